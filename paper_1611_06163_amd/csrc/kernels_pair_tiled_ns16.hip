// kernels_pair_tiled_ns16.hip -- the queued-flux build of the tiled pair
// kernel (pair_tiled.h) for thirteen to sixteen species.
#include "pair_tiled.h"

namespace tdpd {

TDPD_TILED_NS_DECL(16, true);

}  // namespace tdpd
