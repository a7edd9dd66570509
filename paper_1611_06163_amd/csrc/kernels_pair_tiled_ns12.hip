// kernels_pair_tiled_ns12.hip -- the queued-flux build of the tiled pair
// kernel (pair_tiled.h) for nine to twelve species.
#include "pair_tiled.h"

namespace tdpd {

TDPD_TILED_NS_DECL(12, true);

}  // namespace tdpd
