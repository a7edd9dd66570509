// kernels_pair_tiled_ns12.hip -- the queued-flux builds of the tiled pair
// kernel (pair_tiled.h) for nine or ten and for eleven or twelve species.
#include "pair_tiled.h"

namespace tdpd {

TDPD_TILED_NS_DECL(10, true);
TDPD_TILED_NS_DECL(12, true);

}  // namespace tdpd
