// kernels_pair_tiled_rf.hip -- queued-flux builds of the tiled pair kernel
// (pair_tiled.h) for one to four species, the builds that carry the random
// flux of Eqs. (9)-(10).
#include "pair_tiled.h"

namespace tdpd {

TDPD_TILED_NS_DECL(1, true);
TDPD_TILED_NS_DECL(2, true);
TDPD_TILED_NS_DECL(4, true);

}  // namespace tdpd
