// kernels_pair_tiled_ns.hip -- builds of the tiled pair kernel
// (pair_tiled.h) for three or four species (flux in place) and for five to
// eight (queued flux).
#include "pair_tiled.h"

namespace tdpd {

TDPD_TILED_NS_DECL(4, false);
TDPD_TILED_NS_DECL(8, true);

}  // namespace tdpd
