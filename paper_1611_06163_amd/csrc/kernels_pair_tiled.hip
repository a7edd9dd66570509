// kernels_pair_tiled.hip -- the cell-tiled pair kernel (pair_tiled.h): the
// one- and two-species builds, the EMIT build that lists the candidate
// path's pairs, and the dispatch over species counts and tile shapes.  The
// queued-flux builds (random flux, and five or more species) are
// instantiated in kernels_pair_tiled_rf.hip, kernels_pair_tiled_ns.hip,
// kernels_pair_tiled_ns12.hip and kernels_pair_tiled_ns16.hip, so the five
// compile in parallel.
#include "pair_tiled.h"

namespace tdpd {

TDPD_TILED_NS_DECL(1, false);
TDPD_TILED_NS_DECL(2, false);
extern TDPD_TILED_NS_DECL(1, true);
extern TDPD_TILED_NS_DECL(2, true);
extern TDPD_TILED_NS_DECL(4, true);
extern TDPD_TILED_NS_DECL(4, false);
extern TDPD_TILED_NS_DECL(8, true);
extern TDPD_TILED_NS_DECL(10, true);
extern TDPD_TILED_NS_DECL(12, true);
extern TDPD_TILED_NS_DECL(16, true);

// The EMIT build of one shape (one species slot: it evaluates no terms).
template <int W, int KC>
static void launch_emit_shape(const PairConst &pc, const BoxDev *boxes, State s,
                              const uint32_t *cell_start, int64_t ncell, int split, int filter,
                              int64_t n, unsigned long long *nzero, uint32_t *err, bool sheared,
                              const PairEmit &em, hipStream_t st) {
  const int64_t per_xcd = (ncell * split + 7) / 8;
  const dim3 grid(unsigned(per_xcd * 8)), block(64 * W);
  const MemArgs ma{};
  if (sheared)
    hipLaunchKernelGGL((k_pair_tiled<1, W, KC, true, false, true>), grid, block, 0, st, pc, boxes,
                       s, cell_start, ncell, split, filter, per_xcd, n, nullptr, nullptr, nullptr,
                       nzero, err, ma, 0, 0, em);
  else
    hipLaunchKernelGGL((k_pair_tiled<1, W, KC, false, false, true>), grid, block, 0, st, pc, boxes,
                       s, cell_start, ncell, split, filter, per_xcd, n, nullptr, nullptr, nullptr,
                       nzero, err, ma, 0, 0, em);
}

// (each shape is built with and without the stencil filter)
const PairTile kPairTiles[] = {
    {4, 2, 1, 1}, {4, 1, 1, 1}, {4, 3, 1, 1}, {2, 2, 1, 1}, {2, 3, 1, 1}, {2, 4, 1, 1},
    {4, 2, 2, 1}, {4, 1, 2, 1}, {2, 2, 2, 1}, {2, 3, 2, 1}, {2, 4, 2, 1}, {2, 2, 4, 1},
    {2, 3, 4, 1}, {4, 1, 4, 1}, {4, 2, 4, 1},
    {4, 2, 1, 0}, {4, 1, 1, 0}, {4, 3, 1, 0}, {2, 2, 1, 0}, {2, 3, 1, 0}, {2, 4, 1, 0},
    {4, 2, 2, 0}, {4, 1, 2, 0}, {2, 2, 2, 0}, {2, 3, 2, 0}, {2, 4, 2, 0}, {2, 2, 4, 0},
    {2, 3, 4, 0}, {4, 1, 4, 0}, {4, 2, 4, 0}};
const int kNumPairTiles = int(sizeof(kPairTiles) / sizeof(kPairTiles[0]));

// The queued-flux build: with the random flux (a Philox draw per flux pair
// only where a pair is inside r_cc) and from five species on (the flux per
// species evaluated on every lane of every candidate test outweighs the
// queue); one to four species without the random flux keep the flux in
// place, which is faster there.
bool pair_tiled_queued(const PairConst &pc) {
  const bool rflux = pc.ms_rho > 0.f && (pc.terms & TDPD_TERM_FLUX_RANDOM) != 0;
  return rflux || pc.n_species > 4;
}

bool launch_pair_tiled(const PairConst &pc, const BoxDev *boxes, State s,
                       const uint32_t *cell_start, int64_t ncell,
                       int64_t n, const uint32_t *kdev, float *F, float *Q,
                       unsigned long long *nzero, uint32_t *err, const PairTile &tile,
                       bool sheared, const MemArgs &ma, hipStream_t st) {
  if (n <= 0 || ncell <= 0) return true;
  if (tile.split < 1 || tile.split > 8 || tile.filter < 0 || tile.filter > 1) return false;
  const bool qf = pair_tiled_queued(pc);
#define TDPD_NS(NS, QF)                                                                      \
  return launch_tiled_ns<NS, QF>(pc, boxes, s, cell_start, ncell, n, kdev, F, Q, nzero, err, \
                                 tile, sheared, ma, st)
  if (pc.n_species <= 1) {
    if (qf) TDPD_NS(1, true);
    TDPD_NS(1, false);
  }
  if (pc.n_species == 2) {
    if (qf) TDPD_NS(2, true);
    TDPD_NS(2, false);
  }
  if (pc.n_species <= 4) {
    if (qf) TDPD_NS(4, true);
    TDPD_NS(4, false);
  }
  if (pc.n_species <= 8) TDPD_NS(8, true);
  if (pc.n_species <= 10) TDPD_NS(10, true);
  if (pc.n_species <= 12) TDPD_NS(12, true);
  TDPD_NS(16, true);
#undef TDPD_NS
}

bool launch_pair_tiled_emit(const PairConst &pc, const BoxDev *boxes, State s,
                            const uint32_t *cell_start, int64_t ncell, int64_t n, uint32_t k,
                            float rcut2, int32_t *out, int64_t cap, unsigned long long *count,
                            unsigned long long *nzero, uint32_t *err, const PairTile &t,
                            bool sheared, hipStream_t st) {
  if (n <= 0 || ncell <= 0) return true;
  if (t.split < 1 || t.split > 8 || t.filter < 0 || t.filter > 1) return false;
  uint32_t r2bits;
  std::memcpy(&r2bits, &rcut2, sizeof(r2bits));
  const PairEmit em{out, cap, count, r2bits - 1u, k};
#define TDPD_EMIT_SHAPE(W, KC)                                                              \
  if (t.waves == W && t.chunks == KC) {                                                     \
    launch_emit_shape<W, KC>(pc, boxes, s, cell_start, ncell, t.split, t.filter, n, nzero, err, \
                             sheared, em, st);                                              \
    return true;                                                                            \
  }
  TDPD_EMIT_SHAPE(4, 2)
  TDPD_EMIT_SHAPE(4, 1)
  TDPD_EMIT_SHAPE(4, 3)
  TDPD_EMIT_SHAPE(2, 2)
  TDPD_EMIT_SHAPE(2, 3)
  TDPD_EMIT_SHAPE(2, 4)
#undef TDPD_EMIT_SHAPE
  return false;
}

bool pair_tile_built(const PairTile &t, int n_species) {
  for (int i = 0; i < kNumPairTiles; ++i)
    if (kPairTiles[i].waves == t.waves && kPairTiles[i].chunks == t.chunks &&
        kPairTiles[i].split == t.split && kPairTiles[i].filter == t.filter)
      return n_species <= 8 || t.chunks <= 2;
  return false;
}

// LDS of one workgroup of the shape, which the membrane workgroups reuse
// (the in-place build, the smaller of the two, where both exist).
template <int NS, int W, bool QF>
static size_t lds_nsw(int chunks, bool sheared) {
  if (chunks >= 4) return sheared ? sizeof(TiledShared<NS, W, 4, true, QF>) : sizeof(TiledShared<NS, W, 4, false, QF>);
  if (chunks == 3) return sheared ? sizeof(TiledShared<NS, W, 3, true, QF>) : sizeof(TiledShared<NS, W, 3, false, QF>);
  if (chunks == 2) return sheared ? sizeof(TiledShared<NS, W, 2, true, QF>) : sizeof(TiledShared<NS, W, 2, false, QF>);
  return sheared ? sizeof(TiledShared<NS, W, 1, true, QF>) : sizeof(TiledShared<NS, W, 1, false, QF>);
}

template <int NS, bool QF>
static size_t lds_ns(const PairTile &t, bool sheared) {
  return t.waves == 2 ? lds_nsw<NS, 2, QF>(t.chunks, sheared) : lds_nsw<NS, 4, QF>(t.chunks, sheared);
}

bool pair_tiled_takes_membrane(const PairTile &t, int n_species, bool sheared, int max_nv) {
  if (t.waves != 2 && t.waves != 4) return false;
  const size_t have = n_species <= 1   ? lds_ns<1, false>(t, sheared)
                      : n_species == 2 ? lds_ns<2, false>(t, sheared)
                      : n_species <= 4 ? lds_ns<4, false>(t, sheared)
                      : n_species <= 8 ? lds_ns<8, true>(t, sheared)
                      : n_species <= 10 ? lds_ns<10, true>(t, sheared)
                      : n_species <= 12 ? lds_ns<12, true>(t, sheared)
                                        : lds_ns<16, true>(t, sheared);
  return membrane_cell_lds(max_nv, 64 * t.waves) <= have;
}

}  // namespace tdpd
