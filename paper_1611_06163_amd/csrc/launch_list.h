// launch_list.h -- host-side launchers of the Verlet neighbour-list path
// (the per-particle neighbour lists with a skin, rebuilt every few steps,
// that the paper's GPU implementation keeps: Sections 3.1 and 5.2).
#pragma once

#include "launch.h"

namespace tdpd {

// Error bits of the list path (sticky until the host reads them): a particle
// moved more than half the skin since the last rebuild, so a pair inside the
// cutoff may be missing from the list; a particle had more list neighbours
// than the capacity.
constexpr uint32_t kErrSkin = 4u;
constexpr uint32_t kErrListFull = 8u;

// FP32 displacement x_j - x_i of a pair closer than half the box side L,
// rounded as the cell kernels round it: across the periodic boundary the
// coordinate nearer 0 is lifted by L (one rounding), so d_ji = -d_ij.
__device__ __forceinline__ float pair_disp(float xj, float xi, float L) {
  const float raw = __fsub_rn(xj, xi), half = 0.5f * L;
  if (raw > half) return __fsub_rn(xj, __fadd_rn(xi, L));
  if (raw < -half) return __fsub_rn(__fadd_rn(xj, L), xi);
  return raw;
}

// Lanes that share one particle's list: its neighbours are dealt round-robin
// at the build into `lanes` sub-lists (8, or 4 for systems large enough to
// fill the GPU with four), each walked by its own lane, and the lanes'
// partial sums are added by shuffles in a fixed order.
constexpr int kMaxListLanes = 8;
constexpr int64_t kFourLaneParticles = 131072;  // from this many particles on, 4 lanes

// Buffers of the list path, all in the sorted particle order of the last
// rebuild: entry m of sub-list l of particle i at
// nbr[m * (n * lanes) + i * lanes + l] (m < ncnt[i * lanes + l]),
// so that a wavefront's loads of one entry index are contiguous; the
// positions at the rebuild (xref), and per-step packed copies of the
// particle data the pair kernel gathers: p4 = (x, y, z, info bits),
// v4 = (vx, vy, vz, box-local gid bits) and, for up to four species, c4 =
// the concentrations (zero past the last species; null for more species).
struct ListDev {
  uint32_t *nbr, *ncnt;
  float4 *xref, *p4, *v4, *c4;
  uint32_t cap;       // neighbours per particle (a multiple of kMaxListLanes)
  int lanes;          // sub-lists per particle (4 or 8)
  float rl2;          // (max(rc, rcc) + skin)^2
  float drift2;       // squared displacement that invalidates the list
};

// After the binning: lists of every particle, within rl of it, from the 27
// cells around its own (cells must be at least rl wide), and xref, p4, v4
// of the new order.
void launch_list_build(const BoxDev *boxes, int nbox, State s, int nspec,
                       const uint32_t *cell_start, int64_t ncell, int64_t n, const ListDev &L,
                       uint32_t *err, hipStream_t st);

// First half of a step without binning: half kick and drift as k_prekick,
// then the displacement check against xref (kErrSkin) and p4, v4.
void launch_prekick_list(const PairConst &pc, const BoxDev *boxes, State s, const float *F,
                         const float *Q, int64_t n, bool integrate, const uint32_t *kdev,
                         const ListDev &L, uint32_t *err, uint32_t *kstep, hipStream_t st);

// Pair forces and fluxes over the lists (same outputs as the cell kernels).
void launch_pair_list(const PairConst &pc, const BoxDev *boxes, State s, int64_t n,
                      const uint32_t *kdev, const ListDev &L, float *F, float *Q,
                      unsigned long long *nzero, uint32_t *err, hipStream_t st);

// Pairs (gid_i < gid_j) with 0 < d2 < rcut2 taken from the lists.
void launch_list_emit(const BoxDev *boxes, State s, int64_t n, const ListDev &L, float rcut2,
                      int32_t *out, int64_t cap, unsigned long long *count, hipStream_t st);

}  // namespace tdpd
