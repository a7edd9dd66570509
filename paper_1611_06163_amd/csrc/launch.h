// launch.h -- host-side launchers of the library's HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tdpd_device.h"

namespace tdpd {

// ------------------------------------------------------------- membrane
struct MeshDev {
  int nv, ntri, nbond;
  const int32_t *tri;        // [ntri][3]
  const int2 *bond_ab;       // [nbond] local (a, b), a < b
  const float2 *bond_par;    // [nbond] (l_m, k_p)
  const int32_t *bond_off;   // [nv+1]
  const int32_t *bond_inc;   // [2*nbond] bond << 1 | (vertex is b)
  const int32_t *tri_off;    // [nv+1]
  const int4 *tri_inc;       // [nt] (b, c, tri index, -)
  const int32_t *dih_off;    // [nv+1]
  const int4 *dih_inc;       // [nd] (a, b, c, d)
  const uint8_t *dih_role;   // [nd]
  const float *A0t;          // [ntri]
  const int32_t *ring_off;   // [nv+1] 1-ring of each vertex
  const int32_t *ring;       // counter-clockwise from outside, from the smallest index
  float ell;                 // mean rest edge length (surrogate feature scale)
  double A0, V0;             // rest area and volume (FP64, as the totals they are compared with)
  float theta0;
  float p, m_pow, kb, kg, kl, kv, gamma_t, gamma_c;
};

struct MembraneConst {
  float kT, dt;
  int terms;
  int local_only;  // 1: bending and local area only (no K-Gather writes, no global terms)
  int gate;        // > 0: run only at steps k with k % gate == 0
};

// Vertices whose bending and local-area forces come from the surrogate:
// flag[v] != 0 selects Fs[v] instead (global vertex index).
struct SurrUse {
  const uint8_t *flag;
  const float *Fs;
};

// Everything the membrane terms of a set of cells read and write.
struct MemArgs {
  MembraneConst mc;
  const MeshDev *meshes;
  const int32_t *rbc_mesh, *rbc_box;     // [nrbc]
  const int64_t *rbc_first, *rbc_voff;   // [nrbc]
  const uint32_t *slot_of_gid;
  double *av, *centroid;                 // [nrbc][2], [nrbc][3] (FP64 totals)
  float *Fm;                             // [nvert][3] output
  float *Fb;                             // [nrbc][3][bond_stride] per-bond scratch
  int64_t bond_stride;                   // >= nbond of every mesh
  SurrUse su;
  int nrbc;
  int max_nv;                            // largest mesh
};

// Radix sort of (key, value) u32 pairs; keys < 2^key_bits.  tmp buffers of
// the same length; hist needs radix_hist_words(n) words.  Result in
// keys_out/vals_out.  Stable.
size_t radix_hist_words(int64_t n);
void radix_sort(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp,
                uint32_t *vals_tmp, uint32_t *keys_out, uint32_t *vals_out, uint32_t *hist,
                int64_t n, int key_bits, hipStream_t st);

// Membrane forces of an evaluation, indexed by global vertex (launch_membrane).
struct VertexMap {
  const float *Fm;          // [nvert][3] or null
  const int64_t *rbc_first; // [nrbc]
  const int64_t *rbc_voff;  // [nrbc]
};
// First half kick + drift + walls + wrap + cell key (one thread per particle).
// With cell_count, vals gets the particle's unordered rank in its cell (the
// counting binning); else vals = index (the radix binning).  *kdev is the
// counter of this evaluation (sheared boxes take its image offsets).
// finish: the previous step's closing work (launch_postkick's, with `prev`
// its membrane forces) is done first, per particle, with the same
// arithmetic; the counter is then not yet advanced, so this evaluation's is
// *kdev + 1 (the binning advances it: launch_bin_counting's advance).
void launch_prekick(const PairConst &pc, const BoxDev *boxes, State s, float *F,
                    const float *Q, int64_t n, uint32_t *keys, uint32_t *vals, bool integrate,
                    uint32_t *cell_count, uint32_t *kdev, bool finish, VertexMap prev,
                    uint32_t *kstep, hipStream_t st);
// Counting binning after launch_prekick: scan of the cell counts into
// cell_start (counts zeroed for the next step; tile_sum holds
// count_scan_tiles(ncell) words; tmp holds 2n words), scatter, and the rank
// fix-up fused with
// the reorder of every state plane into dst (slot_of_gid of the membrane
// vertices and the sorted keys
// updated).  Same permutation as the stable radix sort.
int64_t count_scan_tiles(int64_t ncell);
// With advance, the scatter also advances the step counter *advance by one.
// With membrane (nrbc > 0), the scan's launch also takes the K-Gather and the
// bond forces of every cell (membrane_elements, `eparts` workgroups per
// cell, counter *kdev + kofs), on the state before the reorder; the pair
// kernel then takes the per-vertex part (launch_pair_tiled).
void launch_bin_counting(State src, State dst, const uint32_t *keys, const uint32_t *rank,
                         uint32_t *cell_count, int64_t ncell, uint32_t *cell_start, uint32_t *tmp,
                         uint32_t *tile_sum, int64_t n, int nspec, uint32_t *slot_of_gid,
                         uint32_t *keys_sorted, uint32_t *advance, const MemArgs &membrane,
                         const BoxDev *boxes, const uint32_t *kdev, int kofs, uint32_t *err,
                         hipStream_t st);
// Workgroups per cell of the scan launch's membrane part; whether its LDS
// holds a cell of max_nv vertices.
int membrane_element_parts(int64_t max_nbond);
bool scan_takes_membrane(int max_nv);
// cell_start[c] = first sorted index of cell c, cell_start[ncell] = n.
void launch_cell_bounds(const uint32_t *sorted_keys, int64_t n, int64_t ncell,
                        uint32_t *cell_start, hipStream_t st);
// dst[p] = src[perm[p]] for every state plane; slot_of_gid[gid] = p for
// membrane vertices (the map serves the membrane gathers only).
void launch_reorder(State src, State dst, const uint32_t *perm, int64_t n, int nspec,
                    uint32_t *slot_of_gid, hipStream_t st);
// Adds the membrane forces Fm (indexed by global vertex, see launch_membrane)
// into F, then (integrate) the second half kick of mobile particles; ends
// the evaluation by advancing the device step counter *kdev by one (the
// kernels of an evaluation at counter k all read k; the next step reads
// k + 1).
void launch_postkick(const PairConst &pc, State s, float *F, const float *Q, int64_t n,
                     VertexMap vm, bool integrate, uint32_t *kdev, hipStream_t st);
// Sets *kdev = k.
void launch_set_counter(uint32_t *kdev, uint32_t k, hipStream_t st);

// Pair forces and fluxes, one thread per particle (sorted order).
// The random-number step counter k is read from device memory (*kdev) so a
// captured graph of a step stays valid from step to step.
void launch_pair_simple(const PairConst &pc, const BoxDev *boxes, State s,
                        const uint32_t *cell_keys,
                        const uint32_t *cell_start, int64_t n, const uint32_t *kdev, float *F,
                        float *Q, unsigned long long *nzero, uint32_t *err, hipStream_t st);
// Tile shape of the cell-tiled pair kernel: wavefronts per workgroup,
// 64-candidate chunks per wavefront held in registers, workgroups per cell,
// and whether the 27-cell stencil is first filtered against the home cell's
// box (1) or tested whole (0).
struct PairTile {
  int waves, chunks, split, filter;
};
extern const PairTile kPairTiles[];  // the shapes the kernel is built for
extern const int kNumPairTiles;
// Whether the shape is built for n_species species.
bool pair_tile_built(const PairTile &t, int n_species);
// Whether the tiled kernel runs its queued-flux build for these parameters
// (the random flux on, or more than four species).
bool pair_tiled_queued(const PairConst &pc);
// Enumerate pairs (gid_i < gid_j) below rcut^2 with the same cell search.
void launch_pair_emit(const PairConst &pc, const BoxDev *boxes, State s,
                      const uint32_t *cell_keys,
                      const uint32_t *cell_start, int64_t n, float rcut2, uint32_t k,
                      int32_t *out, int64_t cap, unsigned long long *count, hipStream_t st);

// FP64 diagnostics in fixed order: [P0,P1,P2, sum v^2, n_mobile, C_0..C_{S-1}]
// FP64 diagnostics: partial sums of kDiagSpan particles per workgroup
// (kDiagFields doubles each) into `partial`, then their fixed-order total
// into out[5 + nspec] (Σv, Σ|v|^2 and the mobile count, ΣC per species).
constexpr int kDiagSpan = 1024;
constexpr int kDiagFields = 5 + kMaxS;
void launch_diag(State s, int64_t n, int nspec, double *partial, double *out, hipStream_t st);
// out[4 + nspec] = (P[3], kT, ΣC[nspec]) from the totals of launch_diag.
void launch_diag_finish(const double *sums, int nspec, double *out, hipStream_t st);

// Copy (SoA -> AoS) in gid order: slot p to row gid[p].
void launch_gid_order(State s, int64_t n, int nspec, const float *F, const float *Q, float *pos,
                      float *vel, float *conc, float *Fo, float *Qo, hipStream_t st);


// All membrane terms of every cell, one workgroup per cell: per-cell FP64
// totals A^t, V^t and centroid (the K-Gather), then per bond the spring,
// viscous and random forces, then per vertex the sum of its bond forces, the
// area/volume constraint forces (K-Apply) and bending, written to
// Fm[rbc_voff[r] + v] (overwritten, not accumulated), so the kernel can run
// beside the pair kernel.  lds_bytes = membrane_lds_bytes(max nv).
size_t membrane_lds_bytes(int max_nv);
void launch_membrane(const MemArgs &ma, const BoxDev *boxes, State s, const uint32_t *kdev,
                     uint32_t *err, size_t lds_bytes, hipStream_t st);

// Pair forces and fluxes, cell-tiled kernel (sheared: some box has
// Lees-Edwards boundaries).  With ma.nrbc > 0 the launch also takes the
// membrane terms of every cell, one cell per extra workgroup (only if
// pair_tiled_takes_membrane for the shape).  Returns false for a shape that
// is not built.
bool launch_pair_tiled(const PairConst &pc, const BoxDev *boxes, State s,
                       const uint32_t *cell_start, int64_t ncell,
                       int64_t n, const uint32_t *kdev, float *F, float *Q,
                       unsigned long long *nzero, uint32_t *err, const PairTile &tile,
                       bool sheared, const MemArgs &ma, hipStream_t st);
// The tiled kernel's candidate path at tile t, listing ordered pairs (home
// gid, candidate gid) with 0 < d^2 < rcut2 of every mobile home into out
// [cap][2] (in no particular order) and their number into *count (cleared by
// the caller); positions at step counter k (the sheared image offset).
// False for a tile shape that is not built.
bool launch_pair_tiled_emit(const PairConst &pc, const BoxDev *boxes, State s,
                            const uint32_t *cell_start, int64_t ncell, int64_t n, uint32_t k,
                            float rcut2, int32_t *out, int64_t cap, unsigned long long *count,
                            unsigned long long *nzero, uint32_t *err, const PairTile &t,
                            bool sheared, hipStream_t st);
// Whether a workgroup of the shape has the LDS for one cell of max_nv vertices.
bool pair_tiled_takes_membrane(const PairTile &t, int n_species, bool sheared, int max_nv);

// ------------------------------------------------------------ surrogate
constexpr int kSurrIn = 20, kSurrHid = 128, kSurrOut = 3;
constexpr int kSurrParams = kSurrHid * kSurrIn + kSurrHid + 2 * (kSurrHid * kSurrHid + kSurrHid) +
                            kSurrOut * kSurrHid + kSurrOut;  // 36,099
constexpr float kSurrDev = 100.f;  // scale of the (A - A0)/A0, (V - V0)/V0 inputs
constexpr int kRingMax = 12;

// offsets of the layers in the flat parameter vector
struct MlpLayout {
  static constexpr int W1 = 0, b1 = W1 + kSurrHid * kSurrIn, W2 = b1 + kSurrHid,
                       b2 = W2 + kSurrHid * kSurrHid, W3 = b2 + kSurrHid,
                       b3 = W3 + kSurrHid * kSurrHid, W4 = b3 + kSurrHid,
                       b4 = W4 + kSurrOut * kSurrHid, end = b4 + kSurrOut;
};
static_assert(MlpLayout::end == kSurrParams, "parameter layout");

enum { kEpiStore = 0, kEpiSilu = 1, kEpiSiluGrad = 2 };
struct GemmArgs {
  const float *A;
  int64_t sa_i, sa_p;
  const float *B;
  int64_t sb_p, sb_j;
  float *C;
  int64_t ldc;
  int64_t M, N, K;
  const float *bias;  // [N] or null
  int epi;
  float *H;           // kEpiSilu: activation out (same layout as C)
  const float *Z;     // kEpiSiluGrad: pre-activation in (same layout as C)
};
void launch_gemm_bf16(const GemmArgs &g, hipStream_t st);
void launch_loss_grad(const float *Y, const float *T, int64_t n, float inv_scale, float *dY,
                      double *part, hipStream_t st);
int64_t loss_grad_blocks(int64_t n);
void launch_sum_parts(const double *part, int64_t n, double *out, hipStream_t st);
void launch_colsum(const float *D, int64_t m, int ld, int ncol, float *out, hipStream_t st);
void launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                 float b2, float eps, float bc1, float bc2, hipStream_t st);

// Network forward pass on n rows of X [n][20] into Y [n][3], one fused
// kernel (weights in LDS, activations on chip); params in the flat layout
// [W1 (128x20), b1, W2, b2, W3, b3, W4 (3x128), b4].  With hdbg the FP32
// hidden activations (before their bfloat16 rounding) also go to hdbg
// [3][n][128] (parity checks).
void mlp_forward(const float *params, const float *X, int64_t n, float *Y, hipStream_t st,
                 float *hdbg = nullptr);
// The same network as four matrix-product launches with the hidden
// activations in Ha, Hb [n][128] (the training path's layout).
void mlp_forward_layers(const float *params, const float *X, int64_t n, float *Ha, float *Hb,
                        float *Y, hipStream_t st);

struct SurrDev {
  const int32_t *vcell, *rbc_mesh, *rbc_box;
  const int64_t *rbc_voff, *rbc_first;
  float *X, *R, *Y, *Fs, *Fp, *stats;
  uint8_t *ok, *flag;
  float s_F, tol;
};
void launch_surr_features(const SurrDev &sd, const BoxDev *boxes, const MeshDev *meshes, State s,
                          const uint32_t *slot_of_gid, const double *av, int64_t nvert,
                          const uint32_t *kdev, float dt, int kofs, hipStream_t st);
void launch_surr_apply(const SurrDev &sd, int64_t nvert, hipStream_t st);
void launch_surr_targets(const SurrDev &sd, float *T, int64_t nvert, hipStream_t st);
void launch_surr_check(const SurrDev &sd, int nrbc, const uint32_t *kdev, int every,
                       hipStream_t st);

}  // namespace tdpd
