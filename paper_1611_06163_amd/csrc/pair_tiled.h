// pair_tiled.h -- cell-tiled tDPD pair kernel (Eqs. 2-10), shared by the
// translation units that instantiate its builds.
//
// One workgroup of W wavefronts per home cell of the cell list (or per part
// of its home particles when a cell is split over several workgroups).  The
// 27 neighbour cells form one candidate list cut into 64-candidate chunks;
// wave w takes chunks w, w + W, ... and holds up to KC of them in registers
// (one lane per candidate).  (W, KC, split) is the tile shape; every shape
// gives a valid result, and the fastest one for a workload is chosen by
// timing them (tdpd_autotune).  Home particles are walked one at a
// time as wave-uniform broadcasts.  For every (home, candidate) test:
//   - the Fickian flux is accumulated in place per lane and summed across
//     the wave with DPP adds (registers only) once per home particle and
//     register block;
//   - force pairs are compacted with a wave ballot into the wave's LDS ring
//     and evaluated 64 at a time, one pair per lane (Philox noise, weights),
//     then summed per home particle with segmented DPP scans.
// The queued-flux build (QF) compacts every candidate inside the largest
// cutoff into a pair queue instead and evaluates the queue 64 entries at a
// time: the Fickian and random fluxes of each pair (Eqs. 8-10), summed per
// home with segmented DPP scans, and the force pairs among them appended to
// the force ring.  It pays where the flux terms are costly, many species or
// the random flux (a Philox draw per flux pair), and is the build for both.
// Each wave keeps its own partial sums; they are added in wave order at the
// end, so the summation order, and the result, does not depend on timing.
// The EMIT build walks the same candidates (stencil, filter, periodic and
// sheared lifts, FP32 distance test) but, instead of evaluating terms, lists
// every (home gid, candidate gid) with 0 < d^2 < the given cutoff, so the
// production candidate path can be checked pair by pair.
#pragma once

#include <cstddef>
#include <cstring>
#include <type_traits>

#include "launch.h"
#include "membrane_cell.h"
#include "pair_terms.h"

namespace tdpd {

constexpr int kRing = 128;     // per-wave force-pair ring (>= 63 + 64)
constexpr int kHome = 64;      // home particles per pass
constexpr uint32_t kJBits = 26;
// 27 neighbour cells; a sheared boundary row replaces its 3 cells by up to 4
constexpr int kMaxSeg = 30;
// candidates of a cell that can reach it are kept in an LDS list (up to
// kMaxList; larger stencils use the raw candidate order)
constexpr int kMaxList = 768;
static_assert((kRing & (kRing - 1)) == 0 && kRing >= 127, "ring");
static_assert(kMaxList <= 1024 && kMaxSeg <= 64, "list entries: 6-bit segment, 10-bit offset");

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                               ROWS, 0xf, true));
}

// Sum over the 64 lanes with DPP: inclusive scans inside each 16-lane row
// (row_shr 1, 2, 4, 8), then row_bcast 15 and 31 carry row totals upward;
// lane 63 ends with the total (other lanes hold partial sums).  Fixed
// order, registers only.  The two row_bcast steps are single DPP adds whose
// row mask leaves the other rows unwritten (as builtins they take a move of
// zero, a DPP move and an add each); the s_nop gives the DPP read of the
// register the previous VALU instruction wrote its two wait states.  Call
// with all lanes active.
__device__ __forceinline__ float wave_sum_to_last(float v) {
  v += dpp<0x111, 0xf>(v);
  v += dpp<0x112, 0xf>(v);
  v += dpp<0x114, 0xf>(v);
  v += dpp<0x118, 0xf>(v);
  asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf"
               : "+v"(v));
  asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf"
               : "+v"(v));
  return v;
}

// Segmented inclusive sums over the 64 lanes: `start` marks the first lane
// of each run, and afterwards every lane holds the sum of its run from the
// run's first lane up to itself.  The DPP pattern of wave_sum_to_last, a
// lane adding its neighbour's partial only while no run starts in between
// (the start flags travel with the partials).  Fixed order, registers only.
template <int CTRL, int ROWS, int NQ>
__device__ __forceinline__ void seg_step(float (&v)[NQ], int &f) {
  const int fo = __builtin_amdgcn_update_dpp(0, f, CTRL, ROWS, 0xf, true);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const float t = dpp<CTRL, ROWS>(v[q]);
    v[q] = f ? v[q] : v[q] + t;
  }
  f |= fo;
}

template <int NQ>
__device__ __forceinline__ void seg_scan(float (&v)[NQ], bool start) {
  int f = start ? 1 : 0;
  seg_step<0x111, 0xf>(v, f);
  seg_step<0x112, 0xf>(v, f);
  seg_step<0x114, 0xf>(v, f);
  seg_step<0x118, 0xf>(v, f);
  seg_step<0x142, 0xa>(v, f);
  seg_step<0x143, 0xc>(v, f);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// a value every lane holds equally, kept in a scalar register
__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return uint32_t(__builtin_amdgcn_readfirstlane(int(v)));
}

// rank of this lane among the set lanes of mask m
__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}

template <int NS, int W, int KC, bool SH, bool QF>
struct TiledShared {
  // The queued builds keep 32 homes per pass (a cell at the densities of
  // the method holds about a dozen particles; more take further passes):
  // their per-wave flux accumulators scale with it.
  static constexpr int kH = QF ? 32 : kHome;
  // Many species (QF, NS > 4): the block table holds slot and info word
  // only, and the queue evaluation reads a partner's concentrations from L2
  // (a full row would hold NS of them per candidate and cap the occupancy).
  static constexpr bool kNarrow = QF && NS > 4;
  // words of a candidate's row in the block table: slot, info word, the
  // concentrations, padded to whole 16-byte loads
  static constexpr int kRow = kNarrow ? 2 : (2 + NS + 3) / 4 * 4;
  // (first: its offsets fit the immediate offsets of the paired LDS reads)
  float kap[NS][kMaxT * kMaxT];
  float hx[kH], hy[kH], hz[kH], hvx[kH], hvy[kH], hvz[kH];
  float hc[NS][kH];
  uint32_t hgid[kH], hinfo[kH];
  float fa[W][3][kH];
  float qa[W][NS][kH];
  int seg_start[kMaxSeg];
  int seg_pref[kMaxSeg + 1];
  int8_t seg_sg[kMaxSeg][4];  // periodic image per axis: -1, 0 or +1 box length
  int8_t seg_le[kMaxSeg];  // 0 plain, 1 home lifted, 2 candidate lifted (sheared image)
  int8_t seg_m[kMaxSeg];   // multiple of L_x added to the lifted x
  // (QF) the candidates of each wave's register block (kk * 64 + lane):
  // slot, info word and concentrations, read when a queued pair is evaluated
  uint4 tab[QF && !kNarrow ? W : 1][QF && !kNarrow ? KC * 64 : 1][QF && !kNarrow ? kRow / 4 : 1];
  uint2 tabn[kNarrow ? W : 1][kNarrow ? KC * 64 : 1];
  // (QF) pair queue of each wave: candidates within the largest cutoff, as
  // (displacement, home index << kJBits | position in the block table)
  float4 fq[QF ? W : 1][QF ? kRing : 1];
  uint8_t fql[QF && SH ? W : 1][QF && SH ? kRing : 1];  // queue: sheared-image code
  // force ring entries: displacement (overwritten by the force) and, as the
  // bits of w, home index << kJBits | candidate slot
  float4 ring[W][kRing];
  uint8_t rl[SH ? W : 1][kRing];  // ring: sheared-image code of the pair (sheared rows only)
  uint16_t list[kMaxList];  // kept candidates: segment << 10 | offset in the segment
  int list_cnt[kMaxList / 64];
  int list_pref[kMaxList / 64 + 1];
};

// Evaluate ring entries [head, head+m) of wave w (m <= 64) and add them to
// that wave's home accumulators; every home index forms one run in the
// window (entries are appended in home order and the ring is flushed at the
// end of each register block), so the per-run sums (segmented DPP scans,
// registers only) land on distinct homes.
template <int NS, int W, bool LE, typename Shm>
__device__ __forceinline__ void flush_ring(const PairConst &pc, const BoxDev &B, const State &s,
                                           Shm &sh, int w, uint32_t head, int m,
                                           uint32_t k, float le_u) {
  const int lane = threadIdx.x & 63;
  const uint32_t e = (head + lane) & (kRing - 1);
  int hi_i = -1;
  float f3[3] = {0.f, 0.f, 0.f};
  wave_sync();
  if (lane < m) {
    const float4 re = sh.ring[w][e];
    const uint32_t wd = __float_as_uint(re.w);
    hi_i = int(wd >> kJBits);
    const uint32_t j = wd & ((1u << kJBits) - 1);
    const float dx = re.x, dy = re.y, dz = re.z;
    float vxi = sh.hvx[hi_i], vxj = s.vx[j];
    if constexpr (LE) {  // the lifted particle's image moves with +u in x
      const int code = sh.rl[w][e];
      if (code == 1) vxi = __fadd_rn(vxi, le_u);
      if (code == 2) vxj = __fadd_rn(vxj, le_u);
    }
    const float3 f = force_term(pc, B, dx, dy, dz, dist2(dx, dy, dz), vxi, sh.hvy[hi_i],
                                sh.hvz[hi_i], vxj, s.vy[j], s.vz[j], info_type(sh.hinfo[hi_i]),
                                info_type(s.info[j]), sh.hgid[hi_i] - B.gid_base,
                                s.gid[j] - B.gid_base, k);
    f3[0] = f.x;
    f3[1] = f.y;
    f3[2] = f.z;
  }
  // a lane starts a run where its home index differs from the previous
  // lane's (lane 0 always; the lanes past m form a run of their own)
  const int ip = __builtin_amdgcn_update_dpp(-1, hi_i, 0x138, 0xf, 0xf, false);  // wave_shr:1
  const bool run0 = hi_i != ip;
  seg_scan<3>(f3, run0);
  const uint64_t rm = ballot(run0);
  if (lane < m && (lane == m - 1 || ((rm >> (lane + 1)) & 1ull))) {  // the run's last lane
    sh.fa[w][0][hi_i] += f3[0];
    sh.fa[w][1][hi_i] += f3[1];
    sh.fa[w][2][hi_i] += f3[2];
  }
  wave_sync();
}

// Output of the EMIT build: ordered pairs, a counter, the cutoff test.
struct PairEmit {
  int32_t *out;                 // [cap][2] (home gid, candidate gid)
  int64_t cap;
  unsigned long long *count;    // pairs found (also beyond cap)
  uint32_t r2m1;                // bit pattern of fl(rcut^2) less one
  uint32_t k;                   // step counter of the positions
};

// The in-place builds of up to two species and three register chunks ask
// for six waves per SIMD (at most 80 VGPRs), which they fit without spills;
// left to itself the compiler spends a few more registers and loses a wave.
template <int NS, int W, int KC, bool SH, bool QF, bool EMIT = false>
__global__ void __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(NS <= 2 && !QF && !SH && KC <= 3 ? 6 : 1)))
k_pair_tiled(PairConst pc, const BoxDev *__restrict__ boxes, State s,
             const uint32_t *__restrict__ cell_start, int64_t ncell, int split, int filter,
             int64_t per_xcd, int64_t n, const uint32_t *__restrict__ kdev,
             float *__restrict__ F, float *__restrict__ Q, unsigned long long *nzero,
             uint32_t *err, MemArgs ma, int nmemb, int vparts, PairEmit em) {
  using Shm = TiledShared<NS, W, KC, SH, QF>;
  __shared__ Shm sh;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t k = EMIT ? em.k : *kdev;  // random-number step counter
  // the first nmemb workgroups (a multiple of 8) take the per-vertex
  // membrane terms of a share of one cell each (K-Gather and bond forces
  // came from the binning launch), in this workgroup's LDS, beside the pair
  // work
  if (int(blockIdx.x) < nmemb) {
    const int q = int(blockIdx.x);
    if (q < ma.nrbc * vparts)
      membrane_vertices(ma, boxes, s, k, err, q / vparts, q % vparts, vparts,
                        reinterpret_cast<char *>(&sh));
    return;
  }
  // Consecutive workgroups go to different XCDs; each XCD takes a
  // contiguous range of the walk order, so neighbouring cells share its L2.
  // The walk takes a box in blocks of kYBlk rows of cells along y, each
  // block z layer by z layer (x fastest): the three z layers a cell's
  // stencil spans then lie within about 3 kYBlk rows of the walk, which an
  // XCD's 4 MB L2 holds for rows of up to a few hundred cells at about 600
  // bytes of particle data per cell (the row-major order would put a whole
  // y-x layer of the box between them).  Any order gives the same results:
  // cells are independent.
  constexpr int kYBlk = 8;
  const int64_t b = int64_t(blockIdx.x) - nmemb;
  const int64_t item = (b & 7) * per_xcd + (b >> 3);
  if (item >= ncell * split) return;
  const int64_t walk = item / split;  // position of the cell in the walk
  const int part = int(item - walk * split);
  const int S = pc.n_species, T = pc.n_types;
  const BoxDev &B = boxes[box_of_cell(boxes, pc.n_boxes, uint32_t(walk))];
  const int nx = B.nc[0], ny = B.nc[1], nz = B.nc[2];
  int cx, cy, cz;
  {  // (a box holds fewer than 2^31 cells)
    const uint32_t lw = uint32_t(walk - B.cell_base), blk = uint32_t(kYBlk * nz) * uint32_t(nx);
    const uint32_t yb = lw / blk, r = lw - yb * blk;
    const uint32_t hb = uint32_t(min(kYBlk, ny - int(yb) * kYBlk));  // rows of this block
    const uint32_t lay = hb * uint32_t(nx);                           // cells of a layer of it
    cz = int(r / lay);
    const uint32_t r2 = r - uint32_t(cz) * lay, row = r2 / uint32_t(nx);
    cy = int(yb) * kYBlk + int(row);
    cx = int(r2 - row * uint32_t(nx));
  }
  const int64_t lc = (int64_t(cz) * ny + cy) * nx + cx;  // cell index inside its box
  const int64_t cell = B.cell_base + lc;
  // In a sheared box the neighbour row across the y boundary is displaced
  // by delta in x: its candidates come from the min(4, n_x) cells around
  // x -/+ delta, taken in the sheared image (the candidate lifted when the
  // home is in the top row, the home lifted when it is in the bottom row).
  const bool lecell = SH && B.shear != 0.f && (cy == 0 || cy == ny - 1);
  const LeOff le = le_offsets(B, k, pc.dt);
  const int nw = nx < 4 ? nx : 4;
  // 9 (dz, dy) groups of 3 cells, or nw for a group across the sheared boundary
  auto gsize = [&](int g) {
    const int qy = cy + (g % 3) - 1;
    return (lecell && (qy < 0 || qy >= ny)) ? nw : 3;
  };
  if (tid < 36) {
    const int g = tid / 4, t = tid % 4;
    const int dz = g / 3 - 1, dy = g % 3 - 1;
    int off = 0;
    for (int q = 0; q < g; ++q) off += gsize(q);
    if (t < gsize(g)) {
      const int seg = off + t;
      int qy = cy + dy, qz = cz + dz, qx;
      float sx = 0.f, sy = 0.f, sz = 0.f;
      int code = 0, mm = 0;
      if (qz < 0) { qz += nz; sz = -B.L[2]; } else if (qz >= nz) { qz -= nz; sz = B.L[2]; }
      const bool cross = qy < 0 || qy >= ny;
      if (qy < 0) { qy += ny; sy = -B.L[1]; } else if (qy >= ny) { qy -= ny; sy = B.L[1]; }
      if (lecell && cross) {
        code = sy > 0.f ? 2 : 1;
        const float cshift = (code == 2 ? -le.delta : le.delta) * B.inv_h[0];
        const int qu = int(floorf(float(cx) + cshift)) - 1 + t;  // unwrapped cell index
        qx = ((qu % nx) + nx) % nx;
        const int wraps = (qu - qx) / nx;                        // floor(qu / nx)
        mm = code == 2 ? wraps : -wraps;
        sy = 0.f;  // the y lift is part of the sheared image
      } else {
        qx = cx + t - 1;
        if (qx < 0) { qx += nx; sx = -B.L[0]; } else if (qx >= nx) { qx -= nx; sx = B.L[0]; }
      }
      const int64_t q = B.cell_base + (int64_t(qz) * ny + qy) * nx + qx;
      const uint32_t a0 = cell_start[q], a1 = cell_start[q + 1];
      sh.seg_start[seg] = int(a0);
      sh.seg_pref[seg + 1] = int(a1 - a0);  // counts, prefixed below
      sh.seg_sg[seg][0] = int8_t(sx > 0.f ? 1 : (sx < 0.f ? -1 : 0));
      sh.seg_sg[seg][1] = int8_t(sy > 0.f ? 1 : (sy < 0.f ? -1 : 0));
      sh.seg_sg[seg][2] = int8_t(sz > 0.f ? 1 : (sz < 0.f ? -1 : 0));
      sh.seg_le[seg] = int8_t(code);
      sh.seg_m[seg] = int8_t(mm);
    }
  }
  int nseg = 0;
  for (int g = 0; g < 9; ++g) nseg += gsize(g);
  __syncthreads();
  if (tid == 0) {
    sh.seg_pref[0] = 0;
    for (int q = 1; q <= nseg; ++q) sh.seg_pref[q] += sh.seg_pref[q - 1];
  }
  __syncthreads();
  const int nraw = sh.seg_pref[nseg];
  // Keep only candidates within r_max of the home cell's box (with cells of
  // edge r_max, about a quarter of the 27 cells' volume lies farther from
  // every point of the cell).  The test is a conservative superset filter
  // (margins of 1e-3 cell edges); the exact pair rule is applied per home
  // below.  Kept candidates stay in raw order (per-chunk ballots, then an
  // exclusive scan of the chunk counts), so the lane of a candidate, and
  // with it every summation order, does not depend on timing.
  const bool use_list = filter != 0 && nraw <= kMaxList;
  int ncand = nraw, nlist = 0;
  if (use_list) {
    const float hx = B.L[0] / float(nx), hy = B.L[1] / float(ny), hz = B.L[2] / float(nz);
    const float lox = (float(cx) - 1e-3f) * hx, hix = (float(cx) + 1.001f) * hx;
    const float loy = (float(cy) - 1e-3f) * hy, hiy = (float(cy) + 1.001f) * hy;
    const float loz = (float(cz) - 1e-3f) * hz, hiz = (float(cz) + 1.001f) * hz;
    const float reach = sqrtf(pc.rmax2) * 1.0002f + 1e-3f * fmaxf(hx, fmaxf(hy, hz));
    const float reach2 = reach * reach;
    const int nrc = (nraw + 63) / 64;
    for (int c = w; c < nrc; c += W) {
      const int t = c * 64 + lane;
      bool keep = false;
      uint32_t ent = 0;
      if (t < nraw) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (sh.seg_pref[mid] <= t) lo = mid;
          else hi = mid - 1;
        }
        const uint32_t j = uint32_t(sh.seg_start[lo] + (t - sh.seg_pref[lo]));
        ent = (uint32_t(lo) << 10) | uint32_t(t - sh.seg_pref[lo]);
        // candidate position in the home cell's frame (approximate)
        float px = s.x[j] + float(sh.seg_sg[lo][0]) * B.L[0],
              py = s.y[j] + float(sh.seg_sg[lo][1]) * B.L[1],
              pz = s.z[j] + float(sh.seg_sg[lo][2]) * B.L[2];
        if (SH && lecell) {
          const float mL = float(sh.seg_m[lo]) * B.L[0];
          if (sh.seg_le[lo] == 2) {
            px = s.x[j] + le.delta + mL;
            py = s.y[j] + B.L[1];
          } else if (sh.seg_le[lo] == 1) {
            px = s.x[j] - le.delta - mL;
            py = s.y[j] - B.L[1];
          }
        }
        const float ex = fmaxf(fmaxf(lox - px, px - hix), 0.f);
        const float ey = fmaxf(fmaxf(loy - py, py - hiy), 0.f);
        const float ez = fmaxf(fmaxf(loz - pz, pz - hiz), 0.f);
        keep = ex * ex + ey * ey + ez * ez < reach2;
      }
      const uint64_t m = ballot(keep);
      if (lane == 0) sh.list_cnt[c] = __popcll(m);
      if (keep)
        sh.list[c * 64 + int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)))] = ent;
    }
    __syncthreads();
    // exclusive prefix of the per-chunk counts: kept candidate t lives in
    // chunk c (list_pref[c] <= t < list_pref[c + 1]) at c * 64 + t - list_pref[c]
    if (w == 0) {
      int v = lane < nrc ? sh.list_cnt[lane] : 0;
#pragma unroll
      for (int o = 1; o < kMaxList / 64; o <<= 1) {
        const int u = __shfl_up(v, o);
        if (lane >= o) v += u;
      }
      if (lane < nrc) sh.list_pref[lane + 1] = v;
      if (lane == 0) sh.list_pref[0] = 0;
    }
    __syncthreads();
    ncand = sh.list_pref[nrc];
    nlist = nrc;
  }
  const int nchunk = (ncand + 63) / 64;
  const int my_chunks = nchunk > w ? (nchunk - w + W - 1) / W : 0;
  // this workgroup's share of the cell's home particles
  const int c0 = int(cell_start[cell]), cnt = int(cell_start[cell + 1]) - c0;
  const int h0 = c0 + int(int64_t(cnt) * part / split);
  const int h1 = c0 + int(int64_t(cnt) * (part + 1) / split);
  uint32_t zero = 0;  // coincident (home, candidate) tests of this wave (wave-uniform)
  // (16 species x 16 type pairs outnumber the threads of a two-wave workgroup)
  for (int e = tid; e < NS * kMaxT * kMaxT; e += 64 * W) {
    const int sp = e / (kMaxT * kMaxT), tt = e % (kMaxT * kMaxT);
    sh.kap[sp][tt] = (sp < S && tt < T * T) ? pc.kappa[sp * T * T + tt] : 0.f;
  }

  constexpr int kH = Shm::kH;
  for (int hb = h0; hb < h1; hb += kH) {
    const int nh = min(kH, h1 - hb);
    if (tid < nh) {
      const int p = hb + tid;
      sh.hx[tid] = s.x[p];
      sh.hy[tid] = s.y[p];
      sh.hz[tid] = s.z[p];
      sh.hvx[tid] = s.vx[p];
      sh.hvy[tid] = s.vy[p];
      sh.hvz[tid] = s.vz[p];
#pragma unroll
      for (int sp = 0; sp < NS; ++sp) sh.hc[sp][tid] = sp < S ? s.C[sp * n + p] : 0.f;
      sh.hgid[tid] = s.gid[p];
      sh.hinfo[tid] = s.info[p];
    }
    {  // every wave's force and flux accumulators, fa and qa (adjacent)
      static_assert(offsetof(Shm, qa) == offsetof(Shm, fa) + sizeof(sh.fa), "fa, qa adjacent");
      float *acc = reinterpret_cast<float *>(reinterpret_cast<char *>(&sh) + offsetof(Shm, fa));
      for (int e = tid; e < W * (3 + NS) * kH; e += 64 * W) acc[e] = 0.f;
    }
    __syncthreads();
    // this wave's cursors (wave-uniform): the force ring (head, tail), or
    // with QF the pair queue (head, tail) and the force ring (fhead, ftail)
    uint32_t head = 0, tail = 0, fhead = 0, ftail = 0;
    const float Lx = B.L[0], Ly = B.L[1], Lz = B.L[2];
    const bool fick = (pc.terms & TDPD_TERM_FLUX_FICK) != 0;
    // the random flux of Eqs. (9)-(10): only the QF build has it
    const bool rflux = QF && pc.ms_rho > 0.f && (pc.terms & TDPD_TERM_FLUX_RANDOM) != 0;
    // cutoff bit patterns less one (with fluxes off no pair passes the flux test)
    const uint32_t rcc2m1 = (fick || rflux) ? __float_as_uint(pc.rcc2) - 1u : 0u;
    const uint32_t rc2m1 = __float_as_uint(pc.rc2) - 1u;
    // (QF) the queue takes 0 <= d2 < r_q^2, r_q the largest cutoff in use;
    // the home itself and coincident particles are sorted out at evaluation
    const uint32_t rq2b = __float_as_uint((fick || rflux) ? fmaxf(pc.rc2, pc.rcc2) : pc.rc2);

    // (QF) Evaluate queue entries [head, head+m) of this wave (m <= 64), one
    // per lane: the fluxes of each pair, summed per home over its run of
    // entries (entries are appended in home order), and the force pairs
    // among them appended to the force ring, which is evaluated 64 at a time.
    auto flush_queue = [&](int m, auto le_tag) __attribute__((always_inline)) {
      constexpr bool LE = decltype(le_tag)::value;
      const uint32_t e = (head + uint32_t(lane)) & uint32_t(kRing - 1);
      wave_sync();
      const bool valid = lane < m;
      float4 re = make_float4(0.f, 0.f, 0.f, 0.f);
      uint8_t code = 0;
      if (valid) {
        re = sh.fq[w][e];
        if constexpr (LE) code = sh.fql[w][e];
      }
      const uint32_t wd = __float_as_uint(re.w);
      const int i = valid ? int(wd >> kJBits) : 0;
      const uint32_t tq = valid ? (wd & ((1u << kJBits) - 1)) : 0u;
      uint32_t row[Shm::kRow];
      if constexpr (Shm::kNarrow) {
        const uint2 r2 = sh.tabn[w][tq];
        row[0] = r2.x;
        row[1] = r2.y;
      } else {
#pragma unroll
        for (int c = 0; c < Shm::kRow / 4; ++c) {
          if (c > 0 && 4 * c >= 2 + S) {  // words past the species in use
            row[4 * c] = row[4 * c + 1] = row[4 * c + 2] = row[4 * c + 3] = 0u;
            continue;
          }
          const uint4 r4 = sh.tab[w][tq][c];
          row[4 * c] = r4.x;
          row[4 * c + 1] = r4.y;
          row[4 * c + 2] = r4.z;
          row[4 * c + 3] = r4.w;
        }
      }
      // (lanes past m read a stale table row: masked)
      const uint32_t j = valid ? row[0] : 0u, infoj = valid ? row[1] : 0u;
      // the partner's concentrations (from the table, or from L2: the loads
      // are issued here, for every lane, so that their latency overlaps the
      // force-pair compaction below; lanes past m read slot 0)
      float cjn[Shm::kNarrow ? NS : 1];
      if constexpr (Shm::kNarrow) {
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) cjn[sp] = sp < S ? s.C[sp * n + j] : 0.f;
      }
      auto cjv = [&](int sp) __attribute__((always_inline)) -> float {
        if constexpr (Shm::kNarrow) return cjn[sp];
        else return __uint_as_float(row[2 + sp]);
      };
      const float d2 = dist2(re.x, re.y, re.z);  // the bits of the test
      const uint32_t d2b = __float_as_uint(d2);
      const uint32_t infoi = sh.hinfo[i];
      if (ballot(valid && d2b == 0u))  // the home itself, or a coincident particle
        zero += uint32_t(__popcll(ballot(valid && d2b == 0u && j != uint32_t(hb + i))));
      // force pairs: inside r_c and not of the home's own cell body
      const int bi = info_body(infoi);
      const bool hitf = valid && (d2b - 1u < rc2m1) && (bi < 0 || info_body(infoj) != bi);
      const uint64_t fm = ballot(hitf);
      if (fm) {
        if (hitf) {
          const uint32_t fe = (lane_rank(fm) + ftail) & uint32_t(kRing - 1);
          sh.ring[w][fe] = make_float4(re.x, re.y, re.z, __uint_as_float((uint32_t(i) << kJBits) | j));
          if constexpr (LE) sh.rl[w][fe] = code;
        }
        ftail = uniform(ftail) + uint32_t(__popcll(fm));
      }
      if (fick || rflux) {
        const bool inq = valid && d2b - 1u < rcc2m1;
        const float wq = inq ? fmaxf(1.f - __builtin_amdgcn_sqrtf(d2) * pc.inv_rcc, 0.f) : 0.f;
        const float wdc = pc.sc_exp == 2.f ? wq * wq : powu(wq, pc.sc_exp);
        const int tt = info_type(infoi) * T + info_type(infoj);
        float q[NS];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
          q[sp] = 0.f;
          if (fick && inq && (NS == 1 || sp < S))
            q[sp] = sh.kap[sp][tt] * wdc * (cjv(sp) - sh.hc[sp][i]);
        }
        if (rflux && inq) {
          // eps_ij w_RC zeta_ij / sqrt(dt) per species, zeta from the pair's
          // Philox draws: stream 0 words (2,3) for species 0, stream m >= 1
          // for species 2m-1 and 2m; zeta_ij = -zeta_ji (the draw belongs to
          // the lower gid)
          const uint32_t gi = sh.hgid[i] - B.gid_base, gj = s.gid[j] - B.gid_base;
          const uint32_t lo = gi < gj ? gi : gj, hi = gi < gj ? gj : gi;
          const float a = (gi > gj ? -pc.isdt : pc.isdt) * powu(wq, pc.sc_half);
          auto add = [&](int sp, float z) __attribute__((always_inline)) {
            const float csum = fmaxf(cjv(sp) + sh.hc[sp][i], 0.f);
            const float eps = __builtin_amdgcn_sqrtf(pc.ms_rho * sh.kap[sp][tt] * csum);
            q[sp] = fmaf(eps * a, z, q[sp]);
          };
          {
            const u32x4 w0 = philox10(k, lo, hi, B.ctr3, B.seed_lo, B.seed_hi);
            add(0, gauss(w0.c, w0.d));
          }
#pragma unroll
          for (int m2 = 1; 2 * m2 - 1 < NS; ++m2) {  // stream m2: species 2 m2 - 1 and 2 m2
            if (2 * m2 - 1 < S) {
              const u32x4 wm = philox10(k, lo, hi, B.ctr3 | uint32_t(m2), B.seed_lo, B.seed_hi);
              add(2 * m2 - 1, gauss(wm.a, wm.b));
              if (2 * m2 < NS && 2 * m2 < S) add(2 * m2, gauss(wm.c, wm.d));
            }
          }
        }
        // runs of equal home index: a lane starts a run where the index
        // differs from the previous lane's (lane 0 always; lanes past m
        // form a run of zeros)
        const int ik = valid ? i : kH;
        const int ip = __builtin_amdgcn_update_dpp(-1, ik, 0x138, 0xf, 0xf, false);  // wave_shr:1
        const bool run0 = ik != ip;
        seg_scan<NS>(q, run0);
        const uint64_t rm = ballot(run0);
        const bool last = valid && (lane == m - 1 || (lane < 63 && ((rm >> (lane + 1)) & 1ull)));
        if (last) {
#pragma unroll
          for (int sp = 0; sp < NS; ++sp)
            if (NS == 1 || sp < S) sh.qa[w][sp][i] += q[sp];
        }
      }
      wave_sync();
      if (uniform(ftail) - uniform(fhead) >= 64u) {
        flush_ring<NS, W, LE>(pc, B, s, sh, w, fhead, 64, k, le.u);
        fhead = uniform(fhead) + 64u;
      }
    };

    // the register blocks, specialised for cells with a sheared boundary row
    auto blocks = [&](auto le_tag) {
      constexpr bool LE = decltype(le_tag)::value;
    for (int cb = 0; cb < my_chunks; cb += KC) {
      // candidate coordinates, lifted by +L where the candidate sits across
      // the high boundary; lift[kk] bit a says the home coordinate is lifted
      // instead (candidate across the low boundary).  In a sheared row the
      // candidate takes its sheared image (code 2), or bits 3-4 select the
      // home's sheared x for the segment's multiple m (code 1, bits 5-6 =
      // m + 2).  Empty lanes hold NaN, which fails every distance test.
      float cxs[KC], cys[KC], czs[KC], cc[KC][NS];
      uint32_t cj[KC], lift[KC];
      int ct[KC], cbody[KC];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const int chunk = w + W * (cb + kk);
        const int t = chunk * 64 + lane;
        cxs[kk] = cys[kk] = czs[kk] = __builtin_nanf("");
        cj[kk] = 0;
        lift[kk] = 0;
        ct[kk] = 0;
        cbody[kk] = -2;
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) cc[kk][sp] = 0.f;
        if ((cb + kk) < my_chunks && t < ncand) {
          int lo;
          uint32_t j;
          if (use_list) {
            int c = 0, chi = nlist - 1;  // chunk of the list holding t
            while (c < chi) {
              const int mid = (c + chi + 1) >> 1;
              if (sh.list_pref[mid] <= t) c = mid;
              else chi = mid - 1;
            }
            const uint32_t ent = sh.list[c * 64 + t - sh.list_pref[c]];
            lo = int(ent >> 10);
            j = uint32_t(sh.seg_start[lo]) + (ent & 1023u);
          } else {
            lo = 0;  // largest segment whose prefix is <= t
            int hi = nseg - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (sh.seg_pref[mid] <= t) lo = mid;
              else hi = mid - 1;
            }
            j = uint32_t(sh.seg_start[lo] + (t - sh.seg_pref[lo]));
          }
          cj[kk] = j;
          const int gx = sh.seg_sg[lo][0], gy = sh.seg_sg[lo][1], gz = sh.seg_sg[lo][2];
          cxs[kk] = gx > 0 ? __fadd_rn(s.x[j], Lx) : s.x[j];
          cys[kk] = gy > 0 ? __fadd_rn(s.y[j], Ly) : s.y[j];
          czs[kk] = gz > 0 ? __fadd_rn(s.z[j], Lz) : s.z[j];
          lift[kk] = (gx < 0 ? 1u : 0u) | (gy < 0 ? 2u : 0u) | (gz < 0 ? 4u : 0u);
          if constexpr (LE) {
            const int code = sh.seg_le[lo];
            const float mL = float(sh.seg_m[lo]) * Lx;
            if (code == 2) {  // candidate in the sheared image above
              cxs[kk] = __fadd_rn(__fadd_rn(s.x[j], le.delta), mL);
              cys[kk] = __fadd_rn(s.y[j], Ly);
              lift[kk] |= 2u << 3;
            } else if (code == 1) {  // home in the sheared image above
              lift[kk] |= 2u | (1u << 3) | (uint32_t(sh.seg_m[lo] + 2) << 5);
            }
          }
          if constexpr (Shm::kNarrow) {
            sh.tabn[w][kk * 64 + lane] = make_uint2(j, s.info[j]);
          } else if constexpr (QF) {
            uint32_t row[Shm::kRow];
            row[0] = j;
            row[1] = s.info[j];
#pragma unroll
            for (int sp = 0; sp < Shm::kRow - 2; ++sp)
              row[2 + sp] = (sp < NS && sp < S) ? __float_as_uint(s.C[sp * n + j]) : 0u;
#pragma unroll
            for (int c = 0; c < Shm::kRow / 4; ++c)
              if (c == 0 || 4 * c < 2 + S)
                sh.tab[w][kk * 64 + lane][c] =
                    make_uint4(row[4 * c], row[4 * c + 1], row[4 * c + 2], row[4 * c + 3]);
          } else {
            const uint32_t inf = s.info[j];
            ct[kk] = info_type(inf);
            cbody[kk] = info_body(inf);
#pragma unroll
            for (int sp = 0; sp < NS; ++sp)
              if (sp < S) cc[kk][sp] = s.C[sp * n + j];
          }
        }
      }
      // chunks without any lifted coordinate take the plain difference
      bool lifted[KC];
      bool blk_lifted = false;
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        lifted[kk] = ballot(lift[kk] != 0u) != 0ull;
        blk_lifted = blk_lifted || lifted[kk];
      }

      // the home loop, built twice: blocks without any lifted lane (all of
      // an interior cell's) take the plain differences with no lane selects
      auto homes = [&](auto lift_tag) {
        constexpr bool LB = decltype(lift_tag)::value;
      for (int i = 0; i < nh; ++i) {
        const uint32_t infoi = uniform(sh.hinfo[i]);
        if (info_frozen(infoi)) continue;  // frozen particles get F = Q = 0
        const float xi = sh.hx[i], yi = sh.hy[i], zi = sh.hz[i];
        float xil = xi, yil = yi, zil = zi;
        if constexpr (LB) {
          xil = __fadd_rn(xi, Lx);
          yil = __fadd_rn(yi, Ly);
          zil = __fadd_rn(zi, Lz);
        }
        float xm[4] = {0.f, 0.f, 0.f, 0.f};  // home x in the sheared image, m = -2..1
        if constexpr (LE) {
          const float X1 = __fadd_rn(xi, le.delta);
#pragma unroll
          for (int c = 0; c < 4; ++c) xm[c] = __fadd_rn(X1, float(c - 2) * Lx);
        }
        // pair forces skip partners of the home's own cell body; body ids
        // are >= -2 (-1 none, -2 empty lane), so -3 matches nothing
        const int bq = info_body(infoi) >= 0 ? info_body(infoi) : -3;
        const int trow = info_type(infoi) * T;
        const uint32_t hbits = uint32_t(i) << kJBits;
        float qp[NS], ci[NS];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
          qp[sp] = 0.f;
          ci[sp] = sh.hc[sp][i];
        }
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
          if (cb + kk >= my_chunks) break;  // wave-uniform
          float dx, dy, dz;
          if (!LB || !lifted[kk]) {
            dx = __fsub_rn(cxs[kk], xi);
            dy = __fsub_rn(cys[kk], yi);
            dz = __fsub_rn(czs[kk], zi);
          } else {
            float hx = (lift[kk] & 1u) ? xil : xi;
            if constexpr (LE) {
              if (((lift[kk] >> 3) & 3u) == 1u) {
                const uint32_t c = (lift[kk] >> 5) & 3u;
                hx = (c & 2u) ? ((c & 1u) ? xm[3] : xm[2]) : ((c & 1u) ? xm[1] : xm[0]);
              }
            }
            dx = __fsub_rn(cxs[kk], hx);
            dy = __fsub_rn(cys[kk], (lift[kk] & 2u) ? yil : yi);
            dz = __fsub_rn(czs[kk], (lift[kk] & 4u) ? zil : zi);
          }
          const float d2 = dist2(dx, dy, dz);
          if (!QF && ballot(d2 == 0.f)) {  // the home itself, or a coincident particle
            const uint32_t self = uint32_t(hb + i);
            zero += uint32_t(__popcll(ballot((d2 == 0.f) & (cj[kk] != self))));
          }
          // 0 < d2 < r^2 as one unsigned compare of the bit patterns (d2 is
          // +0 or above; the NaN of an empty lane lies above every cutoff)
          const uint32_t d2m1 = __float_as_uint(d2) - 1u;
          if constexpr (EMIT) {
            const bool hit = d2m1 < em.r2m1;
            const uint64_t hm = ballot(hit);
            if (hm) {
              unsigned long long base = 0;
              if (lane == 0) base = atomicAdd(em.count, (unsigned long long)__popcll(hm));
              const uint64_t b0 =
                  (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(base >> 32), 0))) << 32) |
                  uint32_t(__builtin_amdgcn_readlane(int(uint32_t(base)), 0));
              if (hit) {
                const uint64_t q = b0 + lane_rank(hm);
                if (int64_t(q) < em.cap) {
                  em.out[2 * q] = int32_t(sh.hgid[i]);
                  em.out[2 * q + 1] = int32_t(s.gid[cj[kk]]);
                }
              }
            }
            continue;
          }
          if constexpr (QF) {
            // queue the candidate when 0 <= d2 < r_q^2 (one unsigned compare
            // of the bit patterns; the NaN of an empty lane lies above)
            const bool hit = __float_as_uint(d2) < rq2b;
            const uint64_t hm = ballot(hit);
            if (hm) {
              if (hit) {
                const uint32_t e = (lane_rank(hm) + tail) & uint32_t(kRing - 1);
                sh.fq[w][e] = make_float4(dx, dy, dz,
                                          __uint_as_float((hbits + uint32_t(kk * 64)) | uint32_t(lane)));
                if constexpr (LE) sh.fql[w][e] = uint8_t((lift[kk] >> 3) & 3u);
              }
              tail = uniform(tail) + uint32_t(__popcll(hm));
              if (tail - uniform(head) >= 64u) {
                flush_queue(64, le_tag);
                head = uniform(head) + 64u;
              }
            }
            continue;
          }
          {  // flux on every lane, with zero weight outside the flux cutoff
            const float wdc = d2m1 < rcc2m1 ? flux_weight(pc, d2) : 0.f;
            const int tt = trow + ct[kk];
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
              if (NS > 2 && sp >= S) break;  // a build for more species than used
              qp[sp] = fmaf(sh.kap[sp][tt] * wdc, cc[kk][sp] - ci[sp], qp[sp]);
            }
          }
          // (a home outside any cell body has bq = -3, which no candidate's
          // body id matches).  The mask is the AND of two ballots of single
          // compares, each of which is the compare's own lane mask (a ballot
          // of the combined predicate would first turn it into a lane value
          // and back)
          const bool inr = d2m1 < rc2m1, other = cbody[kk] != bq;
          const uint64_t fm = ballot(inr) & ballot(other);
          if (fm) {
            if (inr && other) {
              // rank among the set lanes, with the ring's tail as its base
              const uint32_t e =
                  __builtin_amdgcn_mbcnt_hi(uint32_t(fm >> 32),
                                            __builtin_amdgcn_mbcnt_lo(uint32_t(fm), tail)) &
                  uint32_t(kRing - 1);
              sh.ring[w][e] = make_float4(dx, dy, dz, __uint_as_float(hbits | cj[kk]));
              if constexpr (LE) sh.rl[w][e] = uint8_t((lift[kk] >> 3) & 3u);
            }
            // (cursors re-read as scalars, so their arithmetic stays scalar)
            tail = uniform(tail) + uint32_t(__popcll(fm));
            if (tail - uniform(head) >= 64u) {
              flush_ring<NS, W, LE>(pc, B, s, sh, w, head, 64, k, le.u);
              head = uniform(head) + 64u;
            }
          }
        }
        if (fick && !EMIT && !QF) {
#pragma unroll
          for (int sp = 0; sp < NS; ++sp) {
            if (NS > 2 && sp >= S) break;
            const float t = wave_sum_to_last(qp[sp]);
            if (lane == 63) sh.qa[w][sp][i] += t;
          }
        }
      }
      };
      if (LE || blk_lifted) homes(std::true_type{});
      else homes(std::false_type{});
      // end of the register block: empty the ring (with QF the queue, then
      // the force ring) so that no flush window ever mixes entries of two
      // blocks (which would repeat home indices)
      if constexpr (QF) {
        while (tail != head) {
          const int m = int(min(tail - head, 64u));
          flush_queue(m, le_tag);
          head = uniform(head + uint32_t(m));
        }
        while (ftail != fhead) {
          const int m = int(min(ftail - fhead, 64u));
          flush_ring<NS, W, LE>(pc, B, s, sh, w, fhead, m, k, le.u);
          fhead = uniform(fhead + uint32_t(m));
        }
      } else {
        while (tail != head) {
          const int m = int(min(tail - head, 64u));
          flush_ring<NS, W, LE>(pc, B, s, sh, w, head, m, k, le.u);
          head = uniform(head + uint32_t(m));
        }
      }
    }
    };
    // (SH: a build of the kernel that has the sheared-row variant at all)
    if constexpr (SH) {
      if (lecell) blocks(std::true_type{});
      else blocks(std::false_type{});
    } else {
      blocks(std::false_type{});
    }
    __syncthreads();
    if (tid < nh && !EMIT) {
      const int p = hb + tid;
      float fx = 0.f, fy = 0.f, fz = 0.f;
      const bool frozen = info_frozen(sh.hinfo[tid]);
      if (!frozen) {
#pragma unroll
        for (int v = 0; v < W; ++v) {
          fx += sh.fa[v][0][tid];
          fy += sh.fa[v][1][tid];
          fz += sh.fa[v][2][tid];
        }
        if (pc.terms & TDPD_TERM_BODY_FORCE) {
          fx += pc.body_force[0];
          fy += pc.body_force[1];
          fz += pc.body_force[2];
        }
        if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) atomicOr(err, kErrNonfinite);
      }
      F[3 * p] = fx;
      F[3 * p + 1] = fy;
      F[3 * p + 2] = fz;
#pragma unroll
      for (int sp = 0; sp < NS; ++sp) {
        if (sp >= S) break;
        float q = 0.f;
        if (!frozen) {
#pragma unroll
          for (int v = 0; v < W; ++v) q += sh.qa[v][sp][tid];
          if (pc.has_source) q += source_term(pc, sp, info_type(sh.hinfo[tid]), sh.hc[sp][tid]);
        }
        Q[S * p + sp] = q;
      }
    }
    __syncthreads();
  }
  if (!EMIT && zero && lane == 0) atomicAdd(nzero, (unsigned long long)zero);
}

template <int NS, int W, int KC, bool QF>
void launch_shape(const PairConst &pc, const BoxDev *boxes, State s,
                         const uint32_t *cell_start, int64_t ncell, int split, int filter,
                         int64_t n,
                         const uint32_t *kdev, float *F, float *Q, unsigned long long *nzero,
                         uint32_t *err, bool sheared, const MemArgs &ma, hipStream_t st) {
  const int64_t per_xcd = (ncell * split + 7) / 8;
  // one thread per vertex in the membrane workgroups
  const int vparts = ma.nrbc > 0 ? (ma.max_nv + 64 * W - 1) / (64 * W) : 0;
  const int nmemb = (ma.nrbc * vparts + 7) / 8 * 8;
  const dim3 grid(unsigned(per_xcd * 8 + nmemb)), block(64 * W);
  // the sheared-row variant costs registers: only systems with a sheared box get it
  const PairEmit none{};
  if (sheared)
    hipLaunchKernelGGL((k_pair_tiled<NS, W, KC, true, QF>), grid, block, 0, st, pc, boxes, s,
                       cell_start, ncell, split, filter, per_xcd, n, kdev, F, Q, nzero, err, ma,
                       nmemb, vparts, none);
  else
    hipLaunchKernelGGL((k_pair_tiled<NS, W, KC, false, QF>), grid, block, 0, st, pc, boxes, s,
                       cell_start, ncell, split, filter, per_xcd, n, kdev, F, Q, nzero, err, ma,
                       nmemb, vparts, none);
}

// Launch the build of (NS, QF) for tile shape t; false for a shape not
// built.  Each (NS, QF) is instantiated in one translation unit.
template <int NS, bool QF>
bool launch_tiled_ns(const PairConst &pc, const BoxDev *boxes, State s, const uint32_t *cell_start,
                     int64_t ncell, int64_t n, const uint32_t *kdev, float *F, float *Q,
                     unsigned long long *nzero, uint32_t *err, const PairTile &t, bool sheared,
                     const MemArgs &ma, hipStream_t st) {
// (nine or more species: one or two register chunks only, the rest is
// registers for the species)
#define TDPD_SHAPE(W, KC)                                                                    \
  if constexpr (NS <= 8 || KC <= 2) {                                                        \
    if (t.waves == W && t.chunks == KC) {                                                    \
      launch_shape<NS, W, KC, QF>(pc, boxes, s, cell_start, ncell, t.split, t.filter, n, kdev, \
                                  F, Q, nzero, err, sheared, ma, st);                        \
      return true;                                                                           \
    }                                                                                        \
  }
  TDPD_SHAPE(4, 2)
  TDPD_SHAPE(4, 1)
  TDPD_SHAPE(4, 3)
  TDPD_SHAPE(2, 2)
  TDPD_SHAPE(2, 3)
  TDPD_SHAPE(2, 4)
#undef TDPD_SHAPE
  return false;
}

#define TDPD_TILED_NS_DECL(NS, QF)                                                           \
  template bool launch_tiled_ns<NS, QF>(const PairConst &, const BoxDev *, State,           \
                                        const uint32_t *, int64_t, int64_t, const uint32_t *, \
                                        float *, float *, unsigned long long *, uint32_t *,  \
                                        const PairTile &, bool, const MemArgs &, hipStream_t)

}  // namespace tdpd
