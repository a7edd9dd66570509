// kernels_pair_tiled.hip -- cell-tiled tDPD pair kernel (Eqs. 2-10).
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
//     then summed per home particle in ring order.
// Each wave keeps its own partial sums; they are added in wave order at the
// end, so the summation order, and the result, does not depend on timing.
// The EMIT build walks the same candidates (stencil, filter, periodic and
// sheared lifts, FP32 distance test) but, instead of evaluating terms, lists
// every (home gid, candidate gid) with 0 < d^2 < the given cutoff, so the
// production candidate path can be checked pair by pair.
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
// order, registers only.
__device__ __forceinline__ float wave_sum_to_last(float v) {
  v += dpp<0x111, 0xf>(v);
  v += dpp<0x112, 0xf>(v);
  v += dpp<0x114, 0xf>(v);
  v += dpp<0x118, 0xf>(v);
  v += dpp<0x142, 0xa>(v);
  v += dpp<0x143, 0xc>(v);
  return v;
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

template <int NS, int W, bool SH>
struct TiledShared {
  float hx[kHome], hy[kHome], hz[kHome], hvx[kHome], hvy[kHome], hvz[kHome];
  float hc[NS][kHome];
  uint32_t hgid[kHome], hinfo[kHome];
  float fa[W][3][kHome];
  float qa[W][NS][kHome];
  float kap[NS][kMaxT * kMaxT];
  int seg_start[kMaxSeg];
  int seg_pref[kMaxSeg + 1];
  int8_t seg_sg[kMaxSeg][4];  // periodic image per axis: -1, 0 or +1 box length
  int8_t seg_le[kMaxSeg];  // 0 plain, 1 home lifted, 2 candidate lifted (sheared image)
  int8_t seg_m[kMaxSeg];   // multiple of L_x added to the lifted x
  // ring entries: displacement (overwritten by the force) and, as the bits
  // of w, home index << kJBits | candidate slot
  float4 ring[W][kRing];
  uint8_t rl[SH ? W : 1][kRing];  // ring: sheared-image code of the pair (sheared rows only)
  uint16_t list[kMaxList];  // kept candidates: segment << 10 | offset in the segment
  int list_cnt[kMaxList / 64];
  int list_pref[kMaxList / 64 + 1];
};

// Evaluate ring entries [head, head+m) of wave w (m <= 64) and add them to
// that wave's home accumulators; every home index forms one run in the
// window (entries are appended in home order and the ring is flushed at the
// end of each register block), so run leaders never collide.
template <int NS, int W, bool LE, typename Shm>
__device__ __forceinline__ void flush_ring(const PairConst &pc, const BoxDev &B, const State &s,
                                           Shm &sh, int w, uint32_t head, int m,
                                           uint32_t k, float le_u) {
  const int lane = threadIdx.x & 63;
  const uint32_t e = (head + lane) & (kRing - 1);
  int hi_i = -1;
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
    sh.ring[w][e] = make_float4(f.x, f.y, f.z, re.w);
  }
  wave_sync();
  if (lane < m) {
    const bool leader =
        lane == 0 ||
        int(__float_as_uint(sh.ring[w][(head + lane - 1) & (kRing - 1)].w) >> kJBits) != hi_i;
    if (leader) {
      float ax = 0.f, ay = 0.f, az = 0.f;
      for (int q = lane; q < m; ++q) {
        const float4 rq = sh.ring[w][(head + q) & (kRing - 1)];
        if (int(__float_as_uint(rq.w) >> kJBits) != hi_i) break;
        ax += rq.x;
        ay += rq.y;
        az += rq.z;
      }
      sh.fa[w][0][hi_i] += ax;
      sh.fa[w][1][hi_i] += ay;
      sh.fa[w][2][hi_i] += az;
    }
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

template <int NS, int W, int KC, bool SH, bool EMIT = false>
__global__ void __launch_bounds__(64 * W) k_pair_tiled(PairConst pc,
                                                            const BoxDev *__restrict__ boxes,
                                                            State s,
                                                            const uint32_t *__restrict__ cell_start,
                                                            int64_t ncell, int split, int filter,
                                                            int64_t per_xcd, int64_t n,
                                                            const uint32_t *__restrict__ kdev,
                                                            float *__restrict__ F,
                                                            float *__restrict__ Q,
                                                            unsigned long long *nzero,
                                                            uint32_t *err, MemArgs ma, int nmemb,
                                                            int vparts, PairEmit em) {
  __shared__ TiledShared<NS, W, SH> sh;
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
  // consecutive workgroups go to different XCDs; give each XCD a contiguous
  // slab of cells so neighbouring cells share that XCD's L2
  const int64_t b = int64_t(blockIdx.x) - nmemb;
  const int64_t item = (b & 7) * per_xcd + (b >> 3);
  if (item >= ncell * split) return;
  const int64_t cell = item / split;
  const int part = int(item - cell * split);
  const int S = pc.n_species, T = pc.n_types;
  const BoxDev &B = boxes[box_of_cell(boxes, pc.n_boxes, uint32_t(cell))];
  const int nx = B.nc[0], ny = B.nc[1], nz = B.nc[2];
  const int64_t lc = cell - B.cell_base;  // cell index inside its box
  const int cx = int(lc % nx), cy = int((lc / nx) % ny), cz = int(lc / (int64_t(nx) * ny));
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

  for (int hb = h0; hb < h1; hb += kHome) {
    const int nh = min(kHome, h1 - hb);
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
    sh.fa[w][0][lane] = sh.fa[w][1][lane] = sh.fa[w][2][lane] = 0.f;
#pragma unroll
    for (int sp = 0; sp < NS; ++sp) sh.qa[w][sp][lane] = 0.f;
    __syncthreads();
    uint32_t head = 0, tail = 0;  // this wave's ring cursors (wave-uniform)
    const float Lx = B.L[0], Ly = B.L[1], Lz = B.L[2];
    const bool fick = (pc.terms & TDPD_TERM_FLUX_FICK) != 0;
    // cutoff bit patterns less one (with fluxes off no pair passes the flux test)
    const uint32_t rcc2m1 = fick ? __float_as_uint(pc.rcc2) - 1u : 0u;
    const uint32_t rc2m1 = __float_as_uint(pc.rc2) - 1u;

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
          const uint32_t inf = s.info[j];
          ct[kk] = info_type(inf);
          cbody[kk] = info_body(inf);
#pragma unroll
          for (int sp = 0; sp < NS; ++sp)
            if (sp < S) cc[kk][sp] = s.C[sp * n + j];
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
          if (ballot(d2 == 0.f)) {  // the home itself, or a coincident particle
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
          {  // flux on every lane, with zero weight outside the flux cutoff
            const float wdc = d2m1 < rcc2m1 ? flux_weight(pc, d2) : 0.f;
            const int tt = trow + ct[kk];
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
              if (NS > 2 && sp >= S) break;  // a build for more species than used
              qp[sp] = fmaf(sh.kap[sp][tt] * wdc, cc[kk][sp] - ci[sp], qp[sp]);
            }
          }
          // homes outside any cell body test the cutoff alone
          const bool hitf = bq == -3 ? d2m1 < rc2m1 : (d2m1 < rc2m1) & (cbody[kk] != bq);
          const uint64_t fm = ballot(hitf);
          if (fm) {
            if (hitf) {
              const uint32_t e = (lane_rank(fm) + tail) & uint32_t(kRing - 1);
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
        if (fick && !EMIT) {
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
      // end of the register block: empty the ring so that no flush window
      // ever mixes entries of two blocks (which would repeat home indices)
      while (tail != head) {
        const int m = int(min(tail - head, 64u));
        flush_ring<NS, W, LE>(pc, B, s, sh, w, head, m, k, le.u);
        head = uniform(head + uint32_t(m));
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

template <int NS, int W, int KC>
static void launch_shape(const PairConst &pc, const BoxDev *boxes, State s,
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
    hipLaunchKernelGGL((k_pair_tiled<NS, W, KC, true>), grid, block, 0, st, pc, boxes, s,
                       cell_start, ncell, split, filter, per_xcd, n, kdev, F, Q, nzero, err, ma,
                       nmemb, vparts, none);
  else
    hipLaunchKernelGGL((k_pair_tiled<NS, W, KC, false>), grid, block, 0, st, pc, boxes, s,
                       cell_start, ncell, split, filter, per_xcd, n, kdev, F, Q, nzero, err, ma,
                       nmemb, vparts, none);
}

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
    hipLaunchKernelGGL((k_pair_tiled<1, W, KC, true, true>), grid, block, 0, st, pc, boxes, s,
                       cell_start, ncell, split, filter, per_xcd, n, nullptr, nullptr, nullptr,
                       nzero, err, ma, 0, 0, em);
  else
    hipLaunchKernelGGL((k_pair_tiled<1, W, KC, false, true>), grid, block, 0, st, pc, boxes, s,
                       cell_start, ncell, split, filter, per_xcd, n, nullptr, nullptr, nullptr,
                       nzero, err, ma, 0, 0, em);
}

template <int NS>
static bool launch_ns(const PairConst &pc, const BoxDev *boxes, State s, const uint32_t *cell_start,
                      int64_t ncell, int64_t n, const uint32_t *kdev, float *F, float *Q,
                      unsigned long long *nzero, uint32_t *err, const PairTile &t,
                      bool sheared, const MemArgs &ma, hipStream_t st) {
// (16 species: one or two register chunks only, the rest is registers for
// the species)
#define TDPD_SHAPE(W, KC)                                                                    \
  if constexpr (NS < 16 || KC <= 2) {                                                        \
    if (t.waves == W && t.chunks == KC) {                                                    \
      launch_shape<NS, W, KC>(pc, boxes, s, cell_start, ncell, t.split, t.filter, n, kdev, F, \
                              Q, nzero, err, sheared, ma, st);                               \
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

// (each shape is built with and without the stencil filter)
const PairTile kPairTiles[] = {
    {4, 2, 1, 1}, {4, 1, 1, 1}, {4, 3, 1, 1}, {2, 2, 1, 1}, {2, 3, 1, 1}, {2, 4, 1, 1},
    {4, 2, 2, 1}, {4, 1, 2, 1}, {2, 2, 2, 1}, {2, 3, 2, 1}, {2, 4, 2, 1}, {2, 2, 4, 1},
    {2, 3, 4, 1}, {4, 1, 4, 1}, {4, 2, 4, 1},
    {4, 2, 1, 0}, {4, 1, 1, 0}, {4, 3, 1, 0}, {2, 2, 1, 0}, {2, 3, 1, 0}, {2, 4, 1, 0},
    {4, 2, 2, 0}, {4, 1, 2, 0}, {2, 2, 2, 0}, {2, 3, 2, 0}, {2, 4, 2, 0}, {2, 2, 4, 0},
    {2, 3, 4, 0}, {4, 1, 4, 0}, {4, 2, 4, 0}};
const int kNumPairTiles = int(sizeof(kPairTiles) / sizeof(kPairTiles[0]));

bool launch_pair_tiled(const PairConst &pc, const BoxDev *boxes, State s,
                       const uint32_t *cell_start, int64_t ncell,
                       int64_t n, const uint32_t *kdev, float *F, float *Q,
                       unsigned long long *nzero, uint32_t *err, const PairTile &tile,
                       bool sheared, const MemArgs &ma, hipStream_t st) {
  if (n <= 0 || ncell <= 0) return true;
  if (tile.split < 1 || tile.split > 8 || tile.filter < 0 || tile.filter > 1) return false;
  if (pc.n_species <= 1)
    return launch_ns<1>(pc, boxes, s, cell_start, ncell, n, kdev, F, Q, nzero, err, tile, sheared, ma, st);
  if (pc.n_species == 2)
    return launch_ns<2>(pc, boxes, s, cell_start, ncell, n, kdev, F, Q, nzero, err, tile, sheared, ma, st);
  if (pc.n_species <= 4)
    return launch_ns<4>(pc, boxes, s, cell_start, ncell, n, kdev, F, Q, nzero, err, tile, sheared, ma, st);
  if (pc.n_species <= 8)
    return launch_ns<8>(pc, boxes, s, cell_start, ncell, n, kdev, F, Q, nzero, err, tile, sheared, ma, st);
  return launch_ns<16>(pc, boxes, s, cell_start, ncell, n, kdev, F, Q, nzero, err, tile, sheared, ma, st);
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

// LDS of one workgroup of the shape, which the membrane workgroups reuse.
template <int NS>
static size_t lds_ns(const PairTile &t, bool sheared) {
  if (t.waves == 2) return sheared ? sizeof(TiledShared<NS, 2, true>) : sizeof(TiledShared<NS, 2, false>);
  return sheared ? sizeof(TiledShared<NS, 4, true>) : sizeof(TiledShared<NS, 4, false>);
}

bool pair_tiled_takes_membrane(const PairTile &t, int n_species, bool sheared, int max_nv) {
  if (t.waves != 2 && t.waves != 4) return false;
  const size_t have = n_species <= 1   ? lds_ns<1>(t, sheared)
                      : n_species == 2 ? lds_ns<2>(t, sheared)
                      : n_species <= 4 ? lds_ns<4>(t, sheared)
                      : n_species <= 8 ? lds_ns<8>(t, sheared)
                                       : lds_ns<16>(t, sheared);
  return membrane_cell_lds(max_nv, 64 * t.waves) <= have;
}

}  // namespace tdpd
