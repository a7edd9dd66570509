// kernels_pair_tiled.hip -- cell-tiled tDPD pair kernel.
//
// One 64-lane wavefront (one workgroup) per home cell of the cell list.
// The 27 neighbour cells form one candidate list; lanes take candidates
// (64 per chunk, up to kChunks chunks held in registers), home particles are
// walked one at a time as wave-uniform broadcasts from LDS.  For every
// (home, candidate) test:
//   - the Fickian flux (cheap, ~15% hit rate) is accumulated in place per
//     lane and reduced across the wave once per home particle;
//   - force pairs (~4% hit rate, expensive: Philox + Box-Muller + weights)
//     are compacted with a wave ballot into an LDS ring and evaluated 64 at
//     a time, one pair per lane, then summed per home particle in ring order.
// The home loop visits candidates in a fixed order and the ring is consumed
// in append order, so the summation order -- and the result -- is fixed.
#include "launch.h"
#include "pair_terms.h"

namespace tdpd {

constexpr int kChunks = 4;          // candidate chunks of 64 held in registers
constexpr int kRing = 512;          // force-pair ring capacity (>= 63 + 64*kChunks)
constexpr int kHome = 64;           // home particles per pass
constexpr uint32_t kJBits = 26;     // slot bits in a ring entry

static_assert(kRing >= 63 + 64 * kChunks, "ring too small");
static_assert((kRing & (kRing - 1)) == 0, "ring must be a power of two");

__device__ __forceinline__ float sel4(int t, float a0, float a1, float a2, float a3) {
  return t == 0 ? a0 : (t == 1 ? a1 : (t == 2 ? a2 : a3));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

struct TiledShared {
  float hx[kHome], hy[kHome], hz[kHome], hvx[kHome], hvy[kHome], hvz[kHome];
  float hc[kMaxS][kHome];
  uint32_t hgid[kHome], hinfo[kHome];
  float fa[3][kHome];
  float qa[kMaxS][kHome];
  int seg_start[27];
  int seg_pref[28];
  float seg_sh[27][3];
  float rd[3][kRing];     // ring: displacement
  uint32_t rij[kRing];    // ring: home index << kJBits | candidate slot
  float rf[3][64];        // evaluated forces of one batch
};

// Evaluate ring entries [head, head+m) (m <= 64) and add them to the home
// accumulators, summing each run of equal home index in ring order.
__device__ __forceinline__ void flush_ring(const PairConst &pc, const State &s, TiledShared &sh,
                                           uint32_t head, int m, uint32_t k) {
  const int lane = threadIdx.x;
  const uint32_t e = (head + lane) & (kRing - 1);
  int hi_i = -1;
  if (lane < m) {
    const uint32_t w = sh.rij[e];
    hi_i = int(w >> kJBits);
    const uint32_t j = w & ((1u << kJBits) - 1);
    const uint32_t infoi = sh.hinfo[hi_i], infoj = s.info[j];
    const float3 f = force_term(pc, sh.rd[0][e], sh.rd[1][e], sh.rd[2][e],
                                dist2(sh.rd[0][e], sh.rd[1][e], sh.rd[2][e]), sh.hvx[hi_i],
                                sh.hvy[hi_i], sh.hvz[hi_i], s.vx[j], s.vy[j], s.vz[j],
                                info_type(infoi), info_type(infoj), sh.hgid[hi_i], s.gid[j], k);
    sh.rf[0][lane] = f.x;
    sh.rf[1][lane] = f.y;
    sh.rf[2][lane] = f.z;
  }
  __syncthreads();
  if (lane < m) {
    const bool leader =
        lane == 0 || int(sh.rij[(head + lane - 1) & (kRing - 1)] >> kJBits) != hi_i;
    if (leader) {
      float ax = 0.f, ay = 0.f, az = 0.f;
      for (int q = lane; q < m; ++q) {
        if (int(sh.rij[(head + q) & (kRing - 1)] >> kJBits) != hi_i) break;
        ax += sh.rf[0][q];
        ay += sh.rf[1][q];
        az += sh.rf[2][q];
      }
      sh.fa[0][hi_i] += ax;
      sh.fa[1][hi_i] += ay;
      sh.fa[2][hi_i] += az;
    }
  }
  __syncthreads();
}

__global__ void __launch_bounds__(64) k_pair_tiled(PairConst pc, State s,
                                                   const uint32_t *__restrict__ cell_start,
                                                   int64_t ncell, int64_t per_xcd, int64_t n,
                                                   uint32_t k, float *__restrict__ F,
                                                   float *__restrict__ Q,
                                                   unsigned long long *nzero, uint32_t *err) {
  __shared__ TiledShared sh;
  const int lane = threadIdx.x;
  // consecutive workgroups go to different XCDs; give each XCD a contiguous
  // slab of cells so neighbouring cells share that XCD's L2
  const int64_t b = blockIdx.x;
  const int64_t cell = (b & 7) * per_xcd + (b >> 3);
  if (cell >= ncell) return;
  const int S = pc.n_species, T = pc.n_types;
  const int nx = pc.nc[0], ny = pc.nc[1], nz = pc.nc[2];
  const int cx = int(cell % nx), cy = int((cell / nx) % ny), cz = int(cell / (int64_t(nx) * ny));
  if (lane < 27) {
    const int dz = lane / 9 - 1, dy = (lane / 3) % 3 - 1, dx = lane % 3 - 1;
    int qx = cx + dx, qy = cy + dy, qz = cz + dz;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    if (qx < 0) { qx += nx; sx = -pc.L[0]; } else if (qx >= nx) { qx -= nx; sx = pc.L[0]; }
    if (qy < 0) { qy += ny; sy = -pc.L[1]; } else if (qy >= ny) { qy -= ny; sy = pc.L[1]; }
    if (qz < 0) { qz += nz; sz = -pc.L[2]; } else if (qz >= nz) { qz -= nz; sz = pc.L[2]; }
    const int64_t q = (int64_t(qz) * ny + qy) * nx + qx;
    const uint32_t a0 = cell_start[q], a1 = cell_start[q + 1];
    sh.seg_start[lane] = int(a0);
    sh.seg_pref[lane + 1] = int(a1 - a0);  // counts, prefixed below
    sh.seg_sh[lane][0] = sx;
    sh.seg_sh[lane][1] = sy;
    sh.seg_sh[lane][2] = sz;
  }
  __syncthreads();
  if (lane == 0) {
    sh.seg_pref[0] = 0;
    for (int q = 1; q <= 27; ++q) sh.seg_pref[q] += sh.seg_pref[q - 1];
  }
  __syncthreads();
  const int ncand = sh.seg_pref[27];
  const int h0 = int(cell_start[cell]), h1 = int(cell_start[cell + 1]);
  unsigned long long zero = 0;

  for (int hb = h0; hb < h1; hb += kHome) {
    const int nh = min(kHome, h1 - hb);
    if (lane < nh) {
      const int p = hb + lane;
      sh.hx[lane] = s.x[p];
      sh.hy[lane] = s.y[p];
      sh.hz[lane] = s.z[p];
      sh.hvx[lane] = s.vx[p];
      sh.hvy[lane] = s.vy[p];
      sh.hvz[lane] = s.vz[p];
      for (int sp = 0; sp < S; ++sp) sh.hc[sp][lane] = s.C[sp * n + p];
      sh.hgid[lane] = s.gid[p];
      sh.hinfo[lane] = s.info[p];
    }
    sh.fa[0][lane] = sh.fa[1][lane] = sh.fa[2][lane] = 0.f;
    for (int sp = 0; sp < S; ++sp) sh.qa[sp][lane] = 0.f;
    __syncthreads();
    uint32_t head = 0, tail = 0;  // ring cursors (wave-uniform)

    for (int cb = 0; cb < ncand; cb += 64 * kChunks) {
      // candidates of this block into registers
      float cxs[kChunks], cys[kChunks], czs[kChunks], cc[kChunks][kMaxS];
      uint32_t cj[kChunks];
      int ct[kChunks], cbody[kChunks];
      bool cv[kChunks];
#pragma unroll
      for (int kk = 0; kk < kChunks; ++kk) {
        const int t = cb + kk * 64 + lane;
        cv[kk] = t < ncand;
        cxs[kk] = cys[kk] = czs[kk] = 0.f;
        cj[kk] = 0;
        ct[kk] = 0;
        cbody[kk] = -2;
#pragma unroll
        for (int sp = 0; sp < kMaxS; ++sp) cc[kk][sp] = 0.f;
        if (cv[kk]) {
          int lo = 0, hi = 26;  // largest segment with prefix <= t
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sh.seg_pref[mid] <= t) lo = mid;
            else hi = mid - 1;
          }
          const uint32_t j = uint32_t(sh.seg_start[lo] + (t - sh.seg_pref[lo]));
          cj[kk] = j;
          cxs[kk] = __fadd_rn(s.x[j], sh.seg_sh[lo][0]);
          cys[kk] = __fadd_rn(s.y[j], sh.seg_sh[lo][1]);
          czs[kk] = __fadd_rn(s.z[j], sh.seg_sh[lo][2]);
          const uint32_t inf = s.info[j];
          ct[kk] = info_type(inf);
          cbody[kk] = info_body(inf);
#pragma unroll
          for (int sp = 0; sp < kMaxS; ++sp)
            if (sp < S) cc[kk][sp] = s.C[sp * n + j];
        }
      }
      const int nck = min(kChunks, (ncand - cb + 63) / 64);

      for (int i = 0; i < nh; ++i) {
        const uint32_t infoi = sh.hinfo[i];
        if (info_frozen(infoi)) continue;
        const float xi = sh.hx[i], yi = sh.hy[i], zi = sh.hz[i];
        const int ti = info_type(infoi), bi = info_body(infoi);
        const uint32_t self = uint32_t(hb + i);
        float qp[kMaxS], ci[kMaxS], kr[kMaxS][kMaxT];
#pragma unroll
        for (int sp = 0; sp < kMaxS; ++sp) {
          qp[sp] = 0.f;
          ci[sp] = sp < S ? sh.hc[sp][i] : 0.f;
#pragma unroll
          for (int tj = 0; tj < kMaxT; ++tj)
            kr[sp][tj] = (sp < S && tj < T) ? pc.kappa[(sp * T + ti) * T + tj] : 0.f;
        }
#pragma unroll
        for (int kk = 0; kk < kChunks; ++kk) {
          if (kk < nck) {
            const float dx = __fsub_rn(cxs[kk], xi);
            const float dy = __fsub_rn(cys[kk], yi);
            const float dz = __fsub_rn(czs[kk], zi);
            const float d2 = dist2(dx, dy, dz);
            const bool live = cv[kk] && d2 > 0.f;
            const uint64_t zm = __ballot(cv[kk] && d2 == 0.f && cj[kk] != self);
            zero += __popcll(zm);
            if ((pc.terms & TDPD_TERM_FLUX_FICK) && live && d2 < pc.rcc2) {
              const float wdc = flux_weight(pc, d2);
#pragma unroll
              for (int sp = 0; sp < kMaxS; ++sp)
                if (sp < S)
                  qp[sp] -= sel4(ct[kk], kr[sp][0], kr[sp][1], kr[sp][2], kr[sp][3]) * wdc *
                            (ci[sp] - cc[kk][sp]);
            }
            const bool hitf = live && d2 < pc.rc2 && !(bi >= 0 && bi == cbody[kk]);
            const uint64_t fm = __ballot(hitf);
            if (fm) {
              if (hitf) {
                const uint32_t e = (tail + uint32_t(__popcll(fm & __lanemask_lt()))) & (kRing - 1);
                sh.rd[0][e] = dx;
                sh.rd[1][e] = dy;
                sh.rd[2][e] = dz;
                sh.rij[e] = (uint32_t(i) << kJBits) | cj[kk];
              }
              tail += uint32_t(__popcll(fm));
            }
          }
        }
#pragma unroll
        for (int sp = 0; sp < kMaxS; ++sp)
          if (sp < S) {
            const float t = wave_sum(qp[sp]);
            if (lane == 0) sh.qa[sp][i] += t;
          }
        __syncthreads();
        while (tail - head >= 64) {
          flush_ring(pc, s, sh, head, 64, k);
          head += 64;
        }
      }
    }
    while (tail != head) {
      const int m = int(min(tail - head, 64u));
      flush_ring(pc, s, sh, head, m, k);
      head += uint32_t(m);
    }
    if (lane < nh) {
      const int p = hb + lane;
      float fx = 0.f, fy = 0.f, fz = 0.f;
      if (!info_frozen(sh.hinfo[lane])) {
        fx = sh.fa[0][lane];
        fy = sh.fa[1][lane];
        fz = sh.fa[2][lane];
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
      for (int sp = 0; sp < S; ++sp) Q[S * p + sp] = info_frozen(sh.hinfo[lane]) ? 0.f : sh.qa[sp][lane];
    }
    __syncthreads();
  }
  if (lane == 0 && zero) atomicAdd(nzero, zero);
}

void launch_pair_tiled(const PairConst &pc, State s, const uint32_t *cell_start, int64_t ncell,
                       int64_t n, uint32_t k, float *F, float *Q, unsigned long long *nzero,
                       uint32_t *err, hipStream_t st) {
  if (n <= 0 || ncell <= 0) return;
  const int64_t per_xcd = (ncell + 7) / 8;
  hipLaunchKernelGGL(k_pair_tiled, dim3(unsigned(per_xcd * 8)), dim3(64), 0, st, pc, s, cell_start,
                     ncell, per_xcd, n, k, F, Q, nzero, err);
}

}  // namespace tdpd
