// kernels_pair_list.hip -- tDPD pair forces (Eqs. 3-6) and fluxes (Eqs. 8-10)
// over Verlet neighbour lists: every particle keeps the list of neighbours
// within max(rc, rcc) + skin, built from the cell binning every few steps,
// and between rebuilds the pair kernel tests only those (about a quarter of
// a 27-cell scan at the paper's densities).  The paper's GPU code keeps such
// lists, rebuilt every few steps, in a transposed layout (performance
// section); here entry k of particle i sits at nbr[k * n + i] so that a
// wave's loads of one entry index are contiguous.
//
// One thread per particle, full lists (each pair in both lists, each
// particle sums its own row: no atomics, deterministic).  The flux is
// accumulated while the list is walked; force pairs (about one entry in
// seven) are appended to a per-lane queue in LDS and evaluated in a second
// loop, so the Philox noise and the force arithmetic run on queued pairs
// only instead of on every entry of the walk.
#include "launch_list.h"
#include "pair_terms.h"

namespace tdpd {

constexpr int kListThreads = 256;
constexpr int kForceQueue = 32;  // queued force pairs per lane before a flush

template <int NS>
struct ListShared {
  float kap[NS * kMaxT * kMaxT];
  float alpha[kMaxT * kMaxT], gamma[kMaxT * kMaxT], sigma[kMaxT * kMaxT];
  uint32_t queue[kForceQueue][kListThreads];
};

// Force on i of the queued pairs q[0..m): displacement and d2 recomputed by
// the walk's expressions (so the same predicate holds), then Eqs. (3)-(5)
// with the pair noise of the unordered box-local gid pair at counter k.
template <int NS>
__device__ __forceinline__ void flush_forces(const PairConst &pc, const BoxDev &B,
                                             const ListShared<NS> &sh, int tid, int m,
                                             const float4 *__restrict__ p4,
                                             const float4 *__restrict__ v4, float4 pi, float4 vi,
                                             int ti, uint32_t k, float &fx, float &fy,
                                             float &fz) {
  const uint32_t gi = __float_as_uint(vi.w);
  for (int u = 0; u < m; ++u) {
    const uint32_t j = sh.queue[u][tid];
    const float4 pj = p4[j], vj = v4[j];
    const float dx = pair_disp(pj.x, pi.x, B.L[0]);
    const float dy = pair_disp(pj.y, pi.y, B.L[1]);
    const float dz = pair_disp(pj.z, pi.z, B.L[2]);
    const float d2 = dist2(dx, dy, dz);
    const float rinv = __builtin_amdgcn_rsqf(d2);
    const float r = d2 * rinv;
    const float ex = -dx * rinv, ey = -dy * rinv, ez = -dz * rinv;
    const int tt = ti * pc.n_types + info_type(__float_as_uint(pj.w));
    const float wc = fmaxf(1.f - r * pc.inv_rc, 0.f);
    float fs = 0.f;
    if (pc.terms & TDPD_TERM_CONSERVATIVE) fs += sh.alpha[tt] * wc;
    const float wr = powu(wc, pc.s_half);
    if (pc.terms & TDPD_TERM_DISSIPATIVE) {
      const float ev = ex * (vi.x - vj.x) + ey * (vi.y - vj.y) + ez * (vi.z - vj.z);
      fs -= sh.gamma[tt] * wr * wr * ev;
    }
    if (pc.terms & TDPD_TERM_RANDOM) {
      const uint32_t gj = __float_as_uint(vj.w);
      const uint32_t lo = gi < gj ? gi : gj, hi = gi < gj ? gj : gi;
      const u32x4 w = philox10(k, lo, hi, B.ctr3, B.seed_lo, B.seed_hi);
      fs += sh.sigma[tt] * wr * gauss(w.a, w.b) * pc.isdt;
    }
    fx += fs * ex;
    fy += fs * ey;
    fz += fs * ez;
  }
}

// NS: species bound of the build (the system's count S <= NS).
template <int NS>
__global__ void __launch_bounds__(kListThreads) k_pair_list(PairConst pc,
                                                            const BoxDev *__restrict__ boxes,
                                                            State s, int64_t n,
                                                            const uint32_t *__restrict__ kdev,
                                                            ListDev L, float *__restrict__ F,
                                                            float *__restrict__ Q,
                                                            unsigned long long *nzero,
                                                            uint32_t *err) {
  __shared__ ListShared<NS> sh;
  const int tid = int(threadIdx.x);
  const int T = pc.n_types, S = pc.n_species;
  for (int e = tid; e < NS * kMaxT * kMaxT; e += kListThreads)
    sh.kap[e] = e < S * T * T ? pc.kappa[e] : 0.f;
  for (int e = tid; e < kMaxT * kMaxT; e += kListThreads) {
    sh.alpha[e] = pc.alpha[e];
    sh.gamma[e] = pc.gamma[e];
    sh.sigma[e] = pc.sigma[e];
  }
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * kListThreads + tid;
  if (i >= n) return;
  const float4 pi = L.p4[i];
  const uint32_t infoi = __float_as_uint(pi.w);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  float q[NS];
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) q[sp] = 0.f;
  if (!info_frozen(infoi)) {
    const BoxDev &B = boxes[info_box(infoi)];
    const uint32_t k = *kdev;
    const float4 vi = L.v4[i];
    float ci[NS];
#pragma unroll
    for (int sp = 0; sp < NS; ++sp) ci[sp] = sp < S ? s.C[sp * n + i] : 0.f;
    const int ti = info_type(infoi), bi = info_body(infoi);
    const bool fick = (pc.terms & TDPD_TERM_FLUX_FICK) != 0;
    const int cnt = int(L.ncnt[i]);
    const uint32_t *row = L.nbr + i;
    int m = 0;
    unsigned zero = 0;
    for (int e = 0; e < cnt; ++e) {
      const uint32_t j = row[int64_t(e) * n];
      const float4 pj = L.p4[j];
      const float dx = pair_disp(pj.x, pi.x, B.L[0]);
      const float dy = pair_disp(pj.y, pi.y, B.L[1]);
      const float dz = pair_disp(pj.z, pi.z, B.L[2]);
      const float d2 = dist2(dx, dy, dz);
      if (d2 == 0.f) {  // coincident: skipped and counted
        ++zero;
        continue;
      }
      const uint32_t infoj = __float_as_uint(pj.w);
      if (fick && d2 < pc.rcc2) {
        const float w = flux_weight(pc, d2);
        const int tt = ti * T + info_type(infoj);
#pragma unroll
        for (int sp = 0; sp < NS; ++sp)
          if (sp < S) q[sp] -= sh.kap[sp * T * T + tt] * w * (ci[sp] - s.C[sp * n + j]);
      }
      const int bj = info_body(infoj);
      if (d2 < pc.rc2 && !(bi >= 0 && bi == bj)) {
        sh.queue[m][tid] = j;
        if (++m == kForceQueue) {
          flush_forces<NS>(pc, B, sh, tid, m, L.p4, L.v4, pi, vi, ti, k, fx, fy, fz);
          m = 0;
        }
      }
    }
    flush_forces<NS>(pc, B, sh, tid, m, L.p4, L.v4, pi, vi, ti, k, fx, fy, fz);
    if (zero) atomicAdd(nzero, (unsigned long long)zero);
    if (pc.terms & TDPD_TERM_BODY_FORCE) {
      fx += pc.body_force[0];
      fy += pc.body_force[1];
      fz += pc.body_force[2];
    }
    if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) atomicOr(err, kErrNonfinite);
  }
  F[3 * i] = fx;
  F[3 * i + 1] = fy;
  F[3 * i + 2] = fz;
#pragma unroll
  for (int sp = 0; sp < NS; ++sp)
    if (sp < S) Q[int64_t(S) * i + sp] = q[sp];
}

void launch_pair_list(const PairConst &pc, const BoxDev *boxes, State s, int64_t n,
                      const uint32_t *kdev, const ListDev &L, float *F, float *Q,
                      unsigned long long *nzero, uint32_t *err, hipStream_t st) {
  if (n <= 0) return;
  const dim3 g(unsigned((n + kListThreads - 1) / kListThreads)), b(kListThreads);
  const int S = pc.n_species;
  if (S <= 1)
    hipLaunchKernelGGL(k_pair_list<1>, g, b, 0, st, pc, boxes, s, n, kdev, L, F, Q, nzero, err);
  else if (S <= 2)
    hipLaunchKernelGGL(k_pair_list<2>, g, b, 0, st, pc, boxes, s, n, kdev, L, F, Q, nzero, err);
  else if (S <= 4)
    hipLaunchKernelGGL(k_pair_list<4>, g, b, 0, st, pc, boxes, s, n, kdev, L, F, Q, nzero, err);
  else
    hipLaunchKernelGGL(k_pair_list<kMaxS>, g, b, 0, st, pc, boxes, s, n, kdev, L, F, Q, nzero,
                       err);
}

// ------------------------------------------------------------- list build
// One thread per particle in the sorted order of the binning just done: the
// 27 cells around its own (at least rl wide, so they hold every neighbour
// within rl), each entry tested with the pair rule's displacement.
__global__ void __launch_bounds__(256) k_list_build(const BoxDev *__restrict__ boxes, State s,
                                                    const uint32_t *__restrict__ keys_sorted,
                                                    const uint32_t *__restrict__ cell_start,
                                                    int64_t n, ListDev L, uint32_t *err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t info = s.info[i];
  const BoxDev &B = boxes[info_box(info)];
  const float xi = s.x[i], yi = s.y[i], zi = s.z[i];
  L.p4[i] = make_float4(xi, yi, zi, __uint_as_float(info));
  L.v4[i] = make_float4(s.vx[i], s.vy[i], s.vz[i], __uint_as_float(s.gid[i] - B.gid_base));
  L.xref[i] = make_float4(xi, yi, zi, 0.f);
  uint32_t cnt = 0;
  {  // frozen particles too: their rows are not summed, but list pairs
     // between two of them (tdpd_get_pairs)
    const int nx = B.nc[0], ny = B.nc[1], nz = B.nc[2];
    const uint32_t key = keys_sorted[i] - B.cell_base;
    const int cx = int(key % uint32_t(nx));
    const int cy = int((key / uint32_t(nx)) % uint32_t(ny));
    const int cz = int(key / uint32_t(nx * ny));
    for (int oz = -1; oz <= 1; ++oz) {
      int qz = cz + oz;
      float sz = 0.f;
      if (qz < 0) { qz += nz; sz = -B.L[2]; }
      else if (qz >= nz) { qz -= nz; sz = B.L[2]; }
      for (int oy = -1; oy <= 1; ++oy) {
        int qy = cy + oy;
        float sy = 0.f;
        if (qy < 0) { qy += ny; sy = -B.L[1]; }
        else if (qy >= ny) { qy -= ny; sy = B.L[1]; }
        for (int ox = -1; ox <= 1; ++ox) {
          int qx = cx + ox;
          float sx = 0.f;
          if (qx < 0) { qx += nx; sx = -B.L[0]; }
          else if (qx >= nx) { qx -= nx; sx = B.L[0]; }
          const uint32_t c = B.cell_base + uint32_t((qz * ny + qy) * nx + qx);
          const uint32_t j1 = cell_start[c + 1];
          for (uint32_t j = cell_start[c]; j < j1; ++j) {
            if (j == uint32_t(i)) continue;
            const float d2 = dist2(disp(s.x[j], sx, xi), disp(s.y[j], sy, yi),
                                   disp(s.z[j], sz, zi));
            if (d2 < L.rl2) {
              if (cnt < L.cap) L.nbr[int64_t(cnt) * n + i] = j;
              ++cnt;
            }
          }
        }
      }
    }
  }
  if (cnt > L.cap) {
    atomicOr(err, kErrListFull);
    cnt = L.cap;
  }
  L.ncnt[i] = cnt;
}

void launch_list_build(const BoxDev *boxes, State s, const uint32_t *keys_sorted,
                       const uint32_t *cell_start, int64_t n, const ListDev &L, uint32_t *err,
                       hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_list_build, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, boxes, s,
                     keys_sorted, cell_start, n, L, err);
}

// ------------------------------------------------------------- pair listing
__global__ void __launch_bounds__(256) k_list_emit(const BoxDev *__restrict__ boxes, State s,
                                                   int64_t n, ListDev L, float rcut2,
                                                   int32_t *out, int64_t cap,
                                                   unsigned long long *count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 pi = L.p4[i];
  const uint32_t gi = s.gid[i];
  const BoxDev &B = boxes[info_box(__float_as_uint(pi.w))];
  const int cnt = int(L.ncnt[i]);
  for (int e = 0; e < cnt; ++e) {
    const uint32_t j = L.nbr[int64_t(e) * n + i];
    const uint32_t gj = s.gid[j];
    if (gj <= gi) continue;
    const float4 pj = L.p4[j];
    const float d2 = dist2(pair_disp(pj.x, pi.x, B.L[0]), pair_disp(pj.y, pi.y, B.L[1]),
                           pair_disp(pj.z, pi.z, B.L[2]));
    if (d2 > 0.f && d2 < rcut2) {
      const unsigned long long pos = atomicAdd(count, 1ull);
      if (int64_t(pos) < cap) {
        out[2 * pos] = int32_t(gi);
        out[2 * pos + 1] = int32_t(gj);
      }
    }
  }
}

void launch_list_emit(const BoxDev *boxes, State s, int64_t n, const ListDev &L, float rcut2,
                      int32_t *out, int64_t cap, unsigned long long *count, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_list_emit, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, boxes, s, n,
                     L, rcut2, out, cap, count);
}

}  // namespace tdpd
