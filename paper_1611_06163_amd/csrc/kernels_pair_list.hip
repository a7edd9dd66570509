// kernels_pair_list.hip -- tDPD pair forces (Eqs. 3-6) and fluxes (Eqs. 8-10)
// over Verlet neighbour lists: every particle keeps the list of neighbours
// within max(rc, rcc) + skin, built from the cell binning every few steps,
// and between rebuilds the pair kernel tests only those (about a quarter of
// a 27-cell scan at the paper's densities).  The paper's GPU code keeps such
// lists in a locally transposed layout (Section 3.1) and refreshes them
// every 5 steps in its benchmarks (Section 5.2); here a particle's list is
// dealt into 4 or 8 sub-lists in such a layout, so that a wavefront's loads
// of one entry index are contiguous.
//
// One lane per sub-list, and full lists (each pair in both lists, each
// particle sums its own row: no atomics, deterministic; the lanes' partial
// sums are added by shuffles in a fixed order).  Eight lanes per particle
// give even the 24,500-particle single-cell system 3,000 wavefronts; from
// 131,072 particles on, four lanes fill the GPU with fewer shuffles and
// longer walks (the 246,608-particle channel: pair kernel 187 against
// 199 µs).  The flux is accumulated while a sub-list is walked;
// force pairs (about one entry in seven) are appended to a per-lane queue in
// LDS and evaluated in a second loop, so the Philox noise and the force
// arithmetic run on queued pairs only instead of on every entry.
#include "launch_list.h"
#include "pair_terms.h"

namespace tdpd {

constexpr int kListThreads = 256;
constexpr int kForceQueue = 16;  // queued force pairs per lane before a flush

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

// NS: species bound of the build (the system's count S <= NS); LANES:
// sub-lists per particle.
template <int NS, int LANES>
__global__ void __launch_bounds__(kListThreads) k_pair_list(PairConst pc,
                                                            const BoxDev *__restrict__ boxes,
                                                            State s, int64_t n,
                                                            const uint32_t *__restrict__ kdev,
                                                            ListDev L, float *__restrict__ F,
                                                            float *__restrict__ Q,
                                                            unsigned long long *nzero,
                                                            uint32_t *err, int64_t per_xcd) {
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
  // consecutive workgroups go to different XCDs; each XCD takes a
  // contiguous range of particles (cell order), so the neighbours its lists
  // gather stay in its L2
  const int64_t bb = int64_t(blockIdx.x);
  const int64_t t = ((bb & 7) * per_xcd + (bb >> 3)) * kListThreads + tid;
  const int64_t i = t / LANES;  // the LANES lanes of i are adjacent in one wavefront
  const int lane = int(t % LANES);
  if (i >= n) return;
  const float4 pi = L.p4[i];
  const uint32_t infoi = __float_as_uint(pi.w);
  const bool mobile = !info_frozen(infoi);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  float q[NS];
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) q[sp] = 0.f;
  if (mobile) {
    const BoxDev &B = boxes[info_box(infoi)];
    const uint32_t k = *kdev;
    const float4 vi = L.v4[i];
    // up to four species the concentrations come packed with one load
    constexpr bool kPacked = NS <= 4;
    float ci[NS];
    if (kPacked) {
      const float4 c = L.c4[i];
      const float cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
      for (int sp = 0; sp < NS; ++sp) ci[sp] = cc[sp];
    } else {
#pragma unroll
      for (int sp = 0; sp < NS; ++sp) ci[sp] = sp < S ? s.C[sp * n + i] : 0.f;
    }
    const int ti = info_type(infoi), bi = info_body(infoi);
    const bool fick = (pc.terms & TDPD_TERM_FLUX_FICK) != 0;
    const int cnt = int(L.ncnt[t]);
    const uint32_t *row = L.nbr + t;
    const int64_t stride = n * LANES;
    int m = 0;
    unsigned zero = 0;
    for (int e = 0; e < cnt; ++e) {
      const uint32_t j = row[int64_t(e) * stride];
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
        if (kPacked) {
          const float4 c = L.c4[j];
          const float cj[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
          for (int sp = 0; sp < NS; ++sp)
            if (sp < S) q[sp] -= sh.kap[sp * T * T + tt] * w * (ci[sp] - cj[sp]);
        } else {
#pragma unroll
          for (int sp = 0; sp < NS; ++sp)
            if (sp < S) q[sp] -= sh.kap[sp * T * T + tt] * w * (ci[sp] - s.C[sp * n + j]);
        }
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
  }
  // the lanes of i hold the same i, so they all reach the shuffles
#pragma unroll
  for (int off = LANES / 2; off > 0; off >>= 1) {
    fx += __shfl_xor(fx, off);
    fy += __shfl_xor(fy, off);
    fz += __shfl_xor(fz, off);
#pragma unroll
    for (int sp = 0; sp < NS; ++sp)
      if (sp < S) q[sp] += __shfl_xor(q[sp], off);
  }
  if (lane != 0) return;
  if (mobile) {
    if (pc.has_source)
#pragma unroll
      for (int sp = 0; sp < NS; ++sp)
        if (sp < S) q[sp] += source_term(pc, sp, info_type(infoi), s.C[sp * n + i]);
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

template <int LANES>
static void launch_pair_list_lanes(const PairConst &pc, const BoxDev *boxes, State s, int64_t n,
                                   const uint32_t *kdev, const ListDev &L, float *F, float *Q,
                                   unsigned long long *nzero, uint32_t *err, hipStream_t st) {
  const int64_t lanes = n * LANES, per_xcd = ((lanes + kListThreads - 1) / kListThreads + 7) / 8;
  const dim3 g(unsigned(8 * per_xcd)), b(kListThreads);
  const int S = pc.n_species;
  if (S <= 1)
    hipLaunchKernelGGL((k_pair_list<1, LANES>), g, b, 0, st, pc, boxes, s, n, kdev, L, F, Q,
                       nzero, err, per_xcd);
  else if (S <= 2)
    hipLaunchKernelGGL((k_pair_list<2, LANES>), g, b, 0, st, pc, boxes, s, n, kdev, L, F, Q,
                       nzero, err, per_xcd);
  else if (S <= 4)
    hipLaunchKernelGGL((k_pair_list<4, LANES>), g, b, 0, st, pc, boxes, s, n, kdev, L, F, Q,
                       nzero, err, per_xcd);
  else
    hipLaunchKernelGGL((k_pair_list<kMaxS, LANES>), g, b, 0, st, pc, boxes, s, n, kdev, L, F, Q,
                       nzero, err, per_xcd);
}

void launch_pair_list(const PairConst &pc, const BoxDev *boxes, State s, int64_t n,
                      const uint32_t *kdev, const ListDev &L, float *F, float *Q,
                      unsigned long long *nzero, uint32_t *err, hipStream_t st) {
  if (n <= 0) return;
  if (L.lanes == 4)
    launch_pair_list_lanes<4>(pc, boxes, s, n, kdev, L, F, Q, nzero, err, st);
  else
    launch_pair_list_lanes<8>(pc, boxes, s, n, kdev, L, F, Q, nzero, err, st);
}

// ------------------------------------------------------------- list build
// One workgroup per cell (cells at least rl wide, so the 27 around a cell
// hold every neighbour within rl of its particles).  The stencil's
// positions, shifted into the cell's periodic image, are staged in LDS in
// chunks of up to kStageMax, keeping only entries within rl of the cell's
// box (about three quarters of the 27 cells' volume; compacted in stencil
// order); the cell's particles, LANES lanes each, test them there.  A stencil's entries are dealt round the lanes in one
// sequence (lane l takes entries l, l + LANES, ...), so the sub-lists
// stay within one candidate of each other.  Frozen particles get lists too
// (their rows are never summed, but tdpd_get_pairs lists pairs between two
// of them).
constexpr int kBuildThreads = 256;
constexpr int kStageMax = 2048;  // staged entries per chunk

template <int LANES>
__global__ void __launch_bounds__(kBuildThreads) k_list_build(const BoxDev *__restrict__ boxes,
                                                              int nbox, State s, int nspec,
                                                              const uint32_t *__restrict__ cell_start,
                                                              int64_t n, ListDev L,
                                                              uint32_t *err, int64_t ncell,
                                                              int64_t per_xcd) {
  __shared__ float4 stage[kStageMax];
  __shared__ uint32_t cstart[27], cpref[28];
  __shared__ float cshift[27][3];
  __shared__ uint32_t wsum[kBuildThreads / 64];
  const int tid = int(threadIdx.x);
  // a contiguous range of cells per XCD, as in the pair kernels
  const int64_t bb = int64_t(blockIdx.x), cw = (bb & 7) * per_xcd + (bb >> 3);
  if (cw >= ncell) return;  // uniform over the workgroup
  const uint32_t c = uint32_t(cw);
  const BoxDev &B = boxes[box_of_cell(boxes, nbox, c)];
  const uint32_t h0 = cell_start[c], h1 = cell_start[c + 1];
  if (h0 == h1) return;  // uniform over the workgroup
  if (tid < 27) {
    const int nx = B.nc[0], ny = B.nc[1], nz = B.nc[2];
    const uint32_t key = c - B.cell_base;
    const int cx = int(key % uint32_t(nx));
    const int cy = int((key / uint32_t(nx)) % uint32_t(ny));
    const int cz = int(key / uint32_t(nx * ny));
    int qx = cx + tid % 3 - 1, qy = cy + (tid / 3) % 3 - 1, qz = cz + tid / 9 - 1;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    if (qx < 0) { qx += nx; sx = -B.L[0]; } else if (qx >= nx) { qx -= nx; sx = B.L[0]; }
    if (qy < 0) { qy += ny; sy = -B.L[1]; } else if (qy >= ny) { qy -= ny; sy = B.L[1]; }
    if (qz < 0) { qz += nz; sz = -B.L[2]; } else if (qz >= nz) { qz -= nz; sz = B.L[2]; }
    const uint32_t q = B.cell_base + uint32_t((qz * ny + qy) * nx + qx);
    cstart[tid] = cell_start[q];
    cpref[tid + 1] = cell_start[q + 1] - cell_start[q];
    cshift[tid][0] = sx;
    cshift[tid][1] = sy;
    cshift[tid][2] = sz;
  }
  __syncthreads();
  if (tid == 0) {
    cpref[0] = 0;
    for (int u = 0; u < 27; ++u) cpref[u + 1] += cpref[u];
  }
  __syncthreads();
  const uint32_t total = cpref[27];
  // the cell's box, widened by a rounding margin
  float blo[3], bhi[3];
  {
    const uint32_t key = c - B.cell_base;
    const int cc[3] = {int(key % uint32_t(B.nc[0])), int((key / uint32_t(B.nc[0])) % uint32_t(B.nc[1])),
                       int(key / uint32_t(B.nc[0] * B.nc[1]))};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float h = B.L[a] / float(B.nc[a]), eps = 1e-4f * h;
      blo[a] = float(cc[a]) * h - eps;
      bhi[a] = float(cc[a] + 1) * h + eps;
    }
  }
  constexpr int kHomes = kBuildThreads / LANES;  // particles per pass
  const uint32_t capl = L.cap / LANES;
  const int64_t stride = n * LANES;
  const uint32_t lane = uint32_t(tid % LANES);
  for (uint32_t hb = h0; hb < h1; hb += kHomes) {
    const uint32_t i = hb + uint32_t(tid / LANES);
    const bool home = i < h1;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    if (home) {
      xi = s.x[i];
      yi = s.y[i];
      zi = s.z[i];
      if (lane == 0) {
        const uint32_t info = s.info[i];
        L.p4[i] = make_float4(xi, yi, zi, __uint_as_float(info));
        L.v4[i] = make_float4(s.vx[i], s.vy[i], s.vz[i],
                              __uint_as_float(s.gid[i] - B.gid_base));
        L.xref[i] = make_float4(xi, yi, zi, 0.f);
        if (L.c4) {
          const int S = nspec;
          L.c4[i] = make_float4(s.C[i], S > 1 ? s.C[n + i] : 0.f, S > 2 ? s.C[2 * n + i] : 0.f,
                                S > 3 ? s.C[3 * n + i] : 0.f);
        }
      }
    }
    uint32_t cnt = 0;
    uint32_t dealt = 0;  // staged entries of the earlier chunks
    for (uint32_t g0 = 0; g0 < total;) {  // uniform over the workgroup
      uint32_t m = 0;
      __syncthreads();  // the previous chunk has been read
      while (g0 < total && m + kBuildThreads <= uint32_t(kStageMax)) {
        const uint32_t g = g0 + uint32_t(tid);
        bool keep = false;
        float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
        if (g < total) {
          int u = 0;
          while (cpref[u + 1] <= g) ++u;
          const uint32_t j = cstart[u] + (g - cpref[u]);
          e = make_float4(s.x[j] + cshift[u][0], s.y[j] + cshift[u][1], s.z[j] + cshift[u][2],
                          __uint_as_float(j));
          const float ex = fmaxf(fmaxf(blo[0] - e.x, e.x - bhi[0]), 0.f);
          const float ey = fmaxf(fmaxf(blo[1] - e.y, e.y - bhi[1]), 0.f);
          const float ez = fmaxf(fmaxf(blo[2] - e.z, e.z - bhi[2]), 0.f);
          keep = dist2(ex, ey, ez) < L.rl2;
        }
        // compaction in stencil order: lanes before in the wavefront, then
        // the earlier wavefronts' totals
        const uint64_t bal = __ballot(keep);
        const int w = tid >> 6, l = tid & 63;
        if (l == 0) wsum[w] = uint32_t(__popcll(bal));
        __syncthreads();
        uint32_t off = m, tot = 0;
        for (int q = 0; q < kBuildThreads / 64; ++q) {
          if (q < w) off += wsum[q];
          tot += wsum[q];
        }
        if (keep) stage[off + uint32_t(__popcll(bal & ((1ull << l) - 1ull)))] = e;
        __syncthreads();  // wsum is rewritten by the next round
        m += tot;
        g0 += kBuildThreads;
      }
      if (home) {
        for (uint32_t p = (lane - dealt) & uint32_t(LANES - 1); p < m; p += LANES) {
          const float4 e = stage[p];
          const uint32_t j = __float_as_uint(e.w);
          const float dx = e.x - xi, dy = e.y - yi, dz = e.z - zi;
          if (j != i && dist2(dx, dy, dz) < L.rl2) {
            if (cnt < capl) L.nbr[int64_t(cnt) * stride + int64_t(i) * LANES + lane] = j;
            ++cnt;
          }
        }
      }
      dealt += m;
    }
    if (home) {
      if (cnt > capl) {
        atomicOr(err, kErrListFull);
        cnt = capl;
      }
      L.ncnt[int64_t(i) * LANES + lane] = cnt;
    }
  }
}

void launch_list_build(const BoxDev *boxes, int nbox, State s, int nspec,
                       const uint32_t *cell_start, int64_t ncell, int64_t n, const ListDev &L,
                       uint32_t *err, hipStream_t st) {
  if (n <= 0) return;
  const int64_t per_xcd = (ncell + 7) / 8;
  if (L.lanes == 4)
    hipLaunchKernelGGL(k_list_build<4>, dim3(unsigned(8 * per_xcd)), dim3(kBuildThreads), 0, st,
                       boxes, nbox, s, nspec, cell_start, n, L, err, ncell, per_xcd);
  else
    hipLaunchKernelGGL(k_list_build<8>, dim3(unsigned(8 * per_xcd)), dim3(kBuildThreads), 0, st,
                       boxes, nbox, s, nspec, cell_start, n, L, err, ncell, per_xcd);
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
  const int64_t stride = n * L.lanes;
  for (int l = 0; l < L.lanes; ++l) {
    const int64_t t = i * L.lanes + l;
    const int cnt = int(L.ncnt[t]);
    for (int e = 0; e < cnt; ++e) {
      const uint32_t j = L.nbr[int64_t(e) * stride + t];
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
}

void launch_list_emit(const BoxDev *boxes, State s, int64_t n, const ListDev &L, float rcut2,
                      int32_t *out, int64_t cap, unsigned long long *count, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_list_emit, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, boxes, s, n,
                     L, rcut2, out, cap, count);
}

}  // namespace tdpd
