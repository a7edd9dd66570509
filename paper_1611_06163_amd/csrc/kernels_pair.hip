// kernels_pair.hip -- tDPD pair forces (Eqs. 3-6) and concentration fluxes
// (Eqs. 8-10) over the cell list.
//
// Full-shell gather: particle i sums F_ij over every neighbour j itself, so
// no atomics are needed and the result is deterministic.  F_ij and F_ji are
// evaluated by the same expressions with d and v_ij negated and the same
// pair noise (Philox counter keyed by the unordered gid pair), so the two
// evaluations are exact negatives of each other.
#include "launch.h"

namespace tdpd {

// Pair interaction of home particle i with candidate j at FP32 displacement
// d = x_j + s - x_i (d2 = |d|^2 under the exact predicate, 0 < d2 < rmax2).
struct PairAcc {
  float fx, fy, fz;
  float q[kMaxS];
};

__device__ __forceinline__ void pair_term(const PairConst &pc, const BoxDev &B, float dx, float dy,
                                          float dz, float d2,
                                          float vxi, float vyi, float vzi, float vxj, float vyj,
                                          float vzj, const float *ci, const float *cj, int ti,
                                          int tj, bool same_body, uint32_t gi, uint32_t gj,
                                          uint32_t k, PairAcc &acc) {
  const float rinv = __builtin_amdgcn_rsqf(d2);
  const float r = d2 * rinv;
  // e_ij points from j to i: e = -d / r
  const float ex = -dx * rinv, ey = -dy * rinv, ez = -dz * rinv;
  const uint32_t lo = gi < gj ? gi : gj, hi = gi < gj ? gj : gi;
  const bool need_noise =
      (d2 < pc.rc2 && !same_body && (pc.terms & TDPD_TERM_RANDOM)) ||
      (d2 < pc.rcc2 && pc.ms_rho > 0.f && (pc.terms & TDPD_TERM_FLUX_RANDOM));
  u32x4 w = {0, 0, 0, 0};
  if (need_noise) w = philox10(k, lo, hi, B.ctr3, B.seed_lo, B.seed_hi);
  if (d2 < pc.rc2 && !same_body) {
    const int tt = ti * pc.n_types + tj;
    const float wc = fmaxf(1.f - r * pc.inv_rc, 0.f);
    float fs = 0.f;
    if (pc.terms & TDPD_TERM_CONSERVATIVE) fs += pc.alpha[tt] * wc;
    const float wr = powu(wc, pc.s_half);
    if (pc.terms & TDPD_TERM_DISSIPATIVE) {
      const float ev = ex * (vxi - vxj) + ey * (vyi - vyj) + ez * (vzi - vzj);
      fs -= pc.gamma[tt] * wr * wr * ev;
    }
    if (pc.terms & TDPD_TERM_RANDOM) fs += pc.sigma[tt] * wr * gauss(w.a, w.b) * pc.isdt;
    acc.fx += fs * ex;
    acc.fy += fs * ey;
    acc.fz += fs * ez;
  }
  if (d2 < pc.rcc2) {
    const float wq = fmaxf(1.f - r * pc.inv_rcc, 0.f);
    const float wdc = pc.sc_exp == 2.f ? wq * wq : powu(wq, pc.sc_exp);
    for (int sp = 0; sp < pc.n_species; ++sp) {
      const float kap = pc.kappa[(sp * pc.n_types + ti) * pc.n_types + tj];
      float q = 0.f;
      if (pc.terms & TDPD_TERM_FLUX_FICK) q -= kap * wdc * (ci[sp] - cj[sp]);
      if (pc.ms_rho > 0.f && (pc.terms & TDPD_TERM_FLUX_RANDOM)) {
        const float eps = __builtin_amdgcn_sqrtf(pc.ms_rho * kap * fmaxf(ci[sp] + cj[sp], 0.f));
        float z;
        if (sp == 0) {
          z = gauss(w.c, w.d);
        } else {
          const u32x4 w2 = philox10(k, lo, hi, B.ctr3 | uint32_t((sp + 1) >> 1), B.seed_lo,
                                    B.seed_hi);
          z = (sp & 1) ? gauss(w2.a, w2.b) : gauss(w2.c, w2.d);
        }
        if (gi > gj) z = -z;  // zeta_ij = -zeta_ji
        q += eps * powu(wq, pc.sc_half) * pc.isdt * z;
      }
      acc.q[sp] += q;
    }
  }
}


// Visit every candidate j of a home particle at (xi, yi, zi) in local cell
// (cx, cy, cz): fn(j, dx, dy, dz, d2, lift) with the FP32 displacement of
// the pair rule (lift: 0 none, 1 the home, 2 the candidate is taken in the
// sheared image above; the lifted particle's x velocity gains le.u).  In a
// sheared box a neighbour row across the y boundary is displaced by delta:
// its candidates come from the min(4, n_x) cells around x -/+ delta.
template <class Fn>
__device__ __forceinline__ void for_candidates(const BoxDev &B, const LeOff &le, const State &s,
                                               const uint32_t *__restrict__ cell_start, int cx,
                                               int cy, int cz, float xi, float yi, float zi,
                                               Fn &&fn) {
  const int nx = B.nc[0], ny = B.nc[1], nz = B.nc[2];
  for (int dz = -1; dz <= 1; ++dz) {
    int qz = cz + dz;
    float sz = 0.f;
    if (qz < 0) { qz += nz; sz = -B.L[2]; }
    else if (qz >= nz) { qz -= nz; sz = B.L[2]; }
    for (int dy = -1; dy <= 1; ++dy) {
      int qy = cy + dy;
      float sy = 0.f;
      if (qy < 0) { qy += ny; sy = -B.L[1]; }
      else if (qy >= ny) { qy -= ny; sy = B.L[1]; }
      if (B.shear != 0.f && sy != 0.f) {
        const int lift = sy > 0.f ? 2 : 1;  // candidate above the top, or home below the bottom
        const float cshift = (lift == 2 ? -le.delta : le.delta) * B.inv_h[0];
        const int clo = int(floorf(float(cx) + cshift)) - 1;
        const int nw = nx < 4 ? nx : 4;
        for (int t = 0; t < nw; ++t) {
          const int qx = ((clo + t) % nx + nx) % nx;
          const uint32_t c = B.cell_base + uint32_t((qz * ny + qy) * nx + qx);
          for (uint32_t j = cell_start[c]; j < cell_start[c + 1]; ++j) {
            const float xj = s.x[j], yj = s.y[j];
            float dx, dy2;
            if (lift == 2) {
              dx = __fsub_rn(le_lift_x(xj, xi, le.delta, B.L[0]), xi);
              dy2 = __fsub_rn(__fadd_rn(yj, B.L[1]), yi);
            } else {
              dx = __fsub_rn(xj, le_lift_x(xi, xj, le.delta, B.L[0]));
              dy2 = __fsub_rn(yj, __fadd_rn(yi, B.L[1]));
            }
            const float dz2 = disp(s.z[j], sz, zi);
            fn(j, dx, dy2, dz2, dist2(dx, dy2, dz2), lift);
          }
        }
        continue;
      }
      for (int dx = -1; dx <= 1; ++dx) {
        int qx = cx + dx;
        float sx = 0.f;
        if (qx < 0) { qx += nx; sx = -B.L[0]; }
        else if (qx >= nx) { qx -= nx; sx = B.L[0]; }
        const uint32_t c = B.cell_base + uint32_t((qz * ny + qy) * nx + qx);
        for (uint32_t j = cell_start[c]; j < cell_start[c + 1]; ++j) {
          const float ddx = disp(s.x[j], sx, xi);
          const float ddy = disp(s.y[j], sy, yi);
          const float ddz = disp(s.z[j], sz, zi);
          fn(j, ddx, ddy, ddz, dist2(ddx, ddy, ddz), 0);
        }
      }
    }
  }
}

// ------------------------------------------------------------ simple kernel
// One thread per home particle (sorted order), scanning the 27 neighbour
// cells of its own cell in global memory.
__global__ void __launch_bounds__(256) k_pair_simple(PairConst pc,
                                                     const BoxDev *__restrict__ boxes, State s,
                                                     const uint32_t *__restrict__ cell_keys,
                                                     const uint32_t *__restrict__ cell_start,
                                                     int64_t n, const uint32_t *__restrict__ kdev,
                                                     float *__restrict__ F, float *__restrict__ Q,
                                                     unsigned long long *nzero, uint32_t *err) {
  const uint32_t k = *kdev;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int S = pc.n_species;
  const uint32_t infoi = s.info[i];
  const BoxDev &B = boxes[info_box(infoi)];
  const uint32_t key = cell_keys[i] - B.cell_base;
  const int cx = int(key % uint32_t(B.nc[0]));
  const int cy = int((key / uint32_t(B.nc[0])) % uint32_t(B.nc[1]));
  const int cz = int(key / uint32_t(B.nc[0] * B.nc[1]));
  PairAcc acc;
  acc.fx = acc.fy = acc.fz = 0.f;
  for (int sp = 0; sp < kMaxS; ++sp) acc.q[sp] = 0.f;
  if (!info_frozen(infoi)) {
    const float xi = s.x[i], yi = s.y[i], zi = s.z[i];
    const float vxi = s.vx[i], vyi = s.vy[i], vzi = s.vz[i];
    float ci[kMaxS], cj[kMaxS];
    for (int sp = 0; sp < S; ++sp) ci[sp] = s.C[sp * n + i];
    const uint32_t gi = s.gid[i] - B.gid_base;
    const int ti = info_type(infoi), bi = info_body(infoi);
    const LeOff le = le_offsets(B, k, pc.dt);
    unsigned zero = 0;
    for_candidates(B, le, s, cell_start, cx, cy, cz, xi, yi, zi,
                   [&](uint32_t j, float ddx, float ddy, float ddz, float d2, int lift) {
      if (d2 == 0.f) {
        if (j != uint32_t(i)) ++zero;
        return;
      }
      if (!(d2 < pc.rmax2)) return;
      const uint32_t infoj = s.info[j];
      const int bj = info_body(infoj);
      for (int sp = 0; sp < S; ++sp) cj[sp] = s.C[sp * n + j];
      const float vxh = lift == 1 ? __fadd_rn(vxi, le.u) : vxi;
      const float vxj = lift == 2 ? __fadd_rn(s.vx[j], le.u) : s.vx[j];
      pair_term(pc, B, ddx, ddy, ddz, d2, vxh, vyi, vzi, vxj, s.vy[j], s.vz[j], ci, cj, ti,
                info_type(infoj), bi >= 0 && bi == bj, gi, s.gid[j] - B.gid_base, k, acc);
    });
    if (zero) atomicAdd(nzero, (unsigned long long)zero);
    if (pc.has_source)
      for (int sp = 0; sp < S; ++sp) acc.q[sp] += source_term(pc, sp, ti, ci[sp]);
    if (pc.terms & TDPD_TERM_BODY_FORCE) {
      acc.fx += pc.body_force[0];
      acc.fy += pc.body_force[1];
      acc.fz += pc.body_force[2];
    }
    if (!(isfinite(acc.fx) && isfinite(acc.fy) && isfinite(acc.fz))) atomicOr(err, kErrNonfinite);
  }
  F[3 * i] = acc.fx;
  F[3 * i + 1] = acc.fy;
  F[3 * i + 2] = acc.fz;
  for (int sp = 0; sp < S; ++sp) Q[S * i + sp] = acc.q[sp];
}

void launch_pair_simple(const PairConst &pc, const BoxDev *boxes, State s,
                        const uint32_t *cell_keys, const uint32_t *cell_start, int64_t n,
                        const uint32_t *kdev, float *F, float *Q, unsigned long long *nzero,
                        uint32_t *err, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pair_simple, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, pc, boxes, s,
                     cell_keys, cell_start, n, kdev, F, Q, nzero, err);
}

// ------------------------------------------------------------ pair listing
__global__ void __launch_bounds__(256) k_pair_emit(PairConst pc, const BoxDev *__restrict__ boxes,
                                                   State s,
                                                   const uint32_t *__restrict__ cell_keys,
                                                   const uint32_t *__restrict__ cell_start,
                                                   int64_t n, float rcut2, uint32_t k, int32_t *out,
                                                   int64_t cap, unsigned long long *count) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float xi = s.x[i], yi = s.y[i], zi = s.z[i];
  const uint32_t gi = s.gid[i];
  const BoxDev &B = boxes[info_box(s.info[i])];
  const uint32_t key = cell_keys[i] - B.cell_base;
  const int cx = int(key % uint32_t(B.nc[0]));
  const int cy = int((key / uint32_t(B.nc[0])) % uint32_t(B.nc[1]));
  const int cz = int(key / uint32_t(B.nc[0] * B.nc[1]));
  const LeOff le = le_offsets(B, k, pc.dt);
  for_candidates(B, le, s, cell_start, cx, cy, cz, xi, yi, zi,
                 [&](uint32_t j, float, float, float, float d2, int) {
    const uint32_t gj = s.gid[j];
    if (gj <= gi) return;
    if (d2 > 0.f && d2 < rcut2) {
      const unsigned long long pos = atomicAdd(count, 1ull);
      if (int64_t(pos) < cap) {
        out[2 * pos] = int32_t(gi);
        out[2 * pos + 1] = int32_t(gj);
      }
    }
  });
}

void launch_pair_emit(const PairConst &pc, const BoxDev *boxes, State s,
                      const uint32_t *cell_keys, const uint32_t *cell_start, int64_t n,
                      float rcut2, uint32_t k, int32_t *out, int64_t cap,
                      unsigned long long *count, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pair_emit, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, pc, boxes, s,
                     cell_keys, cell_start, n, rcut2, k, out, cap, count);
}

}  // namespace tdpd
