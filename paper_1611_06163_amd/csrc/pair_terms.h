// pair_terms.h -- per-pair tDPD force (Eqs. 3-6) and flux (Eqs. 8-10) terms
// used by every pair kernel.
#pragma once

#include "tdpd_device.h"

namespace tdpd {

// Force of pair (i,j) on i at FP32 displacement d (of x_j seen from x_i)
// with d2 = |d|^2, 0 < d2 < rc2, i and j not in the same cell body.
// e_ij = -d/r points from j to i; v_ij = v_i - v_j; the noise xi is the
// Box-Muller normal of Philox stream 0, words (0,1), for the unordered pair
// of box-local gids at step k under the box's key, so F_ij = -F_ji exactly.
__device__ __forceinline__ float3 force_term(const PairConst &pc, const BoxDev &B, float dx,
                                             float dy, float dz,
                                             float d2, float vxi, float vyi, float vzi, float vxj,
                                             float vyj, float vzj, int ti, int tj, uint32_t gi,
                                             uint32_t gj, uint32_t k) {
  const float rinv = __builtin_amdgcn_rsqf(d2);
  const float r = d2 * rinv;
  const float ex = -dx * rinv, ey = -dy * rinv, ez = -dz * rinv;
  const int tt = ti * pc.n_types + tj;
  const float wc = fmaxf(1.f - r * pc.inv_rc, 0.f);
  float fs = 0.f;
  if (pc.terms & TDPD_TERM_CONSERVATIVE) fs += pc.alpha[tt] * wc;
  const float wr = powu(wc, pc.s_half);
  if (pc.terms & TDPD_TERM_DISSIPATIVE) {
    const float ev = ex * (vxi - vxj) + ey * (vyi - vyj) + ez * (vzi - vzj);
    fs -= pc.gamma[tt] * wr * wr * ev;
  }
  if (pc.terms & TDPD_TERM_RANDOM) {
    const uint32_t lo = gi < gj ? gi : gj, hi = gi < gj ? gj : gi;
    const u32x4 w = philox10(k, lo, hi, B.ctr3, B.seed_lo, B.seed_hi);
    fs += pc.sigma[tt] * wr * gauss(w.a, w.b) * pc.isdt;
  }
  return make_float3(fs * ex, fs * ey, fs * ez);
}

// Fickian flux weight w_DC(r) for 0 < d2 < rcc2 (inside the cutoff 1 - r/rcc
// is at worst a rounding step below zero, which the square leaves harmless)
__device__ __forceinline__ float flux_weight(const PairConst &pc, float d2) {
  const float wq = 1.f - __builtin_amdgcn_sqrtf(d2) * pc.inv_rcc;
  return pc.sc_exp == 2.f ? wq * wq : powu(fmaxf(wq, 0.f), pc.sc_exp);
}

}  // namespace tdpd
