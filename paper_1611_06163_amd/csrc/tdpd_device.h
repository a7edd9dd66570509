// tdpd_device.h -- device-side data structures and inline math shared by the
// HIP kernels of the tDPD + RBC library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tdpd.h"

namespace tdpd {

constexpr int kMaxT = TDPD_MAX_TYPES;
constexpr int kMaxS = TDPD_MAX_SPECIES;

// Internal info word of a particle (the public flags word is converted at
// upload): type bits 0-2 | frozen bit 3 | box bits 4-13 | (body + 1) bits 14-31.
constexpr uint32_t kFrozen = 1u << 3;
constexpr int kMaxBoxes = 1024;
constexpr int kMaxBodies = (1 << 18) - 2;
__host__ __device__ inline int info_type(uint32_t w) { return int(w & 7u); }
__host__ __device__ inline bool info_frozen(uint32_t w) { return (w & kFrozen) != 0; }
__host__ __device__ inline int info_box(uint32_t w) { return int((w >> 4) & 1023u); }
__host__ __device__ inline int info_body(uint32_t w) { return int(w >> 14) - 1; }
__host__ __device__ inline uint32_t make_info(int type, bool frozen, int box, int body) {
  return uint32_t(type) | (frozen ? kFrozen : 0u) | (uint32_t(box) << 4) | (uint32_t(body + 1) << 14);
}

// Error bits written by kernels (sticky until the host reads them).
constexpr uint32_t kErrOverext = 1u;
constexpr uint32_t kErrNonfinite = 2u;

// One periodic box of a (possibly batched) system: geometry, its slice of
// the global cell list and of the gid range, and its noise key and counter
// word (the counter uses box-local gids, so a box behaves the same alone and
// in a batch).
struct BoxDev {
  float L[3], invL[3], inv_h[3];
  int nc[3];
  uint32_t cell_base, ncell;
  uint32_t gid_base;
  uint32_t seed_lo, seed_hi, ctr3;  // ctr3 = box_id << 8
  float shear;                      // Lees-Edwards shear rate, 0 = plain periodic
};

// Parameters shared by every box, passed by value.
struct PairConst {
  float rc, rcc, rc2, rcc2, rmax2;
  float inv_rc, inv_rcc;
  float s_half;       // w_R = w^(s/2)
  float sc_exp, sc_half;
  float isdt;         // 1/sqrt(dt)
  float dt, half_dt;
  float ms_rho;       // m_s^2 * rho
  int n_types, n_species;
  float alpha[kMaxT * kMaxT], gamma[kMaxT * kMaxT], sigma[kMaxT * kMaxT];
  float kappa[kMaxS * kMaxT * kMaxT];
  float body_force[3];
  int wall_axis;
  float wall_w;
  int terms;
  int n_boxes;
  // source term Q^S of Eq. (7): source - decay * C per [species * n_types + type]
  int has_source;
  float source[kMaxS * kMaxT], decay[kMaxS * kMaxT];
  float wall_radius;  // wall_axis 3: tube radius about (L_y/2, L_z/2)
};

// State planes of one particle ordering.
struct State {
  float *x, *y, *z, *vx, *vy, *vz;
  float *C;            // [S][N]
  uint32_t *gid, *info;
};

// Box owning global cell c (boxes hold ascending cell ranges).
__device__ __forceinline__ int box_of_cell(const BoxDev *boxes, int nbox, uint32_t c) {
  int lo = 0, hi = nbox - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (boxes[mid].cell_base <= c) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ Philox
// Philox-4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products whose high halves are mixed into the other counter words with
// the round key; the key advances by the Weyl constants between rounds.
struct u32x4 {
  uint32_t a, b, c, d;
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c0;
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c2;
    const uint32_t n0 = uint32_t(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = uint32_t(p0 >> 32) ^ c3 ^ k1;
    c1 = uint32_t(p1);
    c3 = uint32_t(p0);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// uniform in (0,1): (2*(bits>>9)+1) * 2^-24, exact in FP32
__device__ __forceinline__ float u01(uint32_t bits) {
  return float((bits >> 9) * 2u + 1u) * 5.9604644775390625e-8f;
}

// Box-Muller normal from two words.  v_log_f32 is log2; v_cos_f32 takes its
// argument in revolutions, so cos(2 pi u) is one instruction.
__device__ __forceinline__ float gauss(uint32_t w0, uint32_t w1) {
  const float u0 = u01(w0), u1 = u01(w1);
  const float r2 = -1.3862943611198906f * __builtin_amdgcn_logf(u0);  // -2 ln u0
  return __builtin_amdgcn_sqrtf(r2) * __builtin_amdgcn_cosf(u1);
}

// Both Box-Muller normals of a word pair: r cos(2 pi u1), r sin(2 pi u1).
__device__ __forceinline__ void gauss2(uint32_t w0, uint32_t w1, float &c, float &s) {
  const float u0 = u01(w0), u1 = u01(w1);
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
  c = r * __builtin_amdgcn_cosf(u1);
  s = r * __builtin_amdgcn_sinf(u1);
}

// ------------------------------------------------------------ predicate
// FP32 displacement component of x_j seen from x_i at periodic image shift
// s in {0, +L, -L} of x_j, rounded exactly as specified (no contraction).
// Across the boundary the coordinate nearer 0 is lifted by L, so both
// orientations of a pair round the same value and d_ji = -d_ij exactly.
__device__ __forceinline__ float disp(float xj, float s, float xi) {
  if (s > 0.f) return __fsub_rn(__fadd_rn(xj, s), xi);
  if (s < 0.f) return __fsub_rn(xj, __fadd_rn(xi, -s));
  return __fsub_rn(xj, xi);
}
__device__ __forceinline__ float dist2(float dx, float dy, float dz) {
  return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
}

// Q^S of Eq. (7) for a mobile particle of type t holding concentration c of
// species sp: the zero-order source less the first-order decay.
__device__ __forceinline__ float source_term(const PairConst &pc, int sp, int t, float c) {
  const int e = sp * pc.n_types + t;
  return __fmaf_rn(-pc.decay[e], c, pc.source[e]);
}

// w^e for w in [0,1]; zero at w <= 0
__device__ __forceinline__ float powu(float w, float e) {
  return w > 0.f ? __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(w)) : 0.f;
}

// x^e for x > 0 (any e); zero at x <= 0
__device__ __forceinline__ float powu_any(float x, float e) {
  return x > 0.f ? __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(x)) : 0.f;
}

__device__ __forceinline__ float wrap_coord(float x, float L) {
  if (x < 0.f) x += L;
  if (x >= L) x -= L;
  if (x >= L || x < 0.f) x = 0.f;
  return x;
}

__device__ __forceinline__ int cell_coord(float x, float inv_h, int n) {
  int c = int(x * inv_h);
  c = c < 0 ? 0 : c;
  return c >= n ? n - 1 : c;
}

__device__ __forceinline__ float min_image(float d, float L, float invL) {
  return d - L * rintf(d * invL);
}

// Lees-Edwards offsets of a sheared box at step counter k: the image above
// in y sits delta to the right and moves with +u in x,
//   u = fl32(shear L_y), delta = fl32(fmod(shear L_y * (k dt), L_x)),
// products in FP64 from the FP32 parameters.
struct LeOff {
  float delta, u;
};
__device__ __forceinline__ LeOff le_offsets(const BoxDev &B, uint32_t k, float dt) {
  LeOff o{0.f, 0.f};
  if (B.shear != 0.f) {
    const double a = double(B.shear) * double(B.L[1]);
    const double b = double(k) * double(dt);
    o.u = float(a);
    const float d = float(fmod(a * b, double(B.L[0])));
    o.delta = d >= B.L[0] ? 0.f : d;
  }
  return o;
}

// x of a particle lifted into the image above (y + L_y) of a sheared box,
// nearest to the other particle's x: fl(fl(x + delta) + m L_x) with m in
// {-2, .., 1} decided in FP32 from dx1 = fl(x_o - fl(x + delta)), the same
// sequence whichever particle of the pair evaluates it.
__device__ __forceinline__ float le_lift_x(float x, float xo, float delta, float Lx) {
  const float X1 = __fadd_rn(x, delta);
  const float dx1 = __fsub_rn(xo, X1);
  float m = 0.f;
  if (dx1 > 0.5f * Lx) m = 1.f;
  else if (dx1 < -0.5f * Lx) m = (__fadd_rn(dx1, Lx) < -0.5f * Lx) ? -2.f : -1.f;
  return __fadd_rn(X1, m * Lx);
}

// Nearest-image difference a - o of two coordinates in [0, L): the
// coordinate that moves by a box length is moved first, which is exact
// (Sterbenz: it lies in [L/2, L)), so only the final difference rounds.
__device__ __forceinline__ float near_diff(float a, float o, float L) {
  const float d = a - o;
  if (d > 0.5f * L) return (a - L) - o;
  if (d < -0.5f * L) return a - (o - L);
  return d;
}

// nearest-image difference a - o in a (possibly sheared) box; *ny gets -1
// when a was taken in the image below o (+1 above), which shifts a's x
// velocity by -u (+u)
__device__ __forceinline__ float3 le_rel(const BoxDev &B, float3 a, float3 o, float delta,
                                         int *ny) {
  int s = 0;
  float dx, dy;
  if (B.shear != 0.f) {
    dx = a.x - o.x;
    dy = a.y - o.y;
    if (dy > 0.5f * B.L[1]) {
      dy = (a.y - B.L[1]) - o.y;
      dx -= delta;
      s = -1;
    } else if (dy < -0.5f * B.L[1]) {
      dy = a.y - (o.y - B.L[1]);
      dx += delta;
      s = 1;
    }
    dx = min_image(dx, B.L[0], B.invL[0]);
  } else {
    dx = near_diff(a.x, o.x, B.L[0]);
    dy = near_diff(a.y, o.y, B.L[1]);
  }
  if (ny) *ny = s;
  return make_float3(dx, dy, near_diff(a.z, o.z, B.L[2]));
}

}  // namespace tdpd
