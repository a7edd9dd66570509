// kernels_surrogate.hip -- the membrane surrogate: per-vertex 1-ring
// features, a bfloat16 MFMA matrix product with the network's epilogues
// (bias, SiLU, SiLU derivative), the loss gradient, column sums, Adam, and
// the kernels that apply the network's forces and compare them with the
// plain bending + local-area forces (Eqs. 17 and 19).
//
// Feature reading (the paper has no learned part): ring = neighbours in
// counter-clockwise order seen from outside starting at the smallest mesh
// index; frame rows e1 (ring start projected on the tangent plane), e2 =
// n x e1, n (normalised sum of consecutive ring cross products); inputs =
// local coordinates / ell of up to six ring vectors, then c_dev (A - A0)/A0
// and c_dev (V - V0)/V0 of the cell; only degree-5 and degree-6 vertices
// may use the network.
#include "launch.h"

namespace tdpd {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kGemmTile = 64;   // C tile is 64 x 64, four wavefronts of 32 x 32
constexpr int kGemmK = 16;      // k-step of v_mfma_f32_16x16x16_bf16
constexpr int kGemmPad = 4;     // LDS row padding (in bf16) against bank conflicts

// round to nearest even bfloat16 (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t b = __builtin_bit_cast(uint32_t, f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return uint16_t(b >> 16);
}

// SiLU z sigma(z) with the hardware exponential and reciprocal (a few ulps,
// far inside the bfloat16 rounding that follows)
__device__ __forceinline__ float silu_f(float z) {
  return z * __builtin_amdgcn_rcpf(1.f + __expf(-z));
}

// order this wavefront's LDS writes before its later LDS reads (other lanes)
__device__ __forceinline__ void wave_barrier_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ float silu_grad_f(float z) {
  const float sg = 1.f / (1.f + __expf(-z));
  return sg * (1.f + z * (1.f - sg));
}

// C(i, j) = sum_p A(i, p) B(p, j) with A(i, p) = A[i sa_i + p sa_p] and
// B(p, j) = B[p sb_p + j sb_j], both rounded to bfloat16 on load, FP32
// accumulation on the matrix cores, then the epilogue.
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  __shared__ uint16_t As[kGemmTile][kGemmK + kGemmPad];
  __shared__ uint16_t Bt[kGemmTile][kGemmK + kGemmPad];  // B transposed: [j][p]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t i0 = int64_t(blockIdx.x) * kGemmTile, j0 = int64_t(blockIdx.y) * kGemmTile;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int64_t p0 = 0; p0 < g.K; p0 += kGemmK) {
    // 64 x 16 elements of each operand, four per thread
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int r = e / kGemmK, c = e % kGemmK;  // A: row r of the tile, k offset c
      const int64_t i = i0 + r, p = p0 + c;
      const float va = (i < g.M && p < g.K) ? g.A[i * g.sa_i + p * g.sa_p] : 0.f;
      As[r][c] = to_bf16(va);
      const int64_t j = j0 + r;
      const float vb = (j < g.N && p < g.K) ? g.B[p * g.sb_p + j * g.sb_j] : 0.f;
      Bt[r][c] = to_bf16(vb);
    }
    __syncthreads();
    const int kq = 4 * (lane >> 4), rr = lane & 15;
    v4s a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[t][q] = short(As[wi + 16 * t + rr][kq + q]);
        b[t][q] = short(Bt[wj + 16 * t + rr][kq + q]);
      }
    }
#pragma unroll
    for (int ta = 0; ta < 2; ++ta)
#pragma unroll
      for (int tb = 0; tb < 2; ++tb)
        acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
    __syncthreads();
  }
  // lane holds C[4 (lane / 16) + q][lane % 16] of each 16 x 16 tile
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t i = i0 + wi + 16 * ta + 4 * (lane >> 4) + q;
        const int64_t j = j0 + wj + 16 * tb + (lane & 15);
        if (i >= g.M || j >= g.N) continue;
        float v = acc[ta][tb][q];
        if (g.bias) v += g.bias[j];
        switch (g.epi) {
          case kEpiStore:
            g.C[i * g.ldc + j] = v;
            break;
          case kEpiSilu:  // pre-activation to C (if given), activation to H
            if (g.C) g.C[i * g.ldc + j] = v;
            g.H[i * g.ldc + j] = silu_f(v);
            break;
          case kEpiSiluGrad:  // backward through the SiLU of pre-activation Z
            g.C[i * g.ldc + j] = v * silu_grad_f(g.Z[i * g.ldc + j]);
            break;
        }
      }
}

void launch_gemm_bf16(const GemmArgs &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  const dim3 grid(unsigned((g.M + kGemmTile - 1) / kGemmTile),
                  unsigned((g.N + kGemmTile - 1) / kGemmTile));
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, st, g);
}

// dY = 2 (Y - T / s) / (3 n) and per-block FP64 partial sums of (Y - T / s)^2
__global__ void __launch_bounds__(256) k_loss_grad(const float *__restrict__ Y,
                                                   const float *__restrict__ T, int64_t n,
                                                   float inv_scale, float *__restrict__ dY,
                                                   double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  double sq = 0.0;
  if (e < 3 * n) {
    const float d = Y[e] - T[e] * inv_scale;
    dY[e] = 2.f * d / float(3 * n);
    sq = double(d) * double(d);
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[j] = sum_m D[m ld + j], one workgroup per column, fixed order
__global__ void __launch_bounds__(256) k_colsum(const float *__restrict__ D, int64_t m, int ld,
                                                float *__restrict__ out) {
  __shared__ float red[256];
  const int j = blockIdx.x;
  float s = 0.f;
  for (int64_t r = threadIdx.x; r < m; r += 256) s += D[r * ld + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

void launch_loss_grad(const float *Y, const float *T, int64_t n, float inv_scale, float *dY,
                      double *part, hipStream_t st) {
  const unsigned nb = unsigned((3 * n + 255) / 256);
  hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, st, Y, T, n, inv_scale, dY, part);
}

int64_t loss_grad_blocks(int64_t n) { return (3 * n + 255) / 256; }

void launch_colsum(const float *D, int64_t m, int ld, int ncol, float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3(unsigned(ncol)), dim3(256), 0, st, D, m, ld, out);
}

// Adam (Kingma & Ba) with bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t
__global__ void __launch_bounds__(256) k_adam(float *__restrict__ w, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float bc1, float bc2) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

void launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                 float b2, float eps, float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, w, g, m, v, n, lr,
                     b1, b2, eps, bc1, bc2);
}

// ------------------------------------------------------------ features
__device__ __forceinline__ float3 f3sub(float3 a, float3 b) {
  return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ float3 f3cross(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float f3dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

__global__ void __launch_bounds__(256) k_surr_features(SurrDev sd, const BoxDev *__restrict__ boxes,
                                                       const MeshDev *__restrict__ meshes, State s,
                                                       const uint32_t *__restrict__ slot_of_gid,
                                                       const double *__restrict__ av,
                                                       int64_t nvert,
                                                       const uint32_t *__restrict__ kdev, int kofs,
                                                       float dt) {
  const int64_t vg = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (vg >= nvert) return;
  const int r = sd.vcell[vg];
  const MeshDev &M = meshes[sd.rbc_mesh[r]];
  const BoxDev &B = boxes[sd.rbc_box[r]];
  const int v = int(vg - sd.rbc_voff[r]);
  const int64_t g0 = sd.rbc_first[r];
  auto pos = [&](int u) {
    const uint32_t q = slot_of_gid[g0 + u];
    return make_float3(s.x[q], s.y[q], s.z[q]);
  };
  const float3 pv = pos(v);
  const int r0 = M.ring_off[v], deg = M.ring_off[v + 1] - r0;
  float3 u[kRingMax];
  const LeOff le = le_offsets(B, *kdev + uint32_t(kofs), dt);
  for (int kk = 0; kk < deg && kk < kRingMax; ++kk) u[kk] = le_rel(B, pos(M.ring[r0 + kk]), pv, le.delta, nullptr);
  const int dg = deg < kRingMax ? deg : kRingMax;
  float3 nn = make_float3(0.f, 0.f, 0.f);
  for (int kk = 0; kk < dg; ++kk) {
    const float3 c = f3cross(u[kk], u[(kk + 1) % dg]);
    nn.x += c.x;
    nn.y += c.y;
    nn.z += c.z;
  }
  const float inn = 1.f / sqrtf(f3dot(nn, nn));
  const float3 n = make_float3(nn.x * inn, nn.y * inn, nn.z * inn);
  const float un = f3dot(u[0], n);
  float3 t = make_float3(u[0].x - un * n.x, u[0].y - un * n.y, u[0].z - un * n.z);
  const float it = 1.f / sqrtf(f3dot(t, t));
  const float3 e1 = make_float3(t.x * it, t.y * it, t.z * it);
  const float3 e2 = f3cross(n, e1);
  float *R = sd.R + 9 * vg;
  R[0] = e1.x; R[1] = e1.y; R[2] = e1.z;
  R[3] = e2.x; R[4] = e2.y; R[5] = e2.z;
  R[6] = n.x;  R[7] = n.y;  R[8] = n.z;
  const bool ok = deg == 5 || deg == 6;
  sd.ok[vg] = ok ? 1 : 0;
  float *X = sd.X + kSurrIn * vg;
  const float il = 1.f / M.ell;
  for (int kk = 0; kk < 6; ++kk) {
    float a = 0.f, b = 0.f, c = 0.f;
    if (ok && kk < deg) {
      a = f3dot(u[kk], e1) * il;
      b = f3dot(u[kk], e2) * il;
      c = f3dot(u[kk], n) * il;
    }
    X[3 * kk] = a;
    X[3 * kk + 1] = b;
    X[3 * kk + 2] = c;
  }
  // lagged totals of the cell (zero before the first evaluation)
  const double A = av[2 * r], V = av[2 * r + 1];
  X[18] = A > 0.0 ? float(kSurrDev * (A - M.A0) / M.A0) : 0.f;
  X[19] = A > 0.0 ? float(kSurrDev * (V - M.V0) / M.V0) : 0.f;
}

void launch_surr_features(const SurrDev &sd, const BoxDev *boxes, const MeshDev *meshes, State s,
                          const uint32_t *slot_of_gid, const double *av, int64_t nvert,
                          const uint32_t *kdev, float dt, int kofs, hipStream_t st) {
  if (nvert <= 0) return;
  hipLaunchKernelGGL(k_surr_features, dim3(unsigned((nvert + 255) / 256)), dim3(256), 0, st, sd,
                     boxes, meshes, s, slot_of_gid, av, nvert, kdev, kofs, dt);
}

// Fs = s_F R^T y (global frame) for every vertex
__global__ void __launch_bounds__(256) k_surr_apply(SurrDev sd, int64_t nvert) {
  const int64_t vg = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (vg >= nvert) return;
  const float *R = sd.R + 9 * vg, *y = sd.Y + 3 * vg;
  for (int j = 0; j < 3; ++j)
    sd.Fs[3 * vg + j] = sd.s_F * (R[j] * y[0] + R[3 + j] * y[1] + R[6 + j] * y[2]);
}

void launch_surr_apply(const SurrDev &sd, int64_t nvert, hipStream_t st) {
  if (nvert <= 0) return;
  hipLaunchKernelGGL(k_surr_apply, dim3(unsigned((nvert + 255) / 256)), dim3(256), 0, st, sd,
                     nvert);
}

// T = R Fp: plain forces in the local frame (training targets)
__global__ void __launch_bounds__(256) k_surr_targets(SurrDev sd, float *__restrict__ T,
                                                      int64_t nvert) {
  const int64_t vg = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (vg >= nvert) return;
  const float *R = sd.R + 9 * vg, *f = sd.Fp + 3 * vg;
  for (int i = 0; i < 3; ++i) T[3 * vg + i] = R[3 * i] * f[0] + R[3 * i + 1] * f[1] + R[3 * i + 2] * f[2];
}

void launch_surr_targets(const SurrDev &sd, float *T, int64_t nvert, hipStream_t st) {
  if (nvert <= 0) return;
  hipLaunchKernelGGL(k_surr_targets, dim3(unsigned((nvert + 255) / 256)), dim3(256), 0, st, sd, T,
                     nvert);
}

// Fallback check, one workgroup per cell, on steps k with k % every == 0:
// err_v = |Fs - Fp| / rms over the cell of |Fp|; a vertex uses the network
// until the next check iff it may (degree 5 or 6) and err_v <= tol.
// stats[r] = (vertices on the network, max err, sum err) of the last check.
__global__ void __launch_bounds__(256) k_surr_check(SurrDev sd, const uint32_t *__restrict__ kdev,
                                                    int every) {
  __shared__ float red[256];
  const uint32_t k = *kdev;
  if (every > 0 && (k % uint32_t(every)) != 0u) return;
  const int r = blockIdx.x, tid = threadIdx.x;
  const int64_t v0 = sd.rbc_voff[r], v1 = sd.rbc_voff[r + 1];
  float s2 = 0.f;
  for (int64_t v = v0 + tid; v < v1; v += 256) {
    const float *f = sd.Fp + 3 * v;
    s2 += f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
  }
  red[tid] = s2;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const float rms = sqrtf(red[0] / float(v1 - v0));
  const float inv = rms > 0.f ? 1.f / rms : 0.f;
  __syncthreads();
  float cnt = 0.f, mx = 0.f, sm = 0.f;
  for (int64_t v = v0 + tid; v < v1; v += 256) {
    const float *f = sd.Fp + 3 * v, *g = sd.Fs + 3 * v;
    const float dx = g[0] - f[0], dy = g[1] - f[1], dz = g[2] - f[2];
    const float e = sqrtf(dx * dx + dy * dy + dz * dz) * inv;
    const bool use = sd.ok[v] && e <= sd.tol;
    sd.flag[v] = use ? 1 : 0;
    cnt += use ? 1.f : 0.f;
    if (sd.ok[v]) {
      mx = fmaxf(mx, e);
      sm += e;
    }
  }
  float vals[3] = {cnt, mx, sm};
  for (int q = 0; q < 3; ++q) {
    red[tid] = vals[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) red[tid] = q == 1 ? fmaxf(red[tid], red[tid + off]) : red[tid] + red[tid + off];
      __syncthreads();
    }
    if (tid == 0) sd.stats[3 * r + q] = red[0];
    __syncthreads();
  }
}

void launch_surr_check(const SurrDev &sd, int nrbc, const uint32_t *kdev, int every,
                       hipStream_t st) {
  if (nrbc <= 0) return;
  hipLaunchKernelGGL(k_surr_check, dim3(unsigned(nrbc)), dim3(256), 0, st, sd, kdev, every);
}

}  // namespace tdpd

namespace tdpd {

// out[0] += sum of parts in fixed order (one workgroup)
__global__ void __launch_bounds__(256) k_sum_parts(const double *__restrict__ part, int64_t n,
                                                   double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

void launch_sum_parts(const double *part, int64_t n, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, st, part, n, out);
}

// ------------------------------------------------- fused forward pass
// The whole network in one kernel: a workgroup keeps the four weight
// matrices in LDS as bfloat16 (loaded once) and walks tiles of 128 rows; each
// wavefront owns 16 rows, so its activations never leave its own rows of the
// LDS tile (no barrier between layers).  Layers run on gfx950's
// v_mfma_f32_16x16x32_bf16 (16 x 32 A block, 32 x 16 B block, FP32
// accumulation): lane l holds A[l % 16][8 (l / 16) + 0..7] and
// B[8 (l / 16) + 0..7][l % 16], and receives D[4 (l / 16) + 0..3][l % 16].
// The rounding points are those of the layer-by-layer path: inputs, weights
// and hidden activations to bfloat16 where they enter a product, bias and
// SiLU in FP32.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kFusedRows = 128;                 // rows per tile (8 wavefronts x 16)
constexpr int kFusedThreads = 512;
constexpr int kK1 = 32;                         // first layer's K (20 inputs, padded)
constexpr int kS1 = kK1 + 8;                    // LDS row strides in bfloat16 (16-byte
constexpr int kSH = kSurrHid + 8;               // aligned, offset against bank conflicts)
constexpr int kN4 = 16;                         // last layer's N (3 outputs, padded)

struct FusedShared {
  uint16_t w1[kSurrHid][kS1];
  uint16_t w2[kSurrHid][kSH];
  uint16_t w3[kSurrHid][kSH];
  uint16_t w4[kN4][kSH];
  float b1[kSurrHid], b2[kSurrHid], b3[kSurrHid], b4[kN4];
  uint16_t act[kFusedRows][kSH];
};

__device__ __forceinline__ v8bf lds_v8(const uint16_t *p) {
  return __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4 *>(p));
}

// acc[c] += A (16 rows of this wave, K columns of act) x W^T (column tiles c)
template <int K, int NT, int SA, int SW>
__device__ __forceinline__ void fused_layer(const uint16_t (*act)[kSH], const uint16_t *w, int r0,
                                            int lane, v4f (&acc)[NT]) {
  const int rr = lane & 15, kq = 8 * (lane >> 4);
#pragma unroll
  for (int c = 0; c < NT; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    const v8bf a = lds_v8(&act[r0 + rr][k0 + kq]);
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      const v8bf b = lds_v8(w + (16 * c + rr) * SW + k0 + kq);
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
  }
}

// bias + SiLU of a hidden layer, rounded to bfloat16 into the wave's rows;
// with hdbg the FP32 activations (before that rounding) also go to
// hdbg[row][128] (rows past n are not written)
__device__ __forceinline__ void fused_store_hidden(uint16_t (*act)[kSH], const float *bias,
                                                   int r0, int lane, const v4f (&acc)[8],
                                                   float *hdbg, int64_t row0, int64_t n) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int col = 16 * c + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 4 * (lane >> 4) + q;
      const float h = silu_f(acc[c][q] + bias[col]);
      act[r0 + r][col] = to_bf16(h);
      if (hdbg && row0 + r < n) hdbg[(row0 + r) * kSurrHid + col] = h;
    }
  }
}

__global__ void __launch_bounds__(kFusedThreads) k_mlp_fused(const float *__restrict__ params,
                                                             const float *__restrict__ X, int64_t n,
                                                             float *__restrict__ Y,
                                                             float *__restrict__ hdbg) {
  __shared__ __align__(16) FusedShared sh;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const MlpLayout L;
  // weights and biases, once per workgroup (padding zero)
  for (int e = tid; e < kSurrHid * kS1; e += kFusedThreads) {
    const int o = e / kS1, k = e % kS1;
    sh.w1[o][k] = k < kSurrIn ? to_bf16(params[L.W1 + o * kSurrIn + k]) : uint16_t(0);
  }
  // (four consecutive weights per thread: one 16-byte load, one 8-byte store)
  for (int e = tid; e < kSurrHid * (kSH / 4); e += kFusedThreads) {
    const int o = e / (kSH / 4), k = 4 * (e % (kSH / 4));
    uint2 v2 = make_uint2(0u, 0u), v3 = make_uint2(0u, 0u);
    if (k < kSurrHid) {
      const float4 a = *reinterpret_cast<const float4 *>(params + L.W2 + o * kSurrHid + k);
      const float4 b = *reinterpret_cast<const float4 *>(params + L.W3 + o * kSurrHid + k);
      v2 = make_uint2(uint32_t(to_bf16(a.x)) | (uint32_t(to_bf16(a.y)) << 16),
                      uint32_t(to_bf16(a.z)) | (uint32_t(to_bf16(a.w)) << 16));
      v3 = make_uint2(uint32_t(to_bf16(b.x)) | (uint32_t(to_bf16(b.y)) << 16),
                      uint32_t(to_bf16(b.z)) | (uint32_t(to_bf16(b.w)) << 16));
    }
    *reinterpret_cast<uint2 *>(&sh.w2[o][k]) = v2;
    *reinterpret_cast<uint2 *>(&sh.w3[o][k]) = v3;
  }
  for (int e = tid; e < kN4 * kSH; e += kFusedThreads) {
    const int o = e / kSH, k = e % kSH;
    sh.w4[o][k] = (o < kSurrOut && k < kSurrHid) ? to_bf16(params[L.W4 + o * kSurrHid + k]) : uint16_t(0);
  }
  for (int e = tid; e < kSurrHid; e += kFusedThreads) {
    sh.b1[e] = params[L.b1 + e];
    sh.b2[e] = params[L.b2 + e];
    sh.b3[e] = params[L.b3 + e];
  }
  if (tid < kN4) sh.b4[tid] = tid < kSurrOut ? params[L.b4 + tid] : 0.f;
  __syncthreads();
  const int r0 = 16 * w;  // this wave's rows of the tile
  const int64_t ntiles = (n + kFusedRows - 1) / kFusedRows;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * kFusedRows + r0;
    // inputs of the wave's 16 rows, bfloat16, K padded to 32 (all loads
    // issued before the first is used)
    float xv[16 * kK1 / 64];
#pragma unroll
    for (int u = 0; u < 16 * kK1 / 64; ++u) {
      const int e = lane + 64 * u, r = e / kK1, k = e % kK1;
      const int64_t i = row0 + r;
      xv[u] = (k < kSurrIn && i < n) ? X[i * kSurrIn + k] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 16 * kK1 / 64; ++u) {
      const int e = lane + 64 * u;
      sh.act[r0 + e / kK1][e % kK1] = to_bf16(xv[u]);
    }
    wave_barrier_lds();
    v4f acc[8];
    fused_layer<kK1, 8, kSH, kS1>(sh.act, &sh.w1[0][0], r0, lane, acc);
    wave_barrier_lds();
    fused_store_hidden(sh.act, sh.b1, r0, lane, acc, hdbg ? hdbg + 0 * n * kSurrHid : nullptr,
                       row0, n);
    wave_barrier_lds();
    fused_layer<kSurrHid, 8, kSH, kSH>(sh.act, &sh.w2[0][0], r0, lane, acc);
    wave_barrier_lds();
    fused_store_hidden(sh.act, sh.b2, r0, lane, acc, hdbg ? hdbg + 1 * n * kSurrHid : nullptr,
                       row0, n);
    wave_barrier_lds();
    fused_layer<kSurrHid, 8, kSH, kSH>(sh.act, &sh.w3[0][0], r0, lane, acc);
    wave_barrier_lds();
    fused_store_hidden(sh.act, sh.b3, r0, lane, acc, hdbg ? hdbg + 2 * n * kSurrHid : nullptr,
                       row0, n);
    wave_barrier_lds();
    v4f o[1];
    fused_layer<kSurrHid, 1, kSH, kSH>(sh.act, &sh.w4[0][0], r0, lane, o);
    const int col = lane & 15;
    if (col < kSurrOut) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t i = row0 + 4 * (lane >> 4) + q;
        if (i < n) Y[i * kSurrOut + col] = o[0][q] + sh.b4[col];
      }
    }
    wave_barrier_lds();  // the next tile's inputs overwrite these rows
  }
}

void mlp_forward(const float *params, const float *X, int64_t n, float *Y, hipStream_t st,
                 float *hdbg) {
  if (n <= 0) return;
  const int64_t ntiles = (n + kFusedRows - 1) / kFusedRows;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const unsigned grid = unsigned(ntiles < ncu ? ntiles : ncu);
  hipLaunchKernelGGL(k_mlp_fused, dim3(grid), dim3(kFusedThreads), 0, st, params, X, n, Y, hdbg);
}

// The same network layer by layer (four matrix-product launches with the
// hidden activations in HBM), used by training.
void mlp_forward_layers(const float *params, const float *X, int64_t n, float *Ha, float *Hb,
                        float *Y, hipStream_t st) {
  const MlpLayout L;
  GemmArgs g{};
  g.A = X; g.sa_i = kSurrIn; g.sa_p = 1;
  g.B = params + L.W1; g.sb_p = 1; g.sb_j = kSurrIn;
  g.C = nullptr; g.ldc = kSurrHid; g.M = n; g.N = kSurrHid; g.K = kSurrIn;
  g.bias = params + L.b1; g.epi = kEpiSilu; g.H = Ha;
  launch_gemm_bf16(g, st);
  g.A = Ha; g.sa_i = kSurrHid; g.B = params + L.W2; g.sb_j = kSurrHid; g.K = kSurrHid;
  g.bias = params + L.b2; g.H = Hb;
  launch_gemm_bf16(g, st);
  g.A = Hb; g.B = params + L.W3; g.bias = params + L.b3; g.H = Ha;
  launch_gemm_bf16(g, st);
  g.A = Ha; g.B = params + L.W4; g.C = Y; g.ldc = kSurrOut; g.N = kSurrOut;
  g.bias = params + L.b4; g.epi = kEpiStore; g.H = nullptr;
  launch_gemm_bf16(g, st);
}

}  // namespace tdpd
