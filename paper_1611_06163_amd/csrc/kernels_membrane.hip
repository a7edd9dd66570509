// kernels_membrane.hip -- RBC membrane terms (Section 2.2) as two kernels:
//   k_rbc_gather  (one workgroup per cell): FP64 totals A^t and V^t of every
//                 cell (the paper's K-Gather) and its centroid update;
//   k_membrane    (one thread per vertex): every bonded term acting on the
//                 vertex -- WLC + POW springs, bond viscosity and noise,
//                 global/local area and volume forces (K-Apply), bending --
//                 gathered over the vertex's incident bonds, triangles and
//                 dihedrals, so no atomics and each triangle is recomputed
//                 by its three vertices (as the paper does, Section 3.3).
#include "launch.h"

namespace tdpd {

constexpr int kGatherThreads = 256;

__device__ __forceinline__ float3 load_pos(const State &s, uint32_t slot) {
  return make_float3(s.x[slot], s.y[slot], s.z[slot]);
}
__device__ __forceinline__ float3 rel(const MembraneConst &mc, float3 a, float3 o) {
  return make_float3(min_image(a.x - o.x, mc.L[0], mc.invL[0]),
                     min_image(a.y - o.y, mc.L[1], mc.invL[1]),
                     min_image(a.z - o.z, mc.L[2], mc.invL[2]));
}
__device__ __forceinline__ float3 sub(float3 a, float3 b) {
  return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ float3 crs(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dt3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

__global__ void __launch_bounds__(kGatherThreads) k_rbc_gather(
    MembraneConst mc, const MeshDev *__restrict__ meshes, const int32_t *__restrict__ rbc_mesh,
    const int64_t *__restrict__ rbc_first, State s, const uint32_t *__restrict__ slot_of_gid,
    double *__restrict__ av, double *__restrict__ centroid) {
  __shared__ double red[kGatherThreads];
  const int r = blockIdx.x;
  const MeshDev &M = meshes[rbc_mesh[r]];
  const int64_t g0 = rbc_first[r];
  const double c0x = centroid[3 * r], c0y = centroid[3 * r + 1], c0z = centroid[3 * r + 2];
  const float3 cf = make_float3(float(c0x), float(c0y), float(c0z));
  double acc[5] = {0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < M.ntri; t += kGatherThreads) {
    const float3 a = rel(mc, load_pos(s, slot_of_gid[g0 + M.tri[3 * t]]), cf);
    const float3 b = rel(mc, load_pos(s, slot_of_gid[g0 + M.tri[3 * t + 1]]), cf);
    const float3 c = rel(mc, load_pos(s, slot_of_gid[g0 + M.tri[3 * t + 2]]), cf);
    const float3 nn = crs(sub(b, a), sub(c, a));
    acc[0] += double(0.5f * sqrtf(dt3(nn, nn)));
    acc[1] += double(dt3(a, crs(b, c)) * (1.f / 6.f));
  }
  for (int v = threadIdx.x; v < M.nv; v += kGatherThreads) {
    const float3 a = rel(mc, load_pos(s, slot_of_gid[g0 + v]), cf);
    acc[2] += a.x;
    acc[3] += a.y;
    acc[4] += a.z;
  }
  double tot[5];
  for (int f = 0; f < 5; ++f) {
    red[threadIdx.x] = acc[f];
    __syncthreads();
    for (int off = kGatherThreads / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    tot[f] = red[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    av[2 * r] = tot[0];
    av[2 * r + 1] = tot[1];
    // centroid relative to the float-rounded previous centroid, then shifted
    centroid[3 * r] = double(cf.x) + tot[2] / M.nv;
    centroid[3 * r + 1] = double(cf.y) + tot[3] / M.nv;
    centroid[3 * r + 2] = double(cf.z) + tot[4] / M.nv;
  }
}

void launch_rbc_gather(const MembraneConst &mc, const MeshDev *meshes, const int32_t *rbc_mesh,
                       const int64_t *rbc_first, int nrbc, State s, const uint32_t *slot_of_gid,
                       double *av, double *centroid, hipStream_t st) {
  if (nrbc <= 0) return;
  hipLaunchKernelGGL(k_rbc_gather, dim3(nrbc), dim3(kGatherThreads), 0, st, mc, meshes, rbc_mesh,
                     rbc_first, s, slot_of_gid, av, centroid);
}

// gradient of the signed normal angle of triangles (a,b,c), (d,c,b) with
// respect to the vertex in `role` (0..3 = a,b,c,d); also returns sin/cos.
__device__ __forceinline__ float3 dihedral_grad(float3 a, float3 b, float3 c, float3 d, int role,
                                                float &sn, float &cs) {
  const float3 n1 = crs(sub(b, a), sub(c, a));
  const float3 n2 = crs(sub(c, d), sub(b, d));
  const float3 e = sub(c, b);
  const float le2 = dt3(e, e);
  const float le = sqrtf(le2);
  const float n11 = dt3(n1, n1), n22 = dt3(n2, n2);
  const float inv = __builtin_amdgcn_rsqf(n11 * n22);
  sn = dt3(crs(n1, n2), e) / le * inv;
  cs = dt3(n1, n2) * inv;
  const float f1 = -le / n11, f2 = -le / n22;
  const float3 ga = make_float3(f1 * n1.x, f1 * n1.y, f1 * n1.z);
  const float3 gd = make_float3(f2 * n2.x, f2 * n2.y, f2 * n2.z);
  if (role == 0) return ga;
  if (role == 3) return gd;
  const float ta = dt3(sub(a, b), e) / le2, td = dt3(sub(d, b), e) / le2;
  if (role == 1)
    return make_float3((ta - 1.f) * ga.x + (td - 1.f) * gd.x, (ta - 1.f) * ga.y + (td - 1.f) * gd.y,
                       (ta - 1.f) * ga.z + (td - 1.f) * gd.z);
  return make_float3(-ta * ga.x - td * gd.x, -ta * ga.y - td * gd.y, -ta * ga.z - td * gd.z);
}

__global__ void __launch_bounds__(128) k_membrane(
    MembraneConst mc, const MeshDev *__restrict__ meshes, const int32_t *__restrict__ rbc_mesh,
    const int64_t *__restrict__ rbc_first, const int64_t *__restrict__ rbc_voff, int nrbc,
    int64_t nvert, State s, const uint32_t *__restrict__ slot_of_gid, const double *__restrict__ av,
    uint32_t k, float *__restrict__ F, uint32_t *err) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nvert) return;
  // cell owning global vertex t
  int lo = 0, hi = nrbc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rbc_voff[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  const int r = lo;
  const MeshDev &M = meshes[rbc_mesh[r]];
  const int64_t g0 = rbc_first[r];
  const int v = int(t - rbc_voff[r]);
  const uint32_t sv = slot_of_gid[g0 + v];
  const float3 pv = load_pos(s, sv);
  const float3 vv = make_float3(s.vx[sv], s.vy[sv], s.vz[sv]);
  const uint32_t gv = uint32_t(g0 + v);
  float3 f = make_float3(0.f, 0.f, 0.f);
  const int terms = mc.terms;

  // ---- bonds, Eqs. (13)-(16)
  if (terms & (TDPD_TERM_BOND | TDPD_TERM_BOND_VISCOUS | TDPD_TERM_BOND_RANDOM)) {
    const float amp = sqrtf(2.f * mc.kT / mc.dt);
    const float ct = sqrtf(2.f * M.gamma_t);
    const float cc = sqrtf(fmaxf(3.f * M.gamma_c - M.gamma_t, 0.f)) * (1.f / 3.f);
    for (int b = M.bond_off[v]; b < M.bond_off[v + 1]; ++b) {
      const int w = M.bond_nbr[b];
      const uint32_t sw = slot_of_gid[g0 + w];
      const float3 d = rel(mc, load_pos(s, sw), pv);  // v -> w
      const float l = sqrtf(dt3(d, d));
      const float il = 1.f / l;
      if (terms & TDPD_TERM_BOND) {
        const float2 par = M.bond_par[b];  // (l_m, k_p)
        const float x = l / par.x;
        if (x >= 1.f) {
          atomicOr(err, kErrOverext);
        } else {
          const float om = 1.f - x;
          const float dwlc = mc.kT / M.p * (0.25f / (om * om) - 0.25f + x);
          const float dpow = -par.y * powu_any(l, -M.m_pow);
          const float fs = (dwlc + dpow) * il;
          f.x += fs * d.x;
          f.y += fs * d.y;
          f.z += fs * d.z;
        }
      }
      // e points from w to v (the paper's e_ij with i = v)
      const float3 e = make_float3(-d.x * il, -d.y * il, -d.z * il);
      if (terms & TDPD_TERM_BOND_VISCOUS) {
        const float3 vw = make_float3(s.vx[sw], s.vy[sw], s.vz[sw]);
        const float3 vr = sub(vv, vw);
        const float ve = dt3(vr, e);
        f.x += -M.gamma_t * vr.x - M.gamma_c * ve * e.x;
        f.y += -M.gamma_t * vr.y - M.gamma_c * ve * e.y;
        f.z += -M.gamma_t * vr.z - M.gamma_c * ve * e.z;
      }
      if (terms & TDPD_TERM_BOND_RANDOM) {
        const uint32_t gw = uint32_t(g0 + w);
        const uint32_t lo_g = gv < gw ? gv : gw, hi_g = gv < gw ? gw : gv;
        float W[10];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const u32x4 z = philox10(k, lo_g, hi_g, mc.ctr3 | uint32_t(64 + q), mc.seed_lo, mc.seed_hi);
          W[2 * q] = gauss(z.a, z.b);
          W[2 * q + 1] = gauss(z.c, z.d);
        }
        const float trW = W[0] + W[4] + W[8];  // trace of W and of its symmetric part
        const float ex[3] = {e.x, e.y, e.z};
        float o[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            float m = ct * (0.5f * (W[3 * i + j] + W[3 * j + i]) - (i == j ? trW * (1.f / 3.f) : 0.f));
            if (i == j) m += cc * trW;
            acc += m * ex[j];
          }
          o[i] = amp * acc;
        }
        f.x += o[0];
        f.y += o[1];
        f.z += o[2];
      }
    }
  }

  // ---- area and volume constraints, Eqs. (17)-(18)
  if (terms & (TDPD_TERM_AREA | TDPD_TERM_VOLUME)) {
    const float cg = float(M.kg * (av[2 * r] - M.A0) / M.A0);
    const float cv = float(M.kv * (av[2 * r + 1] - M.V0) / M.V0);
    for (int q = M.tri_off[v]; q < M.tri_off[v + 1]; ++q) {
      const int4 tr = M.tri_inc[q];  // (b, c, triangle, -), v first, counter-clockwise
      const float3 rb = rel(mc, load_pos(s, slot_of_gid[g0 + tr.x]), pv);
      const float3 rc = rel(mc, load_pos(s, slot_of_gid[g0 + tr.y]), pv);
      const float3 nn = crs(rb, rc);
      if (terms & TDPD_TERM_AREA) {
        const float nl = sqrtf(dt3(nn, nn));
        const float At = 0.5f * nl;
        const float a0 = M.A0t[tr.z];
        const float coef = -(cg + M.kl * (At - a0) / a0) * 0.5f / nl;
        const float3 g = crs(nn, sub(rc, rb));  // |n| * (n_hat x (c - b))
        f.x += coef * g.x;
        f.y += coef * g.y;
        f.z += coef * g.z;
      }
      if (terms & TDPD_TERM_VOLUME) {
        const float coef = -cv * (1.f / 6.f);
        f.x += coef * nn.x;
        f.y += coef * nn.y;
        f.z += coef * nn.z;
      }
    }
  }

  // ---- bending, Eq. (19)
  if (terms & TDPD_TERM_BENDING) {
    const float s0 = sinf(M.theta0), c0 = cosf(M.theta0);
    for (int q = M.dih_off[v]; q < M.dih_off[v + 1]; ++q) {
      const int4 D = M.dih_inc[q];
      const int role = M.dih_role[q];
      const float3 a = role == 0 ? make_float3(0.f, 0.f, 0.f) : rel(mc, load_pos(s, slot_of_gid[g0 + D.x]), pv);
      const float3 b = role == 1 ? make_float3(0.f, 0.f, 0.f) : rel(mc, load_pos(s, slot_of_gid[g0 + D.y]), pv);
      const float3 c = role == 2 ? make_float3(0.f, 0.f, 0.f) : rel(mc, load_pos(s, slot_of_gid[g0 + D.z]), pv);
      const float3 d = role == 3 ? make_float3(0.f, 0.f, 0.f) : rel(mc, load_pos(s, slot_of_gid[g0 + D.w]), pv);
      float sn, cs;
      const float3 g = dihedral_grad(a, b, c, d, role, sn, cs);
      const float coef = -M.kb * (sn * c0 - cs * s0);  // -kb sin(theta - theta0)
      f.x += coef * g.x;
      f.y += coef * g.y;
      f.z += coef * g.z;
    }
  }
  F[3 * sv] += f.x;
  F[3 * sv + 1] += f.y;
  F[3 * sv + 2] += f.z;
  if (!(isfinite(f.x) && isfinite(f.y) && isfinite(f.z))) atomicOr(err, kErrNonfinite);
}

void launch_membrane_forces(const MembraneConst &mc, const MeshDev *meshes,
                            const int32_t *rbc_mesh, const int64_t *rbc_first,
                            const int64_t *rbc_voff, int nrbc, int64_t nvert_total, State s,
                            const uint32_t *slot_of_gid, const double *av, uint32_t k, float *F,
                            uint32_t *err, hipStream_t st) {
  if (nrbc <= 0 || nvert_total <= 0) return;
  hipLaunchKernelGGL(k_membrane, dim3(unsigned((nvert_total + 127) / 128)), dim3(128), 0, st, mc,
                     meshes, rbc_mesh, rbc_first, rbc_voff, nrbc, nvert_total, s, slot_of_gid, av, k,
                     F, err);
}

}  // namespace tdpd
