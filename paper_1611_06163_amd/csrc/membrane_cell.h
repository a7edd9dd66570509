// membrane_cell.h -- the RBC membrane terms of one cell (Section 2.2) for
// workgroups of any multiple of 64 threads, in three parts:
//   1. K-Gather: per-triangle area and volume in FP64 (from the FP32
//      positions, relative to the cell's FP64 centroid) summed over the cell
//      in a fixed order (A^t, V^t into av), plus the centroid update;
//   2. per bond, once: WLC + POW spring (Eqs. 13-14), viscosity (Eq. 15) and
//      its random partner (Eq. 16), into the cell's scratch row;
//   3. per vertex: the signed sum of its bond forces, the global/local area
//      and volume constraint forces over its incident triangles (K-Apply,
//      Eqs. 17-18; each triangle recomputed by its three vertices as the
//      paper does, Section 3.3) and bending over its incident dihedrals
//      (Eq. 19), written to Fm.
// membrane_cell runs all three in one workgroup (the membrane kernel);
// membrane_elements runs 1 and a share of 2 (extra workgroups of the cell
// count scan) and membrane_vertices a share of 3 (extra workgroups of the
// pair kernel), the launch boundary between them ordering the parts.
// No atomics; every sum has a fixed order for a given workgroup size.
#pragma once

#include "launch.h"

namespace tdpd {

namespace mem {

__device__ __forceinline__ float3 sub(float3 a, float3 b) {
  return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ float3 crs(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dt3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
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

}  // namespace mem

// LDS layout: vertex slots and positions (16 B per vertex), then the FP64
// wavefront partials (5 per wavefront) and the 5 cell totals.
__host__ __device__ constexpr size_t membrane_cell_lds(int nv, int threads) {
  return (size_t(nv) * 16 + 7) / 8 * 8 + (size_t(threads / 64) * 5 + 5) * sizeof(double);
}

namespace mem {

// One cell as seen by a workgroup: mesh, box, staged positions.
struct Cell {
  const MeshDev *M;
  const BoxDev *B;
  int nv;
  int64_t g0;
  LeOff le;
  const uint32_t *sl;
  const float *px, *py, *pz;
  __device__ float3 P(int v) const { return make_float3(px[v], py[v], pz[v]); }
  __device__ float3 rel(float3 a, float3 o) const { return le_rel(*B, a, o, le.delta, nullptr); }
};

// Stage the cell's vertex slots and positions in LDS (every thread calls it).
__device__ __forceinline__ Cell stage_cell(const MemArgs &ma, const BoxDev *__restrict__ boxes,
                                           const State &s, uint32_t k, int r, char *lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const MeshDev &M = ma.meshes[ma.rbc_mesh[r]];
  const BoxDev &B = boxes[ma.rbc_box[r]];
  const int nv = M.nv;
  uint32_t *sl = reinterpret_cast<uint32_t *>(lds);
  float *px = reinterpret_cast<float *>(sl + nv), *py = px + nv, *pz = py + nv;
  const int64_t g0 = ma.rbc_first[r];
  for (int v = tid; v < nv; v += nt) {
    const uint32_t q = ma.slot_of_gid[g0 + v];
    sl[v] = q;
    px[v] = s.x[q];
    py[v] = s.y[q];
    pz[v] = s.z[q];
  }
  __syncthreads();
  // nearest image (sheared boxes: Lees-Edwards image of the step counter)
  return Cell{&M, &B, nv, g0, le_offsets(B, k, ma.mc.dt), sl, px, py, pz};
}

// Nearest image of a relative to the FP64 point c, in FP64 (the shift of a
// sheared box as in le_rel).
__device__ __forceinline__ double3 rel64(const BoxDev &B, float3 a, double cx, double cy,
                                         double cz, float delta) {
  const double Lx = B.L[0], Ly = B.L[1], Lz = B.L[2];
  double dx = double(a.x) - cx, dy = double(a.y) - cy, dz = double(a.z) - cz;
  if (B.shear != 0.f) {
    if (dy > 0.5 * Ly) {
      dy -= Ly;
      dx -= double(delta);
    } else if (dy < -0.5 * Ly) {
      dy += Ly;
      dx += double(delta);
    }
  } else {
    dy -= Ly * rint(dy / Ly);
  }
  return make_double3(dx - Lx * rint(dx / Lx), dy, dz - Lz * rint(dz / Lz));
}

__device__ __forceinline__ double3 sub64(double3 a, double3 b) {
  return make_double3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ double3 crs64(double3 a, double3 b) {
  return make_double3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double dt64(double3 a, double3 b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}

// 1. K-Gather: A^t, V^t into av[r], centroid[r] moved to the mean position.
// Every triangle's area and volume term is evaluated in FP64 from the FP32
// positions, so the totals, and with them the global area and volume
// coefficients of Eqs. (17)-(18), carry no FP32 rounding.
__device__ __forceinline__ void kgather(const MemArgs &ma, const Cell &C, int r, char *lds) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const MeshDev &M = *C.M;
  double *red = reinterpret_cast<double *>(lds + (size_t(C.nv) * 16 + 7) / 8 * 8);
  double *tot = red + (nt / 64) * 5;
  const double cx = ma.centroid[3 * r], cy = ma.centroid[3 * r + 1], cz = ma.centroid[3 * r + 2];
  const BoxDev &B = *C.B;
  const float del = C.le.delta;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int t = tid; t < M.ntri; t += nt) {
    const double3 a = rel64(B, C.P(M.tri[3 * t]), cx, cy, cz, del);
    const double3 b = rel64(B, C.P(M.tri[3 * t + 1]), cx, cy, cz, del);
    const double3 c = rel64(B, C.P(M.tri[3 * t + 2]), cx, cy, cz, del);
    const double3 nn = crs64(sub64(b, a), sub64(c, a));
    acc[0] += 0.5 * sqrt(dt64(nn, nn));
    acc[1] += dt64(a, crs64(b, c)) * (1.0 / 6.0);
  }
  for (int v = tid; v < C.nv; v += nt) {
    const double3 a = rel64(B, C.P(v), cx, cy, cz, del);
    acc[2] += a.x;
    acc[3] += a.y;
    acc[4] += a.z;
  }
  // fixed-order sums: a butterfly inside each wavefront (partners add the
  // same two values, so every lane ends with the same bits), then the
  // wavefront totals in wavefront order
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double a = acc[f];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) a += __shfl_xor(a, off);
    if ((tid & 63) == 0) red[(tid >> 6) * 5 + f] = a;
  }
  __syncthreads();
  if (tid < 5) {
    double a = 0.0;
    for (int w = 0; w < nt / 64; ++w) a += red[w * 5 + tid];
    tot[tid] = a;
  }
  __syncthreads();
  if (tid == 0 && !ma.mc.local_only) {
    ma.av[2 * r] = tot[0];
    ma.av[2 * r + 1] = tot[1];
    ma.centroid[3 * r] = cx + tot[2] / C.nv;
    ma.centroid[3 * r + 1] = cy + tot[3] / C.nv;
    ma.centroid[3 * r + 2] = cz + tot[4] / C.nv;
  }
}

// 2. bonds [b0, b1), Eqs. (13)-(16): force on the bond's first vertex a,
// into the cell's scratch row [3][nbond].
__device__ __forceinline__ void bond_forces(const MemArgs &ma, const Cell &C, const State &s,
                                            uint32_t k, uint32_t *err, int r, int b0, int b1) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const MeshDev &M = *C.M;
  const BoxDev &B = *C.B;
  const MembraneConst &mc = ma.mc;
  const int terms = mc.terms;
  if (!(terms & (TDPD_TERM_BOND | TDPD_TERM_BOND_VISCOUS | TDPD_TERM_BOND_RANDOM))) return;
  float *fb = ma.Fb + 3 * ma.bond_stride * r;
  const float amp = sqrtf(2.f * mc.kT / mc.dt);
  const float ct = sqrtf(2.f * M.gamma_t);
  const float cc = sqrtf(fmaxf(3.f * M.gamma_c - M.gamma_t, 0.f)) * (1.f / 3.f);
  for (int bnd = b0 + tid; bnd < b1; bnd += nt) {
    const int2 ab = M.bond_ab[bnd];
    int nyb = 0;  // b taken in the sheared image below (-1) or above (+1) a
    const float3 d = le_rel(B, C.P(ab.y), C.P(ab.x), C.le.delta, &nyb);  // a -> b
    const float l = sqrtf(dt3(d, d));
    const float il = 1.f / l;
    float3 f = make_float3(0.f, 0.f, 0.f);
    if (terms & TDPD_TERM_BOND) {
      const float2 par = M.bond_par[bnd];  // (l_m, k_p)
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
    // e points from b to a (the paper's e_ij with i = a)
    const float3 e = make_float3(-d.x * il, -d.y * il, -d.z * il);
    if (terms & TDPD_TERM_BOND_VISCOUS) {
      const uint32_t qa = C.sl[ab.x], qb = C.sl[ab.y];
      const float3 vr = make_float3(s.vx[qa] - s.vx[qb] - float(nyb) * C.le.u, s.vy[qa] - s.vy[qb],
                                    s.vz[qa] - s.vz[qb]);
      const float ve = dt3(vr, e);
      f.x += -M.gamma_t * vr.x - M.gamma_c * ve * e.x;
      f.y += -M.gamma_t * vr.y - M.gamma_c * ve * e.y;
      f.z += -M.gamma_t * vr.z - M.gamma_c * ve * e.z;
    }
    if (terms & TDPD_TERM_BOND_RANDOM) {
      // a < b locally and gids are consecutive, so (g0+a, g0+b) is ordered;
      // the counter takes box-local gids
      const uint32_t ga = uint32_t(C.g0 + ab.x) - B.gid_base, gb = uint32_t(C.g0 + ab.y) - B.gid_base;
      float W[12];  // streams 64..66: (cos, sin) of words (0,1) then (2,3); first 9 used
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const u32x4 z = philox10(k, ga, gb, B.ctr3 | uint32_t(64 + q), B.seed_lo, B.seed_hi);
        gauss2(z.a, z.b, W[4 * q], W[4 * q + 1]);
        gauss2(z.c, z.d, W[4 * q + 2], W[4 * q + 3]);
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
    fb[bnd] = f.x;
    fb[M.nbond + bnd] = f.y;
    fb[2 * M.nbond + bnd] = f.z;
  }
}

// 3. vertices [v0, v1): bond sums, area/volume constraints, bending, into Fm.
// A^t, V^t come from av[r] (part 1, in this workgroup or an earlier launch).
__device__ __forceinline__ void vertex_forces(const MemArgs &ma, const Cell &C, uint32_t *err,
                                              int r, int v0, int v1) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const MeshDev &M = *C.M;
  const MembraneConst &mc = ma.mc;
  const int terms = mc.terms;
  const float *fb = ma.Fb + 3 * ma.bond_stride * r;
  const SurrUse su = ma.su;
  const int64_t voff = ma.rbc_voff[r];
  const float cg = mc.local_only ? 0.f : float(M.kg * (ma.av[2 * r] - M.A0) / M.A0);
  const float cv = mc.local_only ? 0.f : float(M.kv * (ma.av[2 * r + 1] - M.V0) / M.V0);
  const float s0 = sinf(M.theta0), c0 = cosf(M.theta0);
  for (int v = v0 + tid; v < v1; v += nt) {
    const float3 pv = C.P(v);
    float3 f = make_float3(0.f, 0.f, 0.f);
    // bending and local area of this vertex come from the surrogate
    const bool sv = su.flag && su.flag[voff + v];
    if (terms & (TDPD_TERM_BOND | TDPD_TERM_BOND_VISCOUS | TDPD_TERM_BOND_RANDOM)) {
      for (int q = M.bond_off[v]; q < M.bond_off[v + 1]; ++q) {
        const int inc = M.bond_inc[q];
        const int bnd = inc >> 1;
        const float sg = (inc & 1) ? -1.f : 1.f;
        f.x += sg * fb[bnd];
        f.y += sg * fb[M.nbond + bnd];
        f.z += sg * fb[2 * M.nbond + bnd];
      }
    }
    if (terms & (TDPD_TERM_AREA | TDPD_TERM_VOLUME)) {
      for (int q = M.tri_off[v]; q < M.tri_off[v + 1]; ++q) {
        const int4 tr = M.tri_inc[q];  // (b, c, triangle, -), v first, counter-clockwise
        const float3 rb = C.rel(C.P(tr.x), pv);
        const float3 rc = C.rel(C.P(tr.y), pv);
        const float3 nn = crs(rb, rc);
        if (terms & TDPD_TERM_AREA) {
          const float nl = sqrtf(dt3(nn, nn));
          const float At = 0.5f * nl;
          const float a0 = M.A0t[tr.z];
          const float cl = sv ? 0.f : M.kl * (At - a0) / a0;
          const float coef = -(cg + cl) * 0.5f / nl;
          const float3 g = crs(nn, sub(rc, rb));  // |n| * (n_hat x (c - b))
          f.x += coef * g.x;
          f.y += coef * g.y;
          f.z += coef * g.z;
        }
        if (terms & TDPD_TERM_VOLUME) {
          const float coef = -cv * (1.f / 6.f);  // dV/dv = (b - v) x (c - v) / 6
          f.x += coef * nn.x;
          f.y += coef * nn.y;
          f.z += coef * nn.z;
        }
      }
    }
    if ((terms & TDPD_TERM_BENDING) && !sv) {
      const float3 zero3 = make_float3(0.f, 0.f, 0.f);
      for (int q = M.dih_off[v]; q < M.dih_off[v + 1]; ++q) {
        const int4 D = M.dih_inc[q];
        const int role = M.dih_role[q];
        const float3 a = role == 0 ? zero3 : C.rel(C.P(D.x), pv);
        const float3 b = role == 1 ? zero3 : C.rel(C.P(D.y), pv);
        const float3 c = role == 2 ? zero3 : C.rel(C.P(D.z), pv);
        const float3 d = role == 3 ? zero3 : C.rel(C.P(D.w), pv);
        float sn, cs;
        const float3 g = dihedral_grad(a, b, c, d, role, sn, cs);
        const float coef = -M.kb * (sn * c0 - cs * s0);  // -kb sin(theta - theta0)
        f.x += coef * g.x;
        f.y += coef * g.y;
        f.z += coef * g.z;
      }
    }
    const int64_t o = 3 * (voff + v);
    if (sv) {
      f.x += su.Fs[o];
      f.y += su.Fs[o + 1];
      f.z += su.Fs[o + 2];
    }
    ma.Fm[o] = f.x;
    ma.Fm[o + 1] = f.y;
    ma.Fm[o + 2] = f.z;
    if (!(isfinite(f.x) && isfinite(f.y) && isfinite(f.z))) atomicOr(err, kErrNonfinite);
  }
}

}  // namespace mem

// All three parts for cell r in one workgroup.
__device__ __forceinline__ void membrane_cell(const MemArgs &ma, const BoxDev *__restrict__ boxes,
                                              const State &s, uint32_t k, uint32_t *err, int r,
                                              char *lds) {
  if (ma.mc.gate > 0 && (k % uint32_t(ma.mc.gate)) != 0u) return;
  const mem::Cell C = mem::stage_cell(ma, boxes, s, k, r, lds);
  if (ma.mc.local_only) {  // no K-Gather writes: A^t, V^t are not used
  } else {
    mem::kgather(ma, C, r, lds);
  }
  mem::bond_forces(ma, C, s, k, err, r, 0, C.M->nbond);
  __syncthreads();
  mem::vertex_forces(ma, C, err, r, 0, C.nv);
}

// Part 1 (p = 0) or a share of part 2 (p >= 1: bonds [(p-1) nbond / (parts-1),
// p nbond / (parts-1))) of cell r; the state is the one before this
// evaluation's reorder.
__device__ __forceinline__ void membrane_elements(const MemArgs &ma, const BoxDev *__restrict__ boxes,
                                                  const State &s, uint32_t k, uint32_t *err, int r,
                                                  int p, int parts, char *lds) {
  const mem::Cell C = mem::stage_cell(ma, boxes, s, k, r, lds);
  if (p == 0) {
    mem::kgather(ma, C, r, lds);
    return;
  }
  const int64_t nb = C.M->nbond, q = parts - 1;
  mem::bond_forces(ma, C, s, k, err, r, int(nb * (p - 1) / q), int(nb * p / q));
}

// Part 3 for vertices [g nv / parts, (g+1) nv / parts) of cell r.
__device__ __forceinline__ void membrane_vertices(const MemArgs &ma, const BoxDev *__restrict__ boxes,
                                                  const State &s, uint32_t k, uint32_t *err, int r,
                                                  int g, int parts, char *lds) {
  const mem::Cell C = mem::stage_cell(ma, boxes, s, k, r, lds);
  mem::vertex_forces(ma, C, err, r, int(int64_t(C.nv) * g / parts),
                     int(int64_t(C.nv) * (g + 1) / parts));
}

}  // namespace tdpd
