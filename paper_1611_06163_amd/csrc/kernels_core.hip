// kernels_core.hip -- binning (LSD radix sort of cell keys), reordering,
// velocity-Verlet kicks, diagnostics and gid-order gathers.
#include "launch_list.h"
#include "membrane_cell.h"

namespace tdpd {

// ------------------------------------------------------------- radix sort
// LSD radix sort with 8-bit digits.  Each pass: (1) per-tile digit histogram,
// (2) one exclusive scan over [digit][tile] (digit-major, so tiles of equal
// digit are consecutive and the scatter is stable), (3) per-tile scatter with
// ranks from wavefront ballots.  Tiles are 2048 keys: 256 threads x 8 rounds.
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kScanThreads = 1024;

static inline int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }
size_t radix_hist_words(int64_t n) { return size_t(kRadix) * size_t(sort_tiles(n) > 0 ? sort_tiles(n) : 1); }

__global__ void __launch_bounds__(kSortThreads) k_radix_hist(const uint32_t *__restrict__ keys,
                                                             int64_t n, int shift,
                                                             uint32_t *__restrict__ hist,
                                                             int64_t ntiles) {
  __shared__ uint32_t h[kRadix];
  for (int d = threadIdx.x; d < kRadix; d += kSortThreads) h[d] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kSortThreads) hist[int64_t(d) * ntiles + blockIdx.x] = h[d];
}

// Exclusive scan of `total` words in place, one workgroup; thread t owns the
// contiguous chunk [t*chunk, (t+1)*chunk).
__global__ void __launch_bounds__(kScanThreads) k_scan_inplace(uint32_t *__restrict__ a,
                                                               int64_t total) {
  __shared__ uint32_t part[kScanThreads];
  const int64_t chunk = (total + kScanThreads - 1) / kScanThreads;
  const int64_t b = int64_t(threadIdx.x) * chunk;
  const int64_t e = b + chunk < total ? b + chunk : total;
  uint32_t s = 0;
  for (int64_t i = b; i < e; ++i) s += a[i];
  part[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the partial sums
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int64_t i = b; i < e; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(kSortThreads) k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ hist,
    int64_t ntiles) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ uint32_t base[kRadix];
  __shared__ uint32_t wcnt[kWaves][kRadix];
  const int tid = threadIdx.x, wave = tid >> 6;
  for (int d = tid; d < kRadix; d += kSortThreads) base[d] = hist[int64_t(d) * ntiles + blockIdx.x];
  const uint64_t lt = __lanemask_lt();
  const int64_t tile0 = int64_t(blockIdx.x) * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    for (int q = tid; q < kWaves * kRadix; q += kSortThreads) (&wcnt[0][0])[q] = 0;
    __syncthreads();
    const int64_t i = tile0 + r * kSortThreads + tid;
    const bool valid = i < n;
    uint32_t key = 0, val = 0, digit = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
      digit = (key >> shift) & (kRadix - 1);
    }
    // lanes of this wavefront holding the same digit
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (digit >> b) & 1u;
      const uint64_t m = __ballot(bit);
      same &= bit ? m : ~m;
    }
    const uint32_t rank = __popcll(same & lt);
    if (valid && rank == 0) wcnt[wave][digit] = __popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t off = base[digit] + rank;
      for (int w = 0; w < wave; ++w) off += wcnt[w][digit];
      kout[off] = key;
      vout[off] = val;
    }
    __syncthreads();
    for (int d = tid; d < kRadix; d += kSortThreads) {
      uint32_t t = 0;
      for (int w = 0; w < kWaves; ++w) t += wcnt[w][d];
      base[d] += t;
    }
    __syncthreads();
  }
}

void radix_sort(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp,
                uint32_t *vals_tmp, uint32_t *keys_out, uint32_t *vals_out, uint32_t *hist,
                int64_t n, int key_bits, hipStream_t st) {
  if (n <= 0) return;
  const int passes = key_bits <= kRadixBits ? 1 : (key_bits + kRadixBits - 1) / kRadixBits;
  const int64_t ntiles = sort_tiles(n);
  // ping-pong so that the last pass lands in *_out
  const uint32_t *ki = keys_in, *vi = vals_in;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    uint32_t *ko = to_out ? keys_out : keys_tmp;
    uint32_t *vo = to_out ? vals_out : vals_tmp;
    (void)last;
    const int shift = p * kRadixBits;
    hipLaunchKernelGGL(k_radix_hist, dim3(unsigned(ntiles)), dim3(kSortThreads), 0, st, ki, n,
                       shift, hist, ntiles);
    hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(kScanThreads), 0, st, hist,
                       int64_t(kRadix) * ntiles);
    hipLaunchKernelGGL(k_radix_scatter, dim3(unsigned(ntiles)), dim3(kSortThreads), 0, st, ki, vi,
                       ko, vo, n, shift, hist, ntiles);
    ki = ko;
    vi = vo;
  }
}

// ------------------------------------------------------------- integrator
// First half kick, drift, wall reflection, wrap and cell key of every
// particle.  In counting mode the value is the particle's unordered rank in
// its cell: lanes of a wave holding the same key in a run (slots are in the
// previous step's cell order, so most runs are whole cells) take one atomic
// for the run, and each lane adds its offset in the run.
// The closing work of an evaluation for particle i: membrane forces added
// into F, then (integrate) the second half kick of a mobile particle.
// Returns the total force.  With vout (the kick folded into the next step's
// first kick, in the same kernel) the kicked velocity is handed over in
// registers instead of through memory.  Kicks are explicit fused
// multiply-adds, so the folded and the separate kicks give the same bits.
__device__ __forceinline__ float3 close_step(const PairConst &pc, State s, float *F,
                                             const float *Q, int64_t n, const VertexMap &vm,
                                             bool integrate, int64_t i, uint32_t info,
                                             float3 *vout = nullptr) {
  float fx = F[3 * i], fy = F[3 * i + 1], fz = F[3 * i + 2];
  const int body = info_body(info);
  if (vm.Fm && body >= 0) {
    const int64_t v = vm.rbc_voff[body] + (int64_t(s.gid[i]) - vm.rbc_first[body]);
    fx += vm.Fm[3 * v];
    fy += vm.Fm[3 * v + 1];
    fz += vm.Fm[3 * v + 2];
    // the total force is kept for readback, except where the next step
    // begins in the same kernel (its pair kernel overwrites F before anyone
    // reads it; scattered over the vertices, the stores would cost a write
    // granule each)
    if (!vout) {
      F[3 * i] = fx;
      F[3 * i + 1] = fy;
      F[3 * i + 2] = fz;
    }
  }
  if (integrate && !info_frozen(info)) {
    const float h = pc.half_dt;
    const float3 v1 = make_float3(__fmaf_rn(h, fx, s.vx[i]), __fmaf_rn(h, fy, s.vy[i]),
                                  __fmaf_rn(h, fz, s.vz[i]));
    if (vout) {
      *vout = v1;
    } else {
      s.vx[i] = v1.x;
      s.vy[i] = v1.y;
      s.vz[i] = v1.z;
    }
    for (int sp = 0; sp < pc.n_species; ++sp)
      s.C[sp * n + i] = __fmaf_rn(h, Q[pc.n_species * i + sp], s.C[sp * n + i]);
  }
  return make_float3(fx, fy, fz);
}

// Half kick and drift of mobile particle i under force f: velocity and
// concentration kick, drift, wall reflection, sheared-boundary crossing (at
// the offsets of counter *kdev + finish) and wrap; stores the new x and v
// and returns them; with vin the kick starts from *vin (the closing kick of
// the previous step handed over by close_step).
__device__ __forceinline__ void kick_drift(const PairConst &pc, const BoxDev &B, State s, float3 f,
                                           const float *__restrict__ Q, int64_t n, int64_t i,
                                           const uint32_t *__restrict__ kdev, int finish,
                                           const float3 *vin, float &x, float &y, float &z,
                                           float &vx, float &vy, float &vz) {
  const float h = pc.half_dt;
  const float3 v0 = vin ? *vin : make_float3(s.vx[i], s.vy[i], s.vz[i]);
  vx = __fmaf_rn(h, f.x, v0.x);
  vy = __fmaf_rn(h, f.y, v0.y);
  vz = __fmaf_rn(h, f.z, v0.z);
  for (int sp = 0; sp < pc.n_species; ++sp)
    s.C[sp * n + i] = __fmaf_rn(h, Q[pc.n_species * i + sp], s.C[sp * n + i]);
  x += pc.dt * vx;
  y += pc.dt * vy;
  z += pc.dt * vz;
  if (pc.wall_axis == 3) {
    // the tube: a particle farther than R from the axis is mirrored along
    // its radius to 2R - r, its velocity reversed
    const float cy = 0.5f * B.L[1], cz = 0.5f * B.L[2], R = pc.wall_radius;
    const float dy = y - cy, dz = z - cz;
    const float r2 = __fmaf_rn(dz, dz, dy * dy);
    if (r2 > R * R) {
      const float r = __builtin_amdgcn_sqrtf(r2);
      const float f = (2.f * R - r) / r;
      y = __fmaf_rn(dy, f, cy);
      z = __fmaf_rn(dz, f, cz);
      vx = -vx;
      vy = -vy;
      vz = -vz;
    }
  } else if (pc.wall_axis >= 0) {
    float *c = pc.wall_axis == 0 ? &x : (pc.wall_axis == 1 ? &y : &z);
    const float L = B.L[pc.wall_axis], w = pc.wall_w;
    bool hit = false;
    if (*c < w) {
      *c = 2.f * w - *c;
      hit = true;
    } else if (*c > L - w) {
      *c = 2.f * (L - w) - *c;
      hit = true;
    }
    if (hit) {
      vx = -vx;
      vy = -vy;
      vz = -vz;
    }
  }
  if (B.shear != 0.f) {
    // crossing the y boundary of a sheared box: into the image below
    // (above), x by -delta (+delta), x velocity by -u (+u), with the
    // offsets of this step's counter (the positions are at that time)
    const LeOff le = le_offsets(B, *kdev + uint32_t(finish), pc.dt);
    if (y >= B.L[1]) {
      y -= B.L[1];
      x -= le.delta;
      vx -= le.u;
    } else if (y < 0.f) {
      y += B.L[1];
      x += le.delta;
      vx += le.u;
    }
  }
  x = wrap_coord(x, B.L[0]);
  y = wrap_coord(y, B.L[1]);
  z = wrap_coord(z, B.L[2]);
  s.x[i] = x;
  s.y[i] = y;
  s.z[i] = z;
  s.vx[i] = vx;
  s.vy[i] = vy;
  s.vz[i] = vz;
}

__global__ void __launch_bounds__(256) k_prekick(PairConst pc, const BoxDev *__restrict__ boxes,
                                                 State s, float *__restrict__ F,
                                                 const float *__restrict__ Q, int64_t n,
                                                 uint32_t *__restrict__ keys,
                                                 uint32_t *__restrict__ vals, int integrate,
                                                 uint32_t *__restrict__ cell_count,
                                                 uint32_t *__restrict__ kdev, int finish,
                                                 VertexMap vprev, uint32_t *__restrict__ kstep) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool active = i < n;
  // the counter of this evaluation, for kernels on the second stream that
  // run while the scatter advances *kdev
  if (i == 0 && kstep) *kstep = *kdev + uint32_t(finish);
  uint32_t key = 0xffffffffu;
  if (active) {
    const uint32_t info = s.info[i];
    const BoxDev &B = boxes[info_box(info)];
    float x = s.x[i], y = s.y[i], z = s.z[i];
    float3 f, v1;
    const bool carry = finish && integrate;  // this kernel kicks again
    if (finish) {
      f = close_step(pc, s, F, Q, n, vprev, true, i, info, carry ? &v1 : nullptr);
    } else {
      f = make_float3(F[3 * i], F[3 * i + 1], F[3 * i + 2]);
    }
    if (integrate && !info_frozen(info)) {
      float vx, vy, vz;
      kick_drift(pc, B, s, f, Q, n, i, kdev, finish, carry ? &v1 : nullptr, x, y, z, vx, vy, vz);
    }
    const int cx = cell_coord(x, B.inv_h[0], B.nc[0]);
    const int cy = cell_coord(y, B.inv_h[1], B.nc[1]);
    const int cz = cell_coord(z, B.inv_h[2], B.nc[2]);
    key = B.cell_base + uint32_t((cz * B.nc[1] + cy) * B.nc[0] + cx);
    keys[i] = key;
  }
  if (!cell_count) {
    if (active) vals[i] = uint32_t(i);
    return;
  }
  // runs of equal keys inside the wave (every lane takes part)
  const int lane = int(threadIdx.x & 63u);
  const uint32_t prev = uint32_t(__shfl_up(int(key), 1));
  const bool start = lane == 0 || prev != key;
  const uint64_t starts = __ballot(start);
  uint32_t base = 0;
  if (start && active) {
    const uint64_t above = starts & ~((2ull << lane) - 1ull);
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    base = atomicAdd(&cell_count[key], uint32_t(next - lane));
  }
  const int leader = 63 - __clzll((long long)(starts & ((2ull << lane) - 1ull)));
  const uint32_t b0 = uint32_t(__shfl(int(base), leader));
  if (active) vals[i] = b0 + uint32_t(lane - leader);
}

void launch_prekick(const PairConst &pc, const BoxDev *boxes, State s, float *F,
                    const float *Q, int64_t n, uint32_t *keys, uint32_t *vals, bool integrate,
                    uint32_t *cell_count, uint32_t *kdev, bool finish, VertexMap prev,
                    uint32_t *kstep, hipStream_t st) {
  const int64_t nb = n > 0 ? (n + 255) / 256 : 1;
  hipLaunchKernelGGL(k_prekick, dim3(unsigned(nb)), dim3(256), 0, st, pc, boxes, s, F, Q, n, keys,
                     vals, int(integrate), cell_count, kdev, int(finish), prev, kstep);
}

// First half of a step on the neighbour-list path (no binning): half kick
// and drift, then the check that the particle has not moved more than half
// the skin from its position at the last list build, and the packed copies
// the list pair kernel gathers.
__global__ void __launch_bounds__(256) k_prekick_list(PairConst pc,
                                                      const BoxDev *__restrict__ boxes, State s,
                                                      const float *__restrict__ F,
                                                      const float *__restrict__ Q, int64_t n,
                                                      int integrate,
                                                      const uint32_t *__restrict__ kdev,
                                                      ListDev L, uint32_t *err,
                                                      uint32_t *__restrict__ kstep) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i == 0 && kstep) *kstep = *kdev;
  if (i >= n) return;
  const uint32_t info = s.info[i];
  const BoxDev &B = boxes[info_box(info)];
  float x = s.x[i], y = s.y[i], z = s.z[i];
  float vx, vy, vz;
  if (integrate && !info_frozen(info)) {
    const float3 f = make_float3(F[3 * i], F[3 * i + 1], F[3 * i + 2]);
    kick_drift(pc, B, s, f, Q, n, i, kdev, 0, nullptr, x, y, z, vx, vy, vz);
  } else {
    vx = s.vx[i];
    vy = s.vy[i];
    vz = s.vz[i];
  }
  const float4 r = L.xref[i];
  const float dx = pair_disp(x, r.x, B.L[0]), dy = pair_disp(y, r.y, B.L[1]),
              dz = pair_disp(z, r.z, B.L[2]);
  if (dist2(dx, dy, dz) > L.drift2) atomicOr(err, kErrSkin);
  L.p4[i] = make_float4(x, y, z, __uint_as_float(info));
  L.v4[i] = make_float4(vx, vy, vz, __uint_as_float(s.gid[i] - B.gid_base));
  if (L.c4) {
    const int S = pc.n_species;
    L.c4[i] = make_float4(s.C[i], S > 1 ? s.C[n + i] : 0.f, S > 2 ? s.C[2 * n + i] : 0.f,
                          S > 3 ? s.C[3 * n + i] : 0.f);
  }
}

void launch_prekick_list(const PairConst &pc, const BoxDev *boxes, State s, const float *F,
                         const float *Q, int64_t n, bool integrate, const uint32_t *kdev,
                         const ListDev &L, uint32_t *err, uint32_t *kstep, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_prekick_list, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, pc, boxes,
                     s, F, Q, n, int(integrate), kdev, L, err, kstep);
}

// ------------------------------------------------------------- counting binning
// A stable one-digit radix sort (radix = number of cells): the cell counts
// come from atomic increments in k_prekick, one exclusive scan gives
// cell_start, a scatter places every particle at start + its unordered rank,
// and k_rank_gather replaces that rank by the particle's rank in previous
// order among its cell (a count over the cell), so the final order is the
// same as a stable sort's and does not depend on atomic ordering.
constexpr int kCellTile = 4 * kScanThreads;  // cells per scan tile

// Inclusive scan of one value per thread over the block (1024 threads):
// shuffle scans inside each wavefront, then a scan of the 16 wavefront
// totals (sh holds at least 16 words).
__device__ __forceinline__ uint32_t block_scan_incl(uint32_t v, uint32_t *sh) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = uint32_t(__shfl_up(int(v), off));
    if (lane >= off) v += u;
  }
  __syncthreads();  // sh may still be read by the caller's previous scan
  if (lane == 63) sh[w] = v;
  __syncthreads();
  if (w == 0) {
    uint32_t tw = lane < kScanThreads / 64 ? sh[lane] : 0u;
#pragma unroll
    for (int off = 1; off < kScanThreads / 64; off <<= 1) {
      const uint32_t u = uint32_t(__shfl_up(int(tw), off));
      if (lane >= off) tw += u;
    }
    if (lane < kScanThreads / 64) sh[lane] = tw;
  }
  __syncthreads();
  return v + (w > 0 ? sh[w - 1] : 0u);
}

// Sum of the cell counts of each tile of kCellTile cells.
__global__ void __launch_bounds__(kScanThreads) k_count_tiles(const uint32_t *__restrict__ count,
                                                              int64_t ncell,
                                                              uint32_t *__restrict__ tile_sum) {
  __shared__ uint32_t sh[kScanThreads];
  const int64_t c0 = int64_t(blockIdx.x) * kCellTile;
  uint32_t v = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t c = c0 + q * kScanThreads + threadIdx.x;
    if (c < ncell) v += count[c];
  }
  const uint32_t tot = block_scan_incl(v, sh);
  if (threadIdx.x == kScanThreads - 1) tile_sum[blockIdx.x] = tot;
}

// Exclusive scan of the cell counts into cell_start (tile prefix from the
// tile sums, then a block scan of the tile); clears the counts.
// Workgroups past the scan tiles take the membrane K-Gather and bond forces
// of one cell share each (membrane_elements).
__global__ void __launch_bounds__(kScanThreads) k_count_scan(uint32_t *__restrict__ count,
                                                             int64_t ncell, int ntiles,
                                                             const uint32_t *__restrict__ tile_sum,
                                                             uint32_t *__restrict__ start,
                                                             MemArgs ma, int eparts,
                                                             const BoxDev *__restrict__ boxes,
                                                             State s,
                                                             const uint32_t *__restrict__ kdev,
                                                             int kofs, uint32_t *err) {
  __shared__ uint32_t sh[kScanThreads];
  __shared__ uint32_t tile[kCellTile];
  const int t = threadIdx.x;
  if (int(blockIdx.x) >= ntiles) {
    const int q = int(blockIdx.x) - ntiles;
    membrane_elements(ma, boxes, s, *kdev + uint32_t(kofs), err, q / eparts, q % eparts, eparts,
                      reinterpret_cast<char *>(tile));
    return;
  }
  const int64_t c0 = int64_t(blockIdx.x) * kCellTile;
  // prefix of the earlier tiles
  uint32_t pre = 0;
  for (int64_t q = t; q < int64_t(blockIdx.x); q += kScanThreads) pre += tile_sum[q];
  (void)block_scan_incl(pre, sh);
  const uint32_t base = sh[kScanThreads / 64 - 1];  // the block total
  __syncthreads();
  // coalesced load of the tile, then four consecutive cells per thread
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t c = c0 + q * kScanThreads + t;
    uint32_t v = 0;
    if (c < ncell) {
      v = count[c];
      count[c] = 0u;  // ready for the next step
    }
    tile[q * kScanThreads + t] = v;
  }
  __syncthreads();
  const uint32_t a0 = tile[4 * t], a1 = tile[4 * t + 1], a2 = tile[4 * t + 2], a3 = tile[4 * t + 3];
  const uint32_t incl = block_scan_incl(a0 + a1 + a2 + a3, sh);
  const uint32_t ex = base + incl - (a0 + a1 + a2 + a3);
  __syncthreads();
  tile[4 * t] = ex;
  tile[4 * t + 1] = ex + a0;
  tile[4 * t + 2] = ex + a0 + a1;
  tile[4 * t + 3] = ex + a0 + a1 + a2;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t c = c0 + q * kScanThreads + t;
    if (c < ncell) start[c] = tile[q * kScanThreads + t];
  }
  if (int(blockIdx.x) == ntiles - 1 && t == kScanThreads - 1) start[ncell] = ex + a0 + a1 + a2 + a3;
}

int64_t count_scan_tiles(int64_t ncell) { return ncell > 0 ? (ncell + kCellTile - 1) / kCellTile : 1; }

// the K-Gather in one workgroup, the bonds in workgroups of up to
// kBondsPerPart (most lanes then carry one bond, with its three Philox
// blocks, on the critical path)
constexpr int64_t kBondsPerPart = 384;
int membrane_element_parts(int64_t max_nbond) {
  return 1 + int(max_nbond > 0 ? (max_nbond + kBondsPerPart - 1) / kBondsPerPart : 1);
}

bool scan_takes_membrane(int max_nv) {
  return membrane_cell_lds(max_nv, kScanThreads) <= sizeof(uint32_t) * kCellTile;
}

__global__ void __launch_bounds__(256) k_scatter_rank(const uint32_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ rank,
                                                      const uint32_t *__restrict__ start, int64_t n,
                                                      uint32_t *__restrict__ tmp,
                                                      uint32_t *__restrict__ advance) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (advance && i == 0) *advance += 1u;  // nothing in this launch reads it
  if (i >= n) return;
  // the slot's particle, and (in the second half) its cell, so that the
  // fix-up reads both at once
  const uint32_t c = keys[i];
  const uint32_t pos = start[c] + rank[i];
  tmp[pos] = uint32_t(i);
  tmp[n + pos] = c;
}

__global__ void __launch_bounds__(256) k_rank_gather(State a, State b, const uint32_t *__restrict__ tmp,
                                                     const uint32_t *__restrict__ start, int64_t n,
                                                     int nspec, uint32_t *__restrict__ slot_of_gid,
                                                     uint32_t *__restrict__ keys_sorted) {
  const int64_t p0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p0 >= n) return;
  const uint32_t q = tmp[p0], c = tmp[n + p0];
  // the particle's state is loaded before its rank is known, so that those
  // loads overlap the rank count's
  const float x = a.x[q], y = a.y[q], z = a.z[q], vx = a.vx[q], vy = a.vy[q], vz = a.vz[q];
  const uint32_t g = a.gid[q], info = a.info[q];
  float cv[kMaxS];
#pragma unroll
  for (int sp = 0; sp < kMaxS; ++sp) cv[sp] = sp < nspec ? a.C[sp * n + q] : 0.f;
  const uint32_t s0 = start[c], s1 = start[c + 1];
  // rank among the cell's entries by previous slot; eight independent loads
  // per round so that their latencies overlap (past the cell end: no entry)
  uint32_t r = 0;
  for (uint32_t m = s0; m < s1; m += 8) {
    uint32_t t[8];
#pragma unroll
    for (uint32_t u = 0; u < 8; ++u) t[u] = m + u < s1 ? tmp[m + u] : 0xffffffffu;
#pragma unroll
    for (int u = 0; u < 8; ++u) r += t[u] < q ? 1u : 0u;
  }
  const uint32_t p = s0 + r;
  b.x[p] = x;
  b.y[p] = y;
  b.z[p] = z;
  b.vx[p] = vx;
  b.vy[p] = vy;
  b.vz[p] = vz;
#pragma unroll
  for (int sp = 0; sp < kMaxS; ++sp)
    if (sp < nspec) b.C[sp * n + p] = cv[sp];
  b.gid[p] = g;
  b.info[p] = info;
  // the id-to-slot map serves the membrane gathers: vertices only (a
  // scattered 4-byte store per solvent particle would cost a write granule)
  if (info_body(info) >= 0) slot_of_gid[g] = p;
  keys_sorted[p] = c;
}

void launch_bin_counting(State src, State dst, const uint32_t *keys, const uint32_t *rank,
                         uint32_t *cell_count, int64_t ncell, uint32_t *cell_start, uint32_t *tmp,
                         uint32_t *tile_sum, int64_t n, int nspec, uint32_t *slot_of_gid,
                         uint32_t *keys_sorted, uint32_t *advance, const MemArgs &membrane,
                         const BoxDev *boxes, const uint32_t *kdev, int kofs, uint32_t *err,
                         hipStream_t st) {
  const int64_t nt = count_scan_tiles(ncell);
  if (nt > 1)  // one tile needs no tile prefix
    hipLaunchKernelGGL(k_count_tiles, dim3(unsigned(nt)), dim3(kScanThreads), 0, st, cell_count,
                       ncell, tile_sum);
  const int eparts = membrane_element_parts(membrane.bond_stride);
  const int64_t nmem = membrane.nrbc > 0 ? int64_t(membrane.nrbc) * eparts : 0;
  hipLaunchKernelGGL(k_count_scan, dim3(unsigned(nt + nmem)), dim3(kScanThreads), 0, st, cell_count,
                     ncell, int(nt), tile_sum, cell_start, membrane, eparts, boxes, src, kdev, kofs,
                     err);
  if (n <= 0) return;
  const dim3 g(unsigned((n + 255) / 256));
  hipLaunchKernelGGL(k_scatter_rank, g, dim3(256), 0, st, keys, rank, cell_start, n, tmp, advance);
  hipLaunchKernelGGL(k_rank_gather, g, dim3(256), 0, st, src, dst, tmp, cell_start, n, nspec,
                     slot_of_gid, keys_sorted);
}

// F, Q are per particle in sorted order: F [n][3], Q [n][S].  The last
// kernel of an evaluation: it advances the device step counter to the next
// step's value (every kernel of this evaluation has read it already).
__global__ void __launch_bounds__(256) k_postkick(PairConst pc, State s, float *__restrict__ F,
                                                  const float *__restrict__ Q, int64_t n,
                                                  VertexMap vm, int integrate,
                                                  uint32_t *__restrict__ kdev) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i == 0 && kdev) *kdev += 1u;
  if (i >= n) return;
  (void)close_step(pc, s, F, Q, n, vm, integrate != 0, i, s.info[i]);
}

void launch_postkick(const PairConst &pc, State s, float *F, const float *Q, int64_t n,
                     VertexMap vm, bool integrate, uint32_t *kdev, hipStream_t st) {
  const int64_t nb = n > 0 ? (n + 255) / 256 : 1;
  hipLaunchKernelGGL(k_postkick, dim3(unsigned(nb)), dim3(256), 0, st, pc, s, F, Q, n, vm,
                     int(integrate), kdev);
}

__global__ void k_set_counter(uint32_t *kdev, uint32_t k) { *kdev = k; }

void launch_set_counter(uint32_t *kdev, uint32_t k, hipStream_t st) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, kdev, k);
}

// ------------------------------------------------------------- cell bounds
__global__ void __launch_bounds__(256) k_cell_bounds(const uint32_t *__restrict__ keys, int64_t n,
                                                     int64_t ncell, uint32_t *__restrict__ start) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t k = keys[p];
  const int64_t kp = p ? int64_t(keys[p - 1]) : -1;
  for (int64_t c = kp + 1; c <= k; ++c) start[c] = uint32_t(p);
  if (p == n - 1)
    for (int64_t c = k + 1; c <= ncell; ++c) start[c] = uint32_t(n);
}

void launch_cell_bounds(const uint32_t *sorted_keys, int64_t n, int64_t ncell,
                        uint32_t *cell_start, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cell_bounds, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, sorted_keys,
                     n, ncell, cell_start);
}

// ------------------------------------------------------------- reorder
__global__ void __launch_bounds__(256) k_reorder(State a, State b, const uint32_t *__restrict__ perm,
                                                 int64_t n, int nspec,
                                                 uint32_t *__restrict__ slot_of_gid) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t q = perm[p];
  b.x[p] = a.x[q];
  b.y[p] = a.y[q];
  b.z[p] = a.z[q];
  b.vx[p] = a.vx[q];
  b.vy[p] = a.vy[q];
  b.vz[p] = a.vz[q];
  for (int sp = 0; sp < nspec; ++sp) b.C[sp * n + p] = a.C[sp * n + q];
  const uint32_t g = a.gid[q], info = a.info[q];
  b.gid[p] = g;
  b.info[p] = info;
  if (info_body(info) >= 0) slot_of_gid[g] = uint32_t(p);  // vertices only
}

void launch_reorder(State src, State dst, const uint32_t *perm, int64_t n, int nspec,
                    uint32_t *slot_of_gid, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_reorder, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, src, dst, perm,
                     n, nspec, slot_of_gid);
}

// ------------------------------------------------------------- diagnostics
// Fixed-order FP64 reduction: block b sums its contiguous kDiagSpan-particle
// span through an LDS tree; a second one-block pass sums the block partials.
constexpr int kDiagThreads = 256;

__global__ void __launch_bounds__(kDiagThreads) k_diag_partial(State s, int64_t n, int nspec,
                                                               double *__restrict__ partial) {
  __shared__ double red[kDiagThreads];
  double acc[kDiagFields];
  for (int f = 0; f < kDiagFields; ++f) acc[f] = 0.0;
  const int64_t b0 = int64_t(blockIdx.x) * kDiagSpan;
  for (int r = 0; r < kDiagSpan / kDiagThreads; ++r) {
    const int64_t i = b0 + r * kDiagThreads + threadIdx.x;
    if (i >= n) break;
    if (!info_frozen(s.info[i])) {
      const double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
      acc[0] += vx;
      acc[1] += vy;
      acc[2] += vz;
      acc[3] += vx * vx + vy * vy + vz * vz;
      acc[4] += 1.0;
    }
    for (int sp = 0; sp < nspec; ++sp) acc[5 + sp] += s.C[sp * n + i];
  }
  for (int f = 0; f < 5 + nspec; ++f) {
    red[threadIdx.x] = acc[f];
    __syncthreads();
    for (int off = kDiagThreads / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[int64_t(blockIdx.x) * kDiagFields + f] = red[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kDiagThreads) k_diag_final(const double *__restrict__ partial,
                                                             int64_t nblocks, int nfields,
                                                             double *__restrict__ out) {
  __shared__ double red[kDiagThreads];
  for (int f = 0; f < nfields; ++f) {
    double a = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += kDiagThreads) a += partial[b * kDiagFields + f];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int off = kDiagThreads / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[f] = red[0];
    __syncthreads();
  }
}

// The reported values from the reduced sums (momentum, kT over the mobile
// particles, totals per species), in the same FP64 operations and order as
// the host finish of tdpd_diagnostics, without contraction, so both give the
// same bits.
__global__ void k_diag_finish(const double *__restrict__ sums, int nspec, double *__restrict__ out) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  const double nm = sums[4];
  out[0] = sums[0];
  out[1] = sums[1];
  out[2] = sums[2];
  out[3] = nm > 1 ? (sums[3] - (sums[0] * sums[0] + sums[1] * sums[1] + sums[2] * sums[2]) / nm) /
                        (3.0 * (nm - 1))
                  : 0.0;
  for (int sp = 0; sp < nspec; ++sp) out[4 + sp] = sums[5 + sp];
}

void launch_diag_finish(const double *sums, int nspec, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(64), 0, st, sums, nspec, out);
}

void launch_diag(State s, int64_t n, int nspec, double *partial, double *out, hipStream_t st) {
  const int64_t nb = n > 0 ? (n + kDiagSpan - 1) / kDiagSpan : 0;
  if (nb > 0)
    hipLaunchKernelGGL(k_diag_partial, dim3(unsigned(nb)), dim3(kDiagThreads), 0, st, s, n, nspec,
                       partial);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, st, partial, nb, 5 + nspec, out);
}

// ------------------------------------------------------------- gid order
// Copy of the state (and F, Q) in gid order: slot p goes to row gid[p].
__global__ void __launch_bounds__(256) k_to_gid_order(State s, int64_t n, int nspec,
                                                      const float *__restrict__ F,
                                                      const float *__restrict__ Q, float *pos,
                                                      float *vel, float *conc, float *Fo, float *Qo) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t g = s.gid[p];
  if (pos) {
    pos[3 * g] = s.x[p];
    pos[3 * g + 1] = s.y[p];
    pos[3 * g + 2] = s.z[p];
  }
  if (vel) {
    vel[3 * g] = s.vx[p];
    vel[3 * g + 1] = s.vy[p];
    vel[3 * g + 2] = s.vz[p];
  }
  if (conc)
    for (int sp = 0; sp < nspec; ++sp) conc[nspec * g + sp] = s.C[sp * n + p];
  if (Fo) {
    Fo[3 * g] = F[3 * p];
    Fo[3 * g + 1] = F[3 * p + 1];
    Fo[3 * g + 2] = F[3 * p + 2];
  }
  if (Qo)
    for (int sp = 0; sp < nspec; ++sp) Qo[nspec * g + sp] = Q[nspec * p + sp];
}

void launch_gid_order(State s, int64_t n, int nspec, const float *F, const float *Q, float *pos,
                      float *vel, float *conc, float *Fo, float *Qo, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_gid_order, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, s, n,
                     nspec, F, Q, pos, vel, conc, Fo, Qo);
}

}  // namespace tdpd
