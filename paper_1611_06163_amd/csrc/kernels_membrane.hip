// kernels_membrane.hip -- RBC membrane terms (Section 2.2) as a kernel of
// its own, one workgroup per cell (membrane_cell.h); used where the pair
// kernel does not take the cells itself (surrogate runs, the simple pair
// kernel).
#include "membrane_cell.h"

namespace tdpd {

constexpr int kMemThreads = 512;

size_t membrane_lds_bytes(int max_nv) { return membrane_cell_lds(max_nv, kMemThreads); }

__global__ void __launch_bounds__(kMemThreads) k_membrane(MemArgs ma, const BoxDev *__restrict__ boxes,
                                                          State s, const uint32_t *__restrict__ kdev,
                                                          uint32_t *err) {
  extern __shared__ double lds_d[];
  membrane_cell(ma, boxes, s, *kdev, err, int(blockIdx.x), reinterpret_cast<char *>(lds_d));
}

void launch_membrane(const MemArgs &ma, const BoxDev *boxes, State s, const uint32_t *kdev,
                     uint32_t *err, size_t lds_bytes, hipStream_t st) {
  if (ma.nrbc <= 0) return;
  hipLaunchKernelGGL(k_membrane, dim3(ma.nrbc), dim3(kMemThreads), lds_bytes, st, ma, boxes, s,
                     kdev, err);
}

}  // namespace tdpd
