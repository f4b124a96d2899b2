// Small utility kernels: exact widening of fp32 matrices to fp64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace symtd {

// dst[j * ldd + i] = (double) src[j * lds + i] for i < rows, j < cols
__global__ __launch_bounds__(256) void k_widen(const float* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                                               int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / rows, i = e - j * rows;
    dst[j * ldd + i] = (double)src[j * lds + i];
  }
}

void launch_widen(hipStream_t st, const float* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                  int64_t cols) {
  const int64_t total = rows * cols;
  if (total <= 0) return;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_widen, dim3(blocks), dim3(256), 0, st, src, lds, dst, ldd, rows, cols);
}

}  // namespace symtd
