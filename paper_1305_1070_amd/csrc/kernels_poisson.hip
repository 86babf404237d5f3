// Vector kernels of the Newton step of the Schroedinger-Poisson problem:
// the Poisson operator's product (CSR, one row per thread), linear
// combinations, and dot products reduced in a fixed order (per-block
// partials, then one block), so every call gives the same bits.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace ndg {

// The caller's CSR is not trusted: row ranges are clamped to [0, nnz) and
// columns outside [0, n) are skipped, so a malformed matrix gives a wrong
// product, never an out-of-bounds access.
__global__ void __launch_bounds__(256) k_spmv(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                                              const double* val, const double* x, double* y) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double acc = 0.0;
    const int64_t q0 = max(rowptr[i], (int64_t)0), q1 = min(rowptr[i + 1], nnz);
    for (int64_t q = q0; q < q1; ++q) {
      const int32_t j = col[q];
      if (j >= 0 && j < n) acc = fma(val[q], x[j], acc);
    }
    y[i] = acc;
  }
}

// out = a x + b y (out may be x or y)
__global__ void __launch_bounds__(256) k_axpby(int64_t n, double a, const double* x, double b, const double* y,
                                               double* out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = a * x[i] + b * y[i];
}

__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

__global__ void __launch_bounds__(256) k_dot_part(int64_t n, const double* x, const double* y, double* part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    acc = fma(x[i], y[i], acc);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_dot_final(const double* part, int nblk, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int q = threadIdx.x; q < nblk; q += 256) acc += part[q];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) *out = s;
}

namespace {
int vec_blocks(int64_t n) { return (int)std::min<int64_t>(kVecBlocks, std::max<int64_t>(1, (n + 255) / 256)); }
}  // namespace

void launch_spmv(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, const double* val,
                 const double* x, double* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_spmv, dim3(vec_blocks(n)), dim3(256), 0, st, n, nnz, rowptr, col, val, x, y);
}

void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpby, dim3(vec_blocks(n)), dim3(256), 0, st, n, a, x, b, y, out);
}

void launch_dot(int64_t n, const double* x, const double* y, double* part, double* out, hipStream_t st) {
  const int nblk = vec_blocks(n);
  hipLaunchKernelGGL(k_dot_part, dim3(nblk), dim3(256), 0, st, n, x, y, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, part, nblk, out);
}

}  // namespace ndg
