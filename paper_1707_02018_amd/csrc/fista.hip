// FISTA reductions (gfx950): per-block FP64 partials of ||x||_1 for the exact
// objective, the objective's final combination, and fixed-order partial sums,
// so every objective is bitwise reproducible run to run. The proximal /
// momentum update itself runs in the analysis kernels' epilogue
// (wavelet.hip, ana_tile with PROX).
#include "aw_internal.hpp"

namespace aw {

constexpr int kProxThreads = 256;
constexpr int kProxItems = 8;  // elements per thread per block-iteration

int fista_prox_blocks(long long n) {
  long long b = (n + (long long)kProxThreads * kProxItems - 1) / ((long long)kProxThreads * kProxItems);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
__global__ __launch_bounds__(kProxThreads) void l1_partials_kernel(long long n, const T* __restrict__ x,
                                                                   double* __restrict__ partials) {
  __shared__ double red[kProxThreads / 64];
  const T* X = x + (long long)blockIdx.y * n;
  double l1 = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const T v = X[i];
    l1 += (double)(v < T(0) ? -v : v);
  }
  double v[1] = {l1};
  block_sums<kProxThreads, 1>(v, red);
  if (threadIdx.x == 0) partials[(long long)blockIdx.y * gridDim.x + blockIdx.x] = v[0];
}

hipError_t launch_l1_partials(int dtype, int batch, long long n, const void* x, double* partials,
                              hipStream_t s) {
  dim3 grid(fista_prox_blocks(n), batch);
  if (dtype)
    hipLaunchKernelGGL(l1_partials_kernel<double>, grid, dim3(kProxThreads), 0, s, n,
                       static_cast<const double*>(x), partials);
  else
    hipLaunchKernelGGL(l1_partials_kernel<float>, grid, dim3(kProxThreads), 0, s, n,
                       static_cast<const float*>(x), partials);
  return hipGetLastError();
}

__global__ void objective_finalize_kernel(int batch, double lambda, double* obj) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch) obj[3 * i + 2] = obj[3 * i] + lambda * obj[3 * i + 1];
}

hipError_t launch_objective_finalize(int batch, double lambda, double* obj, hipStream_t s) {
  hipLaunchKernelGGL(objective_finalize_kernel, dim3((batch + 63) / 64), dim3(64), 0, s, batch,
                     lambda, obj);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void reduce_partials_kernel(int nparts, const double* __restrict__ p,
                                                              double scale, double* __restrict__ out,
                                                              int out_stride, int out_off) {
  __shared__ double red[256 / 64];
  const double* P = p + (long long)blockIdx.x * nparts;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nparts; i += 256) v[0] += P[i];
  block_sums<256, 1>(v, red);
  if (threadIdx.x == 0) out[(long long)blockIdx.x * out_stride + out_off] = scale * v[0];
}

hipError_t launch_reduce_partials(int batch, int nparts, const double* partials, double scale,
                                  double* out, int out_stride, int out_off, hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(batch), dim3(256), 0, s, nparts, partials, scale,
                     out, out_stride, out_off);
  return hipGetLastError();
}

}  // namespace aw
