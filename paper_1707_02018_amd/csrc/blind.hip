// Multi-channel blind channel estimation with a Huber total variation term
// (Sec. "Example 2", eq. 6), gfx950: the pieces a first-order solver needs
// besides the convolution pair (conv.hip).
//
//   sum_rows   out[n] = sum_c in[c][n], channels in order (the source gradient
//              sum_c H_c^* r_c from per-channel parts)
//   row_sumsq  out[c] = sum_t x[c][t]^2 in FP64 (||r_c||^2)
//   huber_tv   value[b] = sum_j L_delta((D h_b)_j), (D h)_j = h_{j+1} - h_j, and
//              grad[b] += gscale * D^* clip(D h_b, -delta, delta), where
//              (D^* v)_j = v_{j-1} - v_j with v_{-1} = v_{K-1} = 0
//   prox_l1    out = soft(x - step g, thresh) with FP64 stats
//              [sum g (out - x), sum (out - x)^2, sum |out|] for the
//              backtracking test of a proximal gradient step
//
// The vectors are short (channel responses and sources of a few thousand
// samples): one workgroup per row, or one for the whole vector, reduces in a
// fixed order, so every result is bitwise reproducible.
#include "aw_internal.hpp"

namespace aw {

constexpr int kBlindThreads = 256;

template <typename T>
__global__ __launch_bounds__(kBlindThreads) void sum_rows_kernel(int rows, long long n,
                                                                 const T* __restrict__ in,
                                                                 T* __restrict__ out) {
  const long long i = (long long)blockIdx.x * kBlindThreads + threadIdx.x;
  if (i >= n) return;
  T acc = T(0);
  for (int c = 0; c < rows; ++c) acc += in[(long long)c * n + i];
  out[i] = acc;
}

template <typename T>
__global__ __launch_bounds__(kBlindThreads) void row_sumsq_kernel(long long n,
                                                                  const T* __restrict__ x,
                                                                  double* __restrict__ out) {
  __shared__ double red[kBlindThreads / 64];
  const T* X = x + (long long)blockIdx.x * n;
  double v[1] = {0.0};
  for (long long i = threadIdx.x; i < n; i += kBlindThreads) v[0] += (double)X[i] * (double)X[i];
  block_sums<kBlindThreads, 1>(v, red);
  if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

template <typename T>
__global__ __launch_bounds__(kBlindThreads) void huber_tv_kernel(int K, const T* __restrict__ h,
                                                                 T delta, T gscale,
                                                                 T* __restrict__ grad,
                                                                 double* __restrict__ value) {
  __shared__ double red[kBlindThreads / 64];
  const T* H = h + (long long)blockIdx.x * K;
  T* G = grad ? grad + (long long)blockIdx.x * K : nullptr;
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < K; j += kBlindThreads) {
    // clipped differences on both sides of sample j
    const T dl = j > 0 ? H[j] - H[j - 1] : T(0);
    const T dr = j + 1 < K ? H[j + 1] - H[j] : T(0);
    if (j + 1 < K) {
      const T a = dr < T(0) ? -dr : dr;
      v[0] += (double)(a <= delta ? T(0.5) * dr * dr : delta * (a - T(0.5) * delta));
    }
    if (G) {
      const T pl = dl > delta ? delta : (dl < -delta ? -delta : dl);
      const T pr = dr > delta ? delta : (dr < -delta ? -delta : dr);
      G[j] += gscale * (pl - pr);
    }
  }
  if (value) {
    block_sums<kBlindThreads, 1>(v, red);
    if (threadIdx.x == 0) value[blockIdx.x] = v[0];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlindThreads) void prox_l1_kernel(long long n,
                                                                const T* __restrict__ x,
                                                                const T* __restrict__ g, T step,
                                                                T thresh, T* __restrict__ out,
                                                                double* __restrict__ stats) {
  __shared__ double red[3 * kBlindThreads / 64];
  double v[3] = {0.0, 0.0, 0.0};
  for (long long i = threadIdx.x; i < n; i += kBlindThreads) {
    const T u = x[i] - step * g[i];
    const T o = u > thresh ? u - thresh : (u < -thresh ? u + thresh : T(0));
    out[i] = o;
    const double d = (double)o - (double)x[i];
    v[0] += (double)g[i] * d;
    v[1] += d * d;
    v[2] += (double)(o < T(0) ? -o : o);
  }
  if (stats) {
    block_sums<kBlindThreads, 3>(v, red);
    if (threadIdx.x == 0)
      for (int q = 0; q < 3; ++q) stats[q] = v[q];
  }
}

hipError_t launch_sum_rows(int dtype, int rows, long long n, const void* in, void* out,
                           hipStream_t s) {
  const dim3 grid((unsigned)((n + kBlindThreads - 1) / kBlindThreads));
  if (dtype)
    hipLaunchKernelGGL(sum_rows_kernel<double>, grid, dim3(kBlindThreads), 0, s, rows, n,
                       static_cast<const double*>(in), static_cast<double*>(out));
  else
    hipLaunchKernelGGL(sum_rows_kernel<float>, grid, dim3(kBlindThreads), 0, s, rows, n,
                       static_cast<const float*>(in), static_cast<float*>(out));
  return hipGetLastError();
}

hipError_t launch_row_sumsq(int dtype, int rows, long long n, const void* x, double* out,
                            hipStream_t s) {
  if (dtype)
    hipLaunchKernelGGL(row_sumsq_kernel<double>, dim3(rows), dim3(kBlindThreads), 0, s, n,
                       static_cast<const double*>(x), out);
  else
    hipLaunchKernelGGL(row_sumsq_kernel<float>, dim3(rows), dim3(kBlindThreads), 0, s, n,
                       static_cast<const float*>(x), out);
  return hipGetLastError();
}

hipError_t launch_huber_tv(int dtype, int batch, int K, const void* h, double delta,
                           double gscale, void* grad, double* value, hipStream_t s) {
  if (dtype)
    hipLaunchKernelGGL(huber_tv_kernel<double>, dim3(batch), dim3(kBlindThreads), 0, s, K,
                       static_cast<const double*>(h), delta, gscale, static_cast<double*>(grad),
                       value);
  else
    hipLaunchKernelGGL(huber_tv_kernel<float>, dim3(batch), dim3(kBlindThreads), 0, s, K,
                       static_cast<const float*>(h), (float)delta, (float)gscale,
                       static_cast<float*>(grad), value);
  return hipGetLastError();
}

hipError_t launch_prox_l1(int dtype, long long n, const void* x, const void* g, double step,
                          double thresh, void* out, double* stats, hipStream_t s) {
  if (dtype)
    hipLaunchKernelGGL(prox_l1_kernel<double>, dim3(1), dim3(kBlindThreads), 0, s, n,
                       static_cast<const double*>(x), static_cast<const double*>(g), step,
                       thresh, static_cast<double*>(out), stats);
  else
    hipLaunchKernelGGL(prox_l1_kernel<float>, dim3(1), dim3(kBlindThreads), 0, s, n,
                       static_cast<const float*>(x), static_cast<const float*>(g), (float)step,
                       (float)thresh, static_cast<float*>(out), stats);
  return hipGetLastError();
}

}  // namespace aw
