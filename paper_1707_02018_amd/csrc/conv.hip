// Blind-channel convolution adjoint pair (Sec. "Example 2"), gfx950.
//
//   resid  = h * s - x_obs          (full linear convolution, length K+N-1)
//   grad_s = H^* resid: grad_s[n] = sum_{k<K} h[k] resid[n+k]
//   grad_h = S^* resid: grad_h[n] = sum_{k<N} s[k] resid[k+n]
//
// resid and grad_s are sliding dot products with the short filter h: each
// thread owns 8 consecutive outputs and slides a 15-entry register window
// over the signal staged in LDS, so every LDS read feeds 8 FMAs.
// grad_h has few outputs (K lags) and long sums: a workgroup per pair splits
// the k range into slices, each thread keeps 8 lags in registers with the
// same sliding window, and slices are combined in a fixed order.
#include "aw_internal.hpp"

namespace aw {

constexpr int kConvThreads = 256;
constexpr int kConvOut = 8;                              // outputs per thread
constexpr int kConvTile = kConvThreads * kConvOut;       // outputs per block
constexpr int kConvKC = 256;                             // filter taps per LDS chunk

// y[t] = sum_k h[k] x[t - k] - sub[t], t < T (x zero outside [0, nx); pair p
// reads x + p * x_stride: 0 shares one signal across the batch)
template <typename T>
__global__ __launch_bounds__(kConvThreads) void conv_full_kernel(int K, int nx, int Tlen,
                                                                 long long x_stride,
                                                                 const T* __restrict__ h,
                                                                 const T* __restrict__ x,
                                                                 const T* __restrict__ sub,
                                                                 T* __restrict__ y) {
  __shared__ T sh[kConvKC];
  __shared__ T sx[kConvTile + kConvKC + 8];
  const int pair = blockIdx.y;
  const T* H = h + (long long)pair * K;
  const T* X = x + (long long)pair * x_stride;
  const int t0 = blockIdx.x * kConvTile;
  const int tb = threadIdx.x * kConvOut;
  T acc[kConvOut];
#pragma unroll
  for (int i = 0; i < kConvOut; ++i) acc[i] = T(0);

  for (int k0 = 0; k0 < K; k0 += kConvKC) {
    const int kc = min(kConvKC, ((K - k0 + 7) / 8) * 8);
    // window of x: indices [t0 - k0 - kc + 1, t0 + kConvTile - k0)
    const int xo = t0 - k0 - kc + 1;
    __syncthreads();
    for (int i = threadIdx.x; i < kc; i += kConvThreads) sh[i] = (k0 + i < K) ? H[k0 + i] : T(0);
    for (int i = threadIdx.x; i < kConvTile + kc - 1; i += kConvThreads) {
      const int xi = xo + i;
      sx[i] = (xi >= 0 && xi < nx) ? X[xi] : T(0);
    }
    __syncthreads();
    for (int kg = 0; kg < kc; kg += 8) {
      // V[j] = x[t0 + tb - k0 - kg - 7 + j]
      const T* w = sx + (tb - kg + kc - 8);
      T V[15];
#pragma unroll
      for (int j = 0; j < 15; ++j) V[j] = w[j];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const T hk = sh[kg + kk];
#pragma unroll
        for (int i = 0; i < kConvOut; ++i) acc[i] += hk * V[7 + i - kk];
      }
    }
  }
  T* Y = y + (long long)pair * Tlen;
  const T* S = sub ? sub + (long long)pair * Tlen : nullptr;
#pragma unroll
  for (int i = 0; i < kConvOut; ++i) {
    const int t = t0 + tb + i;
    if (t < Tlen) Y[t] = S ? acc[i] - S[t] : acc[i];
  }
}

// g[n] = sum_k h[k] r[n + k], n < N (r has length K + N - 1)
template <typename T>
__global__ __launch_bounds__(kConvThreads) void corr_short_kernel(int K, int N,
                                                                  const T* __restrict__ h,
                                                                  const T* __restrict__ r,
                                                                  T* __restrict__ g) {
  __shared__ T sh[kConvKC];
  __shared__ T sr[kConvTile + kConvKC + 8];
  const int pair = blockIdx.y;
  const int R = K + N - 1;
  const T* H = h + (long long)pair * K;
  const T* Rr = r + (long long)pair * R;
  const int n0 = blockIdx.x * kConvTile;
  const int tb = threadIdx.x * kConvOut;
  T acc[kConvOut];
#pragma unroll
  for (int i = 0; i < kConvOut; ++i) acc[i] = T(0);

  for (int k0 = 0; k0 < K; k0 += kConvKC) {
    const int kc = min(kConvKC, ((K - k0 + 7) / 8) * 8);
    const int ro = n0 + k0;  // window of r: [n0 + k0, n0 + k0 + kConvTile + kc - 1)
    __syncthreads();
    for (int i = threadIdx.x; i < kc; i += kConvThreads) sh[i] = (k0 + i < K) ? H[k0 + i] : T(0);
    for (int i = threadIdx.x; i < kConvTile + kc - 1; i += kConvThreads) {
      const int ri = ro + i;
      sr[i] = (ri < R) ? Rr[ri] : T(0);
    }
    __syncthreads();
    for (int kg = 0; kg < kc; kg += 8) {
      const T* w = sr + tb + kg;  // V[j] = r[n0 + tb + k0 + kg + j]
      T V[15];
#pragma unroll
      for (int j = 0; j < 15; ++j) V[j] = w[j];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const T hk = sh[kg + kk];
#pragma unroll
        for (int i = 0; i < kConvOut; ++i) acc[i] += hk * V[i + kk];
      }
    }
  }
  T* G = g + (long long)pair * N;
#pragma unroll
  for (int i = 0; i < kConvOut; ++i) {
    const int n = n0 + tb + i;
    if (n < N) G[n] = acc[i];
  }
}

// g[n] = sum_{k<N} s[k] r[k + n] for n in a block of 128 lags (pair p reads
// s + p * s_stride).
constexpr int kLagThreads = 512;
constexpr int kLagGroups = 16;                          // 8 lags each -> 128 lags
constexpr int kLagSlices = kLagThreads / kLagGroups;    // 32 k-slices
constexpr int kLagBlock = kLagGroups * 8;               // 128 lags
template <typename T>
struct LagCfg {
  static constexpr int slice = sizeof(T) == 4 ? 128 : 64;  // k per slice per chunk
  static constexpr int chunk = kLagSlices * slice;
};

template <typename T>
__global__ __launch_bounds__(kLagThreads) void corr_long_kernel(int K, int N, long long s_stride,
                                                                const T* __restrict__ s,
                                                                const T* __restrict__ r,
                                                                T* __restrict__ g) {
  constexpr int SL = LagCfg<T>::slice, CH = LagCfg<T>::chunk;
  static_assert(2 * CH + kLagBlock + 8 >= kLagSlices * kLagBlock, "reduction buffer fits");
  __shared__ T buf[2 * CH + kLagBlock + 8];
  T* ss = buf;       // [CH] s chunk
  T* sr = buf + CH;  // [CH + kLagBlock + 8] r chunk
  const int pair = blockIdx.y;
  const int R = K + N - 1;
  const T* S = s + (long long)pair * s_stride;
  const T* Rr = r + (long long)pair * R;
  const int n0 = blockIdx.x * kLagBlock;
  const int lg = threadIdx.x % kLagGroups;
  const int ks = threadIdx.x / kLagGroups;
  T acc[8];
#pragma unroll
  for (int l = 0; l < 8; ++l) acc[l] = T(0);

  // The grid holds one workgroup per pair and lag block (256 at the benchmark
  // shape, one per CU), so nothing else hides the latency of the chunk loads:
  // the next chunk is fetched into registers while the current one is used.
  constexpr int QS = CH / kLagThreads;
  constexpr int RW = CH + kLagBlock + 7;
  constexpr int QR = (RW + kLagThreads - 1) / kLagThreads;
  static_assert(CH % kLagThreads == 0, "s chunk splits evenly over the threads");
  T ps[QS], pr[QR];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int q = 0; q < QS; ++q) {
      const int i = threadIdx.x + q * kLagThreads;
      ps[q] = (c0 + i < N) ? S[c0 + i] : T(0);
    }
#pragma unroll
    for (int q = 0; q < QR; ++q) {
      const int i = threadIdx.x + q * kLagThreads;
      const int ri = c0 + n0 + i;
      pr[q] = (i < RW && ri < R) ? Rr[ri] : T(0);
    }
  };
  fetch(0);
  for (int c0 = 0; c0 < N; c0 += CH) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QS; ++q) ss[threadIdx.x + q * kLagThreads] = ps[q];
#pragma unroll
    for (int q = 0; q < QR; ++q) {
      const int i = threadIdx.x + q * kLagThreads;
      if (i < RW) sr[i] = pr[q];
    }
    __syncthreads();
    if (c0 + CH < N) fetch(c0 + CH);
    const int kb = ks * SL;
    for (int kg = 0; kg < SL; kg += 8) {
      T V[15], Sv[8];
#pragma unroll
      for (int j = 0; j < 15; ++j) V[j] = sr[kb + kg + 8 * lg + j];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) Sv[kk] = ss[kb + kg + kk];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
#pragma unroll
        for (int l = 0; l < 8; ++l) acc[l] += Sv[kk] * V[kk + l];
    }
  }
  __syncthreads();
  T* red = buf;  // [kLagSlices][kLagBlock], reuses the staging buffers
#pragma unroll
  for (int l = 0; l < 8; ++l) red[ks * kLagBlock + 8 * lg + l] = acc[l];
  __syncthreads();
  if (threadIdx.x < kLagBlock) {
    T sum = T(0);
    for (int q = 0; q < kLagSlices; ++q) sum += red[q * kLagBlock + threadIdx.x];
    const int n = n0 + threadIdx.x;
    if (n < K) g[(long long)pair * K + n] = sum;
  }
}

template <typename T>
static hipError_t launch_conv_t(int batch, int K, int N, long long s_stride, const void* h,
                                const void* s, const void* x_obs, void* resid, void* grad_h,
                                void* grad_s, hipStream_t st) {
  const int R = K + N - 1;
  hipLaunchKernelGGL(conv_full_kernel<T>, dim3((R + kConvTile - 1) / kConvTile, batch),
                     dim3(kConvThreads), 0, st, K, N, R, s_stride, static_cast<const T*>(h),
                     static_cast<const T*>(s), static_cast<const T*>(x_obs),
                     static_cast<T*>(resid));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (grad_s) {
    hipLaunchKernelGGL(corr_short_kernel<T>, dim3((N + kConvTile - 1) / kConvTile, batch),
                       dim3(kConvThreads), 0, st, K, N, static_cast<const T*>(h),
                       static_cast<const T*>(resid), static_cast<T*>(grad_s));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (grad_h) {
    hipLaunchKernelGGL(corr_long_kernel<T>, dim3((K + kLagBlock - 1) / kLagBlock, batch),
                       dim3(kLagThreads), 0, st, K, N, s_stride, static_cast<const T*>(s),
                       static_cast<const T*>(resid), static_cast<T*>(grad_h));
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_conv_pair(int dtype, int batch, int K, int N, const void* h, const void* s,
                            const void* x_obs, void* resid, void* grad_h, void* grad_s,
                            hipStream_t st, bool shared_s) {
  const long long ss = shared_s ? 0 : N;
  return dtype ? launch_conv_t<double>(batch, K, N, ss, h, s, x_obs, resid, grad_h, grad_s, st)
               : launch_conv_t<float>(batch, K, N, ss, h, s, x_obs, resid, grad_h, grad_s, st);
}

}  // namespace aw
