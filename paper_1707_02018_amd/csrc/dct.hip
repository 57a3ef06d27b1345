// R by DCT-II diagonalisation (Sec. "Example 1": for reflexive boundaries R
// can be applied in O(N log N)), gfx950.
//
// With half-point reflexive boundaries and a symmetric PSF g (length 2r+1,
// any r: the reflections repeat with period 2N), R along one axis of length N
// is diagonalised by the DCT-II: R = C^{-1} diag(lambda) C with
//   (C x)_k  = sum_n x_n cos(pi k (2n+1) / (2N)),
//   lambda_k = g_0 + 2 sum_{u=1}^{r} g_u cos(pi k u / N).
// The 2-D blur is separable: Y = C_c^{-1} C_r^{-1} (Lambda . C_r C_c X).
//
// Each 1-D transform is one workgroup per row with the row in LDS: the
// DCT-II of a real sequence is the real part of a twiddled N-point complex
// FFT of its even/odd reordering (v_n = x_{2n}, v_{N-1-n} = x_{2n+1}); the
// inverse rebuilds the complex spectrum from y_k and y_{N-k}, untwiddles, runs
// the inverse FFT and undoes the reordering. The FFT is iterative radix-2
// (bit-reversed load, N / 2 butterflies per stage, twiddles from a table
// built once per row in LDS). Columns are transformed
// as rows of a tiled transpose. Passes over the image: row DCT, transpose,
// column DCT + scale + inverse (one kernel), transpose, row inverse.
#include <hip/hip_runtime.h>

#include "aw_internal.hpp"

namespace aw {

constexpr int kDctThreads = 256;

template <typename T>
struct Cx;
template <>
struct Cx<float> {
  using V = float2;
  __device__ static void sincospi_(float x, float* s, float* c) { sincospif(x, s, c); }
};
template <>
struct Cx<double> {
  using V = double2;
  __device__ static void sincospi_(double x, double* s, double* c) { sincospi(x, s, c); }
};

__device__ inline int bitrev(int i, int logN) {
  return logN ? (int)(__brev((unsigned)i) >> (32 - logN)) : 0;
}

// In-place radix-2 FFT of a[0..N) held in bit-reversed order, natural order
// out; sign -1 forward, +1 inverse (unnormalised). tw[j] = (cos, sin)(2 pi j / N),
// j < N / 2; stage s takes exp(sign 2 pi i j / 2^s) = tw[j N / 2^s].
template <typename T>
__device__ void fft_lds(typename Cx<T>::V* a, const typename Cx<T>::V* tw, int N, int logN,
                        T sign) {
  using V = typename Cx<T>::V;
  for (int s = 1; s <= logN; ++s) {
    const int half = 1 << (s - 1);
    __syncthreads();
    for (int b = threadIdx.x; b < N / 2; b += kDctThreads) {
      const int j = b & (half - 1);
      const int i0 = ((b >> (s - 1)) << s) + j, i1 = i0 + half;
      const V t0 = tw[j << (logN - s)];
      const T cs = t0.x, sn = sign * t0.y;
      const V u = a[i0], w = a[i1];
      const V t = {cs * w.x - sn * w.y, cs * w.y + sn * w.x};
      a[i0] = V{u.x + t.x, u.y + t.y};
      a[i1] = V{u.x - t.x, u.y - t.y};
    }
  }
  __syncthreads();
}

// MODE 0: out = C x; MODE 1: out = C^{-1} x; MODE 2: out = C^{-1} (s_row lam . C x)
// with s_row = lam_row[row % rows_per_image]. One workgroup per row of N; in
// may equal out (a row is read whole into LDS before any of it is written).
template <typename T, int MODE>
__global__ __launch_bounds__(kDctThreads) void dct_rows_kernel(int N, int logN, int rows_img,
                                                               const T* in, T* out,
                                                               const T* __restrict__ lam,
                                                               const T* __restrict__ lam_row) {
  using V = typename Cx<T>::V;
  extern __shared__ __align__(16) unsigned char smem[];
  V* a = reinterpret_cast<V*>(smem);
  V* tw = a + N;
  T* yb = reinterpret_cast<T*>(tw + N / 2);
  const long long row = blockIdx.x;
  for (int j = threadIdx.x; j < N / 2; j += kDctThreads) {
    T sn, cs;
    Cx<T>::sincospi_(T(2 * j) / T(N), &sn, &cs);
    tw[j] = V{cs, sn};
  }
  const T* X = in + row * N;
  T* Y = out + row * N;
  const T invN = T(1) / T(N);

  if (MODE != 1) {  // forward: reorder, FFT, twiddle, real part
    for (int n = threadIdx.x; n < N / 2; n += kDctThreads) {
      a[bitrev(n, logN)] = V{X[2 * n], T(0)};
      a[bitrev(N - 1 - n, logN)] = V{X[2 * n + 1], T(0)};
    }
    fft_lds<T>(a, tw, N, logN, T(-1));
    const T sr = MODE == 2 ? lam_row[row % rows_img] : T(1);
    for (int k = threadIdx.x; k < N; k += kDctThreads) {
      T sn, cs;
      Cx<T>::sincospi_(T(k) * T(0.5) * invN, &sn, &cs);
      const T y = a[k].x * cs + a[k].y * sn;
      if (MODE == 0)
        Y[k] = y;
      else
        yb[k] = y * (sr * lam[k]);
    }
  } else {
    for (int k = threadIdx.x; k < N; k += kDctThreads) yb[k] = X[k];
  }
  if (MODE == 0) return;
  __syncthreads();
  // inverse: W_0 = y_0, W_k = y_k - i y_{N-k}; V_k = exp(i pi k / 2N) W_k
  for (int k = threadIdx.x; k < N; k += kDctThreads) {
    const T wr = yb[k], wi = k ? -yb[N - k] : T(0);
    T sn, cs;
    Cx<T>::sincospi_(T(k) * T(0.5) * invN, &sn, &cs);
    a[bitrev(k, logN)] = V{wr * cs - wi * sn, wr * sn + wi * cs};
  }
  fft_lds<T>(a, tw, N, logN, T(1));
  for (int n = threadIdx.x; n < N / 2; n += kDctThreads) {
    Y[2 * n] = a[n].x * invN;
    Y[2 * n + 1] = a[N - 1 - n].x * invN;
  }
}

// out[b][c][r] = in[b][r][c] (rows x cols per image), 32 x 32 tiles.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(int rows, int cols, const T* __restrict__ in,
                                                        T* __restrict__ out) {
  __shared__ T tile[32][33];
  const long long plane = (long long)rows * cols;
  const T* I = in + blockIdx.z * plane;
  T* O = out + blockIdx.z * plane;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + i, c = c0 + tx;
    if (r < rows && c < cols) tile[i][tx] = I[(long long)r * cols + c];
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int c = c0 + i, r = r0 + tx;
    if (r < rows && c < cols) O[(long long)c * rows + r] = tile[tx][i];
  }
}

template <typename T>
static size_t dct_lds(int N) {  // a[N], tw[N / 2], yb[N]
  return sizeof(typename Cx<T>::V) * (size_t)(N + N / 2) + sizeof(T) * (size_t)N;
}

template <typename T, int MODE>
static hipError_t launch_rows(int N, long long nrows, int rows_img, const T* in, T* out,
                              const T* lam, const T* lam_row, hipStream_t s) {
  int logN = 0;
  while ((1 << logN) < N) ++logN;
  const size_t lds = dct_lds<T>(N);
  auto kern = dct_rows_kernel<T, MODE>;
  if (lds >= 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)nrows), dim3(kDctThreads), lds, s, N, logN, rows_img,
                     in, out, lam, lam_row);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_transpose(int rows, int cols, int batch, const T* in, T* out,
                                   hipStream_t s) {
  dim3 grid((cols + 31) / 32, (rows + 31) / 32, batch);
  hipLaunchKernelGGL(transpose_kernel<T>, grid, dim3(256), 0, s, rows, cols, in, out);
  return hipGetLastError();
}

template <typename T>
static hipError_t blur_dct_t(int rows, int cols, int batch, const T* lam_r, const T* lam_c,
                             const T* x, T* y, T* w1, T* w2, hipStream_t s) {
  hipError_t e;
  const long long nr = (long long)batch * rows, nc = (long long)batch * cols;
  // transform along each row (length cols)
  if ((e = launch_rows<T, 0>(cols, nr, rows, x, w1, nullptr, nullptr, s)) != hipSuccess) return e;
  if ((e = launch_transpose<T>(rows, cols, batch, w1, w2, s)) != hipSuccess) return e;
  // along each column (length rows): transform, scale by lam_c[col] lam_r[k], invert
  if ((e = launch_rows<T, 2>(rows, nc, cols, w2, w2, lam_r, lam_c, s)) != hipSuccess) return e;
  if ((e = launch_transpose<T>(cols, rows, batch, w2, w1, s)) != hipSuccess) return e;
  return launch_rows<T, 1>(cols, nr, rows, w1, y, nullptr, nullptr, s);
}

size_t blur_dct_lds(int dtype, int n) { return dtype ? dct_lds<double>(n) : dct_lds<float>(n); }

hipError_t launch_blur_dct(int dtype, int rows, int cols, int batch, const void* lam_r,
                           const void* lam_c, const void* x, void* y, void* w1, void* w2,
                           hipStream_t s) {
  if (dtype)
    return blur_dct_t<double>(rows, cols, batch, static_cast<const double*>(lam_r),
                              static_cast<const double*>(lam_c), static_cast<const double*>(x),
                              static_cast<double*>(y), static_cast<double*>(w1),
                              static_cast<double*>(w2), s);
  return blur_dct_t<float>(rows, cols, batch, static_cast<const float*>(lam_r),
                           static_cast<const float*>(lam_c), static_cast<const float*>(x),
                           static_cast<float*>(y), static_cast<float*>(w1),
                           static_cast<float*>(w2), s);
}

}  // namespace aw
