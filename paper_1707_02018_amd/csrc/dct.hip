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
// Each 1-D transform is one workgroup per row. The DCT-II of a real sequence
// is the real part of a twiddled N-point complex FFT of its even/odd
// reordering (v_n = x_{2n}, v_{N-1-n} = x_{2n+1}):
//   y_k = Re(exp(-i pi k / 2N) FFT(v)_k);
// the inverse rebuilds the complex spectrum from y_k and y_{N-k}
// (W_0 = y_0, W_k = y_k - i y_{N-k}), multiplies by exp(i pi k / 2N), runs the
// inverse FFT and undoes the reordering (x_{2n} = v_n / N,
// x_{2n+1} = v_{N-1-n} / N).
//
// The FFT is the self-sorting Stockham form (natural order in and out): radix-8
// passes, then one radix-4 or radix-2 pass for the remaining factor; a pass
// takes the R inputs of a butterfly at stride N / R, multiplies them by
// exp(-+ 2 pi i r k / (Ns R)) (k = butterfly mod Ns, Ns = product of the
// earlier radices), runs an R-point DFT in registers and writes its outputs at
// stride Ns. A row is read into LDS with 16-byte loads; the first pass takes
// its inputs from there (reordered, or rebuilt from the spectrum), the complex
// row lives in LDS between passes, and the last pass writes the real outputs
// (post-twiddled, or reordered back) to LDS, from where they are stored with
// 16-byte stores (the forward-only transform stores y_k directly). Twiddles
// come from tables built on the host in FP64 (plan creation): per butterfly
// w, w^2 and w^4 are read and the other powers multiplied out. Columns are
// transformed as rows of a tiled transpose. Passes over the image: row DCT,
// transpose, column DCT + scale + inverse (one kernel), transpose, row inverse.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "aw_internal.hpp"

namespace aw {

// A row of N is transformed by max(N / 8, 64) threads: a radix-R pass gives
// each thread 8 / R butterflies (eight complex values in registers whatever
// the radix).
constexpr int kDctMaxN = 4096;
constexpr int kDctMaxThreads = kDctMaxN / 8;
inline int dct_threads(int N) { return N / 8 > 64 ? N / 8 : 64; }

template <typename T>
struct Cx;
template <>
struct Cx<float> {
  using V = float2;
  static constexpr float kRh = 0.70710678118654752f;  // sqrt(1/2)
};
template <>
struct Cx<double> {
  using V = double2;
  static constexpr double kRh = 0.70710678118654752;
};

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V>
__device__ __forceinline__ V cadd(V a, V b) {
  return V{a.x + b.x, a.y + b.y};
}
template <typename V>
__device__ __forceinline__ V csub(V a, V b) {
  return V{a.x - b.x, a.y - b.y};
}
// a exp(s i pi / 2) with s = +-1: (x, y) -> (-s y, s x)
template <typename V, typename T>
__device__ __forceinline__ V cquarter(V a, T s) {
  return V{-s * a.y, s * a.x};
}

// R-point DFT in place, natural order in and out: U_q = sum_r u_r exp(s 2 pi i r q / R).
template <typename T, int R>
__device__ __forceinline__ void dft(typename Cx<T>::V (&u)[R], T s) {
  using V = typename Cx<T>::V;
  if constexpr (R == 2) {
    const V a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const V e0 = cadd(u[0], u[2]), e1 = csub(u[0], u[2]);
    const V o0 = cadd(u[1], u[3]), o1 = cquarter(csub(u[1], u[3]), s);
    u[0] = cadd(e0, o0);
    u[2] = csub(e0, o0);
    u[1] = cadd(e1, o1);
    u[3] = csub(e1, o1);
  } else {  // R == 8: 4-point DFTs of the even and odd inputs, combined
    V e[4] = {u[0], u[2], u[4], u[6]}, o[4] = {u[1], u[3], u[5], u[7]};
    dft<T, 4>(e, s);
    dft<T, 4>(o, s);
    const T h = Cx<T>::kRh;
    // o_q exp(s 2 pi i q / 8), q = 1, 2, 3
    o[1] = V{h * (o[1].x - s * o[1].y), h * (o[1].y + s * o[1].x)};
    o[2] = cquarter(o[2], s);
    o[3] = V{-h * (o[3].x + s * o[3].y), h * (s * o[3].x - o[3].y)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u[q] = cadd(e[q], o[q]);
      u[q + 4] = csub(e[q], o[q]);
    }
  }
}

// Twiddle powers w^1 .. w^(R-1) of w = exp(s 2 pi i j / N), j = k * step,
// from the table fftw[j] = exp(-2 pi i j / N): w, w^2 and (R = 8) w^4 are
// read, the other powers are their products.
template <typename T, int R>
__device__ __forceinline__ void twiddles(const typename Cx<T>::V* __restrict__ fftw, int j, T s,
                                         typename Cx<T>::V (&w)[R]) {
  using V = typename Cx<T>::V;
  auto tab = [&](int i) {
    V v = fftw[i];
    v.y *= -s;  // the table's conjugate for s = +1
    return v;
  };
  w[0] = V{T(1), T(0)};
  w[1] = tab(j);
  if constexpr (R >= 4) {
    w[2] = tab(2 * j);
    w[3] = cmul(w[1], w[2]);
  }
  if constexpr (R == 8) {
    w[4] = tab(4 * j);
    w[5] = cmul(w[1], w[4]);
    w[6] = cmul(w[2], w[4]);
    w[7] = cmul(w[3], w[4]);
  }
}

// One Stockham pass of radix R on a length-N transform: butterflies
// b = tid + i NT < N / R, i < 8 / R (NT = blockDim.x). For each,
// u_r = load(b + r N / R) times exp(s 2 pi i r k / (Ns R)) (k = b mod Ns), the
// R-point DFT, and store(idx + q Ns, U_q) with idx = (b / Ns) Ns R + k. The
// twiddle reads are issued before the loads. With sync, every input is read
// before a barrier and every output written after it (the pass reads and
// writes the same LDS row).
template <typename T, int R, class Load, class Store>
__device__ __forceinline__ void stockham_pass(int N, int Ns, T s,
                                              const typename Cx<T>::V* __restrict__ fftw,
                                              bool sync, Load&& load, Store&& store) {
  using V = typename Cx<T>::V;
  constexpr int MB = 8 / R;
  const int nb = N / R;
  const int step = N / (Ns * R);
  const int NT = blockDim.x;
  V u[MB][R];
  V w[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = threadIdx.x + i * NT;
    if (b < nb && Ns > 1) twiddles<T, R>(fftw, (b % Ns) * step, s, w[i]);
  }
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = threadIdx.x + i * NT;
    if (b < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) u[i][r] = load(b + r * nb);
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) u[i][r] = cmul(u[i][r], w[i][r]);
      }
    }
  }
  if (sync) __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = threadIdx.x + i * NT;
    if (b < nb) {
      dft<T, R>(u[i], s);
      const int k = b % Ns;
      const int idx = (b / Ns) * Ns * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) store(idx + q * Ns, u[i][q]);
    }
  }
}

// Runs the passes of a length-N transform (radix 8 while at least 8 remains,
// then 4 or 2): the first pass loads through first_load, the last stores
// through last_store, the others go through the LDS row a. sync_first: the
// first pass must read everything before anything is written (its input may
// alias its output).
template <typename T, class FirstLoad, class LastStore>
__device__ __forceinline__ void fft_passes(int N, int logN, T s, const typename Cx<T>::V* fftw,
                                           typename Cx<T>::V* a, bool sync_first,
                                           FirstLoad&& first_load, LastStore&& last_store) {
  using V = typename Cx<T>::V;
  const int np = (logN + 2) / 3;  // passes
  int Ns = 1;
  for (int p = 0; p < np; ++p) {
    const int rem = logN - 3 * p;
    const int R = rem >= 3 ? 8 : (1 << rem);
    const bool first = p == 0, last = p == np - 1;
    auto load = [&](int m) -> V { return first ? first_load(m) : a[m]; };
    auto store = [&](int k, V v) {
      if (last)
        last_store(k, v);
      else
        a[k] = v;
    };
    const bool sync = first ? sync_first : true;
    if (R == 8)
      stockham_pass<T, 8>(N, Ns, s, fftw, sync, load, store);
    else if (R == 4)
      stockham_pass<T, 4>(N, Ns, s, fftw, sync, load, store);
    else
      stockham_pass<T, 2>(N, Ns, s, fftw, sync, load, store);
    if (!last) __syncthreads();
    Ns *= R;
  }
}

// Lengths 2^9 .. 2^12 with the pass structure fixed at compile time: every
// thread has exactly 8 / R butterflies in each pass, and the table twiddles
// of all passes are read into registers once, before the row is staged, so
// their latency is off the chain of dependent passes (MODE 2 reuses them,
// conjugated, for the inverse).
template <int LOGN, int P>
struct PassOf {
  static constexpr int N = 1 << LOGN;
  static constexpr int R = LOGN - 3 * P >= 3 ? 8 : 1 << (LOGN - 3 * P);
  static constexpr int NS = 1 << (3 * P);
  static constexpr int MB = 8 / R;
  static constexpr int NP = (LOGN + 2) / 3;
};

template <typename T>
struct TwPre {
  typename Cx<T>::V v[4][4];  // pass, loaded value
};

template <typename T, int LOGN, int P>
__device__ __forceinline__ void preload_pass(const typename Cx<T>::V* __restrict__ fftw,
                                             TwPre<T>& pre) {
  using Q = PassOf<LOGN, P>;
  if constexpr (P >= 1 && P < Q::NP) {
    constexpr int step = Q::N / (Q::NS * Q::R);
    constexpr int NT = Q::N / 8;
#pragma unroll
    for (int i = 0; i < Q::MB; ++i) {
      const int j = ((threadIdx.x + i * NT) % Q::NS) * step;
      if constexpr (Q::R == 8) {
        pre.v[P][0] = fftw[j];
        pre.v[P][1] = fftw[2 * j];
        pre.v[P][2] = fftw[4 * j];
      } else if constexpr (Q::R == 4) {
        pre.v[P][2 * i] = fftw[j];
        pre.v[P][2 * i + 1] = fftw[2 * j];
      } else {
        pre.v[P][i] = fftw[j];
      }
    }
  }
}

template <typename T, int LOGN>
__device__ __forceinline__ void preload_twiddles(const typename Cx<T>::V* __restrict__ fftw,
                                                 TwPre<T>& pre) {
  preload_pass<T, LOGN, 1>(fftw, pre);
  preload_pass<T, LOGN, 2>(fftw, pre);
  preload_pass<T, LOGN, 3>(fftw, pre);
}

// Pass P of the compile-time structure: inputs from first_load (P = 0) or the
// LDS row, outputs to last_store (last pass) or the LDS row; every input read
// before a barrier, every output written after it.
template <typename T, int LOGN, int P, class FirstLoad, class LastStore>
__device__ __forceinline__ void static_pass(T s, const TwPre<T>& pre, typename Cx<T>::V* a,
                                            FirstLoad&& first_load, LastStore&& last_store) {
  using V = typename Cx<T>::V;
  using Q = PassOf<LOGN, P>;
  constexpr int R = Q::R, MB = Q::MB, NS = Q::NS, NT = Q::N / 8, nb = Q::N / R;
  V u[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = threadIdx.x + i * NT;
#pragma unroll
    for (int r = 0; r < R; ++r) u[i][r] = P == 0 ? first_load(b + r * nb) : a[b + r * nb];
    if constexpr (P > 0) {
      auto tw = [&](int q) {
        V v = pre.v[P][q];
        v.y *= -s;  // exp(s 2 pi i j / N)
        return v;
      };
      V w[R];
      if constexpr (R == 8) {
        w[1] = tw(0);
        w[2] = tw(1);
        w[4] = tw(2);
        w[3] = cmul(w[1], w[2]);
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
      } else if constexpr (R == 4) {
        w[1] = tw(2 * i);
        w[2] = tw(2 * i + 1);
        w[3] = cmul(w[1], w[2]);
      } else {
        w[1] = tw(i);
      }
#pragma unroll
      for (int r = 1; r < R; ++r) u[i][r] = cmul(u[i][r], w[r]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int b = threadIdx.x + i * NT;
    dft<T, R>(u[i], s);
    const int idx = (b / NS) * NS * R + b % NS;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if constexpr (P == Q::NP - 1)
        last_store(idx + q * NS, u[i][q]);
      else
        a[idx + q * NS] = u[i][q];
    }
  }
  if constexpr (P < Q::NP - 1) __syncthreads();
}

template <typename T, int LOGN, class FirstLoad, class LastStore>
__device__ __forceinline__ void static_fft(T s, const TwPre<T>& pre, typename Cx<T>::V* a,
                                           FirstLoad&& first_load, LastStore&& last_store) {
  constexpr int NP = PassOf<LOGN, 0>::NP;
  static_pass<T, LOGN, 0>(s, pre, a, first_load, last_store);
  if constexpr (NP > 1) static_pass<T, LOGN, 1>(s, pre, a, first_load, last_store);
  if constexpr (NP > 2) static_pass<T, LOGN, 2>(s, pre, a, first_load, last_store);
  if constexpr (NP > 3) static_pass<T, LOGN, 3>(s, pre, a, first_load, last_store);
}

// Row in memory <-> LDS (T values) with 16-byte accesses where N allows.
template <typename T>
__device__ __forceinline__ void row_to_lds(const T* __restrict__ X, T* xs, int N) {
  constexpr int VW = 16 / sizeof(T);
  using W = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  if (N % VW == 0) {
    for (int e = threadIdx.x * VW; e < N; e += blockDim.x * VW)
      *reinterpret_cast<W*>(xs + e) = *reinterpret_cast<const W*>(X + e);
  } else {
    for (int e = threadIdx.x; e < N; e += blockDim.x) xs[e] = X[e];
  }
}
template <typename T>
__device__ __forceinline__ void lds_to_row(const T* xs, T* __restrict__ Y, int N) {
  constexpr int VW = 16 / sizeof(T);
  using W = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  if (N % VW == 0) {
    for (int e = threadIdx.x * VW; e < N; e += blockDim.x * VW)
      *reinterpret_cast<W*>(Y + e) = *reinterpret_cast<const W*>(xs + e);
  } else {
    for (int e = threadIdx.x; e < N; e += blockDim.x) Y[e] = xs[e];
  }
}

// MODE 0: out = C x; MODE 1: out = C^{-1} x; MODE 2: out = C^{-1} (s_row lam . C x)
// with s_row = lam_row[row % rows_per_image]. One workgroup per row of N; in
// may equal out; dct_threads(N) threads. fftw[j] = exp(-2 pi i j / N),
// dctw[k] = exp(-i pi k / 2N). The row is read into LDS and written from LDS
// with 16-byte accesses; the reordering happens in LDS. LOGN = log2 N for the
// compile-time pass structure (2^9 .. 2^12), 0 for any length.
template <typename T, int MODE, int LOGN>
__global__ __launch_bounds__(kDctMaxThreads) void dct_rows_kernel(
    int N, int logN, int rows_img, const T* in, T* out, const T* __restrict__ lam,
    const T* __restrict__ lam_row, const typename Cx<T>::V* __restrict__ fftw,
    const typename Cx<T>::V* __restrict__ dctw) {
  using V = typename Cx<T>::V;
  extern __shared__ __align__(16) unsigned char smem[];
  V* a = reinterpret_cast<V*>(smem);  // complex row, N
  // real row (input, spectrum, output) over the first half of a: every pass
  // that reads one and writes the other reads all its inputs before a barrier
  T* xs = reinterpret_cast<T*>(a);
  const long long row = blockIdx.x;
  const T* X = in + row * N;
  T* Y = out + row * N;
  const int half = N / 2;
  TwPre<T> pre;
  if constexpr (LOGN > 0) preload_twiddles<T, LOGN>(fftw, pre);
  // the transform with sign s (inputs through ld, outputs through st)
  auto fft = [&](T s, auto&& ld, auto&& st) {
    if constexpr (LOGN > 0)
      static_fft<T, LOGN>(s, pre, a, ld, st);
    else
      fft_passes<T>(N, logN, s, fftw, a, true, ld, st);
  };

  row_to_lds(X, xs, N);
  __syncthreads();
  if (MODE != 1) {
    const T sr = MODE == 2 ? lam_row[row % rows_img] : T(1);
    fft(
        T(-1),
        [&](int m) -> V { return V{m < half ? xs[2 * m] : xs[2 * N - 1 - 2 * m], T(0)}; },
        [&](int k, V v) {
          const V c = dctw[k];  // (cos, -sin)(pi k / 2N)
          const T y = v.x * c.x - v.y * c.y;
          if (MODE == 0)
            Y[k] = y;
          else
            xs[k] = y * (sr * lam[k]);
        });
    if (MODE == 0) return;
    __syncthreads();
  }
  const T invN = T(1) / T(N);
  fft(
      T(1),
      [&](int m) -> V {
        const T wr = xs[m];
        const T wi = m ? -xs[N - m] : T(0);
        V c = dctw[m];
        c.y = -c.y;  // exp(i pi m / 2N)
        return cmul(V{wr, wi}, c);
      },
      [&](int k, V v) { xs[k < half ? 2 * k : 2 * N - 1 - 2 * k] = v.x * invN; });
  __syncthreads();
  lds_to_row(xs, Y, N);
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

// The same for rows and cols multiples of 64: 64 x 64 tiles through LDS with
// 16-byte loads and stores (the LDS tile is padded by one element per row, so
// the column reads of the store phase spread over the banks).
template <typename T>
__global__ __launch_bounds__(256) void transpose64_kernel(int rows, int cols,
                                                          const T* __restrict__ in,
                                                          T* __restrict__ out) {
  constexpr int VW = 16 / sizeof(T), TV = 64 / VW;  // values per vector, vectors per tile row
  using W = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  __shared__ T tile[64][65];
  const long long plane = (long long)rows * cols;
  const T* I = in + blockIdx.z * plane;
  T* O = out + blockIdx.z * plane;
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
#pragma unroll
  for (int v = threadIdx.x; v < 64 * TV; v += 256) {
    const int i = v / TV, j = (v % TV) * VW;
    const W w = *reinterpret_cast<const W*>(I + (long long)(r0 + i) * cols + c0 + j);
    const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
    for (int u = 0; u < VW; ++u) tile[i][j + u] = e[u];
  }
  __syncthreads();
#pragma unroll
  for (int v = threadIdx.x; v < 64 * TV; v += 256) {
    const int c = v / TV, i = (v % TV) * VW;  // output row c0 + c, columns r0 + i ..
    W w;
    T* e = reinterpret_cast<T*>(&w);
#pragma unroll
    for (int u = 0; u < VW; ++u) e[u] = tile[i + u][c];
    *reinterpret_cast<W*>(O + (long long)(c0 + c) * rows + r0 + i) = w;
  }
}

template <typename T>
static size_t dct_lds(int N) {  // a[N] complex (the real row aliases it)
  return sizeof(typename Cx<T>::V) * (size_t)N;
}

template <typename T, int MODE>
static hipError_t launch_rows(int N, long long nrows, int rows_img, const T* in, T* out,
                              const T* lam, const T* lam_row, const T* fftw, const T* dctw,
                              hipStream_t s) {
  using V = typename Cx<T>::V;
  int logN = 0;
  while ((1 << logN) < N) ++logN;
  const size_t lds = dct_lds<T>(N);
  auto kern = logN == 9    ? dct_rows_kernel<T, MODE, 9>
              : logN == 10 ? dct_rows_kernel<T, MODE, 10>
              : logN == 11 ? dct_rows_kernel<T, MODE, 11>
              : logN == 12 ? dct_rows_kernel<T, MODE, 12>
                           : dct_rows_kernel<T, MODE, 0>;
  if (lds >= 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)nrows), dim3(dct_threads(N)), lds, s, N, logN, rows_img,
                     in, out, lam, lam_row, reinterpret_cast<const V*>(fftw),
                     reinterpret_cast<const V*>(dctw));
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_transpose(int rows, int cols, int batch, const T* in, T* out,
                                   hipStream_t s) {
  if (rows % 64 == 0 && cols % 64 == 0) {
    hipLaunchKernelGGL(transpose64_kernel<T>, dim3(cols / 64, rows / 64, batch), dim3(256), 0, s,
                       rows, cols, in, out);
    return hipGetLastError();
  }
  dim3 grid((cols + 31) / 32, (rows + 31) / 32, batch);
  hipLaunchKernelGGL(transpose_kernel<T>, grid, dim3(256), 0, s, rows, cols, in, out);
  return hipGetLastError();
}

template <typename T>
static hipError_t blur_dct_t(int rows, int cols, int batch, const DctTables& tb, const T* x, T* y,
                             T* w1, T* w2, hipStream_t s) {
  hipError_t e;
  const T* lam_r = static_cast<const T*>(tb.lam_r);
  const T* lam_c = static_cast<const T*>(tb.lam_c);
  const long long nr = (long long)batch * rows, nc = (long long)batch * cols;
  const T *fr = static_cast<const T*>(tb.fft_r), *dr = static_cast<const T*>(tb.dct_r);
  const T *fc = static_cast<const T*>(tb.fft_c), *dc = static_cast<const T*>(tb.dct_c);
  // transform along each row (length cols)
  if ((e = launch_rows<T, 0>(cols, nr, rows, x, w1, nullptr, nullptr, fc, dc, s)) != hipSuccess)
    return e;
  if ((e = launch_transpose<T>(rows, cols, batch, w1, w2, s)) != hipSuccess) return e;
  // along each column (length rows): transform, scale by lam_c[col] lam_r[k], invert
  if ((e = launch_rows<T, 2>(rows, nc, cols, w2, w2, lam_r, lam_c, fr, dr, s)) != hipSuccess)
    return e;
  if ((e = launch_transpose<T>(cols, rows, batch, w2, w1, s)) != hipSuccess) return e;
  return launch_rows<T, 1>(cols, nr, rows, w1, y, nullptr, nullptr, fc, dc, s);
}

size_t blur_dct_lds(int dtype, int n) { return dtype ? dct_lds<double>(n) : dct_lds<float>(n); }

hipError_t launch_blur_dct(int dtype, int rows, int cols, int batch, const DctTables& tb,
                           const void* x, void* y, void* w1, void* w2, hipStream_t s) {
  if (rows > kDctMaxN || cols > kDctMaxN) return hipErrorInvalidValue;
  if (dtype)
    return blur_dct_t<double>(rows, cols, batch, tb, static_cast<const double*>(x),
                              static_cast<double*>(y), static_cast<double*>(w1),
                              static_cast<double*>(w2), s);
  return blur_dct_t<float>(rows, cols, batch, tb, static_cast<const float*>(x),
                           static_cast<float*>(y), static_cast<float*>(w1), static_cast<float*>(w2),
                           s);
}

}  // namespace aw
