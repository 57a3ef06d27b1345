// Separable Gaussian blur R with half-point reflexive boundaries and its
// structural adjoint R^* (Sec. "Example 1"), gfx950.
//
// R: a workgroup owns a TR x TC output tile, gathers the (TR+2r) x (TC+2r)
// input window through the reflexive index map into LDS, filters along
// columns, then rows. Optional epilogue for FISTA: subtract the observation b
// and emit a deterministic per-tile FP64 partial of 1/2 ||R x - b||^2.
//
// R^*: correlation with the taps on the extended domain m in [-r, N+r),
// followed by the fold of the halo onto its reflexive preimages. Edge tiles
// widen their window to the reflected preimages (same rule as the wavelet
// fold), so interior tiles run the plain correlation.
#include "aw_internal.hpp"

namespace aw {

template <typename T>
struct BlurTile;
template <>
struct BlurTile<float> {
  static constexpr int TR = 32, TC = 64;
};
template <>
struct BlurTile<double> {
  static constexpr int TR = 16, TC = 64;
};

template <typename T>
struct BlurArgs {
  int rows, cols, radius;
  T taps[2 * kMaxRadius + 1];
};

template <typename T>
static BlurArgs<T> make_blur_args(const BlurDesc& b) {
  BlurArgs<T> a{};
  a.rows = b.rows;
  a.cols = b.cols;
  a.radius = b.radius;
  for (int i = 0; i < 2 * b.radius + 1; ++i) a.taps[i] = (T)b.taps[i];
  return a;
}

__device__ inline int refl(int m, int N) {
  const int j = posmod(m, 2 * N);
  return j < N ? j : 2 * N - 1 - j;
}

// Deterministic block sum of one double per thread (fixed tree order).
__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

template <typename T>
__global__ __launch_bounds__(256) void blur_kernel(BlurArgs<T> a, const T* __restrict__ X,
                                                   T* __restrict__ Yout,
                                                   const T* __restrict__ SUB,
                                                   double* __restrict__ partials) {
  constexpr int TR = BlurTile<T>::TR, TC = BlurTile<T>::TC;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  __shared__ T staps[2 * kMaxRadius + 1];
  __shared__ double red[256];

  const int img = blockIdx.z;
  const int N = a.rows, Mc = a.cols, r = a.radius;
  const int r0 = blockIdx.y * TR, r1 = min(r0 + TR, N);
  const int c0 = blockIdx.x * TC, c1 = min(c0 + TC, Mc);
  const int nr = r1 - r0, nc = c1 - c0;
  const int wr = nr + 2 * r, wc = nc + 2 * r;
  T* sx = smem;            // [wr][wc]
  T* sh = smem + wr * wc;  // [wr][TC]
  if (threadIdx.x < 2 * r + 1) staps[threadIdx.x] = a.taps[threadIdx.x];

  const long long plane = (long long)N * Mc;
  const T* Xi = X + img * plane;
  for (int idx = threadIdx.x; idx < wr * wc; idx += blockDim.x) {
    const int i = idx / wc;
    const int j = idx - i * wc;
    sx[idx] = Xi[(long long)refl(r0 - r + i, N) * Mc + refl(c0 - r + j, Mc)];
  }
  __syncthreads();
  // along columns: sh[i][pc] = sum_v g[v] x[i][pc - v]
  for (int idx = threadIdx.x; idx < wr * nc; idx += blockDim.x) {
    const int i = idx / nc;
    const int pc = idx - i * nc;
    const T* row = sx + i * wc + pc + r;
    T acc = T(0);
    for (int v = -r; v <= r; ++v) acc += staps[v + r] * row[-v];
    sh[i * TC + pc] = acc;
  }
  __syncthreads();
  double part = 0.0;
  T* Yi = Yout + img * plane;
  for (int idx = threadIdx.x; idx < nr * nc; idx += blockDim.x) {
    const int pr = idx / nc;
    const int pc = idx - pr * nc;
    const T* col = sh + (pr + r) * TC + pc;
    T acc = T(0);
    for (int u = -r; u <= r; ++u) acc += staps[u + r] * col[-u * TC];
    const long long off = (long long)(r0 + pr) * Mc + (c0 + pc);
    if (SUB) {
      acc -= SUB[img * plane + off];
      part += 0.5 * (double)acc * (double)acc;
    }
    Yi[off] = acc;
  }
  if (partials) {
    const double s = block_sum(part, red);
    if (threadIdx.x == 0)
      partials[(long long)img * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void blur_adj_kernel(BlurArgs<T> a, const T* __restrict__ Y,
                                                       T* __restrict__ Xout) {
  constexpr int TR = BlurTile<T>::TR, TC = BlurTile<T>::TC;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  __shared__ T staps[2 * kMaxRadius + 1];

  const int img = blockIdx.z;
  const int N = a.rows, Mc = a.cols, r = a.radius;
  const int r0 = blockIdx.y * TR, r1 = min(r0 + TR, N);
  const int c0 = blockIdx.x * TC, c1 = min(c0 + TC, Mc);
  int nlo_r, nhi_r, nlo_c, nhi_c;  // windows in n = m + r (m extended index)
  fold_window(r0, r1, N, r, nlo_r, nhi_r);
  fold_window(c0, c1, Mc, r, nlo_c, nhi_c);
  // y window: rows [nlo_r - 2r, nhi_r), cols [nlo_c - 2r, nhi_c)
  const int yo_r = nlo_r - 2 * r, yo_c = nlo_c - 2 * r;
  const int wyr = nhi_r - yo_r, wyc = nhi_c - yo_c;
  const int nc = c1 - c0, nr = r1 - r0;
  T* sy = smem;              // [wyr][wyc]
  T* sz = smem + wyr * wyc;  // [wyr][TC] correlated along columns + column fold
  if (threadIdx.x < 2 * r + 1) staps[threadIdx.x] = a.taps[threadIdx.x];

  const long long plane = (long long)N * Mc;
  const T* Yi = Y + img * plane;
  for (int idx = threadIdx.x; idx < wyr * wyc; idx += blockDim.x) {
    const int i = idx / wyc;
    const int j = idx - i * wyc;
    const int yr = yo_r + i, yc = yo_c + j;
    sy[idx] = (yr >= 0 && yr < N && yc >= 0 && yc < Mc) ? Yi[(long long)yr * Mc + yc] : T(0);
  }
  __syncthreads();
  // sz[i][pc] = sum_{m: refl(m) = c0+pc} sum_v g[v] y[i][m + v]
  for (int idx = threadIdx.x; idx < wyr * nc; idx += blockDim.x) {
    const int i = idx / nc;
    const int pc = idx - i * nc;
    const T* row = sy + i * wyc;
    T acc = T(0);
    for_each_preimage(c0 + pc, Mc, r, SYM, [&](int n) {
      const T* p = row + (n - nlo_c) + r;  // y column (n - r) + v, v in [-r, r]
      for (int v = -r; v <= r; ++v) acc += staps[v + r] * p[v];
    });
    sz[i * TC + pc] = acc;
  }
  __syncthreads();
  T* Xi = Xout + img * plane;
  for (int idx = threadIdx.x; idx < nr * nc; idx += blockDim.x) {
    const int pr = idx / nc;
    const int pc = idx - pr * nc;
    T acc = T(0);
    for_each_preimage(r0 + pr, N, r, SYM, [&](int n) {
      const T* p = sz + ((n - nlo_r) + r) * TC + pc;
      for (int u = -r; u <= r; ++u) acc += staps[u + r] * p[u * TC];
    });
    Xi[(long long)(r0 + pr) * Mc + (c0 + pc)] = acc;
  }
}

template <typename T>
static size_t blur_lds(const BlurDesc& b) {
  constexpr int TR = BlurTile<T>::TR, TC = BlurTile<T>::TC;
  const int r = b.radius;
  const int wr = TR + 2 * r, wc = TC + 2 * r;
  return sizeof(T) * (size_t)(wr * wc + wr * TC);
}

static int adj_max_window(int N, int r, int tile) {
  int mx = 0;
  for (int p0 = 0; p0 < N; p0 += tile) {
    const int p1 = p0 + tile < N ? p0 + tile : N;
    int nlo, nhi;
    fold_window(p0, p1, N, r, nlo, nhi);
    if (nhi - nlo + 2 * r > mx) mx = nhi - nlo + 2 * r;
  }
  return mx;
}

template <typename T>
static size_t blur_adj_lds(const BlurDesc& b) {
  constexpr int TR = BlurTile<T>::TR, TC = BlurTile<T>::TC;
  const int wyr = adj_max_window(b.rows, b.radius, TR);
  const int wyc = adj_max_window(b.cols, b.radius, TC);
  return sizeof(T) * (size_t)(wyr * wyc + wyr * TC);
}

template <typename T>
static dim3 blur_grid(const BlurDesc& b, int batch) {
  return dim3((b.cols + BlurTile<T>::TC - 1) / BlurTile<T>::TC,
              (b.rows + BlurTile<T>::TR - 1) / BlurTile<T>::TR, batch);
}

int blur_tiles(int dtype, const BlurDesc& b) {
  dim3 g = dtype ? blur_grid<double>(b, 1) : blur_grid<float>(b, 1);
  return (int)(g.x * g.y);
}

template <typename T>
static hipError_t set_lds(const void* kern, size_t lds) {
  if (lds > 64 * 1024)
    return hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

template <typename T>
static hipError_t launch_blur_t(const BlurDesc& b, int batch, const void* x, void* y,
                                const void* sub, double* partials, hipStream_t s) {
  const size_t lds = blur_lds<T>(b);
  hipError_t e = set_lds<T>((const void*)blur_kernel<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(blur_kernel<T>, blur_grid<T>(b, batch), dim3(256), lds, s,
                     make_blur_args<T>(b), static_cast<const T*>(x), static_cast<T*>(y),
                     static_cast<const T*>(sub), partials);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_blur_adj_t(const BlurDesc& b, int batch, const void* y, void* x,
                                    hipStream_t s) {
  const size_t lds = blur_adj_lds<T>(b);
  hipError_t e = set_lds<T>((const void*)blur_adj_kernel<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(blur_adj_kernel<T>, blur_grid<T>(b, batch), dim3(256), lds, s,
                     make_blur_args<T>(b), static_cast<const T*>(y), static_cast<T*>(x));
  return hipGetLastError();
}

hipError_t launch_blur(int dtype, const BlurDesc& b, int batch, const void* x, void* y,
                       const void* sub, double* partials, hipStream_t s) {
  return dtype ? launch_blur_t<double>(b, batch, x, y, sub, partials, s)
               : launch_blur_t<float>(b, batch, x, y, sub, partials, s);
}

hipError_t launch_blur_adjoint(int dtype, const BlurDesc& b, int batch, const void* y, void* x,
                               hipStream_t s) {
  return dtype ? launch_blur_adj_t<double>(b, batch, y, x, s)
               : launch_blur_adj_t<float>(b, batch, y, x, s);
}

}  // namespace aw
