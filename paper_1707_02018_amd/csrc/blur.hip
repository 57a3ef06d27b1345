// Separable blur R with half-point reflexive boundaries and its structural
// adjoint R^* (Sec. "Example 1"), gfx950.
//
// With the reflexive extension x^[q] = x[refl(q)], one dimension reads
//   (R x)[p]   = sum_u g[u] x^[p - u]                       (convolution)
//   (R^* y)[p] = sum_{m : refl(m) = p} sum_u g[u] y[m + u]  (correlation on the
//                extended domain, halo folded back onto its preimages).
// Writing the folded terms against the reflected window q = p - r + k, a
// sample reached through an even number of reflections (every sample inside
// the image) carries the correlation tap g[k - r], one reached through an odd
// number carries the convolution tap g[r - k]. So
//   (R^* y)[p] = sum_k t[k] y^[q] + sum_{k : q odd} (t[2r - k] - t[k]) y^[q],
// with t the correlation taps: the reflected window of R plus a correction on
// the at most r reflected samples of border outputs, which vanishes for a
// symmetric PSF (then R^* = R).
//
// A workgroup owns a TR x TC output tile and stages the reflected
// (TR+2r) x (TC+2r) window in LDS: interior tiles with 16-byte direct-to-LDS
// loads (global_load_lds_dwordx4: no registers, no LDS write instructions), border
// tiles through per-row / per-column reflection tables. The column pass writes
// TR+2r rows of TC filtered values (VW outputs per thread from 16-byte LDS
// reads); the row pass walks each column in chunks of four outputs. An optional
// epilogue subtracts b and emits deterministic per-tile FP64 partials of
// 1/2 ||R x - b||^2 for FISTA.
#include "aw_internal.hpp"

namespace aw {

// Tile shapes; variant 1 halves the rows. NT = 512 threads.
template <typename T, int VAR = 0>
struct BlurCfg;
template <int VAR>
struct BlurCfg<float, VAR> {
  static constexpr int TR = 64 >> VAR, TC = 64, VW = 4, NT = 512;
  using V = float4;
};
template <int VAR>
struct BlurCfg<double, VAR> {
  static constexpr int TR = 32 >> VAR, TC = 32, VW = 2, NT = 512;
  using V = double2;
};

template <typename T, int R, bool ADJ, int VAR>
__device__ __forceinline__ void blur_tile(const BlurArgs<T>& a, const T* __restrict__ X,
                                          T* __restrict__ Y, const T* __restrict__ SUB,
                                          double* __restrict__ part_out, int bx, int by, int img) {
  using Cfg = BlurCfg<T, VAR>;
  using V = typename Cfg::V;
  constexpr int TR = Cfg::TR, TC = Cfg::TC, VW = Cfg::VW, NT = Cfg::NT;
  constexpr int WR = TR + 2 * R;                       // window rows
  constexpr int WC = TC + 2 * R;                       // window cols
  constexpr int RA = ((R + VW - 1) / VW) * VW;         // aligned left halo
  constexpr int OFF = RA - R;                          // sx column of window column 0
  constexpr int SXS = TC + 2 * RA;                     // sx row: global columns c0-RA .. c0+TC+RA
  constexpr int NV = (OFF + VW + 2 * R + VW - 1) / VW; // vectors read per column-pass item
  constexpr int K = 2 * R + 1;
  __shared__ __align__(16) T sx[WR * SXS];
  __shared__ __align__(16) T sh[WR * TC];
  __shared__ int rtab[WR], ctab[WC];
  __shared__ double red[NT / 64];

  const int N = a.rows, M = a.cols;
  const int r0 = by * TR, c0 = bx * TC;
  const long long plane = (long long)N * M;
  const T* Xi = X + img * plane;
  T t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = a.taps[k];

  const bool interior = (r0 >= R) && (r0 + TR + R <= N) && (c0 >= R) && (c0 + TC + R <= M);

  // step-3 ownership (thread = one column, RB consecutive output rows); with
  // SUB, the thread's b values are fetched first so their latency overlaps
  // the window staging
  constexpr int RG = NT / TC;  // row groups
  constexpr int RB = TR / RG;  // rows per thread
  const int pc = threadIdx.x % TC;
  const int rg = threadIdx.x / TC;
  const int p_c = c0 + pc;
  T bsub[RB];
  if (SUB) {
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int p_r = r0 + rg * RB + i;
      bsub[i] = (p_r < N && p_c < M) ? SUB[img * plane + (long long)p_r * M + p_c] : T(0);
    }
  }

  // 1. stage the reflected window: rows r0-R .. r0+TR+R, cols c0-R .. c0+TC+R
  //    (sx holds the aligned columns c0-RA .. c0+TC+RA: window column j at
  //    sx column j + OFF)
  constexpr int WCV = SXS / VW;  // vectors per sx row
  if (interior && (M % VW) == 0) {
    // interior: the 16-byte vectors go from memory straight to LDS, vector
    // idx of sx (row-major, no padding) from lane idx % 64 of a wave
    // instruction that writes 64 consecutive vectors
    constexpr int NVEC = WR * WCV;
    constexpr int IT = (NVEC + NT - 1) / NT;
    const int wbase = threadIdx.x & ~63;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < NVEC) {
        const int i = idx / WCV, jv = idx - (idx / WCV) * WCV;
        __builtin_amdgcn_global_load_lds(
            static_cast<const void*>(Xi + (long long)(r0 - R + i) * M + (c0 - RA) + jv * VW),
            (__attribute__((address_space(3))) void*)(sx + (wbase + it * NT) * VW), 16, 0, 0);
      }
    }
  } else {
    for (int i = threadIdx.x; i < WR; i += NT) rtab[i] = refl_idx(r0 - R + i, N);
    for (int j = threadIdx.x; j < WC; j += NT) ctab[j] = refl_idx(c0 - R + j, M);
    __syncthreads();
    constexpr int IT = (WR * WC + NT - 1) / NT;  // every load issued before any LDS write
    T v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < WR * WC) {
        const int i = idx / WC, j = idx - (idx / WC) * WC;
        v[it] = Xi[(long long)rtab[i] * M + ctab[j]];
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < WR * WC) {
        const int i = idx / WC, j = idx - (idx / WC) * WC;
        sx[i * SXS + OFF + j] = v[it];
      }
    }
  }
  __syncthreads();

  // 2. filter along columns: sh[i][pc] = sum_k t[k] sx[i][pc + k]
  constexpr int QV = TC / VW;
  for (int item = threadIdx.x; item < WR * QV; item += NT) {
    const int i = item / QV, q = item - (item / QV) * QV;
    const T* row = sx + i * SXS + q * VW;
    T w[NV * VW];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      using NV16 = T __attribute__((ext_vector_type(VW)));
      NV16 vv = *reinterpret_cast<const NV16*>(row + v * VW);
      // with the window off the vector grid (OFF > 0) the compiler would
      // split the first and last 16-byte reads into narrower ones for the
      // elements used; an empty asm that takes the whole vector keeps them
      // single 16-byte reads
      if constexpr (OFF > 0) asm volatile("" : "+v"(vv));
      const T* e = reinterpret_cast<const T*>(&vv);
#pragma unroll
      for (int u = 0; u < VW; ++u) w[v * VW + u] = e[u];
    }
    V ov;
    T* o = reinterpret_cast<T*>(&ov);
#pragma unroll
    for (int u = 0; u < VW; ++u) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < K; ++k) acc += t[k] * w[OFF + u + k];
      o[u] = acc;
    }
    *reinterpret_cast<V*>(sh + i * TC + q * VW) = ov;
  }
  const bool fix = ADJ && !interior && !a.symmetric;
  if (fix) {  // R^* border columns: odd-reflection samples take the convolution tap
    __syncthreads();
    for (int item = threadIdx.x; item < WR * TC; item += NT) {
      const int i = item / TC, pc = item - (item / TC) * TC;
      const int p = c0 + pc;
      if (p >= M || (p >= R && p < M - R)) continue;
      T acc = T(0);
#pragma unroll 1
      for (int k = 0; k < K; ++k)
        if (refl_odd(p - R + k, M))
          acc += (a.taps[K - 1 - k] - a.taps[k]) * sx[i * SXS + OFF + pc + k];
      sh[i * TC + pc] += acc;
    }
  }
  __syncthreads();

  // 3. filter along rows: each thread owns one column and RB output rows,
  //    walked in chunks of four
  constexpr int CR = RB < 4 ? RB : 4;
  T* Yi = Y + img * plane;
  double part = 0.0;
  // one chunk of CR output rows from window row offset lr; bs = the chunk's
  // b values (SUB only)
  auto chunk = [&](int lr, const T* bs) {
    T hw[CR + 2 * R];
#pragma unroll
    for (int i = 0; i < CR + 2 * R; ++i) hw[i] = sh[(lr + i) * TC + pc];
#pragma unroll
    for (int i = 0; i < CR; ++i) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < K; ++k) acc += t[k] * hw[i + k];
      const int p_r = r0 + lr + i;
      if (fix && (p_r < R || p_r >= N - R)) {
#pragma unroll 1
        for (int k = 0; k < K; ++k)
          if (refl_odd(p_r - R + k, N))
            acc += (a.taps[K - 1 - k] - a.taps[k]) * sh[(lr + i + k) * TC + pc];
      }
      if (p_r < N && p_c < M) {
        const long long off = (long long)p_r * M + p_c;
        if (bs) {
          acc -= bs[i];
          part += 0.5 * (double)acc * (double)acc;
        }
        Yi[off] = acc;
      }
    }
  };
  if (SUB) {  // unrolled, so the prefetched b values stay in registers
#pragma unroll
    for (int c = 0; c < RB; c += CR) chunk(rg * RB + c, bsub + c);
  } else {
#pragma unroll 1
    for (int c = 0; c < RB; c += CR) chunk(rg * RB + c, nullptr);
  }
  if (part_out) {
    double v[1] = {part};
    block_sums<NT, 1>(v, red);
    if (threadIdx.x == 0) *part_out = v[0];
  }
}

template <typename T, int R, bool ADJ, int VAR>
__global__ __launch_bounds__(512) void blur_tile_kernel(BlurArgs<T> a, const T* __restrict__ X,
                                                        T* __restrict__ Y,
                                                        const T* __restrict__ SUB,
                                                        double* __restrict__ partials) {
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  double* po = partials
                   ? partials + ((long long)tz * gridDim.y + ty) * gridDim.x + tx
                   : nullptr;
  blur_tile<T, R, ADJ, VAR>(a, X, Y, SUB, po, tx, ty, tz);
}

// One launch over tiles of several images: items[i] covers tiles
// [prefix[i], prefix[i+1]); partials (if any) go to the image's tile slots.
template <typename T, int R, bool ADJ, int VAR>
__global__ __launch_bounds__(512) void blur_batch_kernel(const BlurItem<T>* __restrict__ items,
                                                         const int* __restrict__ prefix, int n,
                                                         const int* __restrict__ active) {
  const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int i = find_item(prefix, n, b);
  const BlurItem<T>& it = items[i];
  if (active && !active[it.image]) return;
  const int t = b - prefix[i];
  double* po = it.partials ? it.partials + t : nullptr;
  blur_tile<T, R, ADJ, VAR>(it.a, it.x, it.y, it.sub, po, t % it.tiles_x, t / it.tiles_x, 0);
}

template <typename T, int VAR = 0>
static dim3 blur_grid(const BlurDesc& b, int batch) {
  return dim3((b.cols + BlurCfg<T, VAR>::TC - 1) / BlurCfg<T, VAR>::TC,
              (b.rows + BlurCfg<T, VAR>::TR - 1) / BlurCfg<T, VAR>::TR, batch);
}

int blur_tiles(int dtype, const BlurDesc& b) {
  dim3 g = dtype ? blur_grid<double>(b, 1) : blur_grid<float>(b, 1);
  return (int)(g.x * g.y);
}


template <typename T, int R, bool ADJ>
static hipError_t launch_r(const BlurDesc& b, int batch, const void* x, void* y, const void* sub,
                           double* partials, hipStream_t s) {
  hipLaunchKernelGGL((blur_tile_kernel<T, R, ADJ, 0>), blur_grid<T>(b, batch), dim3(512), 0, s,
                     make_blur_args<T, ADJ>(b), static_cast<const T*>(x), static_cast<T*>(y),
                     static_cast<const T*>(sub), partials);
  return hipGetLastError();
}

template <typename T, bool ADJ>
static hipError_t launch_t(const BlurDesc& b, int batch, const void* x, void* y, const void* sub,
                           double* partials, hipStream_t s) {
  switch (b.radius) {
#define AW_R(r) \
  case r: return launch_r<T, r, ADJ>(b, batch, x, y, sub, partials, s);
    AW_R(0) AW_R(1) AW_R(2) AW_R(3) AW_R(4) AW_R(5) AW_R(6) AW_R(7) AW_R(8) AW_R(9) AW_R(10)
    AW_R(11) AW_R(12)
#undef AW_R
    default: return hipErrorInvalidValue;
  }
}

int blur_tiles_var(int dtype, int var, const BlurDesc& b, int* tiles_x) {
  dim3 g;
  if (dtype)
    g = var ? blur_grid<double, 1>(b, 1) : blur_grid<double, 0>(b, 1);
  else
    g = var ? blur_grid<float, 1>(b, 1) : blur_grid<float, 0>(b, 1);
  if (tiles_x) *tiles_x = (int)g.x;
  return (int)(g.x * g.y);
}

size_t blur_item_size(int dtype) { return dtype ? sizeof(BlurItem<double>) : sizeof(BlurItem<float>); }

void make_blur_item(int dtype, bool adj, const BlurDesc& b, const void* x, void* y, const void* sub,
                    double* partials, int image, int tiles_x, void* out) {
  if (dtype) {
    BlurItem<double> it{adj ? make_blur_args<double, true>(b) : make_blur_args<double, false>(b),
                        static_cast<const double*>(x), static_cast<double*>(y),
                        static_cast<const double*>(sub), partials, image, tiles_x};
    *static_cast<BlurItem<double>*>(out) = it;
  } else {
    BlurItem<float> it{adj ? make_blur_args<float, true>(b) : make_blur_args<float, false>(b),
                       static_cast<const float*>(x), static_cast<float*>(y),
                       static_cast<const float*>(sub), partials, image, tiles_x};
    *static_cast<BlurItem<float>*>(out) = it;
  }
}

template <typename T, int R, bool ADJ, int VAR>
static hipError_t launch_blur_batch_r(const void* items, const int* prefix, int n, int total,
                                      const int* active, hipStream_t s) {
  hipLaunchKernelGGL((blur_batch_kernel<T, R, ADJ, VAR>), dim3(total), dim3(512), 0, s,
                     static_cast<const BlurItem<T>*>(items), prefix, n, active);
  return hipGetLastError();
}

template <typename T, bool ADJ, int VAR>
static hipError_t launch_blur_batch_t(int radius, const void* items, const int* prefix, int n,
                                      int total, const int* active, hipStream_t s) {
  switch (radius) {
#define AW_R(r) \
  case r: return launch_blur_batch_r<T, r, ADJ, VAR>(items, prefix, n, total, active, s);
    AW_R(0) AW_R(1) AW_R(2) AW_R(3) AW_R(4) AW_R(5) AW_R(6) AW_R(7) AW_R(8) AW_R(9) AW_R(10)
    AW_R(11) AW_R(12)
#undef AW_R
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_blur_batch(int dtype, int radius, bool adj, int var, const void* items,
                             const int* prefix, int n, int total, const int* active,
                             hipStream_t s) {
  if (dtype) return hipErrorInvalidValue;  // batched path: FP32
  if (adj)
    return var ? launch_blur_batch_t<float, true, 1>(radius, items, prefix, n, total, active, s)
               : launch_blur_batch_t<float, true, 0>(radius, items, prefix, n, total, active, s);
  return var ? launch_blur_batch_t<float, false, 1>(radius, items, prefix, n, total, active, s)
             : launch_blur_batch_t<float, false, 0>(radius, items, prefix, n, total, active, s);
}

hipError_t launch_blur(int dtype, const BlurDesc& b, int batch, const void* x, void* y,
                       const void* sub, double* partials, hipStream_t s) {
  return dtype ? launch_t<double, false>(b, batch, x, y, sub, partials, s)
               : launch_t<float, false>(b, batch, x, y, sub, partials, s);
}

hipError_t launch_blur_adjoint(int dtype, const BlurDesc& b, int batch, const void* y, void* x,
                               hipStream_t s) {
  return dtype ? launch_t<double, true>(b, batch, y, x, nullptr, nullptr, s)
               : launch_t<float, true>(b, batch, y, x, nullptr, nullptr, s);
}

}  // namespace aw
