// A = R W with the finest synthesis level fused into the blur (opt-in entry
// aw_apply_A_fused; FISTA uses the separate kernels, which measured faster).
//
// A workgroup owns a TR x TC tile of the output. It synthesises the finest
// wavelet level (W's last step, E^dagger Phi^* of the level-1 subbands) over
// the rows and columns the tile's blur window reaches (tile + PSF radius,
// clipped to the image), scattering every value straight into the reflected
// LDS window the blur reads: an image position lands in each window slot
// whose half-point reflection it is. The blur then runs as in blur.hip
// (column pass, row pass) and optionally subtracts b. The full-resolution
// W x never reaches memory, which saves one image write and one image read.
// The cost: the window's halo is synthesised by every tile that needs it,
// and the larger LDS footprint lowers the resident workgroups.
//
// The synthesised values and the blur arithmetic are those of the separate
// kernels, so the result is bitwise identical to synthesis followed by blur.
//
// A^* = W^* R^* with the blur adjoint fused into the finest analysis level
// (opt-in entry aw_apply_A_adjoint_fused): each half-height analysis tile
// computes R^* r over the image samples its window reads and analyses them
// from LDS (ana_tile with a blur radius), so R^* r never reaches memory; the
// coarser levels run as in aw_apply_A_adjoint. Bitwise equal to the
// two-kernel A^*.
#include <algorithm>
#include <type_traits>

#include "ana_tile.hpp"
#include "aw_internal.hpp"
#include "synth_tile.hpp"

namespace aw {
namespace {

constexpr int kFTR = 32, kFTC = 64, kFNT = 512;

template <typename T, int R>
struct FusedGeom {
  static constexpr int WR = kFTR + 2 * R, WC = kFTC + 2 * R;
  static constexpr int VW = 16 / sizeof(T);
  static constexpr int SXS = ((WC + VW - 1) / VW) * VW + VW;  // vector-aligned row stride
  static constexpr int SX = WR * SXS;                         // window elements
  static constexpr int SH = WR * kFTC;                        // column-pass elements
};

// Synthesised image value (p, q) -> every window slot (i, j) whose
// reflection is (p, q). Window row i is image row wr0 + i; lengths of at
// least R + 1 reflect each slot that feeds a stored output at most once.
template <typename T>
struct WindowWriter {
  T* sx;
  int sxs, wr0, wc0, WR, WC, N, M;
  __device__ void put(int p, int q, T v) {
    int is[3], js[3], ni = 0, nj = 0;
    const int i0 = p - wr0, i1 = -1 - p - wr0, i2 = 2 * N - 1 - p - wr0;
    if (i0 >= 0 && i0 < WR) is[ni++] = i0;
    if (i1 >= 0 && i1 < WR) is[ni++] = i1;
    if (i2 >= 0 && i2 < WR) is[ni++] = i2;
    const int j0 = q - wc0, j1 = -1 - q - wc0, j2 = 2 * M - 1 - q - wc0;
    if (j0 >= 0 && j0 < WC) js[nj++] = j0;
    if (j1 >= 0 && j1 < WC) js[nj++] = j1;
    if (j2 >= 0 && j2 < WC) js[nj++] = j2;
    for (int a = 0; a < ni; ++a)
      for (int c = 0; c < nj; ++c) sx[is[a] * sxs + js[c]] = v;
  }
  __device__ void one(int r, int c, T v) { put(r, c, v); }
  __device__ void pair(int r, int c, T v0, T v1) {
    put(r, c, v0);
    put(r, c + 1, v1);
  }
};

template <typename T, int L, int BC, int R>
__global__ __launch_bounds__(kFNT) void synth_blur_kernel(SynthLevel d, Taps<T> f, BlurArgs<T> a,
                                                          const T* __restrict__ SUB,
                                                          T* __restrict__ Y) {
  using G = FusedGeom<T, R>;
  using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  constexpr int TR = kFTR, TC = kFTC, NT = kFNT, VW = G::VW, WR = G::WR, SXS = G::SXS;
  constexpr int NV = (VW + 2 * R + VW - 1) / VW;
  constexpr int K = 2 * R + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  T* sx = reinterpret_cast<T*>(smem);
  unsigned char* scratch = smem + sizeof(T) * G::SX;  // synthesis window, then sh
  T* sh = reinterpret_cast<T*>(scratch);

  const int bx = blockIdx.x, by = blockIdx.y, img = blockIdx.z;
  const int N = a.rows, M = a.cols;
  const int r0 = by * TR, c0 = bx * TC;
  const long long plane = (long long)N * M;

  // 1. window slots no stored output reads stay zero
  for (int i = threadIdx.x; i < G::SX; i += NT) sx[i] = T(0);
  __syncthreads();

  // 2. synthesise the finest level over the window's preimage rectangle
  const int y0 = max(0, r0 - R) & ~1, y1 = min(N, r0 + TR + R);
  const int x0 = max(0, c0 - R) & ~1, x1 = min(M, c0 + TC + R);
  WindowWriter<T> wrt{sx, SXS, r0 - R, c0 - R, WR, G::WC, N, M};
  synth_rect<T, L, BC>(d, f, y0, y1, x0, x1, img, scratch, wrt);
  __syncthreads();

  // 3. blur along columns: sh[i][pc] = sum_k t[k] sx[i][pc + k]
  T t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = a.taps[k];
  constexpr int QV = TC / VW;
  for (int item = threadIdx.x; item < WR * QV; item += NT) {
    const int i = item / QV, q = item - (item / QV) * QV;
    const T* row = sx + i * SXS + q * VW;
    T w[NV * VW];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const V vv = *reinterpret_cast<const V*>(row + v * VW);
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
      for (int k = 0; k < K; ++k) acc += t[k] * w[u + k];
      o[u] = acc;
    }
    *reinterpret_cast<V*>(sh + i * TC + q * VW) = ov;
  }
  __syncthreads();

  // 4. blur along rows (each thread one column, RB rows in chunks of four)
  constexpr int RG = NT / TC;
  constexpr int RB = TR / RG;
  constexpr int CR = RB < 4 ? RB : 4;
  const int pc = threadIdx.x % TC;
  const int rg = threadIdx.x / TC;
  const int p_c = c0 + pc;
  T* Yi = Y + img * plane;
  const T* Si = SUB ? SUB + img * plane : nullptr;
#pragma unroll 1
  for (int c = 0; c < RB; c += CR) {
    const int lr = rg * RB + c;
    T hw[CR + 2 * R];
#pragma unroll
    for (int i = 0; i < CR + 2 * R; ++i) hw[i] = sh[(lr + i) * TC + pc];
#pragma unroll
    for (int i = 0; i < CR; ++i) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < K; ++k) acc += t[k] * hw[i + k];
      const int p_r = r0 + lr + i;
      if (p_r < N && p_c < M) {
        const long long off = (long long)p_r * M + p_c;
        if (Si) acc -= Si[off];
        Yi[off] = acc;
      }
    }
  }
}

// Largest coefficient window and preimage length over the tiles of one axis.
template <int L, int BC>
void fused_axis_max(const Axis& ax, int tile, int R, int& nk_max, int& len_max) {
  nk_max = 0;
  len_max = 0;
  for (int p0 = 0; p0 < ax.N; p0 += tile) {
    const int y0 = std::max(0, p0 - R) & ~1, y1 = std::min(ax.N, p0 + tile + R);
    int kw, nk;
    synth_axis_window(y0, y1, ax.N, BC == SYM ? ax.e : 0, L, BC, kw, nk);
    nk_max = std::max(nk_max, nk);
    len_max = std::max(len_max, y1 - y0);
  }
}

template <typename T, int L, int BC, int R>
size_t fused_lds_t(const SynthLevel& d) {
  int nkr, rows, nkc, cols;
  fused_axis_max<L, BC>(d.r, kFTR, R, nkr, rows);
  fused_axis_max<L, BC>(d.c, kFTC, R, nkc, cols);
  const size_t synth = sizeof(T) * (size_t)(4 * nkr * nkc + 2 * rows * nkc);
  const size_t sh = sizeof(T) * (size_t)FusedGeom<T, R>::SH;
  return sizeof(T) * (size_t)FusedGeom<T, R>::SX + std::max(synth, sh);
}

template <typename T, int L, int BC, int R>
hipError_t launch_fused_t(const SynthLevel& d, const double* lo, const BlurDesc& b,
                          const void* sub, void* y, int batch, hipStream_t s, size_t* lds_query) {
  const size_t lds = fused_lds_t<T, L, BC, R>(d);
  if (lds_query) {
    *lds_query = lds;
    return hipSuccess;
  }
  auto kern = synth_blur_kernel<T, L, BC, R>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((b.cols + kFTC - 1) / kFTC, (b.rows + kFTR - 1) / kFTR, batch);
  hipLaunchKernelGGL(kern, grid, dim3(kFNT), lds, s, d, make_taps<T>(lo, L),
                     make_blur_args<T, false>(b), static_cast<const T*>(sub),
                     static_cast<T*>(y));
  return hipGetLastError();
}

template <typename T, int L, int BC>
hipError_t fused_R(const SynthLevel& d, const double* lo, const BlurDesc& b, const void* sub,
                   void* y, int batch, hipStream_t s, size_t* lds) {
  switch (b.radius) {
#define AW_FUSED_R(r) \
  case r: return launch_fused_t<T, L, BC, r>(d, lo, b, sub, y, batch, s, lds);
    AW_FUSED_R(0) AW_FUSED_R(1) AW_FUSED_R(2) AW_FUSED_R(3) AW_FUSED_R(4) AW_FUSED_R(5)
    AW_FUSED_R(6) AW_FUSED_R(7) AW_FUSED_R(8) AW_FUSED_R(9) AW_FUSED_R(10) AW_FUSED_R(11)
    AW_FUSED_R(12)
#undef AW_FUSED_R
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int L>
hipError_t fused_BC(const SynthLevel& d, const double* lo, const BlurDesc& b, const void* sub,
                    void* y, int batch, hipStream_t s, size_t* lds) {
  switch (d.bc) {
    case ZPD: return fused_R<T, L, ZPD>(d, lo, b, sub, y, batch, s, lds);
    case SYM: return fused_R<T, L, SYM>(d, lo, b, sub, y, batch, s, lds);
    case PER: return fused_R<T, L, PER>(d, lo, b, sub, y, batch, s, lds);
    default: return hipErrorInvalidValue;
  }
}

hipError_t fused_dispatch(int L, const SynthLevel& d, const double* lo, const BlurDesc& b,
                          const void* sub, void* y, int batch, hipStream_t s, size_t* lds) {
  switch (L) {
    case 2: return fused_BC<float, 2>(d, lo, b, sub, y, batch, s, lds);
    case 8: return fused_BC<float, 8>(d, lo, b, sub, y, batch, s, lds);
    case 16: return fused_BC<float, 16>(d, lo, b, sub, y, batch, s, lds);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------- R^* fused into analysis level 1
constexpr int kBlurAnaVar = 1;  // half-height tiles: the blur window fits static LDS

template <int L, int BC, int R>
__global__ __launch_bounds__(512) void blur_ana_kernel(AnaLevel d, Taps<float> f,
                                                       BlurArgs<float> a) {
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  ana_tile<float, L, BC, kBlurAnaVar, false, R>(d, f, tx, ty, tz, ProxEpi{}, &a);
}

template <int L, int BC, int R>
hipError_t launch_blur_ana_t(const double* lo, const AnaLevel& d, const BlurDesc& b, int batch,
                             hipStream_t s) {
  using Tile = AnaTile<float, kBlurAnaVar>;
  dim3 grid((d.c.K + Tile::TKC - 1) / Tile::TKC, (d.r.K + Tile::TKR - 1) / Tile::TKR, batch);
  hipLaunchKernelGGL((blur_ana_kernel<L, BC, R>), grid, dim3(Tile::NT), 0, s, d,
                     make_taps<float>(lo, L), make_blur_args<float, true>(b));
  return hipGetLastError();
}

template <int L, int BC>
hipError_t blur_ana_R(const double* lo, const AnaLevel& d, const BlurDesc& b, int batch,
                      hipStream_t s) {
  switch (b.radius) {
#define AW_BLUR_ANA_R(r) \
  case r: return launch_blur_ana_t<L, BC, r>(lo, d, b, batch, s);
    AW_BLUR_ANA_R(0) AW_BLUR_ANA_R(1) AW_BLUR_ANA_R(2) AW_BLUR_ANA_R(3) AW_BLUR_ANA_R(4)
    AW_BLUR_ANA_R(5) AW_BLUR_ANA_R(6) AW_BLUR_ANA_R(7) AW_BLUR_ANA_R(8) AW_BLUR_ANA_R(9)
    AW_BLUR_ANA_R(10) AW_BLUR_ANA_R(11) AW_BLUR_ANA_R(12)
#undef AW_BLUR_ANA_R
    default: return hipErrorInvalidValue;
  }
}

template <int L>
hipError_t blur_ana_BC(const double* lo, const AnaLevel& d, const BlurDesc& b, int batch,
                       hipStream_t s) {
  switch (d.bc) {
    case ZPD: return blur_ana_R<L, ZPD>(lo, d, b, batch, s);
    case SYM: return blur_ana_R<L, SYM>(lo, d, b, batch, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool blur_ana_supported(int L, const AnaLevel& d, const BlurDesc& b) {
  if (d.bc != ZPD && d.bc != SYM) return false;
  if (d.bc == SYM && (d.r.N < d.r.e || d.c.N < d.c.e)) return false;  // two-step fold
  if (L != 2 && L != 8 && L != 16) return false;
  if (b.radius < 0 || b.radius > kMaxRadius) return false;
  return d.r.N == b.rows && d.c.N == b.cols;
}

hipError_t launch_blur_ana(int L, const double* lo, const AnaLevel& d, const BlurDesc& b,
                           int batch, hipStream_t s) {
  switch (L) {
    case 2: return blur_ana_BC<2>(lo, d, b, batch, s);
    case 8: return blur_ana_BC<8>(lo, d, b, batch, s);
    case 16: return blur_ana_BC<16>(lo, d, b, batch, s);
    default: return hipErrorInvalidValue;
  }
}

bool synth_blur_supported(int L, const SynthLevel& d, const BlurDesc& b) {
  if (d.bc != ZPD && d.bc != SYM && d.bc != PER) return false;
  if (d.bc == SYM && (d.r.N < d.r.e || d.c.N < d.c.e)) return false;  // two-step fold
  if (L != 2 && L != 8 && L != 16) return false;
  if (b.radius < 0 || b.radius > kMaxRadius) return false;
  if (d.r.N != b.rows || d.c.N != b.cols) return false;
  if (b.rows < b.radius + 1 || b.cols < b.radius + 1) return false;  // single reflection
  size_t lds = 0;
  if (fused_dispatch(L, d, nullptr, b, nullptr, nullptr, 1, nullptr, &lds) != hipSuccess)
    return false;
  return lds <= 160 * 1024;
}

hipError_t launch_synth_blur(int L, const double* lo, const SynthLevel& d, const BlurDesc& b,
                             const void* sub, void* y, int batch, hipStream_t s) {
  return fused_dispatch(L, d, lo, b, sub, y, batch, s, nullptr);
}

}  // namespace aw
