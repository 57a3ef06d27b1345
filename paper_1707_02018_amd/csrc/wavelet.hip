// One-level 2-D wavelet synthesis and analysis kernels for gfx950.
//
// Synthesis (W = E^dagger Phi^* per level, Sec. "A few signal extensions"):
// a workgroup owns a TR x TC tile of the level's output. It stages the four
// coefficient subbands of the tile's dependency window in LDS, runs the
// column-direction synthesis with the row fold applied per output row, then
// the row-direction synthesis with the column fold, and writes the tile once.
// Edge tiles widen their window to the reflected preimages, so the fold costs
// nothing on interior tiles.
//
// Analysis (W^dagger = Phi E, and the true adjoint W^* = Phi (E^dagger)^*,
// eq. 2): a workgroup owns TKR x TKC coefficients of every band. It gathers
// the extended input window (extension index map and 1/mult weights applied
// during the gather), filters along columns into LDS, then along rows, and
// writes a, H, V, D.
#include <algorithm>
#include <type_traits>

#include "ana_tile.hpp"
#include "aw_internal.hpp"
#include "synth_tile.hpp"

namespace aw {

template <typename T, int L, int BC, int V>
__device__ __forceinline__ void synth_tile(const SynthLevel& d, const Taps<T>& f, int bx, int by,
                                           int img, unsigned char* smem_raw) {
  constexpr int TR = SynthTile<T, V>::TR, TC = SynthTile<T, V>::TC;
  const int r0 = by * TR, r1 = min(r0 + TR, d.r.N);
  const int c0 = bx * TC, c1 = min(c0 + TC, d.c.N);
  if constexpr (sizeof(T) == 4) {
    const SynthWin w = synth_win<L, BC>(d, r0, r1, c0, c1, img);
    if (synth_fast_ok<L, BC, TR, TC>(d, w, static_cast<T*>(d.out) + (long long)img * d.stride_out)) {
      synth_tile_fast<L, BC, TR>(d, f, w, smem_raw);
      return;
    }
  }
  PlaneWriter<T> wr(static_cast<T*>(d.out) + (long long)img * d.stride_out, d.c.N);
  synth_rect<T, L, BC, true>(d, f, r0, r1, c0, c1, img, smem_raw, wr);
}

template <typename T, int L, int BC, int V>
__global__ __launch_bounds__(512) void synth_level_kernel(SynthLevel d, Taps<T> f) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // XCD-aware tile order: each XCD runs a contiguous range of row-major tiles,
  // so the halo rows and columns neighbouring tiles share stay in one L2
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  synth_tile<T, L, BC, V>(d, f, tx, ty, tz, smem_raw);
}

// One launch over tiles of several images (a tile queue): items[i] covers
// tiles [prefix[i], prefix[i+1]) of its image; inactive images return.
template <typename T, int L, int BC, int V>
__global__ __launch_bounds__(512) void synth_batch_kernel(const SynthItem<T>* __restrict__ items,
                                                          const int* __restrict__ prefix, int n,
                                                          const int* __restrict__ active) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int i = find_item(prefix, n, b);
  const SynthItem<T>& it = items[i];
  if (active && !active[it.image]) return;
  const int t = b - prefix[i];
  const int tx = (it.d.c.N + SynthTile<T, V>::TC - 1) / SynthTile<T, V>::TC;
  synth_tile<T, L, BC, V>(it.d, it.f, t % tx, t / tx, 0, smem_raw);
}

static int synth_max_window(const Axis& a, int L, int bc, int tile) {
  const int e = (bc == SYM) ? a.e : 0;
  int mx = 0;
  for (int p0 = 0; p0 < a.N; p0 += tile) {
    const int p1 = p0 + tile < a.N ? p0 + tile : a.N;
    int nlo, nhi;
    fold_window(p0, p1, a.N, e, nlo, nhi);
    const int nk = synth_k0(nhi - 1, L, bc) + 1 - (synth_k0(nlo, L, bc) - (L / 2 - 1));
    if (nk > mx) mx = nk;
  }
  return mx;
}

template <typename T, int V = 0>
static size_t synth_lds_t(int L, const SynthLevel& d) {
  const int mr = synth_max_window(d.r, L, d.bc, SynthTile<T, V>::TR);
  const int mc = synth_max_window(d.c, L, d.bc, SynthTile<T, V>::TC);
  return sizeof(T) * (size_t)(4 * mr * mc + 2 * SynthTile<T, V>::TR * mc);
}

size_t synth_level_lds(int dtype, int L, const SynthLevel& d) {
  return dtype ? synth_lds_t<double>(L, d) : synth_lds_t<float>(L, d);
}

template <typename T, int L, int BC>
static hipError_t launch_synth_t(const double* lo, const SynthLevel& d, int batch, hipStream_t s) {
  const size_t lds = synth_lds_t<T>(L, d);
  auto kern = synth_level_kernel<T, L, BC, 0>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((d.c.N + SynthTile<T>::TC - 1) / SynthTile<T>::TC,
            (d.r.N + SynthTile<T>::TR - 1) / SynthTile<T>::TR, batch);
  hipLaunchKernelGGL(kern, grid, dim3(512), lds, s, d, make_taps<T>(lo, L));
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t launch_synth_bc(const double* lo, const SynthLevel& d, int batch, hipStream_t s) {
  switch (d.bc) {
    case ZPD: return launch_synth_t<T, L, ZPD>(lo, d, batch, s);
    case SYM: return launch_synth_t<T, L, SYM>(lo, d, batch, s);
    case PER: return launch_synth_t<T, L, PER>(lo, d, batch, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_synth_L(int L, const double* lo, const SynthLevel& d, int batch,
                                 hipStream_t s) {
  switch (L) {
    case 2: return launch_synth_bc<T, 2>(lo, d, batch, s);
    case 8: return launch_synth_bc<T, 8>(lo, d, batch, s);
    case 10: return launch_synth_bc<T, 10>(lo, d, batch, s);
    case 16: return launch_synth_bc<T, 16>(lo, d, batch, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_synth_level(int dtype, int L, const double* lo, const SynthLevel& d, int batch,
                              hipStream_t s) {
  return dtype ? launch_synth_L<double>(L, lo, d, batch, s)
               : launch_synth_L<float>(L, lo, d, batch, s);
}

// ------------------------------------------------ chained small levels
// The coarse synthesis levels are small and latency-bound: one launch per
// level costs a launch and a memory round trip each. The chain kernel runs
// d[nl-1] .. d[0] in one launch: a workgroup owns a tile of d[0]'s output and
// synthesises, coarse to fine, the parts of the intermediate approximation
// bands that tile needs (halos recomputed) into LDS. Every value is computed
// by the same arithmetic as the per-level kernels, so the result is bitwise
// the same.
// Output tile of a chain workgroup (a tile of a_1).
constexpr int kChainTR = 32, kChainTC = 128;

template <typename T, int L, int BC>
__global__ __launch_bounds__(512) void synth_chain_kernel(SynthChain c, Taps<T> f) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int TR = kChainTR, TC = kChainTC;
  const int img = blockIdx.z;
  // rows [ra[k], rb[k]) x columns [ca[k], cb[k]) of level d[k]'s output
  int ra[kChainMax], rb[kChainMax], ca[kChainMax], cb[kChainMax];
  ra[0] = blockIdx.y * TR;
  rb[0] = min(ra[0] + TR, c.d[0].r.N);
  ca[0] = blockIdx.x * TC;
  cb[0] = min(ca[0] + TC, c.d[0].c.N);
#pragma unroll
  for (int k = 0; k + 1 < kChainMax; ++k) {
    if (k + 1 >= c.nl) break;
    int kw, nk;
    synth_axis_window(ra[k], rb[k], c.d[k].r.N, BC == SYM ? c.d[k].r.e : 0, L, BC, kw, nk);
    synth_band_part(kw, nk, c.d[k].r.K, ra[k + 1], rb[k + 1]);
    synth_axis_window(ca[k], cb[k], c.d[k].c.N, BC == SYM ? c.d[k].c.e : 0, L, BC, kw, nk);
    synth_band_part(kw, nk, c.d[k].c.K, ca[k + 1], cb[k + 1]);
  }
  // the finest level's detail bands are fetched first when its tile takes
  // the interior layout, so their latency overlaps the coarse levels
  T* const O = static_cast<T*>(c.d[0].out) + (long long)img * c.d[0].stride_out;
  const SynthWin w0 = synth_win<L, BC>(c.d[0], ra[0], rb[0], ca[0], cb[0], img);
  bool fast0 = false;
  FastPre<L, BC, TR> pre0;
  if constexpr (sizeof(T) == 4) {
    fast0 = synth_fast_ok<L, BC, TR, TC>(c.d[0], w0, O);
    if (fast0) fast_fetch<L, BC, TR, true>(c.d[0], w0, pre0);
  }
  for (int k = c.nl - 1; k >= 1; --k) {
    LdsWriter<T> wr{reinterpret_cast<T*>(smem_raw + c.buf_off[k - 1]), ra[k], ca[k],
                    c.buf_pitch[k - 1]};
    if (k == c.nl - 1) {
      synth_rect<T, L, BC>(c.d[k], f, ra[k], rb[k], ca[k], cb[k], img, smem_raw, wr);
    } else {
      const LdsBand<T> src{reinterpret_cast<const T*>(smem_raw + c.buf_off[k]), ra[k + 1],
                           ca[k + 1], c.buf_pitch[k]};
      synth_rect<T, L, BC>(c.d[k], f, ra[k], rb[k], ca[k], cb[k], img, smem_raw, wr, &src);
    }
    __syncthreads();
  }
  const LdsBand<T> src{reinterpret_cast<const T*>(smem_raw + c.buf_off[0]), ra[1], ca[1],
                       c.buf_pitch[0]};
  if constexpr (sizeof(T) == 4) {
    if (fast0) {
      synth_tile_fast_pre<L, BC, TR, true>(c.d[0], f, w0, smem_raw, pre0, &src);
      return;
    }
  }
  PlaneWriter<T> out(O, c.d[0].c.N);
  synth_rect<T, L, BC, true>(c.d[0], f, ra[0], rb[0], ca[0], cb[0], img, smem_raw, out, &src);
}

// Largest output part, and coefficient window, of each chained level over
// the tiles of one axis (rows: is_row).
template <int L, int BC>
static void chain_axis(const SynthChain& c, bool is_row, int tile, int len[], int nk[]) {
  for (int k = 0; k < c.nl; ++k) len[k] = nk[k] = 0;
  const Axis& a0 = is_row ? c.d[0].r : c.d[0].c;
  for (int p0 = 0; p0 < a0.N; p0 += tile) {
    int lo = p0, hi = std::min(p0 + tile, a0.N);
    for (int k = 0; k < c.nl; ++k) {
      const Axis& a = is_row ? c.d[k].r : c.d[k].c;
      len[k] = std::max(len[k], hi - lo);
      int kw, n;
      synth_axis_window(lo, hi, a.N, BC == SYM ? a.e : 0, L, BC, kw, n);
      nk[k] = std::max(nk[k], n);
      synth_band_part(kw, n, a.K, lo, hi);
    }
  }
}

template <int L, int BC>
static size_t chain_plan_t(SynthChain& c) {
  using T = float;
  int lr[kChainMax], nr[kChainMax], lc[kChainMax], nc[kChainMax];
  chain_axis<L, BC>(c, true, kChainTR, lr, nr);
  chain_axis<L, BC>(c, false, kChainTC, lc, nc);
  size_t scratch = 0;
  for (int k = 0; k < c.nl; ++k)
    scratch = std::max(scratch, sizeof(T) * (size_t)(4 * nr[k] * nc[k] + 2 * lr[k] * nc[k]));
  size_t off = (scratch + 15) / 16 * 16;
  for (int k = 0; k + 1 < c.nl; ++k) {  // buffer k: output of d[k+1]
    c.buf_off[k] = (unsigned)off;
    c.buf_pitch[k] = lc[k + 1];
    off += ((size_t)lr[k + 1] * lc[k + 1] * sizeof(T) + 15) / 16 * 16;
  }
  return off;
}

size_t synth_chain_plan(int dtype, int L, SynthChain& c) {
  if (dtype != 0 || c.nl < 2 || c.nl > kChainMax) return 0;
  const int bc = c.d[0].bc;
  for (int k = 0; k < c.nl; ++k) {
    if (c.d[k].bc != bc) return 0;
    if (bc == SYM && (c.d[k].r.N < c.d[k].r.e || c.d[k].c.N < c.d[k].c.e)) return 0;
  }
  size_t lds = 0;
  if (bc == SYM) {
    lds = L == 2    ? chain_plan_t<2, SYM>(c)
          : L == 8  ? chain_plan_t<8, SYM>(c)
          : L == 10 ? chain_plan_t<10, SYM>(c)
          : L == 16 ? chain_plan_t<16, SYM>(c)
                    : 0;
  } else if (bc == ZPD) {
    lds = L == 2    ? chain_plan_t<2, ZPD>(c)
          : L == 8  ? chain_plan_t<8, ZPD>(c)
          : L == 10 ? chain_plan_t<10, ZPD>(c)
          : L == 16 ? chain_plan_t<16, ZPD>(c)
                    : 0;
  }
  return lds <= 64 * 1024 ? lds : 0;
}

// Largest chain grid, in workgroups, that still beats the per-level launches
// (2.5 per CU). Measured with db4, J = 4 (W, FP32): the chain is faster at
// 297 workgroups (2048^2: 27.1 against 32.4 us) and 340 (4 x 1024^2),
// level by level ties at 594-680 (2 x 2048^2, 8 x 1024^2) and wins from
// about 1000 on (16 x 1024^2: 57.3 against 65.6 us, 4 x 4096^2: 183 against
// 212 us).
constexpr long long kChainMaxGrid = 640;

bool synth_chain_pays(const SynthChain& c, int batch) {
  const long long tiles = (long long)((c.d[0].c.N + kChainTC - 1) / kChainTC) *
                          ((c.d[0].r.N + kChainTR - 1) / kChainTR);
  return tiles * batch <= kChainMaxGrid;
}

template <int L, int BC>
static hipError_t launch_chain_t(const double* lo, const SynthChain& c, size_t lds, int batch,
                                 hipStream_t s) {
  using T = float;
  dim3 grid((c.d[0].c.N + kChainTC - 1) / kChainTC, (c.d[0].r.N + kChainTR - 1) / kChainTR,
            batch);
  hipLaunchKernelGGL((synth_chain_kernel<T, L, BC>), grid, dim3(512), lds, s, c,
                     make_taps<T>(lo, L));
  return hipGetLastError();
}

hipError_t launch_synth_chain(int L, const double* lo, const SynthChain& c, size_t lds, int batch,
                              hipStream_t s) {
  const int bc = c.d[0].bc;
  switch (L) {
    case 2: return bc == SYM ? launch_chain_t<2, SYM>(lo, c, lds, batch, s)
                             : launch_chain_t<2, ZPD>(lo, c, lds, batch, s);
    case 8: return bc == SYM ? launch_chain_t<8, SYM>(lo, c, lds, batch, s)
                             : launch_chain_t<8, ZPD>(lo, c, lds, batch, s);
    case 10: return bc == SYM ? launch_chain_t<10, SYM>(lo, c, lds, batch, s)
                              : launch_chain_t<10, ZPD>(lo, c, lds, batch, s);
    case 16: return bc == SYM ? launch_chain_t<16, SYM>(lo, c, lds, batch, s)
                              : launch_chain_t<16, ZPD>(lo, c, lds, batch, s);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------- analysis
template <typename T, int L, int BC, int VAR>
__global__ __launch_bounds__(512) void ana_level_kernel(AnaLevel d, Taps<T> f) {
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  ana_tile<T, L, BC, VAR>(d, f, tx, ty, tz);
}

template <typename T, int L, int BC, int VAR>
__global__ __launch_bounds__(512) void ana_prox_kernel(AnaLevel d, Taps<T> f, ProxEpi pe) {
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  ana_tile<T, L, BC, VAR, true>(d, f, tx, ty, tz, pe);
}

// Tile variant of a single-image analysis level: the half-height tile when
// the full-height grid has fewer than four tiles per compute unit (the
// small, latency-bound levels: measured 96.2 -> 91.7 us per 2048^2 FISTA
// step); FP64 tiles are already half height.
static int ana_variant(int dtype, const AnaLevel& d, int batch) {
  if (dtype) return 0;
  const long long tiles = (long long)((d.c.K + AnaTile<float>::TKC - 1) / AnaTile<float>::TKC) *
                          ((d.r.K + AnaTile<float>::TKR - 1) / AnaTile<float>::TKR) * batch;
  return tiles < 1024 ? 1 : 0;
}

template <typename T, int L, int BC, int VAR, bool PROX = false>
__global__ __launch_bounds__(512) void ana_batch_kernel(
    const AnaItem<T>* __restrict__ items, const int* __restrict__ prefix, int n,
    const int* __restrict__ active) {
  const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int i = find_item(prefix, n, b);
  const AnaItem<T>& it = items[i];
  if (active && !active[it.image]) return;
  const int t = b - prefix[i];
  const int tx = (it.d.c.K + AnaTile<T, VAR>::TKC - 1) / AnaTile<T, VAR>::TKC;
  if constexpr (PROX)
    ana_tile<T, L, BC, VAR, true>(it.d, it.f, t % tx, t / tx, 0, it.pe);
  else
    ana_tile<T, L, BC, VAR>(it.d, it.f, t % tx, t / tx, 0);
}

template <typename T, int L, int BC, int VAR>
static hipError_t launch_ana_tv(const double* lo, const AnaLevel& d, int batch, hipStream_t s) {
  constexpr int TKR = AnaTile<T, VAR>::TKR, TKC = AnaTile<T, VAR>::TKC;
  dim3 grid((d.c.K + TKC - 1) / TKC, (d.r.K + TKR - 1) / TKR, batch);
  hipLaunchKernelGGL((ana_level_kernel<T, L, BC, VAR>), grid, dim3(AnaTile<T, VAR>::NT), 0, s, d,
                     make_taps<T>(lo, L));
  return hipGetLastError();
}

template <typename T, int L, int BC>
static hipError_t launch_ana_t(const double* lo, const AnaLevel& d, int batch, hipStream_t s) {
  if constexpr (sizeof(T) == 4)
    if (ana_variant(0, d, batch)) return launch_ana_tv<T, L, BC, 1>(lo, d, batch, s);
  return launch_ana_tv<T, L, BC, 0>(lo, d, batch, s);
}

template <typename T, int L>
static hipError_t launch_ana_bc(const double* lo, const AnaLevel& d, int batch, hipStream_t s) {
  switch (d.bc) {
    case ZPD: return launch_ana_t<T, L, ZPD>(lo, d, batch, s);
    case SYM: return launch_ana_t<T, L, SYM>(lo, d, batch, s);
    case PER: return launch_ana_t<T, L, PER>(lo, d, batch, s);
    case PER_EXT: return launch_ana_t<T, L, PER_EXT>(lo, d, batch, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_ana_L(int L, const double* lo, const AnaLevel& d, int batch,
                               hipStream_t s) {
  switch (L) {
    case 2: return launch_ana_bc<T, 2>(lo, d, batch, s);
    case 8: return launch_ana_bc<T, 8>(lo, d, batch, s);
    case 10: return launch_ana_bc<T, 10>(lo, d, batch, s);
    case 16: return launch_ana_bc<T, 16>(lo, d, batch, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ana_level(int dtype, int L, const double* lo, const AnaLevel& d, int batch,
                            hipStream_t s) {
  return dtype ? launch_ana_L<double>(L, lo, d, batch, s) : launch_ana_L<float>(L, lo, d, batch, s);
}

template <typename T, int L, int BC, int VAR>
static hipError_t launch_ana_prox_tv(const double* lo, const AnaLevel& d, const ProxEpi& pe,
                                     int batch, hipStream_t s) {
  constexpr int TKR = AnaTile<T, VAR>::TKR, TKC = AnaTile<T, VAR>::TKC;
  dim3 grid((d.c.K + TKC - 1) / TKC, (d.r.K + TKR - 1) / TKR, batch);
  hipLaunchKernelGGL((ana_prox_kernel<T, L, BC, VAR>), grid, dim3(AnaTile<T, VAR>::NT), 0, s, d,
                     make_taps<T>(lo, L), pe);
  return hipGetLastError();
}

template <typename T, int L, int BC>
static hipError_t launch_ana_prox_t(const double* lo, const AnaLevel& d, const ProxEpi& pe,
                                    int batch, hipStream_t s) {
  if constexpr (sizeof(T) == 4)
    if (ana_variant(0, d, batch)) return launch_ana_prox_tv<T, L, BC, 1>(lo, d, pe, batch, s);
  return launch_ana_prox_tv<T, L, BC, 0>(lo, d, pe, batch, s);
}

template <typename T, int L>
static hipError_t launch_ana_prox_bc(const double* lo, const AnaLevel& d, const ProxEpi& pe,
                                     int batch, hipStream_t s) {
  switch (d.bc) {
    case ZPD: return launch_ana_prox_t<T, L, ZPD>(lo, d, pe, batch, s);
    case SYM: return launch_ana_prox_t<T, L, SYM>(lo, d, pe, batch, s);
    case PER: return launch_ana_prox_t<T, L, PER>(lo, d, pe, batch, s);
    case PER_EXT: return launch_ana_prox_t<T, L, PER_EXT>(lo, d, pe, batch, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t launch_ana_prox_L(int L, const double* lo, const AnaLevel& d, const ProxEpi& pe,
                                    int batch, hipStream_t s) {
  switch (L) {
    case 2: return launch_ana_prox_bc<T, 2>(lo, d, pe, batch, s);
    case 8: return launch_ana_prox_bc<T, 8>(lo, d, pe, batch, s);
    case 10: return launch_ana_prox_bc<T, 10>(lo, d, pe, batch, s);
    case 16: return launch_ana_prox_bc<T, 16>(lo, d, pe, batch, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ana_level_prox(int dtype, int L, const double* lo, const AnaLevel& d,
                                 const ProxEpi& pe, int batch, hipStream_t s) {
  return dtype ? launch_ana_prox_L<double>(L, lo, d, pe, batch, s)
               : launch_ana_prox_L<float>(L, lo, d, pe, batch, s);
}

int ana_level_tiles(int dtype, const AnaLevel& d, int batch) {
  if (dtype)
    return ((d.c.K + AnaTile<double>::TKC - 1) / AnaTile<double>::TKC) *
           ((d.r.K + AnaTile<double>::TKR - 1) / AnaTile<double>::TKR);
  if (ana_variant(0, d, batch))
    return ((d.c.K + AnaTile<float, 1>::TKC - 1) / AnaTile<float, 1>::TKC) *
           ((d.r.K + AnaTile<float, 1>::TKR - 1) / AnaTile<float, 1>::TKR);
  return ((d.c.K + AnaTile<float>::TKC - 1) / AnaTile<float>::TKC) *
         ((d.r.K + AnaTile<float>::TKR - 1) / AnaTile<float>::TKR);
}

// ------------------------------------------------------- batched launchers
template <typename T, int V>
static int synth_tiles_t(const SynthLevel& d) {
  return ((d.c.N + SynthTile<T, V>::TC - 1) / SynthTile<T, V>::TC) *
         ((d.r.N + SynthTile<T, V>::TR - 1) / SynthTile<T, V>::TR);
}
template <typename T, int V>
static int ana_tiles_t(const AnaLevel& d) {
  return ((d.c.K + AnaTile<T, V>::TKC - 1) / AnaTile<T, V>::TKC) *
         ((d.r.K + AnaTile<T, V>::TKR - 1) / AnaTile<T, V>::TKR);
}

int synth_tiles(int dtype, int var, const SynthLevel& d) {
  if (dtype) return var ? synth_tiles_t<double, 1>(d) : synth_tiles_t<double, 0>(d);
  return var ? synth_tiles_t<float, 1>(d) : synth_tiles_t<float, 0>(d);
}
int ana_tiles(int dtype, int var, const AnaLevel& d) {
  if (dtype) return var ? ana_tiles_t<double, 1>(d) : ana_tiles_t<double, 0>(d);
  return var ? ana_tiles_t<float, 1>(d) : ana_tiles_t<float, 0>(d);
}
size_t synth_item_lds(int dtype, int L, int var, const SynthLevel& d) {
  if (dtype) return var ? synth_lds_t<double, 1>(L, d) : synth_lds_t<double, 0>(L, d);
  return var ? synth_lds_t<float, 1>(L, d) : synth_lds_t<float, 0>(L, d);
}
size_t synth_item_size(int dtype) { return dtype ? sizeof(SynthItem<double>) : sizeof(SynthItem<float>); }
size_t ana_item_size(int dtype) { return dtype ? sizeof(AnaItem<double>) : sizeof(AnaItem<float>); }

void make_synth_item(int dtype, const SynthLevel& d, const double* lo, int L, int image, void* out) {
  if (dtype) {
    SynthItem<double> it{d, make_taps<double>(lo, L), image};
    *static_cast<SynthItem<double>*>(out) = it;
  } else {
    SynthItem<float> it{d, make_taps<float>(lo, L), image};
    *static_cast<SynthItem<float>*>(out) = it;
  }
}
void make_ana_item_prox(const AnaLevel& d, const double* lo, int L, int image, const ProxEpi& pe,
                        void* out) {
  AnaItem<float> it{d, make_taps<float>(lo, L), image, pe};
  *static_cast<AnaItem<float>*>(out) = it;
}

void make_ana_item(int dtype, const AnaLevel& d, const double* lo, int L, int image, void* out) {
  if (dtype) {
    AnaItem<double> it{d, make_taps<double>(lo, L), image};
    *static_cast<AnaItem<double>*>(out) = it;
  } else {
    AnaItem<float> it{d, make_taps<float>(lo, L), image};
    *static_cast<AnaItem<float>*>(out) = it;
  }
}

template <typename T, int L, int BC, int V>
static hipError_t launch_synth_batch_t(const void* items, const int* prefix, int n, int total,
                                       const int* active, size_t lds, hipStream_t s) {
  auto kern = synth_batch_kernel<T, L, BC, V>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(total), dim3(512), lds, s, static_cast<const SynthItem<T>*>(items),
                     prefix, n, active);
  return hipGetLastError();
}

template <typename T, int L, int BC, int V>
static hipError_t launch_ana_batch_t(const void* items, const int* prefix, int n, int total,
                                     const int* active, hipStream_t s, bool prox) {
  if (prox)
    hipLaunchKernelGGL((ana_batch_kernel<T, L, BC, V, true>), dim3(total), dim3(512), 0, s,
                       static_cast<const AnaItem<T>*>(items), prefix, n, active);
  else
    hipLaunchKernelGGL((ana_batch_kernel<T, L, BC, V>), dim3(total), dim3(512), 0, s,
                       static_cast<const AnaItem<T>*>(items), prefix, n, active);
  return hipGetLastError();
}

#define AW_BATCH_DISPATCH(FN, ...)                                                        \
  switch ((dtype << 8) | (L << 3) | (bc << 1) | var) {                                    \
    case (0 << 8) | (2 << 3) | (ZPD << 1) | 0: return FN<float, 2, ZPD, 0>(__VA_ARGS__);  \
    case (0 << 8) | (2 << 3) | (ZPD << 1) | 1: return FN<float, 2, ZPD, 1>(__VA_ARGS__);  \
    case (0 << 8) | (2 << 3) | (SYM << 1) | 0: return FN<float, 2, SYM, 0>(__VA_ARGS__);  \
    case (0 << 8) | (2 << 3) | (SYM << 1) | 1: return FN<float, 2, SYM, 1>(__VA_ARGS__);  \
    case (0 << 8) | (2 << 3) | (PER << 1) | 0: return FN<float, 2, PER, 0>(__VA_ARGS__);  \
    case (0 << 8) | (2 << 3) | (PER << 1) | 1: return FN<float, 2, PER, 1>(__VA_ARGS__);  \
    case (0 << 8) | (8 << 3) | (ZPD << 1) | 0: return FN<float, 8, ZPD, 0>(__VA_ARGS__);  \
    case (0 << 8) | (8 << 3) | (ZPD << 1) | 1: return FN<float, 8, ZPD, 1>(__VA_ARGS__);  \
    case (0 << 8) | (8 << 3) | (SYM << 1) | 0: return FN<float, 8, SYM, 0>(__VA_ARGS__);  \
    case (0 << 8) | (8 << 3) | (SYM << 1) | 1: return FN<float, 8, SYM, 1>(__VA_ARGS__);  \
    case (0 << 8) | (8 << 3) | (PER << 1) | 0: return FN<float, 8, PER, 0>(__VA_ARGS__);  \
    case (0 << 8) | (8 << 3) | (PER << 1) | 1: return FN<float, 8, PER, 1>(__VA_ARGS__);  \
    case (0 << 8) | (16 << 3) | (ZPD << 1) | 0: return FN<float, 16, ZPD, 0>(__VA_ARGS__); \
    case (0 << 8) | (16 << 3) | (ZPD << 1) | 1: return FN<float, 16, ZPD, 1>(__VA_ARGS__); \
    case (0 << 8) | (16 << 3) | (SYM << 1) | 0: return FN<float, 16, SYM, 0>(__VA_ARGS__); \
    case (0 << 8) | (16 << 3) | (SYM << 1) | 1: return FN<float, 16, SYM, 1>(__VA_ARGS__); \
    case (0 << 8) | (16 << 3) | (PER << 1) | 0: return FN<float, 16, PER, 0>(__VA_ARGS__); \
    case (0 << 8) | (16 << 3) | (PER << 1) | 1: return FN<float, 16, PER, 1>(__VA_ARGS__); \
    default: return hipErrorInvalidValue;                                                 \
  }

// Batched launches run in FP32 (the batched workload's precision); dtype is
// checked by the caller.
hipError_t launch_synth_batch(int dtype, int L, int bc, int var, const void* items,
                              const int* prefix, int n, int total, const int* active, size_t lds,
                              hipStream_t s) {
  AW_BATCH_DISPATCH(launch_synth_batch_t, items, prefix, n, total, active, lds, s)
}
hipError_t launch_ana_batch(int dtype, int L, int bc, int var, const void* items,
                            const int* prefix, int n, int total, const int* active,
                            hipStream_t s, bool prox) {
  AW_BATCH_DISPATCH(launch_ana_batch_t, items, prefix, n, total, active, s, prox)
}
#undef AW_BATCH_DISPATCH

// ---------------------------------------------------- fold of an extended image
// out[p_r][p_c] = w_r w_c sum over preimages of ext[n_r][n_c]; used for the
// periodic-extension mode, whose preimages lie at the far end of the signal.
template <typename T>
__global__ __launch_bounds__(256) void fold_kernel(FoldLevel d) {
  const int img = blockIdx.z;
  const int Nr = d.r.N, Nc = d.c.N, er = d.r.e, ec = d.c.e;
  const int Mc = Nc + 2 * ec;
  const int pc = blockIdx.x * 64 + (threadIdx.x & 63);
  const int pr = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (pr >= Nr || pc >= Nc) return;
  const T* E = static_cast<const T*>(d.ext) + (long long)img * d.stride_ext;
  T acc = T(0);
  const int cr = for_each_preimage(pr, Nr, er, d.bc, [&](int nr) {
    for_each_preimage(pc, Nc, ec, d.bc, [&](int nc) { acc += E[(long long)nr * Mc + nc]; });
  });
  if (d.pinv) {
    const int cc = multiplicity(pc, Nc, ec, d.bc);
    if (cr * cc > 1) acc = acc / T(cr * cc);
  }
  static_cast<T*>(d.out)[(long long)img * d.stride_out + (long long)pr * Nc + pc] = acc;
}

hipError_t launch_fold_level(int dtype, const FoldLevel& d, int batch, hipStream_t s) {
  dim3 grid((d.c.N + 63) / 64, (d.r.N + 3) / 4, batch);
  if (dtype)
    hipLaunchKernelGGL(fold_kernel<double>, grid, dim3(256), 0, s, d);
  else
    hipLaunchKernelGGL(fold_kernel<float>, grid, dim3(256), 0, s, d);
  return hipGetLastError();
}

}  // namespace aw
