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
#include <type_traits>

#include "aw_internal.hpp"

namespace aw {

// Tile shapes; variant 1 halves the rows (more, smaller tiles for small
// levels). The batched path picks the variant per launch (autotuned).
template <typename T, int V = 0>
struct SynthTile {
  static constexpr int TR = (sizeof(T) == 4 ? 32 : 16) >> V, TC = 64;
};
template <typename T, int V = 0>
struct AnaTile {
  static constexpr int TKR = (sizeof(T) == 4 ? 32 : 16) >> V, TKC = 32, NT = 512;
};

template <typename T>
struct Vec;
template <>
struct Vec<float> {
  using V2 = float2;
  using V4 = float4;
};
template <>
struct Vec<double> {
  using V2 = double2;
  using V4 = double4;
};

template <typename T>
static Taps<T> make_taps(const double* lo, int L) {
  Taps<T> t{};
  for (int k = 0; k < L; ++k) {
    t.h[k] = (T)lo[k];
    t.g[k] = (T)(((k & 1) ? -1.0 : 1.0) * lo[L - 1 - k]);
  }
  return t;
}

// ---------------------------------------------------------------- synthesis
// Column-direction synthesis value of extended position n (any parity) from
// the staged coefficient window; lo = a/H pair, hi = V/D pair.
template <typename T, int L, int BC, typename V4>
__device__ inline void synth_col_any(const V4* sc, int nkc, int j, int kw, int n, const Taps<T>& f,
                                     T& lo, T& hi) {
  const int base = synth_k0(n, L, BC) - kw;
  const bool odd = n & 1;
#pragma unroll
  for (int m = 0; m < L / 2; ++m) {
    const T fh = odd ? f.h[2 * m + 1] : f.h[2 * m];
    const T fg = odd ? f.g[2 * m + 1] : f.g[2 * m];
    const V4 q = sc[(base - m) * nkc + j];
    lo += q.x * fh;
    lo += q.y * fg;
    hi += q.z * fh;
    hi += q.w * fg;
  }
}

template <typename T, int L, int BC, typename V2>
__device__ inline T synth_row_any(const V2* row, int kw, int n, const Taps<T>& f) {
  const int base = synth_k0(n, L, BC) - kw;
  const bool odd = n & 1;
  T acc = T(0);
#pragma unroll
  for (int m = 0; m < L / 2; ++m) {
    const T fh = odd ? f.h[2 * m + 1] : f.h[2 * m];
    const T fg = odd ? f.g[2 * m + 1] : f.g[2 * m];
    const V2 q = row[base - m];
    acc += q.x * fh;
    acc += q.y * fg;
  }
  return acc;
}

// Split of a tile [p0, p1) (p0 even) into output pairs (p0 + 2s, p0 + 2s + 1):
// pairs [sL, sR) are regular (single preimage p + e, both rows inside the
// tile); the rows before 2 sL and from 2 sR on are handled one by one
// (border rows within e of an edge, and a ragged last row). nsp counts them.
__device__ inline void special_range(int p0, int p1, int N, int e, bool shift, int& sL, int& sR,
                                     int& nsp) {
  const int np = (p1 - p0 + 1) / 2;
  sL = shift && e > p0 ? (e - p0 + 1) / 2 : 0;
  if (sL > np) sL = np;
  const int m = shift ? min(N - e, p1) : p1;
  int r = (m - 1 - p0 + 1) / 2;  // ceil((m - 1 - p0) / 2) for m - 1 - p0 >= 0
  if (m - 1 - p0 < 0) r = 0;
  sR = r < sL ? sL : (r > np ? np : r);
  nsp = 2 * sL + ((p1 - p0) - 2 * sR);
}

// t-th position (tile-relative) handled one by one
__device__ inline int special_pos(int t, int sL, int sR) {
  return t < 2 * sL ? t : 2 * sR + (t - 2 * sL);
}

template <typename T, int L, int BC, int V>
__device__ __forceinline__ void synth_tile(const SynthLevel& d, const Taps<T>& f, int bx, int by,
                                           int img, unsigned char* smem_raw) {
  constexpr int TR = SynthTile<T, V>::TR, TC = SynthTile<T, V>::TC;
  constexpr int HL = L / 2;
  // extended modes shift the signal by e = L - 1 (odd): the first row of a
  // pair has odd n and the second row uses the next coefficient row
  constexpr bool SHIFT = (BC == SYM);
  using V2 = typename Vec<T>::V2;
  using V4 = typename Vec<T>::V4;

  const int Nr = d.r.N, Nc = d.c.N, Kr = d.r.K, Kc = d.c.K;
  const int er = SHIFT ? d.r.e : 0;
  const int ec = SHIFT ? d.c.e : 0;
  const int r0 = by * TR, r1 = min(r0 + TR, Nr);
  const int c0 = bx * TC, c1 = min(c0 + TC, Nc);
  int nlo_r, nhi_r, nlo_c, nhi_c;
  fold_window(r0, r1, Nr, er, nlo_r, nhi_r);
  fold_window(c0, c1, Nc, ec, nlo_c, nhi_c);
  const int kwr = synth_k0(nlo_r, L, BC) - (HL - 1);
  const int nkr = synth_k0(nhi_r - 1, L, BC) + 1 - kwr;
  const int kwc = synth_k0(nlo_c, L, BC) - (HL - 1);
  const int nkc = synth_k0(nhi_c - 1, L, BC) + 1 - kwc;

  V4* sc = reinterpret_cast<V4*>(smem_raw);  // [nkr][nkc] (a, H, V, D)
  V2* st = reinterpret_cast<V2*>(sc + nkr * nkc);  // [TR][nkc] (lo, hi) after the row fold

  const T* A = static_cast<const T*>(d.a) + (long long)img * d.stride_a;
  const T* HVD = static_cast<const T*>(d.hvd) + (long long)img * d.stride_hvd;
  const long long band = (long long)Kr * Kc;

  // 1. stage the coefficient window, bands interleaved; each thread issues a
  //    batch of loads before writing LDS
  constexpr int CH = 4;
  for (int base = 0; base < nkr * nkc; base += 512 * CH) {
    V4 q[CH];
#pragma unroll
    for (int it = 0; it < CH; ++it) {
      const int idx = base + threadIdx.x + it * 512;
      q[it].x = q[it].y = q[it].z = q[it].w = T(0);
      if (idx < nkr * nkc) {
        const int i = idx / nkc;
        const int j = idx - i * nkc;
        int kr = kwr + i, kc = kwc + j;
        bool ok;
        if (BC == PER) {
          kr = posmod(kr, Kr);
          kc = posmod(kc, Kc);
          ok = true;
        } else {
          ok = (kr >= 0) && (kr < Kr) && (kc >= 0) && (kc < Kc);
        }
        if (ok) {
          const long long off = (long long)kr * Kc + kc;
          q[it].x = A[off];
          q[it].y = HVD[off];
          q[it].z = HVD[band + off];
          q[it].w = HVD[2 * band + off];
        }
      }
    }
#pragma unroll
    for (int it = 0; it < CH; ++it) {
      const int idx = base + threadIdx.x + it * 512;
      if (idx < nkr * nkc) sc[idx] = q[it];
    }
  }
  __syncthreads();

  // 2. column-direction synthesis. Regular row pairs (single preimage, both
  //    rows in the tile) run the paired fast path; border rows and a ragged
  //    last row run a separate pass, so no wave mixes the two.
  int sL, sR, nsp;
  special_range(r0, r1, Nr, er, SHIFT, sL, sR, nsp);
  for (int item = threadIdx.x; item < (sR - sL) * nkc; item += blockDim.x) {
    const int s = sL + item / nkc;
    const int j = item - (item / nkc) * nkc;
    const int p0 = r0 + 2 * s;
    T lo0 = T(0), hi0 = T(0), lo1 = T(0), hi1 = T(0);
    const int k1 = synth_k0(p0 + er, L, BC) - kwr;
    if (SHIFT) {  // row p0: odd taps at k1; row p0+1: even taps at k1+1
      V4 q[HL + 1];
#pragma unroll
      for (int m = 0; m <= HL; ++m) q[m] = sc[(k1 + 1 - m) * nkc + j];
#pragma unroll
      for (int m = 0; m < HL; ++m) {
        lo0 += q[m + 1].x * f.h[2 * m + 1];
        lo0 += q[m + 1].y * f.g[2 * m + 1];
        hi0 += q[m + 1].z * f.h[2 * m + 1];
        hi0 += q[m + 1].w * f.g[2 * m + 1];
        lo1 += q[m].x * f.h[2 * m];
        lo1 += q[m].y * f.g[2 * m];
        hi1 += q[m].z * f.h[2 * m];
        hi1 += q[m].w * f.g[2 * m];
      }
    } else {  // both rows share k1: even taps, then odd taps
#pragma unroll
      for (int m = 0; m < HL; ++m) {
        const V4 q = sc[(k1 - m) * nkc + j];
        lo0 += q.x * f.h[2 * m];
        lo0 += q.y * f.g[2 * m];
        hi0 += q.z * f.h[2 * m];
        hi0 += q.w * f.g[2 * m];
        lo1 += q.x * f.h[2 * m + 1];
        lo1 += q.y * f.g[2 * m + 1];
        hi1 += q.z * f.h[2 * m + 1];
        hi1 += q.w * f.g[2 * m + 1];
      }
    }
    V2 v0, v1;
    v0.x = lo0;
    v0.y = hi0;
    v1.x = lo1;
    v1.y = hi1;
    st[(2 * s) * nkc + j] = v0;
    st[(2 * s + 1) * nkc + j] = v1;
  }
  // border rows: p + e and, near an edge, the reflected preimage
  // (e - 1 - p on the left, 2N - 1 - p + e on the right), weighted 1/mult
  for (int item = threadIdx.x; item < nsp * nkc; item += blockDim.x) {
    const int t = item / nkc;
    const int j = item - t * nkc;
    const int pr = special_pos(t, sL, sR);
    const int p = r0 + pr;
    T lo = T(0), hi = T(0);
    int cnt = 1;
    synth_col_any<T, L, BC>(sc, nkc, j, kwr, p + er, f, lo, hi);
    if (SHIFT && p < er) {
      synth_col_any<T, L, BC>(sc, nkc, j, kwr, er - 1 - p, f, lo, hi);
      ++cnt;
    }
    if (SHIFT && p >= Nr - er) {
      synth_col_any<T, L, BC>(sc, nkc, j, kwr, 2 * Nr - 1 - p + er, f, lo, hi);
      ++cnt;
    }
    if (d.pinv && cnt > 1) {
      const T wgt = cnt == 2 ? T(0.5) : T(1) / T(cnt);
      lo *= wgt;
      hi *= wgt;
    }
    V2 v;
    v.x = lo;
    v.y = hi;
    st[pr * nkc + j] = v;
  }
  __syncthreads();

  // 3. row-direction synthesis, same split over columns
  int qL, qR, nsc;
  special_range(c0, c1, Nc, ec, SHIFT, qL, qR, nsc);
  T* O = static_cast<T*>(d.out) + (long long)img * d.stride_out;
  constexpr int QC = TC / 2;
  const int nrows = r1 - r0;
  // 2-element stores when every row start keeps the pair alignment
  const bool pair_store =
      (Nc & 1) == 0 && (reinterpret_cast<uintptr_t>(O) & (sizeof(V2) - 1)) == 0;
  for (int item = threadIdx.x; item < nrows * QC; item += blockDim.x) {
    const int pr = item / QC;
    const int q = item - pr * QC;
    if (q < qL || q >= qR) continue;
    const int p = c0 + 2 * q;
    const V2* row = st + pr * nkc;
    T o0 = T(0), o1 = T(0);
    const int k1 = synth_k0(p + ec, L, BC) - kwc;
    if (SHIFT) {
      V2 w[HL + 1];
#pragma unroll
      for (int m = 0; m <= HL; ++m) w[m] = row[k1 + 1 - m];
#pragma unroll
      for (int m = 0; m < HL; ++m) {
        o0 += w[m + 1].x * f.h[2 * m + 1];
        o0 += w[m + 1].y * f.g[2 * m + 1];
        o1 += w[m].x * f.h[2 * m];
        o1 += w[m].y * f.g[2 * m];
      }
    } else {
#pragma unroll
      for (int m = 0; m < HL; ++m) {
        const V2 w = row[k1 - m];
        o0 += w.x * f.h[2 * m];
        o0 += w.y * f.g[2 * m];
        o1 += w.x * f.h[2 * m + 1];
        o1 += w.y * f.g[2 * m + 1];
      }
    }
    T* orow = O + (long long)(r0 + pr) * Nc;
    if (pair_store) {  // p even: one aligned 2-element store
      V2 o;
      o.x = o0;
      o.y = o1;
      *reinterpret_cast<V2*>(orow + p) = o;
    } else {
      orow[p] = o0;
      orow[p + 1] = o1;
    }
  }
  for (int item = threadIdx.x; item < nrows * nsc; item += blockDim.x) {
    const int pr = item / nsc;
    const int t = item - pr * nsc;
    const int p = c0 + special_pos(t, qL, qR);
    const V2* row = st + pr * nkc;
    T acc = synth_row_any<T, L, BC>(row, kwc, p + ec, f);
    int cnt = 1;
    if (SHIFT && p < ec) {
      acc += synth_row_any<T, L, BC>(row, kwc, ec - 1 - p, f);
      ++cnt;
    }
    if (SHIFT && p >= Nc - ec) {
      acc += synth_row_any<T, L, BC>(row, kwc, 2 * Nc - 1 - p + ec, f);
      ++cnt;
    }
    if (d.pinv && cnt > 1) acc *= cnt == 2 ? T(0.5) : T(1) / T(cnt);
    O[(long long)(r0 + pr) * Nc + p] = acc;
  }
}

template <typename T, int L, int BC, int V>
__global__ __launch_bounds__(512) void synth_level_kernel(SynthLevel d, Taps<T> f) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // plain dispatch order: the XCD-aware order (xcd_tile) that speeds up the
  // analysis and blur tiles measured 5 % slower here (2048^2 level 1)
  synth_tile<T, L, BC, V>(d, f, blockIdx.x, blockIdx.y, blockIdx.z, smem_raw);
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
    case 16: return launch_synth_bc<T, 16>(lo, d, batch, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_synth_level(int dtype, int L, const double* lo, const SynthLevel& d, int batch,
                              hipStream_t s) {
  return dtype ? launch_synth_L<double>(L, lo, d, batch, s)
               : launch_synth_L<float>(L, lo, d, batch, s);
}

// ----------------------------------------------------------------- analysis
template <typename T, int L, int BC, int VAR, bool PROX = false>
__device__ __forceinline__ void ana_tile(const AnaLevel& d, const Taps<T>& f, int bx, int by,
                                         int img, const ProxEpi& pe = ProxEpi{}) {
  constexpr int TKR = AnaTile<T, VAR>::TKR, TKC = AnaTile<T, VAR>::TKC, NT = AnaTile<T, VAR>::NT;
  // output ownership of step 3: thread = column kk, KB consecutive rows
  constexpr int RBLK = NT / TKC;
  constexpr int KB = TKR / RBLK;
  const int kk = threadIdx.x % TKC;
  const int rb = threadIdx.x / TKC;
  // fused update: y_k and x_{k-1} of the owned coefficients are fetched
  // first, so their latency overlaps the staging below
  T py[KB][4], px[KB][4];
  if constexpr (PROX) {
    const long long band = (long long)d.r.K * d.c.K;
    const int kc = bx * TKC + kk;
#pragma unroll
    for (int r = 0; r < KB; ++r) {
      const int kr = by * TKR + rb * KB + r;
#pragma unroll
      for (int q = 0; q < 4; ++q) py[r][q] = px[r][q] = T(0);
      if (kr < d.r.K && kc < d.c.K) {
        const long long off = (long long)kr * d.c.K + kc;
        const T* Y = static_cast<const T*>(pe.y_hvd) + (long long)img * d.stride_hvd + off;
        const T* X = static_cast<const T*>(pe.x_hvd) + (long long)img * d.stride_hvd + off;
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          py[r][q] = Y[(q - 1) * band];
          px[r][q] = X[(q - 1) * band];
        }
        if (pe.x_a) {
          py[r][0] = static_cast<const T*>(pe.y_a)[(long long)img * d.stride_a + off];
          px[r][0] = static_cast<const T*>(pe.x_a)[(long long)img * d.stride_a + off];
        }
      }
    }
  }
  constexpr int NWR = 2 * TKR + L - 2, NWC = 2 * TKC + L - 2;
  constexpr int VW = 16 / sizeof(T);                       // elements per 16-byte LDS read
  constexpr int SUS = ((NWC + VW - 1) / VW) * VW + VW;     // input row stride
  constexpr int NV = (2 * VW + L - 2 + VW - 1) / VW;       // vectors per pass-1 item
  using V2 = typename Vec<T>::V2;
  using V4 = typename Vec<T>::V4;
  __shared__ __align__(16) T su[NWR * SUS];
  __shared__ __align__(16) V2 slh[NWR * TKC];

  const int Nr = d.r.N, Nc = d.c.N, Kr = d.r.K, Kc = d.c.K;
  const int er = d.r.e, ec = d.c.e;
  const int kr0 = by * TKR, kr1 = min(kr0 + TKR, Kr);
  const int kc0 = bx * TKC, kc1 = min(kc0 + TKC, Kc);
  const int nlo_r = (BC == PER) ? 2 * kr0 : 2 * kr0 - L + 2;
  const int nlo_c = (BC == PER) ? 2 * kc0 : 2 * kc0 - L + 2;
  const int Mr = Nr + 2 * er, Mc = Nc + 2 * ec;
  const T* Y = static_cast<const T*>(d.in) + (long long)img * d.stride_in;
  const bool interior = (BC == PER) ? (nlo_r + NWR <= Nr && nlo_c + NWC <= Nc)
                                    : (nlo_r >= 2 * er && nlo_r + NWR <= Nr && nlo_c >= 2 * ec &&
                                       nlo_c + NWC <= Nc);

  // 1. gather u(n) = w(src) y[src(n - e)] (zero outside [0, M)); all loads
  //    of a thread are issued before its LDS writes
  if (interior && (Nc % VW) == 0) {
    const int g0 = nlo_c - ec;                  // first input column of the window
    const int a0 = (g0 >= 0 ? g0 / VW : -((-g0 + VW - 1) / VW)) * VW;
    const int off = g0 - a0;                    // 0 .. VW-1
    constexpr int NVR = (NWC + 2 * VW - 2) / VW + 1;  // vectors per row (upper bound)
    constexpr int NVEC = NWR * NVR;
    constexpr int IT = (NVEC + NT - 1) / NT;
    using LV = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    LV buf[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < NVEC) {
        const int i = idx / NVR, jv = idx - (idx / NVR) * NVR;
        const int gc = a0 + jv * VW;
        if (gc + VW <= Nc)
          buf[it] = *reinterpret_cast<const LV*>(Y + (long long)(nlo_r + i - er) * Nc + gc);
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < NVEC) {
        const int i = idx / NVR, jv = idx - (idx / NVR) * NVR;
        const int gc = a0 + jv * VW;
        if (gc + VW <= Nc) {
          T e[VW];
          if constexpr (VW == 4) {
            e[0] = buf[it].x; e[1] = buf[it].y; e[2] = buf[it].z; e[3] = buf[it].w;
          } else {
            e[0] = buf[it].x; e[1] = buf[it].y;
          }
#pragma unroll
          for (int u = 0; u < VW; ++u) {
            const int j = jv * VW + u - off;
            if (j >= 0 && j < NWC) su[i * SUS + j] = e[u];
          }
        }
      }
    }
  } else {
    // per-row / per-column source index and weight (1/mult for W^*, 1 for
    // W^dagger, 0 outside the extended signal), then one gather loop
    __shared__ int rsrc[NWR], csrc[NWC];
    __shared__ T rwt[NWR], cwt[NWC];
    for (int i = threadIdx.x; i < NWR + NWC; i += blockDim.x) {
      const bool isr = i < NWR;
      const int n = isr ? nlo_r + i : nlo_c + (i - NWR);
      const int Nn = isr ? Nr : Nc, ee = isr ? er : ec, Mm = Nn + 2 * ee;
      int src = 0;
      T wgt = T(0);
      if (BC == PER) {
        src = posmod(n, Nn);
        wgt = T(1);
      } else if (n >= 0 && n < Mm) {
        src = src_index(n - ee, Nn, BC);
        wgt = d.pinv ? T(1) / T(multiplicity(src, Nn, ee, BC)) : T(1);
      }
      if (isr) {
        rsrc[i] = src;
        rwt[i] = wgt;
      } else {
        csrc[i - NWR] = src;
        cwt[i - NWR] = wgt;
      }
    }
    __syncthreads();
    constexpr int IT2 = (NWR * NWC + NT - 1) / NT;  // every load issued before any LDS write
    T v[IT2];
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < NWR * NWC) {
        const int i = idx / NWC, j = idx - (idx / NWC) * NWC;
        v[it] = Y[(long long)rsrc[i] * Nc + csrc[j]] * (rwt[i] * cwt[j]);
      }
    }
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int idx = threadIdx.x + it * NT;
      if (idx < NWR * NWC) {
        const int i = idx / NWC, j = idx - (idx / NWC) * NWC;
        su[i * SUS + j] = v[it];
      }
    }
  }
  for (int idx = threadIdx.x; idx < NWR * (SUS - NWC); idx += blockDim.x) {
    const int i = idx / (SUS - NWC), j = idx - (idx / (SUS - NWC)) * (SUS - NWC);
    su[i * SUS + NWC + j] = T(0);
  }
  __syncthreads();

  // 2. filter along columns, two output columns per item:
  //    (lo, hi)[i][kc] = sum_j (h, g)[j] u(i, 2 kc + j)
  constexpr int CP = TKC / 2;
  for (int item = threadIdx.x; item < NWR * CP; item += blockDim.x) {
    const int i = item / CP, cp = item - (item / CP) * CP;
    const T* row = su + i * SUS + 4 * cp;
    T w[NV * VW];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (VW == 4) {
        const float4 q = *reinterpret_cast<const float4*>(row + 4 * v);
        w[4 * v] = q.x; w[4 * v + 1] = q.y; w[4 * v + 2] = q.z; w[4 * v + 3] = q.w;
      } else {
        const double2 q = *reinterpret_cast<const double2*>(row + 2 * v);
        w[2 * v] = q.x; w[2 * v + 1] = q.y;
      }
    }
    T lo0 = T(0), hi0 = T(0), lo1 = T(0), hi1 = T(0);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      lo0 += f.h[j] * w[j];
      hi0 += f.g[j] * w[j];
      lo1 += f.h[j] * w[j + 2];
      hi1 += f.g[j] * w[j + 2];
    }
    V4 o;
    o.x = lo0; o.y = hi0; o.z = lo1; o.w = hi1;
    *reinterpret_cast<V4*>(slh + i * TKC + 2 * cp) = o;
  }
  __syncthreads();

  // 3. filter along rows: thread = column kc and KB consecutive coefficient rows
  constexpr int NW = 2 * KB + L - 2;
  V2 win[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) win[i] = slh[(2 * rb * KB + i) * TKC + kk];
  T* Aout = static_cast<T*>(d.a) + (long long)img * d.stride_a;
  T* HVD = static_cast<T*>(d.hvd) + (long long)img * d.stride_hvd;
  const long long band = (long long)Kr * Kc;
  const int kc = kc0 + kk;
  double l1 = 0.0;
#pragma unroll
  for (int r = 0; r < KB; ++r) {
    T a = T(0), H = T(0), V = T(0), D = T(0);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const V2 q = win[2 * r + j];
      a += f.h[j] * q.x;
      H += f.g[j] * q.x;
      V += f.h[j] * q.y;
      D += f.g[j] * q.y;
    }
    const int kr = kr0 + rb * KB + r;
    if (kr < kr1 && kc < kc1) {
      const long long off = (long long)kr * Kc + kc;
      if constexpr (PROX) {
        const T g[4] = {a, H, V, D};
        T xn[4];
        const T il = (T)pe.inv_L, th = (T)pe.thresh, be = (T)pe.beta;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const T v = py[r][q] - g[q] * il;
          xn[q] = v > th ? v - th : (v < -th ? v + th : T(0));
        }
        T* Xh = static_cast<T*>(pe.x_hvd) + (long long)img * d.stride_hvd + off;
        T* Yh = static_cast<T*>(pe.y_hvd) + (long long)img * d.stride_hvd + off;
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          Yh[(q - 1) * band] = xn[q] + be * (xn[q] - px[r][q]);
          Xh[(q - 1) * band] = xn[q];
          l1 += (double)(xn[q] < T(0) ? -xn[q] : xn[q]);
        }
        if (pe.x_a) {
          const long long oa = (long long)img * d.stride_a + off;
          static_cast<T*>(pe.y_a)[oa] = xn[0] + be * (xn[0] - px[r][0]);
          static_cast<T*>(pe.x_a)[oa] = xn[0];
          l1 += (double)(xn[0] < T(0) ? -xn[0] : xn[0]);
        } else {
          Aout[off] = a;
        }
      } else {
        Aout[off] = a;
        HVD[off] = H;
        HVD[band + off] = V;
        HVD[2 * band + off] = D;
      }
    }
  }
  if constexpr (PROX) {
    if (pe.partials) {  // fixed-order tile sum of |x_k|
      __shared__ double red[NT];
      red[threadIdx.x] = l1;
      __syncthreads();
      for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        const int gx = (Kc + TKC - 1) / TKC;
        pe.partials[(long long)img * pe.pstride + pe.pbase + by * gx + bx] = red[0];
      }
    }
  }
}

template <typename T, int L, int BC, int VAR>
__global__ __launch_bounds__(512) void ana_level_kernel(AnaLevel d, Taps<T> f) {
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  ana_tile<T, L, BC, VAR>(d, f, tx, ty, tz);
}

template <typename T, int L, int BC>
__global__ __launch_bounds__(512) void ana_prox_kernel(AnaLevel d, Taps<T> f, ProxEpi pe) {
  int tx, ty, tz;
  xcd_tile(tx, ty, tz);
  ana_tile<T, L, BC, 0, true>(d, f, tx, ty, tz, pe);
}

template <typename T, int L, int BC, int VAR>
__global__ __launch_bounds__(512) void ana_batch_kernel(
    const AnaItem<T>* __restrict__ items, const int* __restrict__ prefix, int n,
    const int* __restrict__ active) {
  const int b = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int i = find_item(prefix, n, b);
  const AnaItem<T>& it = items[i];
  if (active && !active[it.image]) return;
  const int t = b - prefix[i];
  const int tx = (it.d.c.K + AnaTile<T, VAR>::TKC - 1) / AnaTile<T, VAR>::TKC;
  ana_tile<T, L, BC, VAR>(it.d, it.f, t % tx, t / tx, 0);
}

template <typename T, int L, int BC>
static hipError_t launch_ana_t(const double* lo, const AnaLevel& d, int batch, hipStream_t s) {
  constexpr int TKR = AnaTile<T>::TKR, TKC = AnaTile<T>::TKC;
  dim3 grid((d.c.K + TKC - 1) / TKC, (d.r.K + TKR - 1) / TKR, batch);
  hipLaunchKernelGGL((ana_level_kernel<T, L, BC, 0>), grid, dim3(AnaTile<T>::NT), 0, s, d,
                     make_taps<T>(lo, L));
  return hipGetLastError();
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
    case 16: return launch_ana_bc<T, 16>(lo, d, batch, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ana_level(int dtype, int L, const double* lo, const AnaLevel& d, int batch,
                            hipStream_t s) {
  return dtype ? launch_ana_L<double>(L, lo, d, batch, s) : launch_ana_L<float>(L, lo, d, batch, s);
}

template <typename T, int L, int BC>
static hipError_t launch_ana_prox_t(const double* lo, const AnaLevel& d, const ProxEpi& pe,
                                    int batch, hipStream_t s) {
  constexpr int TKR = AnaTile<T>::TKR, TKC = AnaTile<T>::TKC;
  dim3 grid((d.c.K + TKC - 1) / TKC, (d.r.K + TKR - 1) / TKR, batch);
  hipLaunchKernelGGL((ana_prox_kernel<T, L, BC>), grid, dim3(AnaTile<T>::NT), 0, s, d,
                     make_taps<T>(lo, L), pe);
  return hipGetLastError();
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
    case 16: return launch_ana_prox_bc<T, 16>(lo, d, pe, batch, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ana_level_prox(int dtype, int L, const double* lo, const AnaLevel& d,
                                 const ProxEpi& pe, int batch, hipStream_t s) {
  return dtype ? launch_ana_prox_L<double>(L, lo, d, pe, batch, s)
               : launch_ana_prox_L<float>(L, lo, d, pe, batch, s);
}

int ana_level_tiles(int dtype, const AnaLevel& d) {
  if (dtype)
    return ((d.c.K + AnaTile<double>::TKC - 1) / AnaTile<double>::TKC) *
           ((d.r.K + AnaTile<double>::TKR - 1) / AnaTile<double>::TKR);
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
                                     const int* active, hipStream_t s) {
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
                            hipStream_t s) {
  AW_BATCH_DISPATCH(launch_ana_batch_t, items, prefix, n, total, active, s)
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
