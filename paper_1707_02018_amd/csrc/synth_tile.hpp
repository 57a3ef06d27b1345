// Synthesis tile machinery shared by the per-level kernels (wavelet.hip) and
// the fused synthesis + blur kernel (fused.hip).
#pragma once

#include <cstdint>

#include "aw_internal.hpp"

namespace aw {

// Tile shapes; variant 1 halves the rows (more, smaller tiles for small
// levels). The batched path picks the variant per launch (autotuned). FP32
// tiles are 32 x 128 (at 2048^2 faster than 32 x 64, 32 x 256, 64 x 128,
// 16 x 128 and 16 x 256); 128 columns are the 64 lanes' output pairs of the
// interior layout below.
template <typename T, int V = 0>
struct SynthTile {
  static constexpr int TR = (sizeof(T) == 4 ? 32 : 16) >> V, TC = sizeof(T) == 4 ? 128 : 64;
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

// Taps of one side of a transform: the low-pass h = src[0..L) and the
// high-pass g[k] = (-1)^k f[L-1-k] with f = src[kMaxTaps..kMaxTaps+L) (h
// itself for orthogonal filters, the other side's low-pass for a
// biorthogonal pair).
template <typename T>
static Taps<T> make_taps(const double* src, int L) {
  Taps<T> t{};
  for (int k = 0; k < L; ++k) {
    t.h[k] = (T)src[k];
    t.g[k] = (T)(((k & 1) ? -1.0 : 1.0) * src[kMaxTaps + L - 1 - k]);
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

// Coefficient window [kw, kw + nk) of one axis that the synthesis outputs
// [p0, p1) read (e_eff = e for the symmetric extension, else 0), and the part
// of it inside the band, widened to an even start: [a0, a1).
__host__ __device__ inline void synth_axis_window(int p0, int p1, int N, int e_eff, int L, int bc,
                                                  int& kw, int& nk) {
  int nlo, nhi;
  fold_window(p0, p1, N, e_eff, nlo, nhi);
  kw = synth_k0(nlo, L, bc) - (L / 2 - 1);
  nk = synth_k0(nhi - 1, L, bc) + 1 - kw;
}

__host__ __device__ inline void synth_band_part(int kw, int nk, int K, int& a0, int& a1) {
  a0 = (kw > 0 ? kw : 0) & ~1;
  a1 = kw + nk < K ? kw + nk : K;
}

// A level's approximation band held in LDS over rows [r0, ..) and columns
// [c0, ..) (row pitch `pitch`), in place of the band in memory.
template <typename T>
struct LdsBand {
  const T* p;
  int r0, c0, pitch;
};

// Geometry of one synthesis rectangle: outputs [r0, r1) x [c0, c1) of image
// img, read from the coefficient window [kwr, kwr + nkr) x [kwc, kwc + nkc).
struct SynthWin {
  int r0, r1, c0, c1, img, kwr, nkr, kwc, nkc;
};

template <int L, int BC>
__device__ __forceinline__ SynthWin synth_win(const SynthLevel& d, int r0, int r1, int c0, int c1,
                                              int img) {
  SynthWin w{r0, r1, c0, c1, img, 0, 0, 0, 0};
  synth_axis_window(r0, r1, d.r.N, BC == SYM ? d.r.e : 0, L, BC, w.kwr, w.nkr);
  synth_axis_window(c0, c1, d.c.N, BC == SYM ? d.c.e : 0, L, BC, w.kwc, w.nkc);
  return w;
}

constexpr int kSynthCH = 4;  // window items per thread per load batch (x 512 threads)

// Loads of window items base + threadIdx.x + it * 512 (bands interleaved:
// a, H, V, D), zero outside the bands.
template <typename T, int L, int BC>
__device__ __forceinline__ void synth_load(const SynthLevel& d, const SynthWin& w, int base,
                                           typename Vec<T>::V4 (&q)[kSynthCH],
                                           const LdsBand<T>* abuf) {
  const int Kr = d.r.K, Kc = d.c.K;
  const T* A = static_cast<const T*>(d.a) + (long long)w.img * d.stride_a;
  const T* HVD = static_cast<const T*>(d.hvd) + (long long)w.img * d.stride_hvd;
  const long long band = (long long)Kr * Kc;
#pragma unroll
  for (int it = 0; it < kSynthCH; ++it) {
    const int idx = base + threadIdx.x + it * 512;
    q[it].x = q[it].y = q[it].z = q[it].w = T(0);
    if (idx < w.nkr * w.nkc) {
      const int i = idx / w.nkc;
      const int j = idx - i * w.nkc;
      int kr = w.kwr + i, kc = w.kwc + j;
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
        q[it].x = abuf ? abuf->p[(kr - abuf->r0) * abuf->pitch + (kc - abuf->c0)] : A[off];
        q[it].y = HVD[off];
        q[it].z = HVD[band + off];
        q[it].w = HVD[2 * band + off];
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void synth_put(const SynthWin& w, int base,
                                          const typename Vec<T>::V4 (&q)[kSynthCH],
                                          unsigned char* smem_raw) {
  auto* sc = reinterpret_cast<typename Vec<T>::V4*>(smem_raw);
#pragma unroll
  for (int it = 0; it < kSynthCH; ++it) {
    const int idx = base + threadIdx.x + it * 512;
    if (idx < w.nkr * w.nkc) sc[idx] = q[it];
  }
}

template <typename T, int L, int BC, bool LANES, typename W>
__device__ __forceinline__ void synth_passes(const SynthLevel& d, const Taps<T>& f,
                                             const SynthWin& w, unsigned char* smem_raw, W& wr);

// Lane-mapped layout of the synthesis loops (512 threads = 8 waves): a wave
// takes window rows (row pairs, output rows) wv, wv + 8, ... and its 64 lanes
// the columns 0..63; columns from 64 on (at most kSynthTailC) go to threads
// (t >> 3, 64 + (t & 7)). Every address is then a wave-uniform base plus the
// lane, with no per-item index division.
constexpr int kSynthTailC = 8;
constexpr int kSynthMaxRows = 32;  // window rows staged by the lane-mapped loads

__device__ __forceinline__ bool synth_lanes_ok(const SynthWin& w) {
  return w.nkr <= kSynthMaxRows && w.nkc <= 64 + kSynthTailC && (w.c1 - w.c0 + 1) / 2 <= 64 &&
         (w.r1 - w.r0 + 1) / 2 <= 64;
}

// Window item (i, j) (bands interleaved a, H, V, D), zero outside the bands.
template <typename T, int L, int BC>
__device__ __forceinline__ typename Vec<T>::V4 synth_fetch(const SynthLevel& d, const SynthWin& w,
                                                           int i, int j,
                                                           const LdsBand<T>* abuf) {
  const int Kr = d.r.K, Kc = d.c.K;
  const T* A = static_cast<const T*>(d.a) + (long long)w.img * d.stride_a;
  const T* HVD = static_cast<const T*>(d.hvd) + (long long)w.img * d.stride_hvd;
  const long long band = (long long)Kr * Kc;
  typename Vec<T>::V4 q;
  q.x = q.y = q.z = q.w = T(0);
  int kr = w.kwr + i, kc = w.kwc + j;
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
    q.x = abuf ? abuf->p[(kr - abuf->r0) * abuf->pitch + (kc - abuf->c0)] : A[off];
    q.y = HVD[off];
    q.z = HVD[band + off];
    q.w = HVD[2 * band + off];
  }
  return q;
}

template <typename T, int L, int BC>
__device__ __forceinline__ void synth_stage_lanes(const SynthLevel& d, const SynthWin& w,
                                                  unsigned char* smem_raw,
                                                  const LdsBand<T>* abuf) {
  using V4 = typename Vec<T>::V4;
  constexpr int RPW = kSynthMaxRows / 8;
  V4* sc = reinterpret_cast<V4*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ti = threadIdx.x >> 3, tj = 64 + (threadIdx.x & 7);
  const bool main_col = lane < w.nkc, tail = ti < w.nkr && tj < w.nkc;
  V4 q[RPW], qt;
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int i = wv + 8 * k;
    if (i < w.nkr && main_col) q[k] = synth_fetch<T, L, BC>(d, w, i, lane, abuf);
  }
  if (tail) qt = synth_fetch<T, L, BC>(d, w, ti, tj, abuf);
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int i = wv + 8 * k;
    if (i < w.nkr && main_col) sc[i * w.nkc + lane] = q[k];
  }
  if (tail) sc[ti * w.nkc + tj] = qt;
}

// Synthesis of one level at the output rectangle [r0, r1) x [c0, c1)
// (r0, c0 even) of image `img`; each output value goes to wr.one(row, col, v)
// or, for a column pair (col even), wr.pair(row, col, v0, v1). smem_raw holds
// the staged coefficient window (nkr x nkc x 4 values) followed by the
// column-pass rows ((r1 - r0) x nkc x 2 values). With abuf, the approximation
// band comes from LDS (it must cover the window's part inside the band).
// Needs 512 threads. LANES selects the lane-mapped loops where the window
// fits them (the per-level tiles); otherwise items are spread over threads
// (the chained levels' irregular rectangles, where that measured faster).
template <typename T, int L, int BC, bool LANES = false, typename W>
__device__ __forceinline__ void synth_rect(const SynthLevel& d, const Taps<T>& f, int r0, int r1,
                                           int c0, int c1, int img, unsigned char* smem_raw,
                                           W& wr, const LdsBand<T>* abuf = nullptr) {
  const SynthWin w = synth_win<L, BC>(d, r0, r1, c0, c1, img);
  // 1. stage the coefficient window; each thread issues its loads before
  //    writing LDS
  if (LANES && synth_lanes_ok(w)) {
    synth_stage_lanes<T, L, BC>(d, w, smem_raw, abuf);
  } else {
    for (int base = 0; base < w.nkr * w.nkc; base += 512 * kSynthCH) {
      typename Vec<T>::V4 q[kSynthCH];
      synth_load<T, L, BC>(d, w, base, q, abuf);
      synth_put<T>(w, base, q, smem_raw);
    }
  }
  __syncthreads();
  synth_passes<T, L, BC, LANES>(d, f, w, smem_raw, wr);
}

// Column then row passes over the staged window (steps 2 and 3).
template <typename T, int L, int BC, bool LANES, typename W>
__device__ __forceinline__ void synth_passes(const SynthLevel& d, const Taps<T>& f,
                                             const SynthWin& w, unsigned char* smem_raw, W& wr) {
  constexpr int HL = L / 2;
  // extended modes shift the signal by e = L - 1 (odd): the first row of a
  // pair has odd n and the second row uses the next coefficient row
  constexpr bool SHIFT = (BC == SYM);
  using V2 = typename Vec<T>::V2;
  using V4 = typename Vec<T>::V4;
  const int Nr = d.r.N, Nc = d.c.N;
  const int er = SHIFT ? d.r.e : 0;
  const int ec = SHIFT ? d.c.e : 0;
  const int r0 = w.r0, r1 = w.r1, c0 = w.c0, c1 = w.c1;
  const int kwr = w.kwr, nkc = w.nkc, kwc = w.kwc;
  V4* sc = reinterpret_cast<V4*>(smem_raw);            // [nkr][nkc] (a, H, V, D)
  V2* st = reinterpret_cast<V2*>(sc + w.nkr * w.nkc);  // [rows][nkc] (lo, hi) after the row fold

  // 2. column-direction synthesis. Regular row pairs (single preimage, both
  //    rows in the tile) run the paired fast path; border rows and a ragged
  //    last row run a separate pass, so no wave mixes the two.
  int sL, sR, nsp;
  special_range(r0, r1, Nr, er, SHIFT, sL, sR, nsp);
  auto col_pair = [&](int s, int j) {
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
  };
  const bool lanes = LANES && synth_lanes_ok(w);
  if (lanes) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (lane < nkc)
      for (int s = sL + wv; s < sR; s += 8) col_pair(s, lane);
    const int s = sL + (threadIdx.x >> 3), j = 64 + (threadIdx.x & 7);
    if (s < sR && j < nkc) col_pair(s, j);
  } else {
    for (int item = threadIdx.x; item < (sR - sL) * nkc; item += blockDim.x) {
      const int s = sL + item / nkc;
      col_pair(s, item - (item / nkc) * nkc);
    }
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
  const int QC = (c1 - c0 + 1) / 2;
  const int nrows = r1 - r0;
  auto row_pair = [&](int pr, int q) {
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
    wr.pair(r0 + pr, p, o0, o1);
  };
  if (lanes) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (lane >= qL && lane < qR)
      for (int pr = wv; pr < nrows; pr += 8) row_pair(pr, lane);
  } else {
    for (int item = threadIdx.x; item < nrows * QC; item += blockDim.x) {
      const int pr = item / QC;
      const int q = item - pr * QC;
      if (q >= qL && q < qR) row_pair(pr, q);
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
    wr.one(r0 + pr, p, acc);
  }
}

// ------------------------------------------------ interior synthesis tiles
// An FP32 tile of 128 output columns whose outputs are all regular (a full
// tile, no border row or column, the coefficient window inside the bands)
// runs with a fixed thread layout: one wave per window row, row pair or
// output row and the 64 lanes along the columns, so every LDS and global
// address is a wave-uniform base plus the lane (no per-item index division).
// The taps and their order are those of synth_passes: the values are bitwise
// the same.
template <int L, int BC, int TR>
struct FastSynth {
  static constexpr int HL = L / 2;
  static constexpr bool SHIFT = (BC == SYM);
  static constexpr int NKR = TR / 2 + HL - (SHIFT ? 0 : 1);  // window rows
  static constexpr int NKC = 64 + HL - (SHIFT ? 0 : 1);      // window columns
  static constexpr int TAILC = NKC - 64;                     // columns past the lanes
};

template <int L, int BC, int TR, int TC>
__device__ __forceinline__ bool synth_fast_ok(const SynthLevel& d, const SynthWin& w,
                                              const void* out) {
  using G = FastSynth<L, BC, TR>;
  if constexpr (TC != 128 || (BC != SYM && BC != ZPD && BC != PER)) {
    return false;
  } else {
    if (w.r1 - w.r0 != TR || w.c1 - w.c0 != TC) return false;
    if (BC == SYM && (w.r0 < d.r.e || w.r1 > d.r.N - d.r.e || w.c0 < d.c.e ||
                      w.c1 > d.c.N - d.c.e))
      return false;
    if (w.nkr != G::NKR || w.nkc != G::NKC) return false;
    if (w.kwr < 0 || w.kwr + G::NKR > d.r.K || w.kwc < 0 || w.kwc + G::NKC > d.c.K) return false;
    if ((long long)d.r.K * d.c.K >= (1LL << 31)) return false;  // 32-bit offsets in a band
    return (d.c.N & 1) == 0 && (reinterpret_cast<uintptr_t>(out) & 7) == 0;
  }
}

// Column-direction synthesis of row pair s at window column j (FP32), into
// rows 2s and 2s + 1 of the column-pass output.
template <int L, int BC, int TR>
__device__ __forceinline__ void fast_col_pair(const float4* sc, float2* st, const Taps<float>& f,
                                              int s, int j) {
  using G = FastSynth<L, BC, TR>;
  constexpr int HL = G::HL, NKC = G::NKC;
  float lo0 = 0.f, hi0 = 0.f, lo1 = 0.f, hi1 = 0.f;
  if constexpr (G::SHIFT) {  // row 2s: odd taps; row 2s + 1: even taps one row down
    float4 q[HL + 1];
#pragma unroll
    for (int m = 0; m <= HL; ++m) q[m] = sc[(s + HL - m) * NKC + j];
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
  } else {
#pragma unroll
    for (int m = 0; m < HL; ++m) {
      const float4 q = sc[(s + HL - 1 - m) * NKC + j];
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
  st[(2 * s) * NKC + j] = make_float2(lo0, hi0);
  st[(2 * s + 1) * NKC + j] = make_float2(lo1, hi1);
}

// Window of an interior tile held in registers between its loads and its LDS
// writes: wave rows wv + 8k at lane columns, and one tail item per thread.
template <int L, int BC, int TR>
struct FastPre {
  static constexpr int RPW = (FastSynth<L, BC, TR>::NKR + 7) / 8;
  float4 q[RPW];
  float4 qt;
};

// 1a. loads of an interior tile's window: H, V, D, and a unless LDSA (then a
//     is taken from the LDS band by fast_stage). Wave wv loads rows wv, wv + 8,
//     ... at lanes 0..63; the TAILC columns from 64 on go to threads
//     0 .. NKR * TAILC - 1.
template <int L, int BC, int TR, bool LDSA>
__device__ __forceinline__ void fast_fetch(const SynthLevel& d, const SynthWin& w,
                                           FastPre<L, BC, TR>& pre) {
  using G = FastSynth<L, BC, TR>;
  constexpr int NKR = G::NKR, TAILC = G::TAILC, RPW = FastPre<L, BC, TR>::RPW;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int Kc = d.c.K;
  const long long band = (long long)d.r.K * Kc;
  const float* A = static_cast<const float*>(d.a) + (long long)w.img * d.stride_a;
  const float* H = static_cast<const float*>(d.hvd) + (long long)w.img * d.stride_hvd;
  const float* V = H + band;
  const float* D = V + band;
  const int base = w.kwr * Kc + w.kwc;
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int i = wv + 8 * k;
    if (i < NKR) {
      const int o = base + i * Kc + lane;
      pre.q[k] = make_float4(LDSA ? 0.f : A[o], H[o], V[o], D[o]);
    }
  }
  if constexpr (TAILC > 0) {
    if ((int)threadIdx.x < NKR * TAILC) {
      const int ti = threadIdx.x / TAILC, tj = 64 + (threadIdx.x - ti * TAILC);
      const int o = base + ti * Kc + tj;
      pre.qt = make_float4(LDSA ? 0.f : A[o], H[o], V[o], D[o]);
    }
  }
}

// 1b. the fetched window into LDS (with LDSA, a from abuf)
template <int L, int BC, int TR, bool LDSA>
__device__ __forceinline__ void fast_stage(const SynthWin& w, FastPre<L, BC, TR>& pre,
                                           float4* sc, const LdsBand<float>* abuf) {
  using G = FastSynth<L, BC, TR>;
  constexpr int NKR = G::NKR, NKC = G::NKC, TAILC = G::TAILC, RPW = FastPre<L, BC, TR>::RPW;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int i = wv + 8 * k;
    if (i < NKR) {
      if constexpr (LDSA)
        pre.q[k].x = abuf->p[(w.kwr + i - abuf->r0) * abuf->pitch + (w.kwc + lane - abuf->c0)];
      sc[i * NKC + lane] = pre.q[k];
    }
  }
  if constexpr (TAILC > 0) {
    if ((int)threadIdx.x < NKR * TAILC) {
      const int ti = threadIdx.x / TAILC, tj = 64 + (threadIdx.x - ti * TAILC);
      if constexpr (LDSA)
        pre.qt.x = abuf->p[(w.kwr + ti - abuf->r0) * abuf->pitch + (w.kwc + tj - abuf->c0)];
      sc[ti * NKC + tj] = pre.qt;
    }
  }
}

// 2. columns of an interior tile from its staged window: wave wv takes row
//    pairs wv, wv + 8, ...; the pairs' tail columns go to threads
//    0 .. TR / 2 * TAILC - 1
template <int L, int BC, int TR>
__device__ __forceinline__ void fast_columns(const float4* sc, float2* st, const Taps<float>& f) {
  using G = FastSynth<L, BC, TR>;
  constexpr int TAILC = G::TAILC;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int s = wv; s < TR / 2; s += 8) fast_col_pair<L, BC, TR>(sc, st, f, s, lane);
  if constexpr (TAILC > 0) {
    for (int item = threadIdx.x; item < TR / 2 * TAILC; item += 512) {
      const int s = item / TAILC;
      fast_col_pair<L, BC, TR>(sc, st, f, s, 64 + (item - s * TAILC));
    }
  }
}

// 3. rows of an interior tile: wave wv takes output rows wv, wv + 8, ...;
//    lane = output pair
template <int L, int BC, int TR>
__device__ __forceinline__ void fast_rows(const SynthLevel& d, const SynthWin& w, const float2* st,
                                          const Taps<float>& f) {
  using G = FastSynth<L, BC, TR>;
  constexpr int HL = G::HL, NKC = G::NKC;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float* O = static_cast<float*>(d.out) + (long long)w.img * d.stride_out + w.c0 + 2 * lane;
  for (int pr = wv; pr < TR; pr += 8) {
    const float2* row = st + pr * NKC + lane;
    float o0 = 0.f, o1 = 0.f;
    if constexpr (G::SHIFT) {
      float2 v[HL + 1];
#pragma unroll
      for (int m = 0; m <= HL; ++m) v[m] = row[HL - m];
#pragma unroll
      for (int m = 0; m < HL; ++m) {
        o0 += v[m + 1].x * f.h[2 * m + 1];
        o0 += v[m + 1].y * f.g[2 * m + 1];
        o1 += v[m].x * f.h[2 * m];
        o1 += v[m].y * f.g[2 * m];
      }
    } else {
#pragma unroll
      for (int m = 0; m < HL; ++m) {
        const float2 v = row[HL - 1 - m];
        o0 += v.x * f.h[2 * m];
        o0 += v.y * f.g[2 * m];
        o1 += v.x * f.h[2 * m + 1];
        o1 += v.y * f.g[2 * m + 1];
      }
    }
    *reinterpret_cast<float2*>(O + (long long)(w.r0 + pr) * d.c.N) = make_float2(o0, o1);
  }
}

// Steps 1b, 2 and 3 of an interior tile whose window has been fetched into
// pre (see fast_fetch); with LDSA the approximation band is read from abuf.
template <int L, int BC, int TR, bool LDSA = false>
__device__ __forceinline__ void synth_tile_fast_pre(const SynthLevel& d, const Taps<float>& f,
                                                    const SynthWin& w, unsigned char* smem_raw,
                                                    FastPre<L, BC, TR>& pre,
                                                    const LdsBand<float>* abuf = nullptr) {
  using G = FastSynth<L, BC, TR>;
  float4* sc = reinterpret_cast<float4*>(smem_raw);              // [NKR][NKC] (a, H, V, D)
  float2* st = reinterpret_cast<float2*>(sc + G::NKR * G::NKC);  // [TR][NKC] (lo, hi)
  fast_stage<L, BC, TR, LDSA>(w, pre, sc, abuf);
  __syncthreads();
  fast_columns<L, BC, TR>(sc, st, f);
  __syncthreads();
  fast_rows<L, BC, TR>(d, w, st, f);
}

template <int L, int BC, int TR, bool LDSA = false>
__device__ __forceinline__ void synth_tile_fast(const SynthLevel& d, const Taps<float>& f,
                                                const SynthWin& w, unsigned char* smem_raw,
                                                const LdsBand<float>* abuf = nullptr) {
  FastPre<L, BC, TR> pre;
  fast_fetch<L, BC, TR, LDSA>(d, w, pre);
  synth_tile_fast_pre<L, BC, TR, LDSA>(d, f, w, smem_raw, pre, abuf);
}

// Output of synth_rect into a row-major plane (rows of Nc values).
template <typename T>
struct PlaneWriter {
  using V2 = typename Vec<T>::V2;
  T* O;
  int Nc;
  bool pair_store;  // 2-element stores keep their alignment on every row
  __device__ PlaneWriter(T* o, int nc)
      : O(o), Nc(nc),
        pair_store((nc & 1) == 0 && (reinterpret_cast<uintptr_t>(o) & (sizeof(V2) - 1)) == 0) {}
  __device__ void pair(int r, int c, T v0, T v1) {
    T* row = O + (long long)r * Nc;
    if (pair_store) {
      V2 o;
      o.x = v0;
      o.y = v1;
      *reinterpret_cast<V2*>(row + c) = o;
    } else {
      row[c] = v0;
      row[c + 1] = v1;
    }
  }
  __device__ void one(int r, int c, T v) { O[(long long)r * Nc + c] = v; }
};

// Output of synth_rect into an LDS region (rows from r0, columns from c0).
template <typename T>
struct LdsWriter {
  T* p;
  int r0, c0, pitch;
  __device__ void one(int r, int c, T v) { p[(r - r0) * pitch + (c - c0)] = v; }
  __device__ void pair(int r, int c, T v0, T v1) {
    T* q = p + (r - r0) * pitch + (c - c0);
    q[0] = v0;
    q[1] = v1;
  }
};

}  // namespace aw
