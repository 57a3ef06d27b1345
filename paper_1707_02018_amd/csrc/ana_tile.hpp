// Analysis tile (W^dagger = Phi E per level, and the true adjoint
// W^* = Phi (E^dagger)^*, eq. 2), shared by the per-level and batched kernels
// (wavelet.hip) and the fused blur-adjoint + analysis kernel (fused.hip).
//
// A workgroup owns TKR x TKC coefficients of every band. It gathers the
// extended input window (extension index map and 1/mult weights applied during
// the gather), filters along columns into LDS, then along rows, and writes a,
// H, V, D, or, with PROX, applies the FISTA update to them in place.
//
// With BR >= 0 the window is filled with R^* r instead of read: the blur
// adjoint (radius BR, half-point reflexive boundaries) runs over the image
// samples the window reads, which are scattered to the window positions whose
// source they are, with the same weights. The values equal those R^* writes
// to memory, so the result is bitwise that of R^* followed by the analysis.
#pragma once

#include <climits>
#include <type_traits>

#include "aw_internal.hpp"
#include "synth_tile.hpp"

namespace aw {

// LDS of the fused blur adjoint over an NWR x NWC analysis window: the
// reflected image window (rows + 2 BR, row stride SXS, slack for the
// vector reads past the last column) and the column-pass output (stride SHS,
// rows padded for the four-row chunks of the row pass).
template <typename T, int BR, int NWR, int NWC>
struct BlurAdjGeom {
  static constexpr int VW = 16 / sizeof(T);
  static constexpr int WRM = NWR + 2 * BR, WCM = NWC + 2 * BR;
  static constexpr int SXS = ((WCM + 2 * VW + VW - 1) / VW) * VW;
  static constexpr int SHS = ((NWC + VW - 1) / VW) * VW;
  static constexpr int CR = 4;
  static constexpr int SX = WRM * SXS, SH = (WRM + CR) * SHS;
};

// Extent [z0, z1) of the samples of a signal of length N that an analysis
// window over extended positions [nlo, nlo + NW) reads (zero or half-point
// symmetric extension by e with N >= e; positions outside the extended signal
// read nothing).
__device__ inline void window_sources(int nlo, int NW, int N, int e, int bc, int& z0, int& z1) {
  const int a = max(nlo, 0) - e, b = min(nlo + NW, N + 2 * e) - e;  // signal positions [a, b)
  int lo = INT_MAX, hi = INT_MIN;
  if (max(a, 0) < min(b, N)) {
    lo = max(a, 0);
    hi = min(b, N);
  }
  if (bc == SYM) {
    if (a < min(b, 0)) {  // s < 0 reads -1 - s
      lo = min(lo, -min(b, 0));
      hi = max(hi, -a);
    }
    if (max(a, N) < b) {  // s >= N reads 2N - 1 - s
      lo = min(lo, 2 * N - b);
      hi = max(hi, 2 * N - max(a, N));
    }
  }
  if (lo >= hi) lo = hi = 0;
  z0 = lo;
  z1 = hi;
}

// R^* of the image Y over the samples the window reads, written to the window
// su (stride SUS) at every position whose source each sample is, times the
// extension weights (1/mult when pinv). sx and sh are the LDS of
// BlurAdjGeom; sx may share su's space. Arithmetic and order as in the blur
// tile kernel: correlation taps over the reflected window, then the border
// correction of the odd-reflection samples, columns first.
template <typename T, int BC, int R, int NWR, int NWC, int SUS>
__device__ __forceinline__ void stage_blur_adjoint(const BlurArgs<T>& a, const T* __restrict__ Y,
                                                   int nlo_r, int nlo_c, int er, int ec, int Nr,
                                                   int Nc, int pinv, bool interior, T* su, T* sx,
                                                   T* sh) {
  using G = BlurAdjGeom<T, R, NWR, NWC>;
  using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  constexpr int VW = G::VW, SXS = G::SXS, SHS = G::SHS, CR = G::CR, NT = 512;
  constexpr int K = 2 * R + 1;
  constexpr int NV = (VW + 2 * R + VW - 1) / VW;
  __shared__ int rt[G::WRM], ct[G::WCM];

  int zr0, zr1, zc0, zc1;
  if (interior) {
    zr0 = nlo_r - er;
    zr1 = zr0 + NWR;
    zc0 = nlo_c - ec;
    zc1 = zc0 + NWC;
  } else {
    window_sources(nlo_r, NWR, Nr, er, BC, zr0, zr1);
    window_sources(nlo_c, NWC, Nc, ec, BC, zc0, zc1);
  }
  const int ZR = zr1 - zr0, ZC = zc1 - zc0;
  const int WR = ZR + 2 * R, WC = ZC + 2 * R;
  T t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = a.taps[k];

  // reflected image window: rows zr0 - R .. zr1 + R, columns zc0 - R .. zc1 + R
  for (int i = threadIdx.x; i < WR + WC; i += NT) {
    if (i < WR)
      rt[i] = refl_idx(zr0 - R + i, Nr);
    else
      ct[i - WR] = refl_idx(zc0 - R + (i - WR), Nc);
  }
  __syncthreads();
  constexpr int IT = (G::WRM * G::WCM + NT - 1) / NT;
  T v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx < WR * WC) {
      const int i = idx / WC, j = idx - (idx / WC) * WC;
      v[it] = Y[(long long)rt[i] * Nc + ct[j]];
    }
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx < WR * WC) {
      const int i = idx / WC, j = idx - (idx / WC) * WC;
      sx[i * SXS + j] = v[it];
    }
  }
  for (int idx = threadIdx.x; idx < WR * (SXS - WC); idx += NT) {
    const int i = idx / (SXS - WC), j = idx - (idx / (SXS - WC)) * (SXS - WC);
    sx[i * SXS + WC + j] = T(0);
  }
  __syncthreads();

  // columns: sh[i][pc] = sum_k t[k] sx[i][pc + k], VW outputs per item
  const int QV = (ZC + VW - 1) / VW;
  for (int item = threadIdx.x; item < WR * QV; item += NT) {
    const int i = item / QV, q = item - (item / QV) * QV;
    const T* row = sx + i * SXS + q * VW;
    T w[NV * VW];
#pragma unroll
    for (int vv = 0; vv < NV; ++vv) {
      const V x = *reinterpret_cast<const V*>(row + vv * VW);
      const T* e = reinterpret_cast<const T*>(&x);
#pragma unroll
      for (int u = 0; u < VW; ++u) w[vv * VW + u] = e[u];
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
    *reinterpret_cast<V*>(sh + i * SHS + q * VW) = ov;
  }
  if (!a.symmetric) {  // border columns: odd-reflection samples take the convolution tap
    __syncthreads();
    for (int item = threadIdx.x; item < WR * ZC; item += NT) {
      const int i = item / ZC, pc = item - (item / ZC) * ZC;
      const int p = zc0 + pc;
      if (p >= R && p < Nc - R) continue;
      T acc = T(0);
#pragma unroll 1
      for (int k = 0; k < K; ++k)
        if (refl_odd(p - R + k, Nc)) acc += (a.taps[K - 1 - k] - a.taps[k]) * sx[i * SXS + pc + k];
      sh[i * SHS + pc] += acc;
    }
  }
  __syncthreads();  // sx is dead from here: su may take its space
  if (!interior) {
    for (int idx = threadIdx.x; idx < NWR * SUS; idx += NT) su[idx] = T(0);
    __syncthreads();
  }

  // rows: each item one column and CR consecutive rows
  const int NCH = (ZR + CR - 1) / CR;
  for (int item = threadIdx.x; item < ZC * NCH; item += NT) {
    const int ch = item / ZC, pc = item - (item / ZC) * ZC;
    const int i0 = ch * CR;
    T hw[CR + 2 * R];
#pragma unroll
    for (int i = 0; i < CR + 2 * R; ++i) hw[i] = sh[(i0 + i) * SHS + pc];
#pragma unroll
    for (int i = 0; i < CR; ++i) {
      if (i0 + i >= ZR) break;
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < K; ++k) acc += t[k] * hw[i + k];
      const int p_r = zr0 + i0 + i, p_c = zc0 + pc;
      if (!a.symmetric && (p_r < R || p_r >= Nr - R)) {
#pragma unroll 1
        for (int k = 0; k < K; ++k)
          if (refl_odd(p_r - R + k, Nr))
            acc += (a.taps[K - 1 - k] - a.taps[k]) * sh[(i0 + i + k) * SHS + pc];
      }
      if (interior) {
        su[(i0 + i) * SUS + pc] = acc;
      } else {
        const T wr = pinv ? T(1) / T(multiplicity(p_r, Nr, er, BC)) : T(1);
        const T wc = pinv ? T(1) / T(multiplicity(p_c, Nc, ec, BC)) : T(1);
        const T val = acc * (wr * wc);
        for_each_preimage(p_r, Nr, er, BC, [&](int n) {
          const int si = n - nlo_r;
          if (si < 0 || si >= NWR) return;
          for_each_preimage(p_c, Nc, ec, BC, [&](int m) {
            const int sj = m - nlo_c;
            if (sj >= 0 && sj < NWC) su[si * SUS + sj] = val;
          });
        });
      }
    }
  }
}

template <typename T, int L, int BC, int VAR, bool PROX = false, int BR = -1>
__device__ __forceinline__ void ana_tile(const AnaLevel& d, const Taps<T>& f, int bx, int by,
                                         int img, const ProxEpi& pe = ProxEpi{},
                                         const BlurArgs<T>* ba = nullptr) {
  constexpr int TKR = AnaTile<T, VAR>::TKR, TKC = AnaTile<T, VAR>::TKC, NT = AnaTile<T, VAR>::NT;
  // output ownership of step 3: thread = column kk, KB consecutive rows
  constexpr int RBLK = NT / TKC;
  constexpr int KB = TKR / RBLK;
  const int kk = threadIdx.x % TKC;
  const int rb = threadIdx.x / TKC;
  constexpr int NWR = 2 * TKR + L - 2, NWC = 2 * TKC + L - 2;
  constexpr int VW = 16 / sizeof(T);                       // elements per 16-byte LDS read
  constexpr int SUS = ((NWC + VW - 1) / VW) * VW + VW;     // input row stride
  constexpr int NV = (2 * VW + L - 2 + VW - 1) / VW;       // vectors per pass-1 item
  using V2 = typename Vec<T>::V2;
  using V4 = typename Vec<T>::V4;
  // LDS: the staged input su and the column-pass output slh; with the fused
  // blur adjoint (BR >= 0) the blur window shares su's space and the blur's
  // column pass shares slh's (each is dead before the other is written)
  using BG = BlurAdjGeom<T, (BR < 0 ? 0 : BR), NWR, NWC>;
  constexpr int A_EL = BR < 0 ? 1 : (NWR * SUS > BG::SX ? NWR * SUS : BG::SX);
  constexpr int B_EL = BR < 0 ? 1 : (2 * NWR * TKC > BG::SH ? 2 * NWR * TKC : BG::SH);
  __shared__ __align__(16) T su_s[BR < 0 ? NWR * SUS : 1];
  __shared__ __align__(16) V2 slh_s[BR < 0 ? NWR * TKC : 1];
  __shared__ __align__(16) T lds_a[A_EL];
  __shared__ __align__(16) T lds_b[B_EL];
  T* su = BR < 0 ? su_s : lds_a;
  V2* slh = BR < 0 ? slh_s : reinterpret_cast<V2*>(lds_b);

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
  //    of a thread are issued before its LDS writes. With BR >= 0 the input
  //    is R^* of the image at d.in, computed into the window instead.
  if constexpr (BR >= 0) {
    stage_blur_adjoint<T, BC, BR, NWR, NWC, SUS>(*ba, Y, nlo_r, nlo_c, er, ec, Nr, Nc, d.pinv,
                                                 interior, su, lds_a, lds_b);
  } else if (interior && (Nc % VW) == 0) {
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

  // fused update: y_k and x_{k-1} of the owned coefficients are fetched once
  // the window is staged, so their latency overlaps the column pass (fetched
  // before the staging, they held registers that cost a workgroup per CU)
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
  double l1 = 0.0, dx = 0.0;
  T beta = T(0);
  if constexpr (PROX) {
    if (pe.beta_tab) {
      int k = *pe.counter;
      k = k < 1 ? 1 : (k > pe.beta_len ? pe.beta_len : k);
      beta = (T)pe.beta_tab[k - 1];
    } else {
      beta = (T)pe.beta;
    }
  }
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
        const T il = (T)pe.inv_L, th = (T)pe.thresh, be = beta;
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
          dx += (double)(xn[q] - px[r][q]) * (double)(xn[q] - px[r][q]);
        }
        if (pe.x_a) {
          const long long oa = (long long)img * d.stride_a + off;
          static_cast<T*>(pe.y_a)[oa] = xn[0] + be * (xn[0] - px[r][0]);
          static_cast<T*>(pe.x_a)[oa] = xn[0];
          l1 += (double)(xn[0] < T(0) ? -xn[0] : xn[0]);
          dx += (double)(xn[0] - px[r][0]) * (double)(xn[0] - px[r][0]);
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
    if (pe.partials) {  // fixed-order tile sums of |x_k| (and (x_k - x_{k-1})^2)
      __shared__ double red[2 * NT / 64];
      double v[2] = {l1, dx};
      block_sums<NT, 2>(v, red);
      if (threadIdx.x == 0) {
        const int gx = (Kc + TKC - 1) / TKC;
        const long long slot = (long long)img * pe.pstride + pe.pbase + by * gx + bx;
        pe.partials[slot] = v[0];
        if (pe.dx_partials) pe.dx_partials[slot] = v[1];
      }
    }
  }
}

}  // namespace aw
