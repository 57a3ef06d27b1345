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
#include "aw_internal.hpp"

namespace aw {

template <typename T>
struct SynthTile;
template <>
struct SynthTile<float> {
  static constexpr int TR = 32, TC = 64;
};
template <>
struct SynthTile<double> {
  static constexpr int TR = 16, TC = 64;
};
template <typename T>
struct AnaTile;
template <>
struct AnaTile<float> {
  static constexpr int TKR = 16, TKC = 32;
};
template <>
struct AnaTile<double> {
  static constexpr int TKR = 16, TKC = 32;
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
template <typename T, int L, int BC>
__global__ __launch_bounds__(256) void synth_level_kernel(SynthLevel d, Taps<T> f) {
  constexpr int TR = SynthTile<T>::TR, TC = SynthTile<T>::TC;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);

  const int img = blockIdx.z;
  const int Nr = d.r.N, Nc = d.c.N, Kr = d.r.K, Kc = d.c.K;
  const int er = (BC == SYM) ? d.r.e : 0;
  const int ec = (BC == SYM) ? d.c.e : 0;
  const int r0 = blockIdx.y * TR, r1 = min(r0 + TR, Nr);
  const int c0 = blockIdx.x * TC, c1 = min(c0 + TC, Nc);
  int nlo_r, nhi_r, nlo_c, nhi_c;
  fold_window(r0, r1, Nr, er, nlo_r, nhi_r);
  fold_window(c0, c1, Nc, ec, nlo_c, nhi_c);
  const int kwr = synth_k0(nlo_r, L, BC) - (L / 2 - 1);
  const int nkr = synth_k0(nhi_r - 1, L, BC) + 1 - kwr;
  const int kwc = synth_k0(nlo_c, L, BC) - (L / 2 - 1);
  const int nkc = synth_k0(nhi_c - 1, L, BC) + 1 - kwc;
  const int nwin = nkr * nkc;

  T* sc = smem;             // [4][nkr][nkc] coefficient window: a, H, V, D
  T* st = smem + 4 * nwin;  // [2][TR][nkc]  column-synthesised lo / hi

  const T* A = static_cast<const T*>(d.a) + (long long)img * d.stride_a;
  const T* HVD = static_cast<const T*>(d.hvd) + (long long)img * d.stride_hvd;
  const long long band = (long long)Kr * Kc;

  // 1. stage the coefficient window (zero outside [0,K); circular wraps)
  for (int idx = threadIdx.x; idx < 4 * nwin; idx += blockDim.x) {
    const int b = idx / nwin;
    const int rem = idx - b * nwin;
    const int i = rem / nkc;
    const int j = rem - i * nkc;
    int kr = kwr + i, kc = kwc + j;
    bool ok;
    if (BC == PER) {
      kr = posmod(kr, Kr);
      kc = posmod(kc, Kc);
      ok = true;
    } else {
      ok = (kr >= 0) && (kr < Kr) && (kc >= 0) && (kc < Kc);
    }
    T v = T(0);
    if (ok) {
      const long long off = (long long)kr * Kc + kc;
      v = (b == 0) ? A[off] : HVD[(b - 1) * band + off];
    }
    sc[idx] = v;
  }
  __syncthreads();

  // 2. column-direction synthesis (along rows) with the row fold
  const int nrows = r1 - r0;
  for (int idx = threadIdx.x; idx < nrows * nkc; idx += blockDim.x) {
    const int pr = idx / nkc;
    const int j = idx - pr * nkc;
    T lo = T(0), hi = T(0);
    const int cnt = for_each_preimage(r0 + pr, Nr, er, BC, [&](int n) {
      const int base = synth_k0(n, L, BC) - kwr;
      const bool odd = n & 1;
#pragma unroll
      for (int m = 0; m < L / 2; ++m) {
        const T fh = odd ? f.h[2 * m + 1] : f.h[2 * m];
        const T fg = odd ? f.g[2 * m + 1] : f.g[2 * m];
        const int row = base - m;
        lo += sc[(0 * nkr + row) * nkc + j] * fh + sc[(1 * nkr + row) * nkc + j] * fg;
        hi += sc[(2 * nkr + row) * nkc + j] * fh + sc[(3 * nkr + row) * nkc + j] * fg;
      }
    });
    if (d.pinv && cnt > 1) {
      const T w = T(1) / T(cnt);
      lo *= w;
      hi *= w;
    }
    st[pr * nkc + j] = lo;
    st[(TR + pr) * nkc + j] = hi;
  }
  __syncthreads();

  // 3. row-direction synthesis (along columns) with the column fold
  const int ncols = c1 - c0;
  T* O = static_cast<T*>(d.out) + (long long)img * d.stride_out;
  for (int idx = threadIdx.x; idx < nrows * ncols; idx += blockDim.x) {
    const int pr = idx / ncols;
    const int pc = idx - pr * ncols;
    const T* slo = st + pr * nkc;
    const T* shi = st + (TR + pr) * nkc;
    T acc = T(0);
    const int cnt = for_each_preimage(c0 + pc, Nc, ec, BC, [&](int n) {
      const int base = synth_k0(n, L, BC) - kwc;
      const bool odd = n & 1;
#pragma unroll
      for (int m = 0; m < L / 2; ++m) {
        const T fh = odd ? f.h[2 * m + 1] : f.h[2 * m];
        const T fg = odd ? f.g[2 * m + 1] : f.g[2 * m];
        acc += slo[base - m] * fh + shi[base - m] * fg;
      }
    });
    if (d.pinv && cnt > 1) acc *= T(1) / T(cnt);
    O[(long long)(r0 + pr) * Nc + (c0 + pc)] = acc;
  }
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

template <typename T>
static size_t synth_lds_t(int L, const SynthLevel& d) {
  const int mr = synth_max_window(d.r, L, d.bc, SynthTile<T>::TR);
  const int mc = synth_max_window(d.c, L, d.bc, SynthTile<T>::TC);
  return sizeof(T) * (size_t)(4 * mr * mc + 2 * SynthTile<T>::TR * mc);
}

size_t synth_level_lds(int dtype, int L, const SynthLevel& d) {
  return dtype ? synth_lds_t<double>(L, d) : synth_lds_t<float>(L, d);
}

template <typename T, int L, int BC>
static hipError_t launch_synth_t(const double* lo, const SynthLevel& d, int batch, hipStream_t s) {
  const size_t lds = synth_lds_t<T>(L, d);
  auto kern = synth_level_kernel<T, L, BC>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((d.c.N + SynthTile<T>::TC - 1) / SynthTile<T>::TC,
            (d.r.N + SynthTile<T>::TR - 1) / SynthTile<T>::TR, batch);
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, d, make_taps<T>(lo, L));
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
template <typename T, int L, int BC>
__global__ __launch_bounds__(256) void ana_level_kernel(AnaLevel d, Taps<T> f) {
  constexpr int TKR = AnaTile<T>::TKR, TKC = AnaTile<T>::TKC;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);

  const int img = blockIdx.z;
  const int Nr = d.r.N, Nc = d.c.N, Kr = d.r.K, Kc = d.c.K;
  const int er = d.r.e, ec = d.c.e;
  const int kr0 = blockIdx.y * TKR, kr1 = min(kr0 + TKR, Kr);
  const int kc0 = blockIdx.x * TKC, kc1 = min(kc0 + TKC, Kc);
  const int nlo_r = (BC == PER) ? 2 * kr0 : 2 * kr0 - L + 2;
  const int nlo_c = (BC == PER) ? 2 * kc0 : 2 * kc0 - L + 2;
  const int nwr = 2 * (kr1 - kr0) + L - 2;
  const int nwc = 2 * (kc1 - kc0) + L - 2;
  const int Mr = Nr + 2 * er, Mc = Nc + 2 * ec;

  T* su = smem;             // [nwr][nwc] extended, weighted input window
  T* sl = su + nwr * nwc;   // [nwr][TKC] low-pass along columns
  T* sh = sl + nwr * TKC;   // [nwr][TKC] high-pass along columns

  const T* Y = static_cast<const T*>(d.in) + (long long)img * d.stride_in;
  const bool edge_r = (BC != PER) && (nlo_r < 2 * er || nlo_r + nwr > Nr);
  const bool edge_c = (BC != PER) && (nlo_c < 2 * ec || nlo_c + nwc > Nc);

  // 1. gather u(n) = w(src) y[src(n - e)] (zero outside [0, M))
  for (int idx = threadIdx.x; idx < nwr * nwc; idx += blockDim.x) {
    const int i = idx / nwc;
    const int j = idx - i * nwc;
    const int nr = nlo_r + i, nc = nlo_c + j;
    T v = T(0);
    if (BC == PER) {
      v = Y[(long long)posmod(nr, Nr) * Nc + posmod(nc, Nc)];
    } else if (nr >= 0 && nr < Mr && nc >= 0 && nc < Mc) {
      const int sr = edge_r ? src_index(nr - er, Nr, BC) : nr - er;
      const int scc = edge_c ? src_index(nc - ec, Nc, BC) : nc - ec;
      v = Y[(long long)sr * Nc + scc];
      if (d.pinv) {
        const int m = (edge_r ? multiplicity(sr, Nr, er, BC) : 1) *
                      (edge_c ? multiplicity(scc, Nc, ec, BC) : 1);
        if (m > 1) v = v / T(m);
      }
    }
    su[idx] = v;
  }
  __syncthreads();

  // 2. filter along columns: sl/sh[i][kk] = sum_j f[j] u(i, 2 kk + j)
  const int nkc_t = kc1 - kc0;
  for (int idx = threadIdx.x; idx < nwr * nkc_t; idx += blockDim.x) {
    const int i = idx / nkc_t;
    const int kk = idx - i * nkc_t;
    const T* row = su + i * nwc + 2 * kk;
    T lo = T(0), hi = T(0);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      lo += f.h[j] * row[j];
      hi += f.g[j] * row[j];
    }
    sl[i * TKC + kk] = lo;
    sh[i * TKC + kk] = hi;
  }
  __syncthreads();

  // 3. filter along rows and write the four bands
  T* Aout = static_cast<T*>(d.a) + (long long)img * d.stride_a;
  T* HVD = static_cast<T*>(d.hvd) + (long long)img * d.stride_hvd;
  const long long band = (long long)Kr * Kc;
  const int nkr_t = kr1 - kr0;
  for (int idx = threadIdx.x; idx < nkr_t * nkc_t; idx += blockDim.x) {
    const int ii = idx / nkc_t;
    const int kk = idx - ii * nkc_t;
    T a = T(0), H = T(0), V = T(0), D = T(0);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const T l = sl[(2 * ii + j) * TKC + kk];
      const T h = sh[(2 * ii + j) * TKC + kk];
      a += f.h[j] * l;
      H += f.g[j] * l;
      V += f.h[j] * h;
      D += f.g[j] * h;
    }
    const long long off = (long long)(kr0 + ii) * Kc + (kc0 + kk);
    Aout[off] = a;
    HVD[off] = H;
    HVD[band + off] = V;
    HVD[2 * band + off] = D;
  }
}

template <typename T, int L, int BC>
static hipError_t launch_ana_t(const double* lo, const AnaLevel& d, int batch, hipStream_t s) {
  constexpr int TKR = AnaTile<T>::TKR, TKC = AnaTile<T>::TKC;
  const int nwr = 2 * TKR + L - 2, nwc = 2 * TKC + L - 2;
  const size_t lds = sizeof(T) * (size_t)(nwr * nwc + 2 * nwr * TKC);
  auto kern = ana_level_kernel<T, L, BC>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((d.c.K + TKC - 1) / TKC, (d.r.K + TKR - 1) / TKR, batch);
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, d, make_taps<T>(lo, L));
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
