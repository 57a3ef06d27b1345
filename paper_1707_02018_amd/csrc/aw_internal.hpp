// Internal declarations shared by the kernel files and the C-ABI layer.
//
// Index conventions (Folberth & Becker, Sec. "A few signal extensions"):
//  * A level maps a length-N signal to K coefficients per band. The zero-
//    boundary core reads the extended signal u(n), n in [0, M), M = N + 2e,
//    where u(n) copies y[src(n - e)].
//  * Synthesis core: s(n) = sum_{m < L/2} c_lo[k0(n) - m] h[2m + par(n)]
//                          + c_hi[k0(n) - m] g[2m + par(n)],
//    k0(n) = (n + L - 2) / 2 (zero / extended modes) or n / 2 (circular),
//    par(n) = n mod 2; coefficients outside [0, K) are zero (circular: mod K).
//  * Analysis core: c_f[k] = sum_{j < L} f[j] u(2k + j - L + 2)  (extended)
//                   c_f[k] = sum_{j < L} f[j] y[(2k + j) mod N]   (circular).
//  * Fold: y[p] = w(p) sum_{i : src(i) = p} s(i + e), w = 1/mult (E^dagger)
//    or 1 (E^*).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aw {

enum Bc { ZPD = 0, SYM = 1, PER = 2, PER_EXT = 3 };

constexpr int kMaxTaps = 16;
constexpr int kMaxRadius = 12;

__host__ __device__ inline int floordiv(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
__host__ __device__ inline int posmod(int a, int b) {
  int r = a % b;
  return r < 0 ? r + b : r;
}

// Sums of NV values over an NT-thread workgroup in a fixed order: a butterfly
// within each wave64, then the NT / 64 wave sums in wave order (LDS red:
// NV x NT / 64 doubles). The totals are left in thread 0's v; every thread of
// the workgroup must call it (one barrier).
template <int NT, int NV>
__device__ inline void block_sums(double (&v)[NV], double* red) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v[q] += __shfl_xor(v[q], m, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q * NW + (threadIdx.x >> 6)] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += red[q * NW + w];
      v[q] = s;
    }
}

// ---------------------------------------------------------------------------
// Extension index maps.

// Source sample of extended position i in [-e, N+e). When N >= e every
// extended sample is at most one reflection (or one period) away, which the
// closed forms cover; shorter signals take the general index arithmetic.
__host__ __device__ inline int src_index(int i, int N, int bc) {
  if (bc == SYM) {
    if (i >= -N && i < 2 * N) return i < 0 ? -1 - i : (i >= N ? 2 * N - 1 - i : i);
    const int j = posmod(i, 2 * N);
    return j < N ? j : 2 * N - 1 - j;
  }
  if (bc == PER_EXT) {
    if (i >= -N && i < 2 * N) return i < 0 ? i + N : (i >= N ? i - N : i);
    return posmod(i, N);
  }
  return i;
}

// Half-point reflexive extension of the blur (any distance): the source of
// position m, and whether m is reached through an odd number of reflections
// (orientation reversed).
__host__ __device__ inline int refl_idx(int m, int N) {
  if (m >= -N && m < 2 * N) return m < 0 ? -1 - m : (m >= N ? 2 * N - 1 - m : m);
  const int j = posmod(m, 2 * N);
  return j < N ? j : 2 * N - 1 - j;
}

__host__ __device__ inline bool refl_odd(int m, int N) {
  if (m >= -N && m < 2 * N) return m < 0 || m >= N;
  return (floordiv(m, N) & 1) != 0;
}

// Calls f(n) for every extended position n = i + e, i in [-e, N+e), whose
// source is p (half-point symmetric: i = p or 2N-1-p modulo 2N; periodic:
// i = p modulo N). Returns the number of preimages (the multiplicity).
template <typename F>
__host__ __device__ inline int for_each_preimage(int p, int N, int e, int bc, F&& f) {
  if (e == 0 || bc == ZPD || bc == PER || (p >= e && p < N - e)) {
    f(p + e);
    return 1;
  }
  int cnt = 1;
  if (N >= e) {  // at most one extra preimage on each side
    f(p + e);
    if (bc == SYM) {
      if (p < e) { f(e - 1 - p); ++cnt; }
      if (p >= N - e) { f(2 * N - 1 - p + e); ++cnt; }
    } else {
      if (p < e) { f(p + N + e); ++cnt; }
      if (p >= N - e) { f(p - N + e); ++cnt; }
    }
    return cnt;
  }
  cnt = 0;
  if (bc == SYM) {
    const int P = 2 * N;
    for (int fam = 0; fam < 2; ++fam) {
      const int base = fam ? (P - 1 - p) : p;
      for (int i = base - P * ((base + e) / P); i < N + e; i += P) {
        f(i + e);
        ++cnt;
      }
    }
  } else {  // PER_EXT
    for (int i = p - N * ((p + e) / N); i < N + e; i += N) {
      f(i + e);
      ++cnt;
    }
  }
  return cnt;
}

__host__ __device__ inline int multiplicity(int p, int N, int e, int bc) {
  return for_each_preimage(p, N, e, bc, [](int) {});
}

// ---------------------------------------------------------------------------
// Tile windows (host and device agree on these).

// Extended-position window [nlo, nhi) holding every preimage of outputs
// [p0, p1) of a half-point symmetric (or zero / circular) fold. Preimages
// other than p + e lie in [0, e) only if p < e, and in [N+e, N+2e) only if
// p >= N - e.
__host__ __device__ inline void fold_window(int p0, int p1, int N, int e, int& nlo, int& nhi) {
  nlo = (p0 < e) ? 0 : p0 + e;
  nhi = (p1 > N - e) ? N + 2 * e : p1 + e;
}

__host__ __device__ inline int synth_k0(int n, int L, int bc) {
  return bc == PER ? (n >> 1) : ((n + L - 2) >> 1);
}

// ---------------------------------------------------------------------------
// Descriptors passed to the kernels.

struct Axis {
  int N;  // signal length at this level (synthesis output / analysis input)
  int K;  // coefficients per band
  int e;  // extension width
};

template <typename T>
struct Taps {
  T h[kMaxTaps];
  T g[kMaxTaps];
};

// One synthesis level: (a, H, V, D) -> out (rows.N x cols.N).
struct SynthLevel {
  const void* a;
  const void* hvd;  // H; V = H + Kr*Kc; D = V + Kr*Kc
  long long stride_a, stride_hvd, stride_out;  // per-image strides (elements)
  void* out;
  Axis r, c;
  int bc;
  int pinv;  // fold weights 1/mult (1) or 1 (0)
};

// Consecutive synthesis levels run as one launch: d[0] is the finest (its
// output goes to memory), d[k] the k-th coarser one (its output, the
// approximation band of d[k-1], stays in LDS).
constexpr int kChainMax = 3;
struct SynthChain {
  SynthLevel d[kChainMax];
  int nl;
  unsigned buf_off[kChainMax];  // LDS byte offsets of the band buffers
  int buf_pitch[kChainMax];     // their row pitches (elements)
};

// One analysis level: in (rows.N x cols.N) -> (a, H, V, D).
struct AnaLevel {
  const void* in;
  void* a;
  void* hvd;
  long long stride_in, stride_a, stride_hvd;
  Axis r, c;
  int bc;
  int pinv;  // extension weights 1/mult (W^*) or 1 (W^dagger)
};

// FISTA update fused into an analysis level's epilogue: each gradient
// coefficient g the level produces is consumed at once,
//   x_k = soft(y_k - g inv_L, thresh),  y_{k+1} = x_k + beta (x_k - x_{k-1}),
// in place in x and y (coefficient-vector layout, images stride_hvd apart),
// with optional per-tile FP64 sums of |x_k|.
struct ProxEpi {
  void* x_hvd;  // x and y at this level's H band
  void* y_hvd;
  void* x_a;    // x and y at a_J (last level), else null: a_j is stored
  void* y_a;
  double inv_L, thresh, beta;
  double* partials;  // [image][pstride]; this level's tiles at pbase + tile
  int pbase, pstride;
  // batched plans: beta_k = beta_tab[k - 1] for the device counter k (clamped
  // to [1, beta_len]) instead of `beta`, and per-tile sums of (x_k - x_{k-1})^2
  const double* beta_tab;
  const int* counter;
  int beta_len;
  double* dx_partials;
};

// Fold of a materialised extended image (rows.N+2e x cols.N+2e) -> out.
struct FoldLevel {
  const void* ext;
  void* out;
  long long stride_ext, stride_out;
  Axis r, c;
  int bc;
  int pinv;
};

template <typename T>
struct SynthItem {
  SynthLevel d;
  Taps<T> f;
  int image;
};
template <typename T>
struct AnaItem {
  AnaLevel d;
  Taps<T> f;
  int image;
  ProxEpi pe;  // fused FISTA update (batched plans)
};

// Item owning tile t of a batched launch: prefix[i] <= t < prefix[i+1]
// (binary search over the n + 1 prefix entries).
__device__ inline int find_item(const int* prefix, int n, int t) {
  int lo = 0, hi = n;  // invariant: prefix[lo] <= t < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

struct BlurDesc {
  int rows, cols, radius;
  double taps[2 * kMaxRadius + 1];
};

template <typename T>
struct BlurArgs {
  int rows, cols;
  int symmetric;               // taps symmetric: the R^* border correction vanishes
  T taps[2 * kMaxRadius + 1];  // correlation order: out[p] = sum_k t[k] in[p - r + k]
};

// Kernel taps of R (ADJ = false: the PSF reversed, so both directions run as
// correlations) or R^* (the PSF as given); symmetric flags the vanishing
// R^* border correction.
template <typename T, bool ADJ>
inline BlurArgs<T> make_blur_args(const BlurDesc& b) {
  BlurArgs<T> a{};
  a.rows = b.rows;
  a.cols = b.cols;
  const int K = 2 * b.radius + 1;
  a.symmetric = 1;
  for (int k = 0; k < K; ++k)
    if (b.taps[k] != b.taps[K - 1 - k]) a.symmetric = 0;
  for (int k = 0; k < K; ++k) a.taps[k] = (T)(ADJ ? b.taps[k] : b.taps[K - 1 - k]);
  return a;
}

template <typename T>
struct BlurItem {
  BlurArgs<T> a;
  const T* x;
  T* y;
  const T* sub;
  double* partials;  // per-tile slots of this image, or null
  int image;
  int tiles_x;
};

// Launchers (return hipSuccess or the launch error). dtype: 0 = float, 1 = double.
hipError_t launch_synth_level(int dtype, int L, const double* lo, const SynthLevel& d, int batch,
                              hipStream_t s);
hipError_t launch_ana_level(int dtype, int L, const double* lo, const AnaLevel& d, int batch,
                            hipStream_t s);
hipError_t launch_fold_level(int dtype, const FoldLevel& d, int batch, hipStream_t s);
size_t synth_level_lds(int dtype, int L, const SynthLevel& d);

// Blur: y = R x; optionally y -= sub (same layout) and per-tile partial sums
// of 1/2 y^2 (double) into partials[image][tile]. Returns tiles per image.
hipError_t launch_blur(int dtype, const BlurDesc& b, int batch, const void* x, void* y,
                       const void* sub, double* partials, hipStream_t s);
hipError_t launch_blur_adjoint(int dtype, const BlurDesc& b, int batch, const void* y, void* x,
                               hipStream_t s);
int blur_tiles(int dtype, const BlurDesc& b);

// Blocks per image of launch_l1_partials over n coefficients.
int fista_prox_blocks(long long n);
// Chained synthesis (FP32, zpd / sym without the two-step fold): fills the
// chain's LDS plan and returns its dynamic LDS bytes (0: not supported).
// A = R W with the finest synthesis level and the blur in one tile pass
// (FP32, zpd / sym / per, filter lengths 2, 8, 16); sub = b or NULL.
bool synth_blur_supported(int L, const SynthLevel& d, const BlurDesc& b);
hipError_t launch_synth_blur(int L, const double* lo, const SynthLevel& d, const BlurDesc& b,
                             const void* sub, void* y, int batch, hipStream_t s);
// A^* = W^* R^* with R^* fused into the finest analysis level (FP32; zpd or
// sym; filter lengths 2, 8, 16); d.in is the image R^* applies to.
bool blur_ana_supported(int L, const AnaLevel& d, const BlurDesc& b);
hipError_t launch_blur_ana(int L, const double* lo, const AnaLevel& d, const BlurDesc& b,
                           int batch, hipStream_t s);
size_t synth_chain_plan(int dtype, int L, SynthChain& c);
// Whether the chain beats one launch per level for this batch: its
// workgroups (one per tile of a_1) recompute halos at about one workgroup per
// CU, so past a few workgroups per CU the per-level kernels are faster.
bool synth_chain_pays(const SynthChain& c, int batch);
hipError_t launch_synth_chain(int L, const double* lo, const SynthChain& c, size_t lds, int batch,
                              hipStream_t s);
// Analysis level with the fused FISTA update (see ProxEpi); tiles per image.
hipError_t launch_ana_level_prox(int dtype, int L, const double* lo, const AnaLevel& d,
                                 const ProxEpi& pe, int batch, hipStream_t s);
int ana_level_tiles(int dtype, const AnaLevel& d, int batch);
// Per-block FP64 partials of ||x||_1 (same block count as the prox update).
hipError_t launch_l1_partials(int dtype, int batch, long long n, const void* x, double* partials,
                              hipStream_t s);
// obj[i*3 + 2] = obj[i*3] + lambda * obj[i*3 + 1]
hipError_t launch_objective_finalize(int batch, double lambda, double* obj, hipStream_t s);
// out[i*out_stride + out_off] = scale * sum_j partials[i][j] (fixed order).
hipError_t launch_reduce_partials(int batch, int nparts, const double* partials, double scale,
                                  double* out, int out_stride, int out_off, hipStream_t s);

// Batched (tile-queue) launches; items / prefix are device arrays.
int synth_tiles(int dtype, int var, const SynthLevel& d);
int ana_tiles(int dtype, int var, const AnaLevel& d);
size_t synth_item_lds(int dtype, int L, int var, const SynthLevel& d);
size_t synth_item_size(int dtype);
size_t ana_item_size(int dtype);
size_t blur_item_size(int dtype);
void make_synth_item(int dtype, const SynthLevel& d, const double* lo, int L, int image, void* out);
void make_ana_item(int dtype, const AnaLevel& d, const double* lo, int L, int image, void* out);
int blur_tiles_var(int dtype, int var, const BlurDesc& b, int* tiles_x);
void make_blur_item(int dtype, bool adj, const BlurDesc& b, const void* x, void* y, const void* sub,
                    double* partials, int image, int tiles_x, void* out);
hipError_t launch_synth_batch(int dtype, int L, int bc, int var, const void* items,
                              const int* prefix, int n, int total, const int* active, size_t lds,
                              hipStream_t s);
hipError_t launch_ana_batch(int dtype, int L, int bc, int var, const void* items,
                            const int* prefix, int n, int total, const int* active, hipStream_t s,
                            bool prox = false);
void make_ana_item_prox(const AnaLevel& d, const double* lo, int L, int image, const ProxEpi& pe,
                        void* out);
hipError_t launch_blur_batch(int dtype, int radius, bool adj, int var, const void* items,
                             const int* prefix, int n, int total, const int* active,
                             hipStream_t s);

// shared_s: every pair reads the one signal s (multi-channel blind estimation)
hipError_t launch_conv_pair(int dtype, int batch, int K, int N, const void* h, const void* s,
                            const void* x_obs, void* resid, void* grad_h, void* grad_s,
                            hipStream_t st, bool shared_s = false);

// R by DCT-II diagonalisation (dct.hip). Device tables in the transform's
// dtype: lam_r / lam_c the eigenvalues along the rows axis (length rows) and
// the columns axis (length cols); fft_* [N] complex exp(-2 pi i j / N) and
// dct_* [N] complex exp(-i pi k / 2N) for N = rows (_r) and N = cols (_c),
// complex values as (re, im) pairs. w1, w2 hold batch * rows * cols values
// each; x may alias y.
struct DctTables {
  const void *lam_r, *lam_c, *fft_r, *dct_r, *fft_c, *dct_c;
};
size_t blur_dct_lds(int dtype, int n);
hipError_t launch_blur_dct(int dtype, int rows, int cols, int batch, const DctTables& tb,
                           const void* x, void* y, void* w1, void* w2, hipStream_t s);

// Multi-channel blind channel estimation helpers (blind.hip).
hipError_t launch_sum_rows(int dtype, int rows, long long n, const void* in, void* out,
                           hipStream_t s);
hipError_t launch_row_sumsq(int dtype, int rows, long long n, const void* x, double* out,
                            hipStream_t s);
hipError_t launch_huber_tv(int dtype, int batch, int K, const void* h, double delta,
                           double gscale, void* grad, double* value, hipStream_t s);
hipError_t launch_prox_l1(int dtype, long long n, const void* x, const void* g, double step,
                          double thresh, void* out, double* stats, hipStream_t s);

// ------------------------------------------------------ XCD-aware tile order
// Workgroups are dispatched round-robin over the 8 XCDs (id % 8), each with
// its own L2. Renumbering so that XCD k runs the contiguous range k*n/8 ..
// (k+1)*n/8 of row-major tiles keeps a tile's halo neighbours in the same L2.
// A bijection on [0, n) for every n.
constexpr unsigned kXcds = 8;

__device__ __forceinline__ unsigned xcd_remap(unsigned pid, unsigned n) {
  const unsigned per = (n + kXcds - 1) / kXcds;
  const unsigned tall = n % kXcds == 0 ? kXcds : n % kXcds;  // XCDs with `per` tiles
  const unsigned xcd = pid % kXcds, local = pid / kXcds;
  return xcd < tall ? xcd * per + local : tall * per + (xcd - tall) * (per - 1) + local;
}

// (x, y, z) tile of this workgroup in a 3-D grid, XCD-aware.
__device__ __forceinline__ void xcd_tile(int& tx, int& ty, int& tz) {
  const unsigned gx = gridDim.x, gy = gridDim.y;
  const unsigned n = gx * gy * gridDim.z;
  const unsigned l = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), n);
  tx = (int)(l % gx);
  ty = (int)((l / gx) % gy);
  tz = (int)(l / (gx * gy));
}

// ------------------------------------------------------------ warm-start CNN
// Six 3x3 layers 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 (zero 'same' padding,
// bias, ReLU on the first five). Master parameters are FP32, one flat vector
// layer by layer: weight [out][in][3][3] then bias [out]. Activations are BF16,
// channels last: [image][row][col][32].
constexpr int kCnnCh = 32;
constexpr long long kCnnParams = 37601;
constexpr long long kCnnMasterW1 = 0, kCnnMasterB1 = 288;
constexpr long long cnn_master_mid(int m) { return 320 + 9248LL * m; }  // layers 2..5
constexpr long long kCnnMasterW6 = 320 + 4 * 9248LL, kCnnMasterB6 = kCnnMasterW6 + 288;

// Byte offsets of the packed (device) parameter buffer made from the master vector.
struct CnnPack {
  static constexpr size_t w1 = 0;                          // bf16 [9][32]: W1[c][0][t]
  static constexpr size_t b1 = w1 + 9 * 32 * 2;             // f32 [32]
  static constexpr size_t mid = b1 + 32 * 4;                // four mid layers
  static constexpr size_t mid_fwd = 0;                      // bf16 [9][32 out][32 in]
  static constexpr size_t mid_dgrad = 9 * 32 * 32 * 2;      // bf16 [9][32 in][32 out], taps mirrored
  static constexpr size_t mid_bias = 2 * 9 * 32 * 32 * 2;   // f32 [32]
  static constexpr size_t mid_size = mid_bias + 32 * 4;
  static constexpr size_t w6 = mid + 4 * mid_size;          // bf16 [9][32 out][32 in], out > 0 zero
  static constexpr size_t b6 = w6 + 9 * 32 * 32 * 2;        // f32 [32], entry 0 used
  static constexpr size_t w6d = b6 + 32 * 4;                // bf16 [9][32]: W6[0][c][8 - t]
  static constexpr size_t total = w6d + 9 * 32 * 2;
};

hipError_t launch_cnn_pack(const float* master, void* packed, hipStream_t s);
hipError_t launch_cnn_forward(const void* packed, int n, int H, int W, const float* b, void* acts,
                              float* u, hipStream_t s);
// Scratch (bytes) of launch_cnn_backward for this shape.
size_t cnn_backward_scratch(int n, int H, int W);
hipError_t launch_cnn_backward(const void* packed, int n, int H, int W, const float* b,
                               const void* acts, const float* du, void* dacts, float* grad,
                               void* scratch, hipStream_t s);
hipError_t launch_adam(float* p, float* m, float* v, const float* g, long long n, double lr,
                       double beta1, double beta2, double eps, double c1, double c2,
                       hipStream_t s);
// grad = scale * 2 (c - t) (if grad != null); partials[b] = FP64 block sums of (c - t)^2
int sq_error_blocks(long long n);
hipError_t launch_sq_error(long long n, const float* c, const float* t, float scale, float* grad,
                           double* partials, hipStream_t s);
hipError_t launch_soft_threshold(long long n, const float* in, float tau, float* out,
                                 hipStream_t s);

}  // namespace aw
