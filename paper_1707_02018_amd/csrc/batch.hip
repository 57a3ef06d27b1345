// Batched FISTA over images of uneven size, depth, filter and PSF.
//
// A plan fixes n problems; binding device buffers builds, per pipeline stage,
// a tile queue per kernel class (filter length x boundary mode for the wavelet
// levels, PSF radius for the blur): descriptor items plus a prefix of tile
// counts, uploaded once. One iteration enqueues, for every stage, one launch
// per class over all tiles of all images of that class:
//   W levels J..1 -> R(.) - b (+ residual partials) -> R^* -> W^* levels 1..J,
//   each analysis tile applying the proximal/momentum update to the
//   coefficients it produces (beta_k from a device table indexed by a device
//   iteration counter; per-tile partials of ||x_k||_1 and ||x_k - x_{k-1}||^2)
//   -> per-image objective sums -> counter++.
// Classes of one stage are independent and run on forked streams. Nothing is
// allocated, copied or synchronised per iteration and every kernel reads its
// varying inputs from device memory, so an iteration can be captured once into
// a hipGraph and replayed. Images whose active flag is 0 skip all their tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <cstring>
#include <string>
#include <vector>

#include "aw_internal.hpp"

namespace aw {

template <typename T, bool ADJ>
BlurArgs<T> make_blur_args(const BlurDesc& b);

// ------------------------------------------------------------ device kernels
// obj[i] = {1/2 ||A y - b||^2, ||x||_1, ||x_k - x_{k-1}||^2}: fixed-order sums
// over the image's tile and block ranges; inactive images keep their values.
__global__ __launch_bounds__(256) void batch_reduce_kernel(
    int n, const int* __restrict__ tile_prefix, const double* __restrict__ r_part,
    const int* __restrict__ blk_prefix, const double* __restrict__ l1_part,
    const double* __restrict__ dx_part, const int* __restrict__ active, double* __restrict__ obj) {
  __shared__ double red[3 * 256 / 64];
  const int i = blockIdx.x;
  if (i >= n || (active && !active[i])) return;
  double v[3] = {0.0, 0.0, 0.0};
  for (int t = tile_prefix[i] + threadIdx.x; t < tile_prefix[i + 1]; t += 256) v[0] += r_part[t];
  for (int t = blk_prefix[i] + threadIdx.x; t < blk_prefix[i + 1]; t += 256) {
    v[1] += l1_part[t];
    v[2] += dx_part[t];
  }
  block_sums<256, 3>(v, red);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) obj[3 * i + q] = v[q];
}

__global__ void batch_counter_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] += 1;
}

// counter = 1, active = 1, x = y = 0 (fill kernels, capture-safe)
template <typename T>
__global__ void batch_reset_kernel(int* counter, int* active, int n, T* x, T* y, long long ncoef) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) counter[0] = 1;
  if (i < n) active[i] = 1;
  for (long long j = i; j < ncoef; j += (long long)gridDim.x * blockDim.x) {
    x[j] = T(0);
    y[j] = T(0);
  }
}

}  // namespace aw

// =================================================================== plan
#include "../../include/adjwave.h"

namespace {

constexpr int kBetaLen = 1 << 17;  // beta_k for k <= 131072 (clamped beyond)
constexpr size_t kAlignB = 256;
size_t alignb(size_t x) { return (x + kAlignB - 1) / kAlignB * kAlignB; }

struct Image {
  aw_wavelet w;
  double taps[2 * AW_MAX_TAPS];  // tap source of make_taps: the low-pass in both halves
  aw::BlurDesc b;
  int J, L, bc, e, rows, cols;
  int sr[AW_MAX_LEVELS + 1], sc[AW_MAX_LEVELS + 1];
  long long ncoef, npix;
  long long off_hvd[AW_MAX_LEVELS + 1];
  // workspace offsets (bytes)
  size_t a_off[AW_MAX_LEVELS + 1], tmp_off, res_off;
};

struct Group {        // one launch
  int kind;           // 0 synth, 1 analysis, 2 blur, 3 blur adjoint
  int key0, key1;     // (L, bc) or (radius, 0)
  int var = 0;        // tile-shape variant of this launch
  int stream = 0;     // auxiliary stream (several streams: balanced by estimated cost)
  long long cost = 0; // tiles x taps, the estimate the balancing uses
  int n = 0, total = 0;
  size_t lds = 0;
  std::vector<unsigned char> items;
  std::vector<int> prefix;
  size_t items_dev = 0, prefix_dev = 0;  // offsets in the device blob
};

struct Stage {
  std::vector<Group> groups;
};

}  // namespace

struct aw_batch {
  int n = 0;
  std::vector<Image> img;
  std::vector<long long> coef_off, img_off;
  int var[4] = {0, 0, 0, 4};
  // workspace layout (bytes)
  size_t rpart_off = 0, l1_off = 0, dx_off = 0, obj_off = 0, ctr_off = 0, act_off = 0,
         beta_off = 0, ws_total = 0;
  std::vector<int> r_off;   // per-image first residual-partial slot (n + 1)
  std::vector<int> blk_off; // per-image first analysis-tile partial slot (n + 1)
  // bound state
  bool bound = false;
  const void* b_obs = nullptr;
  void* x = nullptr;
  void* y = nullptr;
  char* ws = nullptr;
  double lambda = 0, Lstep = 1;
  std::vector<Stage> stages;
  size_t rpref_dev = 0, bpref_dev = 0;
  char* blob = nullptr;
  hipStream_t aux[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> events;
};

namespace {

thread_local std::string b_err;
aw_status bfail(aw_status st, const char* msg) {
  b_err = msg;
  return st;
}

// Tables and per-level sizes of one image (validation mirrors the single-image path).
aw_status image_setup(const aw_wavelet& w, const aw_blur& b, Image& im) {
  int64_t n = 0;
  int32_t sr[AW_MAX_LEVELS + 1], sc[AW_MAX_LEVELS + 1];
  aw_status st = aw_wavelet_layout(&w, &n, sr, sc);
  if (st != AW_OK) return bfail(st, aw_last_error());
  if (w.bc == AW_BC_PER_EXT) return bfail(AW_EUNSUPPORTED, "batched path: periodic extension not supported");
  if (w.biorthogonal || w.filter_len == 10)
    return bfail(AW_EUNSUPPORTED, "batched path: orthogonal filters of length 2, 8 or 16 only");
  if (b.rows != w.rows || b.cols != w.cols) return bfail(AW_EINVAL, "wavelet and blur sizes differ");
  if (b.radius < 0 || b.radius > AW_MAX_RADIUS) return bfail(AW_EINVAL, "radius out of range");
  im.w = w;
  for (int k = 0; k < AW_MAX_TAPS; ++k) im.taps[k] = im.taps[AW_MAX_TAPS + k] = w.lo[k];
  im.J = w.levels;
  im.L = w.filter_len;
  im.bc = w.bc;
  im.e = (w.bc == AW_BC_SYM) ? w.filter_len - 1 : 0;
  im.rows = w.rows;
  im.cols = w.cols;
  for (int j = 0; j <= im.J; ++j) {
    im.sr[j] = sr[j];
    im.sc[j] = sc[j];
    if (j < im.J && im.bc == AW_BC_SYM && (sr[j] < im.e || sc[j] < im.e))
      return bfail(AW_EUNSUPPORTED, "batched path: level shorter than the extension width");
  }
  im.ncoef = n;
  im.npix = (long long)w.rows * w.cols;
  long long o = (long long)sr[im.J] * sc[im.J];
  im.off_hvd[im.J] = o;
  for (int j = im.J; j >= 1; --j) {
    o += 3LL * sr[j] * sc[j];
    if (j > 1) im.off_hvd[j - 1] = o;
  }
  im.b.rows = b.rows;
  im.b.cols = b.cols;
  im.b.radius = b.radius;
  for (int i = 0; i < 2 * b.radius + 1; ++i) {
    if (!std::isfinite(b.taps[i])) return bfail(AW_EINVAL, "PSF tap not finite");
    im.b.taps[i] = b.taps[i];
  }
  return AW_OK;
}

void layout(aw_batch* p) {
  size_t off = 0;
  const size_t ts = sizeof(float);
  p->coef_off.assign(p->n + 1, 0);
  p->img_off.assign(p->n + 1, 0);
  for (int i = 0; i < p->n; ++i) {
    p->coef_off[i + 1] = p->coef_off[i] + p->img[i].ncoef;
    p->img_off[i + 1] = p->img_off[i] + p->img[i].npix;
  }
  for (int i = 0; i < p->n; ++i) {
    Image& im = p->img[i];
    for (int j = 1; j < im.J; ++j) {
      im.a_off[j] = off;
      off = alignb(off + (size_t)im.sr[j] * im.sc[j] * ts);
    }
    im.tmp_off = off;
    off = alignb(off + (size_t)im.npix * ts);
    im.res_off = off;
    off = alignb(off + (size_t)im.npix * ts);
  }
  p->r_off.assign(p->n + 1, 0);
  p->blk_off.assign(p->n + 1, 0);
  int amax = 0;  // analysis-tile partial slots for either tile variant
  for (int i = 0; i < p->n; ++i) {
    int tx;
    p->r_off[i + 1] = p->r_off[i] + aw::blur_tiles_var(0, p->var[2] == 1 ? 1 : 0, p->img[i].b, &tx);
    const Image& im = p->img[i];
    for (int j = 1; j <= im.J; ++j) {
      aw::AnaLevel d{};
      d.r = {im.sr[j - 1], im.sr[j], im.e};
      d.c = {im.sc[j - 1], im.sc[j], im.e};
      amax += std::max(aw::ana_tiles(0, 0, d), aw::ana_tiles(0, 1, d));
    }
  }
  // partial slots sized for the larger blur variant so the layout does not
  // depend on the tile configuration
  int rmax = 0;
  for (int i = 0; i < p->n; ++i) {
    int tx;
    rmax += std::max(aw::blur_tiles_var(0, 0, p->img[i].b, &tx), aw::blur_tiles_var(0, 1, p->img[i].b, &tx));
  }
  p->rpart_off = off;
  off = alignb(off + (size_t)rmax * sizeof(double));
  p->l1_off = off;
  off = alignb(off + (size_t)amax * sizeof(double));
  p->dx_off = off;
  off = alignb(off + (size_t)amax * sizeof(double));
  p->obj_off = off;
  off = alignb(off + (size_t)p->n * 3 * sizeof(double));
  p->ctr_off = off;
  off = alignb(off + sizeof(int));
  p->act_off = off;
  off = alignb(off + (size_t)p->n * sizeof(int));
  p->beta_off = off;
  off = alignb(off + (size_t)kBetaLen * sizeof(double));
  p->ws_total = off;
}

Group& group_for(Stage& st, int kind, int k0, int k1) {
  for (Group& g : st.groups)
    if (g.kind == kind && g.key0 == k0 && g.key1 == k1) return g;
  st.groups.push_back(Group{});
  Group& g = st.groups.back();
  g.kind = kind;
  g.key0 = k0;
  g.key1 = k1;
  g.prefix.push_back(0);
  return g;
}

void add_item(Group& g, const void* item, size_t sz, int tiles) {
  const unsigned char* c = static_cast<const unsigned char*>(item);
  g.items.insert(g.items.end(), c, c + sz);
  g.n += 1;
  g.total += tiles;
  g.prefix.push_back(g.total);
}

// Blur tile variant: cfg value 1 half-height tiles; 0 and 2 full-height
// tiles (2: one launch per blur stage, below).
int blur_var(const aw_batch* p) { return p->var[2] == 1 ? 1 : 0; }

// Analysis tile variant of level j for filter length L: cfg value 2 takes
// full-height tiles for the finest level (the large launches) and half-height
// ones for the coarser levels (the short, latency-bound launches), as the
// single-image path does; 3 takes half-height tiles for the 16-tap classes
// (whose full-height tile with the fused update holds only two workgroups per
// CU by its registers) and full-height tiles for the others.
int ana_var(const aw_batch* p, int j, int L) {
  switch (p->var[1]) {
    case 2: return j == 1 ? 0 : 1;
    case 3: return L == 16 ? 1 : 0;
    default: return p->var[1];
  }
}

aw_status build(aw_batch* p) {
  p->stages.clear();
  int Jmax = 0;
  for (const Image& im : p->img) Jmax = std::max(Jmax, im.J);
  char* ws = p->ws;
  double* rpart = reinterpret_cast<double*>(ws + p->rpart_off);
  // recompute residual-partial offsets for the current blur variant
  for (int i = 0; i < p->n; ++i) {
    int tx;
    p->r_off[i + 1] = p->r_off[i] + aw::blur_tiles_var(0, blur_var(p), p->img[i].b, &tx);
  }
  // analysis-tile partial slots for the current analysis variant
  for (int i = 0; i < p->n; ++i) {
    const Image& im = p->img[i];
    int t = 0;
    for (int j = 1; j <= im.J; ++j) {
      aw::AnaLevel d{};
      d.r = {im.sr[j - 1], im.sr[j], im.e};
      d.c = {im.sc[j - 1], im.sc[j], im.e};
      t += aw::ana_tiles(0, ana_var(p, j, im.L), d);
    }
    p->blk_off[i + 1] = p->blk_off[i] + t;
  }
  std::vector<unsigned char> buf(std::max({aw::synth_item_size(0), aw::ana_item_size(0),
                                           aw::blur_item_size(0)}));
  std::vector<int> lvl_base(p->blk_off.begin(), p->blk_off.end() - 1);
  // synthesis levels Jmax .. 1
  for (int j = Jmax; j >= 1; --j) {
    Stage st;
    for (int i = 0; i < p->n; ++i) {
      const Image& im = p->img[i];
      if (im.J < j) continue;
      const float* yi = static_cast<const float*>(p->y) + p->coef_off[i];
      aw::SynthLevel d{};
      d.a = (j == im.J) ? (const void*)yi : (const void*)(ws + im.a_off[j]);
      d.stride_a = 0;
      d.hvd = yi + im.off_hvd[j];
      d.stride_hvd = 0;
      d.out = (j == 1) ? (void*)(ws + im.tmp_off) : (void*)(ws + im.a_off[j - 1]);
      d.stride_out = 0;
      d.r = {im.sr[j - 1], im.sr[j], im.e};
      d.c = {im.sc[j - 1], im.sc[j], im.e};
      d.bc = im.bc;
      d.pinv = 1;
      aw::make_synth_item(0, d, im.taps, im.L, i, buf.data());
      Group& g = group_for(st, 0, im.L, im.bc);
      add_item(g, buf.data(), aw::synth_item_size(0), aw::synth_tiles(0, p->var[0], d));
      g.var = p->var[0];
      g.lds = std::max(g.lds, aw::synth_item_lds(0, im.L, p->var[0], d));
      if (g.lds > 160 * 1024) return bfail(AW_EUNSUPPORTED, "tile window exceeds LDS");
    }
    p->stages.push_back(std::move(st));
  }
  // R y - b and R^* r. With cfg[2] = 2 every image joins one class at the
  // largest radius of the batch, its PSF zero-padded to that radius: one
  // launch per stage, and the same values (the padded taps add exact zeros;
  // the R^* border correction of the padded taps is that of the PSF).
  int rbig = 0;
  for (const Image& im : p->img) rbig = std::max(rbig, im.b.radius);
  for (int adj = 0; adj < 2; ++adj) {
    Stage st;
    for (int i = 0; i < p->n; ++i) {
      const Image& im = p->img[i];
      aw::BlurDesc bd = im.b;
      if (p->var[2] == 2 && im.b.radius < rbig) {
        const int r = im.b.radius;
        bd.radius = rbig;
        for (int k = 0; k < 2 * rbig + 1; ++k) {
          const int u = k - (rbig - r);
          bd.taps[k] = (u >= 0 && u < 2 * r + 1) ? im.b.taps[u] : 0.0;
        }
      }
      int tx;
      const int tiles = aw::blur_tiles_var(0, blur_var(p), bd, &tx);
      const float* bi = static_cast<const float*>(p->b_obs) + p->img_off[i];
      if (!adj)
        aw::make_blur_item(0, false, bd, ws + im.tmp_off, ws + im.res_off, bi, rpart + p->r_off[i],
                           i, tx, buf.data());
      else
        aw::make_blur_item(0, true, bd, ws + im.res_off, ws + im.tmp_off, nullptr, nullptr, i, tx,
                           buf.data());
      Group& g = group_for(st, 2 + adj, bd.radius, 0);
      add_item(g, buf.data(), aw::blur_item_size(0), tiles);
      g.var = blur_var(p);
    }
    p->stages.push_back(std::move(st));
  }
  // analysis levels 1 .. Jmax (W^*: weights 1/mult), each tile applying the
  // FISTA update to the coefficients it produces
  for (int j = 1; j <= Jmax; ++j) {
    Stage st;
    for (int i = 0; i < p->n; ++i) {
      const Image& im = p->img[i];
      if (im.J < j) continue;
      float* xi = static_cast<float*>(p->x) + p->coef_off[i];
      float* yi = static_cast<float*>(p->y) + p->coef_off[i];
      aw::AnaLevel d{};
      d.in = (j == 1) ? (const void*)(ws + im.tmp_off) : (const void*)(ws + im.a_off[j - 1]);
      d.stride_in = 0;
      d.a = (j == im.J) ? nullptr : (void*)(ws + im.a_off[j]);
      d.stride_a = 0;
      d.hvd = nullptr;
      d.stride_hvd = 0;
      d.r = {im.sr[j - 1], im.sr[j], im.e};
      d.c = {im.sc[j - 1], im.sc[j], im.e};
      d.bc = im.bc;
      d.pinv = 1;
      aw::ProxEpi pe{};
      pe.x_hvd = xi + im.off_hvd[j];
      pe.y_hvd = yi + im.off_hvd[j];
      pe.x_a = (j == im.J) ? (void*)xi : nullptr;
      pe.y_a = (j == im.J) ? (void*)yi : nullptr;
      pe.inv_L = 1.0 / p->Lstep;
      pe.thresh = p->lambda / p->Lstep;
      pe.partials = reinterpret_cast<double*>(ws + p->l1_off);
      pe.dx_partials = reinterpret_cast<double*>(ws + p->dx_off);
      pe.pbase = lvl_base[i];
      pe.pstride = 0;
      pe.beta_tab = reinterpret_cast<const double*>(ws + p->beta_off);
      pe.counter = reinterpret_cast<const int*>(ws + p->ctr_off);
      pe.beta_len = kBetaLen;
      const int tiles = aw::ana_tiles(0, ana_var(p, j, im.L), d);
      lvl_base[i] += tiles;
      aw::make_ana_item_prox(d, im.taps, im.L, i, pe, buf.data());
      Group& g = group_for(st, 1, im.L, im.bc);
      add_item(g, buf.data(), aw::ana_item_size(0), tiles);
      g.var = ana_var(p, j, im.L);
    }
    p->stages.push_back(std::move(st));
  }
  // device blob: all groups' items and prefixes, partial-slot prefixes
  size_t off = 0;
  for (Stage& st : p->stages)
    for (Group& g : st.groups) {
      g.items_dev = off;
      off = alignb(off + g.items.size());
      g.prefix_dev = off;
      off = alignb(off + g.prefix.size() * sizeof(int));
    }
  p->rpref_dev = off;
  off = alignb(off + p->r_off.size() * sizeof(int));
  p->bpref_dev = off;
  off = alignb(off + p->blk_off.size() * sizeof(int));
  if (p->blob) {
    const hipError_t fe = hipFree(p->blob);
    p->blob = nullptr;
    if (fe != hipSuccess) return bfail(AW_EHIP, hipGetErrorString(fe));
  }
  if (hipMalloc((void**)&p->blob, off) != hipSuccess) return bfail(AW_EHIP, "plan allocation failed");
  std::vector<unsigned char> host(off, 0);
  for (Stage& st : p->stages)
    for (Group& g : st.groups) {
      std::copy(g.items.begin(), g.items.end(), host.begin() + g.items_dev);
      std::memcpy(host.data() + g.prefix_dev, g.prefix.data(), g.prefix.size() * sizeof(int));
    }
  std::memcpy(host.data() + p->rpref_dev, p->r_off.data(), p->r_off.size() * sizeof(int));
  std::memcpy(host.data() + p->bpref_dev, p->blk_off.data(), p->blk_off.size() * sizeof(int));
  if (hipMemcpy(p->blob, host.data(), off, hipMemcpyHostToDevice) != hipSuccess)
    return bfail(AW_EHIP, "plan upload failed");
  // streams of the classes of each stage: longest estimated launch first,
  // each to the stream with the least work so far
  for (Stage& st : p->stages) {
    std::vector<int> order(st.groups.size());
    for (size_t i = 0; i < order.size(); ++i) {
      Group& g = st.groups[i];
      g.cost = (long long)g.total * (g.kind <= 1 ? g.key0 : 2 * g.key0 + 1);
      order[i] = (int)i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return st.groups[a].cost > st.groups[b].cost;
    });
    long long load[4] = {0, 0, 0, 0};
    const int ns = std::max(1, std::min(p->var[3], 4));
    for (int i : order) {
      int best = 0;
      for (int k = 1; k < ns; ++k)
        if (load[k] < load[best]) best = k;
      st.groups[i].stream = best;
      load[best] += st.groups[i].cost;
    }
  }
  // events for fork / join
  size_t need = 0;
  for (const Stage& st : p->stages) need += st.groups.size() + 1;
  while (p->events.size() < need) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return bfail(AW_EHIP, "event creation failed");
    p->events.push_back(e);
  }
  return AW_OK;
}

aw_status launch_group(aw_batch* p, const Group& g, hipStream_t s) {
  const int* active = reinterpret_cast<const int*>(p->ws + p->act_off);
  const void* items = p->blob + g.items_dev;
  const int* prefix = reinterpret_cast<const int*>(p->blob + g.prefix_dev);
  hipError_t e = hipSuccess;
  if (g.total == 0) return AW_OK;
  switch (g.kind) {
    case 0:
      e = aw::launch_synth_batch(0, g.key0, g.key1, g.var, items, prefix, g.n, g.total, active,
                                 g.lds, s);
      break;
    case 1:
      e = aw::launch_ana_batch(0, g.key0, g.key1, g.var, items, prefix, g.n, g.total, active, s,
                               true);
      break;
    default:
      e = aw::launch_blur_batch(0, g.key0, g.kind == 3, g.var, items, prefix, g.n, g.total,
                                active, s);
  }
  if (e != hipSuccess) return bfail(AW_EHIP, hipGetErrorString(e));
  return AW_OK;
}

// Frees what the plan owns (tables, events, streams) and the plan; the first
// runtime error, if any, is returned after everything has been released.
hipError_t release(aw_batch* p) {
  hipError_t first = hipSuccess;
  auto keep = [&first](hipError_t e) {
    if (first == hipSuccess && e != hipSuccess) first = e;
  };
  if (p->blob) keep(hipFree(p->blob));
  for (hipEvent_t e : p->events) keep(hipEventDestroy(e));
  for (int k = 0; k < 4; ++k)
    if (p->aux[k]) keep(hipStreamDestroy(p->aux[k]));
  delete p;
  return first;
}

}  // namespace

extern "C" {

aw_status aw_batch_create(int32_t n, const aw_wavelet* w, const aw_blur* b, aw_batch** plan) {
  if (!plan || !w || !b || n < 1) return bfail(AW_EINVAL, "invalid plan arguments");
  *plan = nullptr;
  aw_batch* p = new aw_batch();
  p->n = n;
  p->img.resize(n);
  for (int i = 0; i < n; ++i) {
    aw_status st = image_setup(w[i], b[i], p->img[i]);
    if (st != AW_OK) {
      delete p;
      return st;
    }
  }
  layout(p);
  for (int k = 0; k < 4; ++k)
    if (hipStreamCreateWithFlags(&p->aux[k], hipStreamNonBlocking) != hipSuccess) {
      p->aux[k] = nullptr;
      (void)release(p);  // the creation error is the one reported
      return bfail(AW_EHIP, "stream creation failed");
    }
  *plan = p;
  b_err.clear();
  return AW_OK;
}

aw_status aw_batch_destroy(aw_batch* p) {
  if (!p) return AW_OK;
  const hipError_t e = release(p);
  if (e != hipSuccess) return bfail(AW_EHIP, hipGetErrorString(e));
  return AW_OK;
}

aw_status aw_batch_layout(const aw_batch* p, int64_t* coef_off, int64_t* img_off,
                          size_t* workspace_bytes) {
  if (!p) return bfail(AW_EINVAL, "plan is NULL");
  for (int i = 0; i <= p->n; ++i) {
    if (coef_off) coef_off[i] = p->coef_off[i];
    if (img_off) img_off[i] = p->img_off[i];
  }
  if (workspace_bytes) *workspace_bytes = p->ws_total;
  return AW_OK;
}

aw_status aw_batch_set_config(aw_batch* p, const int32_t* var) {
  if (!p || !var) return bfail(AW_EINVAL, "invalid arguments");
  const int vmax[3] = {1, 3, 2};
  for (int k = 0; k < 3; ++k)
    if (var[k] < 0 || var[k] > vmax[k])
      return bfail(AW_EINVAL, "tile variant out of range (synthesis 0..1, analysis 0..3, blur 0..2)");
  if (var[3] < 1 || var[3] > 4) return bfail(AW_EINVAL, "streams must be 1..4");
  for (int k = 0; k < 4; ++k) p->var[k] = var[k];
  if (p->bound) return build(p);
  return AW_OK;
}

aw_status aw_batch_bind(aw_batch* p, const void* b_obs, void* x, void* y, void* workspace,
                        size_t workspace_bytes, double lambda, double L) {
  if (!p || !b_obs || !x || !y || !workspace) return bfail(AW_EINVAL, "NULL argument");
  if (workspace_bytes < p->ws_total) return bfail(AW_EINVAL, "workspace too small");
  if (!(L > 0.0) || !(lambda >= 0.0)) return bfail(AW_EINVAL, "L > 0 and lambda >= 0 required");
  p->b_obs = b_obs;
  p->x = x;
  p->y = y;
  p->ws = static_cast<char*>(workspace);
  p->lambda = lambda;
  p->Lstep = L;
  // beta_k = (t_k - 1) / t_{k+1}, t_1 = 1
  std::vector<double> beta(kBetaLen);
  double t = 1.0;
  for (int k = 0; k < kBetaLen; ++k) {
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    beta[k] = (t - 1.0) / tn;
    t = tn;
  }
  if (hipMemcpy(p->ws + p->beta_off, beta.data(), kBetaLen * sizeof(double),
                hipMemcpyHostToDevice) != hipSuccess)
    return bfail(AW_EHIP, "beta table upload failed");
  p->bound = true;
  aw_status st = build(p);
  if (st == AW_OK) b_err.clear();
  return st;
}

aw_status aw_batch_control(const aw_batch* p, int32_t** counter, int32_t** active, double** obj) {
  if (!p || !p->bound) return bfail(AW_EINVAL, "plan not bound");
  if (counter) *counter = reinterpret_cast<int32_t*>(p->ws + p->ctr_off);
  if (active) *active = reinterpret_cast<int32_t*>(p->ws + p->act_off);
  if (obj) *obj = reinterpret_cast<double*>(p->ws + p->obj_off);
  return AW_OK;
}

aw_status aw_batch_reset(aw_batch* p, void* stream) {
  if (!p || !p->bound) return bfail(AW_EINVAL, "plan not bound");
  const long long nc = p->coef_off[p->n];
  hipLaunchKernelGGL(aw::batch_reset_kernel<float>, dim3(1024), dim3(256), 0, (hipStream_t)stream,
                     reinterpret_cast<int*>(p->ws + p->ctr_off),
                     reinterpret_cast<int*>(p->ws + p->act_off), p->n, static_cast<float*>(p->x),
                     static_cast<float*>(p->y), nc);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AW_OK : bfail(AW_EHIP, hipGetErrorString(e));
}

aw_status aw_batch_step(aw_batch* p, void* stream) {
  if (!p || !p->bound) return bfail(AW_EINVAL, "plan not bound");
  hipStream_t s = (hipStream_t)stream;
  size_t ev = 0;
  for (const Stage& st : p->stages) {
    const int ng = (int)st.groups.size();
    if (ng <= 1 || p->var[3] <= 1) {
      for (const Group& g : st.groups) {
        aw_status r = launch_group(p, g, s);
        if (r != AW_OK) return r;
      }
      continue;
    }
    // fork the classes of this stage over auxiliary streams, then join
    hipEvent_t fork = p->events[ev++];
    if (hipEventRecord(fork, s) != hipSuccess) return bfail(AW_EHIP, "event record failed");
    for (int gi = 0; gi < ng; ++gi) {
      hipStream_t a = p->aux[st.groups[gi].stream];
      if (hipStreamWaitEvent(a, fork, 0) != hipSuccess) return bfail(AW_EHIP, "stream wait failed");
      aw_status r = launch_group(p, st.groups[gi], a);
      if (r != AW_OK) return r;
      hipEvent_t done = p->events[ev++];
      if (hipEventRecord(done, a) != hipSuccess) return bfail(AW_EHIP, "event record failed");
      if (hipStreamWaitEvent(s, done, 0) != hipSuccess) return bfail(AW_EHIP, "stream wait failed");
    }
  }
  char* ws = p->ws;
  hipLaunchKernelGGL(aw::batch_reduce_kernel, dim3(p->n), dim3(256), 0, s, p->n,
                     reinterpret_cast<const int*>(p->blob + p->rpref_dev),
                     reinterpret_cast<const double*>(ws + p->rpart_off),
                     reinterpret_cast<const int*>(p->blob + p->bpref_dev),
                     reinterpret_cast<const double*>(ws + p->l1_off),
                     reinterpret_cast<const double*>(ws + p->dx_off),
                     reinterpret_cast<const int*>(ws + p->act_off),
                     reinterpret_cast<double*>(ws + p->obj_off));
  hipLaunchKernelGGL(aw::batch_counter_kernel, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<int*>(ws + p->ctr_off));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? AW_OK : bfail(AW_EHIP, hipGetErrorString(e));
}

const char* aw_batch_last_error(void) { return b_err.c_str(); }

}  // extern "C"
