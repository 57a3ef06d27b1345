// C ABI (include/adjwave.h): validation, coefficient layout, workspace
// carving, and the per-level launch sequences of W, W^*, W^dagger,
// (W^dagger)^* (orthogonal and biorthogonal filters), R, R^*, A, A^* (two
// kernels or one pass over the finest level), one FISTA iteration, the
// convolution pair and its multi-channel form with the Huber TV pieces, the
// learned warm start's CNN, and the DCT-II route for R.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/adjwave.h"
#include "aw_internal.hpp"

namespace {

thread_local std::string g_err;

aw_status fail(aw_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

aw_status ok() {
  g_err.clear();
  return AW_OK;
}

aw_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(AW_EHIP, "%s: %s", what, hipGetErrorString(e));
  return AW_OK;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------ wavelet plan
struct WavePlan {
  int J = 0, L = 0, bc = 0, e = 0;
  int rows = 0, cols = 0;
  int sr[AW_MAX_LEVELS + 1] = {0}, sc[AW_MAX_LEVELS + 1] = {0};
  long long ncoef = 0;
  long long off_hvd[AW_MAX_LEVELS + 1] = {0};  // offset of H_j in the coefficient vector
  bool bior = false;
  // tap sources of the two sides (low-pass | low-pass whose alternating flip
  // is the high-pass): W and W^* use syn, W^dagger and (W^dagger)^* use ana
  double syn[2 * AW_MAX_TAPS] = {0};
  double ana[2 * AW_MAX_TAPS] = {0};
  // fold weights 1/mult (pinv = 1: W, W^*) or 1 (pinv = 0: W^dagger, its adjoint)
  const double* taps(int pinv) const { return pinv ? syn : ana; }
};

int coef_len(int N, int L, int bc, int e) {
  if (bc == aw::PER) return N / 2;
  return (N + 2 * e + L - 1) / 2;
}

aw_status make_plan(const aw_wavelet* w, WavePlan& p) {
  if (!w) return fail(AW_EINVAL, "wavelet descriptor is NULL");
  if (w->rows < 1 || w->cols < 1) return fail(AW_EINVAL, "image size %dx%d", w->rows, w->cols);
  if (w->levels < 1 || w->levels > AW_MAX_LEVELS)
    return fail(AW_EINVAL, "levels=%d outside [1, %d]", w->levels, AW_MAX_LEVELS);
  if (w->filter_len != 2 && w->filter_len != 8 && w->filter_len != 10 && w->filter_len != 16)
    return fail(AW_EINVAL, "filter_len=%d (supported: 2, 8, 10, 16)", w->filter_len);
  if (w->biorthogonal != 0 && w->biorthogonal != 1)
    return fail(AW_EINVAL, "biorthogonal=%d", w->biorthogonal);
  if (w->bc < AW_BC_ZPD || w->bc > AW_BC_PER_EXT) return fail(AW_EINVAL, "bc=%d", w->bc);
  p.J = w->levels;
  p.L = w->filter_len;
  p.bc = w->bc;
  p.e = (p.bc == aw::SYM || p.bc == aw::PER_EXT) ? p.L - 1 : 0;
  p.rows = w->rows;
  p.cols = w->cols;
  p.bior = w->biorthogonal == 1;
  const double* hs = w->lo;
  const double* ha = p.bior ? w->lo_analysis : w->lo;
  for (int k = 0; k < p.L; ++k) {
    if (!std::isfinite(hs[k]) || !std::isfinite(ha[k]))
      return fail(AW_EINVAL, "filter tap %d is not finite", k);
  }
  // orthonormal (h = h_s = h_a) or biorthogonal even shifts:
  // sum_k h_s[k] h_a[k + 2m] = delta_m for every shift
  for (int m = -(p.L / 2 - 1); m <= p.L / 2 - 1; ++m) {
    double s = 0.0;
    for (int k = 0; k < p.L; ++k)
      if (k + 2 * m >= 0 && k + 2 * m < p.L) s += hs[k] * ha[k + 2 * m];
    if (std::fabs(s - (m == 0 ? 1.0 : 0.0)) > 1e-12)
      return fail(AW_EINVAL, "filter %s (shift %d: %.3e)",
                  p.bior ? "pair is not biorthogonal" : "is not orthonormal", 2 * m, s);
  }
  for (int k = 0; k < p.L; ++k) {
    p.syn[k] = hs[k];
    p.syn[AW_MAX_TAPS + k] = ha[k];
    p.ana[k] = ha[k];
    p.ana[AW_MAX_TAPS + k] = hs[k];
  }
  p.sr[0] = p.rows;
  p.sc[0] = p.cols;
  for (int j = 1; j <= p.J; ++j) {
    if (p.bc == aw::PER && (p.sr[j - 1] % 2 || p.sc[j - 1] % 2))
      return fail(AW_EINVAL, "periodic mode needs even sizes at every level (level %d: %dx%d)", j,
                  p.sr[j - 1], p.sc[j - 1]);
    p.sr[j] = coef_len(p.sr[j - 1], p.L, p.bc, p.e);
    p.sc[j] = coef_len(p.sc[j - 1], p.L, p.bc, p.e);
  }
  const long long lim = (1LL << 31) - 1;
  for (int j = 0; j <= p.J; ++j) {
    const long long ext = (long long)(p.sr[j] + 2 * p.e) * (p.sc[j] + 2 * p.e);
    if (ext > lim) return fail(AW_EINVAL, "level %d plane too large", j);
  }
  long long n = (long long)p.sr[p.J] * p.sc[p.J];
  p.off_hvd[p.J] = n;
  for (int j = p.J; j >= 1; --j) {
    n += 3LL * p.sr[j] * p.sc[j];
    if (j > 1) p.off_hvd[j - 1] = n;
  }
  p.ncoef = n;
  return AW_OK;
}

aw_status make_blur(const aw_blur* b, aw::BlurDesc& d) {
  if (!b) return fail(AW_EINVAL, "blur descriptor is NULL");
  if (b->rows < 1 || b->cols < 1) return fail(AW_EINVAL, "image size %dx%d", b->rows, b->cols);
  if ((long long)b->rows * b->cols > (1LL << 31) - 1) return fail(AW_EINVAL, "image too large");
  if (b->radius < 0 || b->radius > AW_MAX_RADIUS)
    return fail(AW_EINVAL, "radius=%d outside [0, %d]", b->radius, AW_MAX_RADIUS);
  d.rows = b->rows;
  d.cols = b->cols;
  d.radius = b->radius;
  for (int i = 0; i < 2 * b->radius + 1; ++i) {
    if (!std::isfinite(b->taps[i])) return fail(AW_EINVAL, "PSF tap %d is not finite", i);
    d.taps[i] = b->taps[i];
  }
  return AW_OK;
}

size_t dsize(aw_dtype t) { return t == AW_F64 ? 8 : 4; }

aw_status check_dtype(aw_dtype t) {
  if (t != AW_F32 && t != AW_F64) return fail(AW_EINVAL, "dtype=%d", (int)t);
  return AW_OK;
}

// ------------------------------------------------------------ workspace
// [a_1 .. a_{J-1}] [extended plane] [image] [gradient] [partials_r] [partials_l1]
struct WsLayout {
  size_t a_off[AW_MAX_LEVELS + 1] = {0};
  size_t ext_off = 0, img_off = 0, grad_off = 0, pr_off = 0, pl_off = 0;
  size_t wave_end = 0;  // bytes used by the wavelet operators alone
  size_t total = 0;
  int n_pr = 0, n_pl = 0;
  int n_pt = 0;  // FISTA l1 partials: one per analysis tile over all levels
};

WsLayout layout_ws(const WavePlan* p, const aw::BlurDesc* b, aw_dtype dt, int batch) {
  WsLayout l;
  const size_t ts = dsize(dt);
  size_t off = 0;
  if (p) {
    for (int j = 1; j < p->J; ++j) {
      l.a_off[j] = off;
      off = align_up(off + (size_t)p->sr[j] * p->sc[j] * batch * ts);
    }
    l.ext_off = off;
    bool need_ext = p->bc == aw::PER_EXT;
    for (int j = 1; j <= p->J; ++j)
      if (p->bc == aw::SYM && (p->sr[j - 1] < p->e || p->sc[j - 1] < p->e)) need_ext = true;
    if (need_ext) {
      size_t mx = 0;
      for (int j = 1; j <= p->J; ++j) {
        const size_t m = (size_t)(p->sr[j - 1] + 2 * p->e) * (p->sc[j - 1] + 2 * p->e);
        if (m > mx) mx = m;
      }
      off = align_up(off + mx * batch * ts);
    }
  }
  l.wave_end = off;
  const int rows = p ? p->rows : (b ? b->rows : 0);
  const int cols = p ? p->cols : (b ? b->cols : 0);
  l.img_off = off;
  off = align_up(off + (size_t)rows * cols * batch * ts);
  l.grad_off = off;
  if (p) off = align_up(off + (size_t)p->ncoef * batch * ts);
  l.n_pr = b ? aw::blur_tiles(dt == AW_F64, *b) : 0;
  l.n_pl = p ? aw::fista_prox_blocks(p->ncoef) : 0;
  if (p)
    for (int j = 1; j <= p->J; ++j) {
      aw::AnaLevel d{};
      d.r = {p->sr[j - 1], p->sr[j], p->e};
      d.c = {p->sc[j - 1], p->sc[j], p->e};
      l.n_pt += aw::ana_level_tiles(dt == AW_F64, d, batch);
    }
  l.pr_off = off;
  off = align_up(off + (size_t)l.n_pr * batch * sizeof(double));
  l.pl_off = off;
  off = align_up(off + (size_t)std::max(l.n_pl, l.n_pt) * batch * sizeof(double));
  l.total = off;
  return l;
}

char* wsp(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

aw_status need_ws(void* ws, size_t have, size_t need) {
  if (need > 0 && !ws) return fail(AW_EINVAL, "workspace is NULL (%zu bytes needed)", need);
  if (have < need) return fail(AW_EINVAL, "workspace too small: %zu < %zu bytes", have, need);
  return AW_OK;
}

// ---------------------------------------------------------- level sequences
aw::SynthLevel synth_desc(const WavePlan& p, aw_dtype dt, const void* coef, void* img, void* ws,
                          const WsLayout& l, int pinv, int j) {
  const size_t ts = dsize(dt);
  aw::SynthLevel d{};
  d.a = (j == p.J) ? coef : wsp(ws, l.a_off[j]);
  d.stride_a = (j == p.J) ? p.ncoef : (long long)p.sr[j] * p.sc[j];
  d.hvd = static_cast<const char*>(coef) + p.off_hvd[j] * ts;
  d.stride_hvd = p.ncoef;
  d.out = (j == 1) ? img : wsp(ws, l.a_off[j - 1]);
  d.stride_out = (long long)p.sr[j - 1] * p.sc[j - 1];
  d.r = {p.sr[j - 1], p.sr[j], p.e};
  d.c = {p.sc[j - 1], p.sc[j], p.e};
  d.bc = p.bc;
  d.pinv = pinv;
  return d;
}

aw_status run_synthesis(const WavePlan& p, aw_dtype dt, int batch, const void* coef, void* img,
                        void* ws, const WsLayout& l, int pinv, hipStream_t s, int j_lo = 1) {
  const int dtype = dt == AW_F64;
  // levels min(J, 4) .. 2 in one chained launch where supported and faster
  int chain_top = 0;
  size_t chain_lds = 0;
  aw::SynthChain ch{};
  if (j_lo <= 2 && p.J >= 3) {
    chain_top = std::min(p.J, 1 + aw::kChainMax);
    ch.nl = chain_top - 1;
    for (int k = 0; k < ch.nl; ++k) ch.d[k] = synth_desc(p, dt, coef, img, ws, l, pinv, 2 + k);
    chain_lds = aw::synth_chain_plan(dtype, p.L, ch);
    if (!chain_lds || !aw::synth_chain_pays(ch, batch)) chain_top = 0;
  }
  for (int j = p.J; j >= j_lo; --j) {
    if (chain_top && j == chain_top) {
      hipError_t e = aw::launch_synth_chain(p.L, p.taps(pinv), ch, chain_lds, batch, s);
      if (e != hipSuccess) return hip_check(e, "synthesis launch");
      j = 2;  // levels chain_top .. 2 done
      continue;
    }
    aw::SynthLevel d = synth_desc(p, dt, coef, img, ws, l, pinv, j);
    hipError_t e;
    // the tile kernel folds with closed-form preimages, valid when every
    // extended sample is at most one reflection away (N >= e); periodic
    // extension and shorter signals materialise the extended level and fold it
    const bool two_step = p.bc == aw::PER_EXT ||
                          (p.bc == aw::SYM && (p.sr[j - 1] < p.e || p.sc[j - 1] < p.e));
    if (two_step) {
      // extended synthesis (zero-boundary core on length N + 2e), then fold
      aw::SynthLevel z = d;
      z.bc = aw::ZPD;
      z.r = {p.sr[j - 1] + 2 * p.e, p.sr[j], 0};
      z.c = {p.sc[j - 1] + 2 * p.e, p.sc[j], 0};
      z.out = wsp(ws, l.ext_off);
      z.stride_out = (long long)z.r.N * z.c.N;
      if (aw::synth_level_lds(dtype, p.L, z) > 160 * 1024)
        return fail(AW_EUNSUPPORTED, "tile window exceeds LDS at level %d", j);
      e = aw::launch_synth_level(dtype, p.L, p.taps(pinv), z, batch, s);
      if (e != hipSuccess) return hip_check(e, "synthesis launch");
      aw::FoldLevel f{};
      f.ext = z.out;
      f.out = d.out;
      f.stride_ext = z.stride_out;
      f.stride_out = d.stride_out;
      f.r = d.r;
      f.c = d.c;
      f.bc = p.bc;
      f.pinv = pinv;
      e = aw::launch_fold_level(dtype, f, batch, s);
      if (e != hipSuccess) return hip_check(e, "fold launch");
    } else {
      if (aw::synth_level_lds(dtype, p.L, d) > 160 * 1024)
        return fail(AW_EUNSUPPORTED, "tile window exceeds LDS at level %d", j);
      e = aw::launch_synth_level(dtype, p.L, p.taps(pinv), d, batch, s);
      if (e != hipSuccess) return hip_check(e, "synthesis launch");
    }
  }
  return AW_OK;
}

aw::AnaLevel ana_desc(const WavePlan& p, aw_dtype dt, const void* img, void* coef, void* ws,
                      const WsLayout& l, int pinv, int j) {
  const size_t ts = dsize(dt);
  aw::AnaLevel d{};
  d.in = (j == 1) ? img : wsp(ws, l.a_off[j - 1]);
  d.stride_in = (long long)p.sr[j - 1] * p.sc[j - 1];
  d.a = (j == p.J) ? coef : wsp(ws, l.a_off[j]);
  d.stride_a = (j == p.J) ? p.ncoef : (long long)p.sr[j] * p.sc[j];
  d.hvd = static_cast<char*>(coef) + p.off_hvd[j] * ts;
  d.stride_hvd = p.ncoef;
  d.r = {p.sr[j - 1], p.sr[j], p.e};
  d.c = {p.sc[j - 1], p.sc[j], p.e};
  d.bc = p.bc;
  d.pinv = pinv;
  return d;
}

aw_status run_analysis(const WavePlan& p, aw_dtype dt, int batch, const void* img, void* coef,
                       void* ws, const WsLayout& l, int pinv, hipStream_t s, int j_from = 1) {
  const size_t ts = dsize(dt);
  for (int j = j_from; j <= p.J; ++j) {
    aw::AnaLevel d{};
    d.in = (j == 1) ? img : wsp(ws, l.a_off[j - 1]);
    d.stride_in = (long long)p.sr[j - 1] * p.sc[j - 1];
    d.a = (j == p.J) ? coef : wsp(ws, l.a_off[j]);
    d.stride_a = (j == p.J) ? p.ncoef : (long long)p.sr[j] * p.sc[j];
    d.hvd = static_cast<char*>(coef) + p.off_hvd[j] * ts;
    d.stride_hvd = p.ncoef;
    d.r = {p.sr[j - 1], p.sr[j], p.e};
    d.c = {p.sc[j - 1], p.sc[j], p.e};
    d.bc = p.bc;
    d.pinv = pinv;
    hipError_t e = aw::launch_ana_level(dt == AW_F64, p.L, p.taps(pinv), d, batch, s);
    if (e != hipSuccess) return hip_check(e, "analysis launch");
  }
  return AW_OK;
}

// W^* (pinv weights) of the residual image with the FISTA update fused into
// every level's epilogue: x, y updated in place, l1 partials per tile.
aw_status run_analysis_prox(const WavePlan& p, aw_dtype dt, int batch, const void* img, void* x,
                            void* y, void* ws, const WsLayout& l, double inv_L, double thresh,
                            double beta, double* partials, int pinv, hipStream_t s) {
  const size_t ts = dsize(dt);
  int pbase = 0;
  for (int j = 1; j <= p.J; ++j) {
    aw::AnaLevel d{};
    d.in = (j == 1) ? img : wsp(ws, l.a_off[j - 1]);
    d.stride_in = (long long)p.sr[j - 1] * p.sc[j - 1];
    d.a = (j == p.J) ? nullptr : wsp(ws, l.a_off[j]);
    d.stride_a = (j == p.J) ? p.ncoef : (long long)p.sr[j] * p.sc[j];
    d.hvd = nullptr;
    d.stride_hvd = p.ncoef;
    d.r = {p.sr[j - 1], p.sr[j], p.e};
    d.c = {p.sc[j - 1], p.sc[j], p.e};
    d.bc = p.bc;
    d.pinv = pinv;
    aw::ProxEpi pe{};
    pe.x_hvd = static_cast<char*>(x) + p.off_hvd[j] * ts;
    pe.y_hvd = static_cast<char*>(y) + p.off_hvd[j] * ts;
    pe.x_a = (j == p.J) ? x : nullptr;
    pe.y_a = (j == p.J) ? y : nullptr;
    pe.inv_L = inv_L;
    pe.thresh = thresh;
    pe.beta = beta;
    pe.partials = partials;
    pe.pbase = pbase;
    pe.pstride = l.n_pt;
    pbase += aw::ana_level_tiles(dt == AW_F64, d, batch);
    hipError_t e = aw::launch_ana_level_prox(dt == AW_F64, p.L, p.taps(pinv), d, pe, batch, s);
    if (e != hipSuccess) return hip_check(e, "analysis launch");
  }
  return AW_OK;
}

aw_status wave_common(const aw_wavelet* w, aw_dtype dt, int batch, const void* in, void* out,
                      void* ws, size_t wsb, WavePlan& p, WsLayout& l) {
  aw_status st;
  if ((st = check_dtype(dt)) != AW_OK) return st;
  if ((st = make_plan(w, p)) != AW_OK) return st;
  if (batch < 1) return fail(AW_EINVAL, "batch=%d", batch);
  if (!in || !out) return fail(AW_EINVAL, "NULL data pointer");
  l = layout_ws(&p, nullptr, dt, batch);
  return need_ws(ws, wsb, l.wave_end);
}

aw_status op_check(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                   const void* in, const void* out, WavePlan& p, aw::BlurDesc& d,
                   WsLayout& l) {
  aw_status st;
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if ((st = make_plan(w, p)) != AW_OK) return st;
  if ((st = make_blur(b, d)) != AW_OK) return st;
  if (d.rows != p.rows || d.cols != p.cols)
    return fail(AW_EINVAL, "wavelet %dx%d and blur %dx%d sizes differ", p.rows, p.cols, d.rows,
                d.cols);
  if (batch < 1) return fail(AW_EINVAL, "batch=%d", batch);
  if (!in || !out) return fail(AW_EINVAL, "NULL data pointer");
  l = layout_ws(&p, &d, dtype, batch);
  return AW_OK;
}

// ------------------------------------------------------------ FISTA step
// Host-side checks of a FISTA call (no device work): descriptors, sizes,
// pointers, L, lambda, k, t and the gradient map; fills the plan, the blur
// and the workspace layout.
aw_status fista_check(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                      const void* b_obs, double L, double lambda, const aw_fista_state* state,
                      WavePlan& p, aw::BlurDesc& d, WsLayout& l) {
  if (!state) return fail(AW_EINVAL, "state is NULL");
  aw_status st = op_check(w, b, dtype, batch, b_obs, state->resid, p, d, l);
  if (st != AW_OK) return st;
  if (!state->x || !state->y) return fail(AW_EINVAL, "state x / y is NULL");
  if (!(L > 0.0) || !std::isfinite(L)) return fail(AW_EINVAL, "L=%g", L);
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(AW_EINVAL, "lambda=%g", lambda);
  if (state->k < 1) return fail(AW_EINVAL, "k=%lld (iterations count from 1)", (long long)state->k);
  if (!(state->t >= 1.0)) return fail(AW_EINVAL, "t=%g (t_1 = 1, increasing)", state->t);
  if (state->gradient != AW_GRAD_ADJOINT && state->gradient != AW_GRAD_PINV)
    return fail(AW_EINVAL, "gradient=%d (AW_GRAD_ADJOINT or AW_GRAD_PINV)", (int)state->gradient);
  return AW_OK;
}

// The launches of one FISTA iteration on `s` with the workspace at
// `workspace` (at least l.total bytes), then k and t of the state advanced.
aw_status fista_enqueue(const WavePlan& p, const aw::BlurDesc& d, const WsLayout& l,
                        aw_dtype dtype, int32_t batch, const void* b_obs, double L, double lambda,
                        aw_fista_state* state, int32_t want_objective, void* workspace,
                        hipStream_t s) {
  aw_status st;
  const bool obj = want_objective && state->obj;
  const int dtype_i = dtype == AW_F64;
  void* img = wsp(workspace, l.img_off);
  double* pr = reinterpret_cast<double*>(wsp(workspace, l.pr_off));
  double* pl = reinterpret_cast<double*>(wsp(workspace, l.pl_off));
  // r = R W y - b
  if ((st = run_synthesis(p, dtype, batch, state->y, img, workspace, l, 1, s)) != AW_OK) return st;
  if ((st = hip_check(aw::launch_blur(dtype_i, d, batch, img, state->resid, b_obs,
                                      obj ? pr : nullptr, s),
                      "blur launch")) != AW_OK)
    return st;
  // g = W^* R^* r
  if ((st = hip_check(aw::launch_blur_adjoint(dtype_i, d, batch, state->resid, img, s),
                      "blur_adjoint launch")) != AW_OK)
    return st;
  // W^* level by level, each level's gradient coefficients consumed at once
  // by the prox + momentum update (the gradient never reaches memory)
  const double t = state->t;
  const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
  const double beta = (t - 1.0) / tn;
  // the true adjoint folds with the 1/mult weights of (E^dagger)^*; W^dagger
  // extends with weight one
  const int fold_w = state->gradient == AW_GRAD_PINV ? 0 : 1;
  if ((st = run_analysis_prox(p, dtype, batch, img, state->x, state->y, workspace, l, 1.0 / L,
                              lambda / L, beta, obj ? pl : nullptr, fold_w, s)) != AW_OK)
    return st;
  if (obj) {
    if ((st = hip_check(aw::launch_reduce_partials(batch, l.n_pr, pr, 1.0, state->obj, 2, 0, s),
                        "reduce launch")) != AW_OK)
      return st;
    if ((st = hip_check(aw::launch_reduce_partials(batch, l.n_pt, pl, 1.0, state->obj, 2, 1, s),
                        "reduce launch")) != AW_OK)
      return st;
  }
  state->t = tn;
  state->k += 1;
  return ok();
}

// ------------------------------------------------------- static scratch
// The workspace of fista_step_noalloc: a file-scope device array, so that
// call allocates nothing. Every GPU the library runs on holds its own copy
// (64 MiB) from the time the library's code is loaded on it until the
// process ends. In host code `scratch` only names the symbol: its device
// address, per device, comes from hipGetSymbolAddress on the first call on
// that device and is kept in g_scratch.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {nullptr};

aw_status scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_check(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(AW_EUNSUPPORTED, "device index %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(AW_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return AW_OK;
}

}  // namespace

extern "C" {

const char* aw_last_error(void) { return g_err.c_str(); }

aw_status aw_daubechies(int32_t taps, double* lo_out) {
  if (!lo_out) return fail(AW_EINVAL, "output pointer is NULL");
  if (taps < 2 || taps > AW_MAX_TAPS || taps % 2) return fail(AW_EINVAL, "taps=%d", taps);
  typedef std::complex<double> cd;
  const int p = taps / 2;
  std::vector<cd> zeros(p, cd(-1.0, 0.0));
  if (p > 1) {
    // roots of P(y) = sum_{k<p} C(p-1+k, k) y^k by Durand-Kerner iteration
    const int deg = p - 1;
    std::vector<double> c(p);
    for (int k = 0; k < p; ++k) {
      double b = 1.0;
      for (int i = 1; i <= k; ++i) b = b * (p - 1 + i) / i;
      c[k] = b;
    }
    auto P = [&](cd y) {
      cd v = 0.0;
      for (int k = deg; k >= 0; --k) v = v * y + c[k];
      return v;
    };
    auto dP = [&](cd y) {
      cd v = 0.0;
      for (int k = deg; k >= 1; --k) v = v * y + c[k] * (double)k;
      return v;
    };
    std::vector<cd> r(deg);
    for (int i = 0; i < deg; ++i) r[i] = std::pow(cd(0.4, 0.9), i);
    for (int it = 0; it < 2000; ++it) {
      double moved = 0.0;
      for (int i = 0; i < deg; ++i) {
        cd den = c[deg];
        for (int j = 0; j < deg; ++j)
          if (j != i) den *= (r[i] - r[j]);
        const cd step = P(r[i]) / den;
        r[i] -= step;
        moved = std::max(moved, std::abs(step));
      }
      if (moved < 1e-16) break;
    }
    for (int i = 0; i < deg; ++i)  // Newton polish on the original polynomial
      for (int it = 0; it < 3; ++it) {
        const cd d = dP(r[i]);
        if (std::abs(d) > 0) r[i] -= P(r[i]) / d;
      }
    for (int i = 0; i < deg; ++i) {
      const cd b = 2.0 - 4.0 * r[i];
      const cd disc = std::sqrt(b * b - 4.0);
      const cd z1 = (b + disc) / 2.0, z2 = (b - disc) / 2.0;
      zeros.push_back(std::abs(z1) < 1.0 ? z1 : z2);
    }
  }
  std::vector<cd> poly(1, cd(1.0, 0.0));  // descending powers
  for (const cd& z : zeros) {
    std::vector<cd> nx(poly.size() + 1, cd(0.0, 0.0));
    for (size_t i = 0; i < poly.size(); ++i) {
      nx[i] += poly[i];
      nx[i + 1] -= poly[i] * z;
    }
    poly.swap(nx);
  }
  double sum = 0.0;
  for (int k = 0; k < taps; ++k) sum += poly[k].real();
  for (int k = 0; k < taps; ++k) lo_out[k] = poly[k].real() * std::sqrt(2.0) / sum;
  return ok();
}

aw_status aw_cdf97(double* lo_syn_out, double* lo_ana_out) {
  if (!lo_syn_out || !lo_ana_out) return fail(AW_EINVAL, "output pointer is NULL");
  // P(y) = 1 + 4y + 10y^2 + 20y^3 is increasing (P' > 0), so it has one real
  // root: Newton from 0, then the quadratic factor holds the complex pair
  double y1 = 0.0;
  for (int it = 0; it < 100; ++it) {
    const double f = ((20.0 * y1 + 10.0) * y1 + 4.0) * y1 + 1.0;
    const double df = (60.0 * y1 + 20.0) * y1 + 4.0;
    const double step = f / df;
    y1 -= step;
    if (std::fabs(step) < 1e-17) break;
  }
  const double qb = 10.0 + 20.0 * y1, qc = 4.0 + qb * y1;  // P = (y - y1)(20y^2 + qb y + qc)
  const std::complex<double> y2 =
      (-qb + std::sqrt(std::complex<double>(qb * qb - 80.0 * qc, 0.0))) / 40.0;
  const double A = 2.0 * (1.0 / y2).real();  // (1 - y/y2)(1 - y/y3) = 1 - A y + B y^2
  const double B = 1.0 / std::norm(y2);
  // centred taps (index = power of z + half-width) of symmetric Laurent polynomials
  auto conv = [](const std::vector<double>& a, const std::vector<double>& b) {
    std::vector<double> c(a.size() + b.size() - 1, 0.0);
    for (size_t i = 0; i < a.size(); ++i)
      for (size_t k = 0; k < b.size(); ++k) c[i + k] += a[i] * b[k];
    return c;
  };
  const std::vector<double> c2 = {0.25, 0.5, 0.25};   // cos^2(w/2)
  const std::vector<double> s2 = {-0.25, 0.5, -0.25}; // sin^2(w/2)
  const std::vector<double> c4 = conv(c2, c2);
  std::vector<double> f1 = {-s2[0] / y1, 1.0 - s2[1] / y1, -s2[2] / y1};
  const std::vector<double> s4 = conv(s2, s2);
  std::vector<double> f2(5, 0.0);
  f2[2] = 1.0;
  for (int k = 0; k < 3; ++k) f2[k + 1] -= A * s2[k];
  for (int k = 0; k < 5; ++k) f2[k] += B * s4[k];
  const std::vector<double> hs = conv(c4, f1);  // 7 taps
  const std::vector<double> ha = conv(c4, f2);  // 9 taps
  for (int k = 0; k < 10; ++k) lo_syn_out[k] = lo_ana_out[k] = 0.0;
  for (int k = 0; k < 7; ++k) lo_syn_out[1 + k] = std::sqrt(2.0) * hs[k];
  for (int k = 0; k < 9; ++k) lo_ana_out[k] = std::sqrt(2.0) * ha[k];
  return ok();
}

aw_status aw_gaussian_psf(double sigma, int32_t radius, double* taps_out) {
  if (!taps_out) return fail(AW_EINVAL, "output pointer is NULL");
  if (!(sigma > 0.0) || radius < 0 || radius > 16384)
    return fail(AW_EINVAL, "sigma=%g radius=%d", sigma, radius);
  double s = 0.0;
  for (int u = -radius; u <= radius; ++u) {
    taps_out[u + radius] = std::exp(-(double)u * u / (2.0 * sigma * sigma));
    s += taps_out[u + radius];
  }
  for (int i = 0; i < 2 * radius + 1; ++i) taps_out[i] /= s;
  return ok();
}

aw_status aw_wavelet_layout(const aw_wavelet* w, int64_t* ncoef, int32_t* sub_rows,
                            int32_t* sub_cols) {
  WavePlan p;
  aw_status st = make_plan(w, p);
  if (st != AW_OK) return st;
  if (ncoef) *ncoef = p.ncoef;
  for (int j = 0; j <= p.J; ++j) {
    if (sub_rows) sub_rows[j] = p.sr[j];
    if (sub_cols) sub_cols[j] = p.sc[j];
  }
  return ok();
}

aw_status aw_workspace_size(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                            size_t* bytes) {
  aw_status st;
  if (!bytes) return fail(AW_EINVAL, "bytes is NULL");
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if (batch < 1) return fail(AW_EINVAL, "batch=%d", batch);
  WavePlan p;
  aw::BlurDesc bd;
  if (w && (st = make_plan(w, p)) != AW_OK) return st;
  if (b && (st = make_blur(b, bd)) != AW_OK) return st;
  *bytes = layout_ws(w ? &p : nullptr, b ? &bd : nullptr, dtype, batch).total;
  return ok();
}

aw_status wavelet_synth(const aw_wavelet* w, aw_dtype dtype, int32_t batch, const void* coef,
                        void* img, void* workspace, size_t workspace_bytes, void* stream) {
  WavePlan p;
  WsLayout l;
  aw_status st = wave_common(w, dtype, batch, coef, img, workspace, workspace_bytes, p, l);
  if (st != AW_OK) return st;
  st = run_synthesis(p, dtype, batch, coef, img, workspace, l, 1, (hipStream_t)stream);
  return st == AW_OK ? ok() : st;
}

aw_status aw_wavelet_analysis_adjoint(const aw_wavelet* w, aw_dtype dtype, int32_t batch,
                                      const void* coef, void* img, void* workspace,
                                      size_t workspace_bytes, void* stream) {
  WavePlan p;
  WsLayout l;
  aw_status st = wave_common(w, dtype, batch, coef, img, workspace, workspace_bytes, p, l);
  if (st != AW_OK) return st;
  st = run_synthesis(p, dtype, batch, coef, img, workspace, l, 0, (hipStream_t)stream);
  return st == AW_OK ? ok() : st;
}

aw_status wavelet_synth_adjoint(const aw_wavelet* w, aw_dtype dtype, int32_t batch,
                                const void* img, void* coef, void* workspace,
                                size_t workspace_bytes, void* stream) {
  WavePlan p;
  WsLayout l;
  aw_status st = wave_common(w, dtype, batch, img, coef, workspace, workspace_bytes, p, l);
  if (st != AW_OK) return st;
  st = run_analysis(p, dtype, batch, img, coef, workspace, l, 1, (hipStream_t)stream);
  return st == AW_OK ? ok() : st;
}

aw_status aw_wavelet_analysis(const aw_wavelet* w, aw_dtype dtype, int32_t batch,
                              const void* img, void* coef, void* workspace,
                              size_t workspace_bytes, void* stream) {
  WavePlan p;
  WsLayout l;
  aw_status st = wave_common(w, dtype, batch, img, coef, workspace, workspace_bytes, p, l);
  if (st != AW_OK) return st;
  st = run_analysis(p, dtype, batch, img, coef, workspace, l, 0, (hipStream_t)stream);
  return st == AW_OK ? ok() : st;
}

static aw_status blur_common(const aw_blur* b, aw_dtype dtype, int32_t batch, const void* in,
                             void* out, aw::BlurDesc& d) {
  aw_status st;
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if ((st = make_blur(b, d)) != AW_OK) return st;
  if (batch < 1) return fail(AW_EINVAL, "batch=%d", batch);
  if (!in || !out) return fail(AW_EINVAL, "NULL data pointer");
  if (in == out) return fail(AW_EINVAL, "blur input and output must not alias");
  return AW_OK;
}

aw_status blur(const aw_blur* b, aw_dtype dtype, int32_t batch, const void* x, void* y,
               void* stream) {
  aw::BlurDesc d;
  aw_status st = blur_common(b, dtype, batch, x, y, d);
  if (st != AW_OK) return st;
  st = hip_check(aw::launch_blur(dtype == AW_F64, d, batch, x, y, nullptr, nullptr,
                                 (hipStream_t)stream),
                 "blur launch");
  return st == AW_OK ? ok() : st;
}

aw_status blur_adjoint(const aw_blur* b, aw_dtype dtype, int32_t batch, const void* y, void* x,
                       void* stream) {
  aw::BlurDesc d;
  aw_status st = blur_common(b, dtype, batch, y, x, d);
  if (st != AW_OK) return st;
  st = hip_check(aw::launch_blur_adjoint(dtype == AW_F64, d, batch, y, x, (hipStream_t)stream),
                 "blur_adjoint launch");
  return st == AW_OK ? ok() : st;
}

static aw_status op_common(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                           const void* in, void* out, void* ws, size_t wsb, WavePlan& p,
                           aw::BlurDesc& d, WsLayout& l) {
  aw_status st = op_check(w, b, dtype, batch, in, out, p, d, l);
  if (st != AW_OK) return st;
  return need_ws(ws, wsb, l.total);
}

aw_status aw_apply_A(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                     const void* coef, void* img, void* workspace, size_t workspace_bytes,
                     void* stream) {
  WavePlan p;
  aw::BlurDesc d;
  WsLayout l;
  aw_status st = op_common(w, b, dtype, batch, coef, img, workspace, workspace_bytes, p, d, l);
  if (st != AW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  void* tmp = wsp(workspace, l.img_off);
  if ((st = run_synthesis(p, dtype, batch, coef, tmp, workspace, l, 1, s)) != AW_OK) return st;
  st = hip_check(aw::launch_blur(dtype == AW_F64, d, batch, tmp, img, nullptr, nullptr, s),
                 "blur launch");
  return st == AW_OK ? ok() : st;
}

aw_status aw_apply_A_fused(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                           const void* coef, const void* b_obs, void* img, void* workspace,
                           size_t workspace_bytes, void* stream) {
  WavePlan p;
  aw::BlurDesc d;
  WsLayout l;
  aw_status st = op_common(w, b, dtype, batch, coef, img, workspace, workspace_bytes, p, d, l);
  if (st != AW_OK) return st;
  if (dtype != AW_F32) return fail(AW_EUNSUPPORTED, "fused A runs in float32 only");
  const aw::SynthLevel d1 = synth_desc(p, dtype, coef, img, workspace, l, 1, 1);
  if (!aw::synth_blur_supported(p.L, d1, d))
    return fail(AW_EUNSUPPORTED,
                "fused A needs zpd/sym/per, filter length 2, 8 or 16, an image of at least "
                "radius + 1 (and, for sym, L - 1) samples per axis and a window within LDS");
  hipStream_t s = (hipStream_t)stream;
  if ((st = run_synthesis(p, dtype, batch, coef, img, workspace, l, 1, s, 2)) != AW_OK) return st;
  st = hip_check(aw::launch_synth_blur(p.L, p.taps(1), d1, d, b_obs, img, batch, s),
                 "fused synthesis-blur launch");
  return st == AW_OK ? ok() : st;
}

aw_status aw_apply_A_adjoint(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                             const void* img, void* coef, void* workspace, size_t workspace_bytes,
                             void* stream) {
  WavePlan p;
  aw::BlurDesc d;
  WsLayout l;
  aw_status st = op_common(w, b, dtype, batch, img, coef, workspace, workspace_bytes, p, d, l);
  if (st != AW_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  void* tmp = wsp(workspace, l.img_off);
  st = hip_check(aw::launch_blur_adjoint(dtype == AW_F64, d, batch, img, tmp, s),
                 "blur_adjoint launch");
  if (st != AW_OK) return st;
  st = run_analysis(p, dtype, batch, tmp, coef, workspace, l, 1, s);
  return st == AW_OK ? ok() : st;
}

aw_status aw_apply_A_adjoint_fused(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype,
                                   int32_t batch, const void* img, void* coef, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  WavePlan p;
  aw::BlurDesc d;
  WsLayout l;
  aw_status st = op_common(w, b, dtype, batch, img, coef, workspace, workspace_bytes, p, d, l);
  if (st != AW_OK) return st;
  if (dtype != AW_F32) return fail(AW_EUNSUPPORTED, "fused A^* runs in float32 only");
  const aw::AnaLevel d1 = ana_desc(p, dtype, img, coef, workspace, l, 1, 1);
  if (!aw::blur_ana_supported(p.L, d1, d))
    return fail(AW_EUNSUPPORTED,
                "fused A^* needs zpd or sym, filter length 2, 8 or 16 and, for sym, images of "
                "at least L - 1 samples per axis");
  hipStream_t s = (hipStream_t)stream;
  st = hip_check(aw::launch_blur_ana(p.L, p.taps(1), d1, d, batch, s), "fused blur-analysis launch");
  if (st != AW_OK) return st;
  st = run_analysis(p, dtype, batch, img, coef, workspace, l, 1, s, 2);
  return st == AW_OK ? ok() : st;
}

aw_status fista_step(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                     const void* b_obs, double L, double lambda, aw_fista_state* state,
                     int32_t want_objective, void* workspace, size_t workspace_bytes,
                     void* stream) {
  WavePlan p;
  aw::BlurDesc d;
  WsLayout l;
  aw_status st = fista_check(w, b, dtype, batch, b_obs, L, lambda, state, p, d, l);
  if (st != AW_OK) return st;
  if ((st = need_ws(workspace, workspace_bytes, l.total)) != AW_OK) return st;
  return fista_enqueue(p, d, l, dtype, batch, b_obs, L, lambda, state, want_objective, workspace,
                       (hipStream_t)stream);
}

aw_status fista_step_noalloc(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                             const void* b_obs, double L, double lambda, aw_fista_state* state,
                             int32_t want_objective, void* stream) {
  WavePlan p;
  aw::BlurDesc d;
  WsLayout l;
  aw_status st = fista_check(w, b, dtype, batch, b_obs, L, lambda, state, p, d, l);
  if (st != AW_OK) return st;
  if (l.total > kScratchBytes)
    return fail(AW_EINVAL,
                "fista_step_noalloc: the problem needs %zu bytes of workspace, more than the "
                "%zu bytes of the static scratch (call fista_step with a workspace)",
                l.total, kScratchBytes);
  void* ws = nullptr;
  if ((st = scratch_ptr(&ws)) != AW_OK) return st;
  return fista_enqueue(p, d, l, dtype, batch, b_obs, L, lambda, state, want_objective, ws,
                       (hipStream_t)stream);
}

aw_status aw_fista_update(const aw_wavelet* w, aw_dtype dtype, int32_t batch, const void* grad,
                          double L, double lambda, aw_fista_state* state, int32_t want_l1,
                          void* workspace, size_t workspace_bytes, void* stream) {
  WavePlan p;
  aw_status st;
  if (!state) return fail(AW_EINVAL, "state is NULL");
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if ((st = make_plan(w, p)) != AW_OK) return st;
  if (batch < 1) return fail(AW_EINVAL, "batch=%d", batch);
  if (!grad || !state->x || !state->y) return fail(AW_EINVAL, "NULL data pointer");
  if (!(L > 0.0) || !std::isfinite(L)) return fail(AW_EINVAL, "L=%g", L);
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(AW_EINVAL, "lambda=%g", lambda);
  if (state->k < 1) return fail(AW_EINVAL, "k=%lld (iterations count from 1)", (long long)state->k);
  if (!(state->t >= 1.0)) return fail(AW_EINVAL, "t=%g (t_1 = 1, increasing)", state->t);
  if (state->gradient != AW_GRAD_ADJOINT && state->gradient != AW_GRAD_PINV)
    return fail(AW_EINVAL, "gradient=%d (AW_GRAD_ADJOINT or AW_GRAD_PINV)", (int)state->gradient);
  const WsLayout l = layout_ws(&p, nullptr, dtype, batch);
  if ((st = need_ws(workspace, workspace_bytes, l.total)) != AW_OK) return st;
  const bool l1 = want_l1 && state->obj;
  hipStream_t s = (hipStream_t)stream;
  double* pl = reinterpret_cast<double*>(wsp(workspace, l.pl_off));
  const double t = state->t;
  const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
  const double beta = (t - 1.0) / tn;
  const int fold_w = state->gradient == AW_GRAD_PINV ? 0 : 1;
  if ((st = run_analysis_prox(p, dtype, batch, grad, state->x, state->y, workspace, l, 1.0 / L,
                              lambda / L, beta, l1 ? pl : nullptr, fold_w, s)) != AW_OK)
    return st;
  if (l1 && (st = hip_check(aw::launch_reduce_partials(batch, l.n_pt, pl, 1.0, state->obj, 2, 1, s),
                            "reduce launch")) != AW_OK)
    return st;
  state->t = tn;
  state->k += 1;
  return ok();
}

aw_status aw_objective(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                       const void* b_obs, double lambda, const void* x, double* obj,
                       void* workspace, size_t workspace_bytes, void* stream) {
  WavePlan p;
  aw::BlurDesc d;
  WsLayout l;
  aw_status st = op_common(w, b, dtype, batch, b_obs, (void*)x, workspace, workspace_bytes, p, d, l);
  if (st != AW_OK) return st;
  if (!obj) return fail(AW_EINVAL, "obj is NULL");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(AW_EINVAL, "lambda=%g", lambda);
  hipStream_t s = (hipStream_t)stream;
  const int dtype_i = dtype == AW_F64;
  void* img = wsp(workspace, l.img_off);
  void* res = wsp(workspace, l.grad_off);  // ncoef >= rows*cols: holds one image
  double* pr = reinterpret_cast<double*>(wsp(workspace, l.pr_off));
  double* pl = reinterpret_cast<double*>(wsp(workspace, l.pl_off));
  if ((st = run_synthesis(p, dtype, batch, x, img, workspace, l, 1, s)) != AW_OK) return st;
  if ((st = hip_check(aw::launch_blur(dtype_i, d, batch, img, res, b_obs, pr, s), "blur launch")) !=
      AW_OK)
    return st;
  if ((st = hip_check(aw::launch_l1_partials(dtype_i, batch, p.ncoef, x, pl, s), "l1 launch")) !=
      AW_OK)
    return st;
  if ((st = hip_check(aw::launch_reduce_partials(batch, l.n_pr, pr, 1.0, obj, 3, 0, s),
                      "reduce launch")) != AW_OK)
    return st;
  if ((st = hip_check(aw::launch_reduce_partials(batch, l.n_pl, pl, 1.0, obj, 3, 1, s),
                      "reduce launch")) != AW_OK)
    return st;
  st = hip_check(aw::launch_objective_finalize(batch, lambda, obj, s), "finalize launch");
  return st == AW_OK ? ok() : st;
}

aw_status conv_adjoint_pair(aw_dtype dtype, int32_t batch, int32_t K, int32_t N, const void* h,
                            const void* s, const void* x_obs, void* resid, void* grad_h,
                            void* grad_s, void* stream) {
  aw_status st;
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if (batch < 1 || K < 1 || N < 1) return fail(AW_EINVAL, "batch=%d K=%d N=%d", batch, K, N);
  if ((long long)K + N - 1 > (1LL << 31) - 1) return fail(AW_EINVAL, "K+N-1 too large");
  if (!h || !s || !resid) return fail(AW_EINVAL, "NULL data pointer");
  if (resid == h || resid == s || resid == x_obs)
    return fail(AW_EINVAL, "resid must not alias the inputs");
  st = hip_check(aw::launch_conv_pair(dtype == AW_F64, batch, K, N, h, s, x_obs, resid, grad_h,
                                      grad_s, (hipStream_t)stream),
                 "conv launch");
  return st == AW_OK ? ok() : st;
}

// ------------------------------------------------------ R via the DCT-II
struct aw_blur_dct {
  int rows = 0, cols = 0, radius = 0;
  aw_dtype dtype = AW_F32;
  // one device buffer in the plan's dtype: eigenvalues of the rows axis (rows
  // values) and of the columns axis (cols), then the FFT and DCT twiddles of
  // the rows axis (2 rows values each, complex pairs) and of the columns axis
  void* lam = nullptr;
};

static bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

aw_status aw_blur_dct_create(int32_t rows, int32_t cols, int32_t radius, const double* taps,
                             aw_dtype dtype, aw_blur_dct** plan) {
  aw_status st;
  if (!plan) return fail(AW_EINVAL, "plan pointer is NULL");
  *plan = nullptr;
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if (!pow2_in(rows, 2, 4096) || !pow2_in(cols, 2, 4096))
    return fail(AW_EUNSUPPORTED, "DCT blur needs power-of-two sizes in [2, 4096] (%dx%d)", rows,
                cols);
  if (radius < 0 || radius > 16384) return fail(AW_EINVAL, "radius=%d outside [0, 16384]", radius);
  if (!taps) return fail(AW_EINVAL, "taps is NULL");
  double mag = 0.0;
  for (int i = 0; i < 2 * radius + 1; ++i) {
    if (!std::isfinite(taps[i])) return fail(AW_EINVAL, "PSF tap %d is not finite", i);
    mag += std::fabs(taps[i]);
  }
  for (int u = 1; u <= radius; ++u)
    if (std::fabs(taps[radius + u] - taps[radius - u]) > 1e-14 * mag)
      return fail(AW_EUNSUPPORTED, "the DCT-II diagonalises R only for a symmetric PSF");
  const size_t need = aw::blur_dct_lds(dtype == AW_F64, std::max(rows, cols));
  if (need > 160 * 1024) return fail(AW_EUNSUPPORTED, "row of %zu bytes exceeds LDS", need);
  // lambda_k = g_0 + 2 sum_u g_u cos(pi k u / N) along each axis
  std::vector<double> lam((size_t)rows + cols);
  for (int axis = 0; axis < 2; ++axis) {
    const int N = axis ? cols : rows;
    double* L = lam.data() + (axis ? rows : 0);
    for (int k = 0; k < N; ++k) {
      double v = taps[radius];
      for (int u = 1; u <= radius; ++u) v += 2.0 * taps[radius + u] * std::cos(M_PI * k * u / N);
      L[k] = v;
    }
  }
  // twiddles of each axis, FP64 on the host: exp(-2 pi i j / N), exp(-i pi k / 2N)
  for (int axis = 0; axis < 2; ++axis) {
    const int N = axis ? cols : rows;
    for (int j = 0; j < N; ++j) {  // angles reduced to [0, 2 pi) exactly: j / N in [0, 1)
      lam.push_back(std::cos(2.0 * M_PI * j / N));
      lam.push_back(-std::sin(2.0 * M_PI * j / N));
    }
    for (int k = 0; k < N; ++k) {
      lam.push_back(std::cos(M_PI * k / (2.0 * N)));
      lam.push_back(-std::sin(M_PI * k / (2.0 * N)));
    }
  }
  aw_blur_dct* p = new aw_blur_dct;
  p->rows = rows;
  p->cols = cols;
  p->radius = radius;
  p->dtype = dtype;
  const size_t n = lam.size();
  if (hipMalloc(&p->lam, n * dsize(dtype)) != hipSuccess) {
    delete p;
    return fail(AW_EHIP, "eigenvalue table allocation failed");
  }
  hipError_t e;
  if (dtype == AW_F64) {
    e = hipMemcpy(p->lam, lam.data(), n * sizeof(double), hipMemcpyHostToDevice);
  } else {
    std::vector<float> lf(lam.begin(), lam.end());
    e = hipMemcpy(p->lam, lf.data(), n * sizeof(float), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    (void)hipFree(p->lam);
    delete p;
    return hip_check(e, "eigenvalue upload");
  }
  *plan = p;
  return ok();
}

aw_status aw_blur_dct_destroy(aw_blur_dct* plan) {
  if (!plan) return ok();
  const hipError_t e = hipFree(plan->lam);
  delete plan;
  return e == hipSuccess ? ok() : hip_check(e, "plan free");
}

aw_status aw_blur_dct_workspace(const aw_blur_dct* plan, int32_t batch, size_t* bytes) {
  if (!plan || !bytes) return fail(AW_EINVAL, "NULL argument");
  if (batch < 1) return fail(AW_EINVAL, "batch=%d", batch);
  *bytes = 2 * align_up((size_t)batch * plan->rows * plan->cols * dsize(plan->dtype));
  return ok();
}

aw_status aw_blur_dct_apply(const aw_blur_dct* plan, int32_t batch, const void* x, void* y,
                            void* workspace, size_t workspace_bytes, void* stream) {
  size_t need = 0;
  aw_status st = aw_blur_dct_workspace(plan, batch, &need);
  if (st != AW_OK) return st;
  if (!x || !y) return fail(AW_EINVAL, "NULL data pointer");
  if ((st = need_ws(workspace, workspace_bytes, need)) != AW_OK) return st;
  const size_t half = need / 2;
  const int di = plan->dtype == AW_F64;
  const char* base = static_cast<const char*>(plan->lam);
  const size_t es = dsize(plan->dtype);
  const size_t R = plan->rows, C = plan->cols;
  aw::DctTables tb;
  tb.lam_r = base;
  tb.lam_c = base + R * es;
  tb.fft_r = base + (R + C) * es;
  tb.dct_r = base + (3 * R + C) * es;
  tb.fft_c = base + (5 * R + C) * es;
  tb.dct_c = base + (5 * R + 3 * C) * es;
  st = hip_check(aw::launch_blur_dct(di, plan->rows, plan->cols, batch, tb, x, y, workspace,
                                     wsp(workspace, half), (hipStream_t)stream),
                 "DCT blur launch");
  return st == AW_OK ? ok() : st;
}

aw_status aw_conv_multichannel(aw_dtype dtype, int32_t channels, int32_t K, int32_t N,
                               const void* h, const void* s, const void* x_obs, void* resid,
                               void* grad_h, void* grad_s_parts, void* grad_s, double* rnorm,
                               void* stream) {
  aw_status st;
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if (channels < 1 || K < 1 || N < 1)
    return fail(AW_EINVAL, "channels=%d K=%d N=%d", channels, K, N);
  if ((long long)K + N - 1 > (1LL << 31) - 1) return fail(AW_EINVAL, "K+N-1 too large");
  if (!h || !s || !resid) return fail(AW_EINVAL, "NULL data pointer");
  if (resid == h || resid == s || resid == x_obs)
    return fail(AW_EINVAL, "resid must not alias the inputs");
  if (grad_s && !grad_s_parts)
    return fail(AW_EINVAL, "grad_s needs grad_s_parts (channels x N scratch)");
  hipStream_t hs = (hipStream_t)stream;
  const int di = dtype == AW_F64;
  st = hip_check(aw::launch_conv_pair(di, channels, K, N, h, s, x_obs, resid, grad_h,
                                      grad_s_parts, hs, true),
                 "conv launch");
  if (st != AW_OK) return st;
  if (grad_s &&
      (st = hip_check(aw::launch_sum_rows(di, channels, N, grad_s_parts, grad_s, hs),
                      "channel sum launch")) != AW_OK)
    return st;
  if (rnorm && (st = hip_check(aw::launch_row_sumsq(di, channels, (long long)K + N - 1, resid,
                                                    rnorm, hs),
                               "residual norm launch")) != AW_OK)
    return st;
  return ok();
}

aw_status aw_huber_tv(aw_dtype dtype, int32_t batch, int32_t K, const void* h, double delta,
                      double gscale, void* grad, double* value, void* stream) {
  aw_status st;
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if (batch < 1 || K < 1) return fail(AW_EINVAL, "batch=%d K=%d", batch, K);
  if (!h) return fail(AW_EINVAL, "NULL data pointer");
  if (!(delta > 0.0) || !std::isfinite(delta) || !std::isfinite(gscale))
    return fail(AW_EINVAL, "delta=%g gscale=%g", delta, gscale);
  if (grad == h) return fail(AW_EINVAL, "grad must not alias h");
  st = hip_check(aw::launch_huber_tv(dtype == AW_F64, batch, K, h, delta, gscale, grad, value,
                                     (hipStream_t)stream),
                 "huber launch");
  return st == AW_OK ? ok() : st;
}

aw_status aw_prox_l1(aw_dtype dtype, int64_t n, const void* x, const void* g, double step,
                     double thresh, void* out, double* stats, void* stream) {
  aw_status st;
  if ((st = check_dtype(dtype)) != AW_OK) return st;
  if (n < 1) return fail(AW_EINVAL, "n=%lld", (long long)n);
  if (!x || !g || !out) return fail(AW_EINVAL, "NULL data pointer");
  if (out == x || out == g) return fail(AW_EINVAL, "out must not alias x or g");
  if (!(step >= 0.0) || !(thresh >= 0.0) || !std::isfinite(step) || !std::isfinite(thresh))
    return fail(AW_EINVAL, "step=%g thresh=%g", step, thresh);
  st = hip_check(aw::launch_prox_l1(dtype == AW_F64, n, x, g, step, thresh, out, stats,
                                    (hipStream_t)stream),
                 "prox launch");
  return st == AW_OK ? ok() : st;
}

// ------------------------------------------------------- warm-start CNN
static aw_status cnn_shape(int32_t batch, int32_t rows, int32_t cols) {
  if (batch < 1 || rows < 1 || cols < 1)
    return fail(AW_EINVAL, "batch=%d rows=%d cols=%d", batch, rows, cols);
  const long long pix = (long long)batch * rows * cols;
  if (pix > (1LL << 31) / AW_CNN_CHANNELS)
    return fail(AW_EINVAL, "%lld pixels exceed the activation index range", pix);
  return AW_OK;
}

aw_status aw_cnn_sizes(int32_t batch, int32_t rows, int32_t cols, size_t* packed_bytes,
                       size_t* act_bytes, size_t* workspace_bytes) {
  aw_status st;
  if ((st = cnn_shape(batch, rows, cols)) != AW_OK) return st;
  if (packed_bytes) *packed_bytes = aw::CnnPack::total;
  if (act_bytes) *act_bytes = (size_t)batch * rows * cols * AW_CNN_ACT_BYTES;
  if (workspace_bytes) *workspace_bytes = aw::cnn_backward_scratch(batch, rows, cols);
  return ok();
}

aw_status aw_cnn_pack(const float* params, void* packed, void* stream) {
  if (!params || !packed) return fail(AW_EINVAL, "NULL pointer");
  aw_status st = hip_check(aw::launch_cnn_pack(params, packed, (hipStream_t)stream), "cnn pack");
  return st == AW_OK ? ok() : st;
}

aw_status aw_cnn_forward(const void* packed, int32_t batch, int32_t rows, int32_t cols,
                         const float* b, void* acts, float* u, void* stream) {
  aw_status st;
  if ((st = cnn_shape(batch, rows, cols)) != AW_OK) return st;
  if (!packed || !b || !acts || !u) return fail(AW_EINVAL, "NULL pointer");
  if ((const void*)u == (const void*)b) return fail(AW_EINVAL, "u must not alias b");
  st = hip_check(aw::launch_cnn_forward(packed, batch, rows, cols, b, acts, u, (hipStream_t)stream),
                 "cnn forward");
  return st == AW_OK ? ok() : st;
}

aw_status aw_cnn_backward(const void* packed, int32_t batch, int32_t rows, int32_t cols,
                          const float* b, const void* acts, const float* du, void* dacts,
                          float* grad, void* workspace, size_t workspace_bytes, void* stream) {
  aw_status st;
  if ((st = cnn_shape(batch, rows, cols)) != AW_OK) return st;
  if (!packed || !b || !acts || !du || !dacts || !grad || !workspace)
    return fail(AW_EINVAL, "NULL pointer");
  if (dacts == acts) return fail(AW_EINVAL, "dacts must not alias acts");
  const size_t need = aw::cnn_backward_scratch(batch, rows, cols);
  if (workspace_bytes < need)
    return fail(AW_EINVAL, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
  st = hip_check(aw::launch_cnn_backward(packed, batch, rows, cols, b, acts, du, dacts, grad,
                                         workspace, (hipStream_t)stream),
                 "cnn backward");
  return st == AW_OK ? ok() : st;
}

aw_status aw_adam_step(float* params, float* m, float* v, const float* grad, int64_t n,
                       int32_t step, double lr, double beta1, double beta2, double eps,
                       void* stream) {
  if (!params || !m || !v || !grad) return fail(AW_EINVAL, "NULL pointer");
  if (n < 1 || step < 1) return fail(AW_EINVAL, "n=%lld step=%d", (long long)n, step);
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return fail(AW_EINVAL, "lr=%g beta1=%g beta2=%g eps=%g", lr, beta1, beta2, eps);
  const double c1 = 1.0 / (1.0 - std::pow(beta1, step));
  const double c2 = 1.0 / (1.0 - std::pow(beta2, step));
  aw_status st = hip_check(aw::launch_adam(params, m, v, grad, n, lr, beta1, beta2, eps, c1, c2,
                                           (hipStream_t)stream),
                           "adam");
  return st == AW_OK ? ok() : st;
}

aw_status aw_sq_error_workspace(int64_t n, size_t* bytes) {
  if (n < 1 || !bytes) return fail(AW_EINVAL, "n=%lld", (long long)n);
  *bytes = (size_t)aw::sq_error_blocks(n) * sizeof(double);
  return ok();
}

aw_status aw_sq_error(int64_t n, const float* c, const float* target, double scale, float* grad,
                      double* loss, void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 1) return fail(AW_EINVAL, "n=%lld", (long long)n);
  if (!c || !target || !loss || !workspace) return fail(AW_EINVAL, "NULL pointer");
  const int blocks = aw::sq_error_blocks(n);
  if (workspace_bytes < (size_t)blocks * sizeof(double))
    return fail(AW_EINVAL, "workspace too small: %zu < %zu bytes", workspace_bytes,
                (size_t)blocks * sizeof(double));
  double* part = static_cast<double*>(workspace);
  hipStream_t s = (hipStream_t)stream;
  aw_status st = hip_check(aw::launch_sq_error(n, c, target, (float)scale, grad, part, s),
                           "squared error");
  if (st != AW_OK) return st;
  st = hip_check(aw::launch_reduce_partials(1, blocks, part, 1.0, loss, 1, 0, s), "reduce");
  return st == AW_OK ? ok() : st;
}

aw_status aw_soft_threshold(int64_t n, const float* in, double tau, float* out, void* stream) {
  if (n < 1 || !in || !out) return fail(AW_EINVAL, "n=%lld or NULL pointer", (long long)n);
  if (!(tau >= 0.0)) return fail(AW_EINVAL, "tau=%g", tau);
  aw_status st = hip_check(aw::launch_soft_threshold(n, in, (float)tau, out, (hipStream_t)stream),
                           "soft threshold");
  return st == AW_OK ? ok() : st;
}

}  // extern "C"
