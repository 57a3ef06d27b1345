"""Torch-facing wrappers over the C ABI (argument marshalling only).

Every compute step runs in libadjwave.so on the device. Torch supplies device
memory (inputs, outputs, workspace) and the current HIP stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import check, load

BC_NAMES = tuple(_lib.BC)


def daubechies(taps: int) -> np.ndarray:
    """Orthonormal Daubechies scaling filter of length ``taps`` (2, 4, ..., 16)."""
    out = (ctypes.c_double * taps)()
    check("aw_daubechies", load().aw_daubechies(taps, out))
    return np.array(out[:], dtype=np.float64)


def cdf97() -> tuple[np.ndarray, np.ndarray]:
    """Biorthogonal CDF 9/7 low-pass pair (synthesis, analysis), length 10."""
    hs, ha = (ctypes.c_double * 10)(), (ctypes.c_double * 10)()
    check("aw_cdf97", load().aw_cdf97(hs, ha))
    return np.array(hs[:], dtype=np.float64), np.array(ha[:], dtype=np.float64)


def gaussian_psf(sigma: float, radius: int) -> np.ndarray:
    out = (ctypes.c_double * (2 * radius + 1))()
    check("aw_gaussian_psf", load().aw_gaussian_psf(float(sigma), int(radius), out))
    return np.array(out[:], dtype=np.float64)


@dataclass
class WaveletSpec:
    """Multi-level 2-D wavelet transform of a rows x cols image: orthogonal
    Daubechies filters of `taps` taps (or the low-pass `lo`), or, with
    family="cdf97" (or `lo_analysis` given), a biorthogonal pair whose
    synthesis low-pass is `lo` and analysis low-pass `lo_analysis`."""
    rows: int
    cols: int
    levels: int
    taps: int = 8
    bc: str = "sym"
    lo: np.ndarray | None = None
    lo_analysis: np.ndarray | None = None
    family: str = "daubechies"
    _c: _lib.Wavelet = field(init=False, repr=False)

    def __post_init__(self):
        if self.bc not in _lib.BC:
            raise ValueError(f"bc must be one of {BC_NAMES}")
        if self.family == "cdf97":
            self.lo, self.lo_analysis = cdf97()
        elif self.family != "daubechies":
            raise ValueError("family must be 'daubechies' or 'cdf97'")
        if self.lo is None:
            self.lo = daubechies(self.taps)
        self.lo = np.asarray(self.lo, dtype=np.float64)
        self.taps = len(self.lo)
        c = _lib.Wavelet()
        c.rows, c.cols, c.levels, c.filter_len = self.rows, self.cols, self.levels, self.taps
        c.bc = _lib.BC[self.bc]
        for k, v in enumerate(self.lo):
            c.lo[k] = float(v)
        if self.lo_analysis is not None:
            self.lo_analysis = np.asarray(self.lo_analysis, dtype=np.float64)
            if len(self.lo_analysis) != self.taps:
                raise ValueError("lo and lo_analysis must have the same length")
            c.biorthogonal = 1
            for k, v in enumerate(self.lo_analysis):
                c.lo_analysis[k] = float(v)
        self._c = c

    @property
    def filters(self):
        """The oracle's filter argument: lo, or the pair (lo, lo_analysis)."""
        return self.lo if self.lo_analysis is None else (self.lo, self.lo_analysis)

    @property
    def c(self):
        return ctypes.byref(self._c)

    def layout(self):
        """(ncoef, row sizes [N, K_1..K_J], col sizes)."""
        n = ctypes.c_int64()
        sr = (ctypes.c_int32 * (self.levels + 1))()
        sc = (ctypes.c_int32 * (self.levels + 1))()
        check("aw_wavelet_layout", load().aw_wavelet_layout(self.c, ctypes.byref(n), sr, sc))
        return int(n.value), list(sr), list(sc)

    @property
    def ncoef(self) -> int:
        return self.layout()[0]


@dataclass
class BlurSpec:
    """Separable PSF with reflexive boundaries: Gaussian (sigma, radius) or
    explicit taps (length 2*radius+1)."""
    rows: int
    cols: int
    sigma: float | None = None
    radius: int | None = None
    taps: np.ndarray | None = None
    _c: _lib.Blur = field(init=False, repr=False)

    def __post_init__(self):
        if self.taps is None:
            if self.sigma is None or self.radius is None:
                raise ValueError("give sigma and radius, or taps")
            self.taps = gaussian_psf(self.sigma, self.radius)
        self.taps = np.asarray(self.taps, dtype=np.float64)
        self.radius = (len(self.taps) - 1) // 2
        if len(self.taps) > 2 * _lib.MAX_RADIUS + 1:
            raise ValueError(f"radius {self.radius} > {_lib.MAX_RADIUS}: the tile kernels take "
                             "narrower PSFs (BlurDCT applies wider symmetric ones)")
        c = _lib.Blur()
        c.rows, c.cols, c.radius = self.rows, self.cols, self.radius
        for k, v in enumerate(self.taps):
            c.taps[k] = float(v)
        self._c = c

    @property
    def c(self):
        return ctypes.byref(self._c)


# ----------------------------------------------------------------- helpers
def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return _lib.F32
    if t.dtype == torch.float64:
        return _lib.F64
    raise TypeError(f"float32 or float64 tensors expected, got {t.dtype}")


def _dev(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("device tensors expected (the library runs on the GPU only)")
    if not t.is_contiguous():
        raise ValueError("contiguous tensors expected")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def workspace_bytes(w: WaveletSpec | None, b: BlurSpec | None, dtype: torch.dtype,
                    batch: int) -> int:
    n = ctypes.c_size_t()
    code = _lib.F64 if dtype == torch.float64 else _lib.F32
    check("aw_workspace_size", load().aw_workspace_size(
        w.c if w is not None else None, b.c if b is not None else None, code, batch,
        ctypes.byref(n)))
    return int(n.value)


def _workspace(w, b, ref: torch.Tensor, batch: int):
    n = workspace_bytes(w, b, ref.dtype, batch)
    return torch.empty(max(n, 1), dtype=torch.uint8, device=ref.device), n


def _batch_img(x: torch.Tensor, rows: int, cols: int) -> int:
    if x.shape[-2:] != (rows, cols):
        raise ValueError(f"image shape {tuple(x.shape)} does not end in ({rows}, {cols})")
    return int(np.prod(x.shape[:-2])) if x.dim() > 2 else 1


def _batch_coef(x: torch.Tensor, ncoef: int) -> int:
    if x.shape[-1] != ncoef:
        raise ValueError(f"coefficient shape {tuple(x.shape)} does not end in {ncoef}")
    return int(np.prod(x.shape[:-1])) if x.dim() > 1 else 1


# ----------------------------------------------------------- wavelet ops
def _coef_to_img(fn, w: WaveletSpec, coef: torch.Tensor, out=None):
    _dev(coef)
    batch = _batch_coef(coef, w.ncoef)
    if out is None:
        out = torch.empty(coef.shape[:-1] + (w.rows, w.cols), dtype=coef.dtype, device=coef.device)
    ws, n = _workspace(w, None, coef, batch)
    check(fn, getattr(load(), fn)(w.c, _dtype_code(coef), batch, _ptr(coef), _ptr(_dev(out)),
                                   _ptr(ws), n, _stream(coef)))
    return out


def _img_to_coef(fn, w: WaveletSpec, img: torch.Tensor, out=None):
    _dev(img)
    batch = _batch_img(img, w.rows, w.cols)
    if out is None:
        out = torch.empty(img.shape[:-2] + (w.ncoef,), dtype=img.dtype, device=img.device)
    ws, n = _workspace(w, None, img, batch)
    check(fn, getattr(load(), fn)(w.c, _dtype_code(img), batch, _ptr(img), _ptr(_dev(out)),
                                   _ptr(ws), n, _stream(img)))
    return out


def wavelet_synth(w: WaveletSpec, coef: torch.Tensor, out=None) -> torch.Tensor:
    """W coef (synthesis)."""
    return _coef_to_img("wavelet_synth", w, coef, out)


def wavelet_synth_adjoint(w: WaveletSpec, img: torch.Tensor, out=None) -> torch.Tensor:
    """W^* img (true adjoint, eq. 2)."""
    return _img_to_coef("wavelet_synth_adjoint", w, img, out)


def wavelet_analysis(w: WaveletSpec, img: torch.Tensor, out=None) -> torch.Tensor:
    """W^dagger img (analysis)."""
    return _img_to_coef("aw_wavelet_analysis", w, img, out)


def wavelet_analysis_adjoint(w: WaveletSpec, coef: torch.Tensor, out=None) -> torch.Tensor:
    """(W^dagger)^* coef (synthesis with a summing fold)."""
    return _coef_to_img("aw_wavelet_analysis_adjoint", w, coef, out)


# -------------------------------------------------------------- blur ops
def _blur_call(fn, b: BlurSpec, x: torch.Tensor, out=None):
    _dev(x)
    batch = _batch_img(x, b.rows, b.cols)
    if out is None:
        out = torch.empty_like(x)
    check(fn, getattr(load(), fn)(b.c, _dtype_code(x), batch, _ptr(x), _ptr(_dev(out)),
                                   _stream(x)))
    return out


def blur(b: BlurSpec, x: torch.Tensor, out=None) -> torch.Tensor:
    """R x."""
    return _blur_call("blur", b, x, out)


def blur_adjoint(b: BlurSpec, y: torch.Tensor, out=None) -> torch.Tensor:
    """R^* y."""
    return _blur_call("blur_adjoint", b, y, out)


class BlurDCT:
    """R by DCT-II diagonalisation: a symmetric PSF of any radius (taps, host
    float64 array of odd length), power-of-two sizes up to 4096."""

    def __init__(self, rows: int, cols: int, taps, dtype=torch.float32):
        taps = np.ascontiguousarray(np.asarray(taps, dtype=np.float64))
        if taps.ndim != 1 or len(taps) % 2 == 0:
            raise ValueError("taps: odd-length 1-D array")
        self.rows, self.cols, self.dtype = rows, cols, dtype
        self.radius = (len(taps) - 1) // 2
        self._plan = ctypes.c_void_p()
        code = _lib.F64 if dtype == torch.float64 else _lib.F32
        check("aw_blur_dct_create", load().aw_blur_dct_create(
            rows, cols, self.radius, taps.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), code,
            ctypes.byref(self._plan)))

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value:
            load().aw_blur_dct_destroy(plan)
            self._plan = None

    def apply(self, x: torch.Tensor, out=None) -> torch.Tensor:
        _dev(x)
        if x.dtype != self.dtype:
            raise TypeError(f"{self.dtype} tensors expected")
        batch = _batch_img(x, self.rows, self.cols)
        if out is None:
            out = torch.empty_like(x)
        n = ctypes.c_size_t()
        check("aw_blur_dct_workspace", load().aw_blur_dct_workspace(self._plan, batch,
                                                                    ctypes.byref(n)))
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=x.device)
        check("aw_blur_dct_apply", load().aw_blur_dct_apply(
            self._plan, batch, _ptr(x), _ptr(_dev(out)), _ptr(ws), n.value, _stream(x)))
        return out


# -------------------------------------------------------------- A, A^*
def apply_A(w: WaveletSpec, b: BlurSpec, coef: torch.Tensor, out=None) -> torch.Tensor:
    _dev(coef)
    batch = _batch_coef(coef, w.ncoef)
    if out is None:
        out = torch.empty(coef.shape[:-1] + (w.rows, w.cols), dtype=coef.dtype, device=coef.device)
    ws, n = _workspace(w, b, coef, batch)
    check("aw_apply_A", load().aw_apply_A(w.c, b.c, _dtype_code(coef), batch, _ptr(coef),
                                          _ptr(_dev(out)), _ptr(ws), n, _stream(coef)))
    return out


def apply_A_fused(w: WaveletSpec, b: BlurSpec, coef: torch.Tensor, sub=None,
                  out=None) -> torch.Tensor:
    """A coef - sub (sub None: A coef) with the finest synthesis level and the
    blur in one pass (float32; zpd, sym or per; 2, 8 or 16 taps)."""
    _dev(coef)
    batch = _batch_coef(coef, w.ncoef)
    shape = coef.shape[:-1] + (w.rows, w.cols)
    if sub is not None:
        _dev(sub)
        if tuple(sub.shape) != tuple(shape) or sub.dtype != coef.dtype or not sub.is_contiguous():
            raise ValueError(f"sub must be a contiguous {coef.dtype} tensor of shape {tuple(shape)}")
    if out is None:
        out = torch.empty(shape, dtype=coef.dtype, device=coef.device)
    ws, n = _workspace(w, b, coef, batch)
    check("aw_apply_A_fused",
          load().aw_apply_A_fused(w.c, b.c, _dtype_code(coef), batch, _ptr(coef),
                                  _ptr(sub) if sub is not None else None, _ptr(_dev(out)),
                                  _ptr(ws), n, _stream(coef)))
    return out


def apply_A_adjoint(w: WaveletSpec, b: BlurSpec, img: torch.Tensor, out=None) -> torch.Tensor:
    _dev(img)
    batch = _batch_img(img, w.rows, w.cols)
    if out is None:
        out = torch.empty(img.shape[:-2] + (w.ncoef,), dtype=img.dtype, device=img.device)
    ws, n = _workspace(w, b, img, batch)
    check("aw_apply_A_adjoint", load().aw_apply_A_adjoint(w.c, b.c, _dtype_code(img), batch,
                                                          _ptr(img), _ptr(_dev(out)), _ptr(ws), n,
                                                          _stream(img)))
    return out


def apply_A_adjoint_fused(w: WaveletSpec, b: BlurSpec, img: torch.Tensor,
                          out=None) -> torch.Tensor:
    """A^* img with the blur adjoint fused into the finest analysis level
    (float32; zpd or sym; 2, 8 or 16 taps)."""
    _dev(img)
    batch = _batch_img(img, w.rows, w.cols)
    if out is None:
        out = torch.empty(img.shape[:-2] + (w.ncoef,), dtype=img.dtype, device=img.device)
    ws, n = _workspace(w, b, img, batch)
    check("aw_apply_A_adjoint_fused",
          load().aw_apply_A_adjoint_fused(w.c, b.c, _dtype_code(img), batch, _ptr(img),
                                          _ptr(_dev(out)), _ptr(ws), n, _stream(img)))
    return out


# ------------------------------------------------------------------ FISTA
class FistaState:
    """Device buffers and counters of one FISTA run (x, y coefficient
    tensors, residual image, objective partials)."""

    GRADIENTS = {"adjoint": 0, "pinv": 1}

    def __init__(self, w: WaveletSpec, b: BlurSpec, b_obs: torch.Tensor, x0=None,
                 gradient: str = "adjoint"):
        """gradient: "adjoint" (W^* R^*, the true gradient) or "pinv" (W^dagger in
        the place of W^*)."""
        _dev(b_obs)
        if gradient not in self.GRADIENTS:
            raise ValueError(f"gradient must be one of {sorted(self.GRADIENTS)}")
        self.gradient = gradient
        self.w, self.b = w, b
        self.batch = _batch_img(b_obs, w.rows, w.cols)
        lead = b_obs.shape[:-2]
        self.x = (torch.zeros(lead + (w.ncoef,), dtype=b_obs.dtype, device=b_obs.device)
                  if x0 is None else x0.clone().contiguous())
        self.y = self.x.clone()
        self.resid = torch.empty_like(b_obs)
        self.obj = torch.zeros(self.batch, 2, dtype=torch.float64, device=b_obs.device)
        self.k = 1
        self.t = 1.0
        self.ws, self.ws_n = _workspace(w, b, b_obs, self.batch)

    def c_state(self):
        s = _lib.FistaState()
        s.x, s.y, s.resid = self.x.data_ptr(), self.y.data_ptr(), self.resid.data_ptr()
        s.obj = self.obj.data_ptr()
        s.k, s.t = self.k, self.t
        s.gradient = self.GRADIENTS[self.gradient]
        return s


def fista_step(state: FistaState, b_obs: torch.Tensor, lam: float, L: float = 1.0,
               want_objective: bool = False) -> None:
    """One FISTA iteration on the state (in place)."""
    cs = state.c_state()
    check("fista_step", load().fista_step(state.w.c, state.b.c, _dtype_code(b_obs), state.batch,
                                          _ptr(_dev(b_obs)), float(L), float(lam),
                                          ctypes.byref(cs), int(bool(want_objective)),
                                          _ptr(state.ws), state.ws_n, _stream(b_obs)))
    state.k, state.t = int(cs.k), float(cs.t)


def fista_step_noalloc(state: FistaState, b_obs: torch.Tensor, lam: float, L: float = 1.0,
                       want_objective: bool = False) -> None:
    """fista_step with the library's static device scratch as its workspace
    (no allocation; problems up to 64 MiB of workspace). Calls that overlap
    on one GPU share that scratch and race."""
    cs = state.c_state()
    check("fista_step_noalloc",
          load().fista_step_noalloc(state.w.c, state.b.c, _dtype_code(b_obs), state.batch,
                                    _ptr(_dev(b_obs)), float(L), float(lam), ctypes.byref(cs),
                                    int(bool(want_objective)), _stream(b_obs)))
    state.k, state.t = int(cs.k), float(cs.t)


def fista_update(state: FistaState, grad: torch.Tensor, lam: float, L: float = 1.0,
                 want_l1: bool = False) -> None:
    """The update half of a FISTA iteration from an image-space gradient
    grad (R^*(A y - b) for eq. (1)): x, y, k, t of the state advance as in
    fista_step; with want_l1, state.obj[:, 1] = ||x_k||_1."""
    _dev(grad)
    if _batch_img(grad, state.w.rows, state.w.cols) != state.batch:
        raise ValueError("grad batch differs from the state's")
    cs = state.c_state()
    ws, n = _workspace(state.w, None, grad, state.batch)
    check("aw_fista_update", load().aw_fista_update(state.w.c, _dtype_code(grad), state.batch,
                                                    _ptr(grad), float(L), float(lam),
                                                    ctypes.byref(cs), int(bool(want_l1)),
                                                    _ptr(ws), n, _stream(grad)))
    state.k, state.t = int(cs.k), float(cs.t)


def objective(w: WaveletSpec, b: BlurSpec, b_obs: torch.Tensor, x: torch.Tensor, lam: float,
              out: torch.Tensor | None = None) -> torch.Tensor:
    """[batch, 3] FP64 device tensor: 1/2||Ax-b||^2, ||x||_1, F(x) (eq. 1)."""
    _dev(b_obs)
    _dev(x)
    batch = _batch_img(b_obs, w.rows, w.cols)
    if out is None:
        out = torch.empty(batch, 3, dtype=torch.float64, device=x.device)
    ws, n = _workspace(w, b, x, batch)
    check("aw_objective", load().aw_objective(w.c, b.c, _dtype_code(x), batch, _ptr(b_obs),
                                              float(lam), _ptr(x), _ptr(out), _ptr(ws), n,
                                              _stream(x)))
    return out


# -------------------------------------------------------- conv adjoint pair
def conv_adjoint_pair(h: torch.Tensor, s: torch.Tensor, x_obs: torch.Tensor | None = None,
                      need_grad_h: bool = True, need_grad_s: bool = True):
    """(resid, grad_h, grad_s) of f = 1/2 ||h * s - x_obs||^2 for a batch of
    pairs; h: [B, K], s: [B, N], x_obs: [B, K+N-1]."""
    _dev(h)
    _dev(s)
    if h.dim() == 1:
        h, s = h[None], s[None]
        x_obs = x_obs[None] if x_obs is not None else None
    B, K = h.shape
    N = s.shape[1]
    if s.shape[0] != B or s.dtype != h.dtype:
        raise ValueError("h and s must share batch and dtype")
    if x_obs is not None and (tuple(x_obs.shape) != (B, K + N - 1) or x_obs.dtype != h.dtype):
        raise ValueError("x_obs must be [B, K+N-1] of the same dtype")
    resid = torch.empty(B, K + N - 1, dtype=h.dtype, device=h.device)
    gh = torch.empty_like(h) if need_grad_h else None
    gs = torch.empty_like(s) if need_grad_s else None
    check("conv_adjoint_pair", load().conv_adjoint_pair(
        _dtype_code(h), B, K, N, _ptr(h), _ptr(s), _ptr(_dev(x_obs)) if x_obs is not None else None,
        _ptr(resid), _ptr(gh), _ptr(gs), _stream(h)))
    return resid, gh, gs


# ------------------------------------------------------- warm-start CNN
CNN_PARAMS = 37601
CNN_CHANNELS = 32


def cnn_sizes(batch: int, rows: int, cols: int):
    """(packed parameter bytes, activation bytes, backward workspace bytes)."""
    pk, act, ws = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    check("aw_cnn_sizes", load().aw_cnn_sizes(batch, rows, cols, ctypes.byref(pk),
                                              ctypes.byref(act), ctypes.byref(ws)))
    return int(pk.value), int(act.value), int(ws.value)


def _f32(t: torch.Tensor) -> torch.Tensor:
    _dev(t)
    if t.dtype != torch.float32:
        raise ValueError("float32 tensors expected")
    return t


def cnn_pack(params: torch.Tensor, packed: torch.Tensor) -> torch.Tensor:
    """BF16 kernel layouts of the FP32 master parameters (device-side)."""
    _f32(params)
    if params.numel() != CNN_PARAMS:
        raise ValueError(f"{CNN_PARAMS} parameters expected")
    check("aw_cnn_pack", load().aw_cnn_pack(_ptr(params), _ptr(_dev(packed)), _stream(params)))
    return packed


def _img_batch(b: torch.Tensor):
    if b.dim() == 2:
        return 1, b.shape[0], b.shape[1]
    if b.dim() != 3:
        raise ValueError("images [rows, cols] or [batch, rows, cols] expected")
    return b.shape[0], b.shape[1], b.shape[2]


def cnn_forward(packed: torch.Tensor, b: torch.Tensor, acts: torch.Tensor,
                u: torch.Tensor | None = None) -> torch.Tensor:
    """u = b + CNN(b); acts (uint8 buffer of cnn_sizes()[1] bytes) receives y_1..y_5."""
    _f32(b)
    n, H, W = _img_batch(b)
    if u is None:
        u = torch.empty_like(b)
    check("aw_cnn_forward", load().aw_cnn_forward(_ptr(_dev(packed)), n, H, W, _ptr(b),
                                                  _ptr(_dev(acts)), _ptr(_f32(u)), _stream(b)))
    return u


def cnn_backward(packed: torch.Tensor, b: torch.Tensor, acts: torch.Tensor, du: torch.Tensor,
                 dacts: torch.Tensor, grad: torch.Tensor, ws: torch.Tensor) -> torch.Tensor:
    """grad = d<du, CNN(b)>/d params (FP32 master layout, overwritten)."""
    _f32(b)
    n, H, W = _img_batch(b)
    if du.shape != b.shape:
        raise ValueError("du must have the shape of b")
    check("aw_cnn_backward", load().aw_cnn_backward(
        _ptr(_dev(packed)), n, H, W, _ptr(b), _ptr(_dev(acts)), _ptr(_f32(du)),
        _ptr(_dev(dacts)), _ptr(_f32(grad)), _ptr(_dev(ws)), ws.numel() * ws.element_size(),
        _stream(b)))
    return grad


def adam_step(params, m, v, grad, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8) -> None:
    n = params.numel()
    for t in (params, m, v, grad):
        _f32(t)
        if t.numel() != n:
            raise ValueError("params, m, v and grad must have the same size")
    check("aw_adam_step", load().aw_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), n, step,
                                              lr, beta1, beta2, eps, _stream(params)))


def sq_error(c: torch.Tensor, target: torch.Tensor, scale: float = 1.0,
             grad: torch.Tensor | None = None, loss: torch.Tensor | None = None,
             ws: torch.Tensor | None = None) -> torch.Tensor:
    """loss = sum (c - target)^2 (FP64 device scalar); grad = scale * 2 (c - target)."""
    _f32(c)
    _f32(target)
    n = c.numel()
    if target.numel() != n or (grad is not None and grad.numel() != n):
        raise ValueError("size mismatch")
    need = ctypes.c_size_t()
    check("aw_sq_error_workspace", load().aw_sq_error_workspace(n, ctypes.byref(need)))
    if ws is None:
        ws = torch.empty(need.value, dtype=torch.uint8, device=c.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=c.device)
    check("aw_sq_error", load().aw_sq_error(n, _ptr(c), _ptr(target), scale,
                                            _ptr(_f32(grad)) if grad is not None else None,
                                            _ptr(_dev(loss)), _ptr(_dev(ws)),
                                            ws.numel() * ws.element_size(), _stream(c)))
    return loss


def soft_threshold(x: torch.Tensor, tau: float, out: torch.Tensor | None = None) -> torch.Tensor:
    _f32(x)
    if out is None:
        out = torch.empty_like(x)
    check("aw_soft_threshold", load().aw_soft_threshold(x.numel(), _ptr(x), tau, _ptr(_f32(out)),
                                                        _stream(x)))
    return out
