"""Wavelet synthesis W, analysis W^dagger and the true adjoint W^* (oracle).

TEST INFRASTRUCTURE ONLY.

Zero-boundary core (the software transform "for extended signals under zero
boundary conditions", Sec. "A few signal extensions"). For a length-M signal u
and a reconstruction filter f in {h, g} (decomposition filter = f reversed):

    Phi_f u  =  odd-indexed samples of the full linear convolution (f reversed) * u,
    K = floor((M + L - 1) / 2) coefficients per band.

The rows of Phi = [Phi_h; Phi_g] are all even shifts of h and g that overlap
[0, M), so Phi^* Phi = I (Phi is an isometry) for any orthonormal filter pair;
this is the statement W^*_zpd = W^dagger_zpd for orthogonal wavelets.

One level with extension E (oracle.extension):
    W^dagger = Phi E                 (analysis, Sec. "A few signal extensions")
    W        = E^dagger Phi^*        (synthesis = pseudoinverse of analysis)
    W^*      = Phi (E^dagger)^*      (eq. 2: the true adjoint)
    (W^dagger)^* = E^* Phi^*         (synthesis with a summing fold)

Biorthogonal filters (Sec. "The adjoint for biorthogonal wavelets") are passed
as a pair h = (h_syn, h_ana): W and its adjoint W^* use the synthesis side,
W^dagger and (W^dagger)^* the analysis side, so that W^* = W~^dagger_zpd
(E^dagger)^* (eq. 4) is the analysis with the dual (synthesis) filters under
the same (E^dagger)^* fold; W^*_zpd no longer equals W^dagger_zpd.

Mode 'per' is the critically sampled circular transform,
c_f[k] = sum_q f[q] y[(2k+q) mod N], K = N/2, which is square and orthogonal,
so W^* = W^dagger = W^{-1}.

2-D (footnote of Sec. "A few signal extensions": "extended to 2d quite
naturally"): the tensor product of the 1-D maps along rows (axis 0) and
columns (axis 1). Subbands of one level: a = lo/lo, H = hi along rows & lo
along columns, V = lo along rows & hi along columns, D = hi/hi.
Multi-level: a_0 = image; level j maps a_{j-1} -> (a_j, H_j, V_j, D_j); the
coefficient vector is [a_J, H_J, V_J, D_J, H_{J-1}, ..., D_1], each row-major.
"""
from __future__ import annotations

import numpy as np

from . import extension as ext
from .filters import flen, side_taps

MODES = ("zpd", "sym", "per", "per_ext")


# ----------------------------------------------------------------- sizes
def coef_len(N: int, L: int, mode: str) -> int:
    """Coefficients per band after one level of a length-N signal."""
    if mode == "per":
        if N % 2:
            raise ValueError("per mode needs an even length at every level")
        return N // 2
    M = N + 2 * ext.ext_width(mode, L)
    return (M + L - 1) // 2


def level_sizes(N: int, L: int, mode: str, levels: int):
    """[N_0 = N, K_1, ..., K_J] along one axis."""
    sizes = [N]
    for _ in range(levels):
        sizes.append(coef_len(sizes[-1], L, mode))
    return sizes


def layout(rows: int, cols: int, L: int, mode: str, levels: int):
    """(ncoef, row sizes, col sizes) of the coefficient vector."""
    sr = level_sizes(rows, L, mode, levels)
    sc = level_sizes(cols, L, mode, levels)
    n = sr[levels] * sc[levels] + sum(3 * sr[j] * sc[j] for j in range(1, levels + 1))
    return n, sr, sc


# ------------------------------------------------------- 1-D cores, last axis
def _full_conv(u: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Full linear convolution along the last axis: out[n] = sum_m d[m] u[n-m]."""
    M, L = u.shape[-1], len(d)
    out = np.zeros(u.shape[:-1] + (M + L - 1,))
    for m in range(L):
        out[..., m:m + M] += d[m] * u
    return out


def phi(u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Phi_f along the last axis: odd samples of (f reversed) * u."""
    return _full_conv(u, f[::-1])[..., 1::2]


def phi_adj(c: np.ndarray, f: np.ndarray, M: int) -> np.ndarray:
    """Phi_f^* along the last axis (transpose of ``phi``): place c at the odd
    positions of a length M+L-1 signal, convolve with f, keep [L-1, L-1+M)."""
    L = len(f)
    z = np.zeros(c.shape[:-1] + (M + L - 1,))
    z[..., 1::2] = c
    return _full_conv(z, f)[..., L - 1:L - 1 + M]


def per_ana(y: np.ndarray, f: np.ndarray) -> np.ndarray:
    """c[k] = sum_q f[q] y[(2k+q) mod N] along the last axis."""
    N = y.shape[-1]
    k = np.arange(N // 2)
    c = np.zeros(y.shape[:-1] + (N // 2,))
    for q in range(len(f)):
        c += f[q] * y[..., (2 * k + q) % N]
    return c


def per_syn(c: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Transpose of ``per_ana``: y[(2k+q) mod N] += f[q] c[k]."""
    K = c.shape[-1]
    N = 2 * K
    k = np.arange(K)
    y = np.zeros(c.shape[:-1] + (N,))
    for q in range(len(f)):
        np.add.at(y, (Ellipsis, (2 * k + q) % N), f[q] * c)
    return y


# ----------------------------------------------------- 1-D one level, any axis
def ana1(y: np.ndarray, h, mode: str, axis: int, weights: str):
    """One analysis level along ``axis``. weights='ones' -> W^dagger = Phi E;
    weights='pinv' -> W^* = Phi (E^dagger)^*. Returns (lo, hi). For a
    biorthogonal pair W^dagger filters with the analysis side and W^*, the
    adjoint of the synthesis, with the synthesis side (eq. 4)."""
    h, g = side_taps(h, "syn" if weights == "pinv" else "ana")
    y = np.moveaxis(y, axis, -1)
    if mode == "per":
        lo, hi = per_ana(y, h), per_ana(y, g)
    else:
        e = ext.ext_width(mode, len(h))
        u = ext.extend(y, e, mode, axis=-1, weights=weights)
        lo, hi = phi(u, h), phi(u, g)
    return np.moveaxis(lo, -1, axis), np.moveaxis(hi, -1, axis)


def syn1(lo: np.ndarray, hi: np.ndarray, h, mode: str, N: int, axis: int, weights: str):
    """One synthesis level along ``axis``. weights='pinv' -> W = E^dagger Phi^*
    (synthesis side of a biorthogonal pair); weights='ones' ->
    (W^dagger)^* = E^* Phi^* (analysis side)."""
    h, g = side_taps(h, "syn" if weights == "pinv" else "ana")
    lo = np.moveaxis(lo, axis, -1)
    hi = np.moveaxis(hi, axis, -1)
    if mode == "per":
        y = per_syn(lo, h) + per_syn(hi, g)
        if y.shape[-1] != N:
            raise ValueError("per size mismatch")
    else:
        e = ext.ext_width(mode, len(h))
        M = N + 2 * e
        v = phi_adj(lo, h, M) + phi_adj(hi, g, M)
        y = ext.fold(v, N, e, mode, axis=-1, weights=weights)
    return np.moveaxis(y, -1, axis)


# ----------------------------------------------------------- 2-D one level
def ana2(img: np.ndarray, h, mode: str, weights: str):
    """(a, H, V, D) of one 2-D level; rows = axis -2, columns = axis -1."""
    lo_c, hi_c = ana1(img, h, mode, axis=-1, weights=weights)
    a, H = ana1(lo_c, h, mode, axis=-2, weights=weights)
    V, D = ana1(hi_c, h, mode, axis=-2, weights=weights)
    return a, H, V, D


def syn2(a, H, V, D, h, mode: str, rows: int, cols: int, weights: str):
    """Inverse structure of ``ana2`` (synthesis of one 2-D level)."""
    lo_c = syn1(a, H, h, mode, rows, axis=-2, weights=weights)
    hi_c = syn1(V, D, h, mode, rows, axis=-2, weights=weights)
    return syn1(lo_c, hi_c, h, mode, cols, axis=-1, weights=weights)


# ------------------------------------------------------------- multi-level
def _pack(a_J, details):
    """details = [(H_J, V_J, D_J), ..., (H_1, V_1, D_1)] -> flat vector(s)."""
    lead = a_J.shape[:-2]
    parts = [a_J.reshape(lead + (-1,))]
    for H, V, D in details:
        parts += [H.reshape(lead + (-1,)), V.reshape(lead + (-1,)), D.reshape(lead + (-1,))]
    return np.concatenate(parts, axis=-1)


def _unpack(x: np.ndarray, sr, sc, levels: int):
    lead = x.shape[:-1]
    pos = 0

    def take(r, c):
        nonlocal pos
        blk = x[..., pos:pos + r * c].reshape(lead + (r, c))
        pos += r * c
        return blk

    a_J = take(sr[levels], sc[levels])
    details = []
    for j in range(levels, 0, -1):
        details.append((take(sr[j], sc[j]), take(sr[j], sc[j]), take(sr[j], sc[j])))
    if pos != x.shape[-1]:
        raise ValueError("coefficient length mismatch")
    return a_J, details


def analysis(img: np.ndarray, h, mode: str, levels: int, weights: str = "ones"):
    """J-level 2-D analysis. weights='ones' gives W^dagger, 'pinv' gives W^*."""
    img = np.asarray(img, dtype=np.float64)
    a = img
    details = []
    for _ in range(levels):
        a, H, V, D = ana2(a, h, mode, weights)
        details.append((H, V, D))
    return _pack(a, details[::-1])


def synthesis(x: np.ndarray, h, mode: str, levels: int, rows: int, cols: int,
              weights: str = "pinv"):
    """J-level 2-D synthesis. weights='pinv' gives W, 'ones' gives (W^dagger)^*."""
    x = np.asarray(x, dtype=np.float64)
    _, sr, sc = layout(rows, cols, flen(h), mode, levels)
    a, details = _unpack(x, sr, sc, levels)
    for idx, j in enumerate(range(levels, 0, -1)):
        H, V, D = details[idx]
        a = syn2(a, H, V, D, h, mode, sr[j - 1], sc[j - 1], weights)
    return a


def W(x, h, mode, levels, rows, cols):
    """Wavelet synthesis (reconstruction) W: coefficients -> image."""
    return synthesis(x, h, mode, levels, rows, cols, weights="pinv")


def W_adj(img, h, mode, levels):
    """True adjoint W^* = per level Phi (E^dagger)^* (eq. 2)."""
    return analysis(img, h, mode, levels, weights="pinv")


def W_pinv(img, h, mode, levels):
    """Wavelet analysis W^dagger = per level Phi E."""
    return analysis(img, h, mode, levels, weights="ones")


def W_pinv_adj(x, h, mode, levels, rows, cols):
    """(W^dagger)^* = per level E^* Phi^* (synthesis with a summing fold)."""
    return synthesis(x, h, mode, levels, rows, cols, weights="ones")


def dense(fn, n_in: int, in_shape=None) -> np.ndarray:
    """Explicit matrix of a linear map (tiny sizes only): ``fn`` is applied to
    the whole identity at once, as a batch of unit inputs of shape ``in_shape``
    (default: flat vectors of length n_in) along a leading axis."""
    shape = (n_in,) if in_shape is None else tuple(in_shape)
    out = np.asarray(fn(np.eye(n_in).reshape((n_in,) + shape)), dtype=np.float64)
    return out.reshape(n_in, -1).T
