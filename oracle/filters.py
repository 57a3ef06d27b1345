"""Orthonormal Daubechies scaling filters (oracle; test infrastructure only).

The paper uses orthogonal wavelets, "Haar and more generally Daubechies"
(Sec. "The adjoint for orthogonal wavelets"). It prints no coefficients, so
they are derived here from the classical construction: the squared magnitude
response of a p-vanishing-moment scaling filter is

    |H(w)|^2 = 2 cos^{2p}(w/2) P(sin^2(w/2)),   P(y) = sum_{k<p} C(p-1+k, k) y^k,

and the minimum-phase spectral factor keeps, for every root y_i of P, the root
of z + 1/z = 2 - 4 y_i that lies inside the unit circle. H(z) = sum h[n] z^-n
then has p zeros at z = -1 plus those roots; it is scaled so sum h = sqrt(2).

The high-pass (wavelet) filter is the alternating flip
g[k] = (-1)^k h[L-1-k], L = 2p.

Biorthogonal CDF 9/7 (Sec. "The adjoint for biorthogonal wavelets"): the same
product filter with p = 4, 2 cos^8(w/2) P(y), split between two symmetric
low-pass filters instead of a spectral factor and its mirror: each keeps
cos^4(w/2), the 7-tap synthesis filter takes the real root y_1 of P and the
9-tap analysis filter the complex pair,

    H_s(w) = sqrt(2) cos^4(w/2) (1 - y/y_1),
    H_a(w) = sqrt(2) cos^4(w/2) (1 - y/y_2)(1 - y/y_3),   y = sin^2(w/2),

so that H_a conj(H_s) = 2 cos^8(w/2) P(y) (biorthogonality). With
cos^2(w/2) = (z + 2 + 1/z)/4 and sin^2(w/2) = (2 - z - 1/z)/4 both are
symmetric Laurent polynomials; they are stored as length-10 filters centred on
the same index (4), as the software transform pads them: synthesis taps at
1..7, analysis taps at 0..8. A biorthogonal pair is passed around as the tuple
(h_syn, h_ana); the high-pass filters are the alternating flips of the other
side's low-pass, g_syn = highpass(h_ana), g_ana = highpass(h_syn).
"""
from __future__ import annotations

from math import comb

import numpy as np


def daubechies(p: int) -> np.ndarray:
    """Scaling filter with p vanishing moments, length 2p, float64."""
    if p < 1:
        raise ValueError("p >= 1")
    poly_y = [float(comb(p - 1 + k, k)) for k in range(p)]  # ascending powers of y
    zeros = [-1.0 + 0j] * p
    if p > 1:
        for y in np.roots(poly_y[::-1]):
            b = 2.0 - 4.0 * y
            disc = np.sqrt(b * b - 4.0 + 0j)
            z1, z2 = (b + disc) / 2.0, (b - disc) / 2.0
            zeros.append(z1 if abs(z1) < 1.0 else z2)
    # descending-power coefficients of prod (z - z_i) are h[0], h[1], ...
    h = np.real(np.poly(np.array(zeros)))
    return h * (np.sqrt(2.0) / h.sum())


def highpass(h: np.ndarray) -> np.ndarray:
    """Alternating flip g[k] = (-1)^k h[L-1-k]."""
    L = len(h)
    return np.array([(-1.0) ** k * h[L - 1 - k] for k in range(L)])


def by_taps(taps: int) -> np.ndarray:
    """Filter by length: 2 = Haar (db1), 8 = Daubechies-4, 16 = Daubechies-8."""
    if taps % 2:
        raise ValueError("even filter length expected")
    return daubechies(taps // 2)


def _laurent_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Product of two symmetric Laurent polynomials given by centred taps."""
    return np.convolve(a, b)


def cdf97():
    """(h_syn, h_ana): the CDF 9/7 low-pass pair as length-10 filters."""
    p = 4
    poly_y = [float(comb(p - 1 + k, k)) for k in range(p)]  # 1 + 4y + 10y^2 + 20y^3
    roots = np.roots(poly_y[::-1])
    real = [r for r in roots if abs(r.imag) < 1e-12]
    cplx = [r for r in roots if abs(r.imag) >= 1e-12]
    if len(real) != 1 or len(cplx) != 2:
        raise ValueError("unexpected root structure")
    c2 = np.array([0.25, 0.5, 0.25])    # cos^2(w/2) as taps of z^-1, z^0, z^1
    s2 = np.array([-0.25, 0.5, -0.25])  # sin^2(w/2)
    one = np.array([0.0, 1.0, 0.0])
    c4 = _laurent_mul(c2, c2)           # 5 taps

    def factor(y0):                      # 1 - y / y0
        return one - s2 / y0

    hs = np.sqrt(2.0) * _laurent_mul(c4, factor(real[0].real))                 # 7 taps
    qa = np.real(_laurent_mul(factor(cplx[0]), factor(cplx[1])))
    ha = np.sqrt(2.0) * _laurent_mul(c4, qa)                                   # 9 taps
    h_syn = np.zeros(10)
    h_ana = np.zeros(10)
    h_syn[1:8] = hs
    h_ana[0:9] = ha
    return h_syn, h_ana


def flen(h) -> int:
    """Filter length of an orthogonal filter or a biorthogonal pair."""
    return len(h[0]) if isinstance(h, tuple) else len(h)


def side_taps(h, side: str):
    """(low-pass, high-pass) taps of one side of a transform: 'syn' for W and
    its adjoint W^*, 'ana' for W^dagger and (W^dagger)^*. Orthogonal filters
    use h on both sides."""
    if isinstance(h, tuple):
        hs, ha = h
        return (hs, highpass(ha)) if side == "syn" else (ha, highpass(hs))
    return h, highpass(h)
