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
