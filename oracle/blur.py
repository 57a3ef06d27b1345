"""Blur operator R and its adjoint R^* (oracle; test infrastructure only).

Sec. "Example 1": R is a Gaussian point spread function under symmetric
(reflexive) boundary conditions. Reading used here: the PSF is separable,
g[u] proportional to exp(-u^2 / (2 sigma^2)) for |u| <= r, normalised to sum 1,
and applied along rows and along columns. Boundaries are half-point reflexive
(x[-1-k] = x[k], x[N+k] = x[N-1-k]), repeated with period 2N when r >= N:

    (R x)[i] = sum_{u=-r}^{r} g[u] x[refl(i - u)].

The adjoint is built structurally: correlate with g over the extended domain
m in [-r, N+r) (the image is zero outside [0, N)), then fold the halo back by
summation onto the reflexive preimages:

    (R^* y)[n] = sum_{m : refl(m) = n} sum_u g[u] y[m + u].

For a symmetric PSF R^* = R (R is symmetric Toeplitz-plus-Hankel and is
diagonalised by the orthonormal DCT-II; Hansen, Nagy & O'Leary 2006).
2-D: R = R_rows (x) R_cols.
"""
from __future__ import annotations

import numpy as np


def gaussian_taps(sigma: float, radius: int) -> np.ndarray:
    """2r+1 taps, taps[u + r] = g[u], normalised to sum 1."""
    u = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-u * u / (2.0 * sigma * sigma))
    return g / g.sum()


def refl(m, N: int):
    """Half-point reflexive index with period 2N."""
    j = np.mod(m, 2 * N)
    return np.where(j < N, j, 2 * N - 1 - j)


def blur1(x: np.ndarray, taps: np.ndarray, axis: int) -> np.ndarray:
    """R along one axis."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    N = x.shape[-1]
    r = (len(taps) - 1) // 2
    i = np.arange(N)
    y = np.zeros_like(x)
    for u in range(-r, r + 1):
        y += taps[u + r] * x[..., refl(i - u, N)]
    return np.moveaxis(y, -1, axis)


def blur1_adj(y: np.ndarray, taps: np.ndarray, axis: int) -> np.ndarray:
    """R^* along one axis: correlation on the extended domain, then fold."""
    y = np.moveaxis(np.asarray(y, dtype=np.float64), axis, -1)
    N = y.shape[-1]
    r = (len(taps) - 1) // 2
    ypad = np.concatenate([np.zeros(y.shape[:-1] + (2 * r,)), y,
                           np.zeros(y.shape[:-1] + (2 * r,))], axis=-1)
    # z[m + r] = sum_u g[u] y[m + u], m in [-r, N + r)
    z = np.zeros(y.shape[:-1] + (N + 2 * r,))
    for u in range(-r, r + 1):
        z += taps[u + r] * ypad[..., r + u:r + u + N + 2 * r]
    out = np.zeros_like(y)
    for m in range(-r, N + r):
        out[..., int(refl(m, N))] += z[..., m + r]
    return np.moveaxis(out, -1, axis)


def R(x: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """2-D blur: rows (axis -2) then columns (axis -1)."""
    return blur1(blur1(x, taps, -2), taps, -1)


def R_adj(y: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """2-D adjoint blur."""
    return blur1_adj(blur1_adj(y, taps, -1), taps, -2)
