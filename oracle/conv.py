"""Blind-channel convolution and its adjoints (oracle; test infrastructure only).

Sec. "Example 2": x_est = h * s is the full linear convolution (zero boundary)
of a channel h (length K) and a source s (length N), length K+N-1. With the
residual r = x_est - x and f(h, s) = 1/2 ||h * s - x||^2 (eq. 5),

    grad_h f[n] = sum_{k<N} s[k] r[k+n],   n < K   (S^* r, a cross-correlation)
    grad_s f[n] = sum_{k<K} h[k] r[k+n],   n < N   (H^* r)

Real data, so conjugation is the identity. Written as the explicit sums of
the two matrix-vector forms S h and H s, vectorised over a leading batch axis.
"""
from __future__ import annotations

import numpy as np


def conv_full(h: np.ndarray, s: np.ndarray) -> np.ndarray:
    """(h * s)[t] = sum_k h[k] s[t-k], t < K+N-1 (batched over axis 0 if 2-D)."""
    h = np.atleast_2d(np.asarray(h, dtype=np.float64))
    s = np.atleast_2d(np.asarray(s, dtype=np.float64))
    K, N = h.shape[1], s.shape[1]
    y = np.zeros((h.shape[0], K + N - 1))
    for k in range(K):
        y[:, k:k + N] += h[:, k:k + 1] * s
    return y


def grad_h(s: np.ndarray, r: np.ndarray, K: int) -> np.ndarray:
    """S^* r: g[n] = sum_{k<N} s[k] r[k+n]."""
    s = np.atleast_2d(np.asarray(s, dtype=np.float64))
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    N = s.shape[1]
    return np.stack([np.sum(s * r[:, n:n + N], axis=1) for n in range(K)], axis=1)


def grad_s(h: np.ndarray, r: np.ndarray, N: int) -> np.ndarray:
    """H^* r: g[n] = sum_{k<K} h[k] r[k+n]."""
    h = np.atleast_2d(np.asarray(h, dtype=np.float64))
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    K = h.shape[1]
    g = np.zeros((h.shape[0], N))
    for k in range(K):
        g += h[:, k:k + 1] * r[:, k:k + N]
    return g


def conv_adjoint_pair(h, s, x_obs):
    """(resid, grad_h, grad_s) for f(h, s) = 1/2 ||h * s - x_obs||^2."""
    h = np.atleast_2d(np.asarray(h, dtype=np.float64))
    s = np.atleast_2d(np.asarray(s, dtype=np.float64))
    r = conv_full(h, s)
    if x_obs is not None:
        r = r - np.atleast_2d(np.asarray(x_obs, dtype=np.float64))
    return r, grad_h(s, r, h.shape[1]), grad_s(h, r, s.shape[1])


def objective(h, s, x_obs) -> float:
    r = conv_full(h, s) - np.atleast_2d(x_obs)
    return 0.5 * float(np.sum(r * r))
