"""Deblurring objective, gradient and FISTA (oracle; test infrastructure only).

Problem (eq. 1): min_x  F(x) = 1/2 ||R W x - b||^2 + lambda ||x||_1, with
A = R W and, by the chain rule (Sec. "Motivation"), grad f(x) = W^* R^* (A x - b).

FISTA with constant step 1/L (Beck & Teboulle 2009, the solver used in
Sec. "The adjoint for orthogonal wavelets"):

    x_0 given, y_1 = x_0, t_1 = 1
    x_k     = soft(y_k - grad f(y_k) / L, lambda / L)
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
    y_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1})
    soft(v, tau) = sign(v) max(|v| - tau, 0)

The step bound L = 1 follows from ||R|| = 1 and ||W|| = 1 (a reading: the
paper leaves L unstated). The l1 norm covers every coefficient.

The gradient map is W^* R^* by default (gradient="adjoint"). gradient="pinv"
puts W^dagger in the place of W^*, the approximation the paper compares with
the true adjoint in Sec. "The adjoint for orthogonal wavelets" (identical for
zpd and per, where W^* = W^dagger).
"""
from __future__ import annotations

import numpy as np

from . import blur as bl
from . import wavelet as wv


class Problem:
    """A = R W for one image; all maps in float64."""

    def __init__(self, rows, cols, h, mode, levels, taps):
        self.rows, self.cols = rows, cols
        self.h = (tuple(np.asarray(f, dtype=np.float64) for f in h) if isinstance(h, tuple)
                  else np.asarray(h, dtype=np.float64))
        self.mode, self.levels = mode, levels
        self.taps = np.asarray(taps, dtype=np.float64)
        self.ncoef = wv.layout(rows, cols, wv.flen(h), mode, levels)[0]

    def A(self, x):
        return bl.R(wv.W(x, self.h, self.mode, self.levels, self.rows, self.cols), self.taps)

    def A_adj(self, img):
        return wv.W_adj(bl.R_adj(img, self.taps), self.h, self.mode, self.levels)

    def A_adj_pinv(self, img):
        """W^dagger R^* img: the adjoint of W replaced by its left inverse."""
        return wv.W_pinv(bl.R_adj(img, self.taps), self.h, self.mode, self.levels)


def soft(v: np.ndarray, tau: float) -> np.ndarray:
    return np.sign(v) * np.maximum(np.abs(v) - tau, 0.0)


def objective(prob: Problem, x, b, lam: float) -> float:
    r = prob.A(x) - b
    return 0.5 * float(np.sum(r * r)) + lam * float(np.sum(np.abs(x)))


def grad(prob: Problem, x, b, gradient: str = "adjoint"):
    r = prob.A(x) - b
    if gradient == "adjoint":
        return prob.A_adj(r)
    if gradient == "pinv":
        return prob.A_adj_pinv(r)
    raise ValueError(f"gradient={gradient!r}")


def t_next(t: float) -> float:
    return (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0


def momentum(k: int) -> float:
    """beta_k = (t_k - 1) / t_{k+1} with t_1 = 1 (depends on k only)."""
    t = 1.0
    for _ in range(k - 1):
        t = t_next(t)
    return (t - 1.0) / t_next(t)


def fista_step(prob: Problem, x_prev, y, b, beta: float, lam: float, L: float = 1.0,
               gradient: str = "adjoint"):
    """One iteration: x_k = soft(y_k - grad f(y_k)/L, lambda/L) and
    y_{k+1} = x_k + beta_k (x_k - x_{k-1}); returns (x_k, y_{k+1})."""
    x = soft(y - grad(prob, y, b, gradient) / L, lam / L)
    y_next = x + beta * (x - x_prev)
    return x, y_next


def fista(prob: Problem, b, lam: float, iters: int, x0=None, L: float = 1.0,
          callback=None, gradient: str = "adjoint"):
    """Plain FISTA from x0 (zero by default); returns the last x_k."""
    x = np.zeros(prob.ncoef) if x0 is None else np.array(x0, dtype=np.float64)
    y = x.copy()
    t = 1.0
    for k in range(1, iters + 1):
        t_new = t_next(t)
        x, y = fista_step(prob, x, y, b, (t - 1.0) / t_new, lam, L, gradient)
        t = t_new
        if callback is not None:
            callback(k, x)
    return x
