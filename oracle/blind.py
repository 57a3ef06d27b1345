"""Multi-channel blind channel estimation with a Huber total variation term
(oracle; test infrastructure only).

Sec. "Example 2": C channels h_c (length K each) observe one source s
(length N), x_c = h_c * s + noise (full linear convolution, length K+N-1).
The augmented problem (eq. 6) is

    min_{h, s}  sum_c [ f_delta(h_c, s) + lambda_h ||h_c||_1 ] + lambda_s ||s||_1,
    f_delta(h_c, s) = ||h_c * s - x_c||^2 + lambda_tv L_delta(D h_c) / delta,

with (D h)_j = h_{j+1} - h_j (K-1 entries) and the Huber function
L_delta(z) = z^2/2 for |z| <= delta, delta (|z| - delta/2) otherwise, summed
over the entries (a reading: the paper applies L_delta to the vector D h).
The smooth part's gradients:

    grad_{h_c} = 2 S^* r_c + (lambda_tv / delta) D^* clip(D h_c, -delta, delta),
    grad_s     = 2 sum_c H_c^* r_c,            r_c = h_c * s - x_c.

Solver (a reading: the paper used L1General, not available here): alternating
proximal gradient over the two blocks (h, then s; PALM), each step
x+ = soft(x - grad / L, lambda / L) with backtracking on L: L doubles until
f(x+) <= f(x) + <grad, x+ - x> + L/2 ||x+ - x||^2, and the next search starts
from L / 2. Each accepted step does not increase the objective.
"""
from __future__ import annotations

import numpy as np

from . import conv as cv


def huber(z: np.ndarray, delta: float) -> np.ndarray:
    """Elementwise L_delta(z)."""
    a = np.abs(z)
    return np.where(a <= delta, 0.5 * z * z, delta * (a - 0.5 * delta))


def huber_grad(z: np.ndarray, delta: float) -> np.ndarray:
    """L_delta'(z) = z clipped to [-delta, delta]."""
    return np.clip(z, -delta, delta)


def D(h: np.ndarray) -> np.ndarray:
    """(D h)_j = h_{j+1} - h_j along the last axis."""
    return h[..., 1:] - h[..., :-1]


def D_adj(v: np.ndarray) -> np.ndarray:
    """D^* v: (D^* v)_j = v_{j-1} - v_j with v_{-1} = v_{K-1} = 0."""
    z = np.zeros(v.shape[:-1] + (1,))
    p = np.concatenate([z, v, z], axis=-1)
    return p[..., :-1] - p[..., 1:]


def tv_huber(h: np.ndarray, delta: float) -> np.ndarray:
    """L_delta(D h) / delta per row (the softened TV seminorm)."""
    return np.sum(huber(D(h), delta), axis=-1) / delta


def smooth(h, s, x, lam_tv: float, delta: float) -> float:
    """sum_c ||h_c * s - x_c||^2 + lambda_tv sum_c L_delta(D h_c) / delta."""
    h = np.atleast_2d(h)
    r = cv.conv_full(h, np.broadcast_to(s, (h.shape[0], len(s)))) - x
    return float(np.sum(r * r)) + lam_tv * float(np.sum(tv_huber(h, delta)))


def grad_smooth(h, s, x, lam_tv: float, delta: float):
    """(grad_h [C, K], grad_s [N]) of the smooth part."""
    h = np.atleast_2d(h)
    S = np.broadcast_to(s, (h.shape[0], len(s)))
    r = cv.conv_full(h, S) - x
    gh = 2.0 * cv.grad_h(S, r, h.shape[1]) + (lam_tv / delta) * D_adj(huber_grad(D(h), delta))
    gs = 2.0 * np.sum(cv.grad_s(h, r, len(s)), axis=0)
    return gh, gs


def objective(h, s, x, p: dict) -> float:
    """The objective of eq. 6; p holds lam_h, lam_s, lam_tv, delta."""
    return (smooth(h, s, x, p["lam_tv"], p["delta"]) + p["lam_h"] * float(np.sum(np.abs(h)))
            + p["lam_s"] * float(np.sum(np.abs(s))))


def soft(v: np.ndarray, tau: float) -> np.ndarray:
    return np.sign(v) * np.maximum(np.abs(v) - tau, 0.0)


def prox_step(x, g, L: float, lam: float):
    """soft(x - g / L, lam / L)."""
    return soft(x - g / L, lam / L)


def palm(h0, s0, x, p: dict, iters: int, L0=(1.0, 1.0), max_doublings: int = 60,
         callback=None):
    """Alternating proximal gradient with backtracking; returns (h, s, L_h, L_s).
    callback(k, h, s, L_h, L_s) after every iteration."""
    h = np.array(np.atleast_2d(h0), dtype=np.float64)
    s = np.array(s0, dtype=np.float64)
    Lh, Ls = L0
    lt, dl = p["lam_tv"], p["delta"]
    for k in range(1, iters + 1):
        # h block (s fixed)
        gh, _ = grad_smooth(h, s, x, lt, dl)
        f0 = smooth(h, s, x, lt, dl)
        for _ in range(max_doublings):
            hn = prox_step(h, gh, Lh, p["lam_h"])
            d = hn - h
            if smooth(hn, s, x, lt, dl) <= f0 + float(np.sum(gh * d)) + 0.5 * Lh * float(
                    np.sum(d * d)):
                break
            Lh *= 2.0
        h = hn
        Lh *= 0.5
        # s block (h fixed)
        _, gs = grad_smooth(h, s, x, lt, dl)
        f0 = smooth(h, s, x, lt, dl)
        for _ in range(max_doublings):
            sn = prox_step(s, gs, Ls, p["lam_s"])
            d = sn - s
            if smooth(h, sn, x, lt, dl) <= f0 + float(np.sum(gs * d)) + 0.5 * Ls * float(
                    np.sum(d * d)):
                break
            Ls *= 2.0
        s = sn
        Ls *= 0.5
        if callback is not None:
            callback(k, h, s, Lh, Ls)
    return h, s, Lh, Ls
