"""Learned warm start for FISTA (test oracle, FP64; test infrastructure only).

The paper solves eq. (1) from x = 0; the learned warm start replaces that
start with a network prediction and keeps FISTA from zero as the fallback.
It is this project's extension of the deblurring experiment of Sec. "The
adjoint for orthogonal wavelets" (the paper has no network), so every choice
below is a reading, not a statement of the paper:

* network: six 3x3 convolution layers 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1,
  ReLU after the first five, zero 'same' padding, a bias per output channel.
  A layer computes the cross-correlation
      out[o, y, x] = b[o] + sum_{i, ky, kx} w[o, i, ky, kx] in[i, y + ky - 1, x + kx - 1]
  with in = 0 outside the image (the convention of CNN libraries).
* residual image u = b + CNN(b); coefficients c = W^dagger u (wavelet analysis,
  the left inverse of the synthesis W of eq. (2)); start x_0 = soft(c, lambda/L).
* training loss ||c - x*||^2 against coefficients x* from FISTA; its gradient
  with respect to u is 2 (W^dagger)^* (c - x*).
* optimiser: Adam (Kingma & Ba 2015, Algorithm 1) with bias correction.
* fallback: x_0 is rejected (FISTA starts from 0) when it is not finite or
  F(x_0) > F(0) = 1/2 ||b||^2.

Parameters are one flat vector, layer by layer, each as the weight in
(out, in, 3, 3) order followed by the bias (out,).

Parity unpinned: none (forward pinned against a library convolution and
closed forms, backward against finite differences, Adam against its
first-step closed form and a library optimiser; see tests).
"""
from __future__ import annotations

import numpy as np

from . import fista as ofi
from . import wavelet as owv

CHANNELS = 32
LAYERS = [(1, CHANNELS)] + [(CHANNELS, CHANNELS)] * 4 + [(CHANNELS, 1)]


def param_count() -> int:
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def unpack(theta: np.ndarray):
    """Flat parameter vector -> [(w (co, ci, 3, 3), b (co,)), ...]."""
    out, p = [], 0
    for ci, co in LAYERS:
        w = theta[p:p + co * ci * 9].reshape(co, ci, 3, 3)
        p += co * ci * 9
        b = theta[p:p + co]
        p += co
        out.append((w, b))
    assert p == theta.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


def conv3x3(x: np.ndarray, w: np.ndarray, b=None) -> np.ndarray:
    """x (ci, H, W) -> (co, H, W): the layer formula of the module docstring,
    one tap at a time on the zero-padded input."""
    _, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    out = np.zeros((w.shape[0], H, W))
    for ky in range(3):
        for kx in range(3):
            out += np.tensordot(w[:, :, ky, kx], xp[:, ky:ky + H, kx:kx + W], axes=(1, 0))
    if b is not None:
        out += b[:, None, None]
    return out


def conv3x3_input_grad(dout: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Transpose of conv3x3 in its input: dx[i, y, x] = sum_{o, ky, kx}
    w[o, i, ky, kx] dout[o, y - ky + 1, x - kx + 1] (dout = 0 outside)."""
    _, H, W = dout.shape
    dp = np.pad(dout, ((0, 0), (1, 1), (1, 1)))
    dx = np.zeros((w.shape[1], H, W))
    for ky in range(3):
        for kx in range(3):
            dx += np.tensordot(w[:, :, ky, kx], dp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + W],
                               axes=(0, 0))
    return dx


def conv3x3_weight_grad(x: np.ndarray, dout: np.ndarray):
    """dw[o, i, ky, kx] = sum_{y, x} dout[o, y, x] x[i, y + ky - 1, x + kx - 1];
    db[o] = sum_{y, x} dout[o, y, x]."""
    _, H, W = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    dw = np.zeros((dout.shape[0], x.shape[0], 3, 3))
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.tensordot(dout, xp[:, ky:ky + H, kx:kx + W],
                                            axes=([1, 2], [1, 2]))
    return dw, dout.sum(axis=(1, 2))


def relu(v: np.ndarray) -> np.ndarray:
    return np.maximum(v, 0.0)


def layer_forward(k: int, theta: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Layer k (0-based) on its input x (ci, H, W); ReLU on all but the last."""
    w, b = unpack(theta)[k]
    z = conv3x3(x, w, b)
    return z if k == len(LAYERS) - 1 else relu(z)


def forward(theta: np.ndarray, img: np.ndarray):
    """img (H, W) -> (activations [y_1 .. y_5], each (32, H, W); output (H, W))."""
    acts, h = [], img[None]
    for k in range(len(LAYERS)):
        h = layer_forward(k, theta, h)
        if k < len(LAYERS) - 1:
            acts.append(h)
    return acts, h[0]


def backward(theta: np.ndarray, img: np.ndarray, acts, dout: np.ndarray):
    """Gradient of <dout, CNN(img)> with respect to theta (flat), by the chain
    rule through the layers; the ReLU derivative is taken as [y > 0].
    Also returns dz_k, the gradient at the pre-activation of layers 1..5."""
    layers = unpack(theta)
    grads = [None] * len(LAYERS)
    inputs = [img[None]] + acts
    dz = dout[None]
    dzs = [None] * (len(LAYERS) - 1)
    for k in range(len(LAYERS) - 1, -1, -1):
        w, _ = layers[k]
        grads[k] = conv3x3_weight_grad(inputs[k], dz)
        if k > 0:
            dz = conv3x3_input_grad(dz, w) * (acts[k - 1] > 0)
            dzs[k - 1] = dz
    return pack(grads), dzs


def adam(theta, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); step t counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def warm_coefficients(theta, b, h, mode: str, levels: int):
    """c = W^dagger (b + CNN(b)); also returns the activations and u."""
    acts, out = forward(theta, b)
    u = b + out
    return owv.W_pinv(u, h, mode, levels), acts, u


def warm_start(theta, b, h, mode: str, levels: int, lam: float, L: float = 1.0):
    """x_0 = soft(W^dagger (b + CNN(b)), lambda / L)."""
    c, _, _ = warm_coefficients(theta, b, h, mode, levels)
    return ofi.soft(c, lam / L)


def loss_and_grad(theta, b, x_star, h, mode: str, levels: int):
    """||c - x*||^2 with c = W^dagger (b + CNN(b)), and its gradient in theta."""
    c, acts, _ = warm_coefficients(theta, b, h, mode, levels)
    r = c - x_star
    du = owv.W_pinv_adj(2.0 * r, h, mode, levels, b.shape[0], b.shape[1])
    g, _ = backward(theta, b, acts, du)
    return float(r @ r), g


def choose_start(prob, b, x0, lam: float):
    """The fallback rule: x_0 if finite with F(x_0) <= F(0), else zeros."""
    if not np.all(np.isfinite(x0)):
        return np.zeros_like(x0), False
    f0 = 0.5 * float(np.sum(b * b))
    if ofi.objective(prob, x0, b, lam) > f0:
        return np.zeros_like(x0), False
    return x0, True
