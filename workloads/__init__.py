"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module draws random numbers and lays out test inputs. It holds none of
the method's arithmetic: no wavelet filter, no extension map, no blur, no
solver step. Blurred observations b are formed by whichever side is under test
(the oracle in tests, the GPU library in the benchmark), from the clean image
and the noise drawn here.

Workload recipe (stand-in for the resolution test chart of the deblurring
experiment, Sec. "The adjoint for orthogonal wavelets", and for the acoustic
data of the blind channel example, Sec. "Example 2"; neither data set is
available):

* ``gen_image``: background 0; 20 axis-aligned rectangles, each with sorted
  random corners and a U[0,1] intensity, painted in order (later ones overwrite
  earlier ones); plus a linear gradient gu*u + gv*v with u, v in [0,1] and
  gu, gv ~ U[-0.25, 0.25]; clipped to [0,1].
* ``gen_noise``: i.i.d. N(0, sigma^2), sigma = 1e-3 by default.
* ``gen_conv_pair``: h ~ N(0,1) of length K, s ~ N(0,1) of length N.
* ``gen_blind_problem``: multi-channel blind estimation (stand-in for the
  simulated underwater acoustic data): an impulsive source of length N (a few
  impulses of N(0,1) amplitude at sorted random positions), C sparse multipath
  channels of length K (arrivals at random delays, amplitudes N(0,1) decaying
  with delay, each followed by a short geometric tail), N(0, sigma^2) noise
  for each channel output (length K+N-1), and N(0,1) starting guesses of the
  estimated lengths K_est, N_est (K_est + N_est = K + N).
* ``gen_batched_config``: the uneven batch (image sides drawn from
  {512, 768, ..., 4096} independently per axis, levels from {3,4,5}, filters
  from {Haar, Daubechies-4, Daubechies-8}, PSF sigma ~ U[1,4], radius
  ceil(3 sigma)).
"""
from __future__ import annotations

import math

import numpy as np


def rng_for(config_id: int, index: int) -> np.random.Generator:
    """One independent stream per (workload id, item index)."""
    return np.random.default_rng((int(config_id), int(index)))


def gen_image(rng: np.random.Generator, rows: int, cols: int, n_rect: int = 20) -> np.ndarray:
    """Piecewise-constant rectangles plus a linear gradient, float64 in [0,1]."""
    img = np.zeros((rows, cols), dtype=np.float64)
    for _ in range(n_rect):
        c0, c1 = np.sort(rng.integers(0, cols, 2))
        r0, r1 = np.sort(rng.integers(0, rows, 2))
        img[r0:r1 + 1, c0:c1 + 1] = rng.uniform(0.0, 1.0)
    gu, gv = rng.uniform(-0.25, 0.25, 2)
    u = np.linspace(0.0, 1.0, rows)[:, None]
    v = np.linspace(0.0, 1.0, cols)[None, :]
    img = img + gu * u + gv * v
    return np.clip(img, 0.0, 1.0)


def gen_noise(rng: np.random.Generator, shape, sigma: float = 1e-3) -> np.ndarray:
    return rng.normal(0.0, sigma, size=shape)


def gen_conv_pair(rng: np.random.Generator, K: int, N: int):
    """Channel h (length K) and source s (length N), both N(0,1) float64."""
    h = rng.standard_normal(K)
    s = rng.standard_normal(N)
    return h, s


def gen_coefficients(rng: np.random.Generator, n: int, density: float = 1.0) -> np.ndarray:
    """Random coefficient vector (for operator parity); optional sparsity."""
    x = rng.standard_normal(n)
    if density < 1.0:
        x = x * (rng.uniform(0.0, 1.0, n) < density)
    return x


def gen_batched_config(rng: np.random.Generator, n_images: int = 64):
    """Per-image (rows, cols, levels, taps, sigma, radius) for the uneven batch."""
    sides = np.arange(512, 4096 + 1, 256)
    out = []
    for _ in range(n_images):
        rows = int(rng.choice(sides))
        cols = int(rng.choice(sides))
        levels = int(rng.choice([3, 4, 5]))
        taps = int(rng.choice([2, 8, 16]))
        sigma = float(rng.uniform(1.0, 4.0))
        radius = int(math.ceil(3.0 * sigma))
        out.append(dict(rows=rows, cols=cols, levels=levels, taps=taps,
                        sigma=sigma, radius=radius))
    return out


def gen_warm_problem(rng: np.random.Generator):
    """PSF (sigma, radius) of one warm-start training or evaluation image:
    sigma ~ U[1, 3], radius ceil(3 sigma)."""
    sigma = float(rng.uniform(1.0, 3.0))
    return sigma, int(math.ceil(3.0 * sigma))


def gen_cnn_init(rng: np.random.Generator, layers, out_scale: float = 0.1) -> np.ndarray:
    """Initial CNN parameters, flat, layer by layer as (weight (co, ci, 3, 3),
    bias (co,)): weights N(0, 2 / (9 ci)) (He et al. 2015), biases 0, the last
    layer's weights further scaled by ``out_scale`` so the network starts near 0."""
    parts = []
    for k, (ci, co) in enumerate(layers):
        w = rng.normal(0.0, math.sqrt(2.0 / (9.0 * ci)), size=co * ci * 9)
        if k == len(layers) - 1:
            w = w * out_scale
        parts.append(w)
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def gen_blind_problem(rng: np.random.Generator, C: int = 2, K: int = 894, N: int = 1717,
                      K_est: int | None = None, N_est: int | None = None,
                      sigma: float = 0.005, n_arrivals: int = 6, n_impulses: int = 5):
    """(h_true [C, K], s_true [N], noise [C, K+N-1], h0 [C, K_est], s0 [N_est])."""
    K_est = K if K_est is None else K_est
    N_est = N if N_est is None else N_est
    if K_est + N_est != K + N:
        raise ValueError("K_est + N_est must equal K + N (observed length K+N-1)")
    s = np.zeros(N)
    pos = np.sort(rng.choice(N, n_impulses, replace=False))
    s[pos] = rng.standard_normal(n_impulses)
    h = np.zeros((C, K))
    for c in range(C):
        delays = np.sort(rng.choice(K, n_arrivals, replace=False))
        for d in delays:
            amp = rng.standard_normal() * math.exp(-2.0 * d / K)
            for t in range(8):
                if d + t < K:
                    h[c, d + t] += amp * 0.6 ** t
    noise = sigma * rng.standard_normal((C, K + N - 1))
    h0 = rng.standard_normal((C, K_est))
    s0 = rng.standard_normal(N_est)
    return h, s, noise, h0, s0
