"""Pins for the oracle's multi-channel blind channel estimation (eq. 6): the
Huber function's closed forms and TV limit, D^* = D^T, a hand-computed
objective, gradients by finite differences, and the solver's descent and
fixed point (CPU only)."""
import numpy as np
import pytest

from oracle import blind as bl
from oracle import conv as cv

P = {"lam_h": 0.1, "lam_s": 0.01, "lam_tv": 0.01, "delta": 0.1}


def test_huber_closed_forms_and_tv_limit():
    d = 0.1
    assert abs(bl.huber(np.array(0.05), d) - 0.00125) < 1e-15
    assert abs(bl.huber(np.array(-0.3), d) - 0.1 * (0.3 - 0.05)) < 1e-15
    # continuous with a continuous derivative at |z| = delta
    e = 1e-9
    assert abs(bl.huber(np.array(d - e), d) - bl.huber(np.array(d + e), d)) < 1e-9
    assert abs(bl.huber_grad(np.array(0.7), d) - d) < 1e-15
    assert abs(bl.huber_grad(np.array(-0.04), d) + 0.04) < 1e-15
    # when every jump exceeds delta, L_delta(Dh)/delta = ||Dh||_1 - (K-1) delta / 2
    h = np.array([0.0, 1.0, -0.5, 2.0, 2.5])
    tv = np.sum(np.abs(np.diff(h)))
    assert abs(bl.tv_huber(h, d) - (tv - 4 * d / 2)) < 1e-13
    # and tends to the TV seminorm as delta -> 0
    assert abs(bl.tv_huber(h, 1e-7) - tv) < 1e-6


def test_difference_adjoint_is_transpose():
    K = 7
    Dm = np.stack([bl.D(e) for e in np.eye(K)], axis=1)          # (K-1) x K
    Da = np.stack([bl.D_adj(e) for e in np.eye(K - 1)], axis=1)  # K x (K-1)
    np.testing.assert_array_equal(Da, Dm.T)
    assert Dm[0, 0] == -1 and Dm[0, 1] == 1


def test_objective_by_hand():
    """h = [1, 2], s = [3, -1], x = 0: h * s = [3, 5, -2], ||.||^2 = 38;
    D h = [1], L_0.1(1) / 0.1 = 0.95."""
    h = np.array([[1.0, 2.0]])
    s = np.array([3.0, -1.0])
    x = np.zeros((1, 3))
    ref = 38.0 + 0.01 * 0.95 + 0.1 * 3.0 + 0.01 * 4.0
    assert abs(bl.objective(h, s, x, P) - ref) < 1e-12


def test_gradients_by_finite_differences():
    rng = np.random.default_rng(11)
    C, K, N = 2, 6, 9
    h = rng.standard_normal((C, K)) * 0.3
    s = rng.standard_normal(N)
    x = rng.standard_normal((C, K + N - 1))
    gh, gs = bl.grad_smooth(h, s, x, 0.05, 0.1)
    f = lambda hh, ss: bl.smooth(hh, ss, x, 0.05, 0.1)  # noqa: E731
    eps = 1e-6
    for c in range(C):
        for k in range(K):
            e = np.zeros_like(h)
            e[c, k] = eps
            fd = (f(h + e, s) - f(h - e, s)) / (2 * eps)
            assert abs(fd - gh[c, k]) < 1e-6 * max(1.0, abs(fd)), (c, k)
    for n in range(N):
        e = np.zeros(N)
        e[n] = eps
        fd = (f(h, s + e) - f(h, s - e)) / (2 * eps)
        assert abs(fd - gs[n]) < 1e-6 * max(1.0, abs(fd)), n
    # the data term's gradients are the convolution adjoint pair, doubled
    r = cv.conv_full(h, np.broadcast_to(s, (C, N))) - x
    np.testing.assert_allclose(bl.grad_smooth(h, s, x, 0.0, 0.1)[1],
                               2 * cv.grad_s(h, r, N).sum(axis=0), atol=1e-12)


def _problem(seed, C=2, K=24, N=60, noise=0.0):
    rng = np.random.default_rng(seed)
    h = np.zeros((C, K))
    for c in range(C):
        for t in rng.choice(K, 3, replace=False):
            h[c, t] = rng.standard_normal()
    s = np.zeros(N)
    s[rng.choice(N, 6, replace=False)] = rng.standard_normal(6)
    x = cv.conv_full(h, np.broadcast_to(s, (C, N))) + noise * rng.standard_normal((C, K + N - 1))
    return h, s, x, rng


def test_solver_descends_and_reaches_a_fixed_point():
    h_true, s_true, x, rng = _problem(12, noise=0.005)
    h0 = rng.standard_normal(h_true.shape)
    s0 = rng.standard_normal(s_true.shape)
    Fs = []
    h, s, Lh, Ls = bl.palm(h0, s0, x, P, 400,
                           callback=lambda k, hh, ss, a, b: Fs.append(bl.objective(hh, ss, x, P)))
    F0 = bl.objective(h0, s0, x, P)
    assert Fs[0] <= F0
    assert all(b <= a * (1 + 1e-12) for a, b in zip(Fs, Fs[1:]))
    assert Fs[-1] < 0.05 * F0
    # near a fixed point of both prox-gradient maps
    gh, gs = bl.grad_smooth(h, s, x, P["lam_tv"], P["delta"])
    assert np.linalg.norm(h - bl.prox_step(h, gh, 2 * Lh, P["lam_h"])) < 1e-2 * np.linalg.norm(h)
    assert np.linalg.norm(s - bl.prox_step(s, gs, 2 * Ls, P["lam_s"])) < 1e-2 * np.linalg.norm(s)


def test_solver_noiseless_unregularised_fits_the_data():
    """lambda = 0, no noise, started near the truth: the bilinear least-squares
    residual falls by four orders of magnitude in 300 iterations (alternating
    gradient steps converge slowly along the scale ambiguity)."""
    h_true, s_true, x, rng = _problem(13)
    p = {"lam_h": 0.0, "lam_s": 0.0, "lam_tv": 0.0, "delta": 0.1}
    h0 = h_true + 0.05 * rng.standard_normal(h_true.shape)
    s0 = s_true + 0.05 * rng.standard_normal(s_true.shape)
    h, s, _, _ = bl.palm(h0, s0, x, p, 300)
    assert bl.objective(h, s, x, p) < 1e-4 * bl.objective(h0, s0, x, p)


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_prox_step_is_soft_threshold(lam):
    x = np.array([1.0, -0.2, 0.05, 0.0])
    g = np.array([0.5, 1.0, -1.0, 0.0])
    out = bl.prox_step(x, g, 2.0, lam)
    v = x - g / 2.0
    np.testing.assert_allclose(out, np.sign(v) * np.maximum(np.abs(v) - lam / 2.0, 0), atol=1e-15)
