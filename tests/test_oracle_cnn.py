"""Pins of the warm-start oracle (oracle/cnn.py) against things other than
itself: a library convolution, closed forms of special kernels, brute force
over basis weights, finite differences, Adam's first-step closed form and a
library optimiser, and the perfect reconstruction of periodic wavelets."""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from oracle import cnn
from oracle import filters as ofl
from oracle import fista as ofi
from oracle import wavelet as owv
from workloads import gen_cnn_init, gen_image, rng_for

SEED = 11


def rng(i=0):
    return rng_for(SEED, i)


def test_param_count():
    # 9*32 + 32, four times 9*32*32 + 32, 9*32 + 1
    assert cnn.param_count() == 320 + 4 * 9248 + 289 == 37601
    th = gen_cnn_init(rng(), cnn.LAYERS)
    assert th.size == cnn.param_count()
    np.testing.assert_array_equal(cnn.pack(cnn.unpack(th)), th)


@pytest.mark.parametrize("ci,co,H,W", [(1, 4, 7, 9), (3, 5, 6, 6), (32, 32, 5, 8), (32, 1, 4, 3)])
def test_conv_matches_library(ci, co, H, W):
    r = rng(1)
    x = r.standard_normal((ci, H, W))
    w = r.standard_normal((co, ci, 3, 3))
    b = r.standard_normal(co)
    ref = torch.nn.functional.conv2d(torch.tensor(x)[None], torch.tensor(w), torch.tensor(b),
                                     padding=1)[0].numpy()
    np.testing.assert_allclose(cnn.conv3x3(x, w, b), ref, rtol=1e-12, atol=1e-12)


def test_conv_closed_forms():
    x = rng(2).standard_normal((1, 6, 7))
    delta = np.zeros((1, 1, 3, 3))
    delta[0, 0, 1, 1] = 1.0
    np.testing.assert_array_equal(cnn.conv3x3(x, delta), x)
    # tap (ky, kx) = (0, 1) reads the row above: a shift down with zero fill
    up = np.zeros((1, 1, 3, 3))
    up[0, 0, 0, 1] = 1.0
    out = cnn.conv3x3(x, up)
    np.testing.assert_array_equal(out[0, 1:], x[0, :-1])
    np.testing.assert_array_equal(out[0, 0], 0.0)
    # all-ones kernel on a constant image counts the in-image neighbours
    c = np.full((1, 5, 6), 2.5)
    out = cnn.conv3x3(c, np.ones((1, 1, 3, 3)))[0]
    assert out[2, 2] == 9 * 2.5 and out[0, 2] == 6 * 2.5 and out[2, 0] == 6 * 2.5
    assert out[0, 0] == 4 * 2.5 and out[4, 5] == 4 * 2.5


def test_input_grad_is_adjoint_and_matches_library():
    r = rng(3)
    x = r.standard_normal((4, 6, 5))
    d = r.standard_normal((3, 6, 5))
    w = r.standard_normal((3, 4, 3, 3))
    lhs = float(np.sum(cnn.conv3x3(x, w) * d))
    rhs = float(np.sum(x * cnn.conv3x3_input_grad(d, w)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-12
    ref = torch.nn.functional.conv_transpose2d(torch.tensor(d)[None], torch.tensor(w),
                                               padding=1)[0].numpy()
    np.testing.assert_allclose(cnn.conv3x3_input_grad(d, w), ref, rtol=1e-12, atol=1e-12)


def test_weight_grad_by_basis_brute_force():
    r = rng(4)
    x = r.standard_normal((2, 5, 4))
    d = r.standard_normal((3, 5, 4))
    dw, db = cnn.conv3x3_weight_grad(x, d)
    for o in range(3):
        for i in range(2):
            for ky in range(3):
                for kx in range(3):
                    e = np.zeros((3, 2, 3, 3))
                    e[o, i, ky, kx] = 1.0
                    assert abs(np.sum(cnn.conv3x3(x, e) * d) - dw[o, i, ky, kx]) < 1e-12
        eb = np.zeros(3)
        eb[o] = 1.0
        assert abs(np.sum(cnn.conv3x3(x, np.zeros((3, 2, 3, 3)), eb) * d) - db[o]) < 1e-12


def _directional_fd(f, theta, g, r, n_dirs=4, eps=1e-6):
    for _ in range(n_dirs):
        dirn = r.standard_normal(theta.size)
        dirn /= np.linalg.norm(dirn)
        fd = (f(theta + eps * dirn) - f(theta - eps * dirn)) / (2 * eps)
        an = float(g @ dirn)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_backward_finite_differences():
    r = rng(5)
    theta = gen_cnn_init(r, cnn.LAYERS, out_scale=1.0)
    img = r.uniform(0.0, 1.0, (7, 9))
    dout = r.standard_normal((7, 9))
    acts, _ = cnn.forward(theta, img)
    g, dzs = cnn.backward(theta, img, acts, dout)

    def f(th):
        return float(np.sum(cnn.forward(th, img)[1] * dout))

    _directional_fd(f, theta, g, r)
    # per-coordinate brute force on a few biases and weights of each layer
    offs = np.cumsum([0] + [co * ci * 9 + co for ci, co in cnn.LAYERS])
    for k in range(len(cnn.LAYERS)):
        for j in (offs[k], offs[k + 1] - 1):
            e = np.zeros_like(theta)
            e[j] = 1e-6
            fd = (f(theta + e) - f(theta - e)) / 2e-6
            assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])), (k, j)
    # dz of layer 5 is the masked input gradient of the last layer
    w6, _ = cnn.unpack(theta)[5]
    np.testing.assert_allclose(dzs[4], cnn.conv3x3_input_grad(dout[None], w6) * (acts[4] > 0))


def test_adam_first_step_and_library():
    r = rng(6)
    th = r.standard_normal(50)
    g = r.standard_normal(50)
    th1, m, v = cnn.adam(th, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    # m_hat = g, v_hat = g^2 at t = 1
    np.testing.assert_allclose(th1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=1e-15)
    p = torch.nn.Parameter(torch.tensor(th))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    ours, m, v = th.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        gt = r.standard_normal(50)
        p.grad = torch.tensor(gt)
        opt.step()
        ours, m, v = cnn.adam(ours, m, v, gt, t, lr=1e-3)
    np.testing.assert_allclose(ours, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def _problem(rows=16, cols=16, mode="sym", J=2, taps=8, sigma=1.5):
    h = ofl.by_taps(taps)
    psf = obl.gaussian_taps(sigma, int(np.ceil(3 * sigma)))
    return ofi.Problem(rows, cols, h, mode, J, psf), h


def test_loss_gradient_finite_differences():
    r = rng(7)
    prob, h = _problem()
    img = gen_image(r, 16, 16)
    b = obl.R(img, prob.taps)
    x_star = r.standard_normal(prob.ncoef) * 0.1
    theta = gen_cnn_init(r, cnn.LAYERS, out_scale=1.0)
    loss, g = cnn.loss_and_grad(theta, b, x_star, h, "sym", 2)

    def f(th):
        return cnn.loss_and_grad(th, b, x_star, h, "sym", 2)[0]

    assert abs(f(theta) - loss) == 0.0
    _directional_fd(f, theta, g, r)


def test_warm_start_reduces_to_analysis_and_reconstructs():
    r = rng(8)
    prob, h = _problem(16, 16, "per", 2, 8)
    b = r.uniform(0.0, 1.0, (16, 16))
    theta = gen_cnn_init(r, cnn.LAYERS)
    layers = cnn.unpack(theta)
    layers[5] = (np.zeros_like(layers[5][0]), np.zeros(1))
    th0 = cnn.pack(layers)
    # a silent network leaves u = b; periodic orthogonal analysis is inverted by W
    x0 = cnn.warm_start(th0, b, h, "per", 2, lam=0.0)
    np.testing.assert_allclose(owv.W(x0, h, "per", 2, 16, 16), b, atol=1e-12)
    tau = 0.05
    np.testing.assert_allclose(cnn.warm_start(th0, b, h, "per", 2, lam=tau),
                               ofi.soft(x0, tau), atol=0)
    # a bias-only last layer adds a constant image before the analysis
    layers[5] = (np.zeros_like(layers[5][0]), np.array([0.25]))
    x1 = cnn.warm_start(cnn.pack(layers), b, h, "per", 2, lam=0.0)
    np.testing.assert_allclose(owv.W(x1, h, "per", 2, 16, 16), b + 0.25, atol=1e-12)


def test_fallback_rule():
    r = rng(9)
    prob, h = _problem()
    b = obl.R(gen_image(r, 16, 16), prob.taps)
    lam = 2e-5
    z = np.zeros(prob.ncoef)
    x, ok = cnn.choose_start(prob, b, z, lam)
    assert ok and np.array_equal(x, z)          # F(0) <= F(0)
    bad = np.full(prob.ncoef, np.nan)
    x, ok = cnn.choose_start(prob, b, bad, lam)
    assert not ok and np.array_equal(x, z)
    huge = np.full(prob.ncoef, 100.0)
    x, ok = cnn.choose_start(prob, b, huge, lam)
    assert not ok and np.array_equal(x, z)
    good = owv.W_pinv(b, h, "sym", 2)              # reproduces b up to the blur
    x, ok = cnn.choose_start(prob, b, good, lam)
    assert ok and np.array_equal(x, good)
