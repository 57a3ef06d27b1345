"""Pins for the oracle's blur R, R^*, operator A, FISTA and the convolution
adjoint pair (CPU only)."""
import numpy as np
import pytest
import scipy.fft

from oracle import blur as bl
from oracle import conv as cv
from oracle import filters as fl
from oracle import fista as fi
from oracle import wavelet as wv


def blur_matrix_1d(N, taps):
    return wv.dense(lambda x: bl.blur1(x, taps, -1), N)


def blur_adj_matrix_1d(N, taps):
    return wv.dense(lambda x: bl.blur1_adj(x, taps, -1), N)


# ---------------------------------------------------------------------- R
def test_gaussian_taps_hand_value():
    """The width convention exp(-u^2 / (2 sigma^2)): at sigma = 1, r = 1 the
    taps are (e^{-1/2}, 1, e^{-1/2}) / (1 + 2 e^{-1/2}), computed by hand.
    A slip such as exp(-u^2 / sigma^2) gives (e^{-1}, 1, e^{-1}) / (1 + 2/e)."""
    e = np.exp(-0.5)
    want = np.array([e, 1.0, e]) / (1.0 + 2.0 * e)
    np.testing.assert_allclose(bl.gaussian_taps(1.0, 1), want, rtol=0, atol=1e-16)
    # sigma = 2, r = 1: exp(-1/8) at the outer taps
    e2 = np.exp(-0.125)
    np.testing.assert_allclose(bl.gaussian_taps(2.0, 1), np.array([e2, 1.0, e2]) / (1 + 2 * e2),
                               rtol=0, atol=1e-16)


@pytest.mark.parametrize("sigma", [1.0, 1.5, 2.0, 3.0])
def test_gaussian_taps_second_moment(sigma):
    """With the support wide enough that the truncated tail is negligible
    (r = 8 sigma: tail mass below 1e-14), the taps are the integer samples of
    exp(-u^2 / (2 sigma^2)), normalised. By Poisson summation their second
    moment is sigma^2 (1 - 8 pi^2 sigma^2 q / (1 + 2 q)), q = exp(-2 pi^2 sigma^2)
    (the k = +-1 aliases; the next ones are below 1e-30): a relative 2.1e-7
    below sigma^2 at sigma = 1, negligible beyond. A sigma^2 / 2 or 2 sigma^2
    reading of the width fails by a factor of two."""
    r = int(np.ceil(8 * sigma))
    g = bl.gaussian_taps(sigma, r)
    u = np.arange(-r, r + 1)
    m2 = float(np.sum(u * u * g))
    q = np.exp(-2.0 * np.pi ** 2 * sigma ** 2)
    want = sigma ** 2 * (1.0 - 8.0 * np.pi ** 2 * sigma ** 2 * q / (1.0 + 2.0 * q))
    assert abs(m2 - want) <= 1e-13 * sigma ** 2
    assert abs(float(np.sum(u * g))) < 1e-15  # centred


@pytest.mark.parametrize("sigma,r", [(2.0, 4), (3.0, 7), (1.0, 3), (4.0, 12)])
@pytest.mark.parametrize("N", [5, 9, 16, 40])
def test_blur_symmetric_psf(sigma, r, N):
    g = bl.gaussian_taps(sigma, r)
    assert abs(g.sum() - 1.0) < 1e-15
    Rm = blur_matrix_1d(N, g)
    np.testing.assert_allclose(Rm, Rm.T, atol=1e-15)            # R = R^T
    np.testing.assert_allclose(Rm.sum(axis=1), 1.0, atol=1e-14)  # rows sum to 1
    assert abs(np.linalg.norm(Rm, 2) - 1.0) < 1e-12
    # reflexive boundaries + symmetric PSF: diagonalised by the orthonormal
    # DCT-II, eigenvalues g0 + 2 sum_u g_u cos(pi k u / N)
    C = scipy.fft.dct(np.eye(N), type=2, norm="ortho", axis=0)
    D = C @ Rm @ C.T
    k = np.arange(N)
    lam = g[r] + 2.0 * sum(g[r + u] * np.cos(np.pi * k * u / N) for u in range(1, r + 1))
    np.testing.assert_allclose(D, np.diag(lam), atol=1e-13)


@pytest.mark.parametrize("N,r", [(16, 40), (8, 30), (5, 17), (32, 100)])
def test_blur_dct_diagonalisation_any_radius(N, r):
    """The reflexive extension repeats with period 2N, so the DCT-II still
    diagonalises R when the PSF is wider than the signal (several
    reflections), with the same closed-form eigenvalues: the basis of the DCT
    route for wide PSFs."""
    g = bl.gaussian_taps(0.4 * r, r)
    Rm = blur_matrix_1d(N, g)
    C = scipy.fft.dct(np.eye(N), type=2, norm="ortho", axis=0)
    k = np.arange(N)
    lam = g[r] + 2.0 * sum(g[r + u] * np.cos(np.pi * k * u / N) for u in range(1, r + 1))
    np.testing.assert_allclose(C @ Rm @ C.T, np.diag(lam), atol=1e-13)


@pytest.mark.parametrize("N,r", [(7, 3), (12, 5), (3, 4), (20, 12)])
def test_blur_adjoint_is_transpose_any_psf(N, r):
    """Structural R^* (correlate, fold halo) equals R^T, also for a
    non-symmetric PSF where R^* != R."""
    rng = np.random.default_rng(N * 31 + r)
    taps = rng.uniform(0.0, 1.0, 2 * r + 1)
    Rm = blur_matrix_1d(N, taps)
    Ra = blur_adj_matrix_1d(N, taps)
    np.testing.assert_allclose(Ra, Rm.T, atol=1e-14)
    assert np.abs(Rm - Rm.T).max() > 1e-3


def test_blur_interior_is_plain_convolution():
    """Away from the boundary, R is the ordinary linear convolution."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal(50)
    taps = rng.uniform(0.0, 1.0, 9)
    y = bl.blur1(x, taps, -1)
    ref = np.convolve(x, taps, mode="full")[4:4 + 50]
    np.testing.assert_allclose(y[4:-4], ref[4:-4], atol=1e-14)


def test_blur_2d_is_kronecker():
    g = bl.gaussian_taps(2.0, 4)
    R, C = 6, 11
    R2 = wv.dense(lambda x: bl.R(x, g), R * C, (R, C))
    np.testing.assert_allclose(R2, np.kron(blur_matrix_1d(R, g), blur_matrix_1d(C, g)), atol=1e-15)
    Ra2 = wv.dense(lambda x: bl.R_adj(x, g), R * C, (R, C))
    np.testing.assert_allclose(Ra2, R2.T, atol=1e-15)


# ---------------------------------------------------------------------- A
@pytest.mark.parametrize("mode", ["zpd", "sym", "per", "per_ext"])
def test_A_adjoint_explicit(mode):
    R, C, L, J = 8, 12, 8, 2
    h = fl.by_taps(L)
    taps = bl.gaussian_taps(2.0, 4)
    prob = fi.Problem(R, C, h, mode, J, taps)
    Am = wv.dense(prob.A, prob.ncoef)
    Aa = wv.dense(prob.A_adj, R * C, (R, C))
    np.testing.assert_allclose(Aa, Am.T, atol=1e-13)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(prob.ncoef)
    y = rng.standard_normal((R, C))
    lhs, rhs = np.vdot(prob.A(x), y), np.vdot(x, prob.A_adj(y))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(prob.A(x)) * np.linalg.norm(y)


# ------------------------------------------------------------------ FISTA
IDENT = np.array([1.0])  # radius-0 PSF: R = I


def test_fista_orthogonal_A_closed_form():
    """A = W orthogonal (per mode, R = I): the minimiser is soft(W^T b, lambda),
    reached by the first step and kept fixed afterwards."""
    R, C = 8, 16
    h = fl.by_taps(8)
    prob = fi.Problem(R, C, h, "per", 2, IDENT)
    rng = np.random.default_rng(2)
    b = rng.standard_normal((R, C))
    lam = 0.3
    W = wv.dense(lambda x: wv.W(x, h, "per", 2, R, C), prob.ncoef)
    x_star = np.sign(W.T @ b.ravel()) * np.maximum(np.abs(W.T @ b.ravel()) - lam, 0)
    xs = []
    fi.fista(prob, b, lam, 5, callback=lambda k, x: xs.append(x.copy()))
    for x in xs:
        np.testing.assert_allclose(x, x_star, atol=1e-13)
    f0 = fi.objective(prob, x_star, b, lam)
    for _ in range(20):
        assert fi.objective(prob, x_star + 1e-3 * rng.standard_normal(prob.ncoef), b, lam) >= f0


def test_fista_lambda_zero_reconstructs_b():
    R, C = 8, 8
    prob = fi.Problem(R, C, fl.by_taps(2), "per", 3, IDENT)
    b = np.random.default_rng(4).standard_normal((R, C))
    x = fi.fista(prob, b, 0.0, 1)
    np.testing.assert_allclose(prob.A(x), b, atol=1e-13)


def test_momentum_sequence():
    """t_{k+1}^2 - t_{k+1} = t_k^2, t_k >= (k+1)/2, beta_1 = 0, beta increasing to 1."""
    t = 1.0
    betas = [fi.momentum(k) for k in range(1, 60)]
    assert betas[0] == 0.0
    assert all(b2 > b1 for b1, b2 in zip(betas, betas[1:]))
    assert betas[-1] < 1.0
    for k in range(1, 60):
        tn = fi.t_next(t)
        assert abs(tn * tn - tn - t * t) < 1e-10 * tn * tn
        assert t >= (k + 1) / 2.0 - 1e-12
        t = tn


class _Dense:
    """The same A as an explicit matrix (fast for long iteration counts)."""

    def __init__(self, prob):
        self.M = wv.dense(prob.A, prob.ncoef)
        self.shape = (prob.rows, prob.cols)
        self.ncoef = prob.ncoef

    def A(self, x):
        return (self.M @ x).reshape(self.shape)

    def A_adj(self, y):
        return self.M.T @ y.ravel()


def _small_problem():
    R, C = 8, 8
    prob = fi.Problem(R, C, fl.by_taps(2), "sym", 2, bl.gaussian_taps(0.7, 1))
    rng = np.random.default_rng(5)
    b = rng.uniform(0.0, 1.0, (R, C))
    return prob, b


def test_fista_kkt_and_rate():
    """KKT conditions of eq. 1 at convergence, and the O(1/k^2) bound
    F(x_k) - F* <= 2 L ||x_0 - x*||^2 / (k+1)^2 (Beck & Teboulle, Thm 4.4)."""
    prob, b = _small_problem()
    prob = _Dense(prob)
    lam = 1e-2
    x_star = fi.fista(prob, b, lam, 20000)
    g = fi.grad(prob, x_star, b)
    zero = np.abs(x_star) < 1e-12
    assert np.all(np.abs(g[zero]) <= lam * (1 + 1e-6))
    np.testing.assert_allclose(g[~zero], -lam * np.sign(x_star[~zero]), atol=1e-7)
    F_star = fi.objective(prob, x_star, b, lam)
    bound0 = 2.0 * np.sum(x_star ** 2)
    fs = []
    fi.fista(prob, b, lam, 200, callback=lambda k, x: fs.append((k, fi.objective(prob, x, b, lam))))
    for k, F in fs:
        assert F - F_star <= bound0 / (k + 1) ** 2 + 1e-12


def test_fista_step_matches_gradient_step():
    """One iteration from a given state equals soft(y - grad f(y), lambda)."""
    prob, b = _small_problem()
    rng = np.random.default_rng(6)
    y = rng.standard_normal(prob.ncoef)
    xp = rng.standard_normal(prob.ncoef)
    # gradient by central finite differences of f = 1/2 ||A y - b||^2
    f = lambda z: 0.5 * np.sum((prob.A(z) - b) ** 2)
    gd = np.array([(f(y + 1e-6 * e) - f(y - 1e-6 * e)) / 2e-6 for e in np.eye(prob.ncoef)[:40]])
    np.testing.assert_allclose(fi.grad(prob, y, b)[:40], gd, atol=1e-6)
    x, yn = fi.fista_step(prob, xp, y, b, fi.momentum(3), 1e-2)
    v = y - fi.grad(prob, y, b)
    np.testing.assert_allclose(x, np.sign(v) * np.maximum(np.abs(v) - 1e-2, 0), atol=1e-14)


@pytest.mark.parametrize("mode", ["zpd", "per"])
def test_pinv_gradient_equals_adjoint_without_extension(mode):
    """zpd and per involve no fold, so W^dagger = W^* and the two gradient
    maps agree."""
    rows, cols = 24, 32
    h = fl.by_taps(8)
    prob = fi.Problem(rows, cols, h, mode, 2, bl.gaussian_taps(1.5, 3))
    rng = np.random.default_rng(7)
    x = rng.standard_normal(prob.ncoef)
    b = rng.standard_normal((rows, cols))
    g = fi.grad(prob, x, b)
    np.testing.assert_allclose(fi.grad(prob, x, b, "pinv"), g, atol=1e-12 * np.abs(g).max())


@pytest.mark.parametrize("L,levels", [(2, 3), (8, 2)])
def test_pinv_gradient_is_left_inverse_of_W(L, levels):
    """With the symmetric extension W^dagger is a left inverse of W that is not
    its adjoint: W maps the pinv gradient back onto R^*(A x - b) exactly, while
    it differs from the true gradient W^* R^*(A x - b)."""
    rows, cols = 20, 28
    h = fl.by_taps(L)
    psf = bl.gaussian_taps(2.0, 4)
    prob = fi.Problem(rows, cols, h, "sym", levels, psf)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(prob.ncoef)
    b = rng.standard_normal((rows, cols))
    gp = fi.grad(prob, x, b, "pinv")
    img_grad = bl.R_adj(prob.A(x) - b, psf)
    back = wv.W(gp, h, "sym", levels, rows, cols)
    np.testing.assert_allclose(back, img_grad, atol=1e-12 * np.abs(img_grad).max())
    ga = fi.grad(prob, x, b)
    assert np.linalg.norm(gp - ga) > 1e-3 * np.linalg.norm(ga)
    # one step with either map
    xp = rng.standard_normal(prob.ncoef)
    xa, _ = fi.fista_step(prob, xp, x, b, 0.3, 1e-2)
    xq, _ = fi.fista_step(prob, xp, x, b, 0.3, 1e-2, gradient="pinv")
    v = x - gp
    np.testing.assert_allclose(xq, np.sign(v) * np.maximum(np.abs(v) - 1e-2, 0), atol=1e-14)
    assert not np.allclose(xa, xq)
    with pytest.raises(ValueError):
        fi.grad(prob, x, b, "transpose")


# --------------------------------------------------------------- conv pair
def paper_S(s, K):
    """The matrix S of x_est = S h (Sec. 'Example 2'): column j holds s shifted
    down by j."""
    N = len(s)
    S = np.zeros((K + N - 1, K))
    for j in range(K):
        S[j:j + N, j] = s
    return S


def paper_H(h, N):
    K = len(h)
    H = np.zeros((K + N - 1, N))
    for j in range(N):
        H[j:j + K, j] = h
    return H


def test_conv_pair_paper_matrices_K3_N5():
    rng = np.random.default_rng(7)
    h, s = rng.standard_normal(3), rng.standard_normal(5)
    x = rng.standard_normal(7)
    S, H = paper_S(s, 3), paper_H(h, 5)
    assert S.shape == (7, 3) and H.shape == (7, 5)
    r, gh, gs = cv.conv_adjoint_pair(h, s, x)
    np.testing.assert_allclose(r[0], S @ h - x, atol=1e-14)
    np.testing.assert_allclose(r[0], H @ s - x, atol=1e-14)
    np.testing.assert_allclose(gh[0], S.T @ r[0], atol=1e-14)   # grad_h = S^* r
    np.testing.assert_allclose(gs[0], H.T @ r[0], atol=1e-14)   # grad_s = H^* r
    # the printed S^* layout: row n holds s[0..4] starting at column n
    for n in range(3):
        np.testing.assert_array_equal(S.T[n, n:n + 5], s)


@pytest.mark.parametrize("K,N", [(3, 5), (16, 100), (128, 700), (1, 9), (9, 1)])
def test_conv_pair_matches_numpy_convolve(K, N):
    rng = np.random.default_rng(K * 1000 + N)
    h, s = rng.standard_normal(K), rng.standard_normal(N)
    x = rng.standard_normal(K + N - 1)
    r, gh, gs = cv.conv_adjoint_pair(h, s, x)
    np.testing.assert_allclose(r[0], np.convolve(h, s, "full") - x, atol=1e-12)
    np.testing.assert_allclose(gh[0], np.convolve(r[0], s[::-1], "valid"), atol=1e-11)
    np.testing.assert_allclose(gs[0], np.convolve(r[0], h[::-1], "valid"), atol=1e-11)


def test_conv_pair_finite_differences():
    rng = np.random.default_rng(11)
    K, N = 6, 17
    h, s = rng.standard_normal(K), rng.standard_normal(N)
    x = rng.standard_normal(K + N - 1)
    _, gh, gs = cv.conv_adjoint_pair(h, s, x)
    eps = 1e-6
    for i in range(K):
        e = np.zeros(K)
        e[i] = eps
        fd = (cv.objective(h + e, s, x) - cv.objective(h - e, s, x)) / (2 * eps)
        assert abs(fd - gh[0, i]) < 1e-6 * (1 + abs(fd))
    for i in range(N):
        e = np.zeros(N)
        e[i] = eps
        fd = (cv.objective(h, s + e, x) - cv.objective(h, s - e, x)) / (2 * eps)
        assert abs(fd - gs[0, i]) < 1e-6 * (1 + abs(fd))
