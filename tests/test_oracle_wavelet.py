"""Pins for the oracle's wavelet maps W, W^dagger, W^* (CPU only).

Independent checks: hand-derived Haar closed forms, the library
pseudoinverse, isometry and perfect-reconstruction identities, explicit
Kronecker products of 1-D matrices, and the boundary-support statement of
Sec. "The adjoint for orthogonal wavelets" (W^* and W^dagger differ only
through E vs (E^dagger)^*).
"""
import itertools

import numpy as np
import pytest

from oracle import extension as ext
from oracle import filters as fl
from oracle import wavelet as wv

S2 = np.sqrt(2.0)


def mat1d_ana(N, L, mode, weights):
    h = fl.by_taps(L)

    def f(y):
        lo, hi = wv.ana1(y, h, mode, axis=-1, weights=weights)
        return np.concatenate([lo, hi], axis=-1)
    return wv.dense(f, N)


def mat1d_syn(N, L, mode, weights):
    h = fl.by_taps(L)
    K = wv.coef_len(N, L, mode)
    return wv.dense(lambda c: wv.syn1(c[..., :K], c[..., K:], h, mode, N, axis=-1, weights=weights),
                    2 * K)


# ---------------------------------------------------------- Haar closed forms
def test_haar_sym_closed_forms():
    """N = 6, y = 1..6, half-point symmetric extension by L' = 1."""
    y = np.arange(1.0, 7.0)
    h = fl.by_taps(2)
    lo, hi = wv.ana1(y, h, "sym", -1, "ones")          # W^dagger
    np.testing.assert_allclose(lo, [S2 * 1, (2 + 3) / S2, (4 + 5) / S2, S2 * 6], atol=1e-14)
    np.testing.assert_allclose(hi, [0, (2 - 3) / S2, (4 - 5) / S2, 0], atol=1e-14)
    lo, hi = wv.ana1(y, h, "sym", -1, "pinv")          # W^*: edge samples halved
    np.testing.assert_allclose(lo, [1 / S2, (2 + 3) / S2, (4 + 5) / S2, 6 / S2], atol=1e-14)
    np.testing.assert_allclose(hi, [0, (2 - 3) / S2, (4 - 5) / S2, 0], atol=1e-14)


def test_haar_per_closed_form():
    y = np.array([3.0, -1.0, 4.0, 1.0, -5.0, 9.0])
    lo, hi = wv.ana1(y, fl.by_taps(2), "per", -1, "ones")
    np.testing.assert_allclose(lo, (y[0::2] + y[1::2]) / S2, atol=1e-14)
    np.testing.assert_allclose(hi, (y[0::2] - y[1::2]) / S2, atol=1e-14)


def test_haar_zpd_closed_form():
    """Zero boundary, odd phase, N = 5: pairs (y0,y1), (y2,y3), (y4, 0)."""
    y = np.array([2.0, 7.0, 1.0, 8.0, 3.0])
    lo, hi = wv.ana1(y, fl.by_taps(2), "zpd", -1, "ones")
    np.testing.assert_allclose(lo, [(2 + 7) / S2, (1 + 8) / S2, 3 / S2], atol=1e-14)
    np.testing.assert_allclose(hi, [(2 - 7) / S2, (1 - 8) / S2, 3 / S2], atol=1e-14)


def test_haar_2d_subband_orientation():
    """2x2 image, per mode, one level: fixes which band is H, V, D."""
    a_, b_, c_, d_ = 1.0, 2.0, 5.0, 11.0
    img = np.array([[a_, b_], [c_, d_]])
    x = wv.W_pinv(img, fl.by_taps(2), "per", 1)
    np.testing.assert_allclose(x, [(a_ + b_ + c_ + d_) / 2,      # a: lo rows, lo cols
                                   (a_ + b_ - c_ - d_) / 2,      # H: hi along rows
                                   (a_ - b_ + c_ - d_) / 2,      # V: hi along columns
                                   (a_ - b_ - c_ + d_) / 2], atol=1e-14)


# ------------------------------------------------------------ one level, 1-D
@pytest.mark.parametrize("L", [2, 8, 16])
@pytest.mark.parametrize("M", [1, 2, 5, 16, 33])
def test_phi_is_isometry(L, M):
    """Phi^* Phi = I_M: W^*_zpd = W^dagger_zpd for orthogonal wavelets."""
    h = fl.by_taps(L)
    g = fl.highpass(h)
    Phi = np.vstack([wv.dense(lambda u: wv.phi(u, h), M), wv.dense(lambda u: wv.phi(u, g), M)])
    np.testing.assert_allclose(Phi.T @ Phi, np.eye(M), atol=1e-13)
    # the adjoint routine is the transpose
    K = (M + L - 1) // 2
    Pa = wv.dense(lambda c: wv.phi_adj(c[..., :K], h, M) + wv.phi_adj(c[..., K:], g, M), 2 * K)
    np.testing.assert_allclose(Pa, Phi.T, atol=1e-15)


@pytest.mark.parametrize("mode", ["zpd", "sym", "per_ext", "per"])
@pytest.mark.parametrize("L", [2, 8, 16])
@pytest.mark.parametrize("N", [2, 6, 10, 18, 40])
def test_one_level_1d(mode, L, N):
    Wd = mat1d_ana(N, L, mode, "ones")     # W^dagger
    Ws = mat1d_ana(N, L, mode, "pinv")     # W^*
    Wm = mat1d_syn(N, L, mode, "pinv")     # W
    np.testing.assert_allclose(Wm, np.linalg.pinv(Wd), atol=1e-12)   # W = pinv(W^dagger)
    np.testing.assert_allclose(Wm @ Wd, np.eye(N), atol=1e-12)       # perfect reconstruction
    np.testing.assert_allclose(Ws, Wm.T, atol=1e-14)                 # W^* = W^T
    if mode == "per" or N > 2 * (L - 1):
        assert abs(np.linalg.norm(Wm, 2) - 1.0) < 1e-12
    if mode in ("per", "zpd"):
        np.testing.assert_allclose(Ws, Wd, atol=1e-14)               # no extension: W^* = W^dagger
    if mode == "per":
        np.testing.assert_allclose(Wm.T @ Wm, np.eye(N), atol=1e-12)


@pytest.mark.parametrize("mode", ["sym", "per_ext"])
@pytest.mark.parametrize("L", [2, 8])
def test_adjoint_vs_pinv_differ_only_at_boundary(mode, L):
    """W^* - W^dagger = Phi (E diag(1/mult) - E): only coefficients whose
    support touches an extended sample that copies a multiply-used sample can
    differ."""
    N = 30
    Wd = mat1d_ana(N, L, mode, "ones")
    Ws = mat1d_ana(N, L, mode, "pinv")
    diff_rows = np.where(np.abs(Ws - Wd).max(axis=1) > 1e-14)[0]
    e = L - 1
    mult = ext.multiplicity(N, e, mode)
    src = ext.src_map(N, e, mode)
    K = wv.coef_len(N, L, mode)
    touched = set()
    for band in range(2):
        for k in range(K):
            # Phi row k reads extended positions n = 2k + j - L + 2, j < L
            ns = [2 * k + j - L + 2 for j in range(L)]
            if any(0 <= n < N + 2 * e and mult[src[n]] > 1 for n in ns):
                touched.add(band * K + k)
    assert set(diff_rows.tolist()) <= touched
    assert len(diff_rows) > 0
    assert len(touched) < 2 * K  # interior coefficients agree exactly


# ---------------------------------------------------------- 2-D, multi-level
def _kron_level(R, C, L, mode, weights_syn):
    """One 2-D synthesis level as Kronecker products of 1-D matrices, in the
    band order (a, H, V, D) and row-major pixel order."""
    Sr = mat1d_syn(R, L, mode, weights_syn)
    Sc = mat1d_syn(C, L, mode, weights_syn)
    Kr, Kc = Sr.shape[1] // 2, Sc.shape[1] // 2
    lo_r, hi_r = Sr[:, :Kr], Sr[:, Kr:]
    lo_c, hi_c = Sc[:, :Kc], Sc[:, Kc:]
    return np.hstack([np.kron(lo_r, lo_c), np.kron(hi_r, lo_c),
                      np.kron(lo_r, hi_c), np.kron(hi_r, hi_c)])


@pytest.mark.parametrize("mode", ["zpd", "sym", "per", "per_ext"])
@pytest.mark.parametrize("L", [2, 8])
def test_2d_single_level_is_kronecker(mode, L):
    R, C = (6, 10)
    h = fl.by_taps(L)
    n = wv.layout(R, C, L, mode, 1)[0]
    W2 = wv.dense(lambda x: wv.W(x, h, mode, 1, R, C), n)
    np.testing.assert_allclose(W2, _kron_level(R, C, L, mode, "pinv"), atol=1e-13)


CASES = [(m, L, J, R, C) for m, L, J, (R, C) in itertools.product(
    ["zpd", "sym", "per", "per_ext"], [2, 8], [1, 2, 3], [(8, 16), (12, 20), (6, 10)])
    if not (m == "per" and (R % 2 ** J or C % 2 ** J))]


@pytest.mark.parametrize("mode,L,J,R,C", CASES)
def test_multilevel_identities(mode, L, J, R, C):
    h = fl.by_taps(L)
    n = wv.layout(R, C, L, mode, J)[0]
    Wm = wv.dense(lambda x: wv.W(x, h, mode, J, R, C), n)
    Wa = wv.dense(lambda y: wv.W_adj(y, h, mode, J), R * C, (R, C))
    Wp = wv.dense(lambda y: wv.W_pinv(y, h, mode, J), R * C, (R, C))
    Wpa = wv.dense(lambda x: wv.W_pinv_adj(x, h, mode, J, R, C), n)
    np.testing.assert_allclose(Wa, Wm.T, atol=1e-13)        # W^* = W^T
    np.testing.assert_allclose(Wpa, Wp.T, atol=1e-13)       # (W^dagger)^* = (W^dagger)^T
    np.testing.assert_allclose(Wm @ Wp, np.eye(R * C), atol=1e-12)
    if mode in ("zpd", "per"):
        np.testing.assert_allclose(Wm, np.linalg.pinv(Wp), atol=1e-11)
    if mode == "per":
        np.testing.assert_allclose(Wm.T @ Wm, np.eye(n), atol=1e-12)
        np.testing.assert_allclose(Wm @ Wm.T, np.eye(R * C), atol=1e-12)


def test_multilevel_composition_matches_explicit_product():
    """W = W_1 (W_2 (+) I): build level matrices separately and multiply."""
    R, C, L, mode = 12, 20, 8, "sym"
    h = fl.by_taps(L)
    n, sr, sc = wv.layout(R, C, L, mode, 2)
    W2full = wv.dense(lambda x: wv.W(x, h, mode, 2, R, C), n)
    L1 = _kron_level(R, C, L, mode, "pinv")                 # (R*C) x 4 K1r K1c
    L2 = _kron_level(sr[1], sc[1], L, mode, "pinv")         # (K1r K1c) x 4 K2r K2c
    n2 = L2.shape[1]
    blockdiag = np.zeros((4 * sr[1] * sc[1], n))
    blockdiag[:sr[1] * sc[1], :n2] = L2
    blockdiag[sr[1] * sc[1]:, n2:] = np.eye(3 * sr[1] * sc[1])
    np.testing.assert_allclose(W2full, L1 @ blockdiag, atol=1e-13)


def test_layout_sizes():
    """Coefficient counts: K = floor((N + 2e + L - 1)/2), per: N/2."""
    assert wv.level_sizes(2048, 8, "sym", 4) == [2048, 1034, 527, 274, 147]
    assert wv.level_sizes(2048, 8, "zpd", 4) == [2048, 1027, 517, 262, 134]
    assert wv.level_sizes(2048, 8, "per", 4) == [2048, 1024, 512, 256, 128]
    assert wv.layout(2048, 2048, 8, "sym", 4)[0] == 4352319
    assert wv.layout(256, 256, 8, "sym", 3)[0] == 85855
    assert wv.layout(32, 32, 8, "sym", 4)[0] == 6831
    with pytest.raises(ValueError):
        wv.level_sizes(12, 8, "per", 3)


# ------------------------------------------------ biorthogonal CDF 9/7 (eq. 4)
def test_cdf97_filters():
    """Symmetric 7- and 9-tap low-pass filters centred on the same index, each
    summing to sqrt(2), biorthogonal under even shifts, four vanishing moments
    on both high-pass filters, and the product filter of the construction
    (H_a conj H_s = 2 cos^8 P at sampled frequencies)."""
    hs, ha = fl.cdf97()
    assert np.count_nonzero(np.abs(hs) > 1e-15) == 7
    assert np.count_nonzero(np.abs(ha) > 1e-15) == 9
    np.testing.assert_allclose(hs[1:8], hs[1:8][::-1], atol=1e-15)
    np.testing.assert_allclose(ha[0:9], ha[0:9][::-1], atol=1e-15)
    assert abs(hs.sum() - S2) < 1e-14 and abs(ha.sum() - S2) < 1e-14
    for m in range(-4, 5):  # linear cross-correlation at even lags
        r = sum(hs[k] * ha[k + 2 * m] for k in range(10) if 0 <= k + 2 * m < 10)
        assert abs(r - (1.0 if m == 0 else 0.0)) < 1e-14, (m, r)
    k = np.arange(10)
    for g in (fl.highpass(ha), fl.highpass(hs)):
        for p in range(4):
            assert abs(np.sum(g * k ** p)) < 1e-9 * max(1, 10 ** p), p
    w = np.linspace(0, np.pi, 17)
    z = np.exp(-1j * np.outer(w, k - 4))
    Hs, Ha = z @ hs, z @ ha
    y = np.sin(w / 2) ** 2
    P = 1 + 4 * y + 10 * y ** 2 + 20 * y ** 3
    np.testing.assert_allclose(Ha * np.conj(Hs), 2 * np.cos(w / 2) ** 8 * P, atol=1e-13)


def _mats_bior(N, mode):
    h = fl.cdf97()
    K = wv.coef_len(N, 10, mode)

    def ana(weights):
        return wv.dense(lambda y: np.concatenate(wv.ana1(y, h, mode, -1, weights), axis=-1), N)

    def syn(weights):
        return wv.dense(lambda c: wv.syn1(c[..., :K], c[..., K:], h, mode, N, -1, weights), 2 * K)
    return ana("ones"), ana("pinv"), syn("pinv"), syn("ones")


@pytest.mark.parametrize("mode", ["zpd", "sym", "per_ext", "per"])
@pytest.mark.parametrize("N", [10, 18, 40])
def test_cdf97_one_level(mode, N):
    """One level: W W^dagger = I (perfect reconstruction), W^* = W^T,
    (W^dagger)^* = (W^dagger)^T, and, unlike the orthogonal case, W^*_zpd !=
    W^dagger_zpd: the adjoint analyses with the synthesis (dual) filters."""
    Wd, Ws, Wm, Wda = _mats_bior(N, mode)
    np.testing.assert_allclose(Wm @ Wd, np.eye(N), atol=1e-12)
    np.testing.assert_allclose(Ws, Wm.T, atol=1e-14)
    np.testing.assert_allclose(Wda, Wd.T, atol=1e-14)
    assert np.abs(Ws - Wd).max() > 1e-2
    if mode == "zpd":
        # eq. 4 with E = I: W^*_zpd is the analysis W~^dagger_zpd of the dual
        # transform, i.e. the primal analysis with the two sides swapped
        hs, ha = fl.cdf97()
        K = wv.coef_len(N, 10, mode)
        dual = wv.dense(lambda y: np.concatenate(wv.ana1(y, (ha, hs), mode, -1, "ones"),
                                                 axis=-1), N)
        np.testing.assert_allclose(Ws, dual, atol=1e-14)
        assert K == (N + 9) // 2


@pytest.mark.parametrize("mode,J,R,C", [("sym", 2, 12, 20), ("zpd", 2, 10, 14),
                                        ("per", 2, 8, 16), ("per_ext", 1, 12, 10),
                                        ("sym", 3, 10, 6)])
def test_cdf97_multilevel(mode, J, R, C):
    h = fl.cdf97()
    n = wv.layout(R, C, 10, mode, J)[0]
    Wm = wv.dense(lambda x: wv.W(x, h, mode, J, R, C), n)
    Wa = wv.dense(lambda y: wv.W_adj(y, h, mode, J), R * C, (R, C))
    Wp = wv.dense(lambda y: wv.W_pinv(y, h, mode, J), R * C, (R, C))
    Wpa = wv.dense(lambda x: wv.W_pinv_adj(x, h, mode, J, R, C), n)
    np.testing.assert_allclose(Wa, Wm.T, atol=1e-13)
    np.testing.assert_allclose(Wpa, Wp.T, atol=1e-13)
    np.testing.assert_allclose(Wm @ Wp, np.eye(R * C), atol=1e-11)
    assert np.abs(Wa - Wp).max() > 1e-2
