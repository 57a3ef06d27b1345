"""Pins for the oracle's filters and extension operators (CPU only).

Each expected value comes from the paper's printed matrices or from textbook
closed forms, not from the oracle itself.
"""
import numpy as np
import pytest

from oracle import extension as ext
from oracle import filters as fl


# ------------------------------------------------------------------ filters
@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8])
def test_daubechies_defining_identities(p):
    h = fl.daubechies(p)
    L = len(h)
    assert L == 2 * p
    assert abs(h.sum() - np.sqrt(2.0)) < 1e-13
    for m in range(p):  # even-shift orthonormality
        s = sum(h[k] * h[k + 2 * m] for k in range(L - 2 * m))
        assert abs(s - (1.0 if m == 0 else 0.0)) < 1e-13
    g = fl.highpass(h)
    for j in range(p):  # p vanishing moments of the wavelet, scaled by max k^j
        mom = sum(g[k] * k ** j for k in range(L))
        assert abs(mom) <= 1e-12 * max(1.0, (L - 1) ** j)
    # H(z) has p zeros at z = -1; the remaining zeros lie inside the unit
    # circle (minimum phase)
    q = h.copy()
    for _ in range(p):
        q, rem = np.polydiv(q, [1.0, 1.0])
        assert np.max(np.abs(rem)) < 1e-9
    if len(q) > 1:
        assert np.all(np.abs(np.roots(q)) < 1.0)


def test_haar_and_db2_closed_forms():
    np.testing.assert_allclose(fl.daubechies(1), [2 ** -0.5, 2 ** -0.5], atol=1e-15)
    s3 = np.sqrt(3.0)
    db2 = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * np.sqrt(2.0))
    np.testing.assert_allclose(fl.daubechies(2), db2, atol=1e-14)


def test_highpass_is_orthogonal_to_lowpass_shifts():
    for taps in (2, 8, 16):
        h = fl.by_taps(taps)
        g = fl.highpass(h)
        L = len(h)
        for m in range(-(L // 2) + 1, L // 2):
            s = sum(h[k] * g[k - 2 * m] for k in range(L) if 0 <= k - 2 * m < L)
            assert abs(s) < 1e-13
        assert abs(np.dot(g, g) - 1.0) < 1e-13


# ---------------------------------------------------------- extension (paper)
def _rev(n):
    return np.eye(n)[::-1]


def paper_E_sym(N, Lp):
    """Block form of the half-point symmetric extension matrix (Sec. 'A few
    signal extensions', N > 2L')."""
    I, P, Z = np.eye(Lp), _rev(Lp), np.zeros
    mid = N - 2 * Lp
    return np.block([
        [P, Z((Lp, mid)), Z((Lp, Lp))],
        [I, Z((Lp, mid)), Z((Lp, Lp))],
        [Z((mid, Lp)), np.eye(mid), Z((mid, Lp))],
        [Z((Lp, Lp)), Z((Lp, mid)), I],
        [Z((Lp, Lp)), Z((Lp, mid)), P],
    ])


def paper_E_sym_pinv_adj(N, Lp):
    """The paper's closed form of (E_sym^dagger)^*: 1/2 on the reflected blocks."""
    E = paper_E_sym(N, Lp)
    E[:2 * Lp] *= 0.5
    E[-2 * Lp:] *= 0.5
    return E


def paper_E_per(N, Lp):
    """Block form of the periodic extension matrix."""
    Z = np.zeros
    return np.vstack([
        np.hstack([Z((Lp, N - Lp)), np.eye(Lp)]),
        np.eye(N),
        np.hstack([np.eye(Lp), Z((Lp, N - Lp))]),
    ])


def paper_E_per_pinv_adj(N, Lp):
    """Printed closed form of (E_per^dagger)^*; the middle identity block is
    split as (1/2 I, I, 1/2 I)."""
    Z = np.zeros
    mid = N - 2 * Lp
    return np.vstack([
        np.hstack([Z((Lp, N - Lp)), 0.5 * np.eye(Lp)]),
        np.hstack([0.5 * np.eye(Lp), Z((Lp, N - Lp))]),
        np.hstack([Z((mid, Lp)), np.eye(mid), Z((mid, Lp))]),
        np.hstack([Z((Lp, N - Lp)), 0.5 * np.eye(Lp)]),
        np.hstack([0.5 * np.eye(Lp), Z((Lp, N - Lp))]),
    ])


def paper_E_zpd(N, Lp):
    return np.vstack([np.zeros((Lp, N)), np.eye(N), np.zeros((Lp, N))])


@pytest.mark.parametrize("N,L", [(10, 4), (16, 8), (40, 16), (9, 2)])
def test_E_sym_matches_paper(N, L):
    Lp = L - 1
    assert N > 2 * Lp
    np.testing.assert_array_equal(ext.matrix(N, Lp, "sym"), paper_E_sym(N, Lp))
    E = ext.matrix(N, Lp, "sym")
    pa = E / ext.multiplicity(N, Lp, "sym")[None, :]
    np.testing.assert_array_equal(pa, paper_E_sym_pinv_adj(N, Lp))
    np.testing.assert_allclose(np.linalg.pinv(paper_E_sym(N, Lp)).T, pa, atol=1e-13)


@pytest.mark.parametrize("N,L", [(10, 4), (16, 8), (40, 16), (9, 2)])
def test_E_per_matches_paper(N, L):
    Lp = L - 1
    np.testing.assert_array_equal(ext.matrix(N, Lp, "per_ext"), paper_E_per(N, Lp))
    E = ext.matrix(N, Lp, "per_ext")
    pa = E / ext.multiplicity(N, Lp, "per_ext")[None, :]
    np.testing.assert_array_equal(pa, paper_E_per_pinv_adj(N, Lp))
    np.testing.assert_allclose(np.linalg.pinv(paper_E_per(N, Lp)).T, pa, atol=1e-13)


@pytest.mark.parametrize("N,L", [(5, 4), (12, 8)])
def test_E_zpd_orthonormal_columns(N, L):
    E = paper_E_zpd(N, L - 1)
    np.testing.assert_array_equal(E.T @ E, np.eye(N))
    np.testing.assert_allclose(np.linalg.pinv(E), E.T, atol=1e-14)


@pytest.mark.parametrize("mode", ["sym", "per_ext"])
@pytest.mark.parametrize("L", [2, 4, 8, 16])
def test_pinv_adjoint_at_every_size(mode, L):
    """(E^dagger)^* from the library pseudoinverse equals E diag(1/mult) for
    every N, including N <= 2L' where 1/3 and smaller weights appear."""
    Lp = L - 1
    for N in range(1, 3 * L):
        E = ext.matrix(N, Lp, mode)
        pa = E / ext.multiplicity(N, Lp, mode)[None, :]
        np.testing.assert_allclose(np.linalg.pinv(E).T, pa, atol=1e-12)


def test_one_third_weights_appear_when_N_le_2Lp():
    """Sec. 'A few signal extensions': for N <= 2L' some 1/2 become 1/3."""
    N, Lp = 5, 3
    w = 1.0 / ext.multiplicity(N, Lp, "sym")
    assert np.any(np.isclose(w, 1.0 / 3.0))
    w_big = 1.0 / ext.multiplicity(20, Lp, "sym")
    assert set(np.round(w_big, 12)) == {0.5, 1.0}


def test_fold_is_transpose_of_extend():
    rng = np.random.default_rng(3)
    for mode, e in [("sym", 7), ("per_ext", 7), ("sym", 15), ("zpd", 0)]:
        for N in (1, 3, 8, 30):
            if mode == "zpd" and e:
                continue
            y = rng.standard_normal(N)
            v = rng.standard_normal(N + 2 * e)
            lhs = np.dot(ext.extend(y, e, mode), v)
            rhs = np.dot(y, ext.fold(v, N, e, mode, weights="ones"))
            assert abs(lhs - rhs) < 1e-12 * (1 + abs(lhs))
            lhs = np.dot(ext.extend(y, e, mode, weights="pinv"), v)
            rhs = np.dot(y, ext.fold(v, N, e, mode, weights="pinv"))
            assert abs(lhs - rhs) < 1e-12 * (1 + abs(lhs))
