"""SSIM as the adjoint-vs-pseudoinverse study measures it (host code, CPU):
closed forms and a brute-force windowed evaluation."""
import numpy as np

from paper_1707_02018_amd.adjoint_study import ssim

C1, C2 = 0.01 ** 2, 0.03 ** 2


def brute_ssim(a, b):
    """Direct definition: 11 x 11 Gaussian window (sigma 1.5, normalised),
    borders reflected about the edge (a b c | c b a), per-pixel local means,
    variances and covariance, averaged over the image."""
    u = np.arange(-5, 6)
    g1 = np.exp(-u ** 2 / (2 * 1.5 ** 2))
    g1 /= g1.sum()
    win = np.outer(g1, g1)
    pa = np.pad(a, 5, mode="symmetric")
    pb = np.pad(b, 5, mode="symmetric")
    vals = []
    for i in range(a.shape[0]):
        for j in range(a.shape[1]):
            wa = pa[i:i + 11, j:j + 11]
            wb = pb[i:i + 11, j:j + 11]
            ma, mb = np.sum(win * wa), np.sum(win * wb)
            va = np.sum(win * wa * wa) - ma * ma
            vb = np.sum(win * wb * wb) - mb * mb
            cab = np.sum(win * wa * wb) - ma * mb
            vals.append((2 * ma * mb + C1) * (2 * cab + C2) /
                        ((ma * ma + mb * mb + C1) * (va + vb + C2)))
    return float(np.mean(vals))


def test_ssim_identical_and_symmetric():
    rng = np.random.default_rng(0)
    a, b = rng.random((30, 24)), rng.random((30, 24))
    assert abs(ssim(a, a) - 1.0) < 1e-12
    assert abs(ssim(a, b) - ssim(b, a)) < 1e-12
    assert ssim(a, b) < 0.5


def test_ssim_constant_images_closed_form():
    """No variance: only the luminance term (2 c d + C1) / (c^2 + d^2 + C1)."""
    for c, d in ((0.2, 0.7), (0.5, 0.5), (0.0, 1.0)):
        a, b = np.full((16, 16), c), np.full((16, 16), d)
        ref = (2 * c * d + C1) / (c * c + d * d + C1)
        assert abs(ssim(a, b) - ref) < 1e-12


def test_ssim_matches_windowed_definition():
    rng = np.random.default_rng(1)
    a = rng.random((14, 12))
    b = np.clip(a + 0.1 * rng.standard_normal(a.shape), 0, 1)
    assert abs(ssim(a, b) - brute_ssim(a, b)) < 1e-12
