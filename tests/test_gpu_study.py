"""Adjoint-vs-pseudoinverse study on the GPU: each gradient map's measures
(relative error, nonzero share, SSIM of the reconstruction) against the same
measures of the FP64 oracle's FISTA iterates on the same b."""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from oracle import filters as ofl
from oracle import fista as ofi
from oracle import wavelet as owv
from paper_1707_02018_amd import adjoint_study

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


@pytest.mark.parametrize("taps", [2, 8, "cdf97"])
def test_study_measures_match_oracle(taps):
    rows, cols, J, sigma, r, lam, iters = 64, 48, 3, 2.0, 4, 2e-5, 60
    print(f"[study] {rows}x{cols} taps={taps} J={J} {iters} iterations", flush=True)
    fam = "cdf97" if taps == "cdf97" else "daubechies"
    res = adjoint_study.run(rows, cols, 10 if fam == "cdf97" else taps, J, "sym", sigma, r, lam,
                            iters, every=30, device=DEV, family=fam)
    img, b, bsp = adjoint_study.make_problem(rows, cols, sigma, r, 0, DEV)
    bh = b.double().cpu().numpy()
    h = ofl.cdf97() if fam == "cdf97" else ofl.by_taps(taps)
    prob = ofi.Problem(rows, cols, h, "sym", J, bsp.taps)
    assert abs(res["blurred"]["rel_err"] -
               np.linalg.norm(bh - img) / np.linalg.norm(img)) < 1e-12
    for grad in ("adjoint", "pinv"):
        x = ofi.fista(prob, bh, lam, iters, gradient=grad)
        rec = owv.W(x, h, "sym", J, rows, cols)
        rel = np.linalg.norm(rec - img) / np.linalg.norm(img)
        nz = 100.0 * np.count_nonzero(x) / x.size
        got = res[grad]
        assert [c["k"] for c in got["curve"]] == [30, 60]
        assert abs(got["rel_err"] - rel) <= 1e-3 * rel, (grad, got["rel_err"], rel)
        assert abs(got["nonzero_pct"] - nz) <= 0.5, (grad, got["nonzero_pct"], nz)
        assert abs(got["ssim"] - adjoint_study.ssim(rec, img)) <= 1e-4
        F = ofi.objective(prob, x, bh, lam)
        assert abs(got["objective"] - F) <= 1e-4 * F, (grad, got["objective"], F)
