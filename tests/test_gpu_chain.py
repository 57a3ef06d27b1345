"""Chained coarse synthesis levels (one launch for levels min(J, 4) .. 2, the
intermediate approximation bands kept in LDS) against the same transform
built from single-level calls: identical bits for W and (W^dagger)^*, every
mode the chain takes (zpd, sym) and those it leaves to the per-level kernels."""
import numpy as np
import pytest
import torch

from paper_1707_02018_amd import ops
from workloads import gen_coefficients, rng_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [  # rows, cols, levels, taps, bc
    (2048, 2048, 4, 8, "sym"), (256, 256, 3, 8, "sym"), (130, 70, 4, 16, "zpd"),
    (97, 161, 5, 2, "zpd"), (40, 56, 3, 8, "sym"), (512, 384, 4, 2, "sym"),
    (64, 64, 3, 16, "sym"), (300, 200, 6, 8, "zpd"), (256, 256, 4, 8, "per"),
    (96, 80, 3, 8, "per_ext"),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def level_by_level(w, x, op):
    """The J-level transform as J single-level calls (coarse to fine)."""
    _, sr, sc = w.layout()
    J = w.levels
    off = sr[J] * sc[J]
    a = x[:, :off]
    for j in range(J, 0, -1):
        k = sr[j] * sc[j]
        wj = ops.WaveletSpec(sr[j - 1], sc[j - 1], 1, lo=w.lo, bc=w.bc)
        coef = torch.cat([a.reshape(x.shape[0], -1), x[:, off:off + 3 * k]], dim=1).contiguous()
        off += 3 * k
        a = op(wj, coef)
    return a


@pytest.mark.parametrize("case", CASES)
def test_chained_synthesis_equals_level_by_level(case):
    rows, cols, J, L, bc = case
    w = ops.WaveletSpec(rows, cols, J, taps=L, bc=bc)
    rng = rng_for(82, rows + 3 * cols + J)
    x = torch.tensor(np.stack([gen_coefficients(rng, w.ncoef) for _ in range(2)]),
                     dtype=torch.float32, device=DEV)
    for op in (ops.wavelet_synth, ops.wavelet_analysis_adjoint):
        full = op(w, x)
        ref = level_by_level(w, x, op)
        torch.cuda.synchronize()
        assert torch.equal(full, ref), (case, op.__name__, (full - ref).abs().max().item())
