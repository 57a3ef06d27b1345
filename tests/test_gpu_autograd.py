"""A = R W as a torch.autograd.Function whose backward is the hand-written
A^* kernel: FP64 gradcheck at 32 x 32 (4-level db4, symmetric boundaries,
sigma = 2 PSF), finite differences in FP32, and the batch-16 1024 x 1024
shape against the oracle on sampled images."""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from oracle import filters as ofl
from oracle import fista as ofi
from paper_1707_02018_amd import autograd as ag
from paper_1707_02018_amd import ops

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def _specs(n, levels=4, bc="sym"):
    w = ops.WaveletSpec(n, n, levels, lo=ofl.by_taps(8), bc=bc)
    b = ops.BlurSpec(n, n, taps=obl.gaussian_taps(2.0, 4))
    return w, b


@pytest.mark.parametrize("bc", ["sym", "per", "zpd"])
def test_gradcheck_fp64_32(bc):
    """Full FP64 gradcheck at 32 x 32 (db4, J = 4): the whole Jacobian of A
    by central differences against the one the backward (A^*) assembles,
    column by column and row by row (not a random projection), and the same
    for the adjoint operator."""
    print(f"[gradcheck] 32x32 db4 J=4 {bc}", flush=True)
    w, b = _specs(32, 4, bc)
    op = ag.AOperator(w, b)
    assert w.ncoef == {"sym": 6831, "per": 1024, "zpd": 2146}[bc]
    x = torch.randn(w.ncoef, dtype=torch.float64, device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(op, (x,), eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=False)
    y = torch.randn(32, 32, dtype=torch.float64, device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(op.adjoint, (y,), eps=1e-6, atol=1e-8, rtol=1e-6,
                                    fast_mode=False)


def test_backward_is_adjoint_against_oracle():
    """loss = <A x, y>: grad_x must equal the oracle's A^* y."""
    n = 32
    w, b = _specs(n)
    prob = ofi.Problem(n, n, ofl.by_taps(8), "sym", 4, obl.gaussian_taps(2.0, 4))
    rng = np.random.default_rng(0)
    xn = rng.standard_normal(w.ncoef)
    yn = rng.standard_normal((n, n))
    x = torch.tensor(xn, device=DEV, requires_grad=True)
    y = torch.tensor(yn, device=DEV)
    (ag.apply_A(x, w, b) * y).sum().backward()
    ref = prob.A_adj(yn)
    assert np.linalg.norm(x.grad.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-12


def test_finite_differences_fp32():
    n = 64
    w, b = _specs(n, 3)
    gen = torch.Generator(device="cpu").manual_seed(7)
    x = torch.randn(w.ncoef, generator=gen).to(DEV).requires_grad_(True)
    target = torch.randn(n, n, generator=gen).to(DEV)
    loss = 0.5 * ((ag.apply_A(x, w, b) - target) ** 2).sum()
    loss.backward()
    g = x.grad.detach().double().cpu().numpy()
    rng = np.random.default_rng(1)
    d = torch.tensor(rng.standard_normal(w.ncoef), dtype=torch.float32, device=DEV)
    # the loss is quadratic in x, so the central difference has no truncation
    # error at any step: a large step keeps the FP32 rounding of the two loss
    # values far below the difference
    eps = 0.5
    with torch.no_grad():
        fp = 0.5 * ((ops.apply_A(w, b, x + eps * d) - target) ** 2).double().sum().item()
        fm = 0.5 * ((ops.apply_A(w, b, x - eps * d) - target) ** 2).double().sum().item()
    fd = (fp - fm) / (2 * eps)
    an = float(np.dot(g, d.double().cpu().numpy()))
    assert abs(fd - an) <= 1e-3 * abs(an)


def test_batch16_1024_matches_oracle_samples():
    """Batch 16 x 1024 x 1024 FP32 forward/backward; images 0 and 15 are
    recomputed by the oracle."""
    print("[autograd] batch 16 x 1024^2", flush=True)
    n = 1024
    w, b = _specs(n)
    prob = ofi.Problem(n, n, ofl.by_taps(8), "sym", 4, obl.gaussian_taps(2.0, 4))
    x = torch.randn(16, w.ncoef, device=DEV, requires_grad=True)
    out = ag.apply_A(x, w, b)
    g_out = torch.randn_like(out)
    out.backward(g_out)
    torch.cuda.synchronize()
    for i in (0, 15):
        xi = x[i].detach().double().cpu().numpy()
        ref = prob.A(xi)
        assert np.linalg.norm(out[i].detach().double().cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-5
        gi = g_out[i].double().cpu().numpy()
        refg = prob.A_adj(gi)
        got = x.grad[i].double().cpu().numpy()
        assert np.linalg.norm(got - refg) / np.linalg.norm(refg) < 1e-5
