"""Single-pass operators against the two-kernel ones: A = R W with the finest
synthesis level synthesised into the blur's reflected LDS window (with and
without the subtracted observation), and A^* = W^* R^* with the blur adjoint
computed inside the finest analysis tiles. Identical bits over boundary modes,
filter lengths, radii (symmetric and asymmetric PSFs), ragged sizes and
batches; the FP64 oracle on a small case; unsupported requests rejected."""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from oracle import filters as ofl
from oracle import fista as ofi
from paper_1707_02018_amd import ops
from paper_1707_02018_amd._lib import AdjwaveError
from workloads import gen_coefficients, gen_image, rng_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [  # rows, cols, levels, taps, bc, radius, sigma, batch
    (2048, 2048, 4, 8, "sym", 7, 3.0, 1),
    (256, 256, 3, 8, "zpd", 4, 2.0, 2),
    (256, 256, 3, 8, "per", 4, 2.0, 2),
    (130, 70, 4, 16, "zpd", 12, 4.0, 1),
    (97, 161, 5, 2, "zpd", 1, 0.7, 3),
    (40, 56, 3, 8, "sym", 7, 3.0, 2),
    (300, 200, 6, 8, "zpd", 0, 1.0, 1),
    (14, 10, 1, 2, "per", 8, 3.0, 2),
    (8, 8, 1, 8, "sym", 7, 2.5, 1),
    (66, 130, 2, 16, "sym", 5, 2.0, 1),
]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def _problem(case, seed):
    rows, cols, J, L, bc, r, sigma, batch = case
    w = ops.WaveletSpec(rows, cols, J, taps=L, bc=bc)
    b = ops.BlurSpec(rows, cols, sigma=sigma, radius=r)
    rng = rng_for(seed, rows + 7 * cols + J)
    x = torch.tensor(np.stack([gen_coefficients(rng, w.ncoef) for _ in range(batch)]),
                     dtype=torch.float32, device=DEV)
    obs = torch.tensor(np.stack([gen_image(rng, rows, cols) for _ in range(batch)]),
                       dtype=torch.float32, device=DEV)
    return w, b, x, obs


@pytest.mark.parametrize("case", CASES)
def test_fused_A_bitwise_equals_two_kernels(case):
    print(f"[fused A] {case}", flush=True)
    w, b, x, obs = _problem(case, 90)
    ref = ops.apply_A(w, b, x)
    got = ops.apply_A_fused(w, b, x)
    res = ops.apply_A_fused(w, b, x, sub=obs)
    torch.cuda.synchronize()
    assert torch.equal(got, ref), (case, (got - ref).abs().max().item())
    assert torch.equal(res, ref - obs), (case, (res - (ref - obs)).abs().max().item())


def test_fused_A_against_oracle():
    rows, cols = 96, 80
    h = ofl.by_taps(8)
    psf = obl.gaussian_taps(2.0, 4)
    prob = ofi.Problem(rows, cols, h, "sym", 3, psf)
    rng = rng_for(91, 0)
    x = rng.standard_normal(prob.ncoef)
    obs = gen_image(rng, rows, cols)
    ref = prob.A(x) - obs
    w = ops.WaveletSpec(rows, cols, 3, lo=h, bc="sym")
    b = ops.BlurSpec(rows, cols, taps=psf)
    got = ops.apply_A_fused(w, b, torch.tensor(x, dtype=torch.float32, device=DEV),
                            sub=torch.tensor(obs, dtype=torch.float32, device=DEV))
    got = got.double().cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("bad", ["f64", "per_ext", "short"])
def test_fused_A_rejects_unsupported(bad):
    rows, cols, bc, dt, r = 64, 64, "sym", torch.float32, 3
    if bad == "f64":
        dt = torch.float64
    elif bad == "per_ext":
        bc = "per_ext"
    else:
        rows, r, bc = 4, 4, "zpd"  # fewer than radius + 1 rows
    w = ops.WaveletSpec(rows, cols, 1, taps=8, bc=bc)
    b = ops.BlurSpec(rows, cols, sigma=1.5, radius=r)
    x = torch.zeros(w.ncoef, dtype=dt, device=DEV)
    with pytest.raises(AdjwaveError):
        ops.apply_A_fused(w, b, x)


ADJ_CASES = [  # rows, cols, levels, taps, bc, radius, sigma (None: asymmetric PSF), batch
    (2048, 2048, 4, 8, "sym", 7, 3.0, 1),
    (256, 256, 3, 8, "zpd", 4, 2.0, 2),
    (256, 256, 3, 8, "sym", 4, None, 2),
    (130, 70, 4, 16, "zpd", 12, 4.0, 1),
    (130, 70, 4, 16, "sym", 12, None, 1),
    (97, 161, 5, 2, "zpd", 1, None, 3),
    (97, 161, 3, 2, "sym", 3, 1.0, 2),
    (40, 56, 3, 8, "sym", 7, 3.0, 2),
    (300, 200, 6, 8, "zpd", 0, 1.0, 1),
    (8, 8, 1, 8, "sym", 7, None, 1),
    (15, 17, 1, 16, "sym", 12, 4.0, 2),
    (5, 3, 1, 2, "zpd", 12, None, 1),
    (66, 130, 2, 16, "sym", 5, 2.0, 1),
]


def _adj_problem(case, seed):
    rows, cols, J, L, bc, r, sigma, batch = case
    w = ops.WaveletSpec(rows, cols, J, taps=L, bc=bc)
    rng = rng_for(seed, rows + 7 * cols + J + r)
    if sigma is None:  # asymmetric PSF: exercises the R^* border correction
        taps = rng.random(2 * r + 1) + 0.1
        b = ops.BlurSpec(rows, cols, taps=taps / taps.sum())
    else:
        b = ops.BlurSpec(rows, cols, sigma=sigma, radius=r)
    img = torch.tensor(np.stack([gen_image(rng, rows, cols) - 0.5 for _ in range(batch)]),
                       dtype=torch.float32, device=DEV)
    return w, b, img


@pytest.mark.parametrize("case", ADJ_CASES)
def test_fused_A_adjoint_bitwise_equals_two_kernels(case):
    print(f"[fused A*] {case}", flush=True)
    w, b, img = _adj_problem(case, 92)
    ref = ops.apply_A_adjoint(w, b, img)
    got = ops.apply_A_adjoint_fused(w, b, img)
    torch.cuda.synchronize()
    assert torch.equal(got, ref), (case, (got - ref).abs().max().item())


def test_fused_A_adjoint_against_oracle():
    rows, cols = 96, 80
    h = ofl.by_taps(8)
    rng = rng_for(93, 0)
    psf = rng.random(9) + 0.1
    psf /= psf.sum()
    prob = ofi.Problem(rows, cols, h, "sym", 3, psf)
    y = gen_image(rng, rows, cols) - 0.5
    ref = prob.A_adj(y)
    w = ops.WaveletSpec(rows, cols, 3, lo=h, bc="sym")
    b = ops.BlurSpec(rows, cols, taps=psf)
    got = ops.apply_A_adjoint_fused(w, b, torch.tensor(y, dtype=torch.float32, device=DEV))
    got = got.double().cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("bad", ["f64", "per", "per_ext", "sym_short"])
def test_fused_A_adjoint_rejects_unsupported(bad):
    rows, cols, bc, dt = 64, 64, "sym", torch.float32
    if bad == "f64":
        dt = torch.float64
    elif bad in ("per", "per_ext"):
        bc = bad
    else:
        rows = 6  # fewer than L - 1 rows: two-step fold
    w = ops.WaveletSpec(rows, cols, 1, taps=8, bc=bc)
    b = ops.BlurSpec(rows, cols, sigma=1.5, radius=3)
    img = torch.zeros(rows, cols, dtype=dt, device=DEV)
    with pytest.raises(AdjwaveError):
        ops.apply_A_adjoint_fused(w, b, img)
