"""R by DCT-II diagonalisation on the GPU (Sec. "Example 1", the O(N log N)
route): against the FP64 oracle's direct reflexive blur for PSFs narrower and
much wider than the image (several reflections), FP32 and FP64; against the
direct blur kernels where both apply; batches, aliasing, rejected inputs."""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from paper_1707_02018_amd import ops
from paper_1707_02018_amd._lib import AdjwaveError
from workloads import gen_image, rng_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# sizes cover the any-length row kernel (2 .. 256), the compile-time pass
# structures (512 .. 4096: radix 8 passes ending in 8, 2, 4 and 8) and both
# transposes (32 x 32 scalar tiles, 64 x 64 vector tiles)
CASES = [(16, 16, 0), (16, 16, 5), (64, 32, 7), (32, 64, 40), (256, 512, 12), (256, 256, 200),
         (8, 128, 300), (2, 4, 3), (1024, 256, 60), (16, 4096, 9), (4096, 8, 3), (128, 2048, 5)]


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("rows,cols,r", CASES)
def test_dct_blur_against_oracle(dt, rows, cols, r):
    print(f"[dct blur] {rows}x{cols} r={r} {dt}", flush=True)
    rng = rng_for(110, rows * 7 + cols + r)
    g = obl.gaussian_taps(max(0.4 * r, 0.5), r)
    x = np.stack([gen_image(rng, rows, cols) for _ in range(2)])
    ref = obl.R(x, g)
    plan = ops.BlurDCT(rows, cols, g, dt)
    y = plan.apply(torch.tensor(x, dtype=dt, device=DEV))
    torch.cuda.synchronize()
    assert rel(y.double().cpu().numpy(), ref) <= TOL[dt] * max(1.0, np.log2(max(rows, cols)))


def test_dct_blur_matches_direct_kernels_at_full_size():
    """2048^2, the 15x15 sigma = 3 PSF: the DCT route and the tile kernel agree
    to FP32 rounding (R = R^* for the symmetric PSF)."""
    print("[dct blur] 2048x2048 r=7 vs direct", flush=True)
    N = 2048
    g = obl.gaussian_taps(3.0, 7)
    rng = rng_for(111, 0)
    x = torch.tensor(gen_image(rng, N, N), dtype=torch.float32, device=DEV)
    plan = ops.BlurDCT(N, N, g)
    b = ops.BlurSpec(N, N, taps=g)
    y1 = plan.apply(x)
    y2 = ops.blur(b, x)
    y3 = ops.blur_adjoint(b, x)
    torch.cuda.synchronize()
    assert rel(y1.double().cpu().numpy(), y2.double().cpu().numpy()) <= 2e-6
    assert rel(y1.double().cpu().numpy(), y3.double().cpu().numpy()) <= 2e-6
    # in place
    x2 = x.clone()
    plan.apply(x2, out=x2)
    torch.cuda.synchronize()
    assert torch.equal(x2, y1)


def test_dct_blur_rejects():
    g = obl.gaussian_taps(2.0, 4)
    with pytest.raises(AdjwaveError):
        ops.BlurDCT(48, 64, g)
    asym = g.copy()
    asym[0] *= 2
    with pytest.raises(AdjwaveError):
        ops.BlurDCT(64, 64, asym)
    plan = ops.BlurDCT(64, 64, g)
    with pytest.raises(ValueError):
        plan.apply(torch.zeros(64, 32, device=DEV))
    with pytest.raises(TypeError):
        plan.apply(torch.zeros(64, 64, dtype=torch.float64, device=DEV))
