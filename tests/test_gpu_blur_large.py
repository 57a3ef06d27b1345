"""R and R^* (Sec. "Example 1") on grids of several rounds of workgroups.

* A batch of two 2048^2 images (2048 tiles) equals, bit for bit, each image
  blurred alone (1024 tiles), for R, R^* with an asymmetric PSF (border
  correction) and the FISTA residual R y - b with its objective partials:
  the result of a tile depends only on its image and position.
* Radius 12 on 2047 x 2045 (odd width: every window staged through the
  reflection tables) and radius 4 on three 1536 x 1600 images (interior
  vector staging and borders) match the FP64 oracle within the FP32 gate.
"""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from paper_1707_02018_amd import ops
from workloads import gen_image, gen_noise, rng_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    torch.cuda.init()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(x, dt=torch.float32):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _taps(kind, r, rng):
    if kind == "gauss":
        return obl.gaussian_taps(r / 2.0, r)
    return rng.uniform(0.1, 1.0, 2 * r + 1)


@pytest.mark.parametrize("r,kind", [(7, "gauss"), (7, "asym"), (4, "asym")])
def test_batch_equals_single_2048(r, kind):
    print(f"[blur large] 2 x 2048^2 r={r} {kind}", flush=True)
    rng = rng_for(5, 10 * r + (kind == "asym"))
    x = rng.standard_normal((2, 2048, 2048))
    taps = _taps(kind, r, rng)
    b = ops.BlurSpec(2048, 2048, taps=taps)
    xd = dev(x)
    f2, a2 = host(ops.blur(b, xd)), host(ops.blur_adjoint(b, xd))
    for i in range(2):
        f1 = host(ops.blur(b, xd[i:i + 1].contiguous()))
        a1 = host(ops.blur_adjoint(b, xd[i:i + 1].contiguous()))
        assert np.array_equal(f2[i], f1[0]), i
        assert np.array_equal(a2[i], a1[0]), i


def test_batch_fista_residual_2048():
    """Three FISTA steps on a batch of two 2048^2 images against each image's
    own steps: x, y, the residual and the objective partials bitwise."""
    N, J = 2048, 4
    print(f"[blur large] fista step 2 x {N}^2 db4 J={J} sym", flush=True)
    psf = obl.gaussian_taps(3.0, 7)
    w = ops.WaveletSpec(N, N, J, taps=8, bc="sym")
    bs = ops.BlurSpec(N, N, taps=psf)
    imgs, obs = [], []
    for i in range(2):
        rng = rng_for(5, 300 + i)
        img = gen_image(rng, N, N)
        imgs.append(img)
        obs.append(obl.R(img, psf) + gen_noise(rng, img.shape))
    bt = dev(np.stack(obs))
    st2 = ops.FistaState(w, bs, bt)
    for _ in range(3):
        ops.fista_step(st2, bt, 2e-5, want_objective=True)
    X2, Y2, R2, O2 = host(st2.x), host(st2.y), host(st2.resid), host(st2.obj)
    for i in range(2):
        b1 = bt[i:i + 1].contiguous()
        st1 = ops.FistaState(w, bs, b1)
        for _ in range(3):
            ops.fista_step(st1, b1, 2e-5, want_objective=True)
        assert np.array_equal(X2[i], host(st1.x)[0]), i
        assert np.array_equal(Y2[i], host(st1.y)[0]), i
        assert np.array_equal(R2[i], host(st1.resid)[0]), i
        assert np.array_equal(O2[i], host(st1.obj)[0]), i


@pytest.mark.parametrize("n,rows,cols,r", [(1, 2047, 2045, 12), (3, 1536, 1600, 4)])
def test_large_against_oracle(n, rows, cols, r):
    print(f"[blur large] {n} x {rows}x{cols} r={r} vs oracle", flush=True)
    rng = rng_for(5, rows + cols + r)
    x = rng.standard_normal((n, rows, cols))
    for kind in ("gauss", "asym"):
        taps = _taps(kind, r, rng)
        b = ops.BlurSpec(rows, cols, taps=taps)
        xd = dev(x)
        f = host(ops.blur(b, xd)).astype(np.float64)
        a = host(ops.blur_adjoint(b, xd)).astype(np.float64)
        for i in range(n):
            assert rel(f[i], obl.R(x[i], taps)) <= TOL, (kind, i)
            assert rel(a[i], obl.R_adj(x[i], taps)) <= TOL, (kind, i)
