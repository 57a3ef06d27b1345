"""Biorthogonal CDF 9/7 on the GPU (Sec. "The adjoint for biorthogonal
wavelets"): W, the true adjoint W^* (analysis with the dual filters under the
(E^dagger)^* fold, eq. 4), W^dagger and (W^dagger)^* against the FP64 oracle in
every boundary mode, FP32 and FP64, with dot tests; the 2048^2 sym transform;
one FISTA step with either gradient map; requests the batched and single-pass
paths do not cover are rejected."""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from oracle import filters as ofl
from oracle import fista as ofi
from oracle import wavelet as owv
from paper_1707_02018_amd import ops
from paper_1707_02018_amd._lib import AdjwaveError
from workloads import gen_image, gen_noise, rng_for

pytestmark = pytest.mark.gpu
TOL = {torch.float32: 1e-5, torch.float64: 1e-12}
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dev(x, dt):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def dot_test(fwd_x, x, adj_y, y):
    lhs = np.vdot(fwd_x.ravel(), y.ravel())
    rhs = np.vdot(x.ravel(), adj_y.ravel())
    return abs(lhs - rhs) / (np.linalg.norm(fwd_x) * np.linalg.norm(y))


CASES = [(m, r, c, J) for m in ("zpd", "sym", "per", "per_ext")
         for r, c, J in [(37, 53, 2), (64, 96, 3), (256, 200, 4), (18, 10, 1), (130, 70, 4)]
         if not (m == "per" and (r % 2 ** J or c % 2 ** J))]


@pytest.mark.parametrize("mode,rows,cols,J", CASES)
def test_cdf97_ops_parity(mode, rows, cols, J):
    print(f"[cdf97] mode={mode} {rows}x{cols} J={J}", flush=True)
    h = ofl.cdf97()
    rng = rng_for(95, rows * 1000 + cols * 10 + J)
    batch = 2
    n = owv.layout(rows, cols, 10, mode, J)[0]
    x = rng.standard_normal((batch, n))
    y = rng.standard_normal((batch, rows, cols))
    refs = {
        "W": owv.W(x, h, mode, J, rows, cols),
        "Wadj": owv.W_adj(y, h, mode, J),
        "Wpinv": owv.W_pinv(y, h, mode, J),
        "Wpinv_adj": owv.W_pinv_adj(x, h, mode, J, rows, cols),
    }
    w = ops.WaveletSpec(rows, cols, J, bc=mode, family="cdf97")
    assert w.ncoef == n
    for dt in (torch.float32, torch.float64):
        xd, yd = dev(x, dt), dev(y, dt)
        got = {
            "W": host(ops.wavelet_synth(w, xd)),
            "Wadj": host(ops.wavelet_synth_adjoint(w, yd)),
            "Wpinv": host(ops.wavelet_analysis(w, yd)),
            "Wpinv_adj": host(ops.wavelet_analysis_adjoint(w, xd)),
        }
        for k in refs:
            e = rel(got[k], refs[k])
            assert e <= TOL[dt], f"{k} {dt}: rel err {e:.3e}"
        xr, yr = host(xd), host(yd)
        assert dot_test(got["W"], xr, got["Wadj"], yr) <= 1e-6
        assert dot_test(got["Wpinv"], yr, got["Wpinv_adj"], xr) <= 1e-6
        # W W^dagger = I (perfect reconstruction through the two sides)
        pr = host(ops.wavelet_synth(w, ops.wavelet_analysis(w, yd)))
        assert rel(pr, yr) <= TOL[dt]
    # the adjoint is not the analysis: the two maps differ
    assert rel(refs["Wadj"], refs["Wpinv"]) > 1e-3


def test_cdf97_full_size_sym():
    """2048^2, four levels, sym, FP32: W and W^* against the oracle."""
    print("[cdf97 full] 2048x2048 J=4 sym", flush=True)
    N, J = 2048, 4
    h = ofl.cdf97()
    rng = rng_for(96, 0)
    n = owv.layout(N, N, 10, "sym", J)[0]
    x = rng.standard_normal(n)
    y = rng.standard_normal((N, N))
    w = ops.WaveletSpec(N, N, J, bc="sym", family="cdf97")
    assert rel(host(ops.wavelet_synth(w, dev(x, torch.float32))),
               owv.W(x, h, "sym", J, N, N)) <= TOL[torch.float32]
    assert rel(host(ops.wavelet_synth_adjoint(w, dev(y, torch.float32))),
               owv.W_adj(y, h, "sym", J)) <= TOL[torch.float32]


@pytest.mark.parametrize("gradient", ["adjoint", "pinv"])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_cdf97_fista_step(dt, gradient):
    print(f"[cdf97 fista] 256x256 {dt} gradient={gradient}", flush=True)
    rows = cols = 256
    h = ofl.cdf97()
    psf = obl.gaussian_taps(2.0, 4)
    rng = rng_for(97, 0)
    img = gen_image(rng, rows, cols)
    b = obl.R(img, psf) + gen_noise(rng, img.shape)
    prob = ofi.Problem(rows, cols, h, "sym", 3, psf)
    x_prev = rng.standard_normal(prob.ncoef) * 1e-2
    y = rng.standard_normal(prob.ncoef) * 1e-2
    lam, k = 2e-5, 4
    t = 1.0
    for _ in range(k - 1):
        t = ofi.t_next(t)
    beta = (t - 1.0) / ofi.t_next(t)
    x_ref, y_ref = ofi.fista_step(prob, x_prev, y, b, beta, lam, gradient=gradient)
    w = ops.WaveletSpec(rows, cols, 3, bc="sym", family="cdf97")
    bs = ops.BlurSpec(rows, cols, taps=psf)
    bt = dev(b, dt)
    st = ops.FistaState(w, bs, bt, x0=dev(x_prev, dt), gradient=gradient)
    st.y.copy_(dev(y, dt))
    st.k, st.t = k, t
    ops.fista_step(st, bt, lam, want_objective=True)
    assert rel(host(st.x), x_ref) <= TOL[dt]
    assert rel(host(st.y), y_ref) <= TOL[dt]
    assert rel(host(st.resid), prob.A(y) - b) <= TOL[dt]


def test_cdf97_unsupported_paths_rejected():
    w = ops.WaveletSpec(64, 64, 2, bc="sym", family="cdf97")
    b = ops.BlurSpec(64, 64, sigma=1.5, radius=3)
    x = torch.zeros(w.ncoef, dtype=torch.float32, device=DEV)
    img = torch.zeros(64, 64, dtype=torch.float32, device=DEV)
    with pytest.raises(AdjwaveError):
        ops.apply_A_fused(w, b, x)
    with pytest.raises(AdjwaveError):
        ops.apply_A_adjoint_fused(w, b, img)
    from paper_1707_02018_amd.batched import BatchedFista
    with pytest.raises(AdjwaveError):
        BatchedFista([(w, b)], [img], 2e-5)


@pytest.mark.parametrize("mode", ["zpd", "sym", "per", "per_ext"])
def test_cdf97_A_and_adjoint_parity(mode):
    """A = R W and A^* = W^* R^* with the CDF 9/7 pair against the oracle, with
    the dot test (the true adjoint of the biorthogonal synthesis)."""
    print(f"[cdf97 A] 128x96 J=3 {mode}", flush=True)
    rows, cols = 128, 96
    h = ofl.cdf97()
    psf = obl.gaussian_taps(2.0, 4)
    prob = ofi.Problem(rows, cols, h, mode, 3, psf)
    rng = rng_for(102, 0)
    x = rng.standard_normal(prob.ncoef)
    y = rng.standard_normal((rows, cols))
    w = ops.WaveletSpec(rows, cols, 3, bc=mode, family="cdf97")
    b = ops.BlurSpec(rows, cols, taps=psf)
    for dt in (torch.float32, torch.float64):
        f = host(ops.apply_A(w, b, dev(x, dt)))
        a = host(ops.apply_A_adjoint(w, b, dev(y, dt)))
        assert rel(f, prob.A(x)) <= TOL[dt]
        assert rel(a, prob.A_adj(y)) <= TOL[dt]
        assert dot_test(f, host(dev(x, dt)), a, host(dev(y, dt))) <= 1e-6


def test_cdf97_autograd_gradcheck():
    """The autograd operator with the biorthogonal pair: backward is the true
    adjoint (full FP64 gradcheck, 32 x 32, three levels, sym)."""
    from paper_1707_02018_amd import autograd as ag

    w = ops.WaveletSpec(32, 32, 3, bc="sym", family="cdf97")
    b = ops.BlurSpec(32, 32, taps=obl.gaussian_taps(2.0, 4))
    op = ag.AOperator(w, b)
    x = torch.randn(w.ncoef, dtype=torch.float64, device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(op, (x,), eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=False)
    y = torch.randn(32, 32, dtype=torch.float64, device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(op.adjoint, (y,), eps=1e-6, atol=1e-8, rtol=1e-6,
                                    fast_mode=False)
