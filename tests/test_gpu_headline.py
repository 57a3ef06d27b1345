"""Oracle parity at the headline configuration and the tile shapes it runs.

One FISTA iteration (eq. 1, gradient W^* R^* (R W y - b) of Sec. "Example 1")
from an identical state, compared element by element with the FP64 oracle:

* 2048 x 2048 FP32, 4-level Daubechies-4, 15 x 15 Gaussian PSF (sigma 3), in
  the symmetric, periodic and zero boundary modes: the launch configuration
  the benchmark times (level-1 analysis grid of at least 1024 tiles, so the
  full-height analysis tile with the fused update runs);
* the update half alone (``aw_fista_update``) on a one-level 2048^2 transform;
* a batch of 48 images of 256^2 in one call, whose level-1 analysis grid
  (25 tiles per image) crosses 1024 tiles while the coarser levels stay below;
* one iteration of the batched uneven plan from a set state, for a 512 x 768
  problem among others of different size, depth, filter and PSF.

The gate is the per-step one: relative L2 <= 1e-5 for x_k, y_{k+1}, the
residual and the objective partials. The states are 0.9 W^dagger b plus
small noise (x_{k-1}) and a perturbation of it (y_k): the residual stays
about a tenth of b, so FP32 cancellation does not dominate it, and many
detail coefficients sit near the threshold lambda / L.
"""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from oracle import filters as ofl
from oracle import fista as ofi
from oracle import wavelet as owv
from paper_1707_02018_amd import ops
from paper_1707_02018_amd.batched import BatchedFista
from workloads import gen_image, gen_noise, rng_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5
LAM = 2e-5
ANA_TILE = 32  # FP32 analysis tile: 32 x 32 coefficients (full height)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    torch.cuda.init()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dev(x, dt=torch.float32):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _state(rng, b, h, mode, J):
    """x_{k-1} = 0.9 W^dagger b + noise, y_k = x_{k-1} + a smaller perturbation."""
    base = 0.9 * owv.W_pinv(b, h, mode, J)
    x_prev = base + 1e-4 * rng.standard_normal(base.shape)
    y = x_prev + 3e-5 * rng.standard_normal(base.shape)
    return x_prev, y


def _t_of(k):
    t = 1.0
    for _ in range(k - 1):
        t = ofi.t_next(t)
    return t


def _near_threshold_share(v, tau):
    return float(np.mean(np.abs(v) <= tau))


@pytest.fixture(scope="module")
def headline_problem():
    N = 2048
    rng = rng_for(2, 0)
    img = gen_image(rng, N, N)
    psf = obl.gaussian_taps(3.0, 7)
    b = obl.R(img, psf) + gen_noise(rng, img.shape)
    return N, psf, b


@pytest.mark.parametrize("mode", ["sym", "per", "zpd"])
def test_fista_step_2048_from_oracle_state(headline_problem, mode):
    N, psf, b = headline_problem
    J, k = 4, 7
    print(f"[headline step] {N}x{N} db4 J={J} {mode} fp32 k={k}", flush=True)
    h = ofl.by_taps(8)
    prob = ofi.Problem(N, N, h, mode, J, psf)
    _, sr, sc = owv.layout(N, N, 8, mode, J)
    tiles = -(-sr[1] // ANA_TILE) * -(-sc[1] // ANA_TILE)
    assert tiles >= 1024, tiles  # the full-height tile with the fused update
    rng = rng_for(2, 100 + ["sym", "per", "zpd"].index(mode))
    x_prev, y = _state(rng, b, h, mode, J)
    t = _t_of(k)
    beta = (t - 1.0) / ofi.t_next(t)
    r_ref = prob.A(y) - b
    v = y - prob.A_adj(r_ref)
    x_ref = ofi.soft(v, LAM)
    y_ref = x_ref + beta * (x_ref - x_prev)
    assert _near_threshold_share(v, LAM) > 1e-3  # the threshold acts
    assert np.linalg.norm(r_ref) < 0.3 * np.linalg.norm(b)

    w = ops.WaveletSpec(N, N, J, taps=8, bc=mode)
    bs = ops.BlurSpec(N, N, taps=psf)
    bt = dev(b)
    st = ops.FistaState(w, bs, bt, x0=dev(x_prev))
    st.y.copy_(dev(y))
    st.k, st.t = k, t
    ops.fista_step(st, bt, LAM, want_objective=True)
    assert rel(host(st.x), x_ref) <= TOL
    assert rel(host(st.y), y_ref) <= TOL
    assert rel(host(st.resid), r_ref) <= TOL
    obj = host(st.obj)[0]
    half_r2 = 0.5 * float(np.sum(r_ref * r_ref))
    l1 = float(np.sum(np.abs(x_ref)))
    assert abs(obj[0] - half_r2) <= TOL * half_r2
    assert abs(obj[1] - l1) <= TOL * l1
    # zeros where the oracle thresholds to zero (ties aside)
    xs = host(st.x)
    clear = np.abs(v) < 0.5 * LAM
    assert np.all(xs[clear] == 0.0)
    assert st.k == k + 1 and abs(st.t - ofi.t_next(t)) < 1e-15


def test_fista_update_2048_level1(headline_problem):
    """aw_fista_update on a one-level 2048^2 sym transform: W^* of an
    image-space gradient with the proximal / momentum update of the four
    level-1 bands in the full-height tile."""
    N, psf, b = headline_problem
    print(f"[headline update] {N}x{N} db4 J=1 sym fp32", flush=True)
    h = ofl.by_taps(8)
    mode, J, k = "sym", 1, 12
    _, sr, sc = owv.layout(N, N, 8, mode, J)
    assert -(-sr[1] // ANA_TILE) * -(-sc[1] // ANA_TILE) >= 1024
    rng = rng_for(2, 200)
    x_prev, y = _state(rng, b, h, mode, J)
    g = 1e-2 * rng.standard_normal((N, N))
    t = _t_of(k)
    beta = (t - 1.0) / ofi.t_next(t)
    v = y - owv.W_adj(g, h, mode, J)
    x_ref = ofi.soft(v, LAM)
    y_ref = x_ref + beta * (x_ref - x_prev)
    assert _near_threshold_share(v, LAM) > 1e-4
    w = ops.WaveletSpec(N, N, J, taps=8, bc=mode)
    bs = ops.BlurSpec(N, N, taps=psf)
    st = ops.FistaState(w, bs, dev(b), x0=dev(x_prev))
    st.y.copy_(dev(y))
    st.k, st.t = k, t
    ops.fista_update(st, dev(g), LAM, want_l1=True)
    assert rel(host(st.x), x_ref) <= TOL
    assert rel(host(st.y), y_ref) <= TOL
    l1 = float(np.sum(np.abs(x_ref)))
    assert abs(host(st.obj)[0][1] - l1) <= TOL * l1


def test_fista_step_batch48_256():
    """48 images of 256^2 (db4, J = 3, sym, 9 x 9 PSF sigma 2) in one call:
    level 1 runs 1200 full-height analysis tiles, levels 2 and 3 the
    half-height ones; every image against its own oracle step."""
    n, S, J, k = 48, 256, 3, 5
    print(f"[headline batch] {n} x {S}^2 db4 J={J} sym fp32", flush=True)
    h = ofl.by_taps(8)
    psf = obl.gaussian_taps(2.0, 4)
    _, sr, sc = owv.layout(S, S, 8, "sym", J)
    per_img = -(-sr[1] // ANA_TILE) * -(-sc[1] // ANA_TILE)
    assert per_img * n >= 1024 and -(-sr[2] // ANA_TILE) * -(-sc[2] // ANA_TILE) * n < 1024
    prob = ofi.Problem(S, S, h, "sym", J, psf)
    t = _t_of(k)
    beta = (t - 1.0) / ofi.t_next(t)
    bs_, xp_, y_, ref = [], [], [], []
    for i in range(n):
        rng = rng_for(1, 500 + i)
        img = gen_image(rng, S, S)
        b = obl.R(img, psf) + gen_noise(rng, img.shape)
        x_prev, y = _state(rng, b, h, "sym", J)
        r = prob.A(y) - b
        x = ofi.soft(y - prob.A_adj(r), LAM)
        bs_.append(b), xp_.append(x_prev), y_.append(y)
        ref.append((x, x + beta * (x - x_prev), r))
    w = ops.WaveletSpec(S, S, J, taps=8, bc="sym")
    bsp = ops.BlurSpec(S, S, taps=psf)
    bt = dev(np.stack(bs_))
    st = ops.FistaState(w, bsp, bt, x0=dev(np.stack(xp_)))
    st.y.copy_(dev(np.stack(y_)))
    st.k, st.t = k, t
    ops.fista_step(st, bt, LAM, want_objective=True)
    X, Y, Rr, O = host(st.x), host(st.y), host(st.resid), host(st.obj)
    for i, (x, yn, r) in enumerate(ref):
        assert rel(X[i], x) <= TOL, i
        assert rel(Y[i], yn) <= TOL, i
        assert rel(Rr[i], r) <= TOL, i
        hr = 0.5 * float(np.sum(r * r))
        assert abs(O[i, 0] - hr) <= TOL * hr, i
        l1 = float(np.sum(np.abs(x)))
        assert abs(O[i, 1] - l1) <= TOL * l1, i


# (rows, cols, levels, taps, sigma, radius), all sym as in the uneven batch
BATCH_PROBLEMS = [(512, 768, 4, 8, 2.2, 7), (768, 512, 3, 2, 1.2, 4), (640, 576, 5, 16, 3.1, 10),
                  (256, 384, 3, 8, 1.0, 3)]


@pytest.mark.parametrize("graph", [False, True])
def test_batched_plan_step_against_oracle(graph):
    """One iteration of the batched uneven plan from a set state (x_{k-1},
    y_k in the plan's buffers, iteration counter k), each problem against its
    own oracle step."""
    k = 9
    print(f"[headline batched plan] {len(BATCH_PROBLEMS)} problems k={k} graph={graph}",
          flush=True)
    t = _t_of(k)
    beta = (t - 1.0) / ofi.t_next(t)
    specs, obs, states, refs = [], [], [], []
    for i, (r, c, J, L, sg, rad) in enumerate(BATCH_PROBLEMS):
        rng = rng_for(3, 700 + i)
        img = gen_image(rng, r, c)
        psf = obl.gaussian_taps(sg, rad)
        b = obl.R(img, psf) + gen_noise(rng, img.shape)
        h = ofl.by_taps(L)
        x_prev, y = _state(rng, b, h, "sym", J)
        prob = ofi.Problem(r, c, h, "sym", J, psf)
        b32 = b.astype(np.float32).astype(np.float64)  # the plan holds b in FP32
        x = ofi.soft(y - prob.A_adj(prob.A(y) - b32), LAM)
        refs.append((x, x + beta * (x - x_prev)))
        specs.append((ops.WaveletSpec(r, c, J, lo=h, bc="sym"), ops.BlurSpec(r, c, taps=psf)))
        obs.append(dev(b))
        states.append((x_prev, y))
    bf = BatchedFista(specs, obs, LAM)
    for i, (x_prev, y) in enumerate(states):
        bf.x(i).copy_(dev(x_prev))
        bf.y(i).copy_(dev(y))
    bf.counter.fill_(k)
    torch.cuda.synchronize()
    bf.run(1, graph=graph)
    torch.cuda.synchronize()
    assert int(bf.counter.item()) == k + 1
    for i, (x, yn) in enumerate(refs):
        assert rel(host(bf.x(i)), x) <= TOL, i
        assert rel(host(bf.y(i)), yn) <= TOL, i
