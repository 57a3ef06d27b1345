"""Batched uneven FISTA (tile queues over images of different size, depth,
filter, PSF and boundary mode): per-image agreement with the single-image
FISTA step, graph replay equal to eager launches, every tile variant equal,
inactive problems frozen, and the FP64 oracle on one problem."""
import numpy as np
import pytest
import torch

from oracle import blur as obl
from oracle import filters as ofl
from oracle import fista as ofi
from paper_1707_02018_amd import ops
from paper_1707_02018_amd.batched import BatchedFista
from workloads import gen_image, gen_noise, rng_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (rows, cols, levels, taps, bc, sigma, radius)
PROBLEMS = [(40, 56, 2, 8, "sym", 1.0, 3), (64, 64, 3, 2, "sym", 1.3, 4),
            (96, 72, 3, 16, "zpd", 2.3, 7), (130, 70, 4, 8, "sym", 4.0, 12),
            (96, 72, 3, 8, "per", 1.7, 5), (200, 136, 3, 2, "sym", 0.7, 2)]
ITERS = 8
LAM = 2e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


@pytest.fixture(scope="module")
def setup():
    specs, obs, host_b = [], [], []
    for i, (r, c, J, L, bc, sg, rad) in enumerate(PROBLEMS):
        rng = rng_for(3, i)
        img = gen_image(rng, r, c)
        psf = obl.gaussian_taps(sg, rad)
        b = obl.R(img, psf) + gen_noise(rng, img.shape)
        specs.append((ops.WaveletSpec(r, c, J, lo=ofl.by_taps(L), bc=bc),
                      ops.BlurSpec(r, c, taps=psf)))
        obs.append(torch.tensor(b, dtype=torch.float32, device=DEV))
        host_b.append(b)
    return specs, obs, host_b


def single_runs(specs, obs):
    out = []
    for (w, b), bt in zip(specs, obs):
        st = ops.FistaState(w, b, bt)
        for _ in range(ITERS):
            ops.fista_step(st, bt, LAM)
        torch.cuda.synchronize()
        out.append(st.x.clone())
    return out


def test_batched_matches_single_image_path(setup):
    specs, obs, _ = setup
    ref = single_runs(specs, obs)
    bf = BatchedFista(specs, obs, LAM)
    bf.reset()
    bf.run(ITERS, graph=False)
    torch.cuda.synchronize()
    assert int(bf.counter.item()) == ITERS + 1
    for i in range(len(PROBLEMS)):
        d = (bf.x(i) - ref[i]).abs().max().item()
        scale = ref[i].abs().max().item()
        assert d <= 1e-6 * scale, (i, d, scale)


def test_graph_replay_and_variants_equal_eager(setup):
    specs, obs, _ = setup
    bf = BatchedFista(specs, obs, LAM)
    bf.reset()
    bf.run(ITERS, graph=False)
    torch.cuda.synchronize()
    eager = bf.X.clone()
    for cfg in [(0, 0, 0, 4), (1, 1, 1, 1), (0, 1, 0, 2), (1, 0, 1, 4), (0, 2, 0, 3), (0, 2, 2, 4),
                (1, 1, 2, 1), (0, 3, 0, 2), (1, 3, 1, 4)]:
        bf.set_config(cfg)
        bf.reset()
        bf.run(ITERS, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(bf.X, eager), cfg
        # a second replay sequence from a fresh reset reproduces it bitwise
        bf.reset()
        bf.run(ITERS, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(bf.X, eager), cfg


def test_one_launch_blur_stage_with_asymmetric_psfs():
    """Blur variant 2 (every PSF zero-padded to the batch's largest radius,
    one launch per blur stage) equals the per-radius launches bitwise, also
    for asymmetric PSFs, whose R^* border correction the padding must keep."""
    rng = rng_for(3, 40)
    probs = [(48, 40, 2, 8, 3), (72, 96, 3, 2, 9), (33, 50, 2, 8, 0)]
    specs, obs = [], []
    for r, c, J, L, rad in probs:
        img = gen_image(rng, r, c)
        taps = rng.uniform(0.1, 1.0, 2 * rad + 1)
        taps /= taps.sum()
        b = obl.R(img, taps) + gen_noise(rng, img.shape)
        specs.append((ops.WaveletSpec(r, c, J, lo=ofl.by_taps(L), bc="sym"),
                      ops.BlurSpec(r, c, taps=taps)))
        obs.append(torch.tensor(b, dtype=torch.float32, device=DEV))
    bf = BatchedFista(specs, obs, LAM)
    out = []
    for cfg in [(0, 0, 0, 1), (0, 0, 2, 1), (0, 0, 2, 4)]:
        bf.set_config(cfg)
        bf.reset()
        bf.run(ITERS, graph=False)
        torch.cuda.synchronize()
        out.append((bf.X.clone(), bf.obj.clone()))
    for X, O in out[1:]:
        assert torch.equal(X, out[0][0])
        assert torch.equal(O, out[0][1])


def test_inactive_problem_is_frozen(setup):
    specs, obs, _ = setup
    bf = BatchedFista(specs, obs, LAM)
    bf.reset()
    bf.run(3, graph=True)
    torch.cuda.synchronize()
    frozen = bf.x(2).clone()
    moving = bf.x(3).clone()
    bf.set_active(2, False)
    bf.run(3, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(bf.x(2), frozen)
    assert not torch.equal(bf.x(3), moving)


def test_batched_against_oracle(setup):
    specs, obs, host_b = setup
    bf = BatchedFista(specs, obs, LAM)
    bf.reset()
    bf.run(ITERS, graph=True)
    torch.cuda.synchronize()
    i = 3  # 130 x 70, db4, J = 4, sym, radius 12
    r, c, J, L, bc, sg, rad = PROBLEMS[i]
    prob = ofi.Problem(r, c, ofl.by_taps(L), bc, J, obl.gaussian_taps(sg, rad))
    b32 = obs[i].double().cpu().numpy()
    x_ref = ofi.fista(prob, b32, LAM, ITERS)
    got = bf.x(i).double().cpu().numpy()
    assert np.linalg.norm(got - x_ref) / np.linalg.norm(x_ref) <= 1e-4


def test_autotune_picks_a_valid_config(setup, tmp_path, monkeypatch):
    monkeypatch.setenv("ADJWAVE_CACHE_DIR", str(tmp_path))
    specs, obs, _ = setup
    bf = BatchedFista(specs, obs, LAM)
    rec = bf.autotune(iters=2)
    assert not rec["cached"] and len(rec["trials"]) >= 5
    assert bf.config == tuple(rec["config"])
    rec2 = BatchedFista(specs, obs, LAM).autotune(iters=2)
    assert rec2["cached"] and rec2["config"] == rec["config"]


def test_set_config_rejects_out_of_range_values(setup):
    """Tile variants beyond synthesis 0..1, analysis 0..3, blur 0..2 and
    stream counts beyond 1..4 fail with EINVAL and leave the plan as it was."""
    from paper_1707_02018_amd._lib import AdjwaveError
    specs, obs, _ = setup
    bf = BatchedFista(specs, obs, LAM)
    bf.set_config((0, 3, 0, 2))
    for bad in [(2, 0, 0, 2), (0, 4, 0, 2), (0, 0, 3, 2), (-1, 0, 0, 2), (0, 0, 0, 0), (0, 0, 0, 5)]:
        with pytest.raises(AdjwaveError):
            bf.set_config(bad)
    assert bf.config == (0, 3, 0, 2)
    bf.reset()
    bf.run(2, graph=False)
    torch.cuda.synchronize()
    assert int(bf.counter.item()) == 3
