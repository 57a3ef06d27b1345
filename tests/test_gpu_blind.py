"""Multi-channel blind channel estimation on the GPU (Sec. "Example 2", eq. 6):
the shared-source convolution pair, the Huber TV term and the proximal step
against the FP64 oracle; the alternating solver's trajectory (objective and
step sizes, iteration by iteration) against the oracle's in FP64; FP32
descent; the paper-size problem; argument validation."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import blind as obl
from oracle import conv as ocv
from paper_1707_02018_amd import blind, ops
from paper_1707_02018_amd._lib import AdjwaveError, load
from workloads import gen_blind_problem, rng_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def dev(x, dt):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("C,K,N", [(2, 894, 1717), (3, 40, 129), (1, 7, 5), (2, 300, 64)])
def test_multichannel_conv_pair(dt, C, K, N):
    print(f"[blind conv] C={C} K={K} N={N} {dt}", flush=True)
    rng = rng_for(98, C * 1000 + K)
    h = rng.standard_normal((C, K))
    s = rng.standard_normal(N)
    x = rng.standard_normal((C, K + N - 1))
    S = np.broadcast_to(s, (C, N))
    r_ref = ocv.conv_full(h, S) - x
    gh_ref = ocv.grad_h(S, r_ref, K)
    gs_ref = ocv.grad_s(h, r_ref, N).sum(axis=0)
    hd, sd, xd = dev(h, dt), dev(s, dt), dev(x, dt)
    r = torch.empty(C, K + N - 1, dtype=dt, device=DEV)
    gh = torch.empty(C, K, dtype=dt, device=DEV)
    parts = torch.empty(C, N, dtype=dt, device=DEV)
    gs = torch.empty(N, dtype=dt, device=DEV)
    rn = torch.empty(C, dtype=torch.float64, device=DEV)
    code = ops._dtype_code(hd)
    assert load().aw_conv_multichannel(code, C, K, N, ops._ptr(hd), ops._ptr(sd), ops._ptr(xd),
                                       ops._ptr(r), ops._ptr(gh), ops._ptr(parts), ops._ptr(gs),
                                       ops._ptr(rn), _stream()) == 0
    tol = TOL[dt]  # FP32 rounding of these sums measures about 1e-7
    assert rel(host(r), r_ref) <= tol
    assert rel(host(gh), gh_ref) <= tol
    assert rel(host(gs), gs_ref) <= tol
    np.testing.assert_allclose(host(rn), np.sum(host(r) ** 2, axis=1), rtol=1e-12)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("K", [1, 2, 17, 844])
def test_huber_tv(dt, K):
    rng = rng_for(99, K)
    C, delta, gscale = 3, 0.1, 0.7
    h = 0.2 * rng.standard_normal((C, K))
    g0 = rng.standard_normal((C, K))
    ref_v = obl.tv_huber(h, delta) * delta  # sum of L_delta, unscaled
    ref_g = g0 + gscale * obl.D_adj(obl.huber_grad(obl.D(h), delta))
    hd, gd = dev(h, dt), dev(g0, dt)
    val = torch.empty(C, dtype=torch.float64, device=DEV)
    assert load().aw_huber_tv(ops._dtype_code(hd), C, K, ops._ptr(hd), delta, gscale,
                              ops._ptr(gd), ops._ptr(val), _stream()) == 0
    np.testing.assert_allclose(host(val), ref_v, rtol=10 * TOL[dt], atol=1e-300)
    assert rel(host(gd), ref_g) <= 10 * TOL[dt]


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_prox_l1_and_stats(dt):
    rng = rng_for(100, 0)
    n = 3001
    x = rng.standard_normal(n)
    g = rng.standard_normal(n)
    L, lam = 3.0, 0.4
    ref = obl.prox_step(x, 2.0 * g, L, lam)  # step 2/L on g
    xd, gd = dev(x, dt), dev(g, dt)
    out = torch.empty_like(xd)
    st = torch.empty(3, dtype=torch.float64, device=DEV)
    assert load().aw_prox_l1(ops._dtype_code(xd), n, ops._ptr(xd), ops._ptr(gd), 2.0 / L,
                             lam / L, ops._ptr(out), ops._ptr(st), _stream()) == 0
    o = host(out)
    assert rel(o, ref) <= 10 * TOL[dt]
    xr, gr = host(xd), host(gd)
    np.testing.assert_allclose(host(st), [np.sum(gr * (o - xr)), np.sum((o - xr) ** 2),
                                          np.sum(np.abs(o))], rtol=1e-10)


def test_solver_trajectory_matches_oracle():
    """FP64, two channels: objective and both step sizes after every one of 25
    iterations equal the oracle's (same backtracking decisions)."""
    print("[blind solver] trajectory C=2 K=24+36", flush=True)
    h_true, s_true, noise, h0, s0 = gen_blind_problem(rng_for(101, 0), 2, 24, 60, 20, 64)
    x = ocv.conv_full(h_true, np.broadcast_to(s_true, (2, 60))) + noise
    P = blind.PAPER
    ref = []
    obl.palm(h0, s0, x, P, 25, callback=lambda k, h, s, a, b: ref.append(
        (obl.objective(h, s, x, P), a, b, h.copy(), s.copy())))
    sol = blind.BlindChannel(dev(x, torch.float64), dev(h0, torch.float64),
                             dev(s0, torch.float64))
    assert abs(sol.objective() - obl.objective(h0, s0, x, P)) <= 1e-12 * obl.objective(h0, s0, x, P)
    for k in range(25):
        F = sol.step()
        Fr, Lh, Ls, hr, sr = ref[k]
        assert abs(F - Fr) <= 1e-9 * Fr, (k, F, Fr)
        assert (sol.Lh, sol.Ls) == (Lh, Ls), k
    assert rel(host(sol.h), ref[-1][3]) <= 1e-9
    assert rel(host(sol.s), ref[-1][4]) <= 1e-9


def test_solver_fp32_descends_paper_size():
    """The paper's sizes (K = 894, N = 1717 guessed as 844 / 1767), FP32: the
    objective never increases and falls well below its start."""
    print("[blind solver] paper size FP32, 60 iterations", flush=True)
    res = blind.run(iters=60, seed=1, device=DEV)
    assert res["iterations"] == 60
    assert res["monotone"], res
    assert res["F"] < 0.05 * res["F0"], res
    assert all(np.isfinite(res["channel_alignment"]))


def test_entry_points_validate():
    x = torch.zeros(8, device=DEV)
    out = torch.zeros(8, device=DEV)
    lib = load()
    assert lib.aw_prox_l1(0, 8, ops._ptr(x), ops._ptr(x), 1.0, 0.1, ops._ptr(x), None,
                          _stream()) != 0  # out aliases x
    assert lib.aw_prox_l1(0, 8, ops._ptr(x), ops._ptr(x), -1.0, 0.1, ops._ptr(out), None,
                          _stream()) != 0
    assert lib.aw_huber_tv(0, 1, 8, ops._ptr(x), 0.0, 1.0, None, None, _stream()) != 0
    assert lib.aw_conv_multichannel(0, 2, 3, 3, ops._ptr(x), ops._ptr(x), None, ops._ptr(out),
                                    None, None, ops._ptr(out), None, _stream()) != 0
    with pytest.raises(ValueError):
        blind.BlindChannel(torch.zeros(2, 10, device=DEV), torch.zeros(2, 4, device=DEV),
                           torch.zeros(5, device=DEV))
    with pytest.raises(AdjwaveError):
        ops.check("aw_prox_l1", lib.aw_prox_l1(0, 0, ops._ptr(x), ops._ptr(x), 1.0, 0.1,
                                               ops._ptr(out), None, _stream()))
