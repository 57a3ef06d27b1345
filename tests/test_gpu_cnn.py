"""Warm-start CNN kernels (BF16 operands, FP32 accumulation) against the FP64
oracle, layer by layer: each GPU layer is compared with the oracle applied to
the GPU's own BF16 inputs (the FP32 image for the first layer) and BF16-rounded
weights, so the check isolates one kernel at a time.

Tolerances (derived from the arithmetic): a BF16-stored output is within
2^-8 |z| of the exact value z (round to nearest) plus the FP32 accumulation
error, bounded here by 1e-5 of the sum of absolute products S; an FP32 output
(network output u, weight gradients) is within 2e-4 S (FP32 sums of up to a few
thousand terms per accumulator, then FP64 across workgroups)."""
import numpy as np
import pytest
import torch

from oracle import cnn
from paper_1707_02018_amd import ops
from workloads import gen_cnn_init, gen_image, rng_for

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHAPES = [(2, 40, 72), (1, 33, 31), (1, 1, 1), (3, 5, 7), (1, 70, 130)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def bf16(a) -> np.ndarray:
    """Round to BF16 (nearest even) with the library conversion of torch."""
    return torch.tensor(np.asarray(a), dtype=torch.float32).to(torch.bfloat16).double().numpy()


def kernel_params(theta: np.ndarray) -> np.ndarray:
    """What the kernels compute with: BF16 weights, FP32 biases."""
    out = []
    for w, b in cnn.unpack(theta):
        out.append((bf16(w), b.astype(np.float32).astype(np.float64)))
    return cnn.pack(out)


def acts_np(buf: torch.Tensor, n, H, W) -> np.ndarray:
    """[5][n][H][W][32] BF16 buffer -> float64 [5, n, 32, H, W]."""
    a = buf.view(torch.bfloat16).view(5, n, H, W, 32).double().cpu().numpy()
    return a.transpose(0, 1, 4, 2, 3)


class Net:
    def __init__(self, theta: np.ndarray):
        self.theta = theta
        self.params = torch.tensor(theta, dtype=torch.float32, device=DEV)
        pk, _, _ = ops.cnn_sizes(1, 1, 1)
        self.packed = torch.empty(pk, dtype=torch.uint8, device=DEV)
        ops.cnn_pack(self.params, self.packed)

    def forward(self, b: torch.Tensor):
        n, H, W = b.shape
        _, act, _ = ops.cnn_sizes(n, H, W)
        acts = torch.empty(act, dtype=torch.uint8, device=DEV)
        u = ops.cnn_forward(self.packed, b, acts)
        return u, acts

    def backward(self, b, acts, du):
        n, H, W = b.shape
        _, act, ws = ops.cnn_sizes(n, H, W)
        dacts = torch.empty(act, dtype=torch.uint8, device=DEV)
        grad = torch.empty(ops.CNN_PARAMS, dtype=torch.float32, device=DEV)
        wsb = torch.empty(ws, dtype=torch.uint8, device=DEV)
        ops.cnn_backward(self.packed, b, acts, du, dacts, grad, wsb)
        return grad, dacts


def make(shape, seed):
    n, H, W = shape
    r = rng_for(21, seed)
    theta = gen_cnn_init(r, cnn.LAYERS, out_scale=1.0)
    imgs = np.stack([gen_image(r, H, W) for _ in range(n)])
    du = r.standard_normal((n, H, W))
    return theta, imgs, du


def check_bf16_out(got, z, S, what):
    tol = 2.0 ** -8 * np.abs(z) + 1e-5 * S + 1e-30
    bad = np.abs(got - z) > tol
    assert not bad.any(), (what, int(bad.sum()), float(np.max(np.abs(got - z) - tol)))


def layer_ref(k, thk, x):
    """Oracle layer k on input x (ci, H, W): (value, sum of |products| + |bias|)."""
    w, b = cnn.unpack(thk)[k]
    z = cnn.conv3x3(x, w, b)
    S = cnn.conv3x3(np.abs(x), np.abs(w), np.abs(b))
    return z, S


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_layers_match_oracle(shape):
    theta, imgs, _ = make(shape, 0)
    n, H, W = shape
    net = Net(theta)
    b = torch.tensor(imgs, dtype=torch.float32, device=DEV)
    u, acts = net.forward(b)
    torch.cuda.synchronize()
    A = acts_np(acts, n, H, W)
    thk = kernel_params(theta)
    u = u.double().cpu().numpy()
    b32 = imgs.astype(np.float32).astype(np.float64)
    for i in range(n):
        x = b32[i][None]  # the image enters in FP32
        for k in range(5):
            z, S = layer_ref(k, thk, x)
            check_bf16_out(A[k, i], np.maximum(z, 0.0), S, (shape, i, k))
            x = A[k, i]
        z, S = layer_ref(5, thk, x)
        ref = b32[i] + z[0]
        assert np.all(np.abs(u[i] - ref) <= 2e-5 * (S[0] + np.abs(b32[i])) + 1e-7), (shape, i)


@pytest.mark.parametrize("shape", SHAPES)
def test_backward_layers_match_oracle(shape):
    theta, imgs, du_np = make(shape, 1)
    n, H, W = shape
    net = Net(theta)
    b = torch.tensor(imgs, dtype=torch.float32, device=DEV)
    du = torch.tensor(du_np, dtype=torch.float32, device=DEV)
    _, acts = net.forward(b)
    grad, dacts = net.backward(b, acts, du)
    torch.cuda.synchronize()
    A = acts_np(acts, n, H, W)
    D = acts_np(dacts, n, H, W)
    thk = kernel_params(theta)
    layers = cnn.unpack(thk)
    g = grad.double().cpu().numpy()
    du32 = du_np.astype(np.float32).astype(np.float64)
    b32 = imgs.astype(np.float32).astype(np.float64)
    gref = [np.zeros((co, ci, 3, 3)) for ci, co in cnn.LAYERS]
    bref = [np.zeros(co) for ci, co in cnn.LAYERS]
    gabs = [np.zeros((co, ci, 3, 3)) for ci, co in cnn.LAYERS]
    babs = [np.zeros(co) for ci, co in cnn.LAYERS]
    for i in range(n):
        dout = bf16(du32[i])[None]
        # gradient at layer 5's pre-activation from the output layer
        w6 = layers[5][0]
        z = cnn.conv3x3_input_grad(dout, w6) * (A[4, i] > 0)
        S = cnn.conv3x3_input_grad(np.abs(dout), np.abs(w6))
        check_bf16_out(D[4, i], z, S, (shape, i, "dz5"))
        for k in range(4, 0, -1):  # layer k+1 (0-based k) back to layer k
            w = layers[k][0]
            z = cnn.conv3x3_input_grad(D[k, i], w) * (A[k - 1, i] > 0)
            S = cnn.conv3x3_input_grad(np.abs(D[k, i]), np.abs(w))
            check_bf16_out(D[k - 1, i], z, S, (shape, i, f"dz{k}"))
        inputs = [b32[i][None]] + [A[k, i] for k in range(5)]
        douts = [D[k, i] for k in range(5)] + [dout]
        for k in range(6):
            gw, gb = cnn.conv3x3_weight_grad(inputs[k], douts[k])
            aw, ab = cnn.conv3x3_weight_grad(np.abs(inputs[k]), np.abs(douts[k]))
            gref[k] += gw
            gabs[k] += aw
            if k == 5:  # the output bias sees the unrounded gradient
                gb, ab = np.array([du32[i].sum()]), np.array([np.abs(du32[i]).sum()])
            bref[k] += gb
            babs[k] += ab
    ref = cnn.pack(list(zip(gref, bref)))
    Sabs = cnn.pack(list(zip(gabs, babs)))
    err = np.abs(g - ref)
    assert np.all(err <= 2e-4 * Sabs + 1e-6), (shape, float(np.max(err - 2e-4 * Sabs)))


def test_backward_is_deterministic():
    theta, imgs, du_np = make((2, 40, 72), 2)
    net = Net(theta)
    b = torch.tensor(imgs, dtype=torch.float32, device=DEV)
    du = torch.tensor(du_np, dtype=torch.float32, device=DEV)
    _, acts = net.forward(b)
    g1, d1 = net.backward(b, acts, du)
    g2, d2 = net.backward(b, acts, du)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(d1, d2)


def test_band_height_does_not_change_results():
    """64 images of 512^2 run the 32-channel layers in 64-row bands (the grid
    then has 2048 workgroups), one image alone in 16-row bands: activations,
    output and input gradients of sampled images are bitwise the same (every
    output row sums its three input rows in the same order)."""
    theta, _, _ = make((1, 1, 1), 4)
    net = Net(theta)
    gen = torch.Generator(device=DEV).manual_seed(4)
    n, H, W = 64, 512, 512
    b = torch.rand(n, H, W, device=DEV, generator=gen)
    du = torch.randn(n, H, W, device=DEV, generator=gen)
    u, acts = net.forward(b)
    _, dacts = net.backward(b, acts, du)
    A = acts.view(torch.bfloat16).view(5, n, H, W, 32)
    D = dacts.view(torch.bfloat16).view(5, n, H, W, 32)
    for i in (0, 37, 63):
        bi, dui = b[i:i + 1].contiguous(), du[i:i + 1].contiguous()
        ui, ai = net.forward(bi)
        _, di = net.backward(bi, ai, dui)
        torch.cuda.synchronize()
        assert torch.equal(u[i], ui[0]), i
        assert torch.equal(A[:, i], ai.view(torch.bfloat16).view(5, 1, H, W, 32)[:, 0]), i
        assert torch.equal(D[:, i], di.view(torch.bfloat16).view(5, 1, H, W, 32)[:, 0]), i


def test_whole_network_close_to_fp64_oracle():
    """BF16 rounding of weights and activations against the unrounded FP64
    network: a loose sanity bound (rounding compounds over six layers)."""
    theta, imgs, _ = make((1, 48, 64), 3)
    net = Net(theta)
    b = torch.tensor(imgs, dtype=torch.float32, device=DEV)
    u, _ = net.forward(b)
    torch.cuda.synchronize()
    _, out = cnn.forward(theta, imgs[0])
    ref = imgs[0] + out
    got = u[0].double().cpu().numpy()
    assert np.linalg.norm(got - ref) <= 3e-2 * np.linalg.norm(out)


def test_adam_matches_oracle():
    r = rng_for(21, 9)
    n = 5000
    p0 = r.standard_normal(n)
    p = torch.tensor(p0, dtype=torch.float32, device=DEV)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    pr, mr, vr = p.double().cpu().numpy(), np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        g0 = r.standard_normal(n)
        g = torch.tensor(g0, dtype=torch.float32, device=DEV)
        ops.adam_step(p, m, v, g, t, lr=1e-3)
        pr, mr, vr = cnn.adam(pr, mr, vr, g0.astype(np.float32).astype(np.float64), t, lr=1e-3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(p.double().cpu().numpy(), pr, rtol=0, atol=2e-6)
    np.testing.assert_allclose(m.double().cpu().numpy(), mr, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(v.double().cpu().numpy(), vr, rtol=1e-5, atol=1e-9)


def test_squared_error_and_soft_threshold():
    r = rng_for(21, 10)
    n = 100003
    c0, t0 = r.standard_normal(n), r.standard_normal(n)
    c = torch.tensor(c0, dtype=torch.float32, device=DEV)
    t = torch.tensor(t0, dtype=torch.float32, device=DEV)
    g = torch.empty_like(c)
    loss = ops.sq_error(c, t, scale=0.5, grad=g)
    s = ops.soft_threshold(c, 0.3)
    torch.cuda.synchronize()
    c32, t32 = c.double().cpu().numpy(), t.double().cpu().numpy()
    rr = c32 - t32
    assert abs(loss.item() - float(rr @ rr)) <= 1e-6 * float(rr @ rr)
    np.testing.assert_allclose(g.double().cpu().numpy(), rr, rtol=1e-6, atol=1e-7)
    from oracle import fista as ofi
    np.testing.assert_allclose(s.double().cpu().numpy(), ofi.soft(c32, 0.3), rtol=1e-6,
                               atol=1e-7)
