"""Learned warm start for FISTA on eq. (1).

A six-layer 3x3 CNN (1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU, BF16
weights and activations, FP32 accumulation on MFMA) maps the blurred image b
to u = b + CNN(b); the start is x_0 = soft(W^dagger u, lambda / L), where
W^dagger is the wavelet analysis (the left inverse of the synthesis W). FISTA
from zero stays the fallback: x_0 is rejected when it is not finite or when
F(x_0) > F(0) = 1/2 ||b||^2.

Training minimises the mean of (W^dagger u - x*)^2 over pairs (b, x*) whose x*
comes from running this library's FISTA on b; the gradient reaches the image
through (W^dagger)^* and the network through its backward kernels, and Adam
updates FP32 master weights. Every step runs in the library's kernels; torch
holds device memory only.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np
import torch

from . import ops
from .batched import BatchedFista

LAYERS = [(1, 32)] + [(32, 32)] * 4 + [(32, 1)]


def init_params(seed: int, out_scale: float = 0.1) -> np.ndarray:
    """He-normal weights, zero biases; the output layer scaled down so the
    untrained network starts near u = b."""
    rng = np.random.default_rng((31, int(seed)))
    parts = []
    for k, (ci, co) in enumerate(LAYERS):
        w = rng.normal(0.0, math.sqrt(2.0 / (9.0 * ci)), size=co * ci * 9)
        parts += [w * (out_scale if k == len(LAYERS) - 1 else 1.0), np.zeros(co)]
    return np.concatenate(parts)


class WarmStartCNN:
    """FP32 master parameters with Adam state, and their packed BF16 copy."""

    def __init__(self, device="cuda:0", params: np.ndarray | None = None, seed: int = 0):
        self.device = torch.device(device)
        p = init_params(seed) if params is None else np.asarray(params)
        if p.size != ops.CNN_PARAMS:
            raise ValueError(f"{ops.CNN_PARAMS} parameters expected, got {p.size}")
        self.params = torch.tensor(p, dtype=torch.float32, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        pk, _, _ = ops.cnn_sizes(1, 1, 1)
        self.packed = torch.empty(pk, dtype=torch.uint8, device=self.device)
        self.grad = torch.zeros_like(self.params)
        self._bufs = {}
        self.pack()

    def pack(self) -> None:
        ops.cnn_pack(self.params, self.packed)

    def _buffers(self, n, H, W):
        key = (n, H, W)
        if key not in self._bufs:
            _, act, ws = ops.cnn_sizes(n, H, W)
            dev = self.device
            self._bufs[key] = {
                "acts": torch.empty(act, dtype=torch.uint8, device=dev),
                "dacts": torch.empty(act, dtype=torch.uint8, device=dev),
                "ws": torch.empty(ws, dtype=torch.uint8, device=dev),
                "u": torch.empty(n, H, W, dtype=torch.float32, device=dev),
            }
        return self._bufs[key]

    def forward(self, b: torch.Tensor) -> torch.Tensor:
        """u = b + CNN(b) for b [n, H, W] (the activations are kept for backward)."""
        buf = self._buffers(*b.shape)
        return ops.cnn_forward(self.packed, b, buf["acts"], buf["u"])

    def backward(self, b: torch.Tensor, du: torch.Tensor) -> torch.Tensor:
        """Parameter gradient of <du, u> after forward(b)."""
        buf = self._buffers(*b.shape)
        return ops.cnn_backward(self.packed, b, buf["acts"], du, buf["dacts"], self.grad,
                                buf["ws"])

    def adam(self, lr: float) -> None:
        self.step += 1
        ops.adam_step(self.params, self.m, self.v, self.grad, self.step, lr)
        self.pack()

    # ------------------------------------------------------------ checkpoint
    def save(self, path: str, meta: dict | None = None) -> None:
        np.savez(path, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(), step=np.int64(self.step),
                 meta=np.array(json.dumps(meta or {})))

    @classmethod
    def load(cls, path: str, device="cuda:0") -> "WarmStartCNN":
        z = np.load(path, allow_pickle=False)
        net = cls(device, params=z["params"])
        net.m.copy_(torch.from_numpy(z["m"]))
        net.v.copy_(torch.from_numpy(z["v"]))
        net.step = int(z["step"])
        net.meta = json.loads(str(z["meta"]))
        return net


def warm_coefficients(net: WarmStartCNN, w: ops.WaveletSpec, b: torch.Tensor,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """c = W^dagger (b + CNN(b)) for b [n, H, W] -> [n, ncoef]."""
    return ops.wavelet_analysis(w, net.forward(b), out=out)


def warm_start(net: WarmStartCNN, w: ops.WaveletSpec, b: torch.Tensor, lam: float,
               L: float = 1.0, out: torch.Tensor | None = None) -> torch.Tensor:
    """x_0 = soft(W^dagger (b + CNN(b)), lambda / L), [n, ncoef]."""
    c = warm_coefficients(net, w, b, out=out)
    return ops.soft_threshold(c, lam / L, out=c)


def train_step(net: WarmStartCNN, w: ops.WaveletSpec, b: torch.Tensor, x_star: torch.Tensor,
               lr: float, loss: torch.Tensor | None = None) -> torch.Tensor:
    """One Adam step on mean (W^dagger u - x*)^2 over the batch; returns the
    summed squared error (FP64 device scalar) before the step."""
    n = b.shape[0]
    c = warm_coefficients(net, w, b)
    g = torch.empty_like(c)
    loss = ops.sq_error(c, x_star, scale=1.0 / c.numel(), grad=g, loss=loss)
    du = ops.wavelet_analysis_adjoint(w, g)
    net.backward(b, du.view(n, w.rows, w.cols))
    net.adam(lr)
    return loss


# --------------------------------------------------------------- problems
def problem_host(seed: int, start: int, count: int, rows: int, cols: int,
                 noise: float = 1e-3):
    """Host side of images start..start+count-1 of stream `seed`: clean image
    from the rectangle generator, sigma ~ U[1, 3], radius ceil(3 sigma), and
    the noise draw."""
    from workloads import gen_image, gen_noise, gen_warm_problem, rng_for

    out = []
    for i in range(start, start + count):
        rng = rng_for(seed, i)
        img = gen_image(rng, rows, cols)
        sigma, radius = gen_warm_problem(rng)
        out.append((img, sigma, radius, gen_noise(rng, (rows, cols), noise)))
    return out


def problem_upload(host, rows: int, cols: int, device):
    """b = R image + noise on the GPU for each host item; returns (b [n, H, W],
    blur specs)."""
    bs, blurs = [], []
    for img, sigma, radius, nz in host:
        bsp = ops.BlurSpec(rows, cols, sigma=sigma, radius=radius)
        x = torch.tensor(img, dtype=torch.float32, device=device)
        bs.append(ops.blur(bsp, x) + torch.tensor(nz, dtype=torch.float32, device=device))
        blurs.append(bsp)
    return torch.stack(bs), blurs


def problem_batch(seed: int, start: int, count: int, rows: int, cols: int, device,
                  noise: float = 1e-3):
    """Images start..start+count-1 of stream `seed` as (b [n, H, W], blur specs)."""
    return problem_upload(problem_host(seed, start, count, rows, cols, noise), rows, cols,
                          device)


def fista_targets(w: ops.WaveletSpec, blurs, b: torch.Tensor, lam: float, iters: int,
                  out: torch.Tensor) -> None:
    """out[i] = x_iters of FISTA from zero on problem i (batched uneven plan)."""
    bf = BatchedFista([(w, bsp) for bsp in blurs], list(b), lam)
    bf.run(iters, graph=True)
    out.copy_(bf.X.view(len(blurs), -1))


def log(msg: str) -> None:
    """Progress line on stderr (stdout stays free for results)."""
    print(f"[warm-start {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def make_pairs(w: ops.WaveletSpec, n: int, lam: float, iters: int, seed: int, device,
               chunk: int = 64):
    """Training pairs (b [n, H, W], x* [n, ncoef]) resident on the device."""
    B = torch.empty(n, w.rows, w.cols, dtype=torch.float32, device=device)
    X = torch.empty(n, w.ncoef, dtype=torch.float32, device=device)
    t0 = time.time()
    host = problem_host(seed, 0, min(chunk, n), w.rows, w.cols)
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        b, blurs = problem_upload(host, w.rows, w.cols, device)
        B[s:s + c].copy_(b)
        fista_targets(w, blurs, b, lam, iters, X[s:s + c])
        # the next chunk's images are drawn on the host while the GPU iterates
        if s + c < n:
            host = problem_host(seed, s + c, min(chunk, n - s - c), w.rows, w.cols)
        if (s // chunk) % 8 == 0:
            torch.cuda.synchronize(device)
            log(f"pairs {s + c}/{n} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize(device)
    return B, X


def train(net: WarmStartCNN, w: ops.WaveletSpec, B: torch.Tensor, X: torch.Tensor,
          epochs: int, batch: int, lr: float, lr_min: float, seed: int = 0):
    """Adam over shuffled minibatches with a cosine learning-rate decay;
    returns the mean training loss of each epoch."""
    n = B.shape[0]
    steps = epochs * (n // batch)
    rng = np.random.default_rng((32, seed))
    loss = torch.zeros(1, dtype=torch.float64, device=B.device)
    hist = []
    k = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(B.device)
        acc = torch.zeros(1, dtype=torch.float64, device=B.device)
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * k / max(1, steps)))
            train_step(net, w, B[idx].contiguous(), X[idx].contiguous(), cur, loss=loss)
            acc += loss
            k += 1
        mean = acc.item() / ((n // batch) * batch * w.ncoef)
        hist.append(mean)
        log(f"epoch {ep + 1}/{epochs}: mean sq error {mean:.4e} ({time.time() - t0:.1f} s)")
    return hist


# -------------------------------------------------------------- evaluation
def _objectives(w, blurs, b, X, lam, out):
    for i, bsp in enumerate(blurs):
        ops.objective(w, bsp, b[i], X[i], lam, out=out[i:i + 1])
    return out


def objective_curve(bf: BatchedFista, w, blurs, b, lam, x0, iters: int, every: int):
    """FISTA from x0 ([n, ncoef], or None for zero) for `iters` iterations,
    graph-replayed `every` at a time; returns the exact objectives F(x_k) at
    k = every, 2 every, ... as an array [iters // every, n]."""
    n = len(blurs)
    bf.reset()
    if x0 is not None:
        bf.X.view(n, -1).copy_(x0)
        bf.Y.copy_(bf.X)
    obj = torch.empty(n, 3, dtype=torch.float64, device=b.device)
    X = bf.X.view(n, -1)
    out = []
    for _ in range(iters // every):
        bf.run(every, graph=True)
        out.append(_objectives(w, blurs, b, X, lam, obj)[:, 2].cpu().numpy().copy())
    return np.array(out)


def first_hits(curve: np.ndarray, F_star: np.ndarray, tol: float, every: int):
    """Per image, the first checked k with (F(x_k) - F*) / F* <= tol (-1: never)."""
    rel = (curve - F_star[None, :]) / F_star[None, :]
    ok = rel <= tol
    return [int(every * (np.argmax(ok[:, i]) + 1)) if ok[:, i].any() else -1
            for i in range(curve.shape[1])]


def choose_starts(w, blurs, b, x0: torch.Tensor, lam: float):
    """The fallback rule per image: keep x_0 if finite with F(x_0) <= F(0)."""
    n = len(blurs)
    obj = _objectives(w, blurs, b, x0, lam, torch.empty(n, 3, dtype=torch.float64,
                                                          device=b.device))
    F0 = 0.5 * (b.double() ** 2).sum(dim=(1, 2))
    ok = torch.isfinite(obj[:, 2]) & (obj[:, 2] <= F0)
    x0 = torch.where(ok[:, None], x0, torch.zeros_like(x0))
    return x0, ok


def timed_run(bf: BatchedFista, w, blurs, b, lam: float, F_star: np.ndarray, tol: float,
              every: int, max_iters: int, net: WarmStartCNN | None = None, k0: int = 1):
    """FISTA on the batch until every problem reaches (F(x_k) - F*) / F* <= tol,
    converged problems dropping out: every `every` iterations the exact
    objective of each active problem is evaluated, and a problem at or below
    tol is frozen (its tiles skip from then on). With `net`, the start is the
    network's (fallback rule applied) and the momentum sequence starts at
    k0; the start is computed inside the timed region. Returns the first
    checked k of each problem (-1: not within max_iters), the wall time, and
    the fallback flags."""
    n = len(blurs)
    dev = b.device
    obj = torch.empty(n, 3, dtype=torch.float64, device=dev)
    X = bf.X.view(n, -1)
    bf.reset()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    ok = None
    if net is not None:
        x0, ok = choose_starts(w, blurs, b, warm_start(net, w, b, lam), lam)
        X.copy_(x0)
        bf.Y.copy_(bf.X)
        if k0 > 1:
            bf.counter.fill_(k0)
    hits = [-1] * n
    active = list(range(n))
    k = 0
    while active and k < max_iters:
        bf.run(every, graph=True)
        k += every
        for i in active:
            ops.objective(w, blurs[i], b[i], X[i], lam, out=obj[i:i + 1])
        F = obj[:, 2].cpu().numpy()
        still = []
        for i in active:
            if (F[i] - F_star[i]) / F_star[i] <= tol:
                hits[i] = k
                bf.set_active(i, False)
            else:
                still.append(i)
        active = still
    torch.cuda.synchronize(dev)
    dt = time.perf_counter() - t0
    for i in range(n):
        bf.set_active(i, True)
    return hits, dt, ok


def evaluate(net: WarmStartCNN, w: ops.WaveletSpec, n: int, lam: float, seed: int, device,
             tol: float = 1e-4, star_iters: int = 60000, max_iters: int = 40000,
             every: int = 100, chunk: int = 64, k0: int = 1):
    """Plain versus warm FISTA on n fresh images, `chunk` images per batched
    plan. F* of each image is the lowest exact objective over a
    star_iters-iteration plain run (checked every 1000). Each arm then runs
    with converged images dropping out (timed_run): per image, the first k
    (checked every `every`) with (F(x_k) - F*) / F* <= tol, and per batch the
    wall time until its last image gets there (warm: the CNN, the analysis,
    the threshold and the fallback check included)."""
    res = {"plain_iters": [], "warm_iters": [], "plain_s": [], "warm_s": [],
           "fallbacks": 0, "images": 0, "every": every, "tol": tol, "k0": k0,
           "star_iters": star_iters, "max_iters": max_iters, "chunk": chunk}
    for s in range(0, n, chunk):
        c = min(chunk, n - s)
        b, blurs = problem_batch(seed, s, c, w.rows, w.cols, device)
        bf = BatchedFista([(w, bsp) for bsp in blurs], list(b), lam)
        star = objective_curve(bf, w, blurs, b, lam, None, star_iters, 1000)
        F_star = star.min(axis=0)
        p_hit, p_s, _ = timed_run(bf, w, blurs, b, lam, F_star, tol, every, max_iters)
        w_hit, w_s, ok = timed_run(bf, w, blurs, b, lam, F_star, tol, every, max_iters, net=net,
                                   k0=k0)
        res["plain_iters"] += p_hit
        res["warm_iters"] += w_hit
        res["plain_s"].append(p_s)
        res["warm_s"].append(w_s)
        res["fallbacks"] += int((~ok).sum().item())
        res["images"] += c
        del bf
        log(f"eval {s + c}/{n}: plain {p_s:.2f} s (median {np.median(p_hit):.0f} it, "
            f"{sum(h < 0 for h in p_hit)} not reached), warm {w_s:.2f} s (median "
            f"{np.median(w_hit):.0f} it, {sum(h < 0 for h in w_hit)} not reached)")
    return res


def main(argv=None) -> int:
    import argparse
    import os

    ap = argparse.ArgumentParser(description="train and evaluate the warm-start CNN")
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--fista-iters", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-min", type=float, default=2e-5)
    ap.add_argument("--eval-images", type=int, default=1000)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--star-iters", type=int, default=60000)
    ap.add_argument("--max-iters", type=int, default=40000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--k0", type=int, default=1)
    ap.add_argument("--eval-only", metavar="CKPT", default=None,
                    help="evaluate an existing checkpoint instead of training")
    ap.add_argument("--out", required=True, help="directory for the checkpoint and report")
    a = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    lam = 2e-5
    w = ops.WaveletSpec(a.size, a.size, 4, taps=8, bc="sym")
    os.makedirs(a.out, exist_ok=True)
    if a.eval_only:
        net = WarmStartCNN.load(a.eval_only, dev)
        meta = dict(net.meta)
        meta.pop("eval", None)
        meta.pop("eval_per_image", None)
    else:
        t0 = time.time()
        B, X = make_pairs(w, a.pairs, lam, a.fista_iters, seed=40 + a.seed, device=dev)
        t_data = time.time() - t0
        net = WarmStartCNN(dev, seed=a.seed)
        t0 = time.time()
        hist = train(net, w, B, X, a.epochs, a.batch, a.lr, a.lr_min, seed=a.seed)
        t_train = time.time() - t0
        del B, X
        torch.cuda.empty_cache()
        meta = {"pairs": a.pairs, "fista_iters": a.fista_iters, "epochs": a.epochs,
                "batch": a.batch, "lr": a.lr, "lr_min": a.lr_min, "size": a.size, "lambda": lam,
                "wavelet": "db4 J=4 sym", "seed": a.seed, "train_loss": hist,
                "data_s": round(t_data, 1), "train_s": round(t_train, 1)}
    if a.eval_images > 0:
        res = evaluate(net, w, a.eval_images, lam, seed=50 + a.seed, device=dev,
                       star_iters=a.star_iters, max_iters=a.max_iters, every=a.every, k0=a.k0)
        meta["eval"] = summarize(res)
        meta["eval_per_image"] = {"plain_iters": res["plain_iters"],
                                  "warm_iters": res["warm_iters"],
                                  "plain_batch_s": res["plain_s"], "warm_batch_s": res["warm_s"]}
    net.meta = meta
    net.save(os.path.join(a.out, f"warmstart_db4_J4_{a.size}.npz"), meta)
    with open(os.path.join(a.out, f"warmstart_db4_J4_{a.size}.json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(json.dumps(meta.get("eval")))
    return 0


def summarize(res: dict) -> dict:
    """Per-image iteration counts (unreached images counted at the cap) and
    the summed batch wall times of both arms."""
    cap = res["max_iters"]
    p = np.array(res["plain_iters"], dtype=float)
    q = np.array(res["warm_iters"], dtype=float)
    pc, qc = np.where(p > 0, p, cap), np.where(q > 0, q, cap)
    both = (p > 0) & (q > 0)
    return {"images": res["images"], "fallbacks": res["fallbacks"], "tol": res["tol"],
            "checked_every": res["every"], "star_iters": res["star_iters"], "max_iters": cap,
            "k0": res["k0"], "chunk": res["chunk"],
            "plain_iters_mean_capped": float(pc.mean()), "warm_iters_mean_capped": float(qc.mean()),
            "plain_iters_median": float(np.median(pc)), "warm_iters_median": float(np.median(qc)),
            "plain_iters_p90": float(np.percentile(pc, 90)),
            "warm_iters_p90": float(np.percentile(qc, 90)),
            "reached_both": int(both.sum()),
            "plain_iters_mean_both": float(p[both].mean()) if both.any() else None,
            "warm_iters_mean_both": float(q[both].mean()) if both.any() else None,
            "warm_fewer_iters_frac": float(np.mean(qc < pc)),
            "unreached_plain": int(np.sum(p < 0)), "unreached_warm": int(np.sum(q < 0)),
            "plain_total_s": float(np.sum(res["plain_s"])),
            "warm_total_s": float(np.sum(res["warm_s"])),
            "warm_over_plain_time": float(np.sum(res["warm_s"]) / np.sum(res["plain_s"]))}


if __name__ == "__main__":
    raise SystemExit(main())
