"""Batched FISTA over many images of uneven size, depth, filter and PSF.

One plan (C ABI ``aw_batch_*``) covers all problems; an iteration is one
launch per (stage, kernel class) over a tile queue that spans every image of
that class, with independent classes on forked streams. The iteration is
captured once into a hipGraph (``torch.cuda.CUDAGraph``) and replayed, so the
host issues one graph launch per FISTA iteration. ``autotune`` picks the
tile-shape variants and stream count by timing graph replays and caches the
choice per device.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
from typing import Sequence

import torch

from . import _lib, ops
from ._lib import check, load

CONFIG_DEFAULT = (0, 2, 0, 4)


def _cache_path() -> str:
    base = os.environ.get("ADJWAVE_CACHE_DIR",
                          os.path.join(os.path.expanduser("~"), ".cache", "adjwave"))
    return os.path.join(base, "autotune.json")


class BatchedFista:
    """FISTA for problems i = 0..n-1: min 1/2 ||R_i W_i x_i - b_i||^2 + lam ||x_i||_1.

    specs: list of (WaveletSpec, BlurSpec) pairs; b_obs: list of [rows_i, cols_i]
    FP32 device tensors. State lives in three concatenated device buffers
    (images B, coefficients X and Y) plus one workspace.
    """

    def __init__(self, specs: Sequence, b_obs: Sequence[torch.Tensor], lam: float,
                 L: float = 1.0):
        lib = load()
        self.n = len(specs)
        if self.n != len(b_obs) or self.n == 0:
            raise ValueError("one observation per problem")
        self.specs = list(specs)
        W = (_lib.Wavelet * self.n)()
        B = (_lib.Blur * self.n)()
        for i, (w, b) in enumerate(specs):
            W[i] = w._c
            B[i] = b._c
        plan = ctypes.c_void_p()
        check("aw_batch_create", lib.aw_batch_create(self.n, W, B, ctypes.byref(plan)))
        self._plan = plan
        co = (ctypes.c_int64 * (self.n + 1))()
        io = (ctypes.c_int64 * (self.n + 1))()
        wsb = ctypes.c_size_t()
        check("aw_batch_layout", lib.aw_batch_layout(plan, co, io, ctypes.byref(wsb)))
        self.coef_off, self.img_off = list(co), list(io)
        dev = b_obs[0].device
        self.device = dev
        self.B = torch.empty(self.img_off[-1], dtype=torch.float32, device=dev)
        for i, b in enumerate(b_obs):
            w = specs[i][0]
            if tuple(b.shape) != (w.rows, w.cols) or b.dtype != torch.float32:
                raise ValueError(f"problem {i}: expected float32 [{w.rows}, {w.cols}]")
            self.B[self.img_off[i]:self.img_off[i + 1]].copy_(b.reshape(-1))
        self.X = torch.zeros(self.coef_off[-1], dtype=torch.float32, device=dev)
        self.Y = torch.zeros_like(self.X)
        self.WS = torch.empty(max(wsb.value, 1), dtype=torch.uint8, device=dev)
        self.lam, self.L = float(lam), float(L)
        torch.cuda.synchronize(dev)
        check("aw_batch_bind", lib.aw_batch_bind(plan, ops._ptr(self.B), ops._ptr(self.X),
                                                 ops._ptr(self.Y), ops._ptr(self.WS), wsb.value,
                                                 self.lam, self.L))
        ctr, act, obj = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        check("aw_batch_control", lib.aw_batch_control(plan, ctypes.byref(ctr), ctypes.byref(act),
                                                       ctypes.byref(obj)))
        base = self.WS.data_ptr()
        self.counter = self.WS[ctr.value - base:ctr.value - base + 4].view(torch.int32)
        self.active = self.WS[act.value - base:act.value - base + 4 * self.n].view(torch.int32)
        self.obj = self.WS[obj.value - base:obj.value - base + 24 * self.n].view(
            torch.float64).view(self.n, 3)
        self.config = CONFIG_DEFAULT
        self._graph = None
        self._graph_stream = None
        self.reset()

    # ------------------------------------------------------------- control
    def __del__(self):
        try:
            # the captured graph goes before the plan: the plan owns the
            # auxiliary streams, events and device tables the graph was
            # captured with
            self._graph = None
            self._graph_stream = None
            if getattr(self, "_plan", None) is not None and self._plan.value:
                load().aw_batch_destroy(self._plan)
                self._plan = None
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def set_config(self, cfg) -> None:
        arr = (ctypes.c_int32 * 4)(*[int(v) for v in cfg])
        torch.cuda.synchronize(self.device)
        # drop the graph first: rebuilding the plan frees the device tables
        # its kernels were captured with
        self._graph = None
        self._graph_stream = None
        check("aw_batch_set_config", load().aw_batch_set_config(self._plan, arr))
        self.config = tuple(int(v) for v in cfg)

    def reset(self) -> None:
        """k = 1, all problems active, x = y = 0."""
        check("aw_batch_reset", load().aw_batch_reset(self._plan, self._stream()))

    def step(self) -> None:
        """One eager iteration (kernels launched from the host)."""
        check("aw_batch_step", load().aw_batch_step(self._plan, self._stream()))

    def capture(self) -> torch.cuda.CUDAGraph:
        """Capture one iteration into a graph (replayed by ``run``)."""
        torch.cuda.synchronize(self.device)
        s = torch.cuda.Stream(device=self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            check("aw_batch_step",
                  load().aw_batch_step(self._plan, ctypes.c_void_p(s.cuda_stream)))
        self._graph, self._graph_stream = g, s
        return g

    def run(self, iters: int, graph: bool = True) -> None:
        if graph:
            if self._graph is None:
                self.capture()
            for _ in range(iters):
                self._graph.replay()
        else:
            for _ in range(iters):
                self.step()

    # ----------------------------------------------------------- accessors
    def x(self, i: int) -> torch.Tensor:
        return self.X[self.coef_off[i]:self.coef_off[i + 1]]

    def y(self, i: int) -> torch.Tensor:
        return self.Y[self.coef_off[i]:self.coef_off[i + 1]]

    def set_active(self, i: int, on: bool) -> None:
        self.active[i].fill_(1 if on else 0)

    @property
    def npix(self) -> int:
        return self.img_off[-1]

    # ------------------------------------------------------------ autotune
    def signature(self) -> str:
        key = [(w.rows, w.cols, w.levels, w.taps, w.bc, b.radius) for w, b in self.specs]
        h = hashlib.sha1(json.dumps(sorted(key)).encode()).hexdigest()[:16]
        return f"{torch.cuda.get_device_name(self.device)}|{h}"

    def time_iters(self, iters: int = 5) -> float:
        """Average ms per graph-replayed iteration (state is reset first)."""
        self.reset()
        self.run(1, graph=True)
        torch.cuda.synchronize(self.device)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        self.run(iters, graph=True)
        e1.record()
        torch.cuda.synchronize(self.device)
        return e0.elapsed_time(e1) / iters

    def autotune(self, iters: int = 5, use_cache: bool = True) -> dict:
        """Coordinate search over (synthesis tile, analysis tile, blur tile,
        streams); the best configuration is applied and cached per device and
        problem set."""
        path = _cache_path()
        sig = self.signature()
        cache = {}
        if use_cache and os.path.exists(path):
            try:
                cache = json.load(open(path))
            except (OSError, ValueError):
                cache = {}
        if use_cache and sig in cache:
            self.set_config(cache[sig]["config"])
            return dict(cache[sig], cached=True)
        best = list(CONFIG_DEFAULT)
        self.set_config(best)
        best_ms = self.time_iters(iters)
        trials = [(tuple(best), best_ms)]
        for k, choices in ((0, (0, 1)), (1, (0, 1, 2, 3)), (2, (0, 1, 2)), (3, (1, 2, 4))):
            for v in choices:
                if v == best[k]:
                    continue
                cand = list(best)
                cand[k] = v
                self.set_config(cand)
                ms = self.time_iters(iters)
                trials.append((tuple(cand), ms))
                if ms < best_ms:
                    best, best_ms = cand, ms
        self.set_config(best)
        rec = {"config": list(best), "ms_per_iter": best_ms,
               "trials": [[list(c), m] for c, m in trials]}
        if use_cache:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            cache[sig] = rec
            tmp = path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, path)
        self.reset()
        return dict(rec, cached=False)
