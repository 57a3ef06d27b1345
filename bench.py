"""Benchmark: FISTA on eq. (1) at 2048 x 2048 on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--bc sym|per|zpd]

A step is one FISTA iteration (one A = R W and one A^* = W^* R^*
application plus the proximal/momentum update) on a 2048 x 2048 FP32 image:
4-level Daubechies-4 W with symmetric boundaries, 15 x 15 Gaussian PSF
(sigma = 3) with reflexive boundaries, lambda = 2e-5, synthetic
rectangles-plus-gradient image with N(0, 1e-3^2) noise. The headline value is
image Mpix per second through A and A^* (one of each per step).

The roofline reported is the whole iteration's: its algorithmic bytes
(4 (5 ncoef + 3 npix)) over the step time from HIP events on the launching
stream, with the Infinity Cache warm (the 2048^2 working set stays in it)
and, beside it, the same step streaming from HBM (12 problems in rotation).

Also reported: Mpix/s of W, W^*, R, R^*, A, A^* alone (graph-replayed, HIP
events, hot and streaming from HBM), standalone single-kernel
microbenchmarks against 8 TB/s, the time to reach a 1e-4 relative objective
measured end to end, the extra workloads (uneven batch, autograd, the
convolution pair, the learned warm start, R through the DCT, the adjoint
study, blind channel estimation), and the FP64 CPU oracle timed on bounded
samples of the same workloads (host CPU model and core count recorded).

Profiling modes: --only-step K runs K FISTA steps only; --trace-summary and
--pmc-summary turn rocprofv3 output of such a run into the per-launch table
and the step traffic record kept under profiles/.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s for A and A* at 2048²; FISTA time-to-1e-4 rel objective, plain vs warm"
HBM_PEAK_GBS = 8000.0
COPY_REF_BYTES = 256 << 20  # read (and again written) by the --copy-reference kernel


# The eight launches of one FISTA step at 2048^2 (db4, J = 4, sym), in
# launch order: what each reads and writes (FP32 values), from the layout
# sizes K_j (rows = cols): the kernel-level algorithmic bytes.
STEP_KERNELS = ["synth_chain (W levels 4..2)", "synth_level (W level 1)", "blur (R y - b)",
                "blur (R^*)", "ana_prox level 1 (W^* + update)", "ana_prox level 2",
                "ana_prox level 3", "ana_prox level 4 (+ a_4)"]
STEP_SOURCES = ["wavelet.hip", "blur.hip", "api.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_fista2048_sym.md")


def step_kernel_bytes(sr, sc, npix: int, ncoef: int) -> list:
    """Algorithmic bytes of each step launch: every input read once, every
    output written once (intermediates between launches included)."""
    k = [sr[j] * sc[j] for j in range(len(sr))]
    J = len(sr) - 1
    coarse = ncoef - 3 * k[1]  # y's coefficients of levels 2..J and a_J
    out = [coarse + k[1],                    # chain: y levels >= 2 in, a_1 out
           4 * k[1] + npix,                  # level 1: a_1 and y's three bands in, image out
           3 * npix,                         # R y - b: image, b in, r out
           2 * npix,                         # R^*: r in, g out
           npix + 12 * k[1] + k[1]]          # level-1 analysis: g in; x, y of 3 bands in+out; a_1 out
    for j in range(2, J + 1):
        bands = 4 if j == J else 3
        out.append(k[j - 1] + 4 * bands * k[j] + (0 if j == J else k[j]))
    return [4 * v for v in out]


def source_hash(names) -> str:
    """Hash of kernel sources and every internal header they can include."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1707_02018_amd", "csrc")
    h = hashlib.sha256()
    for f in list(names) + sorted(x for x in os.listdir(csrc) if x.endswith(".hpp")):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _step_dispatches(rows, name_key, steps: int):
    """Library dispatches of a --only-step run in dispatch order, the first
    (the blur that forms b) dropped, grouped per step: steps x 8 rows."""
    aw = sorted((r for r in rows if "aw::" in r[name_key]), key=lambda r: int(r["Dispatch_Id"]))
    aw = aw[1:]
    n = len(STEP_KERNELS)
    if len(aw) != steps * n:
        raise SystemExit(f"expected {steps * n} step dispatches, found {len(aw)}")
    return [aw[i * n:(i + 1) * n] for i in range(steps)]


def pmc_summary(fetch_csv: str, write_csv: str, steps: int) -> None:
    """HBM bytes per FISTA step from two rocprofv3 --pmc passes (FETCH_SIZE,
    then WRITE_SIZE) of `bench.py --only-step STEPS --copy-reference`: the
    counters of each step launch, scaled by what the same counters read for
    the known-size copy kernel."""
    import csv

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        return rows

    out = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        rows = load(path, counter)
        ref = [float(r["Counter_Value"]) for r in rows
               if "elementwise" in r["Kernel_Name"] and int(r["Grid_Size"]) == COPY_REF_BYTES // 16]
        factor = (COPY_REF_BYTES / 1024) / (sum(ref) / len(ref))
        groups = _step_dispatches(rows, "Kernel_Name", steps)
        per = [sum(float(g[i]["Counter_Value"]) for g in groups) / steps
               for i in range(len(STEP_KERNELS))]
        out[counter] = (factor, per)
    ff, fk = out["FETCH_SIZE"]
    wf, wk = out["WRITE_SIZE"]
    per_kernel = [int(1024 * (f * ff + w * wf)) for f, w in zip(fk, wk)]
    rec = {"unit": "fista_step_2048_db4_J4_sym", "steps": steps,
           "fetch_factor": round(ff, 5), "write_factor": round(wf, 5),
           "fetch_kib": [round(v, 1) for v in fk], "write_kib": [round(v, 1) for v in wk],
           "bytes_per_kernel": per_kernel, "bytes_per_step": sum(per_kernel),
           "sources": STEP_SOURCES, "source_sha": source_hash(STEP_SOURCES)}
    print("step-traffic-record: " + json.dumps(rec))


def step_traffic():
    """HBM bytes per FISTA step from the committed counter summary, or None
    when there is none or a kernel source changed since it was taken."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        if ln.startswith("step-traffic-record: "):
            rec = json.loads(ln[len("step-traffic-record: "):])
            if rec["source_sha"] == source_hash(rec["sources"]):
                return rec
    return None


def trace_summary(trace_csv: str, steps: int, N: int = 2048) -> None:
    """Per-launch table of the FISTA step from a rocprofv3 kernel trace of
    `bench.py --only-step STEPS`: average duration of each of the eight
    launches and its kernel-level algorithmic bytes against 8 TB/s."""
    import csv

    from paper_1707_02018_amd import ops
    rows = list(csv.DictReader(open(trace_csv)))
    groups = _step_dispatches(rows, "Kernel_Name", steps)
    w = ops.WaveletSpec(N, N, 4, taps=8, bc="sym")
    _, sr, sc = w.layout()
    kb = step_kernel_bytes(sr, sc, N * N, w.ncoef)
    total_us = 0.0
    print("| # | launch | kernel | workgroups | avg us | bytes (MB) | TB/s | of 8 TB/s |")
    print("|---|---|---|---|---|---|---|---|")
    for i, name in enumerate(STEP_KERNELS):
        d = [(int(g[i]["End_Timestamp"]) - int(g[i]["Start_Timestamp"])) / 1e3 for g in groups]
        us = sum(d) / len(d)
        total_us += us
        r0 = groups[0][i]
        wg = (int(r0["Grid_Size_X"]) // int(r0["Workgroup_Size_X"])) * int(r0["Grid_Size_Y"])
        kern = r0["Kernel_Name"].split("(")[0].replace("void ", "")
        print(f"| {i + 1} | {name} | `{kern}` | {wg} | {us:.2f} | {kb[i] / 1e6:.2f} | "
              f"{kb[i] / us / 1e6:.2f} | {100 * kb[i] / us / 1e6 / 8:.1f} % |")
    alg = 4 * (5 * w.ncoef + 3 * N * N)
    print(f"\nSum of the launches: {total_us:.2f} us per step; the iteration's algorithmic "
          f"bytes (4 (5 ncoef + 3 npix) = {alg / 1e6:.1f} MB) over it: "
          f"{alg / total_us / 1e6:.2f} TB/s, {100 * alg / total_us / 1e6 / 8:.1f} % of 8 TB/s.")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--bc", default="sym", choices=["sym", "per", "zpd"])
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-target", action="store_true", help="skip the time-to-1e-4 run")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, autograd and convolution-pair sections")
    ap.add_argument("--batched-iters", type=int, default=300)
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the uneven-batch section and print its JSON (for profiling)")
    ap.add_argument("--only-conv", action="store_true",
                    help="run only the convolution-pair section and print its JSON (for profiling)")
    ap.add_argument("--only-autograd", action="store_true",
                    help="run only the autograd A section and print its JSON (for profiling)")
    ap.add_argument("--only-cnn", action="store_true",
                    help="run only the warm-start CNN timing and print its JSON (for profiling)")
    ap.add_argument("--only-large", action="store_true",
                    help="level-1 W, W*, R, R* and update at 4 x 4096^2, streaming from HBM")
    ap.add_argument("--large-summary", nargs=3, metavar=("TRACE_CSV", "FETCH_CSV", "WRITE_CSV"),
                    help="per-kernel table of --only-large --copy-reference runs")
    ap.add_argument("--only-dct", action="store_true",
                    help="run only the DCT-II blur section and print its JSON (for profiling)")
    ap.add_argument("--warm-images", type=int, default=16)
    ap.add_argument("--only-step", type=int, default=0, metavar="STEPS",
                    help="run only STEPS FISTA steps at the bench size (for profiler passes)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "STEPS"),
                    help="print the step traffic record from two rocprofv3 --pmc counter CSVs "
                         "(FETCH_SIZE, WRITE_SIZE) of --only-step STEPS --copy-reference, then exit")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_CSV", "STEPS"),
                    help="print the per-launch step table from a rocprofv3 kernel trace of "
                         "--only-step STEPS, then exit")
    ap.add_argument("--cpu-leg", action="store_true",
                    help="(internal) run the oracle legs of the CPU baseline and print JSON")
    ap.add_argument("--copy-reference", action="store_true",
                    help="first run a plain 256 MiB copy kernel (x * 1 into y) three times, "
                         "the known-size reference for hardware byte counters")
    return ap.parse_args()


def bench_batched(torch, ops, iters: int) -> dict:
    """64 FP32 images, sides from {512, ..., 4096} per axis, levels {3,4,5},
    filters {Haar, db4, db8}, PSF sigma U[1,4] with radius ceil(3 sigma),
    symmetric boundaries; autotuned tile variants; graph-replayed iterations."""
    from paper_1707_02018_amd.batched import BatchedFista
    from workloads import gen_batched_config, gen_image, rng_for
    dev = torch.device("cuda:0")
    cfg = gen_batched_config(rng_for(3, 0), 64)
    specs, obs = [], []
    for i, c in enumerate(cfg):
        w = ops.WaveletSpec(c["rows"], c["cols"], c["levels"], taps=c["taps"], bc="sym")
        b = ops.BlurSpec(c["rows"], c["cols"], sigma=c["sigma"], radius=c["radius"])
        rng = rng_for(3, 1000 + i)
        img = torch.tensor(gen_image(rng, c["rows"], c["cols"]), dtype=torch.float32, device=dev)
        noise = torch.randn(c["rows"], c["cols"], device=dev,
                            generator=torch.Generator(device=dev).manual_seed(i)) * 1e-3
        obs.append(ops.blur(b, img) + noise)
        specs.append((w, b))
    bf = BatchedFista(specs, obs, 2e-5)
    del obs
    tune = bf.autotune(iters=3, use_cache=False)
    bf.reset()
    bf.run(2, graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    bf.run(iters, graph=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    bf.reset()
    bf.run(2, graph=False)
    torch.cuda.synchronize()
    e0.record()
    bf.run(20, graph=False)
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / 20
    npix, ncoef = bf.img_off[-1], bf.coef_off[-1]
    alg = 4 * (5 * ncoef + 3 * npix)  # y, x_prev, x_k, y_{k+1} coefficients; b, r images
    return {"images": 64, "total_mpix": round(npix / 1e6, 2), "iterations": iters,
            "ms_per_iter_graph": round(ms, 3), "ms_per_iter_eager": round(ms_eager, 3),
            "mpix_iter_per_s": round(npix / (ms * 1e-3) / 1e6, 1),
            "algorithmic_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
            "autotune": {"config": tune["config"], "trials": tune["trials"]}}


LARGE_N, LARGE_BATCH, LARGE_SETS, LARGE_ROUNDS = 4096, 4, 3, 5
LARGE_OPS = ["W_level1", "W*_level1", "R", "R*", "W*prox_level1"]


def large_bytes(ops) -> dict:
    """Algorithmic bytes per launch of the level-1 operators on 4 x 4096^2
    (db4, sym, one level): inputs read once, outputs written once (FP32)."""
    w1 = ops.WaveletSpec(LARGE_N, LARGE_N, 1, taps=8, bc="sym")
    _, sr, sc = w1.layout()
    npix, k1 = LARGE_N * LARGE_N, sr[1] * sc[1]
    b = LARGE_BATCH
    return {"W_level1": 4 * b * (w1.ncoef + npix), "W*_level1": 4 * b * (npix + w1.ncoef),
            "R": 8 * b * npix, "R*": 8 * b * npix, "W*prox_level1": 4 * b * (npix + 16 * k1)}


def bench_large(torch, ops) -> dict:
    """Level-1 synthesis, analysis (W^*), R, R^* (radius 7) and the level-1
    FISTA update on 4 x 4096^2 FP32 (db4, sym), each launch streaming from HBM:
    inputs and outputs rotated over LARGE_SETS buffer sets of about 1.3 GB,
    LARGE_ROUNDS rounds after one untimed round, HIP events on the stream."""
    import ctypes
    from paper_1707_02018_amd import _lib
    lib = _lib.load()
    dev = torch.device("cuda:0")
    N, B = LARGE_N, LARGE_BATCH
    w1 = ops.WaveletSpec(N, N, 1, taps=8, bc="sym")
    bsp = ops.BlurSpec(N, N, sigma=3.0, radius=7)
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    P = ops._ptr
    wsn = ops.workspace_bytes(w1, bsp, torch.float32, B)
    ws = torch.empty(max(wsn, 1), dtype=torch.uint8, device=dev)
    g = torch.Generator(device=dev).manual_seed(5)
    sets = []
    for _ in range(LARGE_SETS):
        st = _lib.FistaState()
        x = torch.randn(B, w1.ncoef, device=dev, generator=g) * 1e-2
        y = torch.randn(B, w1.ncoef, device=dev, generator=g) * 1e-2
        st.x, st.y, st.resid, st.obj = x.data_ptr(), y.data_ptr(), None, None
        st.k, st.t, st.gradient = 1, 1.0, 0
        sets.append({"coef": torch.randn(B, w1.ncoef, device=dev, generator=g) * 1e-2,
                     "img": torch.randn(B, N, N, device=dev, generator=g),
                     "oimg": torch.empty(B, N, N, device=dev),
                     "ocoef": torch.empty(B, w1.ncoef, device=dev), "x": x, "y": y, "st": st})
    calls = {
        "W_level1": lambda s: lib.wavelet_synth(w1.c, 0, B, P(s["coef"]), P(s["oimg"]), P(ws),
                                                wsn, sp),
        "W*_level1": lambda s: lib.wavelet_synth_adjoint(w1.c, 0, B, P(s["img"]), P(s["ocoef"]),
                                                         P(ws), wsn, sp),
        "R": lambda s: lib.blur(bsp.c, 0, B, P(s["img"]), P(s["oimg"]), sp),
        "R*": lambda s: lib.blur_adjoint(bsp.c, 0, B, P(s["img"]), P(s["oimg"]), sp),
        "W*prox_level1": lambda s: lib.aw_fista_update(w1.c, 0, B, P(s["img"]), 1.0, 2e-5,
                                                       ctypes.byref(s["st"]), 0, P(ws), wsn, sp),
    }
    byts = large_bytes(ops)
    out = {}
    for name in LARGE_OPS:
        fn = calls[name]
        for s_ in sets:
            assert fn(s_) == 0, name
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(LARGE_ROUNDS):
            for s_ in sets:
                fn(s_)
        e1.record(stream)
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / (LARGE_ROUNDS * LARGE_SETS)
        out[name] = {"us": round(us, 2), "GBps": round(byts[name] / us / 1e3, 1),
                     "frac": round(byts[name] / us / 1e6 / 8.0, 4)}
    return {"workload": f"{B}x{N}^2 FP32, db4 sym, one level, PSF radius 7",
            "cache": "each launch streams from HBM (buffer sets rotated)", "ops": out}


def large_summary(trace_csv: str, fetch_csv: str, write_csv: str) -> None:
    """Per-kernel table of a `--only-large --copy-reference` run: average
    duration from a rocprofv3 kernel trace, HBM bytes from FETCH_SIZE and
    WRITE_SIZE passes scaled by the copy kernel's counters, against the
    algorithmic bytes."""
    import csv

    from paper_1707_02018_amd import ops

    def launches(path):
        rows = [r for r in csv.DictReader(open(path)) if "aw::" in r["Kernel_Name"]]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    per = LARGE_SETS * (LARGE_ROUNDS + 1)
    trace = launches(trace_csv)
    if len(trace) != per * len(LARGE_OPS):
        raise SystemExit(f"expected {per * len(LARGE_OPS)} launches, found {len(trace)}")

    def factor(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        ref = [float(r["Counter_Value"]) for r in rows
               if "elementwise" in r["Kernel_Name"] and int(r["Grid_Size"]) == COPY_REF_BYTES // 16]
        return (COPY_REF_BYTES / 1024) / (sum(ref) / len(ref))

    def counts(path, counter):
        rows = [r for r in csv.DictReader(open(path))
                if r["Counter_Name"] == counter and "aw::" in r["Kernel_Name"]]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return [float(r["Counter_Value"]) for r in rows]

    ff, wf = factor(fetch_csv, "FETCH_SIZE"), factor(write_csv, "WRITE_SIZE")
    fk, wk = counts(fetch_csv, "FETCH_SIZE"), counts(write_csv, "WRITE_SIZE")
    byts = large_bytes(ops)
    print("| op | kernel | avg us | algorithmic MB | TB/s | of 8 TB/s | HBM MB (fetch + write) "
          "| HBM / algorithmic |")
    print("|---|---|---|---|---|---|---|---|")
    for k, name in enumerate(LARGE_OPS):
        sel = slice(k * per + LARGE_SETS, (k + 1) * per)  # the timed rounds
        rows = trace[sel]
        us = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows) / len(rows) / 1e3
        hbm = 1024 * (ff * sum(fk[sel]) + wf * sum(wk[sel])) / len(rows)
        kern = rows[0]["Kernel_Name"].split("(")[0].replace("void ", "")
        print(f"| {name} | `{kern}` | {us:.1f} | {byts[name] / 1e6:.1f} | "
              f"{byts[name] / us / 1e6:.2f} | {100 * byts[name] / us / 8e6:.1f} % | "
              f"{hbm / 1e6:.1f} | {hbm / byts[name]:.2f} |")
    print(f"\nFETCH_SIZE calibration {ff:.4f}, WRITE_SIZE {wf:.4f} (bytes of the "
          f"{COPY_REF_BYTES >> 20} MiB copy over the KiB counted).")


def bench_autograd(torch, ops) -> dict:
    """A = R W as an autograd Function, batch 16 of 1024 x 1024 FP32 (db4 J=4
    sym, sigma 2 PSF): forward + backward (backward = A^* kernel). The leaf's
    gradient is set to None before each backward, as a training loop's
    zero_grad(set_to_none=True) does, so backward writes it instead of adding
    into it."""
    from paper_1707_02018_amd import autograd as ag
    dev = torch.device("cuda:0")
    w = ops.WaveletSpec(1024, 1024, 4, taps=8, bc="sym")
    b = ops.BlurSpec(1024, 1024, sigma=2.0, radius=4)
    x = torch.randn(16, w.ncoef, device=dev, requires_grad=True)
    g = torch.randn(16, 1024, 1024, device=dev)
    for _ in range(3):
        x.grad = None
        ag.apply_A(x, w, b).backward(g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        x.grad = None
        ag.apply_A(x, w, b).backward(g)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"batch": 16, "image": [1024, 1024], "ms_fwd_bwd": round(ms, 3),
            "mpix_per_s_fwd_bwd": round(16 * 1024 * 1024 / (ms * 1e-3) / 1e6, 1)}


def bench_conv(torch, ops) -> dict:
    """Blind-channel pair: 256 pairs, s of length 65536, h of length 128, FP32."""
    dev = torch.device("cuda:0")
    B, K, N = 256, 128, 65536
    h = torch.randn(B, K, device=dev)
    s_ = torch.randn(B, N, device=dev)
    x = torch.randn(B, K + N - 1, device=dev)
    for _ in range(3):
        ops.conv_adjoint_pair(h, s_, x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record()
    for _ in range(reps):
        ops.conv_adjoint_pair(h, s_, x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = 2.0 * B * (K * N * 3)  # h*s, S^* r and H^* r: K N multiply-adds each
    return {"pairs": B, "K": K, "N": N, "ms": round(ms, 3),
            "GFLOPs": round(flops / (ms * 1e-3) / 1e9, 1),
            "frac_fp32_vector_peak_157T": round(flops / (ms * 1e-3) / 157.3e12, 4),
            # the kernels are built without packed FP32 instructions, whose
            # dual-issue the 157.3 TFLOP/s figure counts: one FMA per lane and
            # cycle gives half of it
            "frac_unpacked_fp32_78T": round(flops / (ms * 1e-3) / 78.65e12, 4)}


def bench_warm(torch, ops, n_images: int) -> dict:
    """Learned warm start against FISTA from zero on fresh 512^2 images
    (db4, J = 4, sym, PSF sigma ~ U[1, 3], lambda = 2e-5) with the committed
    checkpoint, in one batched plan with converged images dropping out:
    iterations to the 1e-4 relative objective per image (capped at 40,000)
    and the batch wall time until its last image gets there (warm: the CNN
    and the start included)."""
    from paper_1707_02018_amd import learned

    ckpt = os.path.join(ROOT, "paper_1707_02018_amd", "weights", "warmstart_db4_J4_512.npz")
    if not os.path.exists(ckpt):
        return {"skipped": "no checkpoint"}
    dev = torch.device("cuda:0")
    net = learned.WarmStartCNN.load(ckpt, dev)
    w = ops.WaveletSpec(512, 512, 4, taps=8, bc="sym")
    # CNN inference alone at the evaluation batch
    b, _ = learned.problem_batch(72, 0, n_images, 512, 512, dev)
    net.forward(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        learned.warm_start(net, w, b, 2e-5)
    torch.cuda.synchronize()
    cnn_ms = 1e3 * (time.perf_counter() - t0) / 10
    res = learned.evaluate(net, w, n_images, 2e-5, seed=72, device=dev, star_iters=60000,
                           max_iters=40000, every=100, chunk=n_images)
    s = learned.summarize(res)
    s["warm_start_map_ms"] = round(cnn_ms, 3)
    s["cnn_gflop_per_image"] = round(2 * 37440 * 512 * 512 / 1e9, 2)
    s["cnn_tflops"] = round(2 * 37440 * 512 * 512 * n_images / (cnn_ms * 1e-3) / 1e12, 1)
    s["training"] = {k: net.meta[k] for k in ("pairs", "fista_iters", "epochs", "batch")}
    s["training_eval"] = net.meta.get("eval")
    return s


def graph_us(torch, stream, fn, name: str, reps: int = 50) -> float:
    """Average us of one call of fn (library launches on `stream`), from a
    captured graph of `reps` calls replayed 4 times, HIP events on the stream."""
    for _ in range(3):
        assert fn() == 0, name
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(4):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    return 1e3 * e0.elapsed_time(e1) / (4 * reps)


def bench_cold(torch, ops, lib, w, w1, bsp, lam: float, stream, nsets: int = 12) -> dict:
    """The single operators with their inputs and outputs rotated over nsets
    distinct buffer sets (more than the 256 MB Infinity Cache holds), so each
    application streams from HBM: us per application (one graph of nsets x 4
    rounds, replayed 3 times, HIP events on the launching stream) and, for the
    level-1 update, its algorithmic GB/s against 8 TB/s."""
    import ctypes
    dev = torch.device("cuda:0")
    N = w.rows
    npix = N * N
    P = ops._ptr
    sp = ctypes.c_void_p(stream.cuda_stream)
    wsn = ops.workspace_bytes(w, bsp, torch.float32, 1)
    ws = torch.empty(wsn, dtype=torch.uint8, device=dev)
    coef = [torch.randn(w.ncoef, device=dev) * 1e-2 for _ in range(nsets)]
    img = [torch.randn(N, N, device=dev) for _ in range(nsets)]
    out_img = [torch.empty(N, N, device=dev) for _ in range(nsets)]
    out_coef = [torch.empty(w.ncoef, device=dev) for _ in range(nsets)]
    x1 = [torch.randn(w1.ncoef, device=dev) * 1e-2 for _ in range(nsets)]
    y1 = [torch.randn(w1.ncoef, device=dev) * 1e-2 for _ in range(nsets)]
    st1 = []
    for i in range(nsets):
        st = __import__("paper_1707_02018_amd._lib", fromlist=["FistaState"]).FistaState()
        st.x, st.y, st.resid, st.obj = x1[i].data_ptr(), y1[i].data_ptr(), None, None
        st.k, st.t, st.gradient = 1, 1.0, 0
        st1.append(st)
    ops_ = {
        "W": lambda i: lib.wavelet_synth(w.c, 0, 1, P(coef[i]), P(out_img[i]), P(ws), wsn, sp),
        "W*": lambda i: lib.wavelet_synth_adjoint(w.c, 0, 1, P(img[i]), P(out_coef[i]), P(ws),
                                                  wsn, sp),
        "R": lambda i: lib.blur(bsp.c, 0, 1, P(img[i]), P(out_img[i]), sp),
        "R*": lambda i: lib.blur_adjoint(bsp.c, 0, 1, P(img[i]), P(out_img[i]), sp),
        "A": lambda i: lib.aw_apply_A(w.c, bsp.c, 0, 1, P(coef[i]), P(out_img[i]), P(ws), wsn,
                                      sp),
        "A*": lambda i: lib.aw_apply_A_adjoint(w.c, bsp.c, 0, 1, P(img[i]), P(out_coef[i]),
                                               P(ws), wsn, sp),
        "W*prox_level1": lambda i: lib.aw_fista_update(w1.c, 0, 1, P(img[i]), 1.0, lam,
                                                       ctypes.byref(st1[i]), 0, P(ws), wsn, sp),
    }
    rounds = 4
    out = {}
    with torch.cuda.stream(stream):
        for name, fn in ops_.items():
            for i in range(nsets):
                assert fn(i) == 0, name
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                for _ in range(rounds):
                    for i in range(nsets):
                        fn(i)
            g.replay()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                g.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            out[name] = round(1e3 * e0.elapsed_time(e1) / (3 * rounds * nsets), 3)
    _, sr, sc = w1.layout()
    k1 = sr[1] * sc[1]
    ub = 4 * (npix + 16 * k1)
    gbs = ub / (out["W*prox_level1"] * 1e-6) / 1e9
    per_set = 4 * (2 * npix + 2 * w.ncoef + 2 * w1.ncoef)
    return {"buffer_sets": nsets, "bytes_rotated": nsets * per_set, "ops_us": out,
            "ops_mpix_s": {k: round(npix / v, 1) for k, v in out.items()},
            "roofline_update": {"op": "W*prox_level1", "algorithmic_bytes": ub,
                                "achieved": round(gbs, 1), "unit": "GB/s",
                                "frac": round(gbs / HBM_PEAK_GBS, 4)}}


def bench_step_cold(torch, ops, w, bsp, b, lam: float, nsets: int = 12, rounds: int = 4) -> dict:
    """The FISTA step over `nsets` independent problems stepped in rotation,
    each with its own b, x, y, residual and workspace (about 107 MB per
    problem at 2048^2, more than the 256 MB Infinity Cache in all), so every
    step streams its operands from HBM; HIP events on the launching stream."""
    states = []
    for _ in range(nsets):
        bi = b.clone()
        st = ops.FistaState(w, bsp, bi)
        for _ in range(3):
            ops.fista_step(st, bi, lam)
        states.append((st, bi))
    torch.cuda.synchronize()
    per_set = (2 * w.ncoef * 4 + 2 * b.numel() * 4 + states[0][0].ws_n)
    cur = torch.cuda.current_stream(b.device)
    for st, bi in states:
        ops.fista_step(st, bi, lam)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for _ in range(rounds):
        for st, bi in states:
            ops.fista_step(st, bi, lam)
    e1.record(cur)
    torch.cuda.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / (rounds * nsets)
    del states
    torch.cuda.empty_cache()
    return {"us_per_step": round(us, 3), "sets": nsets,
            "protocol": f"{nsets} independent 2048^2 problems (b, x, y, residual and workspace "
                        f"each; {nsets * per_set / 1e9:.2f} GB in all) stepped in rotation, "
                        f"{rounds} rounds, HIP events on the launching stream"}


def bench_time_to_target(torch, ops, w, bsp, b, lam: float, ms_per_step: float,
                         total: int = 20000, every: int = 20, check: int = 10) -> dict:
    """Plain FISTA from zero to a relative objective of 1e-4, measured end to
    end. F* is the lowest exact objective over `total` plain iterations
    (checked every `every`). A fresh run from zero then evaluates the exact
    objective every `check` iterations and stops at the first check at or
    below 1e-4; its wall time, objective passes and reads included, is the
    time to target."""
    dev = b.device
    st2 = ops.FistaState(w, bsp, b)
    obj = torch.empty(1, 3, dtype=torch.float64, device=dev)
    Fs = []
    for k in range(1, total + 1):
        ops.fista_step(st2, b, lam)
        if k % every == 0:
            ops.objective(w, bsp, b, st2.x, lam, out=obj)
            Fs.append((k, obj[0, 2].item()))
    F_star = min(F for _, F in Fs)
    del st2
    st3 = ops.FistaState(w, bsp, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k, hit = 0, None
    while k < total:
        for _ in range(check):
            ops.fista_step(st3, b, lam)
        k += check
        ops.objective(w, bsp, b, st3.x, lam, out=obj)
        if (obj[0, 2].item() - F_star) / F_star <= 1e-4:
            hit = k
            break
    dt = time.perf_counter() - t0
    return {"F_star": F_star, "F_star_from": f"min exact F over {total} plain iterations "
                                               f"(every {every})",
            "iters_to_1e-4": hit, "checked_every": check,
            "time_to_1e-4_ms": round(1e3 * dt, 3) if hit else None,
            "measured": f"end to end: wall time from x = 0 to the first check at or below 1e-4, "
                        f"one exact objective pass and one 8-byte read every {check} "
                        f"iterations included",
            "steps_only_ms": round(hit * ms_per_step, 3) if hit else None}


def bench_modes(torch, ops, lib, bsp, b, lam: float, modes, steps: int = 100) -> dict:
    """The same 2048^2 workload with the other boundary modes: FISTA step
    time and Mpix/s, and A, A^* per application."""
    import ctypes

    N = b.shape[-1]
    out = {}
    for bc in modes:
        w = ops.WaveletSpec(N, N, 4, taps=8, bc=bc)
        st = ops.FistaState(w, bsp, b)
        for _ in range(10):
            ops.fista_step(st, b, lam)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ops.fista_step(st, b, lam)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        x = torch.randn(w.ncoef, device=b.device) * 1e-2
        oi = torch.empty(N, N, device=b.device)
        oc = torch.empty(w.ncoef, device=b.device)
        wsn = ops.workspace_bytes(w, bsp, torch.float32, 1)
        ws = torch.empty(wsn, dtype=torch.uint8, device=b.device)
        stream = torch.cuda.Stream(device=b.device)
        sp = ctypes.c_void_p(stream.cuda_stream)
        P = ops._ptr
        with torch.cuda.stream(stream):
            a_us = graph_us(torch, stream, lambda: lib.aw_apply_A(
                w.c, bsp.c, 0, 1, P(x), P(oi), P(ws), wsn, sp), "A")
            at_us = graph_us(torch, stream, lambda: lib.aw_apply_A_adjoint(
                w.c, bsp.c, 0, 1, P(b), P(oc), P(ws), wsn, sp), "A*")
        out[bc] = {"ncoef": w.ncoef, "ms_per_step": round(ms, 4),
                   "mpix_s": round(N * N / (ms * 1e-3) / 1e6, 1),
                   "A_us": round(a_us, 3), "A*_us": round(at_us, 3)}
        del st, x, oi, oc, ws
    return out


def bench_cnn(torch, reps: int = 5) -> dict:
    """Warm-start CNN at batch 64 of 512^2 (random weights): forward and
    backward pass, ms per call from HIP events on the current stream."""
    from paper_1707_02018_amd import learned

    dev = torch.device("cuda:0")
    net = learned.WarmStartCNN(dev, seed=0)
    b = torch.rand(64, 512, 512, device=dev)
    du = torch.ones_like(b)
    for _ in range(2):
        net.forward(b)
        net.backward(b, du)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        net.forward(b)
    ev[1].record()
    for _ in range(reps):
        net.backward(b, du)
    ev[2].record()
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1]) / reps
    flop = 2.0 * 37440 * 512 * 512 * 64
    return {"batch": 64, "image": [512, 512], "forward_ms": round(fwd, 3),
            "backward_ms": round(ev[1].elapsed_time(ev[2]) / reps, 3),
            "forward_tflops": round(flop / (fwd * 1e-3) / 1e12, 1)}


def bench_blur_dct(torch, ops, lib, stream) -> dict:
    """R through the DCT-II (five passes, any radius) against the direct tile
    kernel (radius <= 12) at 2048^2, FP32, us per application (graph replay)."""
    import ctypes

    N = 2048
    dev = torch.device("cuda:0")
    x = torch.randn(N, N, device=dev)
    y = torch.empty_like(x)
    sp = ctypes.c_void_p(stream.cuda_stream)
    P = ops._ptr
    out = {}
    with torch.cuda.stream(stream):
        for r in (7, 12, 64, 512):
            taps = ops.gaussian_psf(max(r / 3.0, 1.0), r)
            plan = ops.BlurDCT(N, N, taps)
            n = ctypes.c_size_t()
            lib.aw_blur_dct_workspace(plan._plan, 1, ctypes.byref(n))
            ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
            us = graph_us(torch, stream, lambda: lib.aw_blur_dct_apply(
                plan._plan, 1, P(x), P(y), P(ws), n.value, sp), "R_dct")
            rec = {"dct_us": round(us, 3)}
            if r <= 12:
                b = ops.BlurSpec(N, N, taps=taps)
                rec["direct_us"] = round(graph_us(torch, stream, lambda: lib.blur(
                    b.c, 0, 1, P(x), P(y), sp), "R"), 3)
            out[f"r{r}"] = rec
            del plan, ws
    return out


def bench_adjoint_study() -> dict:
    """True adjoint W^* against W^dagger in the FISTA gradient, the paper's
    setting (three-level transform, sym, lambda = 2e-5, 2500 iterations) on a
    256^2 synthetic image: relative error, nonzero share and SSIM at the end."""
    from paper_1707_02018_amd import adjoint_study

    out = {}
    for taps, fam, name in ((2, "daubechies", "haar_J3_sym"), (8, "daubechies", "db4_J3_sym"),
                            (10, "cdf97", "cdf97_J3_sym")):
        r = adjoint_study.run(256, 256, taps, 3, "sym", 2.0, 4, 2e-5, 2500, every=500,
                              family=fam)
        out[name] = {"blurred": {k: round(v, 6) for k, v in r["blurred"].items()},
                     **{g: {k: round(r[g][k], 6)
                            for k in ("rel_err", "nonzero_pct", "ssim", "objective")}
                        for g in ("adjoint", "pinv")}}
    return out


def bench_blind() -> dict:
    """Two-channel blind estimation with the Huber TV term at the paper's sizes
    (K = 894, N = 1717, guessed 844 / 1767; synthetic sparse channels and an
    impulsive source, noise 0.005), FP32, up to 10,000 alternating iterations
    (stopping when the objective stalls), two problem seeds."""
    from paper_1707_02018_amd import blind

    def rnd(v):
        if isinstance(v, float):
            return round(v, 6)
        if isinstance(v, list):
            return [round(a, 4) for a in v]
        if isinstance(v, dict):
            return {kk: round(vv, 6) for kk, vv in v.items()}
        return v
    return {f"seed{sd}": {k: rnd(v) for k, v in blind.run(10000, sd, tol=1e-7).items()}
            for sd in (0, 1)}


def _pool_fista(task):
    """One worker of the CPU pool legs: `iters` oracle FISTA iterations on
    one image (single-threaded NumPy); returns its pixel count."""
    rows, cols, levels, taps, sigma, radius, seed, iters = task
    from oracle import blur as bl, filters as fl, fista as fi
    from workloads import gen_image, gen_noise, rng_for
    rng = rng_for(*seed)
    img = gen_image(rng, rows, cols)
    psf = bl.gaussian_taps(sigma, radius)
    b = bl.R(img, psf) + gen_noise(rng, img.shape)
    prob = fi.Problem(rows, cols, fl.by_taps(taps), "sym", levels, psf)
    fi.fista(prob, b, 2e-5, iters)
    return rows * cols * iters


def cpu_leg(size: int, bc: str, iters: int = 2) -> dict:
    """The FP64 NumPy oracle on this host (never in the GPU process): bounded
    samples of the benchmark's workloads. Single-threaded legs run with one
    BLAS thread; the pool legs run one single-threaded worker per core, up
    to 16 (one GPU's share of the host)."""
    import multiprocessing as mp
    import platform

    import numpy as np

    from oracle import blur as bl, conv as cv, filters as fl, fista as fi, wavelet as wv
    from workloads import gen_batched_config, gen_conv_pair, gen_image, gen_noise, rng_for
    out = {}
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        model = platform.processor()
    ncpu = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = ncpu
    out["host"] = {"cpu_model": model, "nproc": ncpu, "affinity_cpus": avail}
    # 1. the headline step at full size
    rng = rng_for(2, 0)
    img = gen_image(rng, size, size)
    psf = bl.gaussian_taps(3.0, 7)
    b = bl.R(img, psf) + gen_noise(rng, img.shape)
    prob = fi.Problem(size, size, fl.by_taps(8), bc, 4, psf)
    t0 = time.perf_counter()
    fi.fista(prob, b, 2e-5, iters)
    out["sec_per_iter"] = (time.perf_counter() - t0) / iters
    h = fl.by_taps(8)
    x = np.random.default_rng(0).standard_normal(prob.ncoef) * 1e-2
    ops_ = {"W": lambda: wv.W(x, h, bc, 4, size, size), "W*": lambda: wv.W_adj(img, h, bc, 4),
            "R": lambda: bl.R(img, psf), "R*": lambda: bl.R_adj(img, psf),
            "A": lambda: prob.A(x), "A*": lambda: prob.A_adj(img)}
    op_s = {}
    for name, fn in ops_.items():
        t1 = time.perf_counter()
        fn()
        op_s[name] = time.perf_counter() - t1
    out["op_s"] = op_s
    # 2. the small configuration: 200 iterations at 256^2, db4 J = 3, 9x9 PSF
    rng = rng_for(1, 0)
    img1 = gen_image(rng, 256, 256)
    psf1 = bl.gaussian_taps(2.0, 4)
    b1 = bl.R(img1, psf1) + gen_noise(rng, img1.shape)
    prob1 = fi.Problem(256, 256, fl.by_taps(8), "sym", 3, psf1)
    t0 = time.perf_counter()
    fi.fista(prob1, b1, 2e-5, 200)
    out["small_200_iters_s"] = time.perf_counter() - t0
    # 3. the convolution pair (K = 128, N = 65536), 64 of the 256 pairs
    rng = rng_for(4, 0)
    pairs = [gen_conv_pair(rng, 128, 65536) for _ in range(64)]
    t0 = time.perf_counter()
    for hh, ss in pairs:
        cv.conv_adjoint_pair(hh[None], ss[None], None)
    dt = time.perf_counter() - t0
    out["conv_pairs"] = {"pairs": 64, "s": dt,
                         "GFLOPs": 2.0 * 64 * 3 * 128 * 65536 / dt / 1e9}
    # 4. pool legs: the 16 smallest images of the uneven batch (one iteration
    #    each), and 512^2 warm-start-sized problems (20 iterations each)
    workers = max(1, min(avail, 16))
    cfg = gen_batched_config(rng_for(3, 0), 64)
    small = sorted(range(64), key=lambda i: cfg[i]["rows"] * cfg[i]["cols"])[:16]
    tasks3 = [(cfg[i]["rows"], cfg[i]["cols"], cfg[i]["levels"], cfg[i]["taps"], cfg[i]["sigma"],
               cfg[i]["radius"], (3, 1000 + i), 1) for i in small]
    tasks5 = [(512, 512, 4, 8, 2.0, 6, (50, i), 20) for i in range(workers)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        for key, tasks in (("pool_uneven_batch", tasks3), ("pool_512", tasks5)):
            t0 = time.perf_counter()
            pix = sum(pool.map(_pool_fista, tasks, chunksize=1))
            dt = time.perf_counter() - t0
            out[key] = {"workers": workers, "images": len(tasks), "s": dt,
                        "mpix_iter_per_s": pix / dt / 1e6}
    return out


def cpu_baseline(size: int, bc: str, iters: int = 2) -> dict:
    """The FP64 NumPy oracle timed on this host in a separate process, on
    bounded samples of the same workloads (about half a minute of CPU work)."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", "--size",
                          str(size), "--bc", bc], capture_output=True, text=True, env=env,
                         timeout=900)
    if out.returncode != 0:
        return {"error": out.stderr[-500:]}
    res = json.loads(out.stdout.strip().splitlines()[-1])
    spi = res["sec_per_iter"]
    pool3, pool5 = res["pool_uneven_batch"], res["pool_512"]
    return {"value": size * size / spi / 1e6, "unit": "Mpix/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} FISTA iterations (one A and one A* each) at {size}x{size}, "
                      f"FP64 NumPy, one thread; {spi:.2f} s/iteration",
            "host": res["host"],
            "ops_mpix_s": {k: round(size * size / v / 1e6, 3) for k, v in res["op_s"].items()},
            "ops_sample": "one application each of W, W*, R, R*, A, A* at the same size, one thread",
            "small_config_200_iters": {"s": round(res["small_200_iters_s"], 3), "cores": 1,
                                       "sample": "256x256 FP64, db4 J=3 sym, 9x9 PSF sigma 2, "
                                                 "200 FISTA iterations from zero"},
            "conv_adjoint_pair": {"GFLOPs": round(res["conv_pairs"]["GFLOPs"], 3), "cores": 1,
                                  "sample": "64 of the 256 pairs (K=128, N=65536): h*s and the "
                                            "two valid correlations, np.convolve FP64"},
            "uneven_batch_pool": {"mpix_iter_per_s": round(pool3["mpix_iter_per_s"], 3),
                                  "cores": pool3["workers"],
                                  "sample": "the 16 smallest images of the 64-image uneven batch, "
                                            "one FISTA iteration each, one single-threaded worker "
                                            f"per core ({pool3['workers']} workers), "
                                            f"{pool3['s']:.1f} s"},
            "warm_start_size_pool": {"mpix_iter_per_s": round(pool5["mpix_iter_per_s"], 3),
                                     "cores": pool5["workers"],
                                     "sample": f"{pool5['images']} 512x512 problems (db4 J=4 sym, "
                                               "13x13 PSF), 20 FISTA iterations each, one worker "
                                               f"per core, {pool5['s']:.1f} s"}}


def main():
    args = parse()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], int(args.pmc_summary[2]))
        return
    if args.trace_summary:
        trace_summary(args.trace_summary[0], int(args.trace_summary[1]), args.size)
        return
    if args.large_summary:
        large_summary(*args.large_summary)
        return
    if args.cpu_leg:
        print(json.dumps(cpu_leg(args.size, args.bc)))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(independent images shard across GPUs without exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1707_02018_amd import _lib, ops
    from workloads import gen_image, gen_noise, rng_for

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only_batched:
        print(json.dumps(bench_batched(torch, ops, args.batched_iters)))
        return
    if args.only_conv:
        print(json.dumps(bench_conv(torch, ops)))
        return
    if args.only_autograd:
        print(json.dumps(bench_autograd(torch, ops)))
        return
    if args.only_cnn:
        print(json.dumps(bench_cnn(torch)))
        return
    if args.only_dct:
        print(json.dumps(bench_blur_dct(torch, ops, _lib.load(), torch.cuda.Stream(device=dev))))
        return
    if args.copy_reference:
        src = torch.ones(COPY_REF_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.only_large:
        print(json.dumps(bench_large(torch, ops)))
        return
    N, J, lam = args.size, 4, 2e-5
    w = ops.WaveletSpec(N, N, J, taps=8, bc=args.bc)
    bsp = ops.BlurSpec(N, N, sigma=3.0, radius=7)
    ncoef = w.ncoef
    npix = N * N
    rng = rng_for(2, 0)
    img = torch.tensor(gen_image(rng, N, N), dtype=torch.float32, device=dev)
    noise = torch.tensor(gen_noise(rng, (N, N)), dtype=torch.float32, device=dev)
    b = ops.blur(bsp, img) + noise
    torch.cuda.synchronize()
    if args.only_step:
        st = ops.FistaState(w, bsp, b)
        for _ in range(args.only_step):
            ops.fista_step(st, b, lam)
        torch.cuda.synchronize()
        print(json.dumps({"only_step": args.only_step}))
        return

    # ---------------------------------------------------------- headline
    st = ops.FistaState(w, bsp, b)
    for _ in range(args.warmup):
        ops.fista_step(st, b, lam)
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(cur)
    for _ in range(args.steps):
        ops.fista_step(st, b, lam)
    ev1.record(cur)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    ms_per_step_events = ev0.elapsed_time(ev1) / args.steps
    value = npix * args.steps / dt / 1e6

    # ------------------------------------------- per-operator graph timings
    lib = _lib.load()
    stream = torch.cuda.Stream(device=dev)
    x = torch.randn(ncoef, device=dev) * 1e-2
    y = torch.randn(N, N, device=dev)
    out_img = torch.empty(N, N, device=dev)
    out_coef = torch.empty(ncoef, device=dev)
    wsn = ops.workspace_bytes(w, bsp, torch.float32, 1)
    ws = torch.empty(wsn, dtype=torch.uint8, device=dev)
    w1 = ops.WaveletSpec(N, N, 1, taps=8, bc=args.bc)  # level 1 alone: one kernel
    P = lambda t: ops._ptr(t)  # noqa: E731
    # the update half of the iteration at level 1 alone (one kernel: W^* of an
    # image-space gradient with the proximal / momentum update of all four
    # level-1 bands), on its own state
    x1 = torch.randn(w1.ncoef, device=dev) * 1e-2
    y1 = torch.randn(w1.ncoef, device=dev) * 1e-2
    st1 = _lib.FistaState()
    st1.x, st1.y, st1.resid, st1.obj = x1.data_ptr(), y1.data_ptr(), None, None
    st1.k, st1.t, st1.gradient = 1, 1.0, 0
    ctypes_ = __import__("ctypes")

    def make_calls(s):
        sp = __import__("ctypes").c_void_p(s.cuda_stream)
        return {
            "W": lambda: lib.wavelet_synth(w.c, 0, 1, P(x), P(out_img), P(ws), wsn, sp),
            "W*": lambda: lib.wavelet_synth_adjoint(w.c, 0, 1, P(y), P(out_coef), P(ws), wsn, sp),
            "R": lambda: lib.blur(bsp.c, 0, 1, P(y), P(out_img), sp),
            "R*": lambda: lib.blur_adjoint(bsp.c, 0, 1, P(y), P(out_img), sp),
            "A": lambda: lib.aw_apply_A(w.c, bsp.c, 0, 1, P(x), P(out_img), P(ws), wsn, sp),
            "A-b_fused": lambda: lib.aw_apply_A_fused(w.c, bsp.c, 0, 1, P(x), P(y), P(out_img),
                                                      P(ws), wsn, sp),
            "A*": lambda: lib.aw_apply_A_adjoint(w.c, bsp.c, 0, 1, P(y), P(out_coef), P(ws), wsn,
                                                 sp),
            "A*_fused": lambda: lib.aw_apply_A_adjoint_fused(w.c, bsp.c, 0, 1, P(y), P(out_coef),
                                                             P(ws), wsn, sp),
            "W*_level1": lambda: lib.wavelet_synth_adjoint(w1.c, 0, 1, P(y), P(out_coef), P(ws),
                                                           wsn, sp),
            "W_level1": lambda: lib.wavelet_synth(w1.c, 0, 1, P(x), P(out_img), P(ws), wsn, sp),
            "W*prox_level1": lambda: lib.aw_fista_update(w1.c, 0, 1, P(y), 1.0, lam,
                                                         ctypes_.byref(st1), 0, P(ws), wsn, sp),
        }

    with torch.cuda.stream(stream):
        calls = make_calls(stream)
        op_us = {name: graph_us(torch, stream, fn, name) for name, fn in calls.items()}
    ops_mpix = {k: round(npix / v, 1) for k, v in op_us.items()}

    # the same operators streaming from HBM (inputs and outputs rotated over
    # buffer sets larger than the Infinity Cache); the figures above are
    # cache-resident
    cold = bench_cold(torch, ops, lib, w, w1, bsp, lam, stream)

    # the reported roofline: the whole FISTA iteration against its
    # algorithmic bytes (y and b read, r written for A y - b; r, y and
    # x_{k-1} read, x_k and y_{k+1} written for A^* and the update), step time
    # from HIP events on the launching stream over the timed region
    step_bytes = 4 * (5 * ncoef + 3 * npix)
    step_gbs = step_bytes / (ms_per_step_events * 1e-3) / 1e9
    trec = step_traffic()
    roofline = {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                "traffic": trec["bytes_per_step"] if trec else None,
                "kernel": "fista_step: one FISTA iteration (8 launches: W levels 4..2, W level 1, "
                          "R y - b, R^*, W^* + update levels 1..4)",
                "algorithmic_bytes": step_bytes, "avg_us": round(1e3 * ms_per_step_events, 3),
                "cache": "hot: the 2048^2 working set stays in the 256 MB Infinity Cache between "
                         "iterations"}
    # the whole step streaming from HBM: 12 independent problems in rotation
    step_cold = bench_step_cold(torch, ops, w, bsp, b, lam)
    roofline["cold_hbm"] = {"avg_us": step_cold["us_per_step"],
                            "achieved": round(step_bytes / (step_cold["us_per_step"] * 1e-6) / 1e9,
                                              1),
                            "frac": round(step_bytes / (step_cold["us_per_step"] * 1e-6) / 1e9 /
                                          HBM_PEAK_GBS, 4),
                            "protocol": step_cold["protocol"]}
    # standalone single-kernel operators (microbenchmarks, not the step's own
    # launches): hot replays and the same streaming from HBM
    _, sr, sc = w.layout()
    k1 = sr[1] * sc[1]
    alg_bytes = {"W*_level1": 4 * (npix + 4 * k1), "W_level1": 4 * (npix + 4 * k1),
                 "R": 8 * npix, "R*": 8 * npix, "W*prox_level1": 4 * (npix + 16 * k1)}
    standalone = {}
    for op, nb in alg_bytes.items():
        rec_ = {"algorithmic_bytes": nb, "hot_us": round(op_us[op], 3),
                "hot_frac": round(nb / (op_us[op] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
        if op in cold["ops_us"]:
            cu = cold["ops_us"][op]
            rec_.update({"cold_us": cu, "cold_frac": round(nb / (cu * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                                           4)})
        standalone[op] = rec_

    # ------------------------------------------------ time to 1e-4 (plain)
    target = None
    if not args.no_target:
        log("time to 1e-4 (2048^2, plain)")
        target = bench_time_to_target(torch, ops, w, bsp, b, lam, ms_per_step)

    extras = {}
    if not args.no_extras:
        del st
        torch.cuda.empty_cache()
        log("other boundary modes")
        extras["other_modes"] = bench_modes(torch, ops, lib, bsp, b, lam,
                                            [m for m in ("per", "zpd", "sym") if m != args.bc])
        log("batched uneven FISTA")
        extras["batched_uneven_fista"] = bench_batched(torch, ops, args.batched_iters)
        torch.cuda.empty_cache()
        log("autograd")
        extras["autograd_A"] = bench_autograd(torch, ops)
        torch.cuda.empty_cache()
        log("convolution pair")
        extras["conv_adjoint_pair"] = bench_conv(torch, ops)
        torch.cuda.empty_cache()
        log("warm start (512^2)")
        extras["warm_start"] = bench_warm(torch, ops, args.warm_images)
        log("R through the DCT-II (2048^2)")
        extras["blur_dct"] = bench_blur_dct(torch, ops, lib, stream)
        log("adjoint vs pseudoinverse gradient (256^2, 2500 iterations)")
        extras["adjoint_vs_pinv"] = bench_adjoint_study()
        log("multi-channel blind channel estimation (eq. 6, up to 10,000 iterations)")
        extras["blind_channel"] = bench_blind()
    log("cpu baseline")

    cpu = None if args.no_cpu_baseline else cpu_baseline(N, args.bc)

    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fista_{N}x{N}_db4_J4_{args.bc}_psf15_sigma3",
                   "image": [N, N], "levels": J, "filter_taps": 8, "bc": args.bc,
                   "psf_radius": 7, "psf_sigma": 3.0, "lambda": lam, "ncoef": ncoef,
                   "batch": 1},
        "fista_iters_per_s": round(1e3 / ms_per_step, 1),
        "ms_per_step_hip_events": round(ms_per_step_events, 4),
        "ops_us": {k: round(v, 3) for k, v in op_us.items()},
        "ops_mpix_s": ops_mpix,
        "ops_cache": "hot: inputs resident in the 256 MB Infinity Cache between replays",
        "ops_cold_hbm": cold,
        "roofline": roofline,
        "standalone_kernels": standalone,
        "time_to_target": target,
        **extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
