"""Benchmark: WECT cell x direction throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
                    [--no-single] [--no-calibrate] [--only WORKLOAD] [--copy-calibration]

Headline workload (the largest single-GPU configuration): 16 uint8 volumes
with sides drawn uniformly from 64..192 per axis (Gaussian random fields,
sigma 6 voxels), voxels with intensity > 100 are vertices, edges / squares /
cubes induced, cell weight = max vertex intensity, 512 Fibonacci-sphere
directions, 256 thresholds on [-sqrt3, sqrt3], int32 output [16, 512, 256],
all volumes in one batched call.  One step = one batched forward over the
whole batch, inputs resident in HBM.  Before the warm-up steps the step runs
back to back for half a second, untimed, so that the GPU's clocks have left
their idle state.

Items = directions x (cells of every dimension, vertices included), whatever
shortcut the kernel takes.  Prints one JSON line: the headline, its roofline
(VALU issue of the histogram kernel, algorithmic lane operations per launch
over its HIP-event duration), the HBM fraction at algorithmic bytes against
the MI355X peak and against a measured device copy, the LDS atomic rate
against a measured conflict-free rate, and under "configs" the same
quantities for every other workload (3D Kuhn mesh forward and adjoint,
differentiation batch forward / forward + adjoint / graph, 2D image batch,
small 2D mesh), each batched against one launch per complex; the CPU oracle
on a bounded sample of the headline, on all host cores and on one.

--only NAME runs one workload (volumes3d, images2d, kuhn3d, diffbatch,
mesh2d) and prints its block: the profiling runs use it so that kernel
statistics and counters belong to one workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WECT simplex·directions/sec fwd & fwd+bwd, batched vs 1-per-launch; HBM GB/s"
UNIT = "simplex·directions/s"
HBM_PEAK_GBPS = 8000.0
# VALU lane-operations per second: 256 CUs x 64 lanes x 2.4 GHz (non-packed, non-fused)
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
WORKLOADS = ("volumes3d", "images2d", "kuhn3d", "diffbatch", "mesh2d")


# ---------------------------------------------------------------------------
# bookkeeping: cells, algorithmic work and bytes
# ---------------------------------------------------------------------------

def cubical_cell_count(C) -> int:
    """Number of cells (vertices, edges, squares, cubes) of an image/volume
    under the inclusion rule: a cell exists iff all of its corners exceed the
    inclusion level.  Bookkeeping for the item count only."""
    import itertools
    import numpy as np
    m = np.asarray(C.intensity) > C.include_above
    n = m.ndim
    total = 0
    for r in range(n + 1):
        for S in itertools.combinations(range(n), r):
            ok = None
            for eps in itertools.product((0, 1), repeat=r):
                sl = [slice(None)] * n
                for k, e in zip(S, eps):
                    a = n - 1 - k
                    sl[a] = slice(e, e + m.shape[a] - 1)
                v = m[tuple(sl)]
                ok = v if ok is None else (ok & v)
            total += int(ok.sum())
    return total


def included_vertices(C) -> int:
    import numpy as np
    return int((np.asarray(C.intensity) > C.include_above).sum())


def staged_vertices(C, device: str = "cuda") -> int:
    """Included vertices with a nonzero combined weight in at least one
    orthant: the vertices the top-corner forward stages (its compaction skips
    the others, which add nothing to any output).  Bookkeeping for the
    measurement only, evaluated with torch on the GPU: for each orthant the
    signed, vertex-max (or unit) weights of the 2^n cells a vertex tops."""
    import itertools
    import numpy as np
    import torch
    I = torch.as_tensor(np.asarray(C.intensity).astype(np.int32), device=device)
    P = I > C.include_above
    n = I.dim()
    Ip = torch.nn.functional.pad(I, (1, 1) * n)
    Pp = torch.nn.functional.pad(P, (1, 1) * n)

    def sh(A, off):  # off[k] along axis k (axis 0 = fastest = last tensor dim)
        sl = tuple(slice(1 + off[n - 1 - a], 1 + off[n - 1 - a] + I.shape[a]) for a in range(n))
        return A[sl]

    anynz = torch.zeros_like(P)
    for o in range(1 << n):
        dirs = [1 if (o >> k) & 1 else -1 for k in range(n)]
        acc = torch.zeros_like(I)
        for S in itertools.product((0, 1), repeat=n):
            pres = torch.ones_like(P)
            mx = torch.zeros_like(I)
            for c in itertools.product(*[(0, 1) if S[k] else (0,) for k in range(n)]):
                off = [c[k] * dirs[k] for k in range(n)]
                pres &= sh(Pp, off)
                mx = torch.maximum(mx, sh(Ip, off))
            val = mx if C.weighted else torch.ones_like(I)
            acc += torch.where(pres, val, torch.zeros_like(I)) * (-1) ** sum(S)
        anynz |= acc != 0
    return int((anynz & P).sum().item())


def search_ops(T: int) -> int:
    return math.ceil(math.log2(T + 1))


def cubical_ops(nverts: int, n: int, T: int, d: int) -> int:
    """Algorithmic VALU lane-ops of the top-corner forward: per included vertex
    and direction, (n-1) adds of the axis heights, the threshold search, one
    select of the combined weight, one add."""
    return nverts * d * ((n - 1) + search_ops(T) + 1 + 1)


def simplicial_ops(counts, n: int, T: int, d: int) -> int:
    """Algorithmic VALU lane-ops of the simplicial forward (and of the adjoint,
    whose gather-add takes the place of the histogram add): per vertex and
    direction (2n-1) for the height, the threshold search, one add; per
    i-simplex and direction, i maxima and one add."""
    per_dir = counts[0] * ((2 * n - 1) + search_ops(T) + 1)
    per_dir += sum(counts[i] * (i + 1) for i in range(1, len(counts)))
    return per_dir * d


def simplicial_bytes(counts, n: int, B: int, d: int, T: int, wmode: str, backward: bool = False) -> int:
    """Algorithmic HBM bytes: coordinates, simplex index rows and weights read
    once, the output written once (adjoint: grad_out read once, the weight
    gradient written once instead)."""
    b = counts[0] * n * 4 + sum(counts[i] * (i + 1) * 4 for i in range(1, len(counts)))
    wbytes = counts[0] * 4 if wmode == "vertex_max" else (sum(counts) * 4 if wmode == "explicit" else 0)
    b += wbytes + B * d * T * 4
    if backward:
        b += wbytes  # the gradient has the shape of the weights
    return b


def cubical_bytes(cx, d: int, T: int) -> int:
    return int(cx.total_voxels) + int(cx.axis.numel()) * 4 + cx.B * d * T * 4


def settle(fn, seconds=0.5):
    """Run fn back to back for about `seconds` of wall time (untimed), so that
    the GPU's clocks have left their idle state before anything is measured."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            fn()
        torch.cuda.synchronize()


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


_FLUSH = []


def warm_cold(a, fn, reps=11):
    """Median time of one call with HIP events on the current stream: warm
    (back to back) and cold (each call after writing a 1 GiB buffer, which
    evicts the 256 MB Infinity Cache and the L2 caches of earlier calls).
    Skipped in the single-workload runs behind the profiles, so that their
    kernel statistics cover warm calls only."""
    import torch
    if getattr(a, "only", None):
        return None
    if not _FLUSH:
        _FLUSH.append(torch.empty(1 << 28, dtype=torch.float32, device="cuda"))
    buf = _FLUSH[0]

    def one(flush):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if flush:
            buf.fill_(float(len(ts)))
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))

    res = {}
    for name, flush in (("warm", False), ("cold", True)):
        ts = []
        for _ in range(reps):
            one(flush)
        res[f"{name}_median_ms"] = sorted(ts)[reps // 2]
    res["reps"] = reps
    res["flush_bytes"] = buf.numel() * 4
    return res


def kernel_ms(W, fn, reps):
    """Average HIP-event duration of the library's main kernels (forward
    histogram, adjoint) per launch, recorded on their own stream."""
    import torch
    W.profile_enable(True)
    W.profile_read(reset=True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    p = W.profile_read(reset=True)
    W.profile_enable(False)
    f = p["fwd_ms"] / p["fwd_launches"] if p["fwd_launches"] else None
    b = p["bwd_ms"] / p["bwd_launches"] if p["bwd_launches"] else None
    return f, b, p


# the sources that decide what a profiled kernel does (its translation unit,
# the shared device helpers, the host runtime that plans its launches)
KERNEL_SOURCES = {
    "cub_fwd": ["k_cub_fwd.hip", "k_reduce.hip", "wect_device.h", "wect_internal.h", "wect_api.cpp"],
    "simp_fwd": ["k_simp_fwd.hip", "k_reduce.hip", "wect_device.h", "wect_internal.h", "wect_api.cpp"],
    "simp_bwd": ["k_simp_bwd.hip", "wect_device.h", "wect_internal.h", "wect_api.cpp"],
}


def kernel_source_hash(which: str = None) -> str:
    """Hash of the kernel sources: all of them, or those of one kernel family."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_03909_amd", "csrc")
    files = KERNEL_SOURCES[which] if which else [f for f in os.listdir(csrc) if f.endswith((".hip", ".cpp", ".h"))]
    for f in sorted(files):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(name: str, family: str):
    """HBM traffic per launch measured with rocprofv3 counters for the current
    sources of the kernel family (profiles/<name>.json), or None when they changed."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash(family):
        return None
    return rec


def roofline(kernel: str, ops: int, bytes_alg: int, k_ms: float, calib, profile_name: str, family: str,
             lds_atomics: int = 0, step_ms: float = None, staged: float = None):
    """VALU-issue roofline of one kernel launch: algorithmic lane-ops over the
    kernel's duration (capped below by the whole step's time when the step is
    that kernel alone), the same over the whole step (every kernel of the call,
    e.g. the voxel records of the cubical forward), the algorithmic-bytes HBM
    fraction, the measured counter traffic when available, and the LDS atomic
    rate."""
    t_ms = k_ms if step_ms is None else min(k_ms, step_ms)
    t = t_ms * 1e-3
    ach = ops / t / 1e12
    gbps = bytes_alg / t / 1e9
    rec = load_counters(profile_name, family)
    r = {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": ach / VALU_PEAK_TOPS,
         "step_frac": (ops / (step_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS) if step_ms else None,
         "traffic": rec.get("traffic_bytes_per_launch") if rec else None,
         "kernel": kernel, "kernel_ms": t_ms, "alg_ops_per_launch": ops,
         "hbm_alg_bytes_per_launch": bytes_alg, "hbm_achieved_GBps": gbps, "hbm_frac": gbps / HBM_PEAK_GBPS}
    if calib and calib.get("copy_GBps"):
        r["hbm_frac_of_measured_copy"] = gbps / calib["copy_GBps"]
    if rec:
        r["counter_GBps"] = rec["traffic_bytes_per_launch"] / t / 1e9
        r["counter_hbm_frac"] = r["counter_GBps"] / HBM_PEAK_GBPS
        if rec.get("sq"):
            r["counters"] = rec["sq"]
    if staged is not None:
        # the top-corner count charges every included vertex; only those with a
        # nonzero combined weight are staged and histogrammed
        r["staged_fraction"] = staged
        r["frac_staged"] = r["frac"] * staged
        r["note"] = ("alg_ops charges every included vertex x direction; the kernel stages only the "
                     f"{100 * staged:.1f} % with a nonzero combined weight, so frac can exceed 1; frac_staged "
                     "counts the staged vertices")
    if lds_atomics:
        r["lds_atomics_per_s"] = lds_atomics / t
        if calib and calib.get("lds_add_per_s"):
            r["lds_atomic_frac_of_measured"] = {k: lds_atomics / t / v for k, v in calib["lds_add_per_s"].items()}
    return r


# ---------------------------------------------------------------------------
# calibration: achievable HBM copy and conflict-free LDS atomics
# ---------------------------------------------------------------------------

def calibrate(W):
    import torch
    from paper_2511_03909_amd import _lib as L
    lib = L.lib()
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        L.check(lib.wect_calib_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream), "copy")
    ts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        L.check(lib.wect_calib_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream), "copy")
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[len(ts) // 2]
    out["copy_GBps"] = 2 * nbytes / (ms * 1e-3) / 1e9  # read + write
    out["copy_bytes"] = nbytes
    del src, dst
    blocks, reps = 2048, 4096
    rates = {}
    for kind, name, width in ((0, "u32", 4), (1, "u64", 8), (2, "f32", 4)):
        buf = torch.empty(blocks * 64 * width, dtype=torch.uint8, device="cuda")
        r = reps if kind != 2 else reps // 16
        L.check(lib.wect_calib_lds_atomics(kind, blocks, r, buf.data_ptr(), stream), "lds")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        L.check(lib.wect_calib_lds_atomics(kind, blocks, r, buf.data_ptr(), stream), "lds")
        e1.record()
        torch.cuda.synchronize()
        rates[name] = blocks * 1024 * r / (e0.elapsed_time(e1) * 1e-3)
    out["lds_add_per_s"] = rates
    out["note"] = ("copy: one 1 GiB device copy (wect_calib_copy), read + write bytes over its HIP-event time; "
                   "LDS: lane-level conflict-free atomic adds per second (wect_calib_lds_atomics, 2048 blocks of "
                   "1024 threads)")
    return out


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def run_volumes3d(W, a, calib, single=True):
    """3D cubical batch: 16 volumes, 512 directions, T = 256, one batched forward."""
    import torch
    import synth
    w = synth.cfg4()
    cx = W.CubicalBatch.from_host(w.complexes, device="cuda")
    g = W.Grid(w.dirs, w.thr, device="cuda")
    d, T, B = g.d, g.T, cx.B
    cells = sum(cubical_cell_count(C) for C in w.complexes)
    nverts = sum(included_vertices(C) for C in w.complexes)
    # (not in the single-workload runs behind the profiles: its many small
    # torch kernels would fill their traces)
    nstaged = None if a.only else sum(staged_vertices(C) for C in w.complexes)
    out = torch.empty((B, d, T), dtype=torch.int32, device="cuda")
    ws = torch.empty(max(1, W.wect_workspace_bytes(cx, g)), dtype=torch.uint8, device="cuda")

    def step():
        W.wect_forward(cx, g, out=out, ws=ws)

    settle(step)
    sec = timed(step, a.steps, a.warmup)
    kf, _, _ = kernel_ms(W, step, max(5, a.steps // 2))
    res = {"workload": w.name, "items": d * cells, "cells": cells, "included_vertices": nverts,
           "staged_vertices": nstaged, "ms": sec * 1e3,
           "items_per_s": d * cells / sec, "per_call": warm_cold(a, step),
           "roofline": roofline("k_cub_fwd<3, vertex-max>", cubical_ops(nverts, 3, T, d), cubical_bytes(cx, d, T),
                                kf, calib, "cubical_fwd_3d_16vol_64-192_d512_T256", "cub_fwd",
                                lds_atomics=(nstaged or nverts) * d, step_ms=sec * 1e3,
                                staged=nstaged / nverts if nstaged else None)}
    if single:
        singles = [W.CubicalBatch.from_host([C], device="cuda") for C in w.complexes]
        outs = [torch.empty((1, d, T), dtype=torch.int32, device="cuda") for _ in singles]
        ws1 = torch.empty(max(1, max(W.wect_workspace_bytes(s, g) for s in singles)), dtype=torch.uint8, device="cuda")
        t1 = timed(lambda: [W.wect_forward(s, g, out=o, ws=ws1) for s, o in zip(singles, outs)], 2, 1)
        res["one_per_launch"] = {"ms": t1 * 1e3, "items_per_s": d * cells / t1, "batched_speedup": t1 / sec}
    return res, w


def run_images2d(W, a, calib, single=True):
    """2D cubical batch: 256 images 128^2, 64 directions, T = 128."""
    import torch
    import synth
    w = synth.cfg2()
    cx = W.CubicalBatch.from_host(w.complexes, device="cuda")
    g = W.Grid(w.dirs, w.thr, device="cuda")
    d, T, B = g.d, g.T, cx.B
    cells = sum(cubical_cell_count(C) for C in w.complexes)
    nverts = sum(included_vertices(C) for C in w.complexes)
    # (not in the single-workload runs behind the profiles: its many small
    # torch kernels would fill their traces)
    nstaged = None if a.only else sum(staged_vertices(C) for C in w.complexes)
    out = torch.empty((B, d, T), dtype=torch.int32, device="cuda")
    ws = torch.empty(max(1, W.wect_workspace_bytes(cx, g)), dtype=torch.uint8, device="cuda")

    def step():
        W.wect_forward(cx, g, out=out, ws=ws)

    settle(step)
    sec = timed(step, max(20, a.steps), a.warmup)
    kf, _, _ = kernel_ms(W, step, 20)
    res = {"workload": w.name, "items": d * cells, "ms": sec * 1e3, "items_per_s": d * cells / sec,
           "per_call": warm_cold(a, step),
           "roofline": roofline("k_cub_fwd<2, vertex-max>", cubical_ops(nverts, 2, T, d), cubical_bytes(cx, d, T),
                                kf, calib, "cubical_fwd_2d_256x128x128_d64_T128", "cub_fwd",
                                lds_atomics=(nstaged or nverts) * d, step_ms=sec * 1e3,
                                staged=nstaged / nverts if nstaged else None)}
    if single:
        singles = [W.CubicalBatch.from_host([C], device="cuda") for C in w.complexes]
        outs = [torch.empty((1, d, T), dtype=torch.int32, device="cuda") for _ in singles]
        ws1 = torch.empty(max(1, max(W.wect_workspace_bytes(s, g) for s in singles)), dtype=torch.uint8, device="cuda")
        t1 = timed(lambda: [W.wect_forward(s, g, out=o, ws=ws1) for s, o in zip(singles, outs)], 5, 2)
        res["one_per_launch"] = {"ms": t1 * 1e3, "items_per_s": d * cells / t1, "batched_speedup": t1 / sec}
    return res, w


def run_kuhn3d(W, a, calib):
    """3D simplicial Kuhn mesh 64^3, float32 weights per simplex, 256
    directions, T = 256: forward, and the adjoint to the simplex weights."""
    import torch
    import synth
    w = synth.cfg3()
    cx = W.SimplicialBatch.from_host(w.complexes, device="cuda")
    g = W.Grid(w.dirs, w.thr, device="cuda")
    d, T = g.d, g.T
    counts = list(cx.counts)
    items = d * sum(counts)
    out = torch.empty((1, d, T), dtype=torch.float32, device="cuda")
    ws = torch.empty(max(1, W.wect_workspace_bytes(cx, g, True)), dtype=torch.uint8, device="cuda")
    gout = torch.randn((1, d, T), device="cuda")
    grads = [torch.empty(k, dtype=torch.float32, device="cuda") for k in counts]

    def fwd():
        W.wect_forward(cx, g, out=out, ws=ws)

    def fwdbwd():
        W.wect_batched(cx, g, gout, out=out, grads=grads, ws=ws)

    settle(fwd)
    t_f = timed(fwd, 10, 2)
    t_fb = timed(fwdbwd, 10, 2)
    kf, kb, _ = kernel_ms(W, fwdbwd, 5)
    ops = simplicial_ops(counts, 3, T, d)
    return {"workload": w.name, "items": items, "fwd_ms": t_f * 1e3, "fwd_bwd_ms": t_fb * 1e3,
            "per_call_fwd": warm_cold(a, fwd), "per_call_fwd_bwd": warm_cold(a, fwdbwd),
            "fwd_items_per_s": items / t_f, "fwd_bwd_items_per_s": items / t_fb,
            "roofline_fwd": roofline("k_simp_fwd<3, explicit, float>", ops,
                                     simplicial_bytes(counts, 3, 1, d, T, "explicit"), kf, calib,
                                     "simplicial_fwd_3d_kuhn64_d256_T256", "simp_fwd", lds_atomics=sum(counts) * d),
            "roofline_bwd": roofline("k_simp_bwd<3, explicit>", ops,
                                     simplicial_bytes(counts, 3, 1, d, T, "explicit", backward=True), kb, calib,
                                     "simplicial_bwd_3d_kuhn64_d256_T256", "simp_bwd")}


def run_diffbatch(W, a, calib, single=True):
    """Differentiation batch: 64 Freudenthal complexes (10k-200k vertices),
    vertex-max float32 weights, 128 directions, T = 128: forward, forward +
    adjoint to the vertex weights, and the pair as one HIP graph."""
    import torch
    import synth
    w = synth.cfg5()
    cx = W.SimplicialBatch.from_host(w.complexes, device="cuda")
    g = W.Grid(w.dirs, w.thr, device="cuda")
    d, T, B = g.d, g.T, cx.B
    counts = list(cx.counts)
    items = d * sum(counts)
    gout = torch.randn((B, d, T), device="cuda")
    out = torch.empty((B, d, T), dtype=torch.float32, device="cuda")
    gv = torch.empty(counts[0], dtype=torch.float32, device="cuda")
    ws = torch.empty(max(1, W.wect_workspace_bytes(cx, g, True)), dtype=torch.uint8, device="cuda")

    def fwd():
        W.wect_batched(cx, g, None, out=out, ws=ws)

    def fwdbwd():
        W.wect_batched(cx, g, gout, out=out, grads=gv, ws=ws)

    settle(fwd)
    t_f = timed(fwd, 10, 2)
    t_fb = timed(fwdbwd, 10, 2)
    kf, kb, _ = kernel_ms(W, fwdbwd, 5)
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fwdbwd()
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(graph):
        fwdbwd()
    t_g = timed(graph.replay, 10, 2)
    ops = simplicial_ops(counts, 2, T, d)
    res = {"workload": w.name, "items": items, "fwd_ms": t_f * 1e3, "fwd_bwd_ms": t_fb * 1e3,
           "fwd_bwd_graph_ms": t_g * 1e3, "per_call_fwd": warm_cold(a, fwd),
           "per_call_fwd_bwd": warm_cold(a, fwdbwd),
           "fwd_items_per_s": items / t_f, "fwd_bwd_items_per_s": items / t_fb,
           "roofline_fwd": roofline("k_simp_fwd<2, vertex-max, float>", ops,
                                    simplicial_bytes(counts, 2, B, d, T, "vertex_max"), kf, calib,
                                    "simplicial_fwd_2d_freudenthal_batch64_d128_T128", "simp_fwd", lds_atomics=sum(counts) * d),
           "roofline_bwd": roofline("k_simp_bwd<2, vertex-max>", ops,
                                    simplicial_bytes(counts, 2, B, d, T, "vertex_max", backward=True), kb, calib,
                                    "simplicial_bwd_2d_freudenthal_batch64_d128_T128", "simp_bwd")}
    if single:
        singles = [W.SimplicialBatch.from_host([K], device="cuda") for K in w.complexes]
        ws1 = torch.empty(max(1, max(W.wect_workspace_bytes(c, g, True) for c in singles)), dtype=torch.uint8,
                          device="cuda")
        go1 = [gout[b:b + 1].contiguous() for b in range(B)]
        o1 = [torch.empty((1, d, T), dtype=torch.float32, device="cuda") for _ in singles]
        gv1 = [torch.empty(c.counts[0], dtype=torch.float32, device="cuda") for c in singles]
        t_f1 = timed(lambda: [W.wect_batched(c, g, None, out=o, ws=ws1) for c, o in zip(singles, o1)], 3, 1)
        t_fb1 = timed(lambda: [W.wect_batched(c, g, gg, out=o, grads=v, ws=ws1)
                               for c, gg, o, v in zip(singles, go1, o1, gv1)], 3, 1)
        res["one_per_launch"] = {"fwd_ms": t_f1 * 1e3, "fwd_bwd_ms": t_fb1 * 1e3,
                                 "fwd_batched_speedup": t_f1 / t_f, "fwd_bwd_batched_speedup": t_fb1 / t_fb}
    return res, (w, cx, g, gout)


def run_mesh2d(W, a, calib):
    """Small 2D mesh (32 x 32 vertices), 32 directions, T = 64: launch-bound."""
    import torch
    import synth
    w = synth.cfg1()
    cx = W.SimplicialBatch.from_host(w.complexes, device="cuda")
    g = W.Grid(w.dirs, w.thr, device="cuda")
    items = g.d * sum(cx.counts)
    out = torch.empty((1, g.d, g.T), dtype=torch.int32, device="cuda")
    ws = torch.empty(max(1, W.wect_workspace_bytes(cx, g)), dtype=torch.uint8, device="cuda")
    t = timed(lambda: W.wect_forward(cx, g, out=out, ws=ws), 200, 20)
    return {"workload": w.name, "items": items, "us_per_call": t * 1e6, "items_per_s": items / t,
            "note": "bound by launch latency: 1.9e5 items per call"}


def run_more(W, a, res, diff):
    """Workloads beyond the scope rows: the general-filter WECF of the
    differentiation batch, a batch of small images, the Freudenthal builder,
    the image ECF, and the sigmoid relaxation."""
    import numpy as np
    import torch
    import synth
    w5, cx5, g5, gout = diff
    it5 = g5.d * sum(cx5.counts)
    F5 = (cx5.coords @ g5.dirs.t()).contiguous()
    o5w = torch.empty((cx5.B, F5.shape[1], g5.T), dtype=torch.float32, device="cuda")
    ws5w = torch.empty(max(1, W.wecf_workspace_bytes(cx5, F5.shape[1], g5.T)), dtype=torch.uint8, device="cuda")
    t_w = timed(lambda: W.wecf_forward(cx5, F5, g5.thr, out=o5w, ws=ws5w), 5, 1)
    res["wecf_filter_array_diffbatch_m128"] = {"fwd_ms": t_w * 1e3, "items_per_s": it5 / t_w}
    # one filter column (Algorithm 1 with a single vertex filter: the first
    # direction's heights), with 64 cells per wavefront instruction and without
    F1 = F5[:, :1].contiguous()
    o1 = torch.empty((cx5.B, 1, g5.T), dtype=torch.float32, device="cuda")
    one = {}
    for name, packing in (("packed", 0), ("unpacked", 1)):
        W.set_launch(cell_packing=packing)
        ws1 = torch.empty(max(1, W.wecf_workspace_bytes(cx5, 1, g5.T)), dtype=torch.uint8, device="cuda")
        t1 = timed(lambda: W.wecf_forward(cx5, F1, g5.thr, out=o1, ws=ws1), 5, 1)
        one[name] = {"fwd_ms": t1 * 1e3, "items_per_s": sum(cx5.counts) / t1}
        del ws1
    W.set_launch()
    one["packing_speedup"] = one["unpacked"]["fwd_ms"] / one["packed"]["fwd_ms"]
    res["wecf_filter_array_diffbatch_m1"] = one
    del F5, o5w, ws5w, F1, o1
    # a batch of small images (1024 of 28^2, the images' recipe otherwise):
    # one block per image, against one call per image
    ws_ = synth.cfg2(n_images=1024, side=28)
    cxs = W.CubicalBatch.from_host(ws_.complexes, device="cuda")
    gs = W.Grid(ws_.dirs, ws_.thr, device="cuda")
    its = gs.d * sum(cubical_cell_count(C) for C in ws_.complexes)
    outs = torch.empty((cxs.B, gs.d, gs.T), dtype=torch.int32, device="cuda")
    wss = torch.empty(max(1, W.wect_workspace_bytes(cxs, gs)), dtype=torch.uint8, device="cuda")
    t_b = timed(lambda: W.wect_forward(cxs, gs, out=outs, ws=wss), 20, 3)
    singles = [W.CubicalBatch.from_host([C], device="cuda") for C in ws_.complexes]
    o1s = [torch.empty((1, gs.d, gs.T), dtype=torch.int32, device="cuda") for _ in singles]
    ws1s = torch.empty(max(1, max(W.wect_workspace_bytes(c, gs) for c in singles)), dtype=torch.uint8,
                       device="cuda")
    t_s = timed(lambda: [W.wect_forward(c, gs, out=o, ws=ws1s) for c, o in zip(singles, o1s)], 2, 1)
    res["images2d_1024x28x28_d64_T128"] = {"ms": t_b * 1e3, "items_per_s": its / t_b,
                                           "one_per_launch_ms": t_s * 1e3, "batched_speedup": t_s / t_b}
    del cxs, singles, o1s, ws1s, outs, wss
    # the 256 images of 128^2 at 1000 and 4096 thresholds (threshold tiles: one
    # pass over the voxels per tile of thresholds that fits LDS)
    wi = synth.cfg2()
    cxi = W.CubicalBatch.from_host(wi.complexes, device="cuda")
    iti = 64 * sum(cubical_cell_count(C) for C in wi.complexes)
    many = {}
    for T in (1000, 4096):
        gi = W.Grid(wi.dirs, synth.uniform_thresholds(T, 1.45), device="cuda")
        oi = torch.empty((cxi.B, gi.d, T), dtype=torch.int32, device="cuda")
        wsi = torch.empty(max(1, W.wect_workspace_bytes(cxi, gi)), dtype=torch.uint8, device="cuda")
        ti = timed(lambda: W.wect_forward(cxi, gi, out=oi, ws=wsi), 10, 2)
        many[f"T{T}"] = {"ms": ti * 1e3, "items_per_s": iti / ti}
        del oi, wsi
    res["images2d_256x128x128_d64_many_thresholds"] = many
    del cxi
    thr5 = w5.thr.astype(np.float64)
    lam5 = float(np.float32(2.0 * (thr5.size - 1) / (thr5[-1] - thr5[0])))
    os5 = torch.empty((cx5.B, g5.d, g5.T), dtype=torch.float32, device="cuda")
    t_build = timed(lambda: W.lower_star_index(cx5, cache=False), 2, 1)
    index5 = W.lower_star_index(cx5)
    relax = {"lam": lam5, "index_build_ms": t_build * 1e3}
    for name, index in (("cells", None), ("lower_star", index5)):
        wss = torch.empty(max(1, W.smooth_workspace_bytes(cx5, g5, lam5, index)), dtype=torch.uint8, device="cuda")
        t_sf = timed(lambda: W.smooth_forward(cx5, g5, lam5, out=os5, ws=wss, index=index), 3, 1)
        t_sb = timed(lambda: W.smooth_backward(cx5, g5, lam5, gout, index=index), 3, 1)
        relax[name] = {"fwd_ms": t_sf * 1e3, "bwd_ms": t_sb * 1e3}
        del wss
    res["relaxation_diffbatch_lam_spacing2"] = relax
    del index5, os5
    w2 = synth.cfg2()
    cxf = W.CubicalBatch.from_host(w2.complexes, device="cuda")
    g2 = W.Grid(w2.dirs, w2.thr, device="cuda")
    t_b = timed(lambda: W.freudenthal_from_images(cxf), 10, 2)
    sbf = W.freudenthal_from_images(cxf)
    of = torch.empty((sbf.B, g2.d, g2.T), dtype=torch.float32, device="cuda")
    wsf = torch.empty(max(1, W.wect_workspace_bytes(sbf, g2)), dtype=torch.uint8, device="cuda")
    t_fw = timed(lambda: W.wect_forward(sbf, g2, out=of, ws=wsf), 10, 2)
    res["freudenthal_images2d"] = {"build_ms": t_b * 1e3, "simplices": sum(sbf.counts), "wect_ms": t_fw * 1e3}
    del cxf, sbf, of, wsf
    ecf = {}
    for shape in ((8192, 8192), (512, 512, 512)):
        C = synth.uniform_image(shape, 0)
        cxe = W.CubicalBatch.from_host([C], device="cuda")
        wse = torch.empty(max(1, W.image_ecf_workspace_bytes(cxe)), dtype=torch.uint8, device="cuda")
        npx = int(np.prod(shape))
        for Te in (1000, 10000):
            thr_e = torch.as_tensor(synth.ecf_thresholds(Te), device="cuda")
            oe = torch.empty((1, Te), dtype=torch.int32, device="cuda")
            te = timed(lambda: W.image_ecf(cxe, thr_e, out=oe, ws=wse), 10, 2)
            ecf["x".join(str(v) for v in shape) + f"_T{Te}"] = {"ms": te * 1e3, "Gpix_per_s": npx / te / 1e9}
        del cxe, wse
    res["image_ecf_uniform"] = ecf


# ---------------------------------------------------------------------------
# CPU oracle baseline on a bounded sample of the headline workload
# ---------------------------------------------------------------------------

def _oracle_task(args):
    C, dirs, thr, dir_index = args
    import oracle
    oracle.wect(C, dirs, thr, dir_index=dir_index)
    return len(dir_index)


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(w, cells_of):
    """The oracle (unchanged, numpy) on all host cores: a process pool over
    (volume, 4 directions) tasks, 2 tasks per volume; and on one core: the
    three smallest volumes, 4 directions each."""
    import numpy as np
    import synth
    tasks = [(C, w.dirs, w.thr, list(range(k * 64, k * 64 + 4))) for C in w.complexes for k in (0, 1)]
    cores = host_cores()
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        tiny = synth.random_tiny_cubical(0, (4, 3, 2))
        pool.map(_oracle_task, [(tiny, w.dirs[:1], w.thr[:4], [0])] * cores)  # start the workers
        t0 = time.perf_counter()
        pool.map(_oracle_task, tasks, chunksize=1)
        t_all = time.perf_counter() - t0
    items_all = sum(cells_of[i // 2] * 4 for i in range(len(tasks)))
    small = list(np.argsort([C.intensity.size for C in w.complexes])[:3])
    t0 = time.perf_counter()
    for b in small:
        _oracle_task((w.complexes[b], w.dirs, w.thr, [0, 1, 2, 3]))
    t_one = time.perf_counter() - t0
    items_one = sum(cells_of[b] * 4 for b in small)
    return {"value": items_all / t_all, "unit": UNIT, "cores": cores, "kind": "oracle",
            "sample": f"all 16 volumes x 8 of 512 directions ({len(tasks)} tasks of 4 directions), "
                      f"{t_all:.1f} s wall on a pool of {cores} processes",
            "one_core": {"value": items_one / t_one, "unit": UNIT, "cores": 1,
                         "sample": f"the 3 smallest volumes x 4 directions, {t_one:.1f} s"},
            "host": {"nproc": os.cpu_count(), "usable": cores, "model": cpu_model()}}


# ---------------------------------------------------------------------------

# ---------------------------------------------------------------------------
# profile summaries (profiles/<name>.md and .json) from rocprofv3 output
# ---------------------------------------------------------------------------

# (profile name, workload, kernel name prefix, source family, roofline key of the --only result)
PROFILES = (
    ("cubical_fwd_3d_16vol_64-192_d512_T256", "volumes3d", "k_cub_fwd<3", "cub_fwd", "roofline"),
    ("cubical_fwd_2d_256x128x128_d64_T128", "images2d", "k_cub_fwd<2", "cub_fwd", "roofline"),
    ("simplicial_fwd_3d_kuhn64_d256_T256", "kuhn3d", "k_simp_fwd<3", "simp_fwd", "roofline_fwd"),
    ("simplicial_bwd_3d_kuhn64_d256_T256", "kuhn3d", "k_simp_bwd<3", "simp_bwd", "roofline_bwd"),
    ("simplicial_fwd_2d_freudenthal_batch64_d128_T128", "diffbatch", "k_simp_fwd<2", "simp_fwd", "roofline_fwd"),
    ("simplicial_bwd_2d_freudenthal_batch64_d128_T128", "diffbatch", "k_simp_bwd<2", "simp_bwd", "roofline_bwd"),
)
SQ_COUNTERS = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
               "SQ_WAIT_INST_LDS SQ_ACTIVE_INST_VALU")


def profile_commands(w: str) -> dict:
    """The rocprofv3 runs behind a workload's profiles (REPO = repository
    root, OUT = the folder that receives the profiler output; write_profiles
    reads that folder)."""
    run = f"python3 -u $REPO/bench.py --only {w}"
    return {
        "stats": f"cd /tmp && rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof_{w} "
                 f"-o {w} -- {run} --steps 10 --warmup 2",
        "FETCH_SIZE": f"cd /tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d "
                      f"$OUT/pmc_FETCH_SIZE_{w} -o pmc -- {run} --steps 3 --warmup 1 --copy-calibration",
        "WRITE_SIZE": f"cd /tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d "
                      f"$OUT/pmc_WRITE_SIZE_{w} -o pmc -- {run} --steps 3 --warmup 1 --copy-calibration",
        "sq": f"cd /tmp && rocprofv3 --pmc {SQ_COUNTERS} --output-format csv -d $OUT/pmc_sq_{w} -o pmc "
              f"-- {run} --steps 3 --warmup 1",
    }


def _csv_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _last_json(path):
    with open(path) as f:
        lines = [ln for ln in f.read().splitlines() if ln.startswith("{")]
    return json.loads(lines[-1])


def _kname(full: str) -> str:
    """A kernel's name without return type, namespaces and argument list."""
    import re
    return re.sub(r"\([^()]*\)\s*$", "", full).split("::")[-1]


def _counter_means(path: str, prefix: str) -> tuple:
    """Per-dispatch mean of every counter of the kernels whose short name
    starts with prefix, and the number of dispatches."""
    import collections
    vals = collections.defaultdict(list)
    for r in _csv_rows(path):
        if _kname(r["Kernel_Name"]).startswith(prefix):
            vals[r["Counter_Name"]].append(float(r["Counter_Value"]))
    n = max((len(v) for v in vals.values()), default=0)
    return {k: sum(v) / len(v) for k, v in vals.items()}, n


def write_profiles(src: str, bench_log: str) -> None:
    """Summaries of the rocprofv3 runs in src (profile_commands) and the
    default bench line in bench_log, for the current kernel sources."""
    live = _last_json(bench_log)
    out_dir = os.path.join(ROOT, "profiles")
    for name, w, prefix, family, key in PROFILES:
        only = _last_json(os.path.join(src, f"only_{w}.log"))["result"]
        roof = only[key]
        cmds = profile_commands(w)
        stats = _csv_rows(os.path.join(src, f"prof_{w}", f"{w}_kernel_stats.csv"))
        main_k = [r for r in stats if _kname(r["Name"]).startswith(prefix)]
        main_k = max(main_k, key=lambda r: float(r["TotalDurationNs"]))
        kname = main_k["Name"]
        kshort = _kname(kname)
        copy = {}
        traffic = {}
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            path = os.path.join(src, f"pmc_{c}_{w}", "pmc_counter_collection.csv")
            cm, _ = _counter_means(path, "k_copy")
            copy[c] = cm[c]
            km, n = _counter_means(path, kshort)
            traffic[c] = (km[c], n)
        ff = 536870912 / (copy["FETCH_SIZE"] * 1024)
        wf = 536870912 / (copy["WRITE_SIZE"] * 1024)
        fetch = traffic["FETCH_SIZE"][0] * 1024 * ff
        write = traffic["WRITE_SIZE"][0] * 1024 * wf
        sq, nsq = _counter_means(os.path.join(src, f"pmc_sq_{w}", "pmc_counter_collection.csv"), kshort)
        sq["launches"] = nsq
        alg_bytes = float(roof["hbm_alg_bytes_per_launch"])
        ops = float(roof["alg_ops_per_launch"])
        avg_us = float(main_k["AverageNs"]) / 1e3
        rec = {"workload": w, "kernel": kname, "source_hash": kernel_source_hash(family),
               "source_files": KERNEL_SOURCES[family], "rocprof_average_us": avg_us,
               "commands": [cmds["stats"], cmds["FETCH_SIZE"], cmds["WRITE_SIZE"], cmds["sq"]],
               "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
               "traffic_bytes_per_launch": fetch + write,
               "copy_calibration": {"bytes": 536870912, "fetch_kib_raw": copy["FETCH_SIZE"],
                                    "write_kib_raw": copy["WRITE_SIZE"], "fetch_factor": ff, "write_factor": wf},
               "launches_counted": {"fetch": traffic["FETCH_SIZE"][1], "write": traffic["WRITE_SIZE"][1]},
               "alg_bytes_per_launch": alg_bytes, "sq": sq}
        with open(os.path.join(out_dir, name + ".json"), "w") as f:
            json.dump(rec, f, indent=1)
        tot = sum(float(r["TotalDurationNs"]) for r in stats)
        L = [f"# rocprofv3: {name} (MI355X)", "", "Kernel statistics, command (REPO = repository root, OUT = profiler output folder):",
             "", "    " + cmds["stats"], "", "| kernel | calls | average (us) | min (us) | max (us) | share |",
             "|---|---|---|---|---|---|"]
        for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:8]:
            nm = r["Name"] if len(r["Name"]) <= 90 else r["Name"][:87] + "..."
            L.append(f"| {nm} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {100 * float(r['TotalDurationNs']) / tot:.1f} % |")
        cyc = 4 * sq.get("SQ_INSTS_VALU", 0) / 1024
        kc = avg_us * 1e-6 * 2.4e9
        L += ["", "## HBM traffic of the main kernel (rocprofv3 --pmc, one counter per run)", "",
              "    " + cmds["FETCH_SIZE"], "    " + cmds["WRITE_SIZE"], "",
              f"- copy calibration: a 512 MiB device copy (wect_calib_copy) read {copy['FETCH_SIZE']:.1f} KiB "
              f"(FETCH_SIZE) and wrote {copy['WRITE_SIZE']:.1f} KiB (WRITE_SIZE): factors {ff:.4f} and {wf:.4f}",
              f"- `{kshort}` per launch: fetch {fetch / 1e6:.3f} MB, write {write / 1e6:.3f} MB (scaled), "
              f"{traffic['FETCH_SIZE'][1]} launches",
              f"- algorithmic bytes per launch: {alg_bytes / 1e6:.3f} MB; counter / algorithmic = "
              f"{(fetch + write) / alg_bytes:.2f}", "",
              "## Instruction counters of the main kernel (rocprofv3 --pmc, SQ block)", "", "    " + cmds["sq"], "",
              f"- per launch ({nsq} launches): {sq.get('SQ_INSTS_VALU', 0):.4g} VALU, {sq.get('SQ_INSTS_LDS', 0):.4g} "
              f"LDS, {sq.get('SQ_INSTS_SALU', 0):.4g} scalar wavefront instructions; {sq.get('SQ_WAVES', 0):.0f} "
              f"wavefronts",
              f"- VALU issue: {cyc:.4g} cycles per SIMD (4 cycles per wavefront instruction, 1024 SIMDs) against "
              f"{kc:.4g} cycles of the kernel at 2.4 GHz: {100 * cyc / kc:.0f} % busy",
              f"- {64 * sq.get('SQ_INSTS_VALU', 0) / ops:.2f} VALU lane-instructions per algorithmic lane-op "
              f"({ops:.4g} algorithmic lane-ops per launch)"]
        cal = live.get("calibration", {}).get("lds_add_per_s", {})
        if sq.get("SQ_WAVE_CYCLES") and cal:
            per_cc = lambda rate: rate / 64 / 256 / 2.4e9  # wavefront instructions per CU-cycle
            L.append(f"- LDS: {sq.get('SQ_INSTS_LDS', 0) / 256 / kc:.3f} wavefront instructions per CU-cycle (reads, "
                     f"writes and atomics); conflict-free atomic adds alone sustain {per_cc(cal['u32']):.3f} (u32) "
                     f"and {per_cc(cal['u64']):.3f} (u64) per CU-cycle (wect_calib_lds_atomics, same run as the live "
                     f"line below); wavefronts wait on LDS for "
                     f"{100 * sq.get('SQ_WAIT_INST_LDS', 0) / sq['SQ_WAVE_CYCLES']:.0f} % of their cycles "
                     f"(SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES)")
        # the same workload in the default bench run
        lr = live["roofline"] if w == "volumes3d" else live["configs"][w][key]
        step = {"volumes3d": live["ms_per_step"], "images2d": live["configs"]["images2d"]["ms"]}.get(w)
        if step is None:
            step = live["configs"][w]["fwd_ms" if key == "roofline_fwd" else "fwd_bwd_ms"]
        L += ["", f"Live measurement in the default `python bench.py` run on the same sources: `{lr['kernel']}` "
              f"{lr['kernel_ms'] * 1e3:.1f} us per launch with HIP events on its stream (rocprofv3 average above: "
              f"{avg_us:.1f} us); {step * 1e3:.1f} us per step; {lr['alg_ops_per_launch']:.4g} algorithmic lane-ops "
              f"per launch = {lr['frac']:.3f} of the 39.3 T lane-ops/s VALU peak"
              + (f" ({lr['frac_staged']:.3f} counting only the {100 * lr['staged_fraction']:.1f} % of included "
                 f"vertices that have a nonzero combined weight and are staged)" if "frac_staged" in lr else "")
              + f"; {lr['hbm_alg_bytes_per_launch'] / 1e6:.2f} MB algorithmic HBM bytes = {lr['hbm_frac']:.4f} of "
              f"8 TB/s."]
        with open(os.path.join(out_dir, name + ".md"), "w") as f:
            f.write("\n".join(L) + "\n")
        print(f"wrote profiles/{name}.md/.json", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-single", action="store_true", help="skip the one-complex-per-launch comparisons")
    ap.add_argument("--no-calibrate", action="store_true", help="skip the copy / LDS atomic calibration")
    ap.add_argument("--only", choices=WORKLOADS, default=None, help="run one workload only (profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (counter calibration for profiling runs)")
    ap.add_argument("--write-profiles", nargs=2, metavar=("RESULTS_DIR", "BENCH_LOG"), default=None,
                    help="write profiles/*.md/.json from rocprofv3 output (no GPU needed)")
    a = ap.parse_args(argv)
    if a.write_profiles:
        write_profiles(*a.write_profiles)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (sharding across GPUs is not implemented); --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)

    import torch

    from paper_2511_03909_amd import _lib as L
    from paper_2511_03909_amd import api as W

    torch.cuda.set_device(0)
    if a.copy_calibration:
        src_t = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")   # 512 MiB
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            L.check(L.lib().wect_calib_copy(dst_t.data_ptr(), src_t.data_ptr(), src_t.numel() * 4,
                                            torch.cuda.current_stream().cuda_stream), "copy")
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src_t.numel() * 4, "launches": 3}), flush=True)
        del src_t, dst_t
    calib = None if (a.no_calibrate or a.only) else calibrate(W)

    if a.only:
        fn = {"volumes3d": lambda: run_volumes3d(W, a, None, single=False)[0],
              "images2d": lambda: run_images2d(W, a, None, single=False)[0],
              "kuhn3d": lambda: run_kuhn3d(W, a, None),
              "diffbatch": lambda: run_diffbatch(W, a, None, single=False)[0],
              "mesh2d": lambda: run_mesh2d(W, a, None)}[a.only]
        print(json.dumps({"only": a.only, "result": fn(), "kernel_sources": kernel_source_hash()}), flush=True)
        return

    head, w4 = run_volumes3d(W, a, calib, single=not a.no_single)
    sec = head["ms"] * 1e-3
    result = {
        "metric": METRIC,
        "value": head["items_per_s"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": w4.name, "volumes": len(w4.complexes), "sides": "64-192 per axis",
                   "directions": int(w4.dirs.shape[0]), "thresholds": int(w4.thr.shape[0]),
                   "cells": head["cells"], "included_vertices": head["included_vertices"],
                   "staged_vertices": head["staged_vertices"],
                   "items_per_step": head["items"], "mode": "batched forward, one call for all volumes"},
        "roofline": head["roofline"],
        "calibration": calib,
        "kernel_sources": kernel_source_hash(),
    }
    result["per_call"] = head["per_call"]
    if "one_per_launch" in head:
        result["one_per_launch"] = head["one_per_launch"]
    print(json.dumps({"progress": "headline done", "ms_per_step": head["ms"]}), file=sys.stderr, flush=True)
    if not a.no_extras:
        configs = {}
        configs["images2d"], _ = run_images2d(W, a, calib, single=not a.no_single)
        configs["kuhn3d"] = run_kuhn3d(W, a, calib)
        configs["diffbatch"], diff = run_diffbatch(W, a, calib, single=not a.no_single)
        configs["mesh2d"] = run_mesh2d(W, a, calib)
        print(json.dumps({"progress": "configs done"}), file=sys.stderr, flush=True)
        more = {}
        run_more(W, a, more, diff)
        result["configs"] = configs
        result["extras"] = more
    if not a.no_cpu:
        cells_of = [cubical_cell_count(C) for C in w4.complexes]
        result["cpu_baseline"] = cpu_baseline(w4, cells_of)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
