"""Benchmark: WECT simplex*directions per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]

Headline workload: 256 uint8 images of 128x128 (Gaussian random fields, sigma
4 px), pixels with intensity > 64 are vertices, cells induced, cell weight =
max vertex intensity, 64 directions on S^1, 128 thresholds on [-sqrt2, sqrt2],
int32 output [256, 64, 128], all images in one batched call.  One step = one
batched forward over the whole batch, inputs resident in HBM.  Before the
warm-up steps the step runs back to back for half a second, untimed, so that
the GPU's clocks have left their idle state.

Items = directions x (cells of every dimension, vertices included), whatever
shortcut the kernel takes.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WECT simplex·directions/sec fwd & fwd+bwd, batched vs 1-per-launch; HBM GB/s"
UNIT = "simplex·directions/s"
HBM_PEAK_GBPS = 8000.0
# VALU lane-operations per second: 256 CUs x 64 lanes x 2.4 GHz (non-packed, non-fused)
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


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


def relaxation_terms(cx, grid, lam: float, chunk: int = 1 << 20, vertices_only: bool = False) -> int:
    """Number of sigmoid window terms of the relaxation: over every simplex (or,
    for the vertex-centric kernels, every vertex) and direction, the thresholds
    within 17 / lam of its maximum height (bookkeeping on the device with torch;
    heights from a float32 matmul)."""
    import torch
    R = 17.0 / lam
    thr = grid.thr
    h = cx.coords @ grid.dirs.t()                     # [V, d]
    total = 0
    offs = [0] + [int(v) for v in (cx.vert_off[1:].tolist() if cx.vert_off is not None else [h.shape[0]])]
    for dim in range(1 if vertices_only else cx.top_dim + 1):
        if dim == 0:
            rows = h
        else:
            simp = cx.simplices[dim].long()
            if cx.simp_off is not None and cx.simp_off[dim] is not None:
                so = cx.simp_off[dim]
                base = torch.repeat_interleave(torch.tensor(offs[:-1], device=h.device), so[1:] - so[:-1])
                simp = simp + base[:, None]
            rows = None
        n = h.shape[0] if dim == 0 else simp.shape[0]
        for i in range(0, n, chunk):
            hm = rows[i:i + chunk] if dim == 0 else h[simp[i:i + chunk]].amax(dim=1)
            lo = torch.searchsorted(thr, (hm - R).contiguous(), right=False)
            hi = torch.searchsorted(thr, (hm + R).contiguous(), right=True)
            total += int((hi - lo).sum())
    return total


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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_03909_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name: str):
    """HBM traffic per launch measured with rocprofv3 counters for the current
    kernel sources (profiles/<name>.json), or None."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_launch")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the one-complex-per-launch comparison (profiling the batched kernel alone)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (counter calibration for profiling runs)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2511_03909_amd import api as W

    torch.cuda.set_device(0)
    dev = "cuda"
    if a.copy_calibration:
        src_t = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)   # 512 MiB
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src_t.numel() * 4, "launches": 3}), flush=True)
        del src_t, dst_t

    # ---------------- headline: cubical 2D batch, batched forward ----------------
    w = synth.cfg2()
    cx = W.CubicalBatch.from_host(w.complexes, device=dev)
    grid = W.Grid(w.dirs, w.thr, device=dev)
    d, T, B = grid.d, grid.T, cx.B
    cells = sum(cubical_cell_count(C) for C in w.complexes)
    nverts = sum(included_vertices(C) for C in w.complexes)
    items = d * cells
    out = torch.empty((B, d, T), dtype=torch.int32, device=dev)
    ws = torch.empty(max(1, W.wect_workspace_bytes(cx, grid)), dtype=torch.uint8, device=dev)

    def step():
        W.wect_forward(cx, grid, out=out, ws=ws)

    settle(step)
    sec = timed(step, a.steps, a.warmup)
    # live kernel timing of the dominant (histogram) kernel with HIP events on its stream
    W.profile_enable(True)
    W.profile_read(reset=True)
    nprof = max(10, a.steps)
    for _ in range(nprof):
        step()
    torch.cuda.synchronize()
    prof = W.profile_read(reset=True)
    W.profile_enable(False)
    k_ms = prof["fwd_ms"] / max(1, prof["fwd_launches"])
    # cold runs: before each, a 1 GiB write evicts the inputs from the caches
    # (L2 and the 256 MiB Infinity Cache), then one step is timed with events
    flush = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    cold = []
    for _ in range(5):
        flush.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1))
    del flush

    # algorithmic work of the histogram kernel (per launch)
    # VALU lane-ops per included vertex x direction (top-corner rule, n = 2):
    #   (n-1) add + ceil(log2(T+1)) search + 1 select + 1 add
    ops_per_vd = (2 - 1) + math.ceil(math.log2(T + 1)) + 1 + 1
    alg_ops = ops_per_vd * nverts * d
    # algorithmic HBM bytes: read every voxel once (uint8) + the axes, write the int32 output once
    alg_bytes = cx.total_voxels * 1 + int(cx.axis.numel()) * 4 + B * d * T * 4
    traffic = load_traffic("cubical_fwd_2d_256x128x128_d64_T128")
    roofline = {
        "bound": "alu",
        "achieved": alg_ops / (k_ms * 1e-3) / 1e12,
        "peak": VALU_PEAK_TOPS,
        "unit": "TOP/s",
        "frac": (alg_ops / (k_ms * 1e-3) / 1e12) / VALU_PEAK_TOPS,
        "traffic": traffic,
        "kernel": "k_cub_fwd<2, vertex-max>",
        "kernel_ms": k_ms,
        "alg_ops_per_launch": alg_ops,
        "hbm_alg_bytes_per_launch": alg_bytes,
        "hbm_frac": (alg_bytes / (k_ms * 1e-3) / 1e9) / HBM_PEAK_GBPS,
        "hbm_achieved_GBps": alg_bytes / (k_ms * 1e-3) / 1e9,
        # one LDS atomic add per included vertex and direction (lane-level)
        "lds_atomics_per_s": nverts * d / (k_ms * 1e-3),
    }
    result = {
        "metric": METRIC,
        "value": items / sec,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": w.name, "images": B, "side": 128, "directions": d, "thresholds": T,
                   "cells": cells, "included_vertices": nverts, "items_per_step": items,
                   "mode": "batched forward, one call for all images"},
        "roofline": roofline,
        "cold_ms_per_step": sorted(cold)[len(cold) // 2],
    }

    result["kernel_sources"] = kernel_source_hash()

    # ---------------- one complex per launch (same images) ----------------
    if a.no_single:
        print(json.dumps(result), flush=True)
        return
    singles = [W.CubicalBatch.from_host([C], device=dev) for C in w.complexes]
    outs = [torch.empty((1, d, T), dtype=torch.int32, device=dev) for _ in singles]
    ws1 = torch.empty(max(1, max(W.wect_workspace_bytes(s, grid) for s in singles)), dtype=torch.uint8,
                      device=dev)

    def step_single():
        for s, o in zip(singles, outs):
            W.wect_forward(s, grid, out=o, ws=ws1)

    sec1 = timed(step_single, max(3, a.steps // 5), 2)
    result["one_per_launch"] = {"value": items / sec1, "ms_per_step": sec1 * 1e3,
                                "batched_speedup": sec1 / sec}

    if not a.no_extras:
        extras = {}
        # differentiation workload: batched forward + adjoint to vertex weights
        w5 = synth.cfg5()
        cx5 = W.SimplicialBatch.from_host(w5.complexes, device=dev)
        g5 = W.Grid(w5.dirs, w5.thr, device=dev)
        n5 = sum(cx5.counts)
        it5 = g5.d * n5
        gout = torch.randn((cx5.B, g5.d, g5.T), device=dev)
        o5 = torch.empty((cx5.B, g5.d, g5.T), dtype=torch.float32, device=dev)
        gv5 = torch.empty(cx5.counts[0], dtype=torch.float32, device=dev)
        ws5 = torch.empty(max(1, W.wect_workspace_bytes(cx5, g5, True)), dtype=torch.uint8, device=dev)
        t_fb = timed(lambda: W.wect_batched(cx5, g5, gout, out=o5, grads=gv5, ws=ws5), 10, 2)
        t_f = timed(lambda: W.wect_batched(cx5, g5, None, out=o5, ws=ws5), 10, 2)
        # graph-captured forward + backward
        graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            W.wect_batched(cx5, g5, gout, out=o5, grads=gv5, ws=ws5)
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(graph):
            W.wect_batched(cx5, g5, gout, out=o5, grads=gv5, ws=ws5)
        t_g = timed(graph.replay, 10, 2)
        # the same 64 complexes, one call per complex (forward, and forward + backward)
        singles5 = [W.SimplicialBatch.from_host([K], device=dev) for K in w5.complexes]
        ws5s = torch.empty(max(1, max(W.wect_workspace_bytes(c, g5, True) for c in singles5)), dtype=torch.uint8,
                           device=dev)
        go5 = [gout[b:b + 1].contiguous() for b in range(cx5.B)]
        o5s = [torch.empty((1, g5.d, g5.T), dtype=torch.float32, device=dev) for _ in singles5]
        gv5s = [torch.empty(c.counts[0], dtype=torch.float32, device=dev) for c in singles5]
        t_f1 = timed(lambda: [W.wect_batched(c, g5, None, out=o, ws=ws5s) for c, o in zip(singles5, o5s)], 3, 1)
        t_fb1 = timed(lambda: [W.wect_batched(c, g5, gg, out=o, grads=gv, ws=ws5s)
                               for c, gg, o, gv in zip(singles5, go5, o5s, gv5s)], 3, 1)
        extras["differentiation_batch64"] = {
            "workload": w5.name, "items": it5, "fwd_items_per_s": it5 / t_f, "fwd_bwd_items_per_s": it5 / t_fb,
            "fwd_ms": t_f * 1e3, "fwd_bwd_ms": t_fb * 1e3, "fwd_bwd_graph_ms": t_g * 1e3,
            "one_per_launch": {"fwd_ms": t_f1 * 1e3, "fwd_bwd_ms": t_fb1 * 1e3,
                               "fwd_batched_speedup": t_f1 / t_f, "fwd_bwd_batched_speedup": t_fb1 / t_fb}}
        # the same complexes through the general vertex-filter WECF, with the filter values
        # given as an array (here the heights of the 128 directions, formed on the device)
        F5 = (cx5.coords @ g5.dirs.t()).contiguous()
        o5w = torch.empty((cx5.B, F5.shape[1], g5.T), dtype=torch.float32, device=dev)
        ws5w = torch.empty(max(1, W.wecf_workspace_bytes(cx5, F5.shape[1], g5.T)), dtype=torch.uint8, device=dev)
        t_w = timed(lambda: W.wecf_forward(cx5, F5, g5.thr, out=o5w, ws=ws5w), 5, 1)
        extras["differentiation_batch64"]["wecf_filter_array_m128"] = {
            "fwd_ms": t_w * 1e3, "items_per_s": it5 / t_w,
            "note": "filter values read from a [V, 128] array instead of formed from coordinates"}
        del singles5, o5s, gv5s, go5, ws5s, F5, o5w, ws5w
        # sigmoid relaxation of the same batch (lam x threshold spacing = 2): forward, and
        # the adjoint to coordinates, directions and vertex weights; per-cell kernels and the
        # vertex-centric kernels over the lower-star index (built once per topology)
        thr5 = w5.thr.astype(np.float64)
        lam5 = float(np.float32(2.0 * (thr5.size - 1) / (thr5[-1] - thr5[0])))
        os5 = torch.empty((cx5.B, g5.d, g5.T), dtype=torch.float32, device=dev)
        t_build = timed(lambda: W.lower_star_index(cx5, cache=False), 3, 1)
        index5 = W.lower_star_index(cx5)
        # algorithmic lane-ops: per sigmoid window term, forward sub, mul, exp2, add, reciprocal,
        # weight product, rounding to the fixed-point grid, accumulate = 8; adjoint the same up to
        # the reciprocal, then two products and two accumulations = 9.  Per coface row and direction
        # (vertex-centric kernels): the other vertices' heights (2n - 1 each), one comparison each,
        # one accumulation.
        nrow_ops = sum((dm + 1) * cx5.counts[dm] * (dm * (2 * cx5.n - 1) + dm + 1)
                       for dm in range(1, cx5.top_dim + 1)) * g5.d
        terms_cells = relaxation_terms(cx5, g5, lam5)
        terms_verts = relaxation_terms(cx5, g5, lam5, vertices_only=True)
        relax = {"lam": lam5, "index_build_ms": t_build * 1e3, "index_bytes": int(index5.numel()),
                 "note": "sigmoid window of |lam (t - h)| <= 17, about 17 thresholds per window; adjoint to "
                         "coordinates [V,2], directions [128,2] and vertex weights"}
        for name, index, terms, extra_ops in (("cells", None, terms_cells, 0),
                                              ("lower_star", index5, terms_verts, nrow_ops)):
            wss = torch.empty(max(1, W.smooth_workspace_bytes(cx5, g5, lam5, index)), dtype=torch.uint8, device=dev)
            t_sf = timed(lambda: W.smooth_forward(cx5, g5, lam5, out=os5, ws=wss, index=index), 5, 1)
            t_sb = timed(lambda: W.smooth_backward(cx5, g5, lam5, gout, index=index), 5, 1)
            W.profile_enable(True)
            W.profile_read(reset=True)
            for _ in range(5):
                W.smooth_forward(cx5, g5, lam5, out=os5, ws=wss, index=index)
                W.smooth_backward(cx5, g5, lam5, gout, index=index)
            torch.cuda.synchronize()
            ps = W.profile_read(reset=True)
            W.profile_enable(False)
            kf_ms = ps["fwd_ms"] / max(1, ps["fwd_launches"])
            kb_ms = ps["bwd_ms"] / max(1, ps["bwd_launches"])
            of, ob = 8 * terms + extra_ops, 9 * terms + extra_ops
            relax[name] = {
                "fwd_ms": t_sf * 1e3, "bwd_ms": t_sb * 1e3, "fwd_kernel_ms": kf_ms, "bwd_kernel_ms": kb_ms,
                "fwd_items_per_s": it5 / t_sf, "bwd_items_per_s": it5 / t_sb, "window_terms": terms,
                "roofline_fwd": {"bound": "alu", "achieved": of / (kf_ms * 1e-3) / 1e12, "peak": VALU_PEAK_TOPS,
                                 "unit": "TOP/s", "frac": of / (kf_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS},
                "roofline_bwd": {"bound": "alu", "achieved": ob / (kb_ms * 1e-3) / 1e12, "peak": VALU_PEAK_TOPS,
                                 "unit": "TOP/s", "frac": ob / (kb_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS}}
            del wss
        if not a.no_cpu:
            # the float64 oracle on a bounded sample: the smallest complex, 8 directions
            from oracle import smooth as osm
            b0 = int(np.argmin([K.coords.shape[0] for K in w5.complexes]))
            t0 = time.perf_counter()
            osm.smooth_wect(w5.complexes[b0], w5.dirs[:8], w5.thr, lam5)
            tc = time.perf_counter() - t0
            relax["cpu_oracle"] = {"value": 8 * sum(w5.complexes[b0].counts()) / tc, "unit": "simplex·directions/s",
                                   "cores": 1, "kind": "oracle",
                                   "sample": f"complex {b0} ({sum(w5.complexes[b0].counts())} simplices), "
                                             f"8 directions, {tc:.1f} s"}
        extras["differentiation_batch64"]["relaxation_lam_spacing2"] = relax
        del cx5, o5, gv5, ws5, gout, os5, index5
        # the relaxation on the 3D Kuhn mesh (tetrahedra; 74 cofaces per inner vertex), vertex-centric
        w3r = synth.cfg3()
        cx3r = W.SimplicialBatch.from_host(w3r.complexes, device=dev)
        g3r = W.Grid(w3r.dirs, w3r.thr, device=dev)
        t3r = w3r.thr.astype(np.float64)
        lam3 = float(np.float32(2.0 * (t3r.size - 1) / (t3r[-1] - t3r[0])))
        idx3 = W.lower_star_index(cx3r)
        o3r = torch.empty((1, g3r.d, g3r.T), dtype=torch.float32, device=dev)
        ws3r = torch.empty(max(1, W.smooth_workspace_bytes(cx3r, g3r, lam3, idx3)), dtype=torch.uint8, device=dev)
        go3 = torch.randn((1, g3r.d, g3r.T), device=dev)
        t3f = timed(lambda: W.smooth_forward(cx3r, g3r, lam3, out=o3r, ws=ws3r, index=idx3), 3, 1)
        t3b = timed(lambda: W.smooth_backward(cx3r, g3r, lam3, go3, index=idx3), 3, 1)
        it3r = g3r.d * sum(cx3r.counts)
        extras["relaxation_3d_kuhn64"] = {"workload": w3r.name, "lam": lam3, "fwd_ms": t3f * 1e3,
                                          "bwd_ms": t3b * 1e3, "items": it3r, "fwd_items_per_s": it3r / t3f,
                                          "path": "lower_star"}
        del cx3r, idx3, o3r, ws3r, go3
        # 3D simplicial, float32 weights
        w3 = synth.cfg3()
        cx3 = W.SimplicialBatch.from_host(w3.complexes, device=dev)
        g3 = W.Grid(w3.dirs, w3.thr, device=dev)
        it3 = g3.d * sum(cx3.counts)
        o3 = torch.empty((1, g3.d, g3.T), dtype=torch.float32, device=dev)
        ws3 = torch.empty(max(1, W.wect_workspace_bytes(cx3, g3)), dtype=torch.uint8, device=dev)
        t3 = timed(lambda: W.wect_forward(cx3, g3, out=o3, ws=ws3), 5, 1)
        extras["simplicial_3d_kuhn64"] = {"workload": w3.name, "items": it3, "items_per_s": it3 / t3,
                                          "ms": t3 * 1e3}
        del cx3, o3, ws3
        # 2D simplicial, small: launch-latency bound
        w1 = synth.cfg1()
        cx1 = W.SimplicialBatch.from_host(w1.complexes, device=dev)
        g1 = W.Grid(w1.dirs, w1.thr, device=dev)
        it1 = g1.d * sum(cx1.counts)
        o1 = torch.empty((1, g1.d, g1.T), dtype=torch.int32, device=dev)
        ws1b = torch.empty(max(1, W.wect_workspace_bytes(cx1, g1)), dtype=torch.uint8, device=dev)
        t1 = timed(lambda: W.wect_forward(cx1, g1, out=o1, ws=ws1b), 50, 5)
        extras["simplicial_2d_32x32"] = {"workload": w1.name, "items": it1, "items_per_s": it1 / t1,
                                         "us_per_call": t1 * 1e6}
        # 3D cubical, 16 volumes of uneven size, one call
        w4 = synth.cfg4()
        cx4 = W.CubicalBatch.from_host(w4.complexes, device=dev)
        g4 = W.Grid(w4.dirs, w4.thr, device=dev)
        cells4 = sum(cubical_cell_count(C) for C in w4.complexes)
        it4 = g4.d * cells4
        o4 = torch.empty((cx4.B, g4.d, g4.T), dtype=torch.int32, device=dev)
        ws4 = torch.empty(max(1, W.wect_workspace_bytes(cx4, g4)), dtype=torch.uint8, device=dev)
        t4 = timed(lambda: W.wect_forward(cx4, g4, out=o4, ws=ws4), 3, 1)
        singles4 = [W.CubicalBatch.from_host([C], device=dev) for C in w4.complexes]
        o4s = [torch.empty((1, g4.d, g4.T), dtype=torch.int32, device=dev) for _ in singles4]
        ws4s = torch.empty(max(1, max(W.wect_workspace_bytes(c, g4) for c in singles4)), dtype=torch.uint8,
                           device=dev)
        t41 = timed(lambda: [W.wect_forward(c, g4, out=o, ws=ws4s) for c, o in zip(singles4, o4s)], 2, 1)
        extras["cubical_3d_16vol"] = {"workload": w4.name, "items": it4, "items_per_s": it4 / t4, "ms": t4 * 1e3,
                                      "one_per_launch_ms": t41 * 1e3, "batched_speedup": t41 / t4}
        del cx4, o4, ws4, singles4, o4s, ws4s
        # the headline images as weighted Freudenthal complexes built on the device
        # (vertex weights = intensities), then their WECT through the simplicial path
        cxf = W.CubicalBatch.from_host(w.complexes, device=dev)
        t_build = timed(lambda: W.freudenthal_from_images(cxf), 10, 2)
        sbf = W.freudenthal_from_images(cxf)
        nf = sum(sbf.counts)
        of = torch.empty((sbf.B, d, T), dtype=torch.float32, device=dev)
        wsf = torch.empty(max(1, W.wect_workspace_bytes(sbf, grid)), dtype=torch.uint8, device=dev)
        t_fw = timed(lambda: W.wect_forward(sbf, grid, out=of, ws=wsf), 10, 2)
        extras["freudenthal_2d_256x128x128"] = {
            "workload": "headline images as Freudenthal complexes (every pixel a vertex, vertex-max weights)",
            "build_ms": t_build * 1e3, "simplices": nf, "wect_ms": t_fw * 1e3, "items_per_s": d * nf / t_fw}
        del cxf, sbf, of, wsf
        # ECF of an image (intensity as the vertex filter), uniform intensities as in the
        # paper's throughput measurement; pixels (voxels) per second at 1,000 and 10,000 thresholds
        ecf = {}
        for shape in ((2048, 2048), (4096, 4096), (8192, 8192), (128, 128, 128), (256, 256, 256), (512, 512, 512)):
            C = synth.uniform_image(shape, 0)
            cxe = W.CubicalBatch.from_host([C], device=dev)
            wse = torch.empty(max(1, W.image_ecf_workspace_bytes(cxe)), dtype=torch.uint8, device=dev)
            npx = int(np.prod(shape))
            key = "x".join(str(v) for v in shape)
            for Te in (1000, 10000):
                thr_e = torch.as_tensor(synth.ecf_thresholds(Te), device=dev)
                oe = torch.empty((1, Te), dtype=torch.int32, device=dev)
                te = timed(lambda: W.image_ecf(cxe, thr_e, out=oe, ws=wse), 20, 3)
                ecf[f"{key}_T{Te}"] = {"ms": te * 1e3, "Gpix_per_s": npx / te / 1e9,
                                       "hbm_GBps_at_1B_per_px": npx / te / 1e9}
            del cxe, wse
        extras["image_ecf"] = {"workload": "uniform uint8 intensities, every pixel a vertex, unweighted ECF",
                               "results": ecf}
        result["extras"] = extras

    # ---------------- CPU oracle on a bounded sample of the headline workload ----------------
    if not a.no_cpu:
        import oracle
        # images in strided order (0, 8, 16, ..., 1, 9, ...) until about 10 s of CPU time or all are done
        order = [b for r in range(8) for b in range(r, B, 8)]
        sample = []
        t0 = time.perf_counter()
        for b in order:
            oracle.wect(w.complexes[b], w.dirs, w.thr)
            sample.append(b)
            if time.perf_counter() - t0 >= 10.0:
                break
        tc = time.perf_counter() - t0
        it_cpu = d * sum(cubical_cell_count(w.complexes[b]) for b in sample)
        result["cpu_baseline"] = {"value": it_cpu / tc, "unit": UNIT, "cores": 1, "kind": "oracle",
                                  "sample": f"{len(sample)} of {B} images (strided order), all {d} directions, "
                                            f"{tc:.1f} s, numpy single thread (no BLAS calls)"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
