"""Launch-shape autotuner.

For one request (a complex batch and a sampling grid) it times the forward for a
set of launch shapes (threads per block, blocks per compute unit, minimum stream
items per block, work decomposition) and keeps the fastest; then, with that
shape, it times how the thresholds are split between LDS-resident tiles: all
thresholds in one pass (when their histogram fits), or tiles of a half or a
third of them, one pass each (a smaller histogram leaves room for more blocks
per compute unit and a larger staging area, at the price of re-reading the
cells).  Results are cached in a JSON file keyed by a signature of the request
(kind, ambient dimension, batch size, total cells rounded to a power of two,
directions, thresholds, dtype), so a workload of the same shape reuses the
choice.  Then, for cubical requests with more than 64 directions, it times one
and two directions per lane (a direction tile of 64 or 128).  Last, for
simplicial requests, it times staging tiles of a half and three quarters of
the block besides the automatic one (fewer staged cells per tile, the same
resident blocks).

    from paper_2511_03909_amd import tune
    shape = tune.tune(cx, grid)        # times, caches, applies
    tune.apply(shape)                  # or later: tune.lookup(cx, grid)
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import api

DEFAULT_CACHE = os.environ.get("WECT_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "wect_tune.json"))

# (block, blocks_per_cu, min_items_per_block, decomposition)
CANDIDATES: Tuple[Tuple[int, int, int, int], ...] = (
    (1024, 0, 0, 1), (1024, 1, 0, 1), (1024, 2, 0, 1),
    (512, 0, 0, 1), (512, 2, 0, 1), (512, 4, 0, 1),
    (256, 0, 0, 1), (256, 4, 0, 1),
    (512, 0, 256, 1), (1024, 0, 256, 1), (512, 0, 8192, 1),
    (1024, 0, 0, 2), (512, 0, 0, 2), (256, 0, 0, 2),
)


def signature(cx, grid) -> str:
    if isinstance(cx, api.CubicalBatch):
        cells = cx.total_voxels
        kind = "cubical"
    else:
        cells = sum(cx.counts)
        kind = "simplicial"
    bucket = 1 << max(0, int(math.ceil(math.log2(max(cells, 1)))))
    return f"{kind}/n{cx.n}/B{cx.B}/cells~{bucket}/d{grid.d}/T{grid.T}/dtype{cx.dtype}"


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: Dict[str, dict]) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(shape: Optional[dict]) -> None:
    if shape:
        api.set_launch(shape["block"], shape["blocks_per_cu"], shape["min_items_per_block"],
                       shape.get("decomposition", 0), shape.get("threshold_tile", 0),
                       shape.get("directions_per_lane", 0), stage_entries=shape.get("stage_entries", 0))
    else:
        api.set_launch()


def tile_candidates(T: int) -> Tuple[int, ...]:
    """Threshold tiles tried after the shape: automatic (0), and about a half
    and a third of T for longer threshold arrays."""
    if T < 96:
        return (0,)
    return (0, -(-T // 2), -(-T // 3))


def lane_candidates(cx, grid) -> Tuple[int, ...]:
    """Directions per lane tried for cubical requests with more than one
    64-direction tile (automatic is 2 there): 1 and 2."""
    if isinstance(cx, api.CubicalBatch) and grid.d > 64:
        return (1, 2)
    return ()


def stage_candidates(cx, block: int) -> Tuple[int, ...]:
    """Staging tiles tried for simplicial requests after the other choices: a
    half and three quarters of the block (the automatic one is already timed)."""
    if isinstance(cx, api.CubicalBatch):
        return ()
    b = block or 1024
    return tuple(sorted({b // 2 // 64 * 64, 3 * b // 4 // 64 * 64} - {0}))


def lookup(cx, grid, cache: str = DEFAULT_CACHE) -> Optional[dict]:
    return _load(cache).get(signature(cx, grid))


def _time_forward(cx, grid, reps: int) -> float:
    out = torch.empty((cx.B, grid.d, grid.T), dtype=torch.float32 if cx.dtype == 1 else torch.int32,
                      device=cx.device)
    ws = torch.empty(max(1, api.wect_workspace_bytes(cx, grid)), dtype=torch.uint8, device=cx.device)
    api.wect_forward(cx, grid, out=out, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        api.wect_forward(cx, grid, out=out, ws=ws)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(cx, grid, candidates: Iterable[Tuple[int, int, int, int]] = CANDIDATES, reps: Optional[int] = None,
         cache: Optional[str] = DEFAULT_CACHE, apply_best: bool = True) -> dict:
    """Time every candidate shape, then the threshold tiles with the fastest
    shape; cache and (by default) apply the best."""
    before = api.get_launch()
    results = []

    def run(block, bpc, mi, dec, tt, dpl, st):
        api.set_launch(block, bpc, mi, dec, tt, dpl, stage_entries=st)
        t1 = _time_forward(cx, grid, 1)
        r = reps or max(2, min(50, int(0.05 / max(t1, 1e-6))))
        results.append((_time_forward(cx, grid, r), block, bpc, mi, dec, tt, dpl, st))

    try:
        for block, bpc, mi, dec in candidates:
            run(block, bpc, mi, dec, 0, 0, 0)
        _, block, bpc, mi, dec, _, _, _ = min(results)
        for tt in tile_candidates(grid.T)[1:]:
            run(block, bpc, mi, dec, tt, 0, 0)
        _, block, bpc, mi, dec, tt, _, _ = min(results)
        for dpl in lane_candidates(cx, grid):
            run(block, bpc, mi, dec, tt, dpl, 0)
        _, block, bpc, mi, dec, tt, dpl, _ = min(results)
        for st in stage_candidates(cx, block):
            run(block, bpc, mi, dec, tt, dpl, st)
    finally:
        api.set_launch(before["block"], before["blocks_per_cu"], before["min_items_per_block"],
                       before["decomposition"], before["threshold_tile"], before["directions_per_lane"],
                       before["cubical_records"], before["cell_packing"], before["stage_entries"])
    t, block, bpc, mi, dec, tt, dpl, st = min(results)
    best = {"block": block, "blocks_per_cu": bpc, "min_items_per_block": mi, "decomposition": dec,
            "threshold_tile": tt, "directions_per_lane": dpl, "stage_entries": st, "ms": t * 1e3,
            "tried": [{"block": b, "blocks_per_cu": c, "min_items_per_block": m, "decomposition": e,
                       "threshold_tile": x, "directions_per_lane": y, "stage_entries": z, "ms": s * 1e3}
                      for s, b, c, m, e, x, y, z in results]}
    if cache:
        data = _load(cache)
        data[signature(cx, grid)] = best
        _save(cache, data)
    if apply_best:
        apply(best)
    return best
