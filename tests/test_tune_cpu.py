"""Autotuner bookkeeping that needs no GPU."""
import numpy as np
import torch

import synth
from paper_2511_03909_amd import api, tune


def test_signature_and_cache_roundtrip(tmp_path):
    K = synth.random_tiny_complex(0, n=2, nv=8, top_dim=2, wmode="ones")
    cx = api.SimplicialBatch.from_host([K], device="cpu")
    g = api.Grid(synth.s1_directions(8), synth.uniform_thresholds(9, 1.5), device="cpu")
    sig = tune.signature(cx, g)
    assert sig.startswith("simplicial/n2/B1/") and "/d8/T9/" in sig
    path = str(tmp_path / "t.json")
    tune._save(path, {sig: {"block": 512, "blocks_per_cu": 0, "min_items_per_block": 0}})
    assert tune.lookup(cx, g, path)["block"] == 512
    C = synth.random_tiny_cubical(0, (5, 4))
    cc = api.CubicalBatch.from_host([C], device="cpu")
    assert tune.signature(cc, g).startswith("cubical/n2/B1/")


def test_candidate_lists():
    K = synth.random_tiny_complex(0, n=2, nv=8, top_dim=2, wmode="ones")
    cx = api.SimplicialBatch.from_host([K], device="cpu")
    C = synth.random_tiny_cubical(0, (5, 4))
    cc = api.CubicalBatch.from_host([C], device="cpu")
    # staging tiles: simplicial only, multiples of 64 below the block
    assert tune.stage_candidates(cx, 1024) == (512, 768)
    assert tune.stage_candidates(cx, 0) == (512, 768)
    assert tune.stage_candidates(cx, 512) == (256, 384)
    assert tune.stage_candidates(cx, 256) == (128, 192)
    assert tune.stage_candidates(cc, 1024) == ()
    # threshold tiles: automatic, then about a half and a third of T
    assert tune.tile_candidates(64) == (0,)
    assert tune.tile_candidates(1000) == (0, 500, 334)
    g = api.Grid(synth.s1_directions(128), synth.uniform_thresholds(9, 1.5), device="cpu")
    assert tune.lane_candidates(cc, g) == (1, 2) and tune.lane_candidates(cx, g) == ()
