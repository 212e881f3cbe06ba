"""C-ABI checks that need no GPU: the library loads, exports every function
include/wect.h declares, and rejects bad metadata before touching the device.

Only error paths that return before any kernel launch are exercised here (the
pointers used are never dereferenced on those paths)."""
import ctypes

import pytest

from paper_2511_03909_amd import _lib as L


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def test_library_exports_every_declared_symbol(lib):
    names = L.declared_functions()
    assert {"wect_forward", "wect_backward", "wect_batched", "wect_validate", "wect_workspace_bytes",
            "wect_status_string"} <= set(names)
    for nm in names:
        assert hasattr(lib, nm), nm


def test_status_strings(lib):
    for s in range(8):
        assert len(L.status_string(s)) > 0
    assert L.status_string(0) == "ok"
    assert lib.wect_version().decode().startswith("wect")


FAKE = 0x100000  # never dereferenced: every call below fails its metadata check first


def _simplicial(**kw):
    c = L.WectComplex()
    c.kind = L.WECT_SIMPLICIAL
    c.n = 2
    c.B = 1
    c.top_dim = 2
    c.wmode = L.WECT_W_ONES
    c.dtype = L.WECT_I32
    c.coords = FAKE
    c.count[0], c.count[1], c.count[2] = 3, 3, 1
    c.simplices[1] = FAKE
    c.simplices[2] = FAKE
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _grid(d=4, T=6):
    return L.WectGrid(FAKE, d, T, FAKE)


def _fwd(lib, c, g, out=FAKE, ws=None, nbytes=0):
    return lib.wect_forward(ctypes.byref(c) if c is not None else None, ctypes.byref(g) if g is not None else None,
                            out, ws, nbytes, None)


def test_null_structs(lib):
    assert _fwd(lib, None, _grid()) == L.WECT_ERR_ARG
    assert _fwd(lib, _simplicial(), None) == L.WECT_ERR_ARG
    assert lib.wect_workspace_bytes(None, None, 0) == 0


@pytest.mark.parametrize("field,value", [
    ("kind", 7), ("n", 0), ("n", 4), ("B", 0), ("top_dim", 4), ("top_dim", -1), ("wmode", 3), ("dtype", 5),
    ("coords", None),
])
def test_bad_metadata(lib, field, value):
    c = _simplicial(**{field: value})
    assert _fwd(lib, c, _grid(), ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG


def test_bad_counts(lib):
    c = _simplicial()
    c.count[3] = 5  # count above top_dim
    assert _fwd(lib, c, _grid(), ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG
    c = _simplicial()
    c.count[1] = -1
    assert _fwd(lib, c, _grid(), ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG
    c = _simplicial()
    c.simplices[2] = None
    assert _fwd(lib, c, _grid(), ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG


def test_weight_mode_dtype_combinations(lib):
    assert _fwd(lib, _simplicial(dtype=L.WECT_F32), _grid(), ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG
    c = _simplicial(wmode=L.WECT_W_VERTEX_MAX, dtype=L.WECT_I32)
    assert _fwd(lib, c, _grid(), ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG
    c = _simplicial(wmode=L.WECT_W_EXPLICIT, dtype=L.WECT_F32)  # weights missing
    assert _fwd(lib, c, _grid(), ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG


def test_batch_needs_offsets(lib):
    c = _simplicial(B=2)
    assert _fwd(lib, c, _grid(), ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG


def test_grid_checks(lib):
    assert _fwd(lib, _simplicial(), L.WectGrid(None, 4, 6, FAKE)) == L.WECT_ERR_ARG
    assert _fwd(lib, _simplicial(), L.WectGrid(FAKE, 4, 6, None)) == L.WECT_ERR_ARG
    assert _fwd(lib, _simplicial(), L.WectGrid(FAKE, -1, 6, FAKE)) == L.WECT_ERR_ARG
    # an empty output needs no work and no workspace
    assert _fwd(lib, _simplicial(), L.WectGrid(FAKE, 0, 6, FAKE), out=None) == L.WECT_OK
    assert _fwd(lib, _simplicial(), L.WectGrid(FAKE, 4, 0, FAKE), out=None) == L.WECT_OK


def test_workspace_too_small(lib):
    c, g = _simplicial(), _grid()
    need = lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 0)
    assert need > 0
    assert _fwd(lib, c, g, ws=None, nbytes=0) == L.WECT_ERR_WORKSPACE
    assert _fwd(lib, c, g, ws=FAKE, nbytes=need - 1) == L.WECT_ERR_WORKSPACE
    assert _fwd(lib, c, g, out=None, ws=FAKE, nbytes=need) == L.WECT_ERR_ARG


def test_cubical_metadata(lib):
    c = L.WectComplex()
    c.kind = L.WECT_CUBICAL
    c.n = 2
    c.B = 1
    c.wmode = L.WECT_W_ONES
    c.dtype = L.WECT_I32
    c.shape = FAKE
    c.axis = FAKE
    c.intensity = FAKE
    c.total_voxels = 4
    g = _grid()
    for field, value in (("n", 1), ("n", 4), ("dtype", L.WECT_F32), ("shape", None), ("axis", None),
                         ("intensity", None), ("include_above", 256), ("B", 2)):
        bad = L.WectComplex.from_buffer_copy(c)
        setattr(bad, field, value)
        assert _fwd(lib, bad, g, ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_ARG, field
    bad = L.WectComplex.from_buffer_copy(c)
    bad.wmode = L.WECT_W_EXPLICIT
    assert _fwd(lib, bad, g, ws=FAKE, nbytes=1 << 40) == L.WECT_ERR_UNSUPPORTED


def test_backward_metadata(lib):
    c, g = _simplicial(), _grid()
    gw = (ctypes.c_void_p * 4)()
    # ones weights have no gradient; cubical backward is not provided
    assert lib.wect_backward(ctypes.byref(c), ctypes.byref(g), FAKE, gw, None, None, 0, None) == L.WECT_ERR_ARG
    c = _simplicial(wmode=L.WECT_W_VERTEX_MAX, dtype=L.WECT_F32)
    c.weights[0] = FAKE
    assert lib.wect_backward(ctypes.byref(c), ctypes.byref(g), FAKE, gw, None, None, 0, None) == L.WECT_ERR_ARG
    assert lib.wect_batched(ctypes.byref(c), ctypes.byref(g), FAKE, FAKE, gw, None, FAKE, 1 << 40,
                            None) == L.WECT_ERR_ARG


def test_launch_shape_roundtrip(lib):
    before = L.WectLaunch()
    assert lib.wect_get_launch(ctypes.byref(before)) == L.WECT_OK
    assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(300, 1, 0, 0))) == L.WECT_ERR_ARG
    assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 2, 1024, 3))) == L.WECT_ERR_ARG
    assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 2, 1024, -1))) == L.WECT_ERR_ARG
    assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 2, 1024, 2, -5))) == L.WECT_ERR_ARG
    assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 2, 1024, 2, 77, 3))) == L.WECT_ERR_ARG
    for bad_stage in (-64, 100, 1088):
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 2, 1024, 2, 77, 2, 0, 0, bad_stage))) \
            == L.WECT_ERR_ARG
    assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 2, 1024, 2, 77, 2, 0, 0, 192))) == L.WECT_OK
    now = L.WectLaunch()
    lib.wect_get_launch(ctypes.byref(now))
    assert (now.block, now.blocks_per_cu, now.min_items_per_block, now.decomposition,
            now.threshold_tile, now.directions_per_lane, now.stage_entries) == (512, 2, 1024, 2, 77, 2, 192)
    assert lib.wect_set_launch(ctypes.byref(before)) == L.WECT_OK


def test_group_decomposition_needs_no_partial_slots(lib):
    """One block per group writes the output directly: integer requests then
    need no workspace at all (float ones keep the small max-|w| area)."""
    before = L.WectLaunch()
    lib.wect_get_launch(ctypes.byref(before))
    c, g = _simplicial(), _grid(d=100, T=64)
    try:
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 0, 0, 1))) == L.WECT_OK
        assert lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 0) > 0
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 0, 0, 2))) == L.WECT_OK
        assert lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 0) == 0
        f = _simplicial(wmode=L.WECT_W_VERTEX_MAX, dtype=L.WECT_F32)
        f.weights[0] = FAKE
        assert 0 < lib.wect_workspace_bytes(ctypes.byref(f), ctypes.byref(g), 0) <= 4096
    finally:
        lib.wect_set_launch(ctypes.byref(before))


def test_workspace_grows_with_batch(lib):
    c, g = _simplicial(), _grid(d=100, T=64)
    a = lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 0)
    assert a % (64 * 64 * 4) == 0  # whole [T][64] slots
    slots = a // (64 * 64 * 4)
    # 100,000 thresholds do not fit one LDS histogram: they run in tiles of at
    # most about 600 (int32), and the partial slots are sized for one tile
    big = lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(L.WectGrid(FAKE, 100, 100000, FAKE)), 0)
    assert 0 < big <= slots * 700 * 64 * 4 + 256


def test_two_directions_per_lane_doubles_the_slot_width(lib):
    """Cubical forward with 130 directions: one lane per direction gives 3
    tiles of 64, two per lane 2 tiles of 128 (slots twice as wide); a
    simplicial request ignores the setting."""
    before = L.WectLaunch()
    lib.wect_get_launch(ctypes.byref(before))
    c = L.WectComplex()
    c.kind, c.n, c.B, c.wmode, c.dtype = L.WECT_CUBICAL, 2, 1, L.WECT_W_VERTEX_MAX, L.WECT_I32
    c.shape, c.axis, c.intensity, c.total_voxels = FAKE, FAKE, FAKE, 5000
    g = _grid(d=130, T=40)
    try:
        sizes = {}
        for dpl in (1, 2):  # without the per-voxel records
            assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 64, 1, 0, dpl, 1))) == L.WECT_OK
            sizes[dpl] = lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 0)
        # partial slots (blocks + groups) and slot sums (groups), each T x 64 dpl x 4 bytes; blocks of at
        # least 64 stream items (tiles x voxels), at most 256 (one per compute unit without a device)
        for dpl, tiles in ((1, 3), (2, 2)):
            blocks = min(256, -(-tiles * 5000 // 64))
            assert sizes[dpl] == (blocks + 2 * tiles) * 40 * 64 * dpl * 4
        s = _simplicial()
        per = []
        for dpl in (1, 2):
            assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 64, 1, 0, dpl))) == L.WECT_OK
            per.append(lib.wect_workspace_bytes(ctypes.byref(s), ctypes.byref(g), 0))
        assert per[0] == per[1]
    finally:
        lib.wect_set_launch(ctypes.byref(before))


def test_cubical_records_add_16_bytes_per_voxel(lib):
    """3D cubical forward with 130 directions (two tiles of 128): the voxel
    records (16 bytes per voxel) are on by default and add exactly their size
    to the workspace; off, or with one tile of directions, they are not
    there."""
    before = L.WectLaunch()
    lib.wect_get_launch(ctypes.byref(before))
    c = L.WectComplex()
    c.kind, c.n, c.B, c.wmode, c.dtype = L.WECT_CUBICAL, 3, 1, L.WECT_W_VERTEX_MAX, L.WECT_I32
    c.shape, c.axis, c.intensity, c.total_voxels = FAKE, FAKE, FAKE, 5000
    try:
        ws = {}
        for rec in (0, 1, 2, 3):
            assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 64, 1, 0, 0, rec))) == L.WECT_OK
            ws[rec] = lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(_grid(d=130, T=40)), 0)
        assert ws[0] == ws[2] == ws[3] == ws[1] + (5000 * 16 + 255) // 256 * 256
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 64, 1, 0, 0, 0))) == L.WECT_OK
        one = lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(_grid(d=64, T=40)), 0)
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 64, 1, 0, 0, 1))) == L.WECT_OK
        assert lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(_grid(d=64, T=40)), 0) == one
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 64, 1, 0, 0, 4))) == L.WECT_ERR_ARG
    finally:
        lib.wect_set_launch(ctypes.byref(before))


def test_threshold_tile_sets_the_slot_size(lib):
    """A caller's threshold tile of 16 for T = 64 sizes the partial slots for
    16 thresholds (a quarter); a tile above T is T; float weights (64-bit
    fixed point) at T = 1000 run in tiles that fit LDS."""
    before = L.WectLaunch()
    lib.wect_get_launch(ctypes.byref(before))
    c, g = _simplicial(), _grid(d=100, T=64)
    try:
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 0, 1, 0))) == L.WECT_OK
        full = lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 0)
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 0, 1, 16))) == L.WECT_OK
        quarter = lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 0)
        assert quarter * 4 == full
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 0, 1, 1000))) == L.WECT_OK
        assert lib.wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 0) == full
        assert lib.wect_set_launch(ctypes.byref(L.WectLaunch(512, 1, 0, 1, 0))) == L.WECT_OK
        f = _simplicial(wmode=L.WECT_W_EXPLICIT, dtype=L.WECT_F32)
        for i in range(3):
            f.weights[i] = FAKE
        ws = lib.wect_workspace_bytes(ctypes.byref(f), ctypes.byref(L.WectGrid(FAKE, 100, 1000, FAKE)), 1)
        assert ws > 0
    finally:
        lib.wect_set_launch(ctypes.byref(before))


def test_binding_rejects_mismatched_buffers():
    """The kernels write out/grads and read grad_out at the sizes the request
    implies: the binding refuses buffers that do not match before any call
    that could launch (CPU tensors here; nothing reaches a kernel)."""
    import numpy as np
    import torch

    import synth
    from paper_2511_03909_amd import api as W
    C = synth.random_tiny_cubical(0, (5, 4), include_above=80)
    cx = W.CubicalBatch.from_host([C], device="cpu")
    g = W.Grid(synth.s1_directions(8), synth.uniform_thresholds(6, 1.5), device="cpu")
    with pytest.raises(ValueError):
        W.wect_forward(cx, g, out=torch.empty((1, 8, 6), dtype=torch.float32))    # wrong dtype
    with pytest.raises(ValueError):
        W.wect_forward(cx, g, out=torch.empty((1, 8, 5), dtype=torch.int32))      # wrong shape
    with pytest.raises(ValueError):
        W.wect_forward(cx, g, out=torch.empty((1, 6, 8), dtype=torch.int32).transpose(1, 2))  # not contiguous
    K = synth.random_tiny_complex(1, n=2, nv=7, top_dim=2, wmode="vertex_max", wdtype=np.float32)
    sx = W.SimplicialBatch.from_host([K], device="cpu")
    with pytest.raises(ValueError):
        W.wect_backward(sx, g, torch.zeros((1, 8, 7)))                            # grad_out shape
    with pytest.raises(ValueError):
        W.wect_batched(sx, g, torch.zeros((1, 8, 6)), grads=torch.zeros(3))        # grads size


def test_cubical_batch_needs_one_inclusion_level():
    import numpy as np

    import synth
    from paper_2511_03909_amd import api as W
    a = synth.uniform_image((4, 3), 0, include_above=-1)
    b = synth.uniform_image((4, 3), 1, include_above=10)
    with pytest.raises(ValueError):
        W.CubicalBatch.from_host([a, b], device="cpu")
    c = synth.uniform_image((4, 3), 2, weighted=True)
    with pytest.raises(ValueError):
        W.CubicalBatch.from_host([a, c], device="cpu")
    assert W.CubicalBatch.from_host([a, synth.uniform_image((2, 5), 3)], device="cpu").B == 2
    del np


def test_wecf_metadata(lib):
    c = _simplicial()
    assert lib.wect_wecf_workspace_bytes(ctypes.byref(c), 70, 16) > 0
    # fvals missing while there are vertices and columns
    assert lib.wect_wecf_forward(ctypes.byref(c), None, 3, FAKE, 6, FAKE, FAKE, 1 << 40, None) == L.WECT_ERR_ARG
    # cubical complexes take wect_image_ecf
    cub = _simplicial(kind=L.WECT_CUBICAL)
    assert lib.wect_wecf_forward(ctypes.byref(cub), FAKE, 3, FAKE, 6, FAKE, FAKE, 1 << 40, None) == L.WECT_ERR_ARG
    assert lib.wect_wecf_forward(ctypes.byref(c), FAKE, -1, FAKE, 6, FAKE, FAKE, 1 << 40, None) == L.WECT_ERR_ARG
    # nothing to compute: no workspace needed, nothing enqueued
    assert lib.wect_wecf_forward(ctypes.byref(c), FAKE, 0, FAKE, 6, None, None, 0, None) == L.WECT_OK


def test_freudenthal_counts():
    from paper_2511_03909_amd import api as W
    assert W.freudenthal_counts([[3, 2, 1]]) == (6, 2 * 2 + 3 * 1 + 2, 4)
    assert W.freudenthal_counts([[1, 1, 1], [4, 1, 1]]) == (5, 3, 0)
    with pytest.raises(L.WectError):
        W.freudenthal_counts([[0, 3, 1]])
    with pytest.raises(L.WectError):
        W.freudenthal_counts([[3, 3, 2]])   # a volume


def test_smooth_metadata(lib):
    """Relaxation: lam must be finite and >= 0; simplicial only; explicit
    weights must be float32.  Every failing call returns before any launch."""
    g = _grid()
    ok = _simplicial()
    nb = lib.wect_smooth_workspace_bytes(ctypes.byref(ok), ctypes.byref(g), 2.0)
    assert nb > 0  # fixed-point partial histograms
    for lam in (-1.0, float("inf"), float("nan")):
        assert lib.wect_smooth_forward(ctypes.byref(ok), ctypes.byref(g), lam, FAKE, FAKE, 1 << 30, None) == \
            L.WECT_ERR_ARG
        assert lib.wect_smooth_backward(ctypes.byref(ok), ctypes.byref(g), lam, FAKE, None, None, None, None,
                                        None) == L.WECT_ERR_ARG
    cub = L.WectComplex()
    cub.kind, cub.n, cub.B, cub.wmode, cub.dtype = L.WECT_CUBICAL, 2, 1, L.WECT_W_ONES, L.WECT_I32
    assert lib.wect_smooth_forward(ctypes.byref(cub), ctypes.byref(g), 1.0, FAKE, FAKE, 1 << 30, None) == \
        L.WECT_ERR_UNSUPPORTED
    exi = _simplicial(wmode=L.WECT_W_EXPLICIT, dtype=L.WECT_I32)
    for i in range(3):
        exi.weights[i] = FAKE
    assert lib.wect_smooth_forward(ctypes.byref(exi), ctypes.byref(g), 1.0, FAKE, FAKE, 1 << 30, None) == \
        L.WECT_ERR_UNSUPPORTED
    # a too small workspace is refused before any launch
    assert lib.wect_smooth_forward(ctypes.byref(ok), ctypes.byref(g), 1.0, FAKE, FAKE, nb - 1, None) == \
        L.WECT_ERR_WORKSPACE
    # unit weights need no maximum-|w| pass: less workspace than float32 weights
    exf = _simplicial(wmode=L.WECT_W_EXPLICIT, dtype=L.WECT_F32)
    for i in range(3):
        exf.weights[i] = FAKE
    assert lib.wect_smooth_workspace_bytes(ctypes.byref(exf), ctypes.byref(g), 1.0) > nb


def test_lower_star_metadata(lib):
    """The lower-star index: its size depends on the counts; a missing or too
    small index is refused before any launch."""
    c, g = _simplicial(), _grid()
    nb = lib.wect_lower_star_bytes(ctypes.byref(c))
    assert nb > 0
    big = _simplicial()
    big.count[0], big.count[1], big.count[2] = 30, 60, 31
    assert lib.wect_lower_star_bytes(ctypes.byref(big)) > nb
    assert lib.wect_lower_star_build(ctypes.byref(c), None, nb, None) == L.WECT_ERR_ARG
    assert lib.wect_lower_star_build(ctypes.byref(c), FAKE, nb - 1, None) == L.WECT_ERR_ARG
    assert lib.wect_lower_star_build(ctypes.byref(c), FAKE + 4, nb, None) == L.WECT_ERR_ARG  # misaligned
    cub = L.WectComplex()
    cub.kind, cub.n, cub.B = L.WECT_CUBICAL, 2, 1
    assert lib.wect_lower_star_bytes(ctypes.byref(cub)) == 0
    ws = lib.wect_smooth_ls_workspace_bytes(ctypes.byref(c), ctypes.byref(g), 2.0)
    assert ws > 0
    assert lib.wect_smooth_ls_forward(ctypes.byref(c), ctypes.byref(g), 2.0, None, 0, FAKE, FAKE, ws, None) == \
        L.WECT_ERR_ARG
    assert lib.wect_smooth_ls_forward(ctypes.byref(c), ctypes.byref(g), 2.0, FAKE, nb - 1, FAKE, FAKE, ws, None) == \
        L.WECT_ERR_ARG
    assert lib.wect_smooth_ls_backward(ctypes.byref(c), ctypes.byref(g), -1.0, FAKE, nb, FAKE, None, None, None,
                                       None, None) == L.WECT_ERR_ARG


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with a message, before touching a device."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
