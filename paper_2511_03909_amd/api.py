"""Python binding of libwect.so: argument marshalling only.

Every step of the transform runs in the HIP kernels behind the C ABI
(include/wect.h).  PyTorch provides device memory and the current stream;
nothing here computes any part of the transform.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

__all__ = [
    "Grid", "SimplicialBatch", "CubicalBatch", "wect_workspace_bytes", "wect_forward", "wect_backward",
    "wect_batched", "wect_validate", "set_launch", "get_launch", "profile_enable", "profile_read",
    "WECTFunction", "wect", "WECT", "smooth_workspace_bytes", "smooth_forward", "smooth_backward",
    "SmoothWECTFunction", "smooth_wect", "SmoothWECT", "lower_star_index", "wecf_backward",
]

_WMODES = {"ones": L.WECT_W_ONES, "explicit": L.WECT_W_EXPLICIT, "vertex_max": L.WECT_W_VERTEX_MAX}


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr() if t.numel() > 0 else None


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Grid:
    """Directions [d, n] and thresholds [T] (float32, device)."""

    def __init__(self, dirs, thr, device="cuda"):
        self.dirs = torch.as_tensor(np.ascontiguousarray(dirs, dtype=np.float32) if isinstance(dirs, np.ndarray)
                                    else dirs).to(device=device, dtype=torch.float32).contiguous()
        self.thr = torch.as_tensor(np.ascontiguousarray(thr, dtype=np.float32) if isinstance(thr, np.ndarray)
                                   else thr).to(device=device, dtype=torch.float32).contiguous()
        self.d = int(self.dirs.shape[0])
        self.T = int(self.thr.shape[0])

    def struct(self) -> L.WectGrid:
        return L.WectGrid(_ptr(self.dirs), self.d, self.T, _ptr(self.thr))


class SimplicialBatch:
    """B simplicial complexes packed back to back on the device (CSR offsets).

    coords [sum V, n] float32; simplices[i] [sum k_i, i+1] int32 with vertex ids
    local to their complex; weights per ``wmode``: 'ones' (none), 'explicit'
    (list per dimension, int32 or float32), 'vertex_max' ([w] float32 [sum V]).
    """

    def __init__(self, coords, simplices, wmode, weights, vert_off=None, simp_off=None, B=1):
        self.coords = coords
        self.simplices = list(simplices)
        self.top_dim = len(self.simplices) - 1
        self.wmode = wmode
        self.weights = list(weights)
        self.vert_off = vert_off
        self.simp_off = simp_off or [None] * 4
        self.B = int(B)
        self.n = int(coords.shape[1])
        self.device = coords.device
        if wmode == "ones":
            self.dtype = L.WECT_I32
        elif wmode == "vertex_max":
            self.dtype = L.WECT_F32
        else:
            self.dtype = L.WECT_F32 if self.weights[0].dtype == torch.float32 else L.WECT_I32

    @property
    def counts(self) -> List[int]:
        c = [int(self.coords.shape[0])]
        for i in range(1, self.top_dim + 1):
            c.append(int(self.simplices[i].shape[0]))
        return c

    def with_weights(self, weights) -> "SimplicialBatch":
        s = SimplicialBatch(self.coords, self.simplices, self.wmode, list(weights), self.vert_off,
                            self.simp_off, self.B)
        return s

    @classmethod
    def from_host(cls, complexes: Sequence, device="cuda") -> "SimplicialBatch":
        """Pack host complexes (objects with coords, simplices, wmode, weights)."""
        complexes = list(complexes)
        B = len(complexes)
        top = max(len(K.simplices) - 1 for K in complexes)
        n = complexes[0].coords.shape[1]
        wmode = complexes[0].wmode
        coords = np.concatenate([np.asarray(K.coords, np.float32) for K in complexes])
        vcount = [K.coords.shape[0] for K in complexes]
        simp = [None]
        offs: list = [None]
        for i in range(1, top + 1):
            parts = [np.asarray(K.simplices[i], np.int32).reshape(-1, i + 1) if i < len(K.simplices)
                     and K.simplices[i] is not None else np.zeros((0, i + 1), np.int32) for K in complexes]
            simp.append(np.concatenate(parts))
            offs.append(np.concatenate([[0], np.cumsum([p.shape[0] for p in parts])]).astype(np.int64))
        weights = []
        if wmode == "explicit":
            for i in range(top + 1):
                weights.append(np.concatenate([np.asarray(K.weights[i]) for K in complexes]))
        elif wmode == "vertex_max":
            weights.append(np.concatenate([np.asarray(K.weights[0], np.float32) for K in complexes]))
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        vert_off = T(np.concatenate([[0], np.cumsum(vcount)]).astype(np.int64)) if B > 1 else None
        simp_off = [None] + [T(o) for o in offs[1:]] if B > 1 else None
        return cls(T(coords), [None] + [T(s) for s in simp[1:]], wmode, [T(w) for w in weights],
                   vert_off, simp_off, B)

    def struct(self) -> L.WectComplex:
        c = L.WectComplex()
        c.kind = L.WECT_SIMPLICIAL
        c.n = self.n
        c.B = self.B
        c.top_dim = self.top_dim
        c.wmode = _WMODES[self.wmode]
        c.dtype = self.dtype
        c.coords = _ptr(self.coords)
        c.vert_off = _ptr(self.vert_off)
        cnt = self.counts
        for i in range(4):
            c.count[i] = cnt[i] if i < len(cnt) else 0
            c.simplices[i] = _ptr(self.simplices[i]) if 1 <= i <= self.top_dim else None
            c.simp_off[i] = _ptr(self.simp_off[i]) if (1 <= i <= self.top_dim and self.simp_off) else None
            c.weights[i] = _ptr(self.weights[i]) if i < len(self.weights) else None
        return c


class CubicalBatch:
    """B uint8 images (n = 2) or volumes (n = 3) on the device.

    intensity: all voxels back to back, axis 0 fastest; shape [B, 3] int32
    (n2 = 1 for images); axis: per complex n0 + n1 (+ n2) float32 coordinates."""

    def __init__(self, n, intensity, shape, grid_off, axis, axis_off, include_above, weighted, B):
        self.n = int(n)
        self.intensity = intensity
        self.shape = shape
        self.grid_off = grid_off
        self.axis = axis
        self.axis_off = axis_off
        self.include_above = int(include_above)
        self.weighted = bool(weighted)
        self.B = int(B)
        self.total_voxels = int(intensity.numel())
        self.device = intensity.device
        self.shape_host = None  # host copy of shape when known (set by from_host)

    @classmethod
    def from_host(cls, images: Sequence, device="cuda") -> "CubicalBatch":
        images = list(images)
        B = len(images)
        n = images[0].intensity.ndim
        # one inclusion level, weight mode and dimension per batch (a single wect_complex)
        for C in images[1:]:
            if (C.include_above != images[0].include_above or bool(C.weighted) != bool(images[0].weighted)
                    or np.asarray(C.intensity).ndim != n):
                raise ValueError("every image of a batch needs the same dimension, include_above and weighting")
        shapes, flat, axes, gv, av = [], [], [], [0], [0]
        for C in images:
            I = np.asarray(C.intensity, np.uint8)
            sxyz = list(I.shape[::-1]) + [1] * (3 - I.ndim)
            shapes.append(sxyz)
            flat.append(np.ascontiguousarray(I).ravel())
            ax = np.concatenate([np.asarray(a, np.float32) for a in C.axes])
            axes.append(ax)
            gv.append(gv[-1] + I.size)
            av.append(av[-1] + ax.size)
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        inc = images[0].include_above
        out = cls(n, T(np.concatenate(flat)), T(np.array(shapes, np.int32)),
                  T(np.array(gv, np.int64)) if B > 1 else None, T(np.concatenate(axes)),
                  T(np.array(av, np.int64)) if B > 1 else None, inc, images[0].weighted, B)
        out.shape_host = np.array(shapes, np.int32)  # for host-side sizes (builders)
        return out

    def struct(self) -> L.WectComplex:
        c = L.WectComplex()
        c.kind = L.WECT_CUBICAL
        c.n = self.n
        c.B = self.B
        c.top_dim = self.n
        c.wmode = L.WECT_W_VERTEX_MAX if self.weighted else L.WECT_W_ONES
        c.dtype = L.WECT_I32
        c.shape = _ptr(self.shape)
        c.grid_off = _ptr(self.grid_off)
        c.intensity = _ptr(self.intensity)
        c.axis = _ptr(self.axis)
        c.axis_off = _ptr(self.axis_off)
        c.total_voxels = self.total_voxels
        c.include_above = self.include_above
        return c

    @property
    def dtype(self):
        return L.WECT_I32


def _out_dtype(cx):
    return torch.float32 if cx.dtype == L.WECT_F32 else torch.int32


def wect_workspace_bytes(cx, grid: Grid, with_backward: bool = False) -> int:
    c, g = cx.struct(), grid.struct()
    return int(L.lib().wect_workspace_bytes(ctypes.byref(c), ctypes.byref(g), int(with_backward)))


def _check_tensor(t: torch.Tensor, name: str, device, dtype=None, shape=None) -> None:
    """Caller-supplied buffers are written by the kernels: reject any that do not
    match what the call will write (a wrong one would be written out of bounds)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != torch.device(device):
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _output(cx, grid, out):
    shape = (cx.B, grid.d, grid.T)
    if out is None:
        return torch.empty(shape, dtype=_out_dtype(cx), device=cx.device)
    _check_tensor(out, "out", cx.device, _out_dtype(cx), shape)
    return out


def _workspace(cx, grid, with_backward, ws):
    need = wect_workspace_bytes(cx, grid, with_backward)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=cx.device)
    else:
        _check_tensor(ws, "ws", cx.device)
    return ws, int(ws.numel()) * ws.element_size()


def wect_forward(cx, grid: Grid, out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """Forward transform -> out [B, d, T] (int32 or float32); see wect_forward in wect.h."""
    out = _output(cx, grid, out)
    ws, nbytes = _workspace(cx, grid, False, ws)
    c, g = cx.struct(), grid.struct()
    st = L.lib().wect_forward(ctypes.byref(c), ctypes.byref(g), _ptr(out), _ptr(ws), ctypes.c_size_t(nbytes),
                              _stream(cx.device))
    L.check(st, "wect_forward")
    return out


def _grad_outputs(cx):
    if cx.wmode == "vertex_max":
        return None, torch.empty(cx.counts[0], dtype=torch.float32, device=cx.device)
    gw = [torch.empty(k, dtype=torch.float32, device=cx.device) for k in cx.counts]
    return gw, None


def _gw_array(gw):
    arr = (ctypes.c_void_p * 4)()
    if gw is not None:
        for i, t in enumerate(gw):
            arr[i] = _ptr(t)
    return arr


def _grad_in(cx, grid, grad_out: torch.Tensor) -> torch.Tensor:
    grad_out = grad_out.to(dtype=torch.float32).contiguous()
    _check_tensor(grad_out, "grad_out", cx.device, torch.float32, (cx.B, grid.d, grid.T))
    return grad_out


def wect_backward(cx, grid: Grid, grad_out: torch.Tensor, ws: Optional[torch.Tensor] = None):
    """Adjoint with respect to the weights: list per dimension (explicit) or [V] (vertex_max)."""
    grad_out = _grad_in(cx, grid, grad_out)
    gw, gv = _grad_outputs(cx)
    ws, nbytes = _workspace(cx, grid, True, ws)
    c, g = cx.struct(), grid.struct()
    st = L.lib().wect_backward(ctypes.byref(c), ctypes.byref(g), _ptr(grad_out), _gw_array(gw), _ptr(gv),
                               _ptr(ws), ctypes.c_size_t(nbytes), _stream(cx.device))
    L.check(st, "wect_backward")
    return gv if gv is not None else gw


def wect_batched(cx, grid: Grid, grad_out: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                 grads=None, ws: Optional[torch.Tensor] = None):
    """Forward (+ backward when grad_out is given) for a batch in one call.
    Returns (out, grads) with grads None when grad_out is None."""
    out = _output(cx, grid, out)
    gw = gv = None
    if grad_out is not None:
        grad_out = _grad_in(cx, grid, grad_out)
        if grads is None:
            gw, gv = _grad_outputs(cx)
        elif cx.wmode == "vertex_max":
            gv = grads
            _check_tensor(gv, "grads", cx.device, torch.float32, (cx.counts[0],))
        else:
            gw = list(grads)
            if len(gw) != len(cx.counts):
                raise ValueError(f"grads needs {len(cx.counts)} tensors, one per dimension")
            for i, (t, k) in enumerate(zip(gw, cx.counts)):
                _check_tensor(t, f"grads[{i}]", cx.device, torch.float32, (k,))
    ws, nbytes = _workspace(cx, grid, grad_out is not None, ws)
    c, g = cx.struct(), grid.struct()
    st = L.lib().wect_batched(ctypes.byref(c), ctypes.byref(g), _ptr(out), _ptr(grad_out), _gw_array(gw), _ptr(gv),
                              _ptr(ws), ctypes.c_size_t(nbytes), _stream(cx.device))
    L.check(st, "wect_batched")
    if grad_out is None:
        return out, None
    return out, (gv if gv is not None else gw)


def wect_validate(cx, grid: Grid) -> None:
    """Synchronous data check; raises WectError on the first failing class."""
    c, g = cx.struct(), grid.struct()
    L.check(L.lib().wect_validate(ctypes.byref(c), ctypes.byref(g), _stream(cx.device)), "wect_validate")


def wecf_workspace_bytes(cx, m: int, T: int) -> int:
    c = cx.struct()
    return int(L.lib().wect_wecf_workspace_bytes(ctypes.byref(c), int(m), int(T)))


def wecf_forward(cx, fvals, thr, out: Optional[torch.Tensor] = None,
                 ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """WECF of m general vertex filters fvals [sum V, m] on a simplicial batch ->
    [B, m, T] (int32 or float32 like wect_forward); see wect_wecf_forward."""
    fvals = torch.as_tensor(fvals, dtype=torch.float32).to(cx.device).contiguous()
    if fvals.dim() != 2 or fvals.shape[0] != cx.counts[0]:
        raise ValueError(f"fvals must be [{cx.counts[0]}, m], got {tuple(fvals.shape)}")
    thr = torch.as_tensor(thr, dtype=torch.float32).to(cx.device).contiguous()
    m, T = int(fvals.shape[1]), int(thr.numel())
    shape = (cx.B, m, T)
    if out is None:
        out = torch.empty(shape, dtype=_out_dtype(cx), device=cx.device)
    else:
        _check_tensor(out, "out", cx.device, _out_dtype(cx), shape)
    need = wecf_workspace_bytes(cx, m, T)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=cx.device)
    else:
        _check_tensor(ws, "ws", cx.device)
    c = cx.struct()
    st = L.lib().wect_wecf_forward(ctypes.byref(c), _ptr(fvals), ctypes.c_int32(m), _ptr(thr), ctypes.c_int32(T),
                                   _ptr(out), _ptr(ws), ctypes.c_size_t(int(ws.numel()) * ws.element_size()),
                                   _stream(cx.device))
    L.check(st, "wect_wecf_forward")
    return out


def wecf_backward(cx, fvals, thr, grad_out: torch.Tensor, ws: Optional[torch.Tensor] = None):
    """Adjoint of ``wecf_forward`` with respect to the (float32) weights: list per
    dimension (explicit) or [V] (vertex_max); see wect_wecf_backward."""
    fvals = torch.as_tensor(fvals, dtype=torch.float32).to(cx.device).contiguous()
    if fvals.dim() != 2 or fvals.shape[0] != cx.counts[0]:
        raise ValueError(f"fvals must be [{cx.counts[0]}, m], got {tuple(fvals.shape)}")
    thr = torch.as_tensor(thr, dtype=torch.float32).to(cx.device).contiguous()
    m, T = int(fvals.shape[1]), int(thr.numel())
    grad_out = grad_out.to(dtype=torch.float32).contiguous()
    _check_tensor(grad_out, "grad_out", cx.device, torch.float32, (cx.B, m, T))
    gw, gv = _grad_outputs(cx)
    need = wecf_workspace_bytes(cx, m, T)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=cx.device)
    else:
        _check_tensor(ws, "ws", cx.device)
    c = cx.struct()
    st = L.lib().wect_wecf_backward(ctypes.byref(c), _ptr(fvals), ctypes.c_int32(m), _ptr(thr), ctypes.c_int32(T),
                                    _ptr(grad_out), _gw_array(gw), _ptr(gv), _ptr(ws),
                                    ctypes.c_size_t(int(ws.numel()) * ws.element_size()), _stream(cx.device))
    L.check(st, "wect_wecf_backward")
    return gv if gv is not None else gw


def freudenthal_counts(shapes) -> Tuple[int, int, int]:
    """Total vertices, edges and triangles of the Freudenthal complexes of
    images with host shapes [B, 3] (n0, n1, 1)."""
    sh = np.ascontiguousarray(np.asarray(shapes, dtype=np.int32).reshape(-1, 3))
    out = (ctypes.c_int64 * 3)()
    L.check(L.lib().wect_freudenthal_counts(int(sh.shape[0]), sh.ctypes.data, out), "wect_freudenthal_counts")
    return int(out[0]), int(out[1]), int(out[2])


def freudenthal_from_images(cx) -> "SimplicialBatch":
    """The weighted Freudenthal complexes of a 2D image batch, built on the device:
    vertex weights = intensities, simplex weight = the largest vertex weight
    ('vertex_max'); see wect_freudenthal_build."""
    if cx.n != 2:
        raise ValueError("the Freudenthal builder takes 2D images")
    shapes = cx.shape_host if getattr(cx, "shape_host", None) is not None else cx.shape.cpu().numpy()
    V, E, F = freudenthal_counts(shapes)
    dev = cx.device
    coords = torch.empty((V, 2), dtype=torch.float32, device=dev)
    vw = torch.empty(V, dtype=torch.float32, device=dev)
    edges = torch.empty((E, 2), dtype=torch.int32, device=dev)
    tris = torch.empty((F, 3), dtype=torch.int32, device=dev)
    offs = [torch.empty(cx.B + 1, dtype=torch.int64, device=dev) for _ in range(3)]
    c = cx.struct()
    L.check(L.lib().wect_freudenthal_build(ctypes.byref(c), _ptr(coords), _ptr(vw), _ptr(edges), _ptr(tris),
                                           _ptr(offs[0]), _ptr(offs[1]), _ptr(offs[2]), _stream(dev)),
            "wect_freudenthal_build")
    return SimplicialBatch(coords, [None, edges, tris], "vertex_max", [vw], offs[0], [None, offs[1], offs[2]],
                           cx.B)


def image_ecf_workspace_bytes(cx) -> int:
    c = cx.struct()
    return int(L.lib().wect_image_ecf_workspace_bytes(ctypes.byref(c)))


def image_ecf(cx, thr, out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """ECF of every image / volume of a cubical batch with the intensity as the
    vertex filter -> int32 [B, T]; see wect_image_ecf in wect.h.  Weighted
    batches (vertex_max) give the WECF with weight = largest corner intensity."""
    thr = torch.as_tensor(thr, dtype=torch.float32).to(cx.device).contiguous()
    T = int(thr.numel())
    shape = (cx.B, T)
    if out is None:
        out = torch.empty(shape, dtype=torch.int32, device=cx.device)
    else:
        _check_tensor(out, "out", cx.device, torch.int32, shape)
    need = image_ecf_workspace_bytes(cx)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=cx.device)
    else:
        _check_tensor(ws, "ws", cx.device)
    c = cx.struct()
    st = L.lib().wect_image_ecf(ctypes.byref(c), _ptr(thr), ctypes.c_int32(T), _ptr(out), _ptr(ws),
                                ctypes.c_size_t(int(ws.numel()) * ws.element_size()), _stream(cx.device))
    L.check(st, "wect_image_ecf")
    return out


DECOMP_AUTO, DECOMP_STREAM, DECOMP_GROUP = 0, 1, 2


def set_launch(block: int = 0, blocks_per_cu: int = 0, min_items_per_block: int = 0,
               decomposition: int = DECOMP_AUTO, threshold_tile: int = 0, directions_per_lane: int = 0,
               cubical_records: int = 0, cell_packing: int = 0, stage_entries: int = 0) -> None:
    """Launch shape of the following calls (0 = automatic for each field); see wect_launch."""
    L.check(L.lib().wect_set_launch(ctypes.byref(L.WectLaunch(block, blocks_per_cu, min_items_per_block,
                                                              decomposition, threshold_tile, directions_per_lane,
                                                              cubical_records, cell_packing,
                                                              stage_entries))), "wect_set_launch")


def get_launch() -> dict:
    w = L.WectLaunch()
    L.check(L.lib().wect_get_launch(ctypes.byref(w)), "wect_get_launch")
    return {"block": w.block, "blocks_per_cu": w.blocks_per_cu, "min_items_per_block": w.min_items_per_block,
            "decomposition": w.decomposition, "threshold_tile": w.threshold_tile,
            "directions_per_lane": w.directions_per_lane, "cubical_records": w.cubical_records,
            "cell_packing": w.cell_packing, "stage_entries": w.stage_entries}


def profile_enable(on: bool = True) -> None:
    L.check(L.lib().wect_profile_enable(int(on)), "wect_profile_enable")


def profile_read(reset: bool = True) -> dict:
    fm, bm = ctypes.c_double(), ctypes.c_double()
    fl, bl = ctypes.c_int64(), ctypes.c_int64()
    L.check(L.lib().wect_profile_read(ctypes.byref(fm), ctypes.byref(fl), ctypes.byref(bm), ctypes.byref(bl),
                                      int(reset)), "wect_profile_read")
    return {"fwd_ms": fm.value, "fwd_launches": fl.value, "bwd_ms": bm.value, "bwd_launches": bl.value}


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

class WECTFunction(torch.autograd.Function):
    """out = WECT(weights); gradients flow to the weights only.

    The output is piecewise constant in coordinates, directions and
    thresholds, so their gradient is zero almost everywhere and None is
    returned for them."""

    @staticmethod
    def forward(ctx, cx, grid, *weights):
        cxw = cx.with_weights(list(w.detach().contiguous() for w in weights))
        out = wect_forward(cxw, grid)
        ctx.cx = cxw
        ctx.grid = grid
        return out

    @staticmethod
    def backward(ctx, grad_out):
        g = wect_backward(ctx.cx, ctx.grid, grad_out)
        if isinstance(g, torch.Tensor):
            g = [g]
        return (None, None, *g)


def wect(cx: SimplicialBatch, grid: Grid, *weights: torch.Tensor) -> torch.Tensor:
    """Differentiable WECT of a simplicial batch with float32 weights
    ('vertex_max': one tensor [V]; 'explicit': one tensor per dimension)."""
    return WECTFunction.apply(cx, grid, *weights)


class WECT(torch.nn.Module):
    """Module form: directions and thresholds as buffers, complexes as input."""

    def __init__(self, dirs, thr):
        super().__init__()
        self.register_buffer("dirs", torch.as_tensor(dirs, dtype=torch.float32))
        self.register_buffer("thr", torch.as_tensor(thr, dtype=torch.float32))

    def forward(self, cx, *weights):
        grid = Grid(self.dirs, self.thr, device=self.dirs.device)
        if weights:
            return wect(cx, grid, *weights)
        return wect_forward(cx, grid)


# ---------------------------------------------------------------------------
# sigmoid relaxation (differentiable in coordinates, directions and weights)
# ---------------------------------------------------------------------------

def _lam(lam) -> float:
    lam = float(lam)
    if not (lam >= 0.0) or lam == float("inf"):
        raise ValueError("lam must be finite and >= 0")
    return lam


def lower_star_index(cx, cache: bool = True) -> torch.Tensor:
    """Device buffer holding the lower-star index of a simplicial batch (see
    wect_lower_star_build); built once and kept on the batch object."""
    idx = getattr(cx, "_lower_star", None) if cache else None
    if idx is not None:
        return idx
    c = cx.struct()
    nbytes = int(L.lib().wect_lower_star_bytes(ctypes.byref(c)))
    if nbytes == 0:
        raise L.WectError(L.WECT_ERR_ARG, "wect_lower_star_bytes")
    idx = torch.empty(nbytes, dtype=torch.uint8, device=cx.device)
    L.check(L.lib().wect_lower_star_build(ctypes.byref(c), _ptr(idx), ctypes.c_size_t(nbytes), _stream(cx.device)),
            "wect_lower_star_build")
    if cache:
        cx._lower_star = idx
    return idx


def _index_arg(index):
    if index is None:
        return None, 0
    return _ptr(index), int(index.numel()) * index.element_size()


def smooth_workspace_bytes(cx, grid: Grid, lam: float, index: Optional[torch.Tensor] = None) -> int:
    c, g = cx.struct(), grid.struct()
    fn = L.lib().wect_smooth_ls_workspace_bytes if index is not None else L.lib().wect_smooth_workspace_bytes
    return int(fn(ctypes.byref(c), ctypes.byref(g), _lam(lam)))


def smooth_forward(cx, grid: Grid, lam: float, out: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None, index: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Sigmoid relaxation S [B, d, T] float32; see wect_smooth_forward in wect.h.
    With ``index`` (from ``lower_star_index``) the vertex-centric kernels run."""
    lam = _lam(lam)
    shape = (cx.B, grid.d, grid.T)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=cx.device)
    else:
        _check_tensor(out, "out", cx.device, torch.float32, shape)
    need = smooth_workspace_bytes(cx, grid, lam, index)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=cx.device)
    else:
        _check_tensor(ws, "ws", cx.device)
    c, g = cx.struct(), grid.struct()
    nws = ctypes.c_size_t(int(ws.numel()) * ws.element_size())
    if index is None:
        st = L.lib().wect_smooth_forward(ctypes.byref(c), ctypes.byref(g), lam, _ptr(out), _ptr(ws), nws,
                                         _stream(cx.device))
    else:
        _check_tensor(index, "index", cx.device, torch.uint8)
        ip, ib = _index_arg(index)
        st = L.lib().wect_smooth_ls_forward(ctypes.byref(c), ctypes.byref(g), lam, ip, ctypes.c_size_t(ib),
                                            _ptr(out), _ptr(ws), nws, _stream(cx.device))
    L.check(st, "wect_smooth_forward")
    return out


def smooth_backward(cx, grid: Grid, lam: float, grad_out: torch.Tensor, coords: bool = True, dirs: bool = True,
                    weights: bool = True, index: Optional[torch.Tensor] = None) -> dict:
    """Adjoint of ``smooth_forward``: {"coords": [V, n] or None, "dirs": [d, n] or None,
    "weights": list per dimension (explicit) / [V] (vertex_max) / None}."""
    lam = _lam(lam)
    grad_out = _grad_in(cx, grid, grad_out)
    dev = cx.device
    gx = torch.empty((cx.counts[0], cx.n), dtype=torch.float32, device=dev) if coords else None
    gd = torch.empty((grid.d, cx.n), dtype=torch.float32, device=dev) if dirs else None
    gw = gv = None
    if weights and cx.wmode != "ones":
        gw, gv = _grad_outputs(cx)
    c, g = cx.struct(), grid.struct()
    if index is None:
        st = L.lib().wect_smooth_backward(ctypes.byref(c), ctypes.byref(g), lam, _ptr(grad_out), _ptr(gx),
                                          _ptr(gd), _gw_array(gw), _ptr(gv), _stream(dev))
    else:
        _check_tensor(index, "index", dev, torch.uint8)
        ip, ib = _index_arg(index)
        st = L.lib().wect_smooth_ls_backward(ctypes.byref(c), ctypes.byref(g), lam, ip, ctypes.c_size_t(ib),
                                             _ptr(grad_out), _ptr(gx), _ptr(gd), _gw_array(gw), _ptr(gv),
                                             _stream(dev))
    L.check(st, "wect_smooth_backward")
    return {"coords": gx, "dirs": gd, "weights": gv if gv is not None else gw}


class SmoothWECTFunction(torch.autograd.Function):
    """S = relaxation(coords, dirs, weights) with gradients to all three."""

    @staticmethod
    def forward(ctx, cx, thr, lam, coords, dirs, *weights):
        ws = [w.detach().contiguous() for w in weights] if weights else list(cx.weights)
        cxw = SimplicialBatch(coords.detach().contiguous(), cx.simplices, cx.wmode, ws, cx.vert_off,
                              cx.simp_off, cx.B)
        grid = Grid(dirs.detach(), thr, device=coords.device)
        index = lower_star_index(cx)  # depends on the topology only: built once per batch object
        ctx.cx, ctx.grid, ctx.lam, ctx.nw, ctx.index = cxw, grid, lam, len(weights), index
        return smooth_forward(cxw, grid, lam, index=index)

    @staticmethod
    def backward(ctx, grad_out):
        need = ctx.needs_input_grad
        r = smooth_backward(ctx.cx, ctx.grid, ctx.lam, grad_out, coords=need[3], dirs=need[4],
                            weights=any(need[5:]), index=ctx.index)
        gw = r["weights"]
        if gw is None:
            gw = [None] * ctx.nw
        elif isinstance(gw, torch.Tensor):
            gw = [gw]
        return (None, None, None, r["coords"], r["dirs"], *gw)


def smooth_wect(cx: SimplicialBatch, thr, lam: float, coords: torch.Tensor, dirs: torch.Tensor,
                *weights: torch.Tensor) -> torch.Tensor:
    """Differentiable relaxation S [B, d, T] of a simplicial batch whose
    coordinates, directions and (float32) weights may require gradients."""
    thr = torch.as_tensor(thr, dtype=torch.float32, device=coords.device)
    return SmoothWECTFunction.apply(cx, thr, _lam(lam), coords, dirs, *weights)


class SmoothWECT(torch.nn.Module):
    """Layer form: learnable directions (optional), fixed thresholds and sharpness."""

    def __init__(self, dirs, thr, lam: float, learn_dirs: bool = True):
        super().__init__()
        d = torch.as_tensor(dirs, dtype=torch.float32)
        if learn_dirs:
            self.dirs = torch.nn.Parameter(d)
        else:
            self.register_buffer("dirs", d)
        self.register_buffer("thr", torch.as_tensor(thr, dtype=torch.float32))
        self.lam = _lam(lam)

    def forward(self, cx, coords, *weights):
        return smooth_wect(cx, self.thr, self.lam, coords, self.dirs, *weights)
