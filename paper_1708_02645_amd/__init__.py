"""Python binding of libqmcspline (periodic tricubic B-spline orbital VGL on MI355X).

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of ``libqmcspline.so``, reached through its C ABI
(``include/qmcspline.h``).  PyTorch provides device memory and the stream.
There is no CPU fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmcspline.so")

DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
ELEM_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}
STATUS = {0: "SPL_OK", -1: "SPL_EINVAL", -2: "SPL_ENOMEM", -3: "SPL_EHIP", -4: "SPL_EUNSUPPORTED"}


class SplineError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("cell", ctypes.c_double * 3)]


class Layout(ctypes.Structure):
    _fields_ = [("row_bytes", ctypes.c_int64), ("n_pad", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("scales_offset", ctypes.c_int64), ("total_bytes", ctypes.c_int64),
                ("elem_bytes", ctypes.c_int32), ("padded", ctypes.c_int32 * 3)]


class Tile(ctypes.Structure):
    _fields_ = [("cw", ctypes.c_int32), ("nch", ctypes.c_int32), ("lpp", ctypes.c_int32), ("pb", ctypes.c_int32)]

    def astuple(self):
        return (self.cw, self.nch, self.lpp, self.pb)


_lib = None


def lib():
    """Load libqmcspline.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libqmcspline.so is not built (run __graft_entry__.build()); "
                              "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        p, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        sigs = {
            "spline_table_bytes": ([p, i32, ctypes.c_int], sz),
            "spline_get_layout": ([p, i32, ctypes.c_int, p], ctypes.c_int),
            "spline_pack_host": ([p, i32, p, ctypes.c_int, p, sz], ctypes.c_int),
            "spline_create": ([p, i32, p, ctypes.c_int, p, sz, p, p], ctypes.c_int),
            "spline_eval_vgl": ([p, p, i64, p, p, p, p], ctypes.c_int),
            "spline_eval_v": ([p, p, i64, p, p], ctypes.c_int),
            "spline_tile_candidates": ([p, p, i32, p], ctypes.c_int),
            "spline_set_tile": ([p, p], ctypes.c_int),
            "spline_get_tile": ([p, p], ctypes.c_int),
            "spline_autotune": ([p, p, i64, p, p, p, i32, ctypes.c_char_p, p, p], ctypes.c_int),
            "spline_get_info": ([p, p, p, p, p], ctypes.c_int),
            "spline_destroy": ([p], ctypes.c_int),
            "spline_last_error": ([], ctypes.c_char_p),
            "spline_plan_workspace_bytes": ([i32, p], sz),
            "spline_plan_create": ([p, i32, p, p, p, p, p, p, sz, i32, p, p], ctypes.c_int),
            "spline_plan_launch": ([p, p], ctypes.c_int),
            "spline_plan_launch_eager": ([p, p], ctypes.c_int),
            "spline_plan_get_info": ([p, p, p, p], ctypes.c_int),
            "spline_plan_destroy": ([p], ctypes.c_int),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def last_error() -> str:
    return lib().spline_last_error().decode()


def check(rc: int) -> None:
    if rc != 0:
        raise SplineError(rc, last_error())


def make_grid(grid, cell=(1.0, 1.0, 1.0)) -> Grid:
    g = Grid()
    for d in range(3):
        g.n[d] = int(grid[d])
        g.cell[d] = float(cell[d])
    return g


def table_bytes(grid, norb: int, dtype: str, cell=(1.0, 1.0, 1.0)) -> int:
    g = make_grid(grid, cell)
    return int(lib().spline_table_bytes(ctypes.byref(g), int(norb), DTYPES[dtype]))


def get_layout(grid, norb: int, dtype: str, cell=(1.0, 1.0, 1.0)) -> Layout:
    g = make_grid(grid, cell)
    out = Layout()
    check(lib().spline_get_layout(ctypes.byref(g), int(norb), DTYPES[dtype], ctypes.byref(out)))
    return out


def pack_host(grid, coefs: np.ndarray, dtype: str, cell=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Host-side packed table (halo layout + scales) as a uint8 array."""
    coefs = np.ascontiguousarray(coefs, dtype=np.float64)
    norb = coefs.shape[-1]
    nb = table_bytes(grid, norb, dtype, cell)
    if nb == 0:
        check(-1)
    buf = np.empty(nb, dtype=np.uint8)
    g = make_grid(grid, cell)
    check(lib().spline_pack_host(ctypes.byref(g), norb, coefs.ctypes.data, DTYPES[dtype], buf.ctypes.data, nb))
    return buf


def _stream_ptr(torch, device, stream):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream), stream


class Spline:
    """A coefficient table resident in device memory and its evaluation.

    coefs: numpy [n0, n1, n2, N] float64 (orbital fastest), copied at creation.
    dtype: storage type "f64" | "f32" | "bf16" | "f16".
    """

    def __init__(self, grid, coefs: np.ndarray, dtype: str = "f32", cell=(1.0, 1.0, 1.0), device="cuda", stream=None):
        import torch

        self._torch = torch
        coefs = np.ascontiguousarray(coefs, dtype=np.float64)
        if coefs.ndim != 4 or tuple(coefs.shape[:3]) != tuple(int(x) for x in grid):
            raise ValueError("coefs must have shape grid + (N,)")
        self.grid = tuple(int(x) for x in grid)
        self.cell = tuple(float(x) for x in cell)
        self.norb = int(coefs.shape[-1])
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        nb = table_bytes(self.grid, self.norb, dtype, self.cell)
        if nb == 0:
            check(-1)
        self.buf = torch.empty(nb, dtype=torch.uint8, device=self.device)
        g = make_grid(self.grid, self.cell)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            sp, _ = _stream_ptr(torch, self.device, stream)
            check(lib().spline_create(ctypes.byref(g), self.norb, coefs.ctypes.data, DTYPES[dtype],
                                      ctypes.c_void_p(self.buf.data_ptr()), nb, sp, ctypes.byref(h)))
        self._h = h
        self.layout = Layout()
        check(lib().spline_get_info(self._h, None, None, None, ctypes.byref(self.layout)))

    @property
    def handle(self):
        return self._h

    @property
    def out_dtype(self):
        return self._torch.float64 if self.dtype == "f64" else self._torch.float32

    def _pos(self, pos):
        torch = self._torch
        if not (isinstance(pos, torch.Tensor) and pos.device == self.device and pos.dtype == torch.float64
                and pos.is_contiguous() and pos.dim() == 2 and pos.shape[1] == 3):
            raise ValueError("pos must be a contiguous float64 [B,3] tensor on %s" % self.device)
        return pos

    def alloc_outputs(self, B: int):
        torch = self._torch
        kw = dict(dtype=self.out_dtype, device=self.device)
        return (torch.empty((B, self.norb), **kw), torch.empty((B, 3, self.norb), **kw),
                torch.empty((B, self.norb), **kw))

    def eval_vgl(self, pos, out=None, stream=None):
        """(V[B,N], G[B,3,N], L[B,N]) at positions pos[B,3] (float64, on device)."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V, G, L = out if out is not None else self.alloc_outputs(B)
        for t, shp in ((V, (B, self.norb)), (G, (B, 3, self.norb)), (L, (B, self.norb))):
            if tuple(t.shape) != shp or t.dtype != self.out_dtype or not t.is_contiguous() or t.device != self.device:
                raise ValueError("output tensor has wrong shape/dtype/device")
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_vgl(self._h, ctypes.c_void_p(pos.data_ptr()), B, ctypes.c_void_p(V.data_ptr()),
                                        ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(L.data_ptr()), sp))
        return V, G, L

    def eval_v(self, pos, out=None, stream=None):
        """V[B,N] at positions pos[B,3] (value only)."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V = out if out is not None else self._torch.empty((B, self.norb), dtype=self.out_dtype, device=self.device)
        if tuple(V.shape) != (B, self.norb) or V.dtype != self.out_dtype or not V.is_contiguous():
            raise ValueError("output tensor has wrong shape/dtype")
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_v(self._h, ctypes.c_void_p(pos.data_ptr()), B, ctypes.c_void_p(V.data_ptr()), sp))
        return V

    def tile_candidates(self):
        n = ctypes.c_int32()
        check(lib().spline_tile_candidates(self._h, None, 0, ctypes.byref(n)))
        arr = (Tile * max(1, n.value))()
        check(lib().spline_tile_candidates(self._h, arr, n.value, ctypes.byref(n)))
        return [arr[i].astuple() for i in range(n.value)]

    def set_tile(self, tile):
        t = Tile(*tile)
        check(lib().spline_set_tile(self._h, ctypes.byref(t)))

    def get_tile(self):
        t = Tile()
        check(lib().spline_get_tile(self._h, ctypes.byref(t)))
        return t.astuple()

    def autotune(self, pos, reps: int = 5, cache_path: str | None = None, out=None, stream=None):
        pos = self._pos(pos)
        B = pos.shape[0]
        V, G, L = out if out is not None else self.alloc_outputs(B)
        t = Tile()
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_autotune(self._h, ctypes.c_void_p(pos.data_ptr()), B, ctypes.c_void_p(V.data_ptr()),
                                        ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(L.data_ptr()), int(reps),
                                        None if cache_path is None else cache_path.encode(), sp, ctypes.byref(t)))
        return t.astuple()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().spline_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Ragged multi-table evaluation: one persistent launch captured in a HIP
    graph.  splines: list of Spline (same storage type); positions: list of
    float64 [B_t, 3] device tensors (B_t may be 0).  Outputs are allocated
    here (or passed as a list of (V, G, L)) and stay bound to the plan."""

    def __init__(self, splines, positions, outs=None, tune_reps: int = 3, stream=None):
        import torch

        self._torch = torch
        n = len(splines)
        if n == 0 or len(positions) != n:
            raise ValueError("need one positions tensor per table")
        self.splines = list(splines)
        self.positions = [s._pos(p) for s, p in zip(splines, positions)]
        self.outs = list(outs) if outs is not None else [s.alloc_outputs(p.shape[0]) for s, p in zip(splines, positions)]
        dev = splines[0].device
        Bs = (ctypes.c_int64 * n)(*[p.shape[0] for p in self.positions])
        nb = int(lib().spline_plan_workspace_bytes(n, Bs))
        if nb == 0:
            check(-1)
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        vp = ctypes.c_void_p
        tabs = (vp * n)(*[s.handle.value for s in splines])
        pos = (vp * n)(*[p.data_ptr() for p in self.positions])
        V = (vp * n)(*[o[0].data_ptr() for o in self.outs])
        G = (vp * n)(*[o[1].data_ptr() for o in self.outs])
        L = (vp * n)(*[o[2].data_ptr() for o in self.outs])
        h = vp()
        L_ = lib()
        with torch.cuda.device(dev):
            sp, _ = _stream_ptr(torch, dev, stream)
            check(L_.spline_plan_create(tabs, n, Bs, pos, V, G, L, vp(self.ws.data_ptr()), nb, int(tune_reps), sp,
                                        ctypes.byref(h)))
        self._h = h
        self.device = dev

    def launch(self, stream=None):
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_plan_launch(self._h, sp))
        return self.outs

    def launch_eager(self, stream=None):
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_plan_launch_eager(self._h, sp))
        return self.outs

    def info(self):
        t = Tile()
        nt, nb = ctypes.c_int32(), ctypes.c_int32()
        check(lib().spline_plan_get_info(self._h, ctypes.byref(t), ctypes.byref(nt), ctypes.byref(nb)))
        return {"tile": t.astuple(), "tasks": nt.value, "blocks": nb.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().spline_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
