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
            "spline_sorted_workspace_bytes": ([p, i64], sz),
            "spline_eval_vgl_sorted": ([p, p, i64, p, p, p, p, sz, p], ctypes.c_int),
            "spline_eval_vgl_sorted_noalloc": ([p, p, i64, p, p, p, p], ctypes.c_int),
            "spline_eval_v_sorted": ([p, p, i64, p, p, sz, p], ctypes.c_int),
            "spline_eval_ratio_vgl_sorted": ([p, p, i64, p, i64, p, p, p, sz, p], ctypes.c_int),
            "spline_eval_ratio_v_sorted": ([p, p, i64, p, i64, p, p, p, sz, p], ctypes.c_int),
            "spline_eval_vgh_sorted": ([p, p, i64, p, p, p, p, sz, p], ctypes.c_int),
            "spline_set_sorted_tile": ([p, p], ctypes.c_int),
            "spline_get_sorted_tile": ([p, p], ctypes.c_int),
            "spline_autotune_sorted": ([p, p, i64, p, p, p, p, sz, ctypes.c_int32, ctypes.c_char_p, p, p],
                                       ctypes.c_int),
            "spline_eval_ratio_vgl": ([p, p, i64, p, i64, p, p, p], ctypes.c_int),
            "spline_det_update": ([p, i32, i64, p, p, p, i64, i64, ctypes.c_int, p], ctypes.c_int),
            "jastrow_bytes": ([p, p], sz),
            "jastrow_create": ([p, p, p, p, p, p, p, sz, p, p], ctypes.c_int),
            "jastrow_destroy": ([p], ctypes.c_int),
            "jastrow_move": ([p, p, i64, i64, p, p, p, i64, p, p], ctypes.c_int),
            "jastrow_evaluate": ([p, p, i64, i64, i64, p, p, p, p], ctypes.c_int),
            "jastrow_dist_rows": ([p, p, i64, i64, p, p, i64, p, p, p, p, p], ctypes.c_int),
            "jastrow_accept": ([p, p, i64, i64, p, p, p, i64, p], ctypes.c_int),
            "spline_dlu_workspace_bytes": ([i32, i32, i64], sz),
            "spline_dlu_create": ([i32, i32, i64, p, sz, p, p], ctypes.c_int),
            "spline_dlu_destroy": ([p], ctypes.c_int),
            "spline_dlu_ratio": ([p, p, i64, p, p, p, p, p, i64, p, p], ctypes.c_int),
            "spline_dlu_accept": ([p, p, i64, p, p, p, i64, p], ctypes.c_int),
            "spline_dlu_accept_ratio": ([p, p, i64, p, p, p, p, p, p, p, i64, p, p], ctypes.c_int),
            "spline_dlu_flush": ([p, p, i64, p], ctypes.c_int),
            "spline_set_lattice": ([p, p], ctypes.c_int),
            "spline_get_lattice": ([p, p], ctypes.c_int),
            "spline_eval_vgh": ([p, p, i64, p, p, p, p], ctypes.c_int),
            "spline_vgh_tile_candidates": ([p, p, i32, p], ctypes.c_int),
            "spline_set_vgh_tile": ([p, p], ctypes.c_int),
            "spline_get_vgh_tile": ([p, p], ctypes.c_int),
            "spline_autotune_vgh": ([p, p, i64, p, p, p, i32, p, p], ctypes.c_int),
            "spline_eval_ratio_v": ([p, p, i64, p, i64, p, p, p], ctypes.c_int),
            "spline_tile_candidates": ([p, p, i32, p], ctypes.c_int),
            "spline_set_tile": ([p, p], ctypes.c_int),
            "spline_get_tile": ([p, p], ctypes.c_int),
            "spline_get_value_tile": ([p, p], ctypes.c_int),
            "spline_get_sorted_value_tile": ([p, p], ctypes.c_int),
            "spline_get_sorted_vgh_tile": ([p, p], ctypes.c_int),
            "spline_autotune": ([p, p, i64, p, p, p, i32, ctypes.c_char_p, p, p], ctypes.c_int),
            "spline_get_info": ([p, p, p, p, p], ctypes.c_int),
            "spline_destroy": ([p], ctypes.c_int),
            "spline_last_error": ([], ctypes.c_char_p),
            "spline_plan_workspace_bytes": ([i32, p], sz),
            "spline_plan_workspace_bytes_sorted": ([i32, p], sz),
            "spline_plan_create": ([p, i32, p, p, p, p, p, p, sz, i32, p, p], ctypes.c_int),
            "spline_plan_create_sorted": ([p, i32, p, p, p, p, p, p, sz, i32, p, p], ctypes.c_int),
            "spline_plan_launch": ([p, p], ctypes.c_int),
            "spline_plan_launch_eager": ([p, p], ctypes.c_int),
            "spline_plan_get_info": ([p, p, p, p], ctypes.c_int),
            "spline_plan_destroy": ([p], ctypes.c_int),
            "spline_probe_stream_read": ([p, sz, p, i32, p], ctypes.c_int),
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


def probe_stream_read(buf, grid: int = 1024, out=None, stream=None):
    """One launch of the library's plain streaming-read kernel over a uint8
    device tensor (for measuring the attainable read bandwidth)."""
    import torch

    if not (isinstance(buf, torch.Tensor) and buf.is_cuda and buf.is_contiguous()):
        raise ValueError("buf must be a contiguous GPU tensor")
    if out is None:
        out = torch.empty(grid * 256, dtype=torch.float32, device=buf.device)
    _need(out, torch.float32, (grid * 256,), buf.device, "out")
    sp, _ = _stream_ptr(torch, buf.device, stream)
    check(lib().spline_probe_stream_read(ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                         ctypes.c_void_p(out.data_ptr()), int(grid), sp))
    return out


def det_update(ainv, k, phi, walkers=None, stream=None):
    """Sherman-Morrison update, in place, of the inverses ainv[W, n, n] (float32
    or float64, contiguous, on a GPU) after accepted moves: slot j updates
    walker walkers[j] (or j) for electron k[j] with orbital values phi[j, :n]."""
    import torch

    if not (isinstance(ainv, torch.Tensor) and ainv.is_cuda and ainv.dim() == 3 and ainv.shape[1] == ainv.shape[2]
            and ainv.is_contiguous() and ainv.dtype in (torch.float32, torch.float64)):
        raise ValueError("ainv must be a contiguous [W, n, n] float32/float64 GPU tensor")
    W_, n = ainv.shape[0], ainv.shape[1]
    count = k.shape[0]
    for t, what in ((k, "k"),) + (((walkers, "walkers"),) if walkers is not None else ()):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.int32 and t.device == ainv.device
                and t.is_contiguous() and tuple(t.shape) == (count,)):
            raise ValueError("%s must be a contiguous int32 [count] tensor on the same device" % what)
    if not (isinstance(phi, torch.Tensor) and phi.dtype == ainv.dtype and phi.device == ainv.device
            and phi.dim() == 2 and phi.shape[0] == count and phi.shape[1] >= n and phi.stride(1) == 1):
        raise ValueError("phi must be a [count, >=n] tensor of the inverse's dtype with unit column stride")
    if walkers is None and count > W_:
        raise ValueError("more slots than walkers")
    if walkers is not None and count and (int(walkers.min().item()) < 0 or int(walkers.max().item()) >= W_):
        raise ValueError("walker index out of range")
    dt = DTYPES["f64" if ainv.dtype == torch.float64 else "f32"]
    with torch.cuda.device(ainv.device):
        sp, _ = _stream_ptr(torch, ainv.device, stream)
        check(lib().spline_det_update(ctypes.c_void_p(ainv.data_ptr()), n, n * n,
                                      ctypes.c_void_p(walkers.data_ptr()) if walkers is not None else None,
                                      ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(phi.data_ptr()), phi.stride(0),
                                      count, dt, sp))
    return ainv


def _stream_ptr(torch, device, stream):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream), stream


def _need(t, dtype, shape, device, what):
    """t itself if it is a contiguous tensor of this dtype, shape and device
    (the kernels receive its raw pointer); ValueError otherwise."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.dtype == dtype and t.device == device and t.is_contiguous()
            and tuple(t.shape) == tuple(shape)):
        raise ValueError("%s must be a contiguous %s tensor of shape %s on %s" % (what, dtype, tuple(shape), device))
    return t


def _need_pos(t, device, what="pos"):
    """Positions: a contiguous float64 [B, 3] tensor on the device."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.dim() == 2):
        raise ValueError("%s must be a float64 [B, 3] tensor" % what)
    return _need(t, torch.float64, (t.shape[0], 3), device, what)


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

    def _vgl_out(self, out, B):
        """(V, G, L) outputs for B positions: allocated, or the caller's, checked."""
        if out is None:
            return self.alloc_outputs(B)
        V, G, L = out
        return (_need(V, self.out_dtype, (B, self.norb), self.device, "V"),
                _need(G, self.out_dtype, (B, 3, self.norb), self.device, "G"),
                _need(L, self.out_dtype, (B, self.norb), self.device, "L"))

    def _vgh_out(self, out, B):
        if out is None:
            return self.alloc_vgh(B)
        V, G, H = out
        return (_need(V, self.out_dtype, (B, self.norb), self.device, "V"),
                _need(G, self.out_dtype, (B, 3, self.norb), self.device, "G"),
                _need(H, self.out_dtype, (B, 6, self.norb), self.device, "H"))

    def _v_out(self, out, B):
        if out is None:
            return self._torch.empty((B, self.norb), dtype=self.out_dtype, device=self.device)
        return _need(out, self.out_dtype, (B, self.norb), self.device, "V")

    def eval_vgl(self, pos, out=None, stream=None):
        """(V[B,N], G[B,3,N], L[B,N]) at positions pos[B,3] (float64, on device)."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V, G, L = self._vgl_out(out, B)
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_vgl(self._h, ctypes.c_void_p(pos.data_ptr()), B, ctypes.c_void_p(V.data_ptr()),
                                        ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(L.data_ptr()), sp))
        return V, G, L

    def eval_v(self, pos, out=None, stream=None):
        """V[B,N] at positions pos[B,3] (value only)."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V = self._v_out(out, B)
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_v(self._h, ctypes.c_void_p(pos.data_ptr()), B, ctypes.c_void_p(V.data_ptr()), sp))
        return V

    def _sorted_ws(self, B: int, workspace):
        nb = lib().spline_sorted_workspace_bytes(self._h, B)
        if workspace is None:
            ws = getattr(self, "_sws", None)
            if ws is None or ws.numel() < nb:
                ws = self._torch.empty(max(nb, 256), dtype=self._torch.uint8, device=self.device)
                self._sws = ws
            workspace = ws
        torch = self._torch
        if not (isinstance(workspace, torch.Tensor) and workspace.device == self.device and workspace.is_contiguous()
                and workspace.numel() * workspace.element_size() >= nb):
            raise ValueError("workspace must be a contiguous tensor of >= %d bytes on %s" % (nb, self.device))
        return ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()

    def eval_vgl_sorted(self, pos, out=None, workspace=None, stream=None):
        """eval_vgl in locality order (same results bit for bit, faster for
        large batches); workspace: uint8 device tensor, kept on the object
        when not given."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V, G, L = self._vgl_out(out, B)
        wp, wn = self._sorted_ws(B, workspace)
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_vgl_sorted(self._h, ctypes.c_void_p(pos.data_ptr()), B,
                                               ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                               ctypes.c_void_p(L.data_ptr()), wp, wn, sp))
        return V, G, L

    def eval_vgl_sorted_noalloc(self, pos, out, stream=None):
        """eval_vgl_sorted through the entry point that allocates nothing (its
        scratch is the library's static device array); out: caller's (V, G, L)."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V, G, L = self._vgl_out(out, B)
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_vgl_sorted_noalloc(self._h, ctypes.c_void_p(pos.data_ptr()), B,
                                                       ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                                       ctypes.c_void_p(L.data_ptr()), sp))
        return V, G, L

    def set_sorted_tile(self, tile):
        t = Tile(*tile)
        check(lib().spline_set_sorted_tile(self._h, ctypes.byref(t)))

    def get_sorted_tile(self):
        t = Tile()
        check(lib().spline_get_sorted_tile(self._h, ctypes.byref(t)))
        return t.astuple()

    def get_sorted_value_tile(self):
        t = Tile()
        check(lib().spline_get_sorted_value_tile(self._h, ctypes.byref(t)))
        return t.astuple()

    def get_sorted_vgh_tile(self):
        t = Tile()
        check(lib().spline_get_sorted_vgh_tile(self._h, ctypes.byref(t)))
        return t.astuple()

    def autotune_sorted(self, pos, reps: int = 5, cache_path: str | None = None, out=None, workspace=None,
                        stream=None):
        """Tile shape of the locality-ordered VGL path (see spline_autotune_sorted)."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V, G, L = self._vgl_out(out, B)
        wp, wn = self._sorted_ws(B, workspace)
        t = Tile()
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_autotune_sorted(self._h, ctypes.c_void_p(pos.data_ptr()), B,
                                               ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                               ctypes.c_void_p(L.data_ptr()), wp, wn, int(reps),
                                               None if cache_path is None else cache_path.encode(), sp,
                                               ctypes.byref(t)))
        return t.astuple()

    def eval_v_sorted(self, pos, out=None, workspace=None, stream=None):
        """eval_v in locality order (same results bit for bit)."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V = self._v_out(out, B)
        wp, wn = self._sorted_ws(B, workspace)
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_v_sorted(self._h, ctypes.c_void_p(pos.data_ptr()), B,
                                             ctypes.c_void_p(V.data_ptr()), wp, wn, sp))
        return V

    def set_lattice(self, lattice):
        """Give the table a general cell: lattice[3,3] has the Cartesian
        lattice vectors as rows; grid axis d runs along row d."""
        lat = np.ascontiguousarray(lattice, dtype=np.float64).reshape(9)
        check(lib().spline_set_lattice(self._h, lat.ctypes.data_as(ctypes.c_void_p)))

    def get_lattice(self) -> np.ndarray:
        lat = np.empty(9)
        check(lib().spline_get_lattice(self._h, lat.ctypes.data_as(ctypes.c_void_p)))
        return lat.reshape(3, 3)

    def alloc_vgh(self, B: int):
        torch = self._torch
        kw = dict(dtype=self.out_dtype, device=self.device)
        return (torch.empty((B, self.norb), **kw), torch.empty((B, 3, self.norb), **kw),
                torch.empty((B, 6, self.norb), **kw))

    def eval_vgh(self, pos, out=None, stream=None):
        """(V[B,N], G[B,3,N], H[B,6,N]) with H = Cartesian xx, xy, xz, yy, yz, zz."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V, G, H = self._vgh_out(out, B)
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_vgh(self._h, ctypes.c_void_p(pos.data_ptr()), B, ctypes.c_void_p(V.data_ptr()),
                                        ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(H.data_ptr()), sp))
        return V, G, H

    def eval_vgh_sorted(self, pos, out=None, workspace=None, stream=None):
        """eval_vgh in locality order (same results bit for bit)."""
        pos = self._pos(pos)
        B = pos.shape[0]
        V, G, H = self._vgh_out(out, B)
        wp, wn = self._sorted_ws(B, workspace)
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_eval_vgh_sorted(self._h, ctypes.c_void_p(pos.data_ptr()), B,
                                               ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                               ctypes.c_void_p(H.data_ptr()), wp, wn, sp))
        return V, G, H

    def get_value_tile(self):
        t = Tile()
        check(lib().spline_get_value_tile(self._h, ctypes.byref(t)))
        return t.astuple()

    def vgh_tile_candidates(self):
        n = ctypes.c_int32()
        check(lib().spline_vgh_tile_candidates(self._h, None, 0, ctypes.byref(n)))
        arr = (Tile * max(1, n.value))()
        check(lib().spline_vgh_tile_candidates(self._h, arr, n.value, ctypes.byref(n)))
        return [arr[i].astuple() for i in range(n.value)]

    def set_vgh_tile(self, tile):
        check(lib().spline_set_vgh_tile(self._h, ctypes.byref(Tile(*tile))))

    def get_vgh_tile(self):
        t = Tile()
        check(lib().spline_get_vgh_tile(self._h, ctypes.byref(t)))
        return t.astuple()

    def autotune_vgh(self, pos, reps: int = 5, out=None, stream=None):
        pos = self._pos(pos)
        V, G, H = self._vgh_out(out, pos.shape[0])
        t = Tile()
        with self._torch.cuda.device(self.device):
            sp, _ = _stream_ptr(self._torch, self.device, stream)
            check(lib().spline_autotune_vgh(self._h, ctypes.c_void_p(pos.data_ptr()), pos.shape[0],
                                            ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                            ctypes.c_void_p(H.data_ptr()), reps, sp, ctypes.byref(t)))
        return t.astuple()

    def _ratio(self, vgl, pos, ainv, ld, rows, out, stream, sorted_ws=None):
        torch = self._torch
        pos = self._pos(pos)
        B = pos.shape[0]
        if not (isinstance(ainv, torch.Tensor) and ainv.device == self.device and ainv.dtype == self.out_dtype
                and ainv.is_contiguous()):
            raise ValueError("ainv must be a contiguous %s tensor on %s" % (self.out_dtype, self.device))
        ld = self.norb if ld is None else int(ld)
        if ld < 0:
            raise ValueError("ld must be >= 0")
        if rows is not None:
            if not (isinstance(rows, torch.Tensor) and rows.dtype == torch.int32 and rows.device == self.device
                    and rows.is_contiguous() and tuple(rows.shape) == (B,)):
                raise ValueError("rows must be a contiguous int32 [B] tensor on %s" % self.device)
            last = int(rows.max().item()) if B else 0
            if B and int(rows.min().item()) < 0:
                raise ValueError("negative row index")
        else:
            last = B - 1
        if B and last * ld + self.norb > ainv.numel():
            raise ValueError("rows of ainv extend past the tensor")
        shape = (B, 5) if vgl else (B,)
        D = out if out is not None else torch.empty(shape, dtype=self.out_dtype, device=self.device)
        if tuple(D.shape) != shape or D.dtype != self.out_dtype or not D.is_contiguous() or D.device != self.device:
            raise ValueError("output tensor must be a contiguous %s %s tensor" % (self.out_dtype, shape))
        args = [self._h, ctypes.c_void_p(pos.data_ptr()), B, ctypes.c_void_p(ainv.data_ptr()), ld,
                ctypes.c_void_p(rows.data_ptr()) if rows is not None else None, ctypes.c_void_p(D.data_ptr())]
        if sorted_ws is not False and sorted_ws is not None:
            fn = lib().spline_eval_ratio_vgl_sorted if vgl else lib().spline_eval_ratio_v_sorted
            args += list(self._sorted_ws(B, None if sorted_ws is True else sorted_ws))
        else:
            fn = lib().spline_eval_ratio_vgl if vgl else lib().spline_eval_ratio_v
        with torch.cuda.device(self.device):
            sp, _ = _stream_ptr(torch, self.device, stream)
            check(fn(*args, sp))
        return D

    def eval_ratio_vgl_sorted(self, pos, ainv, ld=None, rows=None, out=None, workspace=None, stream=None):
        """eval_ratio_vgl in locality order (same results bit for bit)."""
        return self._ratio(True, pos, ainv, ld, rows, out, stream, workspace if workspace is not None else True)

    def eval_ratio_v_sorted(self, pos, ainv, ld=None, rows=None, out=None, workspace=None, stream=None):
        """eval_ratio_v in locality order (same results bit for bit)."""
        return self._ratio(False, pos, ainv, ld, rows, out, stream, workspace if workspace is not None else True)

    def eval_ratio_vgl(self, pos, ainv, ld=None, rows=None, out=None, stream=None):
        """D[B,5]: dot products of each position's row of A^-1 with the orbital
        value, gradient (x, y, z) and Laplacian at that position (determinant
        lemma).  The row of position b starts at element (rows[b] or b) * ld of
        ainv (ld defaults to the orbital count)."""
        return self._ratio(True, pos, ainv, ld, rows, out, stream)

    def eval_ratio_v(self, pos, ainv, ld=None, rows=None, out=None, stream=None):
        """R[B]: determinant ratios only (dot products with orbital values)."""
        return self._ratio(False, pos, ainv, ld, rows, out, stream)

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
        V, G, L = self._vgl_out(out, B)
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

    def __init__(self, splines, positions, outs=None, tune_reps: int = 3, stream=None, sorted=False):
        import torch

        self._torch = torch
        self.sorted = bool(sorted)
        n = len(splines)
        if n == 0 or len(positions) != n:
            raise ValueError("need one positions tensor per table")
        self.splines = list(splines)
        self.positions = [s._pos(p) for s, p in zip(splines, positions)]
        outs = [None] * n if outs is None else list(outs)
        if len(outs) != n:
            raise ValueError("need one (V, G, L) triple per table")
        self.outs = [s._vgl_out(o, p.shape[0]) for s, p, o in zip(splines, self.positions, outs)]
        dev = splines[0].device
        Bs = (ctypes.c_int64 * n)(*[p.shape[0] for p in self.positions])
        nb = int((lib().spline_plan_workspace_bytes_sorted if self.sorted else lib().spline_plan_workspace_bytes)(n, Bs))
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
            create = L_.spline_plan_create_sorted if self.sorted else L_.spline_plan_create
            check(create(tabs, n, Bs, pos, V, G, L, vp(self.ws.data_ptr()), nb, int(tune_reps), sp, ctypes.byref(h)))
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


class MlpDesc(ctypes.Structure):
    _fields_ = [("n_freq", ctypes.c_int32), ("width", ctypes.c_int32 * 4)]


class MlpLayout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n_params", "W1", "b1", "W2", "b2", "W3", "b3", "params", "adam_m", "adam_v", "weights_bf16",
                 "mu", "sd", "loss_w", "freqs", "bin_err", "meta", "total")] + [("max_bins", ctypes.c_int32)]


_MLP_SIGS = {
    "spline_mlp_param_bytes": (["p"], "sz"),
    "spline_mlp_get_layout": (["p", "p"], "i"),
    "spline_mlp_create": (["p", "p", "p", "p", "p", "sz", "p", "p"], "i"),
    "spline_mlp_attach": (["p", "p", "p", "sz", "p", "p"], "i"),
    "spline_mlp_init_output": (["p", "p", "p", "p", "i64", "p"], "i"),
    "spline_mlp_train_workspace_bytes": (["p", "i64"], "sz"),
    "spline_mlp_grad": (["p", "p", "p", "p", "p", "i64", "p", "sz", "p", "p", "p"], "i"),
    "spline_mlp_train_step": (["p", "p", "p", "p", "p", "i64", "f", "p", "sz", "p", "p"], "i"),
    "spline_mlp_forward": (["p", "p", "i64", "p", "p", "p", "p"], "i"),
    "spline_mlp_errmap_workspace_bytes": (["p", "i64"], "sz"),
    "spline_mlp_build_error_map": (["p", "p", "p", "i64", "i32", "p", "sz", "p"], "i"),
    "spline_mlp_eval_workspace_bytes": (["i64"], "sz"),
    "spline_mlp_eval_vgl": (["p", "p", "f", "p", "i64", "p", "p", "p", "p", "sz", "p", "p"], "i"),
    "spline_mlp_get_info": (["p", "p", "p"], "i"),
    "spline_mlp_destroy": (["p"], "i"),
    "spline_mlp_select_frequencies": (["p", "i32", "p", "i32", "i32", "p", "p"], "i"),
}


def _mlp_lib():
    L = lib()
    if not getattr(L, "_mlp_sigs", False):
        T = {"p": ctypes.c_void_p, "sz": ctypes.c_size_t, "i": ctypes.c_int, "i32": ctypes.c_int32,
             "i64": ctypes.c_int64, "f": ctypes.c_float}
        for name, (args, res) in _MLP_SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = [T[a] for a in args]
            fn.restype = T[res]
        L._mlp_sigs = True
    return L


def mlp_desc(norb: int) -> MlpDesc:
    d = MlpDesc()
    d.n_freq = 48
    for i, w in enumerate((96, 256, 256, int(norb))):
        d.width[i] = w
    return d


def mlp_layout(norb: int) -> MlpLayout:
    out = MlpLayout()
    d = mlp_desc(norb)
    check(_mlp_lib().spline_mlp_get_layout(ctypes.byref(d), ctypes.byref(out)))
    return out


def spectral_frequencies(coefs: np.ndarray, count: int = 48, kmax: int = 4, with_energy: bool = False):
    """The `count` integer frequency vectors (one of each +-k pair, 0 < |k| <= kmax)
    carrying the most energy in the table's coefficients, summed over orbitals
    (spline_mlp_select_frequencies).  with_energy=True also returns a dict of
    the chosen pairs' energies, the energy at k = 0 and the whole spectrum's."""
    c = np.ascontiguousarray(coefs, dtype=np.float64)
    if c.ndim != 4:
        raise ValueError("coefs must be [n0, n1, n2, N]")
    g = Grid()
    for d in range(3):
        g.n[d] = c.shape[d]
        g.cell[d] = 1.0
    out = np.zeros((int(count), 3), dtype=np.int32)
    en = np.zeros(int(count) + 2)
    check(_mlp_lib().spline_mlp_select_frequencies(ctypes.byref(g), c.shape[3], c.ctypes.data, int(count), int(kmax),
                                                   out.ctypes.data, en.ctypes.data))
    if with_energy:
        return out, {"pairs": en[:count].copy(), "k0": float(en[count]), "total": float(en[count + 1])}
    return out


def flatten_mlp_params(Ws, bs) -> np.ndarray:
    """Flat FP32 parameter vector [W1 | b1 | W2 | b2 | W3 | b3] (weights [out][in])."""
    parts = []
    for W, b in zip(Ws, bs):
        parts += [np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()]
    return np.concatenate(parts)


class SurrogateMLP:
    """The learned surrogate of a table, state held in one device buffer."""

    def __init__(self, norb: int, freqs=None, params=None, cell=(1.0, 1.0, 1.0), device="cuda", state=None,
                 stream=None):
        import torch

        self._torch = torch
        self.norb = int(norb)
        self.cell = tuple(float(x) for x in cell)
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        L = _mlp_lib()
        self.desc = mlp_desc(norb)
        self.layout = mlp_layout(norb)
        nb = int(L.spline_mlp_param_bytes(ctypes.byref(self.desc)))
        cell_a = (ctypes.c_double * 3)(*self.cell)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            sp, _ = _stream_ptr(torch, self.device, stream)
            if state is not None:  # resume from a saved buffer
                self.buf = state.to(self.device).clone()
                if self.buf.numel() < nb:
                    raise ValueError("state buffer too small")
                check(L.spline_mlp_attach(ctypes.byref(self.desc), cell_a, ctypes.c_void_p(self.buf.data_ptr()),
                                          self.buf.numel(), sp, ctypes.byref(h)))
            else:
                fr = np.ascontiguousarray(freqs, dtype=np.int32)
                pr = np.ascontiguousarray(params, dtype=np.float32)
                if fr.shape != (48, 3) or pr.size != self.layout.n_params:
                    raise ValueError("need freqs [48,3] and %d parameters" % self.layout.n_params)
                self.buf = torch.empty(nb, dtype=torch.uint8, device=self.device)
                check(L.spline_mlp_create(ctypes.byref(self.desc), fr.ctypes.data, cell_a, pr.ctypes.data,
                                          ctypes.c_void_p(self.buf.data_ptr()), nb, sp, ctypes.byref(h)))
        self._h = h
        self._ws = {}

    def _stream(self, stream):
        return _stream_ptr(self._torch, self.device, stream)[0]

    def _workspace(self, key, nbytes):
        t = self._ws.get(key)
        if t is None or t.numel() < nbytes:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
            self._ws[key] = t
        return t

    def _out(self, B):
        kw = dict(dtype=self._torch.float32, device=self.device)
        return (self._torch.empty((B, self.norb), **kw), self._torch.empty((B, 3, self.norb), **kw),
                self._torch.empty((B, self.norb), **kw))

    def _vgl(self, vgl, B, what):
        """A caller's float32 (V, G, L) triple for B positions, checked."""
        f32 = self._torch.float32
        V, G, L = vgl
        return (_need(V, f32, (B, self.norb), self.device, what + " V"),
                _need(G, f32, (B, 3, self.norb), self.device, what + " G"),
                _need(L, f32, (B, self.norb), self.device, what + " L"))

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(t.data_ptr())

    def state(self):
        """A copy of the whole network state (parameters, Adam moments, map)."""
        return self.buf.clone()

    def init_output(self, targets, stream=None):
        V, G, L = self._vgl(targets, targets[0].shape[0], "targets")
        check(_mlp_lib().spline_mlp_init_output(self._h, self._p(V), self._p(G), self._p(L), V.shape[0],
                                                self._stream(stream)))

    def grad(self, pos, targets, stream=None):
        pos = _need_pos(pos, self.device)
        B = pos.shape[0]
        targets = self._vgl(targets, B, "targets")
        L_ = _mlp_lib()
        nb = L_.spline_mlp_train_workspace_bytes(self._h, B)
        ws = self._workspace("train", nb)
        g = self._torch.empty(self.layout.n_params, dtype=self._torch.float32, device=self.device)
        loss = self._torch.zeros(1, dtype=self._torch.float32, device=self.device)
        V, G, L = targets
        check(L_.spline_mlp_grad(self._h, self._p(pos), self._p(V), self._p(G), self._p(L), B, self._p(ws), ws.numel(),
                                 self._p(g), self._p(loss), self._stream(stream)))
        return g, loss

    def train_step(self, pos, targets, lr: float, loss_out=None, stream=None):
        pos = _need_pos(pos, self.device)
        B = pos.shape[0]
        targets = self._vgl(targets, B, "targets")
        if loss_out is not None:
            _need(loss_out, self._torch.float32, (1,), self.device, "loss_out")
        L_ = _mlp_lib()
        nb = L_.spline_mlp_train_workspace_bytes(self._h, B)
        ws = self._workspace("train", nb)
        V, G, L = targets
        check(L_.spline_mlp_train_step(self._h, self._p(pos), self._p(V), self._p(G), self._p(L), B, float(lr),
                                       self._p(ws), ws.numel(),
                                       None if loss_out is None else self._p(loss_out), self._stream(stream)))

    def forward(self, pos, out=None, stream=None):
        pos = _need_pos(pos, self.device)
        B = pos.shape[0]
        V, G, L = self._vgl(out, B, "out") if out is not None else self._out(B)
        check(_mlp_lib().spline_mlp_forward(self._h, self._p(pos), B, self._p(V), self._p(G), self._p(L),
                                            self._stream(stream)))
        return V, G, L

    def build_error_map(self, table, val_pos, bins_per_dim: int = 8, stream=None):
        val_pos = _need_pos(val_pos, self.device, "val_pos")
        L_ = _mlp_lib()
        n = val_pos.shape[0]
        ws = self._workspace("errmap", L_.spline_mlp_errmap_workspace_bytes(self._h, n))
        check(L_.spline_mlp_build_error_map(self._h, table.handle, self._p(val_pos), n, int(bins_per_dim),
                                            self._p(ws), ws.numel(), self._stream(stream)))

    def eval_vgl(self, pos, fallback=None, tol: float = 1e-3, out=None, stream=None):
        """(V, G, L, n_fallback tensor) with routing of untrusted bins to `fallback`."""
        pos = _need_pos(pos, self.device)
        B = pos.shape[0]
        L_ = _mlp_lib()
        V, G, L = self._vgl(out, B, "out") if out is not None else self._out(B)
        ws = self._workspace("eval", L_.spline_mlp_eval_workspace_bytes(B))
        nf = self._torch.zeros(1, dtype=self._torch.int32, device=self.device)
        check(L_.spline_mlp_eval_vgl(self._h, None if fallback is None else fallback.handle, float(tol),
                                     self._p(pos), B, self._p(V), self._p(G), self._p(L), self._p(ws), ws.numel(),
                                     self._p(nf), self._stream(stream)))
        return V, G, L, nf

    def info(self):
        st, nb = ctypes.c_int64(), ctypes.c_int32()
        check(_mlp_lib().spline_mlp_get_info(self._h, ctypes.byref(st), ctypes.byref(nb)))
        return {"step": st.value, "bins_per_dim": nb.value}

    def bin_errors(self):
        """The error map as a float32 numpy array [nb, nb, nb] (bins along x,
        y, z of the fractional position), copied from the state buffer."""
        nb = self.info()["bins_per_dim"]
        lay = self.layout
        raw = self.buf[lay.bin_err:lay.bin_err + 4 * nb ** 3].cpu().numpy()
        return raw.view(np.float32).reshape(nb, nb, nb).copy()

    def params_numpy(self):
        """Parameters as float64 numpy arrays in the oracle's dictionary form."""
        lay = self.layout
        b = self.buf.cpu().numpy()
        P = b[lay.params:lay.params + 4 * lay.n_params].view(np.float32).astype(np.float64)
        H, N = 256, self.norb
        out = dict(W1=P[lay.W1:lay.b1].reshape(H, 96), b1=P[lay.b1:lay.W2], W2=P[lay.W2:lay.b2].reshape(H, H),
                   b2=P[lay.b2:lay.W3], W3=P[lay.W3:lay.b3].reshape(N, H), b3=P[lay.b3:lay.b3 + N])
        out["mu"] = b[lay.mu:lay.mu + 4 * N].view(np.float32).astype(np.float64)
        out["sd"] = b[lay.sd:lay.sd + 4 * N].view(np.float32).astype(np.float64)
        out["freqs"] = b[lay.freqs:lay.freqs + 4 * 144].view(np.int32).reshape(48, 3).copy()
        out["loss_w"] = b[lay.loss_w:lay.loss_w + 12].view(np.float32).astype(np.float64)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _mlp_lib().spline_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class JastrowDesc(ctypes.Structure):
    _fields_ = [("n_elec", ctypes.c_int32), ("n_up", ctypes.c_int32), ("n_ion", ctypes.c_int32),
                ("n_species", ctypes.c_int32), ("cell", ctypes.c_double * 3)]


class Jastrow:
    """One- and two-body Jastrow factor on a GPU (include/qmcjastrow.h).

    f1: one (coefs, rcut) per ion species; uu / ud: the two-body functors for
    equal and opposite spins.  Electron positions are float32 tensors
    [W, 3, ld] (structure of arrays; ``positions`` converts [W, N, 3])."""

    def __init__(self, cell, ions, species, f1, uu, ud, n_elec, n_up, device="cuda", stream=None):
        import torch

        self._torch = torch
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        ions = np.ascontiguousarray(ions, dtype=np.float64).reshape(-1, 3)
        species = np.ascontiguousarray(species, dtype=np.int32).reshape(-1)
        funs = list(f1) + [uu, ud]
        self.n_elec, self.n_up, self.n_ion = int(n_elec), int(n_up), ions.shape[0]
        self.desc = JastrowDesc(self.n_elec, self.n_up, self.n_ion, len(f1), (ctypes.c_double * 3)(*cell))
        iv = np.array([len(c) - 3 for c, _ in funs], dtype=np.int32)
        rc = np.array([float(r) for _, r in funs], dtype=np.float64)
        cf = np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.float64) for c, _ in funs]))
        L = lib()
        nb = L.jastrow_bytes(ctypes.byref(self.desc), iv.ctypes.data)
        if nb == 0:
            raise SplineError(-1, "invalid Jastrow sizes or cell")
        self.buf = torch.empty(nb, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            sp, _ = _stream_ptr(torch, self.device, stream)
            check(L.jastrow_create(ctypes.byref(self.desc), ions.ctypes.data if self.n_ion else None,
                                   species.ctypes.data if self.n_ion else None, iv.ctypes.data, rc.ctypes.data,
                                   cf.ctypes.data, ctypes.c_void_p(self.buf.data_ptr()), nb, sp, ctypes.byref(h)))
        self._h = h
        self.ld = (self.n_elec + 63) // 64 * 64

    def positions(self, R):
        """[W, N, 3] array -> float32 [W, 3, ld] device tensor (padding zero)."""
        R = np.asarray(R, dtype=np.float64)
        out = np.zeros((R.shape[0], 3, self.ld), dtype=np.float32)
        out[:, :, :self.n_elec] = np.transpose(R, (0, 2, 1))
        return self._torch.from_numpy(out).to(self.device)

    def _R(self, R):
        t = self._torch
        if not (isinstance(R, t.Tensor) and R.dtype == t.float32 and R.device == self.device and R.dim() == 3
                and R.shape[1] == 3 and R.shape[2] >= self.n_elec and R.is_contiguous()):
            raise ValueError("R must be a contiguous float32 [W, 3, >=n_elec] tensor on %s" % self.device)
        return R, R.shape[2], 3 * R.shape[2]

    def _slots(self, R, k, r, walkers):
        t = self._torch
        count = k.shape[0]
        if not (isinstance(k, t.Tensor) and k.dtype == t.int32 and k.device == self.device and k.is_contiguous()):
            raise ValueError("k must be a contiguous int32 tensor on %s" % self.device)
        if not (isinstance(r, t.Tensor) and r.dtype == t.float64 and r.device == self.device and r.is_contiguous()
                and tuple(r.shape) == (count, 3)):
            raise ValueError("positions must be a contiguous float64 [count, 3] tensor on %s" % self.device)
        if walkers is not None:
            if not (isinstance(walkers, t.Tensor) and walkers.dtype == t.int32 and walkers.device == self.device
                    and walkers.is_contiguous() and tuple(walkers.shape) == (count,)):
                raise ValueError("walkers must be a contiguous int32 [count] tensor on %s" % self.device)
            if count and (int(walkers.min().item()) < 0 or int(walkers.max().item()) >= R.shape[0]):
                raise ValueError("walker index out of range")
        elif count > R.shape[0]:
            raise ValueError("more slots than walkers")
        return count

    @staticmethod
    def _p(x):
        return ctypes.c_void_p(x.data_ptr()) if x is not None else None

    def move(self, R, k, rnew, walkers=None, out=None, stream=None):
        """[count, 5] float32: Delta J, grad_k J (x, y, z), lap_k J for moving
        electron k[s] of walker walkers[s] (or s) to rnew[s]."""
        t = self._torch
        R, ld, ws = self._R(R)
        count = self._slots(R, k, rnew, walkers)
        out = (_need(out, t.float32, (count, 5), self.device, "out") if out is not None
               else t.empty((count, 5), dtype=t.float32, device=self.device))
        with t.cuda.device(self.device):
            sp, _ = _stream_ptr(t, self.device, stream)
            check(lib().jastrow_move(self._h, self._p(R), ld, ws, self._p(walkers), self._p(k), self._p(rnew), count,
                                     self._p(out), sp))
        return out

    def evaluate(self, R, out=None, stream=None):
        """(J [W], G [W, 3, N], L [W, N]) float32."""
        t = self._torch
        R, ld, ws = self._R(R)
        W_ = R.shape[0]
        kw = dict(dtype=t.float32, device=self.device)
        if out is not None:
            J, G, L = out
            J = _need(J, t.float32, (W_,), self.device, "J")
            G = _need(G, t.float32, (W_, 3, self.n_elec), self.device, "G")
            L = _need(L, t.float32, (W_, self.n_elec), self.device, "L")
        else:
            J, G, L = t.empty(W_, **kw), t.empty((W_, 3, self.n_elec), **kw), t.empty((W_, self.n_elec), **kw)
        with t.cuda.device(self.device):
            sp, _ = _stream_ptr(t, self.device, stream)
            check(lib().jastrow_evaluate(self._h, self._p(R), ld, ws, W_, self._p(J), self._p(G), self._p(L), sp))
        return J, G, L

    def dist_rows(self, R, r, walkers=None, stream=None):
        """(de [c, N], dre [c, 3, N], di [c, n_ion], dri [c, 3, n_ion]) with
        dr = r_other - r (minimum image)."""
        t = self._torch
        R, ld, ws = self._R(R)
        dummy_k = t.zeros(r.shape[0], dtype=t.int32, device=self.device)
        count = self._slots(R, dummy_k, r, walkers)
        kw = dict(dtype=t.float32, device=self.device)
        de, dre = t.empty((count, self.n_elec), **kw), t.empty((count, 3, self.n_elec), **kw)
        di, dri = t.empty((count, self.n_ion), **kw), t.empty((count, 3, self.n_ion), **kw)
        with t.cuda.device(self.device):
            sp, _ = _stream_ptr(t, self.device, stream)
            check(lib().jastrow_dist_rows(self._h, self._p(R), ld, ws, self._p(walkers), self._p(r), count,
                                          self._p(de), self._p(dre), self._p(di) if self.n_ion else None,
                                          self._p(dri) if self.n_ion else None, sp))
        return de, dre, di, dri

    def accept(self, R, k, rnew, walkers=None, stream=None):
        t = self._torch
        R, ld, ws = self._R(R)
        count = self._slots(R, k, rnew, walkers)
        with t.cuda.device(self.device):
            sp, _ = _stream_ptr(t, self.device, stream)
            check(lib().jastrow_accept(self._h, self._p(R), ld, ws, self._p(walkers), self._p(k), self._p(rnew),
                                       count, sp))
        return R

    def close(self):
        if getattr(self, "_h", None):
            lib().jastrow_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DelayedUpdate:
    """Delayed (Woodbury) updates of float32 inverses ainv[W, n, n] with at
    most `delay` pending moves per walker (include/qmcspline.h,
    spline_dlu_*)."""

    def __init__(self, n: int, delay: int, walkers: int, device="cuda", stream=None):
        import torch

        self._torch = torch
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.n, self.delay, self.walkers = int(n), int(delay), int(walkers)
        L = lib()
        nb = L.spline_dlu_workspace_bytes(self.n, self.delay, self.walkers)
        if nb == 0:
            raise SplineError(-1, "need 1 <= n <= 2048, 1 <= delay <= min(64, n), walkers >= 1")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            sp, _ = _stream_ptr(torch, self.device, stream)
            check(L.spline_dlu_create(self.n, self.delay, self.walkers, ctypes.c_void_p(self.ws.data_ptr()), nb, sp,
                                      ctypes.byref(h)))
        self._h = h

    def _ainv(self, ainv):
        t = self._torch
        if not (isinstance(ainv, t.Tensor) and ainv.dtype == t.float32 and ainv.device == self.device
                and ainv.dim() == 3 and tuple(ainv.shape[1:]) == (self.n, self.n) and ainv.is_contiguous()
                and ainv.shape[0] >= self.walkers):
            raise ValueError("ainv must be a contiguous float32 [>=walkers, n, n] tensor on %s" % self.device)
        return ctypes.c_void_p(ainv.data_ptr())

    def _slots(self, k, V, walkers):
        t = self._torch
        if not (isinstance(k, t.Tensor) and k.dim() == 1):
            raise ValueError("k must be a contiguous int32 [count] tensor")
        count = k.shape[0]
        _need(k, t.int32, (count,), self.device, "k")
        _need(V, t.float32, (count, self.n), self.device, "V")
        if walkers is not None:
            _need(walkers, t.int32, (count,), self.device, "walkers")
            # indices are range-checked by the kernels (NaN ratio, skipped accept): no host sync here
        elif count > self.walkers:
            raise ValueError("more slots than walkers")
        return count

    def _ratio_args(self, count, G, L, out):
        """The optional derivative rows and the [count, 5] / [count] output."""
        t = self._torch
        if (G is None) != (L is None):
            raise ValueError("give both G and L, or neither")
        if G is not None:
            _need(G, t.float32, (count, 3, self.n), self.device, "G")
            _need(L, t.float32, (count, self.n), self.device, "L")
        shape = (count, 5) if G is not None else (count,)
        if out is None:
            return t.empty(shape, dtype=t.float32, device=self.device)
        return _need(out, t.float32, shape, self.device, "out")

    @staticmethod
    def _p(x):
        return ctypes.c_void_p(x.data_ptr()) if x is not None else None

    def ratio(self, ainv, k, V, G=None, L=None, walkers=None, out=None, stream=None):
        t = self._torch
        count = self._slots(k, V, walkers)
        out = self._ratio_args(count, G, L, out)
        with t.cuda.device(self.device):
            sp, _ = _stream_ptr(t, self.device, stream)
            check(lib().spline_dlu_ratio(self._h, self._ainv(ainv), self.n * self.n, self._p(walkers), self._p(k),
                                         self._p(V), self._p(G), self._p(L), count, self._p(out), sp))
        return out

    def accept(self, ainv, k, V, walkers=None, stream=None):
        t = self._torch
        count = self._slots(k, V, walkers)
        with t.cuda.device(self.device):
            sp, _ = _stream_ptr(t, self.device, stream)
            check(lib().spline_dlu_accept(self._h, self._ainv(ainv), self.n * self.n, self._p(walkers), self._p(k),
                                          self._p(V), count, sp))

    def accept_ratio(self, ainv, k_acc, V_acc, k, V, G=None, L=None, walkers=None, out=None, stream=None):
        """accept(ainv, k_acc, V_acc) then ratio(ainv, k, V, G, L) in one launch
        (bit-identical to the two calls)."""
        t = self._torch
        count = self._slots(k, V, walkers)
        if self._slots(k_acc, V_acc, walkers) != count:
            raise ValueError("accepted and proposed slots differ in count")
        out = self._ratio_args(count, G, L, out)
        with t.cuda.device(self.device):
            sp, _ = _stream_ptr(t, self.device, stream)
            check(lib().spline_dlu_accept_ratio(self._h, self._ainv(ainv), self.n * self.n, self._p(walkers),
                                                self._p(k_acc), self._p(V_acc), self._p(k), self._p(V), self._p(G),
                                                self._p(L), count, self._p(out), sp))
        return out

    def flush(self, ainv, stream=None):
        t = self._torch
        with t.cuda.device(self.device):
            sp, _ = _stream_ptr(t, self.device, stream)
            check(lib().spline_dlu_flush(self._h, self._ainv(ainv), self.n * self.n, sp))
        return ainv

    def close(self):
        if getattr(self, "_h", None):
            lib().spline_dlu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
