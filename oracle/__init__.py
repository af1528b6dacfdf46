"""FP64 CPU oracle (test infrastructure only).

The tests, the smoke check and the benchmark's CPU-baseline leg are the only
users of this package.  It shares no code with the GPU library: the C part
(``oracle.c``) is compiled on its own with gcc, and the Python part here only
marshals numpy arrays.  Inputs come from :mod:`workloads`.

Parity status of each function is listed in the module docstrings of the
parts; every function here is pinned by ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FMT = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        d, i32, i64, p = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.oracle_basis.argtypes = [d, p, p, p]
        L.oracle_basis.restype = None
        L.oracle_reduce.argtypes = [d, d, i32, p, p]
        L.oracle_reduce.restype = None
        L.oracle_eval_vgl.argtypes = [p, p, i32, p, i64, p, p, p, p, i32]
        L.oracle_eval_vgl.restype = ctypes.c_int
        L.oracle_eval_v.argtypes = [p, p, i32, p, i64, p, p, i32]
        L.oracle_eval_v.restype = ctypes.c_int
        L.oracle_eval_vgh.argtypes = [p, p, i32, p, i64, p, p, p, p, i32]
        L.oracle_eval_vgh.restype = ctypes.c_int
        L.oracle_round_sig.argtypes = [d, i32, i32]
        L.oracle_round_sig.restype = d
        L.oracle_dequantize.argtypes = [p, i64, i32, i32, p, p]
        L.oracle_dequantize.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def basis(t: float):
    """(b[4], db[4], d2b[4]) of the uniform cubic B-spline at offset t."""
    b, db, d2b = (np.zeros(4) for _ in range(3))
    lib().oracle_basis(float(t), _ptr(b), _ptr(db), _ptr(d2b))
    return b, db, d2b


def reduce(r: float, cell: float, n: int):
    """(cell index, fractional offset) of one coordinate."""
    i = np.zeros(1, np.int32)
    t = np.zeros(1)
    lib().oracle_reduce(float(r), float(cell), int(n), _ptr(i), _ptr(t))
    return int(i[0]), float(t[0])


def _grid_args(grid, cell):
    n = np.ascontiguousarray(grid, dtype=np.int32)
    c = np.ascontiguousarray(cell, dtype=np.float64)
    return n, c


def eval_vgl(grid, coefs: np.ndarray, pos: np.ndarray, cell=(1.0, 1.0, 1.0), threads: int = 0):
    """V[B,N], G[B,3,N], L[B,N] in FP64 from coefs[n0,n1,n2,N] at pos[B,3]."""
    coefs = np.ascontiguousarray(coefs, dtype=np.float64)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n, c = _grid_args(grid, cell)
    N = coefs.shape[-1]
    assert coefs.shape == tuple(int(x) for x in grid) + (N,)
    B = pos.shape[0]
    V = np.empty((B, N))
    G = np.empty((B, 3, N))
    L = np.empty((B, N))
    rc = lib().oracle_eval_vgl(_ptr(n), _ptr(c), N, _ptr(coefs), B, _ptr(pos), _ptr(V), _ptr(G), _ptr(L), threads)
    if rc != 0:
        raise ValueError("oracle_eval_vgl: bad arguments")
    return V, G, L


def eval_v(grid, coefs: np.ndarray, pos: np.ndarray, cell=(1.0, 1.0, 1.0), threads: int = 0):
    """V[B,N] in FP64 (value only)."""
    coefs = np.ascontiguousarray(coefs, dtype=np.float64)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n, c = _grid_args(grid, cell)
    N = coefs.shape[-1]
    B = pos.shape[0]
    V = np.empty((B, N))
    rc = lib().oracle_eval_v(_ptr(n), _ptr(c), N, _ptr(coefs), B, _ptr(pos), _ptr(V), threads)
    if rc != 0:
        raise ValueError("oracle_eval_v: bad arguments")
    return V


def eval_vgh(grid, coefs: np.ndarray, pos: np.ndarray, lattice, threads: int = 0):
    """V[B,N], G[B,3,N], H[B,6,N] (xx, xy, xz, yy, yz, zz) in FP64 for a
    general cell: lattice[3,3] has the Cartesian lattice vectors as rows, and
    grid axis d runs along lattice row d."""
    coefs = np.ascontiguousarray(coefs, dtype=np.float64)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n = np.ascontiguousarray(grid, dtype=np.int32)
    lat = np.ascontiguousarray(lattice, dtype=np.float64).reshape(9)
    N = coefs.shape[-1]
    assert coefs.shape == tuple(int(x) for x in grid) + (N,)
    B = pos.shape[0]
    V = np.empty((B, N))
    G = np.empty((B, 3, N))
    H = np.empty((B, 6, N))
    rc = lib().oracle_eval_vgh(_ptr(n), _ptr(lat), N, _ptr(coefs), B, _ptr(pos), _ptr(V), _ptr(G), _ptr(H), threads)
    if rc != 0:
        raise ValueError("oracle_eval_vgh: bad arguments or singular lattice")
    return V, G, H


def round_sig(x: float, p: int, emin: int) -> float:
    return float(lib().oracle_round_sig(float(x), int(p), int(emin)))


def dequantize(coefs: np.ndarray, fmt: str):
    """(s_m * q(c / s_m) as FP64 table, scales[N]) for storage format fmt."""
    coefs = np.ascontiguousarray(coefs, dtype=np.float64)
    N = coefs.shape[-1]
    out = np.empty_like(coefs)
    scales = np.empty(N)
    rc = lib().oracle_dequantize(_ptr(coefs), coefs.size // N, N, FMT[fmt], _ptr(out), _ptr(scales))
    if rc != 0:
        raise ValueError("oracle_dequantize: bad arguments")
    return out, scales


def rel_err(Q: np.ndarray, Qref: np.ndarray) -> float:
    """Per-orbital max-norm relative error, maximised over orbitals.

    Q and Qref have the orbital index last; all other axes (positions, and the
    three gradient components) are pooled.  An orbital whose reference is zero
    everywhere is measured in absolute terms.
    """
    Q = np.asarray(Q, dtype=np.float64)
    Qref = np.asarray(Qref, dtype=np.float64)
    N = Qref.shape[-1]
    if Qref.size == 0:
        return 0.0
    d = np.abs(Q - Qref).reshape(-1, N) if Q.shape == Qref.shape else None
    if d is None:
        raise ValueError("shape mismatch %s vs %s" % (Q.shape, Qref.shape))
    num = d.max(0)
    den = np.abs(Qref).reshape(-1, N).max(0)
    den = np.where(den > 0, den, 1.0)
    return float((num / den).max())  # NaN propagates, so a NaN fails any gate


def rel_rms(Q: np.ndarray, Qref: np.ndarray) -> float:
    """||Q - Qref||_2 / ||Qref||_2 over all entries."""
    Q = np.asarray(Q, dtype=np.float64)
    Qref = np.asarray(Qref, dtype=np.float64)
    den = np.linalg.norm(Qref)
    return float(np.linalg.norm(Q - Qref) / (den if den > 0 else 1.0))
