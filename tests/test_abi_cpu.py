"""CPU-side checks of the C ABI: exported symbols, layout arithmetic,
argument validation, and the host packing (halo layout + quantization),
which is integer/byte work and must match the oracle's dequantized table
bit for bit.  No GPU call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1708_02645_amd as q
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in ("qmcspline.h", "qmcjastrow.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b((?:spline|jastrow)_\w+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_header_symbol():
    names = header_functions()
    assert len(names) >= 12
    L = q.lib()
    for n in names:
        assert hasattr(L, n), n


def test_layout_and_sizes():
    L = q.get_layout((80, 80, 80), 384, "f32")
    assert L.row_bytes == 1536 and L.n_pad == 384
    assert L.table_bytes == 83 ** 3 * 1536
    assert L.total_bytes == L.table_bytes + 1536  # 384 float scales, already 256-aligned
    assert tuple(L.padded) == (83, 83, 83)
    L = q.get_layout((16, 16, 16), 32, "f64")
    assert L.row_bytes == 256 and L.n_pad == 32
    L = q.get_layout((5, 6, 7), 37, "bf16")
    assert L.row_bytes == 128 and L.n_pad == 64
    assert q.table_bytes((5, 6, 7), 37, "bf16") == L.total_bytes
    # rows of at most 256 B pad to 64 B (128 B for FP64), longer rows to 256 B;
    # the scales start on a 256-byte boundary after the table
    for grid, n, dt, row in (((80, 80, 80), 48, "f32", 192), ((8, 8, 8), 40, "f32", 192),
                             ((8, 8, 8), 24, "f32", 128), ((8, 8, 8), 16, "f32", 64),
                             ((8, 8, 8), 24, "f64", 256), ((8, 8, 8), 8, "f64", 128),
                             ((8, 8, 8), 100, "f32", 512), ((8, 8, 8), 96, "f16", 192),
                             ((8, 8, 8), 130, "bf16", 512)):
        L = q.get_layout(grid, n, dt)
        assert L.row_bytes == row, (grid, n, dt, L.row_bytes)
        assert L.n_pad * L.elem_bytes == row
        assert L.table_bytes == (grid[0] + 3) * (grid[1] + 3) * (grid[2] + 3) * row
        assert L.scales_offset % 256 == 0 and 0 <= L.scales_offset - L.table_bytes < 256
        assert L.total_bytes == L.scales_offset + (4 * L.n_pad + 255) // 256 * 256


@pytest.mark.parametrize("args", [
    ((0, 4, 4), 4, "f32", (1, 1, 1)),
    ((4, 4, 4), 0, "f32", (1, 1, 1)),
    ((4, 4, 4), 4, "f32", (1, 0, 1)),
    ((4, 4, 4), 4, "f32", (1, float("inf"), 1)),
    ((4, 4, 4), 4, "f32", (1, float("nan"), 1)),
    ((1 << 20, 1 << 20, 1 << 20), 1 << 30, "f64", (1, 1, 1)),  # overflow
])
def test_invalid_sizes_return_zero_bytes(args):
    grid, n, dt, cell = args
    assert q.table_bytes(grid, n, dt, cell) == 0
    with pytest.raises(q.SplineError) as e:
        q.get_layout(grid, n, dt, cell)
    assert e.value.code in (-1, -2)
    assert q.last_error()


def test_null_and_bad_arguments():
    L = q.lib()
    g = q.make_grid((4, 4, 4))
    h = ctypes.c_void_p()
    c = np.zeros((4, 4, 4, 2))
    assert L.spline_create(None, 2, c.ctypes.data, 1, None, 0, None, ctypes.byref(h)) == -1
    assert L.spline_create(ctypes.byref(g), 2, None, 1, None, 0, None, ctypes.byref(h)) == -1
    assert "NULL" in q.last_error() or "null" in q.last_error().lower()
    assert L.spline_create(ctypes.byref(g), 2, c.ctypes.data, 7, None, 0, None, ctypes.byref(h)) == -1
    assert L.spline_create(ctypes.byref(g), 2, c.ctypes.data, 1, ctypes.c_void_p(256), 16, None,
                           ctypes.byref(h)) == -2  # buffer too small
    assert L.spline_create(ctypes.byref(g), 2, c.ctypes.data, 1, ctypes.c_void_p(260), 1 << 20, None,
                           ctypes.byref(h)) == -1  # misaligned
    assert L.spline_create(ctypes.byref(g), 2, c.ctypes.data, 1, None, 0, None, None) == -1
    assert L.spline_eval_vgl(None, None, 0, None, None, None, None) == -1
    assert L.spline_destroy(None) == 0
    assert L.spline_get_tile(None, None) == -1
    assert L.spline_autotune(None, None, 0, None, None, None, 1, None, None, None) == -1


def test_pack_rejects_nonfinite():
    c = np.zeros((3, 3, 3, 2))
    c[1, 1, 1, 1] = np.nan
    for dt in ("f64", "f32", "bf16", "f16"):
        with pytest.raises(q.SplineError):
            q.pack_host((3, 3, 3), c, dt)


def _unpack(buf, grid, norb, dtype):
    """Decode the halo table and scales of a packed buffer (numpy only)."""
    L = q.get_layout(grid, norb, dtype)
    P = tuple(L.padded)
    rows = np.frombuffer(buf[:L.table_bytes].tobytes(), dtype=np.uint8).reshape(P + (L.row_bytes,))
    sc = np.frombuffer(buf[L.scales_offset:L.scales_offset + 4 * L.n_pad].tobytes(), dtype=np.float32)
    if dtype == "f64":
        vals = rows.view(np.float64)
    elif dtype == "f32":
        vals = rows.view(np.float32).astype(np.float64)
    elif dtype == "f16":
        vals = rows.view(np.float16).astype(np.float64)
    else:
        u = rows.view(np.uint16).astype(np.uint32) << 16
        vals = u.view(np.float32).astype(np.float64)
    return vals, sc.astype(np.float64), L


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_pack_matches_oracle_dequantized_bitwise(oracle, dtype):
    rng = np.random.default_rng(21)
    grid, norb = (5, 3, 6), 37
    c = rng.standard_normal(grid + (norb,)) * np.exp(rng.uniform(-12, 6, norb))
    c[..., 5] = 0.0                  # all-zero orbital -> scale 1
    c[..., 6] *= 1e-3                # includes FP16 subnormals after scaling
    c[0, 0, 0, 6] = 1.0
    buf = q.pack_host(grid, c, dtype)
    vals, sc, L = _unpack(buf, grid, norb, dtype)
    dq, s_or = oracle.dequantize(c, dtype)
    np.testing.assert_array_equal(sc[:norb], s_or)
    assert (sc[norb:] == 1.0).all()
    n = np.array(grid)
    for p0 in range(grid[0] + 3):
        for p1 in range(grid[1] + 3):
            for p2 in range(grid[2] + 3):
                j = ((p0 - 1) % n[0], (p1 - 1) % n[1], (p2 - 1) % n[2])
                got = vals[p0, p1, p2, :norb] * sc[:norb]
                np.testing.assert_array_equal(got, dq[j])
                assert (vals[p0, p1, p2, norb:] == 0).all()


def test_pack_f16_ties_and_extremes(oracle):
    """Values at exact rounding ties and at the FP16 subnormal edge."""
    c = np.zeros((1, 1, 1, 4))
    c[0, 0, 0, 0] = 1.0                         # scale 1
    c[0, 0, 0, 1] = 1.0 + 2.0 ** -11            # tie -> even (1.0), scale 2 -> 0.5+2^-12: tie too
    c[0, 0, 0, 2] = -(2.0 ** -25) * 3           # below half of the smallest subnormal after scale
    c[0, 0, 0, 3] = 2.0 ** -14 + 2.0 ** -25     # near the normal/subnormal boundary
    for dt in ("f16", "bf16"):
        buf = q.pack_host((1, 1, 1), c, dt)
        vals, sc, L = _unpack(buf, (1, 1, 1), 4, dt)
        dq, _ = oracle.dequantize(c, dt)
        np.testing.assert_array_equal(vals[1, 1, 1, :4] * sc[:4], dq[0, 0, 0])


def test_ratio_entry_points_reject_bad_arguments_without_a_gpu():
    """Argument checks of the determinant-ratio calls run before any HIP call."""
    L = q.lib()
    for fn in (L.spline_eval_ratio_vgl, L.spline_eval_ratio_v):
        assert fn(None, None, 4, None, 4, None, None, None) == -1
        assert "handle" in q.last_error()


def test_det_update_rejects_bad_arguments_without_a_gpu():
    L = q.lib()
    assert L.spline_det_update(None, 4, 16, None, None, None, 4, 0, 1, None) == 0  # empty: no-op
    assert L.spline_det_update(None, 4, 16, None, None, None, 4, 1, 1, None) == -1
    assert L.spline_det_update(None, 4, 16, None, None, None, 4, -1, 1, None) == -1


def test_jastrow_sizes_and_argument_checks_without_a_gpu():
    import ctypes

    L = q.lib()
    d = q.JastrowDesc(384, 192, 32, 2, (ctypes.c_double * 3)(1.0, 1.0, 1.0))
    iv = np.array([8, 8, 8, 8], dtype=np.int32)
    nb = L.jastrow_bytes(ctypes.byref(d), iv.ctypes.data)
    assert nb > 0 and nb % 256 == 0
    bad = q.JastrowDesc(384, 400, 32, 2, (ctypes.c_double * 3)(1.0, 1.0, 1.0))  # n_up > n_elec
    assert L.jastrow_bytes(ctypes.byref(bad), iv.ctypes.data) == 0
    iv0 = np.array([8, 0, 8, 8], dtype=np.int32)
    assert L.jastrow_bytes(ctypes.byref(d), iv0.ctypes.data) == 0
    for fn, args in ((L.jastrow_move, (None, None, 384, 3 * 384, None, None, None, 1, None, None)),
                     (L.jastrow_evaluate, (None, None, 384, 3 * 384, 1, None, None, None, None)),
                     (L.jastrow_accept, (None, None, 384, 3 * 384, None, None, None, 1, None))):
        assert fn(*args) == -1 and "handle" in q.last_error()


def test_delayed_update_sizes_without_a_gpu():
    L = q.lib()
    assert L.spline_dlu_workspace_bytes(384, 16, 512) % 256 == 0
    assert L.spline_dlu_workspace_bytes(0, 16, 512) == 0
    assert L.spline_dlu_workspace_bytes(384, 0, 512) == 0
    assert L.spline_dlu_workspace_bytes(8, 9, 512) == 0
    assert L.spline_dlu_ratio(None, None, 64, None, None, None, None, None, 1, None, None) == -1


def test_sorted_plan_workspace_holds_eight_position_tasks():
    """A locality-ordered plan may run 8-position tasks (16-byte task
    records), a plain plan 16-position ones; the sorted plan's workspace also
    holds each table's sort workspace (32768 bucket counts and three int32
    per position).  Its size must cover all of that, or the task list spills
    into the sort workspace that follows it."""
    L = q.lib()
    for Bs in ((196608,), (64, 1000, 4099), (7,)):
        arr = (ctypes.c_int64 * len(Bs))(*Bs)
        plain = L.spline_plan_workspace_bytes(len(Bs), arr)
        srt = L.spline_plan_workspace_bytes_sorted(len(Bs), arr)
        tasks8 = sum((b + 7) // 8 for b in Bs) * 16
        tasks16 = sum((b + 15) // 16 for b in Bs) * 16
        sort_ws = sum(4 * (32768 + 3 * b) for b in Bs)
        assert srt >= plain - tasks16 + tasks8 + sort_ws, (Bs, plain, srt)
