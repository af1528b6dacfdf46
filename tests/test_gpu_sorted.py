"""Locality-ordered evaluation (spline_eval_vgl_sorted / spline_eval_v_sorted)
must give exactly the results of the plain entry points: the same
per-position arithmetic, only in another order.  Outputs are pre-filled with
NaN, so a position the sort dropped would show.  The small case is also
checked against the FP64 oracle; the full-size case runs the 80^3 / N=384
table on the 512 x 384 batch in the launch configuration the bench times.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def q(torch):
    import paper_1708_02645_amd as qq
    qq.lib()
    return qq


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _nan_outputs(torch, s, B):
    V, G, L = s.alloc_outputs(B)
    for t in (V, G, L):
        t.fill_(float("nan"))
    return V, G, L


def _same(torch, a, b):
    for x, y in zip(a, b):
        assert torch.equal(x, y) or bool(((x == y) | (torch.isnan(x) & torch.isnan(y))).all())


def _check_equal(torch, s, pos_np):
    pos = torch.from_numpy(pos_np).cuda()
    B = pos.shape[0]
    ref = s.eval_vgl(pos)
    got = s.eval_vgl_sorted(pos, out=_nan_outputs(torch, s, B))
    _same(torch, got, ref)
    v_ref = s.eval_v(pos)
    v = torch.full_like(v_ref, float("nan"))
    s.eval_v_sorted(pos, out=v)
    _same(torch, (v,), (v_ref,))
    return got


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_small_table_equal_and_against_oracle(torch, q, oracle, dtype):
    grid, N, coefs, _ = W.make_table(1)  # 16^3, 32 orbitals
    s = q.Spline(grid, coefs, dtype)
    pos = W.make_positions(1)  # 1000 positions
    _say("case sorted small", dtype)
    V, G, L = _check_equal(torch, s, pos)
    deq = coefs if dtype == "f64" else oracle.dequantize(coefs, dtype)[0]
    ref = oracle.eval_vgl(grid, deq, pos)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for name, a, b in zip("VGL", (V, G, L), ref):
        e = oracle.rel_err(a.cpu().numpy(), b)
        assert e <= tol, "%s %s: %.3e" % (dtype, name, e)


def test_edges(torch, q):
    rng = np.random.default_rng(3)
    grid = (7, 9, 11)
    coefs = rng.uniform(-1, 1, grid + (40,))
    s = q.Spline(grid, coefs, "f32", cell=(1.3, 0.7, 2.1))
    for B in (1, 17, 300):
        _say("case sorted edge B", B)
        pos = rng.uniform(-40, 40, (B, 3))  # far outside the cell: periodic wrap
        if B == 300:
            pos[5] = np.nan
            pos[6, 1] = np.inf
        _check_equal(torch, s, pos)
    # degenerate grids: one point (every position in cell 0), a flat grid
    for g_small, cell in (((1, 1, 1), (1.0, 1.0, 1.0)), ((2, 3, 1), (0.5, 1.0, 2.0))):
        s1 = q.Spline(g_small, rng.uniform(-1, 1, g_small + (24,)), "f32", cell=cell)
        _say("case sorted grid", g_small)
        _check_equal(torch, s1, rng.uniform(-3, 3, (257, 3)))
        s1.close()
    # B == 0 is a no-op; a short workspace is refused, and the value-only form refuses a general cell
    e = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    s.eval_vgl_sorted(e)
    pos = torch.from_numpy(rng.random((64, 3))).cuda()
    with pytest.raises(ValueError):
        s.eval_vgl_sorted(pos, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    L = q.lib()
    assert L.spline_sorted_workspace_bytes(None, 10) == 0
    assert L.spline_sorted_workspace_bytes(s._h, -1) == 0
    assert L.spline_sorted_workspace_bytes(s._h, 10) % 256 == 0
    s.set_lattice([[1.3, 0, 0], [0.2, 0.7, 0], [0, 0, 2.1]])
    with pytest.raises(q.SplineError):
        s.eval_v_sorted(pos)  # value only: orthorhombic cells
    # the ratio with derivatives serves general cells (parity in test_gpu_vgh)
    D = s.eval_ratio_vgl_sorted(pos, torch.zeros((64, 40), dtype=torch.float32, device="cuda"))
    assert tuple(D.shape) == (64, 5) and bool((D == 0).all())


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_vgh_and_general_cells_equal(torch, q, oracle, dtype):
    """VGH (orthorhombic and a triclinic cell) and the general-cell VGL in
    locality order equal the plain entry points bit for bit; the triclinic
    VGH is also checked against the FP64 oracle."""
    rng = np.random.default_rng(13)
    grid = (10, 12, 9)
    coefs = rng.uniform(-1, 1, grid + (48,))
    s = q.Spline(grid, coefs, dtype)
    lat = np.array([[1.0, 0.0, 0.0], [0.3, 0.9, 0.0], [-0.2, 0.1, 1.2]])
    for general in (False, True):
        if general:
            s.set_lattice(lat)
        for B in (1, 700, 3001):
            _say("case sorted vgh", dtype, general, B)
            pos_np = rng.uniform(-2, 2, (B, 3))
            pos = torch.from_numpy(pos_np).cuda()
            ref = s.eval_vgh(pos)
            got = s.eval_vgh_sorted(pos)
            _same(torch, got, ref)
            st = s.get_sorted_vgh_tile()
            assert st[2] in (16, s.get_vgh_tile()[2]) and 1 <= st[3] <= 8, st
            if general:
                _same(torch, s.eval_vgl_sorted(pos), s.eval_vgl(pos))
    deq = coefs if dtype == "f64" else oracle.dequantize(coefs, dtype)[0]
    ref = oracle.eval_vgh(grid, deq, pos_np[:200], lat)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for name, a, b in zip(("V", "G", "H"), got, ref):
        e = oracle.rel_err(a[:200].cpu().numpy(), b)
        assert e <= tol, "%s %s: %.3e" % (dtype, name, e)


def test_tiles_and_chunk_dealing(torch, q):
    """The index list deals whole chunks of pb sorted slots to the XCDs;
    every tile (pb 8, 16, 32, 64) and batch size (no whole chunk, a partial last
    chunk, chunk counts that do and do not divide by 8) must still cover each
    position exactly once."""
    rng = np.random.default_rng(11)
    grid = (12, 10, 9)
    s = q.Spline(grid, rng.uniform(-1, 1, grid + (64,)), "f32")
    seen = {}
    for t in s.tile_candidates():
        seen.setdefault(t[3], t)
    assert len(seen) >= 2
    t16 = seen[16]
    seen[8] = (t16[0], t16[1], t16[2], 8)  # the sorted autotuner's extra chunk length
    for pb, t in sorted(seen.items()):
        s.set_sorted_tile(t)
        assert tuple(s.get_sorted_tile()) == tuple(t)
        for B in (5, 1000, 16 * 8 * 3, 4099):
            _say("case sorted tile", t, "B", B)
            _check_equal(torch, s, rng.random((B, 3)))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_full_size_equal(torch, q, dtype):
    """80^3 grid, 384 orbitals, 196,608 positions (the bench's batch)."""
    grid, N, coefs, _ = W.make_table(3)
    s = q.Spline(grid, coefs, dtype)
    del coefs
    pos = W.make_positions(3)
    import os
    cache = os.path.join(os.path.dirname(q.__file__), "tune_cache.txt")
    s.autotune(torch.from_numpy(pos).cuda(), reps=2, cache_path=cache)  # the bench's tile (cached)
    _say("case sorted full", dtype, pos.shape, s.get_tile())
    _check_equal(torch, s, pos)
    t = s.autotune_sorted(torch.from_numpy(pos).cuda(), reps=1)  # no cache: searches, cross-checks bitwise
    _say("case sorted full tuned", dtype, t, s.get_sorted_value_tile())
    _check_equal(torch, s, pos)
    t = s.autotune_sorted(torch.from_numpy(pos).cuda(), reps=1, cache_path=cache)  # the bench's shapes
    _say("case sorted full, bench shapes", dtype, t, s.get_sorted_value_tile())
    _check_equal(torch, s, pos)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_ratio_small_equal(torch, q, dtype):
    """Determinant ratio in locality order equals the plain entry points bit
    for bit: rows of stacked inverses (no row list), and a row list with
    repeated rows (quadrature points sharing an electron)."""
    grid, N, coefs, _ = W.make_table(1)
    s = q.Spline(grid, coefs, dtype)
    rng = np.random.default_rng(21)
    B = 1000
    pos = torch.from_numpy(W.make_positions(1)).cuda()
    ainv = torch.from_numpy(rng.normal(size=(B, N)) / np.sqrt(N)).to(s.out_dtype).cuda()
    rows = torch.from_numpy(rng.integers(0, B, B).astype(np.int32)).cuda()
    t = s.get_tile()
    s.set_tile(t)  # the ratio's sums follow the tile shape: compare under one shape (VGL and value)
    s.set_sorted_tile(t)
    assert s.get_value_tile() == s.get_sorted_value_tile() == tuple(t)
    for r in (None, rows):
        _say("case sorted ratio", dtype, r is None)
        _same(torch, (s.eval_ratio_vgl_sorted(pos, ainv, rows=r),), (s.eval_ratio_vgl(pos, ainv, rows=r),))
        _same(torch, (s.eval_ratio_v_sorted(pos, ainv, rows=r),), (s.eval_ratio_v(pos, ainv, rows=r),))
    # 8 positions per workgroup (the sums do not depend on it, only on the shape)
    s.set_sorted_tile((t[0], t[1], t[2], 8))
    _same(torch, (s.eval_ratio_vgl_sorted(pos, ainv, rows=rows),), (s.eval_ratio_vgl(pos, ainv, rows=rows),))
    _same(torch, (s.eval_ratio_v_sorted(pos, ainv),), (s.eval_ratio_v(pos, ainv),))


def test_ratio_full_size_equal(torch, q):
    """80^3 / N=384 / 196,608 positions, rows of the 512 stacked 384 x 384
    inverses (the bench's fused-ratio workload)."""
    grid, N, coefs, _ = W.make_table(3)
    s = q.Spline(grid, coefs, "f32")
    del coefs
    pos_np = W.make_positions(3)
    pos = torch.from_numpy(pos_np).cuda()
    import os
    s.autotune(pos, reps=2, cache_path=os.path.join(os.path.dirname(q.__file__), "tune_cache.txt"))
    ainv = torch.from_numpy(W.make_inverse_rows(3, pos_np.shape[0], N)).cuda()
    st = s.autotune_sorted(pos, reps=1, cache_path=os.path.join(os.path.dirname(q.__file__), "tune_cache.txt"))
    sv = s.get_sorted_value_tile()
    _say("case sorted ratio full", st, sv)
    D = s.eval_ratio_vgl_sorted(pos, ainv)
    R = s.eval_ratio_v_sorted(pos, ainv)
    s.set_tile(sv)  # the plain value path under the sorted value shape
    _same(torch, (R,), (s.eval_ratio_v(pos, ainv),))
    s.set_tile(st)  # the plain path under the sorted shape
    _same(torch, (D,), (s.eval_ratio_vgl(pos, ainv),))
