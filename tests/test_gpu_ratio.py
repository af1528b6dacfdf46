"""GPU parity of the fused determinant-ratio evaluation against the oracle.

Every call goes through the C ABI.  The kernel forms, per position b with
row a (a row of A^-1), D[b] = (sum a V, sum a Gx, sum a Gy, sum a Gz,
sum a L) without writing the orbital values.  Error measure, per position and
quantity q: |D - D_ref| / sum_i |a_i| M_iq, where M_iq is orbital i's largest
|Q_ref| over the batch (gradient components pooled): an error of e * M_iq in
every orbital value moves the dot product by at most e times that scale.
Bars: 1e-12 for FP64 tables; 1e-5 for FP32 accumulation (orbital error
<= 3e-6 on these tables, plus summation over at most (values per lane +
log2 lanes + tiles) terms in FP32, ~1e-6).  16-bit tables are compared with
the oracle on the dequantized coefficients.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE_CACHE = os.path.join(ROOT, "paper_1708_02645_amd", "tune_cache.txt")
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5, "f16": 1e-5}


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


def _table_ref(oracle, coefs, dtype):
    return oracle.dequantize(coefs, dtype)[0] if dtype in ("bf16", "f16") else coefs


def _ref(oracle, grid, coefs, pos, rows, cell=(1.0, 1.0, 1.0)):
    """(D_ref[B,5], scale[B,5]) from the oracle."""
    from oracle import det

    D = det.ratio_vgl(grid, coefs, pos, rows, cell)
    V, G, L = oracle.eval_vgl(grid, coefs, pos, cell)
    M = [np.abs(V).max(axis=0), np.abs(G).max(axis=(0, 1)), np.abs(L).max(axis=0)]
    sv, sg, sl = (det.ratio_scale(rows, m) for m in M)
    return D, np.stack([sv, sg, sg, sg, sl], axis=1)


def _err(D, Dref, scale):
    return float(np.max(np.abs(D - Dref) / np.maximum(scale, 1e-300))) if len(D) else 0.0


def _walker_system(oracle, grid, coefs, walkers, rng):
    """Actual inverses: per walker, A(i,j) = phi_i(r_j) from the oracle for
    norb electrons, inverted in FP64; proposals r'_k for every electron."""
    from oracle import det

    N = coefs.shape[-1]
    rows = np.empty((walkers * N, N))
    for w in range(walkers):
        A = det.slater_matrix(grid, coefs, rng.random((N, 3)))
        rows[w * N:(w + 1) * N] = np.linalg.inv(A)
    return rows, rng.random((walkers * N, 3))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_c1_walkers_with_actual_inverses(torch, q, oracle, dtype):
    grid, N, coefs, _ = W.make_table(1)
    rng = np.random.default_rng(31)
    ref_coefs = _table_ref(oracle, coefs, dtype)
    rows64, pos = _walker_system(oracle, grid, ref_coefs, 8, rng)
    rows = rows64 if dtype == "f64" else rows64.astype(np.float32)
    _say("case ratio c1", dtype, pos.shape)
    s = q.Spline(grid, coefs, dtype)
    pd = torch.from_numpy(pos).cuda()
    ad = torch.from_numpy(rows).cuda()
    D = s.eval_ratio_vgl(pd, ad).cpu().numpy()
    R = s.eval_ratio_v(pd, ad).cpu().numpy()
    Dref, scale = _ref(oracle, grid, ref_coefs, pos, rows)
    e = _err(D, Dref, scale)
    ev = _err(R[:, None], Dref[:, :1], scale[:, :1])
    _say("ratio c1 %s: err VGL %.2e, value-only %.2e" % (dtype, e, ev))
    assert e <= TOL[dtype] and ev <= TOL[dtype]
    # determinant ratios of order one: the rows are actual inverses
    assert np.median(np.abs(Dref[:, 0])) > 1e-3


@pytest.fixture(scope="module")
def c3():
    grid, N, coefs, _ = W.make_table(3)
    return grid, N, coefs


def test_c3_full_batch_sampled(torch, q, oracle, c3):
    """The full 80^3 x 384 FP32 batch (512 walkers x 384 electrons, row b of
    the stacked inverses for position b) in the tile shape the benchmark
    selects; the oracle checks a sample of positions."""
    grid, N, coefs = c3
    pos = W.make_positions(3)
    rows = W.make_inverse_rows(3, len(pos), N)
    _say("case ratio c3 f32 full batch", pos.shape)
    s = q.Spline(grid, coefs, "f32")
    pd = torch.from_numpy(pos).cuda()
    out = s.alloc_outputs(len(pos))
    s.autotune(pd, reps=3, out=out, cache_path=TUNE_CACHE)
    del out
    ad = torch.from_numpy(rows).cuda()
    D = s.eval_ratio_vgl(pd, ad)
    R = s.eval_ratio_v(pd, ad)
    idx = np.concatenate([np.random.default_rng(2).choice(len(pos), 384, replace=False), [0, len(pos) - 1]])
    it = torch.from_numpy(idx).cuda()
    Dg, Rg = D[it].cpu().numpy(), R[it].cpu().numpy()
    Dref, scale = _ref(oracle, grid, coefs, pos[idx], rows[idx])
    e, ev = _err(Dg, Dref, scale), _err(Rg[:, None], Dref[:, :1], scale[:, :1])
    _say("ratio c3 f32 tile %s: err VGL %.2e, value-only %.2e" % (s.get_tile(), e, ev))
    assert e <= TOL["f32"] and ev <= TOL["f32"]


def test_every_tile_shape(torch, q, oracle):
    """Every compiled tile shape (ragged batch over positions per workgroup)
    against the oracle, and bit-for-bit repeatable for a fixed shape."""
    grid, N, coefs, _ = W.make_table(2)
    pos = W.make_positions(2, count=1001)
    rows = W.make_inverse_rows(2, len(pos), N)
    pd, ad = torch.from_numpy(pos).cuda(), torch.from_numpy(rows).cuda()
    for dt in ("f32", "bf16"):
        ref_coefs = _table_ref(oracle, coefs, dt)
        Dref, scale = _ref(oracle, grid, ref_coefs, pos[:300], rows[:300])
        s = q.Spline(grid, coefs, dt)
        for t in s.tile_candidates():
            _say("case ratio tile", dt, t)
            s.set_tile(t)
            D1 = s.eval_ratio_vgl(pd, ad).cpu().numpy()
            D2 = s.eval_ratio_vgl(pd, ad).cpu().numpy()
            np.testing.assert_array_equal(D1, D2)
            R = s.eval_ratio_v(pd, ad).cpu().numpy()
            e = _err(D1[:300], Dref, scale)
            ev = _err(R[:300, None], Dref[:, :1], scale[:, :1])
            assert e <= TOL[dt] and ev <= TOL[dt], (dt, t, e, ev)


@pytest.mark.parametrize("norb", [1, 37, 100, 129])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
def test_ragged_orbitals_and_batches(torch, q, oracle, norb, dtype):
    rng = np.random.default_rng(100 + norb)
    grid = (5, 7, 6)
    coefs = rng.uniform(-1, 1, grid + (norb,))
    ref_coefs = _table_ref(oracle, coefs, dtype)
    s = q.Spline(grid, coefs, dtype)
    npdt = np.float64 if dtype == "f64" else np.float32
    for B in (1, 33, 257):
        _say("case ratio ragged", dtype, norb, B)
        pos = rng.random((B, 3))
        rows = rng.normal(size=(B, norb)).astype(npdt)
        D = s.eval_ratio_vgl(torch.from_numpy(pos).cuda(), torch.from_numpy(rows).cuda()).cpu().numpy()
        Dref, scale = _ref(oracle, grid, ref_coefs, pos, rows)
        assert _err(D, Dref, scale) <= TOL[dtype], (dtype, norb, B)


def test_row_addressing(torch, q, oracle):
    """rows[] indirection (quadrature points sharing an electron's row) and a
    strided base (electron k of every walker: base k*N, ld N*N) give the same
    bits as explicitly gathered rows."""
    grid, N, coefs, _ = W.make_table(1)
    rng = np.random.default_rng(7)
    s = q.Spline(grid, coefs, "f32")
    inv = rng.normal(size=(6, N, N)).astype(np.float32)  # six walkers' inverses
    invd = torch.from_numpy(inv).cuda()
    # quadrature: 12 points per electron, electrons 0..N-1 of walker 2
    npts = 12
    pos = rng.random((N * npts, 3))
    pd = torch.from_numpy(pos).cuda()
    ridx = (2 * N + np.arange(N * npts) // npts).astype(np.int32)
    gathered = torch.from_numpy(np.ascontiguousarray(inv.reshape(-1, N)[ridx])).cuda()
    Ri = s.eval_ratio_v(pd, invd.reshape(-1), ld=N, rows=torch.from_numpy(ridx).cuda())
    Rg = s.eval_ratio_v(pd, gathered)
    np.testing.assert_array_equal(Ri.cpu().numpy(), Rg.cpu().numpy())
    # electron k of every walker
    k = 5
    pw = torch.from_numpy(rng.random((6, 3))).cuda()
    Ds = s.eval_ratio_vgl(pw, invd.reshape(-1)[k * N:], ld=N * N)
    Dg = s.eval_ratio_vgl(pw, torch.from_numpy(np.ascontiguousarray(inv[:, k, :])).cuda())
    np.testing.assert_array_equal(Ds.cpu().numpy(), Dg.cpu().numpy())
    Dref, scale = _ref(oracle, grid, coefs, pw.cpu().numpy(), inv[:, k, :])
    assert _err(Ds.cpu().numpy(), Dref, scale) <= TOL["f32"]


def test_edges_and_consistency_with_stored_values(torch, q, oracle):
    """Empty batch, a non-finite position (NaN row, neighbours untouched),
    and agreement with an FP64 dot product of the same kernel family's stored
    V, G, L (a property of the path: only the summation differs)."""
    grid, N, coefs, _ = W.make_table(2)
    s = q.Spline(grid, coefs, "f32")
    rows = W.make_inverse_rows(2, 513, N)
    pos = W.make_positions(2, count=513)
    pos[100, 1] = np.nan
    pd, ad = torch.from_numpy(pos).cuda(), torch.from_numpy(rows).cuda()
    empty = s.eval_ratio_vgl(pd[:0], ad)
    assert tuple(empty.shape) == (0, 5)
    D = s.eval_ratio_vgl(pd, ad).cpu().numpy()
    assert np.all(np.isnan(D[100])) and np.all(np.isfinite(np.delete(D, 100, axis=0)))
    V, G, L = (t.cpu().numpy().astype(np.float64) for t in s.eval_vgl(pd))
    r64 = rows.astype(np.float64)
    mine = np.stack([np.sum(r64 * V, 1)] + [np.sum(r64 * G[:, d], 1) for d in range(3)] + [np.sum(r64 * L, 1)], 1)
    ok = np.arange(len(pos)) != 100
    M = [np.abs(V[ok]).max(0), np.abs(G[ok]).max((0, 1)), np.abs(L[ok]).max(0)]
    sv, sg, sl = (np.abs(r64) @ m for m in M)
    scale = np.stack([sv, sg, sg, sg, sl], 1)
    e = _err(D[ok], mine[ok], scale[ok])
    _say("ratio vs FP64 dot of stored values: %.2e" % e)
    assert e <= 2e-6


def test_argument_errors(torch, q):
    grid, N, coefs, _ = W.make_table(1)
    s = q.Spline(grid, coefs, "f32")
    pd = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    ad = torch.zeros((4, N), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        s.eval_ratio_vgl(pd, ad.double())
    with pytest.raises(ValueError):
        s.eval_ratio_vgl(pd, ad[:3])
    with pytest.raises(ValueError):
        s.eval_ratio_v(pd, ad, rows=torch.tensor([0, 1, 2, 4], dtype=torch.int32, device="cuda"))
    L = q.lib()
    import ctypes
    rc = L.spline_eval_ratio_vgl(s.handle, ctypes.c_void_p(pd.data_ptr()), 4, None, N, None,
                                 ctypes.c_void_p(ad.data_ptr()), None)
    assert rc == -1 and "NULL" in q.last_error()
    rc = L.spline_eval_ratio_v(s.handle, ctypes.c_void_p(pd.data_ptr()), 4, ctypes.c_void_p(ad.data_ptr() + 2), N,
                               None, ctypes.c_void_p(ad.data_ptr()), None)
    assert rc == -1 and "aligned" in q.last_error()
