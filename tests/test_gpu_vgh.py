"""GPU parity of the value-gradient-Hessian kernels and of general
(triclinic) cells against the FP64 oracle (oracle.eval_vgh).

Error measure: per-orbital max-norm relative error (the components of G
pooled, the six components of H pooled), maximised over orbitals.  Bars as
for VGL: 1e-12 for FP64 tables, 1e-5 for FP32 accumulation; 16-bit tables
against the oracle on the dequantized coefficients.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5, "f16": 1e-5}
HEX = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3.0) / 2.0, 0.0], [0.0, 0.0, 1.6]])
TRI = np.array([[1.1, 0.1, -0.2], [0.3, 0.9, 0.15], [-0.1, 0.25, 1.3]])
LATTICES = {"cubic": np.eye(3), "orthorhombic": np.diag([1.0, 1.3, 0.8]), "hexagonal": HEX, "triclinic": TRI}


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


def _ref_coefs(oracle, coefs, dtype):
    return oracle.dequantize(coefs, dtype)[0] if dtype in ("bf16", "f16", "f32") else coefs


def _np(ts):
    return [t.double().cpu().numpy() for t in ts]


def _check(oracle, got, ref, tol, what):
    errs = [oracle.rel_err(g, r) for g, r in zip(got, ref)]
    _say(what, "eps " + " ".join("%.2e" % e for e in errs))
    for name, e in zip("VGH", errs):
        assert e <= tol, "%s: %s rel err %.3e > %.1e" % (what, name, e, tol)
    return errs


def _positions(rng, B, lat):
    return (rng.random((B, 3)) * 3 - 1) @ lat  # several periods, both signs


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("name", list(LATTICES))
def test_c1_vgh_every_lattice(torch, q, oracle, dtype, name):
    lat = LATTICES[name]
    grid, N, coefs, _ = W.make_table(1)
    pos = _positions(np.random.default_rng(7), 1000, lat)
    _say("case vgh c1", dtype, name)
    s = q.Spline(grid, coefs, dtype, cell=tuple(np.diag(lat)) if name in ("cubic", "orthorhombic") else (1, 1, 1))
    if name not in ("cubic", "orthorhombic"):
        s.set_lattice(lat)
    np.testing.assert_array_equal(s.get_lattice(), lat)
    ref = oracle.eval_vgh(grid, _ref_coefs(oracle, coefs, dtype), pos, lat)
    pd = torch.from_numpy(pos).cuda()
    got = _np(s.eval_vgh(pd))
    _check(oracle, got, ref, TOL[dtype], "vgh c1 %s %s" % (dtype, name))
    # VGL and value only on the same handle
    V, G, L = _np(s.eval_vgl(pd))
    Lref = ref[2][:, 0] + ref[2][:, 3] + ref[2][:, 5]
    _check(oracle, (V, G, L), (ref[0], ref[1], Lref), TOL[dtype], "vgl c1 %s %s" % (dtype, name))
    Vv = _np([s.eval_v(pd)])[0]
    _check(oracle, [Vv], [ref[0]], TOL[dtype], "v c1 %s %s" % (dtype, name))


def test_general_handle_with_diagonal_lattice_matches_orthorhombic(torch, q, oracle):
    """A general handle given a diagonal lattice reproduces the orthorhombic
    handle's VGL within rounding (different kernels and staging)."""
    grid, N, coefs, _ = W.make_table(2)
    cell = (1.0, 1.3, 0.8)
    pos = W.make_positions(2, count=2000) * cell
    pd = torch.from_numpy(pos).cuda()
    so = q.Spline(grid, coefs, "f32", cell=cell)
    sg = q.Spline(grid, coefs, "f32", cell=cell)
    sg.set_lattice(np.diag(cell))
    a = _np(so.eval_vgl(pd))
    b = _np(sg.eval_vgl(pd))
    _check(oracle, b, a, 1e-5, "general(diag) vs orthorhombic")
    Vh, Gh, Hh = _np(so.eval_vgh(pd))
    _check(oracle, (Vh, Gh, Hh[:, 0] + Hh[:, 3] + Hh[:, 5]), a, 1e-5, "vgh trace vs vgl")


def test_every_vgh_tile_shape(torch, q, oracle):
    grid, N, coefs, _ = W.make_table(2)
    pos = _positions(np.random.default_rng(3), 1501, HEX)
    pd = torch.from_numpy(pos).cuda()
    for dt in ("f32", "bf16", "f64"):
        s = q.Spline(grid, coefs, dt)
        s.set_lattice(HEX)
        ref = oracle.eval_vgh(grid, _ref_coefs(oracle, coefs, dt), pos[:300], HEX)
        first = None
        for t in s.vgh_tile_candidates():
            _say("case vgh tile", dt, t)
            s.set_vgh_tile(t)
            got = _np(s.eval_vgh(pd))
            if first is None:
                first = got
                _check(oracle, [g[:300] for g in got], ref, TOL[dt], "vgh tile %s %s" % (dt, t))
            else:
                for x, y in zip(first, got):
                    np.testing.assert_array_equal(x, y)
        chosen = s.autotune_vgh(pd, reps=1)
        assert chosen in s.vgh_tile_candidates()


@pytest.mark.parametrize("norb", [1, 37, 100, 129])
@pytest.mark.parametrize("dtype", ["f64", "f32", "f16"])
def test_ragged_orbitals_and_batches(torch, q, oracle, norb, dtype):
    rng = np.random.default_rng(200 + norb)
    grid = (5, 7, 6)
    coefs = rng.uniform(-1, 1, grid + (norb,))
    s = q.Spline(grid, coefs, dtype)
    s.set_lattice(TRI)
    rc = _ref_coefs(oracle, coefs, dtype)
    gots, poss = [], []
    for B in (1, 33, 257):
        _say("case vgh ragged", dtype, norb, B)
        pos = _positions(rng, B, TRI)
        gots.append(_np(s.eval_vgh(torch.from_numpy(pos).cuda())))
        poss.append(pos)
    got = [np.concatenate([g[i] for g in gots]) for i in range(3)]
    pos = np.concatenate(poss)
    _check(oracle, got, oracle.eval_vgh(grid, rc, pos, TRI), TOL[dtype], "vgh ragged %s N=%d" % (dtype, norb))


@pytest.fixture(scope="module")
def c3():
    grid, N, coefs, _ = W.make_table(3)
    return grid, N, coefs


def test_c3_hexagonal_full_batch_sampled(torch, q, oracle, c3):
    """The 80^3 x 384 FP32 table in a hexagonal cell, full 196608-position
    batch, in the tile the benchmark's autotuner selects; sampled check."""
    grid, N, coefs = c3
    u = W.make_positions(3)
    pos = u @ HEX
    _say("case vgh c3 hexagonal", pos.shape)
    s = q.Spline(grid, coefs, "f32")
    s.set_lattice(HEX)
    pd = torch.from_numpy(pos).cuda()
    out = s.alloc_vgh(len(pos))
    s.autotune_vgh(pd, reps=2, out=out)
    V, G, H = s.eval_vgh(pd, out=out)
    idx = np.concatenate([np.random.default_rng(4).choice(len(pos), 256, replace=False), [0, len(pos) - 1]])
    it = torch.from_numpy(idx).cuda()
    got = _np((V[it], G[it], H[it]))
    _check(oracle, got, oracle.eval_vgh(grid, coefs, pos[idx], HEX), TOL["f32"],
           "vgh c3 hexagonal tile %s" % (s.get_vgh_tile(),))
    # locality order: the whole batch equal bit for bit (VGH and the general-cell VGL)
    plain = [t.clone() for t in (V, G, H)]
    Vs, Gs, Hs = s.eval_vgh_sorted(pd, out=out)
    for a, b in zip((Vs, Gs, Hs), plain):
        assert torch.equal(a, b)
    del plain, out
    for a, b in zip(s.eval_vgl_sorted(pd), s.eval_vgl(pd)):
        assert torch.equal(a, b)


def test_edges_and_unsupported(torch, q, oracle):
    grid, N, coefs, _ = W.make_table(1)
    s = q.Spline(grid, coefs, "f32")
    s.set_lattice(HEX)
    pos = _positions(np.random.default_rng(9), 65, HEX)
    pos[10, 2] = np.inf
    pd = torch.from_numpy(pos).cuda()
    V, G, H = _np(s.eval_vgh(pd))
    assert np.all(np.isnan(V[10])) and np.all(np.isnan(H[10]))
    ok = np.arange(65) != 10
    assert np.all(np.isfinite(V[ok])) and np.all(np.isfinite(H[ok]))
    e = s.eval_vgh(pd[:0])
    assert tuple(e[2].shape) == (0, 6, N)
    # the ratio with derivatives: NaN for the non-finite position only
    rows = torch.ones((65, N), dtype=torch.float32, device="cuda")
    D = s.eval_ratio_vgl(pd, rows).cpu().numpy()
    assert np.all(np.isnan(D[10])) and np.all(np.isfinite(D[ok]))
    # value-only ratio serves general cells
    rows = torch.from_numpy(np.random.default_rng(1).normal(size=(65, N)).astype(np.float32)).cuda()
    R = s.eval_ratio_v(pd, rows).cpu().numpy()
    Vref = oracle.eval_vgh(grid, coefs, pos, HEX)[0]
    r64 = rows.double().cpu().numpy()
    ref = np.sum(r64 * Vref, axis=1)
    scale = np.abs(r64) @ np.abs(Vref[ok]).max(0)
    assert np.max(np.abs(R[ok] - ref[ok]) / scale[ok]) < 1e-5
    with pytest.raises(q.SplineError):
        s.set_lattice(np.zeros((3, 3)))
    # plans serve general cells (the VGH-family plan kernel), NaN rows included
    plan = q.Plan([s], [pd], tune_reps=0)
    s.set_vgh_tile(plan.info()["tile"])
    for a, b in zip(plan.launch()[0], s.eval_vgl(pd)):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("name", ["hexagonal", "triclinic"])
def test_general_ratio_with_derivatives(torch, q, oracle, dtype, name):
    """Fused determinant ratio with derivatives in a general cell (the
    VGH-family kernel with the ratio epilogue), plain and locality-ordered,
    against the oracle's dot products of each row with V, the Cartesian G
    and the trace of the Cartesian Hessian.  Error measure of the ratio
    tests: |D - D_ref| / sum_i |a_i| max|Q_i|; same bars as VGL."""
    from oracle import det

    lat = LATTICES[name]
    grid, N, coefs, _ = W.make_table(1)
    rng = np.random.default_rng(41)
    pos = _positions(rng, 777, lat)
    _say("case general ratio", dtype, name)
    s = q.Spline(grid, coefs, dtype)
    s.set_lattice(lat)
    table = _ref_coefs(oracle, coefs, dtype)
    fdt = np.float64 if dtype == "f64" else np.float32
    # rows through an index map with a stride of 2N (quadrature points
    # sharing an electron's row)
    ainv = rng.standard_normal((400, 2 * N)).astype(fdt)
    idx = rng.integers(0, 400, len(pos)).astype(np.int32)
    rows64 = ainv[idx, :N].astype(np.float64)
    Dref = det.ratio_vgl_lattice(grid, table, pos, rows64, lat)
    V, G, H = oracle.eval_vgh(grid, table, pos, lat)
    M = [np.abs(V).max(0), np.abs(G).max((0, 1)), np.abs(H[:, 0] + H[:, 3] + H[:, 5]).max(0)]
    sv, sg, sl = (det.ratio_scale(rows64, m) for m in M)
    scale = np.stack([sv, sg, sg, sg, sl], 1)
    pd = torch.from_numpy(pos).cuda()
    ad = torch.from_numpy(ainv).cuda()
    rd = torch.from_numpy(idx).cuda()
    for how in ("plain", "sorted"):
        if how == "plain":
            D = s.eval_ratio_vgl(pd, ad, ld=2 * N, rows=rd)
        else:
            D = s.eval_ratio_vgl_sorted(pd, ad, ld=2 * N, rows=rd)
        D = D.double().cpu().numpy()
        e = float(np.max(np.abs(D - Dref) / scale))
        _say("  %s eps %.2e" % (how, e))
        assert e <= TOL[dtype], (how, e)
