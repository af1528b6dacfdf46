"""GPU parity of the HIP spline path against the FP64 oracle.

Every call goes through the C ABI (libqmcspline.so) via the Python binding.
Tolerances (per-orbital max-norm relative error, pooled over positions and
gradient components):
  FP64 table: 1e-12 (FP64 accumulation; only summation order differs)
  FP32 table: 1e-5 against the oracle on the ORIGINAL FP64 coefficients
  BF16/FP16:  1e-5 against the oracle on the DEQUANTIZED coefficients (the
              kernel's own arithmetic); the error against the original
              coefficients is reported, not gated here.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

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


def _ref(oracle, grid, coefs, dtype, pos, cell=(1.0, 1.0, 1.0)):
    if dtype in ("bf16", "f16", "f32"):
        dq = oracle.dequantize(coefs, dtype)[0]
    else:
        dq = coefs
    return oracle.eval_vgl(grid, dq, pos, cell=cell)


def _check(oracle, got, ref, tol, what):
    errs = [oracle.rel_err(g, r) for g, r in zip(got, ref)]
    _say(what, "eps V/G/L = %.2e %.2e %.2e" % tuple(errs))
    for name, e in zip("VGL", errs):
        assert e <= tol, "%s: %s rel err %.3e > %.1e" % (what, name, e, tol)
    return errs


def _np(ts):
    return [t.cpu().numpy() for t in ts]


def test_c1_fp64_and_fp32(torch, q, oracle):
    grid, N, coefs, _ = W.make_table(1)
    pos = W.make_positions(1)
    pd = torch.from_numpy(pos).cuda()
    Vr, Gr, Lr = oracle.eval_vgl(grid, coefs, pos)
    for dt in ("f64", "f32"):
        _say("case c1", dt)
        s = q.Spline(grid, coefs, dt)
        got = _np(s.eval_vgl(pd))
        torch.cuda.synchronize()
        _check(oracle, got, _ref(oracle, grid, coefs, dt, pos), TOL[dt], "c1 %s vs dequantized" % dt)
        _check(oracle, got, (Vr, Gr, Lr), TOL[dt], "c1 %s vs original" % dt)


@pytest.fixture(scope="module")
def c2(oracle):
    grid, N, coefs, ex = W.make_table(2)
    return grid, N, coefs


def test_c2_fp32_full_batch_sampled(torch, q, oracle, c2):
    grid, N, coefs = c2
    pos = W.make_positions(2)
    _say("case c2 f32 full batch", pos.shape)
    s = q.Spline(grid, coefs, "f32")
    V, G, L = s.eval_vgl(torch.from_numpy(pos).cuda())
    idx = np.random.default_rng(0).choice(len(pos), 2048, replace=False)
    idx = np.concatenate([idx, [0, len(pos) - 1]])
    it = torch.from_numpy(idx).cuda()
    got = _np((V[it], G[it], L[it]))
    _check(oracle, got, oracle.eval_vgl(grid, coefs, pos[idx]), TOL["f32"], "c2 f32 vs FP64 oracle")


def test_c2_every_tile_shape_bitwise_and_parity(torch, q, oracle, c2):
    grid, N, coefs = c2
    pos = W.make_positions(2, count=4099)   # ragged tail over every positions-per-workgroup value
    pd = torch.from_numpy(pos).cuda()
    ref = oracle.eval_vgl(grid, coefs, pos[:600])
    for dt in ("f32", "bf16", "f16"):
        s = q.Spline(grid, coefs, dt)
        cands = s.tile_candidates()
        assert len(cands) >= 3
        first = None
        for t in cands:
            _say("case c2 tile", dt, t)
            s.set_tile(t)
            got = _np(s.eval_vgl(pd))
            if first is None:
                first = got
                if dt == "f32":
                    _check(oracle, [g[:600] for g in got], ref, TOL[dt], "c2 f32 tile %s" % (t,))
                else:
                    _check(oracle, [g[:600] for g in got], _ref(oracle, grid, coefs, dt, pos[:600]), TOL[dt],
                           "c2 %s tile %s" % (dt, t))
            else:
                for a, b in zip(first, got):
                    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16"])
def test_c3_full_batch_sampled(torch, q, oracle, dtype, c3):
    grid, N, coefs = c3
    pos = W.make_positions(3)
    _say("case c3 full batch", dtype, pos.shape)
    s = q.Spline(grid, coefs, dtype)
    V, G, L = s.eval_vgl(torch.from_numpy(pos).cuda())
    idx = np.random.default_rng(1).choice(len(pos), 512, replace=False)
    it = torch.from_numpy(idx).cuda()
    got = _np((V[it], G[it], L[it]))
    _check(oracle, got, _ref(oracle, grid, coefs, dtype, pos[idx]), TOL[dtype], "c3 %s vs kernel-precision oracle" % dtype)
    if dtype != "f32":
        errs = [oracle.rel_err(g, r) for g, r in zip(got, oracle.eval_vgl(grid, coefs, pos[idx]))]
        _say("c3 %s quantization error vs FP64 original: eps V/G/L = %.2e %.2e %.2e" % ((dtype,) + tuple(errs)))


@pytest.fixture(scope="module")
def c3():
    grid, N, coefs, _ = W.make_table(3)
    return grid, N, coefs


@pytest.mark.parametrize("norb", [1, 37, 100, 129])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_ragged_orbital_counts(torch, q, oracle, norb, dtype):
    """Ragged orbital counts (partial rows) and batch sizes (partial
    workgroups), each launched on its own; the relative error pools the
    launches, since the per-orbital max-norm of a single position is
    pointwise and ill-conditioned where an orbital crosses zero."""
    rng = np.random.default_rng(norb)
    grid = (5, 7, 6)
    coefs = rng.uniform(-1, 1, grid + (norb,))
    s = q.Spline(grid, coefs, dtype)
    gots, poss = [], []
    for B in (1, 33, 257):
        _say("case ragged", dtype, norb, B)
        pos = rng.random((B, 3))
        gots.append(_np(s.eval_vgl(torch.from_numpy(pos).cuda())))
        poss.append(pos)
    got = [np.concatenate([g[i] for g in gots]) for i in range(3)]
    pos = np.concatenate(poss)
    _check(oracle, got, _ref(oracle, grid, coefs, dtype, pos), TOL[dtype], "ragged %s N=%d" % (dtype, norb))


def test_small_and_orthorhombic_grids(torch, q, oracle):
    rng = np.random.default_rng(5)
    for grid, cell in (((1, 1, 1), (1, 1, 1)), ((2, 3, 1), (0.5, 1.0, 2.0)), ((7, 9, 11), (1.3, 0.7, 2.1))):
        coefs = rng.uniform(-1, 1, grid + (64,))
        pos = rng.uniform(-3, 3, (300, 3)) * np.asarray(cell)
        for dt in ("f64", "f32"):
            _say("case grid", grid, cell, dt)
            s = q.Spline(grid, coefs, dt, cell=cell)
            got = _np(s.eval_vgl(torch.from_numpy(pos).cuda()))
            ref = oracle.eval_vgl(grid, coefs, pos, cell=cell)
            if grid == (1, 1, 1):
                # one coefficient per orbital: V is that constant and every
                # derivative vanishes (the oracle's are pure roundoff)
                assert oracle.rel_err(got[0], ref[0]) <= TOL[dt]
                assert np.abs(got[1]).max() <= 1e-12 and np.abs(got[2]).max() <= 1e-12
                assert np.abs(ref[1]).max() <= 1e-12 and np.abs(ref[2]).max() <= 1e-12
                continue
            _check(oracle, got, ref, TOL[dt], "grid %s cell %s %s" % (grid, cell, dt))


def test_edge_positions(torch, q, oracle):
    rng = np.random.default_rng(6)
    grid = (8, 8, 8)
    coefs = rng.uniform(-1, 1, grid + (64,))
    pos = np.array([
        [0.0, 0.0, 0.0], [-0.0, 0.5, 0.25], [-1e-17, 0.125, 1.0 - 2.0 ** -53], [1.0, 2.0, -3.0],
        [1e6 + 0.3, -1e6 + 0.1, 12345.678], [0.375, 0.5, 0.625], [7 / 8, 1 / 8, 3 / 8],
        [np.nan, 0.1, 0.2], [0.1, np.inf, 0.2], [0.1, 0.2, -np.inf], [0.3, 0.4, 0.5],
    ])
    for dt in ("f64", "f32", "bf16"):
        _say("case edge", dt)
        s = q.Spline(grid, coefs, dt)
        V, G, L = _np(s.eval_vgl(torch.from_numpy(pos).cuda()))
        bad = [7, 8, 9]
        assert np.isnan(V[bad]).all() and np.isnan(G[bad]).all() and np.isnan(L[bad]).all()
        good = [i for i in range(len(pos)) if i not in bad]
        ref = _ref(oracle, grid, coefs, dt, pos[good])
        _check(oracle, (V[good], G[good], L[good]), ref, TOL[dt], "edge %s" % dt)


def test_empty_batch_and_value_only(torch, q, oracle):
    rng = np.random.default_rng(7)
    grid = (6, 6, 6)
    coefs = rng.uniform(-1, 1, grid + (96,))
    for dt in ("f64", "f32", "bf16", "f16"):
        _say("case value-only", dt)
        s = q.Spline(grid, coefs, dt)
        empty = torch.empty((0, 3), dtype=torch.float64, device="cuda")
        V0, G0, L0 = s.eval_vgl(empty)
        assert V0.shape == (0, 96)
        pos = torch.from_numpy(rng.random((513, 3))).cuda()
        V, _, _ = s.eval_vgl(pos)
        Vv = s.eval_v(pos)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(Vv.cpu().numpy(), V.cpu().numpy())


def test_side_stream_and_reuse(torch, q, oracle):
    rng = np.random.default_rng(8)
    grid = (6, 7, 8)
    coefs = rng.uniform(-1, 1, grid + (128,))
    pos = rng.random((1000, 3))
    s = q.Spline(grid, coefs, "f32")
    st = torch.cuda.Stream()
    pd = torch.from_numpy(pos).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        out = s.alloc_outputs(len(pos))
        for _ in range(3):
            s.eval_vgl(pd, out=out)
    st.synchronize()
    _check(oracle, _np(out), _ref(oracle, grid, coefs, "f32", pos), TOL["f32"], "side stream")


def test_autotune_cache(torch, q, oracle, tmp_path):
    rng = np.random.default_rng(9)
    grid = (10, 10, 10)
    coefs = rng.uniform(-1, 1, grid + (192,))
    pos = torch.from_numpy(rng.random((2000, 3))).cuda()
    s = q.Spline(grid, coefs, "f32")
    cache = str(tmp_path / "tune.txt")
    t1 = s.autotune(pos, reps=2, cache_path=cache)
    assert t1 in s.tile_candidates()
    assert os.path.exists(cache)
    s2 = q.Spline(grid, coefs, "f32")
    assert s2.autotune(pos, reps=2, cache_path=cache) == t1     # cache hit
    with open(cache, "w") as f:
        f.write("garbage|x y z\n\x00\x01|1 2\n")
    assert s2.autotune(pos, reps=1, cache_path=cache) in s2.tile_candidates()  # corrupt cache ignored
    got = _np(s2.eval_vgl(pos))
    _check(oracle, got, _ref(oracle, grid, coefs, "f32", pos.cpu().numpy()), TOL["f32"], "after autotune")
