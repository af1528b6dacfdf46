"""GPU tests of ragged multi-table plans (one persistent launch in a graph).

The plan evaluates each orbital with the same arithmetic in the same order
as the single-table kernel, so its outputs must equal spline_eval_vgl's bit
for bit; graph replays must equal the eager launch; and a sample is checked
against the FP64 oracle.
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


def _tables(q, torch, specs, seed, dtype="f32"):
    rng = np.random.default_rng(seed)
    sp, pos, coefs = [], [], []
    for grid, N, B in specs:
        c = rng.uniform(-1, 1, grid + (N,))
        sp.append(q.Spline(grid, c, dtype))
        pos.append(torch.from_numpy(rng.random((B, 3))).cuda())
        coefs.append(c)
    return sp, pos, coefs


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())


SPECS = [((8, 8, 8), 64, 1000), ((10, 9, 8), 128, 257), ((12, 12, 12), 256, 1), ((9, 7, 11), 384, 700)]


@pytest.mark.parametrize("sorted_", [False, True])
@pytest.mark.parametrize("tune", [0, 2])
def test_plan_equals_single_table_bitwise(torch, q, oracle, tune, sorted_):
    """Plain plans (one work queue) and locality-ordered plans (positions
    sorted on the device at each launch, the queue in eight segments)."""
    sp, pos, coefs = _tables(q, torch, SPECS, 11)
    _say("case plan tune", tune, "sorted", sorted_)
    plan = q.Plan(sp, pos, tune_reps=tune, sorted=sorted_)
    info = plan.info()
    _say("plan info", info)
    assert info["tasks"] > 0 and info["blocks"] >= 1
    outs = plan.launch()
    torch.cuda.synchronize()
    for s, p, o, c in zip(sp, pos, outs, coefs):
        ref = s.eval_vgl(p)
        torch.cuda.synchronize()
        _same(o, ref)
        if p.shape[0] < 64:
            continue  # too few positions for the per-orbital max-norm; covered bitwise above
        k = 64
        r = oracle.eval_vgl(s.grid, oracle.dequantize(c, "f32")[0], p[:k].cpu().numpy())
        for g_, r_ in zip(o, r):
            assert oracle.rel_err(g_[:k].cpu().numpy(), r_) <= 1e-5


@pytest.mark.parametrize("sorted_", [False, True])
def test_plan_graph_replays_match_eager(torch, q, sorted_):
    sp, pos, _ = _tables(q, torch, SPECS, 12)
    plan = q.Plan(sp, pos, tune_reps=0, sorted=sorted_)
    plan.launch_eager()
    torch.cuda.synchronize()
    eager = [[t.clone() for t in o] for o in plan.outs]
    for rep in range(4):
        _say("case plan replay", rep)
        for o in plan.outs:
            for t in o:
                t.zero_()
        torch.cuda.synchronize()
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for o, e in zip(plan.outs, eager):
            _same(o, e)
        del x


@pytest.mark.parametrize("sorted_", [False, True])
def test_plan_moving_positions(torch, q, sorted_):
    """Positions may change between launches (same buffers); a locality-
    ordered plan sorts them again at every launch."""
    sp, pos, _ = _tables(q, torch, SPECS[:2], 13)
    plan = q.Plan(sp, pos, tune_reps=0, sorted=sorted_)
    for rep in range(3):
        _say("case plan move", rep)
        for p in plan.positions:
            p.add_(0.137).remainder_(1.0)
        plan.launch()
        torch.cuda.synchronize()
        for s, p, o in zip(sp, plan.positions, plan.outs):
            _same(o, s.eval_vgl(p))


@pytest.mark.parametrize("sorted_", [False, True])
def test_plan_empty_tables(torch, q, sorted_):
    specs = [((8, 8, 8), 64, 0), ((9, 9, 9), 128, 33), ((8, 8, 8), 64, 0)]
    sp, pos, _ = _tables(q, torch, specs, 14)
    plan = q.Plan(sp, pos, tune_reps=1, sorted=sorted_)
    outs = plan.launch()
    torch.cuda.synchronize()
    _same(outs[1], sp[1].eval_vgl(pos[1]))
    sp0, pos0, _ = _tables(q, torch, [((8, 8, 8), 64, 0)], 15)
    plan0 = q.Plan(sp0, pos0, tune_reps=1, sorted=sorted_)
    assert plan0.info()["tasks"] == 0
    plan0.launch()
    torch.cuda.synchronize()


def test_plan_rejects_mixed_storage_and_small_workspace(torch, q):
    rng = np.random.default_rng(16)
    a = q.Spline((6, 6, 6), rng.uniform(-1, 1, (6, 6, 6, 64)), "f32")
    b = q.Spline((6, 6, 6), rng.uniform(-1, 1, (6, 6, 6, 64)), "bf16")
    p = [torch.from_numpy(rng.random((10, 3))).cuda() for _ in range(2)]
    with pytest.raises(q.SplineError) as e:
        q.Plan([a, b], p)
    assert e.value.code == -4
    import ctypes
    L = q.lib()
    Bs = (ctypes.c_int64 * 1)(10)
    nb = L.spline_plan_workspace_bytes(1, Bs)
    assert nb > 0
    assert L.spline_plan_workspace_bytes(1, (ctypes.c_int64 * 1)(-1)) == 0


def test_c4_ragged_workload(torch, q, oracle):
    """The four-table ragged workload (32^3..80^3, N=64..384, walker counts
    U{64..1024}) in one plan, against single-table launches (bitwise) and the
    oracle (sampled)."""
    tabs = W.make_ragged()
    sp, pos = [], []
    for t in tabs:
        _say("case c4 table", t["grid"], t["norb"], t["pos"].shape[0])
        sp.append(q.Spline(t["grid"], t["coefs"], "f32"))
        pos.append(torch.from_numpy(t["pos"]).cuda())
    plan = q.Plan(sp, pos, tune_reps=2)
    _say("c4 plan", plan.info())
    outs = plan.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    for t, s, p, o in zip(tabs, sp, pos, outs):
        ref = s.eval_vgl(p)
        torch.cuda.synchronize()
        idx = torch.from_numpy(rng.choice(p.shape[0], 128, replace=False)).cuda()
        for a, b in zip(o, ref):
            np.testing.assert_array_equal(a[idx].cpu().numpy(), b[idx].cpu().numpy())
        r = oracle.eval_vgl(t["grid"], t["coefs"], t["pos"][idx.cpu().numpy()])
        errs = [oracle.rel_err(a[idx].cpu().numpy(), b) for a, b in zip(o, r)]
        _say("c4", t["grid"], "eps V/G/L = %.2e %.2e %.2e" % tuple(errs))
        assert max(errs) <= 1e-5
    # the locality-ordered plan over the same workload: whole outputs equal
    plain = [[x.clone() for x in o] for o in outs]
    plan_s = q.Plan(sp, pos, tune_reps=2, sorted=True)
    _say("c4 sorted plan", plan_s.info())
    outs_s = plan_s.launch()
    torch.cuda.synchronize()
    for o, e in zip(outs_s, plain):
        for a, b in zip(o, e):
            assert torch.equal(a, b)


HEX = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3.0) / 2.0, 0.0], [0.0, 0.0, 1.6]])
TRI = np.array([[1.1, 0.1, -0.2], [0.3, 0.9, 0.15], [-0.1, 0.25, 1.3]])


@pytest.mark.parametrize("sorted_", [False, True])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_plan_with_general_cells(torch, q, oracle, dtype, sorted_):
    """A plan holding tables with general cells (hexagonal, triclinic) and an
    orthorhombic one: every task runs the VGH-family kernel (V, G, and L as
    the trace of the Cartesian Hessian).  Against the FP64 oracle (the
    general-cell oracle for the lattices) at the VGL bars; the general tables
    equal their own single-table spline_eval_vgl under the plan's shape bit
    for bit; a locality-ordered plan equals the plain one bit for bit."""
    specs = [((8, 9, 10), 64, 700), ((10, 8, 8), 128, 333), ((9, 9, 9), 32, 64)]
    lats = [HEX, TRI, None]
    rng = np.random.default_rng(19)
    sp, pos, coefs = [], [], []
    for (grid, N, B), lat in zip(specs, lats):
        c = rng.uniform(-1, 1, grid + (N,))
        s = q.Spline(grid, c, dtype)
        if lat is not None:
            s.set_lattice(lat)
        frac = rng.uniform(-1, 2, (B, 3))
        sp.append(s)
        pos.append(torch.from_numpy(frac @ lat if lat is not None else frac).cuda())
        coefs.append(c)
    _say("case general plan", dtype, "sorted", sorted_)
    plan = q.Plan(sp, pos, tune_reps=2, sorted=sorted_)
    info = plan.info()
    _say("plan info", info)
    outs = [[t.clone() for t in o] for o in plan.launch()]
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == "f64" else 1e-5
    for s, p, o, c, lat in zip(sp, pos, outs, coefs, lats):
        table = c if dtype == "f64" else oracle.dequantize(c, "f32")[0]
        pn = p.cpu().numpy()
        if lat is not None:
            V, G, H = oracle.eval_vgh(s.grid, table, pn, lat)
            ref = (V, G, H[:, 0] + H[:, 3] + H[:, 5])
            s.set_vgh_tile(info["tile"])
            single = s.eval_vgl(p)
            torch.cuda.synchronize()
            _same(o, single)
        else:
            ref = oracle.eval_vgl(s.grid, table, pn)
        for name, g_, r_ in zip("VGL", o, ref):
            e = oracle.rel_err(g_.double().cpu().numpy(), r_)
            assert e <= tol, (name, e)
    if sorted_:
        # per-orbital arithmetic does not depend on the shape (the tuner
        # checks that bitwise), so the plain plan's default shape gives the
        # same bits
        plain = q.Plan(sp, pos, tune_reps=0)
        _same([t for o in outs for t in o], [t for o in plain.launch() for t in o])
