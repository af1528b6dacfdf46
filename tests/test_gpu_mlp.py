"""GPU tests of the learned surrogate (forward-mode MLP on matrix cores).

- the fused forward kernel against the FP64 oracle with BF16 rounding of
  every product operand emulated (tolerance 2^-7, per-orbital max-norm), and
  against the exact FP64 network (reported);
- the output map and loss weights against the oracle's output_normalisation;
- the training gradient against the oracle's reverse pass under the same BF16
  arithmetic model (relative L2 <= 1e-3 per tensor, for the whole loss and
  for each of its three terms alone);
- the error map against the oracle's, bin by bin, and the routed set against
  the oracle's, exactly;
- training lowers the loss; routed positions equal the spline bit for bit
  and the others equal the network bit for bit; routing everything
  reproduces the spline exactly;
- a saved state resumes with identical outputs;
- what the trained network gains over the table: footprint and speed.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mlp as M

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


def _net(q, N, seed=5):
    freqs, Ws, bs = W.mlp_init(5, seed=seed, widths=(96, 256, 256, N))
    return q.SurrogateMLP(N, freqs, q.flatten_mlp_params(Ws, bs)), freqs


@pytest.fixture(scope="module")
def small_table(q, torch):
    rng = np.random.default_rng(31)
    grid = (12, 12, 12)
    G, a, b = W.planewave_params(rng, 192)
    coefs = W.fit_planewave_coefs(grid, G, a, b)
    return grid, coefs, q.Spline(grid, coefs, "f32")


def test_forward_matches_oracle(torch, q, oracle, small_table):
    grid, coefs, spl = small_table
    net, _ = _net(q, 192)
    pos_np = np.random.default_rng(1).random((1000 + 7, 3))
    pos = torch.from_numpy(pos_np).cuda()
    net.init_output(spl.eval_vgl(pos))
    _say("case mlp forward")
    got = [t.cpu().numpy() for t in net.forward(pos)]
    p = net.params_numpy()
    emu = M.forward(p, pos_np, bf16=True)
    exact = M.forward(p, pos_np)
    e_emu = [oracle.rel_err(g, r) for g, r in zip(got, emu)]
    e_ex = [oracle.rel_err(g, r) for g, r in zip(got, exact)]
    _say("mlp forward vs BF16-emulated oracle eps V/G/L = %.2e %.2e %.2e" % tuple(e_emu))
    _say("mlp forward vs exact FP64 network eps V/G/L = %.2e %.2e %.2e" % tuple(e_ex))
    assert max(e_emu) <= 2.0 ** -7


@pytest.mark.parametrize("N,B", [(16, 1), (64, 17), (128, 31), (160, 5), (208, 19), (240, 33), (256, 47), (256, 16)])
def test_forward_widths_and_ragged_batches(torch, q, oracle, N, B):
    """Every output-block count (1 to 4 blocks of 16 per wave, the last wave's
    share partial at 160), outputs staged through LDS (up to 208 orbitals) and
    stored directly (240, 256), and batches that end inside a workgroup's 16
    positions."""
    net, _ = _net(q, N, seed=11)
    pos_np = np.random.default_rng(N + B).random((B, 3))
    _say("case mlp forward N=%d B=%d" % (N, B))
    got = [t.cpu().numpy() for t in net.forward(torch.from_numpy(pos_np).cuda())]
    emu = M.forward(net.params_numpy(), pos_np, bf16=True)
    e = [oracle.rel_err(g, r) for g, r in zip(got, emu)]
    _say("eps V/G/L = %.2e %.2e %.2e" % tuple(e))
    assert all(np.isfinite(g).all() for g in got)
    assert max(e) <= 2.0 ** -7


def test_forward_full_batch_sampled(torch, q, oracle):
    """The 48^3 / N=192 table's surrogate on its full batch (256 walkers x 192
    electrons = 49152 positions, the benchmark's launch: 3072 workgroups),
    output map set from the table's VGL: 512 sampled rows against the
    BF16-model oracle, at the same 2^-7 bar."""
    grid, N, coefs, _ = W.make_table(5)
    spl = q.Spline(grid, coefs, "f32")
    _, Ws, bs = W.mlp_init(5)
    net = q.SurrogateMLP(N, q.spectral_frequencies(coefs), q.flatten_mlp_params(Ws, bs))
    pos_np = W.make_positions(5)
    pos = torch.from_numpy(pos_np).cuda()
    net.init_output(spl.eval_vgl(pos[:4096]))
    _say("case mlp forward, full batch B=%d" % pos_np.shape[0])
    got = [t.cpu().numpy() for t in net.forward(pos)]
    idx = np.sort(np.random.default_rng(3).choice(pos_np.shape[0], 512, replace=False))
    emu = M.forward(net.params_numpy(), pos_np[idx], bf16=True)
    e = [oracle.rel_err(g[idx], r) for g, r in zip(got, emu)]
    _say("eps V/G/L on 512 sampled rows = %.2e %.2e %.2e" % tuple(e))
    assert all(np.isfinite(g).all() for g in got)
    assert max(e) <= 2.0 ** -7


def _set_loss_weights(torch, net, w):
    lay = net.layout
    net.buf[lay.loss_w:lay.loss_w + 12] = torch.tensor(w, dtype=torch.float32).view(torch.uint8).to(net.buf.device)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_init_output_matches_oracle(torch, q, oracle, small_table):
    """mu, sd and the loss weights set on the device from a target batch
    equal the oracle's output_normalisation of the same FP32 targets.  The
    device sums in FP64 and stores FP32, so 1e-6 relative is 16 FP32 ulps."""
    grid, coefs, spl = small_table
    net, _ = _net(q, 192, seed=8)
    pos_np = np.random.default_rng(9).random((3000, 3))
    tgt = spl.eval_vgl(torch.from_numpy(pos_np).cuda())
    net.init_output(tgt)
    p = net.params_numpy()
    tV, tG, tL = (t.cpu().numpy().astype(np.float64) for t in tgt)
    mu, sd, w = M.output_normalisation(tV, tG, tL)
    _say("case init_output: max |dmu|/sd %.2e, sd %.2e, w %s vs %s" % (
        np.max(np.abs(p["mu"] - mu) / sd), np.max(np.abs(p["sd"] / sd - 1)), p["loss_w"][:3], w))
    assert np.all(np.abs(p["mu"] - mu) <= 1e-6 * (sd + np.abs(mu)))
    np.testing.assert_allclose(p["sd"], sd, rtol=1e-6)
    np.testing.assert_allclose(p["loss_w"][:3], w, rtol=1e-6)


def test_gradient_matches_oracle(torch, q, oracle, small_table):
    """The training gradient against the oracle's reverse pass under the same
    BF16 arithmetic model (every product operand rounded to BF16).  What is
    left between the two is FP32 against FP64 arithmetic in the SiLU streams,
    the loss and the accumulations, and the rare BF16 rounding that the
    slightly different FP32 value sends to the neighbouring BF16 number
    (probability ~1e-6 / 2^-9 per operand, each a 2^-8 change of one term):
    ~1e-4 relative L2 (measured 1e-5 to 2e-4).  Gate 1e-3 per tensor, for the whole loss and for each
    of its three terms alone (loss weights (1,0,0), (0,1,0), (0,0,1)), so a
    dropped G or L contribution cannot hide behind the V term.  The gap to
    the exact FP64 reverse pass (the cost of BF16 operands) is reported."""
    grid, coefs, spl = small_table
    net, _ = _net(q, 192, seed=6)
    pos_np = np.random.default_rng(2).random((256, 3))
    pos = torch.from_numpy(pos_np).cuda()
    tgt = spl.eval_vgl(pos)
    net.init_output(tgt)
    w_init = net.params_numpy()["loss_w"][:3].copy()
    tV, tG, tL = (t.cpu().numpy().astype(np.float64) for t in tgt)
    lay = net.layout
    for case, w in (("all", w_init), ("V", [1.0, 0.0, 0.0]), ("G", [0.0, w_init[1], 0.0]),
                    ("L", [0.0, 0.0, w_init[2]])):
        _set_loss_weights(torch, net, [float(x) for x in w])
        _say("case mlp grad, loss terms %s" % case)
        g, loss = net.grad(pos, tgt)
        torch.cuda.synchronize()
        g = g.cpu().numpy().astype(np.float64)
        p = net.params_numpy()
        wd = p["loss_w"][:3]
        lem, gem = M.loss_and_grads(p, pos_np, tV, tG, tL, wd, bf16=True)
        l64, g64 = M.loss_and_grads(p, pos_np, tV, tG, tL, wd)
        lg = float(loss.cpu()[0])
        _say("  loss gpu %.6g, BF16-model oracle %.6g, FP64 oracle %.6g" % (lg, lem, l64))
        assert abs(lg - lem) <= 1e-4 * lem
        for name, lo, hi in (("W1", lay.W1, lay.b1), ("b1", lay.b1, lay.W2), ("W2", lay.W2, lay.b2),
                             ("b2", lay.b2, lay.W3), ("W3", lay.W3, lay.b3), ("b3", lay.b3, lay.n_params)):
            if not np.any(gem[name]):  # b3 has no part in the G or L terms: exactly zero
                _say("  grad %s: zero in the oracle, max |gpu| %.3g" % (name, np.abs(g[lo:hi]).max()))
                assert not np.any(g[lo:hi]), (case, name)
                continue
            e_em = _rel_l2(g[lo:hi], gem[name].ravel())
            e_64 = _rel_l2(g[lo:hi], g64[name].ravel())
            _say("  grad %s rel L2 vs BF16 model %.3e (vs FP64 %.3e)" % (name, e_em, e_64))
            assert e_em <= 1e-3, (case, name)
    _set_loss_weights(torch, net, [float(x) for x in w_init])


def _errmap_setup(torch, q, cell, empty_bin=77, nb=8, per_bin=12, seed=21):
    """A small table in a non-cubic cell, a network over it, and validation
    positions: per_bin points in every bin but one, shifted by whole periods
    (negative and beyond one), plus points exactly on bin edges."""
    rng = np.random.default_rng(seed)
    grid = (10, 12, 8)
    G, a, b = W.planewave_params(rng, 64)
    coefs = W.fit_planewave_coefs(grid, G, a, b)
    spl = q.Spline(grid, coefs, "f32", cell=cell)
    freqs, Ws, bs = W.mlp_init(5, seed=seed, widths=(96, 256, 256, 64))
    net = q.SurrogateMLP(64, freqs, q.flatten_mlp_params(Ws, bs), cell=cell)
    cellv = np.asarray(cell)
    idx = np.arange(nb ** 3)
    idx = idx[idx != empty_bin]
    ijk = np.stack([idx // (nb * nb), (idx // nb) % nb, idx % nb], 1)
    frac = (np.repeat(ijk, per_bin, 0) + rng.random((len(idx) * per_bin, 3))) / nb
    shift = rng.integers(-2, 3, frac.shape)
    val = (frac + shift) * cellv
    # bin edges: lower edges exactly (they belong to the bin above), not in the empty bin
    edges = np.array([[1, 2, 3], [4, 0, 7], [7, 7, 7], [0, 0, 0]]) / nb
    val = np.concatenate([val, edges * cellv, (edges - 1.0) * cellv])
    net.init_output(spl.eval_vgl(torch.from_numpy(rng.random((4096, 3)) * cellv).cuda()))
    return spl, net, val, rng


def test_error_map_matches_oracle(torch, q, oracle):
    """The device's error map against the oracle's, from the same network and
    spline outputs at the validation positions (both deterministic): finite
    bins within 4 FP32 ulps (each is |a - b| / s in FP32), the empty bin and
    only it +inf; a NaN validation position poisons every normaliser, so
    every bin is +inf on both sides."""
    cell = (1.0, 1.3, 0.8)
    nb = 8
    spl, net, val, _ = _errmap_setup(torch, q, cell)
    vd = torch.from_numpy(val).cuda()
    _say("case error map, %d validation positions, cell %s" % (len(val), cell))
    net.build_error_map(spl, vd, bins_per_dim=nb)
    torch.cuda.synchronize()
    got = net.buf[net.layout.bin_err:net.layout.bin_err + 4 * nb ** 3].cpu().numpy().view(np.float32).astype(np.float64)
    netv = [t.cpu().numpy() for t in net.forward(vd)]
    splv = [t.cpu().numpy() for t in spl.eval_vgl(vd)]
    want = M.error_map(netv, splv, val, nb, cell)
    fin = np.isfinite(want)
    assert list(np.flatnonzero(~fin)) == [77]
    np.testing.assert_array_equal(np.isfinite(got), fin)
    rel = np.abs(got[fin] - want[fin]) / want[fin]
    _say("  bins: max rel diff %.2e, values %.3g .. %.3g" % (rel.max(), want[fin].min(), want[fin].max()))
    assert rel.max() <= 2.0 ** -21
    # a NaN validation position: every bin +inf
    val2 = np.concatenate([val, [[np.nan, 0.1, 0.2]]])
    net.build_error_map(spl, torch.from_numpy(val2).cuda(), bins_per_dim=nb)
    torch.cuda.synchronize()
    got2 = net.buf[net.layout.bin_err:net.layout.bin_err + 4 * nb ** 3].cpu().numpy().view(np.float32)
    netv2 = [t.cpu().numpy() for t in net.forward(torch.from_numpy(val2).cuda())]
    splv2 = [t.cpu().numpy() for t in spl.eval_vgl(torch.from_numpy(val2).cuda())]
    assert np.isinf(M.error_map(netv2, splv2, val2, nb, cell)).all()
    assert np.isinf(got2).all() and (got2 > 0).all()


def test_routing_matches_oracle(torch, q, oracle):
    """Which positions the fallback takes: the oracle's routed set (from the
    device's FP32 map, compared in FP32) equals the device's exactly -- the
    count, the rows that equal the spline bit for bit, and the rows that equal
    the network bit for bit (every test row differs between the two, so the
    rows pin the set).  Tolerances: between neighbouring bin values, exactly
    on a bin value (kept), below all (all routed), +inf (nothing routed, the
    empty bin included: inf <= inf), and a tolerance between two bins of
    the oracle's own FP64 map, where the oracle's map decides alone.  Test
    positions include negative coordinates, coordinates beyond one period and
    bin edges."""
    cell = (1.0, 1.3, 0.8)
    nb = 8
    spl, net, val, rng = _errmap_setup(torch, q, cell)
    vd = torch.from_numpy(val).cuda()
    net.build_error_map(spl, vd, bins_per_dim=nb)
    bmap = net.buf[net.layout.bin_err:net.layout.bin_err + 4 * nb ** 3].cpu().numpy().view(np.float32).copy()
    netv = [t.cpu().numpy() for t in net.forward(vd)]
    splv = [t.cpu().numpy() for t in spl.eval_vgl(vd)]
    omap = M.error_map(netv, splv, val, nb, cell)
    cellv = np.asarray(cell)
    test = np.concatenate([(rng.random((3000, 3)) * 5.0 - 2.5) * cellv,
                           np.array([[0, 0, 0], [1, 1, 1], [-1e-17, 0.5, 0.25], [0.125, 0.25, 0.875]]) * cellv,
                           np.array([[77 // 64 + 0.5, (77 // 8) % 8 + 0.5, 77 % 8 + 0.5]]) / nb * cellv])
    td = torch.from_numpy(test).cuda()
    B = len(test)
    ref = [t.cpu().numpy() for t in spl.eval_vgl(td)]
    plain = [t.cpu().numpy() for t in net.forward(td)]
    assert not np.any(np.all(ref[0] == plain[0], axis=1))
    fin = np.sort(bmap[np.isfinite(bmap)])
    mids = [float((fin[i] + fin[i + 1]) / 2) for i in (len(fin) // 4, len(fin) // 2, 3 * len(fin) // 4)]
    ofin = np.sort(omap[np.isfinite(omap)])
    gaps = np.diff(ofin) / ofin[1:]
    j = int(np.argmax(gaps[len(gaps) // 3:])) + len(gaps) // 3
    otol = float((ofin[j] + ofin[j + 1]) / 2)
    cases = [(t, bmap) for t in mids + [float(fin[len(fin) // 3]), -1.0, float("inf")]] + [(otol, omap)]
    for tol, m in cases:
        want = M.route(test, m, nb, tol, cell)
        _say("case routing tol %.6g (%s map): oracle routes %d of %d" % (tol, "device" if m is bmap else "oracle",
                                                                          len(want), B))
        V, G, L, nf = net.eval_vgl(td, fallback=spl, tol=tol)
        torch.cuda.synchronize()
        assert int(nf.cpu()[0]) == len(want)
        V, G, L = V.cpu().numpy(), G.cpu().numpy(), L.cpu().numpy()
        routed = np.zeros(B, bool)
        routed[want] = True
        for got, r, pl in zip((V, G, L), ref, plain):
            np.testing.assert_array_equal(got[routed], r[routed])
            np.testing.assert_array_equal(got[~routed], pl[~routed])
    assert len(M.route(test, bmap, nb, float("inf"), cell)) == 0


def test_training_error_map_fallback_and_resume(torch, q, oracle, small_table):
    grid, coefs, spl = small_table
    net, _ = _net(q, 192, seed=7)
    rng = np.random.default_rng(3)
    train = torch.from_numpy(rng.random((4096 * 8, 3))).cuda()
    val = torch.from_numpy(rng.random((8 * 8 * 8 * 16, 3))).cuda()
    net.init_output(spl.eval_vgl(train[:4096]))
    loss = torch.zeros(1, device="cuda")
    losses = []
    for step in range(300):
        pos = train[(step % 8) * 4096:(step % 8 + 1) * 4096]
        net.train_step(pos, spl.eval_vgl(pos), lr=1e-3 * (0.5 + 0.5 * np.cos(np.pi * step / 300)), loss_out=loss)
        if step % 50 == 0 or step == 299:
            losses.append(float(loss.cpu()[0]))
    _say("case mlp training losses", ["%.3g" % x for x in losses])
    assert losses[-1] < 0.5 * losses[0]
    assert net.info()["step"] == 300

    net.build_error_map(spl, val, bins_per_dim=8)
    assert net.info()["bins_per_dim"] == 8
    pos = torch.from_numpy(rng.random((5000, 3))).cuda()
    ref = spl.eval_vgl(pos)
    plain = net.forward(pos)
    # tolerance below every bin error: everything is routed -> spline exactly
    V, G, L, nf = net.eval_vgl(pos, fallback=spl, tol=-1.0)
    torch.cuda.synchronize()
    assert int(nf.cpu()[0]) == 5000
    for a, b in zip((V, G, L), ref):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    # a tolerance between bin errors: routed rows equal the spline, the rest the network
    errs = np.sort(net.buf[net.layout.bin_err:net.layout.bin_err + 4 * 512].cpu().numpy().view(np.float32))
    tol = float(errs[len(errs) // 2])
    V, G, L, nf = net.eval_vgl(pos, fallback=spl, tol=tol)
    torch.cuda.synchronize()
    n = int(nf.cpu()[0])
    _say("mlp bins median error %.3e, routed %d of 5000" % (tol, n))
    assert 0 < n < 5000
    same_spl = np.all(V.cpu().numpy() == ref[0].cpu().numpy(), axis=1)
    same_net = np.all(V.cpu().numpy() == plain[0].cpu().numpy(), axis=1)
    assert (same_spl | same_net).all() and same_spl.sum() >= n
    # no fallback table: network only
    V2, _, _, _ = net.eval_vgl(pos, fallback=None)
    np.testing.assert_array_equal(V2.cpu().numpy(), plain[0].cpu().numpy())
    # a tolerance above every bin error: nothing is routed -> network exactly
    V3, G3, L3, nf3 = net.eval_vgl(pos, fallback=spl, tol=float(errs[-1]) * 2 + 1.0)
    torch.cuda.synchronize()
    assert int(nf3.cpu()[0]) == 0
    for a, b in zip((V3, G3, L3), plain):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())

    # resume from a saved state
    st = net.state()
    net2 = q.SurrogateMLP(192, state=st)
    assert net2.info() == net.info()
    for a, b in zip(net2.forward(pos), plain):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    # the resumed network routes by the same map
    V4, _, _, nf4 = net2.eval_vgl(pos, fallback=spl, tol=tol)
    torch.cuda.synchronize()
    assert int(nf4.cpu()[0]) == n
    np.testing.assert_array_equal(V4.cpu().numpy(), V.cpu().numpy())
    net2.train_step(pos[:4096], spl.eval_vgl(pos[:4096]), lr=1e-4)
    assert net2.info()["step"] == 301


def test_surrogate_gain_over_the_table(torch, q, oracle):
    """What the trained network gains over the method without it, on the
    48^3 / N=192 table: a footprint hundreds of times smaller than the table,
    and, at a fixed error tolerance, a part of the cell served by the network
    alone.  At the median bin error of the map t, the routed fraction of
    held-out positions is strictly between 0 and 1, and the combined path's
    error against the spline on the positions it did not route stays within
    2t (the map is an empirical maximum over 64 validation points per bin, so
    new points may exceed it a little).  Timing is the benchmark's job."""
    grid, N, coefs, _ = W.make_table(5)
    spl = q.Spline(grid, coefs, "f32")
    _, Ws, bs = W.mlp_init(5)
    net = q.SurrogateMLP(N, q.spectral_frequencies(coefs), q.flatten_mlp_params(Ws, bs))
    train = torch.from_numpy(W.mlp_samples(5, count=4096 * 50)).cuda()
    net.init_output(spl.eval_vgl(train[:4096]))
    val = torch.from_numpy(W.mlp_samples(5, count=8 * 8 * 8 * 64 + 20000, validation=True)).cuda()
    hv = val[8 * 8 * 8 * 64:]
    ref = [t.cpu().numpy() for t in spl.eval_vgl(hv)]
    e0 = [oracle.rel_err(a.cpu().numpy(), b) for a, b in zip(net.forward(hv), ref)]
    for step in range(400):
        pos = train[(step % 50) * 4096:(step % 50 + 1) * 4096]
        net.train_step(pos, spl.eval_vgl(pos), lr=5e-3 * 0.5 * (1 + np.cos(np.pi * step / 400)) + 1e-5)
    net_out = [a.cpu().numpy() for a in net.forward(hv)]
    e1 = [oracle.rel_err(a, b) for a, b in zip(net_out, ref)]
    table_bytes = spl.layout.total_bytes
    net_bytes = net.layout.n_params * 2
    _say("surrogate: table %.1f MB, network %.0f KB (%.0fx); eps V/G/L untrained %.3g %.3g %.3g, trained %.3g %.3g %.3g"
         % ((table_bytes / 1e6, net_bytes / 1e3, table_bytes / net_bytes) + tuple(e0) + tuple(e1)))
    assert table_bytes > 300 * net_bytes
    assert all(b < a for a, b in zip(e0, e1))  # training moved every quantity toward the table

    net.build_error_map(spl, val[:8 * 8 * 8 * 64], bins_per_dim=8)
    bmap = net.buf[net.layout.bin_err:net.layout.bin_err + 4 * 512].cpu().numpy().view(np.float32)
    tol = float(np.median(bmap))
    V, G, L, nf = net.eval_vgl(hv, fallback=spl, tol=tol)
    torch.cuda.synchronize()
    frac = int(nf.cpu()[0]) / hv.shape[0]
    hv_np = hv.cpu().numpy()
    routed = np.zeros(hv.shape[0], bool)
    routed[M.route(hv_np, bmap, 8, tol)] = True
    assert routed.sum() == int(nf.cpu()[0])
    # point errors of the combined output on the rows served by the network,
    # normalised as the map is (each orbital's largest |Q| of the spline)
    comb = [x.cpu().numpy() for x in (V, G, L)]
    pe = M.point_errors(comb, ref)
    worst = float(pe[~routed].max())
    _say("surrogate at tol %.3g (median bin error): routed %.1f%% of held-out positions, worst unrouted error %.3g "
         "(%.2f tol), routed rows exact: %s" % (tol, 100 * frac, worst, worst / tol, float(pe[routed].max()) == 0.0))
    assert 0.0 < frac < 1.0
    assert float(pe[routed].max()) == 0.0
    assert worst <= 2.0 * tol
