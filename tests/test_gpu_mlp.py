"""GPU tests of the learned surrogate (forward-mode MLP on matrix cores).

- the fused forward kernel against the FP64 oracle with BF16 rounding of
  every product operand emulated (tolerance 2^-7, per-orbital max-norm), and
  against the exact FP64 network (reported);
- the training gradient against the oracle's hand-written reverse pass
  (FP64, no rounding): relative L2 error per tensor <= 5e-2 (BF16 operands);
- training lowers the loss; the error map routes; routed positions equal the
  spline bit for bit and the others equal the network bit for bit; routing
  everything reproduces the spline exactly;
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


def test_gradient_matches_oracle(torch, q, oracle, small_table):
    grid, coefs, spl = small_table
    net, _ = _net(q, 192, seed=6)
    pos_np = np.random.default_rng(2).random((256, 3))
    pos = torch.from_numpy(pos_np).cuda()
    tgt = spl.eval_vgl(pos)
    net.init_output(tgt)
    _say("case mlp grad")
    g, loss = net.grad(pos, tgt)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    p = net.params_numpy()
    tV, tG, tL = (t.cpu().numpy().astype(np.float64) for t in tgt)
    lval, gr = M.loss_and_grads(p, pos_np, tV, tG, tL, p["loss_w"])
    lay = net.layout
    _say("loss gpu %.6g oracle %.6g" % (float(loss.cpu()[0]), lval))
    assert abs(float(loss.cpu()[0]) - lval) <= 2e-2 * lval
    for name, lo, hi in (("W1", lay.W1, lay.b1), ("b1", lay.b1, lay.W2), ("W2", lay.W2, lay.b2),
                         ("b2", lay.b2, lay.W3), ("W3", lay.W3, lay.b3), ("b3", lay.b3, lay.n_params)):
        ref = gr[name].ravel()
        err = np.linalg.norm(g[lo:hi] - ref) / np.linalg.norm(ref)
        _say("grad %s rel L2 err %.3e" % (name, err))
        assert err <= 5e-2, name


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
    48^3 / N=192 table and its 256 x 192 batch: a footprint hundreds of times
    smaller than the table, and a faster evaluation of the batch (network
    only, median of timed launches), at an error against the spline that is
    measured and reported (it does not meet 1e-3: see the error map and the
    fallback test above)."""
    grid, N, coefs, _ = W.make_table(5)
    spl = q.Spline(grid, coefs, "f32")
    _, Ws, bs = W.mlp_init(5)
    net = q.SurrogateMLP(N, q.spectral_frequencies(coefs), q.flatten_mlp_params(Ws, bs))
    train = torch.from_numpy(W.mlp_samples(5, count=4096 * 50)).cuda()
    net.init_output(spl.eval_vgl(train[:4096]))
    hv = torch.from_numpy(W.mlp_samples(5, count=20000, validation=True)).cuda()
    ref = [t.cpu().numpy() for t in spl.eval_vgl(hv)]
    e0 = [oracle.rel_err(a.cpu().numpy(), b) for a, b in zip(net.forward(hv), ref)]
    for step in range(400):
        pos = train[(step % 50) * 4096:(step % 50 + 1) * 4096]
        net.train_step(pos, spl.eval_vgl(pos), lr=5e-3 * 0.5 * (1 + np.cos(np.pi * step / 400)) + 1e-5)
    e1 = [oracle.rel_err(a.cpu().numpy(), b) for a, b in zip(net.forward(hv), ref)]
    table_bytes = spl.layout.total_bytes
    net_bytes = net.layout.n_params * 2
    _say("surrogate: table %.1f MB, network %.0f KB (%.0fx); eps V/G/L untrained %.3g %.3g %.3g, trained %.3g %.3g %.3g"
         % ((table_bytes / 1e6, net_bytes / 1e3, table_bytes / net_bytes) + tuple(e0) + tuple(e1)))
    assert table_bytes > 300 * net_bytes
    assert all(b < a for a, b in zip(e0, e1))  # training moved every quantity toward the table

    pos = torch.from_numpy(W.make_positions(5)).cuda()
    out = net._out(pos.shape[0])
    sout = spl.alloc_outputs(pos.shape[0])
    spl.autotune(pos, reps=2, out=sout)

    def median_ms(fn, n=15):
        for _ in range(3):
            fn()
        ts = []
        for _ in range(n):
            e0_, e1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0_.record()
            fn()
            e1_.record()
            torch.cuda.synchronize()
            ts.append(e0_.elapsed_time(e1_))
        return float(np.median(ts))

    ms_net = median_ms(lambda: net.forward(pos, out=out))
    ms_spl = median_ms(lambda: spl.eval_vgl(pos, out=sout))
    _say("surrogate: network %.3f ms vs spline %.3f ms on %d positions (%.2fx)" % (ms_net, ms_spl, pos.shape[0],
                                                                                  ms_spl / ms_net))
    assert ms_net * 1.3 < ms_spl
