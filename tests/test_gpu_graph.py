"""The kernels of one particle-by-particle step can be captured in a HIP
graph: the determinant ratio with derivatives, the Jastrow move, the
Sherman-Morrison update and the Jastrow accept (a slot with k = -1 is a
rejected move, which both update kernels skip); so can the delayed update,
the locality-ordered evaluation and the surrogate with its spline fallback.  The graph is replayed
several times with eager work and synchronisations in between, and every
replay must equal, bit for bit, the same calls made eagerly on the same
inputs.  No call in the sequence allocates or clears memory.
"""
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


def test_pbyp_step_in_a_graph(torch, q):
    grid, N, coefs, _ = W.make_table(1)  # 16^3, 32 orbitals
    s = q.Spline(grid, coefs, "f32")
    jd = W.make_jastrow(n_elec=N, n_up=N // 2)
    jas = q.Jastrow(jd["cell"], jd["ions"], jd["species"], jd["f1"], jd["uu"], jd["ud"], N, N // 2)
    Wn = 64
    rng = np.random.default_rng(8)
    R0 = W.make_electrons(Wn, N)
    inv0 = (np.eye(N) + 0.1 * rng.normal(size=(Wn, N, N)) / np.sqrt(N)).astype(np.float32)
    inv0 = np.linalg.inv(inv0).astype(np.float32)
    k = 7
    rnew = R0[:, k] + rng.normal(scale=0.03, size=(Wn, 3))
    kacc = np.where(rng.random(Wn) < 0.7, k, -1).astype(np.int32)  # accepted slots keep k, rejected -1
    dev = torch.device("cuda")
    pos = torch.from_numpy(rnew).to(dev)
    kk = torch.full((Wn,), k, dtype=torch.int32, device=dev)
    ka = torch.from_numpy(kacc).to(dev)
    phi = s.eval_v(pos)  # orbital values at the proposals (input of the update)

    def fresh():
        return torch.from_numpy(inv0.copy()).to(dev), jas.positions(R0)

    D = torch.empty((Wn, 5), dtype=torch.float32, device=dev)
    J = torch.empty((Wn, 5), dtype=torch.float32, device=dev)

    def step(ainv, R):
        s.eval_ratio_vgl(pos, ainv.view(-1)[k * N:], ld=N * N, out=D)
        jas.move(R, kk, pos, out=J)
        q.det_update(ainv, ka, phi)
        jas.accept(R, ka, pos)

    ainv_e, R_e = fresh()
    step(ainv_e, R_e)
    torch.cuda.synchronize()
    ref = [t.cpu().numpy().copy() for t in (D, J, ainv_e, R_e)]
    assert np.isfinite(ref[0]).all() and np.isfinite(ref[1]).all()
    # rejected walkers are untouched, accepted ones moved
    rej = kacc < 0
    np.testing.assert_array_equal(ref[2][rej], inv0[rej])
    assert not np.array_equal(ref[2][~rej], inv0[~rej])

    ainv_g, R_g = fresh()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        step(ainv_g, R_g)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step(ainv_g, R_g)
    for rep in range(3):
        a_new, r_new = fresh()
        ainv_g.copy_(a_new)
        R_g.copy_(r_new)
        D.zero_()
        J.zero_()
        torch.cuda.synchronize()
        _ = s.eval_vgl(pos)  # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in (D, J, ainv_g, R_g)]
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)


def test_delayed_batch_in_a_graph(torch, q):
    """Four moves through the delayed update (ratio with derivatives against
    the pending moves, accept of a subset of walkers) and the flush, captured
    once and replayed: every replay equals the eager sequence bit for bit.
    The flush clears the pending moves, so each replay starts from none."""
    grid, N, coefs, _ = W.make_table(1)  # 16^3, 32 orbitals
    s = q.Spline(grid, coefs, "f32")
    Wn, moves = 64, 4
    rng = np.random.default_rng(9)
    inv0 = np.linalg.inv(np.eye(N) + 0.3 * rng.normal(size=(Wn, N, N)) / np.sqrt(N)).astype(np.float32)
    dev = torch.device("cuda")
    pos = [torch.from_numpy(rng.random((Wn, 3))).to(dev) for _ in range(moves)]
    kk = [torch.full((Wn,), 3 * i + 1, dtype=torch.int32, device=dev) for i in range(moves)]
    ka = [torch.from_numpy(np.where(rng.random(Wn) < 0.7, 3 * i + 1, -1).astype(np.int32)).to(dev)
          for i in range(moves)]
    vgl = [s.eval_vgl(p) for p in pos]
    D = [torch.empty((Wn, 5), dtype=torch.float32, device=dev) for _ in range(moves)]

    def batch(dl, ainv):
        for i in range(moves):
            V, G, L = vgl[i]
            dl.ratio(ainv, kk[i], V, G, L, out=D[i])
            dl.accept(ainv, ka[i], V)
        dl.flush(ainv)

    dl_e = q.DelayedUpdate(N, moves, Wn)
    a_e = torch.from_numpy(inv0.copy()).to(dev)
    batch(dl_e, a_e)
    torch.cuda.synchronize()
    ref = [d.cpu().numpy().copy() for d in D] + [a_e.cpu().numpy()]
    assert all(np.isfinite(r).all() for r in ref)

    dl_g = q.DelayedUpdate(N, moves, Wn)
    a_g = torch.from_numpy(inv0.copy()).to(dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch(dl_g, a_g)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch(dl_g, a_g)
    for rep in range(3):
        a_g.copy_(torch.from_numpy(inv0).to(dev))
        for d in D:
            d.zero_()
        torch.cuda.synchronize()
        _ = s.eval_vgl(pos[0])  # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        got = [d.cpu().numpy() for d in D] + [a_g.cpu().numpy()]
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)


def test_sorted_evaluation_in_a_graph(torch, q):
    """The locality-ordered evaluation (device sort + indexed gather) captured
    in a HIP graph: replays equal the eager call bit for bit, also after the
    positions change between replays (the sort runs in every replay)."""
    rng = np.random.default_rng(10)
    grid = (20, 18, 16)
    s = q.Spline(grid, rng.uniform(-1, 1, grid + (96,)), "f32")
    B = 3000
    dev = torch.device("cuda")
    pos = torch.from_numpy(rng.random((B, 3))).to(dev)
    ws = torch.empty(q.lib().spline_sorted_workspace_bytes(s.handle, B), dtype=torch.uint8, device=dev)
    out = s.alloc_outputs(B)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        s.eval_vgl_sorted(pos, out=out, workspace=ws)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.eval_vgl_sorted(pos, out=out, workspace=ws)
    for rep in range(3):
        pos.copy_(torch.from_numpy(rng.random((B, 3))).to(dev))
        for t in out:
            t.zero_()
        torch.cuda.synchronize()
        ref = s.eval_vgl(pos)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_surrogate_in_a_graph(torch, q):
    """The surrogate's forward pass and its evaluation with spline fallback
    (network, routing of the untrusted bins, indexed spline gather) captured
    in one HIP graph: every replay, with new positions and eager work
    between replays, equals the eager calls bit for bit, the fallback count
    included."""
    rng = np.random.default_rng(12)
    grid = (12, 12, 12)
    N = 64
    G, a, b = W.planewave_params(rng, N)
    spl = q.Spline(grid, W.fit_planewave_coefs(grid, G, a, b), "f32")
    freqs, Ws, bs = W.mlp_init(5, seed=4, widths=(96, 256, 256, N))
    net = q.SurrogateMLP(N, freqs, q.flatten_mlp_params(Ws, bs))
    dev = torch.device("cuda")
    net.build_error_map(spl, torch.from_numpy(rng.random((8 * 8 * 8 * 16, 3))).to(dev), bins_per_dim=8)
    tol = float(np.median(net.bin_errors()))
    B = 2000
    pos = torch.from_numpy(rng.random((B, 3))).to(dev)
    out_f = net._out(B)
    out_e = net._out(B)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream: the workspace exists before capture
        net.forward(pos, out=out_f)
        net.eval_vgl(pos, fallback=spl, tol=tol, out=out_e)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        net.forward(pos, out=out_f)
        nf = net.eval_vgl(pos, fallback=spl, tol=tol, out=out_e)[3]
    for rep in range(3):
        pos.copy_(torch.from_numpy(rng.random((B, 3))).to(dev))
        for t in out_f + out_e:
            t.zero_()
        torch.cuda.synchronize()
        ref_f = net.forward(pos)  # eager work between replays
        *ref_e, ref_nf = net.eval_vgl(pos, fallback=spl, tol=tol)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        n_routed = int(nf.cpu()[0])
        assert n_routed == int(ref_nf.cpu()[0]) and 0 < n_routed < B, (rep, n_routed)
        for x, y in zip(out_f + out_e, tuple(ref_f) + tuple(ref_e)):
            np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
