"""GPU parity of the delayed (Woodbury) determinant update (spline_dlu_*)
against the oracle (oracle/det.py: delayed_ratio, delayed_flush).

The oracle runs the same sequence of moves in FP64 with its own orbital
values (oracle.eval_vgl at the same positions) and its own stale inverse;
the accept/reject pattern is fixed in advance.  Error measures: a ratio or
derivative sum against sum |a_k| |q| + sum |u_l| |y_l| (the sizes of the terms
it is formed from); a flushed inverse against its largest entry.  Bars: 1e-4
for one batch of pending moves on well-conditioned matrices (FP32; up to
`delay` bordering steps, each a few roundings relative to those sizes); over
a sweep of real Slater matrices the FP32 state drifts from the FP64 one like
any repeated update, so there the error is held to (steps) n u cond(A), the
drift bound used for the Sherman-Morrison sweep (u = 2^-24).
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-4


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


def _scale(a0, phis, ks, k, qv):
    """sum |a_k||q| + sum_l |u_l||y_l| per row of qv (u = t^T S^-1)."""
    a0 = np.asarray(a0)
    base = np.abs(qv) @ np.abs(a0[k])
    if not ks:
        return base
    P = np.asarray(phis).reshape(len(ks), -1)
    R = a0[list(ks)]
    u = np.linalg.solve((R @ P.T).T, P @ a0[k])
    return base + np.abs(qv @ R.T) @ np.abs(u)


def test_sweep_with_real_slater_matrices(torch, q, oracle):
    from oracle import det

    grid, n, coefs, _ = W.make_table(1)  # 16^3, 32 orbitals = electrons
    s = q.Spline(grid, coefs, "f32")
    Wn, delay = 4, 8
    rng = np.random.default_rng(12)
    R = rng.random((Wn, n, 3))
    ainv_ref = [np.linalg.inv(det.slater_matrix(grid, coefs, R[w])) for w in range(Wn)]
    ainv = torch.from_numpy(np.stack(ainv_ref).astype(np.float32)).cuda()
    dl = q.DelayedUpdate(n, delay, Wn)
    pend = [([], []) for _ in range(Wn)]  # oracle's pending (phis, ks) per walker
    worst_r, worst_f = 0.0, 0.0
    u32 = 2.0 ** -24

    def bound(step):
        return (step + 1) * n * u32 * max(np.linalg.cond(det.slater_matrix(grid, coefs, R[w])) for w in range(Wn))

    for k in range(20):
        if k % delay == 0 and k > 0:
            dl.flush(ainv)
            for w in range(Wn):
                ainv_ref[w] = det.delayed_flush(ainv_ref[w], *pend[w])
                pend[w] = ([], [])
            got = ainv.cpu().numpy().astype(np.float64)
            for w in range(Wn):
                worst_f = max(worst_f, float(np.max(np.abs(got[w] - ainv_ref[w])) / np.max(np.abs(ainv_ref[w])))
                              / bound(k))
        rnew = R[:, k] + rng.normal(scale=0.03, size=(Wn, 3))
        acc = rng.random(Wn) < 0.75
        pos = torch.from_numpy(rnew).cuda()
        V, G, L = s.eval_vgl(pos)
        kd = torch.full((Wn,), k, dtype=torch.int32, device="cuda")
        D = dl.ratio(ainv, kd, V, G, L).cpu().numpy().astype(np.float64)
        Vr, Gr, Lr = oracle.eval_vgl(grid, coefs, rnew)
        for w in range(Wn):
            qv = np.vstack([Vr[w], Gr[w], Lr[w]])
            ref = det.delayed_ratio(ainv_ref[w], pend[w][0], pend[w][1], k, qv)
            sc = _scale(ainv_ref[w], pend[w][0], pend[w][1], k, qv)
            worst_r = max(worst_r, float(np.max(np.abs(D[w] - ref) / sc)) / bound(k))
        ka = torch.from_numpy(np.where(acc, k, -1).astype(np.int32)).cuda()
        dl.accept(ainv, ka, V)
        for w in range(Wn):
            if acc[w]:
                pend[w][0].append(Vr[w])
                pend[w][1].append(k)
                R[w, k] = rnew[w]
    dl.flush(ainv)
    got = ainv.cpu().numpy().astype(np.float64)
    for w in range(Wn):
        ainv_ref[w] = det.delayed_flush(ainv_ref[w], *pend[w])
        worst_f = max(worst_f, float(np.max(np.abs(got[w] - ainv_ref[w])) / np.max(np.abs(ainv_ref[w])))
                      / bound(20))
        # the result is the inverse of the Slater matrix of the final positions
        A = det.slater_matrix(grid, coefs, R[w])
        assert np.max(np.abs(got[w] @ A - np.eye(n))) < 1e-3
    _say("delayed sweep: ratio and flush error / drift bound: %.3f, %.3f" % (worst_r, worst_f))
    assert worst_r < 1.0 and worst_f < 1.0


# flush paths, all with <= 16 pending moves unless noted: matrix cores for n
# a multiple of 16 up to 384 (384 and 128: exact 24- and 8-tile builds; 64
# with 12 moves; 144 and 96: 9 and 6 tiles of a guarded 12-tile build); one
# vector pass for other n % 4 == 0 up to 512 (260: ragged column chunk and
# row block; 512); separate T and update passes otherwise (129, 37: n not a
# multiple of 4; 200 with 20 moves)
@pytest.mark.parametrize("n,delay,walkers", [(384, 16, 64), (128, 16, 4), (64, 12, 7), (144, 16, 6), (96, 8, 5),
                                             (260, 16, 5), (512, 16, 3), (129, 5, 9), (37, 37, 3), (200, 20, 4)])
def test_synthetic_against_oracle_and_sherman_morrison(torch, q, n, delay, walkers):
    """Well-conditioned synthetic inverses, `delay` accepted moves of distinct
    electrons per walker, then a flush; compared with the oracle and with the
    same moves applied one by one by spline_det_update."""
    from oracle import det

    rng = np.random.default_rng(n)
    A = np.eye(n) + rng.normal(size=(walkers, n, n)) * (0.3 / np.sqrt(n))
    inv0 = np.linalg.inv(A).astype(np.float32)
    ks = np.stack([rng.permutation(n)[:delay] for _ in range(walkers)]).astype(np.int32)
    phis = np.empty((walkers, delay, n))
    cur = A.copy()
    for w in range(walkers):
        for i in range(delay):
            phis[w, i] = cur[w][:, ks[w, i]] + rng.normal(size=n) * 0.2
            cur[w][:, ks[w, i]] = phis[w, i]
    phis32 = phis.astype(np.float32)
    a_d = torch.from_numpy(inv0.copy()).cuda()
    a_s = torch.from_numpy(inv0.copy()).cuda()
    dl = q.DelayedUpdate(n, delay, walkers)
    worst = 0.0
    for i in range(delay):
        kd = torch.from_numpy(np.ascontiguousarray(ks[:, i])).cuda()
        Vd = torch.from_numpy(np.ascontiguousarray(phis32[:, i])).cuda()
        r = dl.ratio(a_d, kd, Vd).cpu().numpy().astype(np.float64)
        for w in range(0, walkers, max(1, walkers // 8)):
            ref = det.delayed_ratio(inv0[w].astype(np.float64), phis32[w, :i].astype(np.float64), list(ks[w, :i]),
                                    int(ks[w, i]), phis32[w, i].astype(np.float64))
            sc = _scale(inv0[w].astype(np.float64), phis32[w, :i].astype(np.float64), list(ks[w, :i]), int(ks[w, i]),
                        phis32[w, i][None].astype(np.float64))
            worst = max(worst, float(np.abs(r[w] - ref) / sc[0]))
        dl.accept(a_d, kd, Vd)
        q.det_update(a_s, kd, Vd)
    with pytest.raises(q.SplineError):
        dl.accept(a_d, kd, Vd)  # delay reached
    dl.flush(a_d)
    got = a_d.cpu().numpy().astype(np.float64)
    sm = a_s.cpu().numpy().astype(np.float64)
    ferr = 0.0
    for w in range(walkers):
        ref = det.delayed_flush(inv0[w].astype(np.float64), phis32[w].astype(np.float64), list(ks[w]))
        ferr = max(ferr, float(np.max(np.abs(got[w] - ref)) / np.max(np.abs(ref))))
    smerr = float(np.max(np.abs(got - sm)) / np.max(np.abs(sm)))
    _say("delayed n=%d d=%d: ratio %.2e flush %.2e vs SM %.2e" % (n, delay, worst, ferr, smerr))
    assert worst <= TOL and ferr <= TOL and smerr <= 4 * TOL
    # after the flush no move is pending: plain ratios again
    kd = torch.from_numpy(np.ascontiguousarray(ks[:, 0])).cuda()
    Vd = torch.from_numpy(np.ascontiguousarray(phis32[:, 0])).cuda()
    r = dl.ratio(a_d, kd, Vd).cpu().numpy()
    plain = np.einsum("wn,wn->w", got[np.arange(walkers), ks[:, 0]], phis32[:, 0].astype(np.float64))
    assert np.max(np.abs(r - plain) / (np.abs(got[np.arange(walkers), ks[:, 0]]) @ np.ones(n) + 1)) < 1e-5


def test_argument_errors(torch, q):
    with pytest.raises(q.SplineError):
        q.DelayedUpdate(16, 17, 2)  # delay > n
    with pytest.raises(q.SplineError):
        q.DelayedUpdate(4096, 8, 2)  # n too large
    L = q.lib()
    assert L.spline_dlu_workspace_bytes(384, 16, 512) > 0
    assert L.spline_dlu_workspace_bytes(384, 65, 512) == 0
    dl = q.DelayedUpdate(8, 4, 2)
    a = torch.zeros((2, 8, 8), dtype=torch.float32, device="cuda")
    kk = torch.tensor([99, -5], dtype=torch.int32, device="cuda")
    V = torch.ones((2, 8), dtype=torch.float32, device="cuda")
    r = dl.ratio(a, kk, V).cpu().numpy()
    assert np.all(np.isnan(r))  # out-of-range electrons
    dl.accept(a, kk, V)  # skipped, no effect
    dl.flush(a)
    assert float(a.abs().sum()) == 0.0
    # walker indices outside the workspace: NaN ratio, accept skipped
    wl = torch.tensor([5, -1], dtype=torch.int32, device="cuda")
    k2 = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    r = dl.ratio(a, k2, V, walkers=wl).cpu().numpy()
    assert np.all(np.isnan(r))
    dl.accept(a, k2, V, walkers=wl)
    dl.flush(a)
    assert float(a.abs().sum()) == 0.0
    # with no walker list, more slots than walkers is refused by the library itself
    import ctypes  # the binding's own check fires first, so call the C ABI directly
    k3 = torch.zeros(3, dtype=torch.int32, device="cuda")
    V3 = torch.ones((3, 8), dtype=torch.float32, device="cuda")
    o3 = torch.empty(3, dtype=torch.float32, device="cuda")
    rc = L.spline_dlu_ratio(dl._h, ctypes.c_void_p(a.data_ptr()), 64, None, ctypes.c_void_p(k3.data_ptr()),
                            ctypes.c_void_p(V3.data_ptr()), None, None, 3, ctypes.c_void_p(o3.data_ptr()), None)
    assert rc == -1
    rc = L.spline_dlu_accept(dl._h, ctypes.c_void_p(a.data_ptr()), 64, None, ctypes.c_void_p(k3.data_ptr()),
                             ctypes.c_void_p(V3.data_ptr()), 3, None)
    assert rc == -1


@pytest.mark.parametrize("n,delay,walkers,vgl", [(384, 16, 64, True), (129, 8, 9, False), (2048, 64, 2, True)])
def test_fused_accept_ratio_equals_separate_calls(torch, q, n, delay, walkers, vgl):
    """A step loop that accepts the previous move and forms the next ratio in
    one call equals the same loop with separate accept and ratio calls, bit
    for bit (ratios, derivative sums and the flushed inverses); 2048 / 64
    with derivatives does not fit S^-1 in LDS and runs as two launches."""
    rng = np.random.default_rng(n + delay)
    A = np.eye(n) + rng.normal(size=(walkers, n, n)) * (0.3 / np.sqrt(n))
    inv0 = np.linalg.inv(A).astype(np.float32)
    ks = np.stack([rng.permutation(n)[:delay] for _ in range(walkers)]).astype(np.int32)
    acc = rng.random((delay, walkers)) < 0.7
    dev = torch.device("cuda")
    V = [torch.from_numpy((rng.normal(size=(walkers, n)) / np.sqrt(n)).astype(np.float32)).to(dev)
         for _ in range(delay)]
    G = [torch.from_numpy(rng.normal(size=(walkers, 3, n)).astype(np.float32)).to(dev) if vgl else None
         for _ in range(delay)]
    Lp = [torch.from_numpy(rng.normal(size=(walkers, n)).astype(np.float32)).to(dev) if vgl else None
          for _ in range(delay)]
    kk = [torch.from_numpy(np.ascontiguousarray(ks[:, i])).to(dev) for i in range(delay)]
    ka = [torch.from_numpy(np.where(acc[i], ks[:, i], -1).astype(np.int32)).to(dev) for i in range(delay)]
    a1 = torch.from_numpy(inv0.copy()).to(dev)
    a2 = torch.from_numpy(inv0.copy()).to(dev)
    d1 = q.DelayedUpdate(n, delay, walkers)
    d2 = q.DelayedUpdate(n, delay, walkers)
    sep, fused = [], []
    for i in range(delay):
        sep.append(d1.ratio(a1, kk[i], V[i], G[i], Lp[i]).cpu().numpy())
        d1.accept(a1, ka[i], V[i])
    _say("case fused step", n, delay, walkers, vgl)
    fused.append(d2.ratio(a2, kk[0], V[0], G[0], Lp[0]).cpu().numpy())
    for i in range(1, delay):
        fused.append(d2.accept_ratio(a2, ka[i - 1], V[i - 1], kk[i], V[i], G[i], Lp[i]).cpu().numpy())
    d2.accept(a2, ka[delay - 1], V[delay - 1])
    for i, (x, y) in enumerate(zip(sep, fused)):
        np.testing.assert_array_equal(x, y, err_msg="step %d" % i)
        assert np.isfinite(x).all()
    d1.flush(a1)
    d2.flush(a2)
    np.testing.assert_array_equal(a1.cpu().numpy(), a2.cpu().numpy())


def test_pending_electrons(torch, q):
    """A proposal for an electron that is itself pending gets its ratio (and
    derivative sums) against the current matrix -- row k of the Woodbury
    inverse, whose t carries the [k_i == k] correction -- checked against the
    oracle and against numpy's inverse of the matrix with the pending columns
    in place.  A second accept of a pending electron cannot be held: it is
    not applied, the walker is marked and its ratios are NaN (a flush keeps
    the mark, a new workspace clears it); other walkers are unaffected."""
    from oracle import det

    n, delay, walkers = 96, 8, 3
    rng = np.random.default_rng(77)
    A = np.eye(n) + rng.normal(size=(walkers, n, n)) * (0.3 / np.sqrt(n))
    inv0 = np.linalg.inv(A).astype(np.float32)
    ks = np.stack([rng.permutation(n)[:4] for _ in range(walkers)]).astype(np.int32)
    phis = (A[:, :, 0][:, None, :] * 0 + rng.normal(size=(walkers, 4, n)) * 0.2).astype(np.float32)
    cur = A.copy()
    for w in range(walkers):
        for i in range(4):
            phis[w, i] += A[w][:, ks[w, i]].astype(np.float32)
            cur[w][:, ks[w, i]] = phis[w, i]
    a_d = torch.from_numpy(inv0.copy()).cuda()
    dl = q.DelayedUpdate(n, delay, walkers)
    for i in range(4):
        dl.accept(a_d, torch.from_numpy(np.ascontiguousarray(ks[:, i])).cuda(),
                  torch.from_numpy(np.ascontiguousarray(phis[:, i])).cuda())
    # ratios with derivatives for the electron accepted second (pending)
    kp = np.ascontiguousarray(ks[:, 1])
    Vq = (rng.normal(size=(walkers, n)) / np.sqrt(n)).astype(np.float32)
    Gq = rng.normal(size=(walkers, 3, n)).astype(np.float32)
    Lq = rng.normal(size=(walkers, n)).astype(np.float32)
    D = dl.ratio(a_d, torch.from_numpy(kp).cuda(), torch.from_numpy(Vq).cuda(), torch.from_numpy(Gq).cuda(),
                 torch.from_numpy(Lq).cuda()).cpu().numpy().astype(np.float64)
    for w in range(walkers):
        qv = np.vstack([Vq[w], Gq[w], Lq[w]]).astype(np.float64)
        ref = det.delayed_ratio(inv0[w].astype(np.float64), phis[w].astype(np.float64), list(ks[w]), int(kp[w]), qv)
        direct = qv @ np.linalg.inv(cur[w])[kp[w]]
        sc = np.abs(qv) @ np.abs(np.linalg.inv(cur[w])[kp[w]]) + 1.0
        assert np.max(np.abs(D[w] - ref) / sc) < TOL, w
        assert np.max(np.abs(D[w] - direct) / sc) < TOL, w
    # a second accept of a pending electron, for walker 0 only
    kdup = np.array([ks[0, 2], -1, -1], dtype=np.int32)
    dl.accept(a_d, torch.from_numpy(kdup).cuda(), torch.from_numpy(Vq).cuda())
    k0 = np.array([ks[0, 3], ks[1, 3], ks[2, 3]], dtype=np.int32)
    r = dl.ratio(a_d, torch.from_numpy(k0).cuda(), torch.from_numpy(Vq).cuda()).cpu().numpy()
    assert np.isnan(r[0]) and np.isfinite(r[1:]).all()
    for w in (1, 2):
        ref = det.delayed_ratio(inv0[w].astype(np.float64), phis[w].astype(np.float64), list(ks[w]), int(k0[w]),
                                Vq[w].astype(np.float64))
        assert abs(r[w] - ref) / (np.abs(Vq[w]) @ np.abs(np.linalg.inv(cur[w])[k0[w]]) + 1.0) < TOL
    # the fused call whose accept is the duplicate: NaN for that slot
    kdup2 = np.array([ks[0, 0], -1, -1], dtype=np.int32)
    r2 = dl.accept_ratio(a_d, torch.from_numpy(kdup2).cuda(), torch.from_numpy(Vq).cuda(),
                         torch.from_numpy(k0).cuda(), torch.from_numpy(Vq).cuda()).cpu().numpy()
    assert np.isnan(r2[0]) and np.isfinite(r2[1:]).all()
    dl.flush(a_d)
    r3 = dl.ratio(a_d, torch.from_numpy(k0).cuda(), torch.from_numpy(Vq).cuda()).cpu().numpy()
    assert np.isnan(r3[0]) and np.isfinite(r3[1:]).all()
    # the flushed inverses of the unmarked walkers hold their four moves
    got = a_d.cpu().numpy().astype(np.float64)
    for w in (1, 2):
        assert np.max(np.abs(got[w] @ cur[w] - np.eye(n))) < 1e-3
    dl2 = q.DelayedUpdate(n, delay, walkers)  # a new workspace: no marks
    r4 = dl2.ratio(a_d, torch.from_numpy(k0).cuda(), torch.from_numpy(Vq).cuda()).cpu().numpy()
    assert np.isfinite(r4).all()
