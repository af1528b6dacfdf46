"""The kernels of one particle-by-particle step can be captured in a HIP
graph: the determinant ratio with derivatives, the Jastrow move, the
Sherman-Morrison update and the Jastrow accept (a slot with k = -1 is a
rejected move, which both update kernels skip).  The graph is replayed
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
