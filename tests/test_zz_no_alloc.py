"""GPU test of spline_eval_vgl_sorted_noalloc, the entry point that
allocates nothing (its sort scratch is the library's static device array):
through the C ABI, against spline_eval_vgl_sorted (which takes a caller
workspace) bit for bit, on two calls in a row with the second batch smaller,
so stale scratch contents from the first call must not leak into the second.
Also a general (hexagonal) cell, the size limit and B == 0."""
import ctypes
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


def _positions(rng, B, cell):
    p = (rng.random((B, 3)) * 3.0 - 1.0) * np.asarray(cell)
    p[:4] = [[0.0, 0.0, 0.0], [-1e-17, 0.5, 1.0], [1.0, 1.0, 1.0], [0.25, -0.0, 2.0]]
    return p


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_noalloc_matches_workspace_entry_point(torch, q, dtype):
    rng = np.random.default_rng(71)
    grid = (14, 12, 10)
    G, a, b = W.planewave_params(rng, 48)
    coefs = W.fit_planewave_coefs(grid, G, a, b)
    s = q.Spline(grid, coefs, dtype)
    for B in (20000, 3001):  # second call smaller: the scratch holds the first call's keys and ranks
        pos = torch.from_numpy(_positions(rng, B, (1, 1, 1))).cuda()
        _say("case noalloc %s B=%d" % (dtype, B))
        ref = s.eval_vgl_sorted(pos)
        out = s.alloc_outputs(B)
        for t in out:
            t.fill_(float("nan"))
        got = s.eval_vgl_sorted_noalloc(pos, out)
        plain = s.eval_vgl(pos)
        torch.cuda.synchronize()
        for g, r, p in zip(got, ref, plain):
            assert torch.equal(g, r)
            assert torch.equal(g, p)


def test_noalloc_general_cell(torch, q):
    rng = np.random.default_rng(72)
    grid = (12, 12, 16)
    G, a, b = W.planewave_params(rng, 32)
    coefs = W.fit_planewave_coefs(grid, G, a, b)
    s = q.Spline(grid, coefs, "f32")
    hexl = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3.0) / 2.0, 0.0], [0.0, 0.0, 1.6]])
    s.set_lattice(hexl)
    for B in (9000, 777):
        pos = torch.from_numpy(_positions(rng, B, (1, 1, 1)) @ hexl).cuda()
        _say("case noalloc hexagonal B=%d" % B)
        ref = s.eval_vgl_sorted(pos)
        got = s.eval_vgl_sorted_noalloc(pos, s.alloc_outputs(B))
        torch.cuda.synchronize()
        for g, r in zip(got, ref):
            assert torch.equal(g, r)


def test_noalloc_limits(torch, q):
    grid = (8, 8, 8)
    coefs = np.random.default_rng(73).uniform(-1, 1, grid + (16,))
    s = q.Spline(grid, coefs, "f32")
    L = q.lib()
    # beyond the static scratch: rejected before any pointer is touched
    rc = L.spline_eval_vgl_sorted_noalloc(s._h, None, (1 << 19) + 1, None, None, None, None)
    assert rc == -2 and b"524288" in L.spline_last_error()
    assert L.spline_eval_vgl_sorted_noalloc(s._h, None, 0, None, None, None, None) == 0
    assert L.spline_eval_vgl_sorted_noalloc(s._h, None, -1, None, None, None, None) == -1
    # the largest batch it takes
    B = 1 << 19
    pos = torch.from_numpy(np.random.default_rng(74).random((B, 3))).cuda()
    _say("case noalloc B=%d (maximum)" % B)
    got = s.eval_vgl_sorted_noalloc(pos, s.alloc_outputs(B))
    ref = s.eval_vgl(pos)
    torch.cuda.synchronize()
    for g, r in zip(got, ref):
        assert torch.equal(g, r)
