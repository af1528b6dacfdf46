"""GPU parity for tables whose rows hold at most 256 bytes of orbitals.

Such rows are padded only to 64 B (128 B for FP64) instead of 256 B, and the
16-lane tile shapes that divide them are compiled: 48 FP32 orbitals take a
192-byte row read as one 192-byte tile.  Every call goes through the C ABI.
Checked against the FP64 oracle (the dequantized coefficients for 16-bit
tables), with the bars of the plain evaluation: 1e-12 for FP64 tables, 1e-5
for FP32 accumulation; every tile candidate gives the same bits; the
locality-ordered path equals the plain one bit for bit; VGH and the fused
determinant ratio run on the same short rows.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5, "f16": 1e-5}
GRID = (10, 11, 12)  # unequal axes: strides of every axis are exercised
CASES = [(48, "f32"), (40, "f32"), (24, "f32"), (16, "f32"), (8, "f32"), (40, "bf16"), (96, "f16"),
         (24, "f64"), (8, "f64")]


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


def _table(norb, seed):
    rng = np.random.default_rng(seed)
    coefs = rng.uniform(-1.0, 1.0, GRID + (norb,))
    pos = rng.uniform(-1.5, 2.5, (333, 3))  # ragged count; coordinates beyond one period on both sides
    return coefs, pos


def _dq(oracle, coefs, dt):
    return oracle.dequantize(coefs, dt)[0] if dt in ("bf16", "f16", "f32") else coefs


def _np(ts):
    return [t.double().cpu().numpy() for t in ts]


@pytest.mark.parametrize("norb,dt", CASES)
def test_short_rows_every_tile(torch, q, oracle, norb, dt):
    coefs, pos = _table(norb, 100 + norb)
    L = q.get_layout(GRID, norb, dt)
    want = 64 if dt != "f64" else 128
    assert L.row_bytes % want == 0 and L.row_bytes - norb * L.elem_bytes < want
    pd = torch.from_numpy(pos).cuda()
    ref = oracle.eval_vgl(GRID, _dq(oracle, coefs, dt), pos)
    s = q.Spline(GRID, coefs, dt)
    cands = s.tile_candidates()
    assert cands, "no tile shape fits a %d-byte row" % L.row_bytes
    first = None
    for t in cands:
        _say("case short rows", norb, dt, "row", L.row_bytes, "tile", t)
        s.set_tile(t)
        got = _np(s.eval_vgl(pd))
        v = _np([s.eval_v(pd)])[0]
        torch.cuda.synchronize()
        if first is None:
            first = got
            for name, g, r in zip("VGL", got, ref):
                e = oracle.rel_err(g, r)
                assert e <= TOL[dt], "N=%d %s tile %s: %s rel err %.3e" % (norb, dt, t, name, e)
        else:
            for a, b in zip(first, got):
                np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(v, got[0])
    s.close()


@pytest.mark.parametrize("norb,dt", [(48, "f32"), (40, "bf16"), (24, "f64")])
def test_short_rows_sorted_vgh_ratio(torch, q, oracle, norb, dt):
    from oracle import det

    coefs, pos = _table(norb, 200 + norb)
    pd = torch.from_numpy(pos).cuda()
    table = _dq(oracle, coefs, dt)
    s = q.Spline(GRID, coefs, dt)
    _say("case short rows sorted/vgh/ratio", norb, dt, "tile", s.get_tile(), "vgh tile", s.get_vgh_tile())
    plain = _np(s.eval_vgl(pd))
    srt = _np(s.eval_vgl_sorted(pd))
    for a, b in zip(plain, srt):
        np.testing.assert_array_equal(a, b)

    lat = np.diag([1.0, 1.0, 1.0])
    Vh, Gh, Hh = _np(s.eval_vgh(pd))
    Vr, Gr, Hr = oracle.eval_vgh(GRID, table, pos, lat)
    for name, g, r in zip(("V", "G", "H"), (Vh, Gh, Hh), (Vr, Gr, Hr)):
        e = oracle.rel_err(g, r)
        assert e <= TOL[dt], "VGH N=%d %s: %s rel err %.3e" % (norb, dt, name, e)

    rng = np.random.default_rng(norb)
    rows = rng.standard_normal((len(pos), norb)).astype(np.float64 if dt == "f64" else np.float32)
    rd = torch.from_numpy(rows).cuda()
    D = s.eval_ratio_vgl(pd, rd).double().cpu().numpy()
    Dref = det.ratio_vgl(GRID, table, pos, rows.astype(np.float64))
    V, G, Lp = oracle.eval_vgl(GRID, table, pos)
    M = [np.abs(V).max(axis=0), np.abs(G).max(axis=(0, 1)), np.abs(Lp).max(axis=0)]
    sv, sg, sl = (det.ratio_scale(rows.astype(np.float64), m) for m in M)
    scale = np.stack([sv, sg, sg, sg, sl], axis=1)
    e = float(np.max(np.abs(D - Dref) / scale))
    assert e <= TOL[dt], "ratio N=%d %s: rel err %.3e" % (norb, dt, e)
    s.close()
