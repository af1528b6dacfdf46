"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself:
textbook closed forms (golden file), an independent library B-spline
(scipy's Cox-de Boor basis), exact polynomial reproduction, finite
differences, periodicity, continuity at knots, and correctly rounded
conversions from numpy.  A dropped term, a wrong sign or a shifted index in
the oracle fails at least one of them.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden_basis():
    rows = []
    with open(os.path.join(HERE, "golden", "bspline_basis.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            v = [float(Fraction(x)) for x in line.split()]
            rows.append((v[0], np.array(v[1:5]), np.array(v[5:9]), np.array(v[9:13])))
    return rows


def test_basis_golden(oracle):
    rows = _golden_basis()
    assert len(rows) == 3
    for t, b, db, d2b in rows:
        ob, odb, od2b = oracle.basis(t)
        np.testing.assert_allclose(ob, b, rtol=0, atol=1e-15)
        np.testing.assert_allclose(odb, db, rtol=0, atol=1e-15)
        np.testing.assert_allclose(od2b, d2b, rtol=0, atol=1e-15)


def test_basis_matches_cox_de_boor(oracle):
    """Weight k at offset t is the cardinal cubic B-spline at t + 3 - k."""
    from scipy.interpolate import BSpline

    B = BSpline.basis_element(np.arange(5.0), extrapolate=False)
    dB, d2B = B.derivative(1), B.derivative(2)
    for t in np.linspace(0.0, 1.0, 41)[1:-1]:
        ob, odb, od2b = oracle.basis(t)
        x = t + 3.0 - np.arange(4)
        np.testing.assert_allclose(ob, B(x), atol=1e-14)
        np.testing.assert_allclose(odb, dB(x), atol=1e-13)
        np.testing.assert_allclose(od2b, d2B(x), atol=1e-12)


def test_basis_invariants(oracle):
    for t in np.random.default_rng(0).random(200):
        b, db, d2b = oracle.basis(t)
        assert abs(b.sum() - 1.0) < 1e-15
        assert abs(db.sum()) < 1e-15
        assert abs(d2b.sum()) < 1e-14
        b2, db2, d2b2 = oracle.basis(1.0 - t)
        np.testing.assert_allclose(b, b2[::-1], atol=1e-15)
        np.testing.assert_allclose(db, -db2[::-1], atol=1e-15)
        np.testing.assert_allclose(d2b, d2b2[::-1], atol=1e-14)
        assert (b >= 0).all()


def test_reduce_edges(oracle):
    assert oracle.reduce(0.0, 1.0, 16) == (0, 0.0)
    assert oracle.reduce(0.5, 1.0, 16) == (8, 0.0)
    i, t = oracle.reduce(-1e-17, 1.0, 16)       # wraps to just below 1 -> guard to 0
    assert (i, t) == (0, 0.0)
    for n in (16, 48, 80, 7):                   # largest f below 1: last cell, t just below 1
        i, t = oracle.reduce(1.0 - 2.0**-53, 1.0, n)
        assert i == n - 1 and 1.0 - 1e-13 < t <= 1.0
    i, t = oracle.reduce(-0.0, 1.0, 16)
    assert (i, t) == (0, 0.0)
    i, t = oracle.reduce(1e6 + 0.25, 1.0, 16)
    assert i == 4 and abs(t) < 1e-9
    i, t = oracle.reduce(0.3, 2.0, 10)          # cell length 2: f = 0.15, u = 1.5
    assert i == 1 and abs(t - 0.5) < 1e-15
    i, t = oracle.reduce(float("nan"), 1.0, 16)
    assert i == 0 and np.isnan(t)
    i, t = oracle.reduce(float("inf"), 1.0, 16)
    assert i == 0 and np.isnan(t)


def _rand_pos(rng, B, cell=(1.0, 1.0, 1.0)):
    return rng.random((B, 3)) * np.asarray(cell)


def test_constant_table(oracle):
    grid = (5, 6, 7)
    c = np.empty(grid + (3,))
    c[..., 0], c[..., 1], c[..., 2] = 1.0, -2.5, 0.0
    pos = _rand_pos(np.random.default_rng(1), 50, (1.0, 2.0, 0.5))
    V, G, L = oracle.eval_vgl(grid, c, pos, cell=(1.0, 2.0, 0.5))
    np.testing.assert_allclose(V, np.broadcast_to([1.0, -2.5, 0.0], V.shape), atol=1e-14)
    assert np.abs(G).max() < 1e-12 and np.abs(L).max() < 1e-10


def test_grid_point_stencils(oracle):
    """At a knot: V is the (1,4,1)/6 tensor stencil, G_d the central difference
    (n/L)(c+ - c-)/2 along d, L the (n/L)^2 (1,-2,1) second difference."""
    rng = np.random.default_rng(2)
    grid, cell = (6, 7, 8), (1.0, 1.5, 0.75)
    N = 5
    c = rng.uniform(-1, 1, grid + (N,))
    s = [np.array([1.0, 4.0, 1.0]) / 6.0] * 3
    for _ in range(20):
        j = [int(rng.integers(0, n)) for n in grid]
        pos = np.array([[j[d] * cell[d] / grid[d] for d in range(3)]])
        V, G, L = oracle.eval_vgl(grid, c, pos, cell=cell)
        blk = np.empty((3, 3, 3, N))
        for a in range(3):
            for b in range(3):
                for e in range(3):
                    blk[a, b, e] = c[(j[0] + a - 1) % grid[0], (j[1] + b - 1) % grid[1], (j[2] + e - 1) % grid[2]]
        d1 = np.array([-0.5, 0.0, 0.5])
        d2 = np.array([1.0, -2.0, 1.0])
        ev = lambda w0, w1, w2: np.einsum("a,b,e,abem->m", w0, w1, w2, blk)
        g = [grid[d] / cell[d] for d in range(3)]
        np.testing.assert_allclose(V[0], ev(*s), atol=1e-14)
        np.testing.assert_allclose(G[0, 0], g[0] * ev(d1, s[1], s[2]), atol=1e-12)
        np.testing.assert_allclose(G[0, 1], g[1] * ev(s[0], d1, s[2]), atol=1e-12)
        np.testing.assert_allclose(G[0, 2], g[2] * ev(s[0], s[1], d1), atol=1e-12)
        Lref = g[0] ** 2 * ev(d2, s[1], s[2]) + g[1] ** 2 * ev(s[0], d2, s[2]) + g[2] ** 2 * ev(s[0], s[1], d2)
        np.testing.assert_allclose(L[0], Lref, atol=1e-10)


def test_cubic_reproduction(oracle):
    """Coefficients 1, j, j^2 - 1/3, j^3 - j reproduce 1, u, u^2, u^3 exactly
    (moments of the centred cubic B-spline); tensor products reproduce
    tensor monomials, so V, G, L are analytic where the stencil does not wrap."""
    rng = np.random.default_rng(3)
    grid, cell = (9, 10, 11), (1.0, 1.3, 0.8)
    coef1d = [lambda j: np.ones_like(j), lambda j: j, lambda j: j * j - 1.0 / 3.0, lambda j: j ** 3 - j]
    pows = [(p0, p1, p2) for p0 in range(4) for p1 in range(4) for p2 in range(4)]
    N = len(pows)
    jj = [np.arange(n, dtype=np.float64) for n in grid]
    c = np.empty(grid + (N,))
    for m, (p0, p1, p2) in enumerate(pows):
        c[..., m] = np.einsum("a,b,e->abe", coef1d[p0](jj[0]), coef1d[p1](jj[1]), coef1d[p2](jj[2]))
    # positions whose cells keep the stencil [i-1, i+2] inside [0, n-1]
    B = 64
    u = np.stack([rng.uniform(1.0, n - 2.0, B) for n in grid], 1)
    pos = u * np.asarray(cell) / np.asarray(grid)
    V, G, L = oracle.eval_vgl(grid, c, pos, cell=cell)
    g = np.asarray(grid) / np.asarray(cell)
    for m, p in enumerate(pows):
        mono = [u[:, d] ** p[d] for d in range(3)]
        dmono = [p[d] * u[:, d] ** max(p[d] - 1, 0) for d in range(3)]
        d2mono = [p[d] * (p[d] - 1) * u[:, d] ** max(p[d] - 2, 0) for d in range(3)]
        Vr = mono[0] * mono[1] * mono[2]
        Gr = [g[0] * dmono[0] * mono[1] * mono[2], g[1] * mono[0] * dmono[1] * mono[2], g[2] * mono[0] * mono[1] * dmono[2]]
        Lr = (g[0] ** 2 * d2mono[0] * mono[1] * mono[2] + g[1] ** 2 * mono[0] * d2mono[1] * mono[2]
              + g[2] ** 2 * mono[0] * mono[1] * d2mono[2])
        scale = max(1.0, np.abs(Vr).max())
        np.testing.assert_allclose(V[:, m], Vr, atol=1e-12 * scale)
        for d in range(3):
            np.testing.assert_allclose(G[:, d, m], Gr[d], atol=1e-12 * scale * g.max())
        np.testing.assert_allclose(L[:, m], Lr, atol=1e-11 * scale * g.max() ** 2)


def test_periodicity(oracle):
    rng = np.random.default_rng(4)
    grid, cell = (7, 8, 9), (1.0, 1.1, 0.9)
    c = rng.uniform(-1, 1, grid + (4,))
    pos = _rand_pos(rng, 40, cell)
    V, G, L = oracle.eval_vgl(grid, c, pos, cell=cell)
    for d in range(3):
        for shift in (1.0, -3.0, 17.0):
            p2 = pos.copy()
            p2[:, d] += shift * cell[d]
            V2, G2, L2 = oracle.eval_vgl(grid, c, p2, cell=cell)
            np.testing.assert_allclose(V2, V, atol=1e-12)
            np.testing.assert_allclose(G2, G, atol=1e-10)
            np.testing.assert_allclose(L2, L, atol=1e-8)


def test_finite_differences(oracle):
    """5-point first and 3-point second differences are exact for a cubic
    inside one cell, so G and L must match them up to rounding."""
    rng = np.random.default_rng(5)
    grid, cell = (8, 9, 10), (1.0, 1.2, 0.7)
    N = 6
    c = rng.uniform(-1, 1, grid + (N,))
    B = 30
    i = np.stack([rng.integers(0, n, B) for n in grid], 1)
    t = rng.uniform(0.05, 0.95, (B, 3))
    pos = (i + t) * np.asarray(cell) / np.asarray(grid)
    V, G, L = oracle.eval_vgl(grid, c, pos, cell=cell)
    Lfd = np.zeros_like(L)
    for d in range(3):
        h = 0.01 * cell[d] / grid[d]
        e = np.zeros(3)
        e[d] = h
        f = {k: oracle.eval_vgl(grid, c, pos + k * e, cell=cell)[0] for k in (-2, -1, 1, 2)}
        gfd = (-f[2] + 8 * f[1] - 8 * f[-1] + f[-2]) / (12 * h)
        np.testing.assert_allclose(G[:, d], gfd, rtol=0, atol=1e-9 * np.abs(G[:, d]).max())
        Lfd += (f[1] - 2 * V + f[-1]) / (h * h)
    np.testing.assert_allclose(L, Lfd, rtol=0, atol=1e-6 * np.abs(L).max())


def test_c2_continuity_at_knots(oracle):
    rng = np.random.default_rng(6)
    grid = (6, 6, 6)
    c = rng.uniform(-1, 1, grid + (3,))
    for _ in range(10):
        base = rng.random(3)
        d = int(rng.integers(0, 3))
        base[d] = int(rng.integers(0, 6)) / 6.0
        lo, hi = base.copy(), base.copy()
        lo[d] -= 1e-9
        hi[d] += 1e-9
        Vl, Gl, Ll = oracle.eval_vgl(grid, c, lo[None])
        Vh, Gh, Lh = oracle.eval_vgl(grid, c, hi[None])
        assert np.abs(Vl - Vh).max() < 1e-7
        assert np.abs(Gl - Gh).max() < 1e-5
        assert np.abs(Ll - Lh).max() < 1e-3   # L is C0 across knots up to O(n^2 h)


def test_nonfinite_positions(oracle):
    grid = (4, 4, 4)
    c = np.ones(grid + (2,))
    pos = np.array([[np.nan, 0.1, 0.2], [0.1, np.inf, 0.2], [0.3, 0.2, 0.1]])
    V, G, L = oracle.eval_vgl(grid, c, pos)
    assert np.isnan(V[:2]).all() and np.isnan(G[:2]).all() and np.isnan(L[:2]).all()
    np.testing.assert_allclose(V[2], 1.0)


def test_value_only_matches_vgl(oracle):
    rng = np.random.default_rng(7)
    grid = (5, 7, 6)
    c = rng.uniform(-1, 1, grid + (9,))
    pos = _rand_pos(rng, 33)
    V, _, _ = oracle.eval_vgl(grid, c, pos)
    np.testing.assert_array_equal(oracle.eval_v(grid, c, pos), V)


def test_threads_do_not_change_results(oracle):
    rng = np.random.default_rng(8)
    grid = (6, 6, 6)
    c = rng.uniform(-1, 1, grid + (8,))
    pos = _rand_pos(rng, 257)
    a = oracle.eval_vgl(grid, c, pos, threads=1)
    b = oracle.eval_vgl(grid, c, pos, threads=4)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# ---- reduced-precision storage -------------------------------------------------

def test_round_sig_matches_numpy_f32_f16(oracle):
    rng = np.random.default_rng(9)
    xs = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.integers(-9, 2, 3000),
                         rng.uniform(-1, 1, 1000)])
    for x in xs:
        assert oracle.round_sig(x, 24, -126) == float(np.float32(x))
        if abs(x) <= 1.0:
            assert oracle.round_sig(x, 11, -14) == float(np.float16(x))


def test_round_sig_ties_and_bf16(oracle):
    # exact ties round to even
    one = 1.0
    assert oracle.round_sig(one + 2.0**-8, 8, -126) == 1.0            # halfway 1 and 1+2^-7
    assert oracle.round_sig(one + 3 * 2.0**-8, 8, -126) == 1.0 + 2.0**-6
    assert oracle.round_sig(one + 2.0**-11, 11, -14) == 1.0
    # brute force against the explicit neighbour set for BF16
    rng = np.random.default_rng(10)
    for x in rng.uniform(-1, 1, 2000):
        q = oracle.round_sig(x, 8, -126)
        e = np.floor(np.log2(abs(x)))
        ulp = 2.0 ** (e - 7)
        cands = (np.floor(x / ulp) + np.arange(-1, 3)) * ulp
        best = cands[np.argmin(np.abs(cands - x))]
        assert abs(q - x) <= abs(best - x)
        assert (q / ulp) == np.round(q / ulp)  # on the 8-bit grid of its binade (or the next)


def test_dequantize_scales_and_values(oracle):
    rng = np.random.default_rng(11)
    c = rng.standard_normal((4, 3, 5, 6)) * np.array([1e-3, 0.5, 1.0, 3.0, 1000.0, 0.0])
    for fmt, p, emin in (("bf16", 8, -126), ("f16", 11, -14)):
        dq, s = oracle.dequantize(c, fmt)
        for m in range(6):
            mx = np.abs(c[..., m]).max()
            if mx == 0:
                assert s[m] == 1.0
                assert (dq[..., m] == 0).all()
                continue
            assert s[m] >= mx and s[m] / 2 < mx and np.log2(s[m]) == round(np.log2(s[m]))
            x = c[..., m].ravel()[:20]
            q = dq[..., m].ravel()[:20]
            for a, b in zip(x, q):
                assert b == oracle.round_sig(a / s[m], p, emin) * s[m]
        rel = np.abs(dq - c).max(axis=(0, 1, 2)) / np.where(s > 0, s, 1)
        assert (rel <= 2.0 ** -p).all()
    dq, s = oracle.dequantize(c, "f32")
    np.testing.assert_array_equal(dq, c.astype(np.float32).astype(np.float64))
    assert (s == 1).all()
    dq, s = oracle.dequantize(c, "f64")
    np.testing.assert_array_equal(dq, c)


# ---- the plane-wave table generator (input preparation) ------------------------

def test_fit_matches_fft_cyclic_solve():
    """Closed-form fit equals the cyclic solve of the (1,4,1)/6 system by FFT."""
    rng = np.random.default_rng(12)
    grid = (10, 12, 8)
    G, a, b = W.planewave_params(rng, 7)
    c = W.fit_planewave_coefs(grid, G, a, b)
    j = np.stack(np.meshgrid(*[np.arange(n) / n for n in grid], indexing="ij"), -1).reshape(-1, 3)
    f = W.planewave_values(G, a, b, j).reshape(grid + (7,))
    Fk = np.fft.fftn(f, axes=(0, 1, 2))
    for d, n in enumerate(grid):
        lam = (4.0 + 2.0 * np.cos(2 * np.pi * np.fft.fftfreq(n) * 1.0)) / 6.0
        shp = [1, 1, 1, 1]
        shp[d] = n
        Fk = Fk / lam.reshape(shp)
    c_fft = np.fft.ifftn(Fk, axes=(0, 1, 2)).real
    np.testing.assert_allclose(c, c_fft, atol=1e-12 * np.abs(c).max())


def test_fit_interpolates_planewaves(oracle):
    """The oracle evaluated at grid points reproduces the analytic orbitals."""
    rng = np.random.default_rng(13)
    grid = (12, 12, 12)
    G, a, b = W.planewave_params(rng, 6)
    c = W.fit_planewave_coefs(grid, G, a, b)
    jj = rng.integers(0, 12, (40, 3))
    pos = jj / 12.0
    V, _, _ = oracle.eval_vgl(grid, c, pos)
    np.testing.assert_allclose(V, W.planewave_values(G, a, b, pos), atol=1e-12 * np.abs(V).max())
    # off-grid: O(h^4) interpolation error, only reported as a sanity bound
    off = rng.random((40, 3))
    Voff, _, _ = oracle.eval_vgl(grid, c, off)
    ref = W.planewave_values(G, a, b, off)
    assert np.abs(Voff - ref).max() < 0.5 * np.abs(ref).max()


def test_rel_err_metric(oracle):
    ref = np.array([[1.0, 0.0], [-2.0, 0.0]])
    q = np.array([[1.0, 1e-3], [-2.002, 0.0]])
    assert abs(oracle.rel_err(q, ref) - 1e-3) < 1e-15     # zero orbital: absolute
    assert np.isnan(oracle.rel_err(np.array([[np.nan, 0.0], [0.0, 0.0]]), ref))
