"""Pins of the determinant-ratio oracle (oracle/det.py).

The oracle forms sum_i a_i Q_i(r') with a = row k of A^-1.  It is checked
here against quantities it does not compute: determinants of the moved
Slater matrix built from scratch and factorised by numpy.linalg (the ratio),
and central differences of those determinants in the moved electron's
coordinates (gradient and Laplacian).  Positions stay in the interior of
their grid cells, where the spline is a cubic polynomial along each axis, so
a second central difference is exact up to rounding and a first one is
accurate to h^2 |f'''| / 6.  Using a column of A^-1 instead of a row, a
dropped derivative stream or a wrong chain-rule factor fails these checks.
"""
import numpy as np
import pytest

import workloads as W


def _interior(rng, count, grid, cell=(1.0, 1.0, 1.0), lo=0.25, hi=0.75):
    g = np.asarray(grid)
    idx = rng.integers(0, g, size=(count, 3))
    t = rng.uniform(lo, hi, size=(count, 3))
    return (idx + t) / g * np.asarray(cell)


def _system(cell, seed):
    grid, norb, coefs, _ = W.make_table(1)  # 16^3 grid, 32 orbitals, c ~ U[-1, 1]
    rng = np.random.default_rng(seed)
    R = _interior(rng, norb, grid, cell)
    Rp = _interior(rng, norb, grid, cell)
    return grid, norb, coefs, R, Rp


def _moved_ratio(det, grid, coefs, R, k, r, cell, s0, l0):
    R2 = R.copy()
    R2[k] = r
    s1, l1 = np.linalg.slogdet(det.slater_matrix(grid, coefs, R2, cell))
    return s1 * s0 * np.exp(l1 - l0)


CELLS = [(1.0, 1.0, 1.0), (1.0, 1.3, 0.8)]


@pytest.mark.parametrize("cell", CELLS)
def test_ratio_equals_determinant_ratio(oracle, cell):
    from oracle import det

    grid, n, coefs, R, Rp = _system(cell, 21)
    A = det.slater_matrix(grid, coefs, R, cell)
    assert np.linalg.cond(A) < 1e6
    Ainv = np.linalg.inv(A)
    s0, l0 = np.linalg.slogdet(A)
    got = det.ratio_v(grid, coefs, Rp, Ainv, cell)  # position k uses row k
    want = np.array([_moved_ratio(det, grid, coefs, R, k, Rp[k], cell, s0, l0) for k in range(n)])
    phi = oracle.eval_v(grid, coefs, Rp, cell)
    scale = np.sum(np.abs(Ainv) * np.abs(phi), axis=1)
    assert np.max(np.abs(got - want) / scale) < 1e-9
    # sensitivity: columns of A^-1 in place of rows give a different answer
    wrong = det.ratio_v(grid, coefs, Rp, np.ascontiguousarray(Ainv.T), cell)
    assert np.max(np.abs(wrong - want) / scale) > 1e-3
    # the VGL variant's first entry is the same ratio
    D = det.ratio_vgl(grid, coefs, Rp, Ainv, cell)
    np.testing.assert_allclose(D[:, 0], got, rtol=1e-13, atol=1e-13 * scale.max())


@pytest.mark.parametrize("cell", CELLS)
def test_ratio_derivatives_are_determinant_derivatives(oracle, cell):
    """grad det(A')/det A and lap det(A')/det A by central differences of the
    moved determinant."""
    from oracle import det

    grid, n, coefs, R, Rp = _system(cell, 22)
    A = det.slater_matrix(grid, coefs, R, cell)
    Ainv = np.linalg.inv(A)
    s0, l0 = np.linalg.slogdet(A)
    D = det.ratio_vgl(grid, coefs, Rp, Ainv, cell)
    _, G, L = oracle.eval_vgl(grid, coefs, Rp, cell)
    gscale = np.abs(Ainv) @ np.abs(G).max(axis=(0, 1))
    lscale = np.abs(Ainv) @ np.abs(L).max(axis=0)
    h1, h2 = 1e-5, 1e-3  # every position is >= 0.0125 (a quarter grid spacing) from a knot
    for k in range(0, n, 3):
        f = lambda r: _moved_ratio(det, grid, coefs, R, k, r, cell, s0, l0)  # noqa: E731
        f0 = f(Rp[k])
        lap = 0.0
        for d in range(3):
            e = np.zeros(3)
            e[d] = 1.0
            g = (f(Rp[k] + h1 * e) - f(Rp[k] - h1 * e)) / (2 * h1)
            assert abs(g - D[k, 1 + d]) < 1e-6 * gscale[k], (k, d, g, D[k, 1 + d])
            lap += (f(Rp[k] + h2 * e) - 2 * f0 + f(Rp[k] - h2 * e)) / h2 ** 2
        assert abs(lap - D[k, 4]) < 1e-8 * lscale[k], (k, lap, D[k, 4])


def test_ratio_scale_bounds_perturbation(oracle):
    """An error of e * M_i in orbital i moves the dot product by at most e
    times ratio_scale."""
    from oracle import det

    rng = np.random.default_rng(5)
    rows = rng.normal(size=(7, 11))
    M = rng.uniform(0.5, 2.0, size=11)
    s = det.ratio_scale(rows, M)
    for _ in range(20):
        err = rng.uniform(-1, 1, size=(7, 11)) * M * 1e-3
        assert np.all(np.abs(np.sum(rows * err, axis=1)) <= 1e-3 * s * (1 + 1e-12))


def test_sherman_morrison_is_the_inverse_of_the_moved_matrix(oracle):
    """The updated inverse equals numpy's inverse of the Slater matrix rebuilt
    with the moved electron; a sweep of accepted moves over every electron
    equals the inverse of the final matrix."""
    from oracle import det

    grid, n, coefs, R, Rp = _system((1.0, 1.0, 1.0), 23)
    A = det.slater_matrix(grid, coefs, R)
    Ainv = np.linalg.inv(A)
    R2 = R.copy()
    for k in range(n):
        phi = oracle.eval_v(grid, coefs, Rp[k:k + 1])[0]
        new = det.sherman_morrison(Ainv, k, phi)
        R2[k] = Rp[k]
        want = np.linalg.inv(det.slater_matrix(grid, coefs, R2))
        assert np.max(np.abs(new - want)) < 1e-8 * np.max(np.abs(want)), k
        Ainv = new
    # a wrong sign of the correction or the column in place of the row fails
    a0 = np.linalg.inv(A)
    phi = oracle.eval_v(grid, coefs, Rp[:1])[0]
    R3 = R.copy()
    R3[0] = Rp[0]
    want = np.linalg.inv(det.slater_matrix(grid, coefs, R3))
    t = a0 @ phi
    u = t.copy()
    u[0] -= 1.0
    wrong = a0 + np.outer(u, a0[0]) / t[0]
    assert np.max(np.abs(wrong - want)) > 1e-3 * np.max(np.abs(want))


def test_delayed_update_matches_direct_inverses(oracle):
    """With up to 8 pending accepted moves against a stale inverse, the
    delayed ratio and derivative sums equal those from numpy's inverse of
    the Slater matrix with all pending moves applied, and the flush equals
    that inverse; forgetting the correction term fails."""
    from oracle import det

    grid, n, coefs, R, Rp = _system((1.0, 1.0, 1.0), 24)
    A0inv = np.linalg.inv(det.slater_matrix(grid, coefs, R))
    rng = np.random.default_rng(3)
    order = rng.permutation(n)[:9]
    R2 = R.copy()
    phis, ks = [], []
    for step, k in enumerate(order):
        rnew = rng.random(3)
        V, G, L = oracle.eval_vgl(grid, coefs, rnew[None])
        q = np.vstack([V[0], G[0], L[0]])  # value, gradient x/y/z, Laplacian
        cur = np.linalg.inv(det.slater_matrix(grid, coefs, R2))
        want = q @ cur[k]
        got = det.delayed_ratio(A0inv, phis, ks, int(k), q)
        scale = np.abs(q) @ np.abs(cur[k])
        assert np.max(np.abs(got - want) / scale) < 1e-9, step
        if ks:
            plain = q @ A0inv[k]
            assert np.max(np.abs(plain - want) / scale) > 1e-6  # the pending moves matter
        if step == 8:
            break
        phis.append(V[0])
        ks.append(int(k))
        R2[k] = rnew
    new = det.delayed_flush(A0inv, phis, ks)
    want = np.linalg.inv(det.slater_matrix(grid, coefs, R2))
    assert np.max(np.abs(new - want)) < 1e-8 * np.max(np.abs(want))
    # proposals for electrons that are themselves pending: the ratio against
    # the current matrix (row k of its inverse), which needs the correction
    for k in ks[:4]:
        rnew = rng.random(3)
        V, G, L = oracle.eval_vgl(grid, coefs, rnew[None])
        q = np.vstack([V[0], G[0], L[0]])
        want = q @ np.linalg.inv(det.slater_matrix(grid, coefs, R2))[k]
        got = det.delayed_ratio(A0inv, phis, ks, int(k), q)
        scale = np.abs(q) @ np.abs(np.linalg.inv(det.slater_matrix(grid, coefs, R2))[k])
        assert np.max(np.abs(got - want) / scale) < 1e-9, k


def test_general_cell_ratio(oracle):
    """ratio_vgl_lattice: equal to ratio_vgl for a diagonal lattice;
    covariant under a rotation of lattice and positions (value and Laplacian
    invariant, gradient rotated); and its derivatives are central differences
    of its value in a hexagonal cell."""
    from oracle import det

    rng = np.random.default_rng(31)
    grid = (9, 10, 11)
    N = 7
    coefs = rng.uniform(-1, 1, grid + (N,))
    rows = rng.standard_normal((12, N))
    cell = (1.0, 1.3, 0.8)
    pos = rng.uniform(0, 1, (12, 3)) * np.array(cell)
    np.testing.assert_allclose(det.ratio_vgl_lattice(grid, coefs, pos, rows, np.diag(cell)),
                               det.ratio_vgl(grid, coefs, pos, rows, cell), rtol=1e-11, atol=1e-9)
    hexl = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3.0) / 2.0, 0.0], [0.0, 0.0, 1.6]])
    frac = rng.uniform(0.05, 0.95, (12, 3))
    p = frac @ hexl
    D = det.ratio_vgl_lattice(grid, coefs, p, rows, hexl)
    t = 0.7
    Q = np.array([[np.cos(t), -np.sin(t), 0.0], [np.sin(t), np.cos(t), 0.0], [0.0, 0.0, 1.0]])
    Dr = det.ratio_vgl_lattice(grid, coefs, p @ Q.T, rows, hexl @ Q.T)
    np.testing.assert_allclose(Dr[:, 0], D[:, 0], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(Dr[:, 4], D[:, 4], rtol=1e-9, atol=1e-7)
    np.testing.assert_allclose(Dr[:, 1:4], D[:, 1:4] @ Q.T, rtol=1e-10, atol=1e-9)
    h1, h2 = 1e-6, 1e-3
    lap = np.zeros(len(p))
    for d in range(3):
        e = np.zeros(3)
        e[d] = 1.0
        fp = det.ratio_vgl_lattice(grid, coefs, p + h1 * e, rows, hexl)[:, 0]
        fm = det.ratio_vgl_lattice(grid, coefs, p - h1 * e, rows, hexl)[:, 0]
        np.testing.assert_allclose((fp - fm) / (2 * h1), D[:, 1 + d], rtol=1e-5, atol=1e-5 * np.abs(D[:, 1:4]).max())
        gp = det.ratio_vgl_lattice(grid, coefs, p + h2 * e, rows, hexl)[:, 0]
        gm = det.ratio_vgl_lattice(grid, coefs, p - h2 * e, rows, hexl)[:, 0]
        lap += (gp - 2 * D[:, 0] + gm) / h2 ** 2
    np.testing.assert_allclose(lap, D[:, 4], rtol=1e-3, atol=1e-3 * np.abs(D[:, 4]).max())
