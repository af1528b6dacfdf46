"""Pins of the oracle's general-cell value / gradient / Hessian
(oracle.eval_vgh).

Checked against facts outside the function: the orthorhombic oracle (itself
pinned in test_oracle_pins.py) at the fractional coordinates of a position;
central differences of the value and of the gradient in Cartesian directions
(interior positions, where the spline is a polynomial along any line);
rotation covariance (V invariant, G -> Q G, H -> Q H Q^T when lattice and
positions rotate together), which a transposed inverse lattice fails;
periodicity under every lattice vector; and the orthorhombic Laplacian as the
trace of H.
"""
import numpy as np
import pytest

import workloads as W

HEX = np.array([[1.0, 0.0, 0.0], [-0.5, np.sqrt(3.0) / 2.0, 0.0], [0.0, 0.0, 1.6]])  # graphite-like
TRI = np.array([[1.1, 0.1, -0.2], [0.3, 0.9, 0.15], [-0.1, 0.25, 1.3]])
LATTICES = {"hexagonal": HEX, "triclinic": TRI}


def _table():
    grid, N, coefs, _ = W.make_table(1)  # 16^3, 32 orbitals, c ~ U[-1, 1]
    return grid, coefs


def _interior_fractional(rng, count, grid, lo=0.25, hi=0.75):
    g = np.asarray(grid)
    return (rng.integers(0, g, size=(count, 3)) + rng.uniform(lo, hi, size=(count, 3))) / g


def test_orthorhombic_lattice_matches_vgl_oracle(oracle):
    grid, coefs = _table()
    cell = (1.0, 1.3, 0.8)
    pos = np.random.default_rng(0).random((200, 3)) * cell
    V, G, L = oracle.eval_vgl(grid, coefs, pos, cell)
    V2, G2, H = oracle.eval_vgh(grid, coefs, pos, np.diag(cell))
    s = np.abs(L).max()
    np.testing.assert_allclose(V2, V, rtol=0, atol=1e-13)
    np.testing.assert_allclose(G2, G, rtol=0, atol=1e-12 * np.abs(G).max())
    np.testing.assert_allclose(H[:, 0] + H[:, 3] + H[:, 5], L, rtol=0, atol=1e-12 * s)


@pytest.mark.parametrize("name", list(LATTICES))
def test_value_is_the_cube_spline_at_fractional_coordinates(oracle, name):
    lat = LATTICES[name]
    grid, coefs = _table()
    u = np.random.default_rng(1).random((300, 3)) * 3 - 1  # several periods
    V, _, _ = oracle.eval_vgh(grid, coefs, u @ lat, lat)
    Vc = oracle.eval_v(grid, coefs, u, (1.0, 1.0, 1.0))
    np.testing.assert_allclose(V, Vc, rtol=0, atol=1e-12)


@pytest.mark.parametrize("name", list(LATTICES))
def test_gradient_and_hessian_by_central_differences(oracle, name):
    lat = LATTICES[name]
    grid, coefs = _table()
    rng = np.random.default_rng(2)
    r = _interior_fractional(rng, 40, grid) @ lat
    V, G, H = oracle.eval_vgh(grid, coefs, r, lat)
    h = 1e-5
    hc = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        Vp, Gp, _ = oracle.eval_vgh(grid, coefs, r + e, lat)
        Vm, Gm, _ = oracle.eval_vgh(grid, coefs, r - e, lat)
        fd = (Vp - Vm) / (2 * h)
        assert np.max(np.abs(fd - G[:, c])) < 1e-6 * np.abs(G).max()
        fdh = (Gp - Gm) / (2 * h)  # d G_x / d r_c etc.
        for k, (a, b) in enumerate(hc):
            if b == c:
                assert np.max(np.abs(fdh[:, a] - H[:, k])) < 1e-6 * np.abs(H).max(), (name, a, b)
            if a == c:
                assert np.max(np.abs(fdh[:, b] - H[:, k])) < 1e-6 * np.abs(H).max(), (name, a, b)


@pytest.mark.parametrize("name", list(LATTICES))
def test_rotation_covariance(oracle, name):
    lat = LATTICES[name]
    grid, coefs = _table()
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    r = rng.random((100, 3)) * 2
    V, G, H = oracle.eval_vgh(grid, coefs, r, lat)
    V2, G2, H2 = oracle.eval_vgh(grid, coefs, r @ Q.T, lat @ Q.T)
    np.testing.assert_allclose(V2, V, rtol=0, atol=1e-12)
    np.testing.assert_allclose(G2, np.einsum("cd,bdn->bcn", Q, G), rtol=0, atol=1e-11 * np.abs(G).max())
    idx = np.array([[0, 1, 2], [1, 3, 4], [2, 4, 5]])
    Hf = H[:, idx]  # [B,3,3,N]
    Hr = np.einsum("ca,ed,badn->bcen", Q, Q, Hf)
    H2f = H2[:, idx]
    np.testing.assert_allclose(H2f, Hr, rtol=0, atol=1e-11 * np.abs(H).max())


@pytest.mark.parametrize("name", list(LATTICES))
def test_periodic_under_lattice_vectors(oracle, name):
    lat = LATTICES[name]
    grid, coefs = _table()
    r = _interior_fractional(np.random.default_rng(4), 60, grid) @ lat
    ref = oracle.eval_vgh(grid, coefs, r, lat)
    for d in range(3):
        for k in (-2, 1, 3):
            got = oracle.eval_vgh(grid, coefs, r + k * lat[d], lat)
            for a, b in zip(got, ref):
                np.testing.assert_allclose(a, b, rtol=0, atol=1e-10 * np.abs(b).max())


def test_singular_lattice_rejected(oracle):
    grid, coefs = _table()
    with pytest.raises(ValueError):
        oracle.eval_vgh(grid, coefs, np.zeros((1, 3)), np.array([[1, 0, 0], [2, 0, 0], [0, 0, 1.0]]))
