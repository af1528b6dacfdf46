"""Pins of the Jastrow oracle (oracle/jastrow.py) against facts outside it:
scipy's Cox-de Boor cubic B-spline, exact reproduction of constants and
straight lines by the functor, the cutoff, brute force over the 27 nearest
periodic images, central differences of the full Jastrow value in one
electron's coordinates (gradient and Laplacian), the move's Delta J as the
difference of two full evaluations, and spin-resolved two-body functors.
"""
import numpy as np
import pytest

import workloads as W


def _system(n_elec=12, n_up=None, seed=6):
    from oracle import jastrow as oj

    d = W.make_jastrow(seed=seed, n_elec=n_elec, n_up=n_up)
    return oj.System(d["cell"], d["ions"], d["species"], d["f1"], d["uu"], d["ud"], d["n_up"]), d


def test_bspline_matches_cox_de_boor():
    from scipy.interpolate import BSpline

    from oracle import jastrow as oj

    B = BSpline.basis_element(np.arange(5.0), extrapolate=False)
    x = np.linspace(-2.5, 2.5, 201)
    b, db, d2b = oj.bspline3(x)
    ref = np.nan_to_num(B(x + 2.0))
    np.testing.assert_allclose(b, ref, atol=1e-14)
    inside = np.abs(x) < 2
    np.testing.assert_allclose(db[inside], np.nan_to_num(B.derivative(1)(x[inside] + 2.0)), atol=1e-13)
    np.testing.assert_allclose(d2b[inside], np.nan_to_num(B.derivative(2)(x[inside] + 2.0)), atol=1e-12)


def test_functor_reproduces_constants_and_lines_and_cuts_off():
    from oracle import jastrow as oj

    M, rc = 7, 0.45
    h = rc / M
    r = np.linspace(0, rc, 300, endpoint=False)
    u, du, d2u = oj.functor(r, np.ones(M + 3), rc)
    np.testing.assert_allclose(u, 1.0, atol=1e-14)
    np.testing.assert_allclose(du, 0.0, atol=1e-12)
    c = (np.arange(M + 3) - 1.0) * h  # coefficient j centred at (j - 1) h
    u, du, d2u = oj.functor(r, c, rc)
    np.testing.assert_allclose(u, r, atol=1e-14)
    np.testing.assert_allclose(du, 1.0, atol=1e-12)
    np.testing.assert_allclose(d2u, 0.0, atol=1e-9)
    u, du, d2u = oj.functor(np.array([rc, rc + 0.1, 2.0]), np.ones(M + 3), rc)
    assert np.all(u == 0) and np.all(du == 0) and np.all(d2u == 0)


def test_functor_derivatives_by_central_differences():
    from oracle import jastrow as oj

    _, d = _system()
    c, rc = d["uu"]
    r = np.linspace(0.01, rc - 0.01, 97)
    h = 1e-6
    u, du, d2u = oj.functor(r, c, rc)
    up, dup, _ = oj.functor(r + h, c, rc)
    um, dum, _ = oj.functor(r - h, c, rc)
    np.testing.assert_allclose((up - um) / (2 * h), du, atol=1e-6 * np.abs(du).max())
    np.testing.assert_allclose((dup - dum) / (2 * h), d2u, atol=1e-5 * np.abs(d2u).max())


def test_minimum_image_is_the_nearest_of_27_images():
    from oracle import jastrow as oj

    rng = np.random.default_rng(1)
    cell = np.array([1.0, 1.3, 0.8])
    dr = rng.uniform(-3, 3, size=(500, 3))
    mi = oj.min_image(dr, cell)
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]) * cell
    best = np.min(np.linalg.norm(mi[:, None, :] + shifts[None], axis=2), axis=1)
    np.testing.assert_allclose(np.linalg.norm(mi, axis=1), best, atol=1e-12)
    assert np.all(np.abs(mi) <= cell / 2 + 1e-12)


@pytest.mark.parametrize("k", [0, 5, 11])
def test_derivatives_are_derivatives_of_the_full_value(k):
    """grad_k J and lap_k J by central differences of J(R)."""
    sysj, d = _system()
    R = W.make_electrons(1, d["n_elec"])[0]
    J, G, Lp = sysj.evaluate(R)
    h = 1e-5
    lap = 0.0
    for a in range(3):
        Rp, Rm = R.copy(), R.copy()
        Rp[k, a] += h
        Rm[k, a] -= h
        Jp, Jm = sysj.evaluate(Rp)[0], sysj.evaluate(Rm)[0]
        assert abs((Jp - Jm) / (2 * h) - G[k, a]) < 1e-6 * max(1.0, np.abs(G).max())
        lap += (Jp - 2 * J + Jm) / h ** 2
    assert abs(lap - Lp[k]) < 1e-3 * max(1.0, np.abs(Lp).max())


def test_move_is_the_difference_of_two_evaluations():
    sysj, d = _system()
    R = W.make_electrons(1, d["n_elec"])[0]
    k, disp = W.make_moves(5, d["n_elec"])
    for kk, dd in zip(k, disp):
        R2 = R.copy()
        R2[kk] = R[kk] + dd
        dJ, g, lap = sysj.move(R, kk, R2[kk])
        J0 = sysj.evaluate(R)[0]
        J1, G1, L1 = sysj.evaluate(R2)
        assert abs(dJ - (J1 - J0)) < 1e-12 * max(1.0, abs(J0))
        np.testing.assert_allclose(g, G1[kk], atol=1e-12)
        assert abs(lap - L1[kk]) < 1e-10


def test_spins_select_the_two_body_functor():
    """Swapping which electrons are up changes J exactly as the functor
    choice predicts: with uu == ud the spin split does not matter."""
    from oracle import jastrow as oj

    s1, d = _system(n_up=6)
    s2, _ = _system(n_up=3)
    R = W.make_electrons(1, d["n_elec"])[0]
    assert abs(s1.evaluate(R)[0] - s2.evaluate(R)[0]) > 1e-6
    same1 = oj.System(d["cell"], d["ions"], d["species"], d["f1"], d["uu"], d["uu"], 6)
    same2 = oj.System(d["cell"], d["ions"], d["species"], d["f1"], d["uu"], d["uu"], 3)
    assert abs(same1.evaluate(R)[0] - same2.evaluate(R)[0]) < 1e-12


def test_rows_are_minimum_image_distances():
    sysj, d = _system()
    R = W.make_electrons(1, d["n_elec"])[0]
    de, dre, di, dri = sysj.rows(R, R[3])
    assert de[3] == 0.0
    np.testing.assert_allclose(de, np.linalg.norm(dre, axis=1))
    assert np.all(de <= np.sqrt(3) / 2 + 1e-12) and np.all(di <= np.sqrt(3) / 2 + 1e-12)
