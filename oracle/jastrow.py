"""Jastrow-factor oracle (test infrastructure only; FP64).

What it computes (Section 3, the Jastrow equation and the ratio equations;
Section 7, compute-on-the-fly distance tables and Jastrow):

  J = sum_I sum_i U_{s(I)}(|r_I - r_i|) + sum_{i<j} U_2(|r_i - r_j|)

with one-dimensional cubic B-spline functors U (Section 3: the functors are
1D cubic B-splines) that vanish beyond their cutoff.  Distances use the
minimum image of an orthorhombic periodic cell; every cutoff is at most half
the shortest cell length, so no other image is ever inside a cutoff.  The
two-body functor depends on the spins of the pair (electrons 0..n_up-1 are
up): functor ``uu`` for equal spins, ``ud`` otherwise.  The sum over pairs
counts each pair once, which is what the ratio equation's Delta J_2 (a sum
over i != k of the moved electron's pair terms) implies.

Functor reading (the paper gives no formula): M uniform intervals of width
h = rcut / M on [0, rcut), coefficients c_0 .. c_{M+2}, coefficient j
centred at r = (j - 1) h, and U(r) = sum_j c_j B(r / h - (j - 1)) for
0 <= r < rcut, 0 beyond; B is the centred cardinal cubic B-spline.  U' and U''
are derivatives in r.  A pair at distance 0 contributes U(0) to J and nothing
to the derivatives.

Derivatives with respect to electron k (the "derivatives" step of
Algorithm 1, and the kinetic term of the local energy):
  grad_k J = sum_pairs U'(d) (r_k - r_other) / d,
  lap_k J  = sum_pairs (U''(d) + 2 U'(d) / d).

Everything is written out term by term with numpy; pinned in
``tests/test_oracle_jastrow.py`` against scipy's B-splines, brute force over
periodic images, finite differences and the difference of two full
evaluations.
"""
from __future__ import annotations

import numpy as np


def bspline3(x):
    """Centred cardinal cubic B-spline and its first two derivatives."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    s = np.sign(x)
    b = np.where(a < 1, 2.0 / 3.0 - a * a + 0.5 * a ** 3, np.where(a < 2, (2 - a) ** 3 / 6.0, 0.0))
    db = np.where(a < 1, -2 * a + 1.5 * a * a, np.where(a < 2, -0.5 * (2 - a) ** 2, 0.0)) * s
    d2b = np.where(a < 1, -2 + 3 * a, np.where(a < 2, 2 - a, 0.0))
    return b, db, d2b


def functor(r, coefs, rcut):
    """(U, U', U'') at distances r for coefficients c_0..c_{M+2} on [0, rcut)."""
    c = np.asarray(coefs, dtype=np.float64)
    M = len(c) - 3
    h = rcut / M
    r = np.asarray(r, dtype=np.float64)
    u = np.zeros_like(r)
    du = np.zeros_like(r)
    d2u = np.zeros_like(r)
    for j in range(M + 3):
        b, db, d2b = bspline3(r / h - (j - 1))
        u += c[j] * b
        du += c[j] * db / h
        d2u += c[j] * d2b / h ** 2
    inside = r < rcut
    return np.where(inside, u, 0.0), np.where(inside, du, 0.0), np.where(inside, d2u, 0.0)


def min_image(dr, cell):
    """Minimum-image displacement in an orthorhombic cell."""
    L = np.asarray(cell, dtype=np.float64)
    return dr - L * np.round(dr / L)


class System:
    """Ions, spins and functors of one Jastrow factor.

    ions[n_ion, 3], species[n_ion] in [0, n_species); f1[s] = (coefs, rcut)
    for species s; uu, ud = (coefs, rcut) for the two-body terms.
    """

    def __init__(self, cell, ions, species, f1, uu, ud, n_up):
        self.cell = np.asarray(cell, dtype=np.float64)
        self.ions = np.asarray(ions, dtype=np.float64).reshape(-1, 3)
        self.species = np.asarray(species, dtype=np.int64)
        self.f1 = [(np.asarray(c, dtype=np.float64), float(rc)) for c, rc in f1]
        self.uu = (np.asarray(uu[0], dtype=np.float64), float(uu[1]))
        self.ud = (np.asarray(ud[0], dtype=np.float64), float(ud[1]))
        self.n_up = int(n_up)

    def _same_spin(self, i, j):
        return (np.asarray(i) < self.n_up) == (np.asarray(j) < self.n_up)

    def terms_of(self, R, k, r):
        """(sum of U, grad, lap) of the terms that involve electron k placed at
        r, all other electrons at R (the row of the distance tables for k)."""
        R = np.asarray(R, dtype=np.float64)
        r = np.asarray(r, dtype=np.float64)
        dri = min_image(r - self.ions, self.cell)
        v1, g1, l1 = 0.0, np.zeros(3), 0.0
        for s in range(len(self.f1)):
            sel = self.species == s
            if sel.any():
                a, b, c = _sum_functor(dri[sel], *self.f1[s])
                v1, g1, l1 = v1 + a, g1 + b, l1 + c
        others = np.array([i for i in range(len(R)) if i != k], dtype=np.int64)
        dre = min_image(r - R[others], self.cell)
        same = self._same_spin(k, others)
        v2, g2, l2 = 0.0, np.zeros(3), 0.0
        for sel, f in ((same, self.uu), (~same, self.ud)):
            if sel.any():
                a, b, c = _sum_functor(dre[sel], *f)
                v2, g2, l2 = v2 + a, g2 + b, l2 + c
        return v1 + v2, g1 + g2, l1 + l2

    def move(self, R, k, rnew):
        """(Delta J, grad_k J, lap_k J) for moving electron k to rnew: the
        ratio's exponent (the ratio equation's Delta J_1 + Delta J_2) and the
        derivatives at the new position."""
        v1, g1, l1 = self.terms_of(R, k, rnew)
        v0, _, _ = self.terms_of(R, k, R[k])
        return v1 - v0, g1, l1

    def evaluate(self, R):
        """(J, grad J [N, 3], lap J [N]) for all electrons of one walker.  J is
        the one-body sum plus half the sum, over electrons, of each electron's
        two-body terms (every pair counted once)."""
        R = np.asarray(R, dtype=np.float64)
        N = len(R)
        J = 0.0
        G = np.zeros((N, 3))
        Lp = np.zeros(N)
        for i in range(N):
            v, G[i], Lp[i] = self.terms_of(R, i, R[i])
            v1, _, _ = self.one_body(R[i])
            J += v1 + 0.5 * (v - v1)
        return J, G, Lp

    def one_body(self, r):
        dri = min_image(np.asarray(r, dtype=np.float64) - self.ions, self.cell)
        v, g, l = 0.0, np.zeros(3), 0.0
        for s in range(len(self.f1)):
            sel = self.species == s
            if sel.any():
                a, b, c = _sum_functor(dri[sel], *self.f1[s])
                v, g, l = v + a, g + b, l + c
        return v, g, l

    def rows(self, R, r):
        """Distance-table rows for a position r: (d, dr) to every electron
        [N], [N, 3] and to every ion [n_ion], [n_ion, 3], with dr = r_other - r
        (minimum image)."""
        R = np.asarray(R, dtype=np.float64)
        dre = min_image(R - np.asarray(r, dtype=np.float64), self.cell)
        dri = min_image(self.ions - np.asarray(r, dtype=np.float64), self.cell)
        return np.linalg.norm(dre, axis=1), dre, np.linalg.norm(dri, axis=1), dri


def _sum_functor(dr, coefs, rcut):
    """Sum over rows of dr[m, 3] (each pointing from the other particle to the
    electron whose derivatives are taken) of U(d), U'(d) dr / d and
    U''(d) + 2 U'(d) / d, d = |dr|; rows with d = 0 add U(0) only."""
    d = np.sqrt(np.sum(dr * dr, axis=1))
    u, du, d2u = functor(d, coefs, rcut)
    nz = d > 0.0
    g = np.sum((du[nz] / d[nz])[:, None] * dr[nz], axis=0)
    lap = float(np.sum(d2u[nz] + 2.0 * du[nz] / d[nz]))
    return float(np.sum(u)), g, lap
