"""Determinant-ratio oracle (test infrastructure only; FP64).

Section 3 of the paper: the Slater matrix is A(i, j) = phi_i(r_j).  Moving
electron k from r_k to r'_k replaces column k of A by phi(r'_k); by the matrix
determinant lemma the determinant changes by the factor

    det A' / det A = sum_i Ainv(k, i) phi_i(r'_k),

the dot product of row k of A^-1 with the orbital values at the new position.
The gradient and the Laplacian of det A' with respect to r'_k, divided by
det A, are the same dot product with the orbital gradients and Laplacians
(the "derivatives" step of Algorithm 1), because det A' is linear in column k.

When the move is accepted, A^-1 is updated with the Sherman-Morrison
formula (``sherman_morrison``).

Everything here is the plain definition: the orbital V, G, L from the FP64
spline oracle, then one dot product per position with the given row; the
update is the rank-one formula written out.  Pinned in
``tests/test_oracle_det.py`` against determinants and inverses computed
directly with ``numpy.linalg`` (ratio, update) and against central
differences of those determinants (gradient, Laplacian).
"""
from __future__ import annotations

import numpy as np

from . import eval_v, eval_vgh, eval_vgl


def slater_matrix(grid, coefs: np.ndarray, R: np.ndarray, cell=(1.0, 1.0, 1.0)) -> np.ndarray:
    """A[i, j] = phi_i(r_j) for the n = len(R) electrons of one walker (the
    first n orbitals of the table)."""
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    n = R.shape[0]
    V = eval_v(grid, coefs, R, cell)  # V[j, i] = phi_i(r_j)
    return np.ascontiguousarray(V[:, :n].T)


def ratio_vgl(grid, coefs: np.ndarray, pos: np.ndarray, rows: np.ndarray, cell=(1.0, 1.0, 1.0)) -> np.ndarray:
    """D[B, 5]: for position b and its row a = rows[b] (length N, the table's
    orbital count), (sum a V, sum a Gx, sum a Gy, sum a Gz, sum a L)."""
    V, G, L = eval_vgl(grid, coefs, pos, cell)
    a = np.asarray(rows, dtype=np.float64).reshape(V.shape)
    D = np.empty((V.shape[0], 5))
    D[:, 0] = np.sum(a * V, axis=1)
    for d in range(3):
        D[:, 1 + d] = np.sum(a * G[:, d, :], axis=1)
    D[:, 4] = np.sum(a * L, axis=1)
    return D


def ratio_vgl_lattice(grid, coefs: np.ndarray, pos: np.ndarray, rows: np.ndarray, lattice) -> np.ndarray:
    """ratio_vgl in a general cell (rows of `lattice` are the Cartesian
    lattice vectors): the orbital values, Cartesian gradients and Laplacians
    (the trace of the Cartesian Hessian) from the general-cell oracle, each
    dotted with the position's row."""
    V, G, H = eval_vgh(grid, coefs, pos, lattice)
    L = H[:, 0] + H[:, 3] + H[:, 5]  # xx + yy + zz
    a = np.asarray(rows, dtype=np.float64).reshape(V.shape)
    D = np.empty((V.shape[0], 5))
    D[:, 0] = np.sum(a * V, axis=1)
    for d in range(3):
        D[:, 1 + d] = np.sum(a * G[:, d, :], axis=1)
    D[:, 4] = np.sum(a * L, axis=1)
    return D


def ratio_v(grid, coefs: np.ndarray, pos: np.ndarray, rows: np.ndarray, cell=(1.0, 1.0, 1.0)) -> np.ndarray:
    """R[B]: sum_i rows[b, i] phi_i(pos_b)."""
    V = eval_v(grid, coefs, pos, cell)
    a = np.asarray(rows, dtype=np.float64).reshape(V.shape)
    return np.sum(a * V, axis=1)


def ratio_scale(rows: np.ndarray, Qref_max: np.ndarray) -> np.ndarray:
    """sum_i |a_i| M_i per position: the size against which an error in a dot
    product of a row with orbital quantities of per-orbital magnitude M_i is
    measured (an error of e * M_i in every orbital moves the dot product by at
    most e times this)."""
    return np.abs(np.asarray(rows, dtype=np.float64)) @ np.asarray(Qref_max, dtype=np.float64)


def sherman_morrison(ainv: np.ndarray, k: int, phi: np.ndarray) -> np.ndarray:
    """Inverse after the move of electron k is accepted (Section 3: A^-1 is
    updated with the Sherman-Morrison formula).  Column k of A becomes phi =
    (phi_1(r'_k), ..., phi_n(r'_k)); with t = A^-1 phi and rho = t_k (the
    determinant ratio), the new inverse is A^-1 - (t - e_k) (row k of A^-1) / rho."""
    a = np.asarray(ainv, dtype=np.float64)
    t = a @ np.asarray(phi, dtype=np.float64)
    u = t.copy()
    u[k] -= 1.0
    return a - np.outer(u, a[k]) / t[k]


def delayed_ratio(ainv0: np.ndarray, phis, ks, k: int, q: np.ndarray) -> np.ndarray:
    """Ratio (and, for q of several rows, the derivative sums) for moving
    electron k while j accepted moves are pending against the stale inverse
    ainv0 (the delayed update of the paper's outlook, built on the Woodbury
    identity): with a_i the rows of ainv0, phis[i] the orbital vector accepted
    for electron ks[i], S[i][l] = a_{ks[i]} . phis[l], t[i] = a_k . phis[i]
    - [ks[i] == k] and y[i] = a_{ks[i]} . q, the result is a_k . q -
    t^T S^-1 y: q dotted with row k of the current inverse ainv0 - (ainv0 Phi
    - Q) S^-1 R (the Woodbury form; the [ks[i] == k] term is row k of Q, so an
    electron that is itself pending gets its ratio against the current
    matrix).  q: [n] or [m, n] (one result per row).  The electrons ks must
    be distinct."""
    a = np.asarray(ainv0, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    x = q @ a[k]
    j = len(ks)
    if j == 0:
        return x
    P = np.asarray(phis, dtype=np.float64).reshape(j, -1)
    R = a[list(ks)]
    S = R @ P.T
    t = P @ a[k] - (np.asarray(ks) == k).astype(np.float64)
    y = q @ R.T  # [..., j]
    return x - y @ np.linalg.solve(S.T, t)


def delayed_flush(ainv0: np.ndarray, phis, ks) -> np.ndarray:
    """The inverse after the pending moves: ainv0 - (T - Q) S^-1 R with
    T = ainv0 Phi (columns phis), Q = columns e_{ks}, R = rows ks of ainv0."""
    a = np.asarray(ainv0, dtype=np.float64)
    j = len(ks)
    if j == 0:
        return a.copy()
    P = np.asarray(phis, dtype=np.float64).reshape(j, -1)
    R = a[list(ks)]
    T = a @ P.T
    Q = np.zeros_like(T)
    Q[list(ks), np.arange(j)] = 1.0
    S = R @ P.T
    return a - (T - Q) @ np.linalg.solve(S, R)
