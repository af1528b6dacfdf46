"""Seeded synthetic inputs for the tricubic B-spline orbital workloads.

This module generates inputs only: coefficient tables, positions, walker
counts, and the random draws of the surrogate network (initial weights,
Fourier frequencies, training and validation samples).  It evaluates no
B-spline and no network; both the CPU oracle and the GPU library consume what
it returns, and neither is imported here.

Workloads (the paper's benchmark systems in Table 1 need DFT orbitals that are
not available, so smooth plane-wave orbitals on the same FFT grids stand in;
the 80^3 grid with 384 orbitals mirrors the NiO-32 supercell of Table 1):

  C1  16^3 grid, N=32, coefficients i.i.d. U[-1,1], 1000 positions U[0,1)^3
  C2  48^3 grid, N=192, plane-wave orbitals fitted by periodic interpolation,
      256 walkers x 192 electrons
  C3  80^3 grid, N=384, same generator, 512 walkers x 384 electrons
  C4  four tables 32^3/48^3/64^3/80^3 with N=64/128/256/384, walker counts
      U{64..1024} per table, electrons per walker = N of the table
  C5  the C2 table, with the surrogate's draws

Seeds: ``SeedSequence(k)`` for workload k, spawned into seven streams used in
a fixed order: 0 coefficients/orbitals, 1 positions, 2 walker counts,
3 surrogate initialisation, 4 surrogate training samples, 5 validation
samples, 6 rows of inverse Slater matrices (determinant-ratio workloads).
"""
from __future__ import annotations

import numpy as np

(STREAM_COEFS, STREAM_POS, STREAM_WALKERS, STREAM_MLP_INIT, STREAM_MLP_TRAIN, STREAM_MLP_VAL,
 STREAM_AINV) = range(7)

WORKLOADS = {
    1: dict(grid=(16, 16, 16), norb=32, walkers=1, electrons=1000, kind="uniform"),
    2: dict(grid=(48, 48, 48), norb=192, walkers=256, electrons=192, kind="planewave"),
    3: dict(grid=(80, 80, 80), norb=384, walkers=512, electrons=384, kind="planewave"),
    5: dict(grid=(48, 48, 48), norb=192, walkers=256, electrons=192, kind="planewave"),
}
RAGGED_TABLES = [((32, 32, 32), 64), ((48, 48, 48), 128), ((64, 64, 64), 256), ((80, 80, 80), 384)]


def rngs(k: int, seed: int | None = None) -> list[np.random.Generator]:
    """Seven independent generators for workload ``k`` (``seed`` overrides k).
    Child i of the seed sequence does not depend on how many are spawned."""
    ss = np.random.SeedSequence(k if seed is None else seed)
    return [np.random.default_rng(s) for s in ss.spawn(7)]


def gvectors(rmax: int = 4) -> np.ndarray:
    """All integer 3-vectors with |G|_2 <= rmax (257 of them for rmax=4)."""
    r = np.arange(-rmax, rmax + 1)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    return g[(g * g).sum(1) <= rmax * rmax].astype(np.int64)


def planewave_params(rng: np.random.Generator, norb: int, nq: int = 16, rmax: int = 4):
    """Orbital m = sum over q of alpha cos(2 pi G.r) + beta sin(2 pi G.r).

    G is drawn with replacement from the integer vectors with |G| <= rmax,
    alpha and beta are N(0,1).  Returns (G[norb,nq,3], alpha[norb,nq], beta[norb,nq]).
    """
    pool = gvectors(rmax)
    G = pool[rng.integers(0, len(pool), size=(norb, nq))]
    alpha = rng.standard_normal((norb, nq))
    beta = rng.standard_normal((norb, nq))
    return G, alpha, beta


def planewave_values(G, alpha, beta, r, cell=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Analytic orbitals at positions r[B,3] -> [B, norb] (direct sum)."""
    r = np.asarray(r, dtype=np.float64) / np.asarray(cell, dtype=np.float64)
    ph = 2.0 * np.pi * np.einsum("bd,mqd->bmq", r, G.astype(np.float64))
    return (alpha[None] * np.cos(ph) + beta[None] * np.sin(ph)).sum(-1)


def fit_planewave_coefs(grid, G, alpha, beta) -> np.ndarray:
    """Periodic cubic-spline interpolation coefficients of plane-wave orbitals.

    A plane wave exp(2 pi i g j / n) sampled on the grid is an eigenvector of
    the circulant interpolation system whose stencil is (1, 4, 1)/6, with
    eigenvalue (4 + 2 cos(2 pi g / n)) / 6 >= 1/3; each term is divided by the
    product of those eigenvalues over the three axes.  Evaluated separably as
    three small complex contractions over the 9 frequencies per axis.
    Returns coefs[n0, n1, n2, norb] (orbital fastest), float64.
    """
    n0, n1, n2 = grid
    norb, nq, _ = G.shape
    rmax = int(np.abs(G).max()) if G.size else 0
    nf = 2 * rmax + 1
    lam = []
    E = []
    for d, n in enumerate(grid):
        g = np.arange(-rmax, rmax + 1)
        lam.append((4.0 + 2.0 * np.cos(2.0 * np.pi * g / n)) / 6.0)
        j = np.arange(n)
        E.append(np.exp(2j * np.pi * np.outer(g, j) / n))  # [nf, n]
    A = np.zeros((norb, nf, nf, nf), dtype=np.complex128)
    gi = G + rmax
    amp = (alpha - 1j * beta) / (lam[0][gi[..., 0]] * lam[1][gi[..., 1]] * lam[2][gi[..., 2]])
    m = np.repeat(np.arange(norb), nq)
    np.add.at(A, (m, gi[..., 0].ravel(), gi[..., 1].ravel(), gi[..., 2].ravel()), amp.ravel())
    T1 = np.einsum("mabc,cz->mabz", A, E[2])          # [m, g0, g1, j2]
    T2 = np.einsum("mabz,by->ayzm", T1, E[1])          # [g0, j1, j2, m]
    T2 = T2.reshape(nf, n1 * n2 * norb)                  # [g0, (j1, j2, m)]
    re, im = np.ascontiguousarray(T2.real), np.ascontiguousarray(T2.imag)
    out = np.ascontiguousarray(E[0].real.T) @ re
    out -= np.ascontiguousarray(E[0].imag.T) @ im           # [j0, (j1, j2, m)]
    return out.reshape(n0, n1, n2, norb)


def positions(rng: np.random.Generator, count: int, cell=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Uniform positions in the cell, [count, 3] float64, walker-major order."""
    return rng.random((count, 3)) * np.asarray(cell, dtype=np.float64)


def make_table(k: int, seed: int | None = None):
    """(grid, norb, coefs[n0,n1,n2,norb], extras) for workloads 1, 2, 3, 5."""
    w = WORKLOADS[k]
    r = rngs(k, seed)
    grid, norb = w["grid"], w["norb"]
    if w["kind"] == "uniform":
        coefs = r[STREAM_COEFS].uniform(-1.0, 1.0, size=grid + (norb,))
        return grid, norb, coefs, {}
    G, a, b = planewave_params(r[STREAM_COEFS], norb)
    coefs = fit_planewave_coefs(grid, G, a, b)
    return grid, norb, coefs, dict(G=G, alpha=a, beta=b)


def make_positions(k: int, seed: int | None = None, count: int | None = None) -> np.ndarray:
    w = WORKLOADS[k]
    r = rngs(k, seed)
    return positions(r[STREAM_POS], w["walkers"] * w["electrons"] if count is None else count)


def make_ragged(seed: int = 4, tables=RAGGED_TABLES, wmin: int = 64, wmax: int = 1024):
    """Workload C4: per-table (grid, norb, coefs, positions, walkers).

    Walker counts are U{wmin..wmax}; each walker carries norb electrons.
    """
    r = rngs(4, seed)
    W = r[STREAM_WALKERS].integers(wmin, wmax + 1, size=len(tables))
    out = []
    for (grid, norb), w in zip(tables, W):
        G, a, b = planewave_params(r[STREAM_COEFS], norb)
        coefs = fit_planewave_coefs(grid, G, a, b)
        pos = positions(r[STREAM_POS], int(w) * norb)
        out.append(dict(grid=grid, norb=norb, coefs=coefs, pos=pos, walkers=int(w)))
    return out


def fourier_frequencies(rng: np.random.Generator, count: int = 48, rmax: int = 4) -> np.ndarray:
    """``count`` distinct integer vectors with 1 <= |k| <= rmax, [count, 3] int."""
    pool = gvectors(rmax)
    pool = pool[(pool * pool).sum(1) > 0]
    return pool[np.sort(rng.choice(len(pool), size=count, replace=False))]


def mlp_init(k: int = 5, seed: int | None = None, widths=(96, 256, 256, 192), nfreq: int = 48):
    """Frequencies and He-style initial weights/biases of the surrogate network."""
    r = rngs(k, seed)[STREAM_MLP_INIT]
    freqs = fourier_frequencies(r, nfreq)
    Ws, bs = [], []
    for fin, fout in zip(widths[:-1], widths[1:]):
        Ws.append(r.standard_normal((fout, fin)) * np.sqrt(2.0 / fin))
        bs.append(np.zeros(fout))
    return freqs, Ws, bs


def mlp_samples(k: int = 5, seed: int | None = None, count: int = 10**6, validation: bool = False):
    r = rngs(k, seed)[STREAM_MLP_VAL if validation else STREAM_MLP_TRAIN]
    return positions(r, count)


def make_inverse_rows(k: int, count: int, norb: int, seed: int | None = None, dtype=np.float32) -> np.ndarray:
    """[count][norb] stand-ins for rows of inverse Slater matrices: i.i.d.
    N(0, 1/norb) entries (the size of the entries of the inverse of a
    well-conditioned norb x norb matrix with O(1) entries).  Used where only
    the shape and magnitude of the rows matter (throughput, sampled parity);
    tests that need actual inverses build them from the oracle's matrices."""
    r = rngs(k, seed)[STREAM_AINV]
    out = np.empty((count, norb), dtype=dtype)
    step = max(1, (1 << 24) // max(1, norb))
    for i in range(0, count, step):
        j = min(count, i + step)
        out[i:j] = r.standard_normal((j - i, norb), dtype=np.float64 if dtype == np.float64 else np.float32)
    out *= np.asarray(1.0 / np.sqrt(norb), dtype=dtype)
    return out


# Jastrow workload (J1 + J2 with 1D cubic B-spline functors), seeded by
# SeedSequence(6): stream 0 functor coefficients, stream 1 electron
# positions, stream 2 proposed moves and moved electrons.
JASTROW = dict(cell=(1.0, 1.0, 1.0), n_elec=384, n_up=192, ion_grid=4, intervals=8, rcut=0.5, walkers=512)


def make_jastrow(seed: int = 6, n_elec: int | None = None, n_up: int | None = None, intervals: int | None = None,
                 rcut: float | None = None, cell=None):
    """Ions, species and functors of the Jastrow workload.

    32 ions on the sites of a 4x4x4 grid with even index sum (an fcc
    arrangement in the unit cube, as in a rock-salt oxide's cation or anion
    sublattice), two species alternating with the x index (the paper's NiO:
    Ni and O); n_elec electrons, the first n_up spin up.  Functors: M
    intervals on [0, rcut), the last three coefficients zero (U, U', U''
    vanish at the cutoff), the others a decaying cubic profile of seeded
    amplitude.  Returns dict(cell, ions, species, f1=[(c, rcut)]*2, uu, ud,
    n_elec, n_up)."""
    w = JASTROW
    cell = tuple(cell or w["cell"])
    n_elec = n_elec or w["n_elec"]
    n_up = n_elec // 2 if n_up is None else n_up
    M = intervals or w["intervals"]
    rcut = rcut or w["rcut"]
    r = rngs(6, seed)[0]
    g = w["ion_grid"]
    sites = [(i, j, k) for i in range(g) for j in range(g) for k in range(g) if (i + j + k) % 2 == 0]
    ions = (np.array(sites, dtype=np.float64) + 0.5) / g * np.asarray(cell)
    species = np.array([s[0] % 2 for s in sites], dtype=np.int32)

    def profile(amp):
        x = np.arange(M + 3, dtype=np.float64)
        c = amp * np.clip(1.0 - (x - 1.0) / M, 0.0, None) ** 3 * (1.0 + 0.1 * r.uniform(-1, 1, size=M + 3))
        c[M:] = 0.0
        return c

    f1 = [(profile(-1.5), rcut), (profile(-0.8), rcut)]
    uu = (profile(-0.25), rcut)
    ud = (profile(-0.5), rcut)
    return dict(cell=cell, ions=ions, species=species, f1=f1, uu=uu, ud=ud, n_elec=n_elec, n_up=n_up)


def make_electrons(walkers: int, n_elec: int, seed: int = 6, cell=(1.0, 1.0, 1.0)) -> np.ndarray:
    """[walkers][n_elec][3] uniform positions in the cell."""
    r = rngs(6, seed)[1]
    return r.random((walkers, n_elec, 3)) * np.asarray(cell)


def make_moves(walkers: int, n_elec: int, step: float = 0.05, seed: int = 6):
    """(k[walkers] int32, displacement[walkers][3]): one proposed move per
    walker, a Gaussian step of standard deviation `step` per coordinate."""
    r = rngs(6, seed)[2]
    k = r.integers(0, n_elec, size=walkers).astype(np.int32)
    return k, r.normal(scale=step, size=(walkers, 3))
