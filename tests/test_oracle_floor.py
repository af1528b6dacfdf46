"""The surrogate's representational floor (CPU, FP64).

oracle.mlp.spline_fourier_coefficients gives the spline's Fourier series
from the definition of the tricubic spline and the transform of the cubic
B-spline; it is pinned against the discrete transform of the oracle's own
spline sampled on a fine grid (independent of the closed form), a constant
table, and finite differences of the truncated series.  The floor itself --
the error against the spline of the spline's series cut to the features'
|k| <= 4 ball -- is then measured on the 48^3 / N = 192 table that the
surrogate learns: what no approximant below the table's first alias band can
beat.  The network's own accuracy is parity unpinned (measured, reported).
"""
import numpy as np

import oracle
import workloads as W
from oracle import mlp as M


def test_constant_table():
    c = np.full((6, 7, 8, 2), 3.25)
    K, S = M.spline_fourier_coefficients(c, 2.0)
    z = np.flatnonzero((K == 0).all(1))
    assert len(z) == 1
    np.testing.assert_allclose(S[z[0]], [3.25, 3.25], atol=1e-14)
    S0 = np.delete(S, z[0], axis=0)
    assert np.abs(S0).max() < 1e-14
    pos = np.random.default_rng(0).uniform(-2, 3, (20, 3))
    V, G, L = M.bandlimited_vgl(c, pos, 2.0)
    np.testing.assert_allclose(V, 3.25, atol=1e-13)
    assert np.abs(G).max() < 1e-12 and np.abs(L).max() < 1e-11


def test_coefficients_match_sampled_transform():
    # the oracle's spline sampled 8 points per grid spacing on every axis;
    # the discrete transform of the samples equals the Fourier series up to
    # aliases 8 grids away, ~1e-6 of the largest coefficient here
    rng = np.random.default_rng(5)
    n = (8, 6, 10)
    N = 2
    c = rng.uniform(-1, 1, n + (N,))
    Mg = tuple(8 * x for x in n)
    axes = [np.arange(m) / m for m in Mg]
    P = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    Vs = oracle.eval_v(n, c, P).reshape(Mg + (N,))
    F = np.fft.fftn(Vs, axes=(0, 1, 2)) / float(np.prod(Mg))
    K, S = M.spline_fourier_coefficients(c, 2.5)
    got = F[K[:, 0] % Mg[0], K[:, 1] % Mg[1], K[:, 2] % Mg[2]]
    scale = np.abs(S).max()
    assert scale > 1e-2  # not a trivially small spectrum
    # a centre shifted by a grid point (a phase exp(2 pi i k/n)) or another
    # power of sinc would miss by a sizable fraction of the coefficients
    assert np.abs(got - S).max() <= 1e-5 * scale, np.abs(got - S).max() / scale


def test_truncated_series_derivatives_fd():
    rng = np.random.default_rng(6)
    c = rng.uniform(-1, 1, (8, 8, 8, 3))
    cell = (1.3, 0.9, 1.1)
    pos = rng.uniform(0, 1, (12, 3)) * np.array(cell)
    V, G, L = M.bandlimited_vgl(c, pos, 3.0, cell)
    h = 1e-4
    lap = np.zeros_like(V)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        vp = [M.bandlimited_vgl(c, pos + k * e, 3.0, cell)[0] for k in (-2, -1, 1, 2)]
        g = (-vp[3] + 8 * vp[2] - 8 * vp[1] + vp[0]) / (12 * h)
        np.testing.assert_allclose(G[:, d], g, rtol=1e-6, atol=1e-6 * np.abs(G).max())
        lap += (vp[2] - 2 * V + vp[1]) / (h * h)
    np.testing.assert_allclose(L, lap, rtol=1e-4, atol=1e-4 * np.abs(L).max())


def test_floor_of_the_surrogate_table():
    grid, N, coefs, _ = W.make_table(5)
    # the fitted table is band-limited to the generator's |G| <= 4 ball:
    # every other component of the spline is an alias k + 48 a
    chat = np.fft.fftn(coefs, axes=(0, 1, 2))
    ks = [np.fft.fftfreq(g, 1.0 / g) for g in grid]
    KK = np.stack(np.meshgrid(*ks, indexing="ij"), -1)
    outside = (KK ** 2).sum(-1) > 16.0 + 1e-9
    assert np.abs(chat[outside]).max() <= 1e-9 * np.abs(chat).max()

    pos = W.mlp_samples(5, count=2000, validation=True)
    ref = oracle.eval_vgl(grid, coefs, pos)
    got = M.bandlimited_vgl(coefs, pos, 4.0)
    eps = [oracle.rel_err(g, r) for g, r in zip(got, ref)]
    rms = [oracle.rel_rms(g, r) for g, r in zip(got, ref)]
    print("band-limited floor vs the spline: eps V/G/L = %.2e %.2e %.2e, rel RMS %.2e %.2e %.2e"
          % tuple(eps + rms))
    # values and gradients could meet 1e-3 in principle; the Laplacian cannot:
    # the spline's own Laplacian carries alias components of ~1% of its size
    assert eps[0] < 1e-4 and eps[1] < 1e-3
    assert eps[2] > 5e-3 and rms[2] > 2e-3
