"""The surrogate's feature selection (spline_mlp_select_frequencies, host
code of the library, no GPU) against numpy's FFT of the coefficient table.

numpy.fft.fftn gives the same discrete Fourier transform by a different
algorithm; energies must agree to rounding, and the chosen pairs must be the
most energetic ones (pairs whose energies tie within rounding at the cutoff
may come in either order)."""
import numpy as np
import pytest

import paper_1708_02645_amd as q
import workloads as W


def numpy_pair_energies(coefs, kmax):
    n = coefs.shape[:3]
    F = np.fft.fftn(coefs, axes=(0, 1, 2))
    E = (np.abs(F) ** 2).sum(-1)
    out = {}
    for a in range(-kmax, kmax + 1):
        for b in range(-kmax, kmax + 1):
            for c in range(-kmax, kmax + 1):
                r2 = a * a + b * b + c * c
                if 0 < r2 <= kmax * kmax and (a, b, c) > (-a, -b, -c):
                    out[(a, b, c)] = (E[a % n[0], b % n[1], c % n[2]] + E[-a % n[0], -b % n[1], -c % n[2]])
    return out, float(E[0, 0, 0]), float(E.sum())


@pytest.mark.parametrize("grid,norb,count,kmax", [((12, 10, 8), 40, 48, 4), ((16, 16, 16), 33, 20, 3),
                                                  ((9, 7, 11), 5, 10, 2), ((6, 6, 6), 3, 128, 4)])
def test_selection_matches_numpy_fft(grid, norb, count, kmax):
    rng = np.random.default_rng(sum(grid) + norb)
    G, a, b = W.planewave_params(rng, norb, rmax=kmax)
    coefs = W.fit_planewave_coefs(grid, G, a, b) + 0.01 * rng.standard_normal(tuple(grid) + (norb,))
    ks, en = q.spectral_frequencies(coefs, count=count, kmax=kmax, with_energy=True)
    ref, e0, tot = numpy_pair_energies(coefs, kmax)
    scale = max(ref.values())
    got = [tuple(int(x) for x in k) for k in ks]
    assert len(set(got)) == count and all(k in ref for k in got)
    for k, e in zip(got, en["pairs"]):
        assert abs(e - ref[k]) <= 1e-10 * scale, (k, e, ref[k])
    assert all(np.diff(en["pairs"]) <= 0)                       # most energy first
    cut = en["pairs"][-1]
    for k, e in ref.items():                                    # nothing left out beats the last one chosen
        if k not in got:
            assert e <= cut + 1e-10 * scale, (k, e, cut)
    assert abs(en["k0"] - e0) <= 1e-10 * max(e0, scale)
    assert abs(en["total"] - tot) <= 1e-10 * tot


def test_selection_ties_and_arguments():
    # one plane wave cos(2 pi k.j / n) carries all the energy, in its pair
    grid = (8, 8, 8)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1)
    coefs = np.cos(2 * np.pi * (j @ np.array([1, -2, 0])) / 8.0)[..., None]
    ks, en = q.spectral_frequencies(coefs, count=5, kmax=3, with_energy=True)
    assert tuple(ks[0]) == (1, -2, 0)
    assert abs(en["pairs"][0] - en["total"]) <= 1e-12 * en["total"]     # 2 |512/2|^2 = n sum c^2
    assert np.all(en["pairs"][1:] <= 1e-20 * en["pairs"][0])
    # a zero table: every energy is exactly 0, so the order is increasing k
    ks0 = q.spectral_frequencies(np.zeros((5, 5, 5, 2)), count=10, kmax=2)
    reps = sorted(k for k in ((a, b, c) for a in range(-2, 3) for b in range(-2, 3) for c in range(-2, 3))
                  if 0 < sum(x * x for x in k) <= 4 and k > tuple(-x for x in k))
    assert [tuple(k) for k in ks0] == reps[:10]
    with pytest.raises(q.SplineError):
        q.spectral_frequencies(coefs, count=129, kmax=4)      # only 128 pairs with |k| <= 4
    with pytest.raises(q.SplineError):
        q.spectral_frequencies(coefs, count=4, kmax=0)
