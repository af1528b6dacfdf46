"""Pins of the surrogate-network oracle (CPU, FP64).

SiLU and its derivatives against closed values at 0 and finite differences;
the features' derivative streams against finite differences; the network's
forward-mode gradient and Laplacian against finite differences of its value;
the hand-written reverse pass against finite differences of the loss; the
BF16 rounding against exhaustive properties."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as M


def _params(rng, N=12, F=6, H=16):
    freqs = W.fourier_frequencies(rng, F)
    return dict(freqs=freqs,
                W1=rng.standard_normal((H, 2 * F)) * 0.5, b1=rng.standard_normal(H) * 0.1,
                W2=rng.standard_normal((H, H)) * 0.4, b2=rng.standard_normal(H) * 0.1,
                W3=rng.standard_normal((N, H)) * 0.3, b3=rng.standard_normal(N) * 0.1,
                mu=rng.standard_normal(N), sd=rng.uniform(0.5, 2.0, N))


def test_silu_closed_values_and_fd():
    f0, f1, f2, f3 = M.silu_derivs(np.array([0.0]))
    assert (f0[0], f1[0], f2[0], f3[0]) == (0.0, 0.5, 0.5, 0.0)
    x = np.linspace(-8, 8, 161)
    h = 1e-4
    d = [M.silu_derivs(x + k * h) for k in (-2, -1, 1, 2)]
    for order in range(3):
        fd = (-d[3][order] + 8 * d[2][order] - 8 * d[1][order] + d[0][order]) / (12 * h)
        np.testing.assert_allclose(M.silu_derivs(x)[order + 1], fd, atol=1e-9)
    # large |x|: SiLU -> x (x>0) or 0 (x<0)
    f0, f1, _, _ = M.silu_derivs(np.array([40.0, -40.0]))
    np.testing.assert_allclose(f0, [40.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(f1, [1.0, 0.0], atol=1e-12)


def test_feature_streams_fd():
    rng = np.random.default_rng(1)
    freqs = W.fourier_frequencies(rng, 8)
    cell = (1.0, 1.3, 0.8)
    pos = rng.random((20, 3)) * np.array(cell)
    f = M.features(pos, freqs, cell)
    h = 1e-5
    lap = np.zeros_like(f["v"])
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fp, fm = M.features(pos + e, freqs, cell)["v"], M.features(pos - e, freqs, cell)["v"]
        np.testing.assert_allclose(f["d"][d], (fp - fm) / (2 * h), atol=1e-6 * np.abs(f["d"][d]).max())
        lap += (fp - 2 * f["v"] + fm) / (h * h)
    np.testing.assert_allclose(f["L"], lap, atol=2e-3 * np.abs(f["L"]).max())
    # periodic in the cell
    shifted = M.features(pos + np.array([cell[0], -2 * cell[1], 5 * cell[2]]), freqs, cell)
    np.testing.assert_allclose(shifted["v"], f["v"], atol=1e-12)


def test_forward_mode_matches_fd_of_value():
    rng = np.random.default_rng(2)
    p = _params(rng)
    pos = rng.random((15, 3))
    V, G, L = M.forward(p, pos)
    h = 1e-4
    Lfd = np.zeros_like(L)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        v = {k: M.forward(p, pos + k * e)[0] for k in (-2, -1, 1, 2)}
        gfd = (-v[2] + 8 * v[1] - 8 * v[-1] + v[-2]) / (12 * h)
        np.testing.assert_allclose(G[:, d], gfd, atol=1e-7 * np.abs(G).max())
        Lfd += (-v[2] + 16 * v[1] - 30 * V + 16 * v[-1] - v[-2]) / (12 * h * h)
    np.testing.assert_allclose(L, Lfd, atol=1e-5 * np.abs(L).max())


def test_reverse_pass_matches_fd_of_loss():
    rng = np.random.default_rng(3)
    p = _params(rng)
    pos = rng.random((10, 3))
    tV, tG, tL = (rng.standard_normal((10, 12)), rng.standard_normal((10, 3, 12)), rng.standard_normal((10, 12)))
    w = np.array([1.0, 0.3, 0.05])
    lval, g = M.loss_and_grads(p, pos, tV, tG, tL, w)
    assert abs(lval - M.loss(p, pos, tV, tG, tL, w)) < 1e-12 * abs(lval)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, 6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = M.loss(p, pos, tV, tG, tL, w)
            flat[idx] = old - h
            lm = M.loss(p, pos, tV, tG, tL, w)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(an - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx, an, fd)


def test_bf16_round_properties():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0]])
    r = M.bf16_round(x)
    u = r.astype(np.float32).view(np.uint32)
    assert (u & 0xFFFF == 0).all()                      # representable in BF16
    f = x.astype(np.float32).astype(np.float64)
    nz = f != 0
    assert (np.abs(r[nz] - f[nz]) <= 2.0 ** -8 * np.abs(f[nz])).all()
    assert r[-4] == 1.0 and r[-3] == 1.0 and r[-2] == 1.0 + 2 ** -6   # ties to even
