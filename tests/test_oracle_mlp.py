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


# ---------------------------------------------------------------------------
# Output map and loss weights


def test_output_normalisation_closed_form():
    """V = a_n + c_n (-1)^b has mean a_n and population sd |c_n|; G and L
    alternate about per-orbital means m_n, e_n with half-widths g_n, l_n, so
    the loss weights are 1/mean(g^2/c^2) and 1/mean(l^2/c^2).  Sample
    variances, or variances pooled about one mean for all orbitals, fail."""
    B, N = 6, 4
    a = np.array([0.5, -2.0, 3.0, 0.0])
    c = np.array([1.0, 0.25, -2.0, 4.0])
    m = np.array([7.0, -1.0, 0.0, 2.5])
    gw = np.array([2.0, 0.5, 1.0, 3.0])
    e = np.array([-4.0, 0.0, 1.5, 9.0])
    lw = np.array([1.0, 3.0, 0.5, 2.0])
    sb = (-1.0) ** np.arange(B)
    tV = a[None] + c[None] * sb[:, None]
    sg = (-1.0) ** (np.arange(B)[:, None] + np.arange(3)[None])
    tG = m[None, None] + gw[None, None] * sg[..., None]
    tL = e[None] + lw[None] * sb[:, None]
    mu, sd, w = M.output_normalisation(tV, tG, tL)
    np.testing.assert_allclose(mu, a, rtol=0, atol=1e-15)
    np.testing.assert_allclose(sd, np.abs(c), rtol=1e-15)
    np.testing.assert_allclose(w, [1.0, 1.0 / np.mean(gw ** 2 / c ** 2), 1.0 / np.mean(lw ** 2 / c ** 2)], rtol=1e-14)
    # a constant orbital: sd takes its floor
    tV2 = tV.copy()
    tV2[:, 1] = 3.0
    _, sd2, _ = M.output_normalisation(tV2, tG, tL)
    assert sd2[1] == 1e-12


# ---------------------------------------------------------------------------
# BF16 arithmetic model, pinned by scalar loops with the C oracle's rounding


def _r32_16(x):
    """FP32 then BF16 (8 significant bits), both round-to-nearest-even, through
    the C oracle's generic significand rounding (independent of bf16_round)."""
    import oracle as O
    return O.round_sig(O.round_sig(float(x), 24, -126), 8, -126)


def _silu(h):
    s = 1.0 / (1.0 + np.exp(-h))
    return (h * s, s * (1 + h * (1 - s)), s * (1 - s) * (2 + h * (1 - 2 * s)),
            s * (1 - s) * (3 * (1 - 2 * s) + h * (1 - 6 * s + 6 * s * s)))


def _hand_net(p, pos, tgt=None, w=None, bf16=True, cell=(1.0, 1.0, 1.0)):
    """Forward (and, given targets, the reverse pass) of a tiny network in
    scalar loops, rounding every product operand to BF16 as the model says."""
    r = _r32_16 if bf16 else float
    F = len(p["freqs"])
    B = len(pos)
    S = ("v", "x", "y", "z", "L")
    acts = []  # per layer input: acts[l][b][s][k]
    a0 = []
    for b in range(B):
        u = [pos[b][d] / cell[d] for d in range(3)]
        row = {s: [0.0] * (2 * F) for s in S}
        for j in range(F):
            k = p["freqs"][j]
            th = 2 * np.pi * sum(k[d] * u[d] for d in range(3))
            g = [2 * np.pi * k[d] / cell[d] for d in range(3)]
            g2 = sum(x * x for x in g)
            for col, (val, dv) in ((j, (np.sin(th), np.cos(th))), (F + j, (np.cos(th), -np.sin(th)))):
                row["v"][col] = val
                for d, s in enumerate("xyz"):
                    row[s][col] = dv * g[d]
                row["L"][col] = -g2 * val
        a0.append(row)
    acts.append(a0)
    hs = []
    layers = (("W1", "b1", True), ("W2", "b2", True), ("W3", "b3", False))
    for Wn, bn, act in layers:
        Wm, bias = p[Wn], p[bn]
        out_h, out_z = [], []
        for b in range(B):
            a = acts[-1][b]
            h = {s: [0.0] * Wm.shape[0] for s in S}
            for o in range(Wm.shape[0]):
                for s in S:
                    h[s][o] = sum(r(Wm[o][k]) * r(a[s][k]) for k in range(Wm.shape[1]))
                h["v"][o] += bias[o]
            out_h.append(h)
            if act:
                z = {s: [0.0] * Wm.shape[0] for s in S}
                for o in range(Wm.shape[0]):
                    f0, f1, f2, _ = _silu(h["v"][o])
                    z["v"][o] = f0
                    for s in "xyz":
                        z[s][o] = f1 * h[s][o]
                    z["L"][o] = f1 * h["L"][o] + f2 * sum(h[s][o] ** 2 for s in "xyz")
                out_z.append(z)
        hs.append(out_h)
        if act:
            acts.append(out_z)
    N = p["W3"].shape[0]
    y = hs[-1]
    V = np.array([[p["sd"][n] * y[b]["v"][n] + p["mu"][n] for n in range(N)] for b in range(B)])
    G = np.array([[[p["sd"][n] * y[b][s][n] for n in range(N)] for s in "xyz"] for b in range(B)])
    L = np.array([[p["sd"][n] * y[b]["L"][n] for n in range(N)] for b in range(B)])
    if tgt is None:
        return V, G, L
    tV, tG, tL = tgt
    grads = {}
    # adjoint of the network outputs y (V = sd y + mu)
    dy = []
    for b in range(B):
        d = {s: [0.0] * N for s in S}
        for n in range(N):
            sd = p["sd"][n]
            d["v"][n] = 2 * w[0] * (V[b][n] - tV[b][n]) / sd / (B * N)
            for i, s in enumerate("xyz"):
                d[s][n] = 2 * w[1] * (G[b][i][n] - tG[b][i][n]) / sd / (3 * B * N)
            d["L"][n] = 2 * w[2] * (L[b][n] - tL[b][n]) / sd / (B * N)
        dy.append(d)
    dh = dy
    for li in (2, 1, 0):
        Wn, bn, _ = layers[li]
        Wm = p[Wn]
        a = acts[li]
        dW = np.zeros_like(Wm)
        db = np.zeros(Wm.shape[0])
        for o in range(Wm.shape[0]):
            for k in range(Wm.shape[1]):
                dW[o][k] = sum(r(dh[b][s][o]) * r(a[b][s][k]) for b in range(B) for s in S)
            db[o] = sum(dh[b]["v"][o] for b in range(B))
        grads[Wn], grads[bn] = dW, db
        if li == 0:
            break
        # adjoint of the layer input z, then through the SiLU streams of layer li-1
        hprev = hs[li - 1]
        ndh = []
        for b in range(B):
            dz = {s: [sum(r(dh[b][s][o]) * r(Wm[o][k]) for o in range(Wm.shape[0])) for k in range(Wm.shape[1])]
                  for s in S}
            h = hprev[b]
            d = {s: [0.0] * Wm.shape[1] for s in S}
            for k in range(Wm.shape[1]):
                f0, f1, f2, f3 = _silu(h["v"][k])
                s2 = sum(h[s][k] ** 2 for s in "xyz")
                d["v"][k] = (dz["v"][k] * f1 + sum(dz[s][k] * h[s][k] for s in "xyz") * f2
                             + dz["L"][k] * (f2 * h["L"][k] + f3 * s2))
                for s in "xyz":
                    d[s][k] = dz[s][k] * f1 + 2 * dz["L"][k] * f2 * h[s][k]
                d["L"][k] = dz["L"][k] * f1
            ndh.append(d)
        dh = ndh
    return (V, G, L), grads


def _tiny(rng, N=2, F=2, H=3):
    return _params(rng, N=N, F=F, H=H)


def test_bf16_forward_matches_scalar_loops():
    """The vectorised BF16 model equals scalar loops that round each product
    operand through the C oracle; without rounding both equal the exact
    network, and the rounding moves the result by more than the comparison
    bar (so a skipped rounding point fails)."""
    rng = np.random.default_rng(11)
    p = _tiny(rng)
    pos = rng.random((3, 3)) * 2.0 - 0.5
    got = M.forward(p, pos, bf16=True)
    hand = _hand_net(p, pos, bf16=True)
    exact = M.forward(p, pos)
    hand_exact = _hand_net(p, pos, bf16=False)
    for g, h, x, hx in zip(got, hand, exact, hand_exact):
        scale = np.abs(h).max()
        np.testing.assert_allclose(g, h, rtol=0, atol=1e-13 * scale)
        np.testing.assert_allclose(x, hx, rtol=0, atol=1e-13 * scale)
        assert np.abs(g - x).max() > 1e-6 * scale


def test_bf16_reverse_pass_matches_scalar_loops():
    """Reverse pass of the BF16 model (adjoints, layer inputs and weights of
    both products rounded; bias gradients from unrounded adjoints) against
    scalar loops; the unrounded scalar loops equal the FD-pinned FP64 pass."""
    rng = np.random.default_rng(12)
    p = _tiny(rng)
    pos = rng.random((3, 3))
    tgt = (rng.standard_normal((3, 2)), rng.standard_normal((3, 3, 2)), rng.standard_normal((3, 2)))
    w = np.array([1.0, 0.4, 0.07])
    _, g = M.loss_and_grads(p, pos, *tgt, w, bf16=True)
    _, gh = _hand_net(p, pos, tgt, w, bf16=True)
    _, g64 = M.loss_and_grads(p, pos, *tgt, w)
    _, gh64 = _hand_net(p, pos, tgt, w, bf16=False)
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        sc = np.abs(gh[name]).max()
        np.testing.assert_allclose(g[name], gh[name], rtol=0, atol=1e-12 * sc, err_msg=name)
        np.testing.assert_allclose(g64[name], gh64[name], rtol=0, atol=1e-12 * sc, err_msg=name)
        if name.startswith("W"):
            assert np.abs(g[name] - g64[name]).max() > 1e-7 * sc, name


# ---------------------------------------------------------------------------
# Error map and routing, pinned on hand-built cases


def test_bin_index_edges():
    nb = 8
    cell = (1.0, 2.0, 0.5)
    P = np.array([
        [0.5, 1.0, 0.25],           # every axis exactly half-way: bin 4 (a lower edge belongs to the bin above)
        [-0.0, 0.0, 0.0],           # signed zero
        [-1e-17, 0.0, 0.0],         # just below a period: f rounds to 1 -> last bin
        [1.0, 2.0, 0.5],            # one full period: bin 0
        [-0.3, -2.3, -0.05],        # negative coordinates wrap
        [2.3, 4.5, 1.0],            # beyond one period
        [0.999999999999, 1.9999999999, 0.4999999999],
        [np.nan, 0.5, np.inf],      # non-finite -> bin 0 on that axis
        [0.125, 0.25 * 3, 0.0625 * 7],
    ])
    got = M.bin_index(P, nb, cell)
    want = [(4, 4, 4), (0, 0, 0), (7, 0, 0), (0, 0, 0), (5, 6, 7), (2, 2, 0), (7, 7, 7), (0, 2, 0), (1, 3, 7)]
    assert list(got) == [(i * nb + j) * nb + k for i, j, k in want]


def _grid_points(nb, bins):
    """One point at the centre of each listed bin (unit cell)."""
    out = []
    for k in bins:
        i, j, l = k // (nb * nb), (k // nb) % nb, k % nb
        out.append([(i + 0.5) / nb, (j + 0.5) / nb, (l + 0.5) / nb])
    return np.array(out)


def test_error_map_hand_built():
    """Two bins per axis; one point in each bin but bin 5 (empty -> inf),
    two in bin 0.  The network equals the spline except for one planted
    error per point, so each bin's value is that error over its orbital's
    normaliser; a NaN makes its bin inf; a zero orbital is measured in
    absolute terms; the normaliser is the spline's, not the network's."""
    nb, N = 2, 3
    bins = [0, 0, 1, 2, 3, 4, 6, 7]
    pos = _grid_points(nb, bins)
    pos[1] += 0.1                        # second point of bin 0 elsewhere in it
    B = len(pos)
    rng = np.random.default_rng(5)
    Vs = rng.uniform(-1, 1, (B, N))
    Gs = rng.uniform(-1, 1, (B, 3, N))
    Ls = rng.uniform(-1, 1, (B, N))
    Vs[:, 2] = 0.0                       # orbital 2 has no value anywhere
    Vs[3, 0], Gs[5, 1, 1], Ls[6, 2] = 4.0, -5.0, 8.0   # the normalisers: sV0 = 4, sG1 = 5, sL2 = 8
    sV = np.abs(Vs).max(0)
    sV[2] = 1.0
    sG = np.abs(Gs).max((0, 1))
    sL = np.abs(Ls).max(0)
    V, G, L = Vs.copy(), Gs.copy(), Ls.copy()
    want = np.zeros(nb ** 3)
    plant = [  # (point, quantity, component, orbital, delta)
        (0, "V", 0, 0, 0.02), (1, "V", 0, 1, 0.5), (2, "G", 2, 1, 0.3), (3, "L", 0, 2, -0.4),
        (4, "V", 0, 2, 1e-3), (5, "G", 0, 0, 7.0), (6, "L", 0, 0, 0.0), (7, "V", 0, 0, -0.1)]
    for b, q, d, n, delta in plant:
        if q == "V":
            V[b, n] += delta
            e = abs(delta) / sV[n]
        elif q == "G":
            G[b, d, n] += delta
            e = abs(delta) / sG[n]
        else:
            L[b, n] += delta
            e = abs(delta) / sL[n]
        want[bins[b]] = max(want[bins[b]], e)
    want[5] = np.inf
    got = M.error_map((V, G, L), (Vs, Gs, Ls), pos, nb)
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=0)
    # the network's own magnitudes do not enter the normaliser
    V2 = V.copy()
    V2[2, 0] += 100.0
    got2 = M.error_map((V2, G, L), (Vs, Gs, Ls), pos, nb)
    assert abs(got2[bins[2]] - max(want[bins[2]], 100.0 / sV[0])) <= 1e-13
    # a NaN term makes its bin inf (and only its bin)
    G3 = G.copy()
    G3[4, 1, 0] = np.nan
    got3 = M.error_map((V, G3, L), (Vs, Gs, Ls), pos, nb)
    assert got3[bins[4]] == np.inf
    np.testing.assert_allclose(np.delete(got3, bins[4]), np.delete(want, bins[4]), rtol=1e-14, atol=0)
    # a NaN in the spline poisons the normaliser of its orbital: every bin inf
    Ls4 = Ls.copy()
    Ls4[0, 1] = np.nan
    assert np.isinf(M.error_map((V, G, L), (Vs, Gs, Ls4), pos, nb)).all()


def test_route_hand_built():
    nb = 2
    bin_err = np.array([0.1, 0.5, np.inf, np.nan, 0.2, 0.3, 1e-4, 0.05], dtype=np.float32)
    base = _grid_points(nb, range(8))
    # each bin twice: centre, and a copy shifted by whole periods (negative and beyond one)
    pos = np.concatenate([base, base + np.array([-1.0, 2.0, -3.0])])
    r = M.route(pos, bin_err, nb, 0.2)
    routed_bins = [1, 2, 3, 5]           # 0.5, inf, NaN, 0.3 (0.2 <= 0.2 stays)
    want = sorted(k for k in range(16) if k % 8 in routed_bins)
    assert list(r) == want
    assert list(M.route(pos, bin_err, nb, -1.0)) == list(range(16))
    assert list(M.route(pos, bin_err, nb, float("nan"))) == list(range(16))
    assert list(M.route(pos, bin_err, nb, float("inf"))) == [3, 11]      # only the NaN bin
    assert list(M.route(pos, bin_err, nb, 1.0)) == [2, 3, 10, 11]
    # the FP32 comparison: a tolerance that is 0.2 in FP64 equals the stored FP32 0.2
    assert 4 not in M.route(pos, bin_err, nb, np.float64(0.2))
