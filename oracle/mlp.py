"""FP64 oracle of the surrogate network (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
module; it shares no code with the GPU library.

A small periodic network stands in for a spline table: positions go through
periodic Fourier features, then dense layers with SiLU, and the value,
gradient and Laplacian of the output are carried exactly in forward mode.
The paper has no network; this definition follows the surrogate specified
for this library (features [sin 2pi k.u, cos 2pi k.u] for integer k, layers
96 -> 256 -> 256 -> N, SiLU, a per-orbital affine output map), and is
written out plainly in numpy so that each step can be checked by eye.

  forward-mode streams (one value stream, three first-derivative streams and
  one Laplacian stream) through a layer h = W a + b, z = silu(h):
      h   = W a + b          h_d = W a_d          h_L = W a_L
      z   = s(h)             z_d = s'(h) h_d      z_L = s'(h) h_L + s''(h) sum_d h_d^2
  output:  V = sd * (W3 z + b3) + mu,  G_d = sd * W3 z_d,  L = sd * W3 z_L

The reverse pass (gradients of the Sobolev loss with respect to every weight)
is hand-written; tests pin it against finite differences of the loss.

BF16 arithmetic model (bf16=True): every operand of every matrix product --
features, activations, weights, and in the reverse pass the adjoints -- is
rounded to BF16 (nearest even, from FP32); biases, SiLU streams, the loss and
the bias gradients stay unrounded.

The spline fallback: the cell is cut into bins_per_dim^3 bins; a bin's error
is the largest error of the network against the spline over the validation
points that fall in it, over orbitals and over V, the three components of G
and L, each error taken relative to that orbital's largest |quantity| over the
whole validation set; positions in bins whose error exceeds a tolerance are
routed to the spline.

The representational floor: bandlimited_vgl evaluates the spline's Fourier
series cut to the feature frequencies' ball (from the definition of the
spline and the transform of the cubic B-spline); the error of that against
the spline is the least any approximant whose spectrum stays below the
table's first alias band can reach.

Parity status: every function here is pinned by tests/test_oracle_mlp.py
(closed forms, finite differences, hand-built cases and scalar loops).  The
network's accuracy as a surrogate of a spline table has no reference value:
parity unpinned, measured and reported.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def silu_derivs(x):
    """SiLU x*s(x), s the logistic function, and its first three derivatives."""
    s = 1.0 / (1.0 + np.exp(-x))
    f0 = x * s
    f1 = s * (1.0 + x * (1.0 - s))
    f2 = s * (1.0 - s) * (2.0 + x * (1.0 - 2.0 * s))
    f3 = s * (1.0 - s) * (3.0 * (1.0 - 2.0 * s) + x * (1.0 - 6.0 * s + 6.0 * s * s))
    return f0, f1, f2, f3


def bf16_round(x):
    """Round to BF16 (nearest even) from FP32, returned as float64.

    Emulates the GPU path, where FP32 operands are rounded to BF16 before each
    matrix product."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(pos, freqs, cell=(1.0, 1.0, 1.0)):
    """Streams of the periodic features at positions pos[B,3].

    Returns a dict with 'v' [B,2F], 'd' [3,B,2F] (d/dr_x, d/dr_y, d/dr_z) and
    'L' [B,2F]; columns are [sin(2 pi k_j.u) for j] + [cos(2 pi k_j.u) for j],
    u = r / cell componentwise."""
    pos = np.asarray(pos, dtype=np.float64)
    k = np.asarray(freqs, dtype=np.float64)          # [F,3]
    cell = np.asarray(cell, dtype=np.float64)
    u = pos / cell
    theta = TWO_PI * (u @ k.T)                       # [B,F]
    s, c = np.sin(theta), np.cos(theta)
    g = TWO_PI * k / cell                            # [F,3] d theta / d r_d
    g2 = (g * g).sum(1)                              # [F]
    v = np.concatenate([s, c], 1)
    d = np.stack([np.concatenate([c * g[:, dd], -s * g[:, dd]], 1) for dd in range(3)])
    lap = np.concatenate([-s * g2, -c * g2], 1)
    return {"v": v, "d": d, "L": lap}


def _layer(W, b, a, bf16):
    """Forward-mode linear map of the five streams (value gets the bias)."""
    Wm = bf16_round(W) if bf16 else W
    r = (lambda x: bf16_round(x)) if bf16 else (lambda x: x)
    return {"v": r(a["v"]) @ Wm.T + b, "d": np.stack([r(a["d"][i]) @ Wm.T for i in range(3)]),
            "L": r(a["L"]) @ Wm.T}


def _silu_streams(h):
    f0, f1, f2, _ = silu_derivs(h["v"])
    return {"v": f0, "d": f1[None] * h["d"], "L": f1 * h["L"] + f2 * (h["d"] ** 2).sum(0)}


def forward(params, pos, cell=(1.0, 1.0, 1.0), bf16=False, cache=False):
    """V[B,N], G[B,3,N], L[B,N] of the network at pos[B,3].

    params: dict with freqs[F,3], W1,b1,W2,b2,W3,b3 (W stored [out,in]), mu[N], sd[N].
    bf16=True rounds every matrix-product operand to BF16 (the GPU arithmetic).
    """
    a0 = features(pos, params["freqs"], cell)
    h1 = _layer(params["W1"], params["b1"], a0, bf16)
    z1 = _silu_streams(h1)
    h2 = _layer(params["W2"], params["b2"], z1, bf16)
    z2 = _silu_streams(h2)
    y = _layer(params["W3"], params["b3"], z2, bf16)
    sd, mu = params["sd"], params["mu"]
    V = y["v"] * sd + mu
    G = np.transpose(y["d"], (1, 0, 2)) * sd
    L = y["L"] * sd
    if cache:
        return (V, G, L), dict(a0=a0, h1=h1, z1=z1, h2=h2, z2=z2, y=y)
    return V, G, L


def output_normalisation(tV, tG, tL):
    """Per-orbital output map and loss weights from a batch of targets.

    mu_n, sd_n: mean and (population) standard deviation of orbital n's value
    over the batch (sd floored at 1e-12).  Loss weight of quantity Q (V; G
    with its three components pooled; L): 1 / the variance of Q / sd_n about
    its own per-orbital mean, averaged over orbitals.  For V that is 1 by
    construction.  Returns (mu[N], sd[N], w[3])."""
    tV = np.asarray(tV, dtype=np.float64)
    tG = np.asarray(tG, dtype=np.float64)
    tL = np.asarray(tL, dtype=np.float64)
    N = tV.shape[-1]
    mu = tV.mean(0)
    sd = np.maximum(np.sqrt(((tV - mu) ** 2).mean(0)), 1e-12)
    w = []
    for Q in (tV, tG, tL):
        q = Q.reshape(-1, N)
        var = ((q - q.mean(0)) ** 2).mean(0) / (sd * sd)
        w.append(1.0 / max(var.mean(), 1e-30))
    return mu, sd, np.array(w)


def loss(params, pos, tV, tG, tL, w, cell=(1.0, 1.0, 1.0), bf16=False):
    """Sobolev loss: weighted mean squared errors of the normalised V, G, L."""
    (V, G, L) = forward(params, pos, cell, bf16)
    sd = params["sd"]
    eV = (V - tV) / sd
    eG = (G - tG) / sd
    eL = (L - tL) / sd
    return w[0] * (eV ** 2).mean() + w[1] * (eG ** 2).mean() + w[2] * (eL ** 2).mean()


def _silu_backward(h, dz):
    """Adjoint of the forward-mode SiLU streams: (dz_v, dz_d, dz_L) -> dh."""
    _, f1, f2, f3 = silu_derivs(h["v"])
    hd, hL = h["d"], h["L"]
    s2 = (hd ** 2).sum(0)
    dh_v = dz["v"] * f1 + (dz["d"] * hd).sum(0) * f2 + dz["L"] * (f2 * hL + f3 * s2)
    dh_d = dz["d"] * f1[None] + 2.0 * (dz["L"] * f2)[None] * hd
    dh_L = dz["L"] * f1
    return {"v": dh_v, "d": dh_d, "L": dh_L}


def _linear_backward(W, a, dh, bf16=False):
    """Gradients of W (sum over the five streams), b (value stream) and of the
    layer input streams.  bf16=True rounds the operands of the two products
    (adjoints, layer inputs, weights) to BF16; the bias gradient is a plain
    sum of the unrounded value-stream adjoints."""
    r = bf16_round if bf16 else (lambda x: x)
    Wm = r(W)
    dW = r(dh["v"]).T @ r(a["v"]) + sum(r(dh["d"][i]).T @ r(a["d"][i]) for i in range(3)) + r(dh["L"]).T @ r(a["L"])
    db = dh["v"].sum(0)
    da = {"v": r(dh["v"]) @ Wm, "d": np.stack([r(dh["d"][i]) @ Wm for i in range(3)]), "L": r(dh["L"]) @ Wm}
    return dW, db, da


def loss_and_grads(params, pos, tV, tG, tL, w, cell=(1.0, 1.0, 1.0), bf16=False):
    """Loss and its gradients with respect to W1..b3 (reverse mode), in FP64;
    bf16=True follows the BF16 arithmetic model in both passes."""
    (V, G, L), c = forward(params, pos, cell, bf16=bf16, cache=True)
    sd = params["sd"]
    B, N = V.shape
    eV = (V - tV) / sd
    eG = (G - tG) / sd
    eL = (L - tL) / sd
    lval = w[0] * (eV ** 2).mean() + w[1] * (eG ** 2).mean() + w[2] * (eL ** 2).mean()
    # d loss / d y (network outputs before the affine map: V = sd y + mu)
    dy = {"v": 2.0 * w[0] * eV / (B * N),
          "d": np.transpose(2.0 * w[1] * eG / (3 * B * N), (1, 0, 2)),
          "L": 2.0 * w[2] * eL / (B * N)}
    g = {}
    g["W3"], g["b3"], dz2 = _linear_backward(params["W3"], c["z2"], dy, bf16)
    dh2 = _silu_backward(c["h2"], dz2)
    g["W2"], g["b2"], dz1 = _linear_backward(params["W2"], c["z1"], dh2, bf16)
    dh1 = _silu_backward(c["h1"], dz1)
    g["W1"], g["b1"], _ = _linear_backward(params["W1"], c["a0"], dh1, bf16)
    return lval, g


def bin_index(pos, bins_per_dim, cell=(1.0, 1.0, 1.0)):
    """Error-map bin of each position: (i0 * nb + i1) * nb + i2.

    Along axis d the fractional coordinate f = u - floor(u), u = r_d / cell_d
    (FP64), falls in bin floor(nb * f).  An f that rounds up to 1 (a
    coordinate just below a multiple of the cell) belongs to the last bin; a
    non-finite coordinate is put in bin 0."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    nb = int(bins_per_dim)
    idx = np.zeros(pos.shape[0], dtype=np.int64)
    for d in range(3):
        u = pos[:, d] / float(cell[d])
        with np.errstate(invalid="ignore"):
            f = u - np.floor(u)
            i = np.floor(f * nb)
        i = np.where(np.isfinite(i), i, 0.0)
        i = np.clip(i, 0, nb - 1).astype(np.int64)
        idx = idx * nb + i
    return idx


def point_errors(net_vgl, spline_vgl):
    """Per-position error of the network against the spline: max over
    orbitals of |dV| / sV_n, |dG_d| / sG_n (each component), |dL| / sL_n,
    with sQ_n the largest |Q| of orbital n over all the given positions (1 if
    that is 0).  A NaN anywhere in a position's terms makes its error +inf."""
    V, G, L = (np.asarray(x, dtype=np.float64) for x in net_vgl)
    Vs, Gs, Ls = (np.asarray(x, dtype=np.float64) for x in spline_vgl)
    B, N = Vs.shape
    terms = []
    for Q, Qs in ((V, Vs), (G, Gs), (L, Ls)):
        with np.errstate(invalid="ignore"):
            s = np.abs(Qs).reshape(-1, N).max(0) if B else np.ones(N)
        s = np.where(s == 0, 1.0, s)
        with np.errstate(invalid="ignore"):
            terms.append((np.abs(Q - Qs) / s).reshape(B, -1))
    t = np.concatenate(terms, 1)
    with np.errstate(invalid="ignore"):
        e = t.max(1) if t.shape[1] else np.zeros(B)
    return np.where(np.isnan(t).any(1), np.inf, e)


def error_map(net_vgl, spline_vgl, val_pos, bins_per_dim, cell=(1.0, 1.0, 1.0)):
    """bin_err[nb^3]: per bin the largest point error (point_errors) over the
    validation positions in it; +inf for a bin that holds none."""
    nb = int(bins_per_dim)
    e = point_errors(net_vgl, spline_vgl)
    k = bin_index(val_pos, nb, cell)
    out = np.full(nb ** 3, -np.inf)
    np.maximum.at(out, k, e)
    return np.where(np.isneginf(out), np.inf, out)


def route(pos, bin_err, bins_per_dim, tol, cell=(1.0, 1.0, 1.0)):
    """Sorted indices of the positions routed to the spline: those whose bin
    error is not <= tol (so +inf and NaN bins always route, and a NaN
    tolerance routes everything).  The comparison is taken in FP32, the
    precision of a stored map and tolerance."""
    e = np.asarray(bin_err, dtype=np.float32)[bin_index(pos, bins_per_dim, cell)]
    t = np.float32(tol)
    with np.errstate(invalid="ignore"):
        keep = e <= t
    return np.flatnonzero(~keep).astype(np.int64)


def spline_fourier_coefficients(coefs, kmax, cell=(1.0, 1.0, 1.0)):
    """Fourier coefficients of the periodic tricubic spline at the integer
    frequencies k with |k|_2 <= kmax (each below half the grid on every axis).

    The spline is s(r) = sum_j c_j prod_d beta(n_d r_d / cell_d - j_d), beta
    the centred cubic B-spline, whose Fourier transform is sinc(x)^4 (sinc(x)
    = sin(pi x) / (pi x)).  Its Fourier series coefficient at k is therefore
    chat(k) prod_d sinc(k_d / n_d)^4, with chat(k) = (1/|n|) sum_j c_j
    exp(-2 pi i k.j / n) the discrete transform of the coefficients.  Returns
    (K[m,3] int64, S[m,N] complex128)."""
    c = np.asarray(coefs, dtype=np.float64)
    n = np.array(c.shape[:3])
    N = c.shape[3]
    r = int(np.floor(kmax))
    ax = np.arange(-r, r + 1)
    K = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    K = K[(K ** 2).sum(1) <= kmax * kmax + 1e-9]
    if np.any(2 * np.abs(K) >= n[None, :]):
        raise ValueError("kmax must stay below half the grid on every axis")
    chat = np.fft.fftn(c, axes=(0, 1, 2)) / float(np.prod(n))
    Cs = chat[K[:, 0] % n[0], K[:, 1] % n[1], K[:, 2] % n[2]].reshape(-1, N)
    damp = np.prod(np.sinc(K / n[None, :]) ** 4, axis=1)
    return K, Cs * damp[:, None]


def bandlimited_vgl(coefs, pos, kmax, cell=(1.0, 1.0, 1.0)):
    """V[B,N], G[B,3,N], L[B,N] of the spline's Fourier series truncated to
    |k| <= kmax: the L2-closest function over the cell whose spectrum lies in
    that ball.  For a table fitted to plane waves with |G| <= kmax, every
    other component of the spline sits at an alias k + n a (a != 0), so this
    is the best any approximant reaching only frequencies below the first
    alias band can do (the surrogate's features are such frequencies)."""
    K, S = spline_fourier_coefficients(coefs, kmax, cell)
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    cell = np.asarray(cell, dtype=np.float64)
    kc = TWO_PI * K / cell[None, :]                        # [m,3] Cartesian wave vectors
    ph = np.exp(1j * (pos / cell[None, :] * TWO_PI) @ K.T)  # [B,m]
    V = (ph @ S).real
    G = np.stack([((1j * kc[:, d])[None, :] * ph) @ S for d in range(3)], 1).real
    L = ((-(kc ** 2).sum(1))[None, :] * ph @ S).real
    return V, G, L
