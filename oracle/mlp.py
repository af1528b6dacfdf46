"""FP64 oracle of the surrogate network (test infrastructure only).

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

Parity status: every function here is pinned by tests/test_oracle_mlp.py
(closed forms and finite differences).  The network's accuracy as a
surrogate of a spline table has no reference value: parity unpinned,
measured and reported.
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


def loss_weights(tV, tG, tL, mu, sd):
    """1 / variance of each normalised target quantity (V, G, L)."""
    nv = (tV - mu) / sd
    ng = tG / sd
    nl = tL / sd
    return np.array([1.0 / nv.var(), 1.0 / ng.var(), 1.0 / nl.var()])


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


def _linear_backward(W, a, dh):
    """Gradients of W (sum over the five streams), b (value stream) and of the
    layer input streams."""
    dW = dh["v"].T @ a["v"] + sum(dh["d"][i].T @ a["d"][i] for i in range(3)) + dh["L"].T @ a["L"]
    db = dh["v"].sum(0)
    da = {"v": dh["v"] @ W, "d": np.stack([dh["d"][i] @ W for i in range(3)]), "L": dh["L"] @ W}
    return dW, db, da


def loss_and_grads(params, pos, tV, tG, tL, w, cell=(1.0, 1.0, 1.0)):
    """FP64 loss and its gradients with respect to W1..b3 (reverse mode)."""
    (V, G, L), c = forward(params, pos, cell, cache=True)
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
    g["W3"], g["b3"], dz2 = _linear_backward(params["W3"], c["z2"], dy)
    dh2 = _silu_backward(c["h2"], dz2)
    g["W2"], g["b2"], dz1 = _linear_backward(params["W2"], c["z1"], dh2)
    dh1 = _silu_backward(c["h1"], dz1)
    g["W1"], g["b1"], _ = _linear_backward(params["W1"], c["a0"], dh1)
    return lval, g
