"""Surrogate network of the Monte Carlo step, forward and backward in float64
(test infrastructure only).

The surrogate is not part of the paper: it replaces the table lookups of the
total rates and of the inverse cumulative spectrum (Eq. 7) by two small
multilayer perceptrons (three hidden layers of width 64, SiLU), with the tables
kept as the fallback.

  net A  (log10 chi, logit u) -> r,  s = logit(xi) = r + ln chi + 3 ln u
  net B  log10 chi -> (ln h_rad - ln chi, ln h_pair + 8/(3 chi) - ln chi)

Inputs and outputs are normalised by fixed affine maps (``NORM``).

Layer l computes z = W a + b; hidden activations a = silu(z).  This is the
plain float64 network; the GPU's reduced-precision arithmetic is compared with
it through error bounds derived in the tests, not mirrored here.

Pinned by tests/test_oracle_mlp.py: backward against central finite differences
of the forward, forward against a per-sample loop of scalar products, and SiLU
against its closed-form properties.
"""
import math

import numpy as np

TMAX = math.log((1 - 1e-4) / 1e-4)        # logit u range of net A: |t| <= TMAX
NORM = {
    "x_shift": 0.5, "x_scale": 2.5,      # xt = (log10 chi + 0.5) / 2.5
    "A_shift": -1.0, "A_scale": 2.0,     # r = A_shift + A_scale * y
    "B_shift": (-0.4, -2.0), "B_scale": (0.5, 0.5),
}
SIZES = {"A": (2, 1), "B": (1, 2)}
H = 64


def n_params(net):
    nin, nout = SIZES[net]
    return H * nin + H + 2 * (H * H + H) + nout * H + nout


def unpack(theta, net):
    nin, nout = SIZES[net]
    o = 0
    out = {}
    for name, shape in (("W1", (H, nin)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
                        ("W3", (H, H)), ("b3", (H,)), ("W4", (nout, H)), ("b4", (nout,))):
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p, net):
    return np.concatenate([p[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")])


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(theta, net, X):
    """X: (nin, N) normalised inputs -> outputs (nout, N) and the cache."""
    p = unpack(theta, net)
    z1 = p["W1"] @ X + p["b1"][:, None]
    a1 = silu(z1)
    z2 = p["W2"] @ a1 + p["b2"][:, None]
    a2 = silu(z2)
    z3 = p["W3"] @ a2 + p["b3"][:, None]
    a3 = silu(z3)
    y = p["W4"] @ a3 + p["b4"][:, None]
    return y, dict(X=X, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, p=p)


def loss_and_grad(theta, net, X, T, mask=None):
    """Mean over samples of sum_o mask * (y - T)^2 and its gradient."""
    y, c = forward(theta, net, X)
    N = X.shape[1]
    m = np.ones_like(T) if mask is None else mask
    r = (y - T) * m
    loss = float(np.sum(r * r) / N)
    p = c["p"]
    dy = 2.0 * r / N
    g = {}
    g["W4"] = dy @ c["a3"].T
    g["b4"] = dy.sum(axis=1)
    d3 = (p["W4"].T @ dy) * dsilu(c["z3"])
    g["W3"] = d3 @ c["a2"].T
    g["b3"] = d3.sum(axis=1)
    d2 = (p["W3"].T @ d3) * dsilu(c["z2"])
    g["W2"] = d2 @ c["a1"].T
    g["b2"] = d2.sum(axis=1)
    d1 = (p["W2"].T @ d2) * dsilu(c["z1"])
    g["W1"] = d1 @ X.T
    g["b1"] = d1.sum(axis=1)
    return loss, pack(g, net)


def inputs_A(chi, u):
    lx = np.log10(chi)
    t = np.log(u) - np.log1p(-u)
    return np.stack([(lx + NORM["x_shift"]) / NORM["x_scale"], t / TMAX])


def inputs_B(chi):
    return ((np.log10(chi) + NORM["x_shift"]) / NORM["x_scale"])[None, :]


def xi_from_A(y, chi, u):
    """logit(xi) = r + ln chi + 3 ln u with r = A_shift + A_scale y."""
    r = NORM["A_shift"] + NORM["A_scale"] * y
    return r + np.log(chi) + 3.0 * np.log(u)


def rates_from_B(y, chi):
    """(ln h_rad, ln h_pair) from net B outputs."""
    lr = NORM["B_shift"][0] + NORM["B_scale"][0] * y[0] + np.log(chi)
    lp = NORM["B_shift"][1] + NORM["B_scale"][1] * y[1] + np.log(chi) - 8.0 / (3.0 * chi)
    return lr, lp
