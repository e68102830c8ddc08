"""Pins of the oracle's surrogate network: backward against finite differences,
forward against scalar loops, SiLU against closed forms."""
import math

import numpy as np

from oracle import mlp


def _theta(net, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.4, mlp.n_params(net))


def test_gradient_vs_finite_differences():
    for net in ("A", "B"):
        nin, nout = mlp.SIZES[net]
        rng = np.random.default_rng(1)
        X = rng.uniform(-1, 1, (nin, 37))
        T = rng.normal(size=(nout, 37))
        th = _theta(net, 2)
        _, g = mlp.loss_and_grad(th, net, X, T)
        idx = rng.choice(th.size, 60, replace=False)
        h = 1e-6
        for i in idx:
            tp, tm = th.copy(), th.copy()
            tp[i] += h
            tm[i] -= h
            fd = (mlp.loss_and_grad(tp, net, X, T)[0] - mlp.loss_and_grad(tm, net, X, T)[0]) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9


def test_forward_matches_scalar_loop():
    """The vectorised forward against plain scalar loops over the layer
    definitions (z_j = sum_i W_ji a_i + b_j, a = z / (1 + exp(-z))), with the
    parameters unpacked by index from the documented layout W1 b1 W2 b2 W3 b3 W4
    b4 (row-major [out][in])."""
    for net in ("A", "B"):
        nin, nout = mlp.SIZES[net]
        th = _theta(net, 5)
        rng = np.random.default_rng(6)
        X = rng.uniform(-1, 1, (nin, 3))
        y, _ = mlp.forward(th, net, X)
        H = mlp.H
        sizes = [(H, nin), (H, H), (H, H), (nout, H)]
        for s in range(X.shape[1]):
            a = [float(v) for v in X[:, s]]
            o = 0
            for li, (no, ni) in enumerate(sizes):
                W = th[o:o + no * ni]
                o += no * ni
                b = th[o:o + no]
                o += no
                z = [sum(W[j * ni + i] * a[i] for i in range(ni)) + b[j] for j in range(no)]
                a = z if li == 3 else [zz / (1.0 + math.exp(-zz)) for zz in z]
            assert o == th.size
            np.testing.assert_allclose(y[:, s], a, rtol=1e-12, atol=1e-12)


def test_silu_and_derivative_closed_forms():
    """silu(0) = 0, silu(z) -> z for large z and -> 0 for very negative z,
    silu(-z) = silu(z) - z; dsilu matches a central difference and has its
    minimum of silu at z ~ -1.2785 (where dsilu = 0)."""
    z = np.linspace(-8, 8, 161)
    np.testing.assert_allclose(mlp.silu(-z), mlp.silu(z) - z, atol=1e-14)
    assert mlp.silu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.silu(np.array([40.0]))[0] - 40.0) < 1e-15 * 40 + 1e-14
    assert abs(mlp.silu(np.array([-40.0]))[0]) < 1e-15
    h = 1e-6
    np.testing.assert_allclose(mlp.dsilu(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), atol=1e-9)
    zm = -1.2784645427610738          # root of 1 + z (1 - sigmoid(z)) = 0
    assert abs(mlp.dsilu(np.array([zm]))[0]) < 1e-12
