"""Pins of the oracle's surrogate network: backward against finite differences,
split-BF16 products against exact ones."""
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


def test_split_products_close_to_exact():
    rng = np.random.default_rng(3)
    W = rng.normal(size=(64, 64))
    A = rng.normal(size=(64, 50))
    ex = W.astype(np.float32).astype(np.float64) @ A.astype(np.float32).astype(np.float64)
    sp = mlp.matmul(W, A, "split")
    assert np.max(np.abs(sp - ex)) / np.max(np.abs(ex)) < 2 ** -15
    # bf16 rounding: ties to even, 8 significant bits
    assert mlp.bf16(np.float32(1.0 + 2 ** -8)) == 1.0
    assert mlp.bf16(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6
