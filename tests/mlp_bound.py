"""Error bounds of the GPU surrogate arithmetic against the exact float64
network (test infrastructure).

The GPU evaluates the two 64x64 layers on bf16 matrix cores with every operand
split into x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) and the products
hi*hi + hi*lo + lo*hi accumulated in float32; everything else is float32 with
the hardware exp and reciprocal.  With bf16's unit roundoff 2^-8:
  |x - hi - lo| <= 2^-16 |x|,  |lo| <= 2^-8 |x|,
so one split product misses at most 3 * 2^-16 |w| |a| (lo*lo and the two
remainders), and the float32 accumulation of 3 x 64 terms adds at most
192 * 2^-24 of sum |w| |a|.  SiLU with the hardware exp2 / reciprocal: relative
error <= 2^-21 (2 + |z|); its derivative: absolute error <= 2^-20 (2 + |z|);
|silu'| <= 1.1, |silu''| <= 0.5.  Sums over the N samples of a batch in
float32: (N + 128) * 2^-24 of the sum of absolute values.

Two propagations of these roundoffs through the forward and backward passes,
first order in the roundoffs:
  "abs"  worst case: every error adds in absolute value (|W| @ e); a rigorous
         elementwise bound, but loose for 64-term sums of random signs;
  "rss"  probabilistic (Higham & Mary, "A new approach to probabilistic rounding
         error analysis", SIAM J. Sci. Comput. 2019): roundoffs are independent
         and centred, so standard deviations add in quadrature
         (sqrt(W^2 @ e^2)); per-term standard deviations are the worst-case
         sizes above divided by sqrt(3) (uniform within their bound), which
         gives sigma; a test asserts |error| <= K sigma with K = 8.
The "rss" bound is what can see a dropped split product (an error of ~2^-9 of
sum |w a|); the "abs" bound holds without any assumption."""
import numpy as np

from oracle import mlp

U32 = 2.0 ** -24
EPS_MM = 3 * 2.0 ** -16 + 192 * U32
D2 = 0.5                    # max |silu''|
K_SIGMA = 8.0


class _Prop:
    """Error arithmetic of one propagation mode."""

    def __init__(self, mode):
        self.rss = mode == "rss"
        self.f = 1.0 / np.sqrt(3.0) if self.rss else 1.0   # per-term size -> standard deviation

    def mat(self, W, e):                      # error of W @ x from an error e of x
        return np.sqrt((W * W) @ (e * e)) if self.rss else np.abs(W) @ e

    def rnd(self, W, a, eps):                 # roundoff of the product W @ a itself
        return self.f * eps * (np.sqrt((W * W) @ (a * a)) if self.rss else np.abs(W) @ np.abs(a))

    def add(self, *terms):
        return np.sqrt(sum(t * t for t in terms)) if self.rss else sum(terms)

    def act(self, z, a):                      # roundoff of silu
        return self.f * 2.0 ** -21 * (2.0 + np.abs(z)) * np.abs(a)

    def dact(self, z):                        # roundoff of silu'
        return self.f * 2.0 ** -20 * (2.0 + np.abs(z))


def forward_bound(theta, net, X, mode="abs"):
    """Exact outputs y (nout, N), the bound on |y_gpu - y| (the standard
    deviation sigma in mode "rss") and the intermediate bounds."""
    P = _Prop(mode)
    y, c = mlp.forward(theta, net, X)
    p = c["p"]
    E1 = P.add(P.rnd(p["W1"], X, 4 * U32), P.rnd(p["b1"][:, None], np.ones((1, X.shape[1])), 4 * U32))
    da1 = P.add(np.abs(mlp.dsilu(c["z1"])) * E1, P.act(c["z1"], c["a1"]))
    E2 = P.add(P.mat(p["W2"], da1), P.rnd(p["W2"], c["a1"], EPS_MM))
    da2 = P.add(np.abs(mlp.dsilu(c["z2"])) * E2, P.act(c["z2"], c["a2"]))
    E3 = P.add(P.mat(p["W3"], da2), P.rnd(p["W3"], c["a2"], EPS_MM))
    da3 = P.add(np.abs(mlp.dsilu(c["z3"])) * E3, P.act(c["z3"], c["a3"]))
    Ey = P.add(P.mat(p["W4"], da3), P.rnd(p["W4"], c["a3"], 70 * U32))
    return y, Ey, dict(c=c, E1=E1, E2=E2, E3=E3, da1=da1, da2=da2, da3=da3, P=P)


def grad_bound(theta, net, X, T, M, mode="abs"):
    """Exact gradient of sum_o M (y - T)^2 / N and the elementwise bound on
    |grad_gpu - grad| (sigma in mode "rss"), packed like the parameters."""
    y, Ey, f = forward_bound(theta, net, X, mode)
    P, c = f["P"], f["c"]
    p = c["p"]
    N = X.shape[1]
    ES = (N + 128) * U32                        # float32 sums over the batch
    ones = np.ones((N, 1))
    dy = 2.0 * (y - T) * M / N
    ddy = P.add(2.0 * Ey * M / N, P.f * U32 * np.abs(dy))
    s3, s2, s1 = mlp.dsilu(c["z3"]), mlp.dsilu(c["z2"]), mlp.dsilu(c["z1"])

    def layer_back(Wt, d_up, dd_up, s, E, z, eps):
        h = Wt @ d_up
        dh = P.add(P.mat(Wt, dd_up), P.rnd(Wt, d_up, eps))
        d = h * s
        dd = P.add(dh * np.abs(s), np.abs(h) * D2 * E, np.abs(h) * P.dact(z))
        return d, dd

    d3, dd3 = layer_back(p["W4"].T, dy, ddy, s3, f["E3"], c["z3"], 4 * U32)
    d2, dd2 = layer_back(p["W3"].T, d3, dd3, s2, f["E2"], c["z2"], EPS_MM)
    d1, dd1 = layer_back(p["W2"].T, d2, dd2, s1, f["E1"], c["z1"], EPS_MM)

    def wgrad(d, dd, a, da, eps):             # sum over samples of d a^T
        return P.add(P.mat(dd, np.abs(a).T), P.mat(np.abs(d), da.T), P.rnd(d, a.T, eps + ES))

    def bgrad(d, dd):
        return P.add(P.mat(dd, ones)[:, 0], P.rnd(d, ones, ES)[:, 0])

    zero = np.zeros_like(X)
    b = {"W4": wgrad(dy, ddy, c["a3"], f["da3"], 0.0), "b4": bgrad(dy, ddy),
         "W3": wgrad(d3, dd3, c["a2"], f["da2"], EPS_MM), "b3": bgrad(d3, dd3),
         "W2": wgrad(d2, dd2, c["a1"], f["da1"], EPS_MM), "b2": bgrad(d2, dd2),
         "W1": wgrad(d1, dd1, X, zero, 0.0), "b1": bgrad(d1, dd1)}
    _, g = mlp.loss_and_grad(theta, net, X, T, M)
    return g, mlp.pack(b, net)
