"""Modified Bessel functions K_nu(x) for the spectra (test infrastructure only).

Both functions use the integral representation of K_nu (DLMF 10.32.9)

    K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt ,            x > 0,

and the tail integral obtained by integrating it over x from x to infinity,

    int_x^inf K_nu(s) ds = int_0^inf exp(-x cosh t) cosh(nu t) / cosh t dt .

Both integrands are even, entire functions of t that decay double-exponentially,
so the trapezoid rule on [0, t_max] converges geometrically.  Step and cut:

    h(x)     = min(0.1, 0.35 / sqrt(x))
    t_max(x) = arccosh(1 + 40 / x)      (integrand below e^-40 of its value at t=0)

Pinned by tests/test_oracle_pins.py: scipy.special.kv, mpmath.besselk, the closed
form K_{1/2}(x) = sqrt(pi/2x) e^-x and int_0^inf K_nu = pi / (2 cos(nu pi / 2)).
"""
import numpy as np

_CHUNK = 2048


def _trapezoid(x, integrand):
    """Trapezoid sum over t of integrand(x[:,None], t) with the step/cut rule above."""
    x = np.asarray(x, dtype=np.float64)
    shape = x.shape
    xf = x.reshape(-1)
    out = np.empty_like(xf)
    for a in range(0, xf.size, _CHUNK):
        xc = xf[a:a + _CHUNK]
        h = np.minimum(0.1, 0.35 / np.sqrt(xc))
        n = np.ceil(np.arccosh(1.0 + 40.0 / xc) / h).astype(np.int64)
        j = np.arange(int(n.max()) + 1, dtype=np.float64)
        t = j[None, :] * h[:, None]
        g = integrand(xc[:, None], t)
        g = np.where(j[None, :] <= n[:, None], g, 0.0)
        g[:, 0] *= 0.5
        out[a:a + _CHUNK] = h * g.sum(axis=1)
    return out.reshape(shape)


def bessel_k(nu, x):
    """K_nu(x) for x > 0 (DLMF 10.32.9)."""
    return _trapezoid(x, lambda xx, t: np.exp(-xx * np.cosh(t)) * np.cosh(nu * t))


def bessel_k_tail(nu, x):
    """int_x^inf K_nu(s) ds for x > 0 (DLMF 10.32.9 integrated over x)."""
    return _trapezoid(x, lambda xx, t: np.exp(-xx * np.cosh(t)) * np.cosh(nu * t) / np.cosh(t))


def bessel_k_pair(x):
    """(K_{2/3}(x), int_x^inf K_{1/3}) together, sharing exp(-x cosh t).

    Same rule as bessel_k / bessel_k_tail; the two sums are formed from one
    evaluation of the exponential, which halves the cost of the spectra in
    Eqs. (1) and (6).
    """
    x = np.asarray(x, dtype=np.float64)
    shape = x.shape
    xf = x.reshape(-1)
    k23 = np.empty_like(xf)
    i13 = np.empty_like(xf)
    for a in range(0, xf.size, _CHUNK):
        xc = xf[a:a + _CHUNK]
        h = np.minimum(0.1, 0.35 / np.sqrt(xc))
        n = np.ceil(np.arccosh(1.0 + 40.0 / xc) / h).astype(np.int64)
        j = np.arange(int(n.max()) + 1, dtype=np.float64)
        t = j[None, :] * h[:, None]
        ch = np.cosh(t)
        e = np.exp(-xc[:, None] * ch)
        e = np.where(j[None, :] <= n[:, None], e, 0.0)
        e[:, 0] *= 0.5
        k23[a:a + _CHUNK] = h * np.sum(e * np.cosh((2.0 / 3.0) * t), axis=1)
        i13[a:a + _CHUNK] = h * np.sum(e * np.cosh((1.0 / 3.0) * t) / ch, axis=1)
    return k23.reshape(shape), i13.reshape(shape)
