"""Emission and pair spectra and the quantum parameters (test infrastructure only).

Every spectrum is returned as the dimensionless shape S(xi, chi) defined by

    dW/dxi = (alpha m_e c^2 / hbar) / gamma * S(xi, chi) = RATE_UNIT / gamma * S,

so that the total rate is W = RATE_UNIT * h(chi) / gamma with h = int_0^1 S dxi
(RATE_UNIT = alpha E_S in 1/omega_0).  Arguments may be NumPy arrays.

formula_I   Eq. (1):  S = [(1 - xi + 1/(1-xi)) K_{2/3}(d) - int_d^inf K_{1/3}] / (sqrt3 pi),
            d = 2 xi / (3 (1-xi) chi).
formula_II  Eq. (4):  S = xi / (3 pi^2 chi) * sum_i F_i(xi) J_i(sigma),
            sigma = xi / (3 chi (1-xi)).  The J_i are evaluated after the change
            of variable u = sigma cosh^3(theta), under which (u/sigma)^(2/3) - 1 =
            sinh^2(theta) and the inverse square-root endpoint singularity cancels:
              J_1 = int_0^inf cosh^5 K_{2/3}^2(sigma cosh^3) dtheta
              J_2 = int_0^inf cosh^3 sinh^2 K_{1/3}^2(sigma cosh^3) dtheta
              J_3 = int_0^inf cosh^5 K_{1/3}^2(sigma cosh^3) dtheta
            trapezoid in theta, step min(0.08, 0.3/sqrt(sigma)), cut where
            sigma cosh^3 = sigma + 22.5.
classical   Eq. (5):  S = sqrt3 chi / (2 pi xi) * z int_z^inf K_{5/3}.  The printed
            z = 2 xi / (3 chi^2) is read as z = 2 xi / (3 chi): that is the only form
            that is the hbar -> 0 limit of Eq. (1), which the paper says Eq. (5) is.
pair        Eq. (6):  S = [(1/xi + 1/(1-xi) - 2) K_{2/3}(d) + int_d^inf K_{1/3}] / (sqrt3 pi),
            d = 2 / (3 xi (1-xi) chi), xi = eps_e / eps_ph.  The printed sign of the
            integral term is read as "+": only "+" gives Erber's small-chi asymptote
            h_pair -> 3 sqrt3 / (16 sqrt2) chi exp(-8/(3 chi)) (pinned in the tests);
            sign="printed" evaluates the printed "-" for comparison.

The logit variable s = ln(xi / (1 - xi)) is used by the tables; the *_logit
variants take s and form xi and 1 - xi without cancellation.

chi_lepton / chi_photon: Eqs. (2)-(3) written literally in float64,
    chi = gamma / E_S * sqrt((E + v x B)^2 - (v . E)^2),
with v = p / gamma for a lepton and |v| = 1 for a photon.

Pinned by tests/test_oracle_pins.py: formula I == formula II (identity of the two
published forms), classical limit of Eq. (1), synchrotron-function peak
0.918 at x ~ 0.2858, int F(x)/x dx = 5 pi / 3, small/large-chi rate asymptotes,
closed-form chi in crossed and plane-wave fields.
"""
import math

import numpy as np

from .bessel import bessel_k, bessel_k_pair, bessel_k_tail
from .constants import E_S

SQRT3 = math.sqrt(3.0)
INV_SQRT3_PI = 1.0 / (SQRT3 * math.pi)


def _xi_pair(s):
    """xi and 1 - xi from the logit s, each without cancellation."""
    s = np.asarray(s, dtype=np.float64)
    xi = 1.0 / (1.0 + np.exp(-s))
    om = 1.0 / (1.0 + np.exp(s))
    return xi, om


# ---------------------------------------------------------------- Eq. (1)
def formula_I_logit(s, chi):
    xi, om = _xi_pair(s)
    d = (2.0 / 3.0) * np.exp(s) / chi          # 2 xi / (3 (1-xi) chi)
    k23, i13 = bessel_k_pair(d)
    return INV_SQRT3_PI * ((om + 1.0 / om) * k23 - i13)


def formula_I(xi, chi):
    xi = np.asarray(xi, dtype=np.float64)
    return formula_I_logit(np.log(xi) - np.log1p(-xi), chi)


# ---------------------------------------------------------------- Eq. (4)
def _J(sigma):
    """(J_1, J_2, J_3)(sigma) for scalar sigma > 0, theta-substituted trapezoid."""
    h = min(0.08, 0.3 / math.sqrt(sigma))
    th_max = math.acosh((1.0 + 22.5 / sigma) ** (1.0 / 3.0))
    n = int(math.ceil(th_max / h))
    th = np.arange(n + 1, dtype=np.float64) * h
    ch = np.cosh(th)
    sh = np.sinh(th)
    u = sigma * ch ** 3
    k13 = bessel_k(1.0 / 3.0, u)
    k23 = bessel_k(2.0 / 3.0, u)
    w = np.full(n + 1, h)
    w[0] *= 0.5
    j1 = np.sum(w * ch ** 5 * k23 ** 2)
    j2 = np.sum(w * ch ** 3 * sh ** 2 * k13 ** 2)
    j3 = np.sum(w * ch ** 5 * k13 ** 2)
    return j1, j2, j3


def formula_II_logit(s, chi):
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    chi_b = np.broadcast_to(np.asarray(chi, dtype=np.float64), s.shape)
    out = np.empty_like(s)
    for i, (si, ci) in enumerate(zip(s.reshape(-1), chi_b.reshape(-1))):
        xi, om = _xi_pair(si)
        sigma = math.exp(si) / (3.0 * ci)        # xi / (3 chi (1-xi))
        j1, j2, j3 = _J(sigma)
        f1 = 1.0 + 1.0 / om ** 2
        f2 = 2.0 / om
        f3 = (xi / om) ** 2
        out.reshape(-1)[i] = xi / (3.0 * math.pi ** 2 * ci) * (f1 * j1 + f2 * j2 + f3 * j3)
    return out


def formula_II(xi, chi):
    xi = np.asarray(xi, dtype=np.float64)
    return formula_II_logit(np.log(xi) - np.log1p(-xi), chi)


# ---------------------------------------------------------------- Eq. (5)
def classical(xi, chi):
    xi = np.asarray(xi, dtype=np.float64)
    z = 2.0 * xi / (3.0 * chi)
    return SQRT3 * chi / (2.0 * math.pi * xi) * z * bessel_k_tail(5.0 / 3.0, z)


def synchrotron_F(x):
    """F(x) = x int_x^inf K_{5/3}: the shape inside Eq. (5)."""
    x = np.asarray(x, dtype=np.float64)
    return x * bessel_k_tail(5.0 / 3.0, x)


# ---------------------------------------------------------------- Eq. (6)
def pair_logit(s, chi, sign="+"):
    xi, om = _xi_pair(s)
    d = 2.0 / (3.0 * xi * om * chi)
    sg = 1.0 if sign == "+" else -1.0
    k23, i13 = bessel_k_pair(d)
    return INV_SQRT3_PI * ((1.0 / xi + 1.0 / om - 2.0) * k23 + sg * i13)


def pair(xi, chi, sign="+"):
    xi = np.asarray(xi, dtype=np.float64)
    return pair_logit(np.log(xi) - np.log1p(-xi), chi, sign)


# ---------------------------------------------------------------- Eqs. (2)-(3)
def chi_lepton(p, E, B):
    """Eq. (2) for momenta p [m_e c] (..., 3) in fields E, B (..., 3)."""
    p = np.asarray(p, dtype=np.float64)
    gamma = np.sqrt(1.0 + np.sum(p * p, axis=-1))
    v = p / gamma[..., None]
    f = E + np.cross(v, B)
    rad = np.sum(f * f, axis=-1) - np.sum(v * E, axis=-1) ** 2
    return gamma / E_S * np.sqrt(np.maximum(rad, 0.0))


def chi_photon(k, E, B):
    """Eq. (3) for photon momenta k [m_e c] (..., 3): gamma_ph = |k|, |v| = 1."""
    k = np.asarray(k, dtype=np.float64)
    gph = np.sqrt(np.sum(k * k, axis=-1))
    v = k / np.where(gph > 0, gph, 1.0)[..., None]
    f = E + np.cross(v, B)
    rad = np.sum(f * f, axis=-1) - np.sum(v * E, axis=-1) ** 2
    return gph / E_S * np.sqrt(np.maximum(rad, 0.0))
