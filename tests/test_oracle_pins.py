"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: library
routines (scipy / mpmath), closed forms, published asymptotes, identities
between the paper's two photon formulas, known-answer vectors.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

from oracle import bessel, constants, philox, spectra, tables

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Bessel
@pytest.mark.parametrize("nu", [1.0 / 3.0, 2.0 / 3.0, 5.0 / 3.0])
def test_bessel_k_vs_scipy(nu):
    x = np.array([1e-19, 1e-8, 1e-3, 0.3, 1.0, 7.0, 25.0, 90.0, 300.0, 650.0])
    np.testing.assert_allclose(bessel.bessel_k(nu, x), sp.kv(nu, x), rtol=5e-14)


def test_bessel_k_half_closed_form():
    x = np.logspace(-6, 2.5, 40)
    np.testing.assert_allclose(bessel.bessel_k(0.5, x), np.sqrt(np.pi / (2 * x)) * np.exp(-x), rtol=5e-14)
    # int_x^inf sqrt(pi/2s) e^-s ds = (pi/sqrt2) erfc(sqrt x)
    np.testing.assert_allclose(bessel.bessel_k_tail(0.5, x),
                               np.pi / math.sqrt(2.0) * sp.erfc(np.sqrt(x)), rtol=5e-14)


@pytest.mark.parametrize("nu", [1.0 / 3.0, 2.0 / 3.0])
def test_bessel_tail_vs_quad_and_total(nu):
    x = np.array([1e-3, 0.3, 1.0, 7.0, 25.0])
    ref = [si.quad(lambda s: sp.kv(nu, s), xx, np.inf, epsabs=0, epsrel=1e-13, limit=400)[0] for xx in x]
    np.testing.assert_allclose(bessel.bessel_k_tail(nu, x), ref, rtol=2e-13)
    # int_0^inf K_nu = pi / (2 cos(nu pi / 2)) (DLMF 10.43.19 at mu = 0): the tail at
    # tiny x plus the small-x part int_0^x K_nu ~ Gamma(nu) 2^(nu-1) x^(1-nu) / (1-nu)
    x0 = 1e-30
    small = sp.gamma(nu) * 2 ** (nu - 1) * x0 ** (1 - nu) / (1 - nu)
    total = bessel.bessel_k_tail(nu, np.array([x0]))[0] + small
    assert abs(total / (np.pi / (2 * np.cos(nu * np.pi / 2))) - 1) < 1e-12


def test_bessel_vs_mpmath():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    for x in [1e-12, 0.05, 2.0, 40.0, 250.0]:
        for nu in (1.0 / 3.0, 2.0 / 3.0):
            ref = float(mpmath.besselk(mpmath.mpf(nu), mpmath.mpf(x)))
            assert abs(bessel.bessel_k(nu, np.array([x]))[0] / ref - 1) < 5e-14


# ------------------------------------------------------- synchrotron function
def test_synchrotron_peak():
    """F(x) = x int_x^inf K_{5/3} peaks at ~0.918 near x ~ 0.29 (Eq. 5's shape)."""
    r = (math.sqrt(5) - 1) / 2
    a, b = 0.1, 0.6
    f = lambda x: float(spectra.synchrotron_F(np.array([x]))[0])
    for _ in range(80):
        c, d = b - r * (b - a), a + r * (b - a)
        if f(c) > f(d):
            b = d
        else:
            a = c
    xm = 0.5 * (a + b)
    assert abs(xm - 0.285812) < 2e-5
    assert abs(f(xm) - 0.918012) < 2e-6


def test_synchrotron_integrals():
    # int_0^inf F(x)/x dx = 5 pi / 3 and int_0^inf F dx = 8 pi / (9 sqrt3)
    # (Mellin transform of K_nu, DLMF 10.43.19)
    s = np.linspace(-40.0, 4.5, 20001)
    x = np.exp(s)
    F = spectra.synchrotron_F(x)
    # below x = e^-40, F ~ x^(1/3), so int_0^x0 F/x = 3 F(x0)
    assert abs((np.trapezoid(F, s) + 3 * F[0]) / (5 * np.pi / 3) - 1) < 1e-9
    assert abs(np.trapezoid(F * x, s) / (8 * np.pi / (9 * math.sqrt(3))) - 1) < 1e-9


# ------------------------------------------------------- formula I vs II
def test_formula_I_equals_formula_II():
    """The paper compares Eq. (1) and Eq. (4) (Fig. 1) and finds them nearly the
    same; they are the same function, so the oracle must agree to quadrature
    precision."""
    for chi in (1e-3, 0.1, 1.0, 10.0, 100.0):
        xi = np.array([1e-12, 1e-6, 1e-4, 1e-3, 0.05, 0.3, 0.7, 0.95, 0.999])
        I = spectra.formula_I(xi, chi)
        II = spectra.formula_II(xi, chi)
        ok = I > 1e-250
        np.testing.assert_allclose(II[ok], I[ok], rtol=2e-12)


def test_formula_I_vs_scipy_bessel():
    """Eq. (1) written independently with scipy's K_nu and quad."""
    for chi in (0.1, 1.0, 10.0):
        for xi in (1e-3, 0.2, 0.6):
            d = 2 * xi / (3 * (1 - xi) * chi)
            tail = si.quad(lambda s: sp.kv(1 / 3, s), d, np.inf, epsrel=1e-13, epsabs=0, limit=400)[0]
            ref = ((1 - xi + 1 / (1 - xi)) * sp.kv(2 / 3, d) - tail) / (math.sqrt(3) * math.pi)
            assert abs(spectra.formula_I(np.array([xi]), chi)[0] / ref - 1) < 1e-11


def test_classical_limit_of_formula_I():
    """Eq. (5) (with z = 2 xi / (3 chi)) is the chi -> 0 limit of Eq. (1): at
    fixed x = 2 xi / (3 chi) the ratio tends to 1 linearly in chi."""
    x = np.logspace(-2, 1, 13)
    errs = []
    for chi in (1e-2, 1e-3, 1e-4):
        xi = 1.5 * chi * x
        r = spectra.formula_I(xi, chi) / spectra.classical(xi, chi)
        errs.append(np.max(np.abs(r - 1)))
    assert errs[2] < 0.02 and errs[1] < 0.2
    assert 7 < errs[1] / errs[2] < 13          # linear in chi
    # the printed z = 2 xi / (3 chi^2) is far off
    chi = 0.1
    xi = np.array([0.03, 0.1])
    z2 = 2 * xi / (3 * chi ** 2)
    printed = math.sqrt(3) * chi / (2 * math.pi * xi) * z2 * bessel.bessel_k_tail(5 / 3, z2)
    assert np.all(np.abs(printed / spectra.formula_I(xi, chi) - 1) > 0.3)


# ---------------------------------------------------------- rate integrals
def test_h_rad_vs_scipy_quad():
    """h(chi) = int_0^1 S_I dxi from the oracle's fine-grid quadrature against an
    independent scipy quad over xi of Eq. (1) with scipy Bessel functions."""
    for chi in (0.1, 1.0, 10.0):
        def integrand(lx):
            xi = math.exp(lx)
            if xi >= 1:
                return 0.0
            d = 2 * xi / (3 * (1 - xi) * chi)
            tail = si.quad(lambda s: sp.kv(1 / 3, s), d, np.inf, epsrel=1e-12, epsabs=0, limit=200)[0]
            return xi * ((1 - xi + 1 / (1 - xi)) * sp.kv(2 / 3, d) - tail) / (math.sqrt(3) * math.pi)
        ref = si.quad(integrand, -60.0, math.log(1 - 1e-14), epsrel=1e-11, epsabs=0, limit=400,
                      points=[math.log(chi) - 3, math.log(chi)])[0]
        row = tables.fine_row("I", chi, tables.RAD_M, need_rho=False)
        assert abs(row.total / ref - 1) < 1e-8


def test_h_rad_asymptotes():
    c1, c2 = 5 / (2 * math.sqrt(3)), 8 * math.sqrt(3) / 15
    for chi in (1e-5, 1e-4):
        h = tables.fine_row("I", chi, tables.RAD_M, need_rho=False).total
        assert abs(h / (c1 * chi * (1 - c2 * chi)) - 1) < 5e-6
    big = 14 * sp.gamma(2 / 3) / (9 * 3 ** (1 / 3))
    r4 = tables.fine_row("I", 1e4, tables.RAD_M, need_rho=False).total / 1e4 ** (2 / 3)
    r5 = tables.fine_row("I", 1e5, tables.RAD_M, need_rho=False).total / 1e5 ** (2 / 3)
    assert abs(r5 / big - 1) < abs(r4 / big - 1) < 3e-3


def test_fig1_triples():
    """chi_e from Eq. (2) for the Fig. 1 triples (b0, gamma): the paper states
    0.1, 1 and 10; the normalised E_S (lambda_0 = 1 um) reproduces them."""
    rows = np.loadtxt(os.path.join(GOLDEN, "fig1_triples.txt"))
    for b0, g, chi_paper in rows:
        p = np.array([[math.sqrt(g * g - 1), 0.0, 0.0]])
        chi = spectra.chi_lepton(p, np.zeros((1, 3)), np.array([[0.0, 0.0, b0]]))[0]
        assert abs(chi / chi_paper - 1) < 1e-3


def test_chi_closed_forms():
    E0 = 300.0
    for g in (10.0, 1e3, 1e4):
        pm = math.sqrt(g * g - 1)
        beta = pm / g
        E = np.array([[0.0, E0, 0.0]])
        B = np.array([[0.0, 0.0, E0]])          # plane wave along +x
        for sgn in (+1, -1):
            chi = spectra.chi_lepton(np.array([[sgn * pm, 0, 0]]), E, B)[0]
            one_m = 1.0 / (g * g * (1 + beta))           # 1 - beta without cancellation
            ref = g * (one_m if sgn > 0 else 1 + beta) * E0 / constants.E_S
            # the literal Eq. (2) loses ~eps * gamma^2 when co-propagating
            assert abs(chi / ref - 1) < (2e-15 * g * g if sgn > 0 else 1e-14)
    # photon along the wave's direction: chi_ph = 0; against it: 2 gamma E0 / E_S
    k = np.array([[50.0, 0, 0], [-50.0, 0, 0]])
    chi = spectra.chi_photon(k, np.array([[0, E0, 0]] * 2), np.array([[0, 0, E0]] * 2))
    assert chi[0] == 0.0 and abs(chi[1] / (2 * 50 * E0 / constants.E_S) - 1) < 1e-14


def _chi_upper_f32(p, E, B):
    """The thinned lepton pass's float32 upper bound of chi (restated from the
    kernel's device header), every operation rounded to float32 separately
    (the device contracts some into fused multiply-adds: fewer roundings)."""
    f = np.float32
    px, py, pz = (p[:, i].astype(f) for i in range(3))
    ex, ey, ez = (E[:, i].astype(f) for i in range(3))
    bx, by, bz = (B[:, i].astype(f) for i in range(3))
    g = np.sqrt(f(1) + (px * px + py * py + pz * pz))
    ax = g * ex + (py * bz - pz * by)
    ay = g * ey + (pz * bx - px * bz)
    az = g * ez + (px * by - py * bx)
    s = px * ex + py * ey + pz * ez
    Ax = abs(g * ex) + abs(py * bz) + abs(pz * by)
    Ay = abs(g * ey) + abs(pz * bx) + abs(px * bz)
    Az = abs(g * ez) + abs(px * by) + abs(py * bx)
    S = abs(px * ex) + abs(py * ey) + abs(pz * ez)
    T = ax * ax + ay * ay + az * az - s * s
    D = f(2.0 ** -19) * (Ax * Ax + Ay * Ay + Az * Az + S * S)
    return np.sqrt(np.maximum(T + D, f(0))) * f((1.0 / constants.E_S) * (1.0 + 2.0 ** -20))


def test_float32_chi_bound_lies_above_chi():
    """The thinned lepton pass runs its envelope at a float32 upper bound of chi
    (Eq. 2) rather than chi itself; thinning stays exact only if the bound is
    never below chi.  Reference: chi E_S = sqrt(|gamma E + p x B|^2 - (p.E)^2)
    for the same float32 inputs in extended precision (its rounding is ~1e-19
    of the terms, the bound's margin 2e-6).  Generic inputs (gamma up to 1e6,
    fields up to 1e4) and inputs where E and -v x B cancel to 1e-9 .. 1e-2: the
    bound is always at or above chi, and within 2e-5 of it wherever |a|^2 - s^2
    keeps a tenth of the squared term sums."""
    rng = np.random.default_rng(5)
    n = 200000

    def unit(m):
        v = rng.normal(size=(m, 3))
        return v / np.linalg.norm(v, axis=1)[:, None]

    gam = 10.0 ** rng.uniform(0, 6, n)
    nhat = unit(n)
    p = (np.sqrt(gam * gam - 1.0)[:, None] * nhat).astype(np.float32)
    E = (10.0 ** rng.uniform(-2, 4, n))[:, None] * unit(n)
    B = (10.0 ** rng.uniform(-2, 4, n))[:, None] * unit(n)
    # cancelling half: E perpendicular to p, B = (n x E) / beta (1 + delta)
    h = n // 2
    Eh = E[:h] - np.sum(E[:h] * nhat[:h], axis=1)[:, None] * nhat[:h]
    beta = np.sqrt(1.0 - 1.0 / gam[:h] ** 2)
    delta = rng.choice([-1.0, 1.0], h) * 10.0 ** rng.uniform(-9, -2, h)
    E[:h] = Eh
    B[:h] = np.cross(nhat[:h], Eh) / beta[:, None] * (1.0 + delta)[:, None]
    E = E.astype(np.float32)
    B = B.astype(np.float32)
    up = _chi_upper_f32(p, E, B).astype(np.float64)
    L = np.longdouble
    pl, El, Bl = p.astype(L), E.astype(L), B.astype(L)
    gl = np.sqrt(L(1) + np.sum(pl * pl, axis=1))
    a = gl[:, None] * El + np.cross(pl, Bl)
    T = np.sum(a * a, axis=1) - np.sum(pl * El, axis=1) ** 2
    chi = (np.sqrt(np.maximum(T, L(0))) / L(constants.E_S)).astype(np.float64)
    assert np.all(up >= chi), np.max((chi - up) / np.maximum(chi, 1e-300))
    # the margin's size: (sum of the squared term sums) / T sets the excess
    A2 = np.sum((gl[:, None] * np.abs(El) + np.abs(pl[:, [1, 2, 0]] * Bl[:, [2, 0, 1]])
                 + np.abs(pl[:, [2, 0, 1]] * Bl[:, [1, 2, 0]])) ** 2, axis=1)
    S2 = np.sum(np.abs(pl * El), axis=1) ** 2
    generic = (T >= L(0.1) * (A2 + S2)).astype(bool)
    assert generic.sum() > n // 3 and (~generic).sum() > n // 4
    assert np.max(up[generic] / chi[generic] - 1.0) < 2e-5


# ------------------------------------------------------------------- pairs
def test_pair_erber_asymptote_and_sign():
    """Small chi: h_pair -> 3 sqrt3 / (16 sqrt2) chi exp(-8/(3 chi)) (Erber) only
    with the "+" sign in Eq. (6); the printed "-" gives a third of it."""
    ref = lambda c: 3 * math.sqrt(3) / (16 * math.sqrt(2)) * c * math.exp(-8 / (3 * c))
    r = {}
    for c in (0.01, 0.005):
        row = tables.fine_row("pair", c, tables.PAIR_M, need_rho=False)
        r[c] = 2 * row.total / ref(c)
    assert abs(r[0.005] - 1) < abs(r[0.01] - 1) < 3e-3
    s = np.linspace(-0.5, 0.0, 401)
    plus = np.trapezoid(spectra.pair_logit(s, 0.01) * np.exp(s) / (1 + np.exp(s)) ** 2, s)
    minus = np.trapezoid(spectra.pair_logit(s, 0.01, sign="printed") * np.exp(s) / (1 + np.exp(s)) ** 2, s)
    assert 0.3 < minus / plus < 0.37


def test_pair_symmetry():
    xi = np.array([0.01, 0.1, 0.3, 0.45])
    for c in (0.1, 1.0, 30.0):
        np.testing.assert_allclose(spectra.pair(xi, c), spectra.pair(1 - xi, c), rtol=1e-13)


def test_pair_rate_vs_scipy():
    for c in (0.3, 3.0, 30.0):
        def f(xi):
            d = 2 / (3 * xi * (1 - xi) * c)
            tail = si.quad(lambda s: sp.kv(1 / 3, s), d, np.inf, epsrel=1e-12, epsabs=0, limit=200)[0]
            return ((1 / xi + 1 / (1 - xi) - 2) * sp.kv(2 / 3, d) + tail) / (math.sqrt(3) * math.pi)
        ref = 2 * si.quad(f, 1e-9, 0.5, epsrel=1e-11, epsabs=0, limit=400)[0]
        got = 2 * tables.fine_row("pair", c, tables.PAIR_M, need_rho=False).total
        assert abs(got / ref - 1) < 1e-9


# ------------------------------------------------------------------ tables
def test_quantiles_vs_independent_cdf():
    """Quantile nodes of a rad row: the CDF at the node, integrated independently
    with scipy quad of Eq. (1), equals the node's u."""
    tab = tables.build_rad_table("I", rows=[60, 200])
    u = 1 / (1 + np.exp(-tab.t))
    for i in (60, 200):
        chi = tab.chi[i]
        h = math.exp(tab.ln_h[i])
        for k in (0, 40, 128, 200, 250):
            s_k = tab.s[i, k]
            xi_lo = 1e-15 * chi
            g = lambda s: float(spectra.formula_I_logit(np.array([s]), chi)[0] * math.exp(s) / (1 + math.exp(s)) ** 2)
            s_lo = math.log(xi_lo) - math.log1p(-xi_lo)
            val = tables.rad_ir_tail(chi, xi_lo) + si.quad(g, s_lo, s_k, epsrel=1e-12, epsabs=0, limit=400)[0]
            assert abs(val / h - u[k]) < 1e-9 * max(1.0, u[k] / 1e-4)


def test_rows_monotone_and_complete(rad_table_I, pair_table):
    assert np.all(np.isfinite(rad_table_I.s)) and np.all(np.diff(rad_table_I.s, axis=1) > 0)
    assert np.all(np.isfinite(pair_table.s)) and np.all(np.diff(pair_table.s, axis=1) > 0)
    assert np.all(pair_table.s <= 0)
    # ln h increasing in chi
    assert np.all(np.diff(rad_table_I.ln_h) > 0) and np.all(np.isfinite(pair_table.L))


def test_rate_table_interpolation(rad_table_I):
    """Linear interpolation of ln h between nodes stays within 2e-5 of the
    quadrature at midpoints; below the range the small-chi expansion holds."""
    mids = np.sqrt(rad_table_I.chi[:-1] * rad_table_I.chi[1:])[::16]
    exact = np.array([tables.fine_row("I", c, tables.RAD_M, need_rho=False).total for c in mids])
    got = tables.h_rad(rad_table_I, mids)
    assert np.max(np.abs(got / exact - 1)) < 2e-5
    c = 3e-4
    assert abs(tables.h_rad(rad_table_I, np.array([c]))[0]
               / tables.fine_row("I", c, tables.RAD_M, need_rho=False).total - 1) < 1e-5


def test_wide_range_tables():
    """Tables over chi <= 1e5 (the Fig. 5 cascade, chi_0 ~ 4e4): the nodes end at
    1e5; between nodes the photon rate stays within 1e-4 and the pair rate
    within 2e-5 of the quadrature (wider spacing than the default tables); above
    the range both follow the chi^(2/3) law within the asymptote's own error."""
    hi = 1e5
    chi = tables.chi_nodes(tables.RAD_NCHI, tables.RAD_CHI_MIN, hi)
    assert abs(chi[0] / tables.RAD_CHI_MIN - 1) < 1e-14 and abs(chi[-1] / hi - 1) < 1e-14
    pick = [60, 140, 200, 250]                 # chi ~ 0.04, 6, 290, 4e4
    rows = sorted(set(pick + [i + 1 for i in pick] + [255]))
    tab = tables.build_rad_table("I", rows=rows, chi_max=hi)
    mids = np.sqrt(chi[pick] * chi[[i + 1 for i in pick]])
    exact = np.array([tables.fine_row("I", c, tables.RAD_M, need_rho=False).total for c in mids])
    assert np.max(np.abs(tables.h_rad(tab, mids) / exact - 1)) < 1e-4
    big = 14 * sp.gamma(2 / 3) / (9 * 3 ** (1 / 3))
    assert abs(tables.h_rad(tab, np.array([1e6]))[0] / (big * 1e6 ** (2 / 3)) - 1) < 1e-3
    pchi = tables.chi_nodes(tables.PAIR_NRATE, tables.PAIR_CHI_MIN, hi)
    ppick = [100, 300, 500]                    # chi_ph ~ 0.24, 5.5e2, 7e4
    prows = sorted(set(ppick + [i + 1 for i in ppick]))
    ptab = tables.build_pair_table(rate_rows=prows, cdf_rows=[], chi_max=hi)
    pm = np.sqrt(pchi[ppick] * pchi[[i + 1 for i in ppick]])
    pex = np.array([2 * tables.fine_row("pair", c, tables.PAIR_M, need_rho=False).total for c in pm])
    assert np.max(np.abs(tables.h_pair(ptab, pm) / pex - 1)) < 2e-5


def _exact_cdf(kind, chi):
    row = tables.fine_row(kind, chi, tables.RAD_M if kind != "pair" else tables.PAIR_M)
    P = row.F / row.total
    return row.s, P


@pytest.mark.parametrize("chi", [0.0999628, 1.0, 9.996])
def test_sampled_xi_ks_vs_exact(rad_table_I, chi):
    """xi sampled through the 256 x 256 inverse-CDF table (row mixing + linear
    interpolation in logit u) against the exact CDF from quadrature."""
    n = 400000
    rng = np.random.default_rng(7)
    u = (np.floor(rng.uniform(size=n) * 2 ** 23) + 0.5) * 2.0 ** -23
    ur = (np.floor(rng.uniform(size=n) * 2 ** 23) + 0.5) * 2.0 ** -23
    xi, _ = tables.sample_rad(rad_table_I.s, rad_table_I.t, np.full(n, chi), u, ur)
    s_samp = np.sort(np.log(xi) - np.log1p(-xi))
    s, P = _exact_cdf("I", chi)
    Pe = np.interp(s_samp, s, P)
    ecdf_hi = np.arange(1, n + 1) / n
    ks = max(np.max(np.abs(ecdf_hi - Pe)), np.max(np.abs(ecdf_hi - 1 / n - Pe)))
    assert ks < 1.63 / math.sqrt(n) + 2e-4


def test_sampled_pair_xi_ks_vs_exact(pair_table):
    n = 300000
    rng = np.random.default_rng(8)
    for chi in (0.05, 1.0, 50.0):
        u = (np.floor(rng.uniform(size=n) * 2 ** 23) + 0.5) * 2.0 ** -23
        ur = (np.floor(rng.uniform(size=n) * 2 ** 23) + 0.5) * 2.0 ** -23
        xh, _ = tables.sample_pair_half(pair_table.s, pair_table.t, np.full(n, chi), u, ur)
        s_samp = np.sort(np.log(xh) - np.log1p(-xh))
        s, P = _exact_cdf("pair", chi)
        Pe = np.interp(s_samp, s, P)
        ecdf = np.arange(1, n + 1) / n
        ks = max(np.max(np.abs(ecdf - Pe)), np.max(np.abs(ecdf - 1 / n - Pe)))
        assert ks < 1.63 / math.sqrt(n) + 2e-4


def test_quantized_storage_error(rad_table_I):
    s0, sc, q = tables.quantize_rows(rad_table_I.s)
    d = tables.dequantize_rows(s0, sc, q)
    assert np.max(np.abs(d - rad_table_I.s)) < 1e-3


# ------------------------------------------------------------------ Philox
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if not l.startswith("#")]
    for r in rows:
        v = [int(t, 16) for t in r]
        out = philox.philox4x32_10(np.array(v[0:4], np.uint32), np.array(v[4:6], np.uint32))
        assert [int(o) for o in out] == v[6:10]


def test_uniform_mapping_range():
    x = np.array([0, 511, 512, 0xFFFFFFFF], dtype=np.uint32)
    u = philox.uniform(x)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24 and u[2] == 3 * 2.0 ** -24
    assert u[3] == 1 - 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_classical_tail_matches_formula_I_tail():
    """Eq. 5 and Eq. 1 share the xi -> 0 law S ~ Gamma(2/3) 3^(1/6) / pi (chi/xi)^(2/3),
    so the infrared tail of the tables applies to the classical spectrum too."""
    for chi in (0.01, 1.0, 30.0):
        xi = np.array([1e-14 * chi])
        law = sp.gamma(2 / 3) * 3 ** (1 / 6) / np.pi * (chi / xi) ** (2 / 3)
        assert abs(spectra.classical(xi, chi)[0] / law - 1) < 1e-6
        assert abs(spectra.formula_I(xi, chi)[0] / law - 1) < 1e-6


def test_classical_overestimates_high_energy():
    """The paper's Fig. 1 finding: at the Fig. 1 triples the classical formula
    gives a higher rate dW/dxi than formula I at high photon energies (and a
    larger tail beyond xi = 1/2)."""
    for chi in (0.1, 1.0, 10.0):
        xi = np.array([0.5, 0.8])
        assert np.all(spectra.classical(xi, chi) > spectra.formula_I(xi, chi))
        rI = tables.fine_row("I", chi, tables.RAD_M, need_rho=False)
        rC = tables.fine_row("classical", chi, tables.RAD_M, need_rho=False)
        tailI = rI.total - np.interp(0.0, rI.s, rI.F)
        tailC = rC.total - np.interp(0.0, rC.s, rC.F)
        assert tailC > tailI


def test_thinning_envelopes_bound_the_rates(rad_table_I, pair_table):
    """The surrogate path draws candidate events at closed-form envelope rates and
    keeps each with probability W / W_env, which is exact only if W <= W_env
    everywhere (Poisson thinning).  The envelopes (restated from the kernel's
    lookup header): h_rad_env = 1.002 (5 / (2 sqrt3)) chi (1 + chi)^(-1/3) and
    h_pair_env = 1.002 (3 sqrt3 / (16 sqrt2)) chi exp(-8 / (3 chi)) (1 + chi/4)^(-1/3)
    (zero below chi = 1e-2): the oracle's tabulated rates, with their
    extrapolations outside the table, stay below them by at least the 1.002
    margin over chi in [1e-6, 1e5], and are not far below (acceptance >= 0.89)."""
    c1 = 5.0 / (2.0 * math.sqrt(3.0))
    ce = 3.0 * math.sqrt(3.0) / (16.0 * math.sqrt(2.0))
    chi = np.logspace(-6, 5, 400001)
    env = 1.002 * c1 * chi * (1.0 + chi) ** (-1.0 / 3.0)
    r = tables.h_rad(rad_table_I, chi) / env
    assert r.max() <= 1.0 / 1.002 + 1e-12 and r.min() > 0.89
    cp = chi[chi >= 1e-2]
    envp = 1.002 * ce * cp * np.exp(-8.0 / (3.0 * cp)) * (1.0 + 0.25 * cp) ** (-1.0 / 3.0)
    rp = tables.h_pair(pair_table, cp) / envp
    assert rp.max() <= 1.0 / 1.002 + 1e-12 and rp.min() > 0.89
