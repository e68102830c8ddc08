"""Pins of the oracle's Monte Carlo step: event statistics against the rate
integrals, sampled spectra against the exact CDF, the paper's generator
comparisons, exact push kinematics, brute-force compaction."""
import math

import numpy as np
import pytest

from oracle import mc, philox, spectra, tables
from oracle.constants import E_S, RATE_UNIT

import workloads


@pytest.fixture(scope="module")
def rad(rad_table_I):
    return mc.RadSampler(rad_table_I, "f64")


def _ensemble(n, b0, g, seed=0):
    ens = workloads.uniform_b_ensembles(n, seed=seed, triples=((b0, g),))[0]
    E = np.zeros((n, 3))
    B = np.tile([0.0, 0.0, b0], (n, 1))
    return ens, E, B


def test_boris_gyration_exact():
    """Uniform B, E = 0: |p| is conserved exactly and the Boris rotation angle per
    step is 2 atan(q B dt / (2 gamma))."""
    n, b0, g, dt = 64, 2000.0, 206.0, 0.01
    ens, E, B = _ensemble(n, b0, g)
    p0 = ens["p"].copy()
    p1 = mc.boris(p0, E, B, -1.0, dt)
    np.testing.assert_allclose(np.linalg.norm(p1, axis=1), np.linalg.norm(p0, axis=1), rtol=1e-15)
    ang = np.arctan2(p1[:, 1], p1[:, 0]) - np.arctan2(p0[:, 1], p0[:, 0])
    ang = (ang + np.pi) % (2 * np.pi) - np.pi
    np.testing.assert_allclose(ang, 2 * math.atan(b0 * dt / (2 * g)), rtol=1e-12)


def test_first_event_binomial(rad):
    """P(event within dt) = 1 - exp(-W dt) with tau ~ Exp(1)."""
    n = 200000
    b0, g = 2000.0, 206.0
    ens, E, B = _ensemble(n, b0, g)
    tau = mc.init_tau(ens["id"], seed=0)
    out = mc.lepton_step(ens["x"], ens["p"], tau, ens["id"], E, B, q=-1.0, dt=0.01, step=0,
                         seed=0, sampler=rad, next_id=n)
    chi = spectra.chi_lepton(mc.boris(ens["p"], E, B, -1.0, 0.01)[:1], E[:1], B[:1])[0]
    W = RATE_UNIT * tables.fine_row("I", chi, tables.RAD_M, need_rho=False).total / g
    pr = 1 - math.exp(-W * 0.01)
    k = out["emitters"].size
    assert abs(k - n * pr) < 4 * math.sqrt(n * pr * (1 - pr))


def _poisson_run(rad, dt, steps, n=20000, b0=2000.0, g=206.0):
    ens, E, B = _ensemble(n, b0, g, seed=3)
    tau = mc.init_tau(ens["id"], seed=5)
    x, p = ens["x"], ens["p"]
    total = 0
    for s in range(steps):
        out = mc.lepton_step(x, p, tau, ens["id"], E, B, q=-1.0, dt=dt, step=s, seed=5,
                             sampler=rad, next_id=n, recoil=False)
        x, p, tau = out["x"], out["p"], out["tau"]
        total += out["n_events"]
    return total, out["W"][0]


@pytest.mark.parametrize("dt", [0.01, 0.05])
def test_event_counts_poisson_independent_of_dt(rad, dt):
    """No recoil, constant chi: events over T are Poisson(N W T) for any dt
    (the optical-depth carry makes the step size irrelevant)."""
    T = 0.2
    total, W = _poisson_run(rad, dt, int(round(T / dt)))
    mean = 20000 * W * T
    assert abs(total - mean) < 4 * math.sqrt(mean)


def test_thinning_fraction_and_spectrum(rad):
    """Accepted photons: fraction W_cut / W_full with the cut xi >= 2/gamma (text
    under Eq. 7), and the accepted xi follow the truncated CDF (one-sample KS)."""
    n, b0, g = 200000, 200.0, 206.0
    ens, E, B = _ensemble(n, b0, g, seed=11)
    tau = np.zeros(n)   # every particle emits at the start of the step
    out = mc.lepton_step(ens["x"], ens["p"], tau, ens["id"], E, B, q=-1.0, dt=1e-9, step=0,
                         seed=9, sampler=rad, next_id=n, kmax=1, recoil=False)
    chi = out["chi"][0]
    row = tables.fine_row("I", chi, tables.RAD_M)
    P = row.F / row.total
    xcut = 2.0 / g
    Pcut = float(np.interp(math.log(xcut) - math.log1p(-xcut), row.s, P))
    kept = out["photons"]["gamma"].size
    assert abs(kept / n - (1 - Pcut)) < 4 * math.sqrt((1 - Pcut) * Pcut / n)
    xi = np.sort(out["photons"]["gamma"] / g)
    Pe = (np.interp(np.log(xi) - np.log1p(-xi), row.s, P) - Pcut) / (1 - Pcut)
    m = xi.size
    ks = max(np.max(np.abs(np.arange(1, m + 1) / m - Pe)), np.max(np.abs(np.arange(m) / m - Pe)))
    assert ks < 1.63 / math.sqrt(m) + 2e-4


def test_fig1_kept_fractions(rad):
    """Survey-scratch values of W_cut / W_full for the Fig. 1 triples, recomputed
    from the oracle's CDF: 0.493, 0.683, 0.883."""
    for (b0, g), ref in zip(workloads.FIG1_TRIPLES, (0.49332, 0.68321, 0.88332)):
        chi = g * math.sqrt(1 - 1 / g ** 2) * b0 / E_S
        row = tables.fine_row("I", chi, tables.RAD_M)
        xc = 2.0 / g
        Pc = float(np.interp(math.log(xc) - math.log1p(-xc), row.s, row.F / row.total))
        assert abs((1 - Pc) - ref) < 2e-4


def test_method1_vs_method2_and_dt_study(rad):
    """The paper's generators: method I (W Dt > r_1) and method II (optical
    depth) have the same mean rate for W Dt <= 0.2; at W Dt = 6 method I
    saturates at one event per step (the 'very different' result of Fig. 3)."""
    n, b0, g = 100000, 2000.0, 206.0
    ens, E, B = _ensemble(n, b0, g, seed=4)
    chi = spectra.chi_lepton(ens["p"][:1], E[:1], B[:1])[0]
    W = RATE_UNIT * tables.fine_row("I", chi, tables.RAD_M, need_rho=False).total / g
    for wdt in (0.2, 6.0):
        dt = wdt / W
        ev = mc.lepton_step_method1(ens["p"], None, ens["id"], E, B, q=-1.0, dt=dt, step=0,
                                    seed=1, sampler=rad)
        rate1 = ev.sum() / (n * dt)
        if wdt <= 1:
            assert abs(rate1 / W - 1) < 4 * math.sqrt((1 - wdt) / (n * wdt))
        else:
            assert abs(rate1 - 1 / dt) < 1e-12 / dt and rate1 < W / 5
    # method II with the same dt = 0.2/W: events per unit time = W
    dt = 0.2 / W
    total, _ = _poisson_run(rad, dt, 10, n=20000, b0=b0, g=g)
    mean = 20000 * W * dt * 10
    assert abs(total - mean) < 4 * math.sqrt(mean)


def test_method3_doubles_rate():
    """Method III (emit when P_cum > r_3, P_cum reset after an event) has mean
    waiting 'probability' 1/2, i.e. twice the rate: it is not equivalent to
    methods I and II, contrary to the paper's statement."""
    rng = np.random.default_rng(1)
    W, dt, steps, n = 1.0, 0.01, 2000, 2000
    events = 0
    r3 = rng.uniform(size=n)
    pcum = np.zeros(n)
    for _ in range(steps):
        pcum += W * dt
        fire = pcum > r3
        events += fire.sum()
        pcum[fire] = 0.0
        r3[fire] = rng.uniform(size=fire.sum())
    rate = events / (n * steps * dt)
    assert 1.9 < rate / W < 2.1


def test_compaction_bruteforce():
    rng = np.random.default_rng(0)
    n = 1000
    ids = np.arange(n, dtype=np.uint64)
    dead = rng.uniform(size=n) < 0.3
    ids[dead] = mc.DEAD_ID
    vals = rng.normal(size=(n, 3))
    out_ids, out_vals = mc.compact(ids, vals)
    exp_ids, exp_vals = [], []
    for i in range(n):
        if ids[i] != mc.DEAD_ID:
            exp_ids.append(ids[i])
            exp_vals.append(vals[i])
    assert list(out_ids) == exp_ids
    np.testing.assert_array_equal(out_vals, np.array(exp_vals))


def test_tsc_weights_and_linear_exactness():
    n, L = 16, 16.0
    ix = np.arange(n, dtype=np.float64)
    # field linear in x in the interior, constant in y, z
    Eg = np.zeros((3, n, n, n))
    Eg[0] = (2.0 + 0.5 * ix)[:, None, None]
    Eg[1] = 3.0
    Bg = np.zeros_like(Eg)
    rng = np.random.default_rng(2)
    x = np.column_stack([rng.uniform(3, 12, 100), rng.uniform(0, L, 100), rng.uniform(0, L, 100)])
    E, _ = mc.gather_tsc(Eg, Bg, L, x)
    np.testing.assert_allclose(E[:, 0], 2.0 + 0.5 * x[:, 0], rtol=1e-14)
    np.testing.assert_allclose(E[:, 1], 3.0, rtol=1e-14)


def test_standing_wave_is_vacuum_solution():
    h = 1e-5
    x, t, a0 = np.array([0.3, 1.7, 4.0]), 0.8, 500.0
    E, B = mc.standing_wave(x, t, a0)
    Ep, Bp = mc.standing_wave(x, t + h, a0)
    Em, Bm = mc.standing_wave(x, t - h, a0)
    Ex1, Bx1 = mc.standing_wave(x + h, t, a0)
    Ex0, Bx0 = mc.standing_wave(x - h, t, a0)
    dBdt = (Bp - Bm) / (2 * h)
    dEdt = (Ep - Em) / (2 * h)
    dEdx = (Ex1 - Ex0) / (2 * h)
    dBdx = (Bx1 - Bx0) / (2 * h)
    curlE = np.stack([np.zeros(3), -dEdx[:, 2], dEdx[:, 1]], axis=-1)
    curlB = np.stack([np.zeros(3), -dBdx[:, 2], dBdx[:, 1]], axis=-1)
    np.testing.assert_allclose(dBdt, -curlE, atol=1e-4)
    np.testing.assert_allclose(dEdt, curlB, atol=1e-4)


def test_pair_step_yield_and_kinematics(pair_table):
    ps = mc.PairSampler(pair_table, "f64")
    ph = workloads.pair_photons(50000, E_S, seed=2, chi_lo=0.5, chi_hi=5.0)
    tau = mc.init_tau(ph["id"], seed=2)
    dt = 0.01
    out = mc.photon_step(ph["x"], ph["k"], tau, ph["id"], ph["E"], ph["B"], dt=dt, step=0,
                         seed=2, sampler=ps, next_id=50000, move=False)
    gph = np.linalg.norm(ph["k"], axis=1)
    chi = spectra.chi_photon(ph["k"], ph["E"], ph["B"])
    np.testing.assert_allclose(chi, ph["chi_target"], rtol=1e-10)
    pr = 1 - np.exp(-out["W"] * dt)
    k = out["pairs"].size
    assert abs(k - pr.sum()) < 4 * math.sqrt(np.sum(pr * (1 - pr)))
    ge = np.sqrt(1 + np.sum(out["electrons"]["p"] ** 2, axis=1))
    gp = np.sqrt(1 + np.sum(out["positrons"]["p"] ** 2, axis=1))
    np.testing.assert_allclose(ge + gp, gph[out["pairs"]], rtol=1e-12)
    assert np.all(out["id"][out["pairs"]] == mc.DEAD_ID)
    assert np.all(out["positrons"]["id"] - out["electrons"]["id"] == 1)
    # electron takes xi or 1 - xi with equal probability
    frac = np.mean(out["electrons"]["xi"] > 0.5)
    assert abs(frac - 0.5) < 4 * math.sqrt(0.25 / k)


def test_method1_substep_rates(rad):
    """Method I with adaptive sub-steps (W Dt / N <= 0.2): the event rate matches
    the rate integral for Dt = 0.2/W and Dt = 6/W; without sub-steps Dt = 6/W
    saturates at one event per step (the paper's Fig. 3 discussion)."""
    n, b0, g = 20000, 2000.0, 206.0
    ens, E, B = _ensemble(n, b0, g, seed=6)
    chi = spectra.chi_lepton(ens["p"][:1], E[:1], B[:1])[0]
    W = RATE_UNIT * tables.fine_row("I", chi, tables.RAD_M, need_rho=False).total / g
    for wdt, sub in ((0.2, True), (6.0, True), (6.0, False)):
        dt = wdt / W
        r = mc.lepton_step_method1_full(ens["x"], ens["p"], ens["id"], E, B, q=-1.0, dt=dt, step=0, seed=3,
                                        sampler=rad, next_id=n, recoil=False, kmax=64)
        if not sub:
            r = mc.lepton_step_method1_full(ens["x"], ens["p"], ens["id"], E, B, q=-1.0, dt=dt, step=0,
                                            seed=3, sampler=rad, next_id=n, recoil=False, kmax=64,
                                            substep=False)
        rate = r["n_events"] / (n * dt)
        if sub:
            # events per particle: Binomial(N, W dt / N) with N = ceil(W dt / 0.2)
            N = int(np.ceil(wdt / 0.2 - 1e-12))
            mean, var = n * wdt, n * N * (wdt / N) * (1 - wdt / N)
            assert abs(r["n_events"] - mean) < 4 * math.sqrt(var)
            assert np.all(r["N"] == N)
        else:
            assert r["n_events"] == n and rate < W / 5
