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
    ph = workloads.pair_photons(50000, seed=2, chi_lo=0.5, chi_hi=5.0)
    ph["k"] = ph["khat"] * (ph["chi_target"] / spectra.chi_photon(ph["khat"], ph["E"], ph["B"]))[:, None]
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


def _gamma(p):
    return np.sqrt(1.0 + np.sum(np.asarray(p) ** 2, axis=-1))


@pytest.mark.parametrize("kmax,dt", [(1, 1e-9), (4, 0.3)])
def test_recoil_energy_and_direction(rad, kmax, dt):
    """Recoil (the energies defined under Eq. 1: the photon takes eps_ph = xi eps_e,
    the lepton keeps the rest): per lepton, gamma after the step plus the energies
    of its photons equals gamma after the push, as long as no recoil hits the
    gamma' = 1 floor; photons travel along the lepton's direction and the lepton
    keeps its direction; a lepton whose events were all below the infrared cut
    keeps its momentum; the rate after a recoil is the rate at the new chi and
    gamma.  kmax = 1 with tau = 0: one event per lepton at the start of the step;
    kmax = 4, dt = 0.3 at chi ~ 10: several events per lepton."""
    n, b0, g = 20000, 2000.0, 2060.0
    ens, E, B = _ensemble(n, b0, g, seed=21)
    tau = np.zeros(n) if kmax == 1 else mc.init_tau(ens["id"], seed=21)
    out = mc.lepton_step(ens["x"], ens["p"], tau, ens["id"], E, B, q=-1.0, dt=dt, step=0,
                         seed=21, sampler=rad, next_id=n, kmax=kmax, recoil=True)
    p_push = mc.boris(ens["p"], E, B, -1.0, dt)
    g_push, g_out = _gamma(p_push), _gamma(out["p"])
    ph = out["photons"]
    assert ph["gamma"].size > n // 10
    g_ph = np.bincount(ph["parent"], weights=ph["gamma"], minlength=n)
    emitted = np.bincount(ph["parent"], minlength=n) > 0
    np.testing.assert_allclose(g_out[emitted] + g_ph[emitted], g_push[emitted], rtol=1e-12)
    assert np.all(g_out[emitted] > 1.0)
    # energy really moved: the lepton lost what the photons carry
    assert np.all(g_out[emitted] < g_push[emitted] - 1.9)
    # no photon: momentum untouched (events below the cut do not recoil)
    np.testing.assert_array_equal(out["p"][~emitted], p_push[~emitted])
    # directions: photon k parallel to the pushed momentum, recoiled p as well
    nh = p_push / np.linalg.norm(p_push, axis=1)[:, None]
    kh = ph["k"] / np.linalg.norm(ph["k"], axis=1)[:, None]
    np.testing.assert_allclose(np.sum(kh * nh[ph["parent"]], axis=1), 1.0, rtol=1e-13)
    ph_dir = out["p"][emitted] / np.linalg.norm(out["p"][emitted], axis=1)[:, None]
    np.testing.assert_allclose(np.sum(ph_dir * nh[emitted], axis=1), 1.0, rtol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(ph["k"], axis=1), ph["gamma"], rtol=1e-14)
    # the rate left in W is the one at the recoiled state
    chi_new = spectra.chi_lepton(out["p"][emitted], E[emitted], B[emitted])
    np.testing.assert_allclose(out["W"][emitted], rad.rate(chi_new, g_out[emitted]), rtol=1e-12)
    if kmax > 1:
        assert np.max(np.bincount(ph["parent"], minlength=n)) >= 2


def test_cascade_step_energy_and_bookkeeping(rad_table_I, pair_table):
    """cascade_step in a uniform magnetic field (E = 0: the push does no work):
    the total energy of electrons, positrons and photons is conserved (photon ->
    e- + e+ with xi gamma_ph and (1 - xi) gamma_ph, lepton -> lepton + photon with
    (1 - xi) gamma and xi gamma), up to the gamma' >= 1 floor; every pair adds one
    electron and one positron, at the same rank, with ids next_id + 2r, + 1;
    converted photons are removed; ids stay unique and below next_id."""
    rad = mc.RadSampler(rad_table_I, "f64")
    pair = mc.PairSampler(pair_table, "f64")
    n, g0 = 2000, 1.0e4
    b0 = 20.0 * E_S / g0                          # chi_e = 20 for p perpendicular to B
    rng = np.random.default_rng(5)
    phi = rng.uniform(0, 2 * math.pi, n)
    pm = math.sqrt(g0 * g0 - 1.0)
    st = dict(el=dict(x=np.zeros((n, 3)), p=np.stack([pm * np.cos(phi), pm * np.sin(phi), np.zeros(n)], -1),
                      tau=mc.init_tau(np.arange(n, dtype=np.uint64), seed=7), id=np.arange(n, dtype=np.uint64)),
              po=dict(x=np.zeros((0, 3)), p=np.zeros((0, 3)), tau=np.zeros(0), id=np.zeros(0, np.uint64)),
              ph=dict(x=np.zeros((0, 3)), p=np.zeros((0, 3)), tau=np.zeros(0), id=np.zeros(0, np.uint64)),
              next_id=n)

    def energy():
        return (_gamma(st["el"]["p"]).sum() + _gamma(st["po"]["p"]).sum()
                + np.linalg.norm(st["ph"]["p"], axis=1).sum())

    e0 = energy()
    total_pairs = 0
    for s in range(12):
        ne, npo = st["el"]["id"].size, st["po"]["id"].size
        nid = st["next_id"]
        mc.cascade_step(st, dt=0.05, step=s, seed=7, rad=rad, pair=pair, E0=(0, 0, 0), B0=(0, 0, b0))
        new_e = st["el"]["id"][ne:]
        new_p = st["po"]["id"][npo:]
        assert new_e.size == new_p.size
        total_pairs += new_e.size
        if new_e.size:
            np.testing.assert_array_equal(new_p - new_e, np.ones(new_e.size, np.uint64))
            np.testing.assert_array_equal((new_e - np.uint64(nid)) % np.uint64(2), np.zeros(new_e.size, np.uint64))
        assert not np.any(st["ph"]["id"] == mc.DEAD_ID)
        ids = np.concatenate([st["el"]["id"], st["po"]["id"], st["ph"]["id"]])
        assert np.unique(ids).size == ids.size and ids.max() < st["next_id"]
    assert total_pairs > 20 and st["ph"]["id"].size > n
    assert st["el"]["id"].size == n + total_pairs
    e1 = energy()
    assert abs(e1 - e0) < 1e-11 * e0 + 2.0, (e0, e1)


def test_retirement_is_exact(rad_table_I, pair_table):
    """Photon retirement (a photon whose optical depth exceeds the envelope pair
    rate at its largest reachable chi times the time left cannot convert before
    the end): the same cascade with and without it gives identical electrons and
    positrons (ids, momenta, positions, optical depths), and the photons kept plus
    the tally give the histogram of the photons followed without retirement; most
    photons are retired.  Uniform B = b0 z, E = 0: |E| + |B| = b0."""
    rad = mc.RadSampler(rad_table_I, "f64")
    pair = mc.PairSampler(pair_table, "f64")
    n, g0, steps, dt = 1500, 1.0e4, 10, 0.05
    b0 = 20.0 * E_S / g0
    rng = np.random.default_rng(9)
    phi = rng.uniform(0, 2 * math.pi, n)
    pm = math.sqrt(g0 * g0 - 1.0)

    def run(retire):
        e0 = lambda: dict(x=np.zeros((0, 3)), p=np.zeros((0, 3)), tau=np.zeros(0), id=np.zeros(0, np.uint64))
        st = dict(el=dict(x=np.zeros((n, 3)), p=np.stack([pm * np.cos(phi), pm * np.sin(phi), np.zeros(n)], -1),
                          tau=mc.init_tau(np.arange(n, dtype=np.uint64), seed=3), id=np.arange(n, dtype=np.uint64)),
                  po=e0(), ph=e0(), next_id=n)
        for s in range(steps):
            mc.cascade_step(st, dt=dt, step=s, seed=3, rad=rad, pair=pair, E0=(0, 0, 0), B0=(0, 0, b0),
                            retire=retire)
        return st

    a = run(None)
    b = run((steps * dt, b0))
    for sp in ("el", "po"):
        for k in ("id", "p", "x", "tau"):
            np.testing.assert_array_equal(a[sp][k], b[sp][k])
    assert a["po"]["id"].size > 10
    ga = np.linalg.norm(a["ph"]["p"], axis=1)
    gb = np.linalg.norm(b["ph"]["p"], axis=1)
    ha = np.zeros(mc.TALLY_BINS, dtype=np.int64)
    mc.tally_add(ha, ga)
    hb = b["tally"].copy()
    mc.tally_add(hb, gb)
    np.testing.assert_array_equal(ha, hb)
    # the photons still followed are the unretired ones of the full run, same ids
    assert set(b["ph"]["id"].tolist()) <= set(a["ph"]["id"].tolist())
    assert b["tally"].sum() > 0.5 * ga.size
