"""Emission and pair cascade on the GPU (pairs, both lepton passes, photon
compaction in one loop) against the oracle's cascade on the same particles in
the a0 = 1000 standing wave (float32 on the GPU, float64 in the oracle)."""
import math

import numpy as np
import pytest

from oracle import mc, tables
from tests.gpu_helpers import need_gpu

import workloads

pytestmark = pytest.mark.gpu


def test_cascade_counts_and_spectra(rad_table_I, pair_table):
    torch, q = need_gpu()
    n, ngrid, a0, dt, steps = 20000, 128, 1000.0, 0.01, 40
    L = workloads.BOX_L
    seed = 4
    # energetic seed electrons (momentum spread 1000 m_e c) so that photons reach
    # chi_ph ~ 1 within the test's 40 steps
    ens = workloads.standing_wave_electrons(n, seed=seed, p_spread=1000.0)
    x = ens["x"].astype(np.float32).astype(np.float64)
    p = ens["p"].astype(np.float32).astype(np.float64)
    tau = mc.init_tau(ens["id"], seed=seed)
    # GPU
    ctx = q.Context(seed=seed, kmax=4, flags=q.QED_FLAG_TRACK_DEAD)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    cap_l, cap_p = 8 * n, 40 * n
    el, po, ph = q.Species(cap_l, "f32"), q.Species(cap_l, "f32"), q.Species(cap_p, "f32")
    el.load(x, p, tau, ens["id"])
    po.load(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint64))
    ph.load(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint64))
    ctx.qed_set_next_id(n)
    ctx.qed_reserve(cap_p)
    grid = torch.empty(ngrid ** 3 * 6, dtype=torch.float32, device="cuda")
    fld = q.Fields(q.QED_FIELD_GRID, grid=grid, n=ngrid, L=L)
    for s in range(steps):
        ctx.qed_fill_standing_wave(grid, ngrid, L, a0, s * dt)
        ctx.qed_create_pairs(fld, ph, el, po, dt, s)
        for sp, qq in ((el, -1), (po, 1)):
            ctx.qed_gather_push(fld, sp, qq, dt, s)
            ctx.qed_emit_photons(sp, ph, s)
        ctx.qed_compact(ph)
    st, rc = ctx.qed_get_status()
    assert st["scan_timeouts"] == 0 and st["dropped"] == 0
    # oracle on the same particles and streams
    z = lambda: dict(x=np.zeros((0, 3)), p=np.zeros((0, 3)), tau=np.zeros(0), id=np.zeros(0, np.uint64))
    S = dict(el=dict(x=x, p=p, tau=tau, id=ens["id"].copy()), po=z(), ph=z(), next_id=n)
    rad = mc.RadSampler(rad_table_I, "q16")
    pair = mc.PairSampler(pair_table, "q16")
    for s in range(steps):
        Eg, Bg = mc.standing_wave_grid(ngrid, L, a0, s * dt)
        mc.cascade_step(S, Eg=Eg, Bg=Bg, L=L, dt=dt, step=s, seed=seed, rad=rad, pair=pair)
    n_ph, n_po = ph.n(), po.n()
    o_ph, o_po = S["ph"]["id"].size, S["po"]["id"].size
    print(f"cascade: photons GPU {n_ph} oracle {o_ph}; pairs GPU {n_po} oracle {o_po}; "
          f"electrons GPU {el.n()} oracle {S['el']['id'].size}")
    assert o_po > 30 and o_ph > 1000
    assert abs(n_ph - o_ph) < 4 * math.sqrt(o_ph)
    assert abs(n_po - o_po) < 4 * math.sqrt(o_po) + 3
    assert el.n() - n == n_po
    # photon energy spectra (two-sample KS at the sample sizes' 0.1% level)
    gg = np.sort(np.linalg.norm(ph.to_numpy()["p"], axis=1))
    go = np.sort(np.linalg.norm(S["ph"]["p"], axis=1))
    allv = np.concatenate([gg, go])
    ks = np.max(np.abs(np.searchsorted(gg, allv, side="right") / gg.size
                       - np.searchsorted(go, allv, side="right") / go.size))
    crit = 1.95 * math.sqrt((gg.size + go.size) / (gg.size * go.size))
    print(f"photon energy KS {ks:.2e} (0.1% critical {crit:.2e})")
    assert ks < crit


def test_retirement_cascade_f64_matches_oracle(rad_table_I, pair_table):
    """The cascade with photon retirement (qed_set_retirement), float64, uniform
    B = b0 z (|E| + |B| = b0) with electrons at gamma = 1e4, chi = 20, 10 steps
    of 0.05: electrons, positrons and followed photons (ids, momenta) and the
    tally (retired photons, then the followed ones added by qed_tally_species)
    against the oracle's cascade with the same retirement rule (end time set
    five steps beyond the run, so that some photons are still followed)."""
    torch, q = need_gpu()
    from oracle.constants import E_S
    n, g0, steps, dt, seed = 1500, 1.0e4, 10, 0.05, 3
    t_end = (steps + 5) * dt
    b0 = 20.0 * E_S / g0
    rng = np.random.default_rng(9)
    phi = rng.uniform(0, 2 * math.pi, n)
    pm = math.sqrt(g0 * g0 - 1.0)
    p0 = np.stack([pm * np.cos(phi), pm * np.sin(phi), np.zeros(n)], -1)
    ids = np.arange(n, dtype=np.uint64)
    tau0 = mc.init_tau(ids, seed=seed)
    # oracle
    e0 = lambda: dict(x=np.zeros((0, 3)), p=np.zeros((0, 3)), tau=np.zeros(0), id=np.zeros(0, np.uint64))
    st = dict(el=dict(x=np.zeros((n, 3)), p=p0.copy(), tau=tau0.copy(), id=ids.copy()), po=e0(), ph=e0(), next_id=n)
    rad, pair = mc.RadSampler(rad_table_I, "f64"), mc.PairSampler(pair_table, "f64")
    for s in range(steps):
        mc.cascade_step(st, dt=dt, step=s, seed=seed, rad=rad, pair=pair, E0=(0, 0, 0), B0=(0, 0, b0),
                        retire=(t_end, b0))
    # GPU
    ctx = q.Context(seed=seed, kmax=4, flags=q.QED_FLAG_TRACK_DEAD)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    ctx.qed_set_retirement(t_end, b0)
    el, po, ph = q.Species(4 * n, "f64"), q.Species(4 * n, "f64"), q.Species(40 * n, "f64")
    el.load(np.zeros((n, 3)), p0, tau0, ids)
    z = np.zeros((0, 3))
    po.load(z, z, np.zeros(0), np.zeros(0, np.uint64))
    ph.load(z, z, np.zeros(0), np.zeros(0, np.uint64))
    ctx.qed_set_next_id(n)
    ctx.qed_reserve(40 * n)
    fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, b0))
    for s in range(steps):
        ctx.qed_create_pairs(fld, ph, el, po, dt, s)
        for sp, qq in ((el, -1), (po, 1)):
            ctx.qed_gather_push(fld, sp, qq, dt, s)
            ctx.qed_emit_photons(sp, ph, s)
        ctx.qed_compact(ph)
    stat, rc = ctx.qed_get_status()
    tally_retired = ctx.qed_get_tally()
    ctx.qed_tally_species(ph)
    tally_all = ctx.qed_get_tally()
    g = {k: sp.to_numpy() for k, sp in (("el", el), ("po", po), ("ph", ph))}
    print(f"retirement cascade: electrons {g['el']['id'].size} positrons {g['po']['id'].size} photons followed "
          f"{g['ph']['id'].size}, retired {int(tally_retired.sum())} (oracle {int(st['tally'].sum())})")
    assert g["po"]["id"].size > 10 and g["ph"]["id"].size > 10 and stat["retired"] == int(tally_retired.sum())
    for k in ("el", "po", "ph"):
        np.testing.assert_array_equal(g[k]["id"], st[k]["id"])
        np.testing.assert_allclose(g[k]["p"], st[k]["p"], rtol=1e-9, atol=1e-9 * np.abs(st[k]["p"]).max(initial=1.0))
    np.testing.assert_array_equal(tally_retired, st["tally"])
    want = st["tally"].copy()
    mc.tally_add(want, np.linalg.norm(st["ph"]["p"], axis=1))
    np.testing.assert_array_equal(tally_all, want)
