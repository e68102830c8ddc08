"""Surrogate networks on the GPU: forward and gradient against the exact
float64 oracle network within the derived bound of the GPU's split-bf16
arithmetic, training accuracy against the oracle's rate
quadrature and exact CDF, fallback coverage, and the measured gain over the
table sampler."""
import math
import time

import numpy as np
import pytest

from oracle import mc, mlp, tables
from oracle.constants import E_S, RATE_UNIT
from tests import mlp_bound
from tests.gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


def _rand_theta(net, seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, mlp.n_params(net)).astype(np.float32)


@pytest.mark.parametrize("net,netid", [("A", 0), ("B", 1)])
def test_forward_and_gradient_vs_oracle(net, netid):
    """Forward (inference form) and gradient (training form) of random nets
    against the exact float64 network, elementwise within the first-order bound
    of the GPU's split-bf16 / float32 arithmetic (tests/mlp_bound.py), on 1000
    samples (62 full 16-sample tiles and a ragged one)."""
    torch, q = need_gpu()
    ctx = q.Context()
    th = _rand_theta(net, 10 + netid)
    ctx.qed_surrogate_io(netid, th)
    nin, nout = mlp.SIZES[net]
    n = 1000
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (n, nin)).astype(np.float32)
    T = rng.normal(size=(n, nout)).astype(np.float32)
    M = (rng.uniform(size=(n, nout)) < 0.8).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    y = torch.empty((n, nout), dtype=torch.float32, device="cuda")
    print(f"surrogate forward/gradient: net {net}, {n} samples", flush=True)
    ctx.qed_surrogate_forward(netid, dev(X), y)
    g = torch.empty(mlp.n_params(net), dtype=torch.float32, device="cuda")
    ctx.qed_surrogate_grad(netid, dev(X), dev(T), dev(M), g)
    torch.cuda.synchronize()
    th64 = th.astype(np.float64)
    X64, T64, M64 = (a.T.astype(np.float64) for a in (X, T, M))
    ye, Ey, _ = mlp_bound.forward_bound(th64, net, X64)
    _, sy, _ = mlp_bound.forward_bound(th64, net, X64, mode="rss")
    yg = y.cpu().numpy().T.astype(np.float64)
    err = np.abs(yg - ye)
    print(f"  forward: max |err| {err.max():.2e}, max err/bound {np.max(err / Ey):.3f}, "
          f"max err/sigma {np.max(err / sy):.2f}")
    assert np.all(err <= Ey)
    assert np.all(err <= mlp_bound.K_SIGMA * sy)
    # a sample's output does not depend on where it sits in a 16-sample tile
    # (samples are independent columns of the matrix products): shifting the
    # inputs by 5 moves every sample to another lane and tile, bit for bit the same
    y5 = torch.empty((n - 5, nout), dtype=torch.float32, device="cuda")
    ctx.qed_surrogate_forward(netid, dev(X[5:]), y5)
    torch.cuda.synchronize()
    assert np.array_equal(y5.cpu().numpy(), y.cpu().numpy()[5:])
    ge, bound = mlp_bound.grad_bound(th64, net, X64, T64, M64)
    _, sg = mlp_bound.grad_bound(th64, net, X64, T64, M64, mode="rss")
    gg = g.cpu().numpy().astype(np.float64)
    gerr = np.abs(gg - ge)
    print(f"  gradient: max |err| {gerr.max():.2e} (max |g| {np.abs(ge).max():.2e}), "
          f"max err/bound {np.max(gerr / bound):.3f}, max err/sigma {np.max(gerr / sg):.2f}")
    assert np.all(gerr <= bound)
    assert np.all(gerr <= mlp_bound.K_SIGMA * sg)


@pytest.fixture(scope="module")
def trained():
    torch, q = need_gpu()
    ctx = q.Context(seed=3)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    t0 = time.time()
    ctx.qed_surrogate_train(20000, batch=4096, lr=3e-3, seed=11)
    torch.cuda.synchronize()
    print(f"training: {time.time() - t0:.1f} s for 2 nets x 20000 steps x 4096 samples")
    return ctx


def _sample(ctx, q, torch, chi, gamma, prec, step=0, seed_ids=0):
    n = chi.size
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    ids = np.arange(seed_ids, seed_ids + n, dtype=np.uint64)
    lnw = torch.empty(n, dtype=torch.float32, device="cuda")
    xi = torch.empty_like(lnw)
    lnwp = torch.empty_like(lnw)
    ctx.qed_sample(dev(chi, torch.float64), dev(gamma, torch.float64), dev(ids.view(np.int64), torch.int64),
                   prec, step, lnw, xi, lnwp)
    torch.cuda.synchronize()
    return lnw.cpu().numpy().astype(np.float64), xi.cpu().numpy().astype(np.float64), lnwp.cpu().numpy().astype(np.float64)


def test_trained_rates_vs_oracle(trained, rad_table_I, pair_table):
    """Rate surrogate within 1e-3 of the oracle's rates over chi in [1e-3, 1e2]."""
    torch, q = need_gpu()
    ctx = trained
    chi = np.logspace(-3, 2, 20001)
    gam = np.full(chi.size, 1000.0)
    ctx.qed_get_status(check=False)
    lnw, _, lnwp = _sample(ctx, q, torch, chi, gam, q.QED_SAMPLER_MLP)
    st, _ = ctx.qed_get_status(check=False)
    ref = np.log(tables.rate_rad(rad_table_I, chi, gam))
    err = np.max(np.abs(np.exp(lnw - ref) - 1))
    refp = np.log(tables.rate_pair(pair_table, chi, gam))
    okp = chi >= 1e-2
    errp = np.max(np.abs(np.exp(lnwp[okp] - refp[okp]) - 1))
    print(f"rate surrogate: max rel err rad {err:.2e} pair {errp:.2e}, rate fallbacks {st['mlp_fallback_rate']}")
    assert err < 1e-3 and errp < 1e-3
    assert st["mlp_fallback_rate"] == 0


@pytest.mark.parametrize("chi", [0.01, 0.3, 3.0, 60.0])
def test_trained_xi_ks_1e7(trained, rad_table_I, chi):
    """1e7 xi samples from the surrogate sampler (with residual check and table
    fallback) against the exact CDF (one-sample KS) and the oracle's table sampler
    (two-sample KS), both <= 2e-3."""
    torch, q = need_gpu()
    ctx = trained
    n = 10_000_000
    ctx.qed_get_status(check=False)
    _, xi, _ = _sample(ctx, q, torch, np.full(n, chi), np.full(n, 1e3), q.QED_SAMPLER_MLP, step=5)
    st, _ = ctx.qed_get_status(check=False)
    xi = np.sort(xi)
    row = tables.fine_row("I", chi, tables.RAD_M)
    P = row.F / row.total
    xs = np.clip(xi, 1e-300, 1 - 1e-7)
    s = np.log(xs) - np.log1p(-xs)
    Pe = np.interp(s, row.s, P, left=0.0)
    # below the fine grid the CDF follows the infrared law P ~ xi^(1/3)
    lo = s < row.s[0]
    Pe[lo] = P[0] * (xs[lo] / (1 / (1 + math.exp(-row.s[0])))) ** (1 / 3)
    ks1 = max(np.max(np.arange(1, n + 1) / n - Pe), np.max(Pe - np.arange(n) / n))
    rng = np.random.default_rng(7)
    u = (np.floor(rng.uniform(size=n) * 2 ** 23) + 0.5) * 2.0 ** -23
    ur = (np.floor(rng.uniform(size=n) * 2 ** 23) + 0.5) * 2.0 ** -23
    xo, _ = mc.RadSampler(rad_table_I, "q16").sample(np.full(n, chi), u, ur)
    xo = np.sort(xo)
    allv = np.concatenate([xi, xo])
    ks2 = np.max(np.abs(np.searchsorted(xi, allv, side="right") / n - np.searchsorted(xo, allv, side="right") / n))
    fb = st["mlp_fallback_xi"] / n
    print(f"chi {chi}: KS(exact) {ks1:.2e} KS(table sampler) {ks2:.2e} xi fallback {fb:.4%}")
    assert ks1 < 2e-3 and ks2 < 2e-3
    assert fb < 0.01          # u outside [1e-4, 1-1e-4] alone is 2e-4


def test_sampler_position_independent(trained):
    """qed_sample with the nets: each sample's ln W_rad, xi and ln W_pair are bit
    for bit the same when the inputs are shifted by 37 (other lane, other
    16-sample tile, other wave), with ragged tails on both runs."""
    torch, q = need_gpu()
    ctx = trained
    n, k = 5000 + 37, 37
    rng = np.random.default_rng(12)
    chi = 10.0 ** rng.uniform(-3.5, 2.5, n)          # also outside the trained range
    gam = rng.uniform(1.5, 3e3, n)
    full = _sample(ctx, q, torch, chi, gam, q.QED_SAMPLER_MLP, step=3)
    part = _sample(ctx, q, torch, chi[k:], gam[k:], q.QED_SAMPLER_MLP, step=3, seed_ids=k)
    for a, b in zip(full, part):
        assert np.array_equal(a[k:], b, equal_nan=True)


def test_surrogate_gain_vs_table(trained):
    """What the trained networks gain over the plain table sampler on the same
    1e8 lookups (rate + xi + pair rate for every sample, qed_sample): the
    measured throughput ratio surrogate / table is the result.  On this GPU the
    table (in LDS and the caches) is cheaper than two 3 x 64 networks per sample,
    so the ratio is well below 1: the test states that outcome (0.02 < ratio < 1)
    rather than a gain."""
    torch, q = need_gpu()
    ctx = trained
    n = 100_000_000
    inp_chi = torch.pow(10.0, torch.rand(n, dtype=torch.float64, device="cuda") * 5 - 3)
    gam = torch.full((n,), 1e3, dtype=torch.float64, device="cuda")
    ids = torch.arange(n, dtype=torch.int64, device="cuda")
    lnw = torch.empty(n, dtype=torch.float32, device="cuda")
    xi = torch.empty_like(lnw)
    lnwp = torch.empty_like(lnw)
    res = {}
    for name, prec in (("table_f32", q.QED_F32), ("mlp", q.QED_SAMPLER_MLP)):
        ctx.qed_sample(inp_chi, gam, ids, prec, 1, lnw, xi, lnwp)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            ctx.qed_sample(inp_chi, gam, ids, prec, 1, lnw, xi, lnwp)
        e1.record()
        torch.cuda.synchronize()
        res[name] = n * 3 / (e0.elapsed_time(e1) * 1e-3)
    st, _ = ctx.qed_get_status(check=False)
    ratio = res["mlp"] / res["table_f32"]
    print(f"samples/s: table {res['table_f32']:.3e}  surrogate {res['mlp']:.3e}  "
          f"ratio surrogate/table {ratio:.3f}; xi fallback fraction {st['mlp_fallback_xi'] / (4 * n):.4%}")
    assert 0.02 < ratio < 1.0


def _with_weights(q, trained, **kw):
    ctx = q.Context(**kw)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    for net in (0, 1):
        ctx.qed_surrogate_io(net, trained.qed_surrogate_io(net))
    return ctx


def test_surrogate_step_independent_of_order(trained):
    """One surrogate step (rate net in the lepton pass, xi net and, after each
    recoil, the rate net in the emission pass; up to kmax events) on 2e4
    electrons at chi ~ 1 and ~ 10, and on the same electrons shuffled: every
    electron's momentum and optical depth and the set of photons are bit for bit
    the same, so no result depends on which lanes share a tile or a packed
    forward call."""
    torch, q = need_gpu()
    n, b0 = 20000, 2000.0
    rng = np.random.default_rng(31)
    gam = np.where(rng.uniform(size=n) < 0.5, 206.0, 2060.0)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    pm = np.sqrt(gam ** 2 - 1.0)
    p = np.stack([pm * np.cos(phi), pm * np.sin(phi), np.zeros(n)], axis=-1)
    x = np.zeros((n, 3))
    ids = np.arange(n, dtype=np.uint64)
    tau0 = rng.exponential(size=n)

    def run(order):
        ctx = _with_weights(q, trained, seed=23, kmax=4, flags=q.QED_FLAG_SURROGATE)
        lep = q.Species(n, "f32")
        ph = q.Species(4 * n, "f32")
        lep.load(x[order], p[order], tau=tau0[order], ids=ids[order])
        ctx.qed_set_next_id(n)
        fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, b0))
        ctx.qed_gather_push(fld, lep, -1, 0.2, 0)
        ctx.qed_emit_photons(lep, ph, 0)
        st, _ = ctx.qed_get_status(check=False)
        inv = np.argsort(lep.id[:n].cpu().numpy().view(np.uint64))
        lepton = [a[:n].cpu().numpy()[inv] for a in (lep.px, lep.py, lep.pz, lep.tau)]
        m = ph.n()
        phot = np.stack([a[:m].double().cpu().numpy() for a in (ph.px, ph.py, ph.pz, ph.tau)], axis=1)
        phot = phot[np.lexsort(phot.T[::-1])]
        return lepton, phot, st

    la, pa, sa = run(np.arange(n))
    lb, pb, sb = run(rng.permutation(n))
    print(f"order independence: {pa.shape[0]} photons, events {sa['events']}, capped {sa['capped']}, "
          f"fallbacks xi {sa['mlp_fallback_xi']} rate {sa['mlp_fallback_rate']}")
    assert sa["events"] > 1.5 * n and sa["capped"] > 0        # several events per electron, some capped
    for a, b in zip(la, lb):
        assert np.array_equal(a, b)
    assert np.array_equal(pa, pb)
    assert {k: sa[k] for k in ("events", "photons", "rejected", "capped")} == \
           {k: sb[k] for k in ("events", "photons", "rejected", "capped")}


def test_surrogate_emission_passes(trained):
    """The surrogate emission runs every emitter's first candidate in one pass
    and, with kmax > 1, the emitters with a further candidate within the step in
    a second pass that re-runs their first candidate silently.  The photons of
    the first pass come first: a run with kmax = 1 (no second pass; further
    candidates counted as capped) appends exactly the first photons of the run
    with kmax = 4, bit for bit (positions, momenta, optical depths, ids), and
    the electrons without a further candidate end the step identically.  2e4
    electrons at chi ~ 1 and ~ 10, dt = 0.2: several candidates per electron."""
    torch, q = need_gpu()
    n, b0 = 20000, 2000.0
    rng = np.random.default_rng(37)
    gam = np.where(rng.uniform(size=n) < 0.5, 206.0, 2060.0)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    pm = np.sqrt(gam ** 2 - 1.0)
    p = np.stack([pm * np.cos(phi), pm * np.sin(phi), np.zeros(n)], axis=-1)
    tau0 = rng.exponential(size=n)
    out = {}
    for kmax in (1, 4):
        print(f"surrogate emission passes: kmax {kmax}", flush=True)
        ctx = _with_weights(q, trained, seed=29, kmax=kmax, flags=q.QED_FLAG_SURROGATE)
        lep = q.Species(n, "f32")
        ph = q.Species(4 * n, "f32")
        lep.load(np.zeros((n, 3)), p, tau=tau0, ids=np.arange(n, dtype=np.uint64))
        ctx.qed_set_next_id(n)
        fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, b0))
        ctx.qed_gather_push(fld, lep, -1, 0.2, 0)
        ctx.qed_emit_photons(lep, ph, 0)
        st, _ = ctx.qed_get_status(check=False)
        out[kmax] = (st, lep.to_numpy(), ph.to_numpy())
    (s1, l1, p1), (s4, l4, p4) = out[1], out[4]
    m = p1["id"].size
    print(f"  kmax 1: {m} photons, capped {s1['capped']}; kmax 4: {p4['id'].size} photons, capped {s4['capped']}")
    assert s1["capped"] > 100 and p4["id"].size > m > 1000
    for k in ("x", "p", "tau", "id"):
        np.testing.assert_array_equal(p1[k][:m] if k != "id" else p1[k], p4[k][:m])
    # electrons whose step ended after the first candidate: identical in both runs
    same = np.all(l1["p"] == l4["p"], axis=1) & (l1["tau"] == l4["tau"])
    print(f"  electrons identical in both runs: {same.sum()} of {n}")
    assert same.sum() == n - s1["capped"]     # the capped ones are those the second pass finishes


def test_surrogate_step_spectrum_and_rate(trained):
    """The emission step with QED_FLAG_SURROGATE (candidate events at the rate
    envelope in the lepton pass, kept with the rate net's W / W_env, xi net in
    the emission pass): 1e6 electrons at chi ~ 1 without recoil for 20 steps of
    0.05 (~1e7 photons).  Kept events are Poisson with mean n W T (the optical
    depth with carry makes the step size irrelevant; kmax caps only defer
    candidates to the next step): their count must match the oracle's rate
    integral within the surrogate's 1e-3 rate bar plus 4 sigma; the accepted xi
    against the exact truncated CDF (KS <= 2e-3)."""
    torch, q = need_gpu()
    import workloads
    from oracle.constants import E_S
    n, b0, g, dt, steps = 1_000_000, 2000.0, 206.0, 0.05, 20
    ctx = _with_weights(q, trained, seed=21, kmax=4, flags=q.QED_FLAG_NO_RECOIL | q.QED_FLAG_SURROGATE)
    ens = workloads.uniform_b_ensembles(n, seed=21, triples=((b0, g),))[0]
    lep = q.Species(n, "f32")
    ph = q.Species(12_000_000, "f32")
    lep.load(ens["x"], ens["p"], ids=ens["id"])
    ctx.qed_init_optical_depth(lep, 0)
    ctx.qed_set_next_id(n)
    fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, b0))
    ctx.qed_get_status(check=False)
    for s_ in range(steps):
        ctx.qed_gather_push(fld, lep, -1, dt, s_)
        ctx.qed_emit_photons(lep, ph, s_)
    st, rc = ctx.qed_get_status()
    chi = g * math.sqrt(1 - 1 / g ** 2) * b0 / E_S
    row = tables.fine_row("I", chi, tables.RAD_M)
    W = RATE_UNIT * row.total / g
    mean = n * W * steps * dt
    rel = st["events"] / mean - 1
    print(f"surrogate step: events {st['events']} (oracle mean {mean:.0f}, rel {rel:+.2e}), candidates not kept "
          f"{st['thinned']} ({st['thinned'] / (st['events'] + st['thinned']):.3f}), capped {st['capped']}")
    assert abs(st["events"] - mean) < 1e-3 * mean + 4 * math.sqrt(mean), (st["events"], mean)
    assert st["envelope_exceeded"] == 0
    nph = ph.n()
    gam = torch.sqrt(ph.px[:nph].double() ** 2 + ph.py[:nph].double() ** 2 + ph.pz[:nph].double() ** 2)
    xi = np.sort((gam / g).cpu().numpy())
    P = row.F / row.total
    xc = 2.0 / g
    Pc = float(np.interp(math.log(xc) - math.log1p(-xc), row.s, P))
    Pe = (np.interp(np.log(xi) - np.log1p(-np.minimum(xi, 1 - 1e-7)), row.s, P) - Pc) / (1 - Pc)
    m = xi.size
    ks = max(np.max(np.arange(1, m + 1) / m - Pe), np.max(Pe - np.arange(m) / m))
    print(f"  photons {m}, KS {ks:.2e}, fallbacks xi {st['mlp_fallback_xi']} rate {st['mlp_fallback_rate']}")
    assert m > 9_000_000 and ks < 2e-3
    assert st["mlp_fallback_xi"] < 0.01 * st["events"]


@pytest.mark.parametrize("field_bound", [False, True])
def test_surrogate_pairs_yield_and_spectrum_1e7(trained, pair_table, field_bound):
    """Pair creation with QED_FLAG_SURROGATE (candidates at the envelope
    h_pair_env at the photon's chi, or, with a field bound F from
    qed_set_retirement, at the photon's largest rate h_pair_env(gamma_ph F / E_S)
    with no field gathered for non-candidates; kept with the pair head of the
    rate net): 1e7 photons at chi_ph = 1, one step with W dt = 1.  The pair yield
    against 1 - exp(-W dt) with W from the oracle's quadrature, within the
    surrogate's 1e-3 rate bar plus 4 sigma; the electron energy fraction against
    the exact Eq. (6) CDF (one-sample KS <= 2e-3)."""
    torch, q = need_gpu()
    n, gph, chi = 10_000_000, 1000.0, 1.0
    ctx = _with_weights(q, trained, seed=31, kmax=4, flags=q.QED_FLAG_STATIC_PHOTONS | q.QED_FLAG_SURROGATE)
    if field_bound:                     # |E| + |B| = b; the end far away: nothing is retired
        ctx.qed_set_retirement(1e3, chi * E_S / gph)
    ph, el, po = q.Species(n, "f32"), q.Species(n, "f32"), q.Species(n, "f32")
    b = chi * E_S / gph
    ph.load(np.zeros((n, 3)), np.tile([gph, 0.0, 0.0], (n, 1)), ids=np.arange(n, dtype=np.uint64))
    ctx.qed_init_optical_depth(ph, 0)
    ctx.qed_set_next_id(n)
    fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, b))
    row = tables.fine_row("pair", chi, tables.PAIR_M)
    W = RATE_UNIT * 2 * row.total / gph
    dt = 1.0 / W
    ctx.qed_get_status(check=False)
    ctx.qed_create_pairs(fld, ph, el, po, dt, 0)
    st, rc = ctx.qed_get_status()
    m = el.n()
    pr = 1 - math.exp(-W * dt)
    sig = math.sqrt(n * pr * (1 - pr))
    slack = 1e-3 * n * W * dt * math.exp(-W * dt)      # d(yield) for a 1e-3 rate error
    print(f"surrogate pairs {m} (oracle mean {n * pr:.0f}, z {(m - n * pr) / sig:+.2f}), candidates not kept "
          f"{st['thinned']}, rate fallbacks {st['mlp_fallback_rate']}")
    assert abs(m - n * pr) < slack + 4 * sig
    assert st["envelope_exceeded"] == 0 and st["pairs"] == m and st["retired"] == 0
    ge = torch.sqrt(1 + el.px[:m].double() ** 2 + el.py[:m].double() ** 2 + el.pz[:m].double() ** 2)
    xi = np.sort((ge / gph).cpu().numpy())
    P = row.F / row.total
    s_samp = np.log(xi) - np.log1p(-xi)
    Ph = np.interp(-np.abs(s_samp), row.s, P)
    Pe = np.where(s_samp <= 0, 0.5 * Ph, 1 - 0.5 * Ph)
    ks = max(np.max(np.arange(1, m + 1) / m - Pe), np.max(Pe - np.arange(m) / m))
    print(f"  KS(exact) {ks:.2e}")
    assert ks < 2e-3


def test_surrogate_step_matches_table_step_standing_wave(trained):
    """Standing wave a0 = 500, 2e5 electrons, 30 steps: the surrogate step and the
    table step give the same photon yield (within 4 sigma of their difference)
    and the same photon-energy distribution (two-sample KS)."""
    torch, q = need_gpu()
    import workloads
    n, ngrid, L = 200_000, 128, workloads.BOX_L
    res = {}
    for name, flags in (("table", 0), ("mlp", q.QED_FLAG_SURROGATE)):
        ctx = _with_weights(q, trained, seed=1, kmax=4, flags=flags)
        ens = workloads.standing_wave_electrons(n, seed=1)
        lep = q.Species(n, "f32")
        ph = q.Species(3_000_000, "f32")
        lep.load(ens["x"], ens["p"], ids=ens["id"])
        ctx.qed_init_optical_depth(lep, 0)
        ctx.qed_set_next_id(n)
        grid = torch.empty(ngrid ** 3 * 6, dtype=torch.float32, device="cuda")
        fld = q.Fields(q.QED_FIELD_GRID, grid=grid, n=ngrid, L=L)
        for s in range(30):
            ctx.qed_fill_standing_wave(grid, ngrid, L, 500.0, s * 0.01)
            ctx.qed_gather_push(fld, lep, -1, 0.01, s)
            ctx.qed_emit_photons(lep, ph, s)
        st, rc = ctx.qed_get_status()
        m = ph.n()
        gam = torch.sqrt(ph.px[:m].double() ** 2 + ph.py[:m].double() ** 2 + ph.pz[:m].double() ** 2)
        res[name] = (m, np.sort(gam.cpu().numpy()), st)
    (m1, g1, _), (m2, g2, st2) = res["table"], res["mlp"]
    assert abs(m1 - m2) < 4 * math.sqrt(m1 + m2), (m1, m2)
    allv = np.concatenate([g1, g2])
    ks = np.max(np.abs(np.searchsorted(g1, allv, side="right") / m1 - np.searchsorted(g2, allv, side="right") / m2))
    crit = 1.95 * math.sqrt((m1 + m2) / (m1 * m2))
    print(f"standing wave: photons table {m1} surrogate {m2}; KS {ks:.2e} (0.1% critical {crit:.2e}); "
          f"fallbacks {st2['mlp_fallback_xi']} / {st2['mlp_fallback_rate']}")
    assert ks < crit
