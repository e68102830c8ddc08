"""Throughput of the QED Monte Carlo step on one MI355X.

Headline workload (the cascade configuration): 2e8 electrons in the 128^3 grid
of the circularly polarised standing wave a0 = 1000, float32 state with float64
chi and optical depth, formula II tables, dt = 0.01.  One step = refill the grid
for t = n dt, pair creation for every photon present, gather/push and emission
for electrons and for positrons (photons appended), photon compaction every 10
steps; electrons and positrons (on the table path photons too) re-sorted by
cell every 12 steps (outside the captured graphs).  The step runs as captured hipGraphs, 500 steps in all, with
the photon and positron populations growing in place.  It runs twice: with the
surrogate networks (QED_FLAG_SURROGATE: rates and photon energies from the nets,
candidate events by Poisson thinning, table fallback) and with the plain tables.

Prints one JSON line.  `value` = particle-steps per second of the surrogate
cascade over the timed steps (electrons + positrons + photons present at the
start of each step), `table` the same for the table path, inputs resident in HBM
(initial state, table build and training outside the timed region).  The timed
steps are the last K of the 500 (or of W + K if that is more); the steps before
them run untimed.  `roofline` is for the kernel that takes most of the surrogate
step (measured with HIP events around its launch on eagerly run steps spread
over the timed window, on the stream it runs on).  `oracle_gates` compares both
paths with the float64 CPU oracle run on the 1e5-electron subsample (ids
0..99999, the same initial state and random streams) for the same 500 steps:
two-sample KS of the photon and positron energy spectra, z-test of the pair
yield.  `ks_1e7` is the metric-grade spectrum gate: 1e7 photons of the
surrogate emission step at fixed chi ~ 1 against the oracle's exact CDF.
`cpu_baseline` times that same oracle run on the host's cores.
`other_configs` times the other configurations on the same GPU: the standing
wave with 1e7 electrons (table and surrogate, with its own gather/push
roofline), the uniform-B ensembles in float64, pair creation for 2e7 photons,
and the standalone sampler (table and surrogate) on 1e8 lookups.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# E_S = m_e c^2 / (hbar omega_0) at lambda_0 = 1 um: sets the photon energies of
# the pair workload from their drawn chi_ph
E_S_1UM = 510998.95 / 1.239841984
# committed counter summaries (traffic is null for a workload without one)
PROFILE = os.path.join(ROOT, "profiles", "gather_push_standing_wave_1e7.md")
PROFILE_C5 = os.path.join(ROOT, "profiles", "gather_push_cascade_2e8.md")
# sources the gather/push kernel is compiled from (the counters hold while they are unchanged)
PROFILED_SOURCES = ("step.hip", "qed_device.h", "lookup.h")

# the cascade configuration
C5_N, C5_STEPS, C5_A0, C5_DT, C5_GRID, C5_SEED = 200_000_000, 500, 1000.0, 0.01, 128, 4
C5_SUBSAMPLE = 100_000          # ids 0 .. 99999: drawn on the host, shared with the oracle
C5_SORT_EVERY, C5_COMPACT_EVERY = 12, 10
# fixed-chi emission run of the 1e7-sample spectrum gate (chi ~ 1: b0 = 2000, gamma = 206)
KS_N, KS_B0, KS_GAMMA, KS_DT, KS_STEPS = 1_000_000, 2000.0, 206.0, 0.05, 20




def measured_traffic(profile=PROFILE):
    """HBM bytes per gather/push launch from a committed rocprofv3 counter
    summary, or None if the kernel source changed since it was taken."""
    import hashlib
    try:
        text = open(profile).read()
        src = b"".join(open(os.path.join(ROOT, "paper_1608_06356_amd", "csrc", f), "rb").read()
                       for f in PROFILED_SOURCES)
    except OSError:
        return None
    vals = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith(("traffic_bytes_per_launch", "source")))
    sha = hashlib.sha256(src).hexdigest()[:16]
    if "source" not in vals or sha not in vals["source"]:
        return None
    return int(vals["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=480, help="timed steps of the cascade (the last K of its run)")
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps before them (at least 500 - K run)")
    ap.add_argument("--formula", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (and its gates)")
    ap.add_argument("--no-surrogate", action="store_true", help="table path only")
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--no-other-configs", action="store_true")
    ap.add_argument("--c5-n", type=int, default=C5_N, help="electrons of the cascade (2e8)")
    ap.add_argument("--c5-steps", type=int, default=C5_STEPS, help="steps of the cascade run (500)")
    ap.add_argument("--c5-sort-every", type=int, default=C5_SORT_EVERY, help="re-sort interval of the cascade")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 1 GiB device to device once first (scale of the HBM byte counters)")
    return ap.parse_args()


# ------------------------------------------------------------------ oracle leg
# The float64 CPU oracle on the host cores: the cascade on the 1e5-electron
# subsample for the same steps (its photon and positron spectra and pair yield
# gate the GPU runs; its wall time is the cpu_baseline), and the exact CDF of the
# fixed-chi spectrum gate.  It runs in a process started before anything touches
# the GPU, with a fork pool over contiguous id chunks.

_ORACLE = {}


def _oracle_c5_chunk(job):
    """One contiguous chunk of the subsample through the oracle's cascade step.
    Particles the chunk creates take ids from a range of their own (the GPU's ids
    for them depend on the whole population), so only the initial particles share
    their random streams with the GPU run; the comparison is statistical."""
    from oracle import mc
    import workloads
    c, lo, hi, steps = job
    ens = workloads.standing_wave_electrons(C5_SUBSAMPLE, seed=C5_SEED)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    ids = ens["id"][lo:hi]
    e0 = lambda: dict(x=np.zeros((0, 3)), p=np.zeros((0, 3)), tau=np.zeros(0), id=np.zeros(0, np.uint64))
    st = dict(el=dict(x=f32(ens["x"][lo:hi]), p=f32(ens["p"][lo:hi]), tau=mc.init_tau(ids, seed=C5_SEED), id=ids),
              po=e0(), ph=e0(), next_id=(1 << 40) * (c + 1))
    L = workloads.BOX_L
    t0 = time.perf_counter()
    psteps = 0
    for s in range(steps):
        psteps += st["el"]["id"].size + st["po"]["id"].size + st["ph"]["id"].size
        Eg, Bg = mc.standing_wave_grid(C5_GRID, L, C5_A0, s * C5_DT)
        mc.cascade_step(st, Eg=Eg, Bg=Bg, L=L, dt=C5_DT, step=s, seed=C5_SEED, rad=_ORACLE["rad"],
                        pair=_ORACLE["pair"], retire=(steps * C5_DT, c5_field_bound()))
    wall = time.perf_counter() - t0
    g = lambda p: np.sqrt(np.sum(p * p, axis=1))
    hist = st["tally"].copy()
    mc.tally_add(hist, g(st["ph"]["p"]))          # retired + followed photons
    return dict(photon_hist=hist, retired=int(st["tally"].sum()),
                positron_gamma=np.sqrt(1.0 + g(st["po"]["p"]) ** 2).astype(np.float32),
                electrons=int(st["el"]["id"].size), positrons=int(st["po"]["id"].size),
                photons=int(st["ph"]["id"].size), psteps=psteps, wall=wall)


def _oracle_driver(conn, steps, cores):
    os.nice(10)
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from oracle import mc, tables
    from oracle.constants import E_S
    t0 = time.perf_counter()
    # formula I: the same function as formula II (their identity is pinned),
    # far cheaper to build by quadrature
    _ORACLE["rad"] = mc.RadSampler(tables.build_rad_table("I"), "f64")
    _ORACLE["pair"] = mc.PairSampler(tables.build_pair_table(), "f64")
    chi = KS_GAMMA * math.sqrt(1 - 1 / KS_GAMMA ** 2) * KS_B0 / E_S
    row = tables.fine_row("I", chi, tables.RAD_M)
    t_tab = time.perf_counter() - t0
    conn.send(dict(chi=chi, s=row.s, P=row.F / row.total))      # the fixed-chi CDF, first
    bounds = np.linspace(0, C5_SUBSAMPLE, cores + 1).astype(int)
    jobs = [(c, int(bounds[c]), int(bounds[c + 1]), steps) for c in range(cores)]
    with ProcessPoolExecutor(cores, mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_oracle_c5_chunk, jobs))
    out = dict(photon_hist=sum(r["photon_hist"] for r in res), retired=sum(r["retired"] for r in res),
               positron_gamma=np.sort(np.concatenate([r["positron_gamma"] for r in res])),
               electrons=sum(r["electrons"] for r in res), positrons=sum(r["positrons"] for r in res),
               photons=sum(r["photons"] for r in res), psteps=sum(r["psteps"] for r in res),
               loop_s=max(r["wall"] for r in res), wall_s=time.perf_counter() - t0, table_s=t_tab,
               cores=cores)
    conn.send(out)
    conn.close()


def start_oracle(steps):
    """Starts the oracle leg in its own process (call before the GPU is used),
    on all host cores but two and at a lower scheduling priority, so that the
    process driving the GPU is never starved of a core."""
    import multiprocessing as mp
    cores = max(1, len(os.sched_getaffinity(0)) - 2)
    ctx = mp.get_context("fork")
    rd, wr = ctx.Pipe(duplex=False)
    p = ctx.Process(target=_oracle_driver, args=(wr, steps, cores))
    p.start()
    wr.close()
    return p, rd


def c5_field_bound():
    """|E| + |B| <= a0 (|cos x| + |sin x|) <= sqrt2 a0 in the standing wave, and the
    quadratic-spline interpolation (positive weights summing to 1) of node values
    cannot exceed the largest node value; 1e-5 covers the float32 node rounding."""
    return math.sqrt(2.0) * C5_A0 * (1.0 + 1e-5)


def ks_hist(ha, hb):
    """Two-sample KS statistic of two histograms on the same bins (the ECDFs at
    the bin edges; the true statistic differs by at most the largest bin mass)
    and its 0.1 % critical value."""
    na, nb = int(ha.sum()), int(hb.sum())
    ca, cb = np.cumsum(ha) / na, np.cumsum(hb) / nb
    return (float(np.max(np.abs(ca - cb))), 1.95 * math.sqrt((na + nb) / (na * nb)),
            float(max((ha / na).max(), (hb / nb).max())))


def ks_two_sample_np(a, b):
    """Two-sample KS statistic of sorted arrays and its 0.1 % critical value."""
    allv = np.concatenate([a, b])
    fa = np.searchsorted(a, allv, side="right") / a.size
    fb = np.searchsorted(b, allv, side="right") / b.size
    return float(np.max(np.abs(fa - fb))), 1.95 * math.sqrt((a.size + b.size) / (a.size * b.size))


def oracle_gates(gpu, orc, n_gpu):
    """GPU cascade (full population) against the oracle subsample."""
    out = {}
    ks, crit, binmass = ks_hist(gpu["photon_hist"], orc["photon_hist"])
    out["photon_ks"], out["photon_ks_crit_0.1pct"], out["photon_ks_pass"] = ks, crit, ks <= max(crit, 2e-3)
    out["photon_ks_max_bin_mass"] = binmass
    out["photons_emitted"] = [int(gpu["photon_hist"].sum()), int(orc["photon_hist"].sum())]
    if orc["positron_gamma"].size and gpu["positron_gamma"].size:
        ks, crit = ks_two_sample_np(gpu["positron_gamma"], orc["positron_gamma"])
        out["positron_ks"], out["positron_ks_crit_0.1pct"], out["positron_ks_pass"] = ks, crit, ks <= crit
    # pair yield per initial electron: the oracle's count is Poisson, the GPU's
    # rate (2e8 electrons) is known far better
    r_gpu = gpu["positrons"] / n_gpu
    mean = r_gpu * C5_SUBSAMPLE
    z = (orc["positrons"] - mean) / math.sqrt(max(orc["positrons"], 1))
    out["pairs_per_electron"] = [r_gpu, orc["positrons"] / C5_SUBSAMPLE]
    out["pair_yield_z"], out["pair_yield_pass"] = z, abs(z) <= 3.0
    out["photons_emitted_per_electron"] = [gpu["photon_hist"].sum() / n_gpu, orc["photon_hist"].sum() / C5_SUBSAMPLE]
    out["photons_followed_per_electron"] = [gpu["photons"] / n_gpu, orc["photons"] / C5_SUBSAMPLE]
    return out


# ------------------------------------------------------------ cascade (headline)
def run_cascade(q, torch, args, weights, name):
    """The cascade step (pair creation, both lepton passes with emission, photon
    compaction every C5_COMPACT_EVERY steps) on the standing wave, captured as
    hipGraphs and replayed for the whole run; leptons (on the table path photons
    too) re-sorted by cell every `--c5-sort-every` steps outside the graphs (from
    one set of species buffers into the other; graphs are captured for both
    sets).  Photons converted into
    pairs stay in place as dead slots (pair creation skips them) until the
    compaction: a stable compaction moves every photon behind the first hole.
    The 2e8 electrons: ids 0..99999 from workloads.standing_wave_electrons (the
    oracle's subsample), the rest drawn on the device with the same distributions
    (x uniform in the box, p ~ N(0, 10^2) per component; torch's generator, seed
    4); the initial storage order is by cell (untimed).  Photons that can no
    longer convert before the end of the run are retired into the tally
    (qed_set_retirement with F = sqrt2 a0).  Returns the timing, the counts, the
    photon energy histogram (tally of retired photons plus the photons still
    followed), the positron energies (a uniform sample of up to 1e7), and the
    kernel durations sampled on eager steps."""
    import workloads
    n, L, ngrid = args.c5_n, workloads.BOX_L, C5_GRID
    total = max(args.c5_steps, args.warmup + args.steps)
    timed0 = total - args.steps                  # first timed step
    flags = q.QED_FLAG_TRACK_DEAD | (q.QED_FLAG_SURROGATE if name == "surrogate" else 0)
    ctx = q.Context(seed=C5_SEED, kmax=4, flags=flags)
    ctx.qed_build_tables(args.formula)
    if name == "surrogate":
        for k in (0, 1):
            ctx.qed_surrogate_io(k, weights[k])
    # photons that can no longer convert before the end are retired into the tally
    # (qed_set_retirement; without it the run emits ~15 photons per electron);
    # capacities for the measured growth at a0 = 1000 (pairs ~0.2 per electron)
    ctx.qed_set_retirement(total * C5_DT, c5_field_bound())
    cap_e, cap_p = int(1.4 * n) + 1_000_000, int(0.4 * n) + 1_000_000
    cap_g = min(int(0.012 * n * total) + 10_000_000, (1 << 31) - 1)
    # two sets of species: a re-sort moves every sorted species from the set in
    # use to the other one (graphs are captured for both sets).  The table path
    # gathers the field for every photon and re-sorts them too; the surrogate
    # path gathers it only at candidate events, so its photons keep their
    # creation order (which follows the sorted leptons) in one buffer both sets share
    sorted_species = ("el", "po", "ph") if name == "table" else ("el", "po")
    ph_shared = None if "ph" in sorted_species else q.Species(cap_g, "f32")
    sets = [dict(el=q.Species(cap_e, "f32"), po=q.Species(cap_p, "f32"),
                 ph=ph_shared if ph_shared is not None else q.Species(cap_g, "f32")) for _ in range(2)]
    cur = [0]
    src = sets[1]["el"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(C5_SEED)
    for a in (src.x, src.y, src.z):
        a[:n].uniform_(0.0, L, generator=gen)
    for a in (src.px, src.py, src.pz):
        a[:n].normal_(0.0, 10.0, generator=gen)
    torch.arange(n, out=src.id[:n])
    sub = workloads.standing_wave_electrons(C5_SUBSAMPLE, seed=C5_SEED)
    for a, col in ((src.x, sub["x"][:, 0]), (src.y, sub["x"][:, 1]), (src.z, sub["x"][:, 2]),
                   (src.px, sub["p"][:, 0]), (src.py, sub["p"][:, 1]), (src.pz, sub["p"][:, 2])):
        a[:C5_SUBSAMPLE].copy_(torch.from_numpy(np.ascontiguousarray(col, dtype=np.float32)))
    del sub
    src.count.fill_(n)
    grid = torch.empty(ngrid ** 3 * 6, dtype=torch.float32, device="cuda")
    fld = q.Fields(q.QED_FIELD_GRID, grid=grid, n=ngrid, L=L)
    ctx.qed_reserve(cap_e)             # emitter slots for the leptons; the photons' scan state on first use
    ctx.qed_sort_by_cell(fld, src, sets[0]["el"])
    ctx.qed_init_optical_depth(sets[0]["el"], 0)
    ctx.qed_set_next_id(n)
    ctx.qed_set_step(0)
    stream = torch.cuda.current_stream()

    def one_step(compact, sid, ev=None):
        # ev: events around the parts of the step (pairs, electron push, electron
        # emission, positron push, positron emission, compaction)
        rec = (lambda k: ev[k].record(stream)) if ev is not None else (lambda k: None)
        el, po, ph = sets[sid]["el"], sets[sid]["po"], sets[sid]["ph"]
        ctx.qed_fill_standing_wave_at_step(grid, ngrid, L, C5_A0, 0.0, C5_DT)
        rec(0)
        ctx.qed_create_pairs(fld, ph, el, po, C5_DT, q.QED_STEP_DEVICE)
        rec(1)
        for sp, qq in ((el, -1), (po, 1)):
            ctx.qed_gather_push(fld, sp, qq, C5_DT, q.QED_STEP_DEVICE)
            rec(2 if sp is el else 4)
            ctx.qed_emit_photons(sp, ph, q.QED_STEP_DEVICE)
            rec(3 if sp is el else 5)
        if compact:
            ctx.qed_compact(ph)
        rec(6)
        ctx.qed_advance_step()

    def resort():
        a, b = sets[cur[0]], sets[1 - cur[0]]
        for k in sorted_species:
            ctx.qed_sort_by_cell(fld, a[k], b[k])
        cur[0] ^= 1

    one_step(False, 0)                 # step 0 eagerly, then capture
    resort()                           # allocates the sort's scratch before capture
    graphs = {}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for sid in (0, 1):
        for compact in (False, True):
            graphs[compact, sid] = torch.cuda.CUDAGraph()
            with torch.cuda.stream(side):
                with torch.cuda.graph(graphs[compact, sid], stream=side):
                    one_step(compact, sid)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    processed = torch.zeros(1, dtype=torch.int64, device="cuda")
    samples = []

    def step(k):
        # step k of the run (k >= 1); step 0 ran eagerly above
        if k % args.c5_sort_every == 0:
            resort()
        compact = (k + 1) % C5_COMPACT_EVERY == 0 or k == total - 1
        sp = sets[cur[0]]
        if k >= timed0:
            processed.add_(sp["el"].count + sp["po"].count + sp["ph"].count)
        # every 23rd timed step runs eagerly with events around its parts: 23 is
        # prime to the re-sort interval, so the samples see every phase of it
        if k >= timed0 and (k - timed0) % 23 == 3 % min(args.steps, 23):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
            cnt = [sp["ph"].count.clone(), sp["el"].count.clone(), sp["po"].count.clone()]
            one_step(compact, cur[0], ev)
            samples.append((ev, cnt))
        else:
            graphs[compact, cur[0]].replay()

    for k in range(1, timed0):
        step(k)
    torch.cuda.synchronize()
    st0, rc = ctx.qed_get_status(check=False)
    processed.zero_()
    t0 = time.perf_counter()
    ms = _timed(torch, lambda j: step(timed0 + j), args.steps)
    wall = time.perf_counter() - t0
    st, rc = ctx.qed_get_status(check=False)
    tot = int(processed.item())
    pair_ms = [a[0].elapsed_time(a[1]) for a, _ in samples]
    gp_ms = [a[1].elapsed_time(a[2]) for a, _ in samples]
    pair_n = [int(c[0].item()) for _, c in samples]
    gp_n = [int(c[1].item()) for _, c in samples]
    parts = {name: [a[i].elapsed_time(a[i + 1]) for a, _ in samples] for i, name in
             enumerate(("pairs", "electron_push", "electron_emission", "positron_push", "positron_emission",
                        "compaction"))}
    parts["positrons"] = [int(c[2].item()) for _, c in samples]
    el, po, ph = sets[cur[0]]["el"], sets[cur[0]]["po"], sets[cur[0]]["ph"]
    nph = ph.n()                                 # the last step compacted: no dead slots
    retired = ctx.qed_get_tally()
    ctx.qed_tally_species(ph)                    # + the photons still followed
    photon_hist = ctx.qed_get_tally()
    npo = po.n()
    g2 = torch.Generator(device="cuda")
    g2.manual_seed(7)
    pick = torch.randperm(npo, device="cuda", generator=g2)[:10_000_000]   # positrons are in creation order
    pg = torch.sqrt(1 + po.px[pick].double() ** 2 + po.py[pick].double() ** 2 + po.pz[pick].double() ** 2)
    positron_gamma = torch.sort(pg.float()).values.cpu().numpy()
    del pick, pg
    out = dict(value=tot / (ms * 1e-3), ms_per_step=ms / args.steps, host_wall_s=wall, electrons=el.n(),
               positrons=npo, photons=nph, pairs_timed=st["pairs"], dropped=st["dropped"] + st0["dropped"],
               scan_timeouts=st["scan_timeouts"] + st0["scan_timeouts"], envelope_exceeded=st["envelope_exceeded"],
               fallback_xi=st["mlp_fallback_xi"], fallback_rate=st["mlp_fallback_rate"], thinned=st["thinned"],
               box_fallback=st["box_fallback"],
               retired=int(retired.sum()), photon_hist=photon_hist, positron_gamma=positron_gamma, steps_run=total,
               timed_from=timed0,
               pair_pass_ms=pair_ms, pair_pass_photons=pair_n, lepton_pass_ms=gp_ms, lepton_pass_electrons=gp_n,
               sampled_step_parts_ms=parts,
               capacity_photons=cap_g)
    del graphs, sets, ph_shared, el, po, ph, grid, processed
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def run_fixed_chi_ks(q, torch, weights, row):
    """The metric-grade spectrum gate: the surrogate emission step (candidates at
    the rate envelope, rate and xi nets) on 1e6 electrons at chi ~ 1 (b0 = 2000,
    gamma = 206, no recoil) for 20 steps of 0.05, ~1e7 photons; the accepted xi
    against the oracle's exact truncated CDF (one-sample KS)."""
    import workloads
    ctx = q.Context(seed=21, kmax=4, flags=q.QED_FLAG_NO_RECOIL | q.QED_FLAG_SURROGATE)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    for k in (0, 1):
        ctx.qed_surrogate_io(k, weights[k])
    ens = workloads.uniform_b_ensembles(KS_N, seed=21, triples=((KS_B0, KS_GAMMA),))[0]
    lep, ph = q.Species(KS_N, "f32"), q.Species(12_000_000, "f32")
    lep.load(ens["x"], ens["p"], ids=ens["id"])
    ctx.qed_init_optical_depth(lep, 0)
    ctx.qed_set_next_id(KS_N)
    fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, KS_B0))
    ctx.qed_get_status(check=False)
    for s in range(KS_STEPS):
        ctx.qed_gather_push(fld, lep, -1, KS_DT, s)
        ctx.qed_emit_photons(lep, ph, s)
    st, _ = ctx.qed_get_status(check=False)
    m = ph.n()
    gam = torch.sqrt(ph.px[:m].double() ** 2 + ph.py[:m].double() ** 2 + ph.pz[:m].double() ** 2)
    xi = np.sort((gam / KS_GAMMA).cpu().numpy())
    del gam, lep, ph
    ctx.close()
    xc = 2.0 / KS_GAMMA
    Pc = float(np.interp(math.log(xc) - math.log1p(-xc), row["s"], row["P"]))
    Pe = (np.interp(np.log(xi) - np.log1p(-np.minimum(xi, 1 - 1e-7)), row["s"], row["P"]) - Pc) / (1 - Pc)
    ks = max(np.max(np.arange(1, m + 1) / m - Pe), np.max(Pe - np.arange(m) / m))
    return dict(workload=f"surrogate emission step, {KS_N} electrons at chi = {row['chi']:.4f} (b0 = {KS_B0:g}, "
                         f"gamma = {KS_GAMMA:g}), no recoil, {KS_STEPS} steps of {KS_DT}",
                samples=int(m), ks_vs_oracle_exact_cdf=float(ks), gate=2e-3, pass_=bool(ks <= 2e-3),
                fallback_xi=st["mlp_fallback_xi"], events=st["events"])


def run_workload(args, q, torch, flags, weights=None, n=10_000_000, ngrid=128, a0=500.0, steps=200, warmup=10,
                 sort_every=15):
    """The standing-wave configuration: 1e7 electrons, a0 = 500, float32 state,
    one lepton pass + emission per step, photons appended and compacted,
    electrons re-sorted by cell every `sort_every` steps.  Returns timing,
    counters and the sorted photon energies."""
    import workloads
    dev = "cuda"
    L = workloads.BOX_L
    ctx = q.Context(seed=1, kmax=4, flags=q.QED_FLAG_TRACK_DEAD | flags)
    ctx.qed_build_tables(args.formula)
    if weights is not None:
        for k in (0, 1):
            ctx.qed_surrogate_io(k, weights[k])
    ens = workloads.standing_wave_electrons(n, seed=1)
    # initial storage order by grid cell (input layout, not timed)
    cell = np.floor(ens["x"] / (L / ngrid) + 0.5).astype(np.int64) % ngrid
    order = np.argsort((cell[:, 2] * ngrid + cell[:, 1]) * ngrid + cell[:, 0], kind="stable")
    ens = {k: v[order] for k, v in ens.items()}
    lep = q.Species(n, "f32")
    lep.load(ens["x"], ens["p"], ids=ens["id"])
    lep_b = q.Species(n, "f32") if sort_every > 0 else None
    cur = [lep, lep_b]
    del ens
    ctx.qed_init_optical_depth(lep, 0)
    ctx.qed_set_next_id(n)
    ph_cap = int(n * 0.12 * (steps + warmup)) + 1_000_000
    ph = q.Species(ph_cap, "f32")
    ctx.qed_reserve(max(n, ph_cap))
    grid = torch.empty(ngrid ** 3 * 6, dtype=torch.float32, device=dev)
    fld = q.Fields(q.QED_FIELD_GRID, grid=grid, n=ngrid, L=L)
    stream = torch.cuda.current_stream()

    def step(s, ev=None):
        if sort_every > 0 and s % sort_every == 0:
            ctx.qed_sort_by_cell(fld, cur[0], cur[1])
            cur.reverse()
        lp = cur[0]
        ctx.qed_fill_standing_wave(grid, ngrid, L, a0, s * 0.01)
        if ev is not None:
            ev[0].record(stream)
        ctx.qed_gather_push(fld, lp, -1, 0.01, s)
        if ev is not None:
            ev[1].record(stream)
        ctx.qed_emit_photons(lp, ph, s)
        ctx.qed_compact(ph)

    for s in range(warmup):
        step(s)
    torch.cuda.synchronize()
    ctx.qed_get_status()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for k in range(steps):
        step(warmup + k, evs[k])
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    gp_ms = sum(a.elapsed_time(b) for a, b in evs) / steps
    st, rc = ctx.qed_get_status(check=False)
    if rc != 0:
        print(f"bench.py: status {rc}: {st}", file=sys.stderr)
        sys.exit(1)
    m = ph.n()
    gam = torch.sqrt(ph.px[:m] ** 2 + ph.py[:m] ** 2 + ph.pz[:m] ** 2)
    gam = torch.sort(gam).values
    out = dict(total_ms=total_ms, gp_ms=gp_ms, st=st, photons=m, gamma=gam)
    del ph, lep, lep_b, cur, grid
    ctx.close()
    return out


def stream_copy_gbs(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy bandwidth (read + write bytes per second, GB/s) of
    an nbytes buffer, best of `reps` copies timed with HIP events."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2 * nbytes / (best * 1e-3) / 1e9


def _timed(torch, fn, steps):
    """Milliseconds of `steps` calls of fn(k), HIP events on the current stream."""
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for k in range(steps):
        fn(k)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def run_uniform_b(q, torch, n_per=100_000, steps=100, dt=0.01):
    """Three Fig. 1 ensembles (b0, gamma) = (200, 206), (2000, 206), (2000, 2060)
    of n_per electrons each, float64 state, formula I, photons appended.  The
    ensembles share one species and each electron carries its ensemble's uniform
    field (B = b0 z, E = 0, exact in float32) as a per-particle field: one
    gather/push and one emission per step instead of three of each, which at
    this size are bound by kernel latency, not by the work."""
    import workloads
    ctx = q.Context(seed=0, kmax=4)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    ens = workloads.uniform_b_ensembles(n_per, seed=0)
    n = 3 * n_per
    lep, ph = q.Species(n, "f64"), q.Species(16 * n, "f64")
    lep.load(np.concatenate([e["x"] for e in ens]), np.concatenate([e["p"] for e in ens]), None,
             np.concatenate([e["id"] for e in ens]))
    ctx.qed_init_optical_depth(lep, 0)
    b0 = np.concatenate([np.full(e["id"].size, e["b0"], dtype=np.float32) for e in ens])
    zero = torch.zeros(n, dtype=torch.float32, device="cuda")
    Bz = torch.from_numpy(b0).cuda()
    fld = q.Fields(q.QED_FIELD_PER_PARTICLE, E=[zero, zero, zero], B=[zero, zero, Bz])
    ctx.qed_set_next_id(n)
    ctx.qed_reserve(16 * n)

    def step(s):
        ctx.qed_gather_push(fld, lep, -1, dt, s)
        ctx.qed_emit_photons(lep, ph, s)

    ms = _timed(torch, step, steps)
    st, _ = ctx.qed_get_status()
    out = dict(workload=f"uniform B, 3 x {n_per} electrons (Fig. 1 ensembles, one species, per-particle B), "
                        f"float64, formula I, {steps} steps",
               value=3 * n_per * steps / (ms * 1e-3), unit="particle-steps/s", ms_per_step=ms / steps,
               photons=st["photons"], events=st["events"])
    del lep, ph, fld
    ctx.close()
    return out


def run_pairs(q, torch, n=20_000_000, steps=100, dt=0.01):
    """2e7 static photons, chi_ph log-uniform in [1e-2, 1e2], isotropic, each in its
    own uniform E, B (|E|, |B| <= 2000); pairs appended, float32 state."""
    import workloads
    w = workloads.pair_photons(n, seed=2)
    # photon energy for the drawn chi_ph: gamma_ph = chi_ph E_S / |k x (E + k x B)| (Eq. 3, |v| = 1)
    kh, E, B = w["khat"], w["E"], w["B"]
    perp = np.linalg.norm(np.cross(kh, E + np.cross(kh, B)), axis=1)
    w["k"] = kh * (w["chi_target"] * E_S_1UM / perp)[:, None]
    del kh, E, B, perp
    ctx = q.Context(seed=2, kmax=4, flags=q.QED_FLAG_STATIC_PHOTONS)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    ph, el, po = q.Species(n, "f32"), q.Species(n, "f32"), q.Species(n, "f32")
    ph.load(w["x"], w["k"], None, w["id"])
    e0 = np.zeros((0, 3))
    el.load(e0, e0, np.zeros(0), np.zeros(0, np.uint64))
    po.load(e0, e0, np.zeros(0), np.zeros(0, np.uint64))
    ctx.qed_init_optical_depth(ph, 0)
    Et = [torch.from_numpy(np.ascontiguousarray(w["E"][:, c], dtype=np.float32)).cuda() for c in range(3)]
    Bt = [torch.from_numpy(np.ascontiguousarray(w["B"][:, c], dtype=np.float32)).cuda() for c in range(3)]
    del w
    fld = q.Fields(q.QED_FIELD_PER_PARTICLE, E=Et, B=Bt)
    ctx.qed_set_next_id(n)
    ctx.qed_reserve(n)
    ms = _timed(torch, lambda s: ctx.qed_create_pairs(fld, ph, el, po, dt, s), steps)
    st, _ = ctx.qed_get_status()
    out = dict(workload=f"pair creation, {n} static photons (chi_ph log-uniform 1e-2..1e2, |E|,|B| <= 2000), "
                        f"float32 state, {steps} steps; every photon slot is checked each step",
               value=n * steps / (ms * 1e-3), unit="photon-steps/s", ms_per_step=ms / steps, pairs=st["pairs"],
               chi_out_of_range=st["chi_out_of_range"])
    # per photon and step: read id, k, tau and the photon's E, B (52 B), write tau (8 B); the
    # (rare) pairs and the event list are left out
    ach = 60.0 * n / (ms / steps * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": "photon pass (qed_create_pairs), whole call", "achieved": ach,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                       "algorithmic_bytes_per_call": 60 * n}
    del ph, el, po, Et, Bt
    ctx.close()
    return out


def run_sampler(q, torch, weights, n=100_000_000, reps=5):
    """Standalone lookups: ln W_rad, one xi sample and ln W_pair for n particles with
    log10 chi uniform in [-3, 2] and gamma = 1000, from the tables (float32 copies)
    and from the surrogate nets."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    chi = torch.pow(10.0, torch.rand(n, generator=gen, device="cuda", dtype=torch.float64) * 5.0 - 3.0)
    gamma = torch.full((n,), 1000.0, dtype=torch.float64, device="cuda")
    ids = torch.arange(n, dtype=torch.int64, device="cuda")
    lnw, xi, lnwp = (torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3))
    ctx = q.Context(seed=3)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    out = dict(workload=f"sampler, {n} lookups of ln W_rad, xi and ln W_pair (log10 chi uniform in [-3, 2], "
                        f"gamma = 1000)", unit="samples/s")
    xs = {}
    for name, prec in (("table", q.QED_F32), ("surrogate", q.QED_SAMPLER_MLP)):
        if prec == q.QED_SAMPLER_MLP:
            if weights is None:
                continue
            for k in (0, 1):
                ctx.qed_surrogate_io(k, weights[k])
        ctx.qed_sample(chi, gamma, ids, prec, 0, lnw, xi, lnwp)
        ms = _timed(torch, lambda s: ctx.qed_sample(chi, gamma, ids, prec, 0, lnw, xi, lnwp), reps)
        out[name] = n * reps / (ms * 1e-3)
        xs[name] = torch.sort(xi[: 10_000_000].clone()).values
    st, _ = ctx.qed_get_status()
    if "surrogate" in xs:
        out["ks_xi_surrogate_vs_table_1e7"] = ks_two_sample(xs["table"], xs["surrogate"])
        out["fallback_xi"] = st["mlp_fallback_xi"]
        out["fallback_rate"] = st["mlp_fallback_rate"]
    del chi, gamma, ids, lnw, xi, lnwp, xs
    ctx.close()
    return out


def ks_two_sample(a, b):
    """Two-sample Kolmogorov-Smirnov statistic of sorted device tensors."""
    import torch
    allv = torch.cat([a, b])
    fa = torch.searchsorted(a, allv, right=True).double() / a.numel()
    fb = torch.searchsorted(b, allv, right=True).double() / b.numel()
    return float(torch.max(torch.abs(fa - fb)))


def run_other_configs(q, torch, args, weights):
    """The other configurations on the same GPU."""
    out = {}
    n, ngrid = 10_000_000, 128
    tab = run_workload(args, q, torch, 0)
    grid_bytes = ngrid ** 3 * 6 * 4
    algo = n * 64 + grid_bytes          # read x, p (24 B) and tau (8 B), write them back, + one grid read
    achieved = algo / (tab["gp_ms"] * 1e-3) / 1e9
    copy_gbs = stream_copy_gbs(torch)
    c2 = {"workload": f"standing wave a0=500, {n} electrons, {ngrid}^3 grid, formula "
                      f"{'II' if args.formula == 2 else 'I'} tables, 200 timed steps after 10, electrons re-sorted "
                      f"by cell every 15 steps",
          "unit": "particle-steps/s", "table": n * 200 / (tab["total_ms"] * 1e-3), "table_ms_per_step": tab["total_ms"] / 200,
          "roofline_gather_push": {"bound": "hbm", "kernel": "k_gather_push<float>", "achieved": achieved,
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                                   "traffic": measured_traffic(), "algorithmic_bytes_per_launch": algo,
                                   "avg_launch_ms": tab["gp_ms"], "stream_copy_GBs": copy_gbs,
                                   "frac_of_copy": achieved / copy_gbs},
          "events": tab["st"]}
    if weights is not None:
        sur = run_workload(args, q, torch, q.QED_FLAG_SURROGATE, weights)
        ks = ks_two_sample(tab["gamma"], sur["gamma"])
        c2.update(surrogate=n * 200 / (sur["total_ms"] * 1e-3), surrogate_ms_per_step=sur["total_ms"] / 200,
                  surrogate_gather_push_ms=sur["gp_ms"], ratio_surrogate_vs_table=tab["total_ms"] / sur["total_ms"],
                  ks_photon_energy_surrogate_vs_table=ks, photons=[tab["photons"], sur["photons"]],
                  fallback_xi=sur["st"]["mlp_fallback_xi"], fallback_rate=sur["st"]["mlp_fallback_rate"],
                  thinned=sur["st"]["thinned"])
        del sur
    del tab
    out["standing_wave_1e7"] = c2
    out["uniform_b_f64"] = run_uniform_b(q, torch)
    out["pairs"] = run_pairs(q, torch)
    out["sampler"] = run_sampler(q, torch, weights)
    return out


# ------------------------------------------------------------------------ main
def train_surrogate(q, torch, args):
    ctx = q.Context(seed=11)
    ctx.qed_build_tables(args.formula)
    t0 = time.perf_counter()
    ctx.qed_surrogate_train(args.train_steps, batch=4096, lr=3e-3, seed=11)
    torch.cuda.synchronize()
    w = [ctx.qed_surrogate_io(k) for k in (0, 1)]
    ctx.close()
    return w, time.perf_counter() - t0


def kernel_roofline(res, grid_bytes):
    """Roofline of the kernel taking most of the step, from the launches timed
    with HIP events on eagerly run steps of the timed window: algorithmic bytes
    per launch (pair pass: 60 B per photon slot + the grid; lepton pass: 64 B
    per electron + the grid) over the mean launch duration."""
    cand = []
    if res["pair_pass_ms"]:
        b = np.mean([60.0 * k + grid_bytes for k in res["pair_pass_photons"]])
        cand.append(("photon pass (qed_create_pairs)", b, float(np.mean(res["pair_pass_ms"]))))
    if res["lepton_pass_ms"]:
        b = np.mean([64.0 * k + grid_bytes for k in res["lepton_pass_electrons"]])
        cand.append(("electron gather/push (qed_gather_push)", b, float(np.mean(res["lepton_pass_ms"]))))
    name, b, ms = max(cand, key=lambda c: c[2])
    ach = b / (ms * 1e-3) / 1e9
    # counter-measured HBM bytes per electron launch (mean over the profiled run)
    traffic = measured_traffic(PROFILE_C5) if name.startswith("electron") else None
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": b,
            "avg_launch_ms": ms, "launches_timed": len(res["pair_pass_ms"]),
            "other_kernels": {c[0]: {"avg_launch_ms": c[2], "algorithmic_bytes_per_launch": c[1],
                                     "achieved": c[1] / (c[2] * 1e-3) / 1e9} for c in cand if c[0] != name}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    total = max(args.c5_steps, args.warmup + args.steps)
    oracle = None
    if not args.no_cpu_baseline:
        oracle = start_oracle(total)            # before anything touches the GPU
    import torch
    import paper_1608_06356_amd as q

    if args.calibrate_copy:
        # one plain device-to-device copy of known size: what the byte counters
        # read for it scales their per-dispatch values
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    weights, train_s = (None, None) if args.no_surrogate else train_surrogate(q, torch, args)
    res = {"table": run_cascade(q, torch, args, None, "table")}
    if weights is not None:
        res["surrogate"] = run_cascade(q, torch, args, weights, "surrogate")
    head_name = "surrogate" if "surrogate" in res else "table"
    head = res[head_name]
    grid_bytes = C5_GRID ** 3 * 6 * 4
    out = {
        "metric": "QED MC particle-steps/s, surrogate vs table, at KS<=2e-3 spectrum error",
        "value": head["value"], "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 state; f64 chi and optical depth; bf16 matrix cores (split hi/lo) for the nets",
        "data": "synthetic",
        "config": {"workload": f"cascade step, {head_name} path: standing wave a0={C5_A0:g}, {args.c5_n} electrons "
                               f"at start, {C5_GRID}^3 grid, formula {'II' if args.formula == 2 else 'I'} tables, "
                               f"{total} steps of dt={C5_DT} as hipGraphs (the last {args.steps} timed), photon "
                               f"compaction every {C5_COMPACT_EVERY} steps, leptons (table path: and photons) re-sorted by cell every "
                               f"{args.c5_sort_every}",
                   "global_batch": args.c5_n, "dt": C5_DT, "steps_run": total, "parallelism": "single GPU"},
        "path": head_name,
        "roofline": kernel_roofline(head, grid_bytes),
    }
    for name, r in res.items():
        out[name] = {k: v for k, v in r.items() if k not in ("photon_hist", "positron_gamma")}
    if "surrogate" in res:
        out["ratio_surrogate_vs_table"] = res["surrogate"]["value"] / res["table"]["value"]
        out["surrogate"]["train_s"] = train_s
    row = None
    if oracle is not None:
        row = oracle[1].recv()                 # the fixed-chi CDF (sent once the tables are built)
    if weights is not None and row is not None:
        out["ks_1e7"] = run_fixed_chi_ks(q, torch, weights, row)
    if not args.no_other_configs:
        out["other_configs"] = run_other_configs(q, torch, args, weights)
    if oracle is not None:
        orc = oracle[1].recv()
        oracle[0].join()
        out["oracle_gates"] = {name: oracle_gates(r, orc, args.c5_n) for name, r in res.items()}
        out["oracle_gates"]["oracle_counts"] = {k: orc[k] for k in ("electrons", "positrons", "photons", "retired")}
        out["cpu_baseline"] = {
            "value": orc["psteps"] / orc["loop_s"], "unit": "particle-steps/s", "cores": orc["cores"],
            "kind": "oracle",
            "sample": f"the same cascade on the {C5_SUBSAMPLE}-electron subsample (ids 0..{C5_SUBSAMPLE - 1}), "
                      f"{total} steps, float64 NumPy, formula I tables (the same function as formula II), "
                      f"{orc['cores']} processes over contiguous id chunks; loop {orc['loop_s']:.1f} s, tables "
                      f"{orc['table_s']:.1f} s (excluded), wall {orc['wall_s']:.1f} s"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
