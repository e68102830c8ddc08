"""Throughput of the QED Monte Carlo step on one MI355X.

Default workload (the standing-wave electron configuration): 1e7 electrons in a
128^3 grid holding the circularly polarised standing wave a0 = 500, float32
state with float64 chi and optical depth, formula II tables, dt = 0.01.  One
step = refill the grid for t = n dt, gather/push every electron, finish every
emission event, append the photons (stream-compacted) and compact the photon
arrays (a no-op on the device while no photon has been removed), plus a stable
re-sort of the electrons by grid cell every 15 steps.  Inputs are resident
in HBM before timing; table build and initialisation are outside the timed
region.

Prints one JSON line.  `value` = electron-steps per second over the timed
steps.  `roofline` is for the dominant kernel (the lepton gather/push pass),
whose duration is measured with HIP events on the stream it runs on.
`surrogate` repeats the same workload with the trained networks in place of
the table lookups (QED_FLAG_SURROGATE) and gates it on the two-sample KS
distance of the photon-energy spectra of the two runs (<= 2e-3).
`cpu_baseline` times the CPU oracle on a bounded sample of the same workload.
`other_configs` times the other configurations on the same GPU: the uniform-B
ensembles in float64 (three Fig. 1 ensembles of 1e5 electrons, 100 steps), pair
creation for 2e7 photons (100 steps), the standalone sampler (table and
surrogate) on 1e8 lookups, and the cascade step (pairs, emission, compaction)
captured in a hipGraph for 2e7 electrons at a0 = 1000 (table and surrogate).
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
PROFILE = os.path.join(ROOT, "profiles", "gather_push_standing_wave_1e7.md")
# sources the gather/push kernel is compiled from (the counters hold while they are unchanged)
PROFILED_SOURCES = ("step.hip", "qed_device.h", "lookup.h")


def measured_traffic():
    """HBM bytes per gather/push launch from the committed rocprofv3 counter
    summary, or None if the kernel source changed since it was taken."""
    import hashlib
    try:
        text = open(PROFILE).read()
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
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--a0", type=float, default=500.0)
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--formula", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate-network run of the same workload")
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy 1 GiB with torch (reference kernel for HBM counters)")
    ap.add_argument("--presort", type=int, default=1,
                    help="order the initial electrons by grid cell (outside the timed region)")
    ap.add_argument("--sort-every", type=int, default=15,
                    help="re-sort electrons by cell every K steps inside the timed loop (0: never)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the uniform-B, pair and sampler configurations")
    return ap.parse_args()


def cpu_baseline(args, budget_s):
    """The oracle (float64 NumPy) on a sample of the same workload, in a process
    pool over contiguous particle chunks on the host's cores."""
    from concurrent.futures import ProcessPoolExecutor
    cores = len(os.sched_getaffinity(0))
    n_per = 20000
    steps = 3
    t0 = time.perf_counter()
    with ProcessPoolExecutor(cores) as ex:
        futs = [ex.submit(_oracle_chunk, k, n_per, steps, args.a0, args.grid, args.dt, args.formula)
                for k in range(cores)]
        done = [f.result() for f in futs]
    wall = time.perf_counter() - t0
    # each worker also spent time building its tables; count only the step loop
    steps_done = sum(d[0] for d in done)
    loop_s = max(d[1] for d in done)
    return dict(value=steps_done / loop_s, unit="particle-steps/s", cores=cores, kind="oracle",
                sample=f"{cores} x {n_per} electrons x {steps} steps of the same workload "
                       f"(tables built once per worker, excluded); wall {wall:.1f} s")


_TAB = {}


def _oracle_chunk(k, n, steps, a0, ngrid, dt, formula):
    from oracle import mc, tables
    import workloads
    if "rad" not in _TAB:
        # the sampler needs only the rows the sample reaches; the rate uses ln h of
        # every row, so all rows are built (formula I: identical function, far cheaper)
        _TAB["rad"] = mc.RadSampler(tables.build_rad_table("I"), "q16")
    ens = workloads.standing_wave_electrons(n, seed=100 + k)
    x = ens["x"].astype(np.float32).astype(np.float64)
    p = ens["p"].astype(np.float32).astype(np.float64)
    tau = mc.init_tau(ens["id"], seed=1)
    L = workloads.BOX_L
    t0 = time.perf_counter()
    nid = 10**9
    for s in range(steps):
        Eg, Bg = mc.standing_wave_grid(ngrid, L, a0, s * dt)
        E, B = mc.gather_tsc(Eg, Bg, L, x)
        r = mc.lepton_step(x, p, tau, ens["id"], E, B, q=-1.0, dt=dt, step=s, seed=1,
                           sampler=_TAB["rad"], next_id=nid, L=L)
        x, p, tau, nid = r["x"], r["p"], r["tau"], r["next_id"]
    return n * steps, time.perf_counter() - t0


def run_workload(args, q, torch, flags, train_steps=0):
    """Times the standing-wave step; returns timing, counters and the sorted
    photon energies (for the spectrum comparison)."""
    import workloads
    dev = "cuda"
    n, ngrid, L = args.n, args.grid, workloads.BOX_L
    ctx = q.Context(seed=1, kmax=4, flags=q.QED_FLAG_TRACK_DEAD | flags)
    ctx.qed_build_tables(args.formula)
    train_s = None
    if train_steps:
        t0 = time.perf_counter()
        ctx.qed_surrogate_train(train_steps, batch=4096, lr=3e-3, seed=11)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
    ens = workloads.standing_wave_electrons(n, seed=1)
    if args.presort:
        # initial storage order by grid cell (input layout, not timed)
        cell = np.floor(ens["x"] / (L / ngrid) + 0.5).astype(np.int64) % ngrid
        order = np.argsort((cell[:, 2] * ngrid + cell[:, 1]) * ngrid + cell[:, 0], kind="stable")
        ens = {k: v[order] for k, v in ens.items()}
    lep = q.Species(n, "f32")
    lep.load(ens["x"], ens["p"], ids=ens["id"])
    lep_b = q.Species(n, "f32") if args.sort_every > 0 else None
    cur = [lep, lep_b]
    del ens
    ctx.qed_init_optical_depth(lep, 0)
    ctx.qed_set_next_id(n)
    ph_cap = int(n * 0.12 * (args.steps + args.warmup)) + 1_000_000
    ph = q.Species(ph_cap, "f32")
    ctx.qed_reserve(max(n, ph_cap))
    grid = torch.empty(ngrid ** 3 * 6, dtype=torch.float32, device=dev)
    fld = q.Fields(q.QED_FIELD_GRID, grid=grid, n=ngrid, L=L)
    stream = torch.cuda.current_stream()

    def step(s, ev=None):
        if args.sort_every > 0 and s % args.sort_every == 0:
            ctx.qed_sort_by_cell(fld, cur[0], cur[1])
            cur.reverse()
        lp = cur[0]
        ctx.qed_fill_standing_wave(grid, ngrid, L, args.a0, s * args.dt)
        if ev is not None:
            ev[0].record(stream)
        ctx.qed_gather_push(fld, lp, -1, args.dt, s)
        if ev is not None:
            ev[1].record(stream)
        ctx.qed_emit_photons(lp, ph, s)
        ctx.qed_compact(ph)

    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    ctx.qed_get_status()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for k in range(args.steps):
        step(args.warmup + k, evs[k])
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    gp_ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
    st, rc = ctx.qed_get_status(check=False)
    if rc != 0:
        print(f"bench.py: status {rc}: {st}", file=sys.stderr)
        sys.exit(1)
    m = ph.n()
    gam = torch.sqrt(ph.px[:m] ** 2 + ph.py[:m] ** 2 + ph.pz[:m] ** 2)
    gam = torch.sort(gam).values
    weights = [ctx.qed_surrogate_io(k) for k in (0, 1)] if train_steps else None
    out = dict(total_ms=total_ms, gp_ms=gp_ms, st=st, photons=m, gamma=gam, train_s=train_s, weights=weights)
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


def run_cascade(q, torch, weights, n=200_000_000, steps=100, dt=0.01, a0=1000.0, ngrid=128, sort_every=20,
                compact_every=10):
    """The cascade step (pair creation, both lepton passes with emission, photon
    compaction) on the standing wave at a0 = 1000, captured once as a hipGraph
    and replayed; electrons re-sorted by cell every `sort_every` steps outside the
    graph (sorted into a second buffer and copied back, so that the graph's
    pointers stay valid).  Table path, and surrogate path when weights are given.
    The 2e8 electrons are drawn on the device (torch's generator, seed 4) with
    the distributions of workloads.standing_wave_electrons: x uniform in the box,
    p ~ N(0, 10^2) per component, ids 0..n-1; the initial storage order is by
    cell (qed_sort_by_cell, untimed).  Photons converted into pairs stay in place
    as dead slots (pair creation skips them) until the compaction, which runs
    every `compact_every` steps: a stable compaction moves every photon behind
    the first hole, so removing a few hundred converted photons each step would
    move the whole population each step.  The photons are re-sorted by cell as
    well, right after a compaction, into a second photon buffer (graphs are
    captured for both buffers), which keeps their field gathers in pair creation
    local."""
    import workloads
    L = workloads.BOX_L
    res = {}
    for name in ("table", "surrogate"):
        if name == "surrogate" and weights is None:
            continue
        flags = q.QED_FLAG_TRACK_DEAD | (q.QED_FLAG_SURROGATE if name == "surrogate" else 0)
        ctx = q.Context(seed=4, kmax=4, flags=flags)
        ctx.qed_build_tables(q.QED_FORMULA_II)
        if name == "surrogate":
            for k in (0, 1):
                ctx.qed_surrogate_io(k, weights[k])
        cap_e, cap_p, cap_g = int(1.25 * n), n // 4, 3 * n
        el, el_b = q.Species(cap_e, "f32"), q.Species(cap_e, "f32")
        po = q.Species(cap_p, "f32")
        phs = [q.Species(cap_g, "f32"), q.Species(cap_g, "f32")]
        cur = [0]                       # photon buffer in use
        gen = torch.Generator(device="cuda")
        gen.manual_seed(4)
        for a in (el_b.x, el_b.y, el_b.z):
            a[:n].uniform_(0.0, L, generator=gen)
        for a in (el_b.px, el_b.py, el_b.pz):
            a[:n].normal_(0.0, 10.0, generator=gen)
        torch.arange(n, out=el_b.id[:n])
        el_b.count.fill_(n)
        grid = torch.empty(ngrid ** 3 * 6, dtype=torch.float32, device="cuda")
        fld = q.Fields(q.QED_FIELD_GRID, grid=grid, n=ngrid, L=L)
        ctx.qed_reserve(cap_e)          # scan state and emitter slots; photons add scan state on first use
        ctx.qed_sort_by_cell(fld, el_b, el)
        ctx.qed_init_optical_depth(el, 0)
        ctx.qed_set_next_id(n)
        ctx.qed_set_step(0)

        def one_step(compact=True, pb=0):
            ph = phs[pb]
            ctx.qed_fill_standing_wave_at_step(grid, ngrid, L, a0, 0.0, dt)
            ctx.qed_create_pairs(fld, ph, el, po, dt, q.QED_STEP_DEVICE)
            for sp, qq in ((el, -1), (po, 1)):
                ctx.qed_gather_push(fld, sp, qq, dt, q.QED_STEP_DEVICE)
                ctx.qed_emit_photons(sp, ph, q.QED_STEP_DEVICE)
            if compact:
                ctx.qed_compact(ph)
            ctx.qed_advance_step()

        def resort():
            ctx.qed_sort_by_cell(fld, el, el_b)
            for a, b in ((el.x, el_b.x), (el.y, el_b.y), (el.z, el_b.z), (el.px, el_b.px), (el.py, el_b.py),
                         (el.pz, el_b.pz), (el.tau, el_b.tau), (el.id, el_b.id), (el.count, el_b.count)):
                a.copy_(b)
            ctx.qed_sort_by_cell(fld, phs[cur[0]], phs[1 - cur[0]])
            cur[0] ^= 1

        one_step()                      # first step eagerly (state advances), then capture
        resort()                        # allocates the sort's scratch outside the timed loop
        graphs = {}
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        for pb in (0, 1):               # each photon buffer, the step without and with compaction
            for compact in (False, True):
                graphs[compact, pb] = torch.cuda.CUDAGraph()
                with torch.cuda.stream(side):
                    with torch.cuda.graph(graphs[compact, pb], stream=side):
                        one_step(compact, pb)
        torch.cuda.current_stream().wait_stream(side)
        for g in graphs.values():       # the first replays upload the graphs; not timed
            g.replay()
        torch.cuda.synchronize()
        ctx.qed_get_status()
        processed = torch.zeros(1, dtype=torch.int64, device="cuda")

        def step(k):
            if k % sort_every == 0:     # right after a compaction (sort_every is a multiple of it)
                resort()
            processed.add_(el.count + po.count + phs[cur[0]].count)
            graphs[(k + 1) % compact_every == 0, cur[0]].replay()

        for k in range(1, sort_every + 1):   # untimed warm-up through one re-sort
            step(k)
        torch.cuda.synchronize()
        ctx.qed_get_status(check=False)
        processed.zero_()
        ms = _timed(torch, lambda k: step(k + 1), steps)   # same schedule as the warm-up
        st, rc = ctx.qed_get_status(check=False)
        tot = int(processed.item())
        res[name] = dict(value=tot / (ms * 1e-3), ms_per_step=ms / steps, electrons=el.n(), positrons=po.n(),
                         photons=phs[cur[0]].n(), pairs=st["pairs"], dropped=st["dropped"],
                         scan_timeouts=st["scan_timeouts"])
        del graphs, el, el_b, po, phs, grid
        ctx.close()
        torch.cuda.empty_cache()
    res["workload"] = (f"cascade step on the standing wave a0={a0:g}, {n} electrons at start, {ngrid}^3 grid, "
                       f"formula II, pairs + both lepton passes (+ photon compaction every {compact_every} steps) "
                       f"captured as hipGraphs, {steps} replays, electrons and photons re-sorted every {sort_every} steps")
    res["unit"] = "particle-steps/s (electrons + positrons + photons present at the start of each step)"
    if "surrogate" in res:
        res["ratio_surrogate_vs_table"] = res["surrogate"]["value"] / res["table"]["value"]
    return res


def ks_two_sample(a, b):
    """Two-sample Kolmogorov-Smirnov statistic of sorted device tensors."""
    import torch
    allv = torch.cat([a, b])
    fa = torch.searchsorted(a, allv, right=True).double() / a.numel()
    fb = torch.searchsorted(b, allv, right=True).double() / b.numel()
    return float(torch.max(torch.abs(fa - fb)))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1608_06356_amd as q

    n, ngrid = args.n, args.grid
    tab = run_workload(args, q, torch, 0)
    total_ms, gp_ms, st = tab["total_ms"], tab["gp_ms"], tab["st"]
    ms_per_step = total_ms / args.steps
    value = n * args.steps / (total_ms * 1e-3)
    # algorithmic bytes of one gather/push launch: read x,y,z,px,py,pz (24 B) and
    # tau (8 B), write them back (32 B) per electron, plus one read of the grid
    grid_bytes = ngrid ** 3 * 6 * 4
    per_particle = 64
    algo = n * per_particle + grid_bytes
    achieved = algo / (gp_ms * 1e-3) / 1e9
    copy_gbs = stream_copy_gbs(torch)
    out = {
        "metric": "QED MC particle-steps/s, surrogate vs table, at KS<=2e-3 spectrum error",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (chi, tau f64)", "data": "synthetic",
        "config": {"workload": f"standing wave a0={args.a0:g}, {n} electrons, {ngrid}^3 grid, "
                               f"formula {'II' if args.formula == 2 else 'I'} tables, table sampler, "
                               f"cell sort every {args.sort_every} steps",
                   "global_batch": n, "dt": args.dt, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "k_gather_push<float>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(), "algorithmic_bytes_per_launch": algo,
                     "avg_launch_ms": gp_ms, "stream_copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "events": st,
        "photons": tab["photons"],
    }
    if not args.no_surrogate:
        sur = run_workload(args, q, torch, q.QED_FLAG_SURROGATE, train_steps=args.train_steps)
        ks = ks_two_sample(tab["gamma"], sur["gamma"])
        out["surrogate"] = {
            "value": n * args.steps / (sur["total_ms"] * 1e-3), "ms_per_step": sur["total_ms"] / args.steps,
            "gather_push_ms": sur["gp_ms"], "photons": sur["photons"],
            "ks_photon_energy_vs_table": ks, "ks_gate": 2e-3, "ks_pass": ks <= 2e-3,
            "fallback_xi": sur["st"]["mlp_fallback_xi"], "fallback_rate": sur["st"]["mlp_fallback_rate"],
            "events": sur["st"]["events"], "train_s": sur["train_s"],
            "ratio_vs_table": (sur["total_ms"] and total_ms / sur["total_ms"]),
        }
        weights = sur["weights"]
        del sur
    else:
        weights = None
    del tab
    if not args.no_other_configs:
        out["other_configs"] = {"uniform_b_f64": run_uniform_b(q, torch), "pairs": run_pairs(q, torch),
                                "sampler": run_sampler(q, torch, weights),
                                "cascade_graph": run_cascade(q, torch, weights)}
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
