"""One step captured in a HIP graph (through torch.cuda.graph) and replayed:
with the step index in device memory every replay reproduces the eager step
bit for bit, with eager work and synchronisation between replays."""
import numpy as np
import pytest

from tests.gpu_helpers import need_gpu

import workloads

pytestmark = pytest.mark.gpu


def _setup(q, torch, n, ngrid, flags):
    ctx = q.Context(seed=1, kmax=4, flags=flags)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    ens = workloads.standing_wave_electrons(n, seed=1)
    lep = q.Species(n, "f32")
    ph = q.Species(40 * n, "f32")
    lep.load(ens["x"], ens["p"], ids=ens["id"])
    ctx.qed_init_optical_depth(lep, 0)
    ctx.qed_set_next_id(n)
    ctx.qed_reserve(40 * n)
    grid = torch.empty(ngrid ** 3 * 6, dtype=torch.float32, device="cuda")
    fld = q.Fields(q.QED_FIELD_GRID, grid=grid, n=ngrid, L=workloads.BOX_L)
    return ctx, lep, ph, grid, fld


def test_graph_replay_matches_eager():
    torch, q = need_gpu()
    n, ngrid, a0, dt, steps = 100_000, 64, 500.0, 0.01, 8
    L = workloads.BOX_L
    flags = q.QED_FLAG_TRACK_DEAD
    # eager reference, explicit step indices
    ctx, lep, ph, grid, fld = _setup(q, torch, n, ngrid, flags)
    ref = []
    for s in range(steps):
        ctx.qed_fill_standing_wave(grid, ngrid, L, a0, s * dt)
        ctx.qed_gather_push(fld, lep, -1, dt, s)
        ctx.qed_emit_photons(lep, ph, s)
        ctx.qed_compact(ph)
        torch.cuda.synchronize()
        ref.append((lep.to_numpy(), ph.to_numpy()))
    ctx.close()
    # graph: step index on the device
    ctx, lep, ph, grid, fld = _setup(q, torch, n, ngrid, flags)
    ctx.qed_set_step(0)

    def one_step():
        ctx.qed_fill_standing_wave_at_step(grid, ngrid, L, a0, 0.0, dt)
        ctx.qed_gather_push(fld, lep, -1, dt, q.QED_STEP_DEVICE)
        ctx.qed_emit_photons(lep, ph, q.QED_STEP_DEVICE)
        ctx.qed_compact(ph)
        ctx.qed_advance_step()

    # warm-up outside capture on a scratch copy is not possible (state changes),
    # so the first step runs eagerly and is checked like the replays
    one_step()
    torch.cuda.synchronize()
    g0, p0 = lep.to_numpy(), ph.to_numpy()
    np.testing.assert_array_equal(g0["x"], ref[0][0]["x"])
    np.testing.assert_array_equal(p0["id"], ref[0][1]["id"])
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            one_step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    # capture does not execute: state is still after step 0
    for k in range(1, steps):
        graph.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()      # eager work between replays
        g, p = lep.to_numpy(), ph.to_numpy()
        e, ep = ref[k]
        np.testing.assert_array_equal(g["x"], e["x"])
        np.testing.assert_array_equal(g["p"], e["p"])
        np.testing.assert_array_equal(g["tau"], e["tau"])
        np.testing.assert_array_equal(p["id"], ep["id"])
        np.testing.assert_array_equal(p["p"], ep["p"])
    st, rc = ctx.qed_get_status()
    assert st["scan_timeouts"] == 0


def test_graph_cascade_surrogate_matches_eager():
    """The full cascade step with the surrogate (pairs, both lepton passes with
    emission, photon compaction; the shape of the standing-wave cascade
    workload at a0 = 1000) captured once and replayed: every replay equals the
    eager step bit for bit for all three species."""
    torch, q = need_gpu()
    n, ngrid, a0, dt, steps = 40_000, 64, 1000.0, 0.01, 10
    L = workloads.BOX_L
    flags = q.QED_FLAG_TRACK_DEAD | q.QED_FLAG_SURROGATE
    ens = workloads.standing_wave_electrons(n, seed=4, p_spread=1000.0)
    trainer = q.Context(seed=4)
    trainer.qed_build_tables(q.QED_FORMULA_II)
    trainer.qed_surrogate_train(3000, batch=4096, lr=3e-3, seed=5)
    weights = [trainer.qed_surrogate_io(k) for k in (0, 1)]
    trainer.close()

    def setup():
        ctx = q.Context(seed=4, kmax=4, flags=flags)
        ctx.qed_build_tables(q.QED_FORMULA_II)
        for k in (0, 1):
            ctx.qed_surrogate_io(k, weights[k])
        el, po, ph = q.Species(8 * n, "f32"), q.Species(8 * n, "f32"), q.Species(40 * n, "f32")
        el.load(ens["x"], ens["p"], ids=ens["id"])
        e0 = np.zeros((0, 3))
        po.load(e0, e0, np.zeros(0), np.zeros(0, np.uint64))
        ph.load(e0, e0, np.zeros(0), np.zeros(0, np.uint64))
        ctx.qed_init_optical_depth(el, 0)
        ctx.qed_set_next_id(n)
        ctx.qed_reserve(40 * n)
        grid = torch.empty(ngrid ** 3 * 6, dtype=torch.float32, device="cuda")
        fld = q.Fields(q.QED_FIELD_GRID, grid=grid, n=ngrid, L=L)
        return ctx, el, po, ph, grid, fld

    def step(ctx, el, po, ph, grid, fld, s):
        if s is None:
            ctx.qed_fill_standing_wave_at_step(grid, ngrid, L, a0, 0.0, dt)
            s = q.QED_STEP_DEVICE
        else:
            ctx.qed_fill_standing_wave(grid, ngrid, L, a0, s * dt)
        ctx.qed_create_pairs(fld, ph, el, po, dt, s)
        for sp, qq in ((el, -1), (po, 1)):
            ctx.qed_gather_push(fld, sp, qq, dt, s)
            ctx.qed_emit_photons(sp, ph, s)
        ctx.qed_compact(ph)

    ctx, el, po, ph, grid, fld = setup()
    ref = []
    for s in range(steps):
        step(ctx, el, po, ph, grid, fld, s)
        torch.cuda.synchronize()
        ref.append([sp.to_numpy() for sp in (el, po, ph)])
    st_ref, _ = ctx.qed_get_status()
    ctx.close()
    assert ref[-1][1]["id"].size > 0, "no pairs: the replay would not exercise pair creation"

    ctx, el, po, ph, grid, fld = setup()
    ctx.qed_set_step(0)

    def one_step():
        step(ctx, el, po, ph, grid, fld, None)
        ctx.qed_advance_step()

    one_step()
    torch.cuda.synchronize()
    for a, b in zip([sp.to_numpy() for sp in (el, po, ph)], ref[0]):
        np.testing.assert_array_equal(a["id"], b["id"])
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            one_step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for k in range(1, steps):
        graph.replay()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()      # eager work between replays
        for a, b in zip([sp.to_numpy() for sp in (el, po, ph)], ref[k]):
            np.testing.assert_array_equal(a["id"], b["id"])
            np.testing.assert_array_equal(a["x"], b["x"])
            np.testing.assert_array_equal(a["p"], b["p"])
            np.testing.assert_array_equal(a["tau"], b["tau"])
    st, _ = ctx.qed_get_status()
    print(f"cascade graph: electrons {el.n()} positrons {po.n()} photons {ph.n()}; "
          f"surrogate fallbacks xi {st['mlp_fallback_xi']} rate {st['mlp_fallback_rate']}")
    assert st["scan_timeouts"] == 0 and st["dropped"] == 0
    assert st["pairs"] == st_ref["pairs"] and st["photons"] == st_ref["photons"]
