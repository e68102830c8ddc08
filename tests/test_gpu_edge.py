"""Edge cases and error paths of the C ABI on the GPU: empty species, capacity
overflow, non-finite fields, chi outside the tables, call-order and argument
errors."""
import numpy as np
import pytest

from oracle import mc
from oracle.constants import E_S
from tests.gpu_helpers import need_gpu

import workloads

pytestmark = pytest.mark.gpu


def _ctx(q, **kw):
    ctx = q.Context(**kw)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    return ctx


def test_empty_species_are_noops():
    torch, q = need_gpu()
    ctx = _ctx(q)
    for dt in ("f32", "f64"):
        el, po, ph = q.Species(1000, dt), q.Species(1000, dt), q.Species(1000, dt)
        fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, 100.0))
        ctx.qed_gather_push(fld, el, -1, 0.01, 0)
        ctx.qed_emit_photons(el, ph, 0)
        ctx.qed_create_pairs(fld, ph, el, po, 0.01, 0)
        ctx.qed_compact(ph)
        st, rc = ctx.qed_get_status()
        assert el.n() == po.n() == ph.n() == 0
        assert st["events"] == 0 and st["pairs"] == 0


def test_photon_capacity_overflow_is_reported():
    torch, q = need_gpu()
    ctx = _ctx(q, seed=3)
    n = 20000
    e = workloads.uniform_b_ensembles(n, seed=3, triples=((2000.0, 206.0),))[0]
    lep = q.Species(n, "f64")
    lep.load(e["x"], e["p"], np.zeros(n), e["id"])          # every particle emits
    cap = 1000
    ph = q.Species(cap, "f64")
    ctx.qed_set_next_id(n)
    fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, 2000.0))
    ctx.qed_gather_push(fld, lep, -1, 0.01, 0)
    ctx.qed_emit_photons(lep, ph, 0)
    st, rc = ctx.qed_get_status(check=False)
    assert rc == q.QED_ERR_CAPACITY
    assert ph.n() == cap and st["dropped"] == st["photons"] - cap > 0
    # the kept photons are the first `cap` of the ordered list
    ids = ph.to_numpy()["id"]
    np.testing.assert_array_equal(ids, np.arange(n, n + cap, dtype=np.uint64))


@pytest.mark.parametrize("surrogate", [False, True])
def test_nonfinite_fields_and_chi_range_are_counted(surrogate):
    """Non-finite fields skip the particle (optical depth unchanged) and chi above
    the table range is counted, on the table path and on the surrogate path."""
    torch, q = need_gpu()
    ctx = _ctx(q, seed=1, flags=q.QED_FLAG_SURROGATE if surrogate else 0)
    if surrogate:                                    # any weights: nothing is emitted here
        for net in (0, 1):
            rng0 = np.random.default_rng(net)
            ctx.qed_surrogate_io(net, rng0.normal(0, 0.3, q.lib().qed_surrogate_params(net)).astype(np.float32))
    n = 4096
    rng = np.random.default_rng(0)
    x = np.zeros((n, 3))
    p = np.column_stack([np.full(n, 5e3), np.zeros(n), np.zeros(n)])
    E = np.zeros((n, 3), np.float32)
    B = np.zeros((n, 3), np.float32)
    B[:, 2] = 1e4                                    # chi = gamma b / E_S ~ 121 > 1e2
    B[:100, 2] = np.nan
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    fld = q.Fields(q.QED_FIELD_PER_PARTICLE, E=[dev(E[:, c]) for c in range(3)], B=[dev(B[:, c]) for c in range(3)])
    lep = q.Species(n, "f32")
    ph = q.Species(8 * n, "f32")
    tau0 = 1e6 * np.ones(n)                          # no events
    lep.load(x, p, tau0, np.arange(n, dtype=np.uint64))
    ctx.qed_gather_push(fld, lep, -1, 1e-6, 0)
    ctx.qed_emit_photons(lep, ph, 0)
    st, rc = ctx.qed_get_status()
    assert st["nan_chi"] == 100
    assert st["chi_out_of_range"] == n - 100
    tau = lep.to_numpy()["tau"]
    assert np.all(np.isfinite(tau))
    np.testing.assert_array_equal(tau[:100], tau0[:100])   # skipped: optical depth unchanged


def test_call_order_and_argument_errors():
    torch, q = need_gpu()
    ctx = q.Context()
    lep, ph = q.Species(100, "f32"), q.Species(100, "f64")
    fld = q.Fields(q.QED_FIELD_UNIFORM)
    with pytest.raises(q.QEDError) as e:
        ctx.qed_gather_push(fld, lep, -1, 0.01, 0)          # tables missing
    assert e.value.code == q.QED_ERR_STATE
    ctx.qed_build_tables(q.QED_FORMULA_I)
    with pytest.raises(q.QEDError) as e:
        ctx.qed_emit_photons(lep, q.Species(100, "f32"), 0)   # no gather/push yet
    assert e.value.code == q.QED_ERR_STATE
    with pytest.raises(q.QEDError) as e:
        ctx.qed_gather_push(fld, lep, 0, 0.01, 0)           # charge must be +-1
    assert e.value.code == q.QED_ERR_ARG
    ctx.qed_gather_push(fld, lep, -1, 0.01, 0)
    with pytest.raises(q.QEDError) as e:
        ctx.qed_emit_photons(lep, ph, 0)                    # dtype mismatch
    assert e.value.code == q.QED_ERR_ARG
    with pytest.raises(q.QEDError) as e:
        ctx.qed_reserve(1 << 40)
    assert e.value.code == q.QED_ERR_ARG
    with pytest.raises(q.QEDError) as e:
        ctx.qed_sample(torch.zeros(4, dtype=torch.float64, device="cuda"),
                       torch.ones(4, dtype=torch.float64, device="cuda"),
                       torch.zeros(4, dtype=torch.int64, device="cuda"), q.QED_SAMPLER_MLP, 0,
                       torch.empty(4, device="cuda"), torch.empty(4, device="cuda"))
    assert e.value.code == q.QED_ERR_STATE                 # surrogate not trained


def test_converted_photons_are_not_converted_twice(pair_table):
    """Two pair passes without compaction in between: photons marked dead by the
    first pass are skipped by the second (no second pair, no move, no optical
    depth change), as in the oracle's photon step."""
    torch, q = need_gpu()
    ctx = q.Context(seed=9)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    n, b, chi = 4096, 2000.0, 30.0
    gph = chi * E_S / b
    x = np.zeros((n, 3))
    k = np.tile([gph, 0.0, 0.0], (n, 1))
    tau = np.full(n, 1e-6)                         # every photon converts in the first pass
    ids = np.arange(n, dtype=np.uint64)
    for dt in ("f64", "f32"):
        ph, el, po = q.Species(n, dt), q.Species(2 * n, dt), q.Species(2 * n, dt)
        ph.load(x, k, tau, ids)
        e0 = np.zeros((0, 3))
        el.load(e0, e0, np.zeros(0), np.zeros(0, np.uint64))
        po.load(e0, e0, np.zeros(0), np.zeros(0, np.uint64))
        ctx.qed_set_next_id(n)
        ctx.qed_get_status(check=False)
        fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, b))
        ctx.qed_create_pairs(fld, ph, el, po, 0.01, 0)
        first = ph.to_numpy()
        ctx.qed_create_pairs(fld, ph, el, po, 0.01, 1)
        second = ph.to_numpy()
        st, rc = ctx.qed_get_status()
        assert st["pairs"] == n and el.n() == n and po.n() == n
        assert np.all(first["id"] == mc.DEAD_ID)
        np.testing.assert_array_equal(second["x"], first["x"])
        np.testing.assert_array_equal(second["tau"], first["tau"])
        # the oracle's photon step leaves dead photons alone as well
        E = np.zeros((n, 3))
        B = np.tile([0.0, 0.0, b], (n, 1))
        r = mc.photon_step(first["x"], first["p"], first["tau"], first["id"], E, B, dt=0.01, step=1, seed=9,
                           sampler=mc.PairSampler(pair_table, "f64"), next_id=2 * n)
        assert r["pairs"].size == 0
        np.testing.assert_array_equal(r["x"], first["x"])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pair_capacity_overflow_is_reported(dtype):
    """More pairs than the lepton capacities: the first pairs in photon order are
    kept (ids next_id + 2r and + 1), the rest are dropped and counted, the counts
    stop at the capacities, every converted photon is dead and the status says
    QED_ERR_CAPACITY."""
    torch, q = need_gpu()
    ctx = q.Context(seed=4)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    n, cap, b, chi = 5000, 1234, 2000.0, 30.0
    gph = chi * E_S / b
    ph, el, po = q.Species(n, dtype), q.Species(cap, dtype), q.Species(cap, dtype)
    ph.load(np.zeros((n, 3)), np.tile([gph, 0.0, 0.0], (n, 1)), np.full(n, 1e-6), np.arange(n, dtype=np.uint64))
    e0 = np.zeros((0, 3))
    el.load(e0, e0, np.zeros(0), np.zeros(0, np.uint64))
    po.load(e0, e0, np.zeros(0), np.zeros(0, np.uint64))
    ctx.qed_set_next_id(n)
    fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, b))
    ctx.qed_create_pairs(fld, ph, el, po, 0.01, 0)
    st, rc = ctx.qed_get_status(check=False)
    assert rc == q.QED_ERR_CAPACITY
    assert st["pairs"] == n and st["dropped"] == 2 * (n - cap)
    assert el.n() == cap and po.n() == cap
    np.testing.assert_array_equal(el.to_numpy()["id"], n + 2 * np.arange(cap, dtype=np.uint64))
    np.testing.assert_array_equal(po.to_numpy()["id"], n + 1 + 2 * np.arange(cap, dtype=np.uint64))
    assert np.all(ph.to_numpy()["id"] == mc.DEAD_ID)
    assert ctx.qed_get_next_id() == n + 2 * n
