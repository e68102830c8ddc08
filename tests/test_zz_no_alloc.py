"""qed_compact_static, the compaction entry point that allocates nothing (its
scan state is a static device array of the library), against qed_compact on
the same input: every array and the count bit for bit the same, on two calls in
a row (the second one smaller, so that it reuses the array the first one left
behind), in float32 and float64, and against the oracle's compaction."""
import ctypes

import numpy as np
import pytest

from oracle import mc
from tests.gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


def _fill(q, torch, n, dtype, seed, dead_frac):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 3))
    p = rng.normal(size=(n, 3)) * 100
    tau = rng.exponential(size=n)
    ids = np.arange(1000, 1000 + n, dtype=np.uint64)
    ids[rng.uniform(size=n) < dead_frac] = np.uint64(q.DEAD_ID)
    out = []
    for _ in range(2):
        sp = q.Species(n + 17, dtype)
        sp.load(x, p, tau, ids)
        out.append(sp)
    return out, (x, p, tau, ids)


def _arrays(sp):
    n = sp.n()
    return [a[:n].cpu().numpy() for a in (sp.x, sp.y, sp.z, sp.px, sp.py, sp.pz, sp.tau, sp.id)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_compact_static_matches_compact(dtype):
    torch, q = need_gpu()
    ctx = q.Context(seed=1)
    for call, (n, frac) in enumerate(((70001, 0.3), (1025, 0.5))):   # second call smaller
        (a, b), (x, p, tau, ids) = _fill(q, torch, n, dtype, 10 + call, frac)
        print(f"compact_static call {call}: {dtype}, n = {n}, dead fraction {frac}", flush=True)
        ctx.qed_compact(a)
        ctx.qed_compact_static(b)
        st, rc = ctx.qed_get_status()
        ra, rb = _arrays(a), _arrays(b)
        assert a.n() == b.n() == int(np.count_nonzero(ids != np.uint64(q.DEAD_ID)))
        for u, v in zip(ra, rb):
            assert np.array_equal(u, v)
        want = mc.compact(ids, x[:, 0], tau)
        assert np.array_equal(rb[7].view(np.uint64), want[0])
        assert np.array_equal(rb[6], want[2])


def test_compact_static_rejects_large_species():
    torch, q = need_gpu()
    ctx = q.Context(seed=1)
    sp = q.Species(16, "f32")
    big = q.qed_species_t.from_buffer_copy(sp.c)
    big.capacity = (1 << 26) + 1              # checked on the host: nothing is launched
    rc = q.lib().qed_compact_static(ctx.h, ctypes.byref(big), None)
    assert rc == q.QED_ERR_RANGE
    assert b"2^26" in q.lib().qed_last_error(ctx.h)
