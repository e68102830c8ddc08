"""The paper's generator benchmark (Fig. 2 setting): 128 x 192 cells with one
electron of gamma = 206 per cell, 480 steps of Dt = 0.2/W.  The field of Fig. 2 is
not stated; a uniform B = 2000 (chi ~ 1, Fig. 1(b)) is used, without recoil so that
the rate is stationary.  The average photon generation rate of method I (with the
adaptive sub-step) and of the optical-depth method must both equal the rate of
Eq. (1) above xi_min = 2/gamma."""
import math

import numpy as np
import pytest

from oracle import tables
from oracle.constants import E_S, RATE_UNIT
from tests.gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


def test_fig2_generators_average_rate():
    torch, q = need_gpu()
    nx, ny, b0, g, steps = 128, 192, 2000.0, 206.0, 480
    n = nx * ny
    rng = np.random.default_rng(12)
    xs, ys = np.meshgrid((np.arange(nx) + 0.5), (np.arange(ny) + 0.5), indexing="ij")
    x = np.column_stack([xs.ravel(), ys.ravel(), np.zeros(n)]) * (2 * math.pi / 128)
    phi = rng.uniform(0, 2 * math.pi, n)
    pm = math.sqrt(g * g - 1)
    p = np.column_stack([pm * np.cos(phi), pm * np.sin(phi), np.zeros(n)])
    chi = g * math.sqrt(1 - 1 / g ** 2) * b0 / E_S
    row = tables.fine_row("I", chi, tables.RAD_M)
    W = RATE_UNIT * row.total / g
    xc = 2.0 / g
    kept = 1 - float(np.interp(math.log(xc) - math.log1p(-xc), row.s, row.F / row.total))
    W_cut = W * kept
    dt = 0.2 / W
    fld = q.Fields(q.QED_FIELD_UNIFORM, B=(0, 0, b0))
    rates = {}
    for name, flags in (("method I", q.QED_FLAG_METHOD_I), ("optical depth", 0)):
        ctx = q.Context(seed=12, kmax=4, flags=q.QED_FLAG_NO_RECOIL | flags)
        ctx.qed_build_tables(q.QED_FORMULA_I)
        lep = q.Species(n, "f32")
        ph = q.Species(int(n * steps * 0.2) + 100000, "f32")
        lep.load(x, p, ids=np.arange(n, dtype=np.uint64))
        ctx.qed_init_optical_depth(lep, 0)
        ctx.qed_set_next_id(n)
        for s in range(steps):
            ctx.qed_gather_push(fld, lep, -1, dt, s)
            ctx.qed_emit_photons(lep, ph, s)
        st, rc = ctx.qed_get_status()
        rates[name] = st["photons"] / (n * steps * dt)
        mean = W_cut * n * steps * dt
        print(f"{name}: {st['photons']} photons, rate {rates[name]:.5f} vs Eq. (1) {W_cut:.5f} per omega_0")
        assert abs(st["photons"] - mean) < 4 * math.sqrt(mean)
