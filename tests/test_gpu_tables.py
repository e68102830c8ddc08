"""GPU table builder (qed_build_tables) against the oracle's quadrature."""
import math

import numpy as np
import pytest

from oracle import tables
from tests.gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu_tables():
    torch, q = need_gpu()
    ctx = q.Context(seed=0)
    ctx.qed_build_tables(q.QED_FORMULA_I)
    out = {w: ctx.qed_get_table(w) for w in range(8)}
    ctx.qed_build_tables(q.QED_FORMULA_II)
    out["II_lnh"] = ctx.qed_get_table(0)
    out["II_S"] = ctx.qed_get_table(1)
    ctx.close()
    return out


def test_rad_rates_and_quantiles_formula_I(gpu_tables, rad_table_I):
    np.testing.assert_allclose(gpu_tables[0], rad_table_I.ln_h, rtol=0, atol=1e-11)
    d = np.abs(gpu_tables[1] - rad_table_I.s)
    assert d.max() < 1e-8, d.max()


def test_rad_q16_codes(gpu_tables, rad_table_I):
    s0, sc, q = tables.quantize_rows(rad_table_I.s)
    diff = np.abs(gpu_tables[4].astype(np.int64) - q.astype(np.int64))
    assert diff.max() <= 1 and np.count_nonzero(diff) <= 4
    np.testing.assert_array_equal(gpu_tables[5][:, 0], s0)
    np.testing.assert_allclose(gpu_tables[5][:, 1], sc, rtol=1e-6)


def test_pair_tables(gpu_tables, pair_table):
    np.testing.assert_allclose(gpu_tables[2], pair_table.L, rtol=0, atol=1e-10)
    assert np.abs(gpu_tables[3] - pair_table.s).max() < 1e-8
    s0, sc, q = tables.quantize_rows(pair_table.s)
    diff = np.abs(gpu_tables[6].astype(np.int64) - q.astype(np.int64))
    assert diff.max() <= 1 and np.count_nonzero(diff) <= 4


def test_formula_II_table(gpu_tables, rad_table_I):
    """GPU formula II (Eq. 4) rows against the oracle's formula II quadrature on
    sampled rows, and against formula I everywhere (the same function)."""
    rows = [0, 170]
    ref = tables.build_rad_table("II", rows=rows)
    for i in rows:
        assert abs(gpu_tables["II_lnh"][i] - ref.ln_h[i]) < 1e-11
        assert np.abs(gpu_tables["II_S"][i] - ref.s[i]).max() < 1e-8
    assert np.abs(gpu_tables["II_lnh"] - rad_table_I.ln_h).max() < 1e-10
    assert np.abs(gpu_tables["II_S"] - rad_table_I.s).max() < 1e-7


def test_classical_table_vs_oracle():
    """QED_FORMULA_CLASSICAL (Eq. 5): GPU rows against the oracle's quadrature."""
    torch, q = need_gpu()
    ctx = q.Context()
    ctx.qed_build_tables(q.QED_FORMULA_CLASSICAL)
    lnh, S = ctx.qed_get_table(0), ctx.qed_get_table(1)
    ref = tables.build_rad_table("classical", rows=[0, 90, 200, 255])
    for i in (0, 90, 200, 255):
        assert abs(lnh[i] - ref.ln_h[i]) < 1e-11
        assert np.abs(S[i] - ref.s[i]).max() < 1e-8


def test_wide_range_tables_vs_oracle():
    """qed_build_tables_range up to chi = 1e5 (the Fig. 5 cascade): sampled rows
    of every table against the oracle's quadrature on the same nodes; the
    surrogate entry points refuse tables of a non-default range."""
    torch, q = need_gpu()
    ctx = q.Context()
    ctx.qed_build_tables_range(q.QED_FORMULA_I, 1e5, 1e5)
    lnh, S, L, PS = (ctx.qed_get_table(w) for w in range(4))
    rows = [0, 128, 250, 255]
    ref = tables.build_rad_table("I", rows=rows, chi_max=1e5)
    pref = tables.build_pair_table(rate_rows=[0, 300, 511], cdf_rows=[0, 128, 255], chi_max=1e5)
    for i in rows:
        assert abs(lnh[i] - ref.ln_h[i]) < 1e-11
        assert np.abs(S[i] - ref.s[i]).max() < 1e-8
    for i in (0, 300, 511):
        assert abs(L[i] - pref.L[i]) < 1e-10
    for i in (0, 128, 255):
        assert np.abs(PS[i] - pref.s[i]).max() < 1e-8
    with pytest.raises(q.QEDError):
        ctx.qed_surrogate_train(steps=1, batch=64, lr=1e-3, seed=0, nets=3)
    with pytest.raises(q.QEDError):
        ctx.qed_build_tables_range(q.QED_FORMULA_I, 1e7, 1e5)
    ctx.close()
