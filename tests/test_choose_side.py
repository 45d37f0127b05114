"""Section 6's per-level choice of the low-precision side with the GPU's
instruction-class cost (mlmc_choose_precision, host) against the oracle's restatement
(oracle.errmodel.choose_side) on error models from the oracle's reverse sweep, and
the cost model's own pins (monotone in the work it counts)."""
import numpy as np
import pytest

import paper_2502_07123_amd as M
from oracle import errmodel as em
from oracle.paths import Problem

GBM = dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0)
ARITH = {"fp32": 1, "fp16": 2, "fixed": 3}


def _lib_model(m, scheme, level, q):
    return {"level": level, "scheme": 0 if scheme == "euler" else 1, "table_bits": q, "n_paths": m.n_paths,
            "used": [int(u) for u in m.used], "e": [int(x) for x in m.e], "S": list(m.S), "R": list(m.R),
            "V_level": m.V_level, "mse": m.mse}


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
@pytest.mark.parametrize("level", [0, 2, 5, 8])
@pytest.mark.parametrize("with_fixed", [False, True])
def test_choice_equals_oracle(scheme, level, with_fixed):
    m = em.sensitivities(Problem(scheme, **GBM), level, 4000, 8, 1234)
    fixed_d = None
    fmt = None
    if with_fixed:
        fixed_d = np.where(m.used, 20, 0)
        fmt = {v: (int(fixed_d[i]) + 1, int(fixed_d[i] - m.e[i])) for i, v in enumerate(em.VARS) if m.used[i]}
        fixed_d = np.array([fmt[v][0] - 1 if v in fmt else 0 for v in em.VARS], dtype=np.float64)
    want = em.choose_side(m, scheme, level, fixed_d=fixed_d)
    prec, info = M.choose_precision(_lib_model(m, scheme, level, 8), fixed_fmt=fmt)
    assert (prec.arith, prec.table_bits, bool(prec.packed)) == (ARITH[want[0]], want[1], want[2])
    assert abs(info["objective"] - want[3]) <= 1e-10 * want[3]
    assert abs(info["objective_fp32_q8"] - want[4]) <= 1e-10 * want[4]


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
@pytest.mark.parametrize("level", [0, 1, 4, 9])
def test_side_costs_equal_oracle(scheme, level):
    for arith, q, packed in em.SIDE_CANDIDATES:
        a, c = M.side_costs(arith, q, packed, scheme, level)
        assert abs(a - em.side_cost(arith, q, packed, scheme, level, 1)) <= 1e-12 * a
        assert abs(c - em.side_cost(arith, q, packed, scheme, level, 2)) <= 1e-12 * c


def test_cost_model_orders_the_work():
    # packing more indices per word is cheaper; fixed point dearer than FP32; the
    # correction (FP64 inverse normal) dearer than the approximate estimator; Milstein
    # dearer than Euler above level 0 (the table holds the whole fine multiplier, so
    # only the coarse step differs); FP16's 4-byte table reads cheaper than 8-byte ones
    for level in (0, 3):
        a8, c8 = M.side_costs("fp32", 8, True, "milstein", level)
        a4, _ = M.side_costs("fp32", 4, True, "milstein", level)
        a8u, _ = M.side_costs("fp32", 8, False, "milstein", level)
        af, cf = M.side_costs("fixed", 8, False, "milstein", level)
        ae, _ = M.side_costs("fp32", 8, True, "euler", level)
        ah, _ = M.side_costs("fp16", 8, True, "milstein", level)
        assert a4 < a8 < a8u < af and c8 < cf and a8 < c8 and ah < a8
        assert (ae < a8) if level >= 1 else (ae == a8)


def test_choice_follows_the_variance_split():
    # a level whose correction variance is negligible takes the cheapest side; one
    # whose table term dominates takes a finer table
    m = em.sensitivities(Problem("milstein", **GBM), 3, 4000, 8, 1234)
    cheap = em.Model(S=m.S * 0.0, R=m.R, e=m.e, used=m.used, V_level=m.V_level, mse=m.mse, n_paths=m.n_paths)
    a = em.choose_side(cheap, "milstein", 3)
    assert (a[0], a[1], a[2]) == ("fp16", 8, True)       # q = 7 packs four fields too
    heavy = em.Model(S=m.S * 1e6, R=m.R, e=m.e, used=m.used, V_level=m.V_level, mse=m.mse, n_paths=m.n_paths)
    b = em.choose_side(heavy, "milstein", 3)
    assert b[1] >= 10
