"""Fixed point (Section 4.1) in formats chosen to reach every case of the kernels'
32-bit operations, against the oracle bit for bit: products with a right shift of 0,
below 32, exactly 32 and above 32 bits; sums that round the second operand, the
first, or take the general 64-bit form; saturation to a narrow word, at the 32-bit
boundary and in the coarse chain only.  Each case runs the kernels' per-path code
on the host (no GPU) and, marked gpu, the path kernels with per-path records and
without (the group loop), on the same paths."""
import numpy as np
import pytest

import paper_2502_07123_amd as M
from oracle.paths import Precision, Problem, simulate
from parity import GBM, PAYS, SEED, WIDE_FMT


def _fmt(**kw):
    f = dict(WIDE_FMT)
    f.update(kw)
    return f


# name -> (formats, problem overrides, schemes)
REGIMES = {
    # X in 8 bits: X and mul2 saturate (mul2: shift 26; X + mul2 rounds mul2 by 4 bits)
    "narrow-x": (_fmt(X=(8, 6), mul2=(12, 10)), {}, ("euler", "milstein")),
    # X < 2 in a full 32-bit word: the sum X + mul2 leaves 32 bits for X >= 2
    "x-at-32-bits": (_fmt(X=(32, 30), mul2=(32, 31)), dict(sigma=0.4), ("euler", "milstein")),
    # Zs^2 of the coarse chain saturates (shift 33) while every table value fits
    "coarse-zsq": (_fmt(zsq=(28, 23), zm1=(32, 23)), {}, ("milstein",)),
    # mul1 = con2 * Z with a shift of exactly 32; sum1 rounds con1 by 5 bits
    "shift-32": (_fmt(mul1=(32, 29), sum1=(32, 29), mul3=(32, 29), sum2=(32, 29)), {}, ("euler", "milstein")),
    # mul2 = X * sum1 with no shift; sum1 in the general form (both operands shifted)
    "shift-0": (_fmt(X=(32, 14), mul1=(32, 16), sum1=(32, 16), mul2=(32, 30)), {}, ("euler",)),
    # WIDE formats: X + mul2 with mul2 shifted left (the general form at shift 0)
    "wide": (dict(WIDE_FMT), {}, ("euler", "milstein")),
}

CASES = [(name, scheme, est) for name, (_, _, schemes) in REGIMES.items() for scheme in schemes
         for est in (M.EST_APPROX, M.EST_CORR)]
LEVEL, N, OFF = 3, 4000, 123


def _setup(name, scheme):
    fmt, over, _ = REGIMES[name]
    gbm = {**GBM, **over}
    prob = M.make_problem(scheme, PAYS, **gbm)
    prec = M.make_precision("fixed", 8, False, fmt)
    oprec = Precision("fixed", 8, False, tuple((v, w, f) for v, (w, f) in fmt.items()))
    return gbm, prob, prec, oprec


def _oracle(name, scheme, est):
    gbm, prob, prec, oprec = _setup(name, scheme)
    o = simulate(Problem(scheme, **gbm), LEVEL, np.arange(OFF, OFF + N, dtype=np.uint64), oprec, est, SEED,
                 0, PAYS)
    return prob, prec, o


def _compare(name, est, sums, rec, o):
    assert np.array_equal(rec["XN_raw"], o["XN_approx"]), name
    assert np.array_equal(rec["XcN_raw"], o["XcN_approx"]), name
    assert np.array_equal(rec["saturations"], o["sat"]), name
    for i, p in enumerate(PAYS):
        assert np.array_equal(rec["Yraw"][:, i], o[p]["Y_approx_raw"]), (name, p)
        if est == M.EST_APPROX:
            assert np.array_equal(rec["Y"][:, i], o[p]["Y"]), (name, p)
            oi = [int(v) for v in o[p]["Y_approx_raw"]]
            assert sums[p]["isum1"] == sum(oi) and sums[p]["isum2"] == sum(v * v for v in oi), (name, p)
        assert sums[p]["saturations"] == int(o["sat"].sum()), (name, p)


def test_regimes_saturate_where_intended():
    """The oracle itself: the saturating cases saturate (somewhere on these paths),
    the others do not."""
    for name in REGIMES:
        scheme = REGIMES[name][2][-1]
        _, _, o = _oracle(name, scheme, M.EST_APPROX)
        sat = int(o["sat"].sum())
        if name in ("narrow-x", "x-at-32-bits", "coarse-zsq"):
            assert sat > 0, name
        else:
            assert sat == 0, name


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-{c[2]}")
def test_host_fixed_regimes_match_oracle(case):
    name, scheme, est = case
    prob, prec, o = _oracle(name, scheme, est)
    sums, rec = M.check_paths_host(prob, LEVEL, N, OFF, prec, est, SEED)
    _compare(name, est, sums, rec, o)


@pytest.mark.gpu
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-{c[2]}")
def test_gpu_fixed_regimes_match_oracle(case):
    name, scheme, est = case
    print("fixed regime", case, flush=True)
    prob, prec, o = _oracle(name, scheme, est)
    with M.Context(0, workspace_bytes=64 << 20) as ctx:
        sums, rec = ctx.level_sums(prob, LEVEL, N, OFF, prec, est, SEED, debug=True)
        _compare(name, est, sums, rec, o)
        fast = ctx.level_sums(prob, LEVEL, N, OFF, prec, est, SEED)
        assert fast == sums, name
