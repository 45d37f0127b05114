"""GPU parity: the HIP path through the C ABI against the oracle, element by element
(bars in tests/parity.py).  Per-path records come from the same kernel (a debug
buffer flag).  Sizes span several tiles with a ragged tail at every level."""
import numpy as np
import pytest

import paper_2502_07123_amd as M
from parity import (CASES, GBM, METHOD_CASES, PAYS, SEED, WIDE_FMT, case_q, check_records, library_precision,
                    oracle_run)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0, workspace_bytes=768 << 20)
    yield c
    c.close()


def _n_for(level):
    # several tiles (one block's worth of groups at least per tile) and a ragged tail
    # at every level
    return int(max(3 * (1 << 16) // max(1 << level, 16) + 77, 2000))


@pytest.mark.parametrize("level", [0, 1, 4, 7])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("payoffs", [("euro",), PAYS], ids=["euro", "all"])
def test_paths_and_sums(ctx, case, level, payoffs):
    scheme, est, arith, packed = case
    n, off = _n_for(level), 1000 + level
    prob = M.make_problem(scheme, payoffs, **GBM)
    prec = library_precision(M, case)
    sums, rec = ctx.level_sums(prob, level, n, off, prec, est, SEED, debug=True)
    o = oracle_run(case, level, np.arange(off, off + n, dtype=np.uint64), payoffs)
    check_records(case, level, n, off, payoffs, sums, rec, o)


EXACT_CASES = [c for c in CASES if c[1] != M.EST_APPROX]


@pytest.mark.parametrize("level", [2, 5])
@pytest.mark.parametrize("case", EXACT_CASES, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("ahead", [True, False], ids=["normals-ahead", "normals-inline"])
def test_exact_normals_ahead_and_inline(ctx, case, level, ahead):
    """Exact-normal works with few paths get their normals from the pre-pass kernel;
    with the pre-pass disabled the path kernel computes them: both match the oracle."""
    scheme, est, arith, packed = case
    saved = ctx.get_tuning()
    ctx.set_tuning(zb_max_paths=(1 << 15) if ahead else 0)
    try:
        n, off = 3001, 77
        prob = M.make_problem(scheme, PAYS, **GBM)
        prec = library_precision(M, case)
        sums, rec = ctx.level_sums(prob, level, n, off, prec, est, SEED, debug=True)
        o = oracle_run(case, level, np.arange(off, off + n, dtype=np.uint64), PAYS)
        check_records(case, level, n, off, PAYS, sums, rec, o)
    finally:
        ctx.set_tuning(**saved)


@pytest.mark.parametrize("level", [0, 2, 5])
@pytest.mark.parametrize("mcase", METHOD_CASES, ids=lambda m: f"m{m[0]}-q{m[1]}-" + "-".join(map(str, m[2])))
def test_methods_2_3(ctx, mcase, level):
    """Methods 2 and 3 of Section 3 (tables expanded by the library; Method 2's
    permutation on the exact side of the correction estimator, in the path kernel
    and in the normals-ahead kernel at level 5)."""
    method, q, case = mcase
    scheme, est, arith, packed = case
    n, off = _n_for(level), 500 + level
    prob = M.make_problem(scheme, PAYS, **GBM)
    prec = library_precision(M, case, q=q, method=method)
    sums, rec = ctx.level_sums(prob, level, n, off, prec, est, SEED, debug=True)
    o = oracle_run(case, level, np.arange(off, off + n, dtype=np.uint64), PAYS, method=method, q=q)
    check_records(case, level, n, off, PAYS, sums, rec, o, q=q)


def test_sums_without_debug_equal_debug_run(ctx):
    """The debug buffer is a flag of the same kernel: identical sums either way
    (per-path code, level-0 index histogram, normals computed ahead)."""
    prob = M.make_problem("milstein", PAYS, **GBM)
    prec = M.make_precision("fp32", 8)
    for est, level, n in ((M.EST_PLAIN, 5, 50_000), (M.EST_APPROX, 5, 50_000),
                          (M.EST_CORR, 5, 50_000), (M.EST_APPROX, 0, 300_000),
                          (M.EST_CORR, 6, 5_000), (M.EST_PLAIN, 3, 7_000)):
        a = ctx.level_sums(prob, level, n, 3, prec, est, SEED)
        b, _ = ctx.level_sums(prob, level, n, 3, prec, est, SEED, debug=True)
        assert a == b, (est, level)


@pytest.mark.parametrize("est,arith,method,q", [(M.EST_CORR, "fp32", 1, 8), (M.EST_CORR, "fp16", 1, 8),
                                                (M.EST_CORR, "fp32", 2, 8), (M.EST_CORR, "fp32", 1, 12),
                                                (M.EST_PLAIN, "fp32", 1, 8), (M.EST_PLAIN, "fp64", 1, 8)])
def test_level0_exact_loop_equals_debug_run(ctx, est, arith, method, q):
    """Level 0 of the exact-normal estimators without a debug buffer runs its own loop
    (the correction estimator's approximate side from per-index samples in LDS): the
    same sums as the per-path code of a debug run, bit for bit, over several tiles and
    ragged ends; one payoff (q = 12: the largest per-index table) or all five."""
    for pays in (("euro",), PAYS):
        if q == 12 and len(pays) > 1:
            continue
        prob = M.make_problem("milstein", pays, **GBM)
        prec = M.make_precision(arith, q, method=method)
        n = 1_000_003
        a = ctx.level_sums(prob, 0, n, 5, prec, est, SEED)
        b, _ = ctx.level_sums(prob, 0, n, 5, prec, est, SEED, debug=True)
        assert a == b, (est, arith, method, q, pays)


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
@pytest.mark.parametrize("packed", [True, False], ids=["packed", "unpacked"])
def test_fp16_two_paths_per_lane_equal_debug_run(ctx, scheme, packed):
    """FP16 approximate paths above level 0 run two per lane (packed binary16
    arithmetic) without a debug buffer: the same sums as the one-path-per-lane code of
    a debug run, bit for bit, over odd numbers of groups per thread and ragged path
    ranges; with path functionals (Asian, barrier) a lane keeps one path."""
    prec = M.make_precision("fp16", 8, packed)
    for pays in (("euro",), ("euro", "digital"), PAYS):
        prob = M.make_problem(scheme, pays, **GBM)
        for level, n, off in ((2, 70_001, 3), (4, 50_003, 11), (5, 20_011, 0), (8, 3_001, 7)):
            a = ctx.level_sums(prob, level, n, off, prec, M.EST_APPROX, SEED)
            b, _ = ctx.level_sums(prob, level, n, off, prec, M.EST_APPROX, SEED, debug=True)
            assert a == b, (scheme, packed, pays, level)


@pytest.mark.parametrize("est,arith,pays", [(M.EST_APPROX, "fixed", ("euro",)), (M.EST_APPROX, "fixed", PAYS),
                                             (M.EST_CORR, "fp32", ("euro",))],
                         ids=["fixed-one-payoff", "fixed-all-payoffs", "corr-fp32"])
def test_many_tiles_reduction(ctx, est, arith, pays):
    """A work cut into more than 8192 tiles (several batches of slot loads per lane of
    the fixed-order reduction, and a ragged last one) against the same work in the
    default tiles: the same path count and the same exact integer sums (every slot
    added exactly once), FP64 sums within rounding."""
    prob = M.make_problem("euler", pays, **GBM)
    fmt = WIDE_FMT if arith == "fixed" else None
    prec = M.make_precision(arith, 8, False, fmt)
    n, off = 3_000_001, 17
    ref = ctx.level_sums(prob, 2, n, off, prec, est, SEED)
    saved = ctx.get_tuning()
    ctx.set_tuning(tile_steps=256, min_tiles=1)
    try:
        small = ctx.level_sums(prob, 2, n, off, prec, est, SEED)
    finally:
        ctx.set_tuning(**saved)
    for p in pays:
        a, b = ref[p], small[p]
        assert a["n"] == b["n"] == n, p
        assert a["saturations"] == b["saturations"], p
        if arith == "fixed":
            assert a["isum1"] == b["isum1"] and a["isum2"] == b["isum2"], p
        for k in ("sum1", "sum2", "esum1", "esum2"):
            assert abs(a[k] - b[k]) <= 1e-10 * max(1.0, abs(a[k])), (p, k)


def test_repeatable_and_offset_split(ctx):
    """Bit-identical repeated runs; exact integer sums split over two path ranges add up."""
    prob = M.make_problem("euler", ("euro", "asian"), **GBM)
    prec = M.make_precision("fixed", 8, False, WIDE_FMT)
    a = ctx.level_sums(prob, 6, 100_000, 0, prec, M.EST_APPROX, SEED)
    b = ctx.level_sums(prob, 6, 100_000, 0, prec, M.EST_APPROX, SEED)
    assert a == b
    c1 = ctx.level_sums(prob, 6, 37_001, 0, prec, M.EST_APPROX, SEED)
    c2 = ctx.level_sums(prob, 6, 100_000 - 37_001, 37_001, prec, M.EST_APPROX, SEED)
    for p in ("euro", "asian"):
        assert c1[p]["isum1"] + c2[p]["isum1"] == a[p]["isum1"]
        assert c1[p]["isum2"] + c2[p]["isum2"] == a[p]["isum2"]


@pytest.mark.parametrize("arith,q,packed", [("fp32", 8, True), ("fp32", 4, True), ("fp32", 8, False),
                                            ("fp16", 8, True), ("fixed", 8, False)])
def test_approx_group_loop_equals_debug_run(ctx, arith, q, packed):
    """Levels >= 1 of the approximate estimator without a debug buffer run whole groups
    through a loop with path boundaries placed by construction: the same sums as the
    per-path code of a debug run, bit for bit, over many tiles and ragged ends; one
    payoff and all five (path functionals)."""
    for pays in (("euro",), PAYS):
        prob = M.make_problem("milstein", pays, **GBM)
        prec = M.make_precision(arith, q, packed, WIDE_FMT if arith == "fixed" else None)
        for level in (1, 2, 3, 4, 6):
            n = (1 << 21) // (1 << level) + 7
            a = ctx.level_sums(prob, level, n, 9, prec, M.EST_APPROX, SEED)
            b, _ = ctx.level_sums(prob, level, n, 9, prec, M.EST_APPROX, SEED, debug=True)
            assert a == b, (arith, q, packed, pays, level)


@pytest.mark.parametrize("est,arith,method", [(M.EST_PLAIN, "fp64", 1), (M.EST_PLAIN, "fp32", 1),
                                              (M.EST_CORR, "fp32", 1), (M.EST_CORR, "fp16", 1),
                                              (M.EST_CORR, "fp32", 2)])
def test_exact_group_loop_equals_debug_run(ctx, est, arith, method):
    """Levels >= 1 of the exact-normal estimators without a debug buffer run whole
    groups as (even, odd) step pairs with path boundaries by construction: the same
    sums as the per-path code of a debug run, bit for bit (70,001 paths: more than the
    normals-ahead limit, so every level runs the loop)."""
    for pays in (("euro",), PAYS):
        prob = M.make_problem("milstein", pays, **GBM)
        prec = M.make_precision(arith, 8, method=method)
        for level in (1, 2, 3, 5):
            a = ctx.level_sums(prob, level, 70_001, 11, prec, est, SEED)
            b, _ = ctx.level_sums(prob, level, 70_001, 11, prec, est, SEED, debug=True)
            assert a == b, (est, arith, method, pays, level)
