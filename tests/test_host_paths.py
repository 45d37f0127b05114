"""The kernels' per-path code compiled for the host (mlmc_check_paths_host) against
the oracle, with the same bars as the GPU parity tests (tests/parity.py), without a
GPU.  This pins the kernel arithmetic; the GPU tests add launch, tiling, reductions."""
import math

import numpy as np
import pytest

import paper_2502_07123_amd as M
from oracle.paths import Precision, Problem, simulate
from parity import (CASES, EST_APPROX, EST_CORR, EST_PLAIN, GBM, METHOD_CASES, PAYS, SEED, WIDE_FMT, case_q, library_precision,
                    check_records, oracle_run)


@pytest.mark.parametrize("level", [0, 1, 3, 6])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_host_paths_match_oracle(case, level):
    scheme, est, arith, packed = case
    n, off = 700, 33
    prob = M.make_problem(scheme, PAYS, **GBM)
    prec = library_precision(M, case)
    sums, rec = M.check_paths_host(prob, level, n, off, prec, est, SEED)
    o = oracle_run(case, level, np.arange(off, off + n, dtype=np.uint64), PAYS)
    check_records(case, level, n, off, PAYS, sums, rec, o)


def test_host_narrow_fixed_counts_saturations():
    """A format too narrow for X saturates; the per-path counts match the oracle's."""
    fmt = dict(WIDE_FMT)
    fmt["X"] = (8, 6)
    fmt["mul2"] = (12, 10)
    prob = M.make_problem("euler", ("euro",), **GBM)
    prec = M.make_precision("fixed", 8, False, fmt)
    sums, rec = M.check_paths_host(prob, 4, 3000, 0, prec, M.EST_APPROX, SEED)
    o = simulate(Problem("euler", **GBM), 4, np.arange(3000, dtype=np.uint64),
                 Precision("fixed", 8, False, tuple((v, w, f) for v, (w, f) in fmt.items())),
                 M.EST_APPROX, SEED)
    assert o["sat"].sum() > 0
    assert np.array_equal(rec["saturations"], o["sat"])
    assert sums["euro"]["saturations"] == int(o["sat"].sum())
    assert np.array_equal(rec["XN_raw"], o["XN_approx"])


@pytest.mark.parametrize("level", [0, 3])
@pytest.mark.parametrize("mcase", METHOD_CASES, ids=lambda m: f"m{m[0]}-q{m[1]}-" + "-".join(map(str, m[2])))
def test_host_methods_2_3_match_oracle(mcase, level):
    """Methods 2 and 3 of Section 3: same records as the oracle (Method 2's
    correction estimator with the permuted coupled uniform on the exact side)."""
    method, q, case = mcase
    scheme, est, arith, packed = case
    n, off = 700, 31
    prob = M.make_problem(scheme, PAYS, **GBM)
    prec = library_precision(M, case, q=q, method=method)
    sums, rec = M.check_paths_host(prob, level, n, off, prec, est, SEED)
    o = oracle_run(case, level, np.arange(off, off + n, dtype=np.uint64), PAYS, method=method, q=q)
    check_records(case, level, n, off, PAYS, sums, rec, o, q=q)


EXACT0_CASES = [c for c in CASES if c[1] == EST_PLAIN or (c[1] == EST_CORR and c[2] != "fixed")]


@pytest.mark.parametrize("case", EXACT0_CASES, ids=lambda c: "-".join(map(str, c)))
def test_level0_exact_loop_equals_per_path_code(case):
    """Level 0 of the exact-normal estimators without records runs the kernels'
    level-0 loop (per-index approximate-side samples for the correction estimator):
    its sums equal those of the per-path code bit for bit (same operations, same
    order of accumulation), and with an FP64 exact side they hold the oracle's
    samples (plain FP32 per-path values are pinned by the record tests above)."""
    scheme, est, arith, packed = case
    n, off = 1001, 17                       # a ragged group at each end
    prob = M.make_problem(scheme, PAYS, **GBM)
    prec = library_precision(M, case)
    fast, none = M.check_paths_host(prob, 0, n, off, prec, est, SEED, records=False)
    slow, rec = M.check_paths_host(prob, 0, n, off, prec, est, SEED)
    assert none is None and rec is not None
    o = oracle_run(case, 0, np.arange(off, off + n, dtype=np.uint64), PAYS)
    for name in PAYS:
        a, b = fast[name], slow[name]
        for f in ("n", "sum1", "sum2", "esum1", "esum2", "nonfinite"):
            assert a[f] == b[f], (name, f, a[f], b[f])
        assert a["n"] == n
        if (arith == "fp32" and est == EST_PLAIN) or arith.endswith("x"):
            continue
        Y = o[name]["Y"]
        assert abs(a["sum1"] - math.fsum(Y)) <= 1e-9 * (np.sum(np.abs(Y)) + 1e-300)


@pytest.mark.parametrize("q", [8, 12])
def test_level0_exact_loop_method2_correction(q):
    """Method 2's correction estimator (the exact side inverts the permuted word):
    the level-0 loop's sums equal the per-path code's."""
    case = ("euler", EST_CORR, "fp32", False)
    prob = M.make_problem("euler", PAYS, **GBM)
    prec = M.make_precision("fp32", q, False, WIDE_FMT, method=2)
    fast, _ = M.check_paths_host(prob, 0, 777, 5, prec, EST_CORR, SEED, records=False)
    slow, _ = M.check_paths_host(prob, 0, 777, 5, prec, EST_CORR, SEED)
    for name in PAYS:
        for f in ("n", "sum1", "sum2", "esum1", "esum2", "nonfinite"):
            assert fast[name][f] == slow[name][f], (name, f)


@pytest.mark.parametrize("level", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("arith,q,packed", [("fp32", 8, True), ("fp32", 4, True), ("fp32", 8, False),
                                            ("fp16", 8, True), ("fp32", 6, True)])
@pytest.mark.parametrize("pays", [("euro",), PAYS], ids=["one", "all"])
def test_approx_group_loop_equals_per_path_code(level, arith, q, packed, pays):
    """Above level 0 the approximate estimator's whole groups (no records) run a loop
    that places path starts and ends by construction: the same sums as the per-path
    code, bit for bit, with ragged groups at both ends (q = 6: five fields per word,
    the general code throughout)."""
    n, off = 901, 13
    prob = M.make_problem("milstein", pays, **GBM)
    prec = M.make_precision(arith, q, packed)
    fast, _ = M.check_paths_host(prob, level, n, off, prec, EST_APPROX, SEED, records=False)
    slow, _ = M.check_paths_host(prob, level, n, off, prec, EST_APPROX, SEED)
    for name in pays:
        for f in ("n", "sum1", "sum2", "nonfinite"):
            assert fast[name][f] == slow[name][f], (name, f)


@pytest.mark.parametrize("level", [1, 2, 3, 5])
@pytest.mark.parametrize("case", [("milstein", EST_PLAIN, "fp64"), ("euler", EST_PLAIN, "fp32"),
                                  ("milstein", EST_CORR, "fp32"), ("euler", EST_CORR, "fp16"),
                                  ("milstein", EST_CORR, "fixed")], ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("pays", [("euro",), PAYS], ids=["one", "all"])
def test_exact_group_loop_equals_per_path_code(level, case, pays):
    """Above level 0 the exact-normal estimators' whole groups (no records) run a loop
    of (even, odd) step pairs with path boundaries by construction: the same sums as
    the per-path code, bit for bit (fixed point: the general code throughout)."""
    scheme, est, arith = case
    n, off = 333, 5
    prob = M.make_problem(scheme, pays, **GBM)
    prec = M.make_precision(arith, 8, False, WIDE_FMT if arith == "fixed" else None)
    fast, _ = M.check_paths_host(prob, level, n, off, prec, est, SEED, records=False)
    slow, _ = M.check_paths_host(prob, level, n, off, prec, est, SEED)
    for name in pays:
        for f in ("n", "sum1", "sum2", "esum1", "esum2", "nonfinite", "isum1"):
            assert fast[name][f] == slow[name][f], (name, f)


def test_method2_correction_group_loop():
    """Method 2's permuted coupled word on the exact side, above level 0."""
    prob = M.make_problem("euler", PAYS, **GBM)
    prec = M.make_precision("fp32", 8, False, WIDE_FMT, method=2)
    for level in (1, 3):
        fast, _ = M.check_paths_host(prob, level, 555, 3, prec, EST_CORR, SEED, records=False)
        slow, _ = M.check_paths_host(prob, level, 555, 3, prec, EST_CORR, SEED)
        for name in PAYS:
            for f in ("n", "sum1", "sum2", "esum1", "esum2"):
                assert fast[name][f] == slow[name][f], (name, f, level)


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
@pytest.mark.parametrize("arith,q,packed", [("fixed", 8, False), ("fp32", 8, True), ("fp16", 8, True)])
def test_approx_group_loop_equals_per_path_code(scheme, arith, q, packed):
    """Levels >= 1 of the approximate estimator without records run whole groups with
    path boundaries by construction: the same sums as the per-path code (exact
    integers for fixed point), ragged ends included."""
    fmt = WIDE_FMT if arith == "fixed" else None
    for pays in (("euro",), PAYS):
        prob = M.make_problem(scheme, pays, **GBM)
        prec = M.make_precision(arith, q, packed, fmt)
        for level in (1, 2, 3, 5):
            n = 3001
            fast, _ = M.check_paths_host(prob, level, n, 7, prec, EST_APPROX, SEED, records=False)
            slow, _ = M.check_paths_host(prob, level, n, 7, prec, EST_APPROX, SEED)
            for name in pays:
                for f in ("n", "sum1", "sum2", "isum1", "isum2", "saturations", "nonfinite"):
                    assert fast[name][f] == slow[name][f], (level, name, f)
