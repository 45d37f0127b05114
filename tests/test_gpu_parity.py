"""GPU parity: the HIP path through the C ABI against the oracle, element by element
(bars in tests/parity.py).  Per-path records come from the same kernel (a debug
buffer flag).  Sizes span several tiles with a ragged tail at every level."""
import numpy as np
import pytest

import paper_2502_07123_amd as M
from parity import (CASES, GBM, PAYS, SEED, WIDE_FMT, case_q, check_records, oracle_run)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0, workspace_bytes=768 << 20)
    yield c
    c.close()


def _n_for(level):
    # several tiles (2^16 path-steps each) and a ragged tail at every level
    return int(max(3 * (1 << 16) // max(1 << level, 16) + 77, 2000))


@pytest.mark.parametrize("level", [0, 1, 4, 7])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("payoffs", [("euro",), PAYS], ids=["euro", "all"])
def test_paths_and_sums(ctx, case, level, payoffs):
    scheme, est, arith, packed = case
    n, off = _n_for(level), 1000 + level
    prob = M.make_problem(scheme, payoffs, **GBM)
    prec = M.make_precision(arith, case_q(case), packed, WIDE_FMT)
    sums, rec = ctx.level_sums(prob, level, n, off, prec, est, SEED, debug=True)
    o = oracle_run(case, level, np.arange(off, off + n, dtype=np.uint64), payoffs)
    check_records(case, level, n, off, payoffs, sums, rec, o)


def test_sums_without_debug_equal_debug_run(ctx):
    """The debug buffer is a flag of the same kernel: identical sums either way."""
    prob = M.make_problem("milstein", PAYS, **GBM)
    prec = M.make_precision("fp32", 8)
    for est in (M.EST_PLAIN, M.EST_APPROX, M.EST_CORR):
        a = ctx.level_sums(prob, 5, 50_000, 3, prec, est, SEED)
        b, _ = ctx.level_sums(prob, 5, 50_000, 3, prec, est, SEED, debug=True)
        assert a == b


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
