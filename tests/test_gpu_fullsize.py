"""Parity at the full size of the fixed-point workload: 1,000,000 paths per level,
levels 0..10 (1024 fine steps at the finest), Q-int32 paths with X's fractional bits
b_l = min(24, 14 + l) (reading R19; the other formats wide enough not to saturate
at sigma = 0.2), the q = 8 Method-1 table in Z's fixed-point format, and the
European, Asian and down-and-out barrier (85) payoffs on the same paths (one
launch).  Euler (Algorithm 1) at every level, Milstein at levels 0, 5 and 10.

* per-path records bit-exact against the oracle: every path at levels <= 6, a
  fixed subsample of 65,536 path indices (the same at every level) above;
* the exact integer sums over all 1,000,000 paths equal the sums of the per-path
  integer samples the same kernel wrote, and at levels <= 6 the oracle's."""
import numpy as np
import pytest

import paper_2502_07123_amd as M
from parity import GBM, SEED, WIDE_FMT, oracle_run

pytestmark = pytest.mark.gpu

N_PATHS = 1_000_000
PAYS3 = ("euro", "asian", "barrier")
IDX = {"forward": 0, "euro": 1, "asian": 2, "barrier": 3, "digital": 4}
SAMPLE = np.unique(np.concatenate([
    np.arange(64), N_PATHS - 64 + np.arange(64),
    np.random.default_rng(20250207).choice(N_PATHS, 65_536 - 128, replace=False)]))[:65_536]


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0, workspace_bytes=256 << 20)
    yield c
    c.close()


def _fmt(level):
    b = min(24, 14 + level)
    return {**WIDE_FMT, "X": (32, b)}, b


@pytest.mark.parametrize("scheme,level", [("euler", l) for l in range(11)] +
                         [("milstein", 0), ("milstein", 5), ("milstein", 10)])
def test_fixed_point_full_size(ctx, scheme, level):
    fmt, b = _fmt(level)
    prob = M.make_problem(scheme, PAYS3, **GBM)
    prec = M.make_precision("fixed", 8, False, fmt)
    sums, rec = ctx.level_sums(prob, level, N_PATHS, 0, prec, M.EST_APPROX, SEED, debug=True)
    assert rec.shape[0] == N_PATHS
    # exact integer sums over all paths = sums of the kernel's own per-path samples
    for p in PAYS3:
        s = sums[p]
        assert s["n"] == N_PATHS and s["saturations"] == 0 and s["nonfinite"] == 0
        yi = rec["Yraw"][:, IDX[p]].astype(object)
        assert s["isum1"] == int(np.sum(rec["Yraw"][:, IDX[p]]))
        assert s["isum2"] == int(sum(v * v for v in yi)), p
    # per-path records against the oracle
    idx = np.arange(N_PATHS) if level <= 6 else SAMPLE
    case = (scheme, M.EST_APPROX, "fixed", False)
    from oracle.paths import Precision, Problem, simulate
    paths = idx.astype(np.uint64)
    o = simulate(Problem(scheme, **GBM), level, paths, Precision("fixed", 8, False, tuple(
        (v, w, f) for v, (w, f) in fmt.items())), M.EST_APPROX, SEED, 0, PAYS3)
    r = rec[idx]
    assert np.array_equal(r["XN_raw"], o["XN_approx"])
    assert np.array_equal(r["XcN_raw"], o["XcN_approx"])
    for p in PAYS3:
        assert np.array_equal(r["Yraw"][:, IDX[p]], o[p]["Y_approx_raw"]), p
        assert np.array_equal(r["Y"][:, IDX[p]], o[p]["Y"]), p
        if level <= 6:
            oi = [int(v) for v in o[p]["Y_approx_raw"]]
            assert sums[p]["isum1"] == sum(oi) and sums[p]["isum2"] == sum(v * v for v in oi), p
