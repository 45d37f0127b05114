"""Shared per-path comparison of the library's path records with the oracle.

Bars (the readings behind them are in the design notes):
* uniform words and table indices: bit-exact;
* fixed-point side: terminal values, payoff differences and integer sums bit-exact;
* FP32 / FP16 table side (APPROX, and the approximate side of CORR): Algorithm 1
  is evaluated operation by operation in that type on both sides -> bit-exact;
* FP64 exact side: within 1e-12 of the path scale max(|X_N|, X_0), X_0 = 1 (= S0);
* plain FP32 (own FP32 inverse normal): within the worst-case bound of
  plain32_tol(level), derived from the inverse-normal error and per-step rounding;
* FP64 sums: equal to the sum of the records within the FP64 summation bound.
"""
import math

import numpy as np

from oracle import philox
from oracle.paths import Precision, Problem, simulate

GBM = dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, barrier=85.0)
PAYS = ("forward", "euro", "asian", "barrier", "digital")
SEED = 1234
# formats wide enough that nothing saturates at sigma = 0.2
WIDE = (("X", 32, 29), ("con1", 32, 34), ("con2", 32, 33), ("con3", 32, 36),
        ("Z", 31, 28), ("mul1", 32, 30), ("sum1", 32, 30), ("zsq", 32, 23),
        ("zm1", 32, 23), ("mul3", 32, 29), ("sum2", 32, 29), ("mul2", 32, 27))
WIDE_FMT = {v: (w, f) for v, w, f in WIDE}

EST_PLAIN, EST_APPROX, EST_CORR = 0, 1, 2

# approximate normals of Section 3 beyond Method 1: (method, q, case)
_MC = [("milstein", EST_APPROX, "fp32", False), ("euler", EST_CORR, "fp32", False),
       ("milstein", EST_CORR, "fixed", False), ("euler", EST_APPROX, "fp16", False),
       ("milstein", EST_APPROX, "fp32", True), ("milstein", EST_CORR, "fp16", False)]
METHOD_CASES = ([(2, 8, c) for c in _MC] + [(3, 8, c) for c in _MC] +
                [(2, 12, c) for c in _MC if c[2] != "fixed" and not c[3]] +
                [(3, 11, c) for c in _MC if not c[3]])

CASES = [
    # (scheme, estimator, arith, packed)
    ("euler", EST_PLAIN, "fp64", False),
    ("milstein", EST_PLAIN, "fp64", False),
    ("euler", EST_PLAIN, "fp32", False),
    ("milstein", EST_PLAIN, "fp32", False),
    ("euler", EST_APPROX, "fp32", False),
    ("milstein", EST_APPROX, "fp32", False),
    ("milstein", EST_APPROX, "fp32", True),
    ("euler", EST_APPROX, "fp32", True),
    ("euler", EST_CORR, "fp32", False),
    ("milstein", EST_CORR, "fp32", False),
    ("euler", EST_APPROX, "fixed", False),
    ("milstein", EST_APPROX, "fixed", False),
    ("milstein", EST_CORR, "fixed", False),
    ("euler", EST_APPROX, "fp16", False),
    ("milstein", EST_APPROX, "fp16", True),
    ("milstein", EST_CORR, "fp16", False),
    # correction estimator with an FP32 exact side (reading R21's narrower option):
    # arith "<table side>x"
    ("euler", EST_CORR, "fp32x", False),
    ("milstein", EST_CORR, "fp32x", False),
    ("milstein", EST_CORR, "fp16x", False),
]


def split_arith(arith):
    """(table-side arithmetic, exact side) of a case's arith: 'fp32x' is an FP32
    table side with an FP32 exact side."""
    return (arith[:-1], "fp32") if arith.endswith("x") else (arith, "fp64")


def library_precision(M, case, q=None, fmt=None, method=1):
    scheme, est, arith, packed = case
    base, exact = split_arith(arith)
    return M.make_precision(base, q or case_q(case), packed, fmt if fmt is not None else WIDE_FMT,
                            method=method, exact=exact)


def case_q(case):
    scheme, est, arith, packed = case
    return 8 if not packed else (6 if scheme == "euler" else 8)


def oracle_run(case, level, paths, payoffs, gbm=GBM, seed=SEED, option=0, method=1, q=None):
    scheme, est, arith, packed = case
    arith, exact = split_arith(arith)
    prec = Precision(arith if est != EST_PLAIN else "fp32", q or case_q(case), packed, WIDE, method, exact)
    return simulate(Problem(scheme, **gbm), level, paths, prec, est, seed, option, payoffs,
                    plain_arith=arith if est == EST_PLAIN else "fp64")


# worst-case relative bound of the plain-FP32 estimator's Z against the oracle's
# round-to-FP32 of the exact quantile: the fit's 2.6e-7 (over the 32-bit grid, with
# margin 4e-7) plus the oracle's own half ulp 2^-24
ZREL32 = 4e-7 + 2.0 ** -24


def plain32_tol(level, gbm=GBM):
    """|dX_N| / max(|X_N|, 1) for plain FP32: per step, the multiplier differs by
    con2 |dZ| <= sigma sqrt(h) * ZREL32 * 6.34 (|Z| <= 6.34 on the 32-bit grid), and
    the two roundings of X + X s can land up to one ulp apart on each side; summed
    over N steps: N (sigma sqrt(h) 6.34 ZREL32 + 4 * 2^-24), plus 1e-6."""
    N = 1 << level
    h = gbm["T"] / N
    return 1e-6 + N * (gbm["sigma"] * math.sqrt(h) * 6.34 * ZREL32 + 4 * 2.0 ** -24)


def k_of(gbm):
    return gbm["K"] / gbm["S0"]


def near_count(o, p, gbm):
    """Exact-side paths whose digital / barrier decision lies within 1e-5 of its
    threshold (an FP32 exact side may decide them either way)."""
    return int(near_threshold(o, "exact", p, gbm["K"] / gbm["S0"], gbm["barrier"] / gbm["S0"], 1e-5).sum())


def near_threshold(o, side, p, k, b, margin):
    """Paths whose digital / barrier decision lies within `margin` (relative) of its
    threshold on the fine or coarse path: rounding may put them on either side."""
    f = lambda key: o[key].astype(np.float64)
    if p == "digital":
        return (np.abs(f("XN_" + side) - k) < margin * k) | (np.abs(f("XcN_" + side) - k) < margin * k)
    if p == "barrier":
        return ((np.abs(f("min_" + side) - b) < margin * b) | (np.abs(f("minc_" + side) - b) < margin * b) |
                (np.abs(f("XN_" + side) - k) < margin * k) | (np.abs(f("XcN_" + side) - k) < margin * k))
    return np.zeros(o["n"], dtype=bool)


def check_close(rec, o, side, payoffs, tol, Ykey="Y", gbm=GBM):
    k, b = gbm["K"] / gbm["S0"], gbm["barrier"] / gbm["S0"]
    for key in ("XN_", "XcN_"):
        X, Xo = rec[key + side], o[key + side].astype(np.float64)
        scale = np.maximum(np.abs(Xo), 1.0)
        err = np.abs(X - Xo) / scale
        assert np.all(err <= tol), (key + side, float(err.max()), tol)
    for i, p in enumerate(PAYS):
        if p not in payoffs:
            continue
        d = np.abs(rec["Y"][:, i] - o[p][Ykey])
        # the level difference of 1-Lipschitz payoffs moves by at most the two paths' moves
        bad = (d > 2 * tol * np.maximum(np.abs(o["XN_" + side]), 1.0) * max(k, 1.0) + 1e-300)
        bad &= ~near_threshold(o, side, p, k, b, max(10 * tol, 1e-6))
        assert not bad.any(), (p, float(d.max()), np.flatnonzero(bad)[:5])


def check_records(case, level, n, off, payoffs, sums, rec, o, gbm=GBM, seed=SEED, q=None):
    scheme, est, arith, packed = case
    arith, exact = split_arith(arith)
    q = q or case_q(case)
    paths = np.arange(off, off + n, dtype=np.uint64)
    if not packed:
        J = philox.stream_words(seed, 0, level, est, paths * np.uint64(1 << level))
        assert np.array_equal(rec["first_word"], J)
        if est != EST_PLAIN:
            assert np.array_equal(rec["first_index"], (J >> np.uint32(32 - q)).astype(np.uint32))
    if est == EST_PLAIN:
        tol = 1e-12 if arith == "fp64" else plain32_tol(level, gbm)
        check_close(rec, o, "exact", payoffs, tol, gbm=gbm)
    if est == EST_CORR and exact == "fp64":
        check_close(rec, o, "exact", (), 1e-12, gbm=gbm)
    if est == EST_CORR and exact == "fp32":
        # the approximate side is bit-exact below, so Y differs by the exact side only
        check_close(rec, o, "exact", payoffs, plain32_tol(level, gbm), gbm=gbm)
    if est != EST_PLAIN:
        if arith == "fixed":
            assert np.array_equal(rec["XN_raw"], o["XN_approx"])
            assert np.array_equal(rec["XcN_raw"], o["XcN_approx"])
            for i, p in enumerate(PAYS):
                if p in payoffs:
                    assert np.array_equal(rec["Yraw"][:, i], o[p]["Y_approx_raw"]), p
        else:
            assert np.array_equal(rec["XN_approx"], o["XN_approx"].astype(np.float64))
            assert np.array_equal(rec["XcN_approx"], o["XcN_approx"].astype(np.float64))
            for i, p in enumerate(PAYS):
                if p in payoffs:
                    Ya = rec["Yraw"][:, i].view(np.float64)
                    assert np.array_equal(Ya, o[p]["Y_approx"]), p
    for i, p in enumerate(PAYS):
        if p not in payoffs:
            continue
        if est == EST_APPROX:
            assert np.array_equal(rec["Y"][:, i], o[p]["Y"]), p
        if est == EST_CORR and exact == "fp64":
            assert np.all(np.abs(rec["Y"][:, i] - o[p]["Y"]) <= 1e-12 * (1 + np.abs(o[p]["Y_exact"]))), p
        s = sums[p]
        assert s["n"] == n and s["nonfinite"] == 0 and s["saturations"] == 0
        Y = rec["Y"][:, i]
        assert abs(s["sum1"] - math.fsum(Y)) <= 4 * n * 2.0 ** -53 * (np.sum(np.abs(Y)) + 1e-300)
        assert abs(s["sum2"] - math.fsum(Y * Y)) <= 4 * n * 2.0 ** -53 * np.sum(Y * Y) + 1e-300
        if arith == "fixed" and est == EST_APPROX:
            oi = [int(v) for v in o[p]["Y_approx_raw"]]
            assert s["isum1"] == sum(oi) and s["isum2"] == sum(v * v for v in oi)
        if est == EST_CORR:
            E = o[p]["Y_exact"]
            etol = 1e-10 if exact == "fp64" else 4 * plain32_tol(level, gbm) * max(k_of(gbm), 1.0)
            assert abs(s["esum1"] - math.fsum(E)) <= etol * (np.sum(np.abs(E)) + 1) + near_count(o, p, gbm) * max(k_of(gbm), 1.0)
