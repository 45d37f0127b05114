"""Pins for the oracle's coupled paths (Section 2.1, Algorithm 1, readings R2-R5).

Deterministic pins (from the same stream words, computed here independently):
* Euler on GBM telescopes to a product: X_N = prod (1 + r h + sigma sqrt(h) Z_n);
  Milstein to prod (1 + r h + sigma sqrt(h) Z + sigma^2 h (Z^2 - 1) / 2).
* The coarse path of level l is the fine path of level l-1 driven by
  Z'_m = (Z_2m + Z_2m+1) / sqrt(2) (Section 2.1's coupling, R2).
* Payoffs recomputed from the whole path (trapezoid average, minimum incl. X_0).
* Wide fixed-point formats follow the FP64 path within the rounding bounds.
Statistical pins:
* exact discrete-time moments E[X_N] = (1 + r h)^N and E[X_N^2] (Euler, Milstein,
  and with Method-1 normals E[Z~^2] = 1 - MSE_q);
* strong rates 1/2 (Euler) and 1 (Milstein) against the exact GBM solution;
* Black-Scholes call and digital prices from the MLMC telescoping sum.
"""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import normal, philox
from oracle.mlmc import level_sums, scale_price
from oracle.paths import (EST_APPROX, EST_CORR, EST_PLAIN, Precision, Problem,
                          simulate)

GBM = dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, barrier=85.0)
SEED = 1234

WIDE = (("X", 32, 29), ("con1", 32, 34), ("con2", 32, 33), ("con3", 32, 36),
        ("Z", 32, 28), ("mul1", 32, 30), ("sum1", 32, 30), ("zsq", 32, 23),
        ("zm1", 32, 23), ("mul3", 32, 29), ("sum2", 32, 29), ("mul2", 32, 27))


def bs_call(S0, K, r, s, T):
    d1 = (math.log(S0 / K) + (r + 0.5 * s * s) * T) / (s * math.sqrt(T))
    d2 = d1 - s * math.sqrt(T)
    return S0 * norm.cdf(d1) - K * math.exp(-r * T) * norm.cdf(d2)


def bs_digital(S0, K, r, s, T):
    d2 = (math.log(S0 / K) + (r - 0.5 * s * s) * T) / (s * math.sqrt(T))
    return K * math.exp(-r * T) * norm.cdf(d2)


def test_closed_forms_values():
    # d1 = 0.35, d2 = 0.15 for the paper's call (Section 4.4 parameters)
    assert abs(bs_call(100, 100, 0.05, 0.2, 1) - 10.450583572185565) < 1e-9
    assert abs(bs_digital(100, 100, 0.05, 0.2, 1) - 53.232481545376345) < 1e-8


def words_matrix(level, est, paths, seed=SEED, option=0):
    N = 1 << level
    g = paths[:, None].astype(np.uint64) * np.uint64(N) + np.arange(N, dtype=np.uint64)[None]
    return philox.stream_words(seed, option, level, est, g.ravel()).reshape(len(paths), N)


def euler_factor(r, h, s, Z):
    return 1 + r * h + s * math.sqrt(h) * Z


def milstein_factor(r, h, s, Z):
    return 1 + r * h + s * math.sqrt(h) * Z + 0.5 * s * s * h * (Z * Z - 1)


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
@pytest.mark.parametrize("level", [0, 1, 2, 5])
def test_fp64_paths_equal_product_forms(scheme, level):
    p = Problem(scheme, **GBM)
    paths = np.arange(5, 301, dtype=np.uint64)
    out = simulate(p, level, paths, Precision(), EST_PLAIN, SEED)
    Z = normal.exact_normal(words_matrix(level, EST_PLAIN, paths))
    h = p.T / 2 ** level
    fac = euler_factor if scheme == "euler" else milstein_factor
    Xf = np.prod(fac(p.r, h, p.sigma, Z), axis=1)
    assert np.allclose(out["XN_exact"], Xf, rtol=1e-13, atol=0)
    if level >= 1:
        Zp = (Z[:, 0::2] + Z[:, 1::2]) / math.sqrt(2)         # coarse = fine of level-1
        Xc = np.prod(fac(p.r, 2 * h, p.sigma, Zp), axis=1)
        assert np.allclose(out["XcN_exact"], Xc, rtol=1e-13, atol=0)


@pytest.mark.parametrize("q", [4, 8])
def test_table_side_uses_method1_values(q):
    p = Problem("euler", **GBM)
    level = 3
    paths = np.arange(200, dtype=np.uint64)
    out = simulate(p, level, paths, Precision("fp64", q), EST_CORR, SEED)
    J = words_matrix(level, EST_CORR, paths)
    T = normal.table_float(q, "float64")
    h = p.T / 2 ** level
    Zt = T[normal.table_index(J, q)]
    assert np.allclose(out["XN_approx"], np.prod(euler_factor(p.r, h, p.sigma, Zt), axis=1),
                       rtol=1e-13)
    # the same words drive the exact side (coupling of Section 3)
    Z = normal.exact_normal(J)
    assert np.allclose(out["XN_exact"], np.prod(euler_factor(p.r, h, p.sigma, Z), axis=1),
                       rtol=1e-13)


def test_packed_stream_uses_fields():
    p = Problem("euler", **GBM)
    level, q = 2, 8
    paths = np.arange(64, dtype=np.uint64)
    out = simulate(p, level, paths, Precision("fp64", q, packed=True), EST_APPROX, SEED)
    N, F = 1 << level, 32 // q
    g = paths[:, None] * np.uint64(N) + np.arange(N, dtype=np.uint64)[None]
    J = philox.stream_words(SEED, 0, level, EST_APPROX, (g // np.uint64(F)).ravel())
    j = (g % np.uint64(F)).ravel().astype(np.int64)
    k = ((J.astype(np.int64) >> (32 - q * (j + 1))) & ((1 << q) - 1)).reshape(g.shape)
    Zt = normal.table_float(q, "float64")[k]
    h = p.T / N
    assert np.allclose(out["XN_approx"], np.prod(euler_factor(p.r, h, p.sigma, Zt), axis=1),
                       rtol=1e-13)


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
def test_payoffs_from_whole_path(scheme):
    p = Problem(scheme, **GBM)
    level = 4
    paths = np.arange(400, dtype=np.uint64)
    names = ("forward", "euro", "asian", "barrier", "digital")
    out = simulate(p, level, paths, Precision(), EST_PLAIN, SEED, payoffs=names)
    Z = normal.exact_normal(words_matrix(level, EST_PLAIN, paths))
    h = p.T / 2 ** level
    fac = euler_factor if scheme == "euler" else milstein_factor
    k, b = p.K / p.S0, p.barrier / p.S0

    def pay(X):
        grid = np.concatenate([np.ones((X.shape[0], 1)), X], axis=1)
        XN = grid[:, -1]
        A = np.mean(0.5 * (grid[:, :-1] + grid[:, 1:]), axis=1)
        return {"forward": XN, "euro": np.maximum(XN - k, 0),
                "asian": np.maximum(A - k, 0),
                "barrier": np.where(grid.min(axis=1) > b, np.maximum(XN - k, 0), 0),
                "digital": np.where(XN > k, k, 0.0)}

    Pf = pay(np.cumprod(fac(p.r, h, p.sigma, Z), axis=1))
    Zp = (Z[:, 0::2] + Z[:, 1::2]) / math.sqrt(2)
    Pc = pay(np.cumprod(fac(p.r, 2 * h, p.sigma, Zp), axis=1))
    for n in names:
        assert np.allclose(out[n]["Y"], Pf[n] - Pc[n], rtol=1e-11, atol=1e-13), n


def test_level0_has_no_coarse():
    p = Problem("euler", **GBM)
    paths = np.arange(100, dtype=np.uint64)
    out = simulate(p, 0, paths, Precision(), EST_PLAIN, SEED, payoffs=("euro",))
    assert np.array_equal(out["euro"]["Y"], out["euro"]["Pf_exact"])


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
def test_fixed_wide_follows_fp64_table_path(scheme):
    p = Problem(scheme, **GBM)
    level = 4
    paths = np.arange(500, dtype=np.uint64)
    fixed = simulate(p, level, paths, Precision("fixed", 8, fmt=WIDE), EST_APPROX, SEED,
                     payoffs=("euro", "asian"))
    flt = simulate(p, level, paths, Precision("fp64", 8), EST_APPROX, SEED,
                   payoffs=("euro", "asian"))
    assert fixed["sat"].sum() == 0
    XN = fixed["XN_approx"] * 2.0 ** -29
    # each of the 16 steps rounds ~5 variables at <= 2^-28 relative: 1e-6 is loose
    assert np.allclose(XN, flt["XN_approx"], rtol=1e-6, atol=0)
    for n in ("euro", "asian"):
        assert np.allclose(fixed[n]["Y"], flt[n]["Y"], atol=1e-6)


@pytest.mark.parametrize("arith,u", [("fp32", 2.0 ** -24), ("fp16", 2.0 ** -11)])
@pytest.mark.parametrize("scheme", ["euler", "milstein"])
def test_float_sides_round_at_their_precision(arith, u, scheme):
    """FP32 / FP16 table paths follow the FP64 table path within the per-step
    rounding bound (Algorithm 1: at most ~6 roundings of unit roundoff u per step,
    constants and table values rounded once), and deviate by at least the rounding
    scale -- arithmetic carried out in a wider type would not."""
    p = Problem(scheme, **GBM)
    level, N = 4, 16
    paths = np.arange(2000, dtype=np.uint64)
    lo = simulate(p, level, paths, Precision(arith, 8), EST_APPROX, SEED, payoffs=("euro",))
    ref = simulate(p, level, paths, Precision("fp64", 8), EST_APPROX, SEED, payoffs=("euro",))
    dt = {"fp32": np.float32, "fp16": np.float16}[arith]
    for key in ("XN_approx", "XcN_approx"):
        assert lo[key].dtype == np.dtype(dt)
        err = np.abs(lo[key].astype(np.float64) - ref[key]) / np.maximum(np.abs(ref[key]), 1.0)
        assert err.max() <= 8 * N * u, (key, err.max() / u)
        assert err.mean() >= u / 8, (key, err.mean() / u)


def test_fixed_narrow_saturates_and_counts():
    p = Problem("euler", **GBM)
    fmt = tuple((v, w, f) if v != "X" else ("X", 8, 7) for v, w, f in WIDE)   # X < 1
    out = simulate(p, 3, np.arange(2000, dtype=np.uint64), Precision("fixed", 8, fmt=fmt),
                   EST_APPROX, SEED)
    assert out["sat"].sum() > 0
    assert out["XN_approx"].max() <= 127


def _moment_check(sample, expected, nsig=4.5):
    se = sample.std() / math.sqrt(sample.size)
    assert abs(sample.mean() - expected) < nsig * se, (sample.mean(), expected, se)


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
def test_exact_discrete_moments(scheme):
    p = Problem(scheme, **GBM)
    level = 3
    N, h = 1 << level, p.T / (1 << level)
    out = simulate(p, level, np.arange(200_000, dtype=np.uint64), Precision(), EST_PLAIN, SEED,
                   payoffs=("forward",))
    X = out["XN_exact"]
    _moment_check(X, (1 + p.r * h) ** N)
    m2 = (1 + p.r * h) ** 2 + p.sigma ** 2 * h
    if scheme == "milstein":
        m2 += 0.5 * p.sigma ** 4 * h * h
    _moment_check(X * X, m2 ** N)


@pytest.mark.parametrize("q", [4, 8])
def test_table_discrete_moments(q):
    p = Problem("euler", **GBM)
    level = 3
    N, h = 1 << level, p.T / (1 << level)
    out = simulate(p, level, np.arange(200_000, dtype=np.uint64), Precision("fp64", q),
                   EST_APPROX, SEED, payoffs=("forward",))
    X = out["XN_approx"]
    mse = float(normal.table_mse(q))
    _moment_check(X, (1 + p.r * h) ** N)
    _moment_check(X * X, ((1 + p.r * h) ** 2 + p.sigma ** 2 * h * (1 - mse)) ** N)


@pytest.mark.parametrize("scheme,rate", [("euler", 0.5), ("milstein", 1.0)])
def test_strong_rates(scheme, rate):
    p = Problem(scheme, **GBM)
    paths = np.arange(20_000, dtype=np.uint64)
    errs = []
    for level in (3, 4, 5, 6):
        out = simulate(p, level, paths, Precision(), EST_PLAIN, SEED, payoffs=("forward",))
        Z = normal.exact_normal(words_matrix(level, EST_PLAIN, paths))
        h = p.T / 2 ** level
        XT = np.exp((p.r - 0.5 * p.sigma ** 2) * p.T + p.sigma * math.sqrt(h) * Z.sum(axis=1))
        errs.append(math.sqrt(np.mean((out["XN_exact"] - XT) ** 2)))
    slope = -np.polyfit(np.arange(4), np.log2(errs), 1)[0]
    assert abs(slope - rate) < 0.15, (errs, slope)


def _telescoped(p, L, n, payoff):
    tot, var = 0.0, 0.0
    for l in range(L + 1):
        s = level_sums(p, l, n, 0, Precision(), EST_PLAIN, SEED, payoffs=(payoff,))[payoff]
        tot += s.mean()
        var += s.var() / s.n
        last = s.mean()
    sc = scale_price(p)
    return sc * tot, sc * math.sqrt(var), sc * abs(last)


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
def test_black_scholes_call(scheme):
    p = Problem(scheme, **GBM)
    est, se, lastmean = _telescoped(p, 6, 100_000, "euro")
    ref = bs_call(p.S0, p.K, p.r, p.sigma, p.T)
    assert abs(est - ref) < 4 * se + 2 * lastmean, (est, ref, se, lastmean)


def test_black_scholes_digital():
    p = Problem("milstein", **GBM)
    est, se, lastmean = _telescoped(p, 6, 100_000, "digital")
    ref = bs_digital(p.S0, p.K, p.r, p.sigma, p.T)
    assert abs(est - ref) < 4 * se + 2 * lastmean, (est, ref, se, lastmean)


@pytest.mark.parametrize("scheme,beta", [("euler", 1.0), ("milstein", 2.0)])
def test_variance_decay_beta(scheme, beta):
    p = Problem(scheme, **GBM)
    V = []
    for l in range(2, 7):
        s = level_sums(p, l, 40_000, 0, Precision(), EST_PLAIN, SEED, payoffs=("forward",))["forward"]
        V.append(s.var())
    slope = -np.polyfit(np.arange(2, 7), np.log2(V), 1)[0]
    assert abs(slope - beta) < 0.25, (V, slope)


def test_telescoping_identity_statistical():
    """sum_{l<=L} E[P_l - P_{l-1}] = E[P_L]: the telescoped sum of independent level
    estimators agrees with a direct estimate of E[P_L] (Section 2.1)."""
    p = Problem("euler", **GBM)
    L = 4
    est, se, _ = _telescoped(p, L, 100_000, "euro")
    out = simulate(p, L, np.arange(100_000, 200_000, dtype=np.uint64), Precision(), EST_PLAIN,
                   99, payoffs=("euro",))
    Pf = out["euro"]["Pf_exact"] * scale_price(p)
    se2 = Pf.std() / math.sqrt(Pf.size)
    assert abs(est - Pf.mean()) < 4 * math.sqrt(se * se + se2 * se2)


def test_nested_split_per_path():
    """Correction samples are exactly (exact dP) - (approx dP) on the same J (Section 2.2)."""
    p = Problem("milstein", **GBM)
    for level in (0, 3):
        out = simulate(p, level, np.arange(1000, dtype=np.uint64), Precision("fp32", 6),
                       EST_CORR, SEED, payoffs=("euro", "asian"))
        for n in ("euro", "asian"):
            r = out[n]
            assert np.array_equal(r["Y"], r["Y_exact"] - r["Y_approx"])
            assert r["Y_approx"].dtype == np.float64
