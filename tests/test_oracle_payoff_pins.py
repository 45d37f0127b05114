"""Pins for the oracle's Asian and barrier payoffs (reading R5 on the path's own
grid of Section 2.1), independent of the oracle's own formulas.

Deterministic pins drive the oracle's PathState with chosen normals:
* A worked example whose every grid value is a short dyadic fraction (r = 0,
  sigma = 1/2, h = 1, so con2 = 1/2 and each factor is 1 +- 1/4), so FP64, FP32,
  FP16 and wide fixed point all hold it exactly.  Its trapezoid averages and its
  barrier ties were worked out by hand (values below).
* Constant normals: every path is geometric, X_n = g^n, so the trapezoid average
  is the geometric sum (1 + g) (g^N - 1) / (2 N (g - 1)), the minimum is X_0
  (g > 1) or X_N (g < 1).
Statistical pins:
* E[A] from E[X_n] = (1 + r h)^n (Euler and Milstein, exact normals: E[Z] = 0,
  E[Z^2 - 1] = 0), fine and coarse.
* The down-and-out call monitored on the fine grid against the continuous
  closed form with the Broadie-Glasserman-Kou barrier shift B exp(-0.5826 sigma
  sqrt(T/m)) (a loose pin: the shift is itself an asymptotic correction).

Each pin fails for a dropped X_0 in the minimum, a '>=' knock-out test, or wrong
trapezoid end weights.
"""
from fractions import Fraction
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle.paths import (EST_PLAIN, PathState, Precision, Problem, level_constants,
                          make_side, simulate)

WIDE = (("X", 32, 29), ("con1", 32, 34), ("con2", 32, 33), ("con3", 32, 36),
        ("Z", 32, 28), ("mul1", 32, 30), ("sum1", 32, 30), ("zsq", 32, 23),
        ("zm1", 32, 23), ("mul3", 32, 29), ("sum2", 32, 29), ("mul2", 32, 27))
# formats for the worked example below (con2 = 1/2 needs two integer bits of con2)
EXFMT = tuple((v, 32, 28) if v != "X" else ("X", 32, 29) for v, _, _ in WIDE)
ARITHS = ("fp64", "fp32", "fp16", "fixed")


def _state(prob, level, arith, n, fmt=WIDE):
    prec = Precision(arith, 8, fmt=fmt) if arith == "fixed" else Precision(arith, 8)
    side = make_side(arith, prec, level_constants(prob, level), prob.scheme)
    return PathState(side, n, level)


def _z(side, z):
    """Normals in the side's storage (fixed: Z's format, f = 28)."""
    z = np.asarray(z, dtype=np.float64)
    if hasattr(side, "F"):
        f = side.F["Z"][1]
        q = np.rint(z * 2.0 ** f).astype(np.int64)
        assert np.array_equal(q * 2.0 ** -f, z)            # exactly representable
        return q
    return z.astype(side.t)


def _run(prob, level, arith, zs, fmt=EXFMT):
    """zs: (paths, 2^level) normals; returns the oracle's state after all steps."""
    zs = np.asarray(zs, dtype=np.float64)
    st = _state(prob, level, arith, zs.shape[0], fmt)
    for n in range(zs.shape[1]):
        st.fine(_z(st.side, zs[:, n]), n)
    return st


def _value(st, name):
    """(Y, Pf, Pc) of payoff `name` as FP64 values."""
    Y, Pf, Pc = st.level_diff(name)
    conv = st.side.to_f64
    return conv(Y), conv(Pf), conv(Pc)


# The worked example: level 2 (N = 4, h = T / 4 = 1), r = 0, sigma = 1/2, S0 = 1.
# Fine normals (-1/2, -1/2, +1/2, +1/2): factors 1 + Z/2 = 3/4, 3/4, 5/4, 5/4, so
#   X = 1, 3/4, 9/16, 45/64, 225/256;
#   trapezoid A_f = (1/4) [ (1 + 3/4)/2 + (3/4 + 9/16)/2 + (9/16 + 45/64)/2
#                          + (45/64 + 225/256)/2 ] = 1513/2048;
#   minimum (incl. X_0) = 9/16 at n = 2.
# Coarse: Zs = (-1, +1), step 2h with con1c = 0 and the same con2 = 1/2:
#   factors 1/2, 3/2, so Xc = 1, 1/2, 3/4; A_c = (1/2) [ (1 + 1/2)/2 + (1/2 + 3/4)/2 ]
#   = 11/16; minimum 1/2.
EX_Z = [[-0.5, -0.5, 0.5, 0.5]]
EX_XN, EX_XCN = Fraction(225, 256), Fraction(3, 4)
EX_AF, EX_AC = Fraction(1513, 2048), Fraction(11, 16)
EX_MINF, EX_MINC = Fraction(9, 16), Fraction(1, 2)


def _example(K, B):
    return Problem("euler", S0=1.0, K=K, r=0.0, sigma=0.5, T=4.0, barrier=B)


@pytest.mark.parametrize("arith", ARITHS)
def test_worked_example_paths_exact(arith):
    st = _run(_example(0.25, 0.0), 2, arith, EX_Z)
    conv = st.side.to_f64
    assert conv(st.Xf)[0] == float(EX_XN) and conv(st.Xc)[0] == float(EX_XCN)
    assert conv(st.min_f)[0] == float(EX_MINF) and conv(st.min_c)[0] == float(EX_MINC)
    if arith == "fixed":
        assert int(st.side.sat.sum()) == 0


@pytest.mark.parametrize("arith", ARITHS)
def test_worked_example_asian(arith):
    K = 0.25
    Y, Pf, Pc = _value(_run(_example(K, 0.0), 2, arith, EX_Z), "asian")
    assert Pf[0] == float(EX_AF - Fraction(1, 4))
    assert Pc[0] == float(EX_AC - Fraction(1, 4))
    assert Y[0] == float(EX_AF - EX_AC)


@pytest.mark.parametrize("arith", ARITHS)
def test_worked_example_barrier_ties_knock_out(arith):
    K = 0.25
    euro_f, euro_c = float(EX_XN - Fraction(1, 4)), float(EX_XCN - Fraction(1, 4))
    # barrier just below the fine minimum 9/16 (and above the coarse one, 1/2):
    # the fine path survives, the coarse path is knocked out
    _, Pf, Pc = _value(_run(_example(K, 0.5625 - 2 ** -10), 2, arith, EX_Z), "barrier")
    assert Pf[0] == euro_f and Pc[0] == 0.0
    # barrier equal to the fine minimum X_2 = 9/16: a tie knocks out
    _, Pf, _ = _value(_run(_example(K, 0.5625), 2, arith, EX_Z), "barrier")
    assert Pf[0] == 0.0
    # barrier equal to the coarse minimum 1/2 (a tie) and below the fine one
    _, Pf, Pc = _value(_run(_example(K, 0.5), 2, arith, EX_Z), "barrier")
    assert Pf[0] == euro_f and Pc[0] == 0.0
    # barrier just below the coarse minimum: both survive
    _, Pf, Pc = _value(_run(_example(K, 0.5 - 2 ** -10), 2, arith, EX_Z), "barrier")
    assert Pf[0] == euro_f and Pc[0] == euro_c


@pytest.mark.parametrize("arith", ARITHS)
def test_barrier_minimum_includes_x0(arith):
    """A rising path (every X_n > 1 for n >= 1) is knocked out by a barrier at
    X_0 = 1 (a tie at the start) and survives one just below it."""
    K = 0.25
    z = [[0.5, 0.5, 0.5, 0.5]]                      # factors 5/4: X_n = (5/4)^n
    XN, XcN = (Fraction(5, 4) ** 4, Fraction(3, 2) ** 2)
    _, Pf, Pc = _value(_run(_example(K, 1.0), 2, arith, z), "barrier")
    assert Pf[0] == 0.0 and Pc[0] == 0.0
    _, Pf, Pc = _value(_run(_example(K, 1.0 - 2 ** -10), 2, arith, z), "barrier")
    assert Pf[0] == float(XN - Fraction(1, 4)) and Pc[0] == float(XcN - Fraction(1, 4))


def _geometric_avg(g, N):
    """(1/N) sum_{n<N} (g^n + g^(n+1)) / 2 = (1 + g) (g^N - 1) / (2 N (g - 1))."""
    return (1.0 + g) * (g ** N - 1.0) / (2.0 * N * (g - 1.0))


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
@pytest.mark.parametrize("level", [1, 3, 6])
def test_constant_normals_geometric(scheme, level):
    """Constant normals z per path: X_n = g^n fine, (g_c)^m coarse (Zs = 2z), with
    g = 1 + r h + sigma sqrt(h) z (+ sigma^2 h (z^2 - 1) / 2, Milstein); the
    trapezoid average is the geometric sum and the minimum is X_0 or the end."""
    p = Problem(scheme, S0=100.0, K=1e-6, r=0.05, sigma=0.2, T=1.0, barrier=0.0)
    N = 1 << level
    h = p.T / N
    z = np.array([-1.7, -0.6, -0.05, 0.3, 1.1, 2.4])
    st = _run(p, level, "fp64", np.repeat(z[:, None], N, axis=1))
    k = p.K / p.S0
    g = 1 + p.r * h + p.sigma * math.sqrt(h) * z
    gc = 1 + p.r * 2 * h + p.sigma * math.sqrt(h) * (2 * z)
    if scheme == "milstein":
        g = g + 0.5 * p.sigma ** 2 * h * (z * z - 1)
        gc = gc + 0.5 * p.sigma ** 2 * h * ((2 * z) ** 2 - 2)
    Af, Ac = _geometric_avg(g, N), _geometric_avg(gc, N // 2)
    Y, Pf, Pc = _value(st, "asian")
    assert np.allclose(Pf, Af - k, rtol=1e-13, atol=0)
    assert np.allclose(Pc, Ac - k, rtol=1e-13, atol=0)
    assert np.allclose(st.min_f, np.minimum(1.0, g ** N), rtol=1e-13, atol=0)
    assert np.allclose(st.min_c, np.minimum(1.0, gc ** (N // 2)), rtol=1e-13, atol=0)


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
def test_constant_normals_barrier_geometric(scheme):
    """Falling paths (z < 0) have their minimum at X_N: a barrier just above X_N
    knocks out, just below it does not; rising paths (z > 0) are knocked out by a
    barrier at 1 (a tie with X_0) only."""
    level, N = 4, 16
    h = 1.0 / N
    z = np.array([-1.5, -0.8, 0.7, 1.9])
    sig, r = 0.2, 0.05
    g = 1 + r * h + sig * math.sqrt(h) * z
    if scheme == "milstein":
        g = g + 0.5 * sig ** 2 * h * (z * z - 1)
    XN = g ** N
    for j in range(len(z)):
        row = np.full((1, N), z[j])
        for B, alive in (((XN[j] * (1 + 1e-9) if z[j] < 0 else 1.0), False),
                         ((XN[j] * (1 - 1e-9) if z[j] < 0 else 1.0 - 1e-9), True)):
            p = Problem(scheme, S0=1.0, K=1e-6, r=r, sigma=sig, T=1.0, barrier=B)
            _, Pf, _ = _value(_run(p, level, "fp64", row), "barrier")
            assert (Pf[0] > 0) == alive, (z[j], B, Pf[0])
            if alive:
                assert abs(Pf[0] - (XN[j] - 1e-6)) <= 1e-13 * XN[j]


@pytest.mark.parametrize("scheme", ["euler", "milstein"])
def test_asian_mean_statistical(scheme):
    """E[A_f] and E[A_c] from E[X_n] = (1 + r h)^n (exact normals): the trapezoid
    weights in expectation; the level difference E[Y] from the two sums."""
    p = Problem(scheme, S0=100.0, K=1e-6, r=0.05, sigma=0.2, T=1.0, barrier=0.0)
    level, N = 2, 4
    h = p.T / N
    out = simulate(p, level, np.arange(200_000, dtype=np.uint64), Precision(), EST_PLAIN, 1234,
                   payoffs=("asian",))["asian"]
    k = p.K / p.S0
    Ef = _geometric_avg(1 + p.r * h, N) - k
    Ec = _geometric_avg(1 + p.r * 2 * h, N // 2) - k
    for x, e in ((out["Pf_exact"], Ef), (out["Pc_exact"], Ec), (out["Y"], Ef - Ec)):
        se = x.std() / math.sqrt(x.size)
        assert abs(x.mean() - e) < 4.5 * se, (x.mean(), e, se)
    # the pins separate: a mean over X_1..X_N instead of the trapezoid is far off
    wrong = (1 + p.r * h) * ((1 + p.r * h) ** N - 1) / (N * p.r * h) - k
    assert abs(Ef - wrong) > 10 * out["Pf_exact"].std() / math.sqrt(200_000)


def _bs_call(S, K, r, s, T):
    d1 = (math.log(S / K) + (r + 0.5 * s * s) * T) / (s * math.sqrt(T))
    return S * norm.cdf(d1) - K * math.exp(-r * T) * norm.cdf(d1 - s * math.sqrt(T))


def _down_out_call(S, K, B, r, s, T):
    """Continuously monitored down-and-out call, B <= K (Merton 1973 / Reiner-
    Rubinstein 1991): C - C_di, C_di = S (B/S)^(2 lam) N(y)
    - K e^{-rT} (B/S)^(2 lam - 2) N(y - s sqrt T), lam = (r + s^2/2) / s^2,
    y = ln(B^2 / (S K)) / (s sqrt T) + lam s sqrt T."""
    lam = (r + 0.5 * s * s) / (s * s)
    sq = s * math.sqrt(T)
    y = math.log(B * B / (S * K)) / sq + lam * sq
    di = S * (B / S) ** (2 * lam) * norm.cdf(y) - K * math.exp(-r * T) * (B / S) ** (2 * lam - 2) * norm.cdf(y - sq)
    return _bs_call(S, K, r, s, T) - di


def test_down_out_call_formula_limits():
    # a barrier far below the strike leaves the call; the survival factor is monotone
    assert abs(_down_out_call(100, 100, 1e-3, 0.05, 0.2, 1) - _bs_call(100, 100, 0.05, 0.2, 1)) < 1e-12
    vals = [_down_out_call(100, 100, B, 0.05, 0.2, 1) for B in (80, 85, 90, 95, 99)]
    assert all(a > b for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("B,level", [(95.0, 4), (90.0, 6)])
def test_barrier_price_bgk(B, level):
    """Down-and-out call on the fine grid of level l (m = 2^l monitoring dates plus
    X_0): within 4 SE plus a tenth of the monitoring correction of the continuous
    price at the shifted barrier B exp(-0.5826 sigma sqrt(T/m)), and above the
    continuous price at B (discrete monitoring knocks out less)."""
    p = Problem("milstein", S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, barrier=B)
    m = 1 << level
    out = simulate(p, level, np.arange(200_000, dtype=np.uint64), Precision(), EST_PLAIN, 1234,
                   payoffs=("barrier",))["barrier"]
    P = out["Pf_exact"] * p.S0 * math.exp(-p.r * p.T)
    se = P.std() / math.sqrt(P.size)
    cont = _down_out_call(p.S0, p.K, B, p.r, p.sigma, p.T)
    shifted = _down_out_call(p.S0, p.K, B * math.exp(-0.5826 * p.sigma * math.sqrt(p.T / m)), p.r,
                             p.sigma, p.T)
    assert abs(P.mean() - shifted) < 4 * se + 0.1 * (shifted - cont), (P.mean(), shifted, cont, se)
    assert P.mean() > cont + 10 * se
