"""Coupled fine/coarse GBM paths and level differences (Sections 2.1-2.2, Algorithm 1).

SDE dS = a dt + b dW with GBM a = r S, b = sigma S (Algorithm 1).  Work is in
S0-normalised units X = S / S0 (reading R4; GBM is scale free), so X_0 = 1, the
strike is k = K / S0 and the barrier b = B / S0; prices are scaled back by S0.

Level l: h = 2^-l T, N = 2^l fine steps.

Fine step, Euler-Maruyama in Algorithm 1's order:
    mul1 = con2 * Z,  sum1 = con1 + mul1,  mul2 = X * sum1,  X <- X + mul2,
    con1 = r h, con2 = sqrt(h) sigma.
Fine step, Milstein (reading R3; the paper names Milstein only in its conclusion):
    mul1 = con2 * Z, zsq = Z * Z, zm1 = zsq - 1, mul3 = con3 * zm1,
    sum1 = con1 + mul1, sum2 = sum1 + mul3, mul2 = X * sum2, X <- X + mul2,
    con3 = sigma^2 h / 2.
Coarse step (l >= 1, reading R2): the coarse path of Section 2.1 freezes drift and
volatility over each pair of fine steps; the two sub-steps add up to one step of
size 2h driven by Zs = Z_2m + Z_2m+1, so it is computed as one step with
con1c = r 2h, the same con2 and con3, Zs in place of Z and (Milstein) zm1 = zsq - 2.
Level 0: one step of size T, no coarse path, Delta P_0 = P_0 (convention P_-1 = 0).

Arithmetic of a side (one path generator):
* 'fp64' / 'fp32' / 'fp16': every operation above is rounded to that IEEE type
  (numpy performs each elementwise operation in the type; no fusion).
* 'fixed': every variable has its own (w, f); each operation is an exact integer
  operation rounded once to the destination's f (R7) and saturated (R8).  Zs keeps
  Z's f with one extra integer bit (exact).
Constants con1, con1c, con2, con3, k, b are computed in FP64 in the order written
(con2 = sigma * sqrt(h), con3 = ((0.5 * sigma) * sigma) * h) and rounded once to
the side's type (reading: constants are prepared off the low-precision device).

Normals of a side: 'exact' = Phi^-1(U) (FP64, rounded to the side type), or
'table' = Method-1 table T_q (Section 3.1) stored in the side type.

Payoffs (the paper uses only the European call; the others are reading R5), on
the path's own grid X_0..X_N:
  forward  P = X_N                        euro     P = max(X_N - k, 0)
  asian    A = (1/N) sum_{n<N} (X_n + X_{n+1})/2,  P = max(A - k, 0)
  barrier  P = max(X_N - k, 0) if min_n X_n > b else 0   (down-and-out)
  digital  P = k if X_N > k else 0                (cash-or-nothing paying K)
Discounting e^{-rT} is applied once to the level sums (R5a), not here.

Estimators (Section 2.2):
  plain (0)       Y = P_f - P_c on the exact side.
  approx (1)      Y~ = P~_f - P~_c on the low-precision side with table normals.
  correction (2)  Y_D = (P_f - P_c) - Y~ with both sides driven by the same J.
The correction's exact side is FP64 with FP64 normals (reading R21: the paper's
"double" increment), or, with Precision.exact = 'fp32', FP32 arithmetic with the
exact normal rounded to FP32 (the narrower reading: FP64 only for the sums).

This module is test infrastructure: see the package docstring.
"""
from dataclasses import dataclass, field
import math

import mpmath
import numpy as np

from . import fixedpoint as fx
from . import normal
from .philox import StepWords, stream_words
from . import rngmethods

PAYOFFS = ("forward", "euro", "asian", "barrier", "digital")
EST_PLAIN, EST_APPROX, EST_CORR = 0, 1, 2

# fixed-point variables of the low-precision path (Algorithm 1 + Milstein)
FIXED_VARS = ("X", "con1", "con2", "con3", "Z", "mul1", "sum1",
              "zsq", "zm1", "mul3", "sum2", "mul2")


@dataclass(frozen=True)
class Problem:
    scheme: str          # 'euler' | 'milstein'
    S0: float
    K: float
    r: float
    sigma: float
    T: float
    barrier: float = 0.0


@dataclass(frozen=True)
class Precision:
    """Arithmetic of the low-precision side.  fmt: var -> (w, f) for 'fixed'."""
    arith: str = "fp32"          # fp64 | fp32 | fp16 | fixed
    q: int = 8                   # table bits (d of Section 3)
    packed: bool = False         # approx estimator: floor(32/q) indices per word
    fmt: tuple = ()              # tuple of (var, w, f) for 'fixed'
    method: int = 1              # approximate normals: Method 1, 2 (n = 2) or 3
    exact: str = "fp64"          # correction estimator's exact side: fp64 or fp32 (R21)

    def fmt_of(self, var):
        for v, w, f in self.fmt:
            if v == var:
                return w, f
        raise KeyError(var)


@dataclass
class Constants:
    """FP64 constants of a level (before rounding to a side)."""
    h: float
    con1: float
    con1c: float
    con2: float
    con3: float
    k: float
    b: float


def level_constants(prob: Problem, level: int) -> Constants:
    h = prob.T / float(1 << level)
    return Constants(h=h, con1=prob.r * h, con1c=prob.r * (2.0 * h),
                     con2=prob.sigma * math.sqrt(h),
                     con3=((0.5 * prob.sigma) * prob.sigma) * h,
                     k=prob.K / prob.S0, b=prob.barrier / prob.S0)


# --------------------------------------------------------------------- sides
class FloatSide:
    """Path arithmetic in one IEEE type; each operation is rounded to it."""

    def __init__(self, dtype, c: Constants, scheme):
        self.t = np.dtype(dtype).type
        t = self.t
        self.con1, self.con1c, self.con2, self.con3 = (t(c.con1), t(c.con1c),
                                                       t(c.con2), t(c.con3))
        self.k, self.b = t(c.k), t(c.b)
        self.one, self.two, self.zero, self.half = t(1), t(2), t(0), t(0.5)
        self.milstein = scheme == "milstein"
        self.sat = None

    def x0(self, n):
        return np.full(n, self.one, dtype=self.t)

    def mul(self, a, b, *_):
        return (a * b).astype(self.t)

    def add(self, a, b, *_):
        return (a + b).astype(self.t)

    def sub(self, a, b, *_):
        return (a - b).astype(self.t)

    def step(self, X, Z, coarse):
        con1 = self.con1c if coarse else self.con1
        mul1 = self.mul(self.con2, Z)
        s = self.add(con1, mul1)
        if self.milstein:
            zsq = self.mul(Z, Z)
            zm1 = self.sub(zsq, self.two if coarse else self.one)
            mul3 = self.mul(self.con3, zm1)
            s = self.add(s, mul3)
        mul2 = self.mul(X, s)
        return self.add(X, mul2)

    def zsum(self, za, zb):
        return self.add(za, zb)

    # payoff helpers
    def acc_init(self, n):
        return np.zeros(n, dtype=self.t)

    def acc_add(self, acc, X):
        return self.add(acc, X)

    def asian_avg(self, acc, X0, XN, log2n):
        t = self.sub(acc, self.mul(self.half, XN))
        t = self.add(t, self.mul(self.half, X0))
        return self.mul(t, self.t(2.0 ** -log2n))

    def relu_minus_k(self, A):
        return np.maximum(self.sub(A, self.k), self.zero)

    def digital(self, XN):
        return np.where(XN > self.k, self.k, self.zero).astype(self.t)

    def diff(self, Pf, Pc):
        return self.sub(Pf, Pc)

    def to_f64(self, Y):
        return np.asarray(Y, dtype=np.float64)


class FixedSide:
    """Path arithmetic in fixed point: every variable has its own (w, f)."""

    def __init__(self, prec: Precision, c: Constants, scheme):
        self.F = {v: (w, f) for v, w, f in prec.fmt}
        self.milstein = scheme == "milstein"
        wX, fX = self.F["X"]
        q = lambda x, var: fx.quantize_double(x, self.F[var][1], self.F[var][0])
        self.con1 = q(c.con1, "con1")
        self.con1c = q(c.con1c, "con1")
        self.con2 = q(c.con2, "con2")
        if self.milstein:
            self.con3 = q(c.con3, "con3")
        self.k = q(c.k, "X")
        self.b = q(c.b, "X")
        self.sat = None

    def _count(self, s):
        self.sat = s if self.sat is None else self.sat + s

    def x0(self, n):
        return np.full(n, 1 << self.F["X"][1], dtype=np.int64)

    def op(self, kind, a, fa, b, fb, dst):
        wd, fd = self.F[dst]
        if kind == "mul":
            v, s = fx.mul(a, fa, b, fb, fd, wd)
        else:
            v, s = fx.add(a, fa, b, fb, fd, wd, sub=(kind == "sub"))
        self._count(s)
        return v

    def step(self, X, Z, coarse):
        F = self.F
        fZ = F["Z"][1]
        con1 = self.con1c if coarse else self.con1
        mul1 = self.op("mul", self.con2, F["con2"][1], Z, fZ, "mul1")
        s = self.op("add", con1, F["con1"][1], mul1, F["mul1"][1], "sum1")
        sname = "sum1"
        if self.milstein:
            zsq = self.op("mul", Z, fZ, Z, fZ, "zsq")
            fq = F["zsq"][1]
            c = (2 if coarse else 1) << fq          # the constant 1 or 2, exact in zsq's f
            zm1 = self.op("sub", zsq, fq, c, fq, "zm1")
            mul3 = self.op("mul", self.con3, F["con3"][1], zm1, F["zm1"][1], "mul3")
            s = self.op("add", s, F["sum1"][1], mul3, F["mul3"][1], "sum2")
            sname = "sum2"
        mul2 = self.op("mul", X, F["X"][1], s, F[sname][1], "mul2")
        return self.op("add", X, F["X"][1], mul2, F["mul2"][1], "X")

    def zsum(self, za, zb):
        # exact: Zs has Z's f and one more integer bit (R2)
        return np.asarray(za, dtype=np.int64) + np.asarray(zb, dtype=np.int64)

    def acc_init(self, n):
        return np.zeros(n, dtype=np.int64)

    def acc_add(self, acc, X):
        return acc + X                       # exact (int64; N <= 2^20 terms of < 2^31)

    def asian_avg(self, acc, X0, XN, log2n):
        # 2 * trapezoid sum = 2 acc - X_N + X_0 exactly; A = that / 2^(log2n + 1), R7
        s2 = 2 * acc - XN + X0
        A = fx.round_shift(s2, log2n + 1)
        A, s = fx.saturate(A, self.F["X"][0])
        self._count(s)
        return A

    def relu_minus_k(self, A):
        return np.maximum(A - self.k, 0)     # exact in X's format (one more bit)

    def digital(self, XN):
        return np.where(XN > self.k, self.k, 0).astype(np.int64)

    def diff(self, Pf, Pc):
        return Pf - Pc                        # exact int64

    def to_f64(self, Y):
        return np.asarray(Y, dtype=np.float64) * 2.0 ** -self.F["X"][1]


def make_side(arith, prec, c, scheme):
    if arith == "fixed":
        return FixedSide(prec, c, scheme)
    return FloatSide({"fp64": np.float64, "fp32": np.float32, "fp16": np.float16}[arith],
                     c, scheme)


# ------------------------------------------------------------------ normals
def method_values(prec):
    """FP64 table values of Method 2 or 3 (Section 3.2, 3.3) and Method 2's
    permutation (None otherwise)."""
    if prec.method == 2:
        return rngmethods.method2_table(prec.q, 2)
    if prec.method == 3:
        return rngmethods.method3_table(prec.q), None
    raise ValueError(prec.method)


def side_table(side, prec):
    """The table of approximate normals in the side's storage format: Method 1's
    exact values rounded once; Methods 2 and 3 their FP64 values rounded once."""
    if prec.method == 1:
        if isinstance(side, FixedSide):
            return normal.table_fixed(prec.q, side.F["Z"][1])
        return normal.table_float(prec.q, np.dtype(side.t).name)
    vals, _ = method_values(prec)
    if isinstance(side, FixedSide):
        f = side.F["Z"][1]
        return np.array([normal.round_fixed(mpmath.mpf(float(v)), f) for v in vals], dtype=np.int64)
    return vals.astype(side.t)


# ------------------------------------------------------------------- paths
class PathState:
    """Fine and coarse state of one side plus the payoff functionals."""

    def __init__(self, side, n, level):
        self.side, self.level = side, level
        self.Xf = side.x0(n)
        self.Xc = side.x0(n)
        self.X0 = side.x0(n)
        self.acc_f, self.acc_c = side.acc_init(n), side.acc_init(n)
        self.min_f, self.min_c = self.Xf.copy(), self.Xc.copy()
        self.zprev = None

    def fine(self, Z, n):
        s = self.side
        self.Xf = s.step(self.Xf, Z, coarse=False)
        self.acc_f = s.acc_add(self.acc_f, self.Xf)
        self.min_f = np.minimum(self.min_f, self.Xf)
        if self.level >= 1:
            if n % 2 == 0:
                self.zprev = Z
            else:
                Zs = s.zsum(self.zprev, Z)
                self.Xc = s.step(self.Xc, Zs, coarse=True)
                self.acc_c = s.acc_add(self.acc_c, self.Xc)
                self.min_c = np.minimum(self.min_c, self.Xc)

    def payoff(self, name, XN, acc, mn, log2n):
        s = self.side
        if name == "forward":
            return XN
        if name == "euro":
            return s.relu_minus_k(XN)
        if name == "asian":
            return s.relu_minus_k(s.asian_avg(acc, self.X0, XN, log2n))
        if name == "barrier":
            e = s.relu_minus_k(XN)
            return np.where(mn > s.b, e, np.zeros_like(e))
        if name == "digital":
            return s.digital(XN)
        raise ValueError(name)

    def level_diff(self, name):
        """Y = P_f - P_c in the side's arithmetic (P_c = 0 on level 0)."""
        l = self.level
        Pf = self.payoff(name, self.Xf, self.acc_f, self.min_f, l)
        if l == 0:
            return self.side.diff(Pf, np.zeros_like(Pf)), Pf, np.zeros_like(Pf)
        Pc = self.payoff(name, self.Xc, self.acc_c, self.min_c, l - 1)
        return self.side.diff(Pf, Pc), Pf, Pc


def simulate(prob: Problem, level: int, paths, prec: Precision, estimator: int,
             seed: int, option: int = 0, payoffs=("euro",), plain_arith="fp64"):
    """Simulate the given path indices of one (level, estimator) sample set.

    Returns a dict with, per payoff name, 'Y' (FP64 per path, the estimator's
    sample) and the side results; plus 'sat' (fixed-point saturations per path)
    and the terminal values.
    """
    paths = np.asarray(paths, dtype=np.uint64)
    n = paths.size
    c = level_constants(prob, level)
    N = 1 << level
    words = StepWords(seed, option, level, estimator, paths)

    exact_side = approx_side = None
    if estimator in (EST_PLAIN, EST_CORR):
        exact_side = PathState(make_side(plain_arith if estimator == EST_PLAIN else prec.exact,
                                         prec, c, prob.scheme), n, level)
    if estimator in (EST_APPROX, EST_CORR):
        approx_side = PathState(make_side(prec.arith, prec, c, prob.scheme), n, level)
        table = side_table(approx_side.side, prec)

    packed = prec.packed and estimator == EST_APPROX
    perm = None
    if estimator == EST_CORR and prec.method == 2:
        perm = method_values(prec)[1]
    for step in range(N):
        if packed:
            idx = words.packed_index(step, prec.q)
        else:
            J = words.word(step)
            idx = normal.table_index(J, prec.q)
        if exact_side is not None:
            # Method 2 couples the exact side to the permuted interval pi(j)
            Z = normal.exact_normal(J if perm is None else rngmethods.coupled_words(J, prec.q, perm))
            exact_side.fine(Z.astype(exact_side.side.t), step)
        if approx_side is not None:
            approx_side.fine(table[idx], step)

    out = {"n": n}
    for name in payoffs:
        res = {}
        if exact_side is not None:
            Ye, Pf, Pc = exact_side.level_diff(name)
            res["Y_exact"] = exact_side.side.to_f64(Ye)
            res["Pf_exact"], res["Pc_exact"] = Pf, Pc
        if approx_side is not None:
            Ya, Pf, Pc = approx_side.level_diff(name)
            res["Y_approx_raw"] = Ya
            res["Y_approx"] = approx_side.side.to_f64(Ya)
            res["Pf_approx"], res["Pc_approx"] = Pf, Pc
        if estimator == EST_PLAIN:
            res["Y"] = res["Y_exact"]
        elif estimator == EST_APPROX:
            res["Y"] = res["Y_approx"]
        else:
            res["Y"] = res["Y_exact"] - res["Y_approx"]
        out[name] = res
    if exact_side is not None:
        out["XN_exact"], out["XcN_exact"] = exact_side.Xf, exact_side.Xc
        out["min_exact"], out["minc_exact"] = exact_side.min_f, exact_side.min_c
    if approx_side is not None:
        out["XN_approx"], out["XcN_approx"] = approx_side.Xf, approx_side.Xc
        out["min_approx"], out["minc_approx"] = approx_side.min_f, approx_side.min_c
        sat = approx_side.side.sat
        out["sat"] = np.zeros(n, np.int64) if sat is None else sat
    return out
