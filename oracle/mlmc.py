"""Per-level sums, estimators, sample allocation and the adaptive MLMC driver.

Section 2.1: E[P_L] = sum_l E[P_l - P_{l-1}], level l estimated from N_l samples;
Cost = sum N_l C_l, Variance = sum V_l / N_l; minimising cost at variance eps^2
gives N_l = lambda sqrt(V_l / C_l), lambda = eps^-2 sum_k sqrt(V_k C_k).

Section 2.2 (nested): each level splits into E[dP~_l] (N~_l samples, cost C~_l)
and E[dP_l - dP~_l] (N^D_l samples, cost C^D_l = C_l + C~_l), with
N~_l = lambda_M sqrt(V~_l / C~_l), N^D_l = lambda_M sqrt(V^D_l / C^D_l),
lambda_M = eps^-2 sum_k (sqrt(V~_k C~_k) + sqrt(V^D_k C^D_k)).

Readings:
* R9  variance estimate v = (S2 - S1^2 / n) / (n - 1).
* R10 N_l = ceil(theta^-1 * (formula above)): theta = 1 is Section 2.1 exactly
  (variance eps^2); theta = 1/2 splits eps^2 between variance and squared bias as
  in the adaptive algorithm of Giles (2008) that Section 6 says is used on-line.
* R11 costs: C_l = 2^l c with a per-estimator constant c (Section 5's CPU model
  C_l ~ 2^l C_RNG), never live timings.
* R13 eps is on the S0-normalised price unless eps_units = 'absolute'.
* R5a prices are e^{-rT} S0 times the sum of level means.
* R34 bias test: the remaining bias is estimated from the last three correction
  levels, max over l = max(1, L-2) .. L of |mean_l| 2^(alpha (l - L)) / (2^alpha - 1)
  (Giles' published MLMC test; a single noisy level mean stops too early), with
  alpha = 1, the weak order of both schemes (Section 2.1), rather than a rate fitted
  to two or three noisy level means, which can come out far too large.
* R35 per-level estimator (nested runs): once a level's pilot has landed, the level
  keeps the nested pair only if its cost at the optimum is below the plain
  estimator's, (sqrt(V~ c~) + sqrt(V^D c^D))^2 <= V~ c_plain (Section 6's level
  objective with the plain estimator as the full-precision alternative and V~ as
  its variance); otherwise its approximate and correction samples are dropped and
  it continues with plain samples.  A new level above a plain level l >= 1 starts
  plain.  (Discontinuous payoffs: a table error that moves a path across the
  jump makes V^D as large as V~, and the nested pair costs more than plain.)

This module is test infrastructure: see the package docstring.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from .paths import EST_APPROX, EST_CORR, EST_PLAIN, Problem, Precision, simulate


@dataclass
class Sums:
    n: int = 0
    s1: float = 0.0
    s2: float = 0.0
    i1: int = 0            # exact integer sums (fixed-point approx estimator)
    i2: int = 0
    e1: float = 0.0        # sums of dP on the exact side (correction estimator)
    e2: float = 0.0
    sat: int = 0

    def add(self, other):
        self.n += other.n
        self.s1 += other.s1
        self.s2 += other.s2
        self.i1 += other.i1
        self.i2 += other.i2
        self.e1 += other.e1
        self.e2 += other.e2
        self.sat += other.sat

    def mean(self):
        return self.s1 / self.n if self.n else 0.0

    def var(self):
        """R9."""
        if self.n < 2:
            return 0.0
        return max((self.s2 - self.s1 * self.s1 / self.n) / (self.n - 1), 0.0)


def level_sums(prob: Problem, level, n_paths, path_offset, prec: Precision, estimator,
               seed, option=0, payoffs=("euro",), plain_arith="fp64", chunk=1 << 16):
    """(n, sum Y, sum Y^2) of one (level, estimator) over paths
    [path_offset, path_offset + n_paths).  FP64 sums are correctly rounded
    (math.fsum); fixed-point approx sums are also kept as exact integers."""
    acc = {p: [] for p in payoffs}
    ints = {p: [0, 0] for p in payoffs}
    ex = {p: [] for p in payoffs}
    sat = 0
    for start in range(path_offset, path_offset + n_paths, chunk):
        stop = min(start + chunk, path_offset + n_paths)
        out = simulate(prob, level, np.arange(start, stop, dtype=np.uint64), prec,
                       estimator, seed, option, payoffs, plain_arith)
        if "sat" in out:
            sat += int(out["sat"].sum())
        for p in payoffs:
            acc[p].append(out[p]["Y"])
            if estimator == EST_APPROX and prec.arith == "fixed":
                Yi = [int(v) for v in out[p]["Y_approx_raw"]]
                ints[p][0] += sum(Yi)
                ints[p][1] += sum(v * v for v in Yi)
            if estimator == EST_CORR:
                ex[p].append(out[p]["Y_exact"])
    res = {}
    for p in payoffs:
        Y = np.concatenate(acc[p]) if acc[p] else np.zeros(0)
        s = Sums(n=int(Y.size), s1=math.fsum(Y), s2=math.fsum(Y * Y),
                 i1=ints[p][0], i2=ints[p][1], sat=sat)
        if ex[p]:
            E = np.concatenate(ex[p])
            s.e1, s.e2 = math.fsum(E), math.fsum(E * E)
        res[p] = s
    return res


# ---------------------------------------------------------------- allocation
def optimal_samples(V, C, eps2, theta=1.0):
    """Section 2.1: N_l = ceil(theta^-1 eps^-2 sqrt(V_l/C_l) sum_k sqrt(V_k C_k))."""
    V, C = np.asarray(V, float), np.asarray(C, float)
    lam = np.sum(np.sqrt(V * C)) / (theta * eps2)
    return np.ceil(lam * np.sqrt(V / C)).astype(np.int64)


def nested_samples(Vt, Ct, Vd, Cd, eps2, theta=1.0):
    """Section 2.2: N~_l, N^D_l with the common multiplier lambda_M."""
    Vt, Ct, Vd, Cd = (np.asarray(a, float) for a in (Vt, Ct, Vd, Cd))
    lam = (np.sum(np.sqrt(Vt * Ct)) + np.sum(np.sqrt(Vd * Cd))) / (theta * eps2)
    return (np.ceil(lam * np.sqrt(Vt / Ct)).astype(np.int64),
            np.ceil(lam * np.sqrt(Vd / Cd)).astype(np.int64))


def mlmc_cost(V, C, eps2):
    """Section 2.1, total cost eps^-2 (sum sqrt(V C))^2 (real-valued N)."""
    return float(np.sum(np.sqrt(np.asarray(V) * np.asarray(C)))) ** 2 / eps2


# ------------------------------------------------------------------ adaptive
@dataclass
class RunConfig:
    eps: float = 1e-3
    eps_units: str = "normalised"     # R13
    theta: float = 0.5                # R10
    L_min: int = 2
    L_max: int = 10
    n_pilot: int = 10_000             # R12
    nested: bool = True
    cost_plain: float = 1.0           # R11: cost per fine step
    cost_approx: float = 0.1
    cost_corr: float = 1.1
    plain_arith: str = "fp32"


@dataclass
class Result:
    estimate: float
    variance: float
    L: int
    sums: dict = field(default_factory=dict)     # (level, estimator) -> Sums
    sweeps: int = 0


WEAK_ORDER = 1.0      # alpha: weak order of the Euler and Milstein schemes (Section 2.1)


def remaining_bias(means):
    """R34: max over l = max(1, L-2) .. L of |mean_l| 2^(alpha (l - L)) / (2^alpha - 1)
    with alpha = WEAK_ORDER (L = 0: |mean_0| / (2^alpha - 1))."""
    L = len(means) - 1
    a = WEAK_ORDER
    lo = max(1, L - 2) if L >= 1 else 0
    return max(abs(means[l]) * 2.0 ** (a * (l - L)) for l in range(lo, L + 1)) / (2.0 ** a - 1.0)


def estimate(prob: Problem, payoff, prec: Precision, cfg: RunConfig, seed, option=0):
    """Adaptive (nested) MLMC in the manner of Giles (2008): pilot, allocation,
    sweeps of extra samples, then a bias test that may add a level (R10, R34, R35)."""
    scale = math.exp(-prob.r * prob.T) * (prob.S0 if cfg.eps_units == "absolute" else 1.0)
    eps = cfg.eps / scale                      # target on the normalised sums
    nested = (EST_APPROX, EST_CORR)
    cost = {EST_PLAIN: cfg.cost_plain, EST_APPROX: cfg.cost_approx, EST_CORR: cfg.cost_corr}
    sums = {}
    L = cfg.L_min
    ests = {l: nested if cfg.nested else (EST_PLAIN,) for l in range(L + 1)}
    decided = set()

    def run(level, est, n):
        s = sums.setdefault((level, est), Sums())
        got = level_sums(prob, level, n, s.n, prec, est, seed, option, (payoff,),
                         cfg.plain_arith)[payoff]
        s.add(got)

    for l in range(L + 1):
        for e in ests[l]:
            run(l, e, cfg.n_pilot)
    sweeps = 0
    while True:
        sweeps += 1
        V = {k: max(s.var(), 1e-300) for k, s in sums.items()}
        if cfg.nested:                             # R35, once per level
            switched = False
            for l in range(L + 1):
                if l in decided:
                    continue
                decided.add(l)
                if ests[l] != nested:
                    continue
                Va, Vc = V[(l, EST_APPROX)], V[(l, EST_CORR)]
                root = math.sqrt(Va * cost[EST_APPROX]) + math.sqrt(Vc * cost[EST_CORR])
                if root * root > Va * cost[EST_PLAIN]:
                    ests[l] = (EST_PLAIN,)
                    del sums[(l, EST_APPROX)], sums[(l, EST_CORR)]
                    run(l, EST_PLAIN, cfg.n_pilot)
                    switched = True
            if switched:
                continue
        # Sections 2.1/2.2: one multiplier over every (level, estimator) in use
        # (the formula of optimal_samples, summed in this order: level, then estimator)
        keys = [(l, e) for l in range(L + 1) for e in ests[l]]
        lam = 0.0
        for (l, e) in keys:
            lam += math.sqrt(V[(l, e)] * cost[e] * 2.0 ** l)
        lam /= cfg.theta * eps * eps
        Nk = [math.ceil(lam * math.sqrt(V[(l, e)] / (cost[e] * 2.0 ** l))) for (l, e) in keys]
        extra = {k: int(t) - sums[k].n for k, t in zip(keys, Nk) if t > sums[k].n}
        if extra:
            for (l, e), dn in sorted(extra.items()):
                run(l, e, dn)
            continue
        means = [sum(sums[(l, e)].mean() for e in ests[l]) for l in range(L + 1)]
        if remaining_bias(means) > math.sqrt(1 - cfg.theta) * eps and L < cfg.L_max:
            L += 1
            plain_above = cfg.nested and L - 1 >= 1 and ests[L - 1] == (EST_PLAIN,)
            ests[L] = (EST_PLAIN,) if (plain_above or not cfg.nested) else nested
            if plain_above:
                decided.add(L)
            for e in ests[L]:
                run(L, e, cfg.n_pilot)
            continue
        break
    est = scale_price(prob) * sum(sums[(l, e)].mean() for l in range(L + 1) for e in ests[l])
    var = scale_price(prob) ** 2 * sum(sums[(l, e)].var() / sums[(l, e)].n
                                       for l in range(L + 1) for e in ests[l])
    return Result(estimate=est, variance=var, L=L, sums=sums, sweeps=sweeps)


def scale_price(prob: Problem):
    """Normalised, undiscounted level sums -> price: e^{-rT} S0 (R4, R5a)."""
    return math.exp(-prob.r * prob.T) * prob.S0
