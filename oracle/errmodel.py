"""Rounding-error model and bit-width optimisation (Sections 4-6).

Variables (the fixed-point kernel's per-variable formats, Algorithm 1 with the
Milstein extension R3): X, con1, con2, con3, Z, mul1, sum1, zsq, zm1, mul3, sum2,
mul2.  One level-l sample dP = P(X_N) - P(Xc_{N/2}) (level 0: P(X_1)) of the
European call P(x) = max(x - k, 0) has, per path, instances of each variable:
fine step n: mul1 = con2 Z_n, sum1 = con1 + mul1 (Milstein: zsq = Z_n Z_n,
zm1 = zsq - 1, mul3 = con3 zm1, sum2 = sum1 + mul3), mul2 = X_n s_n,
X_{n+1} = X_n + mul2; coarse step m the same on Zs_m = Z_2m + Z_2m+1 (exact) with
con1c (a second instance of con1) and 2 in zm1; the constants con1, con1c, con2,
con3 once each.  Z's instances are the fine normals.

* Sensitivities x_bar = d dP / d x of every instance by a reverse sweep of these
  operations (Section 4.2), on FP64 paths with exact normals.
* Exponents e: |x| < 2^e for every instance over the calibration paths
  (Section 4.1: the maximum absolute value); Z's from the table the kernel
  quantises (its largest |T_q[k]|).
* Per variable: S = sum over instances of E[x_bar^2] and R = sum over instances of
  sqrt(E[x_bar^2]);  V_indep(d) = (1/12) sum S 4^(e - d)  (eq. optimistic),
  V_corr(d) = (sum R 2^(e - d - 1))^2  (eq. pessimistic).  With approximate normals
  (eq. extended) the RNG term is S_Z * MSE in V'_indep and (R_Z sqrt(MSE))^2 inside
  V'_corr's square -- reading R16: without the printed 1/12, because the normal's
  error is not a uniform rounding error.  Simulation (the tests) puts the Euler
  correction samples within a factor 2 of this term and several times above the
  1/12 form; with Milstein and the table error dominant it is an upper estimate,
  since an error that moves close fine and coarse paths across the payoff's kink
  changes dP far less than the linearised sensitivities say.
* Cost (eq. cost_sq, the separable relaxation): C(d) = sum (1/2) M d^2 + M' d with M
  (M') the number of multiplications (additions) taking the variable as an operand
  per sample, counted on the kernel's operations: the fine step is the table's
  multiplier s_k times X and the add; the coarse step runs the whole chain.
* Optimisation (Section 6): for a multiplier lambda each d_i solves
  ln(4) (S_i / 12) 4^(e_i - d_i) = lambda (M_i d_i + M'_i)  (eq. Lagr, uncoupled);
  the level objective sqrt(V_l C(d)) + sqrt(V^D(d) C_l) (eq. level_cost2, V^D =
  V_indep or V'_indep, C_l = 2^l C_RNG) is minimised over log lambda by golden-section
  search on the bracket spanned by the lambdas of uniform widths 4..16 (the paper's
  scan), then the widths are rounded by the greedy ratio rule (eq. ratio_lagr).
* Formats for the kernel: w = d + 1, f = d - e (Section 4.1).

This module is test infrastructure: see the package docstring.
"""
from dataclasses import dataclass
import math

import numpy as np

from . import normal
from .philox import StepWords
from .paths import EST_CORR, Problem, level_constants

VARS = ("X", "con1", "con2", "con3", "Z", "mul1", "sum1", "zsq", "zm1", "mul3", "sum2", "mul2")
IX = {v: i for i, v in enumerate(VARS)}
MIL_ONLY = ("con3", "zsq", "zm1", "mul3", "sum2")


# widest formats of the int32 kernel: w = d + 1 <= 32 bits (Z: 31)
D_MAX = np.array([30 if v == "Z" else 31 for v in VARS], dtype=np.float64)


def used_vars(scheme):
    return [v for v in VARS if scheme == "milstein" or v not in MIL_ONLY]


@dataclass
class Model:
    S: np.ndarray          # per variable: sum over instances of E[x_bar^2]
    R: np.ndarray          # per variable: sum over instances of sqrt(E[x_bar^2])
    e: np.ndarray          # exponents (int)
    used: np.ndarray       # bool per variable
    V_level: float         # V[dP] on the exact paths
    mse: float             # Method-1 table MSE
    n_paths: int
    zbar: np.ndarray = None  # (N, P) dP / dZ_n per path, when asked for


def _exponent(maxabs):
    """Smallest integer e with |x| < 2^e (frexp: |x| = m 2^e, m in [1/2, 1))."""
    return int(math.frexp(maxabs)[1]) if maxabs > 0 else -1074


def sensitivities(prob: Problem, level, n_paths, q, seed, option=0, path_offset=0, keep_zbar=False):
    """Reverse sweep of the level-l sample on FP64 paths with exact normals from the
    correction estimator's stream.  Returns a Model."""
    assert prob.scheme in ("euler", "milstein")
    mil = prob.scheme == "milstein"
    c = level_constants(prob, level)
    con1, con1c, con2, con3, k = c.con1, c.con1c, c.con2, c.con3, c.k
    N = 1 << level
    paths = np.arange(path_offset, path_offset + n_paths, dtype=np.uint64)
    words = StepWords(seed, option, level, EST_CORR, paths)
    Z = np.stack([normal.exact_normal(words.word(n)) for n in range(N)])     # (N, P)
    maxabs = {v: 0.0 for v in VARS}

    def seen(v, a):
        maxabs[v] = max(maxabs[v], float(np.max(np.abs(a))))

    def chain(z, cc1, cz):
        """Multiplier chain on normal(s) z: returns dict of the intermediates."""
        d = {"mul1": con2 * z}
        d["sum1"] = cc1 + d["mul1"]
        if mil:
            d["zsq"] = z * z
            d["zm1"] = d["zsq"] - cz
            d["mul3"] = con3 * d["zm1"]
            d["sum2"] = d["sum1"] + d["mul3"]
            d["s"] = d["sum2"]
        else:
            d["s"] = d["sum1"]
        return d

    # forward: fine
    X = [np.ones(n_paths)]
    fine = []
    for n in range(N):
        ch = chain(Z[n], con1, 1.0)
        ch["mul2"] = X[-1] * ch["s"]
        X.append(X[-1] + ch["mul2"])
        fine.append(ch)
        for v in ("mul1", "sum1", "mul2") + (("zsq", "zm1", "mul3", "sum2") if mil else ()):
            seen(v, ch[v])
        seen("X", X[-1])
    # forward: coarse
    Xc = [np.ones(n_paths)]
    coarse = []
    if level >= 1:
        for m in range(N // 2):
            zs = Z[2 * m] + Z[2 * m + 1]
            ch = chain(zs, con1c, 2.0)
            ch["zs"] = zs
            ch["mul2"] = Xc[-1] * ch["s"]
            Xc.append(Xc[-1] + ch["mul2"])
            coarse.append(ch)
            for v in ("mul1", "sum1", "mul2") + (("zsq", "zm1", "mul3", "sum2") if mil else ()):
                seen(v, ch[v])
            seen("X", Xc[-1])
    for v, val in (("con1", con1), ("con2", con2)) + ((("con3", con3),) if mil else ()):
        seen(v, np.array([val]))
    if level >= 1:
        seen("con1", np.array([con1c]))
    Tq = normal.table_float(q, "float64")
    seen("Z", Tq)

    P = np.maximum(X[-1] - k, 0.0)
    dP = P - (np.maximum(Xc[-1] - k, 0.0) if level >= 1 else 0.0)
    inst = {v: [] for v in VARS}            # per-instance adjoint arrays (per path)

    def reverse(chs, Xs, zs, xbar_end):
        """Adjoints along one path (fine or coarse) from dP/dX_end: records every
        instance's adjoint in `inst`; returns the adjoint of the normal each step
        used and the constants' adjoints (con1 or con1c, con2, con3)."""
        zbar = [None] * len(chs)
        c1b = np.zeros(n_paths)
        c2b = np.zeros(n_paths)
        c3b = np.zeros(n_paths)
        xb = xbar_end
        for n in range(len(chs) - 1, -1, -1):
            ch = chs[n]
            inst["X"].append(xb)                          # X_{n+1}
            mul2b = xb                                    # X_{n+1} = X_n + mul2
            inst["mul2"].append(mul2b)
            sb = mul2b * Xs[n]                            # mul2 = X_n s_n
            xb_prev = xb + mul2b * ch["s"]
            zb = np.zeros(n_paths)
            if mil:
                inst["sum2"].append(sb)                   # sum2 = sum1 + mul3
                sum1b, mul3b = sb, sb
                inst["mul3"].append(mul3b)                # mul3 = con3 zm1
                c3b += mul3b * ch["zm1"]
                zm1b = mul3b * con3
                inst["zm1"].append(zm1b)                  # zm1 = zsq - c
                zsqb = zm1b
                inst["zsq"].append(zsqb)                  # zsq = z z
                zb += 2.0 * zs[n] * zsqb
            else:
                sum1b = sb
            inst["sum1"].append(sum1b)                    # sum1 = con1 + mul1
            c1b += sum1b
            mul1b = sum1b
            inst["mul1"].append(mul1b)                    # mul1 = con2 z
            c2b += mul1b * zs[n]
            zb += mul1b * con2
            zbar[n] = zb
            xb = xb_prev
        return zbar, c1b, c2b, c3b

    Pp = (X[-1] > k).astype(np.float64)
    zb_f, c1f, c2f, c3f = reverse(fine, X, [Z[n] for n in range(N)], Pp)
    Zbar = [zb_f[n].copy() for n in range(N)]
    con2b, con3b = c2f, c3f
    inst["con1"].append(c1f)
    if level >= 1:
        Ppc = -(Xc[-1] > k).astype(np.float64)
        zb_c, c1c, c2c, c3c = reverse(coarse, Xc, [ch["zs"] for ch in coarse], Ppc)
        for m in range(N // 2):                           # zs = Z_2m + Z_2m+1
            Zbar[2 * m] = Zbar[2 * m] + zb_c[m]
            Zbar[2 * m + 1] = Zbar[2 * m + 1] + zb_c[m]
        inst["con1"].append(c1c)                          # con1c: an instance of con1
        con2b, con3b = con2b + c2c, con3b + c3c
    inst["Z"].extend(Zbar)
    inst["con2"].append(con2b)
    if mil:
        inst["con3"].append(con3b)
    sens = inst
    S = np.zeros(len(VARS))
    R = np.zeros(len(VARS))
    for v, arrs in sens.items():
        for a in arrs:
            m2 = float(np.mean(a * a))
            S[IX[v]] += m2
            R[IX[v]] += math.sqrt(m2)
    used = np.array([v in used_vars(prob.scheme) for v in VARS])
    e = np.array([_exponent(maxabs[v]) if used[i] else 0 for i, v in enumerate(VARS)])
    return Model(S=S, R=R, e=e, used=used, V_level=float(np.var(dP, ddof=1)),
                 mse=float(normal.table_mse(q)), n_paths=n_paths,
                 zbar=np.stack(Zbar) if keep_zbar else None)


# ------------------------------------------------------------------ bounds
def v_indep(m: Model, d, rng=False):
    d = np.asarray(d, dtype=np.float64)
    v = float(np.sum(np.where(m.used, m.S * 4.0 ** (m.e - d), 0.0))) / 12.0
    return v + (m.S[IX["Z"]] * m.mse if rng else 0.0)


def v_corr(m: Model, d, rng=False):
    d = np.asarray(d, dtype=np.float64)
    s = float(np.sum(np.where(m.used, m.R * 2.0 ** (m.e - d - 1), 0.0)))
    if rng:
        s += m.R[IX["Z"]] * math.sqrt(m.mse)
    return s * s


# -------------------------------------------------------------------- cost
def op_counts(scheme, level):
    """(M, M'): per variable, multiplications / additions taking it as an operand,
    per sample, on the kernel's operations (fine: X s_k and the add; coarse: the
    whole chain on Zs)."""
    mil = scheme == "milstein"
    N = 1 << level
    Nc = N // 2 if level >= 1 else 0
    M = np.zeros(len(VARS))
    A = np.zeros(len(VARS))
    s = IX["sum2"] if mil else IX["sum1"]
    for steps in (N, Nc):                   # mul2 = X s ; X = X + mul2
        M[IX["X"]] += steps
        M[s] += steps
        A[IX["X"]] += steps
        A[IX["mul2"]] += steps
    # coarse chain: mul1 = con2 zs ; sum1 = con1 + mul1 (+ Milstein terms)
    M[IX["con2"]] += Nc
    M[IX["Z"]] += Nc                        # zs has Z's format (one more integer bit)
    A[IX["con1"]] += Nc
    A[IX["mul1"]] += Nc
    if mil:
        M[IX["Z"]] += 2 * Nc                # zsq = zs zs
        A[IX["zsq"]] += Nc                  # zm1 = zsq - 2
        M[IX["con3"]] += Nc
        M[IX["zm1"]] += Nc                  # mul3 = con3 zm1
        A[IX["sum1"]] += Nc
        A[IX["mul3"]] += Nc                 # sum2 = sum1 + mul3
    return M, A


def cost(M, A, d, used):
    d = np.asarray(d, dtype=np.float64)
    return float(np.sum(np.where(used, 0.5 * M * d * d + A * d, 0.0)))


# -------------------------------------------------------------- optimiser
@dataclass
class Optimum:
    d_real: np.ndarray
    d_int: np.ndarray
    lam: float
    objective: float
    objective_uniform: float
    best_uniform: int


def _solve_d(S, e, Mi, Ai, lam, lo=0.0, hi=31.0):
    """Root of ln4 (S/12) 4^(e-d) = lam (M d + M') in d on [lo, hi] (bisection);
    a variable that costs nothing (M = M' = 0: table-driven on the device) takes hi."""
    if Mi == 0 and Ai == 0:
        return hi
    f = lambda d: math.log(4.0) * S / 12.0 * 4.0 ** (e - d) - lam * (Mi * d + Ai)
    if f(lo) <= 0:
        return lo
    if f(hi) >= 0:
        return hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def widths_for(m: Model, M, A, lam):
    d = np.zeros(len(VARS))
    for i in range(len(VARS)):
        if m.used[i]:
            d[i] = _solve_d(m.S[i], m.e[i], M[i], A[i], lam, hi=D_MAX[i])
    return d


def level_objective(m: Model, M, A, d, C_l, rng):
    return math.sqrt(m.V_level * cost(M, A, d, m.used)) + math.sqrt(v_indep(m, d, rng) * C_l)


def uniform_lambda(m: Model, M, A, du):
    """The paper's lambda of a uniform width: sum dV/dd + lambda sum dC/dd = 0."""
    dV = -math.log(4.0) / 12.0 * np.sum(np.where(m.used, m.S * 4.0 ** (m.e - du), 0.0))
    dC = np.sum(np.where(m.used, M * du + A, 0.0))
    return -dV / dC


def golden_min(f, a, b, iters=200):
    """Golden-section search of a unimodal f on [a, b]."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(iters):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
    return 0.5 * (a + b)


def greedy_round(m: Model, M, A, d_real, rng):
    """Floor, then add one bit to the variables in decreasing order of the ratio
    (V(d*) - V(d* + e_i)) / (C(d* + e_i) - C(d*)) until V(d*) <= V(d_real)."""
    d = np.floor(d_real)
    target = v_indep(m, d_real, rng)
    ratios = []
    for i in range(len(VARS)):
        if not m.used[i] or d[i] >= D_MAX[i]:
            continue
        up = d.copy()
        up[i] += 1
        dv = v_indep(m, d, rng) - v_indep(m, up, rng)
        dc = cost(M, A, up, m.used) - cost(M, A, d, m.used)
        ratios.append((-(dv / dc) if dc > 0 else -math.inf, i))
    ratios.sort()
    for _, i in ratios:
        if v_indep(m, d, rng) <= target:
            break
        d[i] += 1
    return d.astype(np.int64)


def optimise(m: Model, scheme, level, c_rng=1e4, rng=False, uniform=range(4, 17)):
    """Section 6 for one level: returns an Optimum."""
    M, A = op_counts(scheme, level)
    C_l = (1 << level) * c_rng
    lams = [uniform_lambda(m, M, A, du) for du in uniform]
    lo, hi = math.log(min(lams)), math.log(max(lams))
    obj = lambda t: level_objective(m, M, A, widths_for(m, M, A, math.exp(t)), C_l, rng)
    t = golden_min(obj, lo, hi)
    lam = math.exp(t)
    d_real = widths_for(m, M, A, lam)
    d_int = greedy_round(m, M, A, d_real, rng)
    uni = [(level_objective(m, M, A, np.where(m.used, np.minimum(du, D_MAX), 0.0), C_l, rng), du)
           for du in uniform]
    best_u = min(uni)
    return Optimum(d_real=d_real, d_int=d_int, lam=lam, objective=obj(t),
                   objective_uniform=best_u[0], best_uniform=best_u[1])


def formats(m: Model, d):
    """(w, f) per variable from widths d: w = d + 1, f = d - e (Section 4.1)."""
    d = np.asarray(d, dtype=np.int64)
    return {v: (int(d[i]) + 1, int(d[i] - m.e[i])) for i, v in enumerate(VARS) if m.used[i]}


def kernel_formats(m: Model, d, scheme):
    """formats(m, d) brought into the fixed-point kernel's domain without adding
    rounding error: a result never keeps more fractional bits than its exact value
    has (product f_a + f_b, sum max(f_a, f_b)), two summands differ by at most 30
    fractional bits, zsq keeps at most 30, and words fit 32 bits (Z 31) -- a
    fractional bit above these limits rounds nothing; f is at least 0.  w follows f:
    w = f + e + 1."""
    F = {v: [w, f] for v, (w, f) in formats(m, d).items()}
    e = {v: int(m.e[IX[v]]) for v in F}
    mil = scheme == "milstein"

    def cap(v):
        F[v][1] = max(min(F[v][1], (30 if v == "Z" else 31) - e[v]), 0)
        F[v][0] = F[v][1] + e[v] + 1

    def prod(dst, a, b):
        F[dst][1] = min(F[dst][1], F[a][1] + F[b][1])
        cap(dst)

    def add(dst, a, b):
        hi, lo = (a, b) if F[a][1] >= F[b][1] else (b, a)
        if F[hi][1] - F[lo][1] > 30:
            F[hi][1] = F[lo][1] + 30
            cap(hi)
        F[dst][1] = min(F[dst][1], max(F[a][1], F[b][1]))
        cap(dst)

    for v in F:
        cap(v)
    for _ in range(3):
        prod("mul1", "con2", "Z")
        add("sum1", "con1", "mul1")
        s = "sum1"
        if mil:
            prod("zsq", "Z", "Z")
            F["zsq"][1] = min(F["zsq"][1], 30)
            cap("zsq")
            add("zm1", "zsq", "zsq")
            prod("mul3", "con3", "zm1")
            add("sum2", "sum1", "mul3")
            s = "sum2"
        prod("mul2", "X", s)
        add("X", "X", "mul2")
    return {v: (w, f) for v, (w, f) in F.items()}


# ------------------------------------------- the level's low-precision side (Section 6)
# Section 6 chooses, per level, the low-precision side that minimises the level
# objective sqrt(V~ C~) + sqrt(V^D C^D).  Here the candidates are the GPU's table
# sides and the cost of Section 5 is counted in issue cycles of the instruction
# classes the path kernels use (instructions per fine path-step over issue rates in
# wave-instructions per CU per clock) rather than in FPGA bit operations.
GPU_RATES = {"f32": 1.447, "i32": 1.470, "f64_fma": 0.794, "f64_add": 0.871, "u64_mad": 0.831,
             "lds_b64": 0.250, "lds_b32": 0.500}

SIDE_CANDIDATES = (("fp32", 8, True), ("fp32", 6, True), ("fp32", 4, True), ("fp32", 10, False),
                   ("fp32", 12, False), ("fp16", 8, True), ("fp16", 7, True), ("fp16", 10, False),
                   ("fixed", 8, False), ("fixed", 10, False), ("fixed", 12, False))


def side_instructions(arith, fields, scheme, level, estimator):
    """Instructions per fine path-step by class of one sample of the approximate
    (estimator 1) or correction (2) estimator with this table side."""
    mil = scheme == "milstein"
    n = {k: 0.0 for k in GPU_RATES}
    word_share = 1.0 / fields if estimator == 1 else 1.0
    n["u64_mad"] += 5 * word_share          # Philox4x32-10: 20 widening multiplies per 4 words
    n["i32"] += 7.5 * word_share             # and 30 xors / adds
    n["i32"] += 2.0 if (estimator == 1 and fields > 1) else 1.0     # table index
    half = 0.5 if level >= 1 else 0.0        # a coarse step per two fine steps
    if arith == "fixed":
        n["u64_mad"] += 1 + half * (4 if mil else 2)
        n["i32"] += 17 + half * (69 if mil else 35)
        n["lds_b64"] += 1
    else:
        n["f32"] += 2 + half * (9 if mil else 5)
        n["lds_b32" if arith == "fp16" else "lds_b64"] += 1
    if estimator == 2:
        n["f64_fma"] += 55 + (5 if mil else 2) + half * (9 if mil else 5)
        n["f64_add"] += 5 + 8.0 / 2 ** level
    else:
        n["f64_add"] += 4.0 / 2 ** level
    return n


def side_cost(arith, q, packed, scheme, level, estimator, rates=GPU_RATES):
    n = side_instructions(arith, 32 // q if packed else 1, scheme, level, estimator)
    return sum(n[k] / rates[k] for k in n)


def choose_side(m: Model, scheme, level, rates=GPU_RATES, fixed_d=None):
    """The candidate side with the least level objective (first in order on ties):
    V~ = V_level, V^D = v_indep(d) + S_Z MSE_q with d the significand bits (FP32 24,
    FP16 11) or the fixed widths fixed_d, C = 2^l side_cost.  Returns
    (arith, q, packed, objective, objective of FP32 q = 8 packed)."""
    best = None
    ref = None
    for arith, q, packed in SIDE_CANDIDATES:
        if arith == "fixed":
            if fixed_d is None:
                continue
            d = np.asarray(fixed_d, dtype=np.float64)
        else:
            d = np.full(len(VARS), 24.0 if arith == "fp32" else 11.0)
        vD = v_indep(m, d) + m.S[IX["Z"]] * float(normal.table_mse(q))
        cA = 2 ** level * side_cost(arith, q, packed, scheme, level, 1, rates)
        cC = 2 ** level * side_cost(arith, q, packed, scheme, level, 2, rates)
        obj = math.sqrt(m.V_level * cA) + math.sqrt(vD * cC)
        if ref is None:
            ref = obj
        if best is None or obj < best[3]:
            best = (arith, q, packed, obj)
    return best + (ref,)
