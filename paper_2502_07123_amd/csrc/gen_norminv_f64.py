"""Generate the FP64 inverse-normal coefficients of the exact side (the Z of the
coupled pair (Z, Z~), Section 3.1).

Method: the variable change of M. Giles, "Approximating the erfinv function"
(GPU Computing Gems, 2011).  With y = 2u - 1 and w = -log(1 - y^2) = -log(4u(1-u)),
Phi^-1(u) = y * P(w) on the central range w < W1 -- which holds for all but about
1e-3 of the inputs, so almost every wave runs a single branch with no division --
and Phi^-1(u) = sign(y) * Q(sqrt(w)) beyond.  P and Q are this project's own fits:
Chebyshev interpolants of degree DEG_C / DEG_T computed in 50-digit arithmetic
(mpmath), converted to monomials in the centred variable and rounded to FP64.
The FP64 Horner evaluation is then checked against 50-digit values on a sample of
the 32-bit input grid u = (J + 1/2) 2^-32 used by the kernels.

The logarithm in w is the kernels' own (log_unit below, mirrored in
device/norminv.hpp): frexp, the atanh series of log m with exact Taylor
coefficients, and e ln 2 with ln 2 split so that e * LN2_HI is exact.

Writes device/norminv_f64_coeffs.hpp next to this file.  Run by hand when the
fit changes:  python gen_norminv_f64.py
"""
import math
import os

import mpmath
import numpy as np

mpmath.mp.dps = 50

W1 = 6.25
W_MAX = -math.log(4 * 2.0 ** -33 * (1 - 2.0 ** -33))      # largest w of the 32-bit grid
DEG_C, DEG_T = 24, 20
S_LO, S_HI = math.sqrt(W1), math.sqrt(W_MAX) + 1e-3


def central_target(w):
    """P(w) = Phi^-1(u) / (2u - 1) with 4u(1-u) = exp(-w)."""
    w = mpmath.mpf(w)
    if w == 0:
        return mpmath.sqrt(mpmath.pi / 2)
    y = mpmath.sqrt(-mpmath.expm1(-w))
    return mpmath.sqrt(2) * mpmath.erfinv(y) / y


def tail_target(s):
    """Q(s) = |Phi^-1(u)| with 4u(1-u) = exp(-s^2)."""
    w = mpmath.mpf(s) ** 2
    y = mpmath.sqrt(-mpmath.expm1(-w))
    return mpmath.sqrt(2) * mpmath.erfinv(y)


def cheb_fit(fun, lo, hi, deg):
    """Monomial coefficients in t = x - (lo + hi) / 2 of the Chebyshev interpolant."""
    n = deg + 1
    lo, hi = mpmath.mpf(lo), mpmath.mpf(hi)
    mid, hw = (lo + hi) / 2, (hi - lo) / 2
    xs = [mpmath.cos(mpmath.pi * (j + mpmath.mpf(1) / 2) / n) for j in range(n)]
    fs = [fun(mid + hw * x) for x in xs]
    c = []
    for k in range(n):
        s = mpmath.fsum(fs[j] * mpmath.cos(k * mpmath.pi * (j + mpmath.mpf(1) / 2) / n) for j in range(n))
        c.append(2 * s / n)
    c[0] /= 2
    # Chebyshev series in x -> monomials in x (T_{k+1} = 2x T_k - T_{k-1}) -> in t = hw x
    T = [[mpmath.mpf(1)], [mpmath.mpf(0), mpmath.mpf(1)]]
    for k in range(2, n):
        nxt = [mpmath.mpf(0)] + [2 * v for v in T[k - 1]]
        for i, v in enumerate(T[k - 2]):
            nxt[i] -= v
        T.append(nxt)
    mono = [mpmath.mpf(0)] * n
    for k in range(n):
        for i, v in enumerate(T[k]):
            mono[i] += c[k] * v
    return [mono[i] / hw ** i for i in range(n)], float(mid)


def horner(coef, t):
    """FP64 Horner with fused multiply-adds (as on the device), vectorised."""
    p = np.full_like(t, float(coef[-1]))
    for k in range(len(coef) - 2, -1, -1):
        p = np.array([math.fma(a, b, float(coef[k])) for a, b in zip(p, t)]) if hasattr(math, "fma") \
            else p * t + float(coef[k])
    return p


def ln2_split():
    """ln 2 = LN2_HI + LN2_LO with the low 21 mantissa bits of LN2_HI zero, so that
    e * LN2_HI is exact for |e| < 2^21."""
    ln2 = mpmath.log(2)
    hi = float(ln2)
    hi = float(np.frombuffer((np.frombuffer(np.float64(hi).tobytes(), np.uint64) &
                              np.uint64(~((1 << 21) - 1) & (2 ** 64 - 1))).tobytes(), np.float64)[0])
    return hi, float(ln2 - mpmath.mpf(hi))


LOG_TERMS = 10          # atanh series terms in z = s^2 beyond the leading 2 s


def log_unit(x):
    """The kernel's logarithm of x in (0, 1]: x = 2^e m, m in [1/sqrt 2, sqrt 2),
    log m = 2 atanh(s) = 2 s + s z Q(z), s = (m - 1) / (m + 1), z = s^2,
    Q(z) = sum_k 2 z^(k-1) / (2k + 1); plus e ln 2 (split)."""
    hi, lo = ln2_split()
    m, e = np.frexp(x)
    small = m < 0.70710678118654752440
    m = np.where(small, m * 2.0, m)
    e = np.where(small, e - 1, e).astype(np.float64)
    f = m - 1.0
    s = f / (2.0 + f)
    z = s * s
    q = np.full_like(z, 2.0 / (2 * LOG_TERMS + 1))
    for k in range(LOG_TERMS - 1, 0, -1):
        q = q * z + 2.0 / (2 * k + 1)
    lm = (s * z) * q + 2.0 * s
    return e * hi + (e * lo + lm)


def evaluate(cc, cmid, ct, tmid, J):
    """The kernel's evaluation order for inputs J (uint64 array)."""
    sj = J.astype(np.int64) - 2 ** 31
    y = (sj.astype(np.float64) + 0.5) * 2.0 ** -31                 # 2u - 1, exact
    v = np.minimum(J, 2 ** 32 - 1 - J).astype(np.float64)
    us = (v + 0.5) * 2.0 ** -32                                    # min(u, 1 - u), exact
    # the kernels form 4u(1-u) as the single fma 1 - y^2: the same double, since the
    # real values agree and each form rounds once
    w = -log_unit((us * (1.0 - us)) * 4.0)
    out = np.empty(J.shape)
    cen = w < W1
    out[cen] = y[cen] * horner(cc, w[cen] - cmid)
    out[~cen] = np.sign(y[~cen]) * horner(ct, np.sqrt(w[~cen]) - tmid)
    return out


def reference(J):
    with mpmath.workdps(40):
        return np.array([float(mpmath.sqrt(2) * mpmath.erfinv(2 * ((mpmath.mpf(int(j)) + 0.5) / 2 ** 32) - 1))
                         for j in J])


def main():
    cc, cmid = cheb_fit(central_target, 0.0, W1, DEG_C)
    ct, tmid = cheb_fit(tail_target, S_LO, S_HI, DEG_T)
    cc64 = [float(v) for v in cc]
    ct64 = [float(v) for v in ct]
    rng = np.random.default_rng(0)
    J = np.unique(np.concatenate([
        rng.integers(0, 2 ** 32, 6000, dtype=np.uint64),
        np.arange(0, 600, dtype=np.uint64), 2 ** 32 - 1 - np.arange(0, 600, dtype=np.uint64),
        2 ** 31 + np.arange(-300, 300).astype(np.uint64),
        # around the branch point w = W1 and the tail's far end
        (rng.integers(0, 2 ** 32, 40000, dtype=np.uint64) >> np.uint64(20)),
        (np.uint64(2 ** 32 - 1) - (rng.integers(0, 2 ** 32, 40000, dtype=np.uint64) >> np.uint64(20)))]))
    z = evaluate(cc64, cmid, ct64, tmid, J)
    ref = reference(J)
    rel = np.abs(z - ref) / np.abs(ref)
    print(f"{J.size} points: max rel err {rel.max():.3e}, 99.9% {np.quantile(rel, 0.999):.3e}")
    here = os.path.dirname(os.path.abspath(__file__))
    out = os.path.join(here, "device", "norminv_f64_coeffs.hpp")
    with open(out, "w") as f:
        f.write("// Generated by gen_norminv_f64.py: FP64 inverse normal, Giles (2011) variable\n")
        f.write("// change w = -log(4u(1-u)), own Chebyshev-interpolant fits (50 digits).\n")
        f.write(f"// Max relative error on {J.size} grid points (FP64 Horner): {rel.max():.2e}\n")
        f.write("#pragma once\n\nnamespace mlmc { namespace ninv64 {\n")
        f.write(f"constexpr double W1 = {W1!r};\n")
        f.write(f"constexpr double C_MID = {cmid!r};\n")
        f.write(f"constexpr double T_MID = {tmid!r};\n")
        f.write(f"constexpr int DEG_C = {DEG_C};\nconstexpr int DEG_T = {DEG_T};\n")
        hi, lo = ln2_split()
        f.write(f"constexpr int LOG_TERMS = {LOG_TERMS};\n")
        f.write(f"constexpr double LN2_HI = {hi!r};\nconstexpr double LN2_LO = {lo!r};\n")
        f.write("constexpr double PC[DEG_C + 1] = {\n    " +
                ",\n    ".join(f"{v!r}" for v in cc64) + "};\n")
        f.write("constexpr double PT[DEG_T + 1] = {\n    " +
                ",\n    ".join(f"{v!r}" for v in ct64) + "};\n")
        f.write("}}  // namespace mlmc::ninv64\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
