"""Normal increments: exact Z = Phi^-1(U) and the Method-1 table (Section 3).

* U = 2^-D (J + 1/2) with D = 32 (Section 3.1, coupled full-precision uniform).
  U is exact in FP64 and never 0 or 1.
* Z = Phi^-1(U): scipy.special.ndtri in FP64 (pinned against mpmath in the tests).
* Method 1 (Section 3.1): Phi^-1 is replaced by its mean on each of the 2^q
  uniform intervals [k 2^-q, (k+1) 2^-q); the d-bit integer j is the top q bits of
  J (reading R14: a full 2^q table; the paper's half table plus sign bit holds the
  same values because T[2^q-1-k] = -T[k]).  The optimal constant of Section 3.1 is
  T[k] = 2^q * integral of Phi^-1 over the interval, which by the substitution
  u = Phi(x) equals 2^q (phi(Phi^-1(k 2^-q)) - phi(Phi^-1((k+1) 2^-q))), with
  phi(Phi^-1(0)) = phi(Phi^-1(1)) = 0.

Storage rounding: round-to-nearest from the exact (mpmath) value directly to the
target format; a near-tie raises, so the value is unambiguous.

This module is test infrastructure: see the package docstring.
"""
from functools import lru_cache

import mpmath
import numpy as np
from scipy.special import ndtri

TWO_M32 = 2.0 ** -32


def uniform(J):
    """U = 2^-32 (J + 1/2), exact in FP64."""
    return (np.asarray(J, dtype=np.float64) + 0.5) * TWO_M32


def exact_normal(J):
    """Z = Phi^-1(U) in FP64 (Section 3: the 'double' increment of the coupled pair)."""
    return ndtri(uniform(J))


def table_index(J, q):
    """Method-1 interval index: the top q bits of the 32-bit J."""
    return (np.asarray(J, dtype=np.int64) >> (32 - q)) & ((1 << q) - 1)


def _phi_of_quantile(u):
    """phi(Phi^-1(u)) at high precision; 0 at u = 0 and u = 1."""
    if u == 0 or u == 1:
        return mpmath.mpf(0)
    x = mpmath.sqrt(2) * mpmath.erfinv(2 * u - 1)
    return mpmath.npdf(x)


@lru_cache(maxsize=None)
def table_exact(q):
    """Method-1 table T_q[k], k = 0 .. 2^q - 1, as mpmath values (60 digits)."""
    with mpmath.workdps(60):
        n = 1 << q
        edges = [_phi_of_quantile(mpmath.mpf(k) / n) for k in range(n + 1)]
        return tuple(n * (edges[k] - edges[k + 1]) for k in range(n))


def table_mse(q):
    """E[(Z - T[k(Z)])^2] = 1 - 2^-q sum_k T[k]^2: T[k] is the conditional mean
    of Z on interval k, so the error is orthogonal to T (Section 3.1, the MSE
    that Method 1 minimises)."""
    T = table_exact(q)
    with mpmath.workdps(60):
        return 1 - mpmath.fsum(t * t for t in T) / (1 << q)


_FLOAT_BITS = {np.float32: 24, np.float16: 11, np.float64: 53}


def round_float(x, dtype, margin=1e-9):
    """Round the exact value x (mpmath) to the nearest dtype value (ties to even
    never needed: a value within `margin` ulp of a tie raises)."""
    dtype = np.dtype(dtype).type
    with mpmath.workdps(80):
        c = dtype(float(x))
        cands = {c, np.nextafter(c, dtype(-np.inf)), np.nextafter(c, dtype(np.inf))}
        scored = sorted((abs(mpmath.mpf(float(v)) - x), v) for v in cands
                        if np.isfinite(v))
        (d0, best), (d1, _) = scored[0], scored[1]
        ulp = abs(mpmath.mpf(float(np.nextafter(best, dtype(np.inf)))) - mpmath.mpf(float(best)))
        if ulp > 0 and abs(d1 - d0) < margin * ulp:
            raise ValueError(f"value {x} is within {margin} ulp of a rounding tie")
        return best


def round_fixed(x, frac_bits, margin=1e-9):
    """Round the exact value x to an integer multiple of 2^-f: n = floor(x 2^f + 1/2)
    (round-to-nearest, ties toward +infinity, reading R7).  A value within
    `margin` of a tie raises."""
    with mpmath.workdps(80):
        y = x * mpmath.mpf(2) ** frac_bits
        fl = mpmath.floor(y)
        frac = y - fl
        if abs(frac - mpmath.mpf(0.5)) < margin:
            raise ValueError(f"value {x} is within {margin} of a fixed-point tie")
        return int(mpmath.floor(y + mpmath.mpf(0.5)))


@lru_cache(maxsize=None)
def table_float(q, dtype_name):
    """T_q rounded to float64 / float32 / float16 (numpy dtype name)."""
    dt = np.dtype(dtype_name).type
    return np.array([round_float(t, dt) for t in table_exact(q)], dtype=dt)


@lru_cache(maxsize=None)
def table_fixed(q, frac_bits):
    """T_q as integers n with value n 2^-f (int64 array)."""
    return np.array([round_fixed(t, frac_bits) for t in table_exact(q)], dtype=np.int64)
