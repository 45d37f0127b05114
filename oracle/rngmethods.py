"""Approximate normals from fewer table values: Methods 2 and 3 of Section 3.

Method 1 (normal.py) stores the conditional mean Z_j of Phi^-1 on each of the 2^d
uniform intervals.  The two methods here define other values Z~_j (j = the top d
bits of the uniform word) that need smaller tables on the paper's FPGA; the GPU
library expands them back into a 2^d table, so the values -- and, for Method 2,
the coupled uniform -- are what the oracle fixes.

Common convention (the sign-bit form of Method 1): a b-bit integer whose top bit is
s and whose other b-1 bits are r has the value  +H[r] if s = 1  and  -H[2^(b-1)-1-r]
if s = 0, where H is a table of 2^(b-1) magnitudes; with H the upper half of the
Method-1 table this reproduces Method 1 exactly (T[2^b - 1 - k] = -T[k]).

Method 2 (Section 3.2, sum of n variables).  j is split into n chunks of m = d/n
bits, most significant first; each chunk has the value above over one small table X
of 2^(m-1) entries, and Z~_j is the sum of the n chunk values.  X starts as the
upper half of the m-bit Method-1 table divided by sqrt(n); then, repeatedly, the
Z~_j are ranked in ascending order (pi(j) = rank of Z~_j; equal values ranked by j,
reading R30), and X is replaced by the least-squares solution of
sum_j (Z_{pi(j)} - Z~_j)^2 with Z the d-bit Method-1 values, until pi no longer
changes.  The coupled full-precision uniform of word J is
U = 2^-d pi(j) + 2^-32 (J - 2^(32-d) j + 1/2): the top d bits of J are replaced by
pi(j) (reading R31: D = 32).
Reading R30: Z~_j sums its chunk values in ascending order of value, so that equal
multisets of chunk values give bit-identical sums and ties are exact.

Method 3 (Section 3.3, piecewise linear on dyadic intervals).  j = (s, r) with the
sign-bit convention; on the r side, Z-bar_r = a_i + b_i r where i is the dyadic
interval of r: i = 1 for r in {0, 1}, and i = bit length of r for r >= 2, so the
intervals are {0,1}, [2,3], [4,7], ..., [2^(d-2), 2^(d-1)-1] -- d - 1 of them, the
paper's LUT of d - 1 pairs, whose first two intervals hold two points each (reading
R32).  (a_i, b_i) minimise sum over the interval of (a + b r - Z_r)^2 against the
lower-half Method-1 values Z_r (the paper's reduction of the MSE, eq. for the
dyadic MSE).  The coupled uniform is Method 1's.

MSE.  For any values c_j constant on the uniform intervals of j, E[(c - Phi^-1(U))^2]
= 2^-d sum_j (c_j - Z_j)^2 + MSE_1(d), since Z_j is the conditional mean on
interval j; for Method 2 the interval of j is pi(j).

This module is test infrastructure: see the package docstring.
"""
from functools import lru_cache
import math

import numpy as np

from . import normal


def _sign_split(v, bits):
    """(s, r) of a bits-wide integer: top bit and the other bits."""
    return (v >> (bits - 1)) & 1, v & ((1 << (bits - 1)) - 1)


def _lut_index(s, r, bits):
    """Small-table column and sign of the sign-bit convention."""
    half = 1 << (bits - 1)
    return np.where(s == 1, r, half - 1 - r), np.where(s == 1, 1.0, -1.0)


def method2_design(d, n):
    """cols, signs: (2^d, n) arrays; chunk c of j contributes signs * X[cols]."""
    if d % n:
        raise ValueError("n must divide d")
    m = d // n
    j = np.arange(1 << d, dtype=np.int64)
    cols = np.empty((j.size, n), dtype=np.int64)
    signs = np.empty((j.size, n))
    for c in range(n):
        chunk = (j >> (d - m * (c + 1))) & ((1 << m) - 1)
        s, r = _sign_split(chunk, m)
        cols[:, c], signs[:, c] = _lut_index(s, r, m)
    return cols, signs


def method2_values(X, cols, signs):
    """Z~_j: the chunk values summed in ascending order of value (R30)."""
    v = np.sort(signs * np.asarray(X, dtype=np.float64)[cols], axis=1)
    out = v[:, 0].copy()
    for c in range(1, v.shape[1]):
        out = out + v[:, c]
    return out


def _ranks(values):
    order = np.argsort(values, kind="stable")        # ascending; ties by j
    r = np.empty(values.size, dtype=np.int64)
    r[order] = np.arange(values.size)
    return r


@lru_cache(maxsize=None)
def method2_lut(d, n, max_iter=2000):
    """(X, pi, iterations) of Method 2 for d bits and n variables."""
    m = d // n
    Zd = normal.table_float(d, "float64")
    Hm = normal.table_float(m, "float64")[1 << (m - 1):]       # upper half, ascending
    X = Hm / math.sqrt(n)
    cols, signs = method2_design(d, n)
    A = np.zeros(((1 << d), 1 << (m - 1)))
    for c in range(n):
        np.add.at(A, (np.arange(1 << d), cols[:, c]), signs[:, c])
    pi = None
    for it in range(1, max_iter + 1):
        r = _ranks(method2_values(X, cols, signs))
        if pi is not None and np.array_equal(r, pi):
            return X, pi, it - 1
        pi = r
        X, *_ = np.linalg.lstsq(A, Zd[pi], rcond=None)
    raise RuntimeError("Method 2 permutation did not converge")


def method2_table(d, n):
    """(Z~_j for j = 0 .. 2^d - 1, pi) in FP64."""
    X, pi, _ = method2_lut(d, n)
    cols, signs = method2_design(d, n)
    return method2_values(X, cols, signs), pi


def method2_initial_table(d, n):
    """Z~_j of the initial small table (before the least-squares stage)."""
    m = d // n
    X = normal.table_float(m, "float64")[1 << (m - 1):] / math.sqrt(n)
    cols, signs = method2_design(d, n)
    return method2_values(X, cols, signs)


def coupled_words(J, d, pi):
    """Method 2's coupled word: the top d bits of J replaced by pi(j)."""
    J = np.asarray(J, dtype=np.uint64)
    j = (J >> np.uint64(32 - d)).astype(np.int64)
    low = J & np.uint64((1 << (32 - d)) - 1)
    return (np.asarray(pi, dtype=np.uint64)[j] << np.uint64(32 - d)) | low


def dyadic_interval(r):
    """Method 3's interval of r (R32): 1 for r in {0, 1}, else the bit length of r."""
    r = np.asarray(r, dtype=np.int64)
    bl = np.zeros(r.shape, dtype=np.int64)
    v = r.copy()
    while np.any(v > 0):
        bl += (v > 0)
        v >>= 1
    return np.maximum(bl, 1)


@lru_cache(maxsize=None)
def method3_coeffs(d):
    """(a, b) for intervals i = 1 .. d - 1 (index i - 1), least squares against the
    lower-half Method-1 values."""
    Z = normal.table_float(d, "float64")[: 1 << (d - 1)]
    r = np.arange(1 << (d - 1))
    iv = dyadic_interval(r)
    a = np.empty(d - 1)
    b = np.empty(d - 1)
    for i in range(1, d):
        sel = iv == i
        A = np.stack([np.ones(sel.sum()), r[sel].astype(np.float64)], axis=1)
        (a[i - 1], b[i - 1]), *_ = np.linalg.lstsq(A, Z[sel], rcond=None)
    return a, b


def method3_table(d):
    """Z-bar_j for j = 0 .. 2^d - 1 (sign-bit convention on both halves)."""
    a, b = method3_coeffs(d)
    j = np.arange(1 << d, dtype=np.int64)
    s, r = _sign_split(j, d)
    rr = np.where(s == 1, (1 << (d - 1)) - 1 - r, r)       # lower-half position
    i = dyadic_interval(rr)
    low = a[i - 1] + b[i - 1] * rr
    return np.where(s == 1, -low, low)


def mse(values, d, pi=None):
    """E[(c_j - Phi^-1(U))^2] for values constant on the intervals of j, with the
    interval of j being pi(j) (Method 2) or j (Methods 1, 3)."""
    Zd = normal.table_float(d, "float64")
    target = Zd if pi is None else Zd[np.asarray(pi)]
    return float(np.mean((np.asarray(values) - target) ** 2) + float(normal.table_mse(d)))
