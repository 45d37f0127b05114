"""Fixed-point arithmetic of the low-precision path (Section 4.1).

The paper's format is x~ = (-1)^s 2^(e-d) n with 0 <= n < 2^d and a separate sign
bit, rounding to nearest (Section 4.1, bound |dx| <= 2^(e-d-1)).

Readings:
* R6 (encoding): two's-complement integer of w bits with f fractional bits, value
  n 2^-f, w = d + 1 and f = d - e.  Same value set as sign-magnitude except -2^d.
* R7 (rounding): nearest, ties toward +infinity: n = floor(x 2^f + 1/2).  When the
  result needs no rounding the operation is exact.
* R8 (overflow): saturate to [-2^(w-1), 2^(w-1) - 1] and count each saturation.

Operations take integer operands with their own fractional bits and return the
destination integer: the exact result (product, or sum after exact alignment to
the finer operand) is rounded once to the destination f, then saturated.

`exact_*` functions do the same with fractions.Fraction scalars (the definition);
the numpy versions (int64, |operands| < 2^31) are the ones the paths use and are
tested equal to the Fraction versions on their domain: a product keeps at most
its own fractional bits (f_dst <= f_a + f_b) and a sum at most its finer operand's
(f_dst <= max(f_a, f_b)) with |f_a - f_b| <= 30, so no intermediate exceeds 2^62.

This module is test infrastructure: see the package docstring.
"""
from fractions import Fraction
import math

import numpy as np


# ---------------------------------------------------------------- definitions
def exact_round(x: Fraction, f: int) -> int:
    """Round the rational x to a multiple of 2^-f: floor(x 2^f + 1/2) (R7)."""
    y = x * (Fraction(2) ** f)
    return math.floor(y + Fraction(1, 2))


def exact_saturate(n: int, w: int):
    lo, hi = -(1 << (w - 1)), (1 << (w - 1)) - 1
    if n < lo:
        return lo, 1
    if n > hi:
        return hi, 1
    return n, 0


def exact_mul(a, fa, b, fb, fd, wd):
    x = Fraction(a) * Fraction(2) ** -fa * Fraction(b) * Fraction(2) ** -fb
    return exact_saturate(exact_round(x, fd), wd)


def exact_add(a, fa, b, fb, fd, wd, sub=False):
    x = Fraction(a) * Fraction(2) ** -fa + (-1 if sub else 1) * Fraction(b) * Fraction(2) ** -fb
    return exact_saturate(exact_round(x, fd), wd)


# ---------------------------------------------------------------- numpy forms
def round_shift(p, s):
    """p 2^-s rounded to an integer by R7 (s > 0), or the exact p 2^-s (s <= 0).
    p: int64 array with |p| small enough that p + 2^(s-1) does not overflow."""
    p = np.asarray(p, dtype=np.int64)
    if s <= 0:
        return p << np.int64(-s)
    return (p + np.int64(1 << (s - 1))) >> np.int64(s)


def saturate(n, w):
    """Clip to the w-bit two's-complement range; returns (value, count array)."""
    lo, hi = -(1 << (w - 1)), (1 << (w - 1)) - 1
    n = np.asarray(n, dtype=np.int64)
    sat = ((n < lo) | (n > hi)).astype(np.int64)
    return np.clip(n, lo, hi), sat


def mul(a, fa, b, fb, fd, wd):
    """(a 2^-fa)(b 2^-fb) rounded to f = fd and saturated to w = wd."""
    p = np.asarray(a, dtype=np.int64) * np.asarray(b, dtype=np.int64)
    return saturate(round_shift(p, fa + fb - fd), wd)


def add(a, fa, b, fb, fd, wd, sub=False):
    """a 2^-fa +/- b 2^-fb: exact alignment to max(fa, fb), one rounding to fd,
    saturation to wd."""
    fm = max(fa, fb)
    A = np.asarray(a, dtype=np.int64) << np.int64(fm - fa)
    B = np.asarray(b, dtype=np.int64) << np.int64(fm - fb)
    s = A - B if sub else A + B
    return saturate(round_shift(s, fm - fd), wd)


def quantize_double(x, f, w):
    """Quantise an FP64 value exactly (the double is a dyadic rational)."""
    n = exact_round(Fraction(float(x)), f)
    return exact_saturate(n, w)[0]
