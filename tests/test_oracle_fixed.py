"""Pins for the oracle's fixed-point arithmetic (Section 4.1; readings R6-R8).

* The vectorised int64 operations equal the rational definitions (Fraction,
  round once to nearest with ties up, then saturate): exhaustively for small
  operands, by hypothesis for 32-bit operands.
* Rounding error bound |dx| <= 2^(e-d-1) = 2^-(f+1) (Section 4.1).
* Rounding error moments: mean ~ 0 and E[dx^2] ~ 4^-f / 12, the uniform model the
  optimistic bound uses (Section 4.1).
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import fixedpoint as fx


def test_round_ties_up():
    assert fx.exact_round(Fraction(3, 2), 0) == 2
    assert fx.exact_round(Fraction(-3, 2), 0) == -1
    assert fx.exact_round(Fraction(5, 8), 2) == 3      # 2.5 -> 3
    assert fx.exact_round(Fraction(-5, 8), 2) == -2    # -2.5 -> -2
    assert list(fx.round_shift(np.array([3, -3, 5, -5, 4]), 1)) == [2, -1, 3, -2, 2]


@pytest.mark.parametrize("fa,fb,fd", [(3, 3, 3), (4, 2, 3), (2, 5, 6), (5, 5, 1), (1, 1, 4)])
def test_mul_exhaustive_small(fa, fb, fd):
    vals = np.arange(-32, 32)
    A, B = np.meshgrid(vals, vals)
    got, sat = fx.mul(A.ravel(), fa, B.ravel(), fb, fd, 7)
    for a, b, g, s in zip(A.ravel(), B.ravel(), got, sat):
        ref, rs = fx.exact_mul(int(a), fa, int(b), fb, fd, 7)
        assert (int(g), int(s)) == (ref, rs), (a, b)


@pytest.mark.parametrize("fa,fb,fd,sub", [(3, 3, 3, False), (4, 2, 3, True), (2, 5, 6, False),
                                          (5, 1, 2, True), (0, 6, 6, False)])
def test_add_exhaustive_small(fa, fb, fd, sub):
    vals = np.arange(-32, 32)
    A, B = np.meshgrid(vals, vals)
    got, sat = fx.add(A.ravel(), fa, B.ravel(), fb, fd, 6, sub=sub)
    for a, b, g, s in zip(A.ravel(), B.ravel(), got, sat):
        ref, rs = fx.exact_add(int(a), fa, int(b), fb, fd, 6, sub=sub)
        assert (int(g), int(s)) == (ref, rs), (a, b)


i32 = st.integers(-(2**31), 2**31 - 1)
fr = st.integers(0, 30)


@settings(max_examples=400, deadline=None)
@given(i32, i32, fr, fr, fr, st.integers(2, 32))
def test_mul_32bit(a, b, fa, fb, fd, wd):
    fd = min(fd, fa + fb)                    # the operation's domain (module docstring)
    got, sat = fx.mul(np.array([a]), fa, np.array([b]), fb, fd, wd)
    assert (int(got[0]), int(sat[0])) == fx.exact_mul(a, fa, b, fb, fd, wd)


@settings(max_examples=400, deadline=None)
@given(i32, i32, fr, fr, fr, st.integers(2, 32), st.booleans())
def test_add_32bit(a, b, fa, fb, fd, wd, sub):
    fd = min(fd, max(fa, fb))                # the operation's domain (module docstring)
    got, sat = fx.add(np.array([a]), fa, np.array([b]), fb, fd, wd, sub=sub)
    assert (int(got[0]), int(sat[0])) == fx.exact_add(a, fa, b, fb, fd, wd, sub=sub)


@pytest.mark.parametrize("f", [4, 10, 20])
def test_rounding_error_bound_and_moments(f):
    rng = np.random.default_rng(f)
    a = rng.integers(-(2**20), 2**20, size=200_000)
    b = rng.integers(-(2**20), 2**20, size=200_000)
    fa, fb = 20, 20
    got, sat = fx.mul(a, fa, b, fb, f, 32)
    assert sat.sum() == 0
    exact = (a.astype(np.float64) * b) * 2.0 ** -(fa + fb)      # exact: < 2^53
    d = got * 2.0 ** -f - exact
    assert np.all(np.abs(d) <= 2.0 ** -(f + 1))
    se = np.std(d) / np.sqrt(d.size)
    assert abs(d.mean()) < 5 * se + 2.0 ** -(fa + fb)
    ratio = np.mean(d * d) / (4.0 ** -f / 12)
    assert 0.97 < ratio < 1.03, ratio


def test_saturation_counts():
    v, s = fx.add(np.array([2**30, -(2**30)]), 0, np.array([2**30, -(2**30) - 1]), 0, 0, 32)
    assert list(v) == [2**31 - 1, -(2**31)]
    assert list(s) == [1, 1]
    v, s = fx.mul(np.array([100]), 0, np.array([100]), 0, 0, 8)
    assert int(v[0]) == 127 and int(s[0]) == 1


def test_quantize_double_exact():
    for x in (0.1, -0.37, 1e-3, 2.5):
        for f in (8, 16, 24):
            n = fx.quantize_double(x, f, 32)
            assert abs(Fraction(n, 1 << f) - Fraction(x)) <= Fraction(1, 1 << (f + 1))
