"""Pins for the oracle's normal increments (Section 3.1).

* Phi^-1: scipy's ndtri against mpmath's sqrt(2) erfinv(2u - 1) at 60 digits.
* Table T_q: the closed form against direct quadrature of the paper's definition
  Z_j = 2^d * integral of Phi^-1 over the interval; sum zero; antisymmetry; each
  value inside its interval (the coupling of Section 3.1).
* MSE: 1 - 2^-q sum T^2 against quadrature of the squared error; trend of
  Section 3.4 (the MSE ratio per extra bit tends to 2).
* Storage rounding helpers against brute force.
"""
import mpmath
import numpy as np
import pytest

from oracle import normal


def _mp_quantile(u):
    with mpmath.workdps(60):
        return mpmath.sqrt(2) * mpmath.erfinv(2 * mpmath.mpf(u) - 1)


def test_uniform_exact_and_open():
    J = np.array([0, 1, 2**31 - 1, 2**31, 2**32 - 1], dtype=np.uint64)
    U = normal.uniform(J)
    for j, u in zip(J, U):
        assert mpmath.mpf(float(u)) == (mpmath.mpf(int(j)) + mpmath.mpf(0.5)) / 2**32
    assert U.min() > 0 and U.max() < 1


def test_ndtri_against_mpmath():
    rng = np.random.default_rng(0)
    J = np.concatenate([np.array([0, 1, 2, 2**31 - 2, 2**31 - 1, 2**31, 2**31 + 1,
                                  2**32 - 2, 2**32 - 1], dtype=np.uint64),
                        rng.integers(0, 2**32, size=3000, dtype=np.uint64)])
    Z = normal.exact_normal(J)
    for j, z in zip(J, Z):
        with mpmath.workdps(60):
            u = (mpmath.mpf(int(j)) + mpmath.mpf(0.5)) / mpmath.mpf(2) ** 32
            ref = mpmath.sqrt(2) * mpmath.erfinv(2 * u - 1)
            err = abs(mpmath.mpf(float(z)) - ref)
            assert err <= 2e-15 * max(abs(ref), mpmath.mpf(1e-3)), (int(j), z, ref)
    # |Z| is bounded by the extreme uniforms
    assert np.abs(Z).max() <= float(-_mp_quantile(mpmath.mpf(0.5) / 2**32)) + 1e-12


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_table_closed_form_equals_interval_mean(q):
    T = normal.table_exact(q)
    n = 1 << q
    with mpmath.workdps(30):
        f = lambda u: mpmath.sqrt(2) * mpmath.erfinv(2 * u - 1)
        for k in range(n):
            a, b = mpmath.mpf(k) / n, mpmath.mpf(k + 1) / n
            ref = n * mpmath.quad(f, [a, b])
            assert abs(T[k] - ref) < mpmath.mpf(10) ** -20, (q, k)


@pytest.mark.parametrize("q", [2, 4, 6, 8, 10])
def test_table_invariants(q):
    T = normal.table_exact(q)
    n = 1 << q
    with mpmath.workdps(60):
        assert abs(mpmath.fsum(T)) < mpmath.mpf(10) ** -40
        for k in range(n):
            assert abs(T[k] + T[n - 1 - k]) < mpmath.mpf(10) ** -40
            lo = -mpmath.inf if k == 0 else _mp_quantile(mpmath.mpf(k) / n)
            hi = mpmath.inf if k == n - 1 else _mp_quantile(mpmath.mpf(k + 1) / n)
            assert lo < T[k] < hi
        # increasing
        assert all(T[k] < T[k + 1] for k in range(n - 1))


@pytest.mark.parametrize("q", [1, 2, 3])
def test_mse_identity_against_quadrature(q):
    T = normal.table_exact(q)
    n = 1 << q
    with mpmath.workdps(30):
        f = lambda u: mpmath.sqrt(2) * mpmath.erfinv(2 * u - 1)
        tot = mpmath.fsum(mpmath.quad(lambda u: (T[k] - f(u)) ** 2,
                                      [mpmath.mpf(k) / n, mpmath.mpf(k + 1) / n])
                          for k in range(n))
        assert abs(tot - normal.table_mse(q)) < mpmath.mpf(10) ** -15


def test_mse_trend_per_bit():
    """MSE falls by a factor tending to 2 per extra bit (Section 3.4)."""
    m = [float(normal.table_mse(q)) for q in range(4, 13)]
    ratios = [m[i] / m[i + 1] for i in range(len(m) - 1)]
    assert all(2.0 < r < 2.6 for r in ratios), ratios
    assert all(ratios[i + 1] < ratios[i] for i in range(len(ratios) - 1)), ratios


@pytest.mark.parametrize("q", [4, 8])
def test_coupling_same_interval_and_empirical_mse(q):
    rng = np.random.default_rng(q)
    J = rng.integers(0, 2**32, size=400_000, dtype=np.uint64)
    Z = normal.exact_normal(J)
    k = normal.table_index(J, q)
    T = normal.table_float(q, "float64")
    edges = np.array([-np.inf] + [float(_mp_quantile(mpmath.mpf(i) / (1 << q)))
                                  for i in range(1, 1 << q)] + [np.inf])
    assert np.all(edges[k] <= Z) and np.all(Z <= edges[k + 1])
    emp = np.mean((Z - T[k]) ** 2)
    mse = float(normal.table_mse(q))
    se = np.std((Z - T[k]) ** 2) / np.sqrt(J.size)
    assert abs(emp - mse) < 4 * se


def test_round_helpers_against_brute_force():
    rng = np.random.default_rng(1)
    for x in rng.normal(size=200):
        xm = mpmath.mpf(x) + mpmath.mpf(1e-9)
        r32 = normal.round_float(xm, np.float32)
        # nearest float32 by brute force over neighbours
        c = np.float32(float(xm))
        lo, hi = c, c
        nb = [c]
        for _ in range(3):
            lo, hi = np.nextafter(lo, np.float32(-np.inf)), np.nextafter(hi, np.float32(np.inf))
            nb += [lo, hi]
        best = min(nb, key=lambda v: abs(mpmath.mpf(float(v)) - xm))
        assert r32 == best
        n = normal.round_fixed(xm, 20)
        assert abs(mpmath.mpf(n) / 2**20 - xm) <= mpmath.mpf(2) ** -21
    assert normal.round_fixed(mpmath.mpf(3) / 8 + mpmath.mpf(10) ** -6, 2) == 2
    assert normal.round_fixed(mpmath.mpf(3) / 8 - mpmath.mpf(10) ** -6, 2) == 1
    with pytest.raises(ValueError):
        normal.round_fixed(mpmath.mpf(3) / 8, 2)


@pytest.mark.parametrize("q", [4, 6, 8, 10, 12])
def test_stored_tables_not_near_ties(q):
    """Every stored format the tests use rounds unambiguously (no near-ties)."""
    normal.table_float(q, "float32")
    normal.table_float(q, "float16")
    for f in (12, 16, 20, 24, 28):
        normal.table_fixed(q, f)
