"""Pins for the oracle's MLMC layer (Sections 2.1-2.2; readings R9-R13).

* Allocation formulas against a direct numerical minimisation of the cost at
  fixed variance (Section 2.1 Lagrange solution; Section 2.2 nested form).
* Total-cost formula eps^-2 (sum sqrt(V C))^2 at the optimum.
* Variance estimate R9 against numpy's unbiased variance.
* Adaptive plain and nested estimates agree with Black-Scholes within their
  standard error plus the bias allowance, and with each other.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle.mlmc import (RunConfig, Sums, estimate, mlmc_cost, nested_samples,
                         optimal_samples)
from oracle.paths import Precision, Problem

from test_oracle_paths import GBM, bs_call


def _brute_force(V, C, eps2):
    """Split the variance budget eps^2 into shares x (softmax of z), N_l = V_l / (x_l eps^2),
    and minimise the cost sum N_l C_l over z numerically."""
    V, C = np.asarray(V, float), np.asarray(C, float)

    def shares(z):
        e = np.exp(z - z.max())
        return e / e.sum()

    def cost(z):
        return float(np.sum(V * C / shares(z))) / eps2

    r = minimize(cost, np.zeros_like(V), method="BFGS", options={"gtol": 1e-12, "maxiter": 5000})
    r = minimize(cost, r.x, method="Nelder-Mead",
                 options={"xatol": 1e-12, "fatol": 1e-14, "maxiter": 40000, "maxfev": 40000})
    x = shares(r.x)
    return V / (x * eps2), r.fun


def test_optimal_samples_minimise_cost():
    V = [1e-2, 3e-4, 8e-5, 2e-5, 5e-6]
    C = [1, 2, 4, 8, 16]
    eps2 = 1e-6
    N = optimal_samples(V, C, eps2)
    Nbf, cbf = _brute_force(V, C, eps2)
    assert np.all(np.abs(N - Nbf) <= 1 + 1e-5 * Nbf), (N, Nbf)     # N is the ceiling
    assert abs(mlmc_cost(V, C, eps2) - cbf) / cbf < 1e-6
    assert np.sum(np.asarray(V) / N) <= eps2 * (1 + 1e-12)     # rounded up: feasible


def test_nested_samples_minimise_cost():
    Vt = [1e-2, 3e-4, 8e-5]
    Ct = [0.1, 0.2, 0.4]
    Vd = [1e-5, 2e-6, 9e-7]
    Cd = [1.1, 2.2, 4.4]
    eps2 = 1e-6
    Nt, Nd = nested_samples(Vt, Ct, Vd, Cd, eps2)
    Nbf, _ = _brute_force(Vt + Vd, Ct + Cd, eps2)
    Nall = np.concatenate([Nt, Nd])
    assert np.all(np.abs(Nall - Nbf) <= 1 + 1e-5 * Nbf), (Nall, Nbf)
    theta = 0.5
    Nt2, Nd2 = nested_samples(Vt, Ct, Vd, Cd, eps2, theta)
    assert np.sum(np.asarray(Vt) / Nt2) + np.sum(np.asarray(Vd) / Nd2) <= theta * eps2 * (1 + 1e-12)


def test_variance_estimate_r9():
    rng = np.random.default_rng(0)
    y = rng.normal(0.3, 2.0, size=1000)
    s = Sums(n=y.size, s1=math.fsum(y), s2=math.fsum(y * y))
    assert abs(s.var() - np.var(y, ddof=1)) < 1e-10
    assert abs(s.mean() - y.mean()) < 1e-14


@pytest.fixture(scope="module")
def adaptive_results():
    p = Problem("milstein", **GBM)
    cfg = RunConfig(eps=2e-3, eps_units="normalised", theta=0.5, L_min=2, L_max=8,
                    n_pilot=2000, nested=False, plain_arith="fp64")
    plain = estimate(p, "euro", Precision(), cfg, seed=1234)
    cfgn = RunConfig(**{**cfg.__dict__, "nested": True})
    nested = estimate(p, "euro", Precision("fp32", 6), cfgn, seed=1234)
    return p, cfg, plain, nested


def test_adaptive_plain_matches_black_scholes(adaptive_results):
    p, cfg, plain, _ = adaptive_results
    ref = bs_call(p.S0, p.K, p.r, p.sigma, p.T)
    # theta = 1/2: sampling variance <= eps^2 / 2 and bias <= eps / sqrt(2) (price units)
    eps_price = cfg.eps * p.S0          # R13: eps is on the price / S0
    assert plain.variance <= cfg.theta * eps_price ** 2 * 1.01
    assert abs(plain.estimate - ref) < 4 * math.sqrt(plain.variance) + eps_price, \
        (plain.estimate, ref)


def test_adaptive_nested_matches_plain(adaptive_results):
    p, cfg, plain, nested = adaptive_results
    ref = bs_call(p.S0, p.K, p.r, p.sigma, p.T)
    eps_price = cfg.eps * p.S0          # R13: eps is on the price / S0
    assert nested.variance <= cfg.theta * eps_price ** 2 * 1.01
    assert abs(nested.estimate - ref) < 4 * math.sqrt(nested.variance) + eps_price
    assert abs(nested.estimate - plain.estimate) < 4 * math.sqrt(nested.variance + plain.variance) + eps_price
    # the correction estimator's variance is far below the approximate one's (Section 2.2)
    for l in range(nested.L + 1):
        assert nested.sums[(l, 2)].var() < 0.2 * nested.sums[(l, 1)].var()


def test_remaining_bias_uses_three_levels():
    """R34 with alpha = 1: a level mean that is small by chance does not hide the
    bias that the two levels below it show; with geometric means every term of the
    max agrees."""
    from oracle.mlmc import remaining_bias
    assert remaining_bias([1.0, 0.08, 0.04, 0.02, 0.01]) == 0.01
    assert remaining_bias([1.0, 0.08, 0.04, 0.02, 1e-6]) == 0.01          # 0.02 / 2
    assert remaining_bias([1.0, 0.08, 0.04, -1e-6, 1e-6]) == 0.01         # 0.04 / 4
    assert remaining_bias([1.0, 0.5, 1e-6]) == 0.25                     # level 0 excluded
    assert remaining_bias([0.3]) == 0.3
    assert remaining_bias([0.3, -0.05]) == 0.05


def digital_closed_form(S0, K, r, sigma, T):
    """A digital call paying K: K e^{-rT} N(d2)."""
    d2 = (math.log(S0 / K) + (r - 0.5 * sigma ** 2) * T) / (sigma * math.sqrt(T))
    return K * math.exp(-r * T) * 0.5 * (1 + math.erf(d2 / math.sqrt(2)))


def test_discontinuous_payoff_switches_levels_to_plain():
    """R35: for a digital call the table error moves paths across the jump, the
    correction variance is as large as the approximate one from level 1 on, and
    those levels continue with plain samples (level 0 keeps the nested pair); the
    price stays within the error budget of the closed form.  A European call keeps
    the nested pair on every level."""
    p = Problem("milstein", **GBM)
    cfg = RunConfig(eps=3e-3, eps_units="normalised", theta=0.5, L_min=2, L_max=6,
                    n_pilot=10_000, nested=True, plain_arith="fp64",
                    cost_plain=1.0, cost_approx=0.5, cost_corr=2.9)
    r = estimate(p, "digital", Precision("fp32", 6), cfg, seed=1234)
    assert (0, 1) in r.sums and (0, 2) in r.sums and (0, 0) not in r.sums
    for l in range(1, r.L + 1):
        assert (l, 0) in r.sums and (l, 1) not in r.sums and (l, 2) not in r.sums, l
    ref = digital_closed_form(p.S0, p.K, p.r, p.sigma, p.T)
    eps_price = cfg.eps * p.S0
    assert r.variance <= cfg.theta * eps_price ** 2 * 1.01
    assert abs(r.estimate - ref) < 4 * math.sqrt(r.variance) + eps_price
    e = estimate(p, "euro", Precision("fp32", 6), cfg, seed=1234)
    assert all((l, 1) in e.sums and (l, 2) in e.sums and (l, 0) not in e.sums for l in range(e.L + 1))
