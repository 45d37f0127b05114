"""Parity at the full size of the benchmark's nested workload, in the launch
configuration it is profiled in: the European call on GBM (S0 = K = 100, r = 0.05,
sigma = 0.2, T = 1), Milstein, levels 0..8, the FP32 approximate estimator with
packed q = 8 indices and the correction estimator (FP64 exact side, FP32 table
side) with the sample counts of an allocation at eps = 1e-3 in price units, all 18
works in one two-stream launch sequence (as bench.py enqueues them).

* Level 0 of the approximate estimator (2.5e8 paths): its sample is a function of
  the path's table index alone, so the exact sums are sum_k c_k Y(k) with c_k the
  index counts of the oracle's own Philox words and Y(k) the oracle's FP32 side;
  the GPU's FP64 sums agree to 1e-11 relative.
* Every other work: the oracle path by path; per-path FP32 samples are bit-exact
  (R25), so the sums differ only by FP64 summation order (4 n 2^-53 sum |Y|); the
  correction's FP64 exact side within 1e-10 of its scale (inverse-normal rounding)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import paper_2502_07123_amd as M
from oracle import philox
from oracle.paths import EST_APPROX as O_APPROX
from oracle.paths import PathState, Precision, Problem, level_constants, make_side, side_table, simulate

pytestmark = pytest.mark.gpu

GBM = dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0)
SEED = 1234
Q = 8
# sample counts of the allocation at eps = 1e-3 (price units) after a pilot
N_APPROX = [249_118_410, 4_978_507, 1_835_051, 678_506, 251_495, 90_766, 32_379, 11_487, 4_053]
N_CORR = [4_238_487, 161_375, 53_054, 22_492, 8_470, 3_278, 1_150, 401, 145]
OFFSET = 1_001                # a ragged first group at every level
# the geometry of the committed profiles (two streams: the flight exceeds 2^26 path-steps)
TUNING = dict(block_table=256, block_exact=256, tile_steps=131072, blocks_per_cu=16, min_tiles=512,
              zb_max_paths=32768, zb_max_positions=4194304, overlap_min_steps=67108864)


@pytest.fixture(scope="module")
def sums():
    ctx = M.Context(0, workspace_bytes=1 << 30)
    ctx.set_tuning(**TUNING)
    prob = M.make_problem("milstein", ("euro",), **GBM)
    pa = M.make_precision("fp32", Q, packed=True)
    pc = M.make_precision("fp32", Q, packed=False)
    items = []
    for l in range(9):
        items.append((prob, l, N_APPROX[l], OFFSET, pa, M.EST_APPROX, SEED, 0))
        items.append((prob, l, N_CORR[l], OFFSET, pc, M.EST_CORR, SEED, 0))
    b = ctx.sums_batch(items)
    b.enqueue()
    out = b.wait().copy()
    ctx.close()
    return out


def _level0_counts(n, off):
    """Index counts c_k of approximate level-0 paths [off, off + n): path p takes
    field p mod 4 (from the top) of stream word p div 4."""
    F = 32 // Q
    c = np.zeros(1 << Q, dtype=np.int64)
    w0, w1 = off // F, (off + n - 1) // F + 1
    step = 1 << 22
    for a in range(w0, w1, step):
        w = np.arange(a, min(a + step, w1), dtype=np.uint64)
        J = philox.stream_words(SEED, 0, 0, O_APPROX, w).astype(np.int64)
        for j in range(F):
            p = w.astype(np.int64) * F + j
            k = (J >> (32 - Q * (j + 1))) & ((1 << Q) - 1)
            c += np.bincount(k[(p >= off) & (p < off + n)], minlength=1 << Q)
    return c


def _level0_samples():
    """Y(k) of the approximate estimator's level 0 for every index k (the oracle's
    FP32 side: one Milstein step with the table value, then the payoff)."""
    prob = Problem("milstein", **GBM)
    prec = Precision("fp32", Q, packed=True)
    side = make_side("fp32", prec, level_constants(prob, 0), "milstein")
    ps = PathState(side, 1 << Q, 0)
    ps.fine(side_table(side, prec), 0)
    Y, _, _ = ps.level_diff("euro")
    return side.to_f64(Y)


def test_level0_approximate_full_size(sums):
    s = sums[0, 0]
    n = N_APPROX[0]
    c = _level0_counts(n, OFFSET)
    assert int(c.sum()) == n
    Y = _level0_samples()
    s1 = sum(Fraction(int(ck)) * Fraction(float(y)) for ck, y in zip(c, Y))
    s2 = sum(Fraction(int(ck)) * Fraction(float(y)) ** 2 for ck, y in zip(c, Y))
    assert int(s["n"]) == n and int(s["nonfinite"]) == 0
    assert abs(float(s["sum1"]) - float(s1)) <= 1e-11 * float(s1)
    assert abs(float(s["sum2"]) - float(s2)) <= 1e-11 * float(s2)


def _oracle_sums(level, n, est):
    prob = Problem("milstein", **GBM)
    prec = Precision("fp32", Q, packed=est == O_APPROX)
    Y, E = [], []
    for a in range(OFFSET, OFFSET + n, 1 << 20):
        paths = np.arange(a, min(a + (1 << 20), OFFSET + n), dtype=np.uint64)
        o = simulate(prob, level, paths, prec, est, SEED, 0, ("euro",), plain_arith="fp64")["euro"]
        Y.append(o["Y"])
        if "Y_exact" in o:
            E.append(o["Y_exact"])
    Y = np.concatenate(Y)
    E = np.concatenate(E) if E else None
    return Y, E


@pytest.mark.parametrize("level,est", [(l, M.EST_APPROX) for l in range(1, 9)] +
                         [(l, M.EST_CORR) for l in range(9)])
def test_works_against_oracle_paths(sums, level, est):
    n = (N_APPROX if est == M.EST_APPROX else N_CORR)[level]
    s = sums[2 * level + (1 if est == M.EST_CORR else 0), 0]
    Y, E = _oracle_sums(level, n, est)
    assert int(s["n"]) == n and int(s["nonfinite"]) == 0
    if est == M.EST_APPROX:
        bound = 4 * n * 2.0 ** -53
        assert abs(float(s["sum1"]) - math.fsum(Y)) <= bound * np.sum(np.abs(Y)) + 1e-300
        assert abs(float(s["sum2"]) - math.fsum(Y * Y)) <= bound * np.sum(Y * Y) + 1e-300
    else:
        assert abs(float(s["sum1"]) - math.fsum(Y)) <= 1e-10 * (np.sum(np.abs(Y)) + 1)
        assert abs(float(s["sum2"]) - math.fsum(Y * Y)) <= 1e-10 * (np.sum(Y * Y) + 1)
        assert abs(float(s["esum1"]) - math.fsum(E)) <= 1e-10 * (np.sum(np.abs(E)) + 1)
        assert abs(float(s["esum2"]) - math.fsum(E * E)) <= 1e-10 * (np.sum(E * E) + 1)
