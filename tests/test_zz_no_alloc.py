"""mlmc_level_sums_static (the entry point that allocates nothing) against
mlmc_level_sums on the same arguments, through the C ABI: two calls in a row with
the second smaller, then other variants, then the first again (the scratch array
keeps the previous call's contents).  Integer results bit-exact; FP64 sums to the
FP64 sum tolerance (they are expected to be identical: same kernels, same tiles)."""
import numpy as np
import pytest

import paper_2502_07123_amd as M

GBM = dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0, barrier=85.0)
FMT = {"X": (32, 29), "con1": (32, 34), "con2": (32, 33), "con3": (32, 36), "Z": (31, 28),
       "mul1": (32, 30), "sum1": (32, 30), "zsq": (32, 23), "zm1": (32, 23),
       "mul3": (32, 29), "sum2": (32, 29), "mul2": (32, 27)}

# (scheme, payoffs, level, n_paths, path_offset, precision, estimator, seed, option)
CASES = [
    ("milstein", ("euro",), 3, 3_000_000, 17, ("fp32", 8, True), M.EST_APPROX, 1234, 0),
    ("milstein", ("euro",), 1, 1_001, 5, ("fp32", 8, True), M.EST_APPROX, 1234, 0),
    ("milstein", ("euro", "asian"), 5, 20_000, 0, ("fp32", 8, False), M.EST_CORR, 99, 3),
    ("euler", ("euro", "barrier"), 2, 100_003, 1, ("fixed", 8, False), M.EST_APPROX, 7, 1),
    ("euler", ("digital",), 0, 250_000, 0, ("fp32", 6, False), M.EST_PLAIN, 5, 2),
    ("milstein", ("euro",), 0, 400_001, 3, ("fp32", 8, False), M.EST_CORR, 1234, 0),
]


def _prec(spec):
    arith, q, packed = spec
    if arith == "fixed":
        return M.make_precision("fixed", q, packed, FMT)
    return M.make_precision(arith, q, packed)


def _close(a, b):
    return abs(a - b) <= 1e-12 * max(1.0, abs(a), abs(b))


@pytest.mark.gpu
def test_static_entry_equals_level_sums():
    import torch
    order = list(range(len(CASES))) + [0]
    with M.Context(0, workspace_bytes=256 << 20) as ctx:
        for i in order:
            scheme, pays, level, n, off, pspec, est, seed, opt = CASES[i]
            print(f"case {i}: {scheme} {pays} level {level} n {n} est {est} {pspec}", flush=True)
            prob = M.make_problem(scheme, pays, **GBM)
            prec = _prec(pspec)
            ref = ctx.level_sums(prob, level, n, off, prec, est, seed, opt)
            out = M.level_sums_static(prob, level, n, off, prec, est, seed, opt)
            torch.cuda.synchronize()
            got = M.sums_from_device(out, prob)
            for p in pays:
                r, g = ref[p], got[p]
                for f in ("n", "isum1", "isum2", "saturations", "nonfinite"):
                    assert int(r[f]) == int(g[f]), (i, p, f, r[f], g[f])
                for f in ("sum1", "sum2", "esum1", "esum2"):
                    assert _close(r[f], g[f]), (i, p, f, r[f], g[f])
                assert r["n"] == n
