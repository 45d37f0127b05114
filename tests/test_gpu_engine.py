"""The device sweep engine (mlmc_set_driver: run states on the device, one graph
replay per sweep) against host-driven sweeps, through the C ABI: the same levels,
sample counts, sums and estimates bit for bit, for nested and plain runs, a level
that switches to plain samples (digital), fixed point, path functionals, an FP32
exact side, batches of mixed options, repeated calls (the cached graph replayed
again) and a workspace too small for the engine (host-driven fallback)."""
import numpy as np
import pytest

import paper_2502_07123_amd as M
from parity import GBM, SEED, WIDE_FMT

pytestmark = pytest.mark.gpu

EURO = {k: v for k, v in GBM.items() if k != "barrier"}


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0, workspace_bytes=512 << 20)
    yield c
    c.set_driver(True)
    c.close()


def _cfg(nested, arith="fp32", eps=0.002, L_max=8, q=8, packed=False, exact="fp64", plain="fp32",
         costs=(1.0, 0.1, 1.1), n_pilot=2000):
    fmt = WIDE_FMT if arith == "fixed" else None
    prec = M.make_precision(arith, q, packed, fmt, exact=exact)
    return M.make_run_config(eps, nested=nested, theta=0.5, L_min=2, L_max=L_max, n_pilot=n_pilot,
                             costs=costs, plain_arith=plain, prec=prec)


def _same(a, b, tag):
    for k in ("status", "L", "sweeps", "estimate", "variance", "path_steps", "saturations", "exact_sides"):
        assert a[k] == b[k], (tag, k, a[k], b[k])
    assert a["levels"] == b["levels"], tag


CASES = [
    # eps small enough that L grows past L_min + 1: levels prepared while the run waits
    ("nested-fp32-euro", "milstein", "euro", dict(nested=True, eps=0.0004)),
    ("nested-fp32-packed", "milstein", "euro", dict(nested=True, packed=True, eps=0.0004)),
    ("plain-fp32", "milstein", "euro", dict(nested=False, eps=0.0004)),
    ("plain-fp64-euler", "euler", "euro", dict(nested=False, plain="fp64")),
    ("nested-asian", "milstein", "asian", dict(nested=True)),
    ("nested-digital-switches", "milstein", "digital",
     dict(nested=True, eps=0.003, q=6, plain="fp64", costs=(1.0, 0.5, 2.9), n_pilot=10_000)),
    ("nested-fixed", "euler", "euro", dict(nested=True, arith="fixed")),
    ("nested-exact-fp32", "milstein", "euro", dict(nested=True, exact="fp32")),
    ("nested-fp16", "milstein", "euro", dict(nested=True, arith="fp16")),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_engine_equals_host_driven(ctx, case):
    name, scheme, payoff, kw = case
    print("engine case", name, flush=True)
    cfg = _cfg(**kw)
    prob = M.make_problem(scheme, (payoff,), **EURO)
    ctx.set_driver(False)
    a = ctx.estimate(prob, cfg, SEED, option=5)
    ctx.set_driver(True)
    b = ctx.estimate(prob, cfg, SEED, option=5)
    c = ctx.estimate(prob, cfg, SEED, option=5)          # the engine's graph replayed again
    _same(a, b, name)
    _same(b, c, name + " again")
    assert a["status"] == 0 and a["sweeps"] >= 2
    if kw.get("eps", 0.002) < 0.001:
        assert a["L"] >= 4, a["L"]


def _options(n, seed=7):
    rng = np.random.default_rng(seed)
    out = []
    kinds = ("euro", "asian", "digital")
    for i in range(n):
        out.append(M.make_problem("milstein", (kinds[i % 3],), S0=float(rng.uniform(80, 120)),
                                  K=float(rng.uniform(80, 120)), r=float(rng.uniform(0, 0.08)),
                                  sigma=float(rng.uniform(0.1, 0.5)), T=float(rng.uniform(0.25, 2.0))))
    return out


@pytest.mark.parametrize("nested", [True, False], ids=["nested", "plain"])
def test_engine_batch_equals_host_driven_batch(ctx, nested):
    probs = _options(24)
    cfg = _cfg(nested, eps=0.004, L_max=10, packed=True)
    print("engine batch nested", nested, flush=True)
    ctx.set_driver(False)
    a = ctx.estimate_batch(probs, cfg, SEED)
    ctx.set_driver(True)
    b = ctx.estimate_batch(probs, cfg, SEED)
    for i in range(len(probs)):
        _same(a[i], b[i], f"option {i}")
    # and each equals the option alone on the engine
    for i in (0, 7, 23):
        alone = ctx.estimate(probs[i], cfg, SEED, option=i)
        _same(alone, b[i], f"alone {i}")


def test_engine_small_workspace_falls_back():
    """A workspace that cannot hold the engine's arrays: host-driven sweeps, the same
    results."""
    cfg = _cfg(True, eps=0.004)
    prob = M.make_problem("milstein", ("euro",), **EURO)
    with M.Context(0, workspace_bytes=1 << 20) as small, M.Context(0, workspace_bytes=256 << 20) as big:
        small.set_driver(True)
        a = small.estimate_batch(_options(40), cfg, SEED)
        big.set_driver(False)
        b = big.estimate_batch(_options(40), cfg, SEED)
        for i in range(40):
            _same(a[i], b[i], f"option {i}")
        r1 = small.estimate(prob, cfg, SEED)
        r2 = big.estimate(prob, cfg, SEED)
        _same(r1, r2, "single")


def test_engine_reused_after_another_engine(ctx):
    """Engines of one context share its workspace: a cached engine used again after
    another one ran (here a plain run's engine, then the nested run's again, FP32 and
    FP16 tables built on the device) gives the host-driven result."""
    prob = M.make_problem("milstein", ("euro",), **EURO)
    for arith in ("fp32", "fp16"):
        nested, plain = _cfg(True, arith=arith, packed=True), _cfg(False)
        ctx.set_driver(False)
        ref = ctx.estimate(prob, nested, SEED, option=3)
        ctx.set_driver(True)
        first = ctx.estimate(prob, nested, SEED, option=3)
        ctx.estimate(prob, plain, SEED, option=4)
        again = ctx.estimate(prob, nested, SEED, option=3)
        _same(ref, first, arith)
        _same(ref, again, arith + " after another engine")


def test_auto_driver_equals_both():
    """The default driver (the engine for batches of at least MLMC_ENGINE_MIN_RUNS
    options, host-planned sweeps below) gives the results of either driver."""
    cfg = _cfg(True, eps=0.004, L_max=10, packed=True)
    with M.Context(0, workspace_bytes=256 << 20) as c:
        for n in (8, 70):
            probs = _options(n, seed=11)
            auto = c.estimate_batch(probs, cfg, SEED)
            c.set_driver(False)
            host = c.estimate_batch(probs, cfg, SEED)
            c.set_driver(True)
            eng = c.estimate_batch(probs, cfg, SEED)
            c.set_driver("auto")
            for i in range(n):
                _same(auto[i], host[i], f"{n} options, option {i} host")
                _same(auto[i], eng[i], f"{n} options, option {i} engine")


def test_engine_uploads_in_pieces():
    """Fixed-point runs with q = 12 tables (32 KB per level, built on the host): a
    batch's first upload is several times the engine's device staging area, so it
    goes in pieces (DMA copy, then scatter, per piece); the results equal the
    host-driven ones."""
    rng = np.random.default_rng(5)
    probs = [M.make_problem("euler", ("euro",), S0=float(rng.uniform(90, 110)), K=100.0, r=0.05, sigma=0.2, T=1.0)
             for _ in range(40)]
    prec = M.make_precision("fixed", 12, False, WIDE_FMT)
    cfg = M.make_run_config(0.004, nested=True, theta=0.5, L_min=2, L_max=6, n_pilot=2000,
                            costs=(1.0, 0.1, 1.1), plain_arith="fp32", prec=prec)
    with M.Context(0, workspace_bytes=256 << 20) as c:
        c.set_driver(False)
        a = c.estimate_batch(probs, cfg, SEED)
        c.set_driver(True)
        b = c.estimate_batch(probs, cfg, SEED)
        for i in range(len(probs)):
            _same(a[i], b[i], f"option {i}")
