"""GPU tests of the layers above one level sum, through the C ABI:

* enqueued batches (mlmc_level_sums_enqueue / _wait) equal synchronous runs, also
  when several are in flight, when the workspace ring wraps and when a synchronous
  call runs in between;
* the adaptive estimate follows the oracle's adaptive driver (same levels, same
  sample counts, estimate and variance within the summation-order bound);
* batched estimates and server requests equal the same option priced alone.
"""
import numpy as np
import pytest

import paper_2502_07123_amd as M
from oracle import mlmc as om
from oracle.paths import Precision as OPrecision
from oracle.paths import Problem as OProblem
from parity import GBM, SEED, WIDE, WIDE_FMT

pytestmark = pytest.mark.gpu

EURO = {k: v for k, v in GBM.items() if k != "barrier"}


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0, workspace_bytes=512 << 20)
    yield c
    c.close()


def _items(off=0):
    mil = M.make_problem("milstein", ("euro", "asian"), **GBM)
    eul = M.make_problem("euler", ("euro",), **GBM)
    p32 = M.make_precision("fp32", 8)
    pk = M.make_precision("fp32", 8, True)
    fx = M.make_precision("fixed", 8, False, WIDE_FMT)
    return [(mil, 0, 200_000, off, pk, M.EST_APPROX, SEED, 0),
            (mil, 3, 20_000, off, p32, M.EST_CORR, SEED, 0),
            (eul, 5, 7_001, off, fx, M.EST_APPROX, SEED, 1),
            (mil, 6, 3_000, off, fx, M.EST_CORR, SEED, 2),
            (eul, 2, 9_999, off, M.make_precision("fp64"), M.EST_PLAIN, SEED, 3),
            (mil, 4, 12_345, off, p32, M.EST_PLAIN, SEED, 4)]


def _sync(ctx, items):
    return [ctx.level_sums(p, l, n, o, pr, e, s, opt) for (p, l, n, o, pr, e, s, opt) in items]


def test_enqueued_batches_equal_synchronous_runs(ctx):
    a_items, b_items = _items(0), _items(50_000)
    ref_a, ref_b = _sync(ctx, a_items), _sync(ctx, b_items)
    A, B = ctx.sums_batch(a_items), ctx.sums_batch(b_items)
    ta, tb = A.enqueue(), B.enqueue()
    assert tb > ta > 0
    mid = _sync(ctx, a_items[:2])                      # a synchronous call between them
    B.wait(tb)
    A.wait(ta)
    assert A.as_dicts() == ref_a
    assert B.as_dicts() == ref_b
    assert mid == ref_a[:2]
    assert A.run() is A.sums and A.as_dicts() == ref_a
    assert ctx.level_sums_batch(b_items) == ref_b


def test_more_flights_than_room_land_in_order():
    """A small workspace: plans wrap around the ring and the oldest flights land
    before newer ones are placed."""
    with M.Context(0, workspace_bytes=2 << 20) as c:
        c.set_tuning(zb_max_paths=0)
        prob = M.make_problem("milstein", ("euro",), **GBM)
        prec = M.make_precision("fp32", 8)
        items = [[(prob, 0, 3_000_000, 10_000 * k, prec, M.EST_APPROX, SEED, 0),
                  (prob, 2, 40_000, 10_000 * k, prec, M.EST_CORR, SEED, 0)] for k in range(7)]
        refs = [_sync(c, it) for it in items]
        bs = [c.sums_batch(it) for it in items]
        ts = [b.enqueue() for b in bs]
        for k in (6, 0, 3, 1, 2, 5, 4):
            bs[k].wait(ts[k])
        for b, ref in zip(bs, refs):
            assert b.as_dicts() == ref


def test_ticket_errors(ctx):
    with pytest.raises(M.MlmcError) as e:
        ctx.sums_batch(_items()[:1]).wait(987654321)
    assert e.value.status == -7
    b = ctx.sums_batch(_items()[:1])
    t = b.enqueue()
    b.wait(t)
    with pytest.raises(M.MlmcError) as e:
        b.wait(t)
    assert e.value.status == -7


# ------------------------------------------------------------------ estimates
DRIVER_CASES = [
    # (nested, scheme, arith of the low-precision side / plain arithmetic, payoff)
    (False, "euler", "fp64", "euro"),
    (False, "milstein", "fp32", "euro"),
    (True, "milstein", "fp32", "euro"),
    (True, "euler", "fixed", "euro"),
    # levels >= 1 switch to plain FP64 samples (the table moves paths across the jump)
    (True, "milstein", "fp32", "digital"),
]


def _configs(nested, scheme, arith, eps=0.001, payoff="euro"):
    kw = dict(eps=eps, theta=0.5, L_min=2, L_max=6, n_pilot=2000)
    costs = (1.0, 0.1, 1.1)
    plain = arith if not nested else "fp32"
    q = 8
    if payoff == "digital":
        kw.update(eps=0.003, n_pilot=10_000)
        costs, plain, q = (1.0, 0.5, 2.9), "fp64", 6
    prec = M.make_precision(arith if nested else "fp32", q, False, WIDE_FMT if arith == "fixed" else None)
    cfg = M.make_run_config(nested=nested, plain_arith=plain, prec=prec, costs=costs, **kw)
    ocfg = om.RunConfig(nested=nested, plain_arith=plain, cost_plain=costs[0], cost_approx=costs[1],
                        cost_corr=costs[2], **kw)
    oprec = OPrecision(arith if nested else "fp32", q, False, WIDE if arith == "fixed" else ())
    return cfg, ocfg, oprec


@pytest.mark.parametrize("case", DRIVER_CASES, ids=lambda c: "-".join(map(str, c)))
def test_estimate_follows_the_oracle_driver(ctx, case):
    """Same levels, same estimator per level (R35), same sample counts; estimate and
    variance within the summation-order bound."""
    nested, scheme, arith, payoff = case
    cfg, ocfg, oprec = _configs(nested, scheme, arith, payoff=payoff)
    r = ctx.estimate(M.make_problem(scheme, (payoff,), **EURO), cfg, SEED, option=3)
    o = om.estimate(OProblem(scheme, **EURO), payoff, oprec, ocfg, SEED, option=3)
    assert r["status"] == 0
    assert r["L"] == o.L
    if payoff == "digital":                 # the per-level switch happened
        assert (1, M.EST_PLAIN) in o.sums and (0, M.EST_APPROX) in o.sums
    # plain FP32 uses its own FP32 inverse normal: its sums differ from the oracle's
    # by ~1e-7 relative, so an allocation may round one sample differently
    slack = 1 if (not nested and arith == "fp32") else 0
    same_n = True
    for l in range(o.L + 1):
        for e in (M.EST_PLAIN, M.EST_APPROX, M.EST_CORR):
            want = o.sums[(l, e)].n if (l, e) in o.sums else 0
            d = abs(r["levels"][l]["n"][e] - want)
            assert d <= slack, (l, e)
            same_n = same_n and d == 0
    if not slack:
        tol_m, tol_v = 1e-10, 1e-8          # FP64 summation order only
    elif same_n:
        tol_m, tol_v = 1e-5, 1e-4           # FP32 paths within their derived bound
    else:
        tol_m, tol_v = 2e-3, 1e-2           # one sample more or less somewhere
    assert abs(r["estimate"] - o.estimate) <= tol_m * abs(o.estimate)
    assert abs(r["variance"] - o.variance) <= tol_v * o.variance


def _strikes():
    return [M.make_problem("milstein", ("euro",), **{**EURO, "K": k}) for k in (90.0, 100.0, 110.0)]


def test_batched_estimates_equal_each_alone(ctx):
    cfg, _, _ = _configs(True, "milstein", "fp32", eps=0.003)
    probs = _strikes()
    batch = ctx.estimate_batch(probs, cfg, SEED)
    for i, p in enumerate(probs):
        alone = ctx.estimate(p, cfg, SEED, option=i)
        for k in ("estimate", "variance", "L", "levels", "path_steps"):
            assert batch[i][k] == alone[k], (i, k)


def _collect(ctx, tickets, timeout=60.0):
    import time
    got = {}
    t_end = time.time() + timeout
    while len(got) < len(tickets) and time.time() < t_end:
        for t, r in ctx.poll_done(64):
            got[t] = r
        time.sleep(0.0005)
    return got


def _mix():
    """(problem, eps, nested) of six requests: three strikes, nested and plain FP32."""
    out = []
    for i, p in enumerate(_strikes()):
        out.append((p, 0.003, True))
        out.append((p, 0.004 + 0.001 * i, False))
    return out


@pytest.mark.parametrize("drv", ["engine", "host"])
@pytest.mark.parametrize("max_active,ws", [(1, 512 << 20), (64, 512 << 20), (4, 1 << 20)],
                         ids=["1-slot", "64-slots", "4-slots-1MiB"])
def test_server_results_equal_each_alone(ctx, max_active, ws, drv):
    """Requests submitted in two waves (the second while the first run) with mixed
    eps and estimators: each result equals mlmc_estimate of the same request alone,
    also with one slot and with a 1 MiB workspace (plans of several launch
    sequences), with the runs in device engine slots or planned on the host."""
    import time
    c = ctx if ws == (512 << 20) else M.Context(0, workspace_bytes=ws)
    c.set_driver(drv == "engine")
    try:
        cfg, _, _ = _configs(True, "milstein", "fp32", eps=0.003)
        reqs = _mix()
        alone = []
        for i, (p, eps, nested) in enumerate(reqs):
            cfg.eps, cfg.nested = eps, 1 if nested else 0
            alone.append(c.estimate(p, cfg, SEED + 7, option=10 + i))
        cfg.eps, cfg.nested = 0.003, 1
        c.server_start(cfg, max_active=max_active)
        try:
            tickets = [c.submit(p, eps, SEED + 7, option=10 + i, nested=nested)
                       for i, (p, eps, nested) in enumerate(reqs[:2])]
            time.sleep(0.002)
            tickets += [c.submit(p, eps, SEED + 7, option=12 + i, nested=nested)
                        for i, (p, eps, nested) in enumerate(reqs[2:])]
            got = _collect(c, tickets)
            assert len(got) == len(tickets)
        finally:
            c.server_stop()
        for t, a in zip(tickets, alone):
            assert got[t]["status"] == 0
            assert got[t]["seconds"] > 0
            for k in ("estimate", "variance", "L", "levels", "path_steps"):
                assert got[t][k] == a[k], k
    finally:
        c.set_driver("auto")
        if c is not ctx:
            c.close()


def test_server_poll_and_stop(ctx):
    """mlmc_poll and mlmc_poll_done hand each result out once; stopping cancels the
    requests not yet admitted and finishes the admitted one."""
    cfg, _, _ = _configs(True, "milstein", "fp32", eps=0.003)
    p = _strikes()[1]
    ctx.server_start(cfg, max_active=1)
    try:
        t0 = ctx.submit(p, 0.003, SEED, option=1)
        queued = [ctx.submit(p, 0.003, SEED, option=2 + i) for i in range(3)]
    finally:
        ctx.server_stop()
    with pytest.raises(M.MlmcError):
        ctx.poll(t0)                        # no server any more
    ctx.server_start(cfg, max_active=2)
    try:
        t1 = ctx.submit(p, 0.003, SEED, option=1)
        got = _collect(ctx, [t1])
        assert list(got) == [t1] and got[t1]["status"] == 0
        assert ctx.poll_done(8) == []
        with pytest.raises(M.MlmcError):
            ctx.poll(t1)                    # already handed out
        t2 = ctx.submit(p, 0.003, SEED, option=1)
        r = None
        for _ in range(60000):
            r = ctx.poll(t2)
            if r is not None:
                break
            import time
            time.sleep(0.001)
        assert r is not None and r["estimate"] == got[t1]["estimate"]
        assert ctx.poll_done(8) == []       # taken by mlmc_poll
    finally:
        ctx.server_stop()


def test_autotune_keeps_results_valid():
    """mlmc_autotune picks a geometry from its candidate sets, leaves it on the
    context, and the work list's results stay what they must be: exact integer sums
    identical (they do not depend on the tile split), FP64 sums within rounding."""
    c = M.Context(0, workspace_bytes=256 << 20)
    try:
        items = _items()
        before = c.level_sums_batch(items)
        b = c.sums_batch(items)
        t = c.autotune(b, reps=2)
        assert t == c.get_tuning()
        assert t["block_table"] in (256, 512, 1024) and t["block_exact"] in (64, 128, 256)
        assert t["tile_steps"] in [1 << k for k in range(14, 19)] and t["blocks_per_cu"] in (2, 4, 8, 16)
        assert t["min_tiles"] in (512, 1024, 2048, 4096) and t["zb_max_paths"] in (0, 1 << 13, 1 << 15, 1 << 17)
        assert t["overlap_min_steps"] in (0, 1 << 24, 1 << 26, 1 << 28, (1 << 64) - 1)
        after = c.level_sums_batch(items)
        for i, (a, z) in enumerate(zip(before, after)):
            for p in a:
                assert a[p]["n"] == z[p]["n"] and a[p]["isum1"] == z[p]["isum1"] and a[p]["isum2"] == z[p]["isum2"]
                n = a[p]["n"]
                for k1, k2 in (("sum1", "sum2"), ("esum1", "esum2")):
                    # |Y| summed <= sqrt(n sum Y^2): two summation orders differ by at most
                    # 2 n 2^-53 times that (and 2 n 2^-53 sum Y^2 for the squares)
                    tol1 = 4 * n * 2.0 ** -53 * (n * a[p][k2]) ** 0.5 + 1e-300
                    tol2 = 4 * n * 2.0 ** -53 * a[p][k2] + 1e-300
                    assert abs(a[p][k1] - z[p][k1]) <= tol1, (i, p, k1)
                    assert abs(a[p][k2] - z[p][k2]) <= tol2, (i, p, k2)
    finally:
        c.close()


def _items_with_level0(off=0):
    """_items plus level-0 works of the exact-normal estimators (the level-0 kernel,
    on the third stream of a two-stream flight)."""
    mil = M.make_problem("milstein", ("euro", "asian"), **GBM)
    eul = M.make_problem("euler", ("euro",), **GBM)
    return _items(off) + [(mil, 0, 50_001, off, M.make_precision("fp32", 8), M.EST_CORR, SEED, 5),
                          (eul, 0, 30_000, off, M.make_precision("fp64"), M.EST_PLAIN, SEED, 6)]


@pytest.mark.parametrize("how", ["sync", "enqueued", "estimate", "server"])
def test_two_stream_flights_equal_one_stream(how):
    """Flights that put the approximate works on the second stream (each stream with
    its own plan copy, reduction and download, results returned in work order) and
    the level-0 exact-normal works on a third give the same sums as one-stream
    flights: synchronous batches, several enqueued batches in flight, an adaptive
    estimate and the server."""
    c = M.Context(0, workspace_bytes=256 << 20)
    try:
        items = _items_with_level0()
        runs = []
        for thr in ((1 << 64) - 1, 0):
            c.set_tuning(overlap_min_steps=thr)
            if how == "sync":
                runs.append(c.level_sums_batch(items))
            elif how == "enqueued":
                bs = [c.sums_batch(_items_with_level0(off=1000 * k)) for k in range(3)]
                for b in bs:
                    b.enqueue()
                out = []
                for b in bs:
                    b.wait()
                    out.append(b.as_dicts())
                runs.append(out)
            elif how == "estimate":
                cfg, _, _ = _configs(True, "milstein", "fp32", eps=0.003)
                runs.append([c.estimate(p, cfg, SEED, option=i) for i, p in enumerate(_strikes())])
            else:
                cfg, _, _ = _configs(True, "milstein", "fp32", eps=0.003)
                c.server_start(cfg, max_active=8)
                try:
                    tickets = [c.submit(p, 0.003, SEED, option=i) for i, p in enumerate(_strikes())]
                    got = _collect(c, tickets)
                finally:
                    c.server_stop()
                runs.append([got[t] for t in tickets])
        if how in ("estimate", "server"):
            for r in runs:
                for x in r:
                    x.pop("seconds")                # wall time, not a result
        assert runs[0] == runs[1]
    finally:
        c.close()


def test_estimate_states_its_exact_side(ctx):
    """The correction's exact side (reading R21): FP64 by default, FP32 on request;
    the result says which, and both estimates agree with the closed form within
    their error (the FP32 side changes the correction's samples by ~1e-7)."""
    from math import erf, exp, log, sqrt
    N = lambda x: 0.5 * (1.0 + erf(x / sqrt(2.0)))
    d1 = (log(EURO["S0"] / EURO["K"]) + (EURO["r"] + 0.5 * EURO["sigma"] ** 2) * EURO["T"]) / (
        EURO["sigma"] * sqrt(EURO["T"]))
    bs = EURO["S0"] * N(d1) - EURO["K"] * exp(-EURO["r"] * EURO["T"]) * N(d1 - EURO["sigma"] * sqrt(EURO["T"]))
    prob = M.make_problem("milstein", ("euro",), **EURO)
    out = {}
    for exact, bit in (("fp64", 1), ("fp32", 2)):
        prec = M.make_precision("fp32", 8, exact=exact)
        cfg = M.make_run_config(0.002, nested=True, prec=prec, theta=0.5, L_min=2, L_max=8, n_pilot=5000)
        r = ctx.estimate(prob, cfg, SEED, option=1)
        assert r["status"] == 0 and r["exact_sides"] & 3 == bit
        out[exact] = r
        assert abs(r["estimate"] - bs) < 4 * 0.002 * EURO["S0"], (exact, r["estimate"], bs)
    # same uniforms: the two runs' level-0 correction means differ only by FP32 rounding
    m64 = out["fp64"]["levels"][0]["mean"][M.EST_CORR]
    m32 = out["fp32"]["levels"][0]["mean"][M.EST_CORR]
    assert abs(m64 - m32) < 1e-5
