"""Benchmark: nested MLMC hot path on one MI355X.

Workload (default): the nested approximate-normal MLMC of a European call on GBM
(S0 = K = 100, r = 0.05, sigma = 0.2, T = 1), Milstein, levels 0..8; the
approximate estimator uses the Method-1 table with q = 8 (packed 8-bit indices,
four per 32-bit word) in FP32, the correction estimator FP64 minus FP32 on the same
uniforms; N_l (approximate) and M_l (correction) come from the nested optimal
allocation at eps = 1e-3 in price units (variance eps^2, theta = 1) after an
untimed pilot.  One step = all 18 (level, estimator) level sums in one launch
sequence plus the host combination into the price estimate; consecutive steps are
pipelined (the host marshals and enqueues the next steps while step k runs, three
steps in flight by default).

Printed: one JSON line (metric path-steps/s), with the VALU roofline of the
dominant kernel (the one with the most algorithmic work; HIP-event timing inside
the timed region), the CPU oracle timed on
a bounded sample, and the time to RMSE eps of the nested estimator against plain
FP32 MLMC on the same GPU.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GBM = dict(S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0)
LEVELS = 9
Q = 8
EPS = 1e-3                 # price units
SEED = 1234
N_PILOT = 100_000

# --- algorithmic VALU work per fine path-step (32-bit lane operations; a multiply
# counts one), by kernel class, as the method's own operation counts:
#   uniform word: a quarter of a Philox4x32-10 call (5 32x32 multiplies for the
#     high and low halves, ~7.5 xors/adds), shared by the indices packed in it;
#   table index: 1.5 (shift, mask when packed);
#   exact inverse normal: ~25 (FP32) or ~60 (FP64, with its logarithm);
#   fine step: 2 (FP32/FP16/FP64 FMA pair) or 12 (fixed point: product, rounding,
#     shift, saturation of two operations), Milstein +3 (zsq, zm1, mul3);
#   coarse step, per fine step (levels >= 1): 1.5 (fixed point 6.5), Milstein +1.5;
#   Asian / barrier functionals: +1.5 each per fine step;
#   per path: payoff, level difference and the two sums, ~4 per side.
PHILOX_WORD_OPS = 12.5
INDEX_OPS = 1.5
NORMINV_OPS = {0: 60.0, 1: 25.0}          # arith FP64, FP32
ARITH_FIXED = 3


def side_step_ops(arith, scheme, level, track=0):
    mil = scheme == 1
    fixed = arith == ARITH_FIXED
    ops = (12.0 if fixed else 2.0) + (3.0 if mil else 0.0)
    if level >= 1:
        ops += (6.5 if fixed else 1.5) + (1.5 if mil else 0.0)
    return ops + 1.5 * track


def alg_ops_per_step(est, fields, scheme, level, arith=1, track=0):
    """Algorithmic lane-ops per fine path-step of one sample of estimator est
    (0 plain, 1 approximate, 2 correction); arith: the table side's arithmetic
    (approximate, correction) or the plain side's (plain).  The correction estimator
    runs the FP64 exact side and the table side on one word per step."""
    per_path = 4.0
    if est == 1:
        ops = PHILOX_WORD_OPS / fields + INDEX_OPS + side_step_ops(arith, scheme, level, track)
    elif est == 2:
        ops = (PHILOX_WORD_OPS + INDEX_OPS + NORMINV_OPS[0] + side_step_ops(0, scheme, level, track)
               + side_step_ops(arith, scheme, level, track))
        per_path = 8.0
    else:
        ops = PHILOX_WORD_OPS + NORMINV_OPS[0 if arith == 0 else 1] + side_step_ops(arith, scheme, level, track)
    return ops + per_path / (1 << level)


def dominant_kernel(stats, Na, Nc):
    """The timed kernel with the most algorithmic lane-ops per step, and those ops: its
    works' sample counts (Na for the approximate estimator, Nc otherwise) level by
    level times the ops per path-step.  Event times are no guide: when the two streams'
    kernels run concurrently an event pair also spans the time its kernel waits behind
    the other stream's."""
    def ops(k):
        N = Na if k["estimator"] == 1 else Nc
        return sum(int(N[l]) * (1 << l) * alg_ops_per_step(k["estimator"], k["fields"], k["scheme"], l,
                                                           k.get("arith", 1), k.get("track", 0))
                   for l in range(LEVELS))
    dom = max(stats, key=ops)
    return dom, ops(dom)


def peak_valu():
    """Full-rate 32-bit VALU lane-ops/s of MI355X: 256 CUs x 128 lanes/clk x 2.4 GHz
    (the 157.3 TFLOP/s FP32 vector figure is 78.6e12 FMA lane-ops/s)."""
    return 256 * 128 * 2.4e9


def make_items(M, prob, prec_a, prec_c, Na, Nc, offset):
    items = []
    for l in range(LEVELS):
        items.append((prob, l, int(Na[l]), offset, prec_a, M.EST_APPROX, SEED, 0))
        items.append((prob, l, int(Nc[l]), offset, prec_c, M.EST_CORR, SEED, 0))
    return items


# kernel sources whose change invalidates recorded HBM counters
KERNEL_SOURCES = ("paper_2502_07123_amd/csrc/kernels.hip", "paper_2502_07123_amd/csrc/kernels.hpp",
                  "paper_2502_07123_amd/csrc/common.hpp", "paper_2502_07123_amd/csrc/device/paths.hpp",
                  "paper_2502_07123_amd/csrc/device/philox.hpp", "paper_2502_07123_amd/csrc/device/norminv.hpp",
                  "paper_2502_07123_amd/csrc/device/fixed.hpp", "paper_2502_07123_amd/csrc/device/reduce.hpp")
TRAFFIC_RECORD = "profiles/k_paths_approx_milstein_euro_L0_8_hbm_traffic.md"
SQ_RECORD = "profiles/k_paths_nested_milstein_euro_L0_8_sq_counters.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _record(path, tag, kernel):
    """The JSON record after `tag` in a committed profile summary, if it is for
    `kernel` and the kernel sources have not changed since it was taken."""
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith(tag):
            rec = json.loads(line[len(tag):])
            if rec.get("source_sha256") != kernel_source_hash() or rec.get("kernel") != kernel:
                return None
            return rec
    return None


def recorded_sq(kernel):
    """VALU busy and issue-cost utilisation of `kernel` from the committed SQ counter
    pass (definitions in that summary), or None once the kernel sources changed."""
    rec = _record(SQ_RECORD, "sq_record: ", kernel)
    return None if rec is None else {"valu_busy": rec["valu_busy"], "issue_cost_util": rec["issue_cost_util"]}


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (scaled by the copy-probe factors recorded there), or None
    when the kernel sources changed since the counters were taken."""
    rec = _record(TRAFFIC_RECORD, "traffic_record: ", kernel)
    if rec is None:
        return None
    return rec["fetch_kib"] * 1024 * rec["fetch_scale"] + rec["write_kib"] * 1024 * rec["write_scale"]


def combine_np(S, scale):
    """Price estimate and its standard error from a batch's sums (R9 variances)."""
    import numpy as np
    s = S[:, 0]
    n = s["n"].astype(np.float64)
    m = s["sum1"] / n
    v = np.maximum((s["sum2"] - s["sum1"] ** 2 / n) / (n - 1.0), 0.0)
    return scale * float(m.sum()), scale * math.sqrt(float((v / n).sum()))


def level_mean(S, l, scale):
    """Mean of the level-l correction E[Y_l] (approximate + correction estimator) of a
    batch laid out as make_items lays it out, in price units."""
    s = S[:, 0]
    return scale * float(s["sum1"][2 * l] / s["n"][2 * l] + s["sum1"][2 * l + 1] / s["n"][2 * l + 1])


def _oracle_work(item):
    """One chunk of the CPU baseline: (level, estimator, path offset, paths, packed)."""
    from oracle.mlmc import level_sums
    from oracle.paths import Precision, Problem
    l, est, off, n, packed = item
    level_sums(Problem("milstein", barrier=0.0, **GBM), l, n, off, Precision("fp32", Q, packed), est, SEED, 0,
               ("euro",))
    return n << l


def oracle_pool():
    """Worker processes for the CPU baseline, forked before anything touches the GPU
    (a process that has initialised the GPU forks no workers); one per core of this
    process's affinity set, at most 16."""
    import multiprocessing as mp
    P = max(1, min(16, len(os.sched_getaffinity(0))))
    return mp.get_context("fork").Pool(P), P


def _sample_items(Na, Nc, f, parts):
    items = []
    for l in range(LEVELS):
        for est, N, packed in ((1, Na[l], True), (2, Nc[l], False)):
            n = max(256, int(round(int(N) * f)))
            k = max(1, min(parts, n // 256))
            for j in range(k):
                a, b = n * j // k, n * (j + 1) // k
                items.append((l, est, a, b - a, packed))
    return items


def cpu_baseline(Na, Nc, pool=None, P=1, budget_1core=6e7, budget_per_core=1.5e8):
    """The oracle on a bounded sample of the same works (same levels and estimators,
    sample sizes proportional to N_l, M_l), as it stands (numpy, vectorised across
    paths): first on one core, then over P worker processes with disjoint path
    ranges of a sample P times larger."""
    total = sum(int(Na[l]) << l for l in range(LEVELS)) + sum(int(Nc[l]) << l for l in range(LEVELS))
    f1 = min(1.0, budget_1core / total)
    t0 = time.perf_counter()
    steps1 = sum(_oracle_work(it) for it in _sample_items(Na, Nc, f1, 1))
    one = steps1 / (time.perf_counter() - t0)
    out = {"value": one, "unit": "path-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{steps1:.3g} fine path-steps: the 18 (level, estimator) works with N_l, M_l "
                     f"scaled by {f1:.3g} (>= 256 paths each), numpy on one core",
           "value_1core": one}
    if pool is None or P <= 1:
        return out
    fP = min(1.0, budget_per_core * P / total)
    items = _sample_items(Na, Nc, fP, 4 * P)
    t0 = time.perf_counter()
    stepsP = sum(pool.map(_oracle_work, items, chunksize=1))
    out.update(value=stepsP / (time.perf_counter() - t0), cores=P,
               sample=f"{stepsP:.3g} fine path-steps: the 18 (level, estimator) works with N_l, M_l scaled "
                      f"by {fP:.3g} (>= 256 paths each), split into disjoint path ranges over {P} worker "
                      f"processes (numpy); one core alone: {one:.3g} path-steps/s on {steps1:.3g}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tte", action="store_true", help="skip the time-to-eps comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 256 MiB device-to-device (a known-size kernel that scales "
                         "the HBM byte counters of a profile)")
    ap.add_argument("--batch", action="store_true",
                    help="instead: the 256-option batched workload (nested vs plain FP32)")
    ap.add_argument("--batch-eps", default="1e-2,1e-3,1e-4")
    ap.add_argument("--drivers", default="engine,host",
                    help="sweep drivers of --batch / --serving: engine (device run states, graph "
                         "replays) and/or host (sweeps planned on the host)")
    ap.add_argument("--serving", action="store_true",
                    help="instead: Poisson-arrival serving, p50/p99 latency (nested vs plain FP32)")
    ap.add_argument("--serve-rates", default="1000,5000,20000")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--depth", type=int, default=3,
                    help="steps in flight: marshalled batches that alternate (1..4)")
    ap.add_argument("--tuning", default=None,
                    help="launch geometry as JSON (fields of mlmc_tuning) in place of the tuner")
    ap.add_argument("--per-level", action="store_true",
                    help="instead: path-steps/s per level for each kernel class")
    ap.add_argument("--configs", action="store_true",
                    help="instead: the plain FP64 Euler workload (levels 0..4, 1e5 paths per level) and "
                         "time to eps at fixed L with table sizes q = 4, 6, 8")
    ap.add_argument("--fixed-sweep", action="store_true",
                    help="instead: the fixed-point workload (Euler, 1e6 paths per level, levels 0..10, "
                         "European + Asian + barrier on the same paths)")
    args = ap.parse_args()
    if not 1 <= args.depth <= 4:
        ap.error("--depth must be 1..4")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    if args.batch or args.serving or args.per_level or args.fixed_sweep or args.configs:
        return main_workloads(args)
    pool, P = (None, 1) if args.no_cpu else oracle_pool()
    import numpy as np
    import torch
    import paper_2502_07123_amd as M

    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = M.Context(0, workspace_bytes=1 << 30)
    prob = M.make_problem("milstein", ("euro",), **GBM)
    prec_a = M.make_precision("fp32", Q, packed=True)
    prec_c = M.make_precision("fp32", Q, packed=False)
    scale = math.exp(-GBM["r"] * GBM["T"]) * GBM["S0"]
    eps_int = EPS / scale

    # cost model (R11: per-estimator ns per fine path-step, frozen for the run) from
    # large launches, then the pilot for the variances (all untimed)
    c_a, c_c, c_p = calibrate(M, ctx, prob, prec_a, prec_c)
    pil = ctx.level_sums_batch(make_items(M, prob, prec_a, prec_c, [N_PILOT] * LEVELS,
                                          [N_PILOT] * LEVELS, 0))

    def var(s):
        n = s["n"]
        return max((s["sum2"] - s["sum1"] ** 2 / n) / (n - 1), 1e-300)

    Va = [var(pil[2 * l]["euro"]) for l in range(LEVELS)]
    Vc = [var(pil[2 * l + 1]["euro"]) for l in range(LEVELS)]
    V = np.array(Va + Vc)
    Cst = np.array([c_a * 2 ** l for l in range(LEVELS)] + [c_c * 2 ** l for l in range(LEVELS)])
    N = M.allocate(V, Cst, eps_int ** 2, 1.0)          # Section 2.2 allocation, theta = 1
    Na, Nc = N[:LEVELS], N[LEVELS:]
    path_steps = int(sum(int(Na[l]) << l for l in range(LEVELS)) + sum(int(Nc[l]) << l for l in range(LEVELS)))

    # --depth marshalled batches (3 by default) rotate so that the host prepares the
    # next steps while the GPU runs the current one, with room for the host's own
    # pauses; each step draws fresh paths (path offsets advance)
    batches = [ctx.sums_batch(make_items(M, prob, prec_a, prec_c, Na, Nc, 0)) for _ in range(args.depth)]
    # launch geometry for this work list by the library's tuner (untimed), or the one
    # given (profiled runs: the tuner's timings are not those of an unprofiled run)
    if args.tuning:
        ctx.set_tuning(**json.loads(args.tuning))
        tuning = ctx.get_tuning()
    else:
        tuning = ctx.autotune(batches[0], reps=20)
    off = N_PILOT
    ests, top = [], []

    host = {"enqueue_s": 0.0, "wait_s": 0.0}
    done_at = []                       # completion times of the timed steps (D5)

    def run_steps(k_steps, record):
        nonlocal off
        for k in range(k_steps):
            b = batches[k % args.depth]
            if b._pending is not None:
                t1 = time.perf_counter()
                b.wait()
                host["wait_s"] += time.perf_counter() - t1
                if record:
                    done_at.append(time.perf_counter())
                    ests.append(combine_np(b.sums, scale))
                    top.append(level_mean(b.sums, LEVELS - 1, scale))
            b.offsets[:] = off
            off += int(max(N))
            t1 = time.perf_counter()
            b.enqueue()
            host["enqueue_s"] += time.perf_counter() - t1
        for k in range(k_steps, k_steps + args.depth):
            b = batches[k % args.depth]
            if b._pending is not None:
                b.wait()
                if record:
                    done_at.append(time.perf_counter())
                    ests.append(combine_np(b.sums, scale))
                    top.append(level_mean(b.sums, LEVELS - 1, scale))

    # per-kernel timing on during the warm-up too, so that its events exist before the
    # timed region (they are created on first use); switching it on again clears the
    # warm-up's launches from the statistics (all of them have landed)
    # no Python garbage collection from here through the timed region (as timeit
    # does): a full collection stalls the host longer than the queued steps and leaves
    # its caches cold; it runs before the warm-up, which warms them again
    gc.collect()
    gc.disable()
    ctx.set_timing(True)
    # the warm-up takes the timed steps' own path, the per-step combination of the
    # results included (its first calls are slow); its records are dropped
    run_steps(args.warmup, True)
    del done_at[:], ests[:], top[:]
    host.update(enqueue_s=0.0, wait_s=0.0)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(args.steps, True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gc.enable()
    stats = ctx.kernel_stats()
    ctx.set_timing(False)
    ms_step = dt * 1e3 / args.steps
    value = path_steps / (dt / args.steps)

    # roofline of the dominant kernel
    dom, ops = dominant_kernel(stats, Na, Nc)
    per_step_steps = dom["path_steps"] / args.steps
    # the kernel's time per step (its launches of one step together cover the mix)
    avg_s = dom["ms"] / args.steps * 1e-3
    achieved = ops / avg_s
    kname = (f"k_paths<{dom['estimator']}, {dom['arith']}, {'true' if dom['scheme'] else 'false'}, "
             f"{dom['payoffs']}, {'true' if dom['track'] else 'false'}, {dom['fields']}>")
    sq = recorded_sq(kname)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak_valu() / 1e12,
                "unit": "Tlane-op/s", "frac": achieved / peak_valu(),
                "traffic": recorded_traffic(kname),
                # from the committed SQ pass of the same kernel (null once its sources change)
                "valu_busy": None if sq is None else sq["valu_busy"],
                "issue_cost_util": None if sq is None else sq["issue_cost_util"],
                "kernel": {"estimator": dom["estimator"], "fields": dom["fields"],
                           "launches_per_step": dom["launches"] / args.steps,
                           "avg_launch_ms": dom["ms"] / dom["launches"],
                           "path_steps_per_step": per_step_steps,
                           "alg_lane_ops_per_step": ops}}

    # per-step times: intervals between consecutive step completions in the timed
    # region (steps are pipelined, so these are the throughput intervals)
    iv = np.diff(np.asarray([t0] + done_at)) * 1e3
    step_ms = {"median": float(np.median(iv)), "p10": float(np.percentile(iv, 10)),
               "p90": float(np.percentile(iv, 90)), "steps": int(iv.size)}
    bs = closed_form(dict(GBM, kind="euro"))
    last = ests[-1][0]
    bias = -float(np.mean(top))
    extra = {
        "estimate": float(np.mean([e[0] for e in ests])),
        "rmse_bound": float(ests[-1][1]),
        # one step's estimate against the Black-Scholes price (discretisation bias of
        # levels 0..8 plus sampling error; the step's RMSE target is eps)
        "closed_form": bs, "step_error": last - bs, "step_error_over_eps": (last - bs) / EPS,
        # the finest level's bias, -sum_{l>L} E[Y_l] ~ -E[Y_L] at weak order 1, from the
        # timed steps' level-L means; the step error less it is the sampling error
        "bias_estimate": bias, "step_error_less_bias": last - bs - bias,
        "N_approx": [int(x) for x in Na], "N_corr": [int(x) for x in Nc],
        "ms_per_step_distribution": step_ms,
        "tuning": tuning,
        # host time per timed step in the library's enqueue (planning, copies, launches)
        # and in the wait for the step two back (the GPU still busy)
        "host_us_per_step": {k[:-2]: v * 1e6 / args.steps for k, v in host.items()},
        "kernels": [{"estimator": s["estimator"], "arith": s["arith"], "fields": s["fields"],
                     "level0_kernel": s["level0"], "exact32": s["exact32"],
                     "launches": s["launches"], "ms": s["ms"],
                     "path_steps_per_s": s["path_steps"] / (s["ms"] * 1e-3)} for s in stats],
    }
    if not args.no_tte:
        extra["time_to_eps"] = time_to_eps(M, ctx, prob, prec_a, c_a, c_c, c_p, scale)
    cpu = None if args.no_cpu else cpu_baseline(Na, Nc, pool, P)
    if pool is not None:
        pool.close()
        pool.join()
    line = {
        "metric": "path-steps/s per level; time to RMSE eps, nested low-prec vs plain FP32",
        "value": value, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "nested MLMC, European call on GBM, Milstein, levels 0..8, "
                               "q=8 Method-1 table (packed), FP32 approx + FP64 correction, "
                               "allocation at eps=1e-3 (price units)",
                   "path_steps_per_step": path_steps},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line))
    ctx.close()


def calibrate(M, ctx, prob, prec_a, prec_c, level=4, n=1 << 22, exact32=False):
    """ns per fine path-step of the approximate, correction and plain-FP32 kernels
    (and, with exact32, of the correction with an FP32 exact side), from one large
    launch each (after a warm-up launch)."""
    out = []
    kinds = [(M.EST_APPROX, prec_a), (M.EST_CORR, prec_c), (M.EST_PLAIN, M.make_precision("fp32", Q))]
    if exact32:
        kinds.append((M.EST_CORR, M.make_precision("fp32", Q, exact="fp32")))
    for est, prec in kinds:
        ctx.level_sums(prob, level, n, 0, prec, est, SEED + 99)
        ctx.set_timing(True)
        ctx.level_sums(prob, level, n, n, prec, est, SEED + 99)
        st = ctx.kernel_stats()[0]
        ctx.set_timing(False)
        out.append(st["ms"] * 1e6 / st["path_steps"])
    return tuple(out)


TTE_SEEDS = 32
TTE_PILOT = 10_000         # pilot paths per (level, estimator)
# 2.5% and 97.5% quantiles of chi-square with 32 degrees of freedom: the 95% interval
# of the true RMSE is rmse * sqrt(32 / q) for q in (CHI2_HI, CHI2_LO)
CHI2_LO, CHI2_HI = 18.291, 49.480


def level_reference(M, ctx, prob, scale):
    """E[P_L] of the finest level L = LEVELS - 1 in price units: the Black-Scholes
    price less the discrete-time corrections above L, sum_{l>L} E[Y_l], from plain
    FP64 level sums at L+1 .. L+6 (2^16 paths at L+1, halving per level) plus
    E[Y_{L+6}] once more for the tail (weak order 1).  Returns (value, std error)."""
    prec = M.make_precision("fp64", Q)
    lv = list(range(LEVELS, LEVELS + 6))
    res = ctx.level_sums_batch([(prob, l, (1 << 16) >> i, 0, prec, M.EST_PLAIN, SEED + 77, 0)
                                for i, l in enumerate(lv)])
    m = v = 0.0
    for i, r in enumerate(res):
        s = r["euro"]
        n = s["n"]
        w = 2.0 if i == len(lv) - 1 else 1.0
        m += w * s["sum1"] / n
        v += w * w * max((s["sum2"] - s["sum1"] ** 2 / n) / (n - 1), 0.0) / n
    return closed_form(dict(GBM, kind="euro")) - scale * m, scale * math.sqrt(v)


ARITH_NAMES = {1: "fp32", 2: "fp16", 3: "fixed"}


def chosen_sides(M, ctx, prob, L_max=10, n_paths=1 << 16, q=8):
    """Per-level table sides by Section 6's level objective with the measured
    instruction-class costs (mlmc_choose_precision) from each level's error model
    (sensitivities on the GPU over n_paths paths)."""
    precs, info = [], []
    for l in range(L_max + 1):
        m = ctx.error_model(prob, l, n_paths, q, SEED + 555)
        p, c = M.choose_precision(m)
        precs.append(p)
        info.append({"level": l, "arith": ARITH_NAMES[c["arith"]], "q": c["table_bits"], "packed": c["packed"],
                     "objective_over_fp32_q8": c["objective"] / c["objective_fp32_q8"]})
    return precs, info


def time_to_eps(M, ctx, prob, prec_a, c_a, c_c, c_p, scale):
    """Wall time of one on-line MLMC estimate to RMSE eps (price units), nested (FP32
    table + FP64 correction; also with the correction's exact side in FP32) vs plain
    FP32 (exact FP32 normals), each over TTE_SEEDS seeds, in two settings:
      fixed:    levels 0..8, theta = 1 (the whole budget on the sampling variance at
                the fixed finest level L), RMSE about E[P_L] (the level-L reference);
      adaptive: theta = 1/2, L from 2 up to 10 by the bias test, RMSE about the
                Black-Scholes price (bias and sampling error together).
    Costs are the calibrated ns per path-step of each kernel class."""
    import numpy as np
    ref, ref_se = level_reference(M, ctx, prob, scale)
    bs = closed_form(dict(GBM, kind="euro"))
    c_x = calibrate(M, ctx, prob, prec_a, M.make_precision("fp32", Q), exact32=True)[3]
    prec_x = M.make_precision("fp32", Q, packed=True, exact="fp32")
    chosen, choices = chosen_sides(M, ctx, prob)
    out = {"reference_level_L": ref, "reference_se": ref_se, "closed_form": bs, "seeds": TTE_SEEDS,
           "cost_ns_per_step": {"plain_fp32": c_p, "approx": c_a, "corr": c_c, "corr_exact_fp32": c_x},
           "chosen_sides": choices}
    modes = (("nested", True, prec_a, c_c), ("nested_exact_fp32", True, prec_x, c_x),
             ("nested_chosen", True, chosen, c_c), ("plain_fp32", False, prec_a, c_c))
    for setting, kw, truth in (("fixed", dict(theta=1.0, L_min=8, L_max=8), ref),
                               ("adaptive", dict(theta=0.5, L_min=2, L_max=10), bs)):
        res = {}
        for name, nested, prec, cc in modes:
            cfg = M.make_run_config(EPS, nested=nested, eps_units="absolute", n_pilot=TTE_PILOT,
                                    costs=(c_p, c_a, cc), plain_arith="fp32", prec=prec, **kw)
            ctx.estimate(prob, cfg, SEED + 1)                  # warm (tables, caches)
            ts, ests, steps, Ls = [], [], [], []
            for rep in range(TTE_SEEDS):
                t0 = time.perf_counter()
                r = ctx.estimate(prob, cfg, SEED + 2 + rep)
                ts.append(time.perf_counter() - t0)
                ests.append(r["estimate"])
                steps.append(r["path_steps"])
                Ls.append(r["L"])
            e = np.asarray(ests)
            rmse = float(np.sqrt(np.mean((e - truth) ** 2)))
            ci = [rmse * math.sqrt(TTE_SEEDS / CHI2_HI), rmse * math.sqrt(TTE_SEEDS / CHI2_LO)]
            res[name] = {"seconds": float(np.median(ts)), "p10_s": float(np.percentile(ts, 10)),
                         "p90_s": float(np.percentile(ts, 90)), "mean_estimate": float(e.mean()),
                         "rmse": rmse, "rmse_ci95": ci, "rmse_within_eps": ci[0] <= EPS,
                         "rmse_vs_closed_form": float(np.sqrt(np.mean((e - bs) ** 2))),
                         "L_median": float(np.median(Ls)), "path_steps_median": float(np.median(steps))}
        for name in ("nested", "nested_exact_fp32", "nested_chosen"):
            res[name]["speedup_vs_plain_fp32"] = res["plain_fp32"]["seconds"] / res[name]["seconds"]
            res[name]["faster_at_equal_rmse"] = bool(res[name]["rmse_within_eps"] and
                                                     res["plain_fp32"]["rmse_within_eps"] and
                                                     res[name]["speedup_vs_plain_fp32"] > 1.0)
        out[setting] = res
    out["speedup"] = out["fixed"]["nested"]["speedup_vs_plain_fp32"]
    out["faster_at_equal_rmse"] = out["fixed"]["nested"]["faster_at_equal_rmse"]
    return out


# ------------------------------------------------------- batched pricing, serving
def draw_options(rng, n):
    """Options of the batched / served workloads: S0, K ~ U[80,120], r ~ U[0,0.08],
    sigma ~ U[0.1,0.5], T ~ U[0.25,2] (drawn in that order as arrays of n), payoffs
    50% European, 30% Asian, 20% digital assigned by a permutation."""
    import numpy as np
    S0 = rng.uniform(80, 120, n)
    K = rng.uniform(80, 120, n)
    r = rng.uniform(0.0, 0.08, n)
    sig = rng.uniform(0.1, 0.5, n)
    T = rng.uniform(0.25, 2.0, n)
    n_e, n_a = n // 2, int(round(0.3 * n))
    kinds = np.array(["euro"] * n_e + ["asian"] * n_a + ["digital"] * (n - n_e - n_a))
    kinds = kinds[rng.permutation(n)]
    return [dict(S0=float(S0[i]), K=float(K[i]), r=float(r[i]), sigma=float(sig[i]), T=float(T[i]),
                 kind=str(kinds[i])) for i in range(n)]


def closed_form(o):
    """Black-Scholes price of a European call, or of a digital call paying K; None
    for the Asian option."""
    from math import erf, exp, log, sqrt
    N = lambda x: 0.5 * (1.0 + erf(x / sqrt(2.0)))
    d1 = (log(o["S0"] / o["K"]) + (o["r"] + 0.5 * o["sigma"] ** 2) * o["T"]) / (o["sigma"] * sqrt(o["T"]))
    d2 = d1 - o["sigma"] * sqrt(o["T"])
    if o["kind"] == "euro":
        return o["S0"] * N(d1) - o["K"] * exp(-o["r"] * o["T"]) * N(d2)
    if o["kind"] == "digital":
        return o["K"] * exp(-o["r"] * o["T"]) * N(d2)
    return None


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def _run_cfg(M, nested, eps, costs):
    prec = M.make_precision("fp32", Q, packed=True)
    return M.make_run_config(eps, nested=nested, eps_units="normalised", theta=0.5, L_min=2, L_max=10,
                             n_pilot=10_000, costs=costs, plain_arith="fp32", prec=prec)


def serving(M, ctx, costs, rates, seconds, warm=1.0, drain=30.0, max_active=256, drivers=("engine",)):
    """Poisson arrivals (exponential gaps) of pricing requests at each rate: options
    as draw_options, eps = 10^U[-4,-2] (normalised), Milstein; nested (FP32 table +
    FP64 correction) or plain FP32.  Latency = arrival to result: the submission's
    lag behind the scheduled arrival plus the server's submit-to-result time.
    Requests arriving in [warm, warm + seconds) are measured."""
    import ctypes as C
    import numpy as np
    from paper_2502_07123_amd import _lib as L
    lib = L.lib()
    out = []
    BUF = 512
    tk = (C.c_uint64 * BUF)()
    res = (L.Result * BUF)()
    cnt = C.c_uint32()
    for rate in rates:
        ss = np.random.SeedSequence(1234 + int(rate))
        g_rng, o_rng = (np.random.default_rng(x) for x in ss.spawn(2))
        t_end = warm + seconds
        gaps = g_rng.exponential(1.0 / rate, int(rate * t_end * 1.2) + 16)
        arr = np.cumsum(gaps)
        arr = arr[arr < t_end]
        n = len(arr)
        opts = draw_options(o_rng, n)
        eps = 10.0 ** o_rng.uniform(-4, -2, n)
        for drv, mode in [(d, m) for d in drivers for m in ("nested", "plain_fp32")]:
            ctx.set_driver(drv == "engine")
            nested = mode == "nested"
            reqs = (L.Request * n)()
            for i, o in enumerate(opts):
                q = reqs[i]
                q.struct_size = C.sizeof(L.Request)
                q.option_id = i
                q.problem = M.make_problem("milstein", (o["kind"],), S0=o["S0"], K=o["K"], r=o["r"],
                                           sigma=o["sigma"], T=o["T"])
                q.eps = float(eps[i])
                q.seed = SEED
                q.nested = 1 if nested else 0
            ctx.server_start(_run_cfg(M, nested, 1e-3, costs), max_active=max_active)
            lag = np.zeros(n)
            lat = np.full(n, np.nan)
            done_at = np.full(n, np.nan)
            est = np.full(n, np.nan)
            steps = np.zeros(n)
            index = {}
            t = C.c_uint64()
            i = 0
            t0 = time.perf_counter()

            def collect():
                while True:
                    if lib.mlmc_poll_done(ctx.h, BUF, tk, res, C.byref(cnt)) != 0:
                        raise RuntimeError("mlmc_poll_done failed")
                    now = time.perf_counter() - t0
                    for k in range(cnt.value):
                        j = index.pop(tk[k])
                        r = res[k]
                        if r.status == 0:
                            lat[j] = lag[j] + r.seconds
                            done_at[j] = now
                            est[j] = r.estimate
                            steps[j] = r.path_steps
                    if cnt.value < BUF:
                        return

            while i < n:
                now = time.perf_counter() - t0
                while i < n and arr[i] <= now:
                    if lib.mlmc_submit(ctx.h, C.byref(reqs[i]), C.byref(t)) != 0:
                        raise RuntimeError("mlmc_submit failed: " + ctx.last_error())
                    lag[i] = now - arr[i]
                    index[t.value] = i
                    i += 1
                collect()
                if i < n:
                    wait = arr[i] - (time.perf_counter() - t0)
                    if wait > 2e-4:
                        time.sleep(min(wait - 1e-4, 1e-3))
            meas = (arr >= warm)
            t_stop = time.perf_counter() + drain
            while time.perf_counter() < t_stop and np.isnan(lat[meas]).any():
                collect()
                time.sleep(5e-4)
            sst = ctx.server_stats()
            wall = time.perf_counter() - t0
            ctx.server_stop()
            ok = meas & ~np.isnan(lat)
            span = (np.nanmax(done_at[ok]) - warm) if ok.any() else float("nan")
            cf_err = []
            for j in np.nonzero(ok)[0]:
                v = closed_form(opts[j])
                if v is not None:
                    cf_err.append((est[j] - v) / opts[j]["S0"] / eps[j])
            cf_err = np.asarray(cf_err)
            out.append({
                "rate_per_s": rate, "mode": mode, "driver": drv, "measured": int(meas.sum()),
                "completed": int(ok.sum()),
                "p50_ms": _pct(lat[ok] * 1e3, 50), "p99_ms": _pct(lat[ok] * 1e3, 99),
                "mean_ms": float(np.mean(lat[ok]) * 1e3) if ok.any() else None,
                "options_per_s": float(ok.sum() / span) if ok.any() else 0.0,
                "path_steps_per_s": float(steps[ok].sum() / span) if ok.any() else 0.0,
                "submit_lag_p99_ms": _pct(lag[meas] * 1e3, 99),
                "closed_form_checked": int(cf_err.size),
                "rms_err_over_eps": float(np.sqrt(np.mean(cf_err ** 2))) if cf_err.size else None,
                "wall_s": wall,
                "scheduler": {k: sst[k] for k in ("flights", "works", "plan_seconds", "land_seconds",
                                                  "idle_seconds", "engine", "slots", "bytes_per_request")},
            })
            print(json.dumps({"serving": out[-1]}), file=sys.stderr, flush=True)
    return out


def batch(M, ctx, costs, eps_list, n_opt=256, drivers=("engine",)):
    """The batched workload: n_opt options (draw_options with default_rng(1234)),
    each to RMSE eps (normalised); nested vs plain FP32.  Wall time of the
    mlmc_estimate_batch call (results converted to dicts after it), per sweep
    driver: 'engine' (run states on the device, one graph replay per sweep of all
    options) or 'host' (each sweep planned on the host, one launch sequence)."""
    import numpy as np
    rng = np.random.default_rng(1234)
    opts = draw_options(rng, n_opt)
    probs = [M.make_problem("milstein", (o["kind"],), S0=o["S0"], K=o["K"], r=o["r"], sigma=o["sigma"],
                            T=o["T"]) for o in opts]
    out = []
    for drv in drivers:
        ctx.set_driver(drv == "engine")
        # one untimed call per mode first: the process-wide caches (table values, the
        # kernels' first launches, the engine's graph) are built once, not per request
        first = {}
        for mode in ("nested", "plain_fp32"):
            t0 = time.perf_counter()
            ctx.estimate_batch(probs, _run_cfg(M, mode == "nested", max(eps_list), costs), SEED + 99)
            first[mode] = time.perf_counter() - t0
        for eps in eps_list:
            for mode in ("nested", "plain_fp32"):
                cfg = _run_cfg(M, mode == "nested", eps, costs)
                t0 = time.perf_counter()
                raw = ctx.estimate_batch(probs, cfg, SEED, raw=True)
                dt = time.perf_counter() - t0
                rs = M.results_as_dicts(raw)
                errs = [(r["estimate"] - closed_form(o)) / o["S0"] / eps for r, o in zip(rs, opts)
                        if closed_form(o) is not None]
                ns = [sum(lv["n"][e] for lv in r["levels"] for e in range(3)) for r in rs]
                out.append({"eps": eps, "mode": mode, "driver": drv, "seconds": dt, "options": n_opt,
                            "path_steps": int(sum(r["path_steps"] for r in rs)),
                            "path_steps_per_s": sum(r["path_steps"] for r in rs) / dt,
                            "sweeps_max": max(r["sweeps"] for r in rs), "L_max": max(r["L"] for r in rs),
                            "samples_min": int(min(ns)), "samples_max": int(max(ns)),
                            "closed_form_checked": len(errs),
                            "rms_err_over_eps": float(np.sqrt(np.mean(np.square(errs)))),
                            "first_call_seconds": first[mode]})
                print(json.dumps({"batch": out[-1]}), file=sys.stderr, flush=True)
    ctx.set_driver("auto")
    return out


def per_level(M, ctx, steps_per_work=1 << 27, reps=3):
    """Path-steps/s of one level's work by kernel class and level (HIP events around
    the path kernels of a one-work launch, about 1.3e8 fine path-steps per work)."""
    prob = M.make_problem("milstein", ("euro",), **GBM)
    fixed = M.make_precision("fixed", 8, False, {
        "X": (32, 22), "con1": (32, 34), "con2": (32, 33), "con3": (32, 36), "Z": (31, 28),
        "mul1": (32, 30), "sum1": (32, 30), "zsq": (32, 23), "zm1": (32, 23), "mul3": (32, 29),
        "sum2": (32, 29), "mul2": (32, 27)})
    modes = [("approx_fp32_q8_packed", M.make_precision("fp32", 8, True), M.EST_APPROX),
             ("approx_fp16_q8_packed", M.make_precision("fp16", 8, True), M.EST_APPROX),
             ("approx_fixed_q8", fixed, M.EST_APPROX),
             ("corr_fp32_q8", M.make_precision("fp32", 8), M.EST_CORR),
             ("plain_fp32", M.make_precision("fp32", 8), M.EST_PLAIN),
             ("plain_fp64", M.make_precision("fp64", 8), M.EST_PLAIN)]
    out = []
    for name, prec, est in modes:
        row = {"mode": name}
        for l in range(0, 11):
            n = max(steps_per_work >> l, 4096)
            ctx.level_sums(prob, l, n, 0, prec, est, SEED)            # warm
            ctx.set_timing(True)
            for r in range(reps):
                ctx.level_sums(prob, l, n, n * (r + 1), prec, est, SEED)
            st = ctx.kernel_stats()
            ctx.set_timing(False)
            ms = sum(x["ms"] for x in st) / reps
            row[str(l)] = (n << l) / (ms * 1e-3)
        out.append(row)
        print(json.dumps({"per_level": row}), file=sys.stderr, flush=True)
    return out


def fixed_sweep(M, ctx, n_paths=1_000_000, reps=3):
    """The fixed-point workload: Euler paths with X a signed 32-bit Q-format number
    of b_l = min(24, 14 + l) fractional bits (the other variables' formats those of
    the parity tests), the q = 8 table in Z's format, European, Asian and barrier (85)
    payoffs of the same paths in one launch, 1e6 paths at each level 0..10.  Per
    level: path kernel time (HIP events, mean of reps), path-steps/s and saturations;
    the whole sweep: the sum of the levels' kernel times and its wall time."""
    import torch
    base = {"X": (32, 22), "con1": (32, 34), "con2": (32, 33), "con3": (32, 36), "Z": (31, 28),
            "mul1": (32, 30), "sum1": (32, 30), "zsq": (32, 23), "zm1": (32, 23), "mul3": (32, 29),
            "sum2": (32, 29), "mul2": (32, 27)}
    prob = M.make_problem("euler", ("euro", "asian", "barrier"), **GBM)
    precs = [M.make_precision("fixed", 8, False, {**base, "X": (32, min(24, 14 + l))}) for l in range(11)]
    for l in range(11):
        ctx.level_sums(prob, l, n_paths, 0, precs[l], M.EST_APPROX, SEED)          # warm
    rows, kernel_ms = [], 0.0
    for l in range(11):
        ctx.set_timing(True)
        for r in range(reps):
            sums = ctx.level_sums(prob, l, n_paths, 0, precs[l], M.EST_APPROX, SEED)
        st = ctx.kernel_stats()
        ctx.set_timing(False)
        ms = sum(x["ms"] for x in st) / reps
        kernel_ms += ms
        rows.append({"level": l, "b": min(24, 14 + l), "kernel_ms": ms,
                     "path_steps_per_s": (n_paths << l) / (ms * 1e-3),
                     "saturations": int(sum(s["saturations"] for s in sums.values()))})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        for l in range(11):
            ctx.level_sums(prob, l, n_paths, 0, precs[l], M.EST_APPROX, SEED)
    wall = (time.perf_counter() - t0) / reps
    steps = sum(n_paths << l for l in range(11))
    out = {"workload": "fixed-point Euler, 1e6 paths/level, levels 0..10, euro+asian+barrier(85)",
           "levels": rows, "sweep_kernel_ms": kernel_ms, "sweep_wall_ms": wall * 1e3,
           "path_steps": steps, "path_steps_per_s_kernel": steps / (kernel_ms * 1e-3),
           "path_steps_per_s_wall": steps / wall}
    print(json.dumps({"fixed_sweep": out}), file=sys.stderr, flush=True)
    return out


def plain_fp64_levels(M, ctx, n_paths=100_000, levels=5, reps=5):
    """Plain MLMC of the European call, Euler, FP64 with the exact FP64 inverse normal
    on Philox uniforms (seed 1234), levels 0..4, 1e5 paths per level: the per-level
    sums of P_f - P_c (normalised) and the time of one launch sequence of the five
    works (HIP-event kernel time and wall time, median of reps)."""
    import numpy as np
    import torch
    prob = M.make_problem("euler", ("euro",), **GBM)
    prec = M.make_precision("fp64", Q)
    items = [(prob, l, n_paths, 0, prec, M.EST_PLAIN, SEED, 0) for l in range(levels)]
    ctx.level_sums_batch(items)                                   # warm
    walls, kms = [], []
    for r in range(reps):
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.level_sums_batch(items)
        walls.append(time.perf_counter() - t0)
        kms.append(sum(x["ms"] for x in ctx.kernel_stats()))
        ctx.set_timing(False)
    steps = sum(n_paths << l for l in range(levels))
    lv = [{"level": l, "n": res[l]["euro"]["n"], "sum_dP": res[l]["euro"]["sum1"],
           "sum_dP2": res[l]["euro"]["sum2"]} for l in range(levels)]
    scale = math.exp(-GBM["r"] * GBM["T"]) * GBM["S0"]
    est = scale * sum(x["sum_dP"] / x["n"] for x in lv)
    out = {"workload": "plain MLMC, European call, Euler, FP64 exact normals, levels 0..4, 1e5 paths/level",
           "levels": lv, "estimate": est, "closed_form": closed_form(dict(GBM, kind="euro")),
           "wall_ms": float(np.median(walls)) * 1e3, "kernel_ms": float(np.median(kms)),
           "path_steps": steps, "path_steps_per_s_wall": steps / float(np.median(walls))}
    print(json.dumps({"plain_fp64_levels": out}), file=sys.stderr, flush=True)
    return out


def tte_methods(M, ctx, costs, q=8):
    """Section 3's approximate normals compared on the GPU: Methods 1 (interval
    means), 2 (sum of two small-table variables, coupled through the permutation)
    and 3 (dyadic piecewise linear), each expanded to the 2^q-entry table the kernels
    read (so a path-step costs the same); what differs is the correction variance
    V^D.  Time to RMSE eps at fixed L = 8 (as tte_table_sizes), and V^D per level
    from the runs' level sums."""
    import numpy as np
    c_p, c_a, c_c = costs
    prob = M.make_problem("milstein", ("euro",), **GBM)
    scale = math.exp(-GBM["r"] * GBM["T"]) * GBM["S0"]
    ref, ref_se = level_reference(M, ctx, prob, scale)
    out = {"q": q, "reference_level_L": ref, "seeds": TTE_SEEDS}
    for method in (1, 2, 3):
        prec = M.make_precision("fp32", q, packed=True, method=method)
        cfg = M.make_run_config(EPS, nested=True, eps_units="absolute", n_pilot=TTE_PILOT, theta=1.0,
                                L_min=8, L_max=8, costs=(c_p, c_a, c_c), plain_arith="fp32", prec=prec)
        ctx.estimate(prob, cfg, SEED + 1)
        ts, ests, vd = [], [], []
        for rep in range(TTE_SEEDS):
            t0 = time.perf_counter()
            r = ctx.estimate(prob, cfg, SEED + 2 + rep)
            ts.append(time.perf_counter() - t0)
            ests.append(r["estimate"])
            vd.append([lv["var"][M.EST_CORR] for lv in r["levels"][:9]])
        e = np.asarray(ests)
        rmse = float(np.sqrt(np.mean((e - ref) ** 2)))
        out[f"method{method}"] = {"seconds": float(np.median(ts)), "rmse": rmse,
                                  "V_corr_per_level": [float(x) for x in np.median(np.asarray(vd), axis=0)]}
        print(json.dumps({"tte_method": {method: out[f"method{method}"]}}), file=sys.stderr, flush=True)
    return out


def tte_table_sizes(M, ctx, costs, qs=(4, 6, 8)):
    """Time to RMSE eps = 1e-3 (price units) at fixed L = 8, theta = 1 (the default
    bench's time-to-eps setting), nested with a q-bit table (packed FP32 indices) vs
    plain FP32, over TTE_SEEDS seeds; RMSE about the level-8 reference."""
    import numpy as np
    c_p, c_a, c_c = costs
    prob = M.make_problem("milstein", ("euro",), **GBM)
    scale = math.exp(-GBM["r"] * GBM["T"]) * GBM["S0"]
    ref, ref_se = level_reference(M, ctx, prob, scale)
    out = {"reference_level_L": ref, "reference_se": ref_se, "seeds": TTE_SEEDS}
    modes = [(f"nested_q{q}", True, q) for q in qs] + [("plain_fp32", False, 8)]
    for name, nested, q in modes:
        prec = M.make_precision("fp32", q, packed=True)
        # the approximate estimator's cost per path-step at this q (the packed fields change it)
        ca = calibrate(M, ctx, prob, prec, M.make_precision("fp32", q))[0] if nested else c_a
        cfg = M.make_run_config(EPS, nested=nested, eps_units="absolute", n_pilot=TTE_PILOT, theta=1.0,
                                L_min=8, L_max=8, costs=(c_p, ca, c_c), plain_arith="fp32", prec=prec)
        ctx.estimate(prob, cfg, SEED + 1)
        ts, ests = [], []
        for rep in range(TTE_SEEDS):
            t0 = time.perf_counter()
            r = ctx.estimate(prob, cfg, SEED + 2 + rep)
            ts.append(time.perf_counter() - t0)
            ests.append(r["estimate"])
        e = np.asarray(ests)
        rmse = float(np.sqrt(np.mean((e - ref) ** 2)))
        ci = [rmse * math.sqrt(TTE_SEEDS / CHI2_HI), rmse * math.sqrt(TTE_SEEDS / CHI2_LO)]
        out[name] = {"q": q, "seconds": float(np.median(ts)), "rmse": rmse, "rmse_ci95": ci,
                     "rmse_within_eps": ci[0] <= EPS, "cost_approx_ns": ca}
        print(json.dumps({"tte_q": {name: out[name]}}), file=sys.stderr, flush=True)
    for q in qs:
        out[f"nested_q{q}"]["speedup_vs_plain_fp32"] = out["plain_fp32"]["seconds"] / out[f"nested_q{q}"]["seconds"]
    return out


def main_workloads(args):
    """--batch / --serving: one JSON line with the batched and/or served workloads."""
    import torch
    import paper_2502_07123_amd as M
    ctx = M.Context(0, workspace_bytes=1 << 30)
    prob = M.make_problem("milstein", ("euro",), **GBM)
    c_a, c_c, c_p = calibrate(M, ctx, prob, M.make_precision("fp32", Q, packed=True),
                              M.make_precision("fp32", Q, packed=False))
    costs = (c_p, c_a, c_c)
    line = {"cost_ns_per_step": {"plain_fp32": c_p, "approx": c_a, "corr": c_c}}
    if args.batch:
        line["batch"] = batch(M, ctx, costs, [float(x) for x in args.batch_eps.split(",")],
                              drivers=tuple(args.drivers.split(",")))
    if args.serving:
        line["serving"] = serving(M, ctx, costs, [float(x) for x in args.serve_rates.split(",")],
                                  args.serve_seconds, drivers=tuple(args.drivers.split(",")))
        ctx.set_driver("auto")
    if args.per_level:
        line["per_level_path_steps_per_s"] = per_level(M, ctx)
    if args.fixed_sweep:
        line["fixed_sweep"] = fixed_sweep(M, ctx)
    if args.configs:
        line["plain_fp64_levels"] = plain_fp64_levels(M, ctx)
        line["tte_table_sizes"] = tte_table_sizes(M, ctx, (c_p, c_a, c_c))
        line["tte_methods"] = tte_methods(M, ctx, (c_p, c_a, c_c))
    torch.cuda.synchronize()
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
