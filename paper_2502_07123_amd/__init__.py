"""Nested multilevel Monte Carlo on MI355X (gfx950).

The hot path of Haas & Giles' nested MLMC method -- coupled fine/coarse GBM
paths from counter-based uniforms, exact or Method-1 table normals, FP64 / FP32 /
per-variable fixed-point arithmetic, level sums of payoff differences for the
plain and the two nested estimators -- runs in HIP kernels behind the C ABI of
include/mlmc.h.  This module is the Python binding: argument marshalling, plus
PyTorch for the device workspace and the stream.
"""
import ctypes as C

import numpy as np

from ._lib import (ARITH, EST_APPROX, EST_CORR, EST_PLAIN, LEVELWORK_DTYPE, PAYOFFS, RECORD_DTYPE, SUMS_DTYPE,
                   VARS, ErrorModel, KernelStat, LevelWork, MlmcError, Precision, Problem, Request, Result,
                   RunConfig, ServerConfig, ServerStats, Sums, Tuning, WidthPlan, check, error_model_struct, lib,
                   make_precision, make_problem, make_run_config)

__all__ = ["Context", "level_sums_static", "make_problem", "make_precision", "make_run_config", "build_table",
           "stream_words", "check_paths_host", "allocate", "validate", "optimise_widths", "MlmcError",
           "EST_PLAIN", "EST_APPROX", "EST_CORR", "PAYOFFS", "VARS", "RECORD_DTYPE", "SUMS_DTYPE",
    "gpu_rates", "side_costs", "choose_precision", "inverse_normal_host", "level_sums_static",
           "SumsBatch"]


def _payoff_names(problem):
    return [p for i, p in enumerate(PAYOFFS) if (problem.payoff_mask >> i) & 1]


class Context:
    """A library context on one GPU: workspace (the HBM budget) allocated by
    PyTorch, launches on the given torch stream (default: the current stream)."""

    def __init__(self, device=0, workspace_bytes=256 << 20, stream=None):
        import torch
        self.device = device
        self._ws = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        check(lib().mlmc_context_create(device, C.c_void_p(self._ws.data_ptr()), int(workspace_bytes),
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().mlmc_context_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return lib().mlmc_last_error(self.h).decode()

    def level_sums(self, problem, level, n_paths, path_offset, prec, estimator, seed, option=0,
                   debug=False):
        """Sums per payoff (dicts, in payoff order) and, with debug, per-path records
        (numpy structured array of RECORD_DTYPE)."""
        import torch
        names = _payoff_names(problem)
        out = (Sums * len(names))()
        rec = None
        if debug:
            rec = torch.zeros(int(n_paths) * RECORD_DTYPE.itemsize, dtype=torch.uint8,
                              device=f"cuda:{self.device}")
        st = lib().mlmc_level_sums(self.h, C.byref(problem), level, int(n_paths), int(path_offset),
                                   C.byref(prec), estimator, int(seed), option, out,
                                   C.c_void_p(rec.data_ptr()) if debug else None)
        check(st, self.h)
        sums = {n: out[i].as_dict() for i, n in enumerate(names)}
        if not debug:
            return sums
        return sums, np.frombuffer(rec.cpu().numpy().tobytes(), dtype=RECORD_DTYPE)

    def level_sums_batch(self, items):
        """items: list of (problem, level, n_paths, path_offset, prec, estimator, seed, option).
        One launch sequence; returns one {payoff: sums} dict per item."""
        n = len(items)
        keep = []
        works = (LevelWork * n)()
        outs = []
        for i, (prob, level, npaths, off, prec, est, seed, opt) in enumerate(items):
            names = _payoff_names(prob)
            out = (Sums * len(names))()
            outs.append((names, out))
            keep.append((prob, prec))
            works[i] = LevelWork(C.sizeof(LevelWork), level, est, opt, int(npaths), int(off),
                                 int(seed), C.pointer(prob), C.pointer(prec),
                                 C.cast(out, C.POINTER(Sums)))
        check(lib().mlmc_level_sums_batch(self.h, n, works), self.h)
        return [{nm: out[j].as_dict() for j, nm in enumerate(names)} for names, out in outs]

    def sums_batch(self, items):
        """A reusable batch of level-sum works (see SumsBatch)."""
        return SumsBatch(self, items)

    def get_tuning(self):
        t = Tuning()
        check(lib().mlmc_get_tuning(self.h, C.byref(t)), self.h)
        return t.as_dict()

    def set_tuning(self, **kw):
        """Change launch geometry fields (see mlmc_tuning in include/mlmc.h)."""
        t = Tuning()
        check(lib().mlmc_get_tuning(self.h, C.byref(t)), self.h)
        for k, v in kw.items():
            setattr(t, k, v)
        check(lib().mlmc_set_tuning(self.h, C.byref(t)), self.h)

    def autotune(self, batch, reps=5):
        """Launch geometry chosen for a SumsBatch's works (mlmc_autotune); returns it."""
        t = Tuning()
        t.struct_size = C.sizeof(Tuning)
        check(lib().mlmc_autotune(self.h, batch.n, batch._works, reps, C.byref(t)), self.h)
        return t.as_dict()

    def set_driver(self, engine=True):
        """Estimates' sweeps on the device sweep engine (True), planned on the host
        (False), or "auto" (the default: the engine for batches of at least
        MLMC_ENGINE_MIN_RUNS options)."""
        check(lib().mlmc_set_driver(self.h, 2 if engine == "auto" else (1 if engine else 0)), self.h)

    def set_timing(self, on=True):
        check(lib().mlmc_set_timing(self.h, 1 if on else 0), self.h)

    def kernel_stats(self):
        cnt = C.c_uint32()
        check(lib().mlmc_kernel_stats(self.h, None, 0, C.byref(cnt)), self.h)
        arr = (KernelStat * max(cnt.value, 1))()
        check(lib().mlmc_kernel_stats(self.h, arr, cnt.value, C.byref(cnt)), self.h)
        return [arr[i].as_dict() for i in range(cnt.value)]

    def estimate(self, problem, cfg, seed, option=0):
        r = Result()
        r.struct_size = C.sizeof(Result)
        check(lib().mlmc_estimate(self.h, C.byref(problem), C.byref(cfg), int(seed), option,
                                  C.byref(r)), self.h)
        return r.as_dict()

    def estimate_batch(self, problems, cfg, seed, raw=False):
        """One result dict per problem; raw: the mlmc_result array as returned (for
        timing the call alone; results_as_dicts converts it)."""
        n = len(problems)
        arr = (Problem * n)(*problems)
        res = (Result * n)()
        check(lib().mlmc_estimate_batch(self.h, n, arr, C.byref(cfg), int(seed), res), self.h)
        return res if raw else results_as_dicts(res)

    # ---- serving
    def server_start(self, run_cfg, max_active=256):
        sc = ServerConfig(C.sizeof(ServerConfig), max_active, run_cfg)
        check(lib().mlmc_server_start(self.h, C.byref(sc)), self.h)

    def submit(self, problem, eps, seed, option=0, nested=True):
        req = Request(C.sizeof(Request), option, problem, eps, int(seed), 1 if nested else 0, 0)
        t = C.c_uint64()
        check(lib().mlmc_submit(self.h, C.byref(req), C.byref(t)), self.h)
        return t.value

    def poll(self, ticket):
        """None while pending, else the result dict."""
        r = Result()
        st = lib().mlmc_poll(self.h, int(ticket), C.byref(r))
        if st == 1:
            return None
        check(st, self.h)
        return r.as_dict()

    def poll_done(self, max_n=1024):
        """[(ticket, result dict)] of up to max_n finished requests, oldest first."""
        tk = (C.c_uint64 * max_n)()
        res = (Result * max_n)()
        n = C.c_uint32()
        check(lib().mlmc_poll_done(self.h, max_n, tk, res, C.byref(n)), self.h)
        return [(tk[i], res[i].as_dict()) for i in range(n.value)]

    # ---- rounding-error model and bit widths (Sections 4-6)
    def inverse_normal(self, J, arith="fp64"):
        """Phi^-1((J + 1/2) 2^-32) by the kernels' inverse normal: J a uint32 numpy
        array (or device tensor of int32 bits); returns a numpy array."""
        import torch
        Jt = torch.as_tensor(np.asarray(J, dtype=np.uint32).view(np.int32)).to(f"cuda:{self.device}")
        dt = torch.float64 if arith == "fp64" else torch.float32
        out = torch.empty(Jt.numel(), dtype=dt, device=f"cuda:{self.device}")
        check(lib().mlmc_inverse_normal(self.h, C.c_void_p(Jt.data_ptr()), Jt.numel(), ARITH[arith],
                                        C.c_void_p(out.data_ptr())), self.h)
        return out.cpu().numpy()

    def error_model(self, problem, level, n_paths, q, seed, option=0):
        m = ErrorModel()
        m.struct_size = C.sizeof(ErrorModel)
        check(lib().mlmc_error_model_compute(self.h, C.byref(problem), level, int(n_paths), q, int(seed),
                                             option, C.byref(m)), self.h)
        return m.as_dict()

    def server_stats(self):
        st = ServerStats()
        st.struct_size = C.sizeof(ServerStats)
        check(lib().mlmc_server_stats_get(self.h, C.byref(st)), self.h)
        return {k: getattr(st, k) for k, _ in ServerStats._fields_ if k not in ("struct_size", "pad")}

    def server_stop(self):
        check(lib().mlmc_server_stop(self.h), self.h)


class SumsBatch:
    """A fixed list of works, items as for Context.level_sums_batch, marshalled once.
    `offsets` (numpy view, one per work) and `seeds` may be changed between runs;
    after run() or wait(), `sums` is a numpy array of SUMS_DTYPE per work and payoff
    (shape (n_works, max payoffs per work), payoffs in increasing order).

    enqueue() launches the batch and returns a ticket without waiting; wait(ticket)
    waits for it.  The sums buffer is written when the batch lands, so a second
    enqueue of the same SumsBatch must follow the wait of the first (use two batches
    to keep two in flight)."""

    def __init__(self, ctx, items):
        self.ctx = ctx
        n = len(items)
        self.n = n
        self._keep = []
        self.payoffs = []
        npay = max(bin(it[0].payoff_mask).count("1") for it in items)
        self._out = (Sums * (n * npay))()
        self.sums = np.frombuffer(self._out, dtype=SUMS_DTYPE).reshape(n, npay)
        self._works = (LevelWork * n)()
        w = np.frombuffer(self._works, dtype=LEVELWORK_DTYPE)
        base = C.addressof(self._out)
        for i, (prob, level, npaths, off, prec, est, seed, opt) in enumerate(items):
            self._keep.append((prob, prec))
            self.payoffs.append(_payoff_names(prob))
            w[i] = (C.sizeof(LevelWork), level, est, opt, int(npaths), int(off), int(seed),
                    C.addressof(prob), C.addressof(prec), base + i * npay * C.sizeof(Sums))
        self.offsets = w["path_offset"]
        self.seeds = w["seed"]
        self.n_paths = w["n_paths"]
        self._pending = None

    def run(self):
        check(lib().mlmc_level_sums_batch(self.ctx.h, self.n, self._works), self.ctx.h)
        return self.sums

    def enqueue(self):
        if self._pending is not None:
            raise RuntimeError("this batch is still in flight: wait for it first")
        t = C.c_uint64()
        check(lib().mlmc_level_sums_enqueue(self.ctx.h, self.n, self._works, C.byref(t)), self.ctx.h)
        self._pending = t.value
        return t.value

    def wait(self, ticket=None):
        t = self._pending if ticket is None else ticket
        self._pending = None
        check(lib().mlmc_level_sums_wait(self.ctx.h, int(t)), self.ctx.h)
        return self.sums

    def as_dicts(self):
        """One {payoff: sums dict} per work (as Context.level_sums_batch)."""
        out = []
        for i, names in enumerate(self.payoffs):
            d = {}
            for j, nm in enumerate(names):
                r = self.sums[i, j]
                x = {f: r[f].item() for f in SUMS_DTYPE.names}
                x["isum2"] = (int(r["isum2_hi"]) << 64) | int(r["isum2_lo"])
                d[nm] = x
            out.append(d)
        return out


# ---------------------------------------------------------- host-side helpers
def results_as_dicts(res):
    """The dicts of an mlmc_result array."""
    return [res[i].as_dict() for i in range(len(res))]


def level_sums_static(problem, level, n_paths, path_offset, prec, estimator, seed, option=0,
                      out=None, stream=None):
    """mlmc_level_sums_static: the sums of one level into `out`, a device tensor of at
    least popcount(mask) * SUMS_DTYPE.itemsize bytes (allocated here when None), on
    `stream` (default: the current torch stream), without waiting.  Returns `out`;
    sums_from_device(out, problem) reads it after the stream has reached it."""
    import torch
    names = _payoff_names(problem)
    if out is None:
        out = torch.empty(len(names) * SUMS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    if out.numel() * out.element_size() < len(names) * SUMS_DTYPE.itemsize or not out.is_cuda:
        raise ValueError("out: device tensor too small")
    st = stream if stream is not None else torch.cuda.current_stream(out.device)
    status = lib().mlmc_level_sums_static(C.byref(problem), level, int(n_paths), int(path_offset),
                                          C.byref(prec), estimator, int(seed), option,
                                          C.c_void_p(st.cuda_stream), C.c_void_p(out.data_ptr()))
    if status != 0:
        raise MlmcError(status, lib().mlmc_last_error(None).decode())
    return out


def sums_from_device(out, problem):
    """{payoff: sums dict} from a device tensor written by level_sums_static."""
    names = _payoff_names(problem)
    raw = out.detach().cpu().numpy().tobytes()[:len(names) * SUMS_DTYPE.itemsize]
    arr = np.frombuffer(raw, dtype=SUMS_DTYPE)
    res = {}
    for i, nm in enumerate(names):
        d = {f: arr[i][f].item() for f in SUMS_DTYPE.names}
        d["isum2"] = (int(d["isum2_hi"]) << 64) | int(d["isum2_lo"])
        res[nm] = d
    return res


def gpu_rates(**over):
    """The measured issue rates (mlmc_gpu_rates_default), fields overridden by `over`."""
    from ._lib import GpuRates
    r = GpuRates()
    r.struct_size = C.sizeof(GpuRates)
    check(lib().mlmc_gpu_rates_default(C.byref(r)))
    for k, v in over.items():
        setattr(r, k, v)
    return r


def side_costs(arith, q, packed, scheme, level, rates=None):
    """(c_approx, c_corr) per fine path-step of a table side (mlmc_side_costs)."""
    a, c = C.c_double(), C.c_double()
    r = rates if rates is not None else gpu_rates()
    check(lib().mlmc_side_costs(ARITH[arith], q, 1 if packed else 0, 0 if scheme == "euler" else 1, level,
                                C.byref(r), C.byref(a), C.byref(c)))
    return a.value, c.value


def choose_precision(model, rates=None, fixed_fmt=None):
    """mlmc_choose_precision for one level's error model (a mapping as returned by
    Context.error_model); fixed_fmt: var -> (w, f) formats of the FIXED candidate.
    Returns (Precision, info dict)."""
    from ._lib import LevelChoice
    m = model if isinstance(model, ErrorModel) else error_model_struct(model)
    r = rates if rates is not None else gpu_rates()
    ff = make_precision("fixed", 8, False, fixed_fmt) if fixed_fmt else None
    out = make_precision("fp32", 8)
    info = LevelChoice()
    info.struct_size = C.sizeof(LevelChoice)
    check(lib().mlmc_choose_precision(C.byref(m), C.byref(r), C.byref(ff) if ff is not None else None,
                                      C.byref(out), C.byref(info)))
    return out, info.as_dict()


def inverse_normal_host(J, arith="fp64"):
    """mlmc_inverse_normal_host: the kernels' inverse normal compiled for the host."""
    J = np.ascontiguousarray(np.asarray(J, dtype=np.uint32))
    out = np.empty(J.size, dtype=np.float64 if arith == "fp64" else np.float32)
    check(lib().mlmc_inverse_normal_host(J.ctypes.data_as(C.c_void_p), J.size, ARITH[arith],
                                         out.ctypes.data_as(C.c_void_p)))
    return out


def optimise_widths(model, c_rng=1e4, rng_term=False):
    """Section 6 widths of one level from an error model (dict as Context.error_model
    returns); host only."""
    m = error_model_struct(model)
    out = WidthPlan()
    out.struct_size = C.sizeof(WidthPlan)
    check(lib().mlmc_optimise_widths(C.byref(m), float(c_rng), 1 if rng_term else 0, C.byref(out)))
    return out.as_dict()


def build_table(q, arith="fp32", frac_bits=0):
    dt = {"fp64": np.float64, "fp32": np.float32, "fp16": np.uint16, "fixed": np.int32}[arith]
    out = np.zeros(1 << q, dtype=dt)
    check(lib().mlmc_build_table(q, ARITH[arith], frac_bits, out.ctypes.data_as(C.c_void_p)))
    return out


def stream_words(seed, option, level, estimator, word_index, count):
    out = np.zeros(int(count), dtype=np.uint32)
    check(lib().mlmc_stream_words(int(seed), option, level, estimator, int(word_index), int(count),
                                  out.ctypes.data_as(C.POINTER(C.c_uint32))))
    return out


def check_paths_host(problem, level, n_paths, path_offset, prec, estimator, seed, option=0,
                     records=True):
    """The kernels' per-path code run on the host (a checker; n_paths <= 65536).
    Returns (sums per payoff, per-path records or None without records: the kernels'
    sums-only code, e.g. the level-0 loop of the exact-normal estimators)."""
    names = _payoff_names(problem)
    out = (Sums * len(names))()
    rec = np.zeros(int(n_paths), dtype=RECORD_DTYPE) if records else None
    check(lib().mlmc_check_paths_host(C.byref(problem), level, int(n_paths), int(path_offset),
                                      C.byref(prec), estimator, int(seed), option, out,
                                      rec.ctypes.data_as(C.c_void_p) if records else None))
    return {n: out[i].as_dict() for i, n in enumerate(names)}, rec


def allocate(V, Cost, eps2, theta=1.0):
    V = np.ascontiguousarray(V, dtype=np.float64)
    Cc = np.ascontiguousarray(Cost, dtype=np.float64)
    out = np.zeros(V.size, dtype=np.uint64)
    check(lib().mlmc_allocate(V.size, V.ctypes.data_as(C.POINTER(C.c_double)),
                              Cc.ctypes.data_as(C.POINTER(C.c_double)), eps2, theta,
                              out.ctypes.data_as(C.POINTER(C.c_uint64))))
    return out


def validate(problem, level, n_paths, path_offset, prec, estimator):
    """The library's status code for these arguments (0 = valid)."""
    return lib().mlmc_validate(C.byref(problem), level, int(n_paths), int(path_offset),
                               C.byref(prec), estimator)
