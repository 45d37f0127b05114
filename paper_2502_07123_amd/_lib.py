"""ctypes binding of libmlmc.so (the C ABI declared in include/mlmc.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory (the workspace, debug buffers) and the
stream.  Loading fails loudly when the built library is missing.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlmc.so")

ABI_VERSION = 1
MAX_LEVELS = 21
NPAYOFF = 5
NVARS = 12

EULER, MILSTEIN = 0, 1
PAYOFFS = ("forward", "euro", "asian", "barrier", "digital")
ARITH = {"fp64": 0, "fp32": 1, "fp16": 2, "fixed": 3}
EST_PLAIN, EST_APPROX, EST_CORR = 0, 1, 2
VARS = ("X", "con1", "con2", "con3", "Z", "mul1", "sum1", "zsq", "zm1", "mul3", "sum2", "mul2")

STATUS = {0: "MLMC_OK", 1: "MLMC_PENDING", -1: "MLMC_E_INVALID", -2: "MLMC_E_NOMEM",
          -3: "MLMC_E_DEVICE", -4: "MLMC_E_OVERFLOW", -5: "MLMC_E_BUSY", -6: "MLMC_E_TIMEOUT",
          -7: "MLMC_E_UNKNOWN_TICKET", -8: "MLMC_E_VERSION"}


class MlmcError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


class Problem(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("scheme", C.c_int32), ("payoff_mask", C.c_uint32),
                ("reserved", C.c_int32), ("S0", C.c_double), ("K", C.c_double), ("r", C.c_double),
                ("sigma", C.c_double), ("T", C.c_double), ("barrier", C.c_double)]


class Precision(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("arith", C.c_int32), ("table_bits", C.c_int32),
                ("packed", C.c_int32), ("word_bits", C.c_int32 * NVARS),
                ("frac_bits", C.c_int32 * NVARS), ("rng_method", C.c_int32), ("exact_side", C.c_int32)]


class Sums(C.Structure):
    _fields_ = [("n", C.c_uint64), ("sum1", C.c_double), ("sum2", C.c_double),
                ("isum1", C.c_int64), ("isum2_lo", C.c_uint64), ("isum2_hi", C.c_uint64),
                ("esum1", C.c_double), ("esum2", C.c_double), ("saturations", C.c_uint64),
                ("nonfinite", C.c_uint64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["isum2"] = (int(self.isum2_hi) << 64) | int(self.isum2_lo)
        return d


# numpy views of the same layouts (checked against the ctypes structs in the tests)
SUMS_DTYPE = np.dtype([("n", "<u8"), ("sum1", "<f8"), ("sum2", "<f8"), ("isum1", "<i8"),
                       ("isum2_lo", "<u8"), ("isum2_hi", "<u8"), ("esum1", "<f8"), ("esum2", "<f8"),
                       ("saturations", "<u8"), ("nonfinite", "<u8")])
LEVELWORK_DTYPE = np.dtype([("struct_size", "<u4"), ("level", "<i4"), ("estimator", "<i4"),
                            ("option_id", "<u4"), ("n_paths", "<u8"), ("path_offset", "<u8"),
                            ("seed", "<u8"), ("prob", "<u8"), ("prec", "<u8"), ("out", "<u8")])

RECORD_DTYPE = np.dtype([("Y", "<f8", (NPAYOFF,)), ("Yraw", "<i8", (NPAYOFF,)),
                         ("XN_exact", "<f8"), ("XcN_exact", "<f8"), ("XN_approx", "<f8"),
                         ("XcN_approx", "<f8"), ("XN_raw", "<i8"), ("XcN_raw", "<i8"),
                         ("first_word", "<u4"), ("first_index", "<u4"), ("saturations", "<u4"),
                         ("reserved", "<u4")])


class LevelWork(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("level", C.c_int32), ("estimator", C.c_int32),
                ("option_id", C.c_uint32), ("n_paths", C.c_uint64), ("path_offset", C.c_uint64),
                ("seed", C.c_uint64), ("prob", C.POINTER(Problem)), ("prec", C.POINTER(Precision)),
                ("out", C.POINTER(Sums))]


class KernelStat(C.Structure):
    _fields_ = [("estimator", C.c_int32), ("arith", C.c_int32), ("scheme", C.c_int32),
                ("fields", C.c_int32), ("payoffs", C.c_int32), ("track", C.c_int32),
                ("level0", C.c_int32), ("exact32", C.c_int32), ("launches", C.c_uint64),
                ("ms", C.c_double), ("path_steps", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("pad")}


class Tuning(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("block_table", C.c_uint32), ("block_exact", C.c_uint32),
                ("tile_steps", C.c_uint32), ("blocks_per_cu", C.c_uint32), ("min_tiles", C.c_uint32),
                ("zb_max_paths", C.c_uint64), ("zb_max_positions", C.c_uint64),
                ("overlap_min_steps", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "struct_size"}


class RunConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("nested", C.c_int32), ("eps_units", C.c_int32),
                ("L_min", C.c_int32), ("L_max", C.c_int32), ("plain_arith", C.c_int32),
                ("eps", C.c_double), ("theta", C.c_double), ("n_pilot", C.c_uint64),
                ("cost_plain", C.c_double), ("cost_approx", C.c_double), ("cost_corr", C.c_double),
                ("prec", Precision * MAX_LEVELS)]


class LevelStats(C.Structure):
    _fields_ = [("n", C.c_uint64 * 3), ("mean", C.c_double * 3), ("var", C.c_double * 3)]


class Result(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("status", C.c_int32), ("L", C.c_int32),
                ("sweeps", C.c_int32), ("estimate", C.c_double), ("variance", C.c_double),
                ("seconds", C.c_double), ("path_steps", C.c_uint64), ("saturations", C.c_uint64),
                ("exact_sides", C.c_int32), ("pad", C.c_int32), ("level", LevelStats * MAX_LEVELS)]

    def as_dict(self):
        lv = [{"n": list(self.level[l].n), "mean": list(self.level[l].mean),
               "var": list(self.level[l].var)} for l in range(self.L + 1)]
        return {"status": self.status, "L": self.L, "sweeps": self.sweeps,
                "estimate": self.estimate, "variance": self.variance, "seconds": self.seconds,
                "path_steps": self.path_steps, "saturations": self.saturations,
                "exact_sides": self.exact_sides, "levels": lv}


class ServerConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("max_active", C.c_uint32), ("run", RunConfig)]


class ErrorModel(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("level", C.c_int32), ("scheme", C.c_int32),
                ("table_bits", C.c_int32), ("n_paths", C.c_uint64), ("used", C.c_int32 * NVARS),
                ("e", C.c_int32 * NVARS), ("S", C.c_double * NVARS), ("R", C.c_double * NVARS),
                ("V_level", C.c_double), ("mse", C.c_double)]

    def as_dict(self):
        return {"level": self.level, "scheme": self.scheme, "table_bits": self.table_bits,
                "n_paths": self.n_paths, "used": list(self.used), "e": list(self.e), "S": list(self.S),
                "R": list(self.R), "V_level": self.V_level, "mse": self.mse}


class WidthPlan(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("best_uniform", C.c_int32), ("lambda_", C.c_double),
                ("objective", C.c_double), ("objective_uniform", C.c_double), ("v_indep", C.c_double),
                ("cost", C.c_double), ("d_real", C.c_double * NVARS), ("d_int", C.c_int32 * NVARS),
                ("word_bits", C.c_int32 * NVARS), ("frac_bits", C.c_int32 * NVARS)]

    def as_dict(self):
        return {"best_uniform": self.best_uniform, "lambda": self.lambda_, "objective": self.objective,
                "objective_uniform": self.objective_uniform, "v_indep": self.v_indep, "cost": self.cost,
                "d_real": list(self.d_real), "d_int": list(self.d_int), "word_bits": list(self.word_bits),
                "frac_bits": list(self.frac_bits)}


def error_model_struct(d):
    """An ErrorModel from a mapping with its fields (lists for the per-variable ones)."""
    m = ErrorModel()
    m.struct_size = C.sizeof(ErrorModel)
    for k in ("level", "scheme", "table_bits", "n_paths", "V_level", "mse"):
        setattr(m, k, d[k])
    for k in ("used", "e", "S", "R"):
        arr = getattr(m, k)
        for i in range(NVARS):
            arr[i] = d[k][i]
    return m


class GpuRates(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("pad", C.c_uint32), ("f32", C.c_double), ("i32", C.c_double),
                ("f64_fma", C.c_double), ("f64_add", C.c_double), ("u64_mad", C.c_double),
                ("lds_b64", C.c_double), ("lds_b32", C.c_double)]


class LevelChoice(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("level", C.c_int32), ("arith", C.c_int32),
                ("table_bits", C.c_int32), ("packed", C.c_int32), ("pad", C.c_int32),
                ("v_approx", C.c_double), ("v_corr", C.c_double), ("c_approx", C.c_double),
                ("c_corr", C.c_double), ("objective", C.c_double), ("objective_fp32_q8", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f not in ("struct_size", "pad")}


class ServerStats(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("pad", C.c_uint32), ("flights", C.c_uint64),
                ("works", C.c_uint64), ("requests_done", C.c_uint64), ("queued", C.c_uint64),
                ("active", C.c_uint64), ("plan_seconds", C.c_double), ("land_seconds", C.c_double),
                ("idle_seconds", C.c_double), ("engine", C.c_uint32), ("slots", C.c_uint32),
                ("bytes_per_request", C.c_uint64)]


class Request(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("option_id", C.c_uint32), ("problem", Problem),
                ("eps", C.c_double), ("seed", C.c_uint64), ("nested", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2502_07123_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, u32, u64, st = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_int32
    P = C.POINTER
    sig = {
        "mlmc_abi_version": (i32, []),
        "mlmc_status_string": (C.c_char_p, [i32]),
        "mlmc_last_error": (C.c_char_p, [vp]),
        "mlmc_context_create": (st, [i32, vp, u64, vp, P(vp)]),
        "mlmc_context_destroy": (None, [vp]),
        "mlmc_level_sums": (st, [vp, P(Problem), i32, u64, u64, P(Precision), i32, u64, u32,
                                 P(Sums), vp]),
        "mlmc_level_sums_static": (st, [P(Problem), i32, u64, u64, P(Precision), i32, u64, u32, vp, vp]),
        "mlmc_level_sums_batch": (st, [vp, u32, P(LevelWork)]),
        "mlmc_level_sums_enqueue": (st, [vp, u32, P(LevelWork), P(u64)]),
        "mlmc_level_sums_wait": (st, [vp, u64]),
        "mlmc_set_timing": (st, [vp, i32]),
        "mlmc_set_driver": (st, [vp, i32]),
        "mlmc_get_tuning": (st, [vp, P(Tuning)]),
        "mlmc_set_tuning": (st, [vp, P(Tuning)]),
        "mlmc_autotune": (st, [vp, u32, P(LevelWork), u32, P(Tuning)]),
        "mlmc_kernel_stats": (st, [vp, P(KernelStat), u32, P(u32)]),
        "mlmc_estimate": (st, [vp, P(Problem), P(RunConfig), u64, u32, P(Result)]),
        "mlmc_estimate_batch": (st, [vp, u32, P(Problem), P(RunConfig), u64, P(Result)]),
        "mlmc_server_start": (st, [vp, P(ServerConfig)]),
        "mlmc_submit": (st, [vp, P(Request), P(u64)]),
        "mlmc_poll": (st, [vp, u64, P(Result)]),
        "mlmc_poll_done": (st, [vp, u32, P(u64), P(Result), P(u32)]),
        "mlmc_server_stats_get": (st, [vp, P(ServerStats)]),
        "mlmc_error_model_compute": (st, [vp, P(Problem), i32, u64, i32, u64, u32, P(ErrorModel)]),
        "mlmc_optimise_widths": (st, [P(ErrorModel), C.c_double, i32, P(WidthPlan)]),
        "mlmc_server_stop": (st, [vp]),
        "mlmc_build_table": (st, [i32, i32, i32, vp]),
        "mlmc_build_rng_table": (st, [i32, i32, P(C.c_double), P(C.c_uint16), P(i32)]),
        "mlmc_stream_words": (st, [u64, u32, i32, i32, u64, u64, P(u32)]),
        "mlmc_validate": (st, [P(Problem), i32, u64, u64, P(Precision), i32]),
        "mlmc_check_paths_host": (st, [P(Problem), i32, u64, u64, P(Precision), i32, u64, u32,
                                       P(Sums), vp]),
        "mlmc_allocate": (st, [u32, P(C.c_double), P(C.c_double), C.c_double, C.c_double, P(u64)]),
        "mlmc_inverse_normal": (st, [vp, vp, u64, i32, vp]),
        "mlmc_gpu_rates_default": (st, [P(GpuRates)]),
        "mlmc_side_costs": (st, [i32, i32, i32, i32, i32, P(GpuRates), P(C.c_double), P(C.c_double)]),
        "mlmc_choose_precision": (st, [P(ErrorModel), P(GpuRates), P(Precision), P(Precision), P(LevelChoice)]),
        "mlmc_inverse_normal_host": (st, [vp, u64, i32, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    if L.mlmc_abi_version() != ABI_VERSION:
        raise ImportError("libmlmc.so ABI version mismatch")
    _lib = L
    return L


EXPORTED = ("mlmc_abi_version", "mlmc_status_string", "mlmc_last_error", "mlmc_context_create",
            "mlmc_context_destroy", "mlmc_level_sums", "mlmc_level_sums_static", "mlmc_level_sums_batch",
            "mlmc_level_sums_enqueue", "mlmc_level_sums_wait", "mlmc_set_timing",
            "mlmc_get_tuning", "mlmc_set_tuning", "mlmc_autotune", "mlmc_set_driver",
            "mlmc_kernel_stats", "mlmc_estimate", "mlmc_estimate_batch",
            "mlmc_server_start", "mlmc_submit", "mlmc_poll", "mlmc_poll_done", "mlmc_server_stats_get",
            "mlmc_server_stop", "mlmc_error_model_compute", "mlmc_optimise_widths",
            "mlmc_build_table", "mlmc_build_rng_table", "mlmc_stream_words", "mlmc_validate", "mlmc_check_paths_host",
            "mlmc_allocate", "mlmc_inverse_normal", "mlmc_inverse_normal_host", "mlmc_gpu_rates_default",
            "mlmc_side_costs", "mlmc_choose_precision")


# ------------------------------------------------------------------ builders
def make_problem(scheme="euler", payoffs=("euro",), S0=100.0, K=100.0, r=0.05, sigma=0.2, T=1.0,
                 barrier=0.0):
    mask = 0
    for p in payoffs:
        mask |= 1 << PAYOFFS.index(p)
    return Problem(C.sizeof(Problem), EULER if scheme == "euler" else MILSTEIN, mask, 0,
                   S0, K, r, sigma, T, barrier)


def make_precision(arith="fp32", q=8, packed=False, fmt=None, method=1, exact="fp64"):
    """fmt: mapping var -> (word_bits, frac_bits) for 'fixed'; method: approximate
    normals of Section 3 (1, 2 or 3); exact: the correction's exact side (fp64/fp32)."""
    p = Precision()
    p.struct_size = C.sizeof(Precision)
    p.arith = ARITH[arith]
    p.table_bits = q
    p.packed = 1 if packed else 0
    p.rng_method = method
    p.exact_side = 0 if exact == "fp64" else 1
    if fmt:
        for v, (w, f) in dict(fmt).items():
            i = VARS.index(v)
            p.word_bits[i] = w
            p.frac_bits[i] = f
    return p


def make_run_config(eps, nested=True, eps_units="normalised", theta=0.5, L_min=2, L_max=10,
                    n_pilot=10_000, costs=(1.0, 0.1, 1.1), plain_arith="fp32", prec=None):
    """prec: one Precision for all levels, or a list per level (nested runs)."""
    c = RunConfig()
    c.struct_size = C.sizeof(RunConfig)
    c.nested = 1 if nested else 0
    c.eps_units = 0 if eps_units == "normalised" else 1
    c.L_min, c.L_max = L_min, L_max
    c.plain_arith = ARITH[plain_arith]
    c.eps, c.theta, c.n_pilot = eps, theta, n_pilot
    c.cost_plain, c.cost_approx, c.cost_corr = costs
    if prec is None:
        prec = make_precision("fp32", 8)
    for l in range(MAX_LEVELS):
        c.prec[l] = prec[min(l, len(prec) - 1)] if isinstance(prec, (list, tuple)) else prec
    return c


def check(status, ctx=None):
    if status not in (0, 1):
        msg = lib().mlmc_last_error(ctx).decode() if ctx else ""
        raise MlmcError(status, msg)
    return status
