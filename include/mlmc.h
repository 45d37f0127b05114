/*
 * mlmc.h -- C ABI of the MI355X nested multilevel Monte Carlo library.
 *
 * The library computes the data-parallel hot path of the nested MLMC method of
 * Haas & Giles, "A nested MLMC framework for efficient simulations on FPGAs"
 * (2025): coupled fine/coarse Geometric Brownian Motion paths (Section 2.1,
 * Algorithm 1; Milstein as named in Section 7) driven by counter-based uniforms,
 * mapped to normals either exactly or by the Method-1 piecewise-constant table
 * (Section 3.1), in FP64, FP32 or per-variable fixed point (Section 4.1), and
 * reduced into per-level sums of the payoff differences (Section 2.1) for the
 * plain and the two nested estimators (Section 2.2).  On top sit the optimal
 * sample allocation (Sections 2.1-2.2), an adaptive driver, batched pricing of
 * many options in one launch per sweep, and a continuous-batching server.
 *
 * Units.  Paths are simulated in S0-normalised units X = S / S0; every sum below
 * is of normalised, undiscounted payoff differences.  A price is
 * e^{-rT} * S0 * (sum of level means).
 *
 * Conventions.  All structs are plain data, caller-owned, and begin with
 * struct_size (set it to sizeof(the struct)); the library copies what it keeps
 * before returning.  Pointers documented as "device" are HIP device addresses on
 * the context's device; all others are host addresses.  No call throws; every
 * call returns an mlmc_status and, on a context, leaves a message readable with
 * mlmc_last_error.  MLMC_E_DEVICE poisons the context: every later call on it
 * returns MLMC_E_DEVICE.
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLMC_ABI_VERSION 1
#define MLMC_MAX_LEVELS 21      /* levels 0..20: h = 2^-l T (Section 2.1) */

typedef enum mlmc_status {
    MLMC_OK = 0,
    MLMC_PENDING = 1,           /* mlmc_poll: request still running */
    MLMC_E_INVALID = -1,        /* an argument failed validation */
    MLMC_E_NOMEM = -2,          /* workspace (the HBM budget) too small */
    MLMC_E_DEVICE = -3,         /* a HIP call failed; the context is poisoned */
    MLMC_E_OVERFLOW = -4,       /* fixed-point saturation with strict overflow */
    MLMC_E_BUSY = -5,           /* server not running / already running */
    MLMC_E_TIMEOUT = -6,        /* deadline passed */
    MLMC_E_UNKNOWN_TICKET = -7, /* mlmc_poll: no such ticket */
    MLMC_E_VERSION = -8         /* struct_size does not match this library */
} mlmc_status;

/* Time-stepping scheme: Euler-Maruyama (Section 2.1, Algorithm 1) or Milstein. */
enum { MLMC_EULER = 0, MLMC_MILSTEIN = 1 };

/* Payoffs (bit positions of mlmc_problem.payoff_mask).  The paper prices the
 * European call (Section 4.4); the others are evaluated on the same grid:
 *   FORWARD  X_N (a test functional)
 *   EURO     max(X_N - k, 0)
 *   ASIAN    max(A - k, 0), A = (1/N) sum_{n<N} (X_n + X_{n+1}) / 2
 *   BARRIER  max(X_N - k, 0) if min_{0<=n<=N} X_n > b, else 0 (down-and-out)
 *   DIGITAL  k if X_N > k else 0 (cash-or-nothing paying K)
 * with k = K / S0, b = barrier / S0, on each path's own grid. */
enum { MLMC_PAY_FORWARD = 0, MLMC_PAY_EURO = 1, MLMC_PAY_ASIAN = 2,
       MLMC_PAY_BARRIER = 3, MLMC_PAY_DIGITAL = 4, MLMC_NPAYOFF = 5 };

/* Arithmetic of a path generator. */
enum { MLMC_ARITH_FP64 = 0, MLMC_ARITH_FP32 = 1, MLMC_ARITH_FP16 = 2, MLMC_ARITH_FIXED = 3 };

/* Estimators (Section 2.2): PLAIN samples dP_l with exact normals; APPROX
 * samples the low-precision dP~_l with table normals; CORR samples
 * dP_l - dP~_l with both sides driven by the same uniform integers. */
enum { MLMC_EST_PLAIN = 0, MLMC_EST_APPROX = 1, MLMC_EST_CORR = 2 };

/* Fixed-point variables of the low-precision step (Algorithm 1; the Milstein
 * step adds zsq = Z*Z, zm1 = zsq - 1, mul3 = con3*zm1, sum2 = sum1 + mul3 with
 * con3 = sigma^2 h / 2, and mul2 = X * sum2).  Index into word_bits/frac_bits. */
enum { MLMC_V_X = 0, MLMC_V_CON1, MLMC_V_CON2, MLMC_V_CON3, MLMC_V_Z, MLMC_V_MUL1,
       MLMC_V_SUM1, MLMC_V_ZSQ, MLMC_V_ZM1, MLMC_V_MUL3, MLMC_V_SUM2, MLMC_V_MUL2,
       MLMC_NVARS };

/* The option: GBM dS = r S dt + sigma S dW (Section 2.1, Algorithm 1).
 * Validation: S0, K, sigma, T > 0; r >= 0; barrier < S0 when the barrier payoff
 * is requested; payoff_mask non-zero with bits < MLMC_NPAYOFF. */
typedef struct mlmc_problem {
    uint32_t struct_size;
    int32_t scheme;             /* MLMC_EULER | MLMC_MILSTEIN */
    uint32_t payoff_mask;       /* 1 << MLMC_PAY_* ; several payoffs share paths */
    int32_t reserved;
    double S0, K, r, sigma, T;
    double barrier;             /* down-and-out level B (price units) */
} mlmc_problem;

/* Arithmetic of the low-precision (APPROX, and approx side of CORR) generator,
 * or of the PLAIN generator.
 *   arith        PLAIN: FP64 or FP32 (exact normals in that precision).
 *                APPROX/CORR: FP32, FP16 or FIXED with Method-1 table normals;
 *                the exact side of CORR is set by exact_side.  FP32
 *                and FP16 evaluate Algorithm 1 operation by operation, each result
 *                rounded to the type (IEEE nearest-even, no fused multiply-add);
 *                constants and k, b are rounded once from their FP64 values.
 *   table_bits   q, 1..12: table of 2^q interval means indexed by the top q bits
 *                of the 32-bit uniform (Section 3.1, d = q).
 *   packed       APPROX only: take floor(32/q) q-bit indices per 32-bit word
 *                instead of one (the law of each index is the same); FP32 with
 *                q in {4, 6, 7, 8}, FP16 with q in {7, 8}.
 *   word_bits,   FIXED only, per variable (MLMC_V_*): two's-complement word w
 *   frac_bits    (2..32) and fractional bits f (0..62): value n 2^-f (Section 4.1,
 *                w = d + 1, f = d - e).  Every operation is rounded once to the
 *                destination's f, to nearest with ties toward +infinity, then
 *                saturated to w bits (saturations are counted).  The table entries
 *                use Z's format; the coarse sum of two normals keeps Z's f with one
 *                more integer bit; X's format must hold X_0 = 1 (f <= w - 2); constants and k, b are quantised exactly from
 *                their FP64 values (con1 = r h, con2 = sigma * sqrt(h),
 *                con3 = ((0.5 * sigma) * sigma) * h, k = K / S0, b = B / S0).
 *   rng_method   APPROX/CORR: the approximate normals of Section 3 (0 or 1:
 *                Method 1, the interval means; 2: Method 2 with two variables,
 *                Z~_j = +-X_a +-X_b from a table of 2^(q/2-1) values fitted by least
 *                squares under the sorting permutation pi, q even; the exact side of
 *                CORR then uses the coupled uniform whose top q bits are pi(j);
 *                3: Method 3, piecewise linear on the q - 1 dyadic intervals of
 *                the magnitude bits).  The library expands Methods 2 and 3 into the
 *                2^q-entry table (values formed in FP64, then rounded once to the
 *                side's format).  PLAIN: must be 0 or 1.
 *   exact_side   CORR: the exact side's arithmetic (Section 2.2's full-precision
 *                path on the same uniforms).  0: FP64 arithmetic with the FP64
 *                inverse normal (the paper's "double" increment); 1: FP32 Algorithm 1
 *                arithmetic with the FP32 inverse normal, as the plain-FP32
 *                estimator (FP64 then holds only the sums); needs an FP32 or FP16
 *                table side.  Other estimators: 0 or 1, ignored. */
typedef struct mlmc_precision {
    uint32_t struct_size;
    int32_t arith;
    int32_t table_bits;
    int32_t packed;
    int32_t word_bits[MLMC_NVARS];
    int32_t frac_bits[MLMC_NVARS];
    int32_t rng_method;
    int32_t exact_side;
} mlmc_precision;

/* Sums of one (level, estimator, payoff) over a set of paths (Section 2.1:
 * the per-level Monte Carlo estimator).  Y is the estimator's sample in
 * normalised units.  sum1/sum2 are FP64 sums of Y and Y^2.  For FIXED APPROX,
 * Y is an integer multiple of 2^-f_X and isum1 (int64) and isum2 (unsigned
 * 128-bit, lo/hi) are its exact integer sums; the FP64 view is filled too.
 * For CORR, esum1/esum2 are FP64 sums of the exact side's dP_l (for V_l). */
typedef struct mlmc_sums {
    uint64_t n;
    double sum1, sum2;
    int64_t isum1;
    uint64_t isum2_lo, isum2_hi;
    double esum1, esum2;
    uint64_t saturations;       /* FIXED: saturated operations over all paths */
    uint64_t nonfinite;         /* paths whose Y was not finite */
} mlmc_sums;

/* One record per path of a debug dump (mlmc_level_sums' debug_paths). */
typedef struct mlmc_path_record {
    double Y[MLMC_NPAYOFF];          /* estimator sample per payoff (0 if not asked) */
    int64_t Yraw[MLMC_NPAYOFF];      /* approx side dP~: integer (FIXED) or the FP64
                                        bit pattern of the float value */
    double XN_exact, XcN_exact;      /* fine / coarse terminal values, exact side */
    double XN_approx, XcN_approx;    /* approx side as FP64 (FIXED: n 2^-f_X) */
    int64_t XN_raw, XcN_raw;         /* FIXED approx side: the integers n */
    uint32_t first_word;             /* the 32-bit word holding fine step 0's uniform */
    uint32_t first_index;            /* table index of fine step 0 */
    uint32_t saturations;
    uint32_t reserved;
} mlmc_path_record;

typedef struct mlmc_context mlmc_context;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.
 * workspace: device buffer of workspace_bytes bytes that the context
 * sub-allocates for tables, work lists and sums; it is the context's HBM budget
 * (MLMC_E_NOMEM when a call needs more).  The caller owns it and keeps it alive
 * until mlmc_context_destroy.  NULL asks the library to allocate workspace_bytes
 * itself (freed at destroy).  stream: the hipStream_t launches go to (NULL: the
 * null stream); large launch sequences also use two streams the context creates
 * (see overlap_min_steps), and the library waits for those too before it reports
 * their results.  Errors: MLMC_E_INVALID (bad device, size < 1 MiB),
 * MLMC_E_DEVICE (HIP failure). */
mlmc_status mlmc_context_create(int32_t device, void* workspace, uint64_t workspace_bytes,
                                void* stream, mlmc_context** out);
void mlmc_context_destroy(mlmc_context* ctx);
/* The context's last error message; with ctx NULL, the calling thread's last
 * error of a context-free call (mlmc_level_sums_static). */
const char* mlmc_last_error(const mlmc_context* ctx);
const char* mlmc_status_string(int32_t status);
int32_t mlmc_abi_version(void);

/* --------------------------------------------------------------- level sums */

/* Sums of one level's estimator over paths [path_offset, path_offset + n_paths)
 * (Section 2.1 per-level estimator; Section 2.2 for APPROX/CORR).
 * level: 0..20, h = 2^-level T; level 0 has no coarse path (P_{-1} = 0).
 * seed, option_id: key and counter word of the uniform stream; path i, fine
 * step n uses stream position i 2^level + n (see mlmc_stream_word).
 * out: host array of popcount(payoff_mask) mlmc_sums, in increasing payoff
 * order.  debug_paths: NULL or a device array of n_paths mlmc_path_record
 * (same kernel; each record written once).
 * Synchronous on the context's stream.  Errors: MLMC_E_INVALID (validation, see
 * mlmc_problem / mlmc_precision; n_paths >= 1; path_offset + n_paths <= 2^40),
 * MLMC_E_NOMEM, MLMC_E_DEVICE. */
mlmc_status mlmc_level_sums(mlmc_context* ctx, const mlmc_problem* prob, int32_t level,
                            uint64_t n_paths, uint64_t path_offset,
                            const mlmc_precision* prec, int32_t estimator, uint64_t seed,
                            uint32_t option_id, mlmc_sums* out, void* debug_paths);

/* Many level sums in one launch sequence (one persistent kernel per estimator /
 * arithmetic class over a ragged list of tiles; the block finishing a work's last
 * tile adds the work's tile sums in a fixed order):
 * e.g. every (level, estimator) of a nested MLMC estimate with its own N_l
 * (Section 2.2).  Each work's sums equal those of mlmc_level_sums on the same
 * arguments.  works: host array; each out points at popcount(payoff_mask) sums.
 * Errors as mlmc_level_sums (the index of a failing work is in the message). */
typedef struct mlmc_level_work {
    uint32_t struct_size;
    int32_t level;
    int32_t estimator;
    uint32_t option_id;
    uint64_t n_paths, path_offset, seed;
    const mlmc_problem* prob;
    const mlmc_precision* prec;
    mlmc_sums* out;
} mlmc_level_work;

mlmc_status mlmc_level_sums_batch(mlmc_context* ctx, uint32_t n, const mlmc_level_work* works);

/* The same batch without waiting: validates, plans, uploads and launches it on the
 * context's stream and returns a ticket (> 0).  Batches run in enqueue order; up to
 * four are in flight, each in its own part of the workspace (an enqueue that finds
 * no room waits for the oldest).  The prob/prec structs may be reused at once; each
 * work's out array must stay valid until mlmc_level_sums_wait on the ticket (or on a
 * later one) returns, and is written then, or by any later call on the context that
 * has to wait for the batch.  Results equal mlmc_level_sums_batch's.  Errors as
 * mlmc_level_sums_batch, from the enqueue (nothing was launched) or from the wait. */
mlmc_status mlmc_level_sums_enqueue(mlmc_context* ctx, uint32_t n, const mlmc_level_work* works,
                                    uint64_t* ticket);

/* Waits for an enqueued batch and returns its status (its outs are written).  Every
 * ticket is waited on once; MLMC_E_UNKNOWN_TICKET for a ticket never issued or
 * already waited on. */
mlmc_status mlmc_level_sums_wait(mlmc_context* ctx, uint64_t ticket);

/* For callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  The sums of mlmc_level_sums for one
 * (level, estimator) path range without a context and without allocating: no
 * hipMalloc / hipFree, no pinned host memory, no stream or event, no library call
 * that allocates.  The plan and the per-tile partial sums live in a 4 MiB device
 * array inside the library, one per GPU, held until the process ends; the plan
 * reaches it as kernel arguments.  Every launch goes to `stream` (a hipStream_t on
 * the current device; NULL: the null stream) and the call returns without
 * waiting.
 *   prob, level, n_paths, path_offset, prec, estimator, seed, option_id: as
 *     mlmc_level_sums (host structs, read before the call returns).
 *   out_dev: DEVICE array of popcount(payoff_mask) mlmc_sums, in increasing payoff
 *     order, caller-owned; written by the stream's last kernel of the call.
 * The launch geometry is the library's default (mlmc_tuning defaults); the sums
 * equal mlmc_level_sums' under that geometry while the work needs at most 8192
 * tiles (larger works are split into 8192 tiles: integer sums are unchanged, FP64
 * sums may differ in rounding), without per-path debug records.
 * All calls on one GPU share its array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.  Nothing in
 * the array has to start at zero (every partial sum is written before it is read).
 * Errors: MLMC_E_INVALID (validation as mlmc_level_sums; out_dev NULL),
 * MLMC_E_NOMEM (the plan and partial sums exceed the 4 MiB array), MLMC_E_DEVICE
 * (a HIP call failed).  The message is mlmc_last_error(NULL) on the calling
 * thread. */
mlmc_status mlmc_level_sums_static(const mlmc_problem* prob, int32_t level, uint64_t n_paths,
                                   uint64_t path_offset, const mlmc_precision* prec,
                                   int32_t estimator, uint64_t seed, uint32_t option_id,
                                   void* stream, mlmc_sums* out_dev);

/* Kernel timing.  With timing on, every path-kernel launch is bracketed by HIP
 * events on the context's stream; per kernel class the library accumulates the
 * launches, the summed event time and the fine path-steps processed. */
typedef struct mlmc_kernel_stat {
    int32_t estimator, arith, scheme, fields;  /* fields: indices per 32-bit word */
    int32_t payoffs, track;
    int32_t level0;                            /* 1: the level-0 kernel of an exact-normal estimator */
    int32_t exact32;                           /* 1: correction estimator with an FP32 exact side */
    uint64_t launches;
    double ms;                                 /* summed event time */
    uint64_t path_steps;                       /* fine path-steps (paths * 2^level) */
} mlmc_kernel_stat;

/* Launch geometry of a context.  Results are reproducible for a fixed tuning;
 * FP64 sums may change in the last bits when it changes (summation order), integer
 * sums never do.  Defaults: 256, 256, 131072, 16, 512, 32768, 4194304.
 *   block_table   threads per block of the table-only (APPROX) kernels, 64..1024
 *   block_exact   threads per block of kernels with exact normals, 64..256
 *   tile_steps    target fine path-steps per tile
 *   blocks_per_cu persistent grid = CUs * blocks_per_cu
 *   min_tiles     a work is split into at least this many tiles when it can be
 *   zb_max_paths, zb_max_positions: exact-normal works (levels >= 2) with at most
 *                 this many paths and paths*2^level stream positions get their
 *                 normals computed ahead by a separate kernel (off the paths'
 *                 sequential chains); 0 disables.
 *   overlap_min_steps: launch sequences of at least this many fine path-steps
 *                 run their approximate-estimator kernels, with those works'
 *                 reduction, on a second stream beside the
 *                 exact-normal ones (with its own copy of the plan, uploaded on a
 *                 third stream, so that neither waits for the other), and their
 *                 level-0 exact-normal kernels on the third stream (it waits for
 *                 the context stream's upload; that stream's reduction waits for
 *                 it); smaller sequences use the context's stream alone.  Default
 *                 2^26. */
typedef struct mlmc_tuning {
    uint32_t struct_size;
    uint32_t block_table, block_exact;
    uint32_t tile_steps;
    uint32_t blocks_per_cu;
    uint32_t min_tiles;
    uint64_t zb_max_paths, zb_max_positions;
    uint64_t overlap_min_steps;
} mlmc_tuning;

mlmc_status mlmc_get_tuning(const mlmc_context* ctx, mlmc_tuning* out);
/* Chooses the launch geometry for a work list (host wall time per launch sequence
 * with `reps` sequences enqueued back to back, as a pipelined caller or the server
 * runs them, after a warm-up run; the least of three such rounds): two passes of
 * coordinate descent, the incumbent timed afresh at the start of each, over block_table {256, 512, 1024}, block_exact {64, 128, 256}, tile_steps
 * {2^14..2^18}, blocks_per_cu {2, 4, 8, 16}, min_tiles {512..4096} and zb_max_paths
 * {0, 2^13, 2^15, 2^17} and overlap_min_steps {0, 2^24, 2^26, 2^28, never},
 * starting from the context's current geometry and keeping
 * a change only when it is at least 1% faster (timing noise does not move it).  Sets the result on the context and copies it to
 * out (out->struct_size must be set).  The works' sums are written by every trial
 * run (the last trial's remain); sums of the same work can differ in FP64 rounding
 * between geometries (a different tile split), so tune before pricing.  Errors:
 * those of mlmc_level_sums_batch, MLMC_E_BUSY while a server runs, MLMC_E_INVALID
 * (reps outside 1..100). */
mlmc_status mlmc_autotune(mlmc_context* ctx, uint32_t n, const mlmc_level_work* works, uint32_t reps,
                          mlmc_tuning* out);
mlmc_status mlmc_set_tuning(mlmc_context* ctx, const mlmc_tuning* t);   /* MLMC_E_INVALID if out of range */

mlmc_status mlmc_set_timing(mlmc_context* ctx, int32_t on);  /* also clears the stats */
/* Copies up to max stats into out (host); *n receives the number available. */
mlmc_status mlmc_kernel_stats(mlmc_context* ctx, mlmc_kernel_stat* out, uint32_t max, uint32_t* n);

/* ----------------------------------------------------------- MLMC estimates */

/* On-line nested MLMC (Sections 2.1, 2.2 and 6): pilot samples on levels
 * 0..L_min, optimal allocation N_l = ceil(theta^-1 eps^-2 sqrt(V_l/C_l) Lambda)
 * (plain) or N~_l, N^D_l with the common Lambda (nested), sweeps of the missing
 * samples, then a bias test that adds level L+1 up to L_max while
 * max_{l = max(1, L-2)..L} |mean_l| 2^(alpha (l - L)) / (2^alpha - 1) exceeds
 * sqrt(1 - theta) eps, with alpha = 1 (the schemes' weak order).  Nested runs choose each level's estimator once its pilot
 * has landed: the level keeps the nested pair while
 * (sqrt(V~ c_approx) + sqrt(V^D c_corr))^2 <= V~ c_plain (Section 6's level
 * objective with plain samples as the full-precision alternative), otherwise its
 * nested samples are dropped (their work still counts in path_steps) and it goes
 * on with plain samples of plain_arith; a new level above a plain level >= 1
 * starts plain.  Costs are the deterministic model C_l = 2^l c_estimator
 * (Section 5: C_l ~ 2^l C_RNG).  eps_units 0: eps on the price / S0; 1: eps in
 * price units. */
typedef struct mlmc_run_config {
    uint32_t struct_size;
    int32_t nested;             /* 1: APPROX + CORR per level; 0: PLAIN */
    int32_t eps_units;          /* 0 normalised, 1 absolute */
    int32_t L_min, L_max;       /* 0 <= L_min <= L_max <= 20 */
    int32_t plain_arith;        /* PLAIN generator (plain runs, switched levels): FP64 or FP32 */
    double eps, theta;          /* eps > 0, 0 < theta <= 1 */
    uint64_t n_pilot;           /* >= 2 */
    double cost_plain, cost_approx, cost_corr;   /* cost per fine path-step (> 0) */
    mlmc_precision prec[MLMC_MAX_LEVELS];        /* approx side per level (nested) */
} mlmc_run_config;

typedef struct mlmc_level_stats {
    uint64_t n[3];              /* samples per estimator (PLAIN, APPROX, CORR) */
    double mean[3], var[3];     /* normalised level mean and variance (R9) */
} mlmc_level_stats;

typedef struct mlmc_result {
    uint32_t struct_size;
    int32_t status;
    int32_t L;                  /* finest level used */
    int32_t sweeps;
    double estimate;            /* e^{-rT} S0 sum_l (means) */
    double variance;            /* (e^{-rT} S0)^2 sum_l var / n */
    double seconds;             /* wall time of the estimate */
    uint64_t path_steps;        /* fine path-steps generated, all estimators */
    uint64_t saturations;
    int32_t exact_sides;        /* samples in the estimate: bit 0 correction with an FP64
                                   exact side, bit 1 correction with an FP32 exact side,
                                   bit 2 plain samples (plain_arith) */
    int32_t pad;
    mlmc_level_stats level[MLMC_MAX_LEVELS];
} mlmc_result;

/* Who drives the estimates' sweeps.  MLMC_DRIVER_ENGINE: the device sweep engine --
 * each option's run state (level sums, sample counts = the next path index of each
 * uniform stream, the driver's decisions) stays in device memory; one sweep of all
 * options is one replay of a HIP graph that computes every run's next samples
 * (pilot, per-level estimator, optimal allocation, bias test) on the device, plans
 * their tiles, runs the path kernels and adds each work's fixed-order sums into its
 * run; the host only replays it, prepares the levels a run reaches and collects
 * finished runs.  MLMC_DRIVER_HOST: the host computes each sweep's works from
 * downloaded sums and launches them (a launch sequence per sweep, with only the
 * kernel classes that have work).  MLMC_DRIVER_AUTO (the default): the engine for
 * mlmc_estimate_batch calls of at least MLMC_ENGINE_MIN_RUNS options, the host
 * otherwise and for the server (the engine's sweep has a fixed cost of a few hundred
 * microseconds that few runs do not amortise).  All give the same results bit for
 * bit (same decisions on the same sums, same tiles, same reductions).  A workspace
 * too small for the engine's arrays falls back to host-driven sweeps.  Errors:
 * MLMC_E_INVALID, MLMC_E_BUSY (a server is running). */
enum { MLMC_DRIVER_HOST = 0, MLMC_DRIVER_ENGINE = 1, MLMC_DRIVER_AUTO = 2 };
#define MLMC_ENGINE_MIN_RUNS 64
mlmc_status mlmc_set_driver(mlmc_context* ctx, int32_t driver);

/* One option, one payoff (single bit of payoff_mask).  Errors as
 * mlmc_level_sums plus MLMC_E_INVALID for the run config. */
mlmc_status mlmc_estimate(mlmc_context* ctx, const mlmc_problem* prob,
                          const mlmc_run_config* cfg, uint64_t seed, uint32_t option_id,
                          mlmc_result* out);

/* n options at once (option i uses option_id i and payoff bit of probs[i]); each
 * sweep of all options runs as one persistent launch over a ragged work list.
 * Each option's result equals that of mlmc_estimate alone with the same
 * (seed, option_id). */
mlmc_status mlmc_estimate_batch(mlmc_context* ctx, uint32_t n, const mlmc_problem* probs,
                                const mlmc_run_config* cfg, uint64_t seed,
                                mlmc_result* out);

/* ------------------------------------------------------------------ serving */

/* Continuous batching.  mlmc_server_start launches a scheduler thread on the
 * context.  A request is admitted when one of max_active slots is free; its state
 * (level sums, sample counts) stays on the host.  The scheduler keeps up to two
 * launch sequences in flight: whenever fewer are running it gathers the next
 * samples of every admitted request that has no work in flight (pilot, allocation
 * top-up or a new level; Sections 2.1, 2.2 and 6) into one more sequence, so a
 * request that arrives while others run starts in the next sequence, queued behind
 * the running one.  Device memory is the context's workspace (the HBM budget):
 * each sequence's plan takes a ring slice of it, older sequences land to make
 * room, and a plan larger than the workspace runs as several sequences.  A
 * request's result is the same as mlmc_estimate with its (seed, option_id) and run
 * config; mlmc_result.seconds is its latency, submission to result. */
typedef struct mlmc_server_config {
    uint32_t struct_size;
    uint32_t max_active;        /* slots: requests on the device at once (>= 1) */
    mlmc_run_config run;        /* template; eps and nesting come from each request */
} mlmc_server_config;

typedef struct mlmc_request {
    uint32_t struct_size;
    uint32_t option_id;
    mlmc_problem problem;       /* one payoff bit */
    double eps;                 /* this request's eps (units of run.eps_units) */
    uint64_t seed;
    int32_t nested;
    int32_t reserved;
} mlmc_request;

mlmc_status mlmc_server_start(mlmc_context* ctx, const mlmc_server_config* cfg);
/* Copies the request; returns a ticket.  Thread-safe. */
mlmc_status mlmc_submit(mlmc_context* ctx, const mlmc_request* req, uint64_t* ticket);
/* MLMC_PENDING until done, then MLMC_OK with the result (once).  Thread-safe. */
mlmc_status mlmc_poll(mlmc_context* ctx, uint64_t ticket, mlmc_result* out);
/* Up to max finished requests, oldest completion first: tickets[i] and out[i]
 * (host arrays of max entries); *n receives the count (0 when none).  A result is
 * handed out once, by this call or by mlmc_poll.  Thread-safe.  Errors:
 * MLMC_E_BUSY (no server), MLMC_E_INVALID (NULL pointers). */
mlmc_status mlmc_poll_done(mlmc_context* ctx, uint32_t max, uint64_t* tickets, mlmc_result* out,
                           uint32_t* n);
/* Counters of the running server since its start (host clock). */
typedef struct mlmc_server_stats {
    uint32_t struct_size;
    uint32_t pad;
    uint64_t flights;           /* launch sequences started */
    uint64_t works;             /* (request, level, estimator) works in them */
    uint64_t requests_done;     /* requests that converged */
    uint64_t queued, active;    /* now: waiting for a slot / admitted */
    double plan_seconds;        /* scheduler: next samples, planning, upload, launch */
    double land_seconds;        /* scheduler: landing flights, adding their sums */
    double idle_seconds;        /* scheduler: waiting for a flight or a request */
    uint32_t engine;            /* 1: runs on the device sweep engine (flights: sweeps) */
    uint32_t slots;             /* requests the workspace admits at once */
    uint64_t bytes_per_request; /* engine: device bytes one admitted request holds */
} mlmc_server_stats;

/* out->struct_size must be set.  Errors: MLMC_E_BUSY (no server), MLMC_E_VERSION. */
mlmc_status mlmc_server_stats_get(mlmc_context* ctx, mlmc_server_stats* out);
/* Finishes admitted requests and stops the thread; requests still queued (not
 * admitted) end with status MLMC_E_BUSY. */
mlmc_status mlmc_server_stop(mlmc_context* ctx);

/* ------------------------------------------- rounding-error model (Sections 4-6) */

/* The linear error model of one level of the European call (Section 4.2).
 * For variable v (MLMC_V_*) with instances j (one per fine and per coarse step of a
 * sample, Z one per fine normal, con1 twice: con1 and con1c):
 *   S[v] = sum_j E[xbar_vj^2],  R[v] = sum_j sqrt(E[xbar_vj^2]),
 * xbar the sensitivity d(dP)/dx of the level sample dP = P(X_N) - P(Xc_{N/2}) (level
 * 0: P(X_1)), on FP64 paths with exact normals of the correction estimator's stream.
 * e[v]: the exponent with |x| < 2^e over every instance (Section 4.1); Z's from the
 * q-bit Method-1 table.  V_indep(d) = (1/12) sum_v S[v] 4^(e[v] - d[v]) and
 * V_corr(d) = (sum_v R[v] 2^(e[v] - d[v] - 1))^2; with approximate normals
 * (Section 4.3) the terms S[Z] mse and R[Z] sqrt(mse) are added (without the 1/12:
 * the table's error is not a uniform rounding error).  used[v] = 0: the variable is
 * not in the scheme (Euler: con3, zsq, zm1, mul3, sum2). */
typedef struct mlmc_error_model {
    uint32_t struct_size;
    int32_t level, scheme, table_bits;
    uint64_t n_paths;
    int32_t used[MLMC_NVARS];
    int32_t e[MLMC_NVARS];
    double S[MLMC_NVARS];
    double R[MLMC_NVARS];
    double V_level;             /* V[dP] of the exact paths (normalised units) */
    double mse;                 /* Method-1 table MSE at table_bits */
} mlmc_error_model;

/* Runs the sensitivity kernel over paths 0 .. n_paths-1 of (seed, option_id) at
 * `level` (one wave of 64 paths per lane group, FP64 atomics into the workspace,
 * which it needs whole: in-flight batches are landed first).  prob: one payoff,
 * the European call; q: the table whose MSE and largest value enter the model.
 * out->struct_size must be set.  Errors: MLMC_E_INVALID (payoff, level > 20,
 * n_paths < 2, q outside 1..16), MLMC_E_NOMEM (workspace below 12 (3/2) 2^level
 * doubles), MLMC_E_DEVICE. */
mlmc_status mlmc_error_model_compute(mlmc_context* ctx, const mlmc_problem* prob, int32_t level,
                                     uint64_t n_paths, int32_t q, uint64_t seed, uint32_t option_id,
                                     mlmc_error_model* out);

/* Bit widths of one level (Section 6).  Cost: the separable relaxation of Section 5,
 * C(d) = sum_v (1/2) M_v d_v^2 + M'_v d_v with M (M') the multiplications
 * (additions) that take v as an operand per sample, counted on the kernel's
 * operations (fine step: the table's multiplier times X, and the add; coarse step:
 * the whole chain).  For a multiplier lambda each d_v solves
 * ln4 (S_v / 12) 4^(e_v - d_v) = lambda (M_v d_v + M'_v) on [0, d_max] (d_max = 31,
 * Z 30), lambda minimises the level objective sqrt(V_level C(d)) +
 * sqrt(V^D(d) C_l), C_l = 2^level c_rng, V^D = V_indep (+ the table term when
 * rng_term) by golden-section search over the lambdas of uniform widths 4..16, and
 * d is rounded by the greedy ratio rule (floor, then one bit at a time in order of
 * variance gained per cost until V^D <= V^D(real d)).  word_bits / frac_bits: the
 * kernel's formats of d_int (w = d + 1, f = d - e), with fractional bits that
 * could not change a result dropped (a product keeps at most f_a + f_b, a sum at
 * most max(f_a, f_b), summands differ by at most 30, zsq keeps at most 30), so
 * they pass mlmc_validate.  Host only.  Errors: MLMC_E_INVALID, MLMC_E_VERSION. */
typedef struct mlmc_width_plan {
    uint32_t struct_size;
    int32_t best_uniform;       /* the uniform width of 4..16 with the least objective */
    double lambda;
    double objective;           /* at the real widths */
    double objective_uniform;   /* at best_uniform */
    double v_indep, cost;       /* at d_int */
    double d_real[MLMC_NVARS];
    int32_t d_int[MLMC_NVARS];
    int32_t word_bits[MLMC_NVARS];
    int32_t frac_bits[MLMC_NVARS];
} mlmc_width_plan;

mlmc_status mlmc_optimise_widths(const mlmc_error_model* model, double c_rng, int32_t rng_term,
                                 mlmc_width_plan* out);

/* The exact normal of the coupled pair (Section 3.1): Z = Phi^-1(U) with
 * U = 2^-32 (J + 1/2), for n 32-bit words, by the path kernels' own inverse normal
 * (the four-wide form the exact-normal loops use, on groups of four; a ragged
 * tail with the scalar form).  J_dev: device array of n uint32; out_dev: device
 * array of n doubles (arith MLMC_ARITH_FP64) or floats (MLMC_ARITH_FP32).
 * Synchronous on the context's stream.  Errors: MLMC_E_INVALID (arith, NULL
 * buffers), MLMC_E_DEVICE. */
mlmc_status mlmc_inverse_normal(mlmc_context* ctx, const uint32_t* J_dev, uint64_t n, int32_t arith,
                                void* out_dev);

/* The low-precision side of one level chosen by Section 6's level objective, with
 * the cost of Section 5 measured in gfx950 issue cycles instead of FPGA bit
 * operations.  Issue rates of the instruction classes the path kernels use, in
 * wave-instructions per CU per clock (an instruction's issue cost is the reciprocal):
 * FP32/FP16 arithmetic, 32-bit integer, FP64 FMA and add, 32x32->64 multiply-add,
 * random 8-byte and 4-byte LDS reads. */
typedef struct mlmc_gpu_rates {
    uint32_t struct_size;
    uint32_t pad;
    double f32, i32, f64_fma, f64_add, u64_mad, lds_b64, lds_b32;
} mlmc_gpu_rates;

/* The rates measured on one MI355X by the issue-rate probe.  out->struct_size must
 * be set. */
mlmc_status mlmc_gpu_rates_default(mlmc_gpu_rates* out);

/* Cost per fine path-step (CU issue cycles per 64 path-steps) of the approximate
 * estimator (Philox word share, index, table read, the side's fine step and half a
 * coarse step, the per-path payoff and sums over 2^level steps) and of the
 * correction estimator (one word per step, the FP64 inverse normal and FP64 steps,
 * the table side unpacked), for a table side (arith FP32 / FP16 / FIXED, q, packed)
 * at `level`.  Host only.  Errors: MLMC_E_INVALID, MLMC_E_VERSION. */
mlmc_status mlmc_side_costs(int32_t arith, int32_t table_bits, int32_t packed, int32_t scheme,
                            int32_t level, const mlmc_gpu_rates* rates, double* c_approx, double* c_corr);

typedef struct mlmc_level_choice {
    uint32_t struct_size;
    int32_t level, arith, table_bits, packed;
    int32_t pad;
    double v_approx, v_corr;     /* V~ (= V_level) and the modelled V^D */
    double c_approx, c_corr;     /* 2^level times the costs per fine path-step */
    double objective;            /* sqrt(V~ C~) + sqrt(V^D C^D) of the choice */
    double objective_fp32_q8;    /* the same for FP32 with q = 8 packed indices */
} mlmc_level_choice;

/* Section 6's level objective sqrt(V~ C~) + sqrt(V^D C^D) minimised over the table
 * sides FP32 with q = 8, 6, 4 (packed) and 10, 12; FP16 with q = 8, 7 (packed) and
 * 10; and, when fixed_formats is given, FIXED with those formats and q = 8, 10, 12
 * (the first minimum in that order wins).  V~ = model->V_level; V^D = the linear
 * rounding model (1/12) sum_v S_v 4^(e_v - d_v) with d = the significand bits (FP32
 * 24, FP16 11) or w - 1 of the fixed formats, plus S_Z MSE_q (the Method-1 table of
 * q bits, Section 4.3, without the 1/12); C~, C^D = 2^level mlmc_side_costs.
 * out: the chosen precision (rng_method 1, exact_side 0; fixed: fixed_formats' widths);
 * info (NULL allowed): the numbers behind it.  struct_size of every struct must be
 * set.  Host only.  Errors: MLMC_E_INVALID, MLMC_E_VERSION. */
mlmc_status mlmc_choose_precision(const mlmc_error_model* model, const mlmc_gpu_rates* rates,
                                  const mlmc_precision* fixed_formats, mlmc_precision* out,
                                  mlmc_level_choice* info);

/* ------------------------------------------------- host-side helpers (no GPU) */

/* Method-1 table (Section 3.1): T_q[k] = 2^q (phi(Phi^-1(k 2^-q)) -
 * phi(Phi^-1((k+1) 2^-q))), the mean of Phi^-1 over interval k, rounded to
 * nearest in the target format.  arith FP64 -> double[2^q]; FP32 -> float[2^q];
 * FP16 -> uint16_t[2^q] (binary16 bits); FIXED -> int32_t[2^q] with frac_bits
 * fractional bits.  out: host buffer.  Errors: MLMC_E_INVALID (q outside 1..16). */
mlmc_status mlmc_build_table(int32_t q, int32_t arith, int32_t frac_bits, void* out);

/* Methods 2 and 3 of Section 3 (see mlmc_precision.rng_method): values[2^q] (FP64,
 * before rounding to a side's format) and, for Method 2, perm[2^q] (pi; NULL
 * allowed; untouched for Method 3).  *iterations (NULL allowed): Method 2's
 * least-squares solves until pi repeated.  Host buffers.  Errors: MLMC_E_INVALID
 * (method not 2 or 3; q outside 2..12; odd q for Method 2). */
mlmc_status mlmc_build_rng_table(int32_t q, int32_t method, double* values, uint16_t* perm,
                                 int32_t* iterations);

/* The 32-bit uniform word at stream position `word_index` (Philox4x32-10,
 * Salmon et al. 2011; counter (b mod 2^32, b div 2^32, level | estimator << 8,
 * option_id) for block b = word_index / 4, key = seed) -- host evaluation, for
 * checking.  out: host array of `count` words starting at word_index. */
mlmc_status mlmc_stream_words(uint64_t seed, uint32_t option_id, int32_t level,
                              int32_t estimator, uint64_t word_index, uint64_t count,
                              uint32_t* out);

/* Argument validation as performed by mlmc_level_sums (no device needed). */
mlmc_status mlmc_validate(const mlmc_problem* prob, int32_t level, uint64_t n_paths,
                          uint64_t path_offset, const mlmc_precision* prec,
                          int32_t estimator);

/* The kernels' per-path code compiled for the host, run on paths
 * [path_offset, path_offset + n_paths) with n_paths <= 65536: the same
 * arithmetic and per-path records as mlmc_level_sums (sums are added in path
 * order rather than the kernels' tree order).  A checker of the kernel
 * arithmetic on machines without a GPU; no other entry point calls it.
 * out: as mlmc_level_sums; records: host array of n_paths records or NULL (then
 * the kernels' sums-only code runs where they have one, as without a debug buffer:
 * the level-0 loop of the exact-normal estimators).
 * Errors: MLMC_E_INVALID (validation, n_paths > 65536), MLMC_E_OVERFLOW. */
mlmc_status mlmc_check_paths_host(const mlmc_problem* prob, int32_t level, uint64_t n_paths,
                                  uint64_t path_offset, const mlmc_precision* prec,
                                  int32_t estimator, uint64_t seed, uint32_t option_id,
                                  mlmc_sums* out, mlmc_path_record* records);

/* mlmc_inverse_normal with the kernels' code compiled for the host (FP32: the
 * host's logarithm in place of the device's): host arrays J[n] and out[n]. */
mlmc_status mlmc_inverse_normal_host(const uint32_t* J, uint64_t n, int32_t arith, void* out);

/* Sample allocation (Section 2.1 / 2.2) as used by the drivers:
 * N_i = ceil(theta^-1 eps2^-1 sqrt(V_i / C_i) sum_j sqrt(V_j C_j)) over the m
 * (level, estimator) pairs given.  out: host uint64_t[m]. */
mlmc_status mlmc_allocate(uint32_t m, const double* V, const double* C, double eps2,
                          double theta, uint64_t* out);

#ifdef __cplusplus
}
#endif
#endif /* MLMC_H */
