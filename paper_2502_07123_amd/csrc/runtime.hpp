// Runtime internals: the context, launch planning and execution.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mlmc.h"
#include "common.hpp"
#include "device/advance.hpp"
#include "host/prepare.hpp"
#include "kernels.hpp"

namespace mlmc {

// Launch geometry (chosen per device by the tuner; fixed within a context so that
// sums are reproducible).
struct Tuning {
    uint32_t block_table = 256;     // threads per block, table-only kernels
    uint32_t block_exact = 256;     // threads per block, kernels with exact normals
    uint32_t tile_steps = 1u << 17; // path-steps per tile (target)
    uint32_t blocks_per_cu = 16;    // persistent grid = CUs * blocks_per_cu (cap)
    uint32_t min_tiles = 512;       // a work is split into at least this many tiles when it can be
    // exact-normal works with at most zb_max_paths paths (and zb_max_positions
    // stream positions) get their normals computed ahead, off the paths' chains
    uint64_t zb_max_paths = 1u << 15;
    uint64_t zb_max_positions = 1u << 22;
    // flights of at least this many fine path-steps run their table-only kernels on
    // the second stream (a second plan upload and a second reduction launch, which small
    // flights do not win back)
    uint64_t overlap_min_steps = uint64_t(1) << 26;
};

// The calling thread's last error message of mlmc_level_sums_static ("" if none).
const char* static_last_error();

// Whether a work of variant v at `level` runs in the level-0 kernel of the
// exact-normal estimators (level 0, no debug records, the correction estimator's
// per-index approximate samples fit in LDS).
bool level0_kernel_for(const Variant& v, int level, bool debug, const LevelDev& L);

// Threads per block of a kernel variant under a geometry.
uint32_t block_for(const Tuning& t, const Variant& v, const VariantInfo& vi);

constexpr uint64_t FLIGHT_MAX_TILES = uint64_t(1) << 16;
WorkSplit split_work(const Tuning& t, uint32_t block, uint64_t S, int level, uint64_t path_begin, uint64_t n,
                     uint64_t max_tiles);

// Dynamic LDS bytes the path kernel of variant v needs for level L.
uint32_t lds_bytes_for(const Variant& v, const LevelDev& L);

// One (option, level, estimator) path range of a launch.
struct WorkSpec {
    const mlmc_problem* prob;
    int32_t level;
    const mlmc_precision* prec;
    int32_t est;
    uint64_t seed;
    uint32_t option;
    uint64_t path_begin, n;
    uint64_t debug;                 // device address of records or 0
    const LevelPrep* prep = nullptr;   // the level prepared by the caller, or null
};

struct Server;
struct Engine;

struct PinnedBuf {
    uint8_t* p = nullptr;
    size_t bytes = 0;
    bool busy = false;              // staging a flight that has not landed
};

// One launch sequence on the stream: its plan occupies workspace bytes
// [base, end), its staging buffer holds the uploaded plan and, once `done` has
// fired, the per-work results at down_off.
struct Flight {
    uint64_t ticket = 0;            // 0: an internal synchronous run
    size_t base = 0, end = 0;
    int pin = -1;
    size_t down_off = 0;
    uint32_t n_works = 0;
    hipEvent_t done = nullptr;
    hipEvent_t done_aux = nullptr;  // the second stream's part (two-stream flights)
    hipEvent_t ev_plan = nullptr;   // the plan uploaded (the level-0 stream waits for it)
    hipEvent_t ev_l0 = nullptr;     // the level-0 exact-normal kernels done
    hipEvent_t ev_up2 = nullptr;    // the second stream's plan copy uploaded
    std::vector<uint32_t> order;    // two-stream flights: result position -> work
    struct Timed {
        Variant v;
        uint64_t steps = 0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
    };
    std::vector<Timed> timed;
    std::vector<mlmc_level_work> deliver;   // enqueued batches: where results go
    std::vector<uint32_t> masks;            // their payoff masks
    std::shared_ptr<std::vector<SlotDev>> sink;   // server flights: per-work results
};

}  // namespace mlmc

struct mlmc_context {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t aux_stream = nullptr;    // table-only path kernels beside the exact-normal ones
    hipStream_t l0_stream = nullptr;     // level-0 exact-normal kernels beside the other exact levels
    bool own_ws = false;
    uint8_t* ws = nullptr;
    uint64_t ws_bytes = 0;
    std::string err;
    bool poisoned = false;
    std::vector<mlmc::PinnedBuf> pins;
    int cu_count = 0;
    mlmc::Tuning tune;
    std::mutex dev_mtx;             // one launch sequence at a time on the device
    std::unique_ptr<mlmc::Server> server;
    // device sweep engines of recent batches of estimates (kept for their graphs;
    // each lays its arrays over the workspace while it runs)
    std::vector<std::unique_ptr<mlmc::Engine>> engines;
    int driver = MLMC_DRIVER_AUTO;  // who drives estimates' sweeps (mlmc_set_driver)
    bool ws_held = false;           // a server's sweep engine holds the workspace
    uint64_t tune_key() const;      // the launch geometry, as one number
    // per-context cache of prepared levels (key: problem, level, precision, estimator)
    std::map<std::string, mlmc::LevelPrep> prep_cache;
    // launch sequences in flight (oldest first) and statuses of landed tickets
    std::deque<mlmc::Flight> flights;
    std::map<uint64_t, mlmc_status> finished;
    uint64_t next_ticket = 1;
    std::vector<hipEvent_t> ev_plain, ev_timed;   // free events
    // kernel timing (HIP events around each path-kernel launch)
    bool timing = false;
    std::vector<mlmc_kernel_stat> stats;
    mlmc_context();                 // both defined where Server is complete
    ~mlmc_context();
};

namespace mlmc {

mlmc_status fail(mlmc_context* ctx, mlmc_status s, const std::string& msg);

// Runs the works as one launch sequence (path kernels, one per variant, each
// work's sums reduced in a fixed order) and waits for it; out gets one SlotDev per
// work, in order.  Flights already in progress stay in progress.
mlmc_status run_works(mlmc_context* ctx, const std::vector<WorkSpec>& works, std::vector<SlotDev>& out);
// The same split in two: launch_flight plans, places and launches (caller holds
// dev_mtx and, for an enqueued batch, appends f to ctx->flights); land_flight waits
// for it and delivers the results; drain_oldest / drain_flights land flights in
// order, keeping their statuses in ctx->finished.
mlmc_status launch_flight(mlmc_context* ctx, const std::vector<WorkSpec>& works, Flight& f);
mlmc_status land_flight(mlmc_context* ctx, Flight& f, std::vector<SlotDev>* out);
mlmc_status drain_oldest(mlmc_context* ctx);
mlmc_status drain_flights(mlmc_context* ctx);
// a += b in a fixed field order (host side accumulation of sweep results)
void slot_accumulate(SlotDev& a, const SlotDev& b);
mlmc_status estimate_batch(mlmc_context* ctx, uint32_t n, const mlmc_problem* probs,
                           const mlmc_run_config* cfg, uint64_t seed, const uint32_t* ids,
                           mlmc_result* out);

void slot_to_sums(const SlotDev& s, int np_slot, mlmc_sums& o);
mlmc_status validate_run(const mlmc_problem* prob, const mlmc_run_config* cfg, std::string& err);

// Adaptive nested MLMC for a set of options advancing in lockstep sweeps.
struct OptionRun {
    mlmc_problem prob;
    mlmc_run_config cfg;
    uint64_t seed = 0;
    uint32_t option = 0;
    RunState st;                                // sums, levels, decisions (device/advance.hpp)
    double t_start = 0.0, t_end = 0.0;
    uint64_t saturations = 0;
    // levels prepared for this option (constants, table, variant), per estimator
    std::vector<std::array<std::shared_ptr<const LevelPrep>, 3>> preps;
};

// The option's normalised eps (eps_units) and its RunState's initial values.
double option_eps(const mlmc_problem& prob, const mlmc_run_config& cfg);
void run_state_init(RunState& st, const mlmc_problem& prob, const mlmc_run_config& cfg);
// The payoff slot 0 of a work's result as EstSums.
EstSums est_of_slot(const SlotDev& s);
void result_of_state(const RunState& st, const mlmc_problem& prob, const mlmc_run_config& cfg, double seconds,
                     mlmc_result& r);

void option_init(OptionRun& o);
// Pending (level, estimator, extra samples) of an option, or none when done.
struct Pending {
    int level, est;
    uint64_t n;
};
std::vector<Pending> option_advance(OptionRun& o);
// The option's prepared level (built once per (level, estimator) and kept).
mlmc_status option_prep(OptionRun& o, int level, int est, const mlmc_precision* prec,
                        const LevelPrep*& out, std::string& err);
void option_result(const OptionRun& o, mlmc_result& r);
mlmc_status run_sweeps(mlmc_context* ctx, std::vector<OptionRun*>& opts);
// One sweep over the options that are not done (ran: whether any work was run).
mlmc_status sweep_once(mlmc_context* ctx, const std::vector<OptionRun*>& opts, bool& ran);
double now_seconds();

}  // namespace mlmc
