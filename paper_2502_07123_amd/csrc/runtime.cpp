// C-ABI entry points and the runtime behind them: context and workspace, launch
// planning (works -> tiles -> slots), execution on the caller's stream, the
// adaptive nested MLMC driver (Sections 2.1, 2.2 and 6), batched pricing and the
// continuous-batching server.
#include "runtime.hpp"

#include "device/philox.hpp"
#include "engine_host.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <tuple>
#include <unordered_map>

namespace mlmc {

double now_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

mlmc_status fail(mlmc_context* ctx, mlmc_status s, const std::string& msg);

}  // namespace mlmc

uint64_t mlmc_context::tune_key() const {
    uint64_t h = 1469598103934665603ull;
    const uint64_t f[] = {tune.block_table, tune.block_exact, tune.tile_steps, tune.blocks_per_cu, tune.min_tiles,
                          ws_bytes, reinterpret_cast<uint64_t>(ws)};
    for (uint64_t x : f) h = (h ^ x) * 1099511628211ull;
    return h;
}

namespace mlmc {

mlmc_status fail(mlmc_context* ctx, mlmc_status s, const std::string& msg) {
    if (ctx) {
        ctx->err = msg;
        if (s == MLMC_E_DEVICE) ctx->poisoned = true;
    }
    return s;
}

#define HIPCHK(call)                                                                   \
    do {                                                                               \
        const hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                          \
            return fail(ctx, MLMC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static std::string prep_key(const mlmc_problem* p, int level, const mlmc_precision* prec, int est) {
    std::string k;
    k.append(reinterpret_cast<const char*>(p), sizeof(*p));
    k.append(reinterpret_cast<const char*>(&level), sizeof(level));
    k.append(reinterpret_cast<const char*>(prec), sizeof(*prec));
    k.append(reinterpret_cast<const char*>(&est), sizeof(est));
    return k;
}

void slot_to_sums(const SlotDev& s, int i, mlmc_sums& o) {
    o.n = s.n;
    o.sum1 = s.s1[i];
    o.sum2 = s.s2[i];
    o.isum1 = s.i1[i];
    o.isum2_lo = s.i2lo[i];
    o.isum2_hi = s.i2hi[i];
    o.esum1 = s.e1[i];
    o.esum2 = s.e2[i];
    o.saturations = s.sat;
    o.nonfinite = s.nonfinite;
}

namespace {
using VKey = std::tuple<int, int, int, int, bool, int, bool, bool>;
VKey vkey(const Variant& v) { return VKey{v.est, v.arith, v.scheme, v.np, v.track, v.fields, v.l0, v.exact32}; }

struct LaunchGroup {
    Variant v;
    VariantInfo vi;
    std::vector<uint32_t> works;
    uint32_t w0 = 0, w1 = 0;        // its work-tile descriptors
    uint32_t n_tiles = 0, block = 0, lds = 0;
    uint32_t cnt = 0;               // index of its (work descriptors, tiles) count pair
};

constexpr size_t MAX_FLIGHTS = 4;

// a pinned staging buffer of at least `bytes`, not used by a flight in progress
mlmc_status take_pinned(mlmc_context* ctx, size_t bytes, int& idx) {
    idx = -1;
    for (size_t i = 0; i < ctx->pins.size(); ++i)
        if (!ctx->pins[i].busy && ctx->pins[i].bytes >= bytes) { idx = static_cast<int>(i); break; }
    if (idx < 0) {
        for (size_t i = 0; i < ctx->pins.size(); ++i)
            if (!ctx->pins[i].busy) { idx = static_cast<int>(i); break; }
        if (idx < 0) {
            ctx->pins.emplace_back();
            idx = static_cast<int>(ctx->pins.size() - 1);
        }
        PinnedBuf& pb = ctx->pins[idx];
        if (pb.p) (void)hipHostFree(pb.p);
        pb.p = nullptr;
        pb.bytes = 0;
        const size_t want = std::max<size_t>(bytes, size_t(1) << 20);
        // coherent: the flight's upload kernel reads the plan from it directly
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&pb.p), want, hipHostMallocCoherent));
        pb.bytes = want;
    }
    ctx->pins[idx].busy = true;
    return MLMC_OK;
}

mlmc_status take_event(mlmc_context* ctx, bool timed, hipEvent_t& e) {
    auto& pool = timed ? ctx->ev_timed : ctx->ev_plain;
    if (!pool.empty()) {
        e = pool.back();
        pool.pop_back();
        return MLMC_OK;
    }
    HIPCHK(hipEventCreateWithFlags(&e, timed ? hipEventDefault : hipEventDisableTiming));
    return MLMC_OK;
}

void add_stat(mlmc_context* ctx, const Variant& v, float ms, uint64_t steps) {
    mlmc_kernel_stat* st = nullptr;
    for (auto& x : ctx->stats)
        if (x.estimator == v.est && x.arith == v.arith && x.scheme == v.scheme && x.fields == v.fields &&
            x.payoffs == v.np && x.track == int(v.track) && x.level0 == int(v.l0) &&
            x.exact32 == int(v.exact32))
            st = &x;
    if (!st) {
        mlmc_kernel_stat z;
        std::memset(&z, 0, sizeof(z));
        z.estimator = v.est;
        z.arith = v.arith;
        z.scheme = v.scheme;
        z.fields = v.fields;
        z.payoffs = v.np;
        z.track = v.track ? 1 : 0;
        z.level0 = v.l0 ? 1 : 0;
        z.exact32 = v.exact32 ? 1 : 0;
        ctx->stats.push_back(z);
        st = &ctx->stats.back();
    }
    st->launches += 1;
    st->ms += ms;
    st->path_steps += steps;
}
}  // namespace

bool level0_kernel_for(const Variant& v, int level, bool debug, const LevelDev& L) {
    if (level != 0 || debug || v.est == MLMC_EST_APPROX) return false;
    if (v.est == MLMC_EST_CORR && uint32_t(v.np) * L.table_entries > YTAB_MAX_ENTRIES) return false;
    return has_level0_kernel(v);
}

uint32_t block_for(const Tuning& t, const Variant& v, const VariantInfo& vi) {
    return std::min<uint32_t>(vi.tab_bytes && v.est == MLMC_EST_APPROX ? t.block_table : t.block_exact,
                              static_cast<uint32_t>(vi.max_block));
}

WorkSplit split_work(const Tuning& t, uint32_t block, uint64_t S, int level, uint64_t path_begin, uint64_t n,
                     uint64_t max_tiles) {
    return split_groups(t.tile_steps, t.min_tiles, block, S, level, path_begin, n, max_tiles);
}

// LDS of a work: its step table, plus the level-0 index histogram of the approximate
// estimator or (FP32, small enough) its per-index sample table, or the correction
// estimator's per-index approximate-side samples (float table side).
uint32_t lds_bytes_for(const Variant& v, const LevelDev& L) {
    uint32_t extra = 0;
    const uint32_t ys = static_cast<uint32_t>(v.np) * L.table_entries;
    if (v.est == MLMC_EST_APPROX) {
        extra = 4u * L.table_entries;
        if (v.arith != MLMC_ARITH_FIXED && ys <= YTAB_MAX_ENTRIES) extra = std::max(extra, 8u * ys);
    } else if (v.est == MLMC_EST_CORR && v.arith != MLMC_ARITH_FIXED && ys <= YTAB_MAX_ENTRIES) {
        extra = 8u * ys;
    }
    return L.table_bytes + extra;
}

// Waits for a flight, copies its results (to out, or to the mlmc_sums of its
// enqueued work list) and returns its staging buffer and events to the pools.
mlmc_status land_flight(mlmc_context* ctx, Flight& f, std::vector<SlotDev>* out) {
    hipError_t e = hipEventSynchronize(f.done);
    ctx->ev_plain.push_back(f.done);
    if (f.done_aux) {
        const hipError_t e2 = hipEventSynchronize(f.done_aux);
        if (e == hipSuccess) e = e2;
        ctx->ev_plain.push_back(f.done_aux);
    }
    // the first stream waited for the level-0 stream before recording done
    if (f.ev_plan) ctx->ev_plain.push_back(f.ev_plan);
    if (f.ev_l0) ctx->ev_plain.push_back(f.ev_l0);
    if (f.ev_up2) ctx->ev_plain.push_back(f.ev_up2);
    PinnedBuf& pb = ctx->pins[f.pin];
    pb.busy = false;
    if (e != hipSuccess) {
        for (auto& g : f.timed) { ctx->ev_timed.push_back(g.e0); ctx->ev_timed.push_back(g.e1); }
        return fail(ctx, MLMC_E_DEVICE, std::string("launch sequence failed: ") + hipGetErrorString(e));
    }
    const SlotDev* res = reinterpret_cast<const SlotDev*>(pb.p + f.down_off);
    std::vector<SlotDev> by_work;
    if (!f.order.empty()) {                 // results in stream order: back to work order
        by_work.resize(f.n_works);
        for (uint32_t p = 0; p < f.n_works; ++p) by_work[f.order[p]] = res[p];
        res = by_work.data();
    }
    if (out) out->assign(res, res + f.n_works);
    if (f.sink) f.sink->assign(res, res + f.n_works);
    for (size_t i = 0; i < f.deliver.size(); ++i) {
        const mlmc_level_work& w = f.deliver[i];
        const uint32_t mask = f.masks[i];
        const bool single = popcount32(mask) == 1;
        int j = 0;
        for (int p = 0; p < MLMC_NPAYOFF; ++p)
            if ((mask >> p) & 1u) slot_to_sums(res[i], single ? 0 : p, w.out[j++]);
    }
    for (auto& g : f.timed) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, g.e0, g.e1));
        add_stat(ctx, g.v, ms, g.steps);
        ctx->ev_timed.push_back(g.e0);
        ctx->ev_timed.push_back(g.e1);
    }
    return MLMC_OK;
}

// Lands every flight in order; their statuses wait in ctx->finished for
// mlmc_level_sums_wait.  Returns the first failure.
mlmc_status drain_flights(mlmc_context* ctx) {
    mlmc_status first = MLMC_OK;
    while (!ctx->flights.empty()) {
        Flight f = std::move(ctx->flights.front());
        ctx->flights.pop_front();
        const mlmc_status s = land_flight(ctx, f, nullptr);
        if (f.ticket) ctx->finished[f.ticket] = s;
        if (s != MLMC_OK && first == MLMC_OK) first = s;
    }
    return first;
}

// Plans the works (levels, tables, tiles), places the plan in the workspace behind
// the flights still in progress (landing the oldest when there is no room), uploads
// it and launches the sequence.  Caller holds dev_mtx.
mlmc_status launch_flight(mlmc_context* ctx, const std::vector<WorkSpec>& works, Flight& f) {
    if (ctx->poisoned) return fail(ctx, MLMC_E_DEVICE, "context poisoned by an earlier device error");
    if (ctx->ws_held) return fail(ctx, MLMC_E_BUSY, "a running server's sweep engine holds the workspace");
    HIPCHK(hipSetDevice(ctx->device));

    // 1. levels, tables, works
    std::vector<LevelDev> levels;
    std::vector<Variant> lvl_var;
    std::vector<uint8_t> tables;
    std::map<std::string, uint32_t> lvl_index;
    std::unordered_map<const LevelPrep*, uint32_t> lvl_of_prep;
    std::vector<WorkDev> wdev(works.size());
    if (ctx->prep_cache.size() > 4096) ctx->prep_cache.clear();
    auto add_level = [&](const LevelPrep& lp) {
        LevelDev L = lp.dev;
        if (!lp.table.empty()) {
            L.table_off = static_cast<uint32_t>(tables.size());
            tables.insert(tables.end(), lp.table.begin(), lp.table.end());
        }
        levels.push_back(L);
        lvl_var.push_back(lp.variant);
        return static_cast<uint32_t>(levels.size() - 1);
    };
    for (size_t i = 0; i < works.size(); ++i) {
        const WorkSpec& w = works[i];
        uint32_t li;
        if (w.prep) {                       // prepared by the caller (an option's own level)
            auto it = lvl_of_prep.find(w.prep);
            if (it == lvl_of_prep.end()) {
                li = add_level(*w.prep);
                lvl_of_prep.emplace(w.prep, li);
            } else {
                li = it->second;
            }
        } else {
            const std::string key = prep_key(w.prob, w.level, w.prec, w.est);
            auto it = lvl_index.find(key);
            if (it == lvl_index.end()) {
                auto pc = ctx->prep_cache.find(key);
                if (pc == ctx->prep_cache.end()) {
                    LevelPrep lp;
                    std::string err;
                    const mlmc_status s = prepare_level(w.prob, w.level, w.prec, w.est, lp, err);
                    if (s != MLMC_OK) return fail(ctx, s, err);
                    pc = ctx->prep_cache.emplace(key, std::move(lp)).first;
                }
                li = add_level(pc->second);
                lvl_index.emplace(key, li);
            } else {
                li = it->second;
            }
        }
        WorkDev& d = wdev[i];
        std::memset(&d, 0, sizeof(d));
        d.lvl = li;
        d.c2 = stream_c2(w.level, w.est);
        d.c3 = w.option;
        d.k0 = static_cast<uint32_t>(w.seed);
        d.k1 = static_cast<uint32_t>(w.seed >> 32);
        d.path_begin = w.path_begin;
        d.path_end = w.path_begin + w.n;
        d.debug = w.debug;
    }

    // 2. variants -> tiles (a work's tiles are contiguous; slot = tile index)
    std::map<VKey, LaunchGroup> groups;
    for (size_t i = 0; i < works.size(); ++i) {
        Variant v = lvl_var[wdev[i].lvl];
        v.l0 = level0_kernel_for(v, works[i].level, works[i].debug != 0, levels[wdev[i].lvl]);
        auto& g = groups[vkey(v)];
        g.v = v;
        g.works.push_back(static_cast<uint32_t>(i));
    }
    // longest chains first: a work's tiles start in the order of the tile list, so
    // the fine levels (2^level sequential steps per path, few paths) go first and
    // overlap the short, wide ones instead of forming the launch's tail
    for (auto& kv : groups)
        std::stable_sort(kv.second.works.begin(), kv.second.works.end(),
                         [&](uint32_t a, uint32_t b) { return works[a].level > works[b].level; });
    std::vector<WorkTilesDev> wtiles;
    uint32_t n_slots = 0;
    std::vector<ReduceDev> reds(works.size());
    // works with few, long paths get their exact normals computed ahead (k_normals)
    std::vector<TileDev> ntiles[2];                 // [0]: FP64 normals, [1]: FP32
    std::vector<size_t> zb_bytes(works.size(), 0);
    std::vector<int> zb_f32(works.size(), -1);
    for (auto& kv : groups) {
        LaunchGroup& g = kv.second;
        g.vi = variant_info(g.v);
        if (!g.vi.fn) return fail(ctx, MLMC_E_INVALID, "no compiled kernel for this estimator/arithmetic/packing");
        g.block = block_for(ctx->tune, g.v, g.vi);
        g.w0 = static_cast<uint32_t>(wtiles.size());
        for (uint32_t wi : g.works) {
            const WorkSpec& w = works[wi];
            const uint64_t N = uint64_t(1) << w.level;
            // (and only while the buffer takes at most a quarter of the workspace, so a
            // small workspace still runs every work)
            const bool zb = w.est != MLMC_EST_APPROX && w.level >= 2 && w.n <= ctx->tune.zb_max_paths &&
                            (w.n << w.level) <= ctx->tune.zb_max_positions &&
                            (w.n << w.level) * 12 <= ctx->ws_bytes / 4;
            if (zb) {
                const bool f32 = (w.est == MLMC_EST_PLAIN && w.prec->arith == MLMC_ARITH_FP32) ||
                                 lvl_var[wdev[wi].lvl].exact32;
                zb_f32[wi] = f32 ? 1 : 0;
                const uint64_t pos = w.n << w.level;
                zb_bytes[wi] = align_up(pos * 4, 256) + align_up(pos * (f32 ? 4 : 8), 256);
                // the work's Philox blocks in column order, x = (step / 4) P + path
                // offset (the normals kernel's index), one per thread of a 256-thread
                // normals block: enough workgroups to hide the inverse normal's
                // dependent FP64 chains, and each store a contiguous row segment
                const uint64_t x1 = pos / 4;
                for (uint64_t x = 0; x < x1; x += NORMALS_TILE_BLOCKS) {
                    TileDev t;
                    t.work = wi;
                    t.slot = 0;
                    t.group_begin = x;
                    t.n_groups = static_cast<uint32_t>(std::min<uint64_t>(NORMALS_TILE_BLOCKS, x1 - x));
                    t.pad = 0;
                    ntiles[f32 ? 1 : 0].push_back(t);
                }
            }
            // a buffered work's group is one path
            const uint64_t S = zb ? N : group_span(w.level, static_cast<uint32_t>(g.vi.wpb));
            const WorkSplit sp = split_work(ctx->tune, g.block, S, w.level, w.path_begin, w.n, FLIGHT_MAX_TILES);
            const uint64_t nt = sp.nt;
            if (uint64_t(n_slots) + nt >= (uint64_t(1) << 31)) return fail(ctx, MLMC_E_NOMEM, "too many tiles");
            WorkTilesDev wt;
            wt.g0 = sp.g0;
            wt.g1 = sp.g1;
            wt.per = sp.per;
            wt.work = wi;
            wt.tile_end = g.n_tiles + static_cast<uint32_t>(nt);
            wt.slot_begin = n_slots;
            wt.pad = 0;
            wtiles.push_back(wt);
            reds[wi].slot_begin = n_slots;
            n_slots += static_cast<uint32_t>(nt);
            g.n_tiles += static_cast<uint32_t>(nt);
            reds[wi].slot_end = n_slots;
            reds[wi].kind = (g.v.est == MLMC_EST_CORR ? 1u : 0u) |
                            (g.v.est == MLMC_EST_APPROX && g.v.arith == MLMC_ARITH_FIXED ? 2u : 0u) |
                            (g.v.np == NPAY ? 4u : 0u);
            reds[wi].work = wi;
            // table, plus the level-0 index histogram of the approximate estimator or
            // (FP32, small enough) its per-index sample table, or the correction
            // estimator's per-index approximate-side samples (float table side)
            g.lds = std::max<uint32_t>(g.lds, lds_bytes_for(g.v, levels[wdev[wi].lvl]));
        }
        g.w1 = static_cast<uint32_t>(wtiles.size());
    }

    // large flights with both table-only and exact-normal works run the table-only
    // kernels (and their works' reduction) on the second stream: order the reductions
    // [table-only works | the others]
    uint64_t flight_steps = 0;
    for (const WorkSpec& w : works) flight_steps += w.n << w.level;
    const bool overlap = flight_steps >= ctx->tune.overlap_min_steps;
    bool has_table = false, has_exact = false;
    for (auto& kv : groups) {
        if (!kv.second.n_tiles) continue;
        (kv.second.v.est == MLMC_EST_APPROX ? has_table : has_exact) = true;
    }
    const bool fork = overlap && has_table && has_exact && ctx->aux_stream;
    // results are written in this order (position p holds work order[p]), so that
    // each stream's reduction writes one contiguous part
    uint32_t n_red_aux = 0;
    f.order.clear();
    if (fork) {
        std::vector<ReduceDev> ordered;
        ordered.reserve(reds.size());
        for (int pass = 0; pass < 2; ++pass)
            for (size_t wi = 0; wi < works.size(); ++wi) {
                const bool tab_only = lvl_var[wdev[wi].lvl].est == MLMC_EST_APPROX;
                if (tab_only != (pass == 0)) continue;
                f.order.push_back(static_cast<uint32_t>(wi));
                ordered.push_back(reds[wi]);
                ordered.back().work = static_cast<uint32_t>(ordered.size() - 1);
                n_red_aux += tab_only ? 1u : 0u;
            }
        reds.swap(ordered);
    }

    // 3. layout (offsets from the flight's base):
    //    [levels | works | tables | work tiles | reds | normal tiles | slots | normals]
    //    (the results go straight to the pinned staging buffer)
    const size_t o_lvl = 0;
    const size_t o_work = align_up(o_lvl + levels.size() * sizeof(LevelDev), 256);
    const size_t o_tab = align_up(o_work + wdev.size() * sizeof(WorkDev), 256);
    const size_t o_tile = align_up(o_tab + tables.size(), 256);
    const size_t o_red = align_up(o_tile + wtiles.size() * sizeof(WorkTilesDev), 256);
    const size_t o_nt0 = align_up(o_red + reds.size() * sizeof(ReduceDev), 256);
    const size_t o_nt1 = align_up(o_nt0 + ntiles[0].size() * sizeof(TileDev), 256);
    // per launch group: (work descriptors, tiles), read by its path kernel
    std::vector<uint32_t> counts;
    for (auto& kv : groups) {
        kv.second.cnt = static_cast<uint32_t>(counts.size());
        counts.push_back(kv.second.w1 - kv.second.w0);
        counts.push_back(kv.second.n_tiles);
        counts.push_back(0);                        // the kernel gets its own descriptors' address
        counts.push_back(0);
    }
    const size_t o_cnt = align_up(o_nt1 + ntiles[1].size() * sizeof(TileDev), 256);
    const size_t o_end_plan = align_up(o_cnt + counts.size() * sizeof(uint32_t), 256);
    // the second stream reads its own copy of the plan (uploaded on the third stream,
    // so that neither of the first two streams waits for the other)
    const size_t o_copy = o_end_plan;
    const size_t o_slot = fork ? align_up(o_copy + (o_end_plan - o_lvl), 256) : o_end_plan;
    size_t o_zb = align_up(o_slot + size_t(n_slots) * sizeof(TileSlot), 256);
    std::vector<size_t> zb_off(works.size(), 0);
    for (size_t i = 0; i < works.size(); ++i) {
        if (zb_f32[i] < 0) continue;
        zb_off[i] = o_zb;
        o_zb += zb_bytes[i];
    }
    const size_t total = align_up(o_zb, 256);
    if (total > ctx->ws_bytes)
        return fail(ctx, MLMC_E_NOMEM, "workspace too small: need " + std::to_string(total) + " bytes");

    // 4. place it: a ring over the workspace in flight order
    if (ctx->flights.size() >= MAX_FLIGHTS) {
        const mlmc_status s = drain_oldest(ctx);
        if (s != MLMC_OK && ctx->poisoned) return s;
    }
    size_t base = 0;
    for (;;) {
        if (ctx->flights.empty()) { base = 0; break; }
        const size_t head = ctx->flights.front().base;
        const size_t tail = align_up(ctx->flights.back().end, 256);
        const bool wrapped = ctx->flights.back().base < head;
        if (!wrapped) {
            if (tail + total <= ctx->ws_bytes) { base = tail; break; }
            if (total <= head) { base = 0; break; }
        } else if (tail + total <= head) {
            base = tail;
            break;
        }
        const mlmc_status s = drain_oldest(ctx);
        if (s != MLMC_OK && ctx->poisoned) return s;
    }
    uint8_t* d = ctx->ws + base;
    for (size_t i = 0; i < works.size(); ++i) {
        if (zb_f32[i] < 0) continue;
        const uint64_t pos = works[i].n << works[i].level;
        wdev[i].jbuf = reinterpret_cast<uint64_t>(d + zb_off[i]);
        wdev[i].zbuf = reinterpret_cast<uint64_t>(d + zb_off[i] + align_up(pos * 4, 256));
    }

    // 5. stage and upload [levels .. normal tiles], launch; the reduction writes the
    //    results into the staging buffer behind the plan
    const size_t up_bytes = o_end_plan - o_lvl;
    const size_t down_bytes = works.size() * sizeof(SlotDev);
    f.down_off = align_up(up_bytes, 256);
    mlmc_status st = take_pinned(ctx, f.down_off + down_bytes, f.pin);
    if (st != MLMC_OK) return st;
    bool launched = false;
    auto release = [&]() {
        if (!launched) ctx->pins[f.pin].busy = false;
    };
    uint8_t* h = ctx->pins[f.pin].p;
    std::memset(h, 0, up_bytes);
    std::memcpy(h + (o_lvl - o_lvl), levels.data(), levels.size() * sizeof(LevelDev));
    std::memcpy(h + (o_work - o_lvl), wdev.data(), wdev.size() * sizeof(WorkDev));
    if (!tables.empty()) std::memcpy(h + (o_tab - o_lvl), tables.data(), tables.size());
    std::memcpy(h + (o_tile - o_lvl), wtiles.data(), wtiles.size() * sizeof(WorkTilesDev));
    std::memcpy(h + (o_red - o_lvl), reds.data(), reds.size() * sizeof(ReduceDev));
    if (!ntiles[0].empty()) std::memcpy(h + (o_nt0 - o_lvl), ntiles[0].data(), ntiles[0].size() * sizeof(TileDev));
    if (!ntiles[1].empty()) std::memcpy(h + (o_nt1 - o_lvl), ntiles[1].data(), ntiles[1].size() * sizeof(TileDev));
    if (!counts.empty()) std::memcpy(h + (o_cnt - o_lvl), counts.data(), counts.size() * sizeof(uint32_t));
    hipStream_t s = ctx->stream;
    hipStream_t sa = fork ? ctx->aux_stream : s;
    // The second stream's plan copy is uploaded on the third stream, so that it does
    // not queue behind the previous flight's approximate kernel and reduction.
    hipStream_t s_up2 = ctx->l0_stream ? ctx->l0_stream : sa;
    hipError_t ue = launch_upload(h, d + o_lvl, up_bytes, s);
    if (ue == hipSuccess && fork) ue = launch_upload(h, d + o_copy, up_bytes, s_up2);
    if (ue != hipSuccess) {
        release();
        return fail(ctx, MLMC_E_DEVICE, std::string("upload: ") + hipGetErrorString(ue));
    }
    launched = true;                      // from here the staging buffer belongs to the flight
    f.base = base;
    f.end = base + total;
    f.n_works = static_cast<uint32_t>(works.size());
    if ((st = take_event(ctx, false, f.done)) != MLMC_OK) return st;
    if (fork && (st = take_event(ctx, false, f.done_aux)) != MLMC_OK) return st;
    if (fork && s_up2 != sa) {
        if ((st = take_event(ctx, false, f.ev_up2)) != MLMC_OK) return st;
        HIPCHK(hipEventRecord(f.ev_up2, s_up2));
        HIPCHK(hipStreamWaitEvent(sa, f.ev_up2, 0));
    }
    // In a two-stream flight the level-0 exact-normal kernels run on a third stream,
    // beside the other exact levels' long serial paths (which leave most of the
    // machine idle); they read the first stream's plan once its upload is done.
    bool split_l0 = false;
    if (fork && ctx->l0_stream)
        for (auto& kv : groups)
            if (kv.second.n_tiles && kv.second.v.l0 && kv.second.v.est != MLMC_EST_APPROX) split_l0 = true;
    if (split_l0) {
        if ((st = take_event(ctx, false, f.ev_plan)) != MLMC_OK) return st;
        if ((st = take_event(ctx, false, f.ev_l0)) != MLMC_OK) return st;
        HIPCHK(hipEventRecord(f.ev_plan, s));
        HIPCHK(hipStreamWaitEvent(ctx->l0_stream, f.ev_plan, 0));
    }
    // the second stream's copy of the plan
    uint8_t* da = fork ? d + (o_copy - o_lvl) : d;
    // exact normals ahead of the path kernels for the buffered works
    const uint32_t ngrid = static_cast<uint32_t>(std::max(1, ctx->cu_count)) * 4;
    for (int k = 0; k < 2; ++k) {
        const uint32_t nn = static_cast<uint32_t>(ntiles[k].size());
        if (!nn) continue;
        HIPCHK(launch_normals(k == 1, std::min(nn, ngrid), s,
                              reinterpret_cast<const TileDev*>(d + (k ? o_nt1 : o_nt0)), nn,
                              reinterpret_cast<const WorkDev*>(d + o_work),
                              reinterpret_cast<const LevelDev*>(d + o_lvl), d + o_tab));
    }
    // path kernels, one per variant, then the fixed-order reduction of each work.
    // Table-only (approximate) groups do not wait for the normals-ahead kernel: when a
    // large flight has both kinds they run on the context's second stream, reading
    // that stream's copy of the plan, concurrently with the exact-normal groups.
    const uint32_t max_grid = static_cast<uint32_t>(std::max(1, ctx->cu_count)) * ctx->tune.blocks_per_cu;
    for (auto& kv : groups) {
        LaunchGroup& g = kv.second;
        const uint32_t nt = g.n_tiles;
        if (!nt) continue;
        const bool on_aux = fork && g.v.est == MLMC_EST_APPROX;
        const bool on_l0 = split_l0 && g.v.l0 && g.v.est != MLMC_EST_APPROX;
        hipStream_t gs = on_aux ? sa : (on_l0 ? ctx->l0_stream : s);
        uint8_t* dp = on_aux ? da : d;           // plan copy of that stream
        const uint32_t grid = std::min(nt, max_grid);
        Flight::Timed tm{};
        if (ctx->timing) {
            tm.v = g.v;
            for (uint32_t wi : g.works) tm.steps += works[wi].n << works[wi].level;
            if ((st = take_event(ctx, true, tm.e0)) != MLMC_OK) return st;
            if ((st = take_event(ctx, true, tm.e1)) != MLMC_OK) return st;
            f.timed.push_back(tm);
            HIPCHK(hipEventRecord(tm.e0, gs));
        }
        HIPCHK(launch_paths(g.vi, grid, g.block, g.lds, gs,
                            reinterpret_cast<const WorkTilesDev*>(dp + o_tile) + g.w0,
                            reinterpret_cast<const uint32_t*>(dp + o_cnt) + g.cnt,
                            reinterpret_cast<const WorkDev*>(dp + o_work),
                            reinterpret_cast<const LevelDev*>(dp + o_lvl), dp + o_tab,
                            reinterpret_cast<TileSlot*>(d + o_slot)));
        if (ctx->timing) HIPCHK(hipEventRecord(tm.e1, gs));
    }
    // the reduction writes each work's sums into the pinned staging buffer (coherent
    // host memory): they are on the host when the kernel completes
    const TileSlot* sl_dev = reinterpret_cast<const TileSlot*>(d + o_slot);
    SlotDev* res_host = reinterpret_cast<SlotDev*>(h + f.down_off);
    if (split_l0) {
        HIPCHK(hipEventRecord(f.ev_l0, ctx->l0_stream));
        HIPCHK(hipStreamWaitEvent(s, f.ev_l0, 0));
    }
    if (fork) {
        // each stream reduces its own works (positions [0, n_red_aux) on the second
        // stream) and records its own completion event
        HIPCHK(launch_reduce(n_red_aux, sa, sl_dev, reinterpret_cast<const ReduceDev*>(da + o_red), res_host));
        HIPCHK(hipEventRecord(f.done_aux, sa));
        HIPCHK(launch_reduce(static_cast<uint32_t>(works.size()) - n_red_aux, s, sl_dev,
                             reinterpret_cast<const ReduceDev*>(d + o_red) + n_red_aux, res_host));
    } else {
        HIPCHK(launch_reduce(static_cast<uint32_t>(works.size()), s, sl_dev,
                             reinterpret_cast<const ReduceDev*>(d + o_red), res_host));
    }
    HIPCHK(hipEventRecord(f.done, s));
    return MLMC_OK;
}

mlmc_status drain_oldest(mlmc_context* ctx) {
    if (ctx->flights.empty()) return MLMC_OK;
    Flight f = std::move(ctx->flights.front());
    ctx->flights.pop_front();
    const mlmc_status s = land_flight(ctx, f, nullptr);
    if (f.ticket) ctx->finished[f.ticket] = s;
    return s;
}

mlmc_status run_works(mlmc_context* ctx, const std::vector<WorkSpec>& works, std::vector<SlotDev>& out) {
    if (ctx->poisoned) return fail(ctx, MLMC_E_DEVICE, "context poisoned by an earlier device error");
    out.clear();
    if (works.empty()) return MLMC_OK;
    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    Flight f;
    mlmc_status s = launch_flight(ctx, works, f);
    if (s != MLMC_OK) return s;
    s = land_flight(ctx, f, &out);
    return s;
}

// ------------------------------------------------------------- adaptive MLMC
// The decisions (pilot, per-level estimator, allocation, bias test) are
// run_advance's (device/advance.hpp), on the option's plain-data RunState.

double option_eps(const mlmc_problem& prob, const mlmc_run_config& cfg) {
    const double scale = std::exp(-prob.r * prob.T) * (cfg.eps_units == 1 ? prob.S0 : 1.0);
    return cfg.eps / scale;
}

void run_state_init(RunState& st, const mlmc_problem& prob, const mlmc_run_config& cfg) {
    const double cost[3] = {cfg.cost_plain, cfg.cost_approx, cfg.cost_corr};
    run_init(st, option_eps(prob, cfg), cfg.theta, cost, cfg.n_pilot, cfg.nested ? 1 : 0, cfg.L_min, cfg.L_max);
}

EstSums est_of_slot(const SlotDev& s) {
    EstSums e;
    e.n = s.n;
    e.s1 = s.s1[0];
    e.s2 = s.s2[0];
    e.e1 = s.e1[0];
    e.e2 = s.e2[0];
    e.i1 = s.i1[0];
    e.i2lo = s.i2lo[0];
    e.i2hi = s.i2hi[0];
    e.sat = s.sat;
    e.nonfinite = s.nonfinite;
    return e;
}

void option_init(OptionRun& o) {
    run_state_init(o.st, o.prob, o.cfg);
    o.saturations = 0;
    o.t_start = now_seconds();
    o.t_end = 0.0;
}

std::vector<Pending> option_advance(OptionRun& o) {
    std::vector<Pending> pend;
    if (o.st.done) return pend;
    run_advance(o.st);
    for (int i = 0; i < o.st.n_pend; ++i) pend.push_back({o.st.pend[i].level, o.st.pend[i].est, o.st.pend[i].n});
    if (o.st.done) o.t_end = now_seconds();
    return pend;
}

void result_of_state(const RunState& st, const mlmc_problem& prob, const mlmc_run_config& cfg, double seconds,
                     mlmc_result& r) {
    std::memset(&r, 0, sizeof(r));
    r.struct_size = sizeof(mlmc_result);
    r.status = st.done ? MLMC_OK : MLMC_PENDING;
    r.L = st.L;
    r.sweeps = st.sweeps;
    const double sc = std::exp(-prob.r * prob.T) * prob.S0;       // R4, R5a
    double est = 0.0, var = 0.0;
    uint64_t sat = 0;
    for (int l = 0; l < MLMC_MAX_LEVELS; ++l)
        for (int e = 0; e < 3; ++e) sat += st.sums[l][e].sat;
    for (int l = 0; l <= st.L; ++l)
        for (int e = 0; e < 3; ++e) {
            const EstSums& s = st.sums[l][e];
            r.level[l].n[e] = s.n;
            r.level[l].mean[e] = est_mean(s);
            r.level[l].var[e] = est_var(s);
            if (s.n) {
                est += est_mean(s);
                var += est_var(s) / static_cast<double>(s.n);
                if (e == MLMC_EST_CORR) r.exact_sides |= cfg.prec[l].exact_side == 1 ? 2 : 1;
                if (e == MLMC_EST_PLAIN) r.exact_sides |= 4;
            }
        }
    r.estimate = sc * est;
    r.variance = sc * sc * var;
    r.seconds = seconds;
    r.path_steps = st.path_steps;
    r.saturations = sat;
}

void option_result(const OptionRun& o, mlmc_result& r) {
    result_of_state(o.st, o.prob, o.cfg, o.t_end - o.t_start, r);
}

static mlmc_precision plain_precision(const OptionRun& o) {
    mlmc_precision p;
    std::memset(&p, 0, sizeof(p));
    p.struct_size = sizeof(p);
    p.arith = o.cfg.plain_arith;
    p.table_bits = 8;
    return p;
}

void slot_accumulate(SlotDev& a, const SlotDev& b) {
    for (int p = 0; p < NPAY; ++p) {
        a.s1[p] += b.s1[p];
        a.s2[p] += b.s2[p];
        a.e1[p] += b.e1[p];
        a.e2[p] += b.e2[p];
        a.i1[p] += b.i1[p];
        const uint64_t lo = a.i2lo[p] + b.i2lo[p];
        a.i2hi[p] += b.i2hi[p] + (lo < a.i2lo[p] ? 1u : 0u);
        a.i2lo[p] = lo;
    }
    a.n += b.n;
    a.sat += b.sat;
    a.nonfinite += b.nonfinite;
}

// run_works, split in halves while the workspace cannot hold the plan (a work's
// sums do not depend on the other works of its launch)
static mlmc_status run_works_split(mlmc_context* ctx, const std::vector<WorkSpec>& works,
                                   std::vector<SlotDev>& out) {
    mlmc_status s = run_works(ctx, works, out);
    if (s != MLMC_E_NOMEM || works.size() < 2) return s;
    const size_t h = works.size() / 2;
    std::vector<SlotDev> a, b;
    s = run_works_split(ctx, std::vector<WorkSpec>(works.begin(), works.begin() + h), a);
    if (s != MLMC_OK) return s;
    s = run_works_split(ctx, std::vector<WorkSpec>(works.begin() + h, works.end()), b);
    if (s != MLMC_OK) return s;
    out = std::move(a);
    out.insert(out.end(), b.begin(), b.end());
    return MLMC_OK;
}

mlmc_status option_prep(OptionRun& o, int level, int est, const mlmc_precision* prec,
                        const LevelPrep*& out, std::string& err) {
    if (o.preps.size() <= static_cast<size_t>(level)) o.preps.resize(static_cast<size_t>(level) + 1);
    std::shared_ptr<const LevelPrep>& slot = o.preps[level][est];
    if (!slot) {
        auto lp = std::make_shared<LevelPrep>();
        const mlmc_status s = prepare_level(&o.prob, level, prec, est, *lp, err);
        if (s != MLMC_OK) return s;
        slot = std::move(lp);
    }
    out = slot.get();
    return MLMC_OK;
}

mlmc_status sweep_once(mlmc_context* ctx, const std::vector<OptionRun*>& opts, bool& ran) {
    ran = false;
    std::vector<mlmc_precision> plain(opts.size());
    std::vector<WorkSpec> works;
    std::vector<std::pair<size_t, Pending>> who;
    for (size_t i = 0; i < opts.size(); ++i) {
        OptionRun& o = *opts[i];
        if (o.st.done) continue;
        plain[i] = plain_precision(o);
        for (const Pending& p : option_advance(o)) {
            WorkSpec w;
            w.prob = &o.prob;
            w.level = p.level;
            w.prec = p.est == MLMC_EST_PLAIN ? &plain[i] : &o.cfg.prec[p.level];
            w.est = p.est;
            w.seed = o.seed;
            w.option = o.option;
            w.path_begin = o.st.sums[p.level][p.est].n;
            w.n = p.n;
            w.debug = 0;
            std::string err;
            const mlmc_status ps = option_prep(o, p.level, p.est, w.prec, w.prep, err);
            if (ps != MLMC_OK) return fail(ctx, ps, err);
            works.push_back(w);
            who.emplace_back(i, p);
        }
    }
    if (works.empty()) return MLMC_OK;
    ran = true;
    std::vector<SlotDev> res;
    const mlmc_status s = run_works_split(ctx, works, res);
    if (s != MLMC_OK) return s;
    std::vector<bool> counted(opts.size(), false);
    for (size_t k = 0; k < works.size(); ++k) {
        OptionRun& o = *opts[who[k].first];
        const Pending& p = who[k].second;
        est_accumulate(o.st.sums[p.level][p.est], est_of_slot(res[k]));
        o.st.path_steps += p.n << p.level;
        if (!counted[who[k].first]) { o.st.sweeps += 1; counted[who[k].first] = true; }
    }
    return MLMC_OK;
}

mlmc_status run_sweeps(mlmc_context* ctx, std::vector<OptionRun*>& opts) {
    for (;;) {
        bool ran = false;
        const mlmc_status s = sweep_once(ctx, opts, ran);
        if (s != MLMC_OK || !ran) return s;
    }
}

mlmc_status validate_run(const mlmc_problem* prob, const mlmc_run_config* cfg, std::string& err) {
    mlmc_status s = validate_problem(prob, err);
    if (s != MLMC_OK) return s;
    if (popcount32(prob->payoff_mask) != 1) { err = "an estimate prices exactly one payoff"; return MLMC_E_INVALID; }
    if (!cfg) { err = "run config is NULL"; return MLMC_E_INVALID; }
    if (cfg->struct_size != sizeof(mlmc_run_config)) { err = "mlmc_run_config.struct_size mismatch"; return MLMC_E_VERSION; }
    if (!(cfg->eps > 0.0) || !std::isfinite(cfg->eps)) { err = "eps must be > 0"; return MLMC_E_INVALID; }
    if (!(cfg->theta > 0.0 && cfg->theta <= 1.0)) { err = "theta must be in (0, 1]"; return MLMC_E_INVALID; }
    if (cfg->L_min < 0 || cfg->L_max < cfg->L_min || cfg->L_max >= MLMC_MAX_LEVELS) { err = "need 0 <= L_min <= L_max <= 20"; return MLMC_E_INVALID; }
    if (cfg->n_pilot < 2) { err = "n_pilot must be >= 2"; return MLMC_E_INVALID; }
    if (!(cfg->cost_plain > 0 && cfg->cost_approx > 0 && cfg->cost_corr > 0)) { err = "costs must be > 0"; return MLMC_E_INVALID; }
    if (cfg->eps_units != 0 && cfg->eps_units != 1) { err = "eps_units must be 0 or 1"; return MLMC_E_INVALID; }
    if (cfg->nested) {
        for (int l = 0; l <= cfg->L_max; ++l) {
            if ((s = validate_precision(&cfg->prec[l], MLMC_EST_APPROX, prob, err)) != MLMC_OK) return s;
            mlmc_precision c = cfg->prec[l];
            c.packed = 0;
            if ((s = validate_precision(&c, MLMC_EST_CORR, prob, err)) != MLMC_OK) return s;
        }
    }
    // plain samples: plain runs, and nested levels switched to plain
    if (cfg->plain_arith != MLMC_ARITH_FP64 && cfg->plain_arith != MLMC_ARITH_FP32) {
        err = "plain_arith must be FP64 or FP32";
        return MLMC_E_INVALID;
    }
    return MLMC_OK;
}

mlmc_status estimate_batch(mlmc_context* ctx, uint32_t n, const mlmc_problem* probs,
                           const mlmc_run_config* cfg, uint64_t seed, const uint32_t* ids,
                           mlmc_result* out) {
    if (!ctx) return MLMC_E_INVALID;
    if (ctx->poisoned) return fail(ctx, MLMC_E_DEVICE, "context poisoned by an earlier device error");
    if (!probs || !out || !ids || n == 0) return fail(ctx, MLMC_E_INVALID, "empty batch or NULL pointer");
    std::string err;
    for (uint32_t i = 0; i < n; ++i) {
        const mlmc_status s = validate_run(&probs[i], cfg, err);
        if (s != MLMC_OK) return fail(ctx, s, "option " + std::to_string(i) + ": " + err);
    }
    std::vector<OptionRun> runs(n);
    std::vector<OptionRun*> ptrs(n);
    const double t0 = now_seconds();
    for (uint32_t i = 0; i < n; ++i) {
        runs[i].prob = probs[i];
        runs[i].cfg = *cfg;
        runs[i].seed = seed;
        runs[i].option = ids[i];
        option_init(runs[i]);
        runs[i].t_start = t0;
        ptrs[i] = &runs[i];
    }
    if (ctx->ws_held) return fail(ctx, MLMC_E_BUSY, "a running server's sweep engine holds the workspace");
    mlmc_status s = MLMC_E_NOMEM;
    if (ctx->driver == MLMC_DRIVER_ENGINE || (ctx->driver == MLMC_DRIVER_AUTO && n >= MLMC_ENGINE_MIN_RUNS)) {
        // the device sweep engine owns the workspace while it runs
        std::lock_guard<std::mutex> lock(ctx->dev_mtx);
        s = drain_flights(ctx);
        if (s == MLMC_OK || !ctx->poisoned) s = engine_run_batch(ctx, runs);
    }
    if (s == MLMC_E_NOMEM) {
        // a workspace too small for the engine: sweeps planned on the host
        for (uint32_t i = 0; i < n; ++i) {
            option_init(runs[i]);
            runs[i].t_start = t0;
        }
        s = run_sweeps(ctx, ptrs);
    }
    if (s != MLMC_OK) return s;
    for (uint32_t i = 0; i < n; ++i) option_result(runs[i], out[i]);
    return MLMC_OK;
}


}  // namespace mlmc

using namespace mlmc;

// ====================================================================== ABI
extern "C" {

int32_t mlmc_abi_version(void) { return MLMC_ABI_VERSION; }

const char* mlmc_status_string(int32_t s) {
    switch (s) {
        case MLMC_OK: return "ok";
        case MLMC_PENDING: return "pending";
        case MLMC_E_INVALID: return "invalid argument";
        case MLMC_E_NOMEM: return "workspace too small";
        case MLMC_E_DEVICE: return "device error";
        case MLMC_E_OVERFLOW: return "fixed-point overflow";
        case MLMC_E_BUSY: return "server busy or not running";
        case MLMC_E_TIMEOUT: return "timeout";
        case MLMC_E_UNKNOWN_TICKET: return "unknown ticket";
        case MLMC_E_VERSION: return "struct_size mismatch";
        default: return "unknown status";
    }
}

const char* mlmc_last_error(const mlmc_context* ctx) { return ctx ? ctx->err.c_str() : mlmc::static_last_error(); }

mlmc_status mlmc_context_create(int32_t device, void* workspace, uint64_t workspace_bytes, void* stream,
                                mlmc_context** out) {
    if (!out) return MLMC_E_INVALID;
    *out = nullptr;
    if (workspace_bytes < (uint64_t(1) << 20)) return MLMC_E_INVALID;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return MLMC_E_DEVICE;
    if (device < 0 || device >= n) return MLMC_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return MLMC_E_DEVICE;
    auto* ctx = new mlmc_context();
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(stream);
    ctx->ws_bytes = workspace_bytes;
    if (hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking) != hipSuccess) {
        delete ctx;
        return MLMC_E_DEVICE;
    }
    if (hipStreamCreateWithFlags(&ctx->l0_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(ctx->aux_stream);
        delete ctx;
        return MLMC_E_DEVICE;
    }
    if (hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        (void)hipStreamDestroy(ctx->l0_stream);
        (void)hipStreamDestroy(ctx->aux_stream);
        delete ctx;
        return MLMC_E_DEVICE;
    }
    if (workspace) {
        ctx->ws = static_cast<uint8_t*>(workspace);
    } else {
        if (hipMalloc(reinterpret_cast<void**>(&ctx->ws), workspace_bytes) != hipSuccess) {
            (void)hipStreamDestroy(ctx->l0_stream);
            (void)hipStreamDestroy(ctx->aux_stream);
            delete ctx;
            return MLMC_E_NOMEM;
        }
        ctx->own_ws = true;
    }
    *out = ctx;
    return MLMC_OK;
}

void mlmc_context_destroy(mlmc_context* ctx) {
    if (!ctx) return;
    mlmc_server_stop(ctx);
    {
        std::lock_guard<std::mutex> lock(ctx->dev_mtx);
        (void)drain_flights(ctx);
        ctx->engines.clear();
    }
    if (ctx->aux_stream) (void)hipStreamSynchronize(ctx->aux_stream);
    if (ctx->l0_stream) (void)hipStreamSynchronize(ctx->l0_stream);
    for (hipEvent_t e : ctx->ev_plain) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ev_timed) (void)hipEventDestroy(e);
    if (ctx->aux_stream) (void)hipStreamDestroy(ctx->aux_stream);
    if (ctx->l0_stream) (void)hipStreamDestroy(ctx->l0_stream);
    for (auto& pb : ctx->pins)
        if (pb.p) (void)hipHostFree(pb.p);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    delete ctx;
}

mlmc_status mlmc_level_sums(mlmc_context* ctx, const mlmc_problem* prob, int32_t level, uint64_t n_paths,
                            uint64_t path_offset, const mlmc_precision* prec, int32_t estimator, uint64_t seed,
                            uint32_t option_id, mlmc_sums* out, void* debug_paths) {
    if (!ctx) return MLMC_E_INVALID;
    if (ctx->poisoned) return fail(ctx, MLMC_E_DEVICE, "context poisoned by an earlier device error");
    std::string err;
    mlmc_status s = validate_all(prob, level, n_paths, path_offset, prec, estimator, err);
    if (s != MLMC_OK) return fail(ctx, s, err);
    if (!out) return fail(ctx, MLMC_E_INVALID, "out is NULL");
    WorkSpec w;
    w.prob = prob;
    w.level = level;
    w.prec = prec;
    w.est = estimator;
    w.seed = seed;
    w.option = option_id;
    w.path_begin = path_offset;
    w.n = n_paths;
    w.debug = reinterpret_cast<uint64_t>(debug_paths);
    std::vector<SlotDev> res;
    s = run_works(ctx, {w}, res);
    if (s != MLMC_OK) return s;
    const bool single = popcount32(prob->payoff_mask) == 1;
    int i = 0;
    for (int p = 0; p < MLMC_NPAYOFF; ++p)
        if ((prob->payoff_mask >> p) & 1u) slot_to_sums(res[0], single ? 0 : p, out[i++]);
    return MLMC_OK;
}

static mlmc_status batch_specs(mlmc_context* ctx, uint32_t n, const mlmc_level_work* works,
                               std::vector<WorkSpec>& ws) {
    if (!works || n == 0) return fail(ctx, MLMC_E_INVALID, "empty work list");
    ws.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        const mlmc_level_work& w = works[i];
        if (w.struct_size != sizeof(mlmc_level_work)) return fail(ctx, MLMC_E_VERSION, "mlmc_level_work.struct_size mismatch");
        std::string err;
        const mlmc_status s = validate_all(w.prob, w.level, w.n_paths, w.path_offset, w.prec, w.estimator, err);
        if (s != MLMC_OK) return fail(ctx, s, "work " + std::to_string(i) + ": " + err);
        if (!w.out) return fail(ctx, MLMC_E_INVALID, "work " + std::to_string(i) + ": out is NULL");
        ws[i] = WorkSpec{w.prob, w.level, w.prec, w.estimator, w.seed, w.option_id, w.path_offset, w.n_paths, 0};
    }
    return MLMC_OK;
}

mlmc_status mlmc_level_sums_enqueue(mlmc_context* ctx, uint32_t n, const mlmc_level_work* works,
                                    uint64_t* ticket) {
    if (!ctx || !ticket) return MLMC_E_INVALID;
    *ticket = 0;
    if (ctx->poisoned) return fail(ctx, MLMC_E_DEVICE, "context poisoned by an earlier device error");
    std::vector<WorkSpec> ws;
    mlmc_status s = batch_specs(ctx, n, works, ws);
    if (s != MLMC_OK) return s;
    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    Flight f;
    s = launch_flight(ctx, ws, f);
    if (s != MLMC_OK) return s;
    f.ticket = ctx->next_ticket++;
    f.deliver.assign(works, works + n);
    f.masks.resize(n);
    for (uint32_t i = 0; i < n; ++i) f.masks[i] = works[i].prob->payoff_mask;
    *ticket = f.ticket;
    ctx->flights.push_back(std::move(f));
    return MLMC_OK;
}

mlmc_status mlmc_level_sums_wait(mlmc_context* ctx, uint64_t ticket) {
    if (!ctx) return MLMC_E_INVALID;
    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    for (;;) {
        auto it = ctx->finished.find(ticket);
        if (it != ctx->finished.end()) {
            const mlmc_status s = it->second;
            ctx->finished.erase(it);
            return s;
        }
        bool pending = false;
        for (const Flight& f : ctx->flights) pending = pending || f.ticket == ticket;
        if (!pending) return fail(ctx, MLMC_E_UNKNOWN_TICKET, "no such ticket");
        (void)drain_oldest(ctx);
    }
}

mlmc_status mlmc_level_sums_batch(mlmc_context* ctx, uint32_t n, const mlmc_level_work* works) {
    if (!ctx) return MLMC_E_INVALID;
    if (ctx->poisoned) return fail(ctx, MLMC_E_DEVICE, "context poisoned by an earlier device error");
    std::vector<WorkSpec> ws;
    mlmc_status s = batch_specs(ctx, n, works, ws);
    if (s != MLMC_OK) return s;
    std::vector<SlotDev> res;
    s = run_works(ctx, ws, res);
    if (s != MLMC_OK) return s;
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t mask = works[i].prob->payoff_mask;
        const bool single = popcount32(mask) == 1;
        int j = 0;
        for (int p = 0; p < MLMC_NPAYOFF; ++p)
            if ((mask >> p) & 1u) slot_to_sums(res[i], single ? 0 : p, works[i].out[j++]);
    }
    return MLMC_OK;
}

mlmc_status mlmc_get_tuning(const mlmc_context* ctx, mlmc_tuning* out) {
    if (!ctx || !out) return MLMC_E_INVALID;
    out->struct_size = sizeof(mlmc_tuning);
    out->block_table = ctx->tune.block_table;
    out->block_exact = ctx->tune.block_exact;
    out->tile_steps = ctx->tune.tile_steps;
    out->blocks_per_cu = ctx->tune.blocks_per_cu;
    out->min_tiles = ctx->tune.min_tiles;
    out->zb_max_paths = ctx->tune.zb_max_paths;
    out->zb_max_positions = ctx->tune.zb_max_positions;
    out->overlap_min_steps = ctx->tune.overlap_min_steps;
    return MLMC_OK;
}

mlmc_status mlmc_set_tuning(mlmc_context* ctx, const mlmc_tuning* t) {
    if (!ctx || !t) return MLMC_E_INVALID;
    if (t->struct_size != sizeof(mlmc_tuning)) return fail(ctx, MLMC_E_VERSION, "mlmc_tuning.struct_size mismatch");
    auto pow2ish = [](uint32_t b, uint32_t hi) { return b >= 64 && b <= hi && b % 64 == 0; };
    if (!pow2ish(t->block_table, 1024) || !pow2ish(t->block_exact, 256) || t->tile_steps < 1 ||
        t->blocks_per_cu < 1 || t->blocks_per_cu > 64 || t->min_tiles < 1)
        return fail(ctx, MLMC_E_INVALID, "tuning out of range");
    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    ctx->tune.block_table = t->block_table;
    ctx->tune.block_exact = t->block_exact;
    ctx->tune.tile_steps = t->tile_steps;
    ctx->tune.blocks_per_cu = t->blocks_per_cu;
    ctx->tune.min_tiles = t->min_tiles;
    ctx->tune.zb_max_paths = t->zb_max_paths;
    ctx->tune.zb_max_positions = t->zb_max_positions;
    ctx->tune.overlap_min_steps = t->overlap_min_steps;
    return MLMC_OK;
}

// Launch-geometry tuner: coordinate descent over the tuning fields, each candidate
// timed on the caller's own work list (host wall clock per launch sequence, planning,
// upload, kernels and reduction into pinned memory, with sequences pipelined).
mlmc_status mlmc_autotune(mlmc_context* ctx, uint32_t n, const mlmc_level_work* works, uint32_t reps,
                          mlmc_tuning* out) {
    if (!ctx || !out) return MLMC_E_INVALID;
    if (out->struct_size != sizeof(mlmc_tuning)) return fail(ctx, MLMC_E_VERSION, "mlmc_tuning.struct_size mismatch");
    if (reps < 1 || reps > 100) return fail(ctx, MLMC_E_INVALID, "reps must be 1..100");
    if (ctx->server) return fail(ctx, MLMC_E_BUSY, "stop the server before tuning");
    std::vector<WorkSpec> ws;
    mlmc_status s = batch_specs(ctx, n, works, ws);
    if (s != MLMC_OK) return s;
    {
        std::lock_guard<std::mutex> lock(ctx->dev_mtx);
        if ((s = drain_flights(ctx)) != MLMC_OK) return s;
    }
    std::vector<SlotDev> res;
    // steady-state time per launch sequence: `reps` sequences enqueued back to back
    // (as a pipelined caller or the server runs them), then all landed
    auto measure = [&](const Tuning& t, double& sec) -> mlmc_status {
        {
            std::lock_guard<std::mutex> lock(ctx->dev_mtx);
            ctx->tune = t;
        }
        mlmc_status st = run_works(ctx, ws, res);            // warm (tables, pinned buffers)
        if (st != MLMC_OK) return st;
        std::lock_guard<std::mutex> lock(ctx->dev_mtx);
        // the least of three timed rounds: host jitter only ever adds time
        sec = HUGE_VAL;
        for (int trial = 0; trial < 3; ++trial) {
            const double t0 = now_seconds();
            for (uint32_t r = 0; r < reps; ++r) {
                Flight f;
                if ((st = launch_flight(ctx, ws, f)) != MLMC_OK) {
                    drain_flights(ctx);
                    return st;
                }
                ctx->flights.push_back(std::move(f));
            }
            if ((st = drain_flights(ctx)) != MLMC_OK) return st;
            sec = std::min(sec, (now_seconds() - t0) / reps);
        }
        return MLMC_OK;
    };
    Tuning best = ctx->tune;
    double best_s = 0.0;
    auto try_field = [&](auto set, std::initializer_list<uint64_t> values) -> mlmc_status {
        for (uint64_t v : values) {
            Tuning t = best;
            set(t, v);
            double sec = 0.0;
            const mlmc_status st = measure(t, sec);
            if (st == MLMC_E_NOMEM) continue;                 // a geometry the workspace cannot hold
            if (st != MLMC_OK) return st;
            if (sec < 0.99 * best_s) {                       // at least 1% faster
                best_s = sec;
                best = t;
            }
        }
        return MLMC_OK;
    };
    // two passes of coordinate descent (the fields interact); the incumbent is timed
    // afresh at the start of each pass so that one lucky time does not hold
    const mlmc_status r = [&]() -> mlmc_status {
        for (int pass = 0; pass < 2; ++pass) {
            mlmc_status st;
            if ((st = measure(best, best_s)) != MLMC_OK) return st;
            if ((st = try_field([](Tuning& t, uint64_t v) { t.block_table = uint32_t(v); }, {256, 512, 1024})) != MLMC_OK) return st;
            if ((st = try_field([](Tuning& t, uint64_t v) { t.block_exact = uint32_t(v); }, {64, 128, 256})) != MLMC_OK) return st;
            if ((st = try_field([](Tuning& t, uint64_t v) { t.tile_steps = uint32_t(v); },
                                {1u << 14, 1u << 15, 1u << 16, 1u << 17, 1u << 18})) != MLMC_OK) return st;
            if ((st = try_field([](Tuning& t, uint64_t v) { t.blocks_per_cu = uint32_t(v); }, {2, 4, 8, 16})) != MLMC_OK) return st;
            if ((st = try_field([](Tuning& t, uint64_t v) { t.min_tiles = uint32_t(v); }, {512, 1024, 2048, 4096})) != MLMC_OK) return st;
            if ((st = try_field([](Tuning& t, uint64_t v) { t.zb_max_paths = v; }, {0, 1u << 13, 1u << 15, 1u << 17})) != MLMC_OK) return st;
            if ((st = try_field([](Tuning& t, uint64_t v) { t.overlap_min_steps = v; },
                                {0, uint64_t(1) << 24, uint64_t(1) << 26, uint64_t(1) << 28, UINT64_MAX})) != MLMC_OK)
                return st;
        }
        return MLMC_OK;
    }();
    {
        std::lock_guard<std::mutex> lock(ctx->dev_mtx);
        ctx->tune = best;
    }
    if (r != MLMC_OK) return r;
    return mlmc_get_tuning(ctx, out);
}

mlmc_status mlmc_set_driver(mlmc_context* ctx, int32_t driver) {
    if (!ctx) return MLMC_E_INVALID;
    if (driver != MLMC_DRIVER_HOST && driver != MLMC_DRIVER_ENGINE && driver != MLMC_DRIVER_AUTO)
        return fail(ctx, MLMC_E_INVALID, "driver must be 0 (host), 1 (device engine) or 2 (auto)");
    if (ctx->server) return fail(ctx, MLMC_E_BUSY, "a server is running");
    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    ctx->driver = driver;
    return MLMC_OK;
}

mlmc_status mlmc_set_timing(mlmc_context* ctx, int32_t on) {
    if (!ctx) return MLMC_E_INVALID;
    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    ctx->timing = on != 0;
    ctx->stats.clear();
    return MLMC_OK;
}

mlmc_status mlmc_kernel_stats(mlmc_context* ctx, mlmc_kernel_stat* out, uint32_t max, uint32_t* n) {
    if (!ctx || !n || (max && !out)) return MLMC_E_INVALID;
    std::lock_guard<std::mutex> lock(ctx->dev_mtx);
    *n = static_cast<uint32_t>(ctx->stats.size());
    for (uint32_t i = 0; i < max && i < ctx->stats.size(); ++i) out[i] = ctx->stats[i];
    return MLMC_OK;
}

mlmc_status mlmc_estimate(mlmc_context* ctx, const mlmc_problem* prob, const mlmc_run_config* cfg, uint64_t seed,
                          uint32_t option_id, mlmc_result* out) {
    return estimate_batch(ctx, 1, prob, cfg, seed, &option_id, out);
}

mlmc_status mlmc_estimate_batch(mlmc_context* ctx, uint32_t n, const mlmc_problem* probs,
                                const mlmc_run_config* cfg, uint64_t seed, mlmc_result* out) {
    std::vector<uint32_t> ids(n);
    for (uint32_t i = 0; i < n; ++i) ids[i] = i;
    return estimate_batch(ctx, n, probs, cfg, seed, ids.data(), out);
}

// ------------------------------------------------------------- host helpers
mlmc_status mlmc_build_table(int32_t q, int32_t arith, int32_t frac_bits, void* out) {
    std::string err;
    return build_table_bytes(q, arith, frac_bits, out, err);
}

mlmc_status mlmc_build_rng_table(int32_t q, int32_t method, double* values, uint16_t* perm,
                                 int32_t* iterations) {
    if (!values || (method != 2 && method != 3) || q < 2 || q > 12 || (method == 2 && q % 2)) return MLMC_E_INVALID;
    const MethodTable& t = method_table(q, method);
    std::memcpy(values, t.z.data(), t.z.size() * sizeof(double));
    if (perm && method == 2) std::memcpy(perm, t.perm.data(), t.perm.size() * sizeof(uint16_t));
    if (iterations) *iterations = t.iterations;
    return MLMC_OK;
}

mlmc_status mlmc_stream_words(uint64_t seed, uint32_t option_id, int32_t level, int32_t estimator,
                              uint64_t word_index, uint64_t count, uint32_t* out) {
    if (!out || level < 0 || level > 255 || estimator < 0 || estimator > 255) return MLMC_E_INVALID;
    for (uint64_t i = 0; i < count; ++i) {
        const uint64_t w = word_index + i;
        const uint64_t b = w >> 2;
        const u32x4 r = philox4x32_10(u32x4{static_cast<uint32_t>(b), static_cast<uint32_t>(b >> 32),
                                            stream_c2(level, estimator), option_id},
                                      static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
        const uint32_t words[4] = {r.x, r.y, r.z, r.w};
        out[i] = words[w & 3];
    }
    return MLMC_OK;
}

mlmc_status mlmc_validate(const mlmc_problem* prob, int32_t level, uint64_t n_paths, uint64_t path_offset,
                          const mlmc_precision* prec, int32_t estimator) {
    std::string err;
    return validate_all(prob, level, n_paths, path_offset, prec, estimator, err);
}

mlmc_status mlmc_allocate(uint32_t m, const double* V, const double* C, double eps2, double theta, uint64_t* out) {
    if (!V || !C || !out || m == 0 || !(eps2 > 0) || !(theta > 0 && theta <= 1)) return MLMC_E_INVALID;
    double lam = 0.0;
    for (uint32_t i = 0; i < m; ++i) {
        if (!(V[i] >= 0) || !(C[i] > 0)) return MLMC_E_INVALID;
        lam += std::sqrt(V[i] * C[i]);
    }
    lam /= theta * eps2;
    for (uint32_t i = 0; i < m; ++i) {
        const double t = std::ceil(lam * std::sqrt(V[i] / C[i]));
        out[i] = t > 1.8e19 ? UINT64_MAX : static_cast<uint64_t>(t);
    }
    return MLMC_OK;
}

}  // extern "C"
