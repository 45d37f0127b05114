// Host side of the device sweep engine (engine.hpp): the engine's arrays in the
// context's workspace, its launch classes, the levels of each run (prepared on the
// host when a run first needs them), the sweep captured as a HIP graph, and the
// replay loop of a batch of estimates.
#include "engine_host.hpp"

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <thread>
#include <tuple>

namespace mlmc {

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

using ClassKey = std::tuple<int, int, int, int, bool, int, bool, bool>;
ClassKey class_key(const Variant& v) {
    return ClassKey{v.est, v.arith, v.scheme, v.np, v.track, v.fields, v.l0, v.exact32};
}

mlmc_precision plain_prec_of(const mlmc_run_config& cfg) {
    mlmc_precision p;
    std::memset(&p, 0, sizeof(p));
    p.struct_size = sizeof(p);
    p.arith = cfg.plain_arith;
    p.table_bits = 8;
    return p;
}

}  // namespace

static_assert(offsetof(RunState, sums) % 8 == 0, "a run's state is uploaded as head words and zeros");
static_assert(sizeof(RunState) % 8 == 0 && sizeof(LevelDev) % 8 == 0 && sizeof(EngMeta) % 8 == 0 &&
                  sizeof(EngHeader) % 8 == 0 && sizeof(EngLevelInfo) == 8,
              "engine uploads move 8-byte words");

#define EHIP(call)                                                                       \
    do {                                                                                 \
        const hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, MLMC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Engine::~Engine() {
    if (st) (void)hipStreamSynchronize(st);
    for (auto& x : exec)
        if (x) (void)hipGraphExecDestroy(x);
    for (auto& h : status_h)
        if (h) (void)hipHostFree(h);
    for (auto& e : ev_done)
        if (e) (void)hipEventDestroy(e);
    for (auto& sb : stage) {
        if (sb.p) (void)hipHostFree(sb.p);
        if (sb.ev) (void)hipEventDestroy(sb.ev);
    }
    if (states_h) (void)hipHostFree(states_h);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (st) (void)hipStreamDestroy(st);
}

// Launch classes: every kernel variant a run of these (scheme, payoff kind, nested)
// combinations can need at levels 0..L_max, with the correction's and the plain
// estimator's level-0 kernels.
mlmc_status engine_classes(mlmc_context* ctx, const mlmc_run_config& cfg, const std::vector<EngKind>& kinds,
                           std::vector<EngClass>& out, size_t& tstride) {
    out.clear();
    tstride = 256;
    std::map<ClassKey, int> seen;
    const mlmc_precision plain = plain_prec_of(cfg);
    for (const EngKind& k : kinds) {
        mlmc_problem prob;
        std::memset(&prob, 0, sizeof(prob));
        prob.struct_size = sizeof(prob);
        prob.scheme = k.scheme;
        prob.payoff_mask = k.track ? (1u << MLMC_PAY_ASIAN) : (1u << MLMC_PAY_EURO);
        prob.S0 = prob.K = 1.0;
        prob.sigma = 0.2;
        prob.T = 1.0;
        for (int l = 0; l <= cfg.L_max; ++l)
            for (int e = 0; e < 3; ++e) {
                if (e != MLMC_EST_PLAIN && !k.nested) continue;
                const mlmc_precision* pr = e == MLMC_EST_PLAIN ? &plain : &cfg.prec[l];
                LevelPrep lp;
                std::string err;
                const mlmc_status s = prepare_level(&prob, l, pr, e, lp, err);
                if (s != MLMC_OK) return fail(ctx, s, err);
                Variant v = lp.variant;
                v.l0 = level0_kernel_for(v, l, false, lp.dev);
                tstride = std::max(tstride, al(lp.table.size()));
                const ClassKey key = class_key(v);
                auto it = seen.find(key);
                int ci;
                if (it == seen.end()) {
                    EngClass c;
                    c.v = v;
                    c.vi = variant_info(v);
                    if (!c.vi.fn) return fail(ctx, MLMC_E_INVALID, "no compiled kernel for a level of the run config");
                    c.block = block_for(ctx->tune, v, c.vi);
                    ci = static_cast<int>(out.size());
                    out.push_back(c);
                    seen.emplace(key, ci);
                } else {
                    ci = it->second;
                }
                out[ci].lds = std::max(out[ci].lds, lds_bytes_for(v, lp.dev));
            }
    }
    if (out.size() > ENG_MAX_CLASSES) return fail(ctx, MLMC_E_INVALID, "too many kernel classes for the engine");
    return MLMC_OK;
}

size_t Engine::slot_bytes(uint32_t LV, size_t tstride) {
    const size_t mw = RUN_MAX_PEND;
    return sizeof(RunState) + sizeof(EngMeta) + size_t(LV) * 3 * sizeof(EngLevelInfo) + sizeof(EngPlanScratch) +
           24 * 1024 +
           mw * (sizeof(WorkDev) + sizeof(WorkTilesDev) + sizeof(EngReduce)) + 4 +
           size_t(LV) * 3 * sizeof(LevelDev) + size_t(LV) * 2 * tstride + size_t(LV) * sizeof(EngTableJob);
}

// The Z~ column of every FP32 / FP16 table side the run config's levels use, taken
// from a host-built table (so the device-built tables hold the same values).
mlmc_status Engine::build_bases() {
    base_h.clear();
    base_index.clear();
    if (!cfg.nested) return MLMC_OK;
    for (int l = 0; l <= cfg.L_max; ++l) {
        const mlmc_precision& pr = cfg.prec[l];
        if (pr.arith != MLMC_ARITH_FP32 && pr.arith != MLMC_ARITH_FP16) continue;
        const int method = pr.rng_method > 1 ? pr.rng_method : 1;
        uint32_t off;
        if (base_of(pr.arith, pr.table_bits, method, off)) continue;
        mlmc_problem prob;
        std::memset(&prob, 0, sizeof(prob));
        prob.struct_size = sizeof(prob);
        prob.scheme = MLMC_EULER;
        prob.payoff_mask = 1u << MLMC_PAY_EURO;
        prob.S0 = prob.K = prob.T = 1.0;
        prob.sigma = 0.2;
        LevelPrep lp;
        std::string err;
        const mlmc_status st2 = prepare_level(&prob, 0, &pr, MLMC_EST_APPROX, lp, err);
        if (st2 != MLMC_OK) return fail(ctx, st2, err);
        const size_t zb = pr.arith == MLMC_ARITH_FP32 ? 4 : 2, n = size_t(1) << pr.table_bits;
        off = static_cast<uint32_t>(base_h.size());
        base_h.resize(off + al(n * zb), 0);
        for (size_t k = 0; k < n; ++k) std::memcpy(&base_h[off + k * zb], &lp.table[k * 2 * zb], zb);
        base_index.emplace_back(std::make_tuple(pr.arith, pr.table_bits, method), off);
    }
    return MLMC_OK;
}

bool Engine::base_of(int arith, int q, int method, uint32_t& off) const {
    for (const auto& x : base_index)
        if (x.first == std::make_tuple(arith, q, method)) {
            off = x.second;
            return true;
        }
    return false;
}

// The engine's arrays at the start of the workspace (the tile slots take the rest).
mlmc_status Engine::layout() {
    const size_t MW = size_t(C) * RUN_MAX_PEND;
    size_t o = 0;
    const size_t o_hdr = o;
    o = al(o + sizeof(EngHeader));
    const size_t o_states = o;
    o = al(o + size_t(C) * sizeof(RunState));
    const size_t o_meta = o;
    o = al(o + size_t(C) * sizeof(EngMeta));
    const size_t o_info = o;
    o = al(o + size_t(C) * LV * 3 * sizeof(EngLevelInfo));
    const size_t o_scr = o;
    o = al(o + size_t(C) * sizeof(EngPlanScratch));
    const size_t o_works = o;
    o = al(o + MW * sizeof(WorkDev));
    const size_t o_wt = o;
    o = al(o + MW * sizeof(WorkTilesDev));
    const size_t o_red = o;
    o = al(o + MW * sizeof(EngReduce));
    const size_t o_status = o;
    o = al(o + (size_t(C) + 1) * sizeof(uint32_t));
    const size_t o_base = o;
    o = al(o + base_h.size());
    const size_t o_jobs = o;
    jobs_cap = C * LV;
    o = al(o + size_t(jobs_cap) * sizeof(EngTableJob));
    const size_t o_dstage = o;
    dstage_bytes = std::min<size_t>(std::max<size_t>(size_t(C) * 24 * 1024, size_t(256) << 10), size_t(16) << 20);
    o = al(o + dstage_bytes);
    const size_t o_levels = o;
    o = al(o + size_t(C) * LV * 3 * sizeof(LevelDev));
    const size_t o_tables = o;
    o = al(o + size_t(C) * LV * 2 * tstride);
    const size_t o_slots = o;
    if (o_slots + 64 * sizeof(TileSlot) > ctx->ws_bytes)
        return fail(ctx, MLMC_E_NOMEM, "workspace too small for the sweep engine: need " +
                                           std::to_string(o_slots + 64 * sizeof(TileSlot)) + " bytes");
    slot_cap = std::min<uint64_t>((ctx->ws_bytes - o_slots) / sizeof(TileSlot), uint64_t(1) << 22);
    uint8_t* b = ctx->ws;
    P.hdr = reinterpret_cast<EngHeader*>(b + o_hdr);
    P.states = reinterpret_cast<RunState*>(b + o_states);
    P.meta = reinterpret_cast<EngMeta*>(b + o_meta);
    P.info = reinterpret_cast<EngLevelInfo*>(b + o_info);
    P.scratch = reinterpret_cast<EngPlanScratch*>(b + o_scr);
    P.works = reinterpret_cast<WorkDev*>(b + o_works);
    P.wtiles = reinterpret_cast<WorkTilesDev*>(b + o_wt);
    P.red = reinterpret_cast<EngReduce*>(b + o_red);
    P.slots = reinterpret_cast<TileSlot*>(b + o_slots);
    P.status_out = reinterpret_cast<uint32_t*>(b + o_status);
    base = b + o_base;
    jobs = reinterpret_cast<EngTableJob*>(b + o_jobs);
    dstage = b + o_dstage;
    levels = reinterpret_cast<LevelDev*>(b + o_levels);
    tables = b + o_tables;
    return MLMC_OK;
}

mlmc_status Engine::create(mlmc_context* c, const mlmc_run_config& rc, const std::vector<EngKind>& k, uint32_t n) {
    ctx = c;
    cfg = rc;
    kinds = k;
    C = n;
    LV = static_cast<uint32_t>(rc.L_max) + 1;
    mlmc_status s = engine_classes(ctx, cfg, kinds, cls, tstride);
    if (s != MLMC_OK) return s;
    if ((s = build_bases()) != MLMC_OK) return s;
    if ((s = layout()) != MLMC_OK) return s;
    EHIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    EHIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    EHIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    for (int i = 0; i < 2; ++i) {
        EHIP(hipHostMalloc(reinterpret_cast<void**>(&status_h[i]), (size_t(C) + 1) * sizeof(uint32_t),
                           hipHostMallocDefault));
        std::memset(status_h[i], 0, (size_t(C) + 1) * sizeof(uint32_t));
        EHIP(hipEventCreateWithFlags(&ev_done[i], hipEventDisableTiming));
    }
    EHIP(hipHostMalloc(reinterpret_cast<void**>(&states_h), size_t(C) * sizeof(RunState), hipHostMallocDefault));
    levels_ready.assign(C, 0);
    generation.assign(C, 0);
    for (int i = 0; i < 2; ++i)
        if ((s = capture(i)) != MLMC_OK) return s;
    return MLMC_OK;
}

// One sweep as a graph: advance, plan, the class kernels (table-only classes on a
// second branch beside the exact-normal ones), the reduction, the status copy.
mlmc_status Engine::capture(int k) {
    EHIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_eng_advance(P, C, st);
    if (e == hipSuccess) e = launch_eng_plan(P, st);
    bool forked = false;
    for (size_t c = 0; c < cls.size() && e == hipSuccess; ++c)
        if (cls[c].v.est == MLMC_EST_APPROX) forked = true;
    if (forked && e == hipSuccess) e = hipEventRecord(ev_fork, st);
    if (forked && e == hipSuccess) e = hipStreamWaitEvent(ctx->aux_stream, ev_fork, 0);
    const uint32_t grid = static_cast<uint32_t>(std::max(1, ctx->cu_count)) * ctx->tune.blocks_per_cu;
    for (size_t c = 0; c < cls.size() && e == hipSuccess; ++c) {
        const EngClass& x = cls[c];
        hipStream_t s2 = (forked && x.v.est == MLMC_EST_APPROX) ? ctx->aux_stream : st;
        e = launch_paths(x.vi, grid, x.block, x.lds, s2, P.wtiles, &P.hdr->counts[c][0], P.works, levels, tables,
                         P.slots);
    }
    if (forked && e == hipSuccess) e = hipEventRecord(ev_join, ctx->aux_stream);
    if (forked && e == hipSuccess) e = hipStreamWaitEvent(st, ev_join, 0);
    const uint32_t rgrid = static_cast<uint32_t>(std::min<size_t>(size_t(C) * RUN_MAX_PEND, 1024));
    if (e == hipSuccess) e = launch_eng_reduce(P, rgrid, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(status_h[k], P.status_out, (size_t(C) + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec[k], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(ctx, MLMC_E_DEVICE, std::string("sweep graph: ") + hipGetErrorString(e));
    return MLMC_OK;
}

// ---------------------------------------------------------------- uploads
uint8_t* Engine::Upload::put(const void* src, size_t bytes, uint64_t dst) {
    const size_t off = data.size();
    data.resize(off + ((bytes + 7) & ~size_t(7)), 0);
    if (src) std::memcpy(data.data() + off, src, bytes);
    segs.push_back(EngSeg{off, dst, (bytes + 7) & ~uint64_t(7)});
    return data.data() + off;
}

void Engine::Upload::zero(size_t bytes, uint64_t dst) { segs.push_back(EngSeg{ENG_SEG_ZERO, dst, bytes}); }

// An upload in pieces that fit the device staging area: each piece's data and its
// segment list are one image in a pinned buffer, copied by DMA to the staging area,
// then scattered by a kernel; the stream orders the pieces.
mlmc_status Engine::flush(Upload& u) {
    if (u.segs.empty() && u.jobs.empty()) return MLMC_OK;
    const uint32_t n_jobs = static_cast<uint32_t>(u.jobs.size());
    if (n_jobs > jobs_cap) return fail(ctx, MLMC_E_INVALID, "engine upload: too many step tables in one upload");
    if (n_jobs) u.put(u.jobs.data(), u.jobs.size() * sizeof(EngTableJob), reinterpret_cast<uint64_t>(jobs));
    {   // the scatter copies segments concurrently: they must not overlap
        std::vector<std::pair<uint64_t, uint64_t>> r;
        for (const EngSeg& g : u.segs) r.emplace_back(g.dst, g.dst + g.bytes);
        std::sort(r.begin(), r.end());
        for (size_t i = 1; i < r.size(); ++i)
            if (r[i].first < r[i - 1].second) return fail(ctx, MLMC_E_INVALID, "engine upload: overlapping segments");
    }
    // segments split to at most max_piece data bytes, then grouped into images
    const size_t max_piece = (dstage_bytes / 2) & ~size_t(7);
    struct Image {
        size_t off, data_bytes;
        std::vector<EngSeg> segs;     // src: offset in the image
    };
    std::vector<Image> imgs;
    size_t total = 0;
    auto image_bytes = [](const Image& im) { return al(im.data_bytes) + im.segs.size() * sizeof(EngSeg); };
    auto open_image = [&]() {
        if (!imgs.empty()) total += al(image_bytes(imgs.back()));
        imgs.push_back(Image{total, 0, {}});
    };
    open_image();
    for (const EngSeg& g : u.segs) {
        if (g.src == ENG_SEG_ZERO) {
            if (al(imgs.back().data_bytes) + (imgs.back().segs.size() + 1) * sizeof(EngSeg) > dstage_bytes) open_image();
            imgs.back().segs.push_back(g);
            continue;
        }
        for (uint64_t done = 0; done < g.bytes;) {
            const uint64_t nb = std::min<uint64_t>(g.bytes - done, max_piece);
            Image* im = &imgs.back();
            if (al(im->data_bytes + nb) + (im->segs.size() + 1) * sizeof(EngSeg) > dstage_bytes) {
                open_image();
                im = &imgs.back();
            }
            im->segs.push_back(EngSeg{g.src + done, g.dst + done, nb});   // src rebased below
            im->data_bytes += nb;
            done += nb;
        }
    }
    total += al(image_bytes(imgs.back()));
    // a pinned buffer not in use by an upload the stream has not run yet
    StageBuf* sb = nullptr;
    for (auto& b : stage)
        if (b.bytes >= total && hipEventQuery(b.ev) == hipSuccess) { sb = &b; break; }
    if (!sb) {
        stage.emplace_back();
        sb = &stage.back();
        sb->bytes = std::max<size_t>(total, size_t(1) << 20);
        EHIP(hipHostMalloc(reinterpret_cast<void**>(&sb->p), sb->bytes, hipHostMallocDefault));
        EHIP(hipEventCreateWithFlags(&sb->ev, hipEventDisableTiming));
    }
    for (Image& im : imgs) {
        uint8_t* base = sb->p + im.off;
        size_t d = 0;
        for (EngSeg& g : im.segs) {
            if (g.src == ENG_SEG_ZERO) continue;
            std::memcpy(base + d, u.data.data() + g.src, g.bytes);
            g.src = d;
            d += g.bytes;
        }
        const size_t seg_off = al(im.data_bytes);
        std::memcpy(base + seg_off, im.segs.data(), im.segs.size() * sizeof(EngSeg));
        EHIP(hipMemcpyAsync(dstage, base, image_bytes(im), hipMemcpyHostToDevice, st));
        EHIP(launch_eng_scatter(dstage, reinterpret_cast<const EngSeg*>(dstage + seg_off),
                                static_cast<uint32_t>(im.segs.size()), st));
    }
    // the step tables read the levels' constants the copies have just written
    EHIP(launch_eng_tables(jobs, n_jobs, levels, base, tables, st));
    EHIP(hipEventRecord(sb->ev, st));
    u.data.clear();
    u.segs.clear();
    u.jobs.clear();
    return MLMC_OK;
}

// The header of a fresh engine run (every slot inactive until admitted).
void Engine::stage_reset(Upload& u) {
    EngHeader h;
    std::memset(&h, 0, sizeof(h));
    h.n_slots = C;
    h.n_levels = LV;
    h.n_classes = static_cast<uint32_t>(cls.size());
    h.tile_steps = ctx->tune.tile_steps;
    h.min_tiles = ctx->tune.min_tiles;
    h.max_tiles_work = static_cast<uint32_t>(FLIGHT_MAX_TILES);
    h.slot_cap = slot_cap;
    h.max_works = uint64_t(C) * RUN_MAX_PEND;
    u.put(&h, sizeof(h), reinterpret_cast<uint64_t>(P.hdr));
    // the base tables too: other engines of the context use the same workspace
    if (!base_h.empty()) u.put(base_h.data(), base_h.size(), reinterpret_cast<uint64_t>(base));
    meta_h.assign(C, EngMeta{});
    std::fill(levels_ready.begin(), levels_ready.end(), 0u);
}

// Every slot's meta in one segment (a fresh engine run: inactive slots zero).  The
// segments of one upload are copied concurrently, so no two of them may overlap:
// a run's own meta segment (stage_run with put_meta) is for slots admitted later.
void Engine::stage_meta_all(Upload& u) {
    u.put(meta_h.data(), meta_h.size() * sizeof(EngMeta), reinterpret_cast<uint64_t>(P.meta));
}

// The levels of each task: constants, step tables and launch classes.  FP32 and
// FP16 approximate-side step tables are built on the device (EngTableJob, after the
// copies); the correction estimator shares its level's approximate table; other
// tables (fixed point, Method 2's correction table) are built on the host, on up to
// 8 threads when there are many.  The staging follows in task order.
mlmc_status Engine::stage_tasks(Upload& u, const std::vector<LevelTask>& tasks) {
    const mlmc_precision plain = plain_prec_of(cfg);
    struct Item {
        uint32_t s, l;
        int e;
        const mlmc_problem* prob;
        LevelPrep lp;
        mlmc_status st = MLMC_OK;
        std::string err;
    };
    std::vector<Item> items;
    for (const LevelTask& t : tasks)
        for (uint32_t l = t.from; l < t.to; ++l)
            for (int e = 0; e < 3; ++e)
                if (e == MLMC_EST_PLAIN || t.nested) items.push_back(Item{t.s, l, e, t.prob, {}, MLMC_OK, {}});
    // the correction estimator's table is the approximate one's (same precision) but
    // for Method 2's permutation: not built twice
    auto shares = [&](const Item& it) { return it.e == MLMC_EST_CORR && cfg.prec[it.l].rng_method != 2; };
    // FP32 / FP16 approximate sides: step tables built on the device from a base table
    auto on_device = [&](const Item& it, uint32_t* off) {
        const mlmc_precision& pr = cfg.prec[it.l];
        uint32_t o2;
        return it.e == MLMC_EST_APPROX && (pr.arith == MLMC_ARITH_FP32 || pr.arith == MLMC_ARITH_FP16) &&
               base_of(pr.arith, pr.table_bits, pr.rng_method > 1 ? pr.rng_method : 1, off ? *off : o2);
    };
    auto prep = [&](size_t i0, size_t i1) {
        for (size_t i = i0; i < i1; ++i) {
            Item& it = items[i];
            const mlmc_precision* pr = it.e == MLMC_EST_PLAIN ? &plain : &cfg.prec[it.l];
            it.st = prepare_level(it.prob, static_cast<int>(it.l), pr, it.e, it.lp, it.err,
                                  !shares(it) && !on_device(it, nullptr));
        }
    };
    const size_t n_items = items.size();
    size_t n_host_tables = 0;                           // the items whose tables the host builds
    for (const Item& it : items)
        if (it.e != MLMC_EST_PLAIN && !shares(it) && !on_device(it, nullptr)) ++n_host_tables;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t n_thr = std::min<size_t>({size_t(8), size_t(hw), n_host_tables / 32});
    if (n_thr >= 2) {
        std::vector<std::thread> th;
        const size_t per = (n_items + n_thr - 1) / n_thr;
        for (size_t k = 1; k < n_thr; ++k)
            th.emplace_back(prep, std::min(n_items, k * per), std::min(n_items, (k + 1) * per));
        prep(0, std::min(n_items, per));
        for (auto& t : th) t.join();
    } else {
        prep(0, n_items);
    }
    bool approx_table = false;                          // the (slot, level)'s approximate-side table
    size_t approx_off = 0;
    for (size_t i = 0; i < n_items; ++i) {
        Item& it = items[i];
        if (it.st != MLMC_OK) return fail(ctx, it.st, it.err);
        const uint32_t s = it.s, l = it.l;
        const int e = it.e;
        if (i == 0 || items[i - 1].s != s || items[i - 1].l != l) approx_table = false;
        const LevelPrep& lp = it.lp;
        Variant v = lp.variant;
        v.l0 = level0_kernel_for(v, static_cast<int>(l), false, lp.dev);
        int ci = -1;
        for (size_t c = 0; c < cls.size(); ++c)
            if (class_key(cls[c].v) == class_key(v)) ci = static_cast<int>(c);
        if (ci < 0) return fail(ctx, MLMC_E_INVALID, "a run needs a kernel class the engine was not built for");
        const size_t idx = (size_t(s) * LV + l) * 3 + e;
        LevelDev L = lp.dev;
        uint32_t boff = 0;
        if (shares(it)) {
            if (!approx_table) return fail(ctx, MLMC_E_INVALID, "engine: a correction level without its approximate table");
            L.table_off = static_cast<uint32_t>(approx_off);            // the same bytes: shared
        } else if (on_device(it, &boff)) {
            const size_t toff = ((size_t(s) * LV + l) * 2) * tstride;
            L.table_off = static_cast<uint32_t>(toff);
            u.jobs.push_back(EngTableJob{static_cast<uint32_t>(idx), static_cast<uint32_t>(toff), boff,
                                         static_cast<uint16_t>(cfg.prec[l].arith),
                                         static_cast<uint16_t>(it.prob->scheme == MLMC_MILSTEIN ? 1 : 0)});
            approx_table = true;
            approx_off = toff;
        } else if (!lp.table.empty()) {
            const size_t toff = ((size_t(s) * LV + l) * 2 + (e == MLMC_EST_CORR ? 1 : 0)) * tstride;
            L.table_off = static_cast<uint32_t>(toff);
            u.put(lp.table.data(), lp.table.size(), reinterpret_cast<uint64_t>(tables + toff));
            if (e == MLMC_EST_APPROX) {
                approx_table = true;
                approx_off = toff;
            }
        }
        u.put(&L, sizeof(L), reinterpret_cast<uint64_t>(levels + idx));
        const mlmc_precision* pr = e == MLMC_EST_PLAIN ? &plain : &cfg.prec[l];
        EngLevelInfo in;
        in.cls = static_cast<uint16_t>(ci);
        in.wpb = static_cast<uint16_t>(cls[ci].vi.wpb);
        in.block = static_cast<uint16_t>(cls[ci].block);
        in.kind = static_cast<uint16_t>((e == MLMC_EST_CORR ? 1 : 0) |
                                        (e == MLMC_EST_APPROX && pr->arith == MLMC_ARITH_FIXED ? 2 : 0));
        u.put(&in, sizeof(in), reinterpret_cast<uint64_t>(P.info + idx));
    }
    return MLMC_OK;
}

// A new run in slot s: its state, its first levels and its meta (active), the meta
// as a segment of its own with put_meta, else only in the host mirror (for
// stage_meta_all).
mlmc_status Engine::stage_run(Upload& u, uint32_t s, const mlmc_problem& prob, const mlmc_run_config& rc,
                              uint64_t seed, uint32_t option, bool put_meta, std::vector<LevelTask>* defer) {
    RunState rs;
    run_state_init(rs, prob, rc);
    // the configuration and progress words; the sums and pending works start at zero
    const size_t head = offsetof(RunState, sums);
    u.put(&rs, head, reinterpret_cast<uint64_t>(P.states + s));
    u.zero(sizeof(RunState) - head, reinterpret_cast<uint64_t>(P.states + s) + head);
    const uint32_t first = std::min<uint32_t>(LV, static_cast<uint32_t>(rc.L_min) + 2);
    const LevelTask t{s, &prob, rc.nested != 0, 0, first};
    if (defer) {
        defer->push_back(t);
    } else {
        const mlmc_status st2 = stage_tasks(u, {t});
        if (st2 != MLMC_OK) return st2;
    }
    levels_ready[s] = first;
    generation[s] = (generation[s] + 1) & 0xFFFFu;
    EngMeta m;
    std::memset(&m, 0, sizeof(m));
    m.active = 1;
    m.levels_ready = first;
    m.c3 = option;
    m.k0 = static_cast<uint32_t>(seed);
    m.k1 = static_cast<uint32_t>(seed >> 32);
    m.generation = generation[s];
    meta_h[s] = m;
    if (put_meta) u.put(&m, sizeof(m), reinterpret_cast<uint64_t>(P.meta + s));
    return MLMC_OK;
}

// More levels for a run that waits for `need`: up to need + 1 (one ahead).
mlmc_status Engine::stage_more_levels(Upload& u, uint32_t s, const mlmc_problem& prob, bool nested, uint32_t need,
                                      std::vector<LevelTask>* defer) {
    const uint32_t to = std::min<uint32_t>(LV, need + 2);
    if (to <= levels_ready[s]) return MLMC_OK;
    const LevelTask t{s, &prob, nested, levels_ready[s], to};
    if (defer) {
        defer->push_back(t);
    } else {
        const mlmc_status st2 = stage_tasks(u, {t});
        if (st2 != MLMC_OK) return st2;
    }
    levels_ready[s] = to;
    return MLMC_OK;
}

// The meta's (levels_ready, c3) word pair: uploads move 8-byte words, and these two
// are the host's (pending_valid and status, the device's, are not written).
void Engine::stage_levels_ready(Upload& u, uint32_t s, uint32_t c3) {
    const uint32_t w[2] = {levels_ready[s], c3};
    u.put(w, sizeof(w), reinterpret_cast<uint64_t>(&P.meta[s].levels_ready));
}

mlmc_status Engine::replay(int k) {
    EHIP(hipGraphLaunch(exec[k], st));
    EHIP(hipEventRecord(ev_done[k], st));
    return MLMC_OK;
}

// ------------------------------------------------------------ a batch of runs
mlmc_status engine_run_batch(mlmc_context* ctx, std::vector<OptionRun>& runs) {
    const uint32_t n = static_cast<uint32_t>(runs.size());
    std::vector<EngKind> kinds;
    for (const OptionRun& o : runs) {
        EngKind k;
        k.scheme = o.prob.scheme;
        k.track = ((o.prob.payoff_mask >> MLMC_PAY_ASIAN) & 1u) || ((o.prob.payoff_mask >> MLMC_PAY_BARRIER) & 1u);
        k.nested = o.cfg.nested != 0;
        if (std::find(kinds.begin(), kinds.end(), k) == kinds.end()) kinds.push_back(k);
    }
    std::sort(kinds.begin(), kinds.end());
    Engine* E = nullptr;
    for (auto& x : ctx->engines)
        if (x->C >= n && x->C <= 2 * n + 8 && x->kinds == kinds && x->LV == uint32_t(runs[0].cfg.L_max) + 1 &&
            std::memcmp(x->cfg.prec, runs[0].cfg.prec, sizeof(x->cfg.prec)) == 0 &&
            x->cfg.plain_arith == runs[0].cfg.plain_arith && x->tune_key == ctx->tune_key())
            E = x.get();
    if (!E) {
        auto ne = std::make_unique<Engine>();
        mlmc_status s = ne->create(ctx, runs[0].cfg, kinds, std::max<uint32_t>(n, 1));
        if (s != MLMC_OK) return s;
        ne->tune_key = ctx->tune_key();
        if (ctx->engines.size() >= 6) ctx->engines.erase(ctx->engines.begin());
        ctx->engines.push_back(std::move(ne));
        E = ctx->engines.back().get();
    }
    Engine::Upload u;
    std::vector<Engine::LevelTask> tasks;
    E->stage_reset(u);
    for (uint32_t i = 0; i < n; ++i) {
        const mlmc_status s = E->stage_run(u, i, runs[i].prob, runs[i].cfg, runs[i].seed, runs[i].option, false,
                                           &tasks);
        if (s != MLMC_OK) return s;
    }
    mlmc_status s = E->stage_tasks(u, tasks);
    if (s != MLMC_OK) return s;
    E->stage_meta_all(u);
    s = E->flush(u);
    if (s != MLMC_OK) return s;
    // two sweeps in flight: the host reads sweep j's status while sweep j + 1 runs
    std::vector<uint8_t> finished(n, 0);
    uint32_t left = n;
    int launched = 0, landed = 0;
    const int max_sweeps = 20000;
    while (left > 0) {
        while (launched - landed < 2) {
            if ((s = E->replay(launched & 1)) != MLMC_OK) return s;
            launched += 1;
        }
        const int k = landed & 1;
        hipError_t e = hipEventSynchronize(E->ev_done[k]);
        if (e != hipSuccess) return fail(ctx, MLMC_E_DEVICE, std::string("sweep: ") + hipGetErrorString(e));
        landed += 1;
        const uint32_t* stw = E->status_h[k];
        if (stw[E->C] == 1u) return fail(ctx, MLMC_E_NOMEM, "a run's works need more tile slots than the workspace holds");
        if (stw[E->C]) return fail(ctx, MLMC_E_DEVICE, "sweep engine: a work's level was not prepared");
        tasks.clear();
        for (uint32_t i = 0; i < n; ++i) {
            if (finished[i]) continue;
            const uint32_t w = stw[i];
            if ((w >> 16) != E->generation[i]) continue;
            if (w & ENG_DONE) {
                finished[i] = 1;
                left -= 1;
                runs[i].t_end = now_seconds();
            } else if (w & ENG_WAIT_LEVEL) {
                if ((s = E->stage_more_levels(u, i, runs[i].prob, runs[i].cfg.nested != 0, (w >> 8) & 0xFFu,
                                              &tasks)) != MLMC_OK)
                    return s;
                E->stage_levels_ready(u, i, runs[i].option);
            }
        }
        if (!tasks.empty() && (s = E->stage_tasks(u, tasks)) != MLMC_OK) return s;
        if ((s = E->flush(u)) != MLMC_OK) return s;
        if (landed > max_sweeps) return fail(ctx, MLMC_E_DEVICE, "sweep engine made no progress");
    }
    // the sweep still in flight does nothing for finished runs; then the states
    while (landed < launched) {
        hipError_t e = hipEventSynchronize(E->ev_done[landed & 1]);
        if (e != hipSuccess) return fail(ctx, MLMC_E_DEVICE, std::string("sweep: ") + hipGetErrorString(e));
        landed += 1;
    }
    EHIP(hipMemcpyAsync(E->states_h, E->P.states, size_t(n) * sizeof(RunState), hipMemcpyDeviceToHost, E->st));
    EHIP(hipStreamSynchronize(E->st));
    for (uint32_t i = 0; i < n; ++i) runs[i].st = E->states_h[i];
    return MLMC_OK;
}

}  // namespace mlmc
