// Continuous-batching server: a scheduler thread owns the device work of all
// admitted requests and keeps the device busy with up to two launch sequences
// ("flights") at a time.  Each loop iteration
//   1. admits queued requests while a slot is free;
//   2. lands the flights whose completion event has fired (oldest first) and adds
//      each request's per-work sums into its host sums;
//   3. if fewer than two flights are in progress, asks every admitted request that
//      has no work in flight for its next samples (pilot, allocation top-up or a new
//      level -- the adaptive driver of Sections 2.1/2.2/6), publishes the requests
//      that converged, and launches the rest as one flight.
// A request that arrives while a flight runs therefore starts in the next flight,
// which is queued on the stream behind the running one, instead of waiting for a
// whole sweep of the others.  Device memory: each flight's plan occupies a ring
// over the workspace (the HBM budget); a flight lands older ones to make room, and
// a plan larger than the whole workspace is launched as several flights.
// Each request has at most one flight's worth of work outstanding, its sums are
// its own (one result per (level, estimator) per flight, added on the host) and its
// uniforms depend only on (seed, option_id, level, estimator, path), so its result
// does not depend on what else is in flight.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "engine_host.hpp"
#include "runtime.hpp"

namespace mlmc {

struct Server {
    mlmc_context* ctx = nullptr;
    mlmc_server_config cfg{};
    std::thread th;
    std::mutex m;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_ticket = 1;
    struct Queued {
        uint64_t ticket;
        mlmc_request req;
        double t_submit;
    };
    struct Active {
        uint64_t ticket;
        uint32_t slot;
        int in_flight = 0;          // flights holding this request's work
        OptionRun run;
    };
    struct SFlight {
        uint64_t ticket;            // the context's flight ticket
        std::shared_ptr<std::vector<SlotDev>> sink;
        std::vector<std::pair<Active*, Pending>> who;    // per work
    };
    static constexpr size_t MAX_SF = 2;
    std::deque<Queued> queue;
    std::vector<std::unique_ptr<Active>> active;
    std::deque<SFlight> sflights;
    std::map<uint64_t, mlmc_result> done;
    std::deque<uint64_t> done_order;     // completion order (entries may be taken already)
    std::vector<uint32_t> free_slots;
    uint32_t n_slots = 0;
    mlmc_status error = MLMC_OK;
    std::string error_msg;
    mlmc_server_stats stats{};          // guarded by m
    uint64_t flights_launched = 0;      // scheduler thread only

    // device sweep engine mode: every admitted request's run lives in an engine slot
    std::unique_ptr<Engine> eng;
    struct SlotRun {
        int state = 0;              // 0 free, 1 running on the device, 2 result downloading
        uint64_t ticket = 0;
        mlmc_problem prob{};
        mlmc_run_config rc{};
        double t_submit = 0.0;
        hipEvent_t ev = nullptr;    // the state download
    };
    std::vector<SlotRun> runs;
    bool owned_events = false;
    uint64_t slot_bytes = 0;        // device bytes per admitted request
    ~Server() {
        if (owned_events)
            for (auto& r : runs)
                if (r.ev) (void)hipEventDestroy(r.ev);
    }
    int eng_in_flight = 0;          // sweeps launched and not yet landed
    uint64_t eng_launched = 0, eng_landed = 0;
    mlmc_status engine_start();
    mlmc_status engine_admit(bool& progressed);
    mlmc_status engine_land(bool& progressed);
    void loop_engine();

    void loop();
    void publish(uint64_t ticket, const mlmc_result& r) {    // caller holds m
        done[ticket] = r;
        done_order.push_back(ticket);
    }
    mlmc_status land(bool& progressed);
    mlmc_status launch(std::vector<WorkSpec>& works, std::vector<std::pair<Active*, Pending>>& who,
                       size_t b, size_t e);
    void fail_all(mlmc_status s);
};

// Lands the flights whose completion event has fired, oldest first.
mlmc_status Server::land(bool& progressed) {
    while (!sflights.empty()) {
        SFlight& sf = sflights.front();
        mlmc_status st = MLMC_OK;
        {
            std::lock_guard<std::mutex> dl(ctx->dev_mtx);
            auto it = std::find_if(ctx->flights.begin(), ctx->flights.end(),
                                   [&](const Flight& f) { return f.ticket == sf.ticket; });
            if (it != ctx->flights.end()) {
                // both streams' parts must be complete: landing waits on each
                if (hipEventQuery(it->done) == hipErrorNotReady) return MLMC_OK;
                if (it->done_aux && hipEventQuery(it->done_aux) == hipErrorNotReady) return MLMC_OK;
                for (;;) {                        // land everything up to and including it
                    const uint64_t t = ctx->flights.front().ticket;
                    drain_oldest(ctx);
                    if (t == sf.ticket) break;
                }
            }
            // landed here or by a launch that needed its room: status in finished
            auto fs = ctx->finished.find(sf.ticket);
            if (fs != ctx->finished.end()) {
                st = fs->second;
                ctx->finished.erase(fs);
            }
        }
        if (st != MLMC_OK) return st;
        const std::vector<SlotDev>& res = *sf.sink;
        std::vector<Active*> seen;
        for (size_t k = 0; k < sf.who.size(); ++k) {
            Active* a = sf.who[k].first;
            const Pending& p = sf.who[k].second;
            est_accumulate(a->run.st.sums[p.level][p.est], est_of_slot(res[k]));
            a->run.st.path_steps += p.n << p.level;
            if (std::find(seen.begin(), seen.end(), a) == seen.end()) {
                seen.push_back(a);
                a->run.st.sweeps += 1;
                a->in_flight -= 1;
            }
        }
        sflights.pop_front();
        progressed = true;
    }
    return MLMC_OK;
}

// Launches works [b, e) as one flight; a plan larger than the workspace is halved.
mlmc_status Server::launch(std::vector<WorkSpec>& works, std::vector<std::pair<Active*, Pending>>& who,
                           size_t b, size_t e) {
    const std::vector<WorkSpec> part(works.begin() + b, works.begin() + e);
    Flight f;
    mlmc_status s;
    {
        std::lock_guard<std::mutex> dl(ctx->dev_mtx);
        s = launch_flight(ctx, part, f);
        if (s == MLMC_OK) {
            f.ticket = ctx->next_ticket++;
            f.sink = std::make_shared<std::vector<SlotDev>>();
            SFlight sf{f.ticket, f.sink, {}};
            std::vector<Active*> seen;
            for (size_t k = b; k < e; ++k) {
                sf.who.push_back(who[k]);
                Active* a = who[k].first;
                if (std::find(seen.begin(), seen.end(), a) == seen.end()) {
                    seen.push_back(a);
                    a->in_flight += 1;
                }
            }
            ctx->flights.push_back(std::move(f));
            sflights.push_back(std::move(sf));
            flights_launched += 1;
            return MLMC_OK;
        }
    }
    if (s == MLMC_E_NOMEM && e - b >= 2) {
        const size_t h = b + (e - b) / 2;
        if ((s = launch(works, who, b, h)) != MLMC_OK) return s;
        return launch(works, who, h, e);
    }
    return s;
}

void Server::fail_all(mlmc_status s) {
    std::lock_guard<std::mutex> lk(m);
    error = s;
    error_msg = ctx->err;
    for (SlotRun& r : runs) {
        if (r.state == 0) continue;
        mlmc_result res;
        std::memset(&res, 0, sizeof(res));
        res.struct_size = sizeof(res);
        res.status = s;
        publish(r.ticket, res);
        r.state = 0;
    }
    for (auto& a : active) {
        mlmc_result r;
        option_result(a->run, r);
        r.status = s;
        publish(a->ticket, r);
    }
    active.clear();
    for (auto& q : queue) {
        mlmc_result r;
        std::memset(&r, 0, sizeof(r));
        r.struct_size = sizeof(r);
        r.status = s;
        publish(q.ticket, r);
    }
    queue.clear();
    sflights.clear();           // their flights land later; the sinks own the results
    cv.notify_all();
}

void Server::loop() {
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(m);
            if (sflights.empty())
                cv.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop) {
                // requests not yet admitted are cancelled; admitted ones finish
                for (auto& q : queue) {
                    mlmc_result r;
                    std::memset(&r, 0, sizeof(r));
                    r.struct_size = sizeof(r);
                    r.status = MLMC_E_BUSY;
                    publish(q.ticket, r);
                }
                queue.clear();
                cv.notify_all();
                if (active.empty() && sflights.empty()) return;
            }
            while (!queue.empty() && !free_slots.empty()) {
                Queued q = queue.front();
                queue.pop_front();
                auto a = std::make_unique<Active>();
                a->ticket = q.ticket;
                a->slot = free_slots.back();
                free_slots.pop_back();
                a->run.prob = q.req.problem;
                a->run.cfg = cfg.run;
                a->run.cfg.eps = q.req.eps;
                a->run.cfg.nested = q.req.nested;
                a->run.seed = q.req.seed;
                a->run.option = q.req.option_id;
                option_init(a->run);
                a->run.t_start = q.t_submit;
                active.push_back(std::move(a));
            }
        }
        bool progressed = false;
        const double t_land = now_seconds();
        mlmc_status s = land(progressed);
        if (s != MLMC_OK) { fail_all(s); return; }
        const double t_plan = now_seconds();
        uint64_t n_launched = 0;
        if (sflights.size() < MAX_SF) {
            // plan every admitted request with no work in flight
            std::vector<WorkSpec> works;
            std::vector<std::pair<Active*, Pending>> who;
            std::deque<mlmc_precision> plain;        // stable addresses for the WorkSpecs
            bool retired = false;
            for (auto& up : active) {
                Active* a = up.get();
                if (a->in_flight || a->run.st.done) continue;
                OptionRun& o = a->run;
                mlmc_precision pp;
                std::memset(&pp, 0, sizeof(pp));
                pp.struct_size = sizeof(pp);
                pp.arith = o.cfg.plain_arith;
                pp.table_bits = 8;
                plain.push_back(pp);
                for (const Pending& p : option_advance(o)) {
                    WorkSpec w;
                    w.prob = &o.prob;
                    w.level = p.level;
                    w.prec = p.est == MLMC_EST_PLAIN ? &plain.back() : &o.cfg.prec[p.level];
                    w.est = p.est;
                    w.seed = o.seed;
                    w.option = o.option;
                    w.path_begin = o.st.sums[p.level][p.est].n;
                    w.n = p.n;
                    w.debug = 0;
                    std::string err;
                    const mlmc_status ps = option_prep(o, p.level, p.est, w.prec, w.prep, err);
                    if (ps != MLMC_OK) {
                        fail(ctx, ps, err);
                        fail_all(ps);
                        return;
                    }
                    works.push_back(w);
                    who.emplace_back(a, p);
                }
                retired = retired || o.st.done;
            }
            if (retired) {
                std::lock_guard<std::mutex> lk(m);
                for (auto it = active.begin(); it != active.end();) {
                    if ((*it)->run.st.done) {
                        OptionRun& o = (*it)->run;
                        mlmc_result r;
                        option_result(o, r);
                        publish((*it)->ticket, r);
                        stats.requests_done += 1;
                        free_slots.push_back((*it)->slot);
                        it = active.erase(it);
                    } else {
                        ++it;
                    }
                }
                cv.notify_all();
                progressed = true;
            }
            if (!works.empty()) {
                if ((s = launch(works, who, 0, works.size())) != MLMC_OK) { fail_all(s); return; }
                progressed = true;
                n_launched = works.size();
            }
        }
        const double t_done = now_seconds();
        {
            std::lock_guard<std::mutex> lk(m);
            stats.land_seconds += t_plan - t_land;
            stats.plan_seconds += t_done - t_plan;
            stats.works += n_launched;
            stats.flights = flights_launched;
        }
        if (!progressed && !sflights.empty()) {
            // a flight is running: wake on a new request or poll its event shortly
            std::unique_lock<std::mutex> lk(m);
            cv.wait_for(lk, std::chrono::microseconds(50),
                        [&] { return stop || (!queue.empty() && !free_slots.empty()); });
            stats.idle_seconds += now_seconds() - t_done;
        }
    }
}

// ---------------------------------------------------------- engine mode
// The requests' runs live in the device sweep engine (engine.hpp): their sums,
// sample counts and the driver's decisions stay in device memory and each sweep of
// all admitted runs is one graph replay.  Admission is by device memory: the
// workspace (the HBM budget) holds the engine's arrays for `slots` runs of
// slot_bytes each plus a quarter of the workspace of tile slots; a request is
// admitted when its bytes fit, i.e. when a slot is free.
mlmc_status Server::engine_start() {
    std::vector<EngClass> cls;
    size_t tstride = 256;
    EngKind k0;
    k0.scheme = MLMC_MILSTEIN;
    k0.nested = true;
    std::vector<EngKind> probe{k0};
    mlmc_status s = engine_classes(ctx, cfg.run, probe, cls, tstride);
    if (s != MLMC_OK) return s;
    const uint32_t LV = static_cast<uint32_t>(cfg.run.L_max) + 1;
    slot_bytes = Engine::slot_bytes(LV, tstride);
    const uint64_t reserve = ctx->ws_bytes / 4 + 4096;
    if (ctx->ws_bytes <= reserve + slot_bytes) return MLMC_E_NOMEM;
    const uint64_t fit = (ctx->ws_bytes - reserve) / slot_bytes;
    const uint32_t C = static_cast<uint32_t>(std::min<uint64_t>(fit, cfg.max_active));
    if (C < 1) return MLMC_E_NOMEM;
    {
        std::lock_guard<std::mutex> dl(ctx->dev_mtx);
        s = drain_flights(ctx);
        if (s != MLMC_OK && ctx->poisoned) return s;
    }
    eng = std::make_unique<Engine>();
    // built for nested Milstein runs without path functionals (the tables' size is the
    // run config's); other kinds add their kernels when a request needs them
    if ((s = eng->create(ctx, cfg.run, probe, C)) != MLMC_OK) return s;
    Engine::Upload u;
    eng->stage_reset(u);
    eng->stage_meta_all(u);
    if ((s = eng->flush(u)) != MLMC_OK) return s;
    runs.assign(C, SlotRun{});
    for (auto& r : runs)
        if (hipEventCreateWithFlags(&r.ev, hipEventDisableTiming) != hipSuccess) return MLMC_E_DEVICE;
    owned_events = true;
    n_slots = C;
    free_slots.clear();
    for (uint32_t i = C; i-- > 0;) free_slots.push_back(i);
    return MLMC_OK;
}

// Admits queued requests while a slot (slot_bytes of the workspace) is free.  A
// request of a kind (scheme, path functionals, nested) the engine has no kernels for
// adds them once no sweep is in flight (a new graph).
mlmc_status Server::engine_admit(bool& progressed) {
    Engine::Upload u;
    for (;;) {
        Queued q;
        uint32_t s;
        {
            std::lock_guard<std::mutex> lk(m);
            if (queue.empty() || free_slots.empty()) break;
            q = queue.front();
            EngKind k;
            k.scheme = q.req.problem.scheme;
            k.track = ((q.req.problem.payoff_mask >> MLMC_PAY_ASIAN) & 1u) ||
                      ((q.req.problem.payoff_mask >> MLMC_PAY_BARRIER) & 1u);
            k.nested = q.req.nested != 0;
            if (std::find(eng->kinds.begin(), eng->kinds.end(), k) == eng->kinds.end()) {
                if (!u.segs.empty()) break;                 // first send what is staged
                if (eng_in_flight) return MLMC_PENDING;     // after the sweeps in flight
                std::vector<EngKind> kinds = eng->kinds;
                kinds.push_back(k);
                std::vector<EngClass> cls;
                size_t tstride = 0;
                mlmc_status st2 = engine_classes(ctx, eng->cfg, kinds, cls, tstride);
                if (st2 != MLMC_OK) return st2;
                if (tstride > eng->tstride) return fail(ctx, MLMC_E_INVALID, "engine: table stride changed");
                eng->kinds = kinds;
                eng->cls = cls;
                for (int i = 0; i < 2; ++i) {
                    if (eng->exec[i]) (void)hipGraphExecDestroy(eng->exec[i]);
                    eng->exec[i] = nullptr;
                    if ((st2 = eng->capture(i)) != MLMC_OK) return st2;
                }
                // the header's (n_classes, tile_steps) word pair
                const uint32_t w2[2] = {static_cast<uint32_t>(cls.size()), ctx->tune.tile_steps};
                u.put(w2, sizeof(w2), reinterpret_cast<uint64_t>(&eng->P.hdr->n_classes));
            }
            queue.pop_front();
            s = free_slots.back();
            free_slots.pop_back();
        }
        SlotRun& r = runs[s];
        r.state = 1;
        r.ticket = q.ticket;
        r.prob = q.req.problem;
        r.rc = cfg.run;
        r.rc.eps = q.req.eps;
        r.rc.nested = q.req.nested;
        r.t_submit = q.t_submit;
        const mlmc_status st2 = eng->stage_run(u, s, r.prob, r.rc, q.req.seed, q.req.option_id, true);
        if (st2 != MLMC_OK) return st2;
        progressed = true;
    }
    return eng->flush(u);
}

// Lands the oldest sweep if it has finished: runs that finished get their state
// downloaded, runs that wait for a level get it; downloads that completed become
// results and free their slots.
mlmc_status Server::engine_land(bool& progressed) {
    Engine::Upload u;
    if (eng_in_flight > 0) {
        const int k = static_cast<int>(eng_landed & 1u);
        const hipError_t q = hipEventQuery(eng->ev_done[k]);
        if (q != hipErrorNotReady) {
            if (q != hipSuccess) return fail(ctx, MLMC_E_DEVICE, std::string("sweep: ") + hipGetErrorString(q));
            eng_in_flight -= 1;
            eng_landed += 1;
            progressed = true;
            const uint32_t* stw = eng->status_h[k];
            if (stw[eng->C] == 1u) return fail(ctx, MLMC_E_NOMEM, "a request's works need more tile slots than the workspace holds");
            if (stw[eng->C]) return fail(ctx, MLMC_E_DEVICE, "sweep engine: a work's level was not prepared");
            for (uint32_t s = 0; s < eng->C; ++s) {
                SlotRun& r = runs[s];
                if (r.state != 1) continue;
                const uint32_t w = stw[s];
                if ((w >> 16) != eng->generation[s]) continue;
                if (w & ENG_DONE) {
                    if (hipMemcpyAsync(eng->states_h + s, eng->P.states + s, sizeof(RunState), hipMemcpyDeviceToHost,
                                       eng->st) != hipSuccess ||
                        hipEventRecord(r.ev, eng->st) != hipSuccess)
                        return fail(ctx, MLMC_E_DEVICE, "state download failed");
                    r.state = 2;
                } else if (w & ENG_WAIT_LEVEL) {
                    mlmc_status st2 = eng->stage_more_levels(u, s, r.prob, r.rc.nested != 0, (w >> 8) & 0xFFu);
                    if (st2 != MLMC_OK) return st2;
                    eng->stage_levels_ready(u, s, eng->meta_h[s].c3);
                }
            }
        }
    }
    mlmc_status st2 = eng->flush(u);
    if (st2 != MLMC_OK) return st2;
    bool freed = false;
    for (uint32_t s = 0; s < eng->C; ++s) {
        SlotRun& r = runs[s];
        if (r.state != 2) continue;
        const hipError_t q = hipEventQuery(r.ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(ctx, MLMC_E_DEVICE, std::string("state download: ") + hipGetErrorString(q));
        mlmc_result res;
        result_of_state(eng->states_h[s], r.prob, r.rc, now_seconds() - r.t_submit, res);
        std::lock_guard<std::mutex> lk(m);
        publish(r.ticket, res);
        stats.requests_done += 1;
        free_slots.push_back(s);
        r.state = 0;
        freed = true;
    }
    if (freed) {
        std::lock_guard<std::mutex> lk(m);
        cv.notify_all();
        progressed = true;
    }
    return MLMC_OK;
}

void Server::loop_engine() {
    for (;;) {
        bool running = false;
        for (const SlotRun& r : runs) running = running || r.state != 0;
        {
            std::unique_lock<std::mutex> lk(m);
            if (!running && eng_in_flight == 0)
                cv.wait(lk, [&] { return stop || !queue.empty(); });
            if (stop) {
                for (auto& q : queue) {
                    mlmc_result r;
                    std::memset(&r, 0, sizeof(r));
                    r.struct_size = sizeof(r);
                    r.status = MLMC_E_BUSY;
                    publish(q.ticket, r);
                }
                queue.clear();
                cv.notify_all();
                if (!running && eng_in_flight == 0) return;
            }
        }
        bool progressed = false;
        const double t0 = now_seconds();
        mlmc_status s = engine_admit(progressed);
        if (s != MLMC_OK && s != MLMC_PENDING) { fail_all(s); return; }
        const double t1 = now_seconds();
        running = false;
        for (const SlotRun& r : runs) running = running || r.state == 1;
        if (running && eng_in_flight < 2) {
            if ((s = eng->replay(static_cast<int>(eng_launched & 1u))) != MLMC_OK) { fail_all(s); return; }
            eng_launched += 1;
            eng_in_flight += 1;
            progressed = true;
        }
        const double t2 = now_seconds();
        if ((s = engine_land(progressed)) != MLMC_OK) { fail_all(s); return; }
        const double t3 = now_seconds();
        {
            std::lock_guard<std::mutex> lk(m);
            stats.plan_seconds += (t1 - t0) + (t2 - t1);
            stats.land_seconds += t3 - t2;
            stats.flights = eng_launched;
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(m);
            cv.wait_for(lk, std::chrono::microseconds(20),
                        [&] { return stop || (!queue.empty() && !free_slots.empty()); });
            stats.idle_seconds += now_seconds() - t3;
        }
    }
}
}  // namespace mlmc

mlmc_context::mlmc_context() = default;
mlmc_context::~mlmc_context() = default;

using namespace mlmc;

extern "C" {

mlmc_status mlmc_server_start(mlmc_context* ctx, const mlmc_server_config* cfg) {
    if (!ctx || !cfg) return MLMC_E_INVALID;
    if (cfg->struct_size != sizeof(mlmc_server_config)) return fail(ctx, MLMC_E_VERSION, "mlmc_server_config.struct_size mismatch");
    if (ctx->server) return fail(ctx, MLMC_E_BUSY, "server already running");
    if (cfg->max_active < 1) return fail(ctx, MLMC_E_INVALID, "max_active must be >= 1");
    if (cfg->run.L_max < 0 || cfg->run.L_max >= MLMC_MAX_LEVELS) return fail(ctx, MLMC_E_INVALID, "L_max out of range");
    auto srv = std::make_unique<Server>();
    srv->ctx = ctx;
    srv->cfg = *cfg;
    bool engine = false;
    if (ctx->driver == MLMC_DRIVER_ENGINE) {
        const mlmc_status s = srv->engine_start();
        if (s == MLMC_OK) engine = true;
        else if (s != MLMC_E_NOMEM) return s;
        else srv->eng.reset();               // a workspace too small: host-planned flights
    }
    if (!engine) {
        srv->n_slots = cfg->max_active;
        for (uint32_t i = srv->n_slots; i-- > 0;) srv->free_slots.push_back(i);
    }
    Server* raw = srv.get();
    ctx->server = std::move(srv);
    ctx->ws_held = engine;
    if (engine) raw->th = std::thread([raw] { raw->loop_engine(); });
    else raw->th = std::thread([raw] { raw->loop(); });
    return MLMC_OK;
}

mlmc_status mlmc_submit(mlmc_context* ctx, const mlmc_request* req, uint64_t* ticket) {
    if (!ctx || !req || !ticket) return MLMC_E_INVALID;
    Server* srv = ctx->server.get();
    if (!srv) return MLMC_E_BUSY;
    if (req->struct_size != sizeof(mlmc_request)) return MLMC_E_VERSION;
    mlmc_run_config rc = srv->cfg.run;
    rc.eps = req->eps;
    rc.nested = req->nested;
    std::string err;
    const mlmc_status s = validate_run(&req->problem, &rc, err);
    if (s != MLMC_OK) return s;
    std::lock_guard<std::mutex> lk(srv->m);
    if (srv->stop) return MLMC_E_BUSY;
    if (srv->error != MLMC_OK) return srv->error;
    *ticket = srv->next_ticket++;
    srv->queue.push_back(Server::Queued{*ticket, *req, now_seconds()});
    srv->cv.notify_all();
    return MLMC_OK;
}

mlmc_status mlmc_poll(mlmc_context* ctx, uint64_t ticket, mlmc_result* out) {
    if (!ctx || !out) return MLMC_E_INVALID;
    Server* srv = ctx->server.get();
    if (!srv) return MLMC_E_BUSY;
    std::lock_guard<std::mutex> lk(srv->m);
    auto it = srv->done.find(ticket);
    if (it != srv->done.end()) {
        *out = it->second;
        srv->done.erase(it);
        return out->status == MLMC_OK ? MLMC_OK : static_cast<mlmc_status>(out->status);
    }
    for (auto& q : srv->queue) if (q.ticket == ticket) return MLMC_PENDING;
    for (auto& a : srv->active) if (a->ticket == ticket) return MLMC_PENDING;
    for (auto& r : srv->runs) if (r.state != 0 && r.ticket == ticket) return MLMC_PENDING;
    return MLMC_E_UNKNOWN_TICKET;
}

mlmc_status mlmc_poll_done(mlmc_context* ctx, uint32_t max, uint64_t* tickets, mlmc_result* out,
                           uint32_t* n) {
    if (!ctx || !n || (max && (!tickets || !out))) return MLMC_E_INVALID;
    *n = 0;
    Server* srv = ctx->server.get();
    if (!srv) return MLMC_E_BUSY;
    std::lock_guard<std::mutex> lk(srv->m);
    while (*n < max && !srv->done_order.empty()) {
        const uint64_t t = srv->done_order.front();
        srv->done_order.pop_front();
        auto it = srv->done.find(t);
        if (it == srv->done.end()) continue;        // taken by mlmc_poll
        tickets[*n] = t;
        out[*n] = it->second;
        srv->done.erase(it);
        *n += 1;
    }
    return MLMC_OK;
}

mlmc_status mlmc_server_stats_get(mlmc_context* ctx, mlmc_server_stats* out) {
    if (!ctx || !out) return MLMC_E_INVALID;
    if (out->struct_size != sizeof(mlmc_server_stats)) return MLMC_E_VERSION;
    Server* srv = ctx->server.get();
    if (!srv) return MLMC_E_BUSY;
    std::lock_guard<std::mutex> lk(srv->m);
    *out = srv->stats;
    out->struct_size = sizeof(mlmc_server_stats);
    out->queued = srv->queue.size();
    out->active = srv->active.size();
    for (auto& r : srv->runs) out->active += r.state != 0 ? 1 : 0;
    out->slots = srv->n_slots;
    out->bytes_per_request = srv->slot_bytes;
    out->engine = srv->eng ? 1 : 0;
    return MLMC_OK;
}

mlmc_status mlmc_server_stop(mlmc_context* ctx) {
    if (!ctx) return MLMC_E_INVALID;
    Server* srv = ctx->server.get();
    if (!srv) return MLMC_OK;
    {
        std::lock_guard<std::mutex> lk(srv->m);
        srv->stop = true;
        srv->cv.notify_all();
    }
    if (srv->th.joinable()) srv->th.join();
    ctx->server.reset();
    ctx->ws_held = false;
    return MLMC_OK;
}

}  // extern "C"
