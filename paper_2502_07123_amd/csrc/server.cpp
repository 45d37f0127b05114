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
                if (hipEventQuery(it->done) == hipErrorNotReady) return MLMC_OK;
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
            slot_accumulate(a->run.sums[p.level][p.est], res[k]);
            a->run.path_steps += p.n << p.level;
            if (std::find(seen.begin(), seen.end(), a) == seen.end()) {
                seen.push_back(a);
                a->run.sweeps += 1;
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
                if (a->in_flight || a->run.done) continue;
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
                    w.path_begin = o.sums[p.level][p.est].n;
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
                retired = retired || o.done;
            }
            if (retired) {
                std::lock_guard<std::mutex> lk(m);
                for (auto it = active.begin(); it != active.end();) {
                    if ((*it)->run.done) {
                        OptionRun& o = (*it)->run;
                        o.saturations = 0;
                        for (auto& l : o.sums) for (auto& x : l) o.saturations += x.sat;
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
    srv->n_slots = cfg->max_active;
    for (uint32_t i = srv->n_slots; i-- > 0;) srv->free_slots.push_back(i);
    Server* raw = srv.get();
    ctx->server = std::move(srv);
    raw->th = std::thread([raw] { raw->loop(); });
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
    return MLMC_OK;
}

}  // extern "C"
