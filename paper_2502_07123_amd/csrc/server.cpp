// Continuous-batching server: a scheduler thread owns the device work of all
// admitted requests.  Each iteration (a sweep) admits queued requests while fewer
// than max_active are active, asks every active request for its pending
// samples (pilot, allocation top-up or a new level -- the adaptive driver of
// Sections 2.1/2.2/6), runs all of them as one launch sequence, and retires the
// requests that converged.  Requests submitted meanwhile join the next sweep.
// Each request's sums are its own (added on the host in a fixed order) and its
// uniforms depend only on (seed, option_id, level, estimator, path), so its
// result does not depend on what else is in flight.
#include <algorithm>
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
        double t_submit;
        uint32_t slot;
        OptionRun run;
    };
    std::deque<Queued> queue;
    std::vector<std::unique_ptr<Active>> active;
    std::map<uint64_t, mlmc_result> done;
    std::vector<uint32_t> free_slots;
    uint32_t n_slots = 0;
    mlmc_status error = MLMC_OK;
    std::string error_msg;

    void loop();
};

void Server::loop() {
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(m);
            cv.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop && queue.empty() && active.empty()) return;
            while (!queue.empty() && !free_slots.empty()) {
                Queued q = queue.front();
                queue.pop_front();
                auto a = std::make_unique<Active>();
                a->ticket = q.ticket;
                a->t_submit = q.t_submit;
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
        std::vector<OptionRun*> runs;
        for (auto& a : active) runs.push_back(&a->run);
        // one sweep: every active request's pending work in one launch sequence
        bool ran = false;
        const mlmc_status s = sweep_once(ctx, runs, ran);
        if (s != MLMC_OK) {
            std::lock_guard<std::mutex> lk(m);
            error = s;
            error_msg = ctx->err;
            for (auto& a : active) {
                mlmc_result r;
                option_result(a->run, r);
                r.status = s;
                done[a->ticket] = r;
            }
            active.clear();
            for (auto& q : queue) {
                mlmc_result r;
                std::memset(&r, 0, sizeof(r));
                r.struct_size = sizeof(r);
                r.status = s;
                done[q.ticket] = r;
            }
            queue.clear();
            cv.notify_all();
            return;
        }
        std::lock_guard<std::mutex> lk(m);
        for (auto it = active.begin(); it != active.end();) {
            if ((*it)->run.done) {
                OptionRun& o = (*it)->run;
                o.saturations = 0;
                for (auto& a : o.sums) for (auto& s : a) o.saturations += s.sat;
                mlmc_result r;
                option_result(o, r);
                done[(*it)->ticket] = r;
                free_slots.push_back((*it)->slot);
                it = active.erase(it);
            } else {
                ++it;
            }
        }
        cv.notify_all();
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
    // requests' sums are kept on the host; a sweep whose plan does not fit the
    // workspace runs in parts
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
