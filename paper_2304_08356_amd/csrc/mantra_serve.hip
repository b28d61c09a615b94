// Serving scheduler: continuous batching of the progressive-sampling rounds of
// many requests over one resident graph.
//
// One scheduler thread per graph.  Each pass of its loop admits queued
// requests (FIFO) while the device memory their accumulators need fits the
// budget and the active count is below the limit, gives every active request
// a slice of the pairs of its current phase, runs all slices in ONE sweep
// launch, and then advances each request's state machine: the phase
// reductions and the bound checks of Algorithm 1 run per request, and a
// request that stops leaves the active set at once, so the next pass can
// admit the requests waiting behind it.  A request's pairs, signs and phases
// are functions of its own seed, so its results do not depend on what it
// shares launches with (up to the order of floating-point atomic additions).

#include "mantra_int.h"

namespace mantra {

struct Ticket {
    uint64_t id = 0;
    ReqRun run;
    bool done = false;
    int rc = MANTRA_OK;
    std::string err;
    mantra_result res;
};

struct ServeState {
    std::mutex mu;  // queue, budget, limits, stop
    std::condition_variable cv;
    std::deque<std::shared_ptr<Ticket>> queue;
    size_t budget = 0, used = 0;
    int max_active = 64;
    bool stop = false;
    bool trace = false;  // one stderr line per shared launch (MANTRA_SERVE_TRACE set)
    std::thread th;
};

// tickets outlive nothing but the registry: mantra_poll takes only the id
static std::mutex g_tmu;
static std::condition_variable g_tcv;
static std::map<uint64_t, std::shared_ptr<Ticket>> g_tickets;
static uint64_t g_next_ticket = 1;

static void complete(const std::shared_ptr<Ticket> &t, int rc, const mantra_result &res) {
    std::lock_guard<std::mutex> lk(g_tmu);
    t->rc = rc;
    t->res = res;
    t->res.status = rc;
    // the result names the request's output buffers, filled or not
    t->res.node_bc = t->run.rq.node_bc;
    t->res.edge_bc = (t->run.rq.flags & MANTRA_F_EDGE_BC) ? t->run.rq.edge_bc : nullptr;
    if (rc < 0) t->err = !t->run.err.empty() ? t->run.err : g_err;
    t->done = true;
    g_tcv.notify_all();
}

static size_t default_budget(const mantra_graph *g) { return serve_sums_budget(g); }

// pairs a request may put into one shared launch
static int64_t slice_quota(mantra_graph *g, size_t nactive) {
    const int64_t per_launch = std::max<int64_t>(4 * (int64_t)auto_slabs(g), 1024);
    return std::max<int64_t>(per_launch / (int64_t)std::max<size_t>(nactive, 1), 256);
}

static void serve_loop(mantra_graph *g) {
    ServeState &S = *g->serve;
    std::vector<std::shared_ptr<Ticket>> act;
    for (;;) {
        std::vector<std::shared_ptr<Ticket>> fresh;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait(lk, [&] { return S.stop || !S.queue.empty() || !act.empty(); });
            if (S.stop) break;
            while (!S.queue.empty() && (int)act.size() < S.max_active) {
                std::shared_ptr<Ticket> t = S.queue.front();
                if (S.used + t->run.mem_bytes > S.budget) {
                    if (!act.empty()) break;  // wait for memory to free up
                    // the budget was lowered below what this request needs
                    S.queue.pop_front();
                    mantra_result r;
                    memset(&r, 0, sizeof r);
                    complete(t, fail(MANTRA_E_TOO_LARGE, "request needs %zu device bytes, budget %zu",
                                     t->run.mem_bytes, S.budget), r);
                    continue;
                }
                S.queue.pop_front();
                S.used += t->run.mem_bytes;
                act.push_back(t);
                fresh.push_back(t);
            }
        }
        std::vector<std::shared_ptr<Ticket>> finished;
        {
            std::lock_guard<std::mutex> glk(g->mu);
            hipSetDevice(g->device);
            for (auto &t : fresh) {
                t->run.rc = req_begin(g, t->run);
                if (t->run.rc) { t->run.err = g_err; finished.push_back(t); }
            }
            // one launch over a slice of every active request (one per
            // estimator in use: each has a kernel of its own)
            LaunchSpec sps[3];
            std::vector<std::shared_ptr<Ticket>> ins[3];
            const int64_t quota = slice_quota(g, act.size());
            for (auto &t : act) {
                if (t->run.rc || t->run.phase == ReqRun::DONE) continue;
                const int64_t cnt = std::min(req_pending(t->run), quota);
                if (cnt <= 0) continue;
                const int mi = (t->run.rq.flags & MANTRA_F_RTB) ? 2 : (t->run.rq.flags & MANTRA_F_TRK) ? 1 : 0;
                sps[mi].reqs.push_back(req_slice(t->run, cnt, sps[mi].npairs));
                sps[mi].npairs += cnt;
                ins[mi].push_back(t);
            }
            for (int mi = 0; mi < 3; ++mi) {
                LaunchSpec &sp = sps[mi];
                if (sp.npairs <= 0) continue;
                sp.mode = mi == 2 ? MODE_RTB : mi == 1 ? MODE_TRK : MODE_PAIRS;
                SweepOut o;
                int rc = run_sweep(g, sp, o);
                const std::string launch_err = rc ? g_err : std::string();
                if (S.trace)
                    fprintf(stderr, "serve: launch of %lld pairs from %zu requests, %.1f ms (%d launches, %llu pairs "
                                    "re-run for arc room), rc %d, %zu active\n",
                            (long long)sp.npairs, ins[mi].size(), o.ms, o.launches, (unsigned long long)o.st[5], rc,
                            act.size());
                for (auto &t : ins[mi]) {
                    t->run.R.gpu_ms += o.ms;
                    if (rc) { t->run.rc = rc; t->run.err = launch_err; continue; }
                    t->run.rc = req_advance(g, t->run);
                    if (t->run.rc) t->run.err = g_err;
                }
            }
            for (auto &t : act)
                if ((t->run.rc || t->run.phase == ReqRun::DONE) &&
                    std::find(finished.begin(), finished.end(), t) == finished.end())
                    finished.push_back(t);
            for (auto &t : finished) {
                mantra_result r;
                int rc = req_finish(g, t->run, &r);
                complete(t, rc, r);
            }
        }
        if (!finished.empty()) {
            std::lock_guard<std::mutex> lk(S.mu);
            for (auto &t : finished) {
                S.used -= std::min(S.used, t->run.mem_bytes);
                act.erase(std::remove(act.begin(), act.end(), t), act.end());
            }
        }
    }
    // stopping: every request still held fails
    std::lock_guard<std::mutex> glk(g->mu);
    for (auto &t : act) {
        req_release(t->run);
        mantra_result r;
        memset(&r, 0, sizeof r);
        complete(t, fail(MANTRA_E_INTERNAL, "graph destroyed before the request finished"), r);
    }
}

static int serve_start(mantra_graph *g) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (g->serve) return MANTRA_OK;
    std::unique_ptr<ServeState> S(new ServeState());
    S->budget = default_budget(g);
    S->trace = getenv("MANTRA_SERVE_TRACE") != nullptr;
    g->serve = S.release();
    try {
        g->serve->th = std::thread(serve_loop, g);
    } catch (...) {
        delete g->serve;
        g->serve = nullptr;
        return fail(MANTRA_E_INTERNAL, "could not start the scheduler thread");
    }
    return MANTRA_OK;
}

// queued and active requests finish with MANTRA_E_INTERNAL
void serve_stop(mantra_graph *g) {
    if (!g) return;
    ServeState *S = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        S = g->serve;
    }
    if (!S) return;
    std::deque<std::shared_ptr<Ticket>> left;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        left.swap(S->queue);
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    for (auto &t : left) {
        mantra_result r;
        memset(&r, 0, sizeof r);
        complete(t, fail(MANTRA_E_INTERNAL, "graph destroyed before the request was admitted"), r);
    }
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        g->serve = nullptr;
    }
    delete S;
}

}  // namespace mantra

using namespace mantra;

extern "C" {

int mantra_serve_config(mantra_graph *g, uint64_t mem_budget_bytes, int32_t max_active) {
    if (!g) return fail(MANTRA_E_INVALID, "graph is NULL");
    if (max_active < 0) return fail(MANTRA_E_INVALID, "max_active < 0");
    int rc = serve_start(g);
    if (rc) return rc;
    ServeState &S = *g->serve;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.budget = mem_budget_bytes ? (size_t)mem_budget_bytes : default_budget(g);
        S.max_active = max_active ? max_active : 64;
    }
    S.cv.notify_all();
    return MANTRA_OK;
}

int mantra_submit(mantra_graph *g, const mantra_request *req, uint64_t *ticket) {
    if (!g || !req || !ticket) return fail(MANTRA_E_INVALID, "graph, request or ticket is NULL");
    *ticket = 0;
    int rc = serve_start(g);
    if (rc) return rc;
    // reject now what can never run
    rc = check_request(g, *req);
    if (rc) return rc;
    std::shared_ptr<Ticket> t(new Ticket());
    t->run.rq = *req;
    t->run.mem_bytes = req_mem_bytes(g, *req);
    t->run.t_start = std::chrono::steady_clock::now();
    ServeState &S = *g->serve;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        if (t->run.mem_bytes > S.budget)
            return fail(MANTRA_E_TOO_LARGE, "request needs %zu device bytes, the serving budget is %zu",
                        t->run.mem_bytes, S.budget);
        {
            std::lock_guard<std::mutex> tl(g_tmu);
            t->id = g_next_ticket++;
            g_tickets[t->id] = t;
        }
        S.queue.push_back(t);
    }
    S.cv.notify_all();
    *ticket = t->id;
    return MANTRA_OK;
}

int mantra_poll(uint64_t ticket, mantra_result *out, int32_t timeout_ms) {
    std::unique_lock<std::mutex> lk(g_tmu);
    auto it = g_tickets.find(ticket);
    if (it == g_tickets.end()) return fail(MANTRA_E_INVALID, "unknown or consumed ticket %llu", (unsigned long long)ticket);
    std::shared_ptr<Ticket> t = it->second;
    auto ready = [&] { return t->done; };
    if (timeout_ms < 0) g_tcv.wait(lk, ready);
    else if (timeout_ms > 0) g_tcv.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    if (!t->done) return MANTRA_PENDING;
    g_tickets.erase(ticket);
    if (out) *out = t->res;
    if (t->rc < 0) g_err = t->err;
    return t->rc;
}

}  // extern "C"
