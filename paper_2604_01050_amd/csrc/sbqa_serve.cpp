// Serving loop of the SBQA library: continuous batching of many Ising
// instances on one GPU.
//
// A scheduler thread owns every device call. Requests queue in arrival order;
// the head of the queue is admitted as soon as a slot is free and its device
// footprint fits the remaining budget. Every resident instance then advances
// in step blocks of STEP_BLOCK steps on its slot's own stream, so the kernels
// of different instances overlap on the device; at each block boundary the
// finished instances are read out (best over replicas, Sec. II.B), retired,
// and queued requests take their place. Each instance runs exactly the
// kernels it would run alone, so its result does not depend on the mix.
#include "sbqa_ctx.h"

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

using namespace sbqa;

namespace {

constexpr uint32_t STEP_BLOCK = 64;
typedef std::chrono::steady_clock Clock;

struct Request {
    uint64_t ticket = 0;
    int32_t N = 0, R = 0, runs = 0;
    sbqa_schedule s{};
    std::vector<double> dense, val, h, beta, alpha;
    std::vector<int32_t> row_ptr, col;
    std::vector<float> jp_table;
    InstanceFacts facts;
    size_t bytes = 0;
    Clock::time_point t_submit;
};

struct Result {
    sbqa_status status = SBQA_EAGAIN;
    std::string error;
    std::vector<double> energies;
    std::vector<int8_t> spins;
    double latency_s = 0.0;
};

struct Slot {
    std::unique_ptr<Request> req;
    sbqa_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct sbqa_server {
    size_t budget = 0;
    int32_t max_slots = 0;
    int device = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<Request>> queue;
    std::map<uint64_t, Result> results;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    std::vector<hipStream_t> streams;
    // stats (guarded by mu)
    uint64_t completed = 0;
    double updates = 0.0;
    double busy_s = 0.0;
};

static void finish(sbqa_server *srv, Slot &sl, sbqa_status st, const char *msg) {
    Result res;
    res.status = st;
    if (st == SBQA_OK) {
        res.energies.resize(sl.req->runs);
        res.spins.resize((size_t)sl.req->runs * sl.req->N);
        sbqa_status b = ctx_best(sl.ctx, res.energies.data(), res.spins.data());
        if (b != SBQA_OK) {
            res.status = b;
            res.error = last_error();
        }
    } else {
        res.error = msg ? msg : "";
    }
    res.latency_s = std::chrono::duration<double>(Clock::now() - sl.req->t_submit).count();
    if (sl.ctx) sbqa_destroy(sl.ctx);
    sl.ctx = nullptr;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (res.status == SBQA_OK) {
        srv->completed += 1;
        srv->updates += (double)sl.req->N * sl.req->R * sl.req->runs * sl.req->s.steps;
    }
    srv->results[sl.req->ticket] = std::move(res);
}

static void scheduler(sbqa_server *srv) {
    (void)hipSetDevice(srv->device);
    std::vector<Slot> slots(srv->max_slots);
    for (int q = 0; q < srv->max_slots; ++q) slots[q].stream = srv->streams[q];
    size_t used = 0;
    int resident = 0;
    for (;;) {
        // ---- admission (FIFO, budget and slots)
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            if (resident == 0) {
                srv->cv.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
                if (srv->stop && srv->queue.empty()) break;
            }
            if (srv->stop) srv->queue.clear();
            while (!srv->queue.empty() && resident < srv->max_slots && used + srv->queue.front()->bytes <= srv->budget) {
                std::unique_ptr<Request> rq = std::move(srv->queue.front());
                srv->queue.pop_front();
                int q = 0;
                while (slots[q].req) ++q;
                slots[q].req = std::move(rq);
                slots[q].bytes = slots[q].req->bytes;
                used += slots[q].bytes;
                ++resident;
            }
        }
        auto t0 = Clock::now();
        // ---- create newly admitted contexts
        for (Slot &sl : slots) {
            if (!sl.req || sl.ctx) continue;
            Request &r = *sl.req;
            sbqa_coupling J{};
            if (r.facts.dense) J.dense = r.dense.data();
            else {
                J.row_ptr = r.row_ptr.data();
                J.col = r.col.data();
                J.val = r.val.data();
                J.nnz = (int64_t)r.col.size();
            }
            sbqa_schedule s = r.s;
            s.beta = r.beta.empty() ? nullptr : r.beta.data();
            s.alpha = r.alpha.empty() ? nullptr : r.alpha.data();
            s.jp_table = r.jp_table.empty() ? nullptr : r.jp_table.data();
            sbqa_status st = ctx_create(&J, r.h.empty() ? nullptr : r.h.data(), r.N, r.R, r.runs, &s, r.facts, sl.stream,
                                        &sl.ctx, false);
            if (st != SBQA_OK) {
                sl.ctx = nullptr;
                finish(srv, sl, st, last_error());
                used -= sl.bytes;
                sl.req.reset();
                --resident;
                continue;
            }
            // free what the estimate did not cover
            r.dense.clear(); r.dense.shrink_to_fit();
        }
        // ---- one step block for every resident instance (overlapping streams)
        for (Slot &sl : slots) {
            if (!sl.ctx) continue;
            const uint32_t left = sl.ctx->s.steps - sl.ctx->step;
            const uint32_t n = left < STEP_BLOCK ? left : STEP_BLOCK;
            sbqa_status st = ctx_step(sl.ctx, n);
            if (st != SBQA_OK) {
                finish(srv, sl, st, last_error());
                used -= sl.bytes;
                sl.req.reset();
                --resident;
            }
        }
        // ---- retire finished instances
        for (Slot &sl : slots) {
            if (!sl.ctx || sl.ctx->step < sl.ctx->s.steps) continue;
            finish(srv, sl, SBQA_OK, nullptr);
            used -= sl.bytes;
            sl.req.reset();
            --resident;
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->busy_s += std::chrono::duration<double>(Clock::now() - t0).count();
        }
    }
    for (Slot &sl : slots)
        if (sl.ctx) sbqa_destroy(sl.ctx);
}

extern "C" {

sbqa_status sbqa_server_create(size_t hbm_budget_bytes, int32_t max_slots, sbqa_server **out) {
    clear_error();
    if (!out) return fail(SBQA_EINVAL, "out must be non-NULL");
    *out = nullptr;
    if (hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 1024) return fail(SBQA_EINVAL, "need budget > 0 and 1 <= max_slots <= 1024");
    sbqa_server *srv = new (std::nothrow) sbqa_server();
    if (!srv) return fail(SBQA_ENOMEM, "out of host memory");
    srv->budget = hbm_budget_bytes;
    srv->max_slots = max_slots;
    hipError_t e = hipGetDevice(&srv->device);
    if (e != hipSuccess) { delete srv; return fail(SBQA_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)); }
    for (int q = 0; q < max_slots; ++q) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t x : srv->streams) (void)hipStreamDestroy(x);
            delete srv;
            return fail(SBQA_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        srv->streams.push_back(st);
    }
    srv->worker = std::thread(scheduler, srv);
    *out = srv;
    return SBQA_OK;
}

sbqa_status sbqa_submit(sbqa_server *srv, const sbqa_coupling *J, const double *h, int32_t N, int32_t R, int32_t runs,
                        const sbqa_schedule *s, uint64_t *ticket) {
    clear_error();
    const Clock::time_point t_arrival = Clock::now();   // latency includes validation and copies
    if (!srv || !ticket) return fail(SBQA_EINVAL, "NULL argument");
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return fail(SBQA_ENOMEM, "out of host memory");
    sbqa_status st = validate_instance(J, h, N, R, runs, s, &r->facts);
    if (st != SBQA_OK) return st;
    r->bytes = instance_bytes(N, R, runs, r->facts, s->steps);
    if (r->bytes > srv->budget)
        return fail(SBQA_EBUDGET, "instance needs %zu device bytes, budget is %zu", r->bytes, srv->budget);
    r->N = N;
    r->R = R;
    r->runs = runs;
    r->s = *s;
    if (J->dense) r->dense.assign(J->dense, J->dense + (size_t)N * N);
    else {
        r->row_ptr.assign(J->row_ptr, J->row_ptr + N + 1);
        r->col.assign(J->col, J->col + J->nnz);
        r->val.assign(J->val, J->val + J->nnz);
    }
    if (h) r->h.assign(h, h + N);
    if (s->beta) r->beta.assign(s->beta, s->beta + runs);
    if (s->alpha) r->alpha.assign(s->alpha, s->alpha + runs);
    if (s->jp_kind == SBQA_JP_TABLE) r->jp_table.assign(s->jp_table, s->jp_table + (size_t)runs * s->steps);
    r->t_submit = t_arrival;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return fail(SBQA_ESTATE, "server is shutting down");
        r->ticket = srv->next_ticket++;
        *ticket = r->ticket;
        srv->results[r->ticket] = Result();
        srv->queue.push_back(std::move(r));
    }
    srv->cv.notify_one();
    return SBQA_OK;
}

sbqa_status sbqa_poll(sbqa_server *srv, uint64_t ticket, double *energies, int8_t *spins, double *latency_s) {
    clear_error();
    if (!srv) return fail(SBQA_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->results.find(ticket);
    if (it == srv->results.end()) return fail(SBQA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Result &res = it->second;
    if (res.status == SBQA_EAGAIN) return SBQA_EAGAIN;
    if (res.status != SBQA_OK) {
        sbqa_status st = fail(res.status, "%s", res.error.c_str());
        srv->results.erase(it);
        return st;
    }
    if (energies) std::memcpy(energies, res.energies.data(), sizeof(double) * res.energies.size());
    if (spins) std::memcpy(spins, res.spins.data(), res.spins.size());
    if (latency_s) *latency_s = res.latency_s;
    srv->results.erase(it);
    return SBQA_OK;
}

sbqa_status sbqa_server_stats(sbqa_server *srv, uint64_t *completed, double *updates, double *busy_s) {
    clear_error();
    if (!srv) return fail(SBQA_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (completed) *completed = srv->completed;
    if (updates) *updates = srv->updates;
    if (busy_s) *busy_s = srv->busy_s;
    return SBQA_OK;
}

void sbqa_server_destroy(sbqa_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (hipStream_t st : srv->streams) (void)hipStreamDestroy(st);
    delete srv;
}

}  // extern "C"
