// Serving loop of the SBQA library: continuous batching of many Ising
// instances on one GPU.
//
// A scheduler thread owns every device call. Requests queue in arrival order;
// the head of the queue is admitted as soon as a slot is free and its device
// footprint fits the remaining budget. All resident instances then advance
// together in step blocks of up to STEP_BLOCK steps: every step is one
// grouped launch per kernel specialisation (dense path x m-blocks per wave,
// CSR ballistic x ring by lane reads), a grid-stride loop over the workgroups
// of all instances of the group, driven by a device task table that the
// scheduler rewrites between blocks. Each instance runs exactly the
// workgroups its standalone kernel would run, so its result does not depend
// on the mix. At block boundaries finished instances are read out (best over
// replicas, Sec. II.B) and retired, tracked energies are evaluated, and queued
// requests take their place. A finished instance's readout is enqueued behind
// the block that finished it and collected once an event says it is done (the
// next blocks are queued meanwhile), and its context is released without
// waiting on the server stream, so retirements do not drain the GPU.
#include "sbqa_ctx.h"

#include <algorithm>
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
// Task-table groups: 21 dense (7 contraction paths x m-blocks per wave
// 1/2/4) and 4 CSR (ballistic x ring by lane reads).
constexpr Path DENSE_PATHS[7] = {PATH_F32, PATH_FP8, PATH_BF16X3, PATH_I8, PATH_FP8PK, PATH_FP4, PATH_FP4PK};
constexpr int NDENSE_GROUPS = 21;
constexpr int NGROUPS = NDENSE_GROUPS + 4;
constexpr int DENSE_GRID_CAP = 512;   // workgroups of one grouped dense launch at most
// Groups present in a step block run as parallel branches (one side stream
// each, forked from and joined to the server stream): they touch disjoint
// instances, so the GPU may overlap them.
constexpr int NBRANCH = 4;
constexpr int CSR_GRID_CAP = 2048;
typedef std::chrono::steady_clock Clock;

int group_of(const sbqa_ctx *c) {
    if (c->facts.path == PATH_CSR)
        return NDENSE_GROUPS + 2 * (c->s.fmode == SBQA_F_BALLISTIC ? 1 : 0) + (csr_ring_shfl(c->R) ? 1 : 0);
    const int mi = c->L.mbw == 1 ? 0 : c->L.mbw == 2 ? 1 : 2;
    int pi = 0;
    while (DENSE_PATHS[pi] != c->facts.path) ++pi;
    return pi * 3 + mi;
}

// Table entry of context c for steps [c->step, n_end).
GroupTask make_task(const sbqa_ctx *c, int first_block, uint32_t n_end) {
    GroupTask t;
    std::memset(&t, 0, sizeof t);
    const StepCoef k = step_coef(&c->s, c->c0, c->R, c->step);
    t.first_block = first_block;
    t.n_base = (int)c->step;
    t.n_end = (int)n_end;
    t.S = (int)c->s.steps;
    t.N = c->N;
    t.R = c->R;
    t.C = c->L.C;
    t.fmode = c->s.fmode;
    t.kB = k.kB;
    t.dt = k.dt;
    t.kD = k.kD;
    t.x[0] = c->x[0];
    t.x[1] = c->x[1];
    t.y = c->y;
    t.g[0] = c->g[0];
    t.g[1] = c->g[1];
    t.g_lo[0] = c->g_lo[0];
    t.g_lo[1] = c->g_lo[1];
    t.h = c->h32;
    t.jp = c->jp;
    t.coefA = c->coefA;
    t.delta = c->delta_tab;
    if (c->facts.path == PATH_CSR) {
        t.ld = c->L.Cs;
        t.nchunk = csr_step_chunks(c->L.C);
        t.nblocks = csr_step_blocks(c->N, c->L.C);
        t.row_ptr = c->rp;
        t.col = c->col;
        t.val = c->val;
        t.t3 = c->tri3();
    } else {
        t.ld = c->L.Np;
        t.nkc = c->L.nkc;
        t.nchunk = c->L.Np / DENSE_TN;
        t.nblocks = t.nchunk * (c->L.Cg / (64 * c->L.mbw));
        t.J = c->Jd;
        t.J_lo = c->Jd_lo;
    }
    return t;
}

#define HIP_CHECK_SERVE(expr)                                                                 \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(SBQA_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Request {
    uint64_t ticket = 0;
    int32_t N = 0, R = 0, runs = 0;
    sbqa_schedule s{};
    std::vector<double> dense, val, h, beta, alpha;
    std::vector<uint32_t> jbits;   // dense +-1 J on a bit-packed path: its sign bits instead of `dense`
    std::vector<int32_t> row_ptr, col, tri;
    std::vector<double> K;
    std::vector<float> jp_table;
    InstanceFacts facts;
    size_t bytes = 0;
    Clock::time_point t_submit;
    sbqa_status create_status = SBQA_OK;   // set by the creator thread on failure
    std::string error;
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
    size_t bytes = 0;
    bool retiring = false;      // readout enqueued, waiting for `done`
    hipEvent_t done = nullptr;  // recorded on the server stream behind the readout
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
    hipStream_t stream = nullptr;
    // context creation off the scheduler thread: admitted requests wait in
    // `create` until the creator thread has built their context (on its own
    // stream, so uploads overlap the grouped steps) and moved them to `ready`
    std::thread creator;
    hipStream_t create_stream = nullptr;
    std::deque<std::unique_ptr<Slot>> create, ready;   // guarded by mu
    std::condition_variable cv_create;
    bool stop_creator = false;   // set once the scheduler has drained all admitted work
    // task tables: pinned host copies (two, alternating between blocks) and the device table
    GroupTask *h_tasks[2] = {nullptr, nullptr};
    GroupHeader *h_hdr[2] = {nullptr, nullptr};
    hipEvent_t h_free[2] = {nullptr, nullptr};   // the copy out of host table q has completed
    GroupTask *d_tasks = nullptr;
    GroupHeader *d_hdr = nullptr;
    // full step blocks are replayed from HIP graphs, one per set of groups
    // present (the kernels read membership from the task table)
    std::map<uint32_t, hipGraphExec_t> graphs;
    hipStream_t side[NBRANCH] = {};
    hipEvent_t fork_ev = nullptr, join_ev[NBRANCH] = {};
    // stats (guarded by mu)
    uint64_t completed = 0;
    double updates = 0.0;
    double busy_s = 0.0;
};

static void record_result(sbqa_server *srv, Slot &sl, Result res) {
    res.latency_s = std::chrono::duration<double>(Clock::now() - sl.req->t_submit).count();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (res.status == SBQA_OK) {
        srv->completed += 1;
        srv->updates += (double)sl.req->N * sl.req->R * sl.req->runs * sl.req->s.steps;
    }
    srv->results[sl.req->ticket] = std::move(res);
}

// Enqueue the readout of a finished instance behind its last step block.
static sbqa_status begin_retire(sbqa_server *srv, Slot &sl) {
    if (!sl.done) HIP_CHECK_SERVE(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    const sbqa_status st = ctx_readout_async(sl.ctx);
    if (st != SBQA_OK) return st;
    HIP_CHECK_SERVE(hipEventRecord(sl.done, srv->stream));
    sl.retiring = true;
    return SBQA_OK;
}

// Its results once the readout has completed; the context's work is all
// done, so it is released without a stream synchronisation.
static void end_retire(sbqa_server *srv, Slot &sl) {
    Result res;
    res.status = SBQA_OK;
    res.energies.resize(sl.req->runs);
    res.spins.resize((size_t)sl.req->runs * sl.req->N);
    const sbqa_status b = ctx_readout_collect(sl.ctx, res.energies.data(), res.spins.data());
    if (b != SBQA_OK) {
        res.status = b;
        res.error = last_error();
    }
    delete sl.ctx;
    sl.ctx = nullptr;
    sl.retiring = false;
    record_result(srv, sl, std::move(res));
}

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
    if (sl.ctx) sbqa_destroy(sl.ctx);
    sl.ctx = nullptr;
    sl.retiring = false;
    record_result(srv, sl, std::move(res));
}

// One step block for every resident instance: rewrite the task table, then
// per step one grouped launch per group present. Returns the first failure.
static sbqa_status step_block(sbqa_server *srv, std::vector<Slot> &slots, int parity) {
    GroupTask *ht = srv->h_tasks[parity];
    GroupHeader *hh = srv->h_hdr[parity];
    HIP_CHECK_SERVE(hipEventSynchronize(srv->h_free[parity]));   // host table q no longer read by a copy
    int cnt[NGROUPS] = {0}, total[NGROUPS] = {0};
    uint32_t steps = 0;
    for (Slot &sl : slots) {
        sbqa_ctx *c = sl.ctx;
        if (!c || c->step >= c->s.steps) continue;
        uint32_t n_end = std::min(c->s.steps, c->step + STEP_BLOCK);
        if (c->s.energy_every) n_end = std::min(n_end, (c->step / c->s.energy_every + 1) * c->s.energy_every);
        const int g = group_of(c);
        ht[g * srv->max_slots + cnt[g]] = make_task(c, total[g], n_end);
        total[g] += ht[g * srv->max_slots + cnt[g]].nblocks;
        ++cnt[g];
        steps = std::max(steps, n_end - c->step);
    }
    if (!steps) return SBQA_OK;
    for (int g = 0; g < NGROUPS; ++g) hh[g] = GroupHeader{cnt[g], total[g]};
    HIP_CHECK_SERVE(hipMemcpyAsync(srv->d_hdr, hh, sizeof(GroupHeader) * NGROUPS, hipMemcpyHostToDevice, srv->stream));
    HIP_CHECK_SERVE(hipMemcpyAsync(srv->d_tasks, ht, sizeof(GroupTask) * NGROUPS * srv->max_slots,
                                   hipMemcpyHostToDevice, srv->stream));
    HIP_CHECK_SERVE(hipEventRecord(srv->h_free[parity], srv->stream));
    uint32_t mask = 0;
    for (int g = 0; g < NGROUPS; ++g)
        if (cnt[g]) mask |= 1u << g;
    // full grids (capped) inside graphs, so that a graph serves any membership;
    // the k-th group present runs on branch k % NBRANCH, its steps in order
    int present[NGROUPS], np = 0;
    for (int g = 0; g < NGROUPS; ++g)
        if (mask & (1u << g)) present[np++] = g;
    const int nb = std::min(np, NBRANCH);
    auto launch_all = [&](uint32_t nsteps, bool full_grid) -> sbqa_status {
        HIP_CHECK_SERVE(hipEventRecord(srv->fork_ev, srv->stream));
        for (int b = 0; b < nb; ++b) {
            hipStream_t bs = srv->side[b];
            HIP_CHECK_SERVE(hipStreamWaitEvent(bs, srv->fork_ev, 0));
            for (uint32_t off = 0; off < nsteps; ++off)
                for (int k = b; k < np; k += NBRANCH) {
                    const int g = present[k];
                    const GroupHeader *dh = srv->d_hdr + g;
                    const GroupTask *dt = srv->d_tasks + (size_t)g * srv->max_slots;
                    if (g < NDENSE_GROUPS) {
                        const int mbw = (g % 3 == 0) ? 1 : (g % 3 == 1) ? 2 : 4;
                        const int grid = full_grid ? DENSE_GRID_CAP : std::min(total[g], DENSE_GRID_CAP);
                        HIP_CHECK_SERVE(launch_group_dense(DENSE_PATHS[g / 3], mbw, dh, dt, grid, (int)off, bs));
                    } else {
                        const int q = g - NDENSE_GROUPS;
                        const int grid = full_grid ? CSR_GRID_CAP : std::min(total[g], CSR_GRID_CAP);
                        HIP_CHECK_SERVE(launch_group_csr(q >= 2, q & 1, dh, dt, grid, (int)off, bs));
                    }
                }
            HIP_CHECK_SERVE(hipEventRecord(srv->join_ev[b], bs));
            HIP_CHECK_SERVE(hipStreamWaitEvent(srv->stream, srv->join_ev[b], 0));
        }
        return SBQA_OK;
    };
    if (steps == STEP_BLOCK) {
        auto it = srv->graphs.find(mask);
        if (it == srv->graphs.end()) {
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            HIP_CHECK_SERVE(hipStreamBeginCapture(srv->stream, hipStreamCaptureModeThreadLocal));
            const sbqa_status st = launch_all(STEP_BLOCK, true);
            const hipError_t e = hipStreamEndCapture(srv->stream, &graph);
            if (st != SBQA_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            HIP_CHECK_SERVE(e);
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIP_CHECK_SERVE(ei);
            it = srv->graphs.emplace(mask, exec).first;
        }
        HIP_CHECK_SERVE(hipGraphLaunch(it->second, srv->stream));
    } else {
        const sbqa_status st = launch_all(steps, false);
        if (st != SBQA_OK) return st;
    }
    for (Slot &sl : slots) {
        sbqa_ctx *c = sl.ctx;
        if (!c || c->step >= c->s.steps) continue;
        uint32_t n_end = std::min(c->s.steps, c->step + STEP_BLOCK);
        if (c->s.energy_every) n_end = std::min(n_end, (c->step / c->s.energy_every + 1) * c->s.energy_every);
        c->step = n_end;
        c->cur = (int)(n_end & 1u);
        if (c->s.energy_every && c->step % c->s.energy_every == 0) {
            const sbqa_status st = ctx_evaluate(c);
            if (st != SBQA_OK) return st;
        }
    }
    return SBQA_OK;
}

// Creator thread: builds the contexts of admitted requests on its own stream
// and hands them to the scheduler once their device state is complete.
static void creator(sbqa_server *srv) {
    (void)hipSetDevice(srv->device);
    for (;;) {
        std::unique_ptr<Slot> sl;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv_create.wait(lk, [&] { return srv->stop_creator || !srv->create.empty(); });
            if (srv->create.empty()) break;
            sl = std::move(srv->create.front());
            srv->create.pop_front();
        }
        Request &r = *sl->req;
        sbqa_coupling J{};
        if (r.facts.dense) J.dense = r.dense.data();
        else {
            J.row_ptr = r.row_ptr.data();
            J.col = r.col.data();
            J.val = r.val.data();
            J.nnz = (int64_t)r.col.size();
            J.n3 = (int64_t)r.K.size();
            J.tri = r.tri.empty() ? nullptr : r.tri.data();
            J.K = r.K.empty() ? nullptr : r.K.data();
        }
        sbqa_schedule s = r.s;
        s.beta = r.beta.empty() ? nullptr : r.beta.data();
        s.alpha = r.alpha.empty() ? nullptr : r.alpha.data();
        s.jp_table = r.jp_table.empty() ? nullptr : r.jp_table.data();
        sbqa_status st = ctx_create(&J, r.h.empty() ? nullptr : r.h.data(), r.N, r.R, r.runs, &s, r.facts,
                                    srv->create_stream, &sl->ctx, false, r.jbits.empty() ? nullptr : r.jbits.data());
        if (st == SBQA_OK && hipStreamSynchronize(srv->create_stream) != hipSuccess)
            st = fail(SBQA_EDEVICE, "context set-up did not complete");
        if (st == SBQA_OK) {
            sl->ctx->stream = srv->stream;   // later work is ordered with the grouped steps
        } else {
            if (sl->ctx) sbqa_destroy(sl->ctx);
            sl->ctx = nullptr;
            r.error = last_error();
            r.create_status = st;
        }
        r.dense.clear();
        r.dense.shrink_to_fit();
        r.jbits.clear();
        r.jbits.shrink_to_fit();
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->ready.push_back(std::move(sl));
        }
        srv->cv.notify_one();
    }
}

static void scheduler(sbqa_server *srv) {
    (void)hipSetDevice(srv->device);
    std::vector<Slot> slots(srv->max_slots);
    size_t used = 0;
    int admitted = 0, active = 0, parity = 0;
    for (;;) {
        // ---- admission (FIFO, budget and slots) and hand-over of built contexts
        std::deque<std::unique_ptr<Slot>> got;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            if (active == 0) {
                srv->cv.wait(lk, [&] {
                    return srv->stop || !srv->ready.empty() ||
                           (!srv->queue.empty() && admitted < srv->max_slots &&
                            used + srv->queue.front()->bytes <= srv->budget);
                });
                if (srv->stop && srv->queue.empty() && admitted == 0) break;
            }
            if (srv->stop) srv->queue.clear();
            bool pushed = false;
            while (!srv->queue.empty() && admitted < srv->max_slots && used + srv->queue.front()->bytes <= srv->budget) {
                std::unique_ptr<Slot> sl(new Slot());
                sl->req = std::move(srv->queue.front());
                srv->queue.pop_front();
                sl->bytes = sl->req->bytes;
                used += sl->bytes;
                ++admitted;
                srv->create.push_back(std::move(sl));
                pushed = true;
            }
            if (pushed) srv->cv_create.notify_one();
            got.swap(srv->ready);
        }
        auto t0 = Clock::now();
        for (std::unique_ptr<Slot> &sp : got) {
            if (!sp->ctx) {
                finish(srv, *sp, sp->req->create_status, sp->req->error.c_str());
                used -= sp->bytes;
                --admitted;
                continue;
            }
            int q = 0;
            while (slots[q].req) ++q;
            const hipEvent_t ev = slots[q].done;   // the slot's event outlives its occupants
            slots[q] = std::move(*sp);
            slots[q].done = ev;
            ++active;
        }
        // ---- one step block for every resident instance (grouped launches)
        const sbqa_status st = step_block(srv, slots, parity);
        parity ^= 1;
        if (st != SBQA_OK) {
            const std::string msg = last_error();
            for (Slot &sl : slots) {
                if (!sl.req) continue;
                finish(srv, sl, st, msg.c_str());
                used -= sl.bytes;
                sl.req.reset();
                --admitted;
                --active;
            }
        }
        // ---- retire finished instances: readouts go behind the block just
        // queued; the ones whose readout has completed hand over their results
        bool running = false, waiting = false;
        for (Slot &sl : slots) {
            if (!sl.ctx) continue;
            if (sl.ctx->step < sl.ctx->s.steps) {
                running = true;
                continue;
            }
            if (!sl.retiring) {
                const sbqa_status rs = begin_retire(srv, sl);
                if (rs != SBQA_OK) {
                    const std::string msg = last_error();
                    finish(srv, sl, rs, msg.c_str());
                    used -= sl.bytes;
                    sl.req.reset();
                    --admitted;
                    --active;
                    continue;
                }
            }
            waiting = true;
        }
        if (waiting && !running) {
            // nothing else to queue: wait for the oldest readout instead of spinning
            for (Slot &sl : slots)
                if (sl.ctx && sl.retiring) {
                    (void)hipEventSynchronize(sl.done);
                    break;
                }
        }
        for (Slot &sl : slots) {
            if (!sl.ctx || !sl.retiring || hipEventQuery(sl.done) != hipSuccess) continue;
            end_retire(srv, sl);
            used -= sl.bytes;
            sl.req.reset();
            --admitted;
            --active;
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->busy_s += std::chrono::duration<double>(Clock::now() - t0).count();
        }
    }
    for (Slot &sl : slots) {
        if (sl.ctx) sbqa_destroy(sl.ctx);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
}

static void release(sbqa_server *srv) {
    if (srv->stream) (void)hipStreamSynchronize(srv->stream);
    for (auto &kv : srv->graphs) (void)hipGraphExecDestroy(kv.second);
    for (int q = 0; q < 2; ++q) {
        if (srv->h_tasks[q]) (void)hipHostFree(srv->h_tasks[q]);
        if (srv->h_hdr[q]) (void)hipHostFree(srv->h_hdr[q]);
        if (srv->h_free[q]) (void)hipEventDestroy(srv->h_free[q]);
    }
    if (srv->d_tasks) (void)hipFree(srv->d_tasks);
    if (srv->d_hdr) (void)hipFree(srv->d_hdr);
    for (int b = 0; b < NBRANCH; ++b) {
        if (srv->side[b]) (void)hipStreamSynchronize(srv->side[b]);
        if (srv->side[b]) (void)hipStreamDestroy(srv->side[b]);
        if (srv->join_ev[b]) (void)hipEventDestroy(srv->join_ev[b]);
    }
    if (srv->fork_ev) (void)hipEventDestroy(srv->fork_ev);
    if (srv->stream) (void)hipStreamDestroy(srv->stream);
    if (srv->create_stream) (void)hipStreamDestroy(srv->create_stream);
    delete srv;
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
    const size_t ntask = (size_t)NGROUPS * max_slots;
    e = hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&srv->create_stream, hipStreamNonBlocking);
    for (int b = 0; b < NBRANCH && e == hipSuccess; ++b) {
        e = hipStreamCreateWithFlags(&srv->side[b], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&srv->join_ev[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&srv->fork_ev, hipEventDisableTiming);
    for (int q = 0; q < 2 && e == hipSuccess; ++q) {
        e = hipHostMalloc((void **)&srv->h_tasks[q], sizeof(GroupTask) * ntask, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&srv->h_hdr[q], sizeof(GroupHeader) * NGROUPS, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&srv->h_free[q], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipMalloc(&srv->d_tasks, sizeof(GroupTask) * ntask);
    if (e == hipSuccess) e = hipMalloc(&srv->d_hdr, sizeof(GroupHeader) * NGROUPS);
    if (e != hipSuccess) {
        release(srv);
        return fail(e == hipErrorOutOfMemory ? SBQA_ENOMEM : SBQA_EDEVICE, "server set-up: %s", hipGetErrorString(e));
    }
    srv->worker = std::thread(scheduler, srv);
    srv->creator = std::thread(creator, srv);
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
    // dense +-1 couplings on a bit-packed path travel as sign bits (N^2/8
    // bytes instead of N^2 float64) and keep no float64 copy on the device
    if (J->dense && r->facts.pm1 && path_packed(r->facts.path)) r->facts.jbits = true;
    r->bytes = instance_bytes(N, R, runs, r->facts, s->steps);
    if (r->bytes > srv->budget)
        return fail(SBQA_EBUDGET, "instance needs %zu device bytes, budget is %zu", r->bytes, srv->budget);
    r->N = N;
    r->R = R;
    r->runs = runs;
    r->s = *s;
    if (J->dense && r->facts.jbits) pack_sign_bits(J->dense, N, &r->jbits);
    else if (J->dense) r->dense.assign(J->dense, J->dense + (size_t)N * N);
    else {
        r->row_ptr.assign(J->row_ptr, J->row_ptr + N + 1);
        r->col.assign(J->col, J->col + J->nnz);
        r->val.assign(J->val, J->val + J->nnz);
        if (J->n3 > 0) {
            r->tri.assign(J->tri, J->tri + 3 * J->n3);
            r->K.assign(J->K, J->K + J->n3);
        }
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
    // the scheduler finishes every admitted instance (the creator keeps
    // building the admitted ones meanwhile), then the creator stops
    if (srv->worker.joinable()) srv->worker.join();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop_creator = true;
    }
    srv->cv_create.notify_all();
    if (srv->creator.joinable()) srv->creator.join();
    release(srv);
}

}  // extern "C"
