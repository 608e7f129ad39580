// serve.cpp -- request loop for CP-ALS MTTKRP requests on resident tensors.
//
// Requests (tensor, mode) arrive over time.  A scheduler thread keeps, per
// tensor, a FIFO of its requests (the mode-n update of a sweep must see the
// factors the previous request wrote) and serves them in one of two ways:
//   * batched: continuous batching.  Whenever an epoch slot is free, every
//     ready request (its tensor idle, it is the head of the tensor's FIFO)
//     is admitted, in arrival order, while its workspace fits the HBM budget
//     and the epoch has slots; the epoch runs as one persistent batch launch
//     (deinsum_batch_*) followed by one batched CP-ALS update kernel (an
//     epoch of at most direct_max_jobs requests takes the per-request launches
//     instead).  Up to
//     two epochs are in flight on two streams, so requests that arrive while
//     one epoch runs start on the device before it finishes.
//   * per request: each request is launched on arrival (MTTKRP, then the
//     update) on one stream, in arrival order.
// Latency of a request = host clock when its completion is observed minus its
// scheduled arrival time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "als.h"
#include "internal.h"
#include "kernels.h"
#include "serve_sched.h"

using namespace deinsum;

namespace {

using Clock = std::chrono::steady_clock;

struct STensor {
    int order = 0;
    int64_t dims[DEINSUM_MAX_ORDER] = {0};
    int64_t R = 0;
    int prec = 0;
    const void *X = nullptr;
    void *U[DEINSUM_MAX_ORDER] = {nullptr};
    double *M = nullptr;      // FP64 MTTKRP output, max dim x R (server-owned, one allocation ...)
    double *Xs = nullptr;     // ... unnormalised update, max dim x R
    double *Gp = nullptr;     // ... partial Grams, als_blocks(max dim) x R x R
    double *G = nullptr;      // ... Gram cache, order x R x R
    size_t ws[DEINSUM_MAX_ORDER] = {0};
    bool busy = false;
    std::deque<int64_t> fifo; // pending requests of this tensor, arrival order
};

AlsJob als_job_for(const STensor &t, int mode)
{
    AlsJob aj;
    std::memset(&aj, 0, sizeof(aj));
    aj.order = t.order;
    aj.mode = mode;
    aj.R = static_cast<int32_t>(t.R);
    aj.prec = t.prec;
    for (int m = 0; m < t.order; ++m) {
        aj.dims[m] = t.dims[m];
        aj.U[m] = t.U[m];
    }
    aj.M = t.M;
    aj.Xs = t.Xs;
    aj.Gp = t.Gp;
    aj.G = t.G;
    return aj;
}

struct SRequest {
    int32_t tensor = 0, mode = 0;
    double arrival = 0, done = -1;
    int64_t epoch = -1;
    int32_t status = DEINSUM_REQ_PENDING;  // read by deinsum_server_poll from other threads (atomic access)
    int32_t flags = 0;
};

void store_status(SRequest &rq, int32_t st) { __atomic_store_n(&rq.status, st, __ATOMIC_RELEASE); }
int32_t load_status(const SRequest &rq) { return __atomic_load_n(&rq.status, __ATOMIC_ACQUIRE); }

struct Epoch {
    bool active = false;
    std::vector<int64_t> reqs;
    size_t footprint = 0;
};

deinsum_spec mttkrp_spec_for(int order, int mode)
{
    deinsum_spec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.kind = DEINSUM_MTTKRP;
    sp.order = order;
    sp.free_mode = mode;
    sp.n_factors = order - 1;
    int k = 0;
    for (int m = 0; m < order; ++m) {
        sp.operand_of_mode[m] = -1;
        if (m == mode) continue;
        sp.factor_mode[k] = m;
        sp.operand_of_mode[m] = k;
        ++k;
    }
    return sp;
}

}  // namespace

struct deinsum_server {
    deinsum_server_config cfg{};
    std::vector<STensor> tensors;
    std::vector<SRequest> reqs;
    std::mutex mu;                    // guards reqs growth, `submitted` and the first error
    std::condition_variable cv;       // signalled on submission and on stop
    std::deque<int64_t> submitted;
    std::thread sched;
    std::atomic<bool> stop{false};
    std::string first_error;          // message of the first failed request
    int32_t first_status = DEINSUM_OK;
    std::atomic<int64_t> completed{0};  // requests served successfully
    std::atomic<int64_t> failed{0};     // requests that ended with an error
    int32_t *req_flags = nullptr;       // pinned, one word per request: the update's floor flag
    int64_t nsubmitted = 0;
    Clock::time_point t0;
    bool started = false;
    int device = 0;
    // batched
    deinsum_batch *batch[2] = {nullptr, nullptr};
    hipStream_t stream[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    AlsJob *als_pinned[2] = {nullptr, nullptr};
    AlsJob *als_dev[2] = {nullptr, nullptr};
    Epoch epoch[2];
    size_t footprint_used = 0;
    int64_t epochs = 0, max_batch = 0;
    // per request
    std::deque<std::pair<int64_t, hipEvent_t>> inflight;
    std::vector<hipEvent_t> event_pool;
    // The server's own MTTKRP workspaces, one per stream (stream-ordered reuse): per request
    // on stream 0; batched for epochs of a single request, which launch it directly.
    void *ws[2] = {nullptr, nullptr};
    size_t ws_bytes = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// A request that cannot be served ends with its own status; the server, the other
// requests and later requests of the same tensor go on.
void fail_request(deinsum_server *s, int64_t r, int32_t status, const std::string &msg)
{
    SRequest &rq = s->reqs[r];
    rq.done = s->now();
    STensor &tn = s->tensors[rq.tensor];
    tn.busy = false;
    if (!tn.fifo.empty() && tn.fifo.front() == r) tn.fifo.pop_front();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->first_status == DEINSUM_OK) {
            s->first_status = status;
            s->first_error = "request " + std::to_string(r) + ": " + msg;
        }
    }
    store_status(rq, status);
    ++s->failed;
}

void finish_request(deinsum_server *s, int64_t r, double t)
{
    SRequest &rq = s->reqs[r];
    rq.done = t;
    if (s->cfg.als_update && __atomic_load_n(&s->req_flags[r], __ATOMIC_RELAXED)) rq.flags |= DEINSUM_REQ_REGULARISED;
    STensor &tn = s->tensors[rq.tensor];
    tn.busy = false;
    if (!tn.fifo.empty() && tn.fifo.front() == r) tn.fifo.pop_front();
    store_status(rq, DEINSUM_REQ_DONE);
    ++s->completed;
}

bool enqueue_request(deinsum_server *s, int64_t r, hipStream_t st, void *ws);

bool launch_epoch(deinsum_server *s, int e, std::deque<int64_t> &pending)
{
    Epoch &ep = s->epoch[e];
    ep.reqs.clear();
    ep.footprint = 0;
    const size_t cap = static_cast<size_t>(std::max(1, s->cfg.max_jobs_per_epoch));
    admit_epoch(
        pending, cap, s->footprint_used, s->cfg.hbm_budget_bytes, ep.reqs, ep.footprint,
        [&](int64_t r) { return s->reqs[r].tensor; },
        [&](int64_t r) {
            const STensor &t = s->tensors[s->reqs[r].tensor];
            return !t.fifo.empty() && t.fifo.front() == r;
        },
        [&](int32_t t) { return s->tensors[t].busy; },
        [&](int64_t r) { return s->tensors[s->reqs[r].tensor].ws[s->reqs[r].mode]; },
        [&](int32_t t) { s->tensors[t].busy = true; });
    if (ep.reqs.empty()) return false;
    auto fail_epoch = [&](const std::string &msg) {
        for (int64_t r : ep.reqs) fail_request(s, r, DEINSUM_ERR_DEVICE, msg);
        ep.reqs.clear();
        return false;
    };
    if (static_cast<int64_t>(ep.reqs.size()) <= s->cfg.direct_max_jobs) {
        // A small epoch: the direct launches of the per-request path, one request after
        // the other on this slot's stream with its workspace (no descriptor upload, no
        // persistent batch kernel).  A request that cannot be enqueued ends alone.
        std::vector<int64_t> added;
        size_t footprint = 0;
        for (int64_t r : ep.reqs) {
            if (!enqueue_request(s, r, s->stream[e], s->ws[e])) continue;
            s->reqs[r].epoch = s->epochs;
            footprint += s->tensors[s->reqs[r].tensor].ws[s->reqs[r].mode];
            added.push_back(r);
        }
        ep.reqs.swap(added);
        ep.footprint = footprint;
        if (ep.reqs.empty()) return false;
        if (hipEventRecord(s->ev[e], s->stream[e]) != hipSuccess) return fail_epoch("event record failed");
        ep.active = true;
        s->footprint_used += ep.footprint;
        ++s->epochs;
        s->max_batch = std::max<int64_t>(s->max_batch, static_cast<int64_t>(ep.reqs.size()));
        return true;
    }
    deinsum_batch_reset(s->batch[e]);
    int64_t als_total = 0;
    std::vector<int64_t> added;
    size_t footprint = 0;
    for (size_t k = 0; k < ep.reqs.size(); ++k) {
        const int64_t r = ep.reqs[k];
        SRequest &rq = s->reqs[r];
        STensor &t = s->tensors[rq.tensor];
        const deinsum_spec sp = mttkrp_spec_for(t.order, rq.mode);
        const void *ops[DEINSUM_MAX_ORDER];
        for (int q = 0; q < t.order - 1; ++q) ops[q] = t.U[sp.factor_mode[q]];
        deinsum_opts o;
        deinsum_opts_init(&o);
        o.precision = t.prec;
        o.out_dtype = DEINSUM_F64;
        if (deinsum_status st = deinsum_batch_add_mttkrp(s->batch[e], &sp, t.dims, t.R, t.X, ops, t.M, &o, nullptr)) {
            fail_request(s, r, st, std::string("batch_add: ") + deinsum_last_error());
            continue;
        }
        AlsJob &aj = s->als_pinned[e][added.size()];
        aj = als_job_for(t, rq.mode);
        aj.block_begin = als_total;
        aj.flag = s->req_flags + r;
        als_total += als_blocks(t.dims[rq.mode]);
        rq.epoch = s->epochs;
        footprint += t.ws[rq.mode];
        added.push_back(r);
    }
    ep.reqs.swap(added);
    ep.footprint = footprint;
    if (ep.reqs.empty()) return false;
    for (int64_t r : ep.reqs) store_status(s->reqs[r], DEINSUM_REQ_RUNNING);
    if (deinsum_batch_launch(s->batch[e], s->stream[e]) != DEINSUM_OK)
        return fail_epoch(std::string("batch_launch: ") + deinsum_last_error());
    if (s->cfg.als_update) {
        // One request: its update job goes as a kernel argument (the same kernels, no
        // descriptor copy); several: one table upload and one batched launch.
        deinsum_status st;
        if (ep.reqs.size() == 1) {
            st = launch_als_one(s->als_pinned[e][0], s->stream[e]);
        } else {
            (void)hipMemcpyAsync(s->als_dev[e], s->als_pinned[e], sizeof(AlsJob) * ep.reqs.size(),
                                 hipMemcpyHostToDevice, s->stream[e]);
            st = launch_als_batch(s->als_dev[e], static_cast<int>(ep.reqs.size()), als_total, s->stream[e]);
        }
        if (st != DEINSUM_OK) return fail_epoch(std::string("factor update: ") + deinsum_last_error());
    }
    if (hipEventRecord(s->ev[e], s->stream[e]) != hipSuccess) return fail_epoch("event record failed");
    ep.active = true;
    s->footprint_used += ep.footprint;
    ++s->epochs;
    s->max_batch = std::max<int64_t>(s->max_batch, static_cast<int64_t>(ep.reqs.size()));
    return true;
}

// The epoch's event has completed (device_ok) or reported an error (its requests fail).
void complete_epoch(deinsum_server *s, int e, bool device_ok)
{
    Epoch &ep = s->epoch[e];
    const double t = s->now();
    for (int64_t r : ep.reqs) {
        if (device_ok) finish_request(s, r, t);
        else fail_request(s, r, DEINSUM_ERR_DEVICE, "device error while the epoch ran");
    }
    s->footprint_used -= ep.footprint;
    ep.active = false;
    ep.reqs.clear();
}

// Request r's MTTKRP (deinsum_mttkrp into the tensor's FP64 output) and, if configured,
// its factor update, enqueued on `st` with the stream's own workspace `ws`.  On failure
// the request has ended with its status and false is returned.
bool enqueue_request(deinsum_server *s, int64_t r, hipStream_t st, void *ws)
{
    SRequest &rq = s->reqs[r];
    STensor &t = s->tensors[rq.tensor];
    const deinsum_spec sp = mttkrp_spec_for(t.order, rq.mode);
    const void *ops[DEINSUM_MAX_ORDER];
    for (int q = 0; q < t.order - 1; ++q) ops[q] = t.U[sp.factor_mode[q]];
    deinsum_opts o;
    deinsum_opts_init(&o);
    o.precision = t.prec;
    o.out_dtype = DEINSUM_F64;
    o.workspace = ws;
    o.workspace_bytes = ws ? s->ws_bytes : 0;
    store_status(rq, DEINSUM_REQ_RUNNING);
    deinsum_status rc = deinsum_mttkrp(&sp, t.dims, t.R, t.X, ops, t.M, &o, st);
    if (rc == DEINSUM_ERR_NO_MEMORY && ws) {  // a plan tuned after start needs more: the library pool
        o.workspace = nullptr;
        o.workspace_bytes = 0;
        rc = deinsum_mttkrp(&sp, t.dims, t.R, t.X, ops, t.M, &o, st);
    }
    if (rc != DEINSUM_OK) {
        fail_request(s, r, rc, std::string("mttkrp: ") + deinsum_last_error());
        return false;
    }
    if (s->cfg.als_update) {
        AlsJob aj = als_job_for(t, rq.mode);
        aj.flag = s->req_flags + r;
        if (deinsum_status rc2 = launch_als_one(aj, st)) {
            fail_request(s, r, rc2, std::string("factor update: ") + deinsum_last_error());
            return false;
        }
    }
    return true;
}

bool launch_one(deinsum_server *s, int64_t r)
{
    if (!enqueue_request(s, r, s->stream[0], s->ws[0])) return false;
    hipEvent_t ev;
    if (!s->event_pool.empty()) {
        ev = s->event_pool.back();
        s->event_pool.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        fail_request(s, r, DEINSUM_ERR_DEVICE, "event creation failed");
        return false;
    }
    if (hipEventRecord(ev, s->stream[0]) != hipSuccess) {
        s->event_pool.push_back(ev);
        fail_request(s, r, DEINSUM_ERR_DEVICE, "event record failed");
        return false;
    }
    s->inflight.emplace_back(r, ev);
    s->reqs[r].epoch = s->epochs++;
    return true;
}

void scheduler(deinsum_server *s)
{
    (void)hipSetDevice(s->device);
    std::deque<int64_t> pending;  // arrival order
    std::vector<int64_t> intake;
    for (;;) {
        bool progress = false;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            while (!s->submitted.empty()) {
                const int64_t r = s->submitted.front();
                s->submitted.pop_front();
                intake.push_back(r);
            }
        }
        for (int64_t r : intake) {
            progress = true;
            const SRequest &rq = s->reqs[r];
            const size_t ws = s->tensors[rq.tensor].ws[rq.mode];
            if (ws > s->cfg.hbm_budget_bytes) {  // can never be admitted within the budget
                fail_request(s, r, DEINSUM_ERR_NO_MEMORY,
                             "MTTKRP workspace of " + std::to_string(ws) + " bytes exceeds the HBM budget");
                continue;
            }
            s->tensors[rq.tensor].fifo.push_back(r);
            pending.push_back(r);
        }
        intake.clear();
        if (s->cfg.batched) {
            for (int e = 0; e < 2; ++e) {
                if (!s->epoch[e].active) continue;
                const hipError_t q = hipEventQuery(s->ev[e]);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) (void)hipGetLastError();
                complete_epoch(s, e, q == hipSuccess);
                progress = true;
            }
            const int slots = std::max(1, std::min(2, s->cfg.epochs_in_flight));
            for (int e = 0; e < slots && !pending.empty(); ++e)
                if (!s->epoch[e].active && launch_epoch(s, e, pending)) progress = true;
        } else {
            while (!pending.empty()) {
                const int64_t r = pending.front();
                pending.pop_front();
                (void)launch_one(s, r);  // a failure ends that request only
                progress = true;
            }
            while (!s->inflight.empty()) {
                const hipError_t q = hipEventQuery(s->inflight.front().second);
                if (q == hipErrorNotReady) break;
                const int64_t r = s->inflight.front().first;
                if (q == hipSuccess) {
                    finish_request(s, r, s->now());
                } else {
                    (void)hipGetLastError();
                    fail_request(s, r, DEINSUM_ERR_DEVICE, "device error while the request ran");
                }
                s->event_pool.push_back(s->inflight.front().second);
                s->inflight.pop_front();
                progress = true;
            }
        }
        if (s->stop && pending.empty()) {
            bool idle = s->inflight.empty() && !s->epoch[0].active && !s->epoch[1].active;
            std::lock_guard<std::mutex> lk(s->mu);
            if (idle && s->submitted.empty()) return;
        }
        if (!progress) {
            // Work on the device: poll its events without sleeping (a sleep costs tens of
            // microseconds of latency).  Nothing to do: wait for a submission.
            const bool busy = !pending.empty() || !s->inflight.empty() || s->epoch[0].active || s->epoch[1].active;
            if (busy) {
                std::this_thread::yield();
            } else {
                std::unique_lock<std::mutex> lk(s->mu);
                s->cv.wait_for(lk, std::chrono::milliseconds(1), [&] { return !s->submitted.empty() || s->stop.load(); });
            }
        }
    }
}

}  // namespace

extern "C" {

void deinsum_server_config_init(deinsum_server_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->batched = 1;
    cfg->max_jobs_per_epoch = 256;
    cfg->epochs_in_flight = 2;
    cfg->als_update = 1;
    cfg->max_requests = int64_t(1) << 20;
    cfg->hbm_budget_bytes = size_t(4) << 30;
    cfg->direct_max_jobs = 4;
}

deinsum_status deinsum_server_create(const deinsum_server_config *cfg, deinsum_server **out)
{
    if (!out) return fail(DEINSUM_ERR_INVALID_ARG, "server_create: null out");
    *out = nullptr;
    auto *s = new deinsum_server();
    deinsum_server_config_init(&s->cfg);
    if (cfg) s->cfg = *cfg;
    if (s->cfg.max_jobs_per_epoch < 1 || s->cfg.max_jobs_per_epoch > 65536) {
        delete s;
        return fail(DEINSUM_ERR_INVALID_ARG, "server_create: max_jobs_per_epoch must be 1..65536");
    }
    if (s->cfg.direct_max_jobs < 0 || s->cfg.direct_max_jobs > s->cfg.max_jobs_per_epoch) {
        delete s;
        return fail(DEINSUM_ERR_INVALID_ARG, "server_create: direct_max_jobs must be 0..max_jobs_per_epoch");
    }
    if (s->cfg.max_requests < 1 || s->cfg.max_requests > (int64_t(1) << 28)) {
        delete s;
        return fail(DEINSUM_ERR_INVALID_ARG, "server_create: max_requests must be 1..2^28");
    }
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(DEINSUM_ERR_DEVICE, "server_create: no current device");
    }
    for (int e = 0; e < 2; ++e) {
        if (hipStreamCreateWithFlags(&s->stream[e], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s->ev[e], hipEventDisableTiming) != hipSuccess) {
            deinsum_server_destroy(s);
            return fail(DEINSUM_ERR_DEVICE, "server_create: stream/event creation failed");
        }
        if (s->cfg.batched) {
            if (deinsum_batch_create(s->cfg.max_jobs_per_epoch, &s->batch[e]) != DEINSUM_OK) {
                deinsum_server_destroy(s);
                return DEINSUM_ERR_DEVICE;
            }
            const size_t bytes = sizeof(AlsJob) * static_cast<size_t>(s->cfg.max_jobs_per_epoch);
            if (hipHostMalloc(reinterpret_cast<void **>(&s->als_pinned[e]), bytes, hipHostMallocDefault) != hipSuccess ||
                hipMalloc(reinterpret_cast<void **>(&s->als_dev[e]), bytes) != hipSuccess) {
                deinsum_server_destroy(s);
                return fail(DEINSUM_ERR_NO_MEMORY, "server_create: job table allocation failed");
            }
        }
    }
    *out = s;
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_server_add_tensor(deinsum_server *s, int32_t order, const int64_t *dims, int64_t R,
                                         int32_t precision, const void *X, void *const *U, int32_t *tensor_id)
{
    if (!s || !dims || !X || !U) return fail(DEINSUM_ERR_INVALID_ARG, "server_add_tensor: null argument");
    if (s->started) return fail(DEINSUM_ERR_BUSY, "server_add_tensor: server already started");
    if (order < 2 || order > DEINSUM_MAX_ORDER) return fail(DEINSUM_ERR_SHAPE, "server_add_tensor: order 2..8");
    if (R < 1 || R > kAlsMaxRank) return fail(DEINSUM_ERR_SHAPE, "server_add_tensor: rank 1..64");
    if (precision != DEINSUM_PREC_FP64 && precision != DEINSUM_PREC_FP32)
        return fail(DEINSUM_ERR_UNSUPPORTED, "server_add_tensor: FP64 or FP32 tensors");
    STensor t;
    t.order = order;
    t.R = R;
    t.prec = precision;
    t.X = X;
    int64_t maxd = 0;
    for (int m = 0; m < order; ++m) {
        if (dims[m] < 1) return fail(DEINSUM_ERR_SHAPE, "server_add_tensor: dims >= 1");
        if (!U[m]) return fail(DEINSUM_ERR_INVALID_ARG, "server_add_tensor: null factor");
        t.dims[m] = dims[m];
        t.U[m] = U[m];
        maxd = std::max(maxd, dims[m]);
    }
    const size_t rows_bytes = sizeof(double) * static_cast<size_t>(maxd * R);
    const size_t gp_bytes = sizeof(double) * static_cast<size_t>(als_blocks(maxd) * R * R);
    const size_t g_bytes = sizeof(double) * static_cast<size_t>(order * R * R);
    char *buf = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&buf), 2 * rows_bytes + gp_bytes + g_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DEINSUM_ERR_NO_MEMORY, "server_add_tensor: state allocation failed");
    }
    t.M = reinterpret_cast<double *>(buf);
    t.Xs = reinterpret_cast<double *>(buf + rows_bytes);
    t.Gp = reinterpret_cast<double *>(buf + 2 * rows_bytes);
    t.G = reinterpret_cast<double *>(buf + 2 * rows_bytes + gp_bytes);
    // The caller's X and factors must be ready; the Gram cache starts from them.
    if (hipDeviceSynchronize() != hipSuccess || launch_als_grams(als_job_for(t, 0), s->stream[0]) != DEINSUM_OK ||
        hipStreamSynchronize(s->stream[0]) != hipSuccess) {
        (void)hipFree(buf);
        return fail(DEINSUM_ERR_DEVICE, "server_add_tensor: Gram set-up failed");
    }
    deinsum_opts o;
    deinsum_opts_init(&o);
    o.precision = precision;
    for (int m = 0; m < order; ++m) {
        const deinsum_spec sp = mttkrp_spec_for(order, m);
        size_t ws = 0;
        const int64_t r = R;
        if (deinsum_workspace_size(&sp, dims, &r, &o, &ws) != DEINSUM_OK) ws = 0;
        t.ws[m] = ws;
    }
    if (tensor_id) *tensor_id = static_cast<int32_t>(s->tensors.size());
    s->tensors.push_back(std::move(t));
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_server_start(deinsum_server *s)
{
    if (!s) return fail(DEINSUM_ERR_INVALID_ARG, "server_start: null server");
    if (s->started) return fail(DEINSUM_ERR_BUSY, "server_start: already started");
    s->reqs.reserve(static_cast<size_t>(s->cfg.max_requests));
    if (hipHostMalloc(reinterpret_cast<void **>(&s->req_flags), sizeof(int32_t) * static_cast<size_t>(s->cfg.max_requests),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        s->req_flags = nullptr;
        return fail(DEINSUM_ERR_NO_MEMORY, "server_start: request flag table allocation failed");
    }
    std::memset(s->req_flags, 0, sizeof(int32_t) * static_cast<size_t>(s->cfg.max_requests));
    {
        size_t mx = 0;
        for (auto &t : s->tensors)
            for (int m = 0; m < t.order; ++m) mx = std::max(mx, t.ws[m]);
        const int nws = s->cfg.batched ? 2 : 1;
        for (int e = 0; e < nws && mx; ++e)
            if (hipMalloc(&s->ws[e], mx) != hipSuccess) {
                (void)hipGetLastError();
                s->ws[e] = nullptr;
                return fail(DEINSUM_ERR_NO_MEMORY, "server_start: workspace allocation failed");
            }
        s->ws_bytes = mx;
    }
    s->t0 = Clock::now();
    s->started = true;
    s->sched = std::thread(scheduler, s);
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_server_submit(deinsum_server *s, int32_t tensor_id, int32_t mode, double arrival_s,
                                     int64_t *request_id)
{
    if (!s || !s->started) return fail(DEINSUM_ERR_INVALID_ARG, "server_submit: server not started");
    if (tensor_id < 0 || tensor_id >= static_cast<int32_t>(s->tensors.size()))
        return fail(DEINSUM_ERR_INVALID_ARG, "server_submit: unknown tensor");
    if (mode < 0 || mode >= s->tensors[tensor_id].order) return fail(DEINSUM_ERR_INVALID_ARG, "server_submit: bad mode");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->reqs.size() == s->reqs.capacity())
        return fail(DEINSUM_ERR_BUSY, "server_submit: request table full");  // reqs must not reallocate while served
    SRequest rq;
    rq.tensor = tensor_id;
    rq.mode = mode;
    rq.arrival = arrival_s >= 0 ? arrival_s : s->now();
    s->reqs.push_back(rq);
    const int64_t id = static_cast<int64_t>(s->reqs.size()) - 1;
    s->submitted.push_back(id);
    s->cv.notify_one();
    ++s->nsubmitted;
    if (request_id) *request_id = id;
    return DEINSUM_OK;
}

deinsum_status deinsum_server_replay(deinsum_server *s, int64_t n, const double *arrival_s, const int32_t *tensor_id,
                                     const int32_t *mode)
{
    if (!s || !s->started || !arrival_s || !tensor_id || !mode || n < 0)
        return fail(DEINSUM_ERR_INVALID_ARG, "server_replay: bad argument");
    const Clock::time_point base = s->t0;
    for (int64_t i = 0; i < n; ++i) {
        const Clock::time_point due = base + std::chrono::duration_cast<Clock::duration>(
                                                 std::chrono::duration<double>(arrival_s[i]));
        while (Clock::now() < due) {
            const auto left = due - Clock::now();
            if (left > std::chrono::microseconds(200)) std::this_thread::sleep_for(left - std::chrono::microseconds(150));
        }
        if (deinsum_status st = deinsum_server_submit(s, tensor_id[i], mode[i], arrival_s[i], nullptr)) return st;
    }
    return DEINSUM_OK;
}

deinsum_status deinsum_server_drain(deinsum_server *s)
{
    if (!s || !s->started) return fail(DEINSUM_ERR_INVALID_ARG, "server_drain: server not started");
    for (;;) {
        int64_t nsub;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            nsub = s->nsubmitted;
        }
        if (s->completed + s->failed >= nsub) break;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    if (s->failed > 0) {
        std::lock_guard<std::mutex> lk(s->mu);
        return fail(static_cast<deinsum_status>(s->first_status),
                    std::to_string(s->failed.load()) + " request(s) failed; first: " + s->first_error);
    }
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_server_poll(const deinsum_server *s, int64_t request_id, int32_t *status, int32_t *flags,
                                   double *done_s)
{
    if (!s || !s->started) return fail(DEINSUM_ERR_INVALID_ARG, "server_poll: server not started");
    auto *ms = const_cast<deinsum_server *>(s);
    int64_t n;
    {
        std::lock_guard<std::mutex> lk(ms->mu);
        n = static_cast<int64_t>(s->reqs.size());
    }
    if (request_id < 0 || request_id >= n) return fail(DEINSUM_ERR_INVALID_ARG, "server_poll: unknown request");
    const SRequest &rq = s->reqs[request_id];
    const int32_t st = load_status(rq);  // acquire: done and flags below were written before it
    if (status) *status = st;
    if (flags) *flags = st == DEINSUM_REQ_DONE ? rq.flags : 0;
    if (done_s) *done_s = (st == DEINSUM_REQ_DONE || st < 0) ? rq.done : -1.0;
    return DEINSUM_OK;
}

deinsum_status deinsum_server_results(const deinsum_server *s, int64_t n, double *arrival_s, double *done_s,
                                      int64_t *epoch)
{
    if (!s) return fail(DEINSUM_ERR_INVALID_ARG, "server_results: null server");
    if (n > static_cast<int64_t>(s->reqs.size())) return fail(DEINSUM_ERR_INVALID_ARG, "server_results: n too large");
    for (int64_t i = 0; i < n; ++i) {
        if (arrival_s) arrival_s[i] = s->reqs[i].arrival;
        if (done_s) done_s[i] = s->reqs[i].done;
        if (epoch) epoch[i] = s->reqs[i].epoch;
    }
    return DEINSUM_OK;
}

deinsum_status deinsum_server_stats(const deinsum_server *s, int64_t *completed, int64_t *epochs, int64_t *max_batch)
{
    if (!s) return fail(DEINSUM_ERR_INVALID_ARG, "server_stats: null server");
    if (completed) *completed = s->completed;
    if (epochs) *epochs = s->epochs;
    if (max_batch) *max_batch = s->max_batch;
    return DEINSUM_OK;
}

deinsum_status deinsum_server_destroy(deinsum_server *s)
{
    if (!s) return DEINSUM_OK;
    s->stop = true;
    s->cv.notify_all();
    if (s->sched.joinable()) s->sched.join();
    for (int e = 0; e < 2; ++e) {
        if (s->stream[e]) (void)hipStreamSynchronize(s->stream[e]);
        if (s->batch[e]) deinsum_batch_destroy(s->batch[e]);
        if (s->als_pinned[e]) (void)hipHostFree(s->als_pinned[e]);
        if (s->als_dev[e]) (void)hipFree(s->als_dev[e]);
        if (s->ev[e]) (void)hipEventDestroy(s->ev[e]);
        if (s->stream[e]) (void)hipStreamDestroy(s->stream[e]);
    }
    for (auto &p : s->inflight) (void)hipEventDestroy(p.second);
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (auto &t : s->tensors)
        if (t.M) (void)hipFree(t.M);
    for (void *w : s->ws)
        if (w) (void)hipFree(w);
    if (s->req_flags) (void)hipHostFree(s->req_flags);
    delete s;
    return DEINSUM_OK;
}

}  // extern "C"
