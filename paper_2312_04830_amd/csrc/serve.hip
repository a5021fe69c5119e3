// Property server: chunked admission by device memory, round-robin continuous batching
// across requests, overlap on a pool of streams.
//
// Threads: callers submit; one scheduler thread turns pending requests into chunk
// dispatches whenever a slot is free; one completion thread retires dispatched chunks in
// order, frees their slots and finishes requests.  Slot i always uses stream i % S and
// event i, so a slot is only reused after the work that used it has completed.  In the
// mock executor, host worker threads stand in for the streams (same scheduler, no GPU).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "props_internal.hpp"
#include "trace.hpp"

namespace {

using clk = std::chrono::steady_clock;

constexpr int NOUTF = 10;   // T P Z rho h e cp c mu lambda

struct Slot {
    unsigned char *base = nullptr;
    double *in0, *in1, *Y, *Tg;
    double *out[NOUTF];
    uint8_t *status;
    int *fb_idx, *fb_count;
};

struct Chunk {
    uint64_t ticket;
    int64_t off, m;
    int slot;
    int rc = PROPS_OK;
    bool dispatched = false;   // GPU: copies, kernel and event are enqueued
    bool done = false;         // mock executor: evaluated
};

struct Request {
    props_request r;
    int64_t nchunks = 0, next = 0, done = 0;
    int rc = PROPS_OK;
    double t_submit = 0, t_done = 0;
    bool finished = false;
};

double* out_ptr(const props_out &o, int f)
{
    double *const p[NOUTF] = {o.T, o.P, o.Z, o.rho, o.h, o.e, o.cp, o.c, o.mu, o.lambda};
    return p[f];
}

}  // namespace

using namespace props;

struct props_server_s {
    props_serve_cfg cfg{};
    props_mech_t mech = nullptr;
    props_dnn_t dnn = nullptr;
    int ns = 0, device = 0;
    int64_t C = 0;            // cells per slot
    size_t slot_bytes = 0;
    void *arena = nullptr;
    std::vector<Slot> slots;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;

    std::mutex mu;
    std::condition_variable cv;
    std::map<uint64_t, Request> reqs;
    std::deque<uint64_t> active;    // requests with chunks not yet dispatched (round-robin)
    std::vector<int> free_slots;
    std::deque<Chunk *> inflight;   // dispatch order
    std::deque<Chunk *> mock_q;
    bool stop = false;
    uint64_t next_ticket = 1;
    clk::time_point t0 = clk::now();
    bool any_submit = false;
    double t_first = 0, t_last = 0;
    int64_t submitted = 0, completed = 0, failed = 0, cells_done = 0;
    std::vector<double> lat;

    std::thread sched, compl_thr;
    std::vector<std::thread> workers;

    double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }
};

namespace {

// The two per-cell scalar inputs of a request's mode (Y aside): (P, T), (rho, e) or (h, P).
void mode_inputs(const props_request &q, const double **a, const double **b)
{
    if (q.mode == PROPS_PTY) *a = q.in.P, *b = q.in.T;
    else if (q.mode == PROPS_RHOEY) *a = q.in.rho, *b = q.in.e;
    else *a = q.in.h, *b = q.in.P;
}

// Device-resident request: the chunk's kernels read and write the caller's arrays in place
// (cells [off, off + m) of arrays of n cells, species rows n apart); the slot only lends its
// fallback-list scratch.
int dispatch_device(props_server_s *S, Chunk *ch, const Request &R, hipStream_t st)
{
    const Slot &sl = S->slots[ch->slot];
    const props_request &q = R.r;
    const int64_t m = ch->m, off = ch->off, n = q.n;
    auto at = [off](const double *p) { return p ? p + off : nullptr; };
    auto atw = [off](double *p) { return p ? p + off : nullptr; };
    props_in in{};
    in.P = at(q.in.P), in.T = at(q.in.T), in.rho = at(q.in.rho), in.e = at(q.in.e), in.h = at(q.in.h);
    in.Y = q.in.Y + off;
    in.T_guess = q.mode != PROPS_PTY ? at(q.in.T_guess) : nullptr;
    props_out out{};
    out.T = atw(q.out.T), out.P = atw(q.out.P), out.Z = atw(q.out.Z), out.rho = atw(q.out.rho);
    out.h = atw(q.out.h), out.e = atw(q.out.e), out.cp = atw(q.out.cp), out.c = atw(q.out.c);
    out.mu = atw(q.out.mu), out.lambda = atw(q.out.lambda);
    out.psi = atw(q.out.psi), out.alpha = atw(q.out.alpha);
    out.hRT = q.out.hRT ? q.out.hRT + off : nullptr;
    out.iters = q.out.iters ? q.out.iters + off : nullptr;
    uint8_t *status = q.status ? q.status + off : nullptr;
    int rc;
    if (q.route == PROPS_ROUTE_DNN)
        rc = dnn_eval(S->dnn, S->mech, &in, &out, m, n, status, sl.fb_idx, sl.fb_count, st);
    else
        rc = launch_pr_strided(S->mech, q.mode, q.route == PROPS_ROUTE_PR_FP64 ? PROPS_FP64 : PROPS_MIXED, &in, &out,
                               m, n, status, st);
    if (rc) return rc;
    PROPS_HIP_TRY(hipEventRecord(S->events[ch->slot], st));
    return PROPS_OK;
}

int dispatch_gpu(props_server_s *S, Chunk *ch, const Request &R)
{
    const Slot &sl = S->slots[ch->slot];
    hipStream_t st = S->streams[ch->slot % S->streams.size()];
    const props_request &q = R.r;
    if (q.memory == PROPS_MEM_DEVICE) return dispatch_device(S, ch, R, st);
    // host-staged request: copy the chunk in, evaluate in the slot, copy it out
    const int64_t m = ch->m, off = ch->off, n = q.n;
    const size_t b = (size_t)m * sizeof(double);
    const bool pty = q.mode == PROPS_PTY;
    const double *h0, *h1;
    mode_inputs(q, &h0, &h1);
    PROPS_HIP_TRY(hipMemcpyAsync(sl.in0, h0 + off, b, hipMemcpyHostToDevice, st));
    PROPS_HIP_TRY(hipMemcpyAsync(sl.in1, h1 + off, b, hipMemcpyHostToDevice, st));
    for (int i = 0; i < S->ns; i++)
        PROPS_HIP_TRY(hipMemcpyAsync(sl.Y + (size_t)i * m, q.in.Y + (size_t)i * n + off, b, hipMemcpyHostToDevice, st));
    const bool tg = !pty && q.in.T_guess;
    if (tg) PROPS_HIP_TRY(hipMemcpyAsync(sl.Tg, q.in.T_guess + off, b, hipMemcpyHostToDevice, st));
    props_in in{};
    if (pty) in.P = sl.in0, in.T = sl.in1;
    else if (q.mode == PROPS_RHOEY) in.rho = sl.in0, in.e = sl.in1;
    else in.h = sl.in0, in.P = sl.in1;
    in.Y = sl.Y;
    in.T_guess = tg ? sl.Tg : nullptr;
    props_out out{};
    double **dst[NOUTF] = {&out.T, &out.P, &out.Z, &out.rho, &out.h, &out.e, &out.cp, &out.c, &out.mu, &out.lambda};
    for (int f = 0; f < NOUTF; f++)
        if (out_ptr(q.out, f)) *dst[f] = sl.out[f];
    int rc;
    if (q.route == PROPS_ROUTE_DNN)
        rc = dnn_eval(S->dnn, S->mech, &in, &out, m, m, sl.status, sl.fb_idx, sl.fb_count, st);
    else
        rc = launch_pr(S->mech, q.mode, q.route == PROPS_ROUTE_PR_FP64 ? PROPS_FP64 : PROPS_MIXED, &in, &out, m,
                       sl.status, st);
    if (rc) return rc;
    for (int f = 0; f < NOUTF; f++) {
        double *h = out_ptr(q.out, f);
        if (h) PROPS_HIP_TRY(hipMemcpyAsync(h + off, sl.out[f], b, hipMemcpyDeviceToHost, st));
    }
    if (q.status) PROPS_HIP_TRY(hipMemcpyAsync(q.status + off, sl.status, (size_t)m, hipMemcpyDeviceToHost, st));
    PROPS_HIP_TRY(hipEventRecord(S->events[ch->slot], st));
    return PROPS_OK;
}

// Mock evaluation: a fixed function of each cell's inputs, so that tests can check that
// every cell of every request came back to the right place.
void mock_eval(props_server_s *S, Chunk *ch, const Request &R)
{
    const props_request &q = R.r;
    const double *a, *b;
    mode_inputs(q, &a, &b);
    if (ch->m > 0 && std::isnan(a[ch->off])) {
        ch->rc = fail(PROPS_EINVAL, "mock executor: chunk rejected (NaN first input)");
        return;
    }
    for (int64_t k = ch->off; k < ch->off + ch->m; k++) {
        double ys = 0;
        for (int i = 0; i < S->ns; i++) ys += (i + 1) * q.in.Y[(size_t)i * q.n + k];
        const double v[NOUTF] = {b[k], a[k], ys, a[k] + 2 * b[k], a[k] * b[k], a[k] - b[k], ys * 3,
                                 (double)q.route, (double)q.mode, (double)k};
        for (int f = 0; f < NOUTF; f++) {
            double *h = out_ptr(q.out, f);
            if (h) h[k] = v[f];
        }
        if (q.status) q.status[k] = 0;
    }
}

void scheduler_loop(props_server_s *S)
{
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] { return S->stop || (!S->active.empty() && !S->free_slots.empty()); });
        if (S->stop && (S->active.empty() || S->free_slots.empty())) {
            if (S->active.empty()) break;
            S->cv.wait(lk, [&] { return !S->free_slots.empty() || S->active.empty(); });
            continue;
        }
        const uint64_t t = S->active.front();
        S->active.pop_front();
        Request &R = S->reqs.at(t);
        Chunk *ch = new Chunk{t, R.next * S->C, std::min<int64_t>(S->C, R.r.n - R.next * S->C), S->free_slots.back()};
        S->free_slots.pop_back();
        R.next++;
        if (R.next < R.nchunks) S->active.push_back(t);   // round-robin over active requests
        S->inflight.push_back(ch);
        if (S->cfg.executor == PROPS_EXEC_MOCK) {
            S->mock_q.push_back(ch);
            S->cv.notify_all();
            continue;
        }
        lk.unlock();
        const int rc = dispatch_gpu(S, ch, R);
        lk.lock();
        ch->rc = rc;
        ch->dispatched = true;
        S->cv.notify_all();
    }
}

void mock_worker(props_server_s *S)
{
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] { return !S->mock_q.empty() || (S->stop && S->inflight.empty() && S->active.empty()); });
        if (S->mock_q.empty()) break;
        Chunk *ch = S->mock_q.front();
        S->mock_q.pop_front();
        const Request &R = S->reqs.at(ch->ticket);
        lk.unlock();
        if (S->cfg.mock_ns_per_cell > 0)
            std::this_thread::sleep_for(std::chrono::nanoseconds((int64_t)(S->cfg.mock_ns_per_cell * ch->m)));
        mock_eval(S, ch, R);
        lk.lock();
        ch->done = true;
        S->cv.notify_all();
    }
}

void completion_loop(props_server_s *S)
{
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv.wait(lk, [&] { return !S->inflight.empty() || (S->stop && S->active.empty()); });
        if (S->inflight.empty()) break;
        Chunk *ch = S->inflight.front();
        int rc;
        if (S->cfg.executor == PROPS_EXEC_MOCK) {
            S->cv.wait(lk, [&] { return ch->done; });
            rc = ch->rc;
        } else {
            S->cv.wait(lk, [&] { return ch->dispatched; });
            const int drc = ch->rc;
            lk.unlock();
            hipError_t e = drc ? hipSuccess : hipEventSynchronize(S->events[ch->slot]);
            lk.lock();
            rc = ch->rc ? ch->rc : (e == hipSuccess ? PROPS_OK : fail(PROPS_EHIP, "chunk failed: %s", hipGetErrorString(e)));
        }
        S->inflight.pop_front();
        S->free_slots.push_back(ch->slot);
        Request &R = S->reqs.at(ch->ticket);
        R.done++;
        if (rc) R.rc = rc;
        else S->cells_done += ch->m;
        if (R.done == R.nchunks && R.next == R.nchunks) {
            R.finished = true;
            R.t_done = S->now();
            S->t_last = R.t_done;
            if (R.rc) {
                S->failed++;
            } else {
                S->completed++;
                S->lat.push_back(R.t_done - R.t_submit);
            }
        }
        delete ch;
        S->cv.notify_all();
    }
}

int carve_slots(props_server_s *S)
{
    const size_t C = (size_t)S->C;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t dbl = al(C * sizeof(double));
    S->slot_bytes = dbl * (3 + S->ns + NOUTF) + al(C) + al(C * sizeof(int)) + 256;
    const int64_t nslot = S->cfg.mem_budget / (int64_t)S->slot_bytes;
    if (nslot < 1)
        return fail(PROPS_ETOOBIG, "serve_create: mem_budget %lld B is below one slot of %lld cells (%zu B)",
                    (long long)S->cfg.mem_budget, (long long)S->C, S->slot_bytes);
    int ns = (int)std::min<int64_t>(nslot, 4096);
    if (S->cfg.max_inflight > 0) ns = std::min(ns, S->cfg.max_inflight);
    const size_t total = S->slot_bytes * ns;
    if (S->cfg.executor == PROPS_EXEC_MOCK) {
        S->arena = nullptr;   // the mock executor reads and writes the caller's host arrays
    } else {
        hipError_t e = hipMalloc(&S->arena, total);
        if (e != hipSuccess) return fail(PROPS_ENOMEM, "serve_create: hipMalloc(%zu): %s", total, hipGetErrorString(e));
    }
    S->slots.resize(ns);
    for (int i = 0; i < ns; i++) {
        Slot &sl = S->slots[i];
        unsigned char *p = S->arena ? static_cast<unsigned char *>(S->arena) + S->slot_bytes * i : nullptr;
        auto take = [&](size_t bytes) {
            unsigned char *r = p;
            if (p) p += bytes;
            return r;
        };
        sl.base = p;
        sl.in0 = (double *)take(dbl);
        sl.in1 = (double *)take(dbl);
        sl.Tg = (double *)take(dbl);
        sl.Y = (double *)take(dbl * S->ns);
        for (int f = 0; f < NOUTF; f++) sl.out[f] = (double *)take(dbl);
        sl.status = (uint8_t *)take(al(C));
        sl.fb_idx = (int *)take(al(C * sizeof(int)));
        sl.fb_count = (int *)take(256);
        S->free_slots.push_back(ns - 1 - i);
    }
    return PROPS_OK;
}

void destroy_server(props_server_s *S)
{
    for (hipEvent_t e : S->events) (void)hipEventDestroy(e);
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    if (S->arena) (void)hipFree(S->arena);
    delete S;
}

}  // namespace

extern "C" {

int serve_create(const props_serve_cfg *cfg, props_mech_t mech, props_dnn_t dnn, props_server_t *out)
{
    ApiRange range_("serve_create");
    if (!out) return fail(PROPS_EINVAL, "serve_create: out is NULL");
    *out = nullptr;
    if (!cfg) return fail(PROPS_EINVAL, "serve_create: cfg is required");
    if (!mech && cfg->executor != PROPS_EXEC_MOCK) return fail(PROPS_EINVAL, "serve_create: mech is required");
    if (cfg->executor != PROPS_EXEC_GPU && cfg->executor != PROPS_EXEC_MOCK)
        return fail(PROPS_EINVAL, "serve_create: unknown executor %d", cfg->executor);
    if (cfg->chunk_cells < 0 || cfg->streams < 0 || cfg->max_inflight < 0 || cfg->mem_budget <= 0)
        return fail(PROPS_EINVAL, "serve_create: negative size or non-positive budget");
    props_server_s *S = new (std::nothrow) props_server_s();
    if (!S) return fail(PROPS_ENOMEM, "serve_create: out of host memory");
    S->cfg = *cfg;
    S->mech = mech;
    S->dnn = dnn;
    S->ns = mech ? mech->ns : (cfg->mock_species > 0 ? cfg->mock_species : 8);
    S->C = cfg->chunk_cells ? cfg->chunk_cells : 262144;
    int nstreams = cfg->streams ? cfg->streams : 4;
    int rc;
    if (cfg->executor == PROPS_EXEC_GPU && hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return fail(PROPS_EHIP, "serve_create: hipGetDevice failed");
    }
    if ((rc = carve_slots(S))) {
        destroy_server(S);
        return rc;
    }
    nstreams = std::min<int>(nstreams, (int)S->slots.size());
    if (cfg->executor == PROPS_EXEC_GPU) {
        for (int i = 0; i < nstreams; i++) {
            hipStream_t s;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
                destroy_server(S);
                return fail(PROPS_EHIP, "serve_create: hipStreamCreate failed");
            }
            S->streams.push_back(s);
        }
        for (size_t i = 0; i < S->slots.size(); i++) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                destroy_server(S);
                return fail(PROPS_EHIP, "serve_create: hipEventCreate failed");
            }
            S->events.push_back(e);
        }
    } else {
        for (int i = 0; i < nstreams; i++) S->workers.emplace_back(mock_worker, S);
    }
    S->sched = std::thread(scheduler_loop, S);
    S->compl_thr = std::thread(completion_loop, S);
    *out = S;
    return PROPS_OK;
}

int serve_submit(props_server_t S, const props_request *req, uint64_t *ticket)
{
    ApiRange range_("serve_submit");
    if (!S || !req || !ticket) return fail(PROPS_EINVAL, "serve_submit: null argument");
    const props_request &q = *req;
    if (q.n <= 0) return fail(PROPS_EINVAL, "serve_submit: n = %lld", (long long)q.n);
    if (q.mode != PROPS_PTY && q.mode != PROPS_RHOEY && q.mode != PROPS_HPY)
        return fail(PROPS_EINVAL, "serve_submit: unknown mode %d", q.mode);
    if (q.route < PROPS_ROUTE_PR_FP64 || q.route > PROPS_ROUTE_DNN)
        return fail(PROPS_EINVAL, "serve_submit: unknown route %d", q.route);
    if (q.memory != PROPS_MEM_DEVICE && q.memory != PROPS_MEM_HOST)
        return fail(PROPS_EINVAL, "serve_submit: unknown memory kind %d", q.memory);
    if (S->cfg.executor == PROPS_EXEC_MOCK && q.memory != PROPS_MEM_HOST)
        return fail(PROPS_EINVAL, "serve_submit: the mock executor evaluates host arrays only");
    if (q.route == PROPS_ROUTE_DNN && (!S->dnn || q.mode != PROPS_PTY))
        return fail(PROPS_EINVAL, "serve_submit: the DNN route needs a network and (P, T, Y) inputs");
    // the surrogate predicts rho, h, cp, c, mu and lambda only: any other requested output
    // would come back unwritten
    if (q.route == PROPS_ROUTE_DNN &&
        (q.out.T || q.out.P || q.out.Z || q.out.e || q.out.psi || q.out.alpha || q.out.hRT || q.out.iters))
        return fail(PROPS_EINVAL, "serve_submit: the DNN route returns only rho, h, cp, c, mu and lambda");
    // host-staged requests carry the ten scalar outputs and the status only
    if (q.memory == PROPS_MEM_HOST && (q.out.psi || q.out.alpha || q.out.hRT || q.out.iters))
        return fail(PROPS_EINVAL, "serve_submit: psi, alpha, hRT and iters need device-resident requests");
    const double *a, *b;
    mode_inputs(q, &a, &b);
    if (!q.in.Y || !a || !b) return fail(PROPS_EINVAL, "serve_submit: missing input arrays");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(PROPS_ENOTREADY, "serve_submit: server is shutting down");
    const uint64_t t = S->next_ticket++;
    Request &R = S->reqs[t];
    R.r = q;
    R.nchunks = (q.n + S->C - 1) / S->C;
    R.t_submit = S->now();
    if (!S->any_submit) {
        S->any_submit = true;
        S->t_first = R.t_submit;
    }
    S->active.push_back(t);
    S->submitted++;
    *ticket = t;
    S->cv.notify_all();
    return PROPS_OK;
}

int serve_wait(props_server_t S, uint64_t ticket, int64_t timeout_us, props_result *res)
{
    ApiRange range_("serve_wait");
    if (!S) return fail(PROPS_EINVAL, "serve_wait: null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(PROPS_EINVAL, "serve_wait: unknown or retired ticket %llu", (unsigned long long)ticket);
    Request &R = it->second;
    auto ready = [&] { return R.finished; };
    if (timeout_us < 0) S->cv.wait(lk, ready);
    else if (!S->cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
        return fail(PROPS_ETIMEDOUT, "serve_wait: ticket %llu not done after %lld us", (unsigned long long)ticket,
                    (long long)timeout_us);
    if (res) {
        res->rc = R.rc;
        res->n = R.r.n;
        res->t_submit = R.t_submit;
        res->t_done = R.t_done;
        res->latency_s = R.t_done - R.t_submit;
    }
    const int rc = R.rc;
    S->reqs.erase(it);
    if (rc) return fail(rc, "serve_wait: request %llu failed", (unsigned long long)ticket);
    return PROPS_OK;
}

int serve_stats(props_server_t S, props_serve_stats *st)
{
    if (!S || !st) return fail(PROPS_EINVAL, "serve_stats: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = S->submitted;
    st->completed = S->completed;
    st->failed = S->failed;
    int64_t q = 0;
    for (auto &kv : S->reqs)
        if (!kv.second.finished) q++;
    st->queued_requests = q;
    st->inflight_chunks = (int64_t)S->inflight.size();
    st->cells_done = S->cells_done;
    st->slots = (int64_t)S->slots.size();
    st->slot_bytes = (int64_t)S->slot_bytes;
    st->elapsed_s = S->any_submit ? S->t_last - S->t_first : 0.0;
    st->cells_per_s = st->elapsed_s > 0 ? S->cells_done / st->elapsed_s : 0.0;
    if (!S->lat.empty()) {
        std::vector<double> v = S->lat;
        std::sort(v.begin(), v.end());
        auto rank = [&](double p) {   // nearest-rank percentile
            size_t k = (size_t)std::ceil(p * v.size());
            return v[std::min(v.size() - 1, k ? k - 1 : 0)];
        };
        st->p50_s = rank(0.50);
        st->p99_s = rank(0.99);
        double s = 0;
        for (double x : v) s += x;
        st->mean_s = s / v.size();
        st->max_s = v.back();
    }
    return PROPS_OK;
}

void serve_destroy(props_server_t S)
{
    ApiRange range_("serve_destroy");
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    S->sched.join();
    S->compl_thr.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->cv.notify_all();
    }
    for (auto &w : S->workers) w.join();
    destroy_server(S);
}

}  // extern "C"
