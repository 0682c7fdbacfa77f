// Serving: concurrent GP runs submit population evaluations against
// datasets that stay resident in device memory.  A scheduler thread admits
// requests while their memory fits the budget, fuses the admitted requests
// into one batched launch and keeps up to n_streams launches in flight, so
// work that arrives while the GPU is busy starts as soon as a stream frees
// up (continuous batching).  Each request's fitness is bit-identical to its
// evaluation alone: partial sums are formed per fixed 256-case block.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gp.h"
#include "batch.h"
#include "core_host.h"
#include "runtime.h"

namespace gpx {

using Clock = std::chrono::steady_clock;

enum ReqState { RQ_QUEUED, RQ_RUNNING, RQ_DONE, RQ_CANCELLED, RQ_FAILED };

struct Request {
    uint64_t ticket = 0;
    ProgData pd;
    int32_t ds = 0;
    int32_t kind = 0;
    void* out = nullptr;
    size_t need = 0;
    int64_t gpop = 0;
    int32_t variant = -1;      // kernel variant the request runs with, alone or fused
    ReqState state = RQ_QUEUED;
    gp_status status = GP_OK;
    Clock::time_point t_submit, t_done;
};

struct InFlight {
    int stream = -1;
    hipEvent_t ev = nullptr;
    std::vector<std::shared_ptr<Request>> reqs;
    size_t bytes = 0;
    Clock::time_point t_launch;
    double fake_ms = 0.0;   // dry-run duration
};

struct Server {
    gp_serve_config cfg;
    std::vector<gp_dataset> datasets;
    std::mutex mu;
    std::condition_variable cv_sched;   // wakes the scheduler
    std::condition_variable cv_done;    // wakes waiters
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
    std::vector<InFlight> inflight;
    std::vector<hipStream_t> streams;
    std::vector<std::unique_ptr<BatchScratch>> scratch;
    std::vector<bool> stream_busy;
    size_t bytes_in_flight = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread th;
    // statistics
    int64_t n_submitted = 0, n_admitted = 0, n_completed = 0, n_rejected = 0, n_cancelled = 0, n_failed = 0;
    int64_t n_batches = 0, n_batched_reqs = 0;
    int64_t gpop_done = 0;
    bool have_first = false;
    Clock::time_point t_first, t_last;
    std::vector<double> lat_us;   // ring of recent latencies
    size_t lat_next = 0;
};

static const size_t kLatRing = 1 << 17;

static size_t request_bytes(const ProgData& pd, int64_t N) {
    const int64_t blocks = (N + 255) / 256;
    const int64_t tiles_min = (N + 255) / 256;  // widest tile gives the fewest units; bound with 4-slot tiles
    return pd.code.size() * 4 + pd.progs.size() * sizeof(DevProg) + pd.progs.size() * 4 +
           (size_t)blocks * (size_t)pd.n_prog * sizeof(double) +
           (size_t)tiles_min * (size_t)((pd.n_prog + 7) / 8) * sizeof(UnitDesc) + 4096;
}

static void record_latency(Server& S, double us) {
    if (S.lat_us.size() < kLatRing) S.lat_us.push_back(us);
    else S.lat_us[S.lat_next] = us;
    S.lat_next = (S.lat_next + 1) % kLatRing;
}

static void finish_batch(Server& S, InFlight& f, gp_status st) {
    const Clock::time_point now = Clock::now();
    for (auto& r : f.reqs) {
        if (st == GP_OK) {
            r->state = RQ_DONE;
            S.n_completed++;
            S.gpop_done += r->gpop;
        } else {
            r->state = RQ_FAILED;
            r->status = st;
            S.n_failed++;
        }
        r->t_done = now;
        S.t_last = now;
        record_latency(S, std::chrono::duration<double, std::micro>(now - r->t_submit).count());
        r->pd = ProgData();   // programs are no longer needed
    }
    S.bytes_in_flight -= f.bytes;
    if (f.stream >= 0) S.stream_busy[f.stream] = false;
    if (f.ev) (void)hipEventDestroy(f.ev);
    f.ev = nullptr;
}

// Launch one batch of admitted requests on stream slot k.  Runs on the
// scheduler thread without the server lock: it reads only the immutable
// configuration, the stream's own scratch and the taken requests (ds is a
// copy of the dataset list).
static gp_status launch_batch(Server& S, const std::vector<gp_dataset>& ds, int k,
                              std::vector<std::shared_ptr<Request>>& reqs, InFlight& f) {
    std::vector<BatchJobRef> refs;
    for (auto& r : reqs) refs.push_back(BatchJobRef{&r->pd, r->ds, r->kind, r->out});
    f.stream = k;
    f.reqs = reqs;
    f.t_launch = Clock::now();
    if (S.cfg.dry_run) {
        double gpop = 0;
        for (auto& r : reqs) gpop += (double)r->gpop;
        f.fake_ms = S.cfg.dry_run_gpops > 0 ? gpop / S.cfg.dry_run_gpops * 1e3 : 0.0;
        return GP_OK;
    }
    // every request of a batch has the same variant (the scheduler fuses only those)
    gp_batch_config c = default_config(refs);
    c.variant = reqs[0]->variant;
    if (c.variant < 0) return fail(GP_E_DEPTH, "no kernel variant can hold the batch");
    hipStream_t s = S.streams[(size_t)k % S.streams.size()];
    gp_status st = core_ready(c.variant, s);
    if (st != GP_OK) return st;
    BatchPlan plan;
    st = plan_batch(refs, ds, c, plan);
    if (st != GP_OK) return st;
    BatchScratch& sc = *S.scratch[k];
    std::lock_guard<std::mutex> g(sc.mu);
    // The stream's buffers only grow; when they hold more than this batch needs and more than the
    // stream's share of the budget, free them first, so memory held between batches stays bounded
    // (the free waits for the device, which is rare: only after an unusually large batch).
    const size_t held = sc.code.cap + sc.progs.cap + sc.order.cap + sc.units.cap + sc.jobs.cap + sc.datasets.cap +
                        sc.reduce.cap + sc.partials.cap + sc.counter.cap;
    const size_t need = plan_device_bytes(plan);
    if (held > need && held > S.cfg.memory_budget / (size_t)S.cfg.n_streams) {
        sc.code.release(); sc.progs.release(); sc.order.release(); sc.units.release(); sc.jobs.release();
        sc.datasets.release(); sc.reduce.release(); sc.partials.release(); sc.counter.release();
    }
    if ((st = upload_plan(plan, sc, s)) != GP_OK) return st;
    if ((st = launch_plan(plan, sc, s)) != GP_OK) return st;
    hipError_t e = hipEventCreateWithFlags(&f.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(f.ev, s);
    if (e != hipSuccess) return fail(GP_E_DEVICE, "event: %s", hipGetErrorString(e));
    return GP_OK;
}

static void scheduler(Server* Sp) {
    Server& S = *Sp;
    std::unique_lock<std::mutex> lk(S.mu);
    while (true) {
        // 1. retire finished batches
        bool progress = false;
        for (size_t i = 0; i < S.inflight.size();) {
            InFlight& f = S.inflight[i];
            bool done;
            gp_status st = GP_OK;
            if (S.cfg.dry_run) {
                done = std::chrono::duration<double, std::milli>(Clock::now() - f.t_launch).count() >= f.fake_ms;
            } else {
                hipError_t e = hipEventQuery(f.ev);
                done = e != hipErrorNotReady;
                if (done && e != hipSuccess) st = fail(GP_E_DEVICE, "batch failed: %s", hipGetErrorString(e));
            }
            if (done) {
                finish_batch(S, f, st);
                S.inflight.erase(S.inflight.begin() + (long)i);
                progress = true;
            } else {
                i++;
            }
        }
        if (progress) S.cv_done.notify_all();
        if (S.stop && S.inflight.empty()) break;
        // 2. admit and launch while a stream is free
        while (!S.stop && !S.queue.empty()) {
            int k = -1;
            for (size_t i = 0; i < S.stream_busy.size(); i++)
                if (!S.stream_busy[i]) { k = (int)i; break; }
            if (k < 0) break;
            // The oldest request leads the batch (FIFO: if it does not fit the
            // memory budget, nothing is admitted until memory frees up); later
            // requests join it if they run with the same kernel variant and fit.
            // A fused launch runs one variant: letting requests join the lead's
            // variant whenever it can run their programs fused more (6.4
            // requests per batch) but cost 6 % of throughput on the served
            // workload, since register programs and trees without sin/cos/exp/log
            // then ran on the slower variant with that code.
            std::vector<std::shared_ptr<Request>> take;
            size_t bytes = 0;
            int32_t variant = -1;
            for (auto it = S.queue.begin(); it != S.queue.end() && (int32_t)take.size() < S.cfg.max_batch;) {
                const std::shared_ptr<Request>& r = *it;
                if (r->state == RQ_CANCELLED) { it = S.queue.erase(it); continue; }
                if (!take.empty() && r->variant != variant) { ++it; continue; }
                if (S.bytes_in_flight + bytes + r->need > S.cfg.memory_budget) {
                    if (take.empty()) break;
                    ++it;
                    continue;
                }
                variant = r->variant;
                bytes += r->need;
                take.push_back(r);
                it = S.queue.erase(it);
            }
            if (take.empty()) break;
            for (auto& r : take) r->state = RQ_RUNNING;
            S.n_admitted += (int64_t)take.size();
            S.n_batches++;
            S.n_batched_reqs += (int64_t)take.size();
            InFlight f;
            f.bytes = bytes;
            S.bytes_in_flight += bytes;
            S.stream_busy[k] = true;
            // plan, translate, upload and launch without the lock, so clients keep submitting,
            // polling and waiting meanwhile
            const std::vector<gp_dataset> ds = S.datasets;
            lk.unlock();
            gp_status st = launch_batch(S, ds, k, take, f);
            lk.lock();
            if (st != GP_OK) {
                finish_batch(S, f, st);
                S.cv_done.notify_all();
            } else {
                S.inflight.push_back(f);
            }
        }
        // 3. sleep until something changes; poll the device while batches run
        if (S.inflight.empty()) S.cv_sched.wait(lk, [&] { return S.stop || !S.queue.empty(); });
        else S.cv_sched.wait_for(lk, std::chrono::microseconds(50));
    }
}

}  // namespace gpx

// ===========================================================================
// C ABI
// ===========================================================================
using namespace gpx;

struct gp_server {
    Server S;
};

extern "C" {

gp_status gp_serve_create(const gp_serve_config* cfg, gp_server** out) {
    clear_error();
    if (!out) return fail(GP_E_INVAL, "server pointer is null");
    std::unique_ptr<gp_server> sv(new gp_server());
    Server& S = sv->S;
    memset(&S.cfg, 0, sizeof S.cfg);
    if (cfg) S.cfg = *cfg;
    if (S.cfg.memory_budget == 0) S.cfg.memory_budget = (size_t)4 << 30;
    if (S.cfg.max_queue <= 0) S.cfg.max_queue = 1024;
    if (S.cfg.n_streams <= 0) S.cfg.n_streams = 2;
    if (S.cfg.max_batch <= 0) S.cfg.max_batch = 64;
    if (!S.cfg.batching) {
        S.cfg.n_streams = 1;
        S.cfg.max_batch = 1;
    }
    if (S.cfg.n_streams > 8) return fail(GP_E_INVAL, "at most 8 streams");
    if (S.cfg.hip_streams < 0) return fail(GP_E_INVAL, "hip_streams < 0");
    // one HIP stream by default: measured on the served workload, two batches sharing the CUs on two
    // streams gave 4-7 % over one launch per request with a 3-8 % higher p99; queued on one stream, 6-9 %
    // with the p99 within 1.3 %
    if (S.cfg.hip_streams == 0) S.cfg.hip_streams = 1;
    if (S.cfg.hip_streams > S.cfg.n_streams) S.cfg.hip_streams = S.cfg.n_streams;
    for (int i = 0; i < S.cfg.hip_streams; i++) {
        hipStream_t s = nullptr;
        if (!S.cfg.dry_run) {
            hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e != hipSuccess) {
                for (hipStream_t x : S.streams) (void)hipStreamDestroy(x);
                return fail(GP_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
            }
        }
        S.streams.push_back(s);
    }
    for (int i = 0; i < S.cfg.n_streams; i++) {   // launch slots: each has its own buffers
        S.scratch.emplace_back(new BatchScratch());
        S.stream_busy.push_back(false);
    }
    S.th = std::thread(scheduler, &S);
    *out = sv.release();
    return GP_OK;
}

gp_status gp_serve_add_dataset(gp_server* sv, const float* X, int32_t n_feat, int64_t n_cases, const float* y,
                               int32_t* id) {
    clear_error();
    if (!sv || !id) return fail(GP_E_INVAL, "null argument");
    gp_dataset d{X, n_feat, n_cases, y};
    gp_status st = check_datasets(&d, 1);
    if (st != GP_OK) return st;
    if (!y) return fail(GP_E_INVAL, "dataset needs targets");
    std::lock_guard<std::mutex> g(sv->S.mu);
    sv->S.datasets.push_back(d);
    *id = (int32_t)sv->S.datasets.size() - 1;
    return GP_OK;
}

gp_status gp_serve_submit(gp_server* sv, const gp_job* req, uint64_t* ticket) {
    clear_error();
    if (!sv || !req || !ticket) return fail(GP_E_INVAL, "null argument");
    Server& S = sv->S;
    std::vector<gp_dataset> ds;
    {
        std::lock_guard<std::mutex> g(S.mu);
        ds = S.datasets;  // datasets are only appended
    }
    auto r = std::make_shared<Request>();
    gp_status st = build_job(*req, ds.data(), (int32_t)ds.size(), r->pd);   // lowering on the caller's thread
    if (st != GP_OK) {
        std::lock_guard<std::mutex> g(S.mu);
        S.n_rejected++;
        return st;
    }
    r->ds = req->dataset;
    r->kind = req->kind;
    r->out = req->out;
    r->need = request_bytes(r->pd, ds[req->dataset].n_cases);
    r->gpop = r->pd.n_gpop * ds[req->dataset].n_cases;
    r->variant = pick_core_variant(r->pd.n_load, r->pd.max_depth,
                                   r->pd.n_instr ? (double)r->pd.n_transc / (double)r->pd.n_instr : 0.0,
                                   r->pd.n_transc > 0);
    if (r->variant < 0 && r->pd.n_prog > 0) {
        std::lock_guard<std::mutex> g(S.mu);
        S.n_rejected++;
        return fail(GP_E_DEPTH, "no kernel variant can hold the request's programs");
    }
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> g(S.mu);
    if (r->need > S.cfg.memory_budget) {
        S.n_rejected++;
        return fail(GP_E_NOMEM, "request needs %zu bytes, the budget is %zu", r->need, S.cfg.memory_budget);
    }
    if ((int32_t)S.queue.size() >= S.cfg.max_queue) {
        S.n_rejected++;
        return fail(GP_E_AGAIN, "admission queue is full (%d requests)", S.cfg.max_queue);
    }
    r->ticket = S.next_ticket++;
    if (r->pd.n_prog == 0) {
        r->state = RQ_DONE;
        r->t_done = r->t_submit;
    } else {
        S.queue.push_back(r);
    }
    S.all[r->ticket] = r;
    S.n_submitted++;
    if (!S.have_first) {
        S.have_first = true;
        S.t_first = r->t_submit;
    }
    *ticket = r->ticket;
    S.cv_sched.notify_one();
    return GP_OK;
}

static gp_status request_status(Server& S, uint64_t ticket, std::shared_ptr<Request>& r) {
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return fail(GP_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    r = it->second;
    return GP_OK;
}

gp_status gp_serve_poll(gp_server* sv, uint64_t ticket, int32_t* done) {
    clear_error();
    if (!sv || !done) return fail(GP_E_INVAL, "null argument");
    std::lock_guard<std::mutex> g(sv->S.mu);
    std::shared_ptr<Request> r;
    gp_status st = request_status(sv->S, ticket, r);
    if (st != GP_OK) return st;
    *done = r->state == RQ_DONE || r->state == RQ_FAILED || r->state == RQ_CANCELLED;
    return r->state == RQ_FAILED ? r->status : GP_OK;
}

gp_status gp_serve_wait(gp_server* sv, uint64_t ticket, int64_t timeout_us) {
    clear_error();
    if (!sv) return fail(GP_E_INVAL, "null server");
    Server& S = sv->S;
    std::unique_lock<std::mutex> lk(S.mu);
    std::shared_ptr<Request> r;
    gp_status st = request_status(S, ticket, r);
    if (st != GP_OK) return st;
    auto finished = [&] { return r->state == RQ_DONE || r->state == RQ_FAILED || r->state == RQ_CANCELLED; };
    if (timeout_us < 0) S.cv_done.wait(lk, finished);
    else if (!S.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), finished))
        return fail(GP_E_TIMEOUT, "ticket %llu not finished after %lld us", (unsigned long long)ticket,
                    (long long)timeout_us);
    if (r->state == RQ_FAILED) return r->status;
    if (r->state == RQ_CANCELLED) return fail(GP_E_NOTFOUND, "ticket %llu was cancelled", (unsigned long long)ticket);
    return GP_OK;
}

gp_status gp_serve_cancel(gp_server* sv, uint64_t ticket) {
    clear_error();
    if (!sv) return fail(GP_E_INVAL, "null server");
    Server& S = sv->S;
    std::lock_guard<std::mutex> g(S.mu);
    std::shared_ptr<Request> r;
    gp_status st = request_status(S, ticket, r);
    if (st != GP_OK) return st;
    if (r->state != RQ_QUEUED) return fail(GP_E_AGAIN, "ticket %llu is already admitted", (unsigned long long)ticket);
    r->state = RQ_CANCELLED;
    r->t_done = Clock::now();
    S.n_cancelled++;
    S.cv_done.notify_all();
    return GP_OK;
}

gp_status gp_serve_release(gp_server* sv, uint64_t ticket) {
    clear_error();
    if (!sv) return fail(GP_E_INVAL, "null server");
    Server& S = sv->S;
    std::lock_guard<std::mutex> g(S.mu);
    std::shared_ptr<Request> r;
    gp_status st = request_status(S, ticket, r);
    if (st != GP_OK) return st;
    if (r->state == RQ_QUEUED || r->state == RQ_RUNNING)
        return fail(GP_E_AGAIN, "ticket %llu is still pending", (unsigned long long)ticket);
    S.all.erase(ticket);
    return GP_OK;
}

gp_status gp_serve_stats(gp_server* sv, gp_serve_stats_t* out) {
    clear_error();
    if (!sv || !out) return fail(GP_E_INVAL, "null argument");
    Server& S = sv->S;
    std::lock_guard<std::mutex> g(S.mu);
    memset(out, 0, sizeof *out);
    out->submitted = S.n_submitted;
    out->admitted = S.n_admitted;
    out->completed = S.n_completed;
    out->rejected = S.n_rejected;
    out->cancelled = S.n_cancelled;
    out->failed = S.n_failed;
    out->queue_depth = (int32_t)S.queue.size();
    out->in_flight_batches = (int32_t)S.inflight.size();
    out->bytes_in_flight = (int64_t)S.bytes_in_flight;
    out->batches = S.n_batches;
    out->mean_batch = S.n_batches ? (double)S.n_batched_reqs / (double)S.n_batches : 0.0;
    if (!S.lat_us.empty()) {
        std::vector<double> v = S.lat_us;
        std::sort(v.begin(), v.end());
        out->p50_us = v[(v.size() - 1) / 2];
        out->p99_us = v[(size_t)((v.size() - 1) * 0.99)];
    }
    if (S.have_first && S.n_completed > 0) {
        const double sec = std::chrono::duration<double>(S.t_last - S.t_first).count();
        out->gpops_per_s = sec > 0 ? (double)S.gpop_done / sec : 0.0;
    }
    return GP_OK;
}

gp_status gp_serve_destroy(gp_server* sv) {
    clear_error();
    if (!sv) return GP_OK;
    Server& S = sv->S;
    {
        std::lock_guard<std::mutex> g(S.mu);
        S.stop = true;
        for (auto& r : S.queue) {
            if (r->state == RQ_QUEUED) {
                r->state = RQ_CANCELLED;
                S.n_cancelled++;
            }
        }
        S.queue.clear();
    }
    S.cv_sched.notify_all();
    if (S.th.joinable()) S.th.join();   // drains batches already on the device
    S.cv_done.notify_all();
    for (hipStream_t s : S.streams)
        if (s) (void)hipStreamDestroy(s);
    for (auto& sc : S.scratch) {
        sc->code.release(); sc->progs.release(); sc->order.release(); sc->units.release();
        sc->jobs.release(); sc->datasets.release(); sc->reduce.release(); sc->partials.release();
        sc->counter.release();
        sc->staging.release();
    }
    delete sv;
    return GP_OK;
}

}  // extern "C"
