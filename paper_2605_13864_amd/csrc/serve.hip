// The request loop (serving) in native code: a server thread that admits
// transpose and sum jobs by HBM budget and batches them continuously onto K
// streams (the policy of serve_policy.h), with completion times read from
// device events.  Jobs name device-resident inputs and outputs the caller
// owns; the loop allocates nothing per job.
//
// Clock: steady host nanoseconds (xtr_server_clock_ns).  A job becomes
// visible to the loop at its arrival time (now, or the time it carries, so a
// client may hand over a whole arrival schedule at once).  Its completion time
// is the device time of its unit's completion event, placed on the host clock
// through a reference event recorded (and waited for) when the server starts:
// done = t_ref + elapsed(reference event, completion event).
#include "common.hpp"
#include "serve_policy.h"

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

namespace xtr {
namespace {

int64_t clock_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr int MAX_STREAMS = 8;

// Launches units on the server's streams and reads their completion events.
struct GpuExec {
    hipStream_t streams[MAX_STREAMS] = {};
    int nstreams = 0;
    bool batching = true;
    hipEvent_t ref = nullptr;
    int64_t t_ref = 0;
    std::vector<hipEvent_t> events;     // by handle
    std::vector<int64_t> free_handles;
    const std::vector<xtr_job> *jobs = nullptr;
    int64_t launches = 0;
    std::vector<xtr_tpose_desc> descs;
    std::vector<const void *> srcs;
    std::vector<int64_t> ns;
    std::vector<void *> outs;

    int64_t launch(const std::vector<srv::Pending> &unit, int si) {
        hipStream_t st = streams[si];
        const std::vector<xtr_job> &J = *jobs;
        int rc = XTR_OK;
        if (batching) {
            descs.clear();
            for (const srv::Pending &p : unit) {
                const xtr_job &j = J[p.id];
                if (j.kind != 0) continue;
                descs.push_back(xtr_tpose_desc{j.src, j.dst, j.rows, j.cols, j.cols, j.rows,
                                               j.dtype, 0});
            }
            if (!descs.empty()) {
                rc = tpose_batched(descs.data(), (int64_t)descs.size(), st);
                launches++;
            }
            for (int dt : {XTR_F32, XTR_F16, XTR_BF16, XTR_F8E4M3, XTR_I32, XTR_I64}) {
                srcs.clear();
                ns.clear();
                outs.clear();
                for (const srv::Pending &p : unit) {
                    const xtr_job &j = J[p.id];
                    if (j.kind != 1 || j.dtype != dt) continue;
                    srcs.push_back(j.src);
                    ns.push_back(j.n);
                    outs.push_back(j.dst);
                }
                if (srcs.empty() || rc) continue;
                rc = reduce_sum_batched_scatter(srcs.data(), ns.data(), outs.data(),
                                                (int64_t)srcs.size(), dt, st);
                launches++;
            }
        } else {
            for (const srv::Pending &p : unit) {
                const xtr_job &j = J[p.id];
                rc = j.kind == 0 ? tpose(j.src, j.dst, j.rows, j.cols, j.cols, j.rows, j.dtype, st)
                                 : reduce_sum(j.src, j.n, j.dst, j.dtype, st);
                launches++;
                if (rc) break;
            }
        }
        if (rc) return -1;
        int64_t h;
        if (!free_handles.empty()) {
            h = free_handles.back();
            free_handles.pop_back();
        } else {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            h = (int64_t)events.size();
            events.push_back(e);
        }
        if (hipEventRecord(events[h], st) != hipSuccess) return -1;
        return h;
    }

    int64_t done(int64_t h) {
        const hipError_t q = hipEventQuery(events[h]);
        if (q == hipErrorNotReady) return -1;
        float ms = 0.f;
        if (q != hipSuccess || hipEventElapsedTime(&ms, ref, events[h]) != hipSuccess) {
            free_handles.push_back(h);
            return clock_ns();   // the unit has ended; its device time is unknown
        }
        free_handles.push_back(h);
        return t_ref + (int64_t)((double)ms * 1e6);
    }
};

}  // namespace
}  // namespace xtr

struct xtr_server {
    xtr_server_config cfg{};
    int device = 0;
    xtr::GpuExec ex;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<xtr_job> jobs;            // every job submitted, by id (worker reads [0, seen))
    std::vector<int64_t> arrival;         // arrival time actually used, by id
    std::vector<int64_t> done;            // completion time (-1 pending, -2 failed), by id
    int64_t submitted = 0;                // guarded by mu
    int64_t completed = 0;                // guarded by mu
    bool stop = false;
    int64_t max_inflight = 0, units = 0, failed = 0, launches = 0;
    std::vector<int64_t> admit_order;

    void run();
};

void xtr_server::run() {
    using namespace xtr;
    (void)hipSetDevice(device);
    srv::Scheduler<GpuExec> sch(ex, cfg.budget_bytes, cfg.batching != 0, cfg.nstreams,
                                cfg.small_job_bytes);
    std::vector<int64_t> dn;              // worker-side completion times
    std::vector<int64_t> fin;             // ids finished in this pass
    std::vector<xtr_job> local;           // worker-side copy of the jobs
    int64_t seen = 0, next = 0;
    ex.jobs = &local;
    for (;;) {
        bool stopping;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (seen < submitted) {
                local.insert(local.end(), jobs.begin() + seen, jobs.begin() + submitted);
                dn.resize((size_t)submitted, -1);
                seen = submitted;
            }
            stopping = stop;
        }
        const int64_t now = clock_ns();
        while (next < seen && local[next].arrival_ns <= now) {
            const xtr_job &j = local[next];
            const int eb = elem_bytes(j.dtype);
            const int64_t bytes = j.kind == 0 ? 2 * j.rows * j.cols * eb : j.n * eb + 8;
            sch.arrive(srv::Pending{next, bytes, j.kind, 0});
            next++;
        }
        fin.clear();
        const bool launched = sch.step(now, dn, fin);
        const int64_t newly = (int64_t)fin.size();
        {   // publish
            std::lock_guard<std::mutex> lk(mu);
            for (int64_t id : fin) done[id] = dn[id];
            completed += newly;
            max_inflight = sch.max_used;
            units = sch.units;
            failed = sch.failed;
            launches = ex.launches;
        }
        if (newly) cv_done.notify_all();
        if (stopping && next == seen && sch.idle()) break;
        if (launched) continue;
        if (sch.idle() && next == seen) {      // nothing to do until a submission
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait_for(lk, std::chrono::milliseconds(1),
                             [&] { return submitted > seen || stop; });
            continue;
        }
        if (sch.idle() && next < seen && local[next].arrival_ns - now > 200000)
            std::this_thread::sleep_for(std::chrono::microseconds(50));   // next arrival is far
        else
            std::this_thread::yield();                                     // poll events
    }
    std::lock_guard<std::mutex> lk(mu);
    admit_order = sch.admit_order;
}

extern "C" {

int64_t xtr_server_clock_ns(void) { return xtr::clock_ns(); }

int xtr_server_create(const xtr_server_config *cfg, xtr_server **out) {
    using namespace xtr;
    if (!out) return fail(XTR_EINVAL, "xtr_server_create: null result pointer");
    *out = nullptr;
    if (!cfg) return fail(XTR_EINVAL, "xtr_server_create: null config");
    if (cfg->nstreams < 1 || cfg->nstreams > MAX_STREAMS || cfg->budget_bytes <= 0 ||
        cfg->small_job_bytes < 0)
        return fail(XTR_EINVAL, "xtr_server_create: nstreams in [1, %d], budget > 0, "
                    "small_job_bytes >= 0", MAX_STREAMS);
    auto *s = new (std::nothrow) xtr_server();
    if (!s) return fail(XTR_ENOMEM, "xtr_server_create: out of host memory");
    s->cfg = *cfg;
    s->ex.nstreams = cfg->nstreams;
    s->ex.batching = cfg->batching != 0;
    hipError_t e = hipGetDevice(&s->device);
    for (int i = 0; i < cfg->nstreams && e == hipSuccess; i++)
        e = hipStreamCreateWithFlags(&s->ex.streams[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&s->ex.ref);
    if (e == hipSuccess) e = hipEventRecord(s->ex.ref, s->ex.streams[0]);
    if (e == hipSuccess) e = hipEventSynchronize(s->ex.ref);
    if (e != hipSuccess) {
        for (int i = 0; i < MAX_STREAMS; i++)
            if (s->ex.streams[i]) (void)hipStreamDestroy(s->ex.streams[i]);
        if (s->ex.ref) (void)hipEventDestroy(s->ex.ref);
        delete s;
        return hip_fail(e, "xtr_server_create");
    }
    s->ex.t_ref = clock_ns();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return XTR_OK;
}

int xtr_server_submit(xtr_server *s, const xtr_job *jobs, int64_t count, int64_t *first_id) {
    using namespace xtr;
    if (!s || (count > 0 && !jobs)) return fail(XTR_EINVAL, "xtr_server_submit: null argument");
    if (count < 0) return fail(XTR_EINVAL, "xtr_server_submit: negative count");
    for (int64_t i = 0; i < count; i++) {
        const xtr_job &j = jobs[i];
        const int eb = elem_bytes(j.dtype);
        if (j.kind == 0) {
            if (!eb || j.rows < 0 || j.cols < 0 || ((j.rows && j.cols) && (!j.src || !j.dst)))
                return fail(XTR_EINVAL, "xtr_server_submit: job %lld: bad transpose", (long long)i);
        } else if (j.kind == 1) {
            if (!(is_float_sum_dtype(j.dtype) || is_int_sum_dtype(j.dtype)))
                return fail(XTR_EDTYPE, "xtr_server_submit: job %lld: dtype not summable", (long long)i);
            if (j.n < 0 || !j.dst || (j.n && !j.src))
                return fail(XTR_EINVAL, "xtr_server_submit: job %lld: bad sum", (long long)i);
        } else {
            return fail(XTR_EINVAL, "xtr_server_submit: job %lld: kind %d", (long long)i, j.kind);
        }
        const int64_t bytes = j.kind == 0 ? 2 * j.rows * j.cols * eb : j.n * eb + 8;
        if (bytes > s->cfg.budget_bytes)
            return fail(XTR_EBUDGET, "xtr_server_submit: job %lld needs %lld bytes, more than the "
                        "budget", (long long)i, (long long)bytes);
    }
    const int64_t now = clock_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(XTR_EINVAL, "xtr_server_submit: server stopped");
        if (first_id) *first_id = s->submitted;
        int64_t last = s->jobs.empty() ? 0 : s->jobs.back().arrival_ns;
        for (int64_t i = 0; i < count; i++) {
            xtr_job j = jobs[i];
            if (j.arrival_ns < 0) j.arrival_ns = now;
            if (j.arrival_ns < last) j.arrival_ns = last;   // arrivals never go back in time
            last = j.arrival_ns;
            s->jobs.push_back(j);
            s->arrival.push_back(j.arrival_ns);
            s->done.push_back(-1);
        }
        s->submitted += count;
    }
    s->cv_work.notify_one();
    return XTR_OK;
}

int xtr_server_drain(xtr_server *s, int64_t timeout_ms) {
    using namespace xtr;
    if (!s) return fail(XTR_EINVAL, "xtr_server_drain: null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto all = [&] { return s->completed == s->submitted; };
    if (timeout_ms < 0) s->cv_done.wait(lk, all);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), all))
        return fail(XTR_EINVAL, "xtr_server_drain: %lld of %lld jobs done after %lld ms",
                    (long long)s->completed, (long long)s->submitted, (long long)timeout_ms);
    return s->failed ? fail(XTR_EHIP, "xtr_server_drain: %lld jobs failed to launch",
                            (long long)s->failed)
                     : XTR_OK;
}

int xtr_server_times(xtr_server *s, int64_t first, int64_t count, int64_t *arrival_ns,
                     int64_t *done_ns) {
    using namespace xtr;
    if (!s) return fail(XTR_EINVAL, "xtr_server_times: null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (first < 0 || count < 0 || first + count > s->submitted)
        return fail(XTR_EINVAL, "xtr_server_times: range outside the submitted jobs");
    for (int64_t i = 0; i < count; i++) {
        if (arrival_ns) arrival_ns[i] = s->arrival[first + i];
        if (done_ns) done_ns[i] = s->done[first + i];
    }
    return XTR_OK;
}

int xtr_server_get_stats(xtr_server *s, xtr_server_stats *st) {
    using namespace xtr;
    if (!s || !st) return fail(XTR_EINVAL, "xtr_server_get_stats: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *st = xtr_server_stats{};
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->launches = s->launches;
    st->units = s->units;
    st->max_inflight_bytes = s->max_inflight;
    return XTR_OK;
}

int xtr_server_destroy(xtr_server *s) {
    if (!s) return XTR_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_one();
    if (s->worker.joinable()) s->worker.join();   // it drains every submitted job first
    for (int i = 0; i < xtr::MAX_STREAMS; i++)
        if (s->ex.streams[i]) {
            (void)hipStreamSynchronize(s->ex.streams[i]);
            (void)hipStreamDestroy(s->ex.streams[i]);
        }
    for (hipEvent_t e : s->ex.events) (void)hipEventDestroy(e);
    if (s->ex.ref) (void)hipEventDestroy(s->ex.ref);
    delete s;
    return XTR_OK;
}

}  // extern "C"
