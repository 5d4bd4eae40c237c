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
// Graph mode: at most this many jobs of a kind share a unit, so that every
// batched launch carries its job table in the kernel arguments (no table
// upload, so a unit's graph holds kernel nodes only).
constexpr int GRAPH_MAX_PER_KIND = 24;
constexpr int MAX_GRAPHS = 64;   // cached executable graphs per server

// One executable graph of a unit's launches.  `nodes` are the kernel nodes of
// the graph it was built from (kept alive: they name the exec's nodes); a
// later unit whose captured launches have the same kernels, grids and block
// shapes, on the same stream, is run by giving these nodes the new kernel
// arguments.  `ev` is recorded after each launch: a graph is given new
// arguments only once its previous launch has completed.
struct UnitGraph {
    int stream = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    std::vector<const void *> funcs;
    std::vector<dim3> grids, blocks;
    hipEvent_t ev = nullptr;
};

// Launches units on the server's streams and reads their completion events.
struct GpuExec {
    hipStream_t streams[MAX_STREAMS] = {};
    hipStream_t copy = nullptr;         // host-to-device copies of host-resident inputs
    int nstreams = 0;
    bool batching = true;
    bool graphs = false;
    hipEvent_t ref = nullptr;
    int64_t t_ref = 0;
    std::vector<hipEvent_t> events;     // by handle: the unit's completion
    std::vector<hipEvent_t> copied;     // by handle: its inputs' copies
    std::vector<int64_t> free_handles;
    const std::vector<xtr_job> *jobs = nullptr;
    int64_t launches = 0, graph_launches = 0, graph_builds = 0, host_copies = 0;
    std::vector<xtr_tpose_desc> descs;
    std::vector<const void *> srcs;
    std::vector<int64_t> ns;
    std::vector<void *> outs;
    std::vector<UnitGraph> cache;

    // The unit's launches on stream st (eager, or recorded by a capture).
    // A kind or dtype with a single job in the unit takes the single-job
    // entry point (the same kernels as one launch per job).
    int enqueue(const std::vector<srv::Pending> &unit, hipStream_t st) {
        const std::vector<xtr_job> &J = *jobs;
        int rc = XTR_OK;
        if (!batching) {
            for (const srv::Pending &p : unit) {
                const xtr_job &j = J[p.id];
                rc = j.kind == 0 ? tpose(j.src, j.dst, j.rows, j.cols, j.cols, j.rows, j.dtype, st)
                                 : reduce_sum(j.src, j.n, j.dst, j.dtype, st);
                launches++;
                if (rc) return rc;
            }
            return XTR_OK;
        }
        descs.clear();
        for (const srv::Pending &p : unit) {
            const xtr_job &j = J[p.id];
            if (j.kind != 0) continue;
            descs.push_back(xtr_tpose_desc{j.src, j.dst, j.rows, j.cols, j.cols, j.rows, j.dtype, 0});
        }
        if (descs.size() == 1) {
            const xtr_tpose_desc &d = descs[0];
            rc = tpose(d.src, d.dst, d.rows, d.cols, d.ld_src, d.ld_dst, d.dtype, st);
            launches++;
        } else if (!descs.empty()) {
            rc = tpose_batched(descs.data(), (int64_t)descs.size(), st);
            launches++;
        }
        for (int dt : {XTR_F32, XTR_F16, XTR_BF16, XTR_F8E4M3, XTR_I32, XTR_I64}) {
            if (rc) return rc;
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
            if (srcs.empty()) continue;
            rc = srcs.size() == 1 ? reduce_sum(srcs[0], ns[0], outs[0], dt, st)
                                  : reduce_sum_batched_scatter(srcs.data(), ns.data(), outs.data(),
                                                               (int64_t)srcs.size(), dt, st);
            launches++;
        }
        return rc;
    }

    // The unit's launches captured into a graph and run from a cached
    // executable graph of the same shape (built on first use).  Returns a HIP
    // error, or hipErrorNotSupported when the unit cannot run this way (the
    // caller then launches it eagerly; nothing has been enqueued).
    hipError_t run_graph(const std::vector<srv::Pending> &unit, int si) {
        hipStream_t st = streams[si];
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return e;
        const int64_t l0 = launches;
        const int rc = enqueue(unit, st);
        launches = l0;
        e = hipStreamEndCapture(st, &g);
        if (rc != XTR_OK || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return hipErrorNotSupported;
        }
        size_t n = 0;
        std::vector<hipGraphNode_t> nodes;
        std::vector<hipKernelNodeParams> prm;
        e = hipGraphGetNodes(g, nullptr, &n);
        if (e == hipSuccess && n > 0) {
            nodes.resize(n);
            e = hipGraphGetNodes(g, nodes.data(), &n);
        }
        bool kernels_only = e == hipSuccess && n > 0;
        for (size_t i = 0; kernels_only && i < n; i++) {
            hipGraphNodeType t;
            if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess || t != hipGraphNodeTypeKernel) {
                kernels_only = false;
                break;
            }
            hipKernelNodeParams kp{};
            if (hipGraphKernelNodeGetParams(nodes[i], &kp) != hipSuccess) kernels_only = false;
            prm.push_back(kp);
        }
        if (!kernels_only) {
            (void)hipGraphDestroy(g);
            return hipErrorNotSupported;
        }
        auto same_shape = [&](const UnitGraph &c) {
            if (c.stream != si || c.nodes.size() != n) return false;
            for (size_t i = 0; i < n; i++)
                if (c.funcs[i] != prm[i].func || c.grids[i].x != prm[i].gridDim.x ||
                    c.grids[i].y != prm[i].gridDim.y || c.grids[i].z != prm[i].gridDim.z ||
                    c.blocks[i].x != prm[i].blockDim.x || c.blocks[i].y != prm[i].blockDim.y ||
                    c.blocks[i].z != prm[i].blockDim.z)
                    return false;
            return true;
        };
        UnitGraph *use = nullptr;
        for (UnitGraph &c : cache)
            if (same_shape(c) && hipEventQuery(c.ev) == hipSuccess) {
                use = &c;
                break;
            }
        if (use) {
            for (size_t i = 0; i < n && e == hipSuccess; i++)
                e = hipGraphExecKernelNodeSetParams(use->exec, use->nodes[i], &prm[i]);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
        } else {
            if ((int)cache.size() >= MAX_GRAPHS) {
                (void)hipGraphDestroy(g);
                return hipErrorNotSupported;
            }
            UnitGraph c;
            c.stream = si;
            c.graph = g;
            c.nodes = nodes;
            for (size_t i = 0; i < n; i++) {
                c.funcs.push_back(prm[i].func);
                c.grids.push_back(prm[i].gridDim);
                c.blocks.push_back(prm[i].blockDim);
            }
            e = hipEventCreateWithFlags(&c.ev, hipEventDisableTiming);
            if (e == hipSuccess) e = hipGraphInstantiate(&c.exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                if (c.ev) (void)hipEventDestroy(c.ev);
                (void)hipGraphDestroy(g);
                return e;
            }
            graph_builds++;
            cache.push_back(std::move(c));
            use = &cache.back();
        }
        e = hipGraphLaunch(use->exec, st);
        if (e == hipSuccess) e = hipEventRecord(use->ev, st);
        if (e == hipSuccess) {
            graph_launches++;
            launches += (int64_t)n;
        }
        return e;
    }

    int64_t handle() {
        if (!free_handles.empty()) {
            const int64_t h = free_handles.back();
            free_handles.pop_back();
            return h;
        }
        hipEvent_t e = nullptr, c = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        if (hipEventCreateWithFlags(&c, hipEventDisableTiming) != hipSuccess) {
            (void)hipEventDestroy(e);
            return -1;
        }
        events.push_back(e);
        copied.push_back(c);
        return (int64_t)events.size() - 1;
    }

    int64_t launch(const std::vector<srv::Pending> &unit, int si) {
        hipStream_t st = streams[si];
        const std::vector<xtr_job> &J = *jobs;
        const int64_t h = handle();
        if (h < 0) return -1;
        // host-resident inputs: copied to their device buffers on the copy
        // stream; the unit's kernels wait for those copies only, so they
        // overlap every other unit's kernels
        bool any_host = false;
        for (const srv::Pending &p : unit) {
            const xtr_job &j = J[p.id];
            if (!j.host_src) continue;
            const size_t nb = (size_t)(j.kind == 0 ? j.rows * j.cols : j.n) * elem_bytes(j.dtype);
            if (nb && hipMemcpyAsync(const_cast<void *>(j.src), j.host_src, nb,
                                     hipMemcpyHostToDevice, copy) != hipSuccess) {
                free_handles.push_back(h);
                return -1;
            }
            host_copies++;
            any_host = true;
        }
        if (any_host && (hipEventRecord(copied[h], copy) != hipSuccess ||
                         hipStreamWaitEvent(st, copied[h], 0) != hipSuccess)) {
            free_handles.push_back(h);
            return -1;
        }
        hipError_t ge = hipErrorNotSupported;
        if (graphs) ge = run_graph(unit, si);
        if (ge == hipErrorNotSupported) {
            if (enqueue(unit, st) != XTR_OK) {
                free_handles.push_back(h);
                return -1;
            }
        } else if (ge != hipSuccess) {
            free_handles.push_back(h);
            return -1;
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

    void release() {
        for (UnitGraph &c : cache) {
            if (c.ev) {
                (void)hipEventSynchronize(c.ev);
                (void)hipEventDestroy(c.ev);
            }
            if (c.exec) (void)hipGraphExecDestroy(c.exec);
            if (c.graph) (void)hipGraphDestroy(c.graph);
        }
        cache.clear();
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipEvent_t e : copied) (void)hipEventDestroy(e);
        events.clear();
        copied.clear();
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
    int64_t graph_launches = 0, graph_builds = 0, host_copies = 0;
    std::vector<int64_t> admit_order;

    void run();
};

void xtr_server::run() {
    using namespace xtr;
    (void)hipSetDevice(device);
    srv::Scheduler<GpuExec> sch(ex, cfg.budget_bytes, cfg.batching != 0, cfg.nstreams,
                                cfg.small_job_bytes, cfg.big_lane != 0,
                                cfg.graphs ? GRAPH_MAX_PER_KIND : 0);
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
            graph_launches = ex.graph_launches;
            graph_builds = ex.graph_builds;
            host_copies = ex.host_copies;
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
    s->ex.graphs = cfg->graphs != 0;
    hipError_t e = hipGetDevice(&s->device);
    for (int i = 0; i < cfg->nstreams && e == hipSuccess; i++)
        e = hipStreamCreateWithFlags(&s->ex.streams[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->ex.copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&s->ex.ref);
    if (e == hipSuccess) e = hipEventRecord(s->ex.ref, s->ex.streams[0]);
    if (e == hipSuccess) e = hipEventSynchronize(s->ex.ref);
    if (e != hipSuccess) {
        for (int i = 0; i < MAX_STREAMS; i++)
            if (s->ex.streams[i]) (void)hipStreamDestroy(s->ex.streams[i]);
        if (s->ex.copy) (void)hipStreamDestroy(s->ex.copy);
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
        if (j.host_src && !host_pinned(j.host_src))
            return fail(XTR_EINVAL, "xtr_server_submit: job %lld: host_src is not page-locked "
                        "host memory", (long long)i);
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
    st->graph_launches = s->graph_launches;
    st->graph_builds = s->graph_builds;
    st->host_copies = s->host_copies;
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
    if (s->ex.copy) {
        (void)hipStreamSynchronize(s->ex.copy);
        (void)hipStreamDestroy(s->ex.copy);
    }
    s->ex.release();
    if (s->ex.ref) (void)hipEventDestroy(s->ex.ref);
    delete s;
    return XTR_OK;
}

}  // extern "C"
