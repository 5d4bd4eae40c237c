"""Continuous-batching request loop for transpose and sum jobs on one GPU.

A job arrives at a time given by a Poisson stream and names a device-resident
input (a pool generated once) and an operation.  Each scheduler step

  1. retires finished batches (their completion events have fired), freeing
     HBM budget and output slots;
  2. moves arrived jobs to the pending queue;
  3. admits pending jobs in FIFO order while the in-flight bytes (input +
     output of every admitted, unfinished job) stay within the HBM budget and
     an output slot of the job's class is free;
  4. splits the jobs admitted in this step into launch units -- the jobs
     under 4 MiB of each kind together, every larger job alone (it is
     bandwidth-bound and gains nothing from sharing a launch) unless jobs are
     left waiting, when the larger jobs of a kind share a unit as well (then
     launches are the scarce resource) -- and launches
     each unit at once on the next of K streams: transposes as one persistent
     launch per element size (tpose_batched), sums as one launch per dtype
     (reduce_sum_batched_scatter, straight into each job's output slot); each
     unit ends with its own completion event.

Jobs that arrive while others run therefore join the next unit as soon as
budget and slots free up, and units on different streams overlap on the
device.  Latency is arrival -> completion of the job's unit, the completion
time read from the device event (elapsed time since a reference event whose
host time is known).  With ``batching=False`` every admitted job is its own
unit and launch, with its own event (the comparison).

The policy (`Scheduler`) is separate from the device (`GpuExecutor`), so the
admission and batching rules are tested on the CPU with a fake clock and a
fake executor.

`run_native` serves the same jobs with the library's native loop
(`xtr_server_*`: the same policy in C++, csrc/serve_policy.h, on a server
thread, so no Python runs between an arrival and its launch); `run` is this
module's Python loop with the same policy plus per-class output slots.  The
benchmark uses the native loop.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np


@dataclass
class Pending:
    idx: int
    job: object              # workloads.Job
    nbytes: int
    cls: tuple
    slot: int = -1


@dataclass
class Batch:
    jobs: list
    handle: object


def job_class(j) -> tuple:
    return ("tpose", j.dtype, j.rows) if j.kind == "tpose" else ("sum", j.dtype)


SMALL_JOB_BYTES = 4 << 20


def launch_units(group, batching: bool, backlog: bool = False) -> list:
    """The launch units of the jobs admitted in one step: with batching, the
    small jobs of each kind form one unit (one launch per element size or
    dtype instead of one per job) and every large job is a unit of its own (it
    is bandwidth-bound, so sharing a launch would only make it wait for the
    others) -- unless jobs are left waiting (`backlog`): then launches are the
    scarce resource and the large jobs of a kind share a unit too.  Without
    batching, one unit per job.  Admission order is kept."""
    if not batching:
        return [[p] for p in group]
    shared, units = {}, []
    for p in group:
        if backlog or p.nbytes < SMALL_JOB_BYTES:
            key = (p.job.kind, p.nbytes < SMALL_JOB_BYTES)
            if key not in shared:
                shared[key] = []
                units.append(shared[key])
            shared[key].append(p)
        else:
            units.append([p])
    return units


class SlotPool:
    """Free-lists of output slots per job class (the slot limit of admission)."""

    def __init__(self, counts: dict):
        self.free = {c: list(range(n))[::-1] for c, n in counts.items()}

    def take(self, c) -> int:
        fl = self.free.get(c)
        return fl.pop() if fl else -1

    def give(self, c, s):
        self.free[c].append(s)


class Scheduler:
    """Admission + continuous batching policy, independent of the device."""

    def __init__(self, jobs, arrivals, slots: SlotPool, executor, budget=64 << 30,
                 batching=True, nstreams=4):
        self.jobs, self.arrivals = jobs, arrivals
        self.slots, self.ex = slots, executor
        self.budget, self.batching, self.nstreams = budget, batching, nstreams
        self.pending = collections.deque()
        self.inflight = []
        self.used = 0
        self.max_used = 0
        self.nxt = 0
        self.si = 0
        self.batches = 0
        self.launches = 0
        self.admit_order = []
        self.done_t = np.full(len(jobs), np.nan)

    def finished(self) -> bool:
        return self.nxt >= len(self.jobs) and not self.pending and not self.inflight

    def step(self, now: float) -> bool:
        """One pass at host time `now`; returns True if it launched a batch."""
        still = []
        for b in self.inflight:
            t = self.ex.done(b.handle)
            if t is None:
                still.append(b)
                continue
            for p in b.jobs:
                self.done_t[p.idx] = t
                self.ex.retire(p)
                self.slots.give(p.cls, p.slot)
                self.used -= p.nbytes
        self.inflight = still
        while self.nxt < len(self.jobs) and self.arrivals[self.nxt] <= now:
            j = self.jobs[self.nxt]
            self.pending.append(Pending(self.nxt, j, j.nbytes, job_class(j)))
            self.nxt += 1
        group = []
        while self.pending:
            p = self.pending[0]
            if self.used + p.nbytes > self.budget:
                break                 # FIFO: the head blocks until budget frees
            s = self.slots.take(p.cls)
            if s < 0:
                break
            p.slot = s
            self.used += p.nbytes
            group.append(self.pending.popleft())
            self.admit_order.append(p.idx)
        self.max_used = max(self.max_used, self.used)
        if not group:
            return False
        for unit in launch_units(group, self.batching, backlog=bool(self.pending)):
            h, nl = self.ex.launch(unit, self.si, self.batching)
            self.launches += nl
            self.inflight.append(Batch(unit, h))
            self.si = (self.si + 1) % self.nstreams
            self.batches += 1
        return True

    def next_arrival(self):
        return self.arrivals[self.nxt] if self.nxt < len(self.jobs) else None


class InputPool:
    """One device input per (kind, dtype, size): transposes of side 2^k, sums
    of 2^k elements; drawn once with a seeded device generator."""

    def __init__(self, torch, jobs, seed=12):
        self.t = {}
        gen = torch.Generator("cuda").manual_seed(seed)
        for j in jobs:
            key = self.key(j)
            if key in self.t:
                continue
            if j.kind == "tpose":
                x = torch.rand((j.rows, j.cols), generator=gen, device="cuda") * 2 - 1
                self.t[key] = x.to(torch.bfloat16) if j.dtype == "bf16" else x
            elif j.dtype == "f32":
                self.t[key] = torch.randn(j.n, generator=gen, device="cuda")
            else:
                self.t[key] = torch.randint(-1000, 1001, (j.n,), generator=gen, device="cuda",
                                            dtype=torch.int32)

    @staticmethod
    def key(j):
        return (j.kind, j.dtype, j.rows if j.kind == "tpose" else j.n)

    def get(self, j):
        return self.t[self.key(j)]


class OutputBuffers:
    """Preallocated outputs: a set of dst matrices per transpose class and one
    float64 / int64 vector for the sums."""

    def __init__(self, torch, jobs, slots_per_class=8, sum_slots=4096):
        self.bufs, self.counts = {}, {}
        for c in {job_class(j) for j in jobs if j.kind == "tpose"}:
            _, dt, side = c
            n = slots_per_class if side <= 4096 else max(2, slots_per_class // 2)
            tdt = torch.bfloat16 if dt == "bf16" else torch.float32
            self.bufs[c] = [torch.empty((side, side), dtype=tdt, device="cuda") for _ in range(n)]
            self.counts[c] = n
        self.sum_f = torch.empty(sum_slots, dtype=torch.float64, device="cuda")
        self.sum_i = torch.empty(sum_slots, dtype=torch.int64, device="cuda")
        self.counts[("sum", "f32")] = sum_slots
        self.counts[("sum", "i32")] = sum_slots

    def out(self, c, s):
        if c[0] == "tpose":
            return self.bufs[c][s]
        return (self.sum_f if c[1] == "f32" else self.sum_i)[s:s + 1].view(())


class GpuExecutor:
    """Launches batches on K HIP streams and reads completion from events."""

    def __init__(self, xtr, torch, pool, outs, nstreams=4, keep_results=False):
        self.xtr, self.torch, self.pool, self.outs = xtr, torch, pool, outs
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        self.ref.record(self.streams[0])
        torch.cuda.synchronize()
        self.t_ref = time.perf_counter()
        self.results = {} if keep_results else None

    def launch(self, group, si, batching):
        torch, xtr = self.torch, self.xtr
        st = self.streams[si]
        nl = 0
        with torch.cuda.stream(st):
            tp = [p for p in group if p.job.kind == "tpose"]
            if tp:
                jl = [(self.pool.get(p.job), self.outs.out(p.cls, p.slot)) for p in tp]
                if batching:
                    xtr.tpose_batched(jl)
                    nl += len({p.job.dtype for p in tp})
                else:
                    for s, d in jl:
                        xtr.tpose(s, d)
                    nl += len(jl)
            for dt in ("f32", "i32"):
                sm = [p for p in group if p.job.kind == "sum" and p.job.dtype == dt]
                if not sm:
                    continue
                if batching:
                    xtr.reduce_sum_batched_scatter([self.pool.get(p.job) for p in sm],
                                                   [self.outs.out(p.cls, p.slot) for p in sm],
                                                   dtype=dt)
                    nl += 1
                else:
                    for p in sm:
                        xtr.reduce_sum(self.pool.get(p.job), self.outs.out(p.cls, p.slot),
                                       dtype=dt)
                    nl += len(sm)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(st)
        return ev, nl

    def done(self, ev):
        if not ev.query():
            return None
        return self.t_ref + self.ref.elapsed_time(ev) * 1e-3   # host-clock seconds

    def retire(self, p):
        if self.results is not None:
            self.results[p.idx] = self.outs.out(p.cls, p.slot).clone()


def run(xtr, torch, jobs, *, batching=True, budget=64 << 30, nstreams=4, pool=None, outs=None,
        keep_results=False, log=None):
    """Serve `jobs` (sorted by arrival) in real time; returns stats (and the
    results per job index when keep_results)."""
    pool = pool or InputPool(torch, jobs)
    outs = outs or OutputBuffers(torch, jobs)
    ex = GpuExecutor(xtr, torch, pool, outs, nstreams, keep_results)
    t0 = ex.t_ref
    arrivals = [j.arrival_s for j in jobs]
    sch = Scheduler(jobs, arrivals, SlotPool(outs.counts), ex, budget, batching, nstreams)
    while not sch.finished():
        now = time.perf_counter() - t0
        launched = sch.step(now)
        if not launched and not sch.inflight and not sch.pending:
            na = sch.next_arrival()
            if na is not None:
                wait = na - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
    torch.cuda.synchronize()
    done = sch.done_t - t0
    lat = done - np.asarray(arrivals)
    tot_bytes = sum(j.nbytes for j in jobs)
    span = float(np.nanmax(done) - arrivals[0])
    stats = {
        "jobs": len(jobs), "batching": batching, "streams": nstreams,
        "budget_gib": budget / 2 ** 30, "max_inflight_gib": round(sch.max_used / 2 ** 30, 3),
        "max_inflight_bytes": int(sch.max_used),
        "p50_ms": round(float(np.nanpercentile(lat, 50)) * 1e3, 4),
        "p99_ms": round(float(np.nanpercentile(lat, 99)) * 1e3, 4),
        "mean_ms": round(float(np.nanmean(lat)) * 1e3, 4),
        "max_ms": round(float(np.nanmax(lat)) * 1e3, 4),
        "throughput_gbs": round(tot_bytes / span / 1e9, 1),
        "offered_jobs_per_s": round(len(jobs) / max(arrivals[-1] - arrivals[0], 1e-12), 1),
        "achieved_jobs_per_s": round(len(jobs) / span, 1),
        "launches": sch.launches, "batches": sch.batches,
        "mean_jobs_per_batch": round(len(jobs) / max(sch.batches, 1), 2),
    }
    if log:
        log(f"serve batching={batching}: p50 {stats['p50_ms']} ms p99 {stats['p99_ms']} ms, "
            f"{stats['throughput_gbs']} GB/s, {stats['achieved_jobs_per_s']} jobs/s, "
            f"{stats['launches']} launches in {stats['batches']} batches")
    if keep_results:
        stats["results"] = ex.results
        stats["admit_order"] = sch.admit_order
    return stats


class HostInputs:
    """Page-locked host copies of the pool's inputs, for jobs whose input
    arrives in host memory."""

    def __init__(self, torch, pool, keys):
        self.t = {k: pool.t[k].cpu().pin_memory() for k in keys}

    def get(self, j):
        return self.t[InputPool.key(j)]


def host_resident(jobs, frac, seed, max_input_bytes=16 << 20):
    """Indices of the jobs whose input is in host memory: each job with an
    input of at most max_input_bytes, with probability frac (seeded)."""
    rng = np.random.default_rng(seed)
    pick = rng.random(len(jobs)) < frac
    return {i for i, j in enumerate(jobs)
            if pick[i] and (j.nbytes // 2 if j.kind == "tpose" else j.nbytes) <= max_input_bytes}


def size_classes(jobs, lat):
    """p50 / p99 latency (ms) and job count per size class: algorithmic bytes
    under 4 MiB, 4 to 64 MiB, 64 MiB and more."""
    nb = np.array([j.nbytes for j in jobs], dtype=np.float64)
    out = {}
    for name, lo, hi in (("under_4MiB", 0, 4 << 20), ("4_to_64MiB", 4 << 20, 64 << 20),
                         ("64MiB_up", 64 << 20, float("inf"))):
        m = (nb >= lo) & (nb < hi)
        if m.any():
            out[name] = {"jobs": int(m.sum()),
                         "p50_ms": round(float(np.percentile(lat[m], 50)) * 1e3, 4),
                         "p99_ms": round(float(np.percentile(lat[m], 99)) * 1e3, 4)}
    top = lat >= np.percentile(lat, 99)
    out["top_1pct_mean_mib"] = round(float(nb[top].mean()) / 2 ** 20, 1)
    return out


def run_native(xtr, torch, jobs, *, batching=True, budget=64 << 30, nstreams=4, pool=None,
               outs=None, keep_results=False, lead_s=0.005, log=None, graphs=False,
               big_lane=False, host=None, host_inputs=None):
    """Serve `jobs` with the native request loop (xtr_server_*, the same
    policy as Scheduler, in a server thread of the library): the whole arrival
    schedule is handed over at once and each job becomes visible to the loop
    at its arrival time, so no host-side submission cost enters the
    latencies.  With keep_results every job gets an output of its own (else
    the jobs of a class take that class's output slots in turn: the timing
    does not depend on the values).  `host`: indices of the jobs whose input
    is in page-locked host memory (host_inputs); the loop copies each to the
    pool's device tensor of the same key, which holds the same bytes, so
    concurrent readers see unchanged values.  Returns stats like run()."""
    pool = pool or InputPool(torch, jobs)
    host = host or set()
    if host and host_inputs is None:
        host_inputs = HostInputs(torch, pool, {InputPool.key(jobs[i]) for i in host})
    arr = (xtr.Job * len(jobs))()
    keep = []
    nxt = {}
    if not keep_results:
        outs = outs or OutputBuffers(torch, jobs)
    for i, j in enumerate(jobs):
        x = pool.get(j)
        c = job_class(j)
        if keep_results:
            if j.kind == "tpose":
                o = torch.empty((j.cols, j.rows), dtype=x.dtype, device="cuda")
            else:
                o = torch.empty((), dtype=torch.float64 if j.dtype == "f32" else torch.int64,
                                device="cuda")
            keep.append(o)
        else:
            s = nxt.get(c, 0)
            nxt[c] = (s + 1) % outs.counts[c]
            o = outs.out(c, s)
        a = arr[i]
        a.kind = 0 if j.kind == "tpose" else 1
        a.dtype = xtr.CODES[j.dtype]
        a.src = x.data_ptr()
        a.dst = o.data_ptr()
        a.rows, a.cols, a.n = j.rows, j.cols, j.n
        a.host_src = host_inputs.get(j).data_ptr() if i in host else None
    torch.cuda.synchronize()                     # inputs and outputs exist before serving
    srv = xtr.Server(nstreams=nstreams, batching=batching, budget=budget, graphs=graphs,
                     big_lane=big_lane)
    t0 = xtr.Server.clock_ns() + int(lead_s * 1e9)
    for i, j in enumerate(jobs):
        arr[i].arrival_ns = t0 + int(round(j.arrival_s * 1e9))
    srv.submit(arr)
    srv.drain()
    arrival, done = srv.times()
    st = srv.stats()
    srv.close()
    lat = (done - arrival) * 1e-9
    tot_bytes = sum(j.nbytes for j in jobs)
    span = (done.max() - arrival.min()) * 1e-9
    stats = {
        "jobs": len(jobs), "batching": batching, "streams": nstreams, "loop": "native",
        "budget_gib": budget / 2 ** 30, "max_inflight_gib": round(st["max_inflight_bytes"] / 2 ** 30, 3),
        "max_inflight_bytes": int(st["max_inflight_bytes"]),
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
        "mean_ms": round(float(np.mean(lat)) * 1e3, 4),
        "max_ms": round(float(np.max(lat)) * 1e3, 4),
        "throughput_gbs": round(tot_bytes / span / 1e9, 1),
        "offered_jobs_per_s": round(len(jobs) / max(jobs[-1].arrival_s - jobs[0].arrival_s, 1e-12), 1),
        "achieved_jobs_per_s": round(len(jobs) / span, 1),
        "launches": st["launches"], "batches": st["units"],
        "mean_jobs_per_batch": round(len(jobs) / max(st["units"], 1), 2),
        "graphs": graphs, "big_lane": big_lane, "graph_launches": st["graph_launches"],
        "graph_builds": st["graph_builds"], "host_copies": st["host_copies"],
        "by_size": size_classes(jobs, lat),
    }
    if log:
        log(f"serve (native) batching={batching}: p50 {stats['p50_ms']} ms p99 {stats['p99_ms']} ms, "
            f"{stats['throughput_gbs']} GB/s, {stats['launches']} launches in {stats['batches']} units")
    if keep_results:
        stats["results"] = {i: keep[i] for i in range(len(jobs))}
    return stats


def bench(xtr, torch, log, count=200000, seed=12, rate=20000.0,
          sweep=((60000.0, 120000), (200000.0, 100000))):
    """The serving workload: a Poisson stream (mean 20k jobs/s) of mixed jobs,
    continuous batching vs one launch per job on the same GPU; then the same
    mix at higher arrival rates (the last one beyond what the GPU can serve),
    where the cost of one launch per job shows."""
    import workloads as W
    jobs = W.serving_jobs(count, seed, rate=rate)
    pool = InputPool(torch, jobs)
    outs = OutputBuffers(torch, jobs)
    warm = [j for j in W.serving_jobs(3000, seed + 1000, rate=rate) if InputPool.key(j) in pool.t]
    run(xtr, torch, warm, pool=pool, outs=outs)
    run(xtr, torch, warm, batching=False, pool=pool, outs=outs)
    run_native(xtr, torch, warm, pool=pool, outs=outs)
    out = {"offered_gbs": round(W.mean_job_bytes() * rate / 1e9, 1), "rate_jobs_per_s": rate}
    out["batched"] = run_native(xtr, torch, jobs, batching=True, pool=pool, outs=outs, log=log)
    out["per_job"] = run_native(xtr, torch, jobs, batching=False, pool=pool, outs=outs, log=log)
    out["python_loop_batched"] = run(xtr, torch, jobs[:40000], batching=True, pool=pool, outs=outs,
                                     log=log)
    out["sweep"] = []
    for r, c in sweep:
        js = [j for j in W.serving_jobs(c, seed + int(r), rate=r) if InputPool.key(j) in pool.t]
        ent = {"rate_jobs_per_s": r, "offered_gbs": round(W.mean_job_bytes() * r / 1e9, 1)}
        for name, b in (("batched", True), ("per_job", False)):
            st = run_native(xtr, torch, js, batching=b, pool=pool, outs=outs, log=log)
            ent[name] = {k: st[k] for k in ("jobs", "p50_ms", "p99_ms", "throughput_gbs",
                                            "achieved_jobs_per_s", "launches", "batches")}
        out["sweep"].append(ent)
    return out
