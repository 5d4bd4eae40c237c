#!/usr/bin/env python3
"""Throughput of the transpose and sum-reduction hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--suite step|full] [--no-cpu]

One step = one pass over the large single-job workload: an fp32 16384 x 16384
transpose, a bf16 12288 x 20000 transpose, an fp32 sum of 2^28 N(0,1) values
and an int64 sum of 2^28 values uniform in [-2^40, 2^40].  `value` is the
step's algorithmic bytes (transpose: read + write once; sum: read once) over
the step's device time, in GB/s, with inputs already resident in HBM.
Each kernel is also timed alone with HIP events on the stream it runs on, and
the dominant one is reported against the HBM roofline.  The CPU oracle is
timed on a bounded 1/16 sample of the same workload.

Besides the step, the default run measures the rest of the metric:
  * "batched": the 4096-job fp32 transpose batch (sides uniform in
    [16, 2048]) and the 100k-segment fp32 sum (2^27 values), each as one
    batched call against one launch per job, in GB/s of algorithmic bytes;
  * "serving": the request loop on its Poisson mix (20k jobs/s) for a few
    seconds, continuous batching against one launch per job (and two
    variants: graph-replayed units, a lane for large jobs): p50 / p99 latency
    and aggregate GB/s; then with a share of the inputs in host memory, and
    at 60k and 200k jobs/s;
  * "cpu_baseline": the CPU oracle on one thread, and the same plain loops on
    every host core (OpenMP), with the host's core count and CPU model.
Per-kernel times are reported as medians and means of per-launch HIP events.

`--suite full` adds the precision sweep, paper shapes, piece widths, host
buffers, prefix sums, histograms, matrix products and the serving sweep under
"suite".

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0    # MI355X HBM3E, public spec


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# What decides the kernels of the step and their launches: their sources and
# the tuned launch settings.  Counter summaries are valid for this hash only.
STEP_SOURCES = ("paper_2605_13864_amd/csrc/common.hpp", "paper_2605_13864_amd/csrc/runtime.hip",
                "paper_2605_13864_amd/csrc/tile_map.h", "paper_2605_13864_amd/csrc/tpose_dev.hpp",
                "paper_2605_13864_amd/csrc/tpose.hip", "paper_2605_13864_amd/csrc/tpose_s2.hip",
                "paper_2605_13864_amd/csrc/tpose_s4.hip", "paper_2605_13864_amd/csrc/reduce.hip",
                "paper_2605_13864_amd/tuned/gfx950.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_key: str):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE,
    WRITE_SIZE, scaled by a plain-copy calibration) when the committed counter
    summary was taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel_key)
    return None if k is None else k.get("hbm_bytes_per_launch")


class Step:
    """The four kernels of one step, with their inputs resident on the GPU."""

    def __init__(self, xtr, torch):
        import numpy as np
        import workloads as W
        dev = torch.device("cuda")
        self.xtr, self.torch = xtr, torch
        log("bench: generating inputs ...")
        t0 = time.time()
        a = W.matrix(16384, 16384, 2, "f32")
        self.t32_in = torch.from_numpy(a).to(dev)
        del a
        self.t32_out = torch.empty((16384, 16384), dtype=torch.float32, device=dev)
        b = W.matrix(12288, 20000, 3, "bf16")
        self.t16_in = torch.from_numpy(b.view(np.int16)).to(dev)
        del b
        self.t16_out = torch.empty((20000, 12288), dtype=torch.int16, device=dev)
        self.s32 = torch.from_numpy(W.normal(1 << 28, 4, "f32")).to(dev)
        self.s64 = torch.from_numpy(W.integers(1 << 28, 5, -(1 << 40), 1 << 40, "i64")).to(dev)
        self.o32 = torch.empty((), dtype=torch.float64, device=dev)
        self.o64 = torch.empty((), dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        log(f"bench: inputs ready in {time.time() - t0:.1f}s")
        self.kernels = [
            ("tpose_f32_16384x16384", 2 * 16384 * 16384 * 4,
             lambda: xtr.tpose(self.t32_in, self.t32_out, dtype="f32")),
            ("tpose_bf16_12288x20000", 2 * 12288 * 20000 * 2,
             lambda: xtr.tpose(self.t16_in, self.t16_out, dtype="bf16")),
            ("sum_f32_2^28", (1 << 28) * 4,
             lambda: xtr.reduce_sum(self.s32, self.o32, dtype="f32")),
            ("sum_i64_2^28", (1 << 28) * 8,
             lambda: xtr.reduce_sum(self.s64, self.o64, dtype="i64")),
        ]
        self.bytes = sum(k[1] for k in self.kernels)

    def run(self, events=None):
        for i, (_, _, fn) in enumerate(self.kernels):
            if events is not None:
                events[i][0].record()
            fn()
            if events is not None:
                events[i][1].record()


def copy_ceiling(xtr, torch, nbytes=1 << 30, reps=20):
    """Plain device-to-device copy bandwidth (read + write) of the library's
    streaming copy kernel and of torch's copy_, for context."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    res = {}
    for name, fn in (("xtr_copy", lambda: xtr.copy(b, a)), ("torch_copy", lambda: b.copy_(a))):
        for _ in range(3):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        res[name] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    del a, b
    return res


def host_info():
    """Core count and CPU model of the host the run is on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"os_cpu_count": os.cpu_count(), "cpu_model": model,
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else None}


def cpu_baseline():
    """The oracle, as it stands, on a 1/16 sample of the step's workload
    (single thread), and the same plain loops on every host core (OpenMP, the
    partials-then-combine pattern of Listing 2.2)."""
    import oracle
    import workloads as W
    o = oracle.get()
    b = oracle.omp()
    a = W.matrix(4096, 4096, 2, "f32")
    bb = W.matrix(3072, 5000, 3, "bf16")
    c = W.normal(1 << 24, 4, "f32")
    d = W.integers(1 << 24, 5, -(1 << 40), 1 << 40, "i64")
    names = ("tpose f32 4096x4096", "tpose bf16 3072x5000", "sum f32 2^24", "sum i64 2^24")
    nbytes = (2 * a.nbytes, 2 * bb.nbytes, c.nbytes, d.nbytes)

    def measure(fns, budget_s):
        total_b, total_t, reps = 0, 0.0, 0
        t_start = time.time()
        while reps < 1 or (time.time() - t_start < budget_s and reps < 20):
            for nb, fn in zip(nbytes, fns):
                t0 = time.perf_counter()
                fn()
                total_t += time.perf_counter() - t0
                total_b += nb
            reps += 1
        return total_b / total_t / 1e9, reps, total_t

    v1, r1, t1 = measure((lambda: o.tpose(a), lambda: o.tpose(bb), lambda: o.sum_float(c, "f32"),
                          lambda: o.sum_int(d, "i64")), 8.0)
    vp, rp, tp = measure((lambda: b.tpose(a), lambda: b.tpose(bb),
                          lambda: b.sum_float(c, "f32"), lambda: b.sum_int(d, "i64")), 4.0)
    info = host_info()
    return {"value": round(v1, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"1/16 of the step ({', '.join(names)}), {r1} repetition(s), "
                      f"{t1:.1f}s of CPU time, single thread",
            "all_cores": {"value": round(vp, 3), "unit": "GB/s", "cores": b.threads(),
                          "kind": "oracle loops, OpenMP (Listing 2.2 partials pattern)",
                          "sample": f"the same 1/16 sample, {rp} repetition(s), {tp:.1f}s wall"},
            **info}


def _ev_ms(torch, fn, reps, warm=1):
    """Per-repetition device time (ms) of fn on the current stream: list."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        out.append(s.elapsed_time(e))
    return out


def _median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def _graph(torch, fn):
    """fn captured once in a graph on a side stream."""
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            fn()
    torch.cuda.synchronize()
    return g


def batched_vs_per_job(xtr, torch, per_job=True):
    """The batched configuration: 4096 fp32 transposes with sides uniform in
    [16, 2048] (seed 9) as one tpose_batched call against one tpose launch per
    job; 2^27 fp32 values in 100k lognormal(6, 1.5) segments (seeds 10, 11) as
    one segmented call against one reduce_sum launch per segment.  Values are
    drawn on the device with a seeded generator (a copy's or a sum's speed
    does not depend on them)."""
    import workloads as W
    res = {}
    shapes = W.batched_shapes(4096, 9)
    gen = torch.Generator("cuda").manual_seed(9)
    jobs, nbytes = [], 0
    for r, c in shapes:
        jobs.append((torch.rand((r, c), generator=gen, device="cuda") * 2 - 1,
                     torch.empty((c, r), device="cuda")))
        nbytes += 2 * r * c * 4
    # Device time of the batch as one persistent launch per group (the table
    # built and uploaded once: a plan), against the same 4096 single tpose
    # launches replayed from a graph (no host or binding cost on either side).
    # One tpose_batched call and the eager per-job loop from Python are
    # reported too: their events also see the device idle while Python
    # marshals the jobs.
    plan = xtr.TposePlan(jobs)
    bp = _ev_ms(torch, plan.run, reps=5)
    plan.close()
    bt = _ev_ms(torch, lambda: xtr.tpose_batched(jobs), reps=3)

    def per_job_loop():
        for s_, d_ in jobs:
            xtr.tpose(s_, d_, dtype="f32")
    pg = pe = [float("nan")]
    if per_job:
        pe = _ev_ms(torch, per_job_loop, reps=2)
        g = _graph(torch, per_job_loop)
        pg = _ev_ms(torch, g.replay, reps=3)
        del g
    ok = all(torch.equal(jobs[k][1], jobs[k][0].t()) for k in (0, 2047, 4095))
    res["tpose_4096_jobs_f32"] = {
        "bytes": nbytes,
        "batched_ms": round(_median(bp), 3), "batched_gbs": round(nbytes / _median(bp) / 1e6, 1),
        "per_job_ms": round(_median(pg), 3), "per_job_gbs": round(nbytes / _median(pg) / 1e6, 1),
        "speedup": round(_median(pg) / _median(bp), 2),
        "batched_call_from_python_gbs": round(nbytes / _median(bt) / 1e6, 1),
        "per_job_eager_from_python_gbs": round(nbytes / _median(pe) / 1e6, 1),
        "spot_check_ok": ok}
    del jobs
    torch.cuda.empty_cache()
    total, nseg = 1 << 27, 100000
    off = W.segment_offsets(total, nseg, 11)
    x = torch.randn(total, generator=torch.Generator("cuda").manual_seed(10), device="cuda")
    doff = torch.from_numpy(off).cuda()
    ws = torch.zeros(xtr.segmented_workspace_bytes(nseg, total, "f32"), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty(nseg, dtype=torch.float64, device="cuda")
    sg = _ev_ms(torch, lambda: xtr.reduce_sum_segmented_ws(x, doff, ws, out, dtype="f32"), reps=10)
    views = [x[off[i]:off[i + 1]] for i in range(nseg)]
    per = torch.empty(nseg, dtype=torch.float64, device="cuda")
    outs = [per[i:i + 1].view(()) for i in range(nseg)]

    def per_seg():
        for v, o_ in zip(views, outs):
            xtr.reduce_sum(v, o_, dtype="f32")
    ps = _ev_ms(torch, per_seg, reps=1) if per_job else [float("nan")]
    nb = total * 4
    res["segmented_100k_f32"] = {
        "bytes": nb, "batched_us": round(_median(sg) * 1e3, 1),
        "batched_gbs": round(nb / _median(sg) / 1e6, 1),
        "per_job_us": round(_median(ps) * 1e3, 1), "per_job_gbs": round(nb / _median(ps) / 1e6, 1),
        "per_job_from": "eager reduce_sum calls from Python (100k launches)",
        "speedup": round(_median(ps) / _median(sg), 1),
        "bit_identical_to_alone": bool(torch.equal(per, out)) if per_job else None}
    del x, ws, views, outs
    torch.cuda.empty_cache()
    return res


def serving(xtr, torch, seconds=3.0, rate=20000.0, seed=12, host_frac=0.25,
            sweep=((60000.0, 1.5), (200000.0, 1.0))):
    """The serving workload for a few seconds: Poisson arrivals at `rate`
    jobs/s of the configured mix.  Continuous batching ("batched") against
    one launch per job on the same GPU, and two variants of the batched
    server: launch units replayed from executable graphs, and large jobs in
    order on a lane of their own.  Then the same comparison with a share of
    the inputs arriving in page-locked host memory (copied by the loop on its
    copy stream, overlapping the other jobs' kernels), and at higher arrival
    rates, where launches become the scarce resource."""
    import workloads as W
    from paper_2605_13864_amd import serve
    count = int(seconds * rate)
    jobs = W.serving_jobs(count, seed, rate=rate)
    pool = serve.InputPool(torch, jobs)
    outs = serve.OutputBuffers(torch, jobs)
    warm = [j for j in W.serving_jobs(2000, seed + 1000, rate=rate)
            if serve.InputPool.key(j) in pool.t]
    configs = (("batched", dict(batching=True)),
               ("per_job", dict(batching=False)),
               ("batched_graphs", dict(batching=True, graphs=True)),
               ("batched_large_lane", dict(batching=True, big_lane=True)))
    for _, kw in configs:
        serve.run_native(xtr, torch, warm, pool=pool, outs=outs, **kw)
    keys = ("jobs", "p50_ms", "p99_ms", "mean_ms", "throughput_gbs", "achieved_jobs_per_s",
            "launches", "batches", "mean_jobs_per_batch", "max_inflight_gib", "graph_launches",
            "graph_builds", "host_copies", "by_size")
    res = {"rate_jobs_per_s": rate, "seconds": seconds, "loop": "native (xtr_server)",
           "offered_gbs": round(W.mean_job_bytes() * rate / 1e9, 1)}
    for name, kw in configs:
        st = serve.run_native(xtr, torch, jobs, pool=pool, outs=outs, **kw)
        res[name] = {k: st[k] for k in keys}
        res[name]["config"] = kw
    res["batched_p99_below_per_job"] = res["batched"]["p99_ms"] < res["per_job"]["p99_ms"]
    host = serve.host_resident(jobs, host_frac, seed + 1)
    hin = serve.HostInputs(torch, pool, {serve.InputPool.key(jobs[i]) for i in host})
    hb = sum((jobs[i].nbytes // 2 if jobs[i].kind == "tpose" else jobs[i].nbytes) for i in host)
    ent = {"host_jobs": len(host), "host_input_gbs_offered": round(hb / seconds / 1e9, 2),
           "rule": f"each job with an input of at most 16 MiB, with probability {host_frac}"}
    for name, kw in configs[:2]:
        st = serve.run_native(xtr, torch, jobs, pool=pool, outs=outs, host=host, host_inputs=hin, **kw)
        ent[name] = {k: st[k] for k in keys}
    res["host_inputs"] = ent
    del hin
    res["sweep"] = []
    for r, secs in sweep:
        js = [j for j in W.serving_jobs(int(r * secs), seed + int(r), rate=r)
              if serve.InputPool.key(j) in pool.t]
        e = {"rate_jobs_per_s": r, "offered_gbs": round(W.mean_job_bytes() * r / 1e9, 1),
             "jobs": len(js)}
        for name, kw in configs[:2]:
            st = serve.run_native(xtr, torch, js, pool=pool, outs=outs, **kw)
            e[name] = {k: st[k] for k in ("p50_ms", "p99_ms", "throughput_gbs",
                                          "achieved_jobs_per_s", "launches", "batches")}
        res["sweep"].append(e)
    del pool, outs
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--suite", choices=["step", "full"], default="step")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip batched vs per-job")
    ap.add_argument("--no-serving", action="store_true", help="skip the short serving run")
    ap.add_argument("--no-per-job", action="store_true",
                    help="batched section without the one-launch-per-job loops (profiling)")
    ap.add_argument("--no-step", action="store_true",
                    help="profiling: skip the step (the plain copy still runs)")
    ap.add_argument("--parts", default="paper,widths,batched,segmented,precision,host,scan,hist,matmul,serving",
                    help="suite parts for --suite full (comma-separated)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2605_13864_amd as xtr
    xtr.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"bench: device {torch.cuda.get_device_name(0)}")

    if args.no_step:
        # profiling runs of the other parts: the plain copy (the counters'
        # calibration) and whatever parts are not switched off
        out = {"metric": None, "note": "--no-step: profiling run, no step measured",
               "copy_gbs": copy_ceiling(xtr, torch)}
        rest(args, out, xtr, torch)
        return

    step = Step(xtr, torch)
    for _ in range(args.warmup):
        step.run()
    torch.cuda.synchronize()

    # whole-step timing
    t0 = time.perf_counter()
    s_ev, e_ev = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ev.record()
    for _ in range(args.steps):
        step.run()
    e_ev.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = s_ev.elapsed_time(e_ev) / args.steps
    log(f"bench: {args.steps} steps, {ms_per_step:.3f} ms/step (wall {wall:.2f}s)")

    # per-kernel timing (events on the current stream, which the kernels run on)
    n = len(step.kernels)
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(n)] for _ in range(args.steps)]
    for k in range(args.steps):
        step.run(evs[k])
    torch.cuda.synchronize()
    per = []
    for i, (name, nbytes, _) in enumerate(step.kernels):
        each = [evs[k][i][0].elapsed_time(evs[k][i][1]) * 1e3 for k in range(args.steps)]
        us = sum(each) / len(each)
        med = _median(each)
        gbs = nbytes / (us * 1e-6) / 1e9
        per.append({"kernel": name, "bytes": nbytes, "avg_us": round(us, 2),
                    "median_us": round(med, 2), "gbs": round(gbs, 1),
                    "median_gbs": round(nbytes / (med * 1e-6) / 1e9, 1),
                    "frac": round(gbs / HBM_PEAK_GBS, 4)})
        log(f"bench: {name:28s} {us:9.2f} us (median {med:9.2f})  {gbs:8.1f} GB/s  "
            f"{gbs / HBM_PEAK_GBS:6.1%} of peak")
    dom = max(per, key=lambda p: p["avg_us"])
    value = step.bytes / (ms_per_step * 1e-3) / 1e9
    copy = copy_ceiling(xtr, torch)
    log(f"bench: step {value:.1f} GB/s; plain copy {copy}")

    tr = traffic_from_profile(dom["kernel"])
    out = {
        "metric": "HBM GB/s & % of peak: transpose, sum-reduce; batched vs per-job; p99 latency",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16 (transpose bit copies); f32-pair compensated / int64 (sums)",
        "data": "synthetic",
        "config": {"workload": "large single jobs: tpose f32 16384x16384 + tpose bf16 "
                               "12288x20000 + sum f32 2^28 N(0,1) + sum i64 2^28 U[-2^40,2^40]",
                   "bytes_per_step": step.bytes, "frac_of_peak": round(value / HBM_PEAK_GBS, 4),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["frac"],
                     "traffic": tr, "median_achieved": dom["median_gbs"]},
        "kernels": per,
        "copy_gbs": copy,
    }
    rest(args, out, xtr, torch)


def rest(args, out, xtr, torch):
    """The parts after the step: batched vs per-job, serving, CPU baseline,
    the full suite; then the JSON line."""
    if not args.no_batched:
        t0 = time.time()
        out["batched"] = batched_vs_per_job(xtr, torch, per_job=not args.no_per_job)
        b = out["batched"]
        log(f"bench: batched 4096 transposes {b['tpose_4096_jobs_f32']['batched_gbs']} GB/s vs "
            f"per-job (graph) {b['tpose_4096_jobs_f32']['per_job_gbs']}; segmented 100k "
            f"{b['segmented_100k_f32']['batched_gbs']} GB/s vs per-job "
            f"{b['segmented_100k_f32']['per_job_gbs']} ({time.time() - t0:.1f}s)")
    if not args.no_serving:
        t0 = time.time()
        out["serving"] = serving(xtr, torch)
        v = out["serving"]
        for name in ("batched", "per_job", "batched_graphs", "batched_large_lane"):
            log(f"bench: serving 20k jobs/s {name:16s} p50 {v[name]['p50_ms']} p99 "
                f"{v[name]['p99_ms']} ms {v[name]['throughput_gbs']} GB/s, "
                f"{v[name]['launches']} launches, {v[name]['graph_launches']} graph launches")
        h = v["host_inputs"]
        log(f"bench: serving with {h['host_jobs']} host inputs: batched p99 "
            f"{h['batched']['p99_ms']} ms, per-job p99 {h['per_job']['p99_ms']} ms")
        for e in v["sweep"]:
            log(f"bench: serving {e['rate_jobs_per_s']:.0f} jobs/s: batched p99 "
                f"{e['batched']['p99_ms']} ms {e['batched']['throughput_gbs']} GB/s; per-job p99 "
                f"{e['per_job']['p99_ms']} ms {e['per_job']['throughput_gbs']} GB/s")
        log(f"bench: serving done ({time.time() - t0:.1f}s)")
    if not args.no_cpu:
        log("bench: timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline()
    if args.suite == "full":
        import bench_suite
        out["suite"] = bench_suite.run_all(xtr, torch, log, tuple(args.parts.split(",")))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
