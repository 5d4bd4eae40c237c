"""Extra measurements for `bench.py --suite full`: the precision sweep, batched
transposes and segmented sums against one launch per job, the serving loop,
and the paper's own workload shapes.  Each function returns a small dict that
bench.py puts under "suite" in its JSON line.

Large batched inputs are drawn on the device with torch's seeded generator
(the values do not change a transpose's or a sum's speed); the precision
sweep uses the seeded host generators of `workloads`, because its result is
compared with the CPU oracle.
"""
from __future__ import annotations

import time

HBM_PEAK_GBS = 8000.0


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time_dev(torch, fn, reps=5, warm=1):
    for _ in range(warm):
        fn()
    s, e = _events(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    return s.elapsed_time(e) / reps * 1e-3, wall


def _graph(torch, fn):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn()
    torch.cuda.synchronize()
    return g


# ---------------------------------------------------------------- precision

def precision(xtr, torch, log, n=1 << 30):
    """Relative error of the compensated sum and of the plain fp32 comparators
    against the fp64 oracle on +-lognormal(0, 2) data, per format, as the
    precision workload states it; for fp8-e4m3 also at sigma 1 (key
    f8e4m3_sigma1): sigma 2 needs a per-tensor scale of 0.002 to avoid
    overflow, which flushes most values and leaves nothing for a plain sum to
    lose, while e4m3's 18 binades hold a sigma-1 spread of 2^30 draws
    unscaled."""
    import numpy as np
    import oracle
    import workloads as W
    o = oracle.get()
    out = {}
    for key, dt, seed, sigma in (("bf16", "bf16", 6, 2.0), ("f16", "f16", 7, 2.0),
                                 ("f8e4m3", "f8e4m3", 8, 2.0),
                                 ("f8e4m3_sigma1", "f8e4m3", 8, 1.0)):
        t0 = time.time()
        bits, scale = W.signed_lognormal(n, seed, dt, sigma=sigma)
        ref = o.sum_float(bits, dt)
        sabs = o.sum_abs(bits, dt)
        seq = o.sum_plain_f32(bits, dt)
        d = torch.from_numpy(bits.view(np.int16) if bits.dtype == np.uint16 else bits).cuda()
        comp = xtr.reduce_sum(d, dtype=dt).item()
        plain = xtr.reduce_sum_plain_f32(d, dtype=dt).item()
        sec_c, _ = _time_dev(torch, lambda: xtr.reduce_sum(d, dtype=dt))
        sec_p, _ = _time_dev(torch, lambda: xtr.reduce_sum_plain_f32(d, dtype=dt))
        nbytes = bits.nbytes
        rel = lambda x: abs(x - ref) / abs(ref)
        out[key] = {"n": n, "sigma": sigma, "scale": scale, "kappa": sabs / abs(ref), "ref": ref,
                    "rel_err_compensated": rel(comp), "rel_err_plain_gpu_tree": rel(plain),
                    "rel_err_plain_sequential_cpu": rel(seq),
                    "gbs_compensated": round(nbytes / sec_c / 1e9, 1),
                    "gbs_plain": round(nbytes / sec_p / 1e9, 1),
                    "pass_1e-6": rel(comp) <= 1e-6}
        log(f"suite precision {key}: kappa {sabs / abs(ref):.3g} rel err comp {rel(comp):.2e} "
            f"plain-gpu {rel(plain):.2e} plain-seq {rel(seq):.2e}; "
            f"{nbytes / sec_c / 1e9:.0f} GB/s ({time.time() - t0:.0f}s)")
        del d, bits
    return out


# ---------------------------------------------------------------- batched transposes

def batched_tpose(xtr, torch, log, count=4096, seed=9):
    """4096 fp32 transposes, sides iid U{16..2048}: one persistent launch per
    batch (direct, plan, graph-replayed plan) vs one launch per job (eager and
    graph-replayed)."""
    import workloads as W
    shapes = W.batched_shapes(count, seed)
    gen = torch.Generator("cuda").manual_seed(seed)
    srcs, dsts = [], []
    nbytes = 0
    for r, c in shapes:
        srcs.append(torch.rand((r, c), generator=gen, device="cuda") * 2 - 1)
        dsts.append(torch.empty((c, r), device="cuda"))
        nbytes += 2 * r * c * 4
    jobs = list(zip(srcs, dsts))
    res = {"count": count, "bytes": nbytes}

    sec, wall = _time_dev(torch, lambda: xtr.tpose_batched(jobs), reps=5)
    res["batched_direct"] = {"gbs": round(nbytes / sec / 1e9, 1), "ms": round(sec * 1e3, 3),
                             "host_ms": round(wall * 1e3, 3)}
    plan = xtr.TposePlan(jobs)
    sec, wall = _time_dev(torch, plan.run, reps=5)
    res["batched_plan"] = {"gbs": round(nbytes / sec / 1e9, 1), "ms": round(sec * 1e3, 3)}
    g = _graph(torch, plan.run)
    sec, wall = _time_dev(torch, g.replay, reps=5)
    res["batched_graph"] = {"gbs": round(nbytes / sec / 1e9, 1), "ms": round(sec * 1e3, 3)}
    del g

    def per_job():
        for s, d in jobs:
            xtr.tpose(s, d, dtype="f32")
    sec, wall = _time_dev(torch, per_job, reps=2)
    res["per_job_eager"] = {"gbs": round(nbytes / sec / 1e9, 1), "ms": round(sec * 1e3, 3),
                            "host_ms": round(wall * 1e3, 3)}
    g = _graph(torch, per_job)
    sec, wall = _time_dev(torch, g.replay, reps=3)
    res["per_job_graph"] = {"gbs": round(nbytes / sec / 1e9, 1), "ms": round(sec * 1e3, 3)}
    del g
    # spot-check correctness of the batched path on a few jobs
    xtr.tpose_batched(jobs)
    torch.cuda.synchronize()
    for k in (0, count // 2, count - 1):
        assert torch.equal(dsts[k], srcs[k].t()), k
    plan.close()
    res["speedup_batched_vs_per_job_graph"] = round(res["per_job_graph"]["ms"] /
                                                    res["batched_graph"]["ms"], 2)
    log(f"suite batched tpose: {count} jobs {nbytes / 1e9:.1f} GB: batched {res['batched_direct']['gbs']}"
        f" / plan {res['batched_plan']['gbs']} / graph {res['batched_graph']['gbs']} GB/s; per-job eager "
        f"{res['per_job_eager']['gbs']} / graph {res['per_job_graph']['gbs']} GB/s")
    del srcs, dsts, jobs
    torch.cuda.empty_cache()
    return res


def batched_probe(xtr, torch, log, seed=9):
    """Where batched transposes lose: the same 4096-job fp32 batch (plan,
    device time) against batches that differ in one respect each -- sides
    rounded up to multiples of 32 (every row on cache lines, 16-byte pieces),
    4096 equal 1024^2 and 1023^2 jobs (no size spread; aligned / not), 16
    jobs of 8192^2 (few large jobs) -- and a single 16383^2 transpose."""
    import workloads as W
    res = {}
    shapes = W.batched_shapes(4096, seed)
    cases = {"config": shapes,
             "rounded_32": [((r + 31) // 32 * 32, (c + 31) // 32 * 32) for r, c in shapes],
             "equal_1024": [(1024, 1024)] * 4096, "equal_1023": [(1023, 1023)] * 4096,
             "large_8192": [(8192, 8192)] * 16}
    gen = torch.Generator("cuda").manual_seed(seed)
    for name, shp in cases.items():
        jobs, nb = [], 0
        for r, c in shp:
            jobs.append((torch.rand((r, c), generator=gen, device="cuda"),
                         torch.empty((c, r), device="cuda")))
            nb += 2 * r * c * 4
        plan = xtr.TposePlan(jobs)
        sec, _ = _time_dev(torch, plan.run, reps=5, warm=1)
        plan.close()
        res[name] = {"gbs": round(nb / sec / 1e9, 1), "ms": round(sec * 1e3, 3),
                     "bytes": nb, "jobs": len(shp)}
        del jobs
        torch.cuda.empty_cache()
    x = torch.rand((16383, 16383), generator=gen, device="cuda")
    y = torch.empty((16383, 16383), device="cuda")
    sec, _ = _time_dev(torch, lambda: xtr.tpose(x, y, dtype="f32"), reps=10, warm=2)
    res["single_16383"] = {"gbs": round(2 * 16383 * 16383 * 4 / sec / 1e9, 1)}
    del x, y
    torch.cuda.empty_cache()
    log("suite batched probe: " + ", ".join(f"{k} {v['gbs']}" for k, v in res.items()))
    return res


# ---------------------------------------------------------------- segmented sums

def segmented(xtr, torch, log, total=1 << 27, nseg=100000):
    """2^27 fp32 N(0,1) values in 100k lognormal(6, 1.5) segments: one
    segmented launch vs one reduce_sum launch per segment."""
    import workloads as W
    off = W.segment_offsets(total, nseg, 11)
    gen = torch.Generator("cuda").manual_seed(10)
    x = torch.randn(total, generator=gen, device="cuda")
    doff = torch.from_numpy(off).cuda()
    nbytes = total * 4
    res = {"total": total, "nseg": nseg, "bytes": nbytes}
    ws = torch.zeros(xtr.segmented_workspace_bytes(nseg, total, "f32"), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty(nseg, dtype=torch.float64, device="cuda")
    fn = lambda: xtr.reduce_sum_segmented_ws(x, doff, ws, out, dtype="f32")
    sec, wall = _time_dev(torch, fn, reps=10)
    res["segmented_ws"] = {"gbs": round(nbytes / sec / 1e9, 1), "us": round(sec * 1e6, 1)}
    g = _graph(torch, fn)
    sec, wall = _time_dev(torch, g.replay, reps=10)
    res["segmented_graph"] = {"gbs": round(nbytes / sec / 1e9, 1), "us": round(sec * 1e6, 1)}
    del g
    sec, wall = _time_dev(torch, lambda: xtr.reduce_sum_segmented(x, doff, out, dtype="f32"),
                          reps=5)
    res["segmented_readback"] = {"gbs": round(nbytes / sec / 1e9, 1), "us": round(sec * 1e6, 1),
                                 "host_us": round(wall * 1e6, 1)}
    seg_out = out.clone()
    views = [x[off[i]:off[i + 1]] for i in range(nseg)]
    per = torch.empty(nseg, dtype=torch.float64, device="cuda")
    outs = [per[i:i + 1] for i in range(nseg)]

    def per_job():
        for v, o in zip(views, outs):
            xtr.reduce_sum(v, o.view(()), dtype="f32")
    sec, wall = _time_dev(torch, per_job, reps=1, warm=1)
    res["per_job_eager"] = {"gbs": round(nbytes / sec / 1e9, 1), "us": round(sec * 1e6, 1),
                            "host_us": round(wall * 1e6, 1)}
    same = bool(torch.equal(per, seg_out))
    res["per_segment_bit_identical_to_alone"] = same
    res["speedup_segmented_vs_per_job"] = round(res["per_job_eager"]["us"] /
                                                res["segmented_ws"]["us"], 1)
    log(f"suite segmented: {res['segmented_ws']['gbs']} GB/s ({res['segmented_ws']['us']} us); "
        f"graph {res['segmented_graph']['gbs']}; per-job {res['per_job_eager']['gbs']} GB/s; "
        f"bit-identical to alone: {same}")
    del x, ws
    torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------- piece widths

def piece_widths(xtr, torch, log):
    """Large single transposes whose row pitches allow 16-, 8-, 4-byte or only
    element-wide global accesses (the tile routine picks the widest piece that
    divides both pointers and both pitches), and line-aligned fp32 rows whose
    pitch is not a power of two (16416) or not a multiple of the line (16388)."""
    cases = [("f32", 16384, 16384, 16), ("f32", 16416, 16416, 16), ("f32", 16388, 16388, 16),
             ("f32", 16382, 16382, 8), ("f32", 16383, 16383, 4),
             ("bf16", 12288, 20000, 16), ("bf16", 12292, 20004, 8), ("bf16", 12290, 20002, 4),
             ("bf16", 12289, 20001, 0), ("u8", 32768, 32768, 16), ("u8", 32764, 32764, 4),
             ("u8", 32767, 32767, 0), ("f64", 16384, 8192, 16), ("f64", 16383, 8191, 8)]
    tdt = {"f32": torch.float32, "bf16": torch.int16, "u8": torch.uint8, "f64": torch.float64}
    eb = {"f32": 4, "bf16": 2, "u8": 1, "f64": 8}
    res = {}
    for dt, r, c, w in cases:
        src = torch.empty((r, c), dtype=tdt[dt], device="cuda")
        src.view(torch.uint8).random_(0, 255, generator=torch.Generator("cuda").manual_seed(r))
        dst = torch.empty((c, r), dtype=tdt[dt], device="cuda")
        sec, _ = _time_dev(torch, lambda: xtr.tpose(src, dst, dtype=dt), reps=10, warm=2)
        nb = 2 * r * c * eb[dt]
        key = f"{dt}_{r}x{c}_w{w}"
        res[key] = {"gbs": round(nb / sec / 1e9, 1), "us": round(sec * 1e6, 1)}
        if r == 16383 and dt == "f32":   # bit comparison (random bits include NaNs)
            assert torch.equal(dst.view(torch.int32), src.view(torch.int32).t()), key
        del src, dst
    torch.cuda.empty_cache()
    log("suite piece widths: " + ", ".join(f"{k} {v['gbs']}" for k, v in res.items()))
    return res


# ---------------------------------------------------------------- prefix sums

def prefix_sums(xtr, torch, log, n=1 << 28):
    """Inclusive prefix sums of 2^28 fp32 N(0,1) and int32 values (outputs fp64
    / int64): algorithmic bytes = read n * elem + write n * 8."""
    res = {}
    gen = torch.Generator("cuda").manual_seed(21)
    for dt in ("f32", "i32"):
        x = (torch.randn(n, generator=gen, device="cuda") if dt == "f32" else
             torch.randint(-1000, 1001, (n,), generator=gen, device="cuda", dtype=torch.int32))
        out = torch.empty(n, dtype=torch.float64 if dt == "f32" else torch.int64, device="cuda")
        sec, _ = _time_dev(torch, lambda: xtr.scan_sum(x, out), reps=10, warm=2)
        nb = n * 4 + n * 8
        res[f"scan_{dt}_2^28"] = {"gbs": round(nb / sec / 1e9, 1), "us": round(sec * 1e6, 1)}
        del x, out
    torch.cuda.empty_cache()
    log("suite prefix sums: " + ", ".join(f"{k} {v['gbs']} GB/s" for k, v in res.items()))
    return res


def histograms(xtr, torch, log, n=1 << 28):
    """Histograms (algorithmic bytes = the input read once; the counts are a
    few KiB): 2^28 fp32 N(0,1) values in 1024 bins over [-4, 4); 2^30 uint8
    values, uniform, in 256 bins; 2^28 int32 values, uniform in [0, 2^20), in
    4096 bins of width 256; 2^29 bf16 and 2^30 fp8 N(0,1) values in 256 bins;
    and constant inputs (every element in one bin)."""
    res = {}
    gen = torch.Generator("cuda").manual_seed(23)
    cases = (
        ("f32_normal_1024", lambda: torch.randn(n, generator=gen, device="cuda"),
         lambda x: xtr.histogram_float(x, -4.0, 4.0, 1024)),
        ("u8_uniform_256", lambda: torch.randint(0, 256, (4 * n,), generator=gen, device="cuda",
                                                 dtype=torch.uint8),
         lambda x: xtr.histogram_int(x, 0, 1, 256)),
        ("i32_uniform_4096", lambda: torch.randint(0, 1 << 20, (n,), generator=gen,
                                                   device="cuda", dtype=torch.int32),
         lambda x: xtr.histogram_int(x, 0, 256, 4096)),
        ("f32_constant_1024", lambda: torch.full((n,), 0.5, device="cuda"),
         lambda x: xtr.histogram_float(x, -4.0, 4.0, 1024)),
        ("bf16_normal_256", lambda: torch.randn(2 * n, generator=gen, device="cuda",
                                                dtype=torch.bfloat16),
         lambda x: xtr.histogram_float(x, -4.0, 4.0, 256)),
        ("f8e4m3_normal_256", lambda: torch.randn(4 * n, generator=gen, device="cuda").to(
            torch.float8_e4m3fn), lambda x: xtr.histogram_float(x, -4.0, 4.0, 256)),
        ("u8_constant_256", lambda: torch.full((4 * n,), 7, device="cuda", dtype=torch.uint8),
         lambda x: xtr.histogram_int(x, 0, 1, 256)),
    )
    for name, make, call in cases:
        x = make()
        sec, _ = _time_dev(torch, lambda: call(x), reps=10, warm=2)
        nb = x.numel() * x.element_size()
        res[name] = {"gbs": round(nb / sec / 1e9, 1), "us": round(sec * 1e6, 1)}
        del x
    torch.cuda.empty_cache()
    log("suite histograms: " + ", ".join(f"{k} {v['gbs']} GB/s" for k, v in res.items()))
    return res


def matmuls(xtr, torch, log):
    """Matrix products on the matrix cores, TFLOP/s = 2 M N K / time: bf16 and
    fp16 8192^3 with B given transposed (one launch) and row-major (transpose
    into the workspace first), bf16 4096^3; torch.matmul (the vendor BLAS)
    on the same operands for context (fp32 output from bf16 inputs is not a
    torch op: it writes bf16)."""
    res = {}
    gen = torch.Generator("cuda").manual_seed(25)
    for n, dt, tdt in ((8192, "bf16", torch.bfloat16), (8192, "f16", torch.float16),
                       (4096, "bf16", torch.bfloat16)):
        a = torch.randn((n, n), generator=gen, device="cuda").to(tdt)
        b = torch.randn((n, n), generator=gen, device="cuda").to(tdt)
        c = torch.empty((n, n), device="cuda")
        flop = 2.0 * n ** 3
        for tb in (True, False):
            sec, _ = _time_dev(torch, lambda: xtr.matmul(a, b, c, trans_b=tb), reps=10, warm=2)
            res[f"{dt}_{n}_{'nt' if tb else 'nn'}"] = {"tflops": round(flop / sec / 1e12, 1),
                                                      "us": round(sec * 1e6, 1)}
        sec, _ = _time_dev(torch, lambda: torch.matmul(a, b), reps=10, warm=2)
        res[f"{dt}_{n}_torch_nn"] = {"tflops": round(flop / sec / 1e12, 1),
                                     "us": round(sec * 1e6, 1)}
        del a, b, c
    torch.cuda.empty_cache()
    log("suite matmul: " + ", ".join(f"{k} {v['tflops']} TFLOP/s" for k, v in res.items()))
    return res


# ---------------------------------------------------------------- host buffers

def host_buffers(xtr, torch, log):
    """End-to-end rates (copy in + kernel + copy out, wall clock) of the
    host-buffer entry points on the bench step's fp32 shapes, for page-locked
    and pageable host memory, beside plain page-locked copy rates."""
    import numpy as np
    res = {}

    def wall(fn, reps):
        fn()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        return (time.perf_counter() - t0) / reps

    nb = 1 << 30
    hp = torch.empty(nb // 4, dtype=torch.float32, pin_memory=True)
    d = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
    sec = wall(lambda: (d.copy_(hp, non_blocking=True), torch.cuda.synchronize()), 5)
    res["pinned_h2d_gbs"] = round(nb / sec / 1e9, 1)
    sec = wall(lambda: (hp.copy_(d, non_blocking=True), torch.cuda.synchronize()), 5)
    res["pinned_d2h_gbs"] = round(nb / sec / 1e9, 1)
    del d
    n = 16384
    for pinned in (True, False):
        tag = "pinned" if pinned else "pageable"
        src = (torch.empty(n * n, dtype=torch.float32, pin_memory=pinned) if pinned
               else torch.empty(n * n, dtype=torch.float32))
        src.view(torch.int32).random_(0, 1 << 30)
        dst = (torch.empty(n * n, dtype=torch.float32, pin_memory=pinned) if pinned
               else torch.empty(n * n, dtype=torch.float32))
        sec = wall(lambda: xtr.tpose_host(src, dst, rows=n, cols=n, dtype="f32"), 3)
        res[f"tpose_host_f32_16384_{tag}_gbs"] = round(2 * n * n * 4 / sec / 1e9, 1)
        if not pinned:
            s2 = src.view(n, n)
            assert torch.equal(dst.view(n, n)[:64, :64].view(torch.int32),
                               s2[:64, :64].t().contiguous().view(torch.int32))
        m = 1 << 28
        sec = wall(lambda: xtr.reduce_sum_host(src[:m], n=m, dtype="f32"), 3)
        res[f"sum_host_f32_2^28_{tag}_gbs"] = round(m * 4 / sec / 1e9, 1)
        del src, dst
    log("suite host buffers: " + ", ".join(f"{k} {v}" for k, v in res.items()))
    return res


# ---------------------------------------------------------------- paper shapes

def paper_shapes(xtr, torch, log):
    """The paper's workloads (a 4096 x 4096 fp32 transpose and a 16M-element
    sum, Section 7.1), rotating over enough buffers (> 1 GiB in total) that
    the 256 MB last-level cache cannot serve repeats."""
    res = {}
    k = 12
    srcs = [torch.rand((4096, 4096), device="cuda") for _ in range(k)]
    dsts = [torch.empty((4096, 4096), device="cuda") for _ in range(k)]
    it = [0]

    def tp():
        i = it[0] % k
        it[0] += 1
        xtr.tpose(srcs[i], dsts[i], dtype="f32")
    sec, _ = _time_dev(torch, tp, reps=48, warm=12)
    nb = 2 * 4096 * 4096 * 4
    res["tpose_f32_4096"] = {"gbs": round(nb / sec / 1e9, 1), "us": round(sec * 1e6, 2)}
    del srcs, dsts
    sums = [torch.randn(1 << 24, device="cuda") for _ in range(k)]
    o = torch.empty((), dtype=torch.float64, device="cuda")
    it[0] = 0

    def sm():
        i = it[0] % k
        it[0] += 1
        xtr.reduce_sum(sums[i], o, dtype="f32")
    sec, _ = _time_dev(torch, sm, reps=48, warm=12)
    nb = (1 << 24) * 4
    res["sum_f32_2^24"] = {"gbs": round(nb / sec / 1e9, 1), "us": round(sec * 1e6, 2)}
    res["paper_rtx5060_context_gbs"] = {"tpose_optigpu": 297.7, "tpose_cuda_samples": 340.6,
                                        "reduce_optigpu": 297.9, "reduce3": 349.4,
                                        "reduce6": 376.8}
    log(f"suite paper shapes: tpose 4096^2 f32 {res['tpose_f32_4096']['gbs']} GB/s, "
        f"sum 2^24 f32 {res['sum_f32_2^24']['gbs']} GB/s")
    del sums
    torch.cuda.empty_cache()
    return res


def run_all(xtr, torch, log, parts=("paper", "widths", "batched", "segmented", "precision",
                                   "host", "scan", "hist", "matmul", "serving")):
    out = {}
    for name, fn in (("paper", paper_shapes), ("widths", piece_widths), ("batched", batched_tpose),
                     ("bprobe", batched_probe),
                     ("host", host_buffers), ("scan", prefix_sums), ("hist", histograms),
                     ("matmul", matmuls),
                     ("segmented", segmented), ("precision", precision)):
        if name in parts:
            t0 = time.time()
            out[name] = fn(xtr, torch, log)
            log(f"suite: {name} done in {time.time() - t0:.1f}s")
    if "serving" in parts:
        try:
            from paper_2605_13864_amd import serve
        except ImportError:
            serve = None
        if serve is not None:
            t0 = time.time()
            out["serving"] = serve.bench(xtr, torch, log)
            log(f"suite: serving done in {time.time() - t0:.1f}s")
    return out
