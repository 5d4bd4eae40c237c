"""Batch plans and hipGraph capture: a plan's run launches kernels only, so
it can be captured and replayed; every replay (with eager work and
synchronisations between replays) must equal the eager result."""
import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _tpose_jobs(torch, n, seed, dtypes=("f32", "bf16", "u8", "f64")):
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs, hosts = [], []
    for i in range(n):
        dt = dtypes[i % len(dtypes)]
        r, c = (int(x) for x in rng.integers(1, 700, 2))
        eb = {"f32": 4, "bf16": 2, "u8": 1, "f64": 8}[dt]
        a = W.random_bits(r * c, 500 + i, eb).reshape(r, c)
        s = to_dev(a)
        d = torch.empty((c, r), dtype=s.dtype, device=s.device)
        jobs.append({"src": s, "dst": d, "rows": r, "cols": c, "dtype": dt})
        hosts.append(a)
    return jobs, hosts


@pytest.mark.parametrize("xcd", [1, 3])
def test_tpose_plan_runs_and_replays(xtr, orc, xcd):
    """A transpose plan run eagerly, then captured and replayed; with xcd = 3
    the launches take their slots from counters in the plan's table, which
    every run must leave at zero for the next one."""
    import torch
    origs = {eb: xtr.tpose_config(eb, "batched") for eb in (1, 2, 4, 8)}
    for eb in origs:
        xtr.set_tpose_config(eb, "batched", xcd=xcd, blocks_per_cu=2)
    try:
        _plan_replays(xtr, orc, torch)
    finally:
        for eb, o in origs.items():
            xtr.set_tpose_config(eb, "batched", **o)


def _plan_replays(xtr, orc, torch):
    jobs, hosts = _tpose_jobs(torch, 40, 3)
    for k in range(8, 40):                            # a group of more than 24 jobs: a table
        r, c = (int(x) for x in np.random.Generator(np.random.PCG64(k)).integers(200, 900, 2))
        a = W.random_bits(r * c, 900 + k, 4).reshape(r, c)
        s = to_dev(a)
        jobs.append({"src": s, "dst": torch.empty((c, r), dtype=s.dtype, device=s.device),
                     "rows": r, "cols": c, "dtype": "f32"})
        hosts.append(a)
    plan = xtr.TposePlan(jobs)
    plan.run()
    plan.run()                                        # eager runs back to back
    torch.cuda.synchronize()
    for j, a in zip(jobs, hosts):
        assert np.array_equal(to_host(j["dst"], a.dtype), orc.tpose(a))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for j in jobs:
            j["dst"].zero_()                          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j, a in zip(jobs, hosts):
            assert np.array_equal(to_host(j["dst"], a.dtype), orc.tpose(a)), rep
    plan.close()


def test_sum_plan_runs_and_replays(xtr):
    import torch
    rng = np.random.Generator(np.random.PCG64(4))
    ns = [0, 1, 33, 8192, 8193] + [int(x) for x in rng.integers(1, 3 << 20, 20)]
    bits = [W.normal(n, 700 + i, "f32") for i, n in enumerate(ns)]
    devs = [to_dev(b) for b in bits]
    eager = xtr.reduce_sum_batched(devs, dtype="f32").cpu()
    plan = xtr.SumPlan(devs, dtype="f32")
    assert torch.equal(plan.run().cpu(), eager)
    assert torch.equal(plan.run().cpu(), eager)     # the plan's workspace is reusable
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.run()
    torch.cuda.synchronize()
    for rep in range(4):
        plan.out.fill_(-1.0)                          # eager work between replays
        xtr.reduce_sum(devs[3], dtype="f32")          # another library call in between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(plan.out.cpu(), eager), rep
    ints = [to_dev(W.integers(n, 800 + i, -1000, 1000, "i32")) for i, n in enumerate(ns)]
    p2 = xtr.SumPlan(ints, dtype="i32")
    assert torch.equal(p2.run().cpu(), xtr.reduce_sum_batched(ints, dtype="i32").cpu())
    plan.close()
    p2.close()


def test_scan_histogram_matmul_replay(xtr, orc):
    """Prefix sums (one-pass integer and three-pass float), histograms (LDS,
    fp8-by-code and global-atomic forms) and matrix products (both layouts of
    B) captured in one graph: their flags, counters and partial tables are
    cleared by fill kernels inside the graph, so every replay, with other
    library work and synchronisations between replays, equals the eager
    result."""
    import torch
    n = 3 * 16384 * 4 + 11
    xi = to_dev(W.integers(n, 900, -1000, 1000, "i32"))
    xf = to_dev(W.normal(n, 901, "f32"))
    x8 = to_dev(W.signed_lognormal(n, 902, "f8e4m3", sigma=1.0)[0])
    a = torch.randn((300, 200), device="cuda").to(torch.bfloat16)
    b = torch.randn((200, 260), device="cuda").to(torch.bfloat16)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    outs = {}

    def work():
        outs["si"] = xtr.scan_sum(xi, outs.get("si"), dtype="i32")
        outs["sf"] = xtr.scan_sum(xf, outs.get("sf"), dtype="f32", exclusive=True)
        outs["hf"] = xtr.histogram_float(xf, -3.0, 3.0, 700, outs.get("hf"))
        outs["h8"] = xtr.histogram_float(x8, -2.0, 2.0, 64, outs.get("h8"), dtype="f8e4m3")
        outs["hg"] = xtr.histogram_int(xi, -1000, 1, 20001, outs.get("hg"))
        outs["mn"] = xtr.matmul(a, b, outs.get("mn"))
        outs["mt"] = xtr.matmul(a, b.t().contiguous(), outs.get("mt"), trans_b=True)

    with torch.cuda.stream(s):
        work()                                        # grows the stream's workspaces
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in outs.items()}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            work()
    torch.cuda.synchronize()
    for rep in range(3):
        for v in outs.values():
            v.fill_(7)                                # eager work between replays
        xtr.scan_sum(xi, dtype="i32")                 # other library calls in between
        xtr.histogram_int(xi, 0, 3, 100)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in outs:
            assert torch.equal(outs[k], eager[k]), (k, rep)
    want = orc.scan(xi.cpu().numpy(), "i32")
    assert np.array_equal(eager["si"].cpu().numpy(), want)


def test_replay_after_workspace_growth(xtr, orc):
    """A graph captured from calls that use the library workspace keeps the
    buffer it saw; a later, larger eager call on the same stream grows (and
    replaces) the workspace.  The old buffer must stay valid: every replay
    after the growth still equals the eager result."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    n = 5 * 16384 + 3
    xi = to_dev(W.integers(n, 910, -1000, 1000, "i32"))
    xf = to_dev(W.normal(n, 911, "f32"))
    outs = {}

    def work():
        outs["r"] = xtr.reduce_sum(xf, outs.get("r"), dtype="f32")
        outs["si"] = xtr.scan_sum(xi, outs.get("si"), dtype="i32")
        outs["h"] = xtr.histogram_int(xi, -1000, 4, 501, outs.get("h"))

    with torch.cuda.stream(s):
        work()
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in outs.items()}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            work()
    torch.cuda.synchronize()
    big = 64 << 20
    bi = to_dev(W.integers(big, 912, -1000, 1000, "i32"))
    bf = to_dev(W.normal(big, 913, "f32"))
    for rep in range(3):
        with torch.cuda.stream(s):                    # grows every workspace of the stream
            r = xtr.reduce_sum(bf[:big // (3 - rep)], dtype="f32")
            sc = xtr.scan_sum(bi[:big // (3 - rep)], dtype="i32")
            hh = xtr.histogram_int(bi[:big // (3 - rep)], -1000, 4, 501)
        torch.cuda.synchronize()
        for v in outs.values():
            v.fill_(7)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        for k in outs:
            assert torch.equal(outs[k], eager[k]), (k, rep)
        del r, sc, hh
    want = orc.scan(xi.cpu().numpy(), "i32")
    assert np.array_equal(eager["si"].cpu().numpy(), want)


@pytest.mark.parametrize("streams", [0, 1])
def test_segmented_ws_replay(xtr, streams):
    """The segmented sum with a caller workspace captured in a graph, on one
    stream or forked to the library's second stream (the small segments) and
    joined back: every replay equals the eager result."""
    import torch
    total, nseg = 400000, 3000
    off = W.segment_offsets(total, nseg, 97)
    d, doff = to_dev(W.normal(total, 98, "f32")), to_dev(off)
    ws = torch.zeros(xtr.segmented_workspace_bytes(nseg, total, "f32"), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty(nseg, dtype=torch.float64, device="cuda")
    orig = xtr.reduce_config("f32", "batched")
    try:
        xtr.set_reduce_config("f32", "batched", seg_fused=0, seg_streams=streams,
                              seg_small_per_cu=2 if streams else 0,
                              seg_chunk_per_cu=4 if streams else 0)
        eager = xtr.reduce_sum_segmented_ws(d, doff, ws, out, total=total, dtype="f32").clone()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                xtr.reduce_sum_segmented_ws(d, doff, ws, out, total=total, dtype="f32")
        torch.cuda.synchronize()
        for rep in range(4):
            out.fill_(-1.0)
            xtr.reduce_sum(d, dtype="f32")            # another library call in between
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), rep
    finally:
        xtr.set_reduce_config("f32", "batched", **orig)
