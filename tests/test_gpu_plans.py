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


def test_tpose_plan_runs_and_replays(xtr, orc):
    import torch
    jobs, hosts = _tpose_jobs(torch, 40, 3)
    plan = xtr.TposePlan(jobs)
    plan.run()
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
