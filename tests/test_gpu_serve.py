"""The serving loop on the GPU: every job's result in the mix equals the same
job run alone (bit for bit: transposes are bit copies, integer sums are exact,
and float sums use the same canonical chunking alone and in a batch), matches
the CPU oracle, and the in-flight bytes never exceed the budget."""
import numpy as np
import pytest

import workloads as W
from gpu_util import check_float_sum

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("batching", [True, False])
def test_results_same_alone_and_in_mix(xtr, orc, batching):
    import torch
    from paper_2605_13864_amd import serve
    jobs = W.serving_jobs(600, 21, rate=20000.0, tpose_k=(5, 10), sum_k=(10, 20))
    budget = 96 << 20
    st = serve.run(xtr, torch, jobs, batching=batching, budget=budget, keep_results=True)
    assert st["max_inflight_bytes"] <= budget
    assert sorted(st["results"]) == list(range(len(jobs)))
    assert st["admit_order"] == sorted(st["admit_order"])
    pool = serve.InputPool(torch, jobs)           # same seed: same inputs
    for i, j in enumerate(jobs):
        x = pool.get(j)
        got = st["results"][i]
        if j.kind == "tpose":
            alone = xtr.tpose(x)
            assert torch.equal(got.view(torch.int16) if x.dtype == torch.bfloat16 else got,
                               alone.view(torch.int16) if x.dtype == torch.bfloat16 else alone), i
            if i % 25 == 0:
                h = x.cpu().view(torch.int16).numpy() if x.dtype == torch.bfloat16 else x.cpu().numpy()
                want = orc.tpose(h)
                g = got.cpu().view(torch.int16).numpy() if x.dtype == torch.bfloat16 else got.cpu().numpy()
                assert np.array_equal(g, want), i
        else:
            alone = xtr.reduce_sum(x)
            assert got.item() == alone.item(), (i, got.item(), alone.item())
            if i % 10 == 0:
                h = x.cpu().numpy()
                if j.dtype == "i32":
                    assert got.item() == orc.sum_int(h, "i32")[0]
                else:
                    check_float_sum(got.item(), orc.sum_float(h, "f32"), orc.sum_abs(h, "f32"), i)


@pytest.mark.parametrize("batching", [True, False])
def test_native_loop_same_alone_and_in_mix(xtr, orc, batching):
    """The native request loop (xtr_server_*): every job's result in the mix
    equals the job run alone, bit for bit; the in-flight bytes stay within a
    tight budget; every job completes after it arrives."""
    import torch
    from paper_2605_13864_amd import serve
    jobs = W.serving_jobs(800, 22, rate=20000.0, tpose_k=(5, 10), sum_k=(10, 20))
    budget = 64 << 20
    st = serve.run_native(xtr, torch, jobs, batching=batching, budget=budget, keep_results=True)
    assert 0 < st["max_inflight_bytes"] <= budget
    assert st["p50_ms"] > 0 and st["max_ms"] < 5000
    pool = serve.InputPool(torch, jobs)
    for i, j in enumerate(jobs):
        x = pool.get(j)
        got = st["results"][i]
        if j.kind == "tpose":
            alone = xtr.tpose(x)
            a = got.view(torch.int16) if x.dtype == torch.bfloat16 else got.view(torch.int32)
            b = alone.view(torch.int16) if x.dtype == torch.bfloat16 else alone.view(torch.int32)
            assert torch.equal(a, b), i
        else:
            alone = xtr.reduce_sum(x)
            assert got.item() == alone.item(), (i, got.item(), alone.item())
            if i % 20 == 0 and j.dtype == "i32":
                assert got.item() == orc.sum_int(x.cpu().numpy(), "i32")[0]


def test_native_loop_validation(xtr):
    """Submission refuses bad jobs before anything is queued: an unknown kind,
    a dtype the sums do not take, a job larger than the budget."""
    import torch
    x = torch.zeros(64, dtype=torch.float32, device="cuda")
    o = torch.zeros((), dtype=torch.float64, device="cuda")
    srv = xtr.Server(budget=1 << 20)
    bad = [xtr.Job(7, 0, x.data_ptr(), o.data_ptr(), 0, 0, 64, -1),
           xtr.Job(1, xtr.CODES["u8"], x.data_ptr(), o.data_ptr(), 0, 0, 64, -1),
           xtr.Job(1, 0, x.data_ptr(), o.data_ptr(), 0, 0, 1 << 20, -1)]
    for j, code in zip(bad, (-1, -2, -7)):
        with pytest.raises(xtr.XtrError) as e:
            srv.submit([j])
        assert e.value.code == code
    srv.submit([xtr.Job(1, 0, x.data_ptr(), o.data_ptr(), 0, 0, 64, -1)])
    srv.drain(10000)
    assert srv.stats()["completed"] == 1 and o.item() == 0.0
    srv.close()


def test_native_loop_configured_sizes(xtr, orc):
    """The serving mix at its configured sizes (transposes of side 2^5 ..
    2^13, bf16 and fp32; sums of 2^10 .. 2^26 fp32 / int32 elements), 300
    jobs at 20k jobs/s under a 4 GiB budget, every job with its own output:
    each result equals the job run alone, bit for bit; the small ones are
    checked against the oracle too."""
    import torch
    from paper_2605_13864_amd import serve
    jobs = W.serving_jobs(300, 23, rate=20000.0)
    budget = 4 << 30
    st = serve.run_native(xtr, torch, jobs, batching=True, budget=budget, keep_results=True)
    assert st["max_inflight_bytes"] <= budget
    pool = serve.InputPool(torch, jobs)
    for i, j in enumerate(jobs):
        x = pool.get(j)
        got = st["results"][i]
        if j.kind == "tpose":
            alone = xtr.tpose(x)
            a = got.view(torch.int16) if x.dtype == torch.bfloat16 else got.view(torch.int32)
            b = alone.view(torch.int16) if x.dtype == torch.bfloat16 else alone.view(torch.int32)
            assert torch.equal(a, b), i
            if j.rows <= 1024 and i % 3 == 0:
                h = x.view(torch.int16).cpu().numpy() if x.dtype == torch.bfloat16 else x.cpu().numpy()
                g = a.cpu().numpy()
                assert np.array_equal(g, orc.tpose(h).view(g.dtype)), i
            del alone
        else:
            alone = xtr.reduce_sum(x)
            assert got.item() == alone.item(), (i, got.item(), alone.item())
            if j.n <= (1 << 22):
                h = x.cpu().numpy()
                if j.dtype == "i32":
                    assert got.item() == orc.sum_int(h, "i32")[0], i
                else:
                    check_float_sum(got.item(), orc.sum_float(h, "f32"), orc.sum_abs(h, "f32"), i)
    del st
    torch.cuda.empty_cache()


@pytest.mark.parametrize("graphs,big_lane,host_frac,rate",
                         [(True, False, 0.0, 300000.0), (True, True, 0.3, 300000.0),
                          (False, True, 0.3, 20000.0), (True, False, 0.0, 20000.0)])
def test_native_loop_graphs_lane_host_inputs(xtr, orc, graphs, big_lane, host_frac, rate):
    """Launch units replayed from executable graphs, the large-job lane, and
    inputs that arrive in page-locked host memory (copied by the loop on its
    copy stream): every result equals the job run alone, bit for bit; graph
    mode runs units from graphs; every host input is copied once."""
    import torch
    from paper_2605_13864_amd import serve
    jobs = W.serving_jobs(800, 24, rate=rate, tpose_k=(5, 10), sum_k=(10, 20))
    host = serve.host_resident(jobs, host_frac, 25)
    st = serve.run_native(xtr, torch, jobs, batching=True, budget=64 << 20, keep_results=True,
                          graphs=graphs, big_lane=big_lane, host=host)
    assert st["max_inflight_bytes"] <= 64 << 20
    assert st["host_copies"] == len(host)
    if graphs:
        assert st["graph_launches"] > 0 and st["graph_builds"] <= st["graph_launches"]
    if rate > 100000:
        assert st["mean_jobs_per_batch"] > 1.0
    pool = serve.InputPool(torch, jobs)
    for i, j in enumerate(jobs):
        x = pool.get(j)
        got = st["results"][i]
        if j.kind == "tpose":
            alone = xtr.tpose(x)
            a = got.view(torch.int16) if x.dtype == torch.bfloat16 else got.view(torch.int32)
            b = alone.view(torch.int16) if x.dtype == torch.bfloat16 else alone.view(torch.int32)
            assert torch.equal(a, b), (i, i in host)
        else:
            alone = xtr.reduce_sum(x)
            assert got.item() == alone.item(), (i, i in host, got.item(), alone.item())
            if i % 20 == 0 and j.dtype == "i32":
                assert got.item() == orc.sum_int(x.cpu().numpy(), "i32")[0]
