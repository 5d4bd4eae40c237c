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
