"""reduce_sum_noalloc (the entry point for callers that cannot allocate)
against reduce_sum, through the C ABI: bit-identical results on two calls in a
row on one GPU, the second with a smaller input (the fixed scratch array keeps
the first call's contents), for every summable format, on both combine paths;
sizes beyond the fixed scratch are refused before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

CH = {"f32": 8192, "i32": 8192, "i64": 4096, "bf16": 16384, "f16": 16384, "f8e4m3": 32768}


def data(dt, n, seed):
    if dt == "i32":
        return W.integers(n, seed, -1000, 1000, "i32")
    if dt == "i64":
        return W.integers(n, seed, -(1 << 40), 1 << 40, "i64")
    if dt == "f32":
        return W.normal(n, seed, "f32")
    return W.signed_lognormal(n, seed, dt)[0]


def call(fn, t, n, dt, torch):
    out = torch.zeros((), dtype=torch.int64 if dt in ("i32", "i64") else torch.float64,
                      device="cuda")
    import paper_2605_13864_amd as X
    rc = fn(C.c_void_p(t.data_ptr()), n, C.c_void_p(out.data_ptr()), X.CODES[dt],
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, (rc, X.load().xtr_last_error())
    return out.item()


@pytest.mark.parametrize("dt", ["f32", "i32", "i64", "bf16", "f16", "f8e4m3"])
def test_noalloc_equals_reduce_sum(xtr, dt):
    import torch
    lib = xtr.load()
    c = CH[dt]
    # large (split combine: partials + combine launches), then smaller (ticket
    # combine), then a ragged tail with an unaligned start
    for k, (n, off) in enumerate([(2048 * c + 17, 0), (37 * c + 5, 0), (3 * c + 1, 1), (1, 0), (0, 0)]):
        bits = data(dt, n + off, 1400 + k)
        t = to_dev(bits)[off:]
        a = call(lib.reduce_sum_noalloc, t, n, dt, torch)
        b = call(lib.reduce_sum, t, n, dt, torch)
        assert a == b or (np.isnan(a) and np.isnan(b)), (dt, n, off, a, b)


def test_noalloc_refuses_beyond_scratch(xtr):
    import torch
    lib = xtr.load()
    t = torch.zeros(16, dtype=torch.float32, device="cuda")
    out = torch.zeros((), dtype=torch.float64, device="cuda")
    rc = lib.reduce_sum_noalloc(C.c_void_p(t.data_ptr()), 1 << 40, C.c_void_p(out.data_ptr()), 0,
                                C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -7 and b"scratch" in lib.xtr_last_error()
    torch.cuda.synchronize()
    assert out.item() == 0.0                     # nothing was enqueued
