"""GPU parity of the host-buffer entry points (copy in, kernel, copy out in
panels, the end-to-end form of the paper's host code): transposes bit-exact
against the oracle, sums bit-identical to reduce_sum of an aligned device copy
and within the float bar of the oracle, for page-locked and pageable host
buffers, several panels, ragged last panels and leading dimensions."""
import numpy as np
import pytest

import workloads as W
from gpu_util import check_float_sum

pytestmark = pytest.mark.gpu

SD = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}
NAME = {1: "u8", 2: "bf16", 4: "f32", 8: "f64"}


def host_buf(n, dtype, pinned):
    """A host buffer of n elements: page-locked (torch pin_memory) or numpy."""
    import torch
    if not pinned:
        return np.empty(n, dtype=dtype)
    tdt = {np.uint8: torch.uint8, np.uint16: torch.int16, np.uint32: torch.int32,
           np.uint64: torch.int64, np.float32: torch.float32, np.int32: torch.int32,
           np.int64: torch.int64}[dtype]
    return torch.empty(n, dtype=tdt, pin_memory=True).numpy().view(dtype)


@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("eb,rows,cols,pad_s,pad_d", [
    (4, 20000, 1000, 0, 0),        # three row panels, the last one ragged
    (4, 777, 1031, 5, 3),          # one panel, leading dimensions
    (2, 30001, 1200, 0, 1),        # bf16, two panels
    (1, 1500, 70000, 2, 0),        # u8, wide rows (panel = minimum height)
    (8, 9000, 513, 1, 0),          # f64
])
def test_tpose_host(xtr, orc, eb, rows, cols, pad_s, pad_d, pinned):
    ld_s, ld_d = cols + pad_s, rows + pad_d
    src = host_buf(rows * ld_s, SD[eb], pinned)
    src[:] = W.random_bits(rows * ld_s, 3000 + rows, eb)
    canary = np.frombuffer(bytes([0x5A]) * eb, dtype=SD[eb])[0]
    dst = host_buf(cols * ld_d, SD[eb], pinned)
    dst[:] = canary
    xtr.tpose_host(src, dst, rows=rows, cols=cols, ld_src=ld_s, ld_dst=ld_d, dtype=NAME[eb])
    want = np.full(cols * ld_d, canary, dtype=SD[eb])
    orc.tpose(src, rows, cols, ld_s, ld_d, dst=want)
    assert np.array_equal(dst, want)


def test_tpose_host_empty_and_errors(xtr):
    a = np.zeros(16, dtype=np.float32)
    xtr.tpose_host(a, a.copy(), rows=0, cols=4, dtype="f32")
    with pytest.raises(xtr.XtrError):
        xtr.tpose_host(a, a, rows=4, cols=4, dtype="f32")      # in place: overlap


@pytest.mark.parametrize("pinned", [True, False])
@pytest.mark.parametrize("dt,n", [("f32", 20_000_001), ("i32", 8192 * 1024 + 5), ("bf16", 33_000_000),
                                  ("i64", 3), ("f8e4m3", 0), ("f32", 8192)])
def test_sum_host(xtr, orc, dt, n, pinned):
    import torch
    if dt == "i32":
        bits = W.integers(n, 90, -1000, 1000, "i32")
    elif dt == "i64":
        bits = W.integers(n, 91, -(1 << 40), 1 << 40, "i64")
    elif dt == "f32":
        bits = W.normal(n, 92, "f32")
    else:
        bits = W.signed_lognormal(n, 93, dt)[0] if n else np.zeros(0, dtype=np.uint8)
    host = host_buf(max(n, 1), bits.dtype.type if bits.dtype != np.float32 else np.float32, pinned)[:n]
    host[:] = bits
    got = xtr.reduce_sum_host(host, n=n, dtype=dt)
    dev = torch.from_numpy(bits.view(np.int16) if bits.dtype == np.uint16 else bits).cuda()
    alone = xtr.reduce_sum(dev, n=n, dtype=dt).item()
    assert got == alone, (dt, n, got, alone)              # aligned device copy, bit for bit
    if dt in ("i32", "i64"):
        assert got == orc.sum_int(bits, dt)[0]
    else:
        check_float_sum(got, orc.sum_float(bits, dt), orc.sum_abs(bits, dt), (dt, n))
