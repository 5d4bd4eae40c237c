"""GPU parity of the prefix sums against the CPU oracle: integer scans
bit-exact, float scans within the sum bar on every prefix (1e-6 relative, or
2^-40 of the prefix's sum of magnitudes), deterministic, across tiles, ragged
tails, unaligned starts, non-finite values, inclusive and exclusive."""
import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

TILE = {"f32": 4096, "i32": 4096, "i64": 2048, "bf16": 8192, "f16": 8192, "f8e4m3": 16384}
SIGN = {"f32": np.uint32(0x7FFFFFFF), "bf16": np.uint16(0x7FFF), "f16": np.uint16(0x7FFF),
        "f8e4m3": np.uint8(0x7F)}


def data(dt, n, seed):
    if dt == "i32":
        return W.integers(n, seed, -(1 << 30), 1 << 30, "i32")
    if dt == "i64":
        return W.integers(n, seed, -(1 << 62), 1 << 62, "i64")
    if dt == "f32":
        return W.normal(n, seed, "f32")
    return W.signed_lognormal(n, seed, dt)[0]


def magnitudes(bits, dt):
    """The same elements with the sign bit cleared (|x| for every format)."""
    if dt == "f32":
        return (bits.view(np.uint32) & SIGN[dt]).view(np.float32)
    return bits & SIGN[dt]


def check_scan(orc, got, bits, dt, exclusive, what=""):
    want = orc.scan(bits, dt, exclusive)
    if dt in ("i32", "i64"):
        assert np.array_equal(got, want), what
        return
    absum = orc.scan(magnitudes(bits, dt), dt, exclusive)
    fin = np.isfinite(want)
    assert np.array_equal(np.isnan(got), np.isnan(want)), what
    assert np.array_equal(got[np.isinf(want)], want[np.isinf(want)]), what
    err = np.abs(got[fin] - want[fin])
    bar = np.maximum(1e-6 * np.abs(want[fin]), 2.0 ** -40 * absum[fin])
    bad = np.nonzero(err > bar)[0]
    assert bad.size == 0, (what, int(bad[0]), err[bad[0]], bar[bad[0]])


def gpu_scan(xtr, bits, dt, exclusive, off=0):
    t = to_dev(bits)
    out = xtr.scan_sum(t[off:], dtype=dt, exclusive=exclusive)
    return out.cpu().numpy()


@pytest.mark.parametrize("dt", ["f32", "i32", "i64", "bf16", "f16", "f8e4m3"])
@pytest.mark.parametrize("exclusive", [False, True])
def test_scan_sizes(xtr, orc, dt, exclusive):
    t = TILE[dt]
    for k, n in enumerate([1, 2, 7, 63, 64, t - 1, t, t + 1, 3 * t + 17, 37 * t + 5]):
        bits = data(dt, n, 500 + k)
        check_scan(orc, gpu_scan(xtr, bits, dt, exclusive), bits, dt, exclusive, (dt, n))


@pytest.mark.parametrize("dt", ["f32", "i32", "bf16", "f8e4m3"])
def test_scan_unaligned_start(xtr, orc, dt):
    n = 5 * TILE[dt] + 3
    for off in (1, 3):
        bits = data(dt, n + off, 600 + off)
        got = gpu_scan(xtr, bits, dt, False, off)
        check_scan(orc, got, bits[off:], dt, False, (dt, off))


def test_scan_large_and_deterministic(xtr, orc):
    n = (1 << 26) + 12345            # 16k tiles: several tile offsets per scan thread
    bits = W.normal(n, 610, "f32")
    a = gpu_scan(xtr, bits, "f32", False)
    b = gpu_scan(xtr, bits, "f32", False)
    assert np.array_equal(a, b)
    check_scan(orc, a, bits, "f32", False, "large f32")
    ints = W.integers(n, 611, -1000, 1000, "i32")
    check_scan(orc, gpu_scan(xtr, ints, "i32", True), ints, "i32", True, "large i32")


def test_scan_nonfinite(xtr, orc):
    x = W.normal(3 * TILE["f32"] + 10, 620, "f32")
    x[5000] = np.inf                 # from here on +inf ...
    x[9000] = -np.inf                # ... and NaN after the -inf
    got = gpu_scan(xtr, x, "f32", False)
    assert np.isfinite(got[:5000]).all() and (got[5000:9000] == np.inf).all()
    assert np.isnan(got[9000:]).all()
    check_scan(orc, got, x, "f32", False, "nonfinite")
    gx = gpu_scan(xtr, x, "f32", True)
    check_scan(orc, gx, x, "f32", True, "nonfinite exclusive")


def test_scan_empty_and_errors(xtr):
    import torch
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    assert xtr.scan_sum(e).numel() == 0
    a = torch.zeros(64, dtype=torch.int64, device="cuda")
    with pytest.raises(xtr.XtrError):
        xtr.scan_sum(a, a)                                   # out overlaps src
    with pytest.raises(xtr.XtrError):
        xtr.scan_sum(a, dtype="u8")                          # not summable


@pytest.mark.parametrize("dt", ["i32", "i64", "f32", "bf16", "f8e4m3"])
@pytest.mark.parametrize("exclusive", [False, True])
def test_many_tiles(xtr, orc, dt, exclusive):
    """Hundreds of 64 KiB tiles with a ragged last one: integers run in one
    pass with a look-back spanning several 64-tile windows (bit-exact),
    floats in three passes (within the bar); the same bits on a second call
    (the look-back's ticket and flags start from zero every call)."""
    lb_tile = 4 * TILE[dt]
    n = 300 * lb_tile + 77
    bits = data(dt, n, 620)
    a = gpu_scan(xtr, bits, dt, exclusive)
    check_scan(orc, a, bits, dt, exclusive, (dt, n))
    b = gpu_scan(xtr, bits, dt, exclusive)
    assert np.array_equal(a, b)


def test_int_single_pass_unaligned_output(xtr, orc):
    """Outputs that do not start on 16 bytes (element stores) over many tiles."""
    import torch
    n = 70 * 4 * TILE["i32"] + 5
    bits = data("i32", n, 630)
    t = to_dev(bits)
    out = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    xtr.scan_sum(t, out[1:], dtype="i32")
    check_scan(orc, out[1:].cpu().numpy(), bits, "i32", False, "unaligned out")


def test_int_single_pass_large(xtr, orc):
    """2^26 + 12345 int32 values (4097 tiles of the one-pass form)."""
    n = (1 << 26) + 12345
    bits = data("i32", n, 640)
    got = gpu_scan(xtr, bits, "i32", False)
    check_scan(orc, got, bits, "i32", False, "large i32")


def test_nonfinite_across_tiles(xtr, orc):
    """+inf in one 64 KiB tile, -inf in a later one: the prefixes are finite
    before, +inf between, NaN after, across the tile offsets."""
    lb_tile = 4 * TILE["f32"]
    n = 9 * lb_tile + 5
    x = W.normal(n, 650, "f32")
    x[2 * lb_tile + 17] = np.inf
    x[5 * lb_tile + 3] = -np.inf
    got = gpu_scan(xtr, x, "f32", False)
    check_scan(orc, got, x, "f32", False, "nonfinite tiles")
    a, b = 2 * lb_tile + 17, 5 * lb_tile + 3
    assert np.isfinite(got[:a]).all() and (got[a:b] == np.inf).all() and np.isnan(got[b:]).all()


@pytest.mark.parametrize("dt", ["i32", "i64"])
def test_lookback_bound_reached(xtr, orc, dt):
    """The one-pass integer scan with its wait bound forced to 0 polls: every
    workgroup that finds a nearer predecessor silent sums that tile's elements
    itself instead of waiting.  The results must not change (integer sums are
    exact in any order); the kernels exit normally."""
    t = TILE[dt] * 4                                   # elements of a look-back tile
    old = xtr.scan_lookback_bound(0)
    try:
        for k, n in enumerate([5, t - 1, t + 1, 700 * t + 13]):
            bits = data(dt, n, 1300 + k)
            for excl in (False, True):
                got = gpu_scan(xtr, bits, dt, excl)
                check_scan(orc, got, bits, dt, excl, (dt, n, excl))
    finally:
        assert xtr.scan_lookback_bound(old) == 0
