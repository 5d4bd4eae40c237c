"""GPU parity of the histograms against the CPU oracle: every count exact
(integer work, bit-exact bar), for every input format, for the three integer
bin rules (shift, multiply-high, division), for the LDS path and the
global-atomic path, across workgroups, ragged tails, unaligned starts, the
range ends, NaN and infinities, constant and sorted inputs, empty inputs, and
at the benchmark's full size."""
import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

FLOATS = ["f32", "bf16", "f16", "f8e4m3"]
SIZES = [1, 2, 5, 17, 63, 1000, 65536 + 3, 1_000_003]


def fdata(dt, n, seed):
    if dt == "f32":
        return W.normal(n, seed, "f32")
    return W.signed_lognormal(n, seed, dt, sigma=1.0)[0]


def gpu_hist_float(xtr, bits, dt, lo, hi, nb, off=0):
    t = to_dev(bits)
    return xtr.histogram_float(t[off:], lo, hi, nb, dtype=dt).cpu().numpy()


def gpu_hist_int(xtr, a, dt, lo, width, nb, off=0):
    t = to_dev(a)
    return xtr.histogram_int(t[off:], lo, width, nb, dtype=dt).cpu().numpy()


@pytest.mark.parametrize("dt", FLOATS)
def test_float_sizes(xtr, orc, dt):
    for k, n in enumerate(SIZES):
        bits = fdata(dt, n, 700 + k)
        for lo, hi, nb in ((-4.0, 4.0, 256), (-1.0, 2.5, 1000), (-3.0, 3.0, 1)):
            got = gpu_hist_float(xtr, bits, dt, lo, hi, nb)
            want = orc.histogram_float(bits, dt, lo, hi, nb)
            assert np.array_equal(got, want), (dt, n, lo, hi, nb)


@pytest.mark.parametrize("dt", FLOATS)
def test_float_bin_counts_up_to_lds_limit_and_past_it(xtr, orc, dt):
    bits = fdata(dt, 300_007, 710)
    for nb in (4095, 16384, 16385, 100_000):         # LDS path, its limit, global path
        got = gpu_hist_float(xtr, bits, dt, -2.0, 3.0, nb)
        want = orc.histogram_float(bits, dt, -2.0, 3.0, nb)
        assert np.array_equal(got, want), (dt, nb)


@pytest.mark.parametrize("dt", ["f32", "bf16", "f8e4m3"])
def test_float_unaligned_start(xtr, orc, dt):
    bits = fdata(dt, 50_000, 720)
    for off in (1, 3, 7):
        got = gpu_hist_float(xtr, bits, dt, -1.5, 1.5, 300, off)
        want = orc.histogram_float(bits[off:], dt, -1.5, 1.5, 300)
        assert np.array_equal(got, want), (dt, off)


def test_float_range_ends_and_nonfinite(xtr, orc):
    lo, hi, nb = -1.0, 1.0, 8
    special = np.array([lo, hi, np.nextafter(np.float32(hi), np.float32(0)),
                        np.nextafter(np.float32(lo), np.float32(-2)), np.nan, np.inf, -np.inf,
                        0.0, -0.0, 0.25, 1e-40, -1e-40, 0.75, 3.0], dtype=np.float32)
    bits = np.concatenate([np.tile(special, 97), W.normal(10_000, 730, "f32")])
    got = gpu_hist_float(xtr, bits, "f32", lo, hi, nb)
    want = orc.histogram_float(bits, "f32", lo, hi, nb)
    assert np.array_equal(got, want)
    # lo counts, hi does not, NaN and infinities never
    one = lambda v: gpu_hist_float(xtr, np.full(5, v, np.float32), "f32", lo, hi, nb).sum()
    assert one(lo) == 5 and one(hi) == 0 and one(np.nan) == 0 and one(np.inf) == 0


def test_float_bins_near_edges(xtr, orc):
    """Values at and one ulp around every bin edge of a range whose edges are
    not representable: the fp64 rule decides each, bit for bit."""
    lo, hi, nb = -0.7, 2.3, 300
    edges = lo + (hi - lo) * np.arange(nb + 1) / nb
    e32 = edges.astype(np.float32)
    vals = np.concatenate([e32, np.nextafter(e32, np.float32(-10)),
                           np.nextafter(e32, np.float32(10))]).astype(np.float32)
    got = gpu_hist_float(xtr, vals, "f32", lo, hi, nb)
    assert np.array_equal(got, orc.histogram_float(vals, "f32", lo, hi, nb))


INT_CASES = [
    ("i32", -(1 << 20), 1 << 20, [(-(1 << 20), 1, 4096), (-(1 << 20), 256, 8192),
                                  (-1000, 7, 1000), (0, 1000, 700)]),
    ("i64", -(1 << 40), 1 << 40, [(-(1 << 40), 1 << 30, 2048), (-(1 << 30), 3, 1 << 14),
                                  (-(1 << 40), 3_000_000_007, 300)]),   # span > 2^32: division
    ("u8", 0, 255, [(0, 1, 256), (10, 3, 80), (0, 16, 16)]),
    ("u16", 0, 65535, [(0, 1, 16384), (0, 1, 65536), (100, 10, 6000)]),
]


@pytest.mark.parametrize("dt,vlo,vhi,rules", INT_CASES, ids=[c[0] for c in INT_CASES])
def test_int_rules_and_sizes(xtr, orc, dt, vlo, vhi, rules):
    for k, n in enumerate(SIZES):
        a = W.integers(n, 740 + k, vlo, vhi, dt)
        for lo, width, nb in rules:
            got = gpu_hist_int(xtr, a, dt, lo, width, nb)
            want = orc.histogram_int(a, dt, lo, width, nb)
            assert np.array_equal(got, want), (dt, n, lo, width, nb)


def test_int_extremes(xtr, orc):
    """int64 values at the ends of the type and offsets near 2^64."""
    i64 = np.iinfo(np.int64)
    a = np.array([i64.min, i64.min + 1, -1, 0, 1, i64.max - 1, i64.max] * 50, dtype=np.int64)
    for lo, width, nb in ((i64.min, 1 << 62, 4), (i64.min, 1, 1000), (-1, 1, 3),
                          (i64.min, (1 << 62) + 1, 4), (0, 1 << 61, 4)):
        got = gpu_hist_int(xtr, a, "i64", lo, width, nb)
        assert np.array_equal(got, orc.histogram_int(a, "i64", lo, width, nb)), (lo, width, nb)


@pytest.mark.parametrize("dt", ["i32", "u8", "u16"])
def test_one_bin_of_width_2_32(xtr, orc, dt):
    """width = 2^32 with one bin spans the whole 32-bit range from lo: the
    bin index is a shift by 32, which the 32-bit rules cannot take (it goes to
    the 64-bit shift rule).  Regression test: every element in range counts."""
    vlo, vhi = {"i32": (-(1 << 31), (1 << 31) - 1), "u8": (0, 255), "u16": (0, 65535)}[dt]
    a = W.integers(100_003, 760, vlo, vhi, dt)
    for lo in (-(1 << 31), 0, -5, vlo + 1):
        got = gpu_hist_int(xtr, a, dt, lo, 1 << 32, 1)
        want = orc.histogram_int(a, dt, lo, 1 << 32, 1)
        assert np.array_equal(got, want), (dt, lo, got, want)
    assert gpu_hist_int(xtr, a, dt, -(1 << 31), 1 << 32, 1)[0] == a.size


@pytest.mark.parametrize("dt", ["i32", "u8", "u16"])
def test_int_unaligned_start(xtr, orc, dt):
    vhi = {"i32": 5000, "u8": 255, "u16": 65535}[dt]
    a = W.integers(40_000, 750, 0, vhi, dt)
    for off in (1, 2, 5):
        got = gpu_hist_int(xtr, a, dt, 0, 7, 1000, off)
        assert np.array_equal(got, orc.histogram_int(a[off:], dt, 0, 7, 1000)), (dt, off)


def test_constant_and_sorted_inputs(xtr, orc):
    """Runs of one bin (one atomic add per run): a constant input puts every
    element in one bin, a sorted one walks the bins in order."""
    n = 3_000_001
    c = np.full(n, 0.5, dtype=np.float32)
    got = gpu_hist_float(xtr, c, "f32", 0.0, 1.0, 64)
    assert got[32] == n and got.sum() == n
    s = np.sort(W.normal(n, 760, "f32"))
    assert np.array_equal(gpu_hist_float(xtr, s, "f32", -3.0, 3.0, 1000),
                          orc.histogram_float(s, "f32", -3.0, 3.0, 1000))
    u = np.zeros(n, dtype=np.uint8)
    assert gpu_hist_int(xtr, u, "u8", 0, 1, 256)[0] == n


def test_empty_input_zero_fills(xtr):
    import torch
    counts = torch.full((300,), 7, dtype=torch.int64, device="cuda")
    x = torch.empty(0, dtype=torch.float32, device="cuda")
    xtr.histogram_float(x, 0.0, 1.0, 300, counts)
    assert int(counts.abs().sum()) == 0
    counts.fill_(7)
    xtr.histogram_int(torch.empty(0, dtype=torch.int32, device="cuda"), 0, 1, 300, counts)
    assert int(counts.abs().sum()) == 0


def test_repeated_calls_reuse_workspace(xtr, orc):
    """A large call then a small one on the same stream (the partial table is
    reused, never carried over)."""
    big = W.normal(1 << 22, 770, "f32")
    small = W.normal(999, 771, "f32")
    for bits in (big, small, big):
        got = gpu_hist_float(xtr, bits, "f32", -4.0, 4.0, 2048)
        assert np.array_equal(got, orc.histogram_float(bits, "f32", -4.0, 4.0, 2048))


def test_full_size_and_deterministic(xtr, orc):
    """The benchmark's workloads at full size: 2^28 fp32 normal values in
    1024 bins over [-4, 4), and 2^30 uint8 values in 256 bins."""
    import torch
    n = 1 << 28
    bits = W.normal(n, 780, "f32")
    t = to_dev(bits)
    a = xtr.histogram_float(t, -4.0, 4.0, 1024).cpu().numpy()
    b = xtr.histogram_float(t, -4.0, 4.0, 1024).cpu().numpy()
    assert np.array_equal(a, b)
    assert np.array_equal(a, orc.histogram_float(bits, "f32", -4.0, 4.0, 1024))
    del t
    u = W.integers(1 << 30, 781, 0, 255, "u8")
    tu = torch.from_numpy(u).to("cuda")
    got = xtr.histogram_int(tu, 0, 1, 256).cpu().numpy()
    assert np.array_equal(got, orc.histogram_int(u, "u8", 0, 1, 256))
    del tu
    torch.cuda.empty_cache()
