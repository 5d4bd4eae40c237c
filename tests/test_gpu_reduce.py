"""GPU parity of the sum path against the CPU oracle: integer sums bit-exact,
float sums within 1e-6 relative error of the fp64 oracle, across chunk
boundaries, ragged tails, unaligned starts, special values, every fp8 / bf16 /
fp16 code, the batched and segmented forms and the full-size workloads."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_util import check_float_sum, to_dev

pytestmark = pytest.mark.gpu

CH = {"f32": 8192, "i32": 8192, "i64": 4096, "bf16": 16384, "f16": 16384, "f8e4m3": 32768}
SIZES = [0, 1, 2, 3, 7, 63, 64, 255, 256, 1023, 4095]


def sizes_for(dt):
    c = CH[dt]
    return SIZES + [c - 1, c, c + 1, 3 * c + 17, 256 * c - 5, 256 * c + 3 * c + 1]


def data(dt, n, seed):
    if dt == "i32":
        return W.integers(n, seed, -1000, 1000, "i32")
    if dt == "i64":
        return W.integers(n, seed, -(1 << 40), 1 << 40, "i64")
    if dt == "f32":
        return W.normal(n, seed, "f32")
    return W.signed_lognormal(n, seed, dt)[0]


def gpu_sum(xtr, bits, dt, off=0):
    """Sum of bits[off:] with the device buffer starting `off` elements into an
    allocation (so off != 0 exercises unaligned starts)."""
    t = to_dev(bits)
    r = xtr.reduce_sum(t[off:], dtype=dt)
    return r.item()


def check(orc, got, bits, dt, what="", extreme_kappa=False):
    if dt in ("i32", "i64"):
        assert got == orc.sum_int(bits, dt)[0], (what, got)
    else:
        check_float_sum(got, orc.sum_float(bits, dt), orc.sum_abs(bits, dt), what,
                        extreme_kappa=extreme_kappa)


def test_pr1_int32(xtr, orc):
    """PR1 workload: 2^20 int32 uniform in [-1000, 1000], seed 1: bit-exact."""
    bits = W.integers(1 << 20, 1, -1000, 1000, "i32")
    assert gpu_sum(xtr, bits, "i32") == orc.sum_int(bits, "i32")[0]


@pytest.mark.parametrize("dt", ["i32", "i64", "f32", "bf16", "f16", "f8e4m3"])
def test_sizes_and_offsets(xtr, orc, dt):
    for k, n in enumerate(sizes_for(dt)):
        for off in (0, 1, 3):
            bits = data(dt, n + off, 10 * k + off)
            got = gpu_sum(xtr, bits, dt, off)
            check(orc, got, bits[off:], dt, (dt, n, off))


def test_mixed_sizes_share_workspace(xtr, orc):
    """Calls of very different chunk counts back to back on one stream share
    the library workspace; each must see clean tickets (regression test)."""
    c = CH["i32"]
    for k, n in enumerate([300 * c + 5, c + 1, 17 * c + 3, 2 * c, 256 * c + 1, c + 1, 3,
                           513 * c + 7, 2 * c + 1]):
        bits = data("i32", n, 900 + k)
        assert gpu_sum(xtr, bits, "i32") == orc.sum_int(bits, "i32")[0], n
        fb = data("f32", n, 950 + k)
        check(orc, gpu_sum(xtr, fb, "f32"), fb, "f32", n)


@pytest.mark.parametrize("dt", ["f32", "bf16", "f8e4m3", "i32", "i64", "f16"])
def test_split_combine_matches_tickets(xtr, orc, dt):
    """Plain partials + combine launches give bit-identical results to the
    in-kernel ticket combine, over one, two and three combine levels, ragged
    tails and unaligned heads."""
    orig = xtr.reduce_config(dt, "single")
    c = CH[dt]
    try:
        for k, (n, off) in enumerate([(3 * c, 0), (1000 * c + 17, 1), (2 * c - 1, 3),
                                      (256 * c, 2), (5 * c + c // 2, 0), (70000 * c + 5, 1)]):
            if n * np.dtype(data(dt, 1, 0).dtype).itemsize > (1 << 31):
                continue
            bits = data(dt, n + off, 1100 + k)
            xtr.set_reduce_config(dt, "single", split_chunks=0)
            a = gpu_sum(xtr, bits, dt, off)
            for sc in (1, 2, 3 * c):
                xtr.set_reduce_config(dt, "single", split_chunks=sc)
                b = gpu_sum(xtr, bits, dt, off)
                assert a == b or (math.isnan(a) and math.isnan(b)), (dt, n, off, sc, a, b)
            check(orc, a, bits[off:], dt, (dt, n, off))
    finally:
        xtr.set_reduce_config(dt, "single", **orig)


def test_split_combine_three_levels(xtr, orc):
    """More than 256^2 chunks (three combine levels): int32 against the oracle
    bit for bit, and the split and ticket combines agree."""
    orig = xtr.reduce_config("i32", "single")
    n = 65537 * CH["i32"] + 3
    bits = data("i32", n, 1200)
    d = to_dev(bits)
    try:
        xtr.set_reduce_config("i32", "single", split_chunks=1)
        a = xtr.reduce_sum(d, dtype="i32").item()
        xtr.set_reduce_config("i32", "single", split_chunks=0)
        b = xtr.reduce_sum(d, dtype="i32").item()
    finally:
        xtr.set_reduce_config("i32", "single", **orig)
    assert a == b == orc.sum_int(bits, "i32")[0]


def test_int64_wraps(xtr, orc):
    big = np.full(10000, 2 ** 62 + 12345, dtype=np.int64)
    want, ov = orc.sum_int(big, "i64")
    assert ov
    assert gpu_sum(xtr, big, "i64") == want
    mixed = W.integers(50000, 77, -(2 ** 63), 2 ** 63 - 1, "i64")
    assert gpu_sum(xtr, mixed, "i64") == orc.sum_int(mixed, "i64")[0]


def test_float_special_values(xtr, orc):
    f = np.float32
    cases = [
        np.array([1, np.inf, 2] * 5000, f),
        np.array([-np.inf, 1, -np.inf] * 5000, f),
        np.concatenate([np.full(20000, 1, f), [np.inf], np.full(9000, 2, f), [-np.inf]]).astype(f),
        np.concatenate([W.normal(40000, 3, "f32"), np.array([np.nan], f)]),
        np.array([-0.0] * 100, f),
        np.array([1e37, -1e37] * 1000, f),       # large magnitudes, partial sums in range
    ]
    for i, c in enumerate(cases):
        check(orc, gpu_sum(xtr, c, "f32"), c, "f32", i)
    # outside the domain: fp32 partial sums exceed FLT_MAX and become non-finite
    big = np.array([3.4e38, -3.4e38] * 1000, f)
    assert not math.isfinite(gpu_sum(xtr, big, "f32"))
    # sum|x| / |sum x| = 1e30 is outside what the method resolves, so this is no
    # parity check: the rounding error of the compensation term itself (about
    # u^2 |s| per addition, u = 2^-24) exceeds the exact sum 8192 here, and
    # the derived bound (d^2 u^2 + 17 * 2^-53) sum|x| is ~1e19.  Only that
    # bound and a finite result are asserted; the binding high-kappa cases are
    # in test_high_kappa.
    c = np.array([1e30, 1, -1e30, 1] * 4096, f)
    got = gpu_sum(xtr, c, "f32")
    assert math.isfinite(got)
    check(orc, got, c, "f32", "kappa 1e30", extreme_kappa=True)
    # subnormals are kept (no flush to zero)
    sub = np.full(100000, np.float32(1e-42), f)
    check(orc, gpu_sum(xtr, sub, "f32"), sub, "f32", "subnormal")
    assert gpu_sum(xtr, sub, "f32") != 0.0


@pytest.mark.parametrize("kappa,seed", [(1e6, 400), (1e8, 401)])
def test_high_kappa(xtr, orc, kappa, seed):
    """Heavy cancellation under the 1e-6 relative bar: 2^19 values N(0, 1e4)
    with their negations, plus S ones, shuffled, so sum|x| / |sum x| is about
    kappa.  At kappa = 1e6 the derived bound d^2 u^2 kappa (chain depth
    d <= 18, u = 2^-24) is ~1e-6, so the bar holds by construction; at 1e8
    it holds because the compensation terms stay small here (their own
    rounding is ~u^2 of the partial sums' magnitudes)."""
    rng = np.random.default_rng(seed)
    m = 1 << 19
    b = (rng.standard_normal(m) * 1e4).astype(np.float32)
    total_abs = 2.0 * float(np.abs(b.astype(np.float64)).sum())
    ones = max(1, int(round(total_abs / kappa)))
    x = np.concatenate([b, -b, np.ones(ones, np.float32)])
    rng.shuffle(x)
    ref = orc.sum_float(x, "f32")
    k = orc.sum_abs(x, "f32") / abs(ref)
    assert ref == float(ones) and kappa / 2 <= k <= kappa * 2, (ref, k)
    for off in (0, 1):
        xs = np.concatenate([np.zeros(off, np.float32), x])
        got = gpu_sum(xtr, xs, "f32", off)
        assert abs(got - ref) <= 1e-6 * abs(ref), (kappa, off, got, ref)


def test_cancellation_pairs(xtr, orc):
    x = W.normal(300000, 8, "f32")
    pairs = np.empty(600000, np.float32)
    pairs[0::2], pairs[1::2] = x, -x
    check(orc, gpu_sum(xtr, pairs, "f32"), pairs, "f32")


@pytest.mark.parametrize("dt,codes", [("f8e4m3", 256), ("bf16", 65536), ("f16", 65536)])
def test_every_code(xtr, orc, dt, codes):
    """Every element code of the 8- and 16-bit formats summed alone (n = 1,
    through one batched launch) equals the oracle's exact decode."""
    sd = np.uint8 if codes == 256 else np.uint16
    allc = np.arange(codes, dtype=np.uint32).astype(sd)
    dev = to_dev(allc)
    srcs = [dev[i:i + 1] for i in range(codes)]
    got = xtr.reduce_sum_batched(srcs, dtype=dt).cpu().numpy()
    want = orc.decode(allc, dt)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])


def test_determinism_and_batched_equals_single(xtr):
    import torch
    bits = [data("bf16", n, 200 + n % 97) for n in (0, 5, 16384, 50001, 300000, 1 << 20)]
    devs = [to_dev(b) for b in bits]
    singles = [xtr.reduce_sum(d, dtype="bf16").item() for d in devs]
    again = [xtr.reduce_sum(d, dtype="bf16").item() for d in devs]
    assert singles == again
    batched = xtr.reduce_sum_batched(devs, dtype="bf16").cpu().tolist()
    assert batched == singles                     # bit-identical alone and in the batch
    torch.cuda.synchronize()


@pytest.mark.parametrize("dt", ["f32", "i32", "f8e4m3"])
def test_batched_vs_oracle(xtr, orc, dt):
    rng = np.random.Generator(np.random.PCG64(31))
    ns = [0, 1, 17] + [int(x) for x in rng.integers(1, 200000, 40)]
    bits = [data(dt, n, 300 + i) for i, n in enumerate(ns)]
    got = xtr.reduce_sum_batched([to_dev(b) for b in bits], dtype=dt).cpu().tolist()
    for b, g in zip(bits, got):
        check(orc, g, b, dt)


@pytest.mark.parametrize("dt", ["f32", "i32", "bf16"])
def test_segmented_small(xtr, orc, dt):
    total = 200000
    off = W.segment_offsets(total, 3000, 61)
    off[1500] = off[1499]                         # force an empty segment
    off[1501] = max(off[1501], off[1500])
    bits = data(dt, total, 62)
    d = to_dev(bits)
    doff = to_dev(off)
    got = xtr.reduce_sum_segmented(d, doff, dtype=dt).cpu().numpy()
    want = orc.sum_segmented(bits, off, dt)
    if dt == "i32":
        assert np.array_equal(got, want)
    else:
        for i in range(off.size - 1):
            seg = bits[off[i]:off[i + 1]]
            check_float_sum(float(got[i]), float(want[i]),
                            orc.sum_abs(seg, dt) if seg.size else 0.0, i)
    # each segment equals reduce_sum on that segment alone, bit for bit
    for i in list(range(0, 3000, 97)) + [1500]:
        alone = xtr.reduce_sum(d[off[i]:off[i + 1]], dtype=dt).item()
        assert alone == got[i] or (isinstance(alone, float) and math.isnan(alone)
                                   and math.isnan(got[i])), i


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16", "f8e4m3", "i32", "i64"])
def test_segmented_wave_and_chunk_paths(xtr, orc, dt):
    """Segments around the size where one wave instead of a workgroup chunk
    takes a segment (bodies of 2 * 256 * V elements, V = 16 / element size),
    starting at every alignment: every result equals reduce_sum on that
    segment alone, bit for bit, and the oracle to the usual bar."""
    eb = {"f32": 4, "bf16": 2, "f16": 2, "f8e4m3": 1, "i32": 4, "i64": 8}[dt]
    v = 16 // eb
    sm = 2 * 256 * v
    lens = []
    for base in (0, 1, 5, v - 1, v, 256 * v - 1, 256 * v + 1, sm - v, sm - 1, sm, sm + 1,
                 sm + v, 2 * sm, 4 * sm - 1, 4 * sm + 3, 9 * sm + 7):
        lens += [base, base + 1, max(base - 1, 0)]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64) + 3    # odd start
    total = int(off[-1]) + 5
    bits = data(dt, total, 91)
    d = to_dev(bits)
    got = xtr.reduce_sum_segmented(d, to_dev(off), dtype=dt).cpu().numpy()
    for i in range(len(lens)):
        seg = bits[off[i]:off[i + 1]]
        alone = xtr.reduce_sum(d[off[i]:off[i + 1]], dtype=dt).item()
        assert alone == got[i], (i, lens[i], alone, got[i])
        check(orc, int(got[i]) if dt in ("i32", "i64") else float(got[i]), seg, dt, (i, lens[i]))


def test_segmented_ws_and_invalid_table(xtr):
    import torch
    bits = data("f32", 100000, 71)
    off = W.segment_offsets(100000, 500, 72)
    d, doff = to_dev(bits), to_dev(off)
    nb = xtr.segmented_workspace_bytes(500, 100000, "f32")
    ws = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    a = xtr.reduce_sum_segmented_ws(d, doff, ws, total=100000, dtype="f32").cpu()
    b = xtr.reduce_sum_segmented_ws(d, doff, ws, total=100000, dtype="f32").cpu()   # reused
    c = xtr.reduce_sum_segmented(d, doff, dtype="f32").cpu()
    e = xtr.reduce_sum_segmented_ws(d, doff, ws, dtype="f32").cpu()   # chunk space from ws
    big = torch.zeros(4 * nb, dtype=torch.uint8, device="cuda")
    f = xtr.reduce_sum_segmented_ws(d, doff, big, dtype="f32").cpu()
    assert torch.equal(a, b) and torch.equal(a, c) and torch.equal(a, e) and torch.equal(a, f)
    # a workspace too small for the table's chunk space: every output NaN, and
    # the workspace stays usable
    off_long = np.array([0, 100000], dtype=np.int64)      # one segment of 13 chunks
    small_ws = torch.zeros(3072, dtype=torch.uint8, device="cuda")   # holds 10 chunk slots
    g = xtr.reduce_sum_segmented_ws(d, to_dev(off_long), small_ws, dtype="f32").cpu()
    assert torch.isnan(g).all()
    h = xtr.reduce_sum_segmented_ws(d[:10], to_dev(np.array([0, 10], np.int64)), small_ws,
                                    dtype="f32").cpu()
    assert h[0].item() == xtr.reduce_sum(d[:10], dtype="f32").item()
    bad = off.copy()
    bad[10], bad[11] = bad[11], bad[10] - 1        # a decreasing pair
    out = xtr.reduce_sum_segmented(d, to_dev(bad), dtype="f32").cpu()
    assert torch.isnan(out).all()
    again = xtr.reduce_sum_segmented(d, doff, dtype="f32").cpu()   # workspace still clean
    assert torch.equal(again, c)


def test_reduce_ws_reuse(xtr, orc):
    import torch
    n = 3 * (1 << 20) + 5
    bits = data("f32", n, 81)
    d = to_dev(bits)
    ws = torch.zeros(xtr.reduce_workspace_bytes(n, "f32"), dtype=torch.uint8, device="cuda")
    r1 = xtr.reduce_sum_ws(d, ws, dtype="f32").item()
    r2 = xtr.reduce_sum_ws(d[:n // 2], ws, dtype="f32").item()
    r3 = xtr.reduce_sum(d, dtype="f32").item()
    assert r1 == r3
    check(orc, r2, bits[:n // 2], "f32")


def test_plain_comparator(xtr, orc):
    """The uncompensated fp32 path runs the same structure; on the lognormal
    precision workload it is measurably worse than the compensated one."""
    bits, _ = W.signed_lognormal(1 << 22, 6, "bf16")
    d = to_dev(bits)
    ref = orc.sum_float(bits, "bf16")
    comp = xtr.reduce_sum(d, dtype="bf16").item()
    plain = xtr.reduce_sum_plain_f32(d, dtype="bf16").item()
    assert abs(comp - ref) <= 1e-6 * abs(ref)
    assert abs(plain - ref) <= 1e-2 * abs(ref)
    assert abs(comp - ref) <= abs(plain - ref)


@pytest.mark.parametrize("dt,n,seed", [("f32", 1 << 28, 4), ("i64", 1 << 28, 5)])
def test_full_size_scale(xtr, orc, dt, n, seed):
    bits = data(dt, n, seed)
    check(orc, gpu_sum(xtr, bits, dt), bits, dt, (dt, n))


@pytest.mark.parametrize("dt,seed", [("bf16", 6), ("f16", 7), ("f8e4m3", 8)])
def test_full_size_precision(xtr, orc, dt, seed):
    """Precision workload: 2^30 elements, +-lognormal(0, 2), scaled per tensor."""
    bits, _ = W.signed_lognormal(1 << 30, seed, dt)
    check(orc, gpu_sum(xtr, bits, dt), bits, dt, (dt, 1 << 30))


def test_segmented_full_config(xtr, orc):
    """Segmented workload: 2^27 fp32 N(0,1), 100k lognormal(6, 1.5) segments."""
    total = 1 << 27
    off = W.segment_offsets(total, 100000, 11)
    bits = W.normal(total, 10, "f32")
    got = xtr.reduce_sum_segmented(to_dev(bits), to_dev(off), dtype="f32").cpu().numpy()
    want = orc.sum_segmented(bits, off, "f32")
    nz = want != 0
    rel = np.abs(got[nz] - want[nz]) / np.abs(want[nz])
    assert rel.max() <= 1e-6, rel.max()
    assert np.all(got[~nz] == 0)


@pytest.mark.parametrize("dt", ["f32", "bf16", "f8e4m3", "i32", "i64"])
def test_segmented_fused_launch_same(xtr, orc, dt):
    """The segmented sum's two passes in one launch (seg_fused), or on two
    streams (seg_streams, with and without per-CU caps), and grids beyond the
    resident workgroups (seg_over), give the same bits as two launches on one
    stream, for small, chunked and empty segments; an invalid table still
    gives NaN / 0 everywhere."""
    import torch
    total = 300000
    off = W.segment_offsets(total, 2000, 95)
    off[700] = off[699]
    bits = data(dt, total, 96)
    d, doff = to_dev(bits), to_dev(off)
    orig = xtr.reduce_config(dt, "batched")
    try:
        res = {}
        modes = {0: dict(seg_fused=0, seg_streams=0, seg_over=1),
                 1: dict(seg_fused=1, seg_streams=0, seg_over=1),
                 2: dict(seg_fused=0, seg_streams=1, seg_small_per_cu=2, seg_chunk_per_cu=4),
                 3: dict(seg_fused=0, seg_streams=1, seg_small_per_cu=0, seg_chunk_per_cu=0),
                 4: dict(seg_fused=1, seg_streams=0, seg_over=4),
                 5: dict(seg_fused=0, seg_streams=0, seg_over=16)}
        for m, kw in modes.items():
            xtr.set_reduce_config(dt, "batched", **kw)
            res[m] = xtr.reduce_sum_segmented(d, doff, dtype=dt).cpu()
        for m in (1, 2, 3, 4, 5):
            assert torch.equal(res[0], res[m]), m
        want = orc.sum_segmented(bits, off, dt)
        if dt in ("i32", "i64"):
            assert np.array_equal(res[1].numpy(), want)
        bad = off.copy()
        bad[10], bad[11] = bad[11], bad[10] - 1
        for m in (1, 2, 4):
            xtr.set_reduce_config(dt, "batched", **modes[m])
            out = xtr.reduce_sum_segmented(d, to_dev(bad), dtype=dt).cpu()
            if dt in ("i32", "i64"):
                assert (out == 0).all()
            else:
                assert torch.isnan(out).all()
    finally:
        xtr.set_reduce_config(dt, "batched", **orig)


def test_segmented_more_than_4096_blocks(xtr, orc):
    """A table of 4.3M segments (more than 4096 planning blocks of 1024
    segments: the block totals go through the one-workgroup scan), int32
    (exact), lengths 0 .. 15 with a few long segments (several chunks each)."""
    rng = np.random.default_rng(99)
    nseg = 4_300_000
    lens = rng.integers(0, 16, nseg)
    lens[rng.integers(0, nseg, 40)] = rng.integers(20000, 200000, 40)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    bits = W.integers(int(off[-1]), 100, -1000, 1000, "i32")
    got = xtr.reduce_sum_segmented(to_dev(bits), to_dev(off), dtype="i32").cpu().numpy()
    assert np.array_equal(got, orc.sum_segmented(bits, off, "i32"))
