"""Pins of the CPU oracle: checks against what mathematics, the paper's
definitions, independent libraries (numpy, torch CPU casts, math.fsum) and
brute force fix.  Each pin takes an ``Oracle`` instance and raises
AssertionError on a mismatch, so the same pins can be run against the real
oracle and against deliberately broken builds of it (mutation tests)."""
from __future__ import annotations

import json
import math
import os

import numpy as np

import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SD = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------------ transpose

def pin_tpose_golden(o):
    """Hand-worked examples of out[x][y] = in[y][x] (Listing 3.5)."""
    for case in _gold("tpose_small.json")["cases"]:
        a = np.array(case["in"], dtype=np.int32)
        want = np.array(case["out"], dtype=np.int32)
        got = o.tpose(a)
        assert got.shape == want.shape and np.array_equal(got, want), (case, got)


def pin_tpose_iota(o):
    """Closed form: src[r][c] = r*cols + c gives dst[c][r] = r*cols + c."""
    for eb in (1, 2, 4, 8):
        for rows, cols in ((1, 1), (3, 5), (17, 9), (64, 65), (70, 33)):
            iota = (np.arange(rows * cols, dtype=np.uint64)).astype(SD[eb]).reshape(rows, cols)
            got = o.tpose(iota)
            r = np.arange(rows)[None, :]
            c = np.arange(cols)[:, None]
            want = (r * cols + c).astype(np.uint64).astype(SD[eb])
            assert np.array_equal(got, want), (eb, rows, cols)


def pin_tpose_library(o):
    """Special case that reduces to a library routine: numpy's ``.T.copy()``
    (bitwise, so NaN payloads and -0.0 must survive)."""
    for eb in (1, 2, 4, 8):
        a = W.random_bits(37 * 91, 101 + eb, eb).reshape(37, 91)
        assert np.array_equal(o.tpose(a), a.T.copy())
    f = np.array([[np.nan, -0.0], [np.inf, 1.5]], dtype=np.float32)
    f.view(np.uint32)[0, 0] = 0x7fc12345                   # NaN with a payload
    got = o.tpose(f).view(np.uint32)
    assert np.array_equal(got, f.view(np.uint32).T.copy())


def pin_tpose_involution_and_ld(o):
    """tpose(tpose(A)) == A through padded leading dimensions; padding and
    canary bytes around dst are never written."""
    rng = np.random.Generator(np.random.PCG64(7))
    for eb in (1, 2, 4, 8):
        for rows, cols, pad_s, pad_d in ((5, 7, 0, 3), (33, 2, 17, 1), (1, 40, 1, 0), (16, 16, 5, 5)):
            ld_s, ld_d = cols + pad_s, rows + pad_d
            src = rng.integers(0, 255, (rows * ld_s) * eb, dtype=np.uint8).view(SD[eb])
            canary = np.array(0xA5, dtype=np.uint8).repeat(eb).view(SD[eb])[0]
            dst = np.full((cols - 1) * ld_d + rows + 13, canary, dtype=SD[eb])
            o.tpose(src, rows, cols, ld_s, ld_d, dst=dst)
            for c in range(cols - 1):             # padding after each dst row untouched
                assert np.all(dst[c * ld_d + rows:(c + 1) * ld_d] == canary)
            assert np.all(dst[(cols - 1) * ld_d + rows:] == canary)   # canary after the end
            back = np.full(rows * ld_s, canary, dtype=SD[eb])
            o.tpose(dst, cols, rows, ld_d, ld_s, dst=back)
            for r in range(rows):
                assert np.array_equal(back[r * ld_s:r * ld_s + cols], src[r * ld_s:r * ld_s + cols])


def pin_tpose_permutation(o):
    """The output is a permutation of the input: equal sorted multisets."""
    a = W.random_bits(61 * 47, 5, 2).reshape(61, 47)
    got = o.tpose(a)
    assert np.array_equal(np.sort(got, axis=None), np.sort(a, axis=None))


def pin_tpose_bruteforce(o):
    """Tiny exhaustive enumeration against a pure-Python double loop."""
    for eb in (1, 4):
        for rows in range(1, 9):
            for cols in range(1, 9):
                a = W.random_bits(rows * cols, rows * 31 + cols, eb)
                want = [a[r * cols + c] for c in range(cols) for r in range(rows)]
                got = o.tpose(a.reshape(rows, cols)).ravel()
                assert list(got) == want, (eb, rows, cols)


# ------------------------------------------------------------------ integer sums

def pin_int_golden(o):
    g = _gold("sum_small.json")
    for case in g["int_cases"]:
        for dt in ("i32", "i64"):
            a = np.array(case["A"], dtype=np.int32 if dt == "i32" else np.int64)
            assert o.sum_int(a, dt) == (case["sum"], False), (case, dt)


def pin_int_closed_forms(o):
    """Gauss: sum_{i<n} i = n(n-1)/2; alternating sum_{i<n} (-1)^i i."""
    for n in (0, 1, 2, 3, 1000, 65537, 1 << 20):
        a = np.arange(n, dtype=np.int64)
        assert o.sum_int(a, "i64")[0] == n * (n - 1) // 2
        assert o.sum_int(a.astype(np.int32), "i32")[0] == n * (n - 1) // 2
        alt = np.where(a % 2 == 0, a, -a)
        want = -(n // 2) if n % 2 == 0 else (n - 1) // 2     # pairs (2k, -(2k+1)) give -1
        assert o.sum_int(alt, "i64")[0] == want, n


def pin_int_bruteforce_shuffle(o):
    """Brute force with Python integers; invariance under random shuffles;
    numpy's int64 sum (same modulo-2^64 semantics) where it applies."""
    rng = np.random.Generator(np.random.PCG64(11))
    for n in (0, 1, 5, 127, 4099):
        a32 = W.integers(n, 40 + n, -1000, 1000, "i32")
        want = sum(int(v) for v in a32)
        assert o.sum_int(a32, "i32") == (want, False)
        assert o.sum_int(rng.permutation(a32), "i32")[0] == want
        a64 = W.integers(n, 50 + n, -(1 << 40), 1 << 40, "i64")
        want = sum(int(v) for v in a64)
        assert o.sum_int(a64, "i64") == (want, False)
        assert o.sum_int(rng.permutation(a64), "i64")[0] == int(np.sum(a64, dtype=np.int64))


def pin_int_wrap(o):
    """int64 sums wrap modulo 2^64, and the overflow flag says so."""
    big = np.array([2 ** 63 - 1, 2 ** 63 - 1], dtype=np.int64)
    assert o.sum_int(big, "i64") == (-2, True)
    lo = np.array([-2 ** 63, -1], dtype=np.int64)
    assert o.sum_int(lo, "i64") == (2 ** 63 - 1, True)
    back = np.array([2 ** 63 - 1, 1, -1], dtype=np.int64)   # leaves the range, comes back
    assert o.sum_int(back, "i64") == (2 ** 63 - 1, False)
    mx = np.full(1 << 16, np.iinfo(np.int32).max, dtype=np.int32)   # int32 never wraps in int64
    assert o.sum_int(mx, "i32") == ((1 << 16) * (2 ** 31 - 1), False)


# ------------------------------------------------------------------ decoders

def pin_decode_golden(o):
    g = _gold("decode_codes.json")
    for dt in ("f8e4m3", "bf16", "f16"):
        sd = np.uint8 if dt == "f8e4m3" else np.uint16
        for code, val in g[dt]:
            got = o.decode(np.array([int(code, 16)], dtype=sd), dt)[0]
            if val == "nan":
                assert math.isnan(got), (dt, code)
                continue
            want = float.fromhex(val) if "0x" in val else float(val)
            assert got == want and math.copysign(1, got) == math.copysign(1, want), (dt, code, got)


def pin_decode_all_codes(o):
    """Every code of the 8- and 16-bit formats against torch's CPU casts
    (independent library), NaN positions included."""
    import torch
    u8 = np.arange(256, dtype=np.uint8)
    want = torch.from_numpy(u8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = o.decode(u8, "f8e4m3")
    assert np.array_equal(np.isnan(got), np.isnan(want))
    m = ~np.isnan(want)
    assert np.array_equal(got[m].view(np.uint64), want[m].view(np.uint64))
    u16 = np.arange(65536, dtype=np.uint16)
    want = torch.from_numpy(u16.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    got = o.decode(u16, "bf16")
    assert np.array_equal(np.isnan(got), np.isnan(want))
    m = ~np.isnan(want)
    assert np.array_equal(got[m].view(np.uint64), want[m].view(np.uint64))
    want = u16.view(np.float16).astype(np.float64)
    got = o.decode(u16, "f16")
    assert np.array_equal(np.isnan(got), np.isnan(want))
    m = ~np.isnan(want)
    assert np.array_equal(got[m].view(np.uint64), want[m].view(np.uint64))
    f = W.random_bits(4096, 3, 4).view(np.float32)
    got = o.decode(f, "f32")
    with np.errstate(invalid="ignore"):
        want = f.astype(np.float64)
    m = ~np.isnan(want)
    assert np.array_equal(np.isnan(got), ~m) and np.array_equal(got[m], want[m])


# ------------------------------------------------------------------ float sums

def pin_float_golden(o):
    g = _gold("sum_small.json")
    for case in g["float_cases_exact"]:
        a = np.array(case["A"], dtype=np.float32)
        assert o.sum_float(a, "f32") == case["sum"], case
    for case in g["plain_f32_cases"]:
        a = np.array(case["A"], dtype=np.float32)
        assert o.sum_plain_f32(a, "f32") == case["sum"], case


def pin_float_fsum(o):
    """Against math.fsum (correctly rounded): the fp64 Neumaier oracle is
    within a couple of ulps of the exactly rounded sum, per input format."""
    cases = [("f32", W.normal(1 << 16, 21, "f32")),
             ("f32", W.uniform(12345, 22, "f32")),
             ("bf16", W.signed_lognormal(1 << 15, 23, "bf16")[0]),
             ("f16", W.signed_lognormal(1 << 15, 24, "f16")[0]),
             ("f8e4m3", W.signed_lognormal(1 << 15, 25, "f8e4m3")[0])]
    for dt, bits in cases:
        vals = o.decode(bits, dt)
        exact = math.fsum(vals.tolist())
        got = o.sum_float(bits, dt)
        tol = 4 * math.ulp(abs(exact)) + 1e-300
        assert abs(got - exact) <= tol, (dt, got, exact)


def pin_float_closed_forms(o):
    """Sums fixed by arithmetic: 2^k copies of 1.0, x/-x pairs, a geometric
    series of powers of two; n = 0 and n = 1."""
    one_bf16 = np.full((1 << 20) + 3, 0x3F80, dtype=np.uint16)
    assert o.sum_float(one_bf16, "bf16") == float((1 << 20) + 3)
    one_f8 = np.full(1000, 0x38, dtype=np.uint8)
    assert o.sum_float(one_f8, "f8e4m3") == 1000.0
    x = W.normal(5000, 31, "f32")
    pairs = np.empty(10000, dtype=np.float32)
    pairs[0::2], pairs[1::2] = x, -x
    assert o.sum_float(pairs, "f32") == 0.0
    geo = np.array([2.0 ** -k for k in range(0, 41)], dtype=np.float32)
    assert o.sum_float(geo, "f32") == 2.0 - 2.0 ** -40
    assert o.sum_float(geo[::-1].copy(), "f32") == 2.0 - 2.0 ** -40
    assert o.sum_float(np.zeros(0, np.float32), "f32") == 0.0
    v = np.array([-3.25], dtype=np.float32)
    assert o.sum_float(v, "f32") == -3.25
    # cancellation a plain fp64 left-to-right sum gets wrong
    c = np.array([1.0, 1e30, 1.0, -1e30], dtype=np.float32)
    assert o.sum_float(c, "f32") == 2.0


def pin_float_nonfinite(o):
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    assert o.sum_float(np.array([1, inf, 2], np.float32), "f32") == math.inf
    assert o.sum_float(np.array([1, -inf, -inf], np.float32), "f32") == -math.inf
    assert math.isnan(o.sum_float(np.array([inf, 1, -inf], np.float32), "f32"))
    assert math.isnan(o.sum_float(np.array([1, nan, 1], np.float32), "f32"))
    assert math.isnan(o.sum_float(np.array([0x38, 0x7F], np.uint8), "f8e4m3"))


def pin_plain_f32(o):
    """Listing 2.1 as written: a sequential float accumulator.  numpy's
    float32 cumsum is the same left-to-right recurrence; at 2^24 + k ones the
    accumulator stagnates at 2^24 while the exact sum keeps counting."""
    for dt, bits in (("f32", W.normal(9999, 41, "f32")), ("f32", W.uniform(777, 42, "f32"))):
        want = float(np.cumsum(bits.astype(np.float32), dtype=np.float32)[-1])
        assert o.sum_plain_f32(bits, dt) == want
    ones = np.full((1 << 24) + 100, 0x3F80, dtype=np.uint16)
    assert o.sum_plain_f32(ones, "bf16") == float(1 << 24)
    assert o.sum_float(ones, "bf16") == float((1 << 24) + 100)


def pin_segmented(o):
    """Per-segment sums equal the single-range oracle on each segment; empty
    segments give 0."""
    off = W.segment_offsets(20000, 300, 61)
    bits = W.normal(20000, 62, "f32")
    got = o.sum_segmented(bits, off, "f32")
    for i in range(300):
        seg = bits[off[i]:off[i + 1]]
        assert got[i] == (o.sum_float(seg, "f32") if seg.size else 0.0)
        assert abs(got[i] - math.fsum(seg.astype(np.float64).tolist())) <= \
            4 * math.ulp(max(abs(got[i]), 1e-300))
    ints = W.integers(20000, 63, -1000, 1000, "i32")
    goti = o.sum_segmented(ints, off, "i32")
    for i in range(300):
        assert goti[i] == int(ints[off[i]:off[i + 1]].astype(np.int64).sum())
    off2 = np.array([0, 0, 3, 3, 5], dtype=np.int64)
    assert list(o.sum_segmented(np.arange(5, dtype=np.int32), off2, "i32")) == [0, 3, 0, 7]


def pin_sum_abs(o):
    """The sum of magnitudes (the scale of every float error bound): against
    math.fsum of |x| (correctly rounded, magnitudes taken with numpy, not the
    oracle) per format; closed forms on mixed signs (the integers -k..k give
    k(k + 1); +-2^-j for j < 41 give 2 - 2^-40); the triangle inequality
    sum|x| >= |sum x|, with equality on non-negative data; the IEEE rules
    (an infinity of either sign gives +inf, NaN gives NaN); n = 0 gives 0."""
    cases = [("f32", W.normal(1 << 15, 201, "f32")),
             ("bf16", W.signed_lognormal(1 << 14, 202, "bf16")[0]),
             ("f16", W.signed_lognormal(1 << 14, 203, "f16")[0]),
             ("f8e4m3", W.signed_lognormal(1 << 14, 204, "f8e4m3")[0])]
    for dt, bits in cases:
        if dt == "f32":
            mags = np.abs(bits.astype(np.float64))
        elif dt == "bf16":
            mags = np.abs(_bf16_values(bits))
        elif dt == "f16":
            mags = np.abs(bits.view(np.float16).astype(np.float64))
        else:
            import torch
            mags = np.abs(torch.from_numpy(bits).view(torch.float8_e4m3fn).to(torch.float64).numpy())
        exact = math.fsum(mags.tolist())
        got = o.sum_abs(bits, dt)
        assert abs(got - exact) <= 4 * math.ulp(exact), (dt, got, exact)
        assert got >= abs(o.sum_float(bits, dt))
    k = 3000
    ints = np.arange(-k, k + 1, dtype=np.float32)
    np.random.default_rng(205).shuffle(ints)
    assert o.sum_abs(ints, "f32") == float(k * (k + 1))
    assert o.sum_float(ints, "f32") == 0.0
    geo = np.array([(-1) ** j * 2.0 ** -j for j in range(41)], dtype=np.float32)
    assert o.sum_abs(geo, "f32") == 2.0 - 2.0 ** -40
    # magnitudes an uncompensated fp64 sum drops: 2^60 followed by 1000 ones of
    # either sign; the exact 2^60 + 1000 rounds to the fp64 value 2^60 + 1024
    wide = np.array([-2.0 ** 60] + [(-1.0) ** j for j in range(1000)], dtype=np.float32)
    assert o.sum_abs(wide, "f32") == float(2 ** 60 + 1000)
    pos = W.uniform(5000, 206, "f32", 0.0, 1.0)
    assert o.sum_abs(pos, "f32") == o.sum_float(pos, "f32")
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    assert o.sum_abs(np.array([1, -inf, 2], np.float32), "f32") == math.inf
    assert o.sum_abs(np.array([inf, -inf], np.float32), "f32") == math.inf
    assert math.isnan(o.sum_abs(np.array([1, nan, -inf], np.float32), "f32"))
    assert o.sum_abs(np.zeros(0, np.float32), "f32") == 0.0
    assert o.sum_abs(np.array([0xB8], np.uint8), "f8e4m3") == 1.0      # fp8 -1.0


# ------------------------------------------------------------------ prefix sums

def pin_scan_int(o):
    """Integer prefix sums: the iota closed form i(i+1)/2, numpy's int64 cumsum,
    Python-integer brute force modulo 2^64, and exclusive = inclusive - x."""
    for n in (0, 1, 2, 7, 1000):
        a = np.arange(1, n + 1, dtype=np.int32)
        inc = o.scan(a, "i32")
        assert [int(v) for v in inc] == [i * (i + 1) // 2 for i in range(1, n + 1)]
        exc = o.scan(a, "i32", exclusive=True)
        assert [int(v) for v in exc] == [i * (i - 1) // 2 for i in range(1, n + 1)]
    a = W.integers(50000, 71, -(1 << 30), 1 << 30, "i32")
    inc = o.scan(a, "i32")
    assert np.array_equal(inc, np.cumsum(a.astype(np.int64)))
    assert np.array_equal(o.scan(a, "i32", exclusive=True), inc - a.astype(np.int64))
    big = W.integers(3000, 72, -(1 << 62), 1 << 62, "i64")
    run, want = 0, []
    for v in big.tolist():
        run += v
        want.append((run + (1 << 63)) % (1 << 64) - (1 << 63))   # two's-complement wrap
    assert [int(v) for v in o.scan(big, "i64")] == want


def pin_scan_float(o):
    """Float prefix sums: every prefix within 4 ulp of math.fsum of that prefix
    (correctly rounded), the exclusive scan shifted by one with a leading 0,
    the last inclusive prefix equal to the full fsum, and the IEEE rules."""
    for dt, seed in (("f32", 73), ("bf16", 74), ("f8e4m3", 75)):
        bits = W.signed_lognormal(700, seed, dt)[0] if dt != "f32" else W.normal(700, seed, "f32")
        x = o.decode(bits, dt).tolist()
        inc = o.scan(bits, dt)
        exc = o.scan(bits, dt, exclusive=True)
        for i in range(len(x)):
            ref = math.fsum(x[:i + 1])
            assert abs(inc[i] - ref) <= 4 * math.ulp(max(abs(ref), 1e-300)), (dt, i)
        assert exc[0] == 0.0 and np.array_equal(exc[1:], inc[:-1])
        assert inc[-1] == o.sum_float(bits, dt)
    f = np.array([1.0, np.inf, 2.0, -np.inf, 3.0], dtype=np.float32)
    got = o.scan(f, "f32")
    assert got[0] == 1.0 and got[1] == np.inf and got[2] == np.inf and np.isnan(got[3:]).all()
    gotx = o.scan(f, "f32", exclusive=True)
    assert gotx[0] == 0.0 and gotx[1] == 1.0 and gotx[2] == np.inf and np.isnan(gotx[4])
    g = np.array([1.0, np.nan, 2.0], dtype=np.float32)
    assert o.scan(g, "f32")[0] == 1.0 and np.isnan(o.scan(g, "f32")[1:]).all()
    # 1 + 1e30 - 1e30 + 1: the compensated running sum keeps both ones
    c = np.array([1.0, 1e30, -1e30, 1.0], dtype=np.float32)
    assert list(o.scan(c, "f32")) == [1.0, float(np.float32(1e30)) + 1.0, 1.0, 2.0]


# ------------------------------------------------------------------ histograms

def pin_histogram_int(o):
    """Integer bins against numpy.histogram on exact integer edges, brute force
    on small inputs, and the total = the number of in-range elements."""
    a = W.integers(100000, 81, -5000, 5000, "i32")
    for lo, width, nb in ((-5000, 10, 1000), (-1234, 7, 300), (0, 1, 4096), (-6000, 100, 150)):
        got = o.histogram_int(a, "i32", lo, width, nb)
        hi = lo + nb * width                         # numpy closes the last bin: drop x == hi
        want, _ = np.histogram(a[a != hi].astype(np.float64), bins=nb, range=(lo, hi))
        assert np.array_equal(got, want), (lo, width, nb)
        inr = int(((a >= lo) & (a < lo + nb * width)).sum())
        assert got.sum() == inr
    b = np.array([0, 1, 2, 3, 255, 7, 8, 9], dtype=np.uint8)
    got = o.histogram_int(b, "u8", 2, 3, 3)           # bins [2,5) [5,8) [8,11)
    assert list(got) == [2, 1, 2]
    big = np.array([-(1 << 62), 1 << 62, 5, 6], dtype=np.int64)
    assert list(o.histogram_int(big, "i64", 5, 1, 2)) == [1, 1]


def pin_histogram_u16(o):
    """The uint16 branch: every one of the 65536 codes once, in width-1 bins
    (each bin holds exactly its code) and in bins that start above 2^15 (the
    codes must read as unsigned); random data against numpy.bincount of the
    bin index computed with Python integers; brute force on a small input."""
    codes = np.arange(1 << 16, dtype=np.uint16)
    np.random.default_rng(207).shuffle(codes)
    assert np.array_equal(o.histogram_int(codes, "u16", 0, 1, 1 << 16), np.ones(1 << 16, np.int64))
    got = o.histogram_int(codes, "u16", 40000, 1000, 30)      # [40000, 70000): 25536 codes
    want = [1000] * 25 + [536] + [0] * 4
    assert list(got) == want, got
    assert list(o.histogram_int(codes, "u16", -5, 16, 4)) == [11, 16, 16, 16]
    x = W.integers(200000, 208, 0, 65535, "i32").astype(np.uint16)
    for lo, width, nb in ((0, 256, 256), (-300, 7, 10000), (32000, 3, 500)):
        d = x.astype(np.int64) - lo
        keep = (d >= 0) & (d < width * nb)
        want = np.bincount((d[keep] // width).astype(np.int64), minlength=nb)
        assert np.array_equal(o.histogram_int(x, "u16", lo, width, nb), want), (lo, width, nb)
    small = np.array([65535, 0, 32768, 32767, 65534, 1], dtype=np.uint16)
    want = [0, 0, 0]
    for v in small.tolist():                       # brute force, Python integers
        d = v - 32767
        if 0 <= d < 3 * 16384:
            want[d // 16384] += 1
    assert want == [2, 1, 1]
    assert list(o.histogram_int(small, "u16", 32767, 16384, 3)) == want


def _check_vs_numpy(got, xd, lo, hi, nb):
    """``got`` against numpy.histogram over the same fp64 values.  numpy closes
    its last bin, so x == hi is dropped first.  With dyadic edges both rules
    are exact and must agree bin for bin; otherwise numpy places an element
    against rounded linspace edges, so the two may differ only for elements
    within rounding of an interior edge."""
    xd = xd[np.isfinite(xd) & (xd != hi)]
    want, edges = np.histogram(xd, bins=nb, range=(lo, hi))
    width = hi - lo
    if (nb & (nb - 1)) == 0 and math.frexp(width)[0] == 0.5 and (lo / (width / nb)).is_integer():
        assert np.array_equal(got, want), (lo, hi, nb)
        return
    inner = edges[1:-1]
    k = np.clip(np.searchsorted(inner, xd), 1, max(len(inner), 1)) if len(inner) else None
    near = 0
    if len(inner):
        d = np.minimum(np.abs(xd - inner[k - 1]), np.abs(xd - inner[np.minimum(k, len(inner) - 1)]))
        near = int((d <= 1e-12 * np.maximum(1.0, np.abs(xd))).sum())
    assert got.sum() == want.sum() and np.abs(got - want).sum() <= 2 * near, (lo, hi, nb)


def pin_histogram_float(o):
    """Float bins against numpy.histogram (its uniform-bin rule, in fp64), the
    half-open range (lo counted, hi not), NaN and infinities not counted."""
    x = W.normal(200000, 82, "f32")
    xd = x.astype(np.float64)
    for lo, hi, nb in ((-4.0, 4.0, 256), (-1.0, 2.5, 1000), (0.0, 1.0, 7), (-0.5, 3.0, 1)):
        _check_vs_numpy(o.histogram_float(x, "f32", lo, hi, nb), xd, lo, hi, nb)
    e = np.array([0.0, 1.0, 0.5, np.nan, np.inf, -np.inf, 0.999999, -1e-30], dtype=np.float32)
    got = o.histogram_float(e, "f32", 0.0, 1.0, 2)
    assert list(got) == [1, 2], got                  # 0.0 -> bin 0; 0.5, 0.999999 -> bin 1
    bits, _ = W.signed_lognormal(50000, 83, "bf16")
    vals = o.decode(bits, "bf16")
    _check_vs_numpy(o.histogram_float(bits, "bf16", -10.0, 10.0, 64), vals, -10.0, 10.0, 64)
    _check_vs_numpy(o.histogram_float(bits, "bf16", -8.0, 8.0, 64), vals, -8.0, 8.0, 64)


PINS_TPOSE = [pin_tpose_golden, pin_tpose_iota, pin_tpose_library, pin_tpose_involution_and_ld,
              pin_tpose_permutation, pin_tpose_bruteforce]
PINS_INT = [pin_int_golden, pin_int_closed_forms, pin_int_bruteforce_shuffle, pin_int_wrap]
PINS_FLOAT = [pin_decode_golden, pin_decode_all_codes, pin_float_golden, pin_float_fsum,
              pin_float_closed_forms, pin_float_nonfinite, pin_plain_f32, pin_segmented]
PINS_ABS = [pin_sum_abs]
PINS_SCAN = [pin_scan_int, pin_scan_float]
# ------------------------------------------------------------------ matmul

def _bf16_values(bits):
    """Values of bf16 bits by the format definition (the top half of binary32),
    with numpy only: independent of the oracle's decoder."""
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def pin_matmul_exact_small(o):
    """Against exact rational arithmetic (Python fractions) on small random
    bf16 and fp16 matrices, both layouts of B: within one rounding of the exact
    product sum."""
    from fractions import Fraction
    for dt, M, N, K, seed in (("bf16", 5, 7, 13, 90), ("f16", 6, 3, 17, 91), ("bf16", 1, 1, 40, 92)):
        a = W.to_bits(np.random.default_rng(seed).standard_normal((M, K)) * 3, dt)
        b = W.to_bits(np.random.default_rng(seed + 1).standard_normal((K, N)) * 3, dt)
        av = _bf16_values(a) if dt == "bf16" else a.view(np.float16).astype(np.float64)
        bv = _bf16_values(b) if dt == "bf16" else b.view(np.float16).astype(np.float64)
        got = o.matmul(a, b, dt)
        got_t = o.matmul(a, np.ascontiguousarray(b.T), dt, trans_b=True)
        assert np.array_equal(got, got_t)
        for i in range(M):
            for j in range(N):
                ex = sum(Fraction(float(av[i, k])) * Fraction(float(bv[k, j])) for k in range(K))
                assert abs(Fraction(got[i, j]) - ex) <= abs(ex) * Fraction(1, 2 ** 52), (dt, i, j)


def pin_matmul_integers(o):
    """Integer-valued bf16 matrices: every product and sum is exact, so the
    result equals numpy's int64 matrix product exactly."""
    rng = np.random.default_rng(93)
    ai = rng.integers(-16, 17, (33, 70))
    bi = rng.integers(-16, 17, (70, 21))
    a = W.to_bits(ai.astype(np.float64), "bf16")
    b = W.to_bits(bi.astype(np.float64), "bf16")
    assert np.array_equal(o.matmul(a, b, "bf16"), (ai @ bi).astype(np.float64))


def pin_matmul_closed_forms(o):
    """A[i][k] = i, B[k][j] = j + 1: C[i][j] = i * K * (j + 1).  Identity:
    A @ I = A.  Cancellation: 2^100 * 1 + 1 * 1 + (-2^100) * 1 = 1, which a
    plain fp64 sum gets wrong (0)."""
    M, N, K = 9, 11, 24
    a = W.to_bits(np.repeat(np.arange(M, dtype=np.float64)[:, None], K, axis=1), "bf16")
    b = W.to_bits(np.repeat(np.arange(1, N + 1, dtype=np.float64)[None, :], K, axis=0), "bf16")
    want = np.arange(M)[:, None] * K * np.arange(1, N + 1)[None, :]
    assert np.array_equal(o.matmul(a, b, "bf16"), want.astype(np.float64))
    x = W.to_bits(np.random.default_rng(94).standard_normal((6, 8)), "bf16")
    eye = W.to_bits(np.eye(8), "bf16")
    assert np.array_equal(o.matmul(x, eye, "bf16"), _bf16_values(x))
    ca = W.to_bits(np.array([[2.0 ** 100, 1.0, -2.0 ** 100]]), "bf16")
    cb = W.to_bits(np.ones((3, 1)), "bf16")
    assert o.matmul(ca, cb, "bf16")[0, 0] == 1.0


def pin_matmul_leading_dims_and_entries(o):
    """Padded leading dimensions give the packed result; sampled entries equal
    the full product's; B^T storage equals B storage."""
    rng = np.random.default_rng(95)
    M, N, K = 13, 10, 29
    a = W.to_bits(rng.standard_normal((M, K)), "bf16")
    b = W.to_bits(rng.standard_normal((K, N)), "bf16")
    full = o.matmul(a, b, "bf16")
    ap = np.zeros((M, K + 5), np.uint16)
    ap[:, :K] = a
    ap[:, K:] = 0x7FC0                                  # NaN padding must never be read
    bp = np.full((K, N + 3), 0x7FC0, np.uint16)
    bp[:, :N] = b
    assert np.array_equal(o.matmul(ap, bp, "bf16", M=M, N=N, K=K, lda=K + 5, ldb=N + 3), full)
    bt = np.full((N, K + 2), 0x7FC0, np.uint16)
    bt[:, :K] = b.T
    assert np.array_equal(o.matmul(a, bt, "bf16", trans_b=True, N=N, ldb=K + 2), full)
    r = rng.integers(0, M, 20)
    c = rng.integers(0, N, 20)
    assert np.array_equal(o.matmul_entries(a, b, "bf16", r, c), full[r, c])


def pin_matmul_nonfinite(o):
    """inf * 0 is NaN; inf + -inf is NaN; one infinite product gives inf."""
    inf = np.inf
    a = W.to_bits(np.array([[inf, 1.0], [inf, 1.0], [inf, -inf]]), "f32")
    b = W.to_bits(np.array([[0.0, 2.0], [1.0, 1.0]]), "f32")
    got = o.matmul(a, b, "f32")
    assert np.isnan(got[0, 0]) and got[0, 1] == inf and np.isnan(got[2, 1])


PINS_HIST = [pin_histogram_int, pin_histogram_u16, pin_histogram_float]
PINS_MM = [pin_matmul_exact_small, pin_matmul_integers, pin_matmul_closed_forms,
           pin_matmul_leading_dims_and_entries, pin_matmul_nonfinite]
ALL_PINS = PINS_TPOSE + PINS_INT + PINS_FLOAT + PINS_ABS + PINS_SCAN + PINS_HIST + PINS_MM
