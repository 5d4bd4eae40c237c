"""GPU parity of the matrix product against the CPU oracle: every entry within
the fp32-accumulation bound K * 2^-24 * sum_k |A[i][k] B[k][j]| of the
oracle's (exact products, compensated fp64 sums), for bf16 and fp16, both
layouts of B, one MFMA block, several tiles with ragged edges in M, N and K,
the element-wise load path (K or a leading dimension not a multiple of 8),
padded leading dimensions, K = 0, NaN propagation, and sampled entries at the
benchmark's full size."""
import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

SIGN = np.uint16(0x7FFF)


def operands(M, N, K, dt, seed, trans_b=False, scale=1.0):
    rng = np.random.default_rng(seed)
    a = W.to_bits(rng.standard_normal((M, K)) * scale, dt)
    b = W.to_bits(rng.standard_normal((N, K) if trans_b else (K, N)) * scale, dt)
    return a, b


def check(orc, got, a, b, dt, trans_b, what, **kw):
    ref = orc.matmul(a, b, dt, trans_b=trans_b, **kw)
    absref = orc.matmul(a & SIGN, b & SIGN, dt, trans_b=trans_b, **kw)
    K = kw.get("K", a.shape[1])
    bar = K * 2.0 ** -24 * absref + 1e-30
    err = np.abs(got.astype(np.float64) - ref)
    bad = np.argwhere(err > bar)
    assert bad.size == 0, (what, bad[:3].tolist(), err[tuple(bad[0])], bar[tuple(bad[0])])


def gpu_mm(xtr, a, b, dt, trans_b, **kw):
    ta, tb = to_dev(a), to_dev(b)
    return xtr.matmul(ta, tb, trans_b=trans_b, dtype=dt, **kw).cpu().numpy()


SHAPES = [(1, 1, 1), (32, 32, 16), (128, 128, 64), (129, 130, 72), (7, 300, 40),
          (300, 7, 520), (257, 129, 1000), (512, 384, 256)]


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("trans_b", [False, True])
def test_shapes(xtr, orc, dt, trans_b):
    for k, (M, N, K) in enumerate(SHAPES):
        a, b = operands(M, N, K, dt, 800 + k, trans_b)
        check(orc, gpu_mm(xtr, a, b, dt, trans_b), a, b, dt, trans_b, (dt, trans_b, M, N, K))


@pytest.mark.parametrize("trans_b", [False, True])
def test_elementwise_load_path(xtr, orc, trans_b):
    """K not a multiple of 8 (and so rows not 16-byte aligned): the loads go
    element by element."""
    for k, (M, N, K) in enumerate([(33, 65, 3), (130, 70, 77), (64, 64, 129)]):
        a, b = operands(M, N, K, "bf16", 820 + k, trans_b)
        check(orc, gpu_mm(xtr, a, b, "bf16", trans_b), a, b, "bf16", trans_b, (M, N, K))


def test_padded_leading_dimensions(xtr, orc):
    import torch
    M, N, K = 150, 90, 136
    a, b = operands(M, N, K, "bf16", 830)
    ap = np.full((M, K + 24), 0x7FC0, np.uint16)      # NaN padding must never be read
    ap[:, :K] = a
    bp = np.full((K, N + 10), 0x7FC0, np.uint16)
    bp[:, :N] = b
    c = torch.full((M, N + 6), 3.0, device="cuda")
    xtr.matmul(to_dev(ap), to_dev(bp), c, M=M, N=N, K=K, lda=K + 24, ldb=N + 10, ldc=N + 6,
               dtype="bf16")
    got = c.cpu().numpy()
    check(orc, got[:, :N], a, b, "bf16", False, "padded")
    assert (got[:, N:] == 3.0).all()                   # outside the M x N block: untouched
    bt = np.full((N, K + 8), 0x7FC0, np.uint16)
    bt[:, :K] = b.T
    got = xtr.matmul(to_dev(a), to_dev(bt), trans_b=True, N=N, ldb=K + 8,
                     dtype="bf16").cpu().numpy()
    check(orc, got, a, b, "bf16", False, "padded Bt")


def test_k_zero_and_empty(xtr):
    import torch
    a = torch.empty((5, 0), dtype=torch.bfloat16, device="cuda")
    b = torch.empty((0, 7), dtype=torch.bfloat16, device="cuda")
    c = torch.full((5, 7), 9.0, device="cuda")
    xtr.matmul(a, b, c)
    assert (c == 0).all()
    xtr.matmul(torch.empty((0, 4), dtype=torch.bfloat16, device="cuda"),
               torch.ones((4, 3), dtype=torch.bfloat16, device="cuda"))


def test_nan_propagates(xtr, orc):
    M, N, K = 70, 40, 96
    a, b = operands(M, N, K, "bf16", 840)
    a[3, 17] = 0x7FC0
    got = gpu_mm(xtr, a, b, "bf16", False)
    assert np.isnan(got[3]).all()
    rest = np.delete(np.arange(M), 3)
    ref = orc.matmul(a, b, "bf16")
    assert np.isfinite(got[rest]).all() and np.isfinite(ref[rest]).all()


@pytest.mark.parametrize("trans_b", [False, True])
def test_large_tiles_ragged(xtr, orc, trans_b):
    """A product big enough for the 256 x 256 workgroup tiles, with M, N and K
    not multiples of the tile: 3000 sampled entries, every edge row and column
    among them, against the oracle."""
    M, N, K = 4100, 4000, 200
    a, b = operands(M, N, K, "bf16", 845, trans_b)
    got = gpu_mm(xtr, a, b, "bf16", trans_b)
    rng = np.random.default_rng(846)
    edge_r = np.concatenate([np.arange(M - 4, M), np.arange(4096 - 2, 4096 + 2)])
    edge_c = np.concatenate([np.arange(N - 4, N), np.arange(3840 - 2, 3840 + 2)])
    rows = np.concatenate([rng.integers(0, M, 2000), np.repeat(edge_r, 64),
                           rng.integers(0, M, edge_c.size * 64)])
    cols = np.concatenate([rng.integers(0, N, 2000), rng.integers(0, N, edge_r.size * 64),
                           np.repeat(edge_c, 64)])
    ref = orc.matmul_entries(a, b, "bf16", rows, cols, trans_b=trans_b)
    absref = orc.matmul_entries(a & SIGN, b & SIGN, "bf16", rows, cols, trans_b=trans_b)
    err = np.abs(got[rows, cols].astype(np.float64) - ref)
    assert (err <= K * 2.0 ** -24 * absref + 1e-30).all(), err.max()


@pytest.mark.parametrize("trans_b", [False, True])
def test_full_size_sampled(xtr, orc, trans_b):
    """8192 x 8192 x 8192 bf16 (the benchmark's product): 256 sampled entries
    against the oracle, one by one."""
    import torch
    n = 8192
    gen = torch.Generator("cuda").manual_seed(850)
    ta = torch.randn((n, n), generator=gen, device="cuda").to(torch.bfloat16)
    tb = torch.randn((n, n), generator=gen, device="cuda").to(torch.bfloat16)
    c = xtr.matmul(ta, tb, trans_b=trans_b)
    a = ta.view(torch.int16).cpu().numpy().view(np.uint16)
    b = tb.view(torch.int16).cpu().numpy().view(np.uint16)
    rng = np.random.default_rng(851)
    rows = np.concatenate([rng.integers(0, n, 250), [0, n - 1, 0, n - 1, 4095, 4096]])
    cols = np.concatenate([rng.integers(0, n, 250), [0, n - 1, n - 1, 0, 4096, 4095]])
    got = c[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy()
    ref = orc.matmul_entries(a, b, "bf16", rows, cols, trans_b=trans_b)
    absref = orc.matmul_entries(a & SIGN, b & SIGN, "bf16", rows, cols, trans_b=trans_b)
    err = np.abs(got.astype(np.float64) - ref)
    assert (err <= n * 2.0 ** -24 * absref).all(), err.max()
    del ta, tb, c
    torch.cuda.empty_cache()


@pytest.mark.parametrize("trans_b", [False, True])
def test_deep_path_every_element(xtr, orc, trans_b):
    """4096 x 4096 x 96 bf16: 256 workgroup tiles of 256 x 256, as many as
    the CUs, so the product runs on the large-tile kernel; every one of the
    16.7M entries against the oracle (computed in row blocks on 16 threads)."""
    from concurrent.futures import ThreadPoolExecutor
    M = N = 4096
    K = 96
    a, b = operands(M, N, K, "bf16", 860, trans_b)
    got = gpu_mm(xtr, a, b, "bf16", trans_b)
    aa, ba = a & SIGN, b & SIGN

    def block(i0):
        i1 = min(M, i0 + 256)
        ref = orc.matmul(np.ascontiguousarray(a[i0:i1]), b, "bf16", trans_b=trans_b, N=N, K=K)
        absref = orc.matmul(np.ascontiguousarray(aa[i0:i1]), ba, "bf16", trans_b=trans_b, N=N, K=K)
        err = np.abs(got[i0:i1].astype(np.float64) - ref)
        return bool((err <= K * 2.0 ** -24 * absref + 1e-30).all()), float(err.max())

    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(block, range(0, M, 256)))
    assert all(ok for ok, _ in res), max(e for _, e in res)
