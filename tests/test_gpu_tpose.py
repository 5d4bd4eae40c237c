"""GPU parity of the transpose path against the CPU oracle: bit-exact in
every element size, across tiles, ragged edges, padded and unaligned leading
dimensions, unaligned pointers, batched launches and the full-size shapes."""
import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

SD = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}
NAME = {1: "u8", 2: "bf16", 4: "f32", 8: "f64"}
TILE = {1: 256, 2: 128, 4: 64, 8: 32}      # tile side in elements (256 bytes)
CANARY = 0xA5


def run_tpose(xtr, orc, rows, cols, eb, pad_s=0, pad_d=0, off_s=0, off_d=0, seed=0):
    """Transpose a random-bit rows x cols matrix with leading dimensions
    cols+pad_s / rows+pad_d, src and dst starting off_s / off_d elements into
    their buffers; compare every dst byte (padding and canaries included)."""
    import torch
    ld_s, ld_d = cols + pad_s, rows + pad_d
    n_src = off_s + (rows * ld_s if rows else 0)
    src = W.random_bits(max(n_src, 1), 1000 + seed, eb)
    dst_len = off_d + (cols * ld_d if cols else 0) + 7
    canary = np.frombuffer(bytes([CANARY]) * eb, dtype=SD[eb])[0]
    dst0 = np.full(dst_len, canary, dtype=SD[eb])
    d_src, d_dst = to_dev(src), to_dev(dst0)
    rc_src = d_src[off_s:] if off_s else d_src
    rc_dst = d_dst[off_d:] if off_d else d_dst
    xtr.tpose(rc_src, rc_dst, rows=rows, cols=cols, ld_src=ld_s, ld_dst=ld_d, dtype=NAME[eb])
    torch.cuda.synchronize()
    got = to_host(d_dst, SD[eb])
    want = dst0.copy()
    if rows and cols:
        orc.tpose(src[off_s:], rows, cols, ld_s, ld_d, dst=want[off_d:])
    assert np.array_equal(got, want), (rows, cols, eb, pad_s, pad_d, off_s, off_d)


def test_pr1_fp32_1024(xtr, orc):
    """PR1 workload: 1024 x 1024 fp32, U[-1, 1], seed 0."""
    import torch
    a = W.matrix(1024, 1024, 0, "f32")
    got = xtr.tpose(to_dev(a))
    torch.cuda.synchronize()
    assert np.array_equal(to_host(got, np.uint32), orc.tpose(a).view(np.uint32))


@pytest.mark.parametrize("eb", [1, 2, 4, 8])
def test_shapes_across_tiles(xtr, orc, eb):
    T = TILE[eb]
    shapes = [(1, 1), (1, 3 * T + 1), (2 * T + 5, 1), (17, 33), (T, T), (T - 1, T + 1),
              (2 * T + 3, 3 * T + 5), (3 * T, 2 * T)]
    for i, (r, c) in enumerate(shapes):
        run_tpose(xtr, orc, r, c, eb, seed=i)


@pytest.mark.parametrize("eb", [1, 2, 4, 8])
def test_leading_dims_and_alignment(xtr, orc, eb):
    T = TILE[eb]
    v = 16 // eb
    r, c = 2 * T + 7, T + 9
    run_tpose(xtr, orc, 2 * T, 2 * T, eb, pad_s=v, pad_d=2 * v)          # aligned padding: vector path
    run_tpose(xtr, orc, 2 * T, 2 * T, eb, pad_s=1, pad_d=0)              # unaligned ld: element path
    run_tpose(xtr, orc, 2 * T, 2 * T, eb, pad_s=0, pad_d=3)
    run_tpose(xtr, orc, r, c, eb, pad_s=5, pad_d=11)
    if eb < 16:
        run_tpose(xtr, orc, 2 * T, 2 * T, eb, off_s=1, off_d=0)          # unaligned pointers
        run_tpose(xtr, orc, T + 3, 2 * T, eb, off_s=0, off_d=1)


def _ld_with_piece(n, eb, w):
    """Smallest leading dimension >= n whose byte pitch admits W-byte pieces
    exactly (divisible by w, and not by 2w unless w = 16)."""
    ld = n
    while (ld * eb) % w or (w < 16 and (ld * eb) % (2 * w) == 0):
        ld += 1
    return ld


@pytest.mark.parametrize("eb,w", [(1, 4), (1, 8), (1, 16), (2, 4), (2, 8), (2, 16), (4, 4),
                                  (4, 8), (4, 16), (8, 8), (8, 16)])
def test_every_piece_width(xtr, orc, eb, w):
    """Each (element size, piece width) of the tile routine: whole tiles, and
    ragged rows / cols that cut a piece (partial pieces stored per element)."""
    T = TILE[eb]
    epw = w // eb
    for i, (r, c) in enumerate([(2 * T, 2 * T), (2 * T + epw - 1 if epw > 1 else 2 * T + 1, T + 3),
                                (T + 1, 3 * T - 1)]):
        ld_s, ld_d = _ld_with_piece(c, eb, w), _ld_with_piece(r, eb, w)
        run_tpose(xtr, orc, r, c, eb, pad_s=ld_s - c, pad_d=ld_d - r, seed=40 + i)


@pytest.mark.parametrize("eb", [1, 2])
def test_unaligned_rows(xtr, orc, eb):
    """Rows that are not 4-byte aligned (odd pitches, odd pointer offsets):
    interior tiles move funnel-shifted 4-byte pieces built from aligned
    dwords, edge tiles go element by element.  Every dst byte is compared,
    padding and canaries included, so a store outside a row segment shows;
    every src and dst misalignment occurs among the rows."""
    T = TILE[eb]
    if eb == 1:
        cases = [(1, 0, 0, 0), (0, 1, 0, 0), (3, 5, 1, 2), (2, 2, 3, 1), (1, 3, 2, 3),
                 (0, 0, 1, 3), (0, 0, 2, 0)]
    else:
        cases = [(1, 0, 0, 0), (0, 1, 0, 0), (3, 5, 1, 1), (2, 1, 1, 0), (0, 0, 1, 1)]
    for i, (pad_s, pad_d, off_s, off_d) in enumerate(cases):
        for j, (r, c) in enumerate([(3 * T + 5, 2 * T + 7), (4 * T, 4 * T)]):
            run_tpose(xtr, orc, r, c, eb, pad_s=pad_s, pad_d=pad_d, off_s=off_s, off_d=off_d,
                      seed=200 + 10 * i + j)


@pytest.mark.parametrize("eb", [2, 4, 8])
@pytest.mark.parametrize("tile", [1, 2, 3, 4])
def test_tile_geometries(xtr, orc, eb, tile):
    """512-byte src (tile 1), dst (tile 2) or both (tile 3), or 1 KiB dst row
    segments (tile 4; 2-byte elements keep the default for 3 and 4): whole and ragged tiles, 16-byte pieces,
    against the oracle; wide_min 0 lets every size take the wide geometry, the
    tuned threshold one large matrix."""
    orig = xtr.tpose_config(eb, "single")
    T = TILE[eb]
    try:
        xtr.set_tpose_config(eb, "single", tile=tile, wide_min=0)
        for i, (r, c) in enumerate([(8 * T, 16 * T), (16 * T + 3, 8 * T + 5),
                                    (12 * T - 1, 12 * T + 1), (T + 1, 2 * T - 1), (1, 1),
                                    (32 * T, 64 * T)]):
            if i == 5:
                xtr.set_tpose_config(eb, "single", wide_min=8)   # 2048 tiles: wide
            v = 16 // eb
            pad_s = (-c) % v + v * (i % 2)          # keep 16-byte pitches: 16-byte pieces
            pad_d = (-r) % v
            run_tpose(xtr, orc, r, c, eb, pad_s=pad_s, pad_d=pad_d, seed=60 + i)
    finally:
        xtr.set_tpose_config(eb, "single", **orig)


@pytest.mark.parametrize("geo", [1, 2, 3, 4])
@pytest.mark.parametrize("eb,w", [(2, 4), (2, 8), (2, 16), (4, 4), (4, 8), (4, 16), (8, 8),
                                  (8, 16)])
def test_tile_geometry_shared_rows(xtr, orc, eb, w, geo):
    """512-byte src (tile_shared = 1), dst (2) or both (3) row segments, or
    1 KiB dst ones (4), for rows that do not start on cache lines, with every piece width, whole
    and ragged tiles."""
    orig = xtr.tpose_config(eb, "single")
    T = TILE[eb]
    try:
        xtr.set_tpose_config(eb, "single", tile_shared=geo, wide_min=0)
        # every size in the wide geometry (one ragged tile included)
        for i, (r, c) in enumerate([(16 * T, 8 * T), (16 * T + 3, 8 * T + 5),
                                    (10 * T - 1, 12 * T + 1), (2 * T - 1, T + 1)]):
            ld_s, ld_d = _ld_with_piece(c, eb, w), _ld_with_piece(r, eb, w)
            if (ld_s * eb) % 128 == 0:
                ld_s += 16 // eb                     # rows must not start on lines
            run_tpose(xtr, orc, r, c, eb, pad_s=ld_s - c, pad_d=ld_d - r, seed=80 + i)
    finally:
        xtr.set_tpose_config(eb, "single", **orig)


@pytest.mark.parametrize("bpc,tile", [(1, 0), (2, 3), (1, 1), (3, 2), (2, 4)])
@pytest.mark.parametrize("eb,w", [(1, 16), (1, 4), (2, 16), (2, 8), (4, 16), (4, 8), (4, 4), (8, 16),
                                  (8, 8)])
def test_persistent_single(xtr, orc, eb, w, bpc, tile):
    """Persistent single launches (blocks_per_cu > 0, fewer workgroups than
    tiles): each workgroup takes several tiles in turn, interior and edge
    tiles, each tile geometry (wide_min 0), against the oracle, twice in a
    row."""
    orig = xtr.tpose_config(eb, "single")
    T = TILE[eb]
    try:
        xtr.set_tpose_config(eb, "single", blocks_per_cu=bpc, tile=tile, tile_shared=tile,
                             wide_min=0)
        for i, (r, c) in enumerate([(40 * T + 3, 36 * T + 5), (48 * T, 40 * T)]):
            ld_s, ld_d = _ld_with_piece(c, eb, w), _ld_with_piece(r, eb, w)
            for rep in range(2):
                run_tpose(xtr, orc, r, c, eb, pad_s=ld_s - c, pad_d=ld_d - r, seed=300 + 2 * i + rep)
    finally:
        xtr.set_tpose_config(eb, "single", **orig)


@pytest.mark.parametrize("run,xcd,narrow", [(0, 1, 0), (3, 1, 0), (0, 2, 0), (3, 2, 1), (0, 3, 1),
                                            (3, 3, 0)])
@pytest.mark.parametrize("wide", [0, 1, 2, 3, 4])
def test_batched_geometries(xtr, orc, wide, run, xcd, narrow):
    """Batched transposes with each tile geometry (512-byte src rows: 1, dst
    rows: 2, both: 3, 1 KiB dst rows: 4) for jobs whose rows share lines, mixed with small and aligned
    jobs, every element size and every piece width, in each XCD order (per round;
    one contiguous eighth of the launch order per XCD, with static slots or
    slots taken from counters), with or without one piece width per element
    size; each job against the oracle."""
    import torch
    rng = np.random.Generator(np.random.PCG64(19))
    origs = {eb: xtr.tpose_config(eb, "batched") for eb in (1, 2, 4, 8)}
    try:
        for eb in (2, 4, 8):
            xtr.set_tpose_config(eb, "batched", tile_shared=wide, tile=wide, run=run, xcd=xcd,
                                 narrow=narrow)
        xtr.set_tpose_config(1, "batched", run=run, xcd=xcd, narrow=narrow)
        jobs, hosts = [], []
        for i in range(112):                 # 28 jobs per element size: with one piece
            eb = [1, 2, 4, 8][i % 4]         # width per size, groups above 24 jobs (a table)
            r, c = (int(x) for x in rng.integers(1, 1500, 2))
            if i % 5 == 0:
                r, c = 8 * TILE[eb] + 3, 6 * TILE[eb] + 1      # many tiles: takes the geometry
            a = W.random_bits(r * c, 700 + i, eb).reshape(r, c)
            s = to_dev(a)
            d = torch.empty((c, r), dtype=s.dtype, device=s.device)
            jobs.append({"src": s, "dst": d, "rows": r, "cols": c, "dtype": NAME[eb]})
            hosts.append(a)
        for use_plan in (False, True):
            for j in jobs:
                j["dst"].fill_(0)
            if use_plan:
                p = xtr.TposePlan(jobs)
                p.run()
                p.run()                      # a second run (counters left at zero)
            else:
                xtr.tpose_batched(jobs)
            torch.cuda.synchronize()
            for j, a in zip(jobs, hosts):
                assert np.array_equal(to_host(j["dst"], a.dtype), orc.tpose(a)), (a.shape, a.dtype)
            if use_plan:
                p.close()
    finally:
        for eb, o in origs.items():
            xtr.set_tpose_config(eb, "batched", **o)


def test_tiny_enumeration(xtr, orc):
    for eb in (1, 4):
        for r in range(1, 12):
            for c in range(1, 12):
                run_tpose(xtr, orc, r, c, eb, seed=r * 16 + c)


def test_empty_is_noop(xtr, orc):
    run_tpose(xtr, orc, 0, 17, 4)
    run_tpose(xtr, orc, 9, 0, 2)


def test_involution_nan_payloads(xtr):
    import torch
    bits = W.random_bits(777 * 1031, 5, 4)
    a = to_dev(bits.reshape(777, 1031))
    back = xtr.tpose(xtr.tpose(a, dtype="f32"), dtype="f32")
    torch.cuda.synchronize()
    assert torch.equal(back, a)


def test_batched_mixed(xtr, orc):
    import torch
    rng = np.random.Generator(np.random.PCG64(9))
    jobs, hosts = [], []
    for i in range(48):
        eb = [1, 2, 4, 8][i % 4]
        r, c = (int(x) for x in rng.integers(1, 600, 2))
        a = W.random_bits(r * c, 50 + i, eb).reshape(r, c)
        s = to_dev(a)
        d = torch.empty((c, r), dtype=s.dtype, device=s.device)
        jobs.append({"src": s, "dst": d, "rows": r, "cols": c, "dtype": NAME[eb]})
        hosts.append(a)
    xtr.tpose_batched(jobs)
    torch.cuda.synchronize()
    for j, a in zip(jobs, hosts):
        got = to_host(j["dst"], a.dtype)
        assert np.array_equal(got, orc.tpose(a)), (a.shape, a.dtype)


def test_batched_fp32_config_shapes(xtr, orc):
    """Shapes of the batched workload (sides U{16..2048}, fp32), 256 jobs."""
    import torch
    shapes = W.batched_shapes(256, 9)
    jobs, hosts = [], []
    for i, (r, c) in enumerate(shapes):
        a = W.matrix(r, c, 100 + i, "f32")
        s = to_dev(a)
        jobs.append((s, torch.empty((c, r), dtype=s.dtype, device=s.device)))
        hosts.append(a)
    xtr.tpose_batched(jobs)
    torch.cuda.synchronize()
    for (s, d), a in zip(jobs, hosts):
        assert np.array_equal(to_host(d, np.uint32), orc.tpose(a).view(np.uint32))


@pytest.mark.parametrize("rows,cols,dt,seed", [(16384, 16384, "f32", 2), (12288, 20000, "bf16", 3)])
def test_full_size(xtr, orc, rows, cols, dt, seed):
    """The large single-job shapes, compared in full against the oracle."""
    import torch
    a = W.matrix(rows, cols, seed, dt)
    d = to_dev(a)
    got = xtr.tpose(d, dtype=dt)
    torch.cuda.synchronize()
    del d
    want = orc.tpose(a)
    assert np.array_equal(to_host(got, a.dtype), want)


def test_batched_config_every_job(xtr, orc):
    """The whole batched workload: 4096 fp32 transposes with rows and cols
    uniform in [16, 2048] (seed 9), random bit patterns (NaN payloads
    included), one tpose_batched call; every element of every job against
    the oracle (the oracle runs per job on 16 threads)."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    shapes = W.batched_shapes(4096, 9)

    def make(i):
        r, c = shapes[i]
        return W.random_bits(r * c, 20000 + i, 4).reshape(r, c)

    with ThreadPoolExecutor(16) as ex:
        hosts = list(ex.map(make, range(len(shapes))))
    jobs = []
    for a in hosts:
        s = to_dev(a)
        jobs.append((s, torch.empty((a.shape[1], a.shape[0]), dtype=s.dtype, device=s.device)))
    xtr.tpose_batched(jobs)
    torch.cuda.synchronize()

    def check(i):
        want = orc.tpose(hosts[i])
        got = to_host(jobs[i][1], np.uint32)
        return bool(np.array_equal(got, want))

    bad = []
    for k0 in range(0, len(jobs), 256):          # bounded host memory for the outputs
        with ThreadPoolExecutor(16) as ex:
            ok = list(ex.map(check, range(k0, min(len(jobs), k0 + 256))))
        bad += [k0 + i for i, v in enumerate(ok) if not v]
    assert not bad, (len(bad), [shapes[i] for i in bad[:5]])
