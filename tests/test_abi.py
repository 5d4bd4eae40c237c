"""The C-ABI library on the CPU: it loads, exports every entry point that
include/xtr.h declares, and rejects invalid arguments before touching HIP
(these calls never reach a GPU)."""
import ctypes as C
import os
import re

import pytest

import paper_2605_13864_amd as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xtr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(X.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return X.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tpose", "reduce_sum", "reduce_sum_plain_f32", "tpose_batched",
              "reduce_sum_segmented", "reduce_sum_batched", "reduce_sum_ws",
              "reduce_sum_segmented_ws", "xtr_reduce_workspace_bytes",
              "xtr_segmented_workspace_bytes", "xtr_last_error"):
        assert n in names, n


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding describes every one of them
    assert sorted(X._SIGS) == names


def test_info_entry_points(lib):
    assert X.version() >= (0, 1)
    for name, eb in X.ELEM_BYTES.items():
        assert lib.xtr_elem_bytes(X.CODES[name]) == eb
    assert lib.xtr_elem_bytes(99) == 0


FAKE = 0x7f0000001000   # never dereferenced: every call below fails validation


@pytest.mark.parametrize("args,code", [
    ((FAKE, FAKE + (1 << 30), 4, 4, 4, 4, 99), -2),        # unknown dtype
    ((FAKE, FAKE + (1 << 30), -1, 4, 4, 4, 0), -1),        # negative rows
    ((FAKE, FAKE + (1 << 30), 4, 8, 7, 4, 0), -1),         # ld_src < cols
    ((FAKE, FAKE + (1 << 30), 4, 8, 8, 3, 0), -1),         # ld_dst < rows
    ((0, FAKE, 4, 4, 4, 4, 0), -1),                        # null src
    ((FAKE + 2, FAKE + (1 << 30), 4, 4, 4, 4, 0), -4),     # fp32 pointer not 4-byte aligned
    ((FAKE, FAKE + 32, 4, 4, 4, 4, 0), -3),                # dst overlaps src
])
def test_tpose_rejects(lib, args, code):
    rc = lib.tpose(*[C.c_void_p(a) if i < 2 else a for i, a in enumerate(args)], None)
    assert rc == code
    assert lib.xtr_last_error()


def test_tpose_empty_is_noop(lib):
    assert lib.tpose(C.c_void_p(FAKE), C.c_void_p(FAKE), 0, 5, 5, 1, 0, None) == 0
    assert lib.tpose(C.c_void_p(0), C.c_void_p(0), 7, 0, 1, 7, 0, None) == 0


def test_tpose_batched_validates_every_descriptor(lib):
    arr = (X.TposeDesc * 3)()
    arr[0] = X.TposeDesc(FAKE, FAKE + (1 << 30), 4, 4, 4, 4, 0, 0)
    arr[1] = X.TposeDesc(FAKE + (1 << 31), FAKE + (3 << 30), 4, 4, 2, 4, 0, 0)   # bad ld
    arr[2] = X.TposeDesc(FAKE, FAKE + (1 << 30), 4, 4, 4, 4, 0, 0)
    assert lib.tpose_batched(C.cast(arr, C.c_void_p), 3, None) == -1
    assert b"descriptor 1" in lib.xtr_last_error()
    assert lib.tpose_batched(None, 0, None) == 0
    assert lib.tpose_batched(None, -1, None) == -1


@pytest.mark.parametrize("args,code", [
    ((FAKE, 10, FAKE + 4096, 99), -2),     # unknown dtype
    ((FAKE, 10, FAKE + 4096, 6), -2),      # f64 is transpose-only
    ((FAKE, -1, FAKE + 4096, 0), -1),      # negative n
    ((FAKE, 10, 0, 0), -1),                # null out
    ((0, 10, FAKE + 4096, 0), -1),         # null src
    ((FAKE + 1, 10, FAKE + 4096, 0), -4),  # misaligned fp32 src
    ((FAKE, 10, FAKE + 4100, 0), -4),      # misaligned double out
])
def test_reduce_sum_rejects(lib, args, code):
    src, n, out, dt = args
    assert lib.reduce_sum(C.c_void_p(src), n, C.c_void_p(out), dt, None) == code


def test_plain_comparator_takes_floats_only(lib):
    assert lib.reduce_sum_plain_f32(C.c_void_p(FAKE), 8, C.c_void_p(FAKE + 4096), 4, None) == -2


def test_workspace_sizes(lib):
    for dt in ("f32", "bf16", "f8e4m3", "i32", "i64", "f16"):
        a = lib.xtr_reduce_workspace_bytes(1 << 20, X.CODES[dt])
        b = lib.xtr_reduce_workspace_bytes(1 << 28, X.CODES[dt])
        assert 0 < a <= b
    assert lib.xtr_reduce_workspace_bytes(10, 6) == 0
    assert lib.xtr_segmented_workspace_bytes(100000, 1 << 27, 0) > 0
    # too-small caller workspace is refused before any launch
    assert lib.reduce_sum_ws(C.c_void_p(FAKE), 1 << 20, C.c_void_p(FAKE + (1 << 26)), 0,
                             C.c_void_p(FAKE + (1 << 27)), 16, None) == -7


def test_segmented_and_batched_validation(lib):
    assert lib.reduce_sum_segmented(C.c_void_p(FAKE), C.c_void_p(FAKE + 4096), 0,
                                    C.c_void_p(FAKE + 8192), 0, None) == 0
    assert lib.reduce_sum_segmented(C.c_void_p(FAKE), C.c_void_p(FAKE + 4096), -1,
                                    C.c_void_p(FAKE + 8192), 0, None) == -1
    assert lib.reduce_sum_segmented(C.c_void_p(FAKE), C.c_void_p(FAKE + 4097), 5,
                                    C.c_void_p(FAKE + 8192), 0, None) == -4
    assert lib.reduce_sum_segmented_ws_total(C.c_void_p(FAKE), C.c_void_p(FAKE + 4096), 5, 100,
                                             C.c_void_p(FAKE + 8192), 0,
                                             C.c_void_p(FAKE + 16384), 8, None) == -7
    # the workspace-only form sizes its chunk space from the workspace: 8 bytes hold none
    assert lib.reduce_sum_segmented_ws(C.c_void_p(FAKE), C.c_void_p(FAKE + 4096), 5,
                                       C.c_void_p(FAKE + 8192), 0, C.c_void_p(FAKE + 16384), 8,
                                       None) == -7
    assert lib.reduce_sum_batched(None, None, 0, C.c_void_p(FAKE), 0, None) == 0
    ptrs = (C.c_void_p * 2)(FAKE, FAKE + 3)
    ns = (C.c_int64 * 2)(4, 4)
    assert lib.reduce_sum_batched(C.cast(ptrs, C.c_void_p), C.cast(ns, C.c_void_p), 2,
                                  C.c_void_p(FAKE + 8192), 0, None) == -4
    assert b"job 1" in lib.xtr_last_error()


@pytest.mark.parametrize("args,code", [
    ((FAKE, 10, 0, 0, 1, 16, FAKE + 4096), -2),           # f32 is not an integer format
    ((FAKE, 10, 6, 0, 1, 16, FAKE + 4096), -2),           # nor f64
    ((FAKE, -1, 4, 0, 1, 16, FAKE + 4096), -1),           # negative n
    ((FAKE, 10, 4, 0, 0, 16, FAKE + 4096), -1),           # width 0
    ((FAKE, 10, 4, 0, 1, 0, FAKE + 4096), -1),            # no bins
    ((FAKE, 10, 4, 0, 1, (1 << 28) + 1, FAKE + 4096), -1),  # too many bins
    ((FAKE, 10, 4, 0, 1, 16, 0), -1),                     # null counts
    ((0, 10, 4, 0, 1, 16, FAKE + 4096), -1),              # null src
    ((FAKE + 2, 10, 4, 0, 1, 16, FAKE + 4096), -4),       # misaligned int32 src
    ((FAKE, 10, 4, 0, 1, 16, FAKE + 4100), -4),           # misaligned counts
    ((FAKE, 10, 4, 0, 1, 16, FAKE + 8), -3),              # counts overlap src
])
def test_histogram_int_rejects(lib, args, code):
    src, n, dt, lo, width, nb, counts = args
    assert lib.histogram_int(C.c_void_p(src), n, dt, lo, width, nb, C.c_void_p(counts),
                             None) == code
    assert lib.xtr_last_error()


@pytest.mark.parametrize("args,code", [
    ((FAKE, 10, 4, 0.0, 1.0, 16, FAKE + 4096), -2),               # i32 is not a float format
    ((FAKE, 10, 0, 1.0, 1.0, 16, FAKE + 4096), -1),               # empty range
    ((FAKE, 10, 0, 2.0, 1.0, 16, FAKE + 4096), -1),               # lo > hi
    ((FAKE, 10, 0, float("nan"), 1.0, 16, FAKE + 4096), -1),      # NaN bound
    ((FAKE, 10, 0, float("-inf"), 1.0, 16, FAKE + 4096), -1),     # infinite bound
    ((FAKE, 10, 0, -1.7e308, 1.7e308, 16, FAKE + 4096), -1),      # hi - lo overflows
    ((FAKE, 10, 0, 0.0, 5e-324, 16, FAKE + 4096), -1),            # nbins / (hi - lo) overflows
    ((FAKE, 10, 0, 0.0, 1.0, 0, FAKE + 4096), -1),                # no bins
    ((FAKE + 1, 10, 0, 0.0, 1.0, 16, FAKE + 4096), -4),           # misaligned fp32 src
])
def test_histogram_float_rejects(lib, args, code):
    src, n, dt, lo, hi, nb, counts = args
    assert lib.histogram_float(C.c_void_p(src), n, dt, lo, hi, nb, C.c_void_p(counts),
                               None) == code
    assert lib.xtr_last_error()


def test_histogram_rejects_int8_without_dtype():
    import torch
    with pytest.raises(TypeError):
        X.histogram_int(torch.zeros(4, dtype=torch.int8), 0, 1, 4)


@pytest.mark.parametrize("args,code", [
    ((FAKE, FAKE + (1 << 30), FAKE + (1 << 31), 4, 4, 4, 4, 4, 4, 0, 0), -2),   # f32 operands
    ((FAKE, FAKE + (1 << 30), FAKE + (1 << 31), -1, 4, 4, 4, 4, 4, 0, 2), -1),  # negative M
    ((FAKE, FAKE + (1 << 30), FAKE + (1 << 31), 4, 4, 8, 7, 4, 4, 0, 2), -1),   # lda < K
    ((FAKE, FAKE + (1 << 30), FAKE + (1 << 31), 4, 4, 8, 8, 4, 4, 1, 2), -1),   # ldb < K (Bt)
    ((FAKE, FAKE + (1 << 30), FAKE + (1 << 31), 4, 6, 8, 8, 6, 5, 0, 2), -1),   # ldc < N
    ((0, FAKE + (1 << 30), FAKE + (1 << 31), 4, 4, 4, 4, 4, 4, 0, 2), -1),      # null a
    ((FAKE + 1, FAKE + (1 << 30), FAKE + (1 << 31), 4, 4, 4, 4, 4, 4, 0, 2), -4),  # odd a
    ((FAKE, FAKE + (1 << 30), FAKE + (1 << 31) + 2, 4, 4, 4, 4, 4, 4, 0, 2), -4),  # c not 4-aligned
    ((FAKE, FAKE + (1 << 30), FAKE + 8, 4, 4, 4, 4, 4, 4, 0, 2), -3),           # c overlaps a
])
def test_matmul_rejects(lib, args, code):
    a, b, c, M, N, K, lda, ldb, ldc, tb, dt = args
    assert lib.matmul(C.c_void_p(a), C.c_void_p(b), C.c_void_p(c), M, N, K, lda, ldb, ldc, tb, dt,
                      None) == code
    assert lib.xtr_last_error()


def test_matmul_empty_is_noop(lib):
    assert lib.matmul(None, None, C.c_void_p(FAKE), 0, 4, 4, 4, 4, 4, 0, 2, None) == 0
    assert lib.matmul(None, None, C.c_void_p(FAKE), 4, 0, 4, 4, 4, 4, 0, 2, None) == 0


def test_launch_config_validation(lib):
    """The launch settings are range-checked (they change scheduling only);
    a rejected setting leaves the class's settings as they were."""
    orig = X.tpose_config(4, "batched")
    try:
        X.set_tpose_config(4, "batched", xcd=2)
        assert X.tpose_config(4, "batched")["xcd"] == 2
        for bad in ({"xcd": 4}, {"xcd": -1}, {"group": 0}, {"run": 65}, {"tile": 5},
                    {"blocks_per_cu": 65}, {"narrow": 2}, {"wide_min": 1025},
                    {"wide_min": -1}):
            with pytest.raises(X.XtrError) as e:
                X.set_tpose_config(4, "batched", **bad)
            assert e.value.code == -1, bad
        assert X.tpose_config(4, "batched")["xcd"] == 2
    finally:
        X.set_tpose_config(4, "batched", **orig)
    assert X.tpose_config(4, "batched") == orig
    ro = X.reduce_config("f32", "batched")
    try:
        X.set_reduce_config("f32", "batched", seg_over=16)
        for bad in ({"seg_over": 17}, {"seg_over": -1}, {"seg_chunk_per_cu": 65}):
            with pytest.raises(X.XtrError) as e:
                X.set_reduce_config("f32", "batched", **bad)
            assert e.value.code == -1, bad
        assert X.reduce_config("f32", "batched")["seg_over"] == 16
    finally:
        X.set_reduce_config("f32", "batched", **ro)
    assert X.reduce_config("f32", "batched") == ro
