"""CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path never does.

It wraps ``oracle.c`` (plain single-threaded C, built with gcc) through ctypes:

* ``tpose(src2d, ...)``        out[x][y] = in[y][x], Listing 3.5, as a bit copy.
* ``sum_int(bits, dtype)``      Listing 2.1 / reduce_sum over int32 or int64
                                (int64 wraps modulo 2^64; overflow is reported).
* ``sum_float(bits, dtype)``    Listing 2.1 / reduce_sum over fp32, bf16, fp16 or
                                fp8-e4m3fn, exact decode to fp64 + fp64 Neumaier.
* ``sum_plain_f32(bits, dtype)`` Listing 2.1 exactly as written (float accumulator).
* ``decode(bits, dtype)``       exact fp64 value of every element.
* ``sum_segmented(...)``        the sum above per CSR segment.
* ``tpose_batched(jobs)``       the transpose above per job.
* ``scan(bits, dtype, excl)``   inclusive / exclusive prefix sums, same arithmetic as the sums.
* ``histogram_int(...)``        counts in ``nbins`` bins of ``width`` from ``lo`` (exact).
* ``histogram_float(...)``      counts in ``nbins`` equal bins of [lo, hi), fp64 bin rule.
* ``matmul(a, b, dtype)``       fp64 C = A @ B (exact products, compensated sums in k order).
* ``matmul_entries(...)``       sampled entries of the same product.

``Oracle(path)`` loads any build of ``oracle.c`` (the mutation tests load
deliberately broken copies to show that the pins catch them).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
OMP_SRC = os.path.join(HERE, "oracle_omp.c")        # all-cores baseline (bench cpu leg)
OMP_LIB = os.path.join(HERE, "liboracle_omp.so")

# oracle-local dtype codes (mirror the enum in oracle.c, not the product's)
CODES = {"f32": 0, "f16": 1, "bf16": 2, "f8e4m3": 3, "i32": 4, "i64": 5}
HCODES = {"i32": 4, "i64": 5, "u8": 7, "u16": 8}       # integer histogram inputs
FLOATS = ("f32", "f16", "bf16", "f8e4m3")
INTS = ("i32", "i64")


def build(src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compile ``src`` into the shared library ``out`` with gcc (no -ffast-math,
    no FMA contraction, so the fp64 arithmetic is exactly what is written)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
           "-fno-fast-math", *extra, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def build_omp(src: str = OMP_SRC, out: str = OMP_LIB) -> str:
    """Compile the OpenMP build of the same plain loops (the all-cores CPU
    baseline of the benchmark)."""
    return build(src, out, extra=("-fopenmp",))


def _stale(lib: str, src: str) -> bool:
    return not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    def __init__(self, path: str = LIB):
        if path == LIB and _stale(LIB, SRC):
            build()
        lib = C.CDLL(path)
        i64, vp = C.c_int64, C.c_void_p
        lib.oracle_tpose.argtypes = [vp, vp, i64, i64, i64, i64, C.c_int]
        lib.oracle_tpose.restype = C.c_int
        lib.oracle_sum_int.argtypes = [vp, i64, C.c_int, C.POINTER(C.c_int)]
        lib.oracle_sum_int.restype = C.c_int64
        lib.oracle_sum_float.argtypes = [vp, i64, C.c_int]
        lib.oracle_sum_float.restype = C.c_double
        lib.oracle_sum_abs.argtypes = [vp, i64, C.c_int]
        lib.oracle_sum_abs.restype = C.c_double
        lib.oracle_sum_plain_f32.argtypes = [vp, i64, C.c_int]
        lib.oracle_sum_plain_f32.restype = C.c_float
        lib.oracle_decode_all.argtypes = [vp, i64, C.c_int, vp]
        lib.oracle_decode_all.restype = C.c_int
        lib.oracle_sum_segmented.argtypes = [vp, vp, i64, C.c_int, vp]
        lib.oracle_sum_segmented.restype = C.c_int
        lib.oracle_elem_bytes.argtypes = [C.c_int]
        lib.oracle_elem_bytes.restype = C.c_int
        lib.oracle_scan_int.argtypes = [vp, i64, C.c_int, C.c_int, vp]
        lib.oracle_scan_int.restype = C.c_int
        lib.oracle_scan_float.argtypes = [vp, i64, C.c_int, C.c_int, vp]
        lib.oracle_scan_float.restype = C.c_int
        lib.oracle_histogram_int.argtypes = [vp, i64, C.c_int, i64, i64, i64, vp]
        lib.oracle_histogram_int.restype = C.c_int
        lib.oracle_histogram_float.argtypes = [vp, i64, C.c_int, C.c_double, C.c_double, i64, vp]
        lib.oracle_histogram_float.restype = C.c_int
        lib.oracle_matmul.argtypes = [vp, vp, vp, i64, i64, i64, i64, i64, i64, C.c_int, C.c_int]
        lib.oracle_matmul.restype = C.c_int
        lib.oracle_matmul_entries.argtypes = [vp, vp, i64, i64, i64, i64, i64, C.c_int, C.c_int,
                                              i64, vp, vp, vp]
        lib.oracle_matmul_entries.restype = C.c_int
        self.lib = lib
        self.path = path

    # ------------------------------------------------------------ transpose
    def tpose(self, src: np.ndarray, rows: int | None = None, cols: int | None = None,
              ld_src: int | None = None, ld_dst: int | None = None,
              dst: np.ndarray | None = None) -> np.ndarray:
        """Transpose of the ``rows x cols`` matrix stored with leading dimension
        ``ld_src`` in the flat or 2-D array ``src``.  Without ``dst`` a fresh
        ``cols x rows`` array is returned; with ``dst`` (flat, length
        >= (cols-1)*ld_dst + rows) it is written in place."""
        src = np.ascontiguousarray(src)
        if rows is None:
            rows, cols = src.shape
        ld_src = cols if ld_src is None else ld_src
        if dst is None:
            ld_dst = rows if ld_dst is None else ld_dst
            dst = np.zeros(max(cols, 1) * ld_dst if rows and cols else 0, dtype=src.dtype)
            rc = self.lib.oracle_tpose(_ptr(src), _ptr(dst), rows, cols, ld_src, ld_dst,
                                       src.itemsize)
            if rc:
                raise ValueError("oracle_tpose: invalid arguments")
            if ld_dst == rows:
                return dst.reshape(cols, rows)
            return dst
        assert dst.flags.c_contiguous
        rc = self.lib.oracle_tpose(_ptr(src), _ptr(dst), rows, cols, ld_src, ld_dst, src.itemsize)
        if rc:
            raise ValueError("oracle_tpose: invalid arguments")
        return dst

    def tpose_batched(self, srcs):
        """One fresh transpose per 2-D input array."""
        return [self.tpose(s) for s in srcs]

    # ------------------------------------------------------------ sums
    def sum_int(self, bits: np.ndarray, dtype: str):
        """(wrapped int64 sum, overflow flag) over int32 or int64 elements."""
        assert dtype in INTS
        bits = np.ascontiguousarray(bits)
        ov = C.c_int(0)
        v = self.lib.oracle_sum_int(_ptr(bits), bits.size, CODES[dtype], C.byref(ov))
        return int(v), bool(ov.value)

    def sum_float(self, bits: np.ndarray, dtype: str) -> float:
        assert dtype in FLOATS
        bits = np.ascontiguousarray(bits)
        return float(self.lib.oracle_sum_float(_ptr(bits), bits.size, CODES[dtype]))

    def sum(self, bits: np.ndarray, dtype: str):
        """fp64 sum for float formats, wrapped int64 sum for integer formats."""
        return self.sum_int(bits, dtype)[0] if dtype in INTS else self.sum_float(bits, dtype)

    def sum_abs(self, bits: np.ndarray, dtype: str) -> float:
        bits = np.ascontiguousarray(bits)
        return float(self.lib.oracle_sum_abs(_ptr(bits), bits.size, CODES[dtype]))

    def sum_plain_f32(self, bits: np.ndarray, dtype: str) -> float:
        bits = np.ascontiguousarray(bits)
        return float(np.float32(self.lib.oracle_sum_plain_f32(_ptr(bits), bits.size,
                                                               CODES[dtype])))

    def decode(self, bits: np.ndarray, dtype: str) -> np.ndarray:
        bits = np.ascontiguousarray(bits)
        out = np.empty(bits.size, dtype=np.float64)
        if self.lib.oracle_decode_all(_ptr(bits), bits.size, CODES[dtype], _ptr(out)):
            raise ValueError(dtype)
        return out

    def sum_segmented(self, bits: np.ndarray, offsets: np.ndarray, dtype: str) -> np.ndarray:
        bits = np.ascontiguousarray(bits)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        nseg = offsets.size - 1
        out = np.empty(nseg, dtype=np.int64 if dtype in INTS else np.float64)
        if self.lib.oracle_sum_segmented(_ptr(bits), _ptr(offsets), nseg, CODES[dtype], _ptr(out)):
            raise ValueError("oracle_sum_segmented: bad offsets")
        return out

    def scan(self, bits: np.ndarray, dtype: str, exclusive: bool = False) -> np.ndarray:
        """Inclusive (or exclusive) prefix sums: int64 for integer formats,
        float64 for float formats."""
        bits = np.ascontiguousarray(bits)
        n = bits.size
        if dtype in ("i32", "i64"):
            out = np.empty(n, dtype=np.int64)
            rc = self.lib.oracle_scan_int(_ptr(bits), n, CODES[dtype], int(exclusive), _ptr(out))
        else:
            out = np.empty(n, dtype=np.float64)
            rc = self.lib.oracle_scan_float(_ptr(bits), n, CODES[dtype], int(exclusive), _ptr(out))
        if rc:
            raise ValueError(f"oracle scan: dtype {dtype}")
        return out

    def histogram_int(self, bits: np.ndarray, dtype: str, lo: int, width: int,
                      nbins: int) -> np.ndarray:
        bits = np.ascontiguousarray(bits)
        out = np.empty(nbins, dtype=np.int64)
        if self.lib.oracle_histogram_int(_ptr(bits), bits.size, HCODES[dtype], lo, width, nbins,
                                         _ptr(out)):
            raise ValueError("oracle_histogram_int: bad arguments")
        return out

    def histogram_float(self, bits: np.ndarray, dtype: str, lo: float, hi: float,
                        nbins: int) -> np.ndarray:
        bits = np.ascontiguousarray(bits)
        out = np.empty(nbins, dtype=np.int64)
        if self.lib.oracle_histogram_float(_ptr(bits), bits.size, CODES[dtype], lo, hi, nbins,
                                           _ptr(out)):
            raise ValueError("oracle_histogram_float: bad arguments")
        return out

    # ------------------------------------------------------------ matmul
    def matmul(self, a: np.ndarray, b: np.ndarray, dtype: str, trans_b: bool = False,
               M=None, N=None, K=None, lda=None, ldb=None) -> np.ndarray:
        """fp64 C = A @ B (or A @ B^T with trans_b, B given as N x K) over the
        raw-bit 2-D arrays a and b of format dtype."""
        a = np.ascontiguousarray(a)
        b = np.ascontiguousarray(b)
        M = a.shape[0] if M is None else M
        K = a.shape[1] if K is None else K
        N = (b.shape[0] if trans_b else b.shape[1]) if N is None else N
        lda = a.shape[1] if lda is None else lda
        ldb = b.shape[1] if ldb is None else ldb
        out = np.empty((M, N), dtype=np.float64)
        if self.lib.oracle_matmul(_ptr(a), _ptr(b), _ptr(out), M, N, K, lda, ldb, N,
                                  int(bool(trans_b)), CODES[dtype]):
            raise ValueError("oracle_matmul: bad arguments")
        return out

    def matmul_entries(self, a: np.ndarray, b: np.ndarray, dtype: str, rows, cols,
                       trans_b: bool = False, M=None, N=None, K=None, lda=None,
                       ldb=None) -> np.ndarray:
        """The entries C[rows[t]][cols[t]] of the product above."""
        a = np.ascontiguousarray(a)
        b = np.ascontiguousarray(b)
        M = a.shape[0] if M is None else M
        K = a.shape[1] if K is None else K
        N = (b.shape[0] if trans_b else b.shape[1]) if N is None else N
        lda = a.shape[1] if lda is None else lda
        ldb = b.shape[1] if ldb is None else ldb
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(rows.size, dtype=np.float64)
        if self.lib.oracle_matmul_entries(_ptr(a), _ptr(b), M, N, K, lda, ldb,
                                          int(bool(trans_b)), CODES[dtype], rows.size,
                                          _ptr(rows), _ptr(cols), _ptr(out)):
            raise ValueError("oracle_matmul_entries: bad arguments")
        return out


class OmpBaseline:
    """The plain loops of the oracle on every host core (OpenMP, the
    tile-partials-then-serial-combine pattern of Listing 2.2): the benchmark's
    all-cores CPU baseline.  Transposes and integer sums equal the oracle bit
    for bit; float sums are associated per tile of 128 elements."""

    def __init__(self, path: str = OMP_LIB):
        if path == OMP_LIB and _stale(OMP_LIB, OMP_SRC):
            build_omp()
        lib = C.CDLL(path)
        i64, vp = C.c_int64, C.c_void_p
        lib.omp_threads.argtypes = []
        lib.omp_threads.restype = C.c_int
        lib.omp_tpose.argtypes = [vp, vp, i64, i64, i64, i64, C.c_int]
        lib.omp_tpose.restype = C.c_int
        lib.omp_sum_int.argtypes = [vp, i64, C.c_int]
        lib.omp_sum_int.restype = C.c_int64
        lib.omp_sum_float.argtypes = [vp, i64, C.c_int]
        lib.omp_sum_float.restype = C.c_double
        self.lib = lib

    def threads(self) -> int:
        return int(self.lib.omp_threads())

    def tpose(self, src: np.ndarray) -> np.ndarray:
        src = np.ascontiguousarray(src)
        rows, cols = src.shape
        dst = np.empty((cols, rows), dtype=src.dtype)
        if self.lib.omp_tpose(_ptr(src), _ptr(dst), rows, cols, cols, rows, src.itemsize):
            raise ValueError("omp_tpose: invalid arguments")
        return dst

    def sum_int(self, bits: np.ndarray, dtype: str) -> int:
        bits = np.ascontiguousarray(bits)
        return int(self.lib.omp_sum_int(_ptr(bits), bits.size, CODES[dtype]))

    def sum_float(self, bits: np.ndarray, dtype: str) -> float:
        bits = np.ascontiguousarray(bits)
        return float(self.lib.omp_sum_float(_ptr(bits), bits.size, CODES[dtype]))


_default: Oracle | None = None
_omp: OmpBaseline | None = None


def omp() -> OmpBaseline:
    global _omp
    if _omp is None:
        _omp = OmpBaseline()
    return _omp


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def __getattr__(name):  # module-level convenience: oracle.tpose(...), oracle.sum(...)
    if name in ("tpose", "tpose_batched", "sum_int", "sum_float", "sum", "sum_abs",
                "sum_plain_f32", "decode", "sum_segmented", "scan", "histogram_int",
                "histogram_float", "matmul", "matmul_entries"):
        return getattr(get(), name)
    raise AttributeError(name)


if __name__ == "__main__":
    build()
    build_omp()
    print(LIB, OMP_LIB, file=sys.stderr)
