"""xtr: out-of-place transpose and compensated sum reduction for MI355X (gfx950).

Thin Python binding over the C ABI of ``libxtr.so`` (declared in
``include/xtr.h``).  Every function here only marshals arguments -- tensor
data pointers, sizes, the current HIP stream -- and calls the library; all
work runs in the library's HIP kernels.  There is no fallback: if the library
is missing or fails to load, ``load()`` raises.

Tensors are torch tensors on the GPU.  Element formats are given by name
("f32", "f16", "bf16", "f8e4m3", "i32", "i64", "f64", "u8", "u16") or taken
from the tensor's dtype; raw-bit tensors (e.g. uint16 holding bf16 bits) pass
``dtype=`` explicitly.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxtr.so")

CODES = {"f32": 0, "f16": 1, "bf16": 2, "f8e4m3": 3, "i32": 4, "i64": 5, "f64": 6,
         "u8": 7, "u16": 8}
ELEM_BYTES = {"f32": 4, "f16": 2, "bf16": 2, "f8e4m3": 1, "i32": 4, "i64": 8, "f64": 8,
              "u8": 1, "u16": 2}
FLOAT_SUM = ("f32", "f16", "bf16", "f8e4m3")
INT_SUM = ("i32", "i64")
ERRORS = {0: "XTR_OK", -1: "XTR_EINVAL", -2: "XTR_EDTYPE", -3: "XTR_EOVERLAP",
          -4: "XTR_EALIGN", -5: "XTR_EHIP", -6: "XTR_ENOMEM", -7: "XTR_EBUDGET"}


class XtrError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__(f"{fn} -> {ERRORS.get(code, code)}: {msg}")
        self.code = code


class TposeConfig(C.Structure):
    _fields_ = [("nt_load", C.c_int32), ("nt_store", C.c_int32), ("xcd", C.c_int32),
                ("group", C.c_int32), ("blocks_per_cu", C.c_int32), ("nt_store_shared", C.c_int32),
                ("nt_load_shared", C.c_int32), ("tile", C.c_int32), ("tile_shared", C.c_int32),
                ("run", C.c_int32), ("narrow", C.c_int32), ("wide_min", C.c_int32)]


class ReduceConfig(C.Structure):
    _fields_ = [("nt_load", C.c_int32), ("split_chunks", C.c_int32), ("seg_fused", C.c_int32),
                ("seg_streams", C.c_int32), ("seg_small_per_cu", C.c_int32),
                ("seg_chunk_per_cu", C.c_int32), ("seg_over", C.c_int32),
                ("_reserved", C.c_int32 * 1)]


class Job(C.Structure):
    _fields_ = [("kind", C.c_int32), ("dtype", C.c_int32), ("src", C.c_void_p),
                ("dst", C.c_void_p), ("rows", C.c_int64), ("cols", C.c_int64), ("n", C.c_int64),
                ("arrival_ns", C.c_int64), ("host_src", C.c_void_p)]


class ServerConfig(C.Structure):
    _fields_ = [("nstreams", C.c_int32), ("batching", C.c_int32), ("budget_bytes", C.c_int64),
                ("small_job_bytes", C.c_int64), ("graphs", C.c_int32), ("big_lane", C.c_int32),
                ("_reserved", C.c_int64 * 3)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("launches", C.c_int64), ("units", C.c_int64), ("max_inflight_bytes", C.c_int64),
                ("graph_launches", C.c_int64), ("graph_builds", C.c_int64),
                ("host_copies", C.c_int64), ("_reserved", C.c_int64)]


class TposeDesc(C.Structure):
    _fields_ = [("src", C.c_void_p), ("dst", C.c_void_p), ("rows", C.c_int64),
                ("cols", C.c_int64), ("ld_src", C.c_int64), ("ld_dst", C.c_int64),
                ("dtype", C.c_int32), ("_pad", C.c_int32)]


_lib = None

# C signatures of every entry point in include/xtr.h
_SIGS = {
    "tpose": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int,
               C.c_void_p], C.c_int),
    "reduce_sum": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "reduce_sum_plain_f32": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "xtr_reduce_workspace_bytes": ([C.c_int64, C.c_int], C.c_size_t),
    "reduce_sum_ws": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t,
                       C.c_void_p], C.c_int),
    "reduce_sum_noalloc": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "tpose_batched": ([C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "reduce_sum_segmented": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int,
                              C.c_void_p], C.c_int),
    "xtr_segmented_workspace_bytes": ([C.c_int64, C.c_int64, C.c_int], C.c_size_t),
    "reduce_sum_segmented_ws": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int,
                                 C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "reduce_sum_segmented_ws_total": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                       C.c_int, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "xtr_scan_lookback_bound": ([C.c_uint32], C.c_uint32),
    "reduce_sum_batched": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int,
                            C.c_void_p], C.c_int),
    "reduce_sum_batched_scatter": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                    C.c_void_p], C.c_int),
    "xtr_copy": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p], C.c_int),
    "xtr_tpose_host": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                        C.c_int], C.c_int),
    "xtr_reduce_sum_host": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_int], C.c_int),
    "scan_sum": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "histogram_int": ([C.c_void_p, C.c_int64, C.c_int, C.c_int64, C.c_int64, C.c_int64,
                       C.c_void_p, C.c_void_p], C.c_int),
    "histogram_float": ([C.c_void_p, C.c_int64, C.c_int, C.c_double, C.c_double, C.c_int64,
                         C.c_void_p, C.c_void_p], C.c_int),
    "matmul": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_void_p], C.c_int),
    "xtr_tpose_plan_create": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "xtr_tpose_plan_run": ([C.c_void_p, C.c_void_p], C.c_int),
    "xtr_tpose_plan_destroy": ([C.c_void_p], C.c_int),
    "xtr_sum_plan_create": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p,
                             C.c_void_p], C.c_int),
    "xtr_sum_plan_run": ([C.c_void_p, C.c_void_p], C.c_int),
    "xtr_sum_plan_destroy": ([C.c_void_p], C.c_int),
    "xtr_tpose_get_class_config": ([C.c_int, C.c_int, C.c_void_p], C.c_int),
    "xtr_tpose_set_class_config": ([C.c_int, C.c_int, C.c_void_p], C.c_int),
    "xtr_reduce_get_class_config": ([C.c_int, C.c_int, C.c_void_p], C.c_int),
    "xtr_reduce_set_class_config": ([C.c_int, C.c_int, C.c_void_p], C.c_int),
    "xtr_tpose_get_config": ([C.c_int, C.c_void_p], C.c_int),
    "xtr_tpose_set_config": ([C.c_int, C.c_void_p], C.c_int),
    "xtr_reduce_get_config": ([C.c_int, C.c_void_p], C.c_int),
    "xtr_reduce_set_config": ([C.c_int, C.c_void_p], C.c_int),
    "xtr_server_clock_ns": ([], C.c_int64),
    "xtr_server_create": ([C.c_void_p, C.c_void_p], C.c_int),
    "xtr_server_submit": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "xtr_server_drain": ([C.c_void_p, C.c_int64], C.c_int),
    "xtr_server_times": ([C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "xtr_server_get_stats": ([C.c_void_p, C.c_void_p], C.c_int),
    "xtr_server_destroy": ([C.c_void_p], C.c_int),
    "xtr_last_error": ([], C.c_char_p),
    "xtr_elem_bytes": ([C.c_int], C.c_int),
    "xtr_version": ([], C.c_int),
    "xtr_release": ([], C.c_int),
}


def load(path: str = LIB_PATH):
    """Load libxtr.so (once).  torch is imported first so that the process has a
    single HIP runtime: torch's, which the library then binds to."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (must precede the library: one HIP runtime per process)
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          f"`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    if os.environ.get("XTR_NO_TUNED") != "1" and torch.cuda.is_available():
        # launch settings measured by the autotuner (scheduling only, never results)
        from . import tune
        arch = tune.arch_name(torch)
        tune.load_tuned(__import__(__name__), os.path.join(tune.TUNED_DIR, f"{arch}.json"))
    return lib


def _check(rc: int, fn: str):
    if rc != 0:
        raise XtrError(rc, fn, (_lib.xtr_last_error() or b"").decode())


def _code(dtype) -> int:
    if isinstance(dtype, int):
        return dtype
    return CODES[dtype]


def dtype_of(t) -> str:
    import torch
    if not isinstance(t, torch.Tensor):   # numpy array
        m = {"float32": "f32", "float16": "f16", "int32": "i32", "int64": "i64",
             "float64": "f64", "uint8": "u8", "uint16": "u16", "int16": "u16", "int8": "u8"}
        if str(t.dtype) not in m:
            raise TypeError(f"unsupported array dtype {t.dtype}; pass dtype=")
        return m[str(t.dtype)]
    m = {torch.float32: "f32", torch.float16: "f16", torch.bfloat16: "bf16",
         torch.float8_e4m3fn: "f8e4m3", torch.int32: "i32", torch.int64: "i64",
         torch.float64: "f64", torch.uint8: "u8", torch.uint16: "u16", torch.int16: "u16",
         torch.int8: "u8"}
    if t.dtype not in m:
        raise TypeError(f"unsupported tensor dtype {t.dtype}")
    return m[t.dtype]


def _stream(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


# ---------------------------------------------------------------- transpose

def tpose(src, out=None, *, rows=None, cols=None, ld_src=None, ld_dst=None, dtype=None,
          stream=None):
    """out[c, r] = src[r, c].  ``src`` is a 2-D tensor (any row stride with unit
    column stride) or a flat buffer with explicit rows/cols/ld_src; ``out``
    defaults to a new contiguous (cols, rows) tensor."""
    import torch
    lib = load()
    dt = dtype or dtype_of(src)
    if rows is None:
        assert src.dim() == 2 and (src.stride(1) == 1 or src.shape[1] <= 1)
        rows, cols = src.shape
        ld_src = src.stride(0) if rows > 1 else max(cols, 1)
    if ld_src is None:
        ld_src = cols
    if out is None:
        out = torch.empty((cols, rows), dtype=src.dtype, device=src.device)
    if ld_dst is None:
        if out.dim() == 2:
            assert out.stride(1) == 1 or out.shape[1] <= 1
            ld_dst = out.stride(0) if out.shape[0] > 1 else max(rows, 1)
        else:
            ld_dst = rows
    rc = lib.tpose(C.c_void_p(src.data_ptr()), C.c_void_p(out.data_ptr()), rows, cols, ld_src,
                   ld_dst, _code(dt), _stream(stream))
    _check(rc, "tpose")
    return out


def _tpose_descs(jobs):
    arr = (TposeDesc * len(jobs))()
    for i, j in enumerate(jobs):
        if isinstance(j, dict):
            s, d = j["src"], j["dst"]
            rows, cols = j["rows"], j["cols"]
            lds, ldd = j.get("ld_src", cols), j.get("ld_dst", rows)
            dt = j.get("dtype") or dtype_of(s)
        else:
            s, d = j
            rows, cols = s.shape
            lds = s.stride(0) if rows > 1 else max(cols, 1)
            ldd = d.stride(0) if d.shape[0] > 1 else max(rows, 1)
            dt = dtype_of(s)
        arr[i] = TposeDesc(s.data_ptr(), d.data_ptr(), rows, cols, lds, ldd, _code(dt), 0)
    return arr


def tpose_batched(jobs, *, stream=None):
    """jobs: list of (src, dst) 2-D tensor pairs, or of dicts with keys
    src, dst, rows, cols, ld_src, ld_dst, dtype (as tpose)."""
    lib = load()
    arr = _tpose_descs(jobs)
    rc = lib.tpose_batched(C.cast(arr, C.c_void_p), len(jobs), _stream(stream))
    _check(rc, "tpose_batched")


class TposePlan:
    """A validated, uploaded batch of transposes; run() only launches kernels
    (capturable in a graph).  Keep the tensors alive while the plan lives."""

    def __init__(self, jobs, *, stream=None):
        lib = load()
        self._jobs = jobs
        arr = _tpose_descs(jobs)
        h = C.c_void_p()
        _check(lib.xtr_tpose_plan_create(C.cast(arr, C.c_void_p), len(jobs), _stream(stream),
                                         C.byref(h)), "xtr_tpose_plan_create")
        self._h = h

    def run(self, *, stream=None):
        _check(_lib.xtr_tpose_plan_run(self._h, _stream(stream)), "xtr_tpose_plan_run")

    def close(self):
        if self._h:
            _lib.xtr_tpose_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SumPlan:
    """A validated batch of sums with its own workspace; run() launches one
    kernel (capturable).  Keep the tensors alive while the plan lives."""

    def __init__(self, srcs, out=None, *, ns=None, dtype=None, stream=None):
        lib = load()
        count = len(srcs)
        dt = dtype or (dtype_of(srcs[0]) if count else "f32")
        if out is None:
            out = _sum_out(dt, srcs[0].device if count else "cuda", count)
        self.out = out
        self._srcs = srcs
        ptrs = (C.c_void_p * count)(*[s.data_ptr() for s in srcs])
        lens = (C.c_int64 * count)(*[(s.numel() if ns is None else ns[i])
                                     for i, s in enumerate(srcs)])
        h = C.c_void_p()
        _check(lib.xtr_sum_plan_create(C.cast(ptrs, C.c_void_p), C.cast(lens, C.c_void_p), count,
                                       _code(dt), C.c_void_p(out.data_ptr()), _stream(stream),
                                       C.byref(h)), "xtr_sum_plan_create")
        self._h = h

    def run(self, *, stream=None):
        _check(_lib.xtr_sum_plan_run(self._h, _stream(stream)), "xtr_sum_plan_run")
        return self.out

    def close(self):
        if self._h:
            _lib.xtr_sum_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- sums

def _sum_out(dt, device, count=None):
    import torch
    shape = () if count is None else (count,)
    if dt in INT_SUM:
        return torch.empty(shape, dtype=torch.int64, device=device)
    return torch.empty(shape, dtype=torch.float64, device=device)


def reduce_sum(src, out=None, *, n=None, dtype=None, stream=None):
    """Sum of the elements of a contiguous tensor: a 0-d float64 tensor for
    float formats, int64 for int32/int64."""
    lib = load()
    dt = dtype or dtype_of(src)
    n = src.numel() if n is None else n
    if out is None:
        out = _sum_out(dt, src.device)
    rc = lib.reduce_sum(C.c_void_p(src.data_ptr()), n, C.c_void_p(out.data_ptr()), _code(dt),
                        _stream(stream))
    _check(rc, "reduce_sum")
    return out


def reduce_sum_plain_f32(src, out=None, *, n=None, dtype=None, stream=None):
    """Uncompensated fp32 comparator: a 0-d float32 tensor."""
    import torch
    lib = load()
    dt = dtype or dtype_of(src)
    n = src.numel() if n is None else n
    if out is None:
        out = torch.empty((), dtype=torch.float32, device=src.device)
    rc = lib.reduce_sum_plain_f32(C.c_void_p(src.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                  _code(dt), _stream(stream))
    _check(rc, "reduce_sum_plain_f32")
    return out


def reduce_workspace_bytes(n: int, dtype) -> int:
    return int(load().xtr_reduce_workspace_bytes(n, _code(dtype)))


def reduce_sum_ws(src, ws, out=None, *, n=None, dtype=None, stream=None):
    """reduce_sum with a caller-owned zero-initialised device workspace tensor."""
    lib = load()
    dt = dtype or dtype_of(src)
    n = src.numel() if n is None else n
    if out is None:
        out = _sum_out(dt, src.device)
    rc = lib.reduce_sum_ws(C.c_void_p(src.data_ptr()), n, C.c_void_p(out.data_ptr()), _code(dt),
                           C.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                           _stream(stream))
    _check(rc, "reduce_sum_ws")
    return out


def reduce_sum_segmented(src, offsets, out=None, *, dtype=None, stream=None):
    """Per-segment sums; ``offsets`` is a device int64 tensor of nseg+1 entries."""
    lib = load()
    dt = dtype or dtype_of(src)
    nseg = offsets.numel() - 1
    if out is None:
        out = _sum_out(dt, src.device, nseg)
    rc = lib.reduce_sum_segmented(C.c_void_p(src.data_ptr()), C.c_void_p(offsets.data_ptr()),
                                  nseg, C.c_void_p(out.data_ptr()), _code(dt), _stream(stream))
    _check(rc, "reduce_sum_segmented")
    return out


def segmented_workspace_bytes(nseg: int, total: int, dtype) -> int:
    return int(load().xtr_segmented_workspace_bytes(nseg, total, _code(dtype)))


def reduce_sum_segmented_ws(src, offsets, ws, out=None, *, total=None, dtype=None,
                            stream=None):
    """Segmented sums with a caller-owned zero-initialised workspace, fully
    asynchronous.  Without ``total`` the chunk space is what the workspace
    holds (reduce_sum_segmented_ws); with it, it is sized from the element
    total (reduce_sum_segmented_ws_total)."""
    lib = load()
    dt = dtype or dtype_of(src)
    nseg = offsets.numel() - 1
    if out is None:
        out = _sum_out(dt, src.device, nseg)
    wsb = ws.numel() * ws.element_size()
    if total is None:
        rc = lib.reduce_sum_segmented_ws(C.c_void_p(src.data_ptr()),
                                         C.c_void_p(offsets.data_ptr()), nseg,
                                         C.c_void_p(out.data_ptr()), _code(dt),
                                         C.c_void_p(ws.data_ptr()), wsb, _stream(stream))
        _check(rc, "reduce_sum_segmented_ws")
    else:
        rc = lib.reduce_sum_segmented_ws_total(C.c_void_p(src.data_ptr()),
                                               C.c_void_p(offsets.data_ptr()), nseg, total,
                                               C.c_void_p(out.data_ptr()), _code(dt),
                                               C.c_void_p(ws.data_ptr()), wsb, _stream(stream))
        _check(rc, "reduce_sum_segmented_ws_total")
    return out


class Server:
    """The native request loop (xtr_server_*): submit jobs on device-resident
    tensors, drain, read arrival / completion times (ns, server clock)."""

    def __init__(self, *, nstreams=4, batching=True, budget=64 << 30, small_job_bytes=4 << 20,
                 graphs=False, big_lane=False):
        lib = load()
        cfg = ServerConfig(nstreams, int(bool(batching)), int(budget), int(small_job_bytes),
                           int(bool(graphs)), int(bool(big_lane)))
        h = C.c_void_p()
        _check(lib.xtr_server_create(C.byref(cfg), C.byref(h)), "xtr_server_create")
        self._h = h
        self.count = 0

    @staticmethod
    def clock_ns() -> int:
        return int(load().xtr_server_clock_ns())

    def submit(self, jobs) -> int:
        """jobs: a ctypes array of Job (or a list of Job); returns the first id."""
        if not isinstance(jobs, C.Array):
            arr = (Job * len(jobs))(*jobs)
        else:
            arr = jobs
        first = C.c_int64(0)
        _check(_lib.xtr_server_submit(self._h, C.cast(arr, C.c_void_p), len(arr), C.byref(first)),
               "xtr_server_submit")
        self.count += len(arr)
        return first.value

    def drain(self, timeout_ms: int = -1):
        _check(_lib.xtr_server_drain(self._h, int(timeout_ms)), "xtr_server_drain")

    def times(self, first: int = 0, count: int | None = None):
        import numpy as np
        count = self.count - first if count is None else count
        arr = np.empty(count, dtype=np.int64)
        done = np.empty(count, dtype=np.int64)
        _check(_lib.xtr_server_times(self._h, first, count, arr.ctypes.data_as(C.c_void_p),
                                     done.ctypes.data_as(C.c_void_p)), "xtr_server_times")
        return arr, done

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.xtr_server_get_stats(self._h, C.byref(st)), "xtr_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_ if k != "_reserved"}

    def close(self):
        if self._h:
            _lib.xtr_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scan_lookback_bound(polls: int) -> int:
    """Sets the bound on each look-back wait of the one-pass integer scan
    (results never depend on it); returns the previous bound."""
    return int(load().xtr_scan_lookback_bound(polls))


def reduce_sum_batched(srcs, out=None, *, ns=None, dtype=None, stream=None):
    """Sums of several independent contiguous tensors of one format."""
    lib = load()
    count = len(srcs)
    dt = dtype or (dtype_of(srcs[0]) if count else "f32")
    if out is None:
        import torch
        dev = srcs[0].device if count else torch.device("cuda")
        out = _sum_out(dt, dev, count)
    ptrs = (C.c_void_p * count)(*[s.data_ptr() for s in srcs])
    lens = (C.c_int64 * count)(*[(s.numel() if ns is None else ns[i]) for i, s in enumerate(srcs)])
    rc = lib.reduce_sum_batched(C.cast(ptrs, C.c_void_p), C.cast(lens, C.c_void_p), count,
                                C.c_void_p(out.data_ptr()), _code(dt), _stream(stream))
    _check(rc, "reduce_sum_batched")
    return out


def copy(dst, src, nbytes=None, *, stream=None):
    """Plain device copy of nbytes (default: all of src) -- the bandwidth reference."""
    nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
    rc = load().xtr_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes,
                         _stream(stream))
    _check(rc, "xtr_copy")
    return dst


SHAPE_CLASSES = {"single": 0, "batched": 1}


def tpose_config(elem_bytes: int, shape: str = "single") -> dict:
    """Launch settings of the transposes of one element size, for single
    calls or batched launches."""
    c = TposeConfig()
    _check(load().xtr_tpose_get_class_config(elem_bytes, SHAPE_CLASSES[shape], C.byref(c)),
           "xtr_tpose_get_class_config")
    return {"nt_load": c.nt_load, "nt_store": c.nt_store, "xcd": c.xcd, "group": c.group,
            "blocks_per_cu": c.blocks_per_cu, "nt_store_shared": c.nt_store_shared,
            "nt_load_shared": c.nt_load_shared, "tile": c.tile, "tile_shared": c.tile_shared,
            "run": c.run, "narrow": c.narrow, "wide_min": c.wide_min}


def set_tpose_config(elem_bytes: int, shape: str | None = None, **kw):
    """Change settings of one shape class ("single" / "batched"), or of every
    class (shape=None, starting from the single-call settings)."""
    cur = tpose_config(elem_bytes, shape or "single")
    bad = set(kw) - set(cur)
    if bad:
        raise TypeError(f"set_tpose_config: unknown settings {sorted(bad)}")
    cur.update(kw)
    c = TposeConfig(cur["nt_load"], cur["nt_store"], cur["xcd"], cur["group"],
                    cur["blocks_per_cu"], cur["nt_store_shared"], cur["nt_load_shared"],
                    cur["tile"], cur["tile_shared"], cur["run"], cur["narrow"],
                    cur["wide_min"])
    if shape is None:
        _check(load().xtr_tpose_set_config(elem_bytes, C.byref(c)), "xtr_tpose_set_config")
    else:
        _check(load().xtr_tpose_set_class_config(elem_bytes, SHAPE_CLASSES[shape], C.byref(c)),
               "xtr_tpose_set_class_config")


def reduce_config(dtype, shape: str = "single") -> dict:
    c = ReduceConfig()
    _check(load().xtr_reduce_get_class_config(_code(dtype), SHAPE_CLASSES[shape], C.byref(c)),
           "xtr_reduce_get_class_config")
    return {"nt_load": c.nt_load, "split_chunks": c.split_chunks, "seg_fused": c.seg_fused,
            "seg_streams": c.seg_streams, "seg_small_per_cu": c.seg_small_per_cu,
            "seg_chunk_per_cu": c.seg_chunk_per_cu, "seg_over": c.seg_over}


def set_reduce_config(dtype, shape: str | None = None, **kw):
    cur = reduce_config(dtype, shape or "single")
    bad = set(kw) - set(cur)
    if bad:
        raise TypeError(f"set_reduce_config: unknown settings {sorted(bad)}")
    cur.update(kw)
    c = ReduceConfig(cur["nt_load"], cur["split_chunks"], cur["seg_fused"], cur["seg_streams"],
                     cur["seg_small_per_cu"], cur["seg_chunk_per_cu"], cur["seg_over"])
    if shape is None:
        _check(load().xtr_reduce_set_config(_code(dtype), C.byref(c)), "xtr_reduce_set_config")
    else:
        _check(load().xtr_reduce_set_class_config(_code(dtype), SHAPE_CLASSES[shape], C.byref(c)),
               "xtr_reduce_set_class_config")


def reduce_sum_batched_scatter(srcs, outs, *, ns=None, dtype=None, stream=None):
    """Sums of several tensors, result i written to the 0-d tensor outs[i]."""
    lib = load()
    count = len(srcs)
    dt = dtype or (dtype_of(srcs[0]) if count else "f32")
    ptrs = (C.c_void_p * count)(*[s.data_ptr() for s in srcs])
    lens = (C.c_int64 * count)(*[(s.numel() if ns is None else ns[i]) for i, s in enumerate(srcs)])
    optr = (C.c_void_p * count)(*[o.data_ptr() for o in outs])
    rc = lib.reduce_sum_batched_scatter(C.cast(ptrs, C.c_void_p), C.cast(lens, C.c_void_p),
                                        C.cast(optr, C.c_void_p), count, _code(dt),
                                        _stream(stream))
    _check(rc, "reduce_sum_batched_scatter")


def scan_sum(src, out=None, *, n=None, dtype=None, exclusive=False, stream=None):
    """Prefix sums of a contiguous tensor: float64 output for float formats,
    int64 for int32/int64; exclusive=True shifts by one (out[0] = 0)."""
    import torch
    lib = load()
    dt = dtype or dtype_of(src)
    n = src.numel() if n is None else n
    if out is None:
        out = torch.empty(n, dtype=torch.float64 if dt in FLOAT_SUM else torch.int64,
                          device=src.device)
    rc = lib.scan_sum(C.c_void_p(src.data_ptr()), n, C.c_void_p(out.data_ptr()), _code(dt),
                      int(bool(exclusive)), _stream(stream))
    _check(rc, "scan_sum")
    return out


def _hist_dtype(src, dtype):
    import torch
    if dtype is None and src.dtype in (torch.int8, torch.int16):
        raise TypeError("int8/int16 tensors have no signed histogram format; pass dtype='u8' or "
                        "'u16' to count their raw bits as unsigned")
    return dtype or dtype_of(src)


def histogram_int(src, lo: int, width: int, nbins: int, counts=None, *, n=None, dtype=None,
                  stream=None):
    """Exact integer histogram: counts[b] = #{x : lo + b*width <= x < lo + (b+1)*width}
    over an int32 / int64 / uint8 / uint16 tensor; returns int64[nbins]."""
    import torch
    lib = load()
    dt = _hist_dtype(src, dtype)
    n = src.numel() if n is None else n
    if counts is None:
        counts = torch.empty(nbins, dtype=torch.int64, device=src.device)
    rc = lib.histogram_int(C.c_void_p(src.data_ptr()), n, _code(dt), int(lo), int(width),
                           int(nbins), C.c_void_p(counts.data_ptr()), _stream(stream))
    _check(rc, "histogram_int")
    return counts


def histogram_float(src, lo: float, hi: float, nbins: int, counts=None, *, n=None, dtype=None,
                    stream=None):
    """Histogram of a float tensor over [lo, hi) in nbins equal bins (bin
    floor((x - lo) * nbins / (hi - lo)) in fp64, capped at nbins - 1; NaN and
    values outside [lo, hi) are not counted); returns int64[nbins]."""
    import torch
    lib = load()
    dt = _hist_dtype(src, dtype)
    n = src.numel() if n is None else n
    if counts is None:
        counts = torch.empty(nbins, dtype=torch.int64, device=src.device)
    rc = lib.histogram_float(C.c_void_p(src.data_ptr()), n, _code(dt), float(lo), float(hi),
                             int(nbins), C.c_void_p(counts.data_ptr()), _stream(stream))
    _check(rc, "histogram_float")
    return counts


def matmul(a, b, c=None, *, trans_b=False, M=None, N=None, K=None, lda=None, ldb=None,
           ldc=None, dtype=None, stream=None):
    """C (float32, M x N) = A @ B on the matrix cores, for bf16 or fp16 2-D
    tensors A (M x K) and B (K x N; with trans_b, B given as N x K).  Strides
    come from the tensors (rows must be contiguous) unless given."""
    import torch
    lib = load()
    dt = dtype or dtype_of(a)
    M = a.shape[0] if M is None else M
    K = a.shape[1] if K is None else K
    N = (b.shape[0] if trans_b else b.shape[1]) if N is None else N
    if lda is None:
        assert a.stride(-1) == 1, "rows of A must be contiguous"
        lda = a.stride(0) if a.dim() == 2 else K
    if ldb is None:
        assert b.stride(-1) == 1, "rows of B must be contiguous"
        ldb = b.stride(0) if b.dim() == 2 else (K if trans_b else N)
    if c is None:
        c = torch.empty((M, N), dtype=torch.float32, device=a.device)
    if ldc is None:
        ldc = c.stride(0) if c.dim() == 2 else N
    rc = lib.matmul(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.c_void_p(c.data_ptr()),
                    M, N, K, lda, ldb, ldc, int(bool(trans_b)), _code(dt), _stream(stream))
    _check(rc, "matmul")
    return c


def _host_ptr(a):
    """Address of a host buffer: a CPU torch tensor or a numpy array."""
    if hasattr(a, "data_ptr"):
        assert not a.is_cuda, "host-buffer entry points take CPU tensors"
        return a.data_ptr()
    return a.ctypes.data


def tpose_host(src, dst, *, rows=None, cols=None, ld_src=None, ld_dst=None, dtype=None):
    """dst[c, r] = src[r, c] for host arrays (CPU tensors or numpy arrays, page-
    locked or not), through the GPU; returns when dst is written."""
    lib = load()
    dt = dtype or dtype_of(src)
    if rows is None:
        rows, cols = src.shape
    if ld_src is None:
        ld_src = cols
    if ld_dst is None:
        ld_dst = rows
    _check(lib.xtr_tpose_host(C.c_void_p(_host_ptr(src)), C.c_void_p(_host_ptr(dst)), rows, cols,
                              ld_src, ld_dst, _code(dt)), "xtr_tpose_host")
    return dst


def reduce_sum_host(src, *, n=None, dtype=None):
    """Sum of a host array (CPU tensor or numpy array) through the GPU: a Python
    float (float dtypes) or int (integer dtypes)."""
    lib = load()
    dt = dtype or dtype_of(src)
    if n is None:
        n = src.numel() if hasattr(src, "numel") else src.size
    res = C.c_double() if dt in FLOAT_SUM else C.c_int64()
    _check(lib.xtr_reduce_sum_host(C.c_void_p(_host_ptr(src)), n, C.byref(res), _code(dt)),
           "xtr_reduce_sum_host")
    return res.value


def release():
    _check(load().xtr_release(), "xtr_release")


def version() -> tuple:
    v = load().xtr_version()
    return (v >> 16, v & 0xffff)
