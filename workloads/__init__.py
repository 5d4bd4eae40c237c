"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and stores them in the element formats
the library works on (fp32, bf16, fp16, fp8-e4m3fn, int32, int64).  It holds
none of the transpose or summation arithmetic: the oracle and the HIP path
each do their own.

Every array is a flat or 2-D numpy array of raw element bits (bf16 and fp16
as ``uint16``, fp8 as ``uint8``), plus the dtype name, so that both sides read
exactly the same bytes.

Draws are made block by block: block ``k`` of a stream with seed ``s`` uses
``numpy.random.Generator(PCG64(SeedSequence([s, k])))``, so large inputs can be
drawn in parallel and any block can be redrawn on its own.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

BLOCK = 1 << 22  # elements per independently seeded block

# dtype name -> (element bytes, numpy storage dtype)
DTYPES = {
    "f32": (4, np.float32),
    "f16": (2, np.uint16),
    "bf16": (2, np.uint16),
    "f8e4m3": (1, np.uint8),
    "i32": (4, np.int32),
    "i64": (8, np.int64),
    "f64": (8, np.float64),
    "u8": (1, np.uint8),
    "u16": (2, np.uint16),
}

# Largest finite value of each storable float format (format definitions).
MAX_FINITE = {"f16": 65504.0, "bf16": 3.3895313892515355e38, "f8e4m3": 448.0,
              "f32": 3.4028234663852886e38}


def _rng(seed: int, block: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, block])))


def _blocked(n: int, seed: int, fill, out: np.ndarray, threads: int | None = None):
    """Fill ``out[:n]`` block by block; ``fill(rng, lo, hi)`` writes out[lo:hi]."""
    nblk = (n + BLOCK - 1) // BLOCK
    if nblk <= 1:
        if n:
            fill(_rng(seed, 0), 0, n)
        return out
    threads = threads or min(16, os.cpu_count() or 1)

    def one(k):
        lo = k * BLOCK
        fill(_rng(seed, k), lo, min(n, lo + BLOCK))

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, range(nblk)))
    return out


# ---------------------------------------------------------------- casts
# Round-to-nearest-even casts from float64/float32 to the 16- and 8-bit
# storage formats go through torch's CPU casts (an independent library),
# imported lazily so that numpy-only users of this module do not need torch.

def to_bits(x: np.ndarray, dtype: str) -> np.ndarray:
    """Store float values ``x`` in format ``dtype`` (RNE) and return raw bits."""
    if dtype == "f32":
        return x.astype(np.float32)
    if dtype == "f64":
        return x.astype(np.float64)
    if dtype == "f16":
        return x.astype(np.float16).view(np.uint16)
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
    if dtype == "bf16":
        return t.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    if dtype == "f8e4m3":
        return t.to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    raise ValueError(dtype)


# ---------------------------------------------------------------- generators

def uniform(n: int, seed: int, dtype: str = "f32", lo: float = -1.0, hi: float = 1.0):
    """``n`` values U[lo, hi) stored as ``dtype`` (float formats only)."""
    eb, sd = DTYPES[dtype]
    out = np.empty(n, dtype=sd)

    def fill(rng, a, b):
        out[a:b] = to_bits(rng.uniform(lo, hi, b - a), dtype)

    return _blocked(n, seed, fill, out)


def normal(n: int, seed: int, dtype: str = "f32"):
    """``n`` values N(0, 1) stored as ``dtype``."""
    eb, sd = DTYPES[dtype]
    out = np.empty(n, dtype=sd)

    def fill(rng, a, b):
        out[a:b] = to_bits(rng.standard_normal(b - a), dtype)

    return _blocked(n, seed, fill, out)


def integers(n: int, seed: int, lo: int, hi: int, dtype: str = "i32"):
    """``n`` integers uniform in the closed range [lo, hi]."""
    eb, sd = DTYPES[dtype]
    out = np.empty(n, dtype=sd)

    def fill(rng, a, b):
        out[a:b] = rng.integers(lo, hi, b - a, dtype=np.int64, endpoint=True).astype(sd)

    return _blocked(n, seed, fill, out)


def signed_lognormal(n: int, seed: int, dtype: str, sigma: float = 2.0):
    """``n`` values ``sign * exp(sigma * Z)`` with a fair random sign, scaled per
    tensor so that the largest magnitude lands on the format's largest finite
    value when it would otherwise overflow (scale ``s = min(1, max_finite / max|x|)``),
    then stored as ``dtype`` with RNE.  Returns ``(bits, s)``; the stored values
    are what gets summed, ``s`` is not undone."""
    eb, sd = DTYPES[dtype]
    raw = np.empty(n, dtype=np.float64)

    def fill(rng, a, b):
        z = rng.standard_normal(b - a)
        sign = np.where(rng.integers(0, 2, b - a) == 0, -1.0, 1.0)
        raw[a:b] = sign * np.exp(sigma * z)

    _blocked(n, seed, fill, raw)
    m = float(np.max(np.abs(raw))) if n else 1.0
    s = min(1.0, MAX_FINITE[dtype] / m) if m > 0 else 1.0
    out = np.empty(n, dtype=sd)

    def store(rng, a, b):  # rng unused: deterministic scaling, blocked for speed
        out[a:b] = to_bits(raw[a:b] * s, dtype)

    _blocked(n, seed, store, out)
    return out, s


def matrix(rows: int, cols: int, seed: int, dtype: str = "f32"):
    """A row-major ``rows x cols`` matrix of U[-1, 1) values stored as ``dtype``;
    integer and raw-bit formats get uniformly random bit patterns instead."""
    n = rows * cols
    if dtype in ("f32", "f16", "bf16", "f8e4m3", "f64"):
        flat = uniform(n, seed, dtype)
    else:
        eb, sd = DTYPES[dtype]
        flat = np.empty(n, dtype=sd)
        info = np.iinfo(sd)

        def fill(rng, a, b):
            flat[a:b] = rng.integers(info.min, info.max, b - a, dtype=sd, endpoint=True)

        _blocked(n, seed, fill, flat)
    return flat.reshape(rows, cols)


def random_bits(n: int, seed: int, elem_bytes: int) -> np.ndarray:
    """``n`` elements of uniformly random bits of width ``elem_bytes``
    (covers NaN payloads, signed zeros and subnormals of every float format)."""
    sd = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[elem_bytes]
    out = np.empty(n, dtype=sd)

    def fill(rng, a, b):
        out[a:b] = rng.integers(0, np.iinfo(sd).max, b - a, dtype=sd, endpoint=True)

    return _blocked(n, seed, fill, out)


# ---------------------------------------------------------------- batched / segmented

def batched_shapes(count: int, seed: int, lo: int = 16, hi: int = 2048):
    """``count`` (rows, cols) pairs, each side iid uniform in [lo, hi]."""
    rng = _rng(seed, 0)
    rc = rng.integers(lo, hi, (count, 2), dtype=np.int64, endpoint=True)
    return [(int(r), int(c)) for r, c in rc]


def segment_offsets(total: int, nseg: int, seed: int, mu: float = 6.0, sigma: float = 1.5):
    """CSR offsets (int64, length nseg+1) of ``nseg`` segments whose lengths are
    lognormal(mu, sigma) draws scaled to sum exactly to ``total`` by
    largest-remainder rounding (empty segments allowed)."""
    rng = _rng(seed, 0)
    w = rng.lognormal(mu, sigma, nseg)
    q = w * (total / w.sum())
    base = np.floor(q).astype(np.int64)
    short = int(total - base.sum())
    if short:
        order = np.argsort(-(q - base), kind="stable")
        base[order[:short]] += 1
    off = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(base, out=off[1:])
    assert off[-1] == total
    return off


# ---------------------------------------------------------------- serving

@dataclass
class Job:
    arrival_s: float   # arrival time since the start of the stream
    kind: str          # "tpose" or "sum"
    dtype: str
    rows: int = 0      # tpose: square side
    cols: int = 0
    n: int = 0         # sum: element count

    @property
    def nbytes(self) -> int:
        eb = DTYPES[self.dtype][0]
        return 2 * self.rows * self.cols * eb if self.kind == "tpose" else self.n * eb


def serving_jobs(count: int, seed: int, rate: float = 20000.0, p_tpose: float = 0.6,
                 tpose_k=(5, 13), sum_k=(10, 26)):
    """A Poisson stream of ``count`` mixed jobs: with probability ``p_tpose`` a
    square transpose of side 2^k, k uniform in ``tpose_k``, bf16 or fp32 with
    equal odds; otherwise a sum of 2^k elements, k uniform in ``sum_k``, fp32
    or int32 with equal odds."""
    rng = _rng(seed, 0)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    kinds = rng.random(count) < p_tpose
    pick = rng.integers(0, 2, count)
    ktp = rng.integers(tpose_k[0], tpose_k[1], count, endpoint=True)
    ksm = rng.integers(sum_k[0], sum_k[1], count, endpoint=True)
    jobs = []
    for i in range(count):
        if kinds[i]:
            side = 1 << int(ktp[i])
            jobs.append(Job(float(t[i]), "tpose", "bf16" if pick[i] == 0 else "f32", side, side))
        else:
            jobs.append(Job(float(t[i]), "sum", "f32" if pick[i] == 0 else "i32", n=1 << int(ksm[i])))
    return jobs


def mean_job_bytes(p_tpose=0.6, tpose_k=(5, 13), sum_k=(10, 26)) -> float:
    """Expected algorithmic bytes of one serving job (closed form)."""
    kt = range(tpose_k[0], tpose_k[1] + 1)
    ks = range(sum_k[0], sum_k[1] + 1)
    tp = sum(2 * 4 ** k * 3.0 for k in kt) / len(kt)      # mean over bf16 (2 B) and fp32 (4 B)
    sm = sum(2 ** k * 4.0 for k in ks) / len(ks)          # fp32 and int32 are both 4 B
    return p_tpose * tp + (1 - p_tpose) * sm


__all__ = ["DTYPES", "MAX_FINITE", "BLOCK", "to_bits", "uniform", "normal", "integers",
           "signed_lognormal", "matrix", "random_bits", "batched_shapes", "segment_offsets",
           "Job", "serving_jobs", "mean_job_bytes"]
