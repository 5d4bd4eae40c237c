"""Helpers for the GPU parity tests: moving raw-bit numpy arrays to and from
the device, and the float-sum acceptance rule."""
import math

import numpy as np

_SIGNED = {np.dtype(np.uint8): np.uint8, np.dtype(np.uint16): np.int16,
           np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}


def to_dev(a: np.ndarray, device="cuda"):
    """numpy array -> torch tensor on the device with the same bytes."""
    import torch
    a = np.ascontiguousarray(a)
    view = a.view(_SIGNED[a.dtype]) if a.dtype in _SIGNED else a
    return torch.from_numpy(view).to(device)


def to_host(t, like: np.dtype) -> np.ndarray:
    """torch tensor -> numpy array reinterpreted as dtype ``like``."""
    return t.detach().cpu().contiguous().numpy().view(like)


REL_TOL = 1e-6            # relative error bound for float sums against the fp64 oracle
ABS_TOL_FACTOR = 2.0 ** -40   # |got - ref| bound relative to sum|x| when ref == 0


def check_float_sum(got: float, ref: float, sum_abs: float, what="", extreme_kappa=False):
    """Accept `got` for the exact sum `ref`: NaN/inf must match; otherwise
    |got - ref| <= 1e-6 |ref|, or, when ref == 0, |got| <= 2^-40 sum|x|.
    ``extreme_kappa`` marks inputs built so that sum|x| / |sum x| is far beyond
    what any fp32-pair accumulation resolves (e.g. 1e30 + 1 - 1e30); for them
    only the method's absolute error bound applies: the compensation terms are
    themselves rounded, about u^2 (u = 2^-24) of the partial sums per
    addition over a chain of depth d <= 18, plus the fp64 combine, i.e.
    (d^2 u^2 + 17 * 2^-53) sum|x| ~ 1.2e-12 sum|x| in the worst case.  The
    test bar 2^-40 sum|x| (9.1e-13 sum|x|) sits just inside that worst case:
    typical rounding errors are orders of magnitude smaller."""
    if extreme_kappa and math.isfinite(ref):
        assert abs(got - ref) <= ABS_TOL_FACTOR * sum_abs, (what, got, ref, sum_abs)
        return
    if math.isnan(ref):
        assert math.isnan(got), (what, got, ref)
        return
    if math.isinf(ref):
        assert got == ref, (what, got, ref)
        return
    if ref != 0.0:
        assert abs(got - ref) <= REL_TOL * abs(ref), (what, got, ref, abs(got - ref) / abs(ref))
    else:
        assert abs(got) <= ABS_TOL_FACTOR * sum_abs, (what, got, sum_abs)
