"""The CPU oracle against its pins (no GPU)."""
import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(orc, pin):
    pin(orc)


def test_all_cores_baseline_matches_oracle(orc):
    """The OpenMP build of the plain loops (the benchmark's all-cores CPU
    baseline) computes what the oracle computes: transposes and integer sums
    bit for bit, float sums within 4 ulp of math.fsum."""
    import math

    import numpy as np

    import oracle
    import workloads as W
    b = oracle.omp()
    assert b.threads() >= 1
    for eb, (r, c) in ((4, (300, 517)), (2, (129, 1000)), (1, (77, 33))):
        a = W.random_bits(r * c, 600 + eb, eb).reshape(r, c)
        assert np.array_equal(b.tpose(a), orc.tpose(a))
    for n in (0, 1, 127, 128, 129, 100003):
        x = W.integers(n, 610, -(1 << 40), 1 << 40, "i64")
        assert b.sum_int(x, "i64") == orc.sum_int(x, "i64")[0]
        y = W.integers(n, 611, -1000, 1000, "i32")
        assert b.sum_int(y, "i32") == orc.sum_int(y, "i32")[0]
    for dt in ("f32", "bf16", "f16", "f8e4m3"):
        bits = W.normal(50001, 612, "f32") if dt == "f32" else W.signed_lognormal(50001, 613, dt)[0]
        exact = math.fsum(orc.decode(bits, dt).tolist())
        assert abs(b.sum_float(bits, dt) - exact) <= 4 * math.ulp(abs(exact))
    inf = np.float32(np.inf)
    assert b.sum_float(np.array([1, inf, 2] * 100, np.float32), "f32") == math.inf
    assert math.isnan(b.sum_float(np.array([inf] + [1] * 300 + [-inf], np.float32), "f32"))
