"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake (a transposed index, a dropped term, a
wrong sign, an off-by-one exponent bias, ...) in a private copy of
``oracle/oracle.c``, builds it with gcc into a temporary library, and checks
that at least one pin of the matching group rejects it.  The real oracle is
never modified."""
import os

import pytest

import oracle
import oracle_pins as P

MUTANTS = [
    # (name, original text, planted mistake, pin group)
    ("tpose_dst_index_transposed", "d + (c * ld_dst + r) * elem_bytes",
     "d + (r * ld_dst + c) * elem_bytes", P.PINS_TPOSE),
    ("tpose_src_index_transposed", "s + (r * ld_src + c) * elem_bytes",
     "s + (c * ld_src + r) * elem_bytes", P.PINS_TPOSE),
    ("tpose_ld_ignored", "d + (c * ld_dst + r) * elem_bytes",
     "d + (c * rows + r) * elem_bytes", P.PINS_TPOSE),
    ("tpose_last_col_dropped", "for (int64_t c = 0; c < cols; c++)",
     "for (int64_t c = 0; c < cols - 1; c++)", P.PINS_TPOSE),
    ("int32_last_term_dropped", "acc += (int64_t)a[i];",
     "if (i + 1 < n) acc += (int64_t)a[i];", P.PINS_INT),
    ("int32_accumulates_in_int32", "acc += (int64_t)a[i];",
     "acc = (int32_t)(acc + a[i]);", P.PINS_INT),
    ("int64_overflow_flag_wrong", "*overflow = (exact > (__int128)INT64_MAX",
     "*overflow = (exact >= (__int128)INT64_MAX", P.PINS_INT),
    ("int64_sign_flipped", "w += (uint64_t)a[i];", "w -= (uint64_t)a[i];", P.PINS_INT),
    ("neumaier_wrong_sign", "if (fabs(s) >= fabs(x)) c += (s - t) + x;",
     "if (fabs(s) >= fabs(x)) c += (t - s) + x;", P.PINS_FLOAT),
    ("neumaier_dropped_term", "else c += (x - t) + s;", "else c += (x - t);", P.PINS_FLOAT),
    ("neumaier_no_compensation", "return s + c;\n}\n\n/* Sum of magnitudes",
     "return s;\n}\n\n/* Sum of magnitudes", P.PINS_FLOAT),
    ("f16_subnormal_scale", "ldexp((double)m, -24)", "ldexp((double)m, -25)", P.PINS_FLOAT),
    ("bf16_bias_off_by_one", "e - 134", "e - 133", P.PINS_FLOAT),
    ("f8_nan_code_wrong", "if (e == 15 && m == 7) return NAN;",
     "if (e == 15 && m == 6) return NAN;", P.PINS_FLOAT),
    ("f8_subnormal_as_normal", "if (e == 0) v = ldexp((double)m, -9);",
     "if (e == 0) v = ldexp((double)(8 + m), -10);", P.PINS_FLOAT),
    ("inf_returns_nan", "if (pinf) return INFINITY;", "if (pinf) return NAN;", P.PINS_FLOAT),
    ("plain_f32_in_double", "float s = 0.0f;\n    for (int64_t i = 0; i < n; i++) s += (float)",
     "double s = 0.0;\n    for (int64_t i = 0; i < n; i++) s += (double)", P.PINS_FLOAT),
    ("segment_bounds_shifted", "int64_t lo = offsets[i], hi = offsets[i + 1];",
     "int64_t lo = offsets[i], hi = offsets[i + 1] - (i > 0);", P.PINS_FLOAT),
    ("scan_exclusive_includes_own_term", "        if (exclusive) {\n            memcpy(&out[i], &w, 8);\n            w += x;",
     "        if (exclusive) {\n            w += x;\n            memcpy(&out[i], &w, 8);", P.PINS_SCAN),
    ("scan_int32_sign_dropped", "(uint64_t)(int64_t)((const int32_t *)src)[i]",
     "(uint64_t)(uint32_t)((const int32_t *)src)[i]", P.PINS_SCAN),
    ("scan_float_no_compensation", "ninf ? -INFINITY : s + c;\n            out[i] = prefix;\n        }\n    }",
     "ninf ? -INFINITY : s;\n            out[i] = prefix;\n        }\n    }", P.PINS_SCAN),
    ("abs_sign_kept", "double x = fabs(oracle_decode(src, i, dtype));",
     "double x = oracle_decode(src, i, dtype);", P.PINS_ABS),
    ("abs_no_compensation", "if (inf) return INFINITY;\n    return s + c;",
     "if (inf) return INFINITY;\n    return s;", P.PINS_ABS),
    ("abs_inf_gives_nan", "if (isinf(x)) { inf = 1; continue; }", "(void)inf;", P.PINS_ABS),
    ("abs_comparison_flipped", "if (s >= x) c += (s - t) + x;", "if (s < x) c += (s - t) + x;",
     P.PINS_ABS),
    ("hist_u16_read_signed", "case OR_U16: *x = ((const uint16_t *)src)[i]; return 0;",
     "case OR_U16: *x = ((const int16_t *)src)[i]; return 0;", P.PINS_HIST),
    ("hist_int_hi_included", "if (d < 0 || d >= span) continue;", "if (d < 0 || d > span) continue; if (d == span) d = span - 1;",
     P.PINS_HIST),
    ("hist_int_bin_rounds", "counts[(int64_t)(d / width)] += 1;",
     "counts[(int64_t)((d + width / 2) / width) % nbins] += 1;", P.PINS_HIST),
    ("hist_float_lo_excluded", "if (!(x >= lo && x < hi)) continue;",
     "if (!(x > lo && x < hi)) continue;", P.PINS_HIST),
    ("hist_float_scale_off", "const double scale = (double)nbins / (hi - lo);",
     "const double scale = (double)(nbins - 1) / (hi - lo);", P.PINS_HIST),
    ("mm_b_transposed", "trans_b ? j * ldb + k : k * ldb + j", "trans_b ? k * ldb + j : j * ldb + k",
     P.PINS_MM),
    ("mm_last_k_dropped", "for (int64_t k = 0; k < K; k++) {\n        const double x",
     "for (int64_t k = 0; k < K - 1; k++) {\n        const double x", P.PINS_MM),
    ("mm_lda_ignored", "oracle_decode(a, i * lda + k, dtype)", "oracle_decode(a, i * K + k, dtype)",
     P.PINS_MM),
    ("mm_uncompensated", "ninf ? -INFINITY : s + c;\n}\n\nstatic int mm_dtype_ok",
     "ninf ? -INFINITY : s;\n}\n\nstatic int mm_dtype_ok", P.PINS_MM),
    ("mm_inf_times_zero", "if (isnan(p)) {\n            nan = 1;\n        } else if (isinf(p)) {\n            if (p > 0) pinf = 1; else ninf = 1;\n        } else {\n            const double t",
     "if (isnan(p)) {\n            (void)p;\n        } else if (isinf(p)) {\n            if (p > 0) pinf = 1; else ninf = 1;\n        } else {\n            const double t", P.PINS_MM),
]


@pytest.mark.parametrize("name,orig,bad,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_mutant(tmp_path, name, orig, bad, pins):
    with open(oracle.SRC) as f:
        src = f.read()
    assert src.count(orig) >= 1, f"mutation site for {name} not found in oracle.c"
    mut_src = os.path.join(tmp_path, f"{name}.c")
    with open(mut_src, "w") as f:
        f.write(src.replace(orig, bad, 1))
    lib = oracle.build(mut_src, os.path.join(tmp_path, f"lib{name}.so"))
    mutant = oracle.Oracle(lib)
    caught = []
    for pin in pins:
        try:
            pin(mutant)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
            break
    assert caught, f"no pin rejects mutant {name}"
