/*
 * CPU oracle for the transpose and sum-reduction paths.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library and its Python binding) never links, loads or calls it, and this
 * file includes nothing from the product sources.
 *
 * Every routine is the plain definition written out as single-threaded loops:
 *
 *   transpose   out[x][y] = in[y][x] for an H x W row-major `in` and a W x H
 *               row-major `out` (the sequential transpose of Listing 3.5, the
 *               specification the tiled kernels of Listings 3.8, 3.10 and 6.21
 *               are derived from).  Written here with rows = H, cols = W and
 *               explicit leading dimensions:  dst[c*ld_dst + r] = src[r*ld_src + c].
 *               It copies element bits (memcpy), not values, so NaN payloads
 *               and signed zeros survive.
 *
 *   sum         the sequential reduction of Listing 2.1 and its specification
 *               reduce_sum: reduce_sum(0, A) = 0 and
 *               reduce_sum(i+1, A) = reduce_sum(i, A) + A(i)  (Section 2.1).
 *               Integers: int32 inputs accumulate in int64 (exact for n < 2^32);
 *               int64 inputs give the sum modulo 2^64, and an __int128 shadow sum
 *               reports whether that wrap happened.
 *               Floats (fp32, bf16, fp16, fp8-e4m3fn): every element is decoded
 *               exactly to fp64 and summed left to right with Neumaier's
 *               compensated update in fp64.  Non-finite inputs follow IEEE
 *               semantics of the exact sum (any NaN -> NaN; +inf with -inf ->
 *               NaN; otherwise the infinity).
 *
 *   plain fp32  the reduce of Listing 2.1 as specified there: a single fp32
 *               accumulator, one rounding per element, elements taken in index
 *               order.  It is the uncompensated comparator, not a reference.
 *
 *   sum of |x|  sum over i of |A(i)|, decoded exactly and summed like the float
 *               sum above (the magnitude sum that scales the float error bounds
 *               and the condition number sum|x| / |sum x|).  Any NaN gives NaN,
 *               any infinity gives +inf.
 *
 *   prefix sum  the parallel prefix sum the conclusion names as the next case
 *               study: the inclusive scan out[i] = A(0) + ... + A(i), or the
 *               exclusive scan out[i] = A(0) + ... + A(i-1) (out[0] = 0), i.e.
 *               reduce_sum of every prefix.  Same arithmetic as the sums:
 *               int64 (modulo 2^64) for integers, a running fp64 Neumaier sum
 *               of exact decodes for floats, each output rounded to fp64.
 *
 *   histogram   the other case study the conclusion names: counts of the
 *               elements in equal bins.  Integers: bin b holds
 *               lo + b*width <= x < lo + (b+1)*width, b < nbins (exact).
 *               Floats: x decoded exactly; bin floor((x - lo) * s) with
 *               s = nbins / (hi - lo), both evaluated in fp64 with round to
 *               nearest, capped at nbins - 1; x outside [lo, hi) and NaN are
 *               not counted.
 *
 *   matmul      the matrix multiplication case study the conclusion says was
 *               started: C[i][j] = sum over k of A[i][k] * B[k][j] for row-major
 *               A (M x K, leading dimension lda) and B (K x N, ldb; or, with
 *               trans_b, B stored as its N x K transpose).  Every element is
 *               decoded exactly; each product is exact in fp64 (at most 24-bit
 *               significands); the K products are summed in k order with
 *               Neumaier's update, non-finite products by the IEEE rules of the
 *               exact sum.
 *
 * The element decoders are written from the format definitions (IEEE 754
 * binary16; bfloat16 = the top half of binary32; OCP 8-bit E4M3 "FN": bias 7,
 * no infinities, S.1111.111 is NaN, largest finite 448).
 *
 * Pins (checked by the CPU test suite against values fixed by mathematics, by
 * independent libraries and by brute force): see the tests named test_oracle_*.
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>

/* Oracle-local element format codes (kept independent of the product's). */
enum { OR_F32 = 0, OR_F16 = 1, OR_BF16 = 2, OR_F8E4M3 = 3, OR_I32 = 4, OR_I64 = 5, OR_U8 = 7,
       OR_U16 = 8 };

int oracle_elem_bytes(int dtype) {
    switch (dtype) {
    case OR_F32: return 4;
    case OR_F16: return 2;
    case OR_BF16: return 2;
    case OR_F8E4M3: return 1;
    case OR_I32: return 4;
    case OR_I64: return 8;
    case OR_U8: return 1;
    case OR_U16: return 2;
    default: return 0;
    }
}

/* ------------------------------------------------------------------ transpose */

/* dst[c*ld_dst + r] = src[r*ld_src + c] for 0 <= r < rows, 0 <= c < cols.
 * Bytes of dst outside those positions (ld padding) are not touched.
 * Returns 0, or -1 on invalid arguments. */
int oracle_tpose(const void *src, void *dst, int64_t rows, int64_t cols,
                 int64_t ld_src, int64_t ld_dst, int elem_bytes) {
    if (rows < 0 || cols < 0 || elem_bytes <= 0) return -1;
    if (rows == 0 || cols == 0) return 0;
    if (ld_src < cols || ld_dst < rows) return -1;
    const unsigned char *s = (const unsigned char *)src;
    unsigned char *d = (unsigned char *)dst;
    for (int64_t r = 0; r < rows; r++)
        for (int64_t c = 0; c < cols; c++)
            memcpy(d + (c * ld_dst + r) * elem_bytes, s + (r * ld_src + c) * elem_bytes,
                   (size_t)elem_bytes);
    return 0;
}

/* ------------------------------------------------------------------ decoders */

static double dec_f16(uint16_t h) {
    int sign = h >> 15, e = (h >> 10) & 0x1f, m = h & 0x3ff;
    double v;
    if (e == 0) v = ldexp((double)m, -24);                 /* subnormal: m * 2^-24 */
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexp((double)(1024 + m), e - 25);            /* (1 + m/2^10) * 2^(e-15) */
    return sign ? -v : v;
}

static double dec_bf16(uint16_t b) {
    int sign = b >> 15, e = (b >> 7) & 0xff, m = b & 0x7f;
    double v;
    if (e == 0) v = ldexp((double)m, -133);                /* subnormal: m * 2^-133 */
    else if (e == 255) v = m ? NAN : INFINITY;
    else v = ldexp((double)(128 + m), e - 134);            /* (1 + m/2^7) * 2^(e-127) */
    return sign ? -v : v;
}

static double dec_f8e4m3(uint8_t q) {
    int sign = q >> 7, e = (q >> 3) & 0xf, m = q & 0x7;
    double v;
    if (e == 15 && m == 7) return NAN;                      /* only NaN encoding, no inf */
    if (e == 0) v = ldexp((double)m, -9);                  /* subnormal: m/8 * 2^(1-7) */
    else v = ldexp((double)(8 + m), e - 10);               /* (1 + m/8) * 2^(e-7) */
    return sign ? -v : v;
}

static double dec_f32(const unsigned char *p) {
    float f;
    memcpy(&f, p, 4);
    return (double)f;
}

/* Element i of a float-format array, exactly, as fp64. */
double oracle_decode(const void *src, int64_t i, int dtype) {
    const unsigned char *p = (const unsigned char *)src;
    switch (dtype) {
    case OR_F32: return dec_f32(p + 4 * i);
    case OR_F16: { uint16_t h; memcpy(&h, p + 2 * i, 2); return dec_f16(h); }
    case OR_BF16: { uint16_t b; memcpy(&b, p + 2 * i, 2); return dec_bf16(b); }
    case OR_F8E4M3: return dec_f8e4m3(p[i]);
    default: return NAN;
    }
}

int oracle_decode_all(const void *src, int64_t n, int dtype, double *out) {
    if (dtype != OR_F32 && dtype != OR_F16 && dtype != OR_BF16 && dtype != OR_F8E4M3) return -1;
    for (int64_t i = 0; i < n; i++) out[i] = oracle_decode(src, i, dtype);
    return 0;
}

/* ------------------------------------------------------------------ sums */

/* Integer sum.  int32: exact in int64.  int64: modulo 2^64; *overflow (if
 * non-null) is set to 1 when the exact sum leaves the int64 range. */
int64_t oracle_sum_int(const void *src, int64_t n, int dtype, int *overflow) {
    int64_t acc = 0;
    __int128 exact = 0;
    if (dtype == OR_I32) {
        const int32_t *a = (const int32_t *)src;
        for (int64_t i = 0; i < n; i++) {
            acc += (int64_t)a[i];
            exact += a[i];
        }
    } else if (dtype == OR_I64) {
        const int64_t *a = (const int64_t *)src;
        uint64_t w = 0;
        for (int64_t i = 0; i < n; i++) {
            w += (uint64_t)a[i];                         /* two's-complement wrap */
            exact += a[i];
        }
        memcpy(&acc, &w, 8);
    }
    if (overflow) *overflow = (exact > (__int128)INT64_MAX || exact < (__int128)INT64_MIN);
    return acc;
}

/* Float sum: exact decode to fp64, left-to-right Neumaier compensated sum.
 * IEEE semantics of the exact sum for non-finite inputs. */
double oracle_sum_float(const void *src, int64_t n, int dtype) {
    double s = 0.0, c = 0.0;
    int nan = 0, pinf = 0, ninf = 0;
    for (int64_t i = 0; i < n; i++) {
        double x = oracle_decode(src, i, dtype);
        if (isnan(x)) { nan = 1; continue; }
        if (isinf(x)) { if (x > 0) pinf = 1; else ninf = 1; continue; }
        double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    if (nan || (pinf && ninf)) return NAN;
    if (pinf) return INFINITY;
    if (ninf) return -INFINITY;
    return s + c;
}

/* Sum of magnitudes: |x| decoded exactly, fp64 Neumaier sum (both operands
 * are >= 0, so the larger one is the one with the larger value).  A NaN gives
 * NaN, an infinity +inf (the exact sum of the magnitudes). */
double oracle_sum_abs(const void *src, int64_t n, int dtype) {
    double s = 0.0, c = 0.0;
    int nan = 0, inf = 0;
    for (int64_t i = 0; i < n; i++) {
        double x = fabs(oracle_decode(src, i, dtype));
        if (isnan(x)) { nan = 1; continue; }
        if (isinf(x)) { inf = 1; continue; }
        double t = s + x;
        if (s >= x) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    if (nan) return NAN;
    if (inf) return INFINITY;
    return s + c;
}

/* The comparator: one fp32 accumulator, one rounding per element (Listing 2.1). */
float oracle_sum_plain_f32(const void *src, int64_t n, int dtype) {
    float s = 0.0f;
    for (int64_t i = 0; i < n; i++) s += (float)oracle_decode(src, i, dtype);
    return s;
}

/* ------------------------------------------------------------------ segmented */

/* Segment i is [offsets[i], offsets[i+1]).  Float formats write fp64 sums,
 * integer formats write int64 sums.  Returns -1 on non-monotone offsets. */
int oracle_sum_segmented(const void *src, const int64_t *offsets, int64_t nseg, int dtype,
                         void *out) {
    int eb = oracle_elem_bytes(dtype);
    if (!eb) return -1;
    for (int64_t i = 0; i < nseg; i++) {
        int64_t lo = offsets[i], hi = offsets[i + 1];
        if (hi < lo || lo < 0) return -1;
        const unsigned char *p = (const unsigned char *)src + lo * eb;
        if (dtype == OR_I32 || dtype == OR_I64)
            ((int64_t *)out)[i] = oracle_sum_int(p, hi - lo, dtype, NULL);
        else
            ((double *)out)[i] = oracle_sum_float(p, hi - lo, dtype);
    }
    return 0;
}

/* ------------------------------------------------------------------ prefix sums */

/* Integer scan into int64 out[n] (modulo 2^64 for int64 inputs). */
int oracle_scan_int(const void *src, int64_t n, int dtype, int exclusive, int64_t *out) {
    if (dtype != OR_I32 && dtype != OR_I64) return -1;
    uint64_t w = 0;
    for (int64_t i = 0; i < n; i++) {
        const uint64_t x = dtype == OR_I32 ? (uint64_t)(int64_t)((const int32_t *)src)[i]
                                           : (uint64_t)((const int64_t *)src)[i];
        if (exclusive) {
            memcpy(&out[i], &w, 8);
            w += x;
        } else {
            w += x;
            memcpy(&out[i], &w, 8);
        }
    }
    return 0;
}

/* Float scan into double out[n]: each output is the compensated running sum of
 * the exact decodes (Neumaier, fp64) rounded to fp64, with the IEEE rules of
 * the exact prefix for non-finite values. */
int oracle_scan_float(const void *src, int64_t n, int dtype, int exclusive, double *out) {
    if (dtype != OR_F32 && dtype != OR_F16 && dtype != OR_BF16 && dtype != OR_F8E4M3) return -1;
    double s = 0.0, c = 0.0;
    int nan = 0, pinf = 0, ninf = 0;
    for (int64_t i = 0; i < n; i++) {
        double prefix;
        if (exclusive) {
            prefix = (nan || (pinf && ninf)) ? NAN : pinf ? INFINITY : ninf ? -INFINITY : s + c;
            out[i] = prefix;
        }
        double x = oracle_decode(src, i, dtype);
        if (isnan(x)) {
            nan = 1;
        } else if (isinf(x)) {
            if (x > 0) pinf = 1; else ninf = 1;
        } else {
            double t = s + x;
            if (fabs(s) >= fabs(x)) c += (s - t) + x;
            else c += (x - t) + s;
            s = t;
        }
        if (!exclusive) {
            prefix = (nan || (pinf && ninf)) ? NAN : pinf ? INFINITY : ninf ? -INFINITY : s + c;
            out[i] = prefix;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ histograms */

static int int_elem(const void *src, int64_t i, int dtype, __int128 *x) {
    switch (dtype) {
    case OR_I32: *x = ((const int32_t *)src)[i]; return 0;
    case OR_I64: *x = ((const int64_t *)src)[i]; return 0;
    case OR_U8: *x = ((const uint8_t *)src)[i]; return 0;
    case OR_U16: *x = ((const uint16_t *)src)[i]; return 0;
    default: return -1;
    }
}

/* Integer histogram: counts[b] = #{i : lo + b*width <= x_i < lo + (b+1)*width}. */
int oracle_histogram_int(const void *src, int64_t n, int dtype, int64_t lo, int64_t width,
                         int64_t nbins, int64_t *counts) {
    if (width < 1 || nbins < 0) return -1;
    for (int64_t b = 0; b < nbins; b++) counts[b] = 0;
    const __int128 span = (__int128)width * nbins;
    for (int64_t i = 0; i < n; i++) {
        __int128 x;
        if (int_elem(src, i, dtype, &x)) return -1;
        __int128 d = x - lo;
        if (d < 0 || d >= span) continue;
        counts[(int64_t)(d / width)] += 1;
    }
    return 0;
}

/* Float histogram over [lo, hi): bin floor((x - lo) * (nbins / (hi - lo))) in
 * fp64, capped at nbins - 1; NaN and x outside [lo, hi) are not counted. */
int oracle_histogram_float(const void *src, int64_t n, int dtype, double lo, double hi,
                           int64_t nbins, int64_t *counts) {
    if (dtype != OR_F32 && dtype != OR_F16 && dtype != OR_BF16 && dtype != OR_F8E4M3) return -1;
    if (!(hi > lo) || !isfinite(lo) || !isfinite(hi) || nbins < 1) return -1;
    const double scale = (double)nbins / (hi - lo);
    if (!isfinite(hi - lo) || !isfinite(scale)) return -1;   /* the bin rule needs both finite */
    for (int64_t b = 0; b < nbins; b++) counts[b] = 0;
    for (int64_t i = 0; i < n; i++) {
        const double x = oracle_decode(src, i, dtype);
        if (!(x >= lo && x < hi)) continue;             /* NaN fails both */
        double t = (x - lo) * scale;
        int64_t b = (int64_t)floor(t);
        if (b > nbins - 1) b = nbins - 1;
        counts[b] += 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ matmul */

/* One entry C[i][j] = sum_k A[i][k] * B[k][j]: exact products, Neumaier sum in k order. */
static double mm_entry(const void *a, const void *b, int64_t K, int64_t lda, int64_t ldb,
                       int trans_b, int dtype, int64_t i, int64_t j) {
    double s = 0.0, c = 0.0;
    int nan = 0, pinf = 0, ninf = 0;
    for (int64_t k = 0; k < K; k++) {
        const double x = oracle_decode(a, i * lda + k, dtype);
        const double y = oracle_decode(b, trans_b ? j * ldb + k : k * ldb + j, dtype);
        const double p = x * y;
        if (isnan(p)) {
            nan = 1;
        } else if (isinf(p)) {
            if (p > 0) pinf = 1; else ninf = 1;
        } else {
            const double t = s + p;
            if (fabs(s) >= fabs(p)) c += (s - t) + p;
            else c += (p - t) + s;
            s = t;
        }
    }
    return (nan || (pinf && ninf)) ? NAN : pinf ? INFINITY : ninf ? -INFINITY : s + c;
}

static int mm_dtype_ok(int dtype) {
    return dtype == OR_F32 || dtype == OR_F16 || dtype == OR_BF16 || dtype == OR_F8E4M3;
}

/* c[i*ldc + j] = C[i][j] for the whole M x N product. */
int oracle_matmul(const void *a, const void *b, double *c, int64_t M, int64_t N, int64_t K,
                  int64_t lda, int64_t ldb, int64_t ldc, int trans_b, int dtype) {
    if (!mm_dtype_ok(dtype) || M < 0 || N < 0 || K < 0 || lda < K || ldc < N ||
        ldb < (trans_b ? K : N))
        return -1;
    for (int64_t i = 0; i < M; i++)
        for (int64_t j = 0; j < N; j++)
            c[i * ldc + j] = mm_entry(a, b, K, lda, ldb, trans_b, dtype, i, j);
    return 0;
}

/* out[t] = C[rows[t]][cols[t]] for t < count (sampled entries of a large product). */
int oracle_matmul_entries(const void *a, const void *b, int64_t M, int64_t N, int64_t K,
                          int64_t lda, int64_t ldb, int trans_b, int dtype, int64_t count,
                          const int64_t *rows, const int64_t *cols, double *out) {
    if (!mm_dtype_ok(dtype) || lda < K || ldb < (trans_b ? K : N)) return -1;
    for (int64_t t = 0; t < count; t++) {
        if (rows[t] < 0 || rows[t] >= M || cols[t] < 0 || cols[t] >= N) return -1;
        out[t] = mm_entry(a, b, K, lda, ldb, trans_b, dtype, rows[t], cols[t]);
    }
    return 0;
}
