/*
 * All-cores CPU baseline for the transpose and sum paths.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: only the benchmark's CPU-baseline
 * leg and the test suite load this library; the product path never does, and
 * nothing here is shared with the HIP sources.
 *
 * The same plain loops as oracle.c, spread over the host cores with OpenMP in
 * the two-level pattern of Listing 2.2 (Section 2.2): the iteration space is
 * cut into tiles that threads take in parallel, each tile produces a partial
 * result, and the partials are combined serially in tile order.
 *
 *   transpose   dst[c*ld_dst + r] = src[r*ld_src + c]; the rows of src are
 *               split over the threads (each element is still one memcpy).
 *   int sum     int64 partial sums of tiles of TILE elements (modulo 2^64 for
 *               int64 inputs), added serially in tile order: exact, so equal to
 *               the sequential oracle bit for bit.
 *   float sum   exact fp64 decodes; each tile summed with Neumaier's update,
 *               the tile values (s + c) combined serially with the same update.
 *               The association differs from the sequential oracle, so the
 *               result may differ from it by a few ulp.
 *
 * Non-finite float inputs follow the IEEE rules of the exact sum (any NaN ->
 * NaN, +inf with -inf -> NaN, else the infinity), as in oracle.c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

enum { OM_F32 = 0, OM_F16 = 1, OM_BF16 = 2, OM_F8E4M3 = 3, OM_I32 = 4, OM_I64 = 5 };

#define TILE 128   /* elements per partial sum, as in Listing 2.2 */

int omp_threads(void) { return omp_get_max_threads(); }

int omp_tpose(const void *src, void *dst, int64_t rows, int64_t cols, int64_t ld_src,
              int64_t ld_dst, int eb) {
    if (rows < 0 || cols < 0 || eb <= 0) return -1;
    if (rows == 0 || cols == 0) return 0;
    if (ld_src < cols || ld_dst < rows) return -1;
    const unsigned char *s = (const unsigned char *)src;
    unsigned char *d = (unsigned char *)dst;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; r++)
        for (int64_t c = 0; c < cols; c++)
            memcpy(d + (c * ld_dst + r) * eb, s + (r * ld_src + c) * eb, (size_t)eb);
    return 0;
}

int64_t omp_sum_int(const void *src, int64_t n, int dtype) {
    const int64_t nt = (n + TILE - 1) / TILE;
    uint64_t *ps = (uint64_t *)malloc((size_t)(nt > 0 ? nt : 1) * sizeof(uint64_t));
    if (!ps) return 0;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < nt; t++) {
        const int64_t lo = t * TILE, hi = lo + TILE < n ? lo + TILE : n;
        uint64_t acc = 0;
        if (dtype == OM_I32)
            for (int64_t i = lo; i < hi; i++) acc += (uint64_t)(int64_t)((const int32_t *)src)[i];
        else
            for (int64_t i = lo; i < hi; i++) acc += (uint64_t)((const int64_t *)src)[i];
        ps[t] = acc;
    }
    uint64_t sum = 0;
    for (int64_t t = 0; t < nt; t++) sum += ps[t];
    free(ps);
    int64_t r;
    memcpy(&r, &sum, 8);
    return r;
}

static double dec(const void *src, int64_t i, int dtype) {
    const unsigned char *p = (const unsigned char *)src;
    if (dtype == OM_F32) {
        float f;
        memcpy(&f, p + 4 * i, 4);
        return (double)f;
    }
    if (dtype == OM_BF16) {
        uint16_t b;
        memcpy(&b, p + 2 * i, 2);
        uint32_t w = (uint32_t)b << 16;          /* bf16 is the top half of binary32 */
        float f;
        memcpy(&f, &w, 4);
        return (double)f;
    }
    if (dtype == OM_F16) {
        uint16_t h;
        memcpy(&h, p + 2 * i, 2);
        const int sg = h >> 15, e = (h >> 10) & 0x1f, m = h & 0x3ff;
        double v = e == 0 ? ldexp((double)m, -24)
                 : e == 31 ? (m ? NAN : INFINITY) : ldexp((double)(1024 + m), e - 25);
        return sg ? -v : v;
    }
    const uint8_t q = p[i];                      /* OCP E4M3 "FN" */
    const int sg = q >> 7, e = (q >> 3) & 0xf, m = q & 0x7;
    if (e == 15 && m == 7) return NAN;
    double v = e == 0 ? ldexp((double)m, -9) : ldexp((double)(8 + m), e - 10);
    return sg ? -v : v;
}

static void neumaier(double *s, double *c, double x) {
    const double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

double omp_sum_float(const void *src, int64_t n, int dtype) {
    const int64_t nt = (n + TILE - 1) / TILE;
    double *ps = (double *)malloc((size_t)(nt > 0 ? nt : 1) * sizeof(double));
    int nan = 0, pinf = 0, ninf = 0;
    if (!ps) return NAN;
#pragma omp parallel for schedule(static) reduction(| : nan, pinf, ninf)
    for (int64_t t = 0; t < nt; t++) {
        const int64_t lo = t * TILE, hi = lo + TILE < n ? lo + TILE : n;
        double s = 0.0, c = 0.0;
        for (int64_t i = lo; i < hi; i++) {
            const double x = dec(src, i, dtype);
            if (isnan(x)) { nan = 1; continue; }
            if (isinf(x)) { if (x > 0) pinf = 1; else ninf = 1; continue; }
            neumaier(&s, &c, x);
        }
        ps[t] = s + c;
    }
    double s = 0.0, c = 0.0;
    for (int64_t t = 0; t < nt; t++) neumaier(&s, &c, ps[t]);
    free(ps);
    if (nan || (pinf && ninf)) return NAN;
    if (pinf) return INFINITY;
    if (ninf) return -INFINITY;
    return s + c;
}
