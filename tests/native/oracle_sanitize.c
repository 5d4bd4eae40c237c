/* Drives every entry point of the CPU oracle (oracle/oracle.c) and of the
 * all-cores baseline (oracle/oracle_omp.c) over edge cases -- empty inputs,
 * single elements, padded leading dimensions, every 8- and 16-bit code,
 * integer extremes, non-finite values -- so that a build with
 * -fsanitize=address,undefined reports any out-of-bounds access, leak or
 * undefined behaviour.  Exit status 0 when every call returned what the
 * plain definitions give on these tiny cases. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_tpose(const void *, void *, int64_t, int64_t, int64_t, int64_t, int);
int oracle_decode_all(const void *, int64_t, int, double *);
int64_t oracle_sum_int(const void *, int64_t, int, int *);
double oracle_sum_float(const void *, int64_t, int);
double oracle_sum_abs(const void *, int64_t, int);
float oracle_sum_plain_f32(const void *, int64_t, int);
int oracle_sum_segmented(const void *, const int64_t *, int64_t, int, void *);
int oracle_scan_int(const void *, int64_t, int, int, int64_t *);
int oracle_scan_float(const void *, int64_t, int, int, double *);
int oracle_histogram_int(const void *, int64_t, int, int64_t, int64_t, int64_t, int64_t *);
int oracle_histogram_float(const void *, int64_t, int, double, double, int64_t, int64_t *);
int oracle_matmul(const void *, const void *, double *, int64_t, int64_t, int64_t, int64_t,
                  int64_t, int64_t, int, int);
int oracle_matmul_entries(const void *, const void *, int64_t, int64_t, int64_t, int64_t,
                          int64_t, int, int, int64_t, const int64_t *, const int64_t *,
                          double *);
int omp_tpose(const void *, void *, int64_t, int64_t, int64_t, int64_t, int);
int64_t omp_sum_int(const void *, int64_t, int);
double omp_sum_float(const void *, int64_t, int);

static int bad = 0;
#define EXPECT(c)                                                         \
    do {                                                                  \
        if (!(c)) {                                                       \
            bad++;                                                        \
            fprintf(stderr, "unexpected result, line %d: %s\n", __LINE__, #c); \
        }                                                                 \
    } while (0)

int main(void) {
    /* transposes: exact-size buffers (heap, so ASan sees every edge) */
    for (int eb = 1; eb <= 8; eb *= 2)
        for (int rows = 1; rows <= 5; rows++)
            for (int cols = 1; cols <= 5; cols++)
                for (int pad = 0; pad <= 2; pad++) {
                    const int64_t lds = cols + pad, ldd = rows + pad;
                    unsigned char *s = malloc((size_t)((rows - 1) * lds + cols) * eb);
                    unsigned char *d = malloc((size_t)((cols - 1) * ldd + rows) * eb);
                    unsigned char *d2 = malloc((size_t)((cols - 1) * ldd + rows) * eb);
                    for (int64_t i = 0; i < ((rows - 1) * lds + cols) * eb; i++) s[i] = (unsigned char)i;
                    memset(d, 0, (size_t)((cols - 1) * ldd + rows) * eb);
                    memset(d2, 0, (size_t)((cols - 1) * ldd + rows) * eb);
                    EXPECT(oracle_tpose(s, d, rows, cols, lds, ldd, eb) == 0);
                    EXPECT(omp_tpose(s, d2, rows, cols, lds, ldd, eb) == 0);
                    EXPECT(memcmp(d, d2, (size_t)((cols - 1) * ldd + rows) * eb) == 0);
                    EXPECT(memcmp(d + (cols - 1) * ldd * eb, s + (cols - 1) * eb, (size_t)eb) == 0);
                    free(s);
                    free(d);
                    free(d2);
                }
    EXPECT(oracle_tpose(NULL, NULL, 0, 7, 7, 1, 4) == 0);
    EXPECT(oracle_tpose(NULL, NULL, 3, 3, 2, 3, 4) == -1);

    /* every 8- and 16-bit code decoded, summed, scanned */
    uint16_t *c16 = malloc(65536 * 2);
    double *dv = malloc(65536 * sizeof(double));
    int64_t *iv = malloc(65536 * sizeof(int64_t));
    for (int i = 0; i < 65536; i++) c16[i] = (uint16_t)i;
    for (int dt = 1; dt <= 3; dt++) {
        const int64_t n = dt == 3 ? 256 : 65536;
        uint8_t *c8 = malloc(256);
        for (int i = 0; i < 256; i++) c8[i] = (uint8_t)i;
        const void *src = dt == 3 ? (const void *)c8 : (const void *)c16;
        EXPECT(oracle_decode_all(src, n, dt, dv) == 0);
        EXPECT(isnan(oracle_sum_float(src, n, dt)));          /* NaN codes present */
        EXPECT(isnan(oracle_sum_abs(src, n, dt)));
        (void)oracle_sum_plain_f32(src, n, dt);
        EXPECT(oracle_scan_float(src, n, dt, 0, dv) == 0);
        EXPECT(oracle_scan_float(src, n, dt, 1, dv) == 0 && dv[0] == 0.0);
        int64_t cnt[7];
        EXPECT(oracle_histogram_float(src, n, dt, -2.0, 2.0, 7, cnt) == 0);
        (void)omp_sum_float(src, n, dt);
        free(c8);
    }
    float one = 1.0f;
    EXPECT(oracle_sum_float(&one, 1, 0) == 1.0 && oracle_sum_float(&one, 0, 0) == 0.0);
    EXPECT(omp_sum_float(&one, 1, 0) == 1.0 && omp_sum_float(&one, 0, 0) == 0.0);

    /* integers: extremes, wrap, histograms over the whole int64 range */
    int64_t ext[6] = {INT64_MIN, INT64_MIN + 1, -1, 0, INT64_MAX - 1, INT64_MAX};
    int ov = 0;
    (void)oracle_sum_int(ext, 6, 5, &ov);
    EXPECT(omp_sum_int(ext, 6, 5) == oracle_sum_int(ext, 6, 5, NULL));
    EXPECT(oracle_scan_int(ext, 6, 5, 0, iv) == 0 && oracle_scan_int(ext, 6, 5, 1, iv) == 0);
    int64_t h4[4];
    EXPECT(oracle_histogram_int(ext, 6, 5, INT64_MIN, (int64_t)1 << 62, 4, h4) == 0);
    EXPECT(h4[0] == 2 && h4[1] == 1 && h4[2] == 1 && h4[3] == 2);
    EXPECT(oracle_histogram_int(c16, 65536, 8, 0, 1, 65536, iv) == 0 && iv[65535] == 1);
    int32_t i32[3] = {INT32_MIN, 0, INT32_MAX};
    int64_t h1[1];
    EXPECT(oracle_histogram_int(i32, 3, 4, INT32_MIN, (int64_t)1 << 32, 1, h1) == 0 && h1[0] == 3);
    EXPECT(oracle_sum_int(i32, 0, 4, &ov) == 0 && ov == 0);

    /* segmented: empty segments, a decreasing pair */
    float seg[5] = {1, 2, 3, 4, 5};
    int64_t off[5] = {0, 0, 3, 3, 5}, bad_off[3] = {0, 3, 2};
    double so[4];
    EXPECT(oracle_sum_segmented(seg, off, 4, 0, so) == 0 && so[0] == 0 && so[1] == 6 && so[3] == 9);
    EXPECT(oracle_sum_segmented(seg, bad_off, 2, 0, so) == -1);

    /* matmul: K = 0, padded leading dimensions, sampled entries */
    uint16_t a[3 * 5], b[5 * 4];
    for (int i = 0; i < 15; i++) a[i] = (uint16_t)(0x3F80 + i);
    for (int i = 0; i < 20; i++) b[i] = (uint16_t)(0x3F00 + i);
    double c[3 * 4];
    EXPECT(oracle_matmul(a, b, c, 3, 4, 0, 5, 4, 4, 0, 2) == 0 && c[0] == 0.0);
    EXPECT(oracle_matmul(a, b, c, 3, 4, 5, 5, 4, 4, 0, 2) == 0);
    EXPECT(oracle_matmul(a, b, c, 3, 4, 4, 5, 5, 4, 1, 2) == 0);   /* B^T stored 4 x 5 */
    int64_t rr[2] = {0, 2}, cc[2] = {3, 1};
    double ee[2];
    EXPECT(oracle_matmul_entries(a, b, 3, 4, 5, 5, 4, 0, 2, 2, rr, cc, ee) == 0);
    rr[1] = 3;
    EXPECT(oracle_matmul_entries(a, b, 3, 4, 5, 5, 4, 0, 2, 2, rr, cc, ee) == -1);

    free(c16);
    free(dv);
    free(iv);
    if (bad) return 1;
    puts("oracle under sanitizers: ok");
    return 0;
}
