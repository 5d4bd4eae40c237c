/*
 * xtr — out-of-place matrix transpose and tree-based sum reduction on
 * AMD Instinct MI355X (gfx950).  C ABI of libxtr.so.
 *
 * The two operations are the case studies of "Source-to-Source
 * Transformations for GPU Code Generation" (de Castelnau, 2026):
 *   - transpose: the sequential specification of Listing 3.5
 *     (out[x][y] = in[y][x], in is H x W, out is W x H, both row-major),
 *     computed with LDS-staged tiles and a block barrier at the point where
 *     tile ownership moves from the loading threads to the storing threads
 *     (Listings 3.8 and 3.10, Section 3.3);
 *   - sum: the sequential reduce of Listing 2.1 (specification reduce_sum,
 *     Section 2.1), computed as per-thread register accumulators, a
 *     cross-lane wavefront reduction, an LDS tree across the waves of a
 *     workgroup (the tree reduction of Section 7.2, with the register
 *     accumulator of Listing 7.22) and a grid-level combine of per-workgroup
 *     partials (the partial-sums-then-combine split of Listing 2.2).
 *
 * Conventions for every entry point:
 *   - Data pointers are DEVICE pointers unless the comment says "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls only enqueue work; results are valid once the stream has
 *     reached that point (hipStreamSynchronize or an event).
 *   - The caller owns every data buffer; the library never frees them.
 *     The library owns its internal workspace (per device and stream, grown
 *     on demand and kept until xtr_release or process exit) and its pinned
 *     host staging for descriptor tables.  A grown workspace replaces the old
 *     buffer without freeing it (queued work or a captured graph may still
 *     use it); replaced buffers are freed by xtr_release.
 *   - Graphs: calls that use the library workspace can be captured once the
 *     workspace is large enough (it cannot grow during capture: ENOMEM).  A
 *     captured graph keeps the workspace address it saw, so its replays share
 *     that buffer with eager calls on the capture stream: replay it on that
 *     stream (or order the streams), and keep the graph's replays from
 *     overlapping each other.  The *_ws entry points and the batch plans take
 *     caller-owned state instead.
 *   - Return value: XTR_OK (0) or a negative XTR_E* code.  On a validation
 *     error (EINVAL, EDTYPE, EOVERLAP, EALIGN) nothing has been enqueued.
 *     EHIP means a HIP call failed (message in xtr_last_error()).  No C++
 *     exception crosses this interface.
 *   - Sizes and leading dimensions are in ELEMENTS, never bytes.
 */
#ifndef XTR_H
#define XTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element formats.  Transpose accepts all of them (it copies element bits);
 * the sums accept F32, F16, BF16, F8E4M3 (OCP E4M3 "FN": bias 7, no inf,
 * S.1111.111 = NaN) and I32, I64. */
typedef enum {
    XTR_F32 = 0, XTR_F16 = 1, XTR_BF16 = 2, XTR_F8E4M3 = 3,
    XTR_I32 = 4, XTR_I64 = 5, XTR_F64 = 6, XTR_U8 = 7, XTR_U16 = 8
} xtr_dtype;

enum {
    XTR_OK = 0,
    XTR_EINVAL = -1,    /* null pointer, negative size, ld too small, bad offsets table */
    XTR_EDTYPE = -2,    /* unknown dtype, or a dtype the operation does not take   */
    XTR_EOVERLAP = -3,  /* src and dst byte ranges overlap (transpose is out-of-place) */
    XTR_EALIGN = -4,    /* a pointer is not aligned to its element size             */
    XTR_EHIP = -5,      /* a HIP runtime call failed                               */
    XTR_ENOMEM = -6,    /* workspace allocation failed                             */
    XTR_EBUDGET = -7    /* caller workspace too small                              */
};

/* ------------------------------------------------------------------------
 * tpose — out-of-place transpose (Listing 3.5; tiled form Listings 3.8/3.10).
 *
 *   dst[c*ld_dst + r] = src[r*ld_src + c]   for 0 <= r < rows, 0 <= c < cols
 *
 * src: rows x cols, row-major, leading dimension ld_src >= max(cols, 1).
 * dst: cols x rows, row-major, leading dimension ld_dst >= max(rows, 1).
 * The copy is of element bits (NaN payloads, -0.0 survive).  Elements of dst
 * in columns [rows, ld_dst) of each dst row are not written.
 * rows == 0 or cols == 0 is a no-op returning XTR_OK.
 * Any alignment of src/dst (to the element size) and any ld is accepted.
 * Global accesses move the widest piece (16, 8 or 4 bytes, and at least one
 * element) that divides src, dst, ld_src*elem and ld_dst*elem; 1- and 2-byte
 * elements with no such piece are moved one element per lane.  The result is
 * the same whichever width is used; only the speed differs.
 * Errors: EINVAL (null, negative, small ld), EDTYPE, EOVERLAP, EALIGN.
 */
int tpose(const void *src, void *dst, int64_t rows, int64_t cols,
          int64_t ld_src, int64_t ld_dst, int dtype, void *stream);

/* ------------------------------------------------------------------------
 * reduce_sum — sum of n elements (Listing 2.1; reduce_sum of Section 2.1).
 *
 * out: for F32/F16/BF16/F8E4M3 a device double*, for I32/I64 a device int64_t*.
 *   - Integers: exact int64 sum for I32; sum modulo 2^64 for I64.  Bit-exact
 *     and independent of order.
 *   - Floats: elements are decoded exactly to fp32 and accumulated in fp32
 *     pairs (s, c) with an error-free two-sum per element (compensated,
 *     Neumaier style); pairs are combined with the same pair arithmetic
 *     across lanes and waves; the per-workgroup pairs are combined in fp64
 *     in a fixed order.  The result is a deterministic function of
 *     (data, n, dtype, src alignment).  NaN in -> NaN out; +inf and -inf ->
 *     NaN; a single-signed inf -> that inf.  The domain is |partial sums| <
 *     FLT_MAX (the fp32 accumulators overflow to inf beyond it).
 * n == 0 writes 0.  Uses library workspace (per device/stream); see
 * reduce_sum_ws for a caller-provided one.
 * Errors: EINVAL, EDTYPE, EALIGN, ENOMEM, EHIP.
 */
int reduce_sum(const void *src, int64_t n, void *out, int dtype, void *stream);

/* Same reduction structure with plain (uncompensated) fp32 adds at every
 * level and an fp32 grid combine; writes one float.  Float dtypes only.  It
 * is the comparator that shows what the compensation buys. */
int reduce_sum_plain_f32(const void *src, int64_t n, float *out, int dtype, void *stream);

/* Workspace bytes reduce_sum_ws needs for (n, dtype). */
size_t xtr_reduce_workspace_bytes(int64_t n, int dtype);

/* reduce_sum with caller-owned device workspace `ws` of `ws_bytes` bytes
 * (>= xtr_reduce_workspace_bytes(n, dtype)).  The workspace must be zeroed
 * before its first use; every call leaves its ticket counters at zero again,
 * so the workspace can be reused by later calls on the same stream without
 * clearing.  Calls that share one workspace must not overlap in time.  Errors
 * as reduce_sum, plus EBUDGET when ws_bytes is too small. */
int reduce_sum_ws(const void *src, int64_t n, void *out, int dtype,
                  void *ws, size_t ws_bytes, void *stream);

/* reduce_sum for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result and errors as reduce_sum (bit for bit), but the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine):
 * its workspace is a fixed device array of XTR_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends (its
 * address is looked up once per device).  n is limited to what that array
 * holds: 209715 chunks, i.e. about 1.7e9 fp32 or int32, 3.4e9 bf16 or fp16,
 * 6.9e9 fp8 and 8.6e8 int64 elements; larger n returns XTR_EBUDGET with
 * nothing enqueued.  Every call
 * on one GPU shares that GPU's array, whatever the stream: calls that overlap
 * in time on one GPU race (serialize them on one stream or with events).
 * The call clears what must start at zero with a fill kernel on `stream`. */
#define XTR_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int reduce_sum_noalloc(const void *src, int64_t n, void *out, int dtype, void *stream);

/* ------------------------------------------------------------------------
 * Batched and segmented forms (one persistent launch per batch).
 */
typedef struct {
    const void *src;   /* device */
    void *dst;         /* device */
    int64_t rows, cols, ld_src, ld_dst;
    int32_t dtype, _pad;
} xtr_tpose_desc;

/* Transposes descs[0..count) (host array), each as tpose().  Jobs are grouped
 * by (element size, piece width, whether 32-bit offsets suffice); each group
 * runs as one persistent launch whose workgroups stride over the concatenated
 * tile space of its jobs.  count == 0 is a no-op.
 * Every descriptor is validated before anything is enqueued.  dst ranges of
 * different jobs must not overlap each other or any src. */
int tpose_batched(const xtr_tpose_desc *descs, int64_t count, void *stream);

/* Sum of each CSR segment: segment i is src[offsets[i] .. offsets[i+1]).
 * offsets: device int64_t[nseg + 1], non-decreasing, offsets[0] >= 0.
 * out: device double[nseg] (float dtypes) or int64_t[nseg] (integer dtypes).
 * Empty segments give 0.  Each segment is reduced with exactly the chunking
 * and combine order of reduce_sum on that segment alone, so the result equals
 * reduce_sum(src + offsets[i], len_i) bit for bit.
 * This entry point reads offsets[nseg] back to the host (a blocking 8-byte
 * copy) to size its chunk space; reduce_sum_segmented_ws takes the total from
 * the caller and stays fully asynchronous.
 * Invalid tables (a decreasing pair, or lengths summing to more than
 * offsets[nseg]) are detected on the device: every output of the call is then
 * NaN (float dtypes) or 0 (integer dtypes); nothing is read out of the ranges
 * the table names. */
int reduce_sum_segmented(const void *src, const int64_t *offsets, int64_t nseg,
                         void *out, int dtype, void *stream);

/* Workspace bytes reduce_sum_segmented_ws needs for nseg segments holding
 * total_elems elements in all (total_elems = offsets[nseg] - offsets[0]). */
size_t xtr_segmented_workspace_bytes(int64_t nseg, int64_t total_elems, int dtype);

/* reduce_sum_segmented with a caller-owned device workspace `ws` of
 * `ws_bytes` bytes (zeroed before first use; left reusable, as for
 * reduce_sum_ws), fully asynchronous: nothing is read back.  The chunk space
 * is as large as the workspace holds; ws_bytes >=
 * xtr_segmented_workspace_bytes(nseg, offsets[nseg] - offsets[0], dtype)
 * holds every table whose lengths sum to that total.  A table that needs
 * more chunk space than the workspace holds is treated like an invalid table
 * (every output NaN for float dtypes, 0 for integer dtypes), which is
 * detected on the device.
 * Errors: as reduce_sum_segmented, plus EBUDGET when the workspace cannot
 * hold nseg + 1 chunks. */
int reduce_sum_segmented_ws(const void *src, const int64_t *offsets, int64_t nseg, void *out,
                            int dtype, void *ws, size_t ws_bytes, void *stream);

/* The same with the element total (offsets[nseg] - offsets[0]) given by the
 * caller: the chunk space is sized from it, and EBUDGET is returned when the
 * workspace is smaller than xtr_segmented_workspace_bytes(nseg, total_elems,
 * dtype). */
int reduce_sum_segmented_ws_total(const void *src, const int64_t *offsets, int64_t nseg,
                                  int64_t total_elems, void *out, int dtype, void *ws,
                                  size_t ws_bytes, void *stream);

/* Sums of `count` independent arrays: srcs (host array of device pointers),
 * ns (host array of lengths), out device double[count] / int64_t[count]. */
int reduce_sum_batched(const void *const *srcs, const int64_t *ns, int64_t count,
                       void *out, int dtype, void *stream);

/* reduce_sum_batched with one output location per job: outs is a host array
 * of `count` device pointers (double* for float dtypes, int64_t* for
 * integer dtypes, each 8-byte aligned).  Lets a request loop write each
 * result straight into the job's own output slot. */
int reduce_sum_batched_scatter(const void *const *srcs, const int64_t *ns, void *const *outs,
                               int64_t count, int dtype, void *stream);

/* ------------------------------------------------------------------------
 * scan_sum -- prefix sums, the parallel prefix sum the thesis's conclusion
 * names as the next case study: reduce_sum (Section 2.1) of every prefix.
 *
 *   inclusive (exclusive == 0): out[i] = src[0] + ... + src[i]
 *   exclusive (exclusive != 0): out[i] = src[0] + ... + src[i-1], out[0] = 0
 *
 * out: device double[n] for F32/F16/BF16/F8E4M3, int64_t[n] for I32/I64
 * (8-byte aligned; must not overlap src).  Integers: exact 64-bit sums
 * (modulo 2^64 for I64).  Floats: exact decodes accumulated in fp64 in a
 * fixed order (deterministic); every output is within about 300 * 2^-53 of
 * the sum of magnitudes of its prefix from the exact prefix sum, and
 * non-finite values follow the IEEE rules of the exact prefix (NaN -> NaN
 * from there on; +inf with -inf -> NaN).  Floats: four launches on `stream`
 * (tile sums, two levels of their scan, the tile rescans).  Integers with a
 * 16-byte aligned src: two (a fill of the tile flags, then one pass whose
 * workgroups look back over the totals their predecessors publish).  Library
 * workspace per stream.
 * n == 0 is a no-op.  Errors: EINVAL, EDTYPE, EALIGN, EOVERLAP, ENOMEM, EHIP.
 */
int scan_sum(const void *src, int64_t n, void *out, int dtype, int exclusive, void *stream);

/* Bound on each wait of the one-pass integer scan: a workgroup that has polled
 * a window of 64 predecessor tiles `polls` times while a nearer one has still
 * published nothing stops waiting and sums that tile's elements itself (the
 * decoupled look-back's waits end anyway, since a tile waits only on tiles
 * taken earlier; the bound only caps how long).  Results never depend on it:
 * integer sums are exact in any order.  Process-wide; applies to launches
 * issued after the call.  Default 2^18; 0 or 1 computes at once.  Returns the
 * previous bound. */
uint32_t xtr_scan_lookback_bound(uint32_t polls);

/* ------------------------------------------------------------------------
 * Histograms: the third case study the thesis's conclusion names (after the
 * reduction and the prefix sum).  The thesis's system has no atomics
 * (Section 1.2); these kernels use them.
 *
 * counts: device int64_t[nbins] (8-byte aligned; must not overlap src),
 * fully overwritten with exact counts (deterministic).  src: device array of
 * n elements, aligned to its element size.  1 <= nbins <= XTR_HIST_MAX_BINS.
 * Up to 16384 bins the elements are counted in per-workgroup LDS histograms
 * whose rows are summed by a second launch (library workspace per stream);
 * more bins are counted with 64-bit device atomics into counts (zero-filled
 * first).  n == 0 zero-fills counts.  Asynchronous on `stream`.
 * Errors: EINVAL (n < 0, nbins or width out of range, a bad float range,
 * null pointer), EDTYPE, EALIGN, EOVERLAP, ENOMEM, EHIP.
 */
#define XTR_HIST_MAX_BINS ((int64_t)1 << 28)

/* Integer bins: counts[b] = number of x with lo + b*width <= x < lo + (b+1)*width
 * (exact; elements outside [lo, lo + nbins*width) are not counted).
 * dtype: I32, I64, U8 or U16.  width >= 1. */
int histogram_int(const void *src, int64_t n, int dtype, int64_t lo, int64_t width,
                  int64_t nbins, int64_t *counts, void *stream);

/* Float bins over [lo, hi): x is decoded exactly to fp64 and counted in bin
 * floor((x - lo) * s), s = nbins / (hi - lo), capped at nbins - 1, with every
 * operation an fp64 operation rounded to nearest.  x < lo, x >= hi and NaN are
 * not counted.  lo, hi, hi - lo and s must be finite, lo < hi.
 * dtype: F32, F16, BF16 or F8E4M3. */
int histogram_float(const void *src, int64_t n, int dtype, double lo, double hi,
                    int64_t nbins, int64_t *counts, void *stream);

/* ------------------------------------------------------------------------
 * matmul -- matrix multiplication on the matrix cores, the case study the
 * thesis's conclusion says was started (Chapter 9):
 *
 *   C[i][j] = sum over k of A[i][k] * B[k][j],   0 <= i < M, 0 <= j < N
 *
 * a: device, row-major M x K (leading dimension lda >= K).
 * b: device, row-major K x N (ldb >= N); with trans_b != 0, B is given as its
 *    N x K transpose, row-major (ldb >= K).
 * c: device float[M x N], row-major (ldc >= N), fully overwritten; must not
 *    overlap a or b.
 * dtype: BF16 or F16 (both operands).  Products are exact in fp32 and are
 * summed in fp32 by the matrix cores in k order, so |C - exact| <=
 * K * 2^-24 * sum_k |A[i][k] B[k][j]|.  K == 0 gives C = 0; M == 0 or N == 0
 * is a no-op.  With trans_b == 0 the library first transposes B into its
 * workspace (per stream) with tpose(); with trans_b != 0 the product runs in
 * one launch.  Asynchronous on `stream`.
 * Errors: EINVAL, EDTYPE, EALIGN (a, b not 2-byte or c not 4-byte aligned),
 * EOVERLAP, ENOMEM, EHIP.
 */
int matmul(const void *a, const void *b, float *c, int64_t M, int64_t N, int64_t K,
           int64_t lda, int64_t ldb, int64_t ldc, int trans_b, int dtype, void *stream);

/* ------------------------------------------------------------------------
 * Host buffers: the end-to-end form of the paper's host code (Listing 3.6:
 * copy in, kernel, copy out), for data that lives in host memory.
 *
 * src / dst / out are HOST pointers, page-locked (hipHostMalloc, or torch's
 * pin_memory) or pageable.  The calls are synchronous: they return when the
 * result is in host memory.  The data moves in panels of about 32 MiB
 * through library-owned device buffers on three internal streams (copy in,
 * kernel, copy out), so the copies of one panel overlap the kernel of the
 * next; page-locked buffers are copied by DMA directly, pageable ones pass
 * through the library's pinned staging (one host memcpy per panel).  The
 * internal streams have default priority and are ordered only against each
 * other, not against caller streams.  Calls on one device are serialized.
 */

/* Host transpose: as tpose(), with src and dst in host memory.
 * Errors: as tpose(), plus ENOMEM and EHIP. */
int xtr_tpose_host(const void *src, void *dst, int64_t rows, int64_t cols,
                   int64_t ld_src, int64_t ld_dst, int dtype);

/* Host sum: as reduce_sum(), with src and *out (double or int64_t) in host
 * memory.  The result equals reduce_sum() of the same n values at a
 * 16-byte-aligned device address, bit for bit.
 * Errors: as reduce_sum(), plus EHIP. */
int xtr_reduce_sum_host(const void *src, int64_t n, void *out, int dtype);

/* ------------------------------------------------------------------------
 * Batch plans: a batch whose buffers and shapes repeat (a serving slot, a
 * training step) is validated and uploaded once; each run then only launches
 * kernels, with no host allocation, copy or memset, so a run can be captured
 * in a hipGraph and replayed.  The plan owns its device job table (with the
 * slot counters of the transposes' dynamic order, which every run leaves at
 * zero, and, for sums, a zeroed workspace that every run leaves reusable);
 * the caller owns the data buffers, which must stay valid for the plan's
 * lifetime.  Runs of one plan must not overlap in time (they share its
 * counters and workspace).
 */
typedef struct xtr_tpose_plan xtr_tpose_plan;

/* Validates and uploads descs[0..count) (host array, as tpose_batched); the
 * upload is synchronous on `stream`.  *plan = NULL on error.
 * Errors: as tpose_batched, plus ENOMEM. */
int xtr_tpose_plan_create(const xtr_tpose_desc *descs, int64_t count, void *stream,
                          xtr_tpose_plan **plan);
/* Enqueues the plan's persistent launches on `stream` (kernels only). */
int xtr_tpose_plan_run(const xtr_tpose_plan *plan, void *stream);
int xtr_tpose_plan_destroy(xtr_tpose_plan *plan);

typedef struct xtr_sum_plan xtr_sum_plan;

/* A plan for reduce_sum_batched(srcs, ns, count, out, dtype); same arguments
 * and errors, plus ENOMEM.  The setup is synchronous on `stream`. */
int xtr_sum_plan_create(const void *const *srcs, const int64_t *ns, int64_t count, int dtype,
                        void *out, void *stream, xtr_sum_plan **plan);
/* Enqueues the plan's reduction on `stream` (one kernel, no other work). */
int xtr_sum_plan_run(const xtr_sum_plan *plan, void *stream);
int xtr_sum_plan_destroy(xtr_sum_plan *plan);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching (the serving workload;
 * the paper has no serving).  A server owns a thread, `nstreams` compute
 * streams and one copy stream, all of default priority, on the device current
 * at creation.  Each job names a device input and output the caller owns
 * (they must stay valid, and the input ready, until the job completes); the
 * loop allocates nothing per job.  A job becomes visible to the loop at its
 * arrival time; the loop admits arrived jobs in FIFO order while the
 * in-flight bytes (input + output of every admitted, unfinished job) stay
 * within budget_bytes, and launches the jobs admitted in one pass as units,
 * each unit with a completion event: with batching, jobs under
 * small_job_bytes share one unit per kind (one tpose_batched /
 * reduce_sum_batched_scatter launch per element size or dtype; a kind with
 * one job in the unit takes tpose / reduce_sum) and larger jobs are units of
 * their own unless jobs are left waiting; without batching, one launch per
 * job.  Results are the entry points' own (tpose, reduce_sum), bit for bit
 * whatever the mix.
 *
 * Host-resident inputs (the host side of Listing 3.6 inside the loop): a job
 * with host_src != NULL has its input in page-locked host memory at host_src;
 * when the job is launched the loop copies it to `src` (a device buffer of the
 * input's size, owned by the caller) on the copy stream, and the job's unit
 * waits for that copy only, so copies overlap the kernels of other units.
 * Outputs stay in device memory.
 */
typedef struct {
    int32_t kind;        /* 0: transpose (tpose of a contiguous rows x cols matrix),
                            1: sum (reduce_sum of n elements)                       */
    int32_t dtype;
    const void *src;     /* device input (with host_src: where it is copied to)      */
    void *dst;           /* device output: cols x rows matrix, or the sum's result  */
    int64_t rows, cols;  /* transpose                                               */
    int64_t n;           /* sum                                                     */
    int64_t arrival_ns;  /* arrival on xtr_server_clock_ns(); < 0: at submission.
                            Arrivals are non-decreasing in submission order (a time
                            before the previous job's is raised to it).             */
    const void *host_src;  /* NULL, or the input in page-locked host memory         */
} xtr_job;

typedef struct {
    int32_t nstreams;         /* 1..8                                              */
    int32_t batching;         /* 1: continuous batching; 0: one launch per job     */
    int64_t budget_bytes;     /* HBM budget of the in-flight jobs                  */
    int64_t small_job_bytes;  /* jobs below this share launch units                */
    int32_t graphs;           /* 1: each unit's launches are captured into a graph
                                 and run from a cached executable graph of the same
                                 shape (same kernels and grids, same stream), given
                                 the unit's kernel arguments; a shared unit then
                                 holds at most 24 jobs of a kind (job tables in the
                                 kernel arguments, so the graph has kernel nodes
                                 only).  A unit that cannot be captured so runs
                                 eagerly.                                          */
    int32_t big_lane;         /* 1 (with nstreams >= 2): every unit holding a job of
                                 at least small_job_bytes runs on stream 0, in
                                 admission order; the others take streams 1..K-1.  */
    int64_t _reserved[3];
} xtr_server_config;

typedef struct {
    int64_t submitted, completed, failed, launches, units, max_inflight_bytes;
    int64_t graph_launches;   /* units run from an executable graph               */
    int64_t graph_builds;     /* executable graphs instantiated                   */
    int64_t host_copies;      /* host-to-device input copies                      */
    int64_t _reserved;
} xtr_server_stats;

typedef struct xtr_server xtr_server;

/* The loop's clock: steady host time in nanoseconds. */
int64_t xtr_server_clock_ns(void);
/* Starts a server on the current device.  Errors: EINVAL, ENOMEM, EHIP. */
int xtr_server_create(const xtr_server_config *cfg, xtr_server **srv);
/* Hands jobs[0..count) (host array, copied) to the loop; *first_id (may be
 * NULL) receives the id of jobs[0], ids being consecutive in submission
 * order.  Validated first: EINVAL / EDTYPE for a bad job, EBUDGET for a job
 * larger than the budget; then nothing is submitted. */
int xtr_server_submit(xtr_server *srv, const xtr_job *jobs, int64_t count, int64_t *first_id);
/* Waits until every submitted job has completed (timeout_ms < 0: no limit).
 * EHIP if some job's launch failed (its completion time is -2). */
int xtr_server_drain(xtr_server *srv, int64_t timeout_ms);
/* Arrival and completion times (ns, server clock; completion -1 while
 * pending, -2 if its launch failed) of jobs [first, first + count); either
 * output array may be NULL. */
int xtr_server_times(xtr_server *srv, int64_t first, int64_t count, int64_t *arrival_ns,
                     int64_t *done_ns);
int xtr_server_get_stats(xtr_server *srv, xtr_server_stats *stats);
/* Completes every submitted job, then stops the loop and frees the server. */
int xtr_server_destroy(xtr_server *srv);

/* ------------------------------------------------------------------------
 * Launch configuration (the autotuner's interface).  The settings change how
 * the work is scheduled, never the result: transposes are bit copies, and
 * the reduction's chunking and combine order do not depend on them.
 */
typedef struct {
    int32_t nt_load;        /* 1: nontemporal (streaming) loads of src rows that   */
                            /*    start on 128-byte lines (base and pitch)         */
    int32_t nt_store;       /* 1: nontemporal stores of such dst rows              */
    int32_t xcd;            /* 1: each XCD takes a contiguous range of tiles (per  */
                            /*    round of a persistent launch); 2: a persistent   */
                            /*    launch of at least 8 workgroups gives each XCD a */
                            /*    contiguous eighth of the whole launch order; 3:  */
                            /*    chunks of the order dealt to the XCDs in turn, a */
                            /*    workgroup taking the next free slot of its XCD's */
                            /*    chunks from a counter in the batch table         */
                            /*    (batches with a table; others take 3 as 1);      */
                            /*    0..3, single launches take 2 and 3 as 1          */
    int32_t group;          /* tile rows per band of the launch order, 1..64       */
    int32_t blocks_per_cu;  /* 0: one workgroup per tile; k in 1..64: persistent   */
    int32_t nt_store_shared;/* 1: nontemporal stores of dst rows that do not start */
                            /*    on lines (neighbouring tiles share edge lines)   */
    int32_t nt_load_shared; /* 1: nontemporal loads of such src rows               */
    int32_t tile;           /* tile geometry of single transposes of 2- to 8-byte   */
                            /*    elements with line-aligned rows: 0 = 256 x 256   */
                            /*    bytes, 1 = 512-byte src row segments, 2 = 512-   */
                            /*    byte dst row segments, 3 = 512 x 512 bytes, 4 =   */
                            /*    1 KiB dst row segments of 256-byte src ones (3   */
                            /*    and 4: 4- and 8-byte elements; others take 0)    */
    int32_t tile_shared;    /* the same for rows that do not start on lines (in the */
                            /*    batched class: the geometry of every batch job)   */
    int32_t run;            /* batched class: tiles a workgroup takes one after     */
                            /*    another in the launch order (0 or 1: one), so    */
                            /*    neighbouring tiles, which share the cache lines   */
                            /*    at their edges, meet in one CU; 0..64             */
    int32_t narrow;         /* batched class: 1 = every job whose pieces could be  */
                            /*    wider takes the narrowest piece of its element  */
                            /*    size (4 bytes; 8 for 8-byte elements), so the   */
                            /*    jobs of one element size share one launch; 0..1  */
    int32_t wide_min;       /* single class: a matrix of fewer than wide_min       */
                            /*    256 x 256-byte tiles per CU takes 256 x 256      */
                            /*    bytes whatever tile / tile_shared say (wider     */
                            /*    tiles leave CUs idle there); 0..1024             */
} xtr_tpose_config;

/* Shape classes of the launch configurations: single calls (tpose,
 * reduce_sum and their _ws / host / no-allocation forms) and batched ones
 * (tpose_batched and its plans, reduce_sum_batched(_scatter), sum plans,
 * reduce_sum_segmented).  Each class has its own tuned settings. */
enum { XTR_SHAPE_SINGLE = 0, XTR_SHAPE_BATCHED = 1 };

/* Current / new configuration of tpose for one element size (1, 2, 4, 8) and
 * shape class.  In the batched class blocks_per_cu caps the workgroups of a
 * group's persistent launch per CU (0: as many as are resident at once).
 * Process-wide; not synchronized with launches in flight on other threads.
 * Errors: EINVAL. */
int xtr_tpose_get_class_config(int elem_bytes, int shape_class, xtr_tpose_config *cfg);
int xtr_tpose_set_class_config(int elem_bytes, int shape_class, const xtr_tpose_config *cfg);
/* The single-call class; set applies to every class. */
int xtr_tpose_get_config(int elem_bytes, xtr_tpose_config *cfg);
int xtr_tpose_set_config(int elem_bytes, const xtr_tpose_config *cfg);

typedef struct {
    int32_t nt_load;        /* 1: nontemporal (streaming) 16-byte loads            */
    int32_t split_chunks;   /* single ranges of >= split_chunks chunks (and > 1):   */
                            /*    workgroups store plain per-chunk partials and     */
                            /*    small follow-up kernels add them level by level;  */
                            /*    smaller ranges (or 0 = always) combine in-kernel  */
                            /*    through atomic tickets.  Same result either way.  */
    int32_t seg_fused;      /* segmented sums: 1 = the chunked segments and the     */
                            /*    small ones in one launch (each workgroup takes    */
                            /*    chunks first, then its waves take small           */
                            /*    segments); 0 = two launches.  Same result.        */
    int32_t seg_streams;    /* segmented sums, two launches: 1 = the small          */
                            /*    segments run on a library-owned second stream     */
                            /*    while the chunks run on the caller's (the call    */
                            /*    still completes in the caller's stream order)     */
    int32_t seg_small_per_cu; /* workgroups per CU of the small-segment launch     */
                            /*    (0: as many as are resident)                      */
    int32_t seg_chunk_per_cu; /* the same for the chunk launch                     */
    int32_t seg_over;       /* segmented launches: grids of this many times the    */
                            /*    resident workgroups (0 or 1: the resident ones;  */
                            /*    up to 16), the others starting as earlier ones   */
                            /*    finish, so the dispatcher balances the work      */
    int32_t _reserved[1];
} xtr_reduce_config;

/* Current / new configuration of the sums for one dtype and shape class
 * (split_chunks applies to single ranges only).  Errors: EINVAL. */
int xtr_reduce_get_class_config(int dtype, int shape_class, xtr_reduce_config *cfg);
int xtr_reduce_set_class_config(int dtype, int shape_class, const xtr_reduce_config *cfg);
/* The single-call class; set applies to every class. */
int xtr_reduce_get_config(int dtype, xtr_reduce_config *cfg);
int xtr_reduce_set_config(int dtype, const xtr_reduce_config *cfg);

/* ------------------------------------------------------------------------
 * Misc.
 */
/* Plain device-to-device copy of nbytes (16-byte vectors when src, dst and
 * nbytes are 16-byte aligned, bytes otherwise).  It is the reference for the
 * achievable HBM bandwidth (the effective-bandwidth convention of Section 7.1
 * applied to a copy) and for scaling HBM byte counters.
 * Errors: EINVAL (null), EOVERLAP. */
int xtr_copy(void *dst, const void *src, size_t nbytes, void *stream);

/* Thread-local message describing the last nonzero return on this thread. */
const char *xtr_last_error(void);

/* Element size of a dtype in bytes, 0 if unknown. */
int xtr_elem_bytes(int dtype);

/* Library version, (major << 16) | minor. */
int xtr_version(void);

/* Frees the library's workspaces and staging buffers (the caller must have
 * synchronized every stream that used them). */
int xtr_release(void);

#ifdef __cplusplus
}
#endif
#endif /* XTR_H */
