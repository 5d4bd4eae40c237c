// Matrix multiplication for gfx950 on the matrix cores (MFMA): the case study
// the thesis's conclusion says was started (its CPU transformations done, no
// GPU code yet).  The thesis's system has no tensor-core instructions
// (Section 1.2); this is the first path here that uses them.
//
// What is computed: C[i][j] = sum over k of A[i][k] * B[k][j], C in fp32
// (M x N, leading dimension ldc), A row-major M x K (lda), B row-major K x N
// (ldb) or, with trans_b, given as its N x K transpose Bt (ldb).  Inputs are
// bf16 or fp16; every product is exact in fp32 and the products are summed in
// fp32 by the matrix cores (32x32x16 MFMA blocks, in k order).
//
// How:
//   * The kernels multiply A by Bt: both operands are k-contiguous, so every
//     lane's MFMA fragment (8 consecutive k of one row) is one 16-byte LDS
//     read.  A row-major B is first transposed into a workspace with the
//     library's own transpose (the thesis's other case study).
//   * Products whose 256 x 256 tiles fill the GPU (k_matmul_deep): a
//     workgroup of 512 threads (8 waves, 2 x 4, two per SIMD) owns a 256 x 256
//     tile of C, a wave 128 x 64 = 4 x 2 MFMA blocks of 32 x 32 (128 fp32
//     accumulators per lane).  Operands go straight from global memory into LDS (no
//     staging registers) through four stages of k blocks of 32, three blocks
//     ahead of the MFMAs; an explicit schedule interleaves the MFMAs with the
//     loads and the fragment reads.
//   * Smaller products and operands whose rows are not 16-byte aligned
//     (k_matmul): 128 x 128 tiles, a wave 64 x 64; k blocks of 64 staged
//     through registers into two LDS buffers whose rows are padded to 144
//     bytes, so the 16-byte fragment reads of 16 lanes hit 16 bank groups.
//   * Operand chunks outside the matrices are read from a zero chunk, so no
//     load is predicated and no select waits for a load.
//   * Tiles are numbered so that the workgroups one XCD runs (the hardware
//     deals workgroups to the 8 XCDs in turn) are neighbours in groups of 4
//     tile rows, sharing operand tiles in that XCD's L2.
#include "common.hpp"

namespace xtr {
namespace {

constexpr int MM_NT = 256;          // threads per workgroup
constexpr int BK = 64;              // k per LDS block
constexpr int LROW = BK + 8;        // LDS row in elements (144 bytes)
constexpr int GROUP_M = 4;          // tile rows per group of the tile order
constexpr int NXCD = 8;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t mu32x4 __attribute__((ext_vector_type(4)));

template <int DT> __device__ __forceinline__ f32x16 mfma(const mu32x4 &a, const mu32x4 &b,
                                                         const f32x16 &c) {
    if constexpr (DT == XTR_BF16)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}

// 16 zero bytes: the source of every operand chunk outside the matrix, so that
// edge chunks need no select after their load (which would wait for it).
__device__ __attribute__((aligned(16))) uint32_t g_mm_zero[4];

// Chunk q (0..Q-1) of this thread in a (32 Q) x 64 operand block: row = c / 8,
// 8-element column chunk = c % 8, c = t + 256 q.
// VEC: rows are 16-byte aligned and K % 8 == 0, so a chunk is one 16-byte load
// (all or nothing); otherwise element by element.  Out-of-range elements are 0.
template <bool VEC, int Q>
__device__ __forceinline__ void load_block(const uint16_t *__restrict__ p, int64_t ld,
                                           int64_t rows_left, int64_t k0, int64_t K, int t,
                                           mu32x4 (&r)[Q]) {
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int c = t + MM_NT * q;
        const int row = c >> 3;
        const int64_t k = k0 + (c & 7) * 8;
        if constexpr (VEC) {
            // branch-free: a chunk outside the operand loads the zero chunk
            const bool ok = row < rows_left && k < K;
            const mu32x4 *src = ok ? reinterpret_cast<const mu32x4 *>(p + (int64_t)row * ld + k)
                                   : reinterpret_cast<const mu32x4 *>(g_mm_zero);
            r[q] = *src;
        } else {
            uint32_t w[4] = {0, 0, 0, 0};
            if (row < rows_left) {
                const uint16_t *s = p + (int64_t)row * ld;
#pragma unroll
                for (int e = 0; e < 8; e++)
                    if (k + e < K) w[e >> 1] |= (uint32_t)s[k + e] << (16 * (e & 1));
            }
            r[q] = mu32x4{w[0], w[1], w[2], w[3]};
        }
    }
}

template <int Q>
__device__ __forceinline__ void store_block(uint16_t *lds, int t, const mu32x4 (&r)[Q]) {
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int c = t + MM_NT * q;
        *reinterpret_cast<mu32x4 *>(lds + (c >> 3) * LROW + (c & 7) * 8) = r[q];
    }
}

// The tile (tm, tn) workgroup b computes.
__device__ __forceinline__ void tile_of(int64_t b, int64_t nb, int64_t tiles_m, int64_t tiles_n,
                                        int64_t &tm, int64_t &tn) {
    // workgroups b, b + 8, b + 16, ... run on one XCD: give them consecutive ids
    int64_t id = b;
    if (nb % NXCD == 0) id = (b % NXCD) * (nb / NXCD) + b / NXCD;
    // groups of GROUP_M tile rows, column-major inside a group
    const int64_t per_group = (int64_t)GROUP_M * tiles_n;
    const int64_t g = id / per_group;
    const int64_t first = g * GROUP_M;
    const int64_t gm = (tiles_m - first) < GROUP_M ? (tiles_m - first) : GROUP_M;
    const int64_t in = id - g * per_group;
    tm = first + in % gm;
    tn = in / gm;
}

// One workgroup: 2 x 2 waves, each owning TM x TN MFMA blocks of 32 x 32, so
// the workgroup tile is BM x BN = 64 TM x 64 TN.
template <int DT, bool VEC, int TM, int TN>
__global__ __launch_bounds__(MM_NT) void k_matmul(const uint16_t *__restrict__ A,
                                                  const uint16_t *__restrict__ Bt,
                                                  float *__restrict__ C, int64_t M, int64_t N,
                                                  int64_t K, int64_t lda, int64_t ldb,
                                                  int64_t ldc, int64_t tiles_m, int64_t tiles_n) {
    constexpr int BM = 64 * TM, BN = 64 * TN, QA = BM / 32, QB = BN / 32;
    __shared__ __attribute__((aligned(16))) uint16_t sa[2][BM * LROW];
    __shared__ __attribute__((aligned(16))) uint16_t sb[2][BN * LROW];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    int64_t tm, tn;
    tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const uint16_t *pa = A + m0 * lda;
    const uint16_t *pb = Bt + n0 * ldb;
    const int64_t ma = M - m0, nbl = N - n0;

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) acc[i][j] = f32x16{};

    const int64_t nk = (K + BK - 1) / BK;
    mu32x4 ra[QA], rb[QB];
    if (nk > 0) {
        load_block<VEC, QA>(pa, lda, ma, 0, K, t, ra);
        load_block<VEC, QB>(pb, ldb, nbl, 0, K, t, rb);
        store_block<QA>(sa[0], t, ra);
        store_block<QB>(sb[0], t, rb);
    }
    __syncthreads();
    // lane l's fragment: row l % 32 of a 32-row block, k chunk l / 32 of a 16-k step
    const int fr = l & 31, fk = (l >> 5) * 8;
    for (int64_t kb = 0; kb < nk; kb++) {
        const int cur = kb & 1;
        // the block after this one (past the end: zero chunks, into the
        // buffer nobody reads any more)
        load_block<VEC, QA>(pa, lda, ma, (kb + 1) * BK, K, t, ra);
        load_block<VEC, QB>(pb, ldb, nbl, (kb + 1) * BK, K, t, rb);
        const uint16_t *la = sa[cur] + (wr * 32 * TM + fr) * LROW + fk;
        const uint16_t *lb = sb[cur] + (wc * 32 * TN + fr) * LROW + fk;
        // fragments of step ks + 1 are read while the MFMAs of step ks run; the
        // next block's LDS stores go to the other buffer (last read before the
        // previous barrier) in the second half
        mu32x4 fa[2][TM], fb[2][TN];
#pragma unroll
        for (int i = 0; i < TM; i++) fa[0][i] = *reinterpret_cast<const mu32x4 *>(la + i * 32 * LROW);
#pragma unroll
        for (int j = 0; j < TN; j++) fb[0][j] = *reinterpret_cast<const mu32x4 *>(lb + j * 32 * LROW);
#pragma unroll
        for (int ks = 0; ks < BK / 16; ks++) {
            const int c = ks & 1;
            if (ks + 1 < BK / 16) {
#pragma unroll
                for (int i = 0; i < TM; i++)
                    fa[c ^ 1][i] =
                        *reinterpret_cast<const mu32x4 *>(la + i * 32 * LROW + (ks + 1) * 16);
#pragma unroll
                for (int j = 0; j < TN; j++)
                    fb[c ^ 1][j] =
                        *reinterpret_cast<const mu32x4 *>(lb + j * 32 * LROW + (ks + 1) * 16);
            }
#pragma unroll
            for (int i = 0; i < TM; i++)
#pragma unroll
                for (int j = 0; j < TN; j++) acc[i][j] = mfma<DT>(fa[c][i], fb[c][j], acc[i][j]);
            if (ks == 2) store_block<QA>(sa[cur ^ 1], t, ra);
            if (ks == 3) store_block<QB>(sb[cur ^ 1], t, rb);
        }
        __syncthreads();
    }
    // accumulator v of block (i, j): row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) {
            const int64_t col = n0 + wc * 32 * TN + j * 32 + (l & 31);
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int64_t row =
                    m0 + wr * 32 * TM + i * 32 + 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
                if (row < M && col < N) C[row * ldc + col] = acc[i][j][v];
            }
        }
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void global_void;

// The large-tile kernel with direct global -> LDS loads: each load instruction
// moves 64 lanes x 16 bytes from global memory straight into 1 KiB of LDS (8
// rows of the 128-byte k block), with no register staging and no LDS store
// instructions.  Rows are not padded; instead chunk c of row r sits in slot
// c ^ ((r / 2) % 8).  Two 128-byte rows span the 64 banks, so the 16 lanes an
// LDS pass serves (16 consecutive rows, one chunk) hit 16 different 16-byte
// bank groups: even rows the first 8, odd rows the other 8, and within each
// parity 8 different slots.  Lane i of a load instruction fills slot i % 8 of
// row i / 8 of its 8-row group and fetches the chunk that belongs there.
// ---------------------------------------------------------------- deep pipeline
// The large-tile kernel with four LDS stages of k blocks of 32: the loads of
// block kb + 3 are issued while block kb is multiplied, so each load has three
// blocks of MFMA work (about 3000 cycles) to arrive, against one in the
// two-stage form.  A stage holds 256 rows x 64 bytes per operand; chunk c of
// row r sits in slot c ^ ((r / 4) % 4), so the 16 lanes of an LDS pass (16
// consecutive rows, one chunk) hit 16 different 16-byte bank groups.
constexpr int DBK = 32;
constexpr int MM_DEEP_WAVES = 8;

// NW = 8 waves per workgroup: 2 x 4 waves of 128 x 64, two per SIMD, so one
// wave's MFMAs cover the other's waits (6% faster at 8192^3 than 2 x 2 waves
// of 128 x 128, one per SIMD, despite 1.5x the LDS fragment reads); WC waves
// along N, TN MFMA blocks of 32 columns per wave.
template <int NW> struct DeepGeo {
    static constexpr int WC = NW / 2, TN = 8 / WC, QPW = 16 / NW;
};

template <int DT, int NW>
__device__ __forceinline__ void deep_issue(const uint16_t *pa, const uint16_t *pb, int64_t lda,
                                           int64_t ldb, int64_t ma, int64_t nbl, int64_t kb,
                                           int64_t K, int w, int lrow, int lchunk, uint16_t *ya,
                                           uint16_t *yb) {
    const int64_t k = kb * DBK + lchunk * 8;
#pragma unroll
    for (int q = 0; q < DeepGeo<NW>::QPW; q++) {
        const int g = w * DeepGeo<NW>::QPW + q;   // 16-row group of this load instruction
        const int row = g * 16 + lrow;
        const void *ga = (row < ma && k < K) ? (const void *)(pa + (int64_t)row * lda + k)
                                             : (const void *)g_mm_zero;
        __builtin_amdgcn_global_load_lds((global_void *)ga, (lds_void *)(ya + g * 16 * DBK), 16,
                                         0, 0);
        const void *gb = (row < nbl && k < K) ? (const void *)(pb + (int64_t)row * ldb + k)
                                              : (const void *)g_mm_zero;
        __builtin_amdgcn_global_load_lds((global_void *)gb, (lds_void *)(yb + g * 16 * DBK), 16,
                                         0, 0);
    }
}

// One step: wait for block kb (this wave's loads of the two blocks after it may
// still fly), barrier, issue block kb + 3 into the stage block kb - 1 used,
// multiply block kb.
template <int DT, int NW>
__device__ __forceinline__ void deep_step(f32x16 (&acc)[4][DeepGeo<NW>::TN], const uint16_t *xa,
                                          const uint16_t *xb, uint16_t *ya, uint16_t *yb,
                                          const uint16_t *pa, const uint16_t *pb, int64_t lda,
                                          int64_t ldb, int64_t ma, int64_t nbl, int64_t kb,
                                          int64_t K, int w, int lrow, int lchunk, int wr, int wc,
                                          int fr, int fh, int sw) {
    constexpr int TN = DeepGeo<NW>::TN;
    // this wave's loads of block kb are in LDS (those of kb + 1 and kb + 2 may
    // still fly); the barrier then makes every wave's block kb visible.  Written
    // as one statement: a plain __syncthreads() would wait for every load.
    static_assert(NW == 8, "the wait count and the schedule below are for 8 waves");
    asm volatile("s_waitcnt vmcnt(8)\n\ts_barrier" ::: "memory");
    deep_issue<DT, NW>(pa, pb, lda, ldb, ma, nbl, kb + 3, K, w, lrow, lchunk, ya, yb);
    const uint16_t *la = xa + (wr * 128 + fr) * DBK;
    const uint16_t *lb = xb + (wc * 32 * TN + fr) * DBK;
    mu32x4 fa[2][4], fb[2][TN];
#pragma unroll
    for (int ks = 0; ks < 2; ks++) {
        const int slot = ((2 * ks + fh) ^ sw) << 3;
#pragma unroll
        for (int i = 0; i < 4; i++)
            fa[ks][i] = *reinterpret_cast<const mu32x4 *>(la + i * 32 * DBK + slot);
#pragma unroll
        for (int j = 0; j < TN; j++)
            fb[ks][j] = *reinterpret_cast<const mu32x4 *>(lb + j * 32 * DBK + slot);
    }
#pragma unroll
    for (int ks = 0; ks < 2; ks++)
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < TN; j++) acc[i][j] = mfma<DT>(fa[ks][i], fb[ks][j], acc[i][j]);
    // order: step 0's fragments; its MFMAs with the loads and step 1's
    // fragments; step 1's MFMAs
    __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
}

template <int DT, int NW>
__global__ __launch_bounds__(64 * NW) void k_matmul_deep(const uint16_t *__restrict__ A,
                                                         const uint16_t *__restrict__ Bt,
                                                         float *__restrict__ C, int64_t M,
                                                         int64_t N, int64_t K, int64_t lda,
                                                         int64_t ldb, int64_t ldc,
                                                         int64_t tiles_m, int64_t tiles_n) {
    constexpr int BM = 256, BN = 256, WC = DeepGeo<NW>::WC, TN = DeepGeo<NW>::TN;
    __shared__ __attribute__((aligned(1024))) uint16_t sa0[BM * DBK];
    __shared__ __attribute__((aligned(1024))) uint16_t sb0[BN * DBK];
    __shared__ __attribute__((aligned(1024))) uint16_t sa1[BM * DBK];
    __shared__ __attribute__((aligned(1024))) uint16_t sb1[BN * DBK];
    __shared__ __attribute__((aligned(1024))) uint16_t sa2[BM * DBK];
    __shared__ __attribute__((aligned(1024))) uint16_t sb2[BN * DBK];
    __shared__ __attribute__((aligned(1024))) uint16_t sa3[BM * DBK];
    __shared__ __attribute__((aligned(1024))) uint16_t sb3[BN * DBK];
    const int t = threadIdx.x, l = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int wr = w / WC, wc = w % WC;
    int64_t tm, tn;
    tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const uint16_t *pa = A + m0 * lda;
    const uint16_t *pb = Bt + n0 * ldb;
    const int64_t ma = M - m0, nbl = N - n0;

    f32x16 acc[4][TN];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) acc[i][j] = f32x16{};

    // load lane l: row l / 4 of its 16-row group, slot l % 4, chunk
    // (l % 4) ^ ((row / 4) % 4) = (l % 4) ^ (l / 16)
    const int lrow = l >> 2, lchunk = (l & 3) ^ (l >> 4);
    // fragment lane l: row l % 32 of a 32-row block, chunk 2 ks + l / 32
    const int fr = l & 31, fh = l >> 5, sw = (fr >> 2) & 3;
    const int64_t nk = (K + DBK - 1) / DBK;
    deep_issue<DT, NW>(pa, pb, lda, ldb, ma, nbl, 0, K, w, lrow, lchunk, sa0, sb0);
    deep_issue<DT, NW>(pa, pb, lda, ldb, ma, nbl, 1, K, w, lrow, lchunk, sa1, sb1);
    deep_issue<DT, NW>(pa, pb, lda, ldb, ma, nbl, 2, K, w, lrow, lchunk, sa2, sb2);
#define XTR_DS(X, Y, KB)                                                                      \
    deep_step<DT, NW>(acc, sa##X, sb##X, sa##Y, sb##Y, pa, pb, lda, ldb, ma, nbl, KB, K, w,     \
                      lrow, lchunk, wr, wc, fr, fh, sw)
    for (int64_t kb = 0; kb < nk; kb += 4) {
        XTR_DS(0, 3, kb);
        if (kb + 1 < nk) XTR_DS(1, 0, kb + 1);
        if (kb + 2 < nk) XTR_DS(2, 1, kb + 2);
        if (kb + 3 < nk) XTR_DS(3, 2, kb + 3);
    }
#undef XTR_DS
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // no load may outlive the workgroup's LDS
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) {
            const int64_t col = n0 + wc * 32 * TN + j * 32 + (l & 31);
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int64_t row = m0 + wr * 128 + i * 32 + 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
                if (row < M && col < N) C[row * ldc + col] = acc[i][j][v];
            }
        }
}

int matmul_impl(const void *a, const void *b, float *c, int64_t M, int64_t N, int64_t K,
                int64_t lda, int64_t ldb, int64_t ldc, int trans_b, int dtype, hipStream_t st) {
    const char *who = "matmul";
    if (dtype != XTR_BF16 && dtype != XTR_F16)
        return fail(XTR_EDTYPE, "%s: dtype %d is not bf16 or fp16", who, dtype);
    if (M < 0 || N < 0 || K < 0) return fail(XTR_EINVAL, "%s: negative size", who);
    if (lda < K || ldc < N || ldb < (trans_b ? K : N))
        return fail(XTR_EINVAL, "%s: leading dimension smaller than its row", who);
    if (M == 0 || N == 0) return XTR_OK;
    if (!c || (K > 0 && (!a || !b))) return fail(XTR_EINVAL, "%s: null pointer", who);
    if ((uintptr_t)a % 2 || (uintptr_t)b % 2 || (uintptr_t)c % 4)
        return fail(XTR_EALIGN, "%s: pointer not aligned to its element", who);
    const uintptr_t c0 = (uintptr_t)c, c1 = c0 + (uintptr_t)((M - 1) * ldc + N) * 4;
    if (K > 0) {
        const uintptr_t a0 = (uintptr_t)a, a1 = a0 + (uintptr_t)((M - 1) * lda + K) * 2;
        const int64_t brows = trans_b ? N : K, bcols = trans_b ? K : N;
        const uintptr_t b0 = (uintptr_t)b, b1 = b0 + (uintptr_t)((brows - 1) * ldb + bcols) * 2;
        if ((a0 < c1 && c0 < a1) || (b0 < c1 && c0 < b1))
            return fail(XTR_EOVERLAP, "%s: C overlaps an operand", who);
    }
    const uint16_t *bt = static_cast<const uint16_t *>(b);
    int64_t ldbt = ldb;
    if (!trans_b && K > 0) {
        // Bt = B^T (N x K) in the workspace, rows padded to 8 elements
        ldbt = (K + 7) / 8 * 8;
        void *ws = nullptr;
        int rc = workspace(WS_MM, st, (size_t)N * (size_t)ldbt * 2, &ws);
        if (rc) return rc;
        rc = tpose(b, ws, K, N, ldb, ldbt, dtype, st);
        if (rc) return rc;
        bt = static_cast<const uint16_t *>(ws);
    }
    const bool vec = K % 8 == 0 && lda % 8 == 0 && ldbt % 8 == 0 && (uintptr_t)a % 16 == 0 &&
                     (uintptr_t)bt % 16 == 0;
    // 256 x 256 tiles (a wave owns 128 x 128: half the LDS reads per MFMA) once
    // they fill the GPU; 128 x 128 otherwise
    const int64_t big_tiles = ((M + 255) / 256) * ((N + 255) / 256);
    const bool big = vec && big_tiles >= cu_count();
    const int64_t bm = big ? 256 : 128;
    const int64_t tiles_m = (M + bm - 1) / bm, tiles_n = (N + bm - 1) / bm;
    const int64_t nb = tiles_m * tiles_n;
    if (nb > 0x7fffffff) return fail(XTR_EINVAL, "%s: too many tiles", who);
    const uint16_t *pa = static_cast<const uint16_t *>(a);
#define XTR_MM(D, V, T)                                                                       \
    hipLaunchKernelGGL((k_matmul<D, V, T, T>), dim3((unsigned)nb), dim3(MM_NT), 0, st, pa, bt, c, \
                       M, N, K, lda, ldbt, ldc, tiles_m, tiles_n)
    if (big) {
        constexpr int NW = MM_DEEP_WAVES;
        if (dtype == XTR_BF16)
            hipLaunchKernelGGL((k_matmul_deep<XTR_BF16, NW>), dim3((unsigned)nb), dim3(64 * NW), 0,
                               st, pa, bt, c, M, N, K, lda, ldbt, ldc, tiles_m, tiles_n);
        else
            hipLaunchKernelGGL((k_matmul_deep<XTR_F16, NW>), dim3((unsigned)nb), dim3(64 * NW), 0,
                               st, pa, bt, c, M, N, K, lda, ldbt, ldc, tiles_m, tiles_n);
    } else if (dtype == XTR_BF16) {
        if (vec) XTR_MM(XTR_BF16, true, 2);
        else XTR_MM(XTR_BF16, false, 2);
    } else {
        if (vec) XTR_MM(XTR_F16, true, 2);
        else XTR_MM(XTR_F16, false, 2);
    }
#undef XTR_MM
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

}  // namespace
}  // namespace xtr

extern "C" int matmul(const void *a, const void *b, float *c, int64_t M, int64_t N, int64_t K,
                      int64_t lda, int64_t ldb, int64_t ldc, int trans_b, int dtype,
                      void *stream) {
    return xtr::matmul_impl(a, b, c, M, N, K, lda, ldb, ldc, trans_b, dtype, (hipStream_t)stream);
}
