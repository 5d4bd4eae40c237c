// Histograms for gfx950: the third case study the thesis's conclusion names
// after the reduction and the prefix sum.  The thesis's system has no atomics
// (Section 1.2 lists them among the GPU features it leaves out); a histogram
// needs them, so this kernel is written directly against the hardware.
//
// What is computed, counts[b] for b in [0, nbins):
//   integers (int32, int64, uint8, uint16): the elements x with
//       lo + b*width <= x < lo + (b+1)*width          (exact integer arithmetic)
//   floats (fp32, fp16, bf16, fp8-e4m3fn): the elements x, decoded exactly to
//       fp64, with lo <= x < hi and floor((x - lo) * s) == b (capped at
//       nbins - 1), where s = nbins / (hi - lo) and every operation is an
//       fp64 operation rounded to nearest; NaN is never counted.
// The counts are exact 64-bit integers, so the result does not depend on the
// order of the work: it is deterministic and equal to any serial count.
//
// How (two launches):
//   1. k_hist: G workgroups of 1024 threads stream the input as 16-byte
//      vectors (grid-stride, four vectors in flight per thread) and count in
//      32-bit counters in the workgroup's LDS.  Up to 511 bins there are 32
//      copies of the histogram, interleaved bin-major, and thread t adds 1 to
//      copy t % 32 for every element, without a branch (elements outside the
//      range go to a spare bin): the 32 lanes of an LDS pass never share a
//      bank or a counter, whatever the data.  With more bins the copies
//      shrink to what 64 KiB holds and each thread adds runs of equal bins
//      within its vector (one atomic add per run).  At the end the workgroup
//      folds its copies into row g of a partial table in the workspace.  G
//      keeps every workgroup under 2^31 elements, so the 32-bit counters
//      cannot overflow.
//   2. k_hist_merge: one workgroup per 64 bins sums the G rows in 64 bits
//      and writes counts.
// More bins than one LDS histogram holds take the global path: counts is
// zero-filled and every run is added with a 64-bit device-scope atomic.
// fp8 inputs are counted per code (256 bins of the byte values), and the 256
// code counts are then added to the bins of their values.
#include "common.hpp"

#include <math.h>

#pragma clang fp contract(off)

namespace xtr {
namespace {

constexpr int HNT = 1024;                    // threads per workgroup (16 waves)
constexpr int HUNROLL = 4;                   // 16-byte vectors in flight per thread
constexpr int64_t LDS_WORDS = 16384;         // 64 KiB of 32-bit LDS counters per workgroup
constexpr int64_t WG_MAX_ELEMS = (int64_t)1 << 31;
constexpr int MERGE_NT = 1024;               // merge: 16 waves x 64 bins

// How an integer offset d = x - lo in [0, span) becomes its bin d / width.
// The *32 forms serve inputs of at most 32 bits with lo in the int32 range and
// span <= 2^32: x and lo are compared and subtracted as 32-bit values, biased
// by 2^31 so that unsigned order is signed order.
enum { BIN_FLOAT = 0, BIN_SHIFT = 1, BIN_MAGIC = 2, BIN_DIV = 3, BIN_SHIFT32 = 4, BIN_MAGIC32 = 5 };

typedef uint32_t hu32x4 __attribute__((ext_vector_type(4)));

struct HistArgs {
    int64_t nbins;
    int64_t head;          // elements before the first 16-byte boundary of src
    int64_t nvec;          // whole 16-byte vectors after the head
    int64_t n;
    // integer rule
    int64_t lo_i;
    uint64_t span_m1;      // min(width * nbins, 2^64) - 1
    uint64_t width;
    uint64_t magic;        // ceil(2^64 / width)      (BIN_MAGIC)
    int shift;             // log2(width)             (BIN_SHIFT, BIN_SHIFT32)
    uint32_t lo32;         // lo ^ 2^31, order-preserving 32-bit form  (BIN_*32)
    uint32_t span_m1_32;   // width * nbins - 1                        (BIN_*32)
    int rs;                // log2 of the LDS copies per bin
    // float rule
    double lo_f, hi_f, scale;
};

template <int DT> struct HistT;
template <> struct HistT<XTR_F32> { static constexpr int EB = 4; };
template <> struct HistT<XTR_F16> { static constexpr int EB = 2; };
template <> struct HistT<XTR_BF16> { static constexpr int EB = 2; };
template <> struct HistT<XTR_I32> { static constexpr int EB = 4; };
template <> struct HistT<XTR_I64> { static constexpr int EB = 8; };
template <> struct HistT<XTR_U8> { static constexpr int EB = 1; };
template <> struct HistT<XTR_U16> { static constexpr int EB = 2; };

// exact fp64 value of a float element given its raw bits (low EB*8 bits of r)
template <int DT> __device__ __forceinline__ double fdecode(uint32_t r) {
    if constexpr (DT == XTR_F32) return (double)__uint_as_float(r);
    else if constexpr (DT == XTR_BF16) return (double)__uint_as_float(r << 16);
    else if constexpr (DT == XTR_F16) return (double)(float)__builtin_bit_cast(_Float16, (uint16_t)r);
    else return (double)__builtin_amdgcn_cvt_pk_f32_fp8((int)r, false)[0];
}

// value of an integer element given its raw bits
template <int DT> __device__ __forceinline__ int64_t idecode(uint64_t r) {
    if constexpr (DT == XTR_I32) return (int64_t)(int32_t)(uint32_t)r;
    else if constexpr (DT == XTR_I64) return (int64_t)r;
    else if constexpr (DT == XTR_U8) return (int64_t)(r & 0xffu);
    else return (int64_t)(r & 0xffffu);
}

// The bin of the element with raw bits r when it is counted, else nbins (a
// spare bin that collects the elements outside the range and is never
// reported).  Only the 32-bit and float rules have this form; it lets the
// branch-free loop add 1 for every element.
template <int DT, int MODE>
__device__ __forceinline__ uint32_t bin_or_spare(uint64_t r, const HistArgs &a) {
    const uint32_t nb = (uint32_t)a.nbins;
    if constexpr (MODE == BIN_FLOAT) {
        const double x = fdecode<DT>((uint32_t)r);
        const bool ok = x >= a.lo_f && x < a.hi_f;                     // NaN fails both
        const double t = (x - a.lo_f) * a.scale;
        // t >= 0 when ok, so truncation is the floor
        const uint32_t b = (uint32_t)(int)t;
        return ok ? (b < nb - 1 ? b : nb - 1) : nb;
    } else {
        static_assert(MODE == BIN_SHIFT32 || MODE == BIN_MAGIC32, "32-bit integer rules only");
        const uint32_t ux = (uint32_t)(int32_t)idecode<DT>(r) ^ 0x80000000u;
        uint32_t d;
        const bool below = __builtin_sub_overflow(ux, a.lo32, &d);     // x < lo
        const bool ok = !below && d <= a.span_m1_32;
        uint32_t q;
        if constexpr (MODE == BIN_SHIFT32) {
            q = d >> a.shift;
        } else {
            const uint64_t p0 = (uint64_t)d * (uint32_t)a.magic;       // as in BIN_MAGIC
            const uint64_t p1 = (uint64_t)d * (uint32_t)(a.magic >> 32);
            q = (uint32_t)((p1 + (p0 >> 32)) >> 32);
        }
        return ok ? q : nb;
    }
}

// The bin of the element with raw bits r, or -1 when it is not counted.
template <int DT, int MODE>
__device__ __forceinline__ int bin_of(uint64_t r, const HistArgs &a) {
    if constexpr (MODE == BIN_FLOAT) {
        const double x = fdecode<DT>((uint32_t)r);
        if (!(x >= a.lo_f && x < a.hi_f)) return -1;               // NaN fails both
        const double t = (x - a.lo_f) * a.scale;
        const int b = (int)floor(t);
        return b < (int)a.nbins - 1 ? b : (int)a.nbins - 1;
    } else if constexpr (MODE == BIN_SHIFT32 || MODE == BIN_MAGIC32) {
        const uint32_t ux = (uint32_t)(int32_t)idecode<DT>(r) ^ 0x80000000u;
        uint32_t d;
        if (__builtin_sub_overflow(ux, a.lo32, &d)) return -1;    // x < lo
        if (d > a.span_m1_32) return -1;
        if constexpr (MODE == BIN_SHIFT32) {
            return (int)(d >> a.shift);
        } else {
            const uint64_t p0 = (uint64_t)d * (uint32_t)a.magic;   // as in BIN_MAGIC
            const uint64_t p1 = (uint64_t)d * (uint32_t)(a.magic >> 32);
            return (int)((p1 + (p0 >> 32)) >> 32);
        }
    } else {
        const int64_t x = idecode<DT>(r);
        if (x < a.lo_i) return -1;
        const uint64_t d = (uint64_t)x - (uint64_t)a.lo_i;        // exact: x - lo in [0, 2^64)
        if (d > a.span_m1) return -1;
        if constexpr (MODE == BIN_SHIFT) {
            return (int)(d >> a.shift);
        } else if constexpr (MODE == BIN_MAGIC) {
            // d < 2^32 and width <= 2^32: floor(d / width) = floor(d * c / 2^64) with
            // c = ceil(2^64 / width) (Lemire, Kaser and Kurz, "Faster remainder by direct
            // computation", 2019, Theorem 1 with F = 64, N = 32)
            const uint32_t d32 = (uint32_t)d;
            const uint64_t p0 = (uint64_t)d32 * (uint32_t)a.magic;
            const uint64_t p1 = (uint64_t)d32 * (uint32_t)(a.magic >> 32);
            return (int)((p1 + (p0 >> 32)) >> 32);
        } else {
            return (int)(d / a.width);
        }
    }
}

// Where the LDS counters live: R = 2^rs copies of the histogram, interleaved
// bin-major (counter (b, c) at word b * R + c); thread t adds to copy t % R.
// With R = 32 the 32 lanes an LDS pass serves hit 32 different banks whatever
// their bins, and no two of them share a counter.
template <bool GLOBAL> __device__ __forceinline__ void add_run(uint32_t *h, uint64_t *g, int b,
                                                               uint32_t c, const HistArgs &a,
                                                               uint32_t lr) {
    if constexpr (GLOBAL)
        __hip_atomic_fetch_add(g + b, (uint64_t)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_fetch_add(h + (((uint32_t)b << a.rs) | lr), c, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int EB> __device__ __forceinline__ uint64_t raw_of(const uint32_t (&w)[4], int i) {
    if constexpr (EB == 8) return (uint64_t)w[2 * i] | ((uint64_t)w[2 * i + 1] << 32);
    else if constexpr (EB == 4) return w[i];
    else if constexpr (EB == 2) return (w[i >> 1] >> (16 * (i & 1))) & 0xffffu;
    else return (w[i >> 2] >> (8 * (i & 3))) & 0xffu;
}

// Bins the V elements of one 16-byte vector.  RUNS: one atomic add per run of
// equal bins (a constant or sorted input costs one add per vector, not V).
// Without RUNS (32 LDS copies, where lanes never share a counter): one add of
// 1 per element, with no branch: an element that is not counted goes to the
// spare bin nbins.
template <int DT, int MODE, bool GLOBAL, bool RUNS>
__device__ __forceinline__ void count_vec(const hu32x4 &v, const HistArgs &a, uint32_t *h,
                                          uint64_t *g, uint32_t lr) {
    constexpr int EB = HistT<DT>::EB, V = 16 / EB;
    const uint32_t w[4] = {v[0], v[1], v[2], v[3]};
    if constexpr (!RUNS) {
#pragma unroll
        for (int i = 0; i < V; i++) {
            const uint32_t b = bin_or_spare<DT, MODE>(raw_of<EB>(w, i), a);
            __hip_atomic_fetch_add(h + ((b << 5) | lr), 1u, __ATOMIC_RELAXED,   // R = 32 copies
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        return;
    }
    int cur = -1;
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < V; i++) {
        const int b = bin_of<DT, MODE>(raw_of<EB>(w, i), a);
        if (b != cur) {
            if (cur >= 0) add_run<GLOBAL>(h, g, cur, cnt, a, lr);
            cur = b;
            cnt = 0;
        }
        cnt++;
    }
    if (cur >= 0) add_run<GLOBAL>(h, g, cur, cnt, a, lr);
}

template <int DT> __device__ __forceinline__ uint64_t raw_at(const unsigned char *p) {
    constexpr int EB = HistT<DT>::EB;
    if constexpr (EB == 8) return *reinterpret_cast<const uint64_t *>(p);
    else if constexpr (EB == 4) return *reinterpret_cast<const uint32_t *>(p);
    else if constexpr (EB == 2) return *reinterpret_cast<const uint16_t *>(p);
    else return *p;
}

// Streams the input; GLOBAL = false: LDS histogram, then row blockIdx.x of part;
// GLOBAL = true: 64-bit atomics straight into counts (zero-filled before).
template <int DT, int MODE, bool GLOBAL, bool RUNS>
__global__ __launch_bounds__(HNT) void k_hist(const unsigned char *__restrict__ src, HistArgs a,
                                             uint32_t *__restrict__ part,
                                             uint64_t *__restrict__ counts) {
    constexpr int EB = HistT<DT>::EB, V = 16 / EB;
    // static, so that LDS addresses need no base (two workgroups per CU fit)
    __shared__ uint32_t h[GLOBAL ? 1 : LDS_WORDS];
    const uint32_t lr = threadIdx.x & ((1u << a.rs) - 1);
    if constexpr (!GLOBAL) {
        for (int j = threadIdx.x; j < ((int)a.nbins + (RUNS ? 0 : 1)) << a.rs; j += HNT) h[j] = 0;
        __syncthreads();
    }
    const hu32x4 *vs = reinterpret_cast<const hu32x4 *>(src + a.head * EB);
    const int64_t stride = (int64_t)gridDim.x * HNT;
    int64_t i = (int64_t)blockIdx.x * HNT + threadIdx.x;
    for (; i + (HUNROLL - 1) * stride < a.nvec; i += HUNROLL * stride) {
        hu32x4 v[HUNROLL];
#pragma unroll
        for (int k = 0; k < HUNROLL; k++) v[k] = __builtin_nontemporal_load(vs + i + k * stride);
#pragma unroll
        for (int k = 0; k < HUNROLL; k++) count_vec<DT, MODE, GLOBAL, RUNS>(v[k], a, h, counts, lr);
    }
    for (; i < a.nvec; i += stride) {
        const hu32x4 v = __builtin_nontemporal_load(vs + i);
        count_vec<DT, MODE, GLOBAL, RUNS>(v, a, h, counts, lr);
    }
    // the < V elements before the first 16-byte boundary and the < V after the
    // last whole vector
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x < 2 * V) {
        const int t = threadIdx.x;
        const int64_t e = t < V ? (int64_t)t : a.head + a.nvec * V + (t - V);
        const bool in = t < V ? e < a.head : e < a.n;
        if (in) {
            const int b = bin_of<DT, MODE>(raw_at<DT>(src + e * EB), a);
            if (b >= 0) add_run<GLOBAL>(h, counts, b, 1u, a, lr);
        }
    }
    if constexpr (!GLOBAL) {
        __syncthreads();
        uint32_t *row = part + (int64_t)blockIdx.x * a.nbins;
        const int R = 1 << a.rs;
        for (int j = threadIdx.x; j < (int)a.nbins; j += HNT) {
            uint32_t t = 0;
            for (int c = 0; c < R; c++) t += h[(j << a.rs) + ((c + j) & (R - 1))];   // rotated: no bank conflicts
            row[j] = t;
        }
    }
}

// counts[j] = sum over the G rows of part[g][j]; one workgroup per 64 bins,
// wave w sums rows w, w + 16, ... and the 16 wave sums meet in LDS.
__global__ __launch_bounds__(MERGE_NT) void k_hist_merge(const uint32_t *__restrict__ part, int G,
                                                        int64_t nbins,
                                                        int64_t *__restrict__ counts) {
    constexpr int NW = MERGE_NT / 64;
    __shared__ uint64_t s[NW][64];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + l;
    uint64_t acc = 0;
    if (j < nbins) {
        int g = w;
        for (; g + 3 * NW < G; g += 4 * NW) {
            const uint32_t c0 = part[(int64_t)g * nbins + j];
            const uint32_t c1 = part[(int64_t)(g + NW) * nbins + j];
            const uint32_t c2 = part[(int64_t)(g + 2 * NW) * nbins + j];
            const uint32_t c3 = part[(int64_t)(g + 3 * NW) * nbins + j];
            acc += (uint64_t)c0 + c1 + c2 + c3;
        }
        for (; g < G; g += NW) acc += part[(int64_t)g * nbins + j];
    }
    s[w][l] = acc;
    __syncthreads();
    if (w == 0 && j < nbins) {
        uint64_t t = 0;
#pragma unroll
        for (int k = 0; k < NW; k++) t += s[k][l];
        counts[j] = (int64_t)t;
    }
}

// counts == nullptr: the counts go to the first nbins * 8 bytes of the
// workspace (returned in *ws_counts), ahead of the partial table.
template <int DT, int MODE>
int launch_hist(const void *src, const HistArgs &a0, int64_t *counts, hipStream_t st,
                int64_t **ws_counts = nullptr) {
    constexpr int EB = HistT<DT>::EB, V = 16 / EB;
    HistArgs a = a0;
    const uintptr_t p = (uintptr_t)src;
    const int64_t to16 = (int64_t)(((16 - p % 16) % 16) / EB);
    a.head = to16 < a.n ? to16 : a.n;
    a.nvec = (a.n - a.head) / V;
    const unsigned char *s = static_cast<const unsigned char *>(src);
    uint64_t *c64 = reinterpret_cast<uint64_t *>(counts);
    const int64_t want = (a.nvec + (int64_t)HNT * HUNROLL - 1) / ((int64_t)HNT * HUNROLL);
    if (!counts && a.nbins > LDS_WORDS) return fail(XTR_EINVAL, "histogram: internal bins");
    if (a.nbins > LDS_WORDS) {
        int rc = zero_fill(counts, (size_t)a.nbins * 8, st);
        if (rc) return rc;
        a.rs = 0;
        int64_t G = resident_blocks((const void *)k_hist<DT, MODE, true, true>, HNT);
        if (G > want) G = want;
        if (G < 1) G = 1;
        hipLaunchKernelGGL((k_hist<DT, MODE, true, true>), dim3((unsigned)G), dim3(HNT), 0, st, s,
                           a, (uint32_t *)nullptr, c64);
        XTR_HIP(hipGetLastError());
        return XTR_OK;
    }
    // as many copies per bin (up to 32) as the LDS budget holds; the
    // branch-free loop needs 32 copies of nbins + 1 bins (the spare one)
    constexpr bool flat = MODE == BIN_FLOAT || MODE == BIN_SHIFT32 || MODE == BIN_MAGIC32;
    const bool runs = !flat || ((a.nbins + 1) << 5) > LDS_WORDS;
    a.rs = 5;
    if (runs) {
        a.rs = 0;
        while (a.rs < 5 && (a.nbins << (a.rs + 1)) <= LDS_WORDS) a.rs++;
    }
    const void *kern = runs ? (const void *)k_hist<DT, MODE, false, true>
                            : (const void *)k_hist<DT, MODE, false, !flat>;
    // at most 2 workgroups per CU: more only lengthens the partial table
    int occ = 0;
    XTR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, HNT, 0));
    if (occ < 1) occ = 1;
    if (occ > 2) occ = 2;
    int64_t G = (int64_t)occ * cu_count();
    if (G > want) G = want;
    const int64_t floor_g = (a.n + WG_MAX_ELEMS - 1) / WG_MAX_ELEMS;   // 32-bit counters
    if (G < floor_g) G = floor_g;
    if (G < 1) G = 1;
    if (G > 0x7fffffff) return fail(XTR_EINVAL, "histogram: input too large");
    void *ws = nullptr;
    const size_t reserve = counts ? 0 : ((size_t)a.nbins * 8 + 255) / 256 * 256;
    int rc = workspace(WS_HIST, st, reserve + (size_t)G * (size_t)a.nbins * 4, &ws);
    if (rc) return rc;
    uint32_t *part = reinterpret_cast<uint32_t *>(static_cast<unsigned char *>(ws) + reserve);
    if (!counts) {
        counts = static_cast<int64_t *>(ws);
        *ws_counts = counts;
    }
    if (runs)
        hipLaunchKernelGGL((k_hist<DT, MODE, false, true>), dim3((unsigned)G), dim3(HNT), 0, st,
                           s, a, part, (uint64_t *)nullptr);
    else
        hipLaunchKernelGGL((k_hist<DT, MODE, false, !flat>), dim3((unsigned)G), dim3(HNT), 0, st,
                           s, a, part, (uint64_t *)nullptr);
    hipLaunchKernelGGL(k_hist_merge, dim3((unsigned)((a.nbins + 63) / 64)), dim3(MERGE_NT), 0, st,
                       part, (int)G, a.nbins, counts);
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

// fp8 histograms through their 256 codes: the counts of every code (the fast
// one-byte histogram), then one thread per code adds its count to the bin the
// float rule gives the code's value (the same bin_of as the direct form).
__global__ __launch_bounds__(256) void k_hist_codes(const int64_t *__restrict__ codes, HistArgs a,
                                                    uint64_t *__restrict__ counts) {
    const uint32_t c = threadIdx.x;
    const int b = bin_of<XTR_F8E4M3, BIN_FLOAT>(c, a);
    if (b >= 0 && codes[c] != 0)
        __hip_atomic_fetch_add(counts + b, (uint64_t)codes[c], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

int hist_fp8_by_codes(const void *src, const HistArgs &a, int64_t *counts, hipStream_t st) {
    HistArgs ac{};
    ac.n = a.n;
    ac.nbins = 256;
    ac.lo_i = 0;
    ac.width = 1;
    ac.shift = 0;
    ac.lo32 = 0x80000000u;          // lo = 0, biased
    ac.span_m1 = 255;
    ac.span_m1_32 = 255;
    int64_t *codes = nullptr;
    int rc = launch_hist<XTR_U8, BIN_SHIFT32>(src, ac, nullptr, st, &codes);
    if (rc) return rc;
    rc = zero_fill(counts, (size_t)a.nbins * 8, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_hist_codes, dim3(1), dim3(256), 0, st, codes, a,
                       reinterpret_cast<uint64_t *>(counts));
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

int check_common(const char *who, const void *src, int64_t n, int dtype, int64_t nbins,
                 const int64_t *counts) {
    if (n < 0) return fail(XTR_EINVAL, "%s: negative n", who);
    if (nbins < 1 || nbins > XTR_HIST_MAX_BINS)
        return fail(XTR_EINVAL, "%s: nbins %lld outside [1, %lld]", who, (long long)nbins,
                    (long long)XTR_HIST_MAX_BINS);
    if (!counts) return fail(XTR_EINVAL, "%s: null counts", who);
    if (n > 0 && !src) return fail(XTR_EINVAL, "%s: null src", who);
    if ((uintptr_t)counts % 8) return fail(XTR_EALIGN, "%s: counts not 8-byte aligned", who);
    const int eb = elem_bytes(dtype);
    if (n > 0 && (uintptr_t)src % eb)
        return fail(XTR_EALIGN, "%s: src not aligned to its element", who);
    const uintptr_t s0 = (uintptr_t)src, s1 = s0 + (uintptr_t)n * eb;
    const uintptr_t d0 = (uintptr_t)counts, d1 = d0 + (uintptr_t)nbins * 8;
    if (n > 0 && s0 < d1 && d0 < s1) return fail(XTR_EOVERLAP, "%s: src and counts overlap", who);
    return XTR_OK;
}

template <int MODE>
int dispatch_int(const void *src, int dtype, const HistArgs &a, int64_t *counts, hipStream_t st) {
    switch (dtype) {
    case XTR_I32: return launch_hist<XTR_I32, MODE>(src, a, counts, st);
    case XTR_I64: return launch_hist<XTR_I64, MODE>(src, a, counts, st);
    case XTR_U8: return launch_hist<XTR_U8, MODE>(src, a, counts, st);
    default: return launch_hist<XTR_U16, MODE>(src, a, counts, st);
    }
}

template <int MODE>
int dispatch_int32(const void *src, int dtype, const HistArgs &a, int64_t *counts,
                   hipStream_t st) {
    switch (dtype) {
    case XTR_I32: return launch_hist<XTR_I32, MODE>(src, a, counts, st);
    case XTR_U8: return launch_hist<XTR_U8, MODE>(src, a, counts, st);
    default: return launch_hist<XTR_U16, MODE>(src, a, counts, st);
    }
}

int histogram_int_impl(const void *src, int64_t n, int dtype, int64_t lo, int64_t width,
                       int64_t nbins, int64_t *counts, hipStream_t st) {
    const char *who = "histogram_int";
    if (dtype != XTR_I32 && dtype != XTR_I64 && dtype != XTR_U8 && dtype != XTR_U16)
        return fail(XTR_EDTYPE, "%s: dtype %d is not an integer format", who, dtype);
    if (width < 1) return fail(XTR_EINVAL, "%s: width %lld < 1", who, (long long)width);
    int rc = check_common(who, src, n, dtype, nbins, counts);
    if (rc) return rc;
    if (n == 0) return zero_fill(counts, (size_t)nbins * 8, st);
    HistArgs a{};
    a.n = n;
    a.nbins = nbins;
    a.lo_i = lo;
    a.width = (uint64_t)width;
    const unsigned __int128 span = (unsigned __int128)(uint64_t)width * (uint64_t)nbins;
    a.span_m1 = span > ((unsigned __int128)1 << 64) ? ~(uint64_t)0 : (uint64_t)(span - 1);
    const bool pow2 = (a.width & (a.width - 1)) == 0;
    const bool small = span <= ((unsigned __int128)1 << 32);
    if (pow2) a.shift = __builtin_ctzll(a.width);
    // c = ceil(2^64 / width) = floor((2^64 - 1) / width) + 1 (width is not a power of two)
    else if (small) a.magic = ~(uint64_t)0 / a.width + 1;
    // The 32-bit rules need every shift below 32: width = 2^32 (one bin
    // spanning the whole 32-bit range) takes the 64-bit shift rule.
    const bool rule32_ok = !(pow2 && a.shift >= 32);
    if (dtype != XTR_I64 && small && rule32_ok && lo >= INT32_MIN && lo <= INT32_MAX) {
        a.lo32 = (uint32_t)(int32_t)lo ^ 0x80000000u;
        a.span_m1_32 = (uint32_t)a.span_m1;
        return pow2 ? dispatch_int32<BIN_SHIFT32>(src, dtype, a, counts, st)
                    : dispatch_int32<BIN_MAGIC32>(src, dtype, a, counts, st);
    }
    if (pow2) return dispatch_int<BIN_SHIFT>(src, dtype, a, counts, st);
    if (small) return dispatch_int<BIN_MAGIC>(src, dtype, a, counts, st);
    return dispatch_int<BIN_DIV>(src, dtype, a, counts, st);
}

int histogram_float_impl(const void *src, int64_t n, int dtype, double lo, double hi,
                         int64_t nbins, int64_t *counts, hipStream_t st) {
    const char *who = "histogram_float";
    if (!is_float_sum_dtype(dtype))
        return fail(XTR_EDTYPE, "%s: dtype %d is not a float format", who, dtype);
    if (!(hi > lo) || !isfinite(lo) || !isfinite(hi))
        return fail(XTR_EINVAL, "%s: need finite lo < hi", who);
    const double scale = (double)nbins / (hi - lo);
    if (!isfinite(hi - lo) || !isfinite(scale))
        return fail(XTR_EINVAL, "%s: hi - lo and nbins / (hi - lo) must be finite", who);
    int rc = check_common(who, src, n, dtype, nbins, counts);
    if (rc) return rc;
    if (n == 0) return zero_fill(counts, (size_t)nbins * 8, st);
    HistArgs a{};
    a.n = n;
    a.nbins = nbins;
    a.lo_f = lo;
    a.hi_f = hi;
    a.scale = scale;
    switch (dtype) {
    case XTR_F32: return launch_hist<XTR_F32, BIN_FLOAT>(src, a, counts, st);
    case XTR_F16: return launch_hist<XTR_F16, BIN_FLOAT>(src, a, counts, st);
    case XTR_BF16: return launch_hist<XTR_BF16, BIN_FLOAT>(src, a, counts, st);
    default: return hist_fp8_by_codes(src, a, counts, st);
    }
}

}  // namespace
}  // namespace xtr

extern "C" int histogram_int(const void *src, int64_t n, int dtype, int64_t lo, int64_t width,
                             int64_t nbins, int64_t *counts, void *stream) {
    return xtr::histogram_int_impl(src, n, dtype, lo, width, nbins, counts, (hipStream_t)stream);
}

extern "C" int histogram_float(const void *src, int64_t n, int dtype, double lo, double hi,
                               int64_t nbins, int64_t *counts, void *stream) {
    return xtr::histogram_float_impl(src, n, dtype, lo, hi, nbins, counts, (hipStream_t)stream);
}
