// Tree-based sum reduction for gfx950 (single, batched, segmented).
//
// What is computed: the sequential reduce of Listing 2.1, i.e. its
// specification reduce_sum(n, A) = A(0) + ... + A(n-1) (Section 2.1), for
// int32 / int64 (exact, modulo 2^64 for int64) and for fp32 / bf16 / fp16 /
// fp8-e4m3fn inputs (compensated fp32 accumulation, fp64 only in the final
// cross-workgroup combine).
//
// Structure (the split of Listing 2.2 into partial sums and a combine, with the
// register accumulator and the halving tree of Section 7.2 / Listing 7.22):
//   1. Canonical chunking.  A range (ptr, n) is split into a head of at most
//      V-1 elements up to the first 16-byte boundary, then chunks of
//      CH = 256 threads x U vectors x V elements.  Every chunk is reduced by
//      one workgroup of 256 threads (4 wave64s).
//   2. Thread level: U 16-byte vector loads per thread (vector u of thread t is
//      vector u*256 + t of the chunk, so each wave-level load reads 1 KiB of
//      contiguous HBM), decoded to fp32 and accumulated in registers: four
//      independent (s, c) pairs per thread updated with an error-free two-sum
//      (Knuth) per element, so the rounding error of every addition is kept
//      in c.  fp8-e4m3fn takes a shortcut that is exact: every e4m3 value is a
//      multiple of 2^-9 of magnitude <= 448, so an fp32 sum of up to 73 of them
//      stays an exact multiple of 2^-9 below 2^15; each accumulator sums at most
//      47 per chunk exactly and the pair starts from that exact value.
//      Integers accumulate in 64-bit registers (wrap-around adds).
//   3. Wave level: a 64-lane butterfly of pair additions built from DPP
//      (quad_perm xor 1, xor 2; row_half_mirror and row_mirror on data already
//      uniform across the quad / half-row) and readlane for the four rows.
//   4. Workgroup level: one LDS slot per wave, a barrier, and the pairwise
//      combine ((w0 + w1) + (w2 + w3)).
//   5. Grid level: each chunk's pair becomes one fp64 partial (s + c, exact);
//      partials are combined in fp64 by a radix-256 tree, each group of 256
//      with a fixed pairwise tree, level by level.  Large single ranges store
//      plain partials and small follow-up launches sum the levels; other
//      ranges combine in-kernel: the last workgroup of every group (atomic
//      ticket) sums it and passes the result one level up.  The order is
//      fixed, so the result is a deterministic function of (data, n, dtype,
//      alignment of ptr) -- the same alone, batched, as a segment, or summed
//      from host memory.
//   6. Small segments (body within two vector rows of a chunk) are reduced by
//      one wave that replays the chunk arithmetic of the whole workgroup.
// The plain mode repeats the structure with uncompensated fp32 adds
// everywhere (comparator).
#include "common.hpp"

#include <cstring>

#include <algorithm>
#include <new>
#include <vector>

#pragma clang fp contract(off)

namespace xtr {
namespace {

constexpr int NTHR = 256;        // threads per workgroup
constexpr int NW = NTHR / 64;    // waves per workgroup
constexpr int U = 8;             // 16-byte vectors per thread per chunk
constexpr int RADIX = 256;       // fan-in of the grid combine tree
constexpr int MAXLEV = 5;

enum Mode { COMP = 0, PLAIN = 1, INTM = 2 };

template <int DT> struct DTI;
template <> struct DTI<XTR_F32>    { static constexpr int EB = 4; };
template <> struct DTI<XTR_F16>    { static constexpr int EB = 2; };
template <> struct DTI<XTR_BF16>   { static constexpr int EB = 2; };
template <> struct DTI<XTR_F8E4M3> { static constexpr int EB = 1; };
template <> struct DTI<XTR_I32>    { static constexpr int EB = 4; };
template <> struct DTI<XTR_I64>    { static constexpr int EB = 8; };

template <int DT> constexpr int vec_elems() { return 16 / DTI<DT>::EB; }
template <int DT> constexpr int64_t chunk_elems() { return (int64_t)NTHR * U * vec_elems<DT>(); }

int64_t chunk_elems_rt(int dtype) { return (int64_t)NTHR * U * (16 / elem_bytes(dtype)); }

// ---------------------------------------------------------------- arithmetic

struct Pair {
    float s, c;
};

// Knuth's two-sum: s + e == a + b exactly (round-to-nearest, no FMA involved).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ Pair pair_add(Pair x, Pair y) {
    Pair r;
    float e;
    two_sum(x.s, y.s, r.s, e);
    r.c = (x.c + y.c) + e;
    return r;
}

// fp64 value of a compensated pair; a non-finite s carries the IEEE result of
// the exact sum (inf or NaN) and c is ignored (it is NaN after an inf).
__device__ __forceinline__ double pair_value(Pair p) {
    if (!__builtin_isfinite(p.s)) return (double)p.s;
    return (double)p.s + (double)p.c;
}

// ---------------------------------------------------------------- cross-lane

template <int CTRL> __device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ float dppf(float v) {
    return __uint_as_float(dpp<CTRL>(__float_as_uint(v)));
}
template <int CTRL> __device__ __forceinline__ uint64_t dpp64(uint64_t v) {
    return (uint64_t)dpp<CTRL>((uint32_t)v) | ((uint64_t)dpp<CTRL>((uint32_t)(v >> 32)) << 32);
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
    return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane) |
           ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane) << 32);
}

constexpr int DPP_XOR1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7-i within each 8 lanes
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15-i within each row of 16

// Integer wave sum (the planning kernels' counts): symmetric DPP butterfly
// (after xor1/xor2 the four lanes of a quad hold identical values, so the
// half-row mirror exchanges whole quads and the row mirror the half-rows),
// then the four row totals.
__device__ __forceinline__ uint64_t wave_reduce(uint64_t v) {
    v = v + dpp64<DPP_XOR1>(v);
    v = v + dpp64<DPP_XOR2>(v);
    v = v + dpp64<DPP_HALF_MIRROR>(v);
    v = v + dpp64<DPP_MIRROR>(v);
    return (readlane_u64(v, 0) + readlane_u64(v, 16)) + (readlane_u64(v, 32) + readlane_u64(v, 48));
}
// fp64 butterfly for the grid combine (xor 1 .. 32, a balanced pairwise tree)
__device__ __forceinline__ double wave_reduce_f64(double v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = v + __shfl_xor(v, m, 64);
    return v;
}

// ---------------------------------------------------------------- per-thread state

template <int DT, int MODE> struct Acc;

// compensated float accumulators
template <int DT> struct Acc<DT, COMP> {
    Pair p[4];
    float g[4];   // fp8: exact fp32 group sums
    __device__ void init() {
#pragma unroll
        for (int a = 0; a < 4; a++) p[a] = Pair{0.f, 0.f}, g[a] = 0.f;
    }
    __device__ __forceinline__ void add(int a, float x) {
        if constexpr (DT == XTR_F8E4M3) {
            g[a] = g[a] + x;
        } else {
            float s, e;
            two_sum(p[a].s, x, s, e);
            p[a].s = s;
            p[a].c = p[a].c + e;
        }
    }
    // add into an accumulator that is still (+0, +0): two_sum(+0, x) gives
    // s = +0 + x and e = +0 exactly, and c = +0 + +0 = +0, so this is add()
    // bit for bit while s is finite (once s is not, c is never used).
    __device__ __forceinline__ void add_first(int a, float x) {
        if constexpr (DT == XTR_F8E4M3) {
            g[a] = g[a] + x;
        } else {
            p[a].s = 0.f + x;
            p[a].c = 0.f;
        }
    }
    __device__ Pair finish() {
        if constexpr (DT == XTR_F8E4M3) {
#pragma unroll
            for (int a = 0; a < 4; a++) p[a] = Pair{g[a], 0.f};
        }
        return pair_add(pair_add(p[0], p[1]), pair_add(p[2], p[3]));
    }
};

// plain fp32 accumulators (comparator)
template <int DT> struct Acc<DT, PLAIN> {
    float s[4];
    __device__ void init() {
#pragma unroll
        for (int a = 0; a < 4; a++) s[a] = 0.f;
    }
    __device__ __forceinline__ void add(int a, float x) { s[a] = s[a] + x; }
    __device__ __forceinline__ void add_first(int a, float x) { add(a, x); }
    __device__ float finish() { return (s[0] + s[1]) + (s[2] + s[3]); }
};

// 64-bit wrap-around integer accumulators
template <int DT> struct Acc<DT, INTM> {
    uint64_t s[2];
    __device__ void init() { s[0] = s[1] = 0; }
    __device__ __forceinline__ void add(int a, uint64_t x) { s[a & 1] += x; }
    __device__ __forceinline__ void add_first(int a, uint64_t x) { add(a, x); }
    __device__ uint64_t finish() { return s[0] + s[1]; }
};

// ---------------------------------------------------------------- decode

__device__ __forceinline__ float f16_lo(uint32_t d) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(d & 0xffffu));
}
__device__ __forceinline__ float f16_hi(uint32_t d) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(d >> 16));
}

template <bool FIRST, class A, class X> __device__ __forceinline__ void acc_put(A &acc, int a, X x) {
    if constexpr (FIRST) acc.add_first(a, x);
    else acc.add(a, x);
}

// accumulate element i (0 <= i < V) of a decoded vector into accumulator i % 4
// (FIRST: every accumulator it reaches is still zero -- the thread's first
// vector, with no head before it)
template <int DT, int MODE, bool FIRST = false>
__device__ __forceinline__ void acc_vec(Acc<DT, MODE> &acc, const uint4 &v) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    if constexpr (DT == XTR_F32) {
#pragma unroll
        for (int i = 0; i < 4; i++) acc_put<FIRST>(acc, i, __uint_as_float(w[i]));
    } else if constexpr (DT == XTR_BF16) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            // elements 4..7 reach accumulators 0..3 a second time
            if (k < 2) {
                acc_put<FIRST>(acc, (2 * k) & 3, __uint_as_float(w[k] << 16));
                acc_put<FIRST>(acc, (2 * k + 1) & 3, __uint_as_float(w[k] & 0xffff0000u));
            } else {
                acc.add((2 * k) & 3, __uint_as_float(w[k] << 16));
                acc.add((2 * k + 1) & 3, __uint_as_float(w[k] & 0xffff0000u));
            }
        }
    } else if constexpr (DT == XTR_F16) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (k < 2) {
                acc_put<FIRST>(acc, (2 * k) & 3, f16_lo(w[k]));
                acc_put<FIRST>(acc, (2 * k + 1) & 3, f16_hi(w[k]));
            } else {
                acc.add((2 * k) & 3, f16_lo(w[k]));
                acc.add((2 * k + 1) & 3, f16_hi(w[k]));
            }
        }
    } else if constexpr (DT == XTR_F8E4M3) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[k], false);   // bytes 0, 1
            auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[k], true);    // bytes 2, 3
            acc_put<FIRST>(acc, 0, lo[0]);
            acc_put<FIRST>(acc, 1, lo[1]);
            acc_put<FIRST>(acc, 2, hi[0]);
            acc_put<FIRST>(acc, 3, hi[1]);
        }
    } else if constexpr (DT == XTR_I32) {
#pragma unroll
        for (int i = 0; i < 4; i++) acc_put<FIRST>(acc, i, (uint64_t)(int64_t)(int32_t)w[i]);
    } else {  // I64
        acc_put<FIRST>(acc, 0, (uint64_t)w[0] | ((uint64_t)w[1] << 32));
        acc_put<FIRST>(acc, 1, (uint64_t)w[2] | ((uint64_t)w[3] << 32));
    }
}

// one element at byte address p, as element i of its vector
template <int DT, int MODE>
__device__ __forceinline__ void acc_elem(Acc<DT, MODE> &acc, const unsigned char *p, int i) {
    if constexpr (DT == XTR_F32) {
        acc.add(i & 3, *reinterpret_cast<const float *>(p));
    } else if constexpr (DT == XTR_BF16) {
        acc.add(i & 3, __uint_as_float((uint32_t)*reinterpret_cast<const uint16_t *>(p) << 16));
    } else if constexpr (DT == XTR_F16) {
        acc.add(i & 3, f16_lo(*reinterpret_cast<const uint16_t *>(p)));
    } else if constexpr (DT == XTR_F8E4M3) {
        auto f = __builtin_amdgcn_cvt_pk_f32_fp8((int)(uint32_t)*p, false);
        acc.add(i & 3, f[0]);
    } else if constexpr (DT == XTR_I32) {
        acc.add(i, (uint64_t)(int64_t)*reinterpret_cast<const int32_t *>(p));
    } else {
        acc.add(i, *reinterpret_cast<const uint64_t *>(p));
    }
}

// ---------------------------------------------------------------- ranges

// One array reduced into *dst.
struct Range {
    const unsigned char *ptr;  // first element
    int64_t n;                 // elements
    int64_t chunk_base;        // global index of its first chunk (slot base in the level arrays)
    int64_t nchunks;           // >= 1 (an empty range still has one chunk that writes 0)
    unsigned char *dst;        // where the result goes (double, float or int64)
    int32_t head;              // elements before the first 16-byte boundary
    int32_t _pad;
};

// Level arrays of the grid combine: level l has a partial array indexed by
// chunk_base + (group index at that level); the ticket of group g at level l
// is ctr[(chunk_base + g) * MAXLEV + l].
struct Levels {
    unsigned char *part[MAXLEV];
    uint32_t *ctr;
};

template <int MODE> struct PartT;
template <> struct PartT<COMP> { using T = double; };
template <> struct PartT<PLAIN> { using T = float; };
template <> struct PartT<INTM> { using T = uint64_t; };

// ---------------------------------------------------------------- one chunk

// wave_reduce4 (defined below): the four 64-lane butterflies of a workgroup
// and their ((w0 + w1) + (w2 + w3)) combination, by one wave.
template <typename T> __device__ __forceinline__ T wave_reduce4(const T (&p)[NW]);

// Thread accumulators -> the chunk's value (fp64 for compensated pairs, fp32
// plain, int64): each thread's accumulators combined, then the wave butterfly
// over each wave's 64 threads and ((w0 + w1) + (w2 + w3)) over the 4 waves.
// The threads' values go through LDS to wave 0, which performs exactly those
// additions in one reduce-scatter pass (wave_reduce4) instead of four waves
// running a butterfly each; the value is returned to the threads of wave 0
// (the callers use it there only).
template <int DT, int MODE>
__device__ __forceinline__ typename PartT<MODE>::T chunk_tree(Acc<DT, MODE> &acc) {
    auto tv = acc.finish();
    using W = decltype(tv);
    __shared__ W vals[NTHR];
    const int t = threadIdx.x;
    vals[t] = tv;
    __syncthreads();
    typename PartT<MODE>::T res{};
    if (t < 64) {
        W p[NW];
#pragma unroll
        for (int w = 0; w < NW; w++) p[w] = vals[t + 64 * w];
        const W r = wave_reduce4(p);
        if constexpr (MODE == COMP) res = pair_value(r);
        else res = r;
    }
    __syncthreads();   // vals[] is reused by the next chunk
    return res;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16-byte load of device memory through a global-memory pointer (a pointer
// that went through a struct or a select may reach here as a generic one; a
// generic load would also count against the scalar-load counter, so waiting
// for a scalar load would wait for it too).
typedef __attribute__((address_space(1))) const u32x4 gu32x4;
template <bool NT> __device__ __forceinline__ uint4 load16(const uint4 *p) {
    gu32x4 *g = (gu32x4 *)p;
    u32x4 v;
    if constexpr (NT) v = __builtin_nontemporal_load(g);
    else v = *g;
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Element i of a 16-byte vector, decoded as acc_elem decodes it, added to
// accumulator a (the slot acc_elem uses for element i of a vector).
template <int DT, int MODE, bool FIRST = false>
__device__ __forceinline__ void acc_from_vec(Acc<DT, MODE> &acc, const uint4 &v, int i, int a) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    if constexpr (DT == XTR_F32) {
        acc_put<FIRST>(acc, a, __uint_as_float(w[i]));
    } else if constexpr (DT == XTR_BF16) {
        acc_put<FIRST>(acc, a, __uint_as_float(((w[i >> 1] >> (16 * (i & 1))) & 0xffffu) << 16));
    } else if constexpr (DT == XTR_F16) {
        acc_put<FIRST>(acc, a, f16_lo(w[i >> 1] >> (16 * (i & 1))));
    } else if constexpr (DT == XTR_F8E4M3) {
        auto f = __builtin_amdgcn_cvt_pk_f32_fp8((int)((w[i >> 2] >> (8 * (i & 3))) & 0xffu), false);
        acc_put<FIRST>(acc, a, f[0]);
    } else if constexpr (DT == XTR_I32) {
        acc_put<FIRST>(acc, a, (uint64_t)(int64_t)(int32_t)w[i]);
    } else {
        acc_put<FIRST>(acc, a, (uint64_t)w[2 * i] | ((uint64_t)w[2 * i + 1] << 32));
    }
}

// The first m elements of a 16-byte vector (m may be <= 0 or >= V), the
// others zeroed.  Adding a zero element is an exact no-op on every
// accumulator: the running values are never -0 (they start at +0, and a sum
// is -0 only when both terms are), so s + 0 = s, the two-sum error is +0 and
// c + 0 = c; an integer sum adds 0.  A zeroed element therefore leaves the
// same state as an element that is not added at all.
template <int DT> __device__ __forceinline__ uint4 first_elems(uint4 v, int m) {
    constexpr int EB = DTI<DT>::EB, V = vec_elems<DT>();
    const int nb = (m < 0 ? 0 : (m > V ? V : m)) * EB;   // bytes kept
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int kb = nb - 4 * k;   // bytes kept in dword k
        if constexpr (EB >= 4) {
            w[k] = kb > 0 ? w[k] : 0u;
        } else {
            w[k] = kb >= 4 ? w[k] : (kb <= 0 ? 0u : w[k] & ((1u << (8 * kb)) - 1u));
        }
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Chunk j of range rg, by one workgroup.  Every load is issued before any
// element is added (no load sits behind a branch, so none waits where
// branches join): the head (the elements before the first 16-byte boundary,
// added by thread 0 of chunk 0) comes from the aligned vector that holds it,
// and in a partial chunk a lane whose vector lies past the body reloads the
// body's last vector (a partial last vector is loaded whole); the elements
// outside the body are zeroed before they are added, which leaves the
// accumulators as they are.  A 16-byte aligned vector holding a byte of the
// range lies on a page the range touches.  A chunk with no body or head (an
// empty range) loads the vector holding the range's output slot instead.
template <int DT, int MODE, bool NT>
__device__ __forceinline__ typename PartT<MODE>::T reduce_chunk(const Range &rg, int64_t j) {
    constexpr int EB = DTI<DT>::EB;
    constexpr int V = vec_elems<DT>();
    constexpr int64_t CH = chunk_elems<DT>();
    const int t = threadIdx.x;
    Acc<DT, MODE> acc;
    acc.init();
    const unsigned char *body = rg.ptr + (int64_t)rg.head * EB;
    const int64_t body_n = rg.n - rg.head;
    const int64_t e0 = j * CH;
    const unsigned char *sb = rg.n > 0 ? rg.ptr : rg.dst;   // a byte that exists
    const uint4 *safe = reinterpret_cast<const uint4 *>(sb - ((uintptr_t)sb & 15));
    if (e0 + CH <= body_n) {
        const uint4 *vp = reinterpret_cast<const uint4 *>(body + e0 * EB) + t;
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = load16<NT>(vp + u * NTHR);
        uint4 hv = make_uint4(0, 0, 0, 0);
        if (j == 0 && rg.head > 0) hv = load16<NT>(safe);   // uniform: the first chunk only
        if (j == 0 && t == 0 && rg.head > 0) {
            const int h0 = (int)((uintptr_t)rg.ptr & 15) / EB;
#pragma unroll
            for (int i = 1; i < V; i++)
                if (i >= h0 && i < h0 + rg.head) acc_from_vec(acc, hv, i, 0);
        }
#pragma unroll
        for (int u = 0; u < U; u++) acc_vec(acc, v[u]);
    } else {
        // partial chunk: clamped loads, then the elements in range
        const uint4 *bv = reinterpret_cast<const uint4 *>(body);
        const bool has_body = body_n > e0;
        const int64_t last = has_body ? (body_n - 1) / V : 0;   // last vector of the body
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t q = e0 / V + (int64_t)(u * NTHR + t);
            v[u] = load16<NT>(has_body ? bv + (q < last ? q : last) : safe);
        }
        const uint4 hv = load16<NT>(safe);
        if (j == 0 && t == 0 && rg.head > 0) {
            const int h0 = (int)((uintptr_t)rg.ptr & 15) / EB;
#pragma unroll
            for (int i = 1; i < V; i++)
                if (i >= h0 && i < h0 + rg.head) acc_from_vec(acc, hv, i, 0);
        }
        // per wave and vector row (uniform): all of the wave's vectors in the
        // body, none, or the row holding the body's end, where each lane keeps
        // the elements of its vector that lie in the body (zeroed elements
        // leave the accumulators exactly as they are)
        const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
        const int64_t ew = e0 + (int64_t)(wv * 64) * V;   // the wave's first element
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t eu = ew + (int64_t)(u * NTHR) * V;
            if (eu >= body_n) continue;
            if (eu + 64 * V <= body_n) {
                acc_vec(acc, v[u]);
            } else {
                const int64_t m = body_n - (eu + (int64_t)(t & 63) * V);
                acc_vec(acc, first_elems<DT>(v[u], m < 0 ? 0 : (m > V ? V : (int)m)));
            }
        }
    }
    return chunk_tree<DT, MODE>(acc);
}

// Ranges whose body fits in the first two vector rows of a chunk
// (body <= 2 * 256 * V elements) are "small": one wave computes their value.
template <int DT> constexpr int64_t small_max() { return (int64_t)2 * NTHR * vec_elems<DT>(); }

// Value of the single chunk of a small range, computed by ONE wave with
// exactly the arithmetic of reduce_chunk + chunk_tree on a whole workgroup:
// lane l plays threads l, l + 64, l + 128 and l + 192, keeps their
// accumulators apart, reduces each set of 64 with the same wave butterfly,
// and adds the four wave values in the order of the LDS tree.  The result is
// therefore bit-identical to the workgroup form (and to reduce_sum alone).
// A set of 64 threads that holds no element (its first vector lies past the
// body, and it does not take the head) has zero accumulators, whose butterfly
// gives exactly zero: it is skipped, and so is a vector row no lane reaches.
//
// Every input byte of the range is loaded up front as whole aligned 16-byte
// vectors (SmallRegs), so the value is then computed from registers alone and
// a wave can keep the next range's loads in flight meanwhile: the head (the
// elements before the first 16-byte boundary) from the aligned vector that
// holds them, and a partial last vector whole.  Such a vector holds at least
// one element of the range, and a 16-byte aligned vector never crosses a
// page, so it lies on a page the range touches; the bytes outside the range
// are never used.
template <int US> struct SmallRegs {
    uint4 v[US][NW];   // vector row u, thread set w (vector u * 256 + w * 64 + lane)
    uint4 hv;          // the aligned vector holding the head (lane 0 only)
};

// Every load is issued unconditionally (a branch around a load would make the
// wave wait for it where the branches join): a lane whose vector lies past the
// body reads the body's last vector again, and a range that is not reduced
// here (`use` false), or has no body or no head, reads the aligned vector that
// holds `safe` (any valid device address) instead.  A wave-instruction whose
// lanes all read one vector touches one cache line.  Such values are never
// used.
template <int DT, int US, bool NT>
__device__ __forceinline__ void small_load(const Range &rg, bool use, const void *safe,
                                           SmallRegs<US> &r) {
    constexpr int EB = DTI<DT>::EB;
    constexpr int V = vec_elems<DT>();
    const int l = threadIdx.x & 63;
    // (pointer arithmetic, not integer casts, so that the loads stay global loads)
    const unsigned char *sb = static_cast<const unsigned char *>(safe);
    const uint4 *sv = reinterpret_cast<const uint4 *>(sb - ((uintptr_t)sb & 15));
    // a small range's body has at most 2 * 256 * V elements: 32-bit sizes, and
    // one wave-uniform base with a 32-bit byte offset per lane (q <= 511)
    const int32_t body_n = __builtin_amdgcn_readfirstlane((int32_t)(rg.n - rg.head));
    const bool has_body = use && body_n > 0;
    const unsigned char *base = has_body ? rg.ptr + (int64_t)rg.head * EB
                                         : reinterpret_cast<const unsigned char *>(sv);
    const uint32_t last =
        __builtin_amdgcn_readfirstlane(has_body ? (uint32_t)((body_n - 1) / V) : 0u);
    r.hv = load16<NT>(use && rg.head > 0
                          ? reinterpret_cast<const uint4 *>(rg.ptr - ((uintptr_t)rg.ptr & 15))
                          : sv);
#pragma unroll
    for (int u = 0; u < US; u++)
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const uint32_t q = (uint32_t)(u * NTHR + w * 64 + l);
            const uint32_t byte = (q < last ? q : last) << 4;
            r.v[u][w] = load16<NT>(reinterpret_cast<const uint4 *>(base + (uint64_t)byte));
        }
}


// The canonical combination of a workgroup's 256 thread values: each set of
// 64 (threads 64 w .. 64 w + 63) reduced by the symmetric wave butterfly B
// (xor 1, xor 2, half-row mirror, row mirror -- every lane of a row then holds
// the row total -- and the rows as (r0 + r1) + (r2 + r3)), and the four set
// values as ((B(p0) + B(p1)) + (B(p2) + B(p3))).  One wave performs all of it
// in one pass (a reduce-scatter): p[w] is this lane's value of thread
// l + 64 w; it makes the same additions as the four butterflies (each
// addition is commutative bit for bit), only spread over the lanes.  At the first two
// levels the two lanes of a pair keep different values: after the xor-1 step
// a lane holds two of the four values, after the xor-2 step one, so that in
// every quad the lanes j = 0..3 hold values (0, 2, 1, 3) (even quads) or
// (3, 1, 2, 0) (odd quads).  That layout is symmetric under the half-row and
// row mirrors, so those two steps pair lanes that hold the same value, as in
// B.  Rows are then combined as (r0 + r1) + (r2 + r3) by the
// xor-16 and xor-32 exchanges (lane swaps), and the four values as
// (v0 + v1) + (v2 + v3) by the xor-2 and xor-1 steps inside each quad; every
// lane ends with the result.
__device__ __forceinline__ Pair vadd(Pair a, Pair b) { return pair_add(a, b); }
__device__ __forceinline__ float vadd(float a, float b) { return a + b; }
__device__ __forceinline__ uint64_t vadd(uint64_t a, uint64_t b) { return a + b; }
template <int CTRL> __device__ __forceinline__ Pair vdpp(Pair p) {
    return Pair{dppf<CTRL>(p.s), dppf<CTRL>(p.c)};
}
template <int CTRL> __device__ __forceinline__ float vdpp(float v) { return dppf<CTRL>(v); }
template <int CTRL> __device__ __forceinline__ uint64_t vdpp(uint64_t v) { return dpp64<CTRL>(v); }
// The xor-16 and xor-32 levels through gfx950's lane swaps (plain VALU
// instructions, no LDS round trip).  With both operands a copy of v,
// permlane16_swap leaves x = (row 0, row 0, row 2, row 2) and
// y = (row 1, row 1, row 3, row 3), and permlane32_swap leaves x = low half,
// y = high half in every lane: vadd(x, y) is the xor-16 (xor-32) butterfly
// step, with the lower row (half) as the first operand in every lane, which
// gives the same bits as either order since the additions are commutative.
template <int M> __device__ __forceinline__ void lane_swap(uint32_t &x, uint32_t &y) {
    static_assert(M == 16 || M == 32, "row or half-wave swap");
    if constexpr (M == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    }
}
template <int M> __device__ __forceinline__ float vswapadd(float v) {
    uint32_t x = __float_as_uint(v), y = x;
    lane_swap<M>(x, y);
    return __uint_as_float(x) + __uint_as_float(y);
}
template <int M> __device__ __forceinline__ Pair vswapadd(Pair v) {
    uint32_t xs = __float_as_uint(v.s), ys = xs, xc = __float_as_uint(v.c), yc = xc;
    lane_swap<M>(xs, ys);
    lane_swap<M>(xc, yc);
    return pair_add(Pair{__uint_as_float(xs), __uint_as_float(xc)},
                    Pair{__uint_as_float(ys), __uint_as_float(yc)});
}
template <int M> __device__ __forceinline__ uint64_t vswapadd(uint64_t v) {
    uint32_t xl = (uint32_t)v, yl = xl, xh = (uint32_t)(v >> 32), yh = xh;
    lane_swap<M>(xl, yl);
    lane_swap<M>(xh, yh);
    return ((uint64_t)xl | ((uint64_t)xh << 32)) + ((uint64_t)yl | ((uint64_t)yh << 32));
}

template <typename T> __device__ __forceinline__ T wave_reduce4(const T (&p)[NW]) {
    static_assert(NW == 4, "four values per lane");
    const int l = threadIdx.x & 63, j = l & 3;
    const bool odd = ((l >> 2) & 1) != 0;
    // xor 1: "A" lanes keep values 0 and 1, their partners values 2 and 3
    const bool a = ((j & 1) == 0) != odd;
    const T q0 = vadd(a ? p[0] : p[2], vdpp<DPP_XOR1>(a ? p[2] : p[0]));
    const T q1 = vadd(a ? p[1] : p[3], vdpp<DPP_XOR1>(a ? p[3] : p[1]));
    // xor 2: one of the two
    const bool f = ((j & 2) == 0) != odd;
    T r = vadd(f ? q0 : q1, vdpp<DPP_XOR2>(f ? q1 : q0));
    r = vadd(r, vdpp<DPP_HALF_MIRROR>(r));
    r = vadd(r, vdpp<DPP_MIRROR>(r));
    r = vswapadd<16>(r);
    r = vswapadd<32>(r);
    r = vadd(r, vdpp<DPP_XOR2>(r));
    return vadd(r, vdpp<DPP_XOR1>(r));
}

template <int DT, int MODE, int US>
__device__ __forceinline__ typename PartT<MODE>::T small_value(const Range &rg,
                                                               const SmallRegs<US> &r) {
    constexpr int EB = DTI<DT>::EB;
    constexpr int V = vec_elems<DT>();
    const int l = threadIdx.x & 63;
    // (a small range's body has at most 2 * 256 * V elements)
    const int32_t body_n = __builtin_amdgcn_readfirstlane((int32_t)(rg.n - rg.head));
    Acc<DT, MODE> a0;
    a0.init();
    using WV = decltype(a0.finish());
    WV tv[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const bool any = (w == 0 && rg.head > 0) || w * 64 * V < body_n;   // uniform
        if (!any) {
            if constexpr (MODE == COMP) tv[w] = Pair{0.f, 0.f};
            else tv[w] = WV(0);
            continue;
        }
        Acc<DT, MODE> acc;
        acc.init();
        if (w == 0 && l == 0 && rg.head > 0) {
            // the head, in order, into accumulator 0 (as reduce_chunk adds it)
            const int h0 = (int)((uintptr_t)rg.ptr & 15) / EB;
#pragma unroll
            for (int i = 1; i < V; i++)
                if (i >= h0 && i < h0 + rg.head) acc_from_vec(acc, r.hv, i, 0);
        }
        // row 0 reaches each accumulator first (unless the head came before
        // it, in set 0): the zero-accumulator shortcut, bit-identical
        const bool first_ok = !(w == 0 && rg.head > 0);   // uniform
#pragma unroll
        for (int u = 0; u < US; u++) {
            const int v0 = (u * NTHR + w * 64) * V;   // first element of the slot
            if (v0 >= body_n) continue;                // uniform: no lane has data
            uint4 v = r.v[u][w];
            // the slot that holds the end of the body: each lane keeps the
            // elements of its vector that lie in the body (a lane past the
            // end, which loaded a copy of the last vector, keeps none)
            if (v0 + 64 * V > body_n) v = first_elems<DT>(v, body_n - (v0 + l * V));   // uniform
            if (u == 0 && first_ok) acc_vec<DT, MODE, true>(acc, v);
            else acc_vec(acc, v);
        }
        tv[w] = acc.finish();
    }
    const WV res = wave_reduce4(tv);
    if constexpr (MODE == COMP) return pair_value(res);
    else return res;
}


// ---------------------------------------------------------------- grid combine

// Wave-level butterfly for the grid combine (xor 1 .. 32).
template <typename P> __device__ __forceinline__ P wave_butterfly(P v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        if constexpr (sizeof(P) == 8) {
            const uint64_t b = __builtin_bit_cast(uint64_t, v);
            const uint64_t o = (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)b, m, 64) |
                               ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(b >> 32), m, 64) << 32);
            v = v + __builtin_bit_cast(P, o);
        } else {
            v = v + __builtin_bit_cast(P, __shfl_xor(__builtin_bit_cast(int, v), m, 64));
        }
    }
    return v;
}

// Partials and tickets are exchanged only through agent-scope atomic
// read-modify-writes, which are performed at the device's coherence point (the
// L2s of the 8 XCDs are not coherent with each other).  No cache-maintenance
// fence is used: a writer waits for its partial's exchange to return before it
// takes a ticket, and the group's last workgroup reads the partials back with
// atomic RMWs, so it sees every value published before the tickets it counted.
template <typename P> __device__ __forceinline__ void publish(P *p, P v) {
    if constexpr (sizeof(P) == 8) {
        __hip_atomic_exchange(reinterpret_cast<uint64_t *>(p), __builtin_bit_cast(uint64_t, v),
                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_exchange(reinterpret_cast<uint32_t *>(p), __builtin_bit_cast(uint32_t, v),
                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}
template <typename P> __device__ __forceinline__ P fetch(P *p) {
    if constexpr (sizeof(P) == 8) {
        return __builtin_bit_cast(P, __hip_atomic_fetch_or(reinterpret_cast<uint64_t *>(p),
                                                           (uint64_t)0, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
    } else {
        return __builtin_bit_cast(P, __hip_atomic_fetch_or(reinterpret_cast<uint32_t *>(p), 0u,
                                                           __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
    }
}
// wait until every memory operation this wave issued has completed
__device__ __forceinline__ void drain() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Group sum of up to 256 partials by one wave: lane l adds its four
// consecutive partials as (p[4l] + p[4l+1]) + (p[4l+2] + p[4l+3]), then the
// xor butterfly over the 64 lanes -- a balanced pairwise tree over the 256
// indices (zero-padded), the same association at every call site.
// ATOMIC: read through agent-scope RMWs (partials published by workgroups of
// the same launch); otherwise plain loads (partials written by an earlier
// launch on the stream).  The arithmetic is the same either way.
template <typename P, bool ATOMIC = true>
__device__ __forceinline__ P group_sum(const P *part, int64_t gsize) {
    const int l = threadIdx.x & 63;
    P q[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (4 * l + i >= gsize) q[i] = (P)0;
        else if constexpr (ATOMIC) q[i] = fetch(const_cast<P *>(&part[4 * l + i]));
        else q[i] = part[4 * l + i];
    }
    return wave_butterfly<P>((q[0] + q[1]) + (q[2] + q[3]));
}

// Grid combine, run by the first wave of a workgroup only (the other waves
// have already left, so they never wait on the atomics' round trips).
template <int MODE>
__device__ void grid_combine(const Range &rg, int64_t j, typename PartT<MODE>::T value,
                             const Levels &lv) {
    using P = typename PartT<MODE>::T;
    const int l = threadIdx.x & 63;
    int64_t idx = j, cnt = rg.nchunks;
    for (int level = 0;; level++) {
        if (cnt == 1) {
            if (l == 0) *reinterpret_cast<P *>(rg.dst) = value;
            return;
        }
        const int64_t g = idx / RADIX;
        const int64_t gsize = (cnt - g * RADIX) < RADIX ? (cnt - g * RADIX) : RADIX;
        P *part = reinterpret_cast<P *>(lv.part[level]);
        uint32_t *ticket = lv.ctr + (rg.chunk_base + g) * MAXLEV + level;
        int mine = 0;
        if (l == 0) {
            publish(&part[rg.chunk_base + idx], value);
            drain();           // the partial is at the coherence point before the ticket
            uint32_t old = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
            mine = (old == (uint32_t)(gsize - 1));
        }
        if (!__shfl(mine, 0, 64)) return;
        value = group_sum<P>(part + rg.chunk_base + g * RADIX, gsize);
        if (l == 0)            // leave the ticket at zero for the next call
            __hip_atomic_exchange(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        idx = g;
        cnt = (cnt + RADIX - 1) / RADIX;
    }
}

// ---------------------------------------------------------------- kernels

// Single range (reduce_sum): one workgroup per chunk.
template <int DT, int MODE, bool NT>
__global__ void __launch_bounds__(NTHR) k_reduce_one(Range rg, Levels lv) {
    const int64_t j = blockIdx.x;
    auto v = reduce_chunk<DT, MODE, NT>(rg, j);
    if (threadIdx.x >= 64) return;
    grid_combine<MODE>(rg, j, v, lv);
}

// Single range, split combine: each workgroup writes its chunk's value with a
// plain store and retires at once (no atomics, no waiting); k_combine_level
// launches then add the partials level by level.
template <int DT, int MODE, bool NT>
__global__ void __launch_bounds__(NTHR) k_reduce_parts(Range rg, Levels lv) {
    using P = typename PartT<MODE>::T;
    const int64_t j = blockIdx.x;
    const P v = reduce_chunk<DT, MODE, NT>(rg, j);
    if (threadIdx.x == 0) reinterpret_cast<P *>(lv.part[0])[rg.chunk_base + j] = v;
}

// One level of the combine tree: wave g sums partials [256 g, 256 g + 256) of
// `in` (cnt of them) exactly as the last workgroup of a ticket group does, and
// writes the level's partial g, or the result when the level has one group.
template <typename P>
__global__ void __launch_bounds__(NTHR) k_combine_level(const P *__restrict__ in, int64_t cnt,
                                                        P *__restrict__ out, P *__restrict__ dst) {
    const int64_t g = (int64_t)blockIdx.x * NW + (threadIdx.x >> 6);
    const int64_t ng = (cnt + RADIX - 1) / RADIX;
    if (g >= ng) return;
    const int64_t gsize = (cnt - g * RADIX) < RADIX ? (cnt - g * RADIX) : RADIX;
    const P v = group_sum<P, false>(in + g * RADIX, gsize);
    if ((threadIdx.x & 63) == 0) {
        if (ng == 1) *dst = v;
        else out[g] = v;
    }
}

// Many ranges from a host-built table (reduce_sum_batched): workgroup b takes
// global chunk b and finds its range by binary search over chunk_base.
template <int DT, int MODE, bool NT>
__device__ __forceinline__ void table_chunk(const Range *tab, int nr, const Levels &lv) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].chunk_base <= b) lo = mid; else hi = mid - 1;
    }
    const Range rg = tab[lo];
    const int64_t j = b - rg.chunk_base;
    if (j >= rg.nchunks) return;
    auto v = reduce_chunk<DT, MODE, NT>(rg, j);
    if (threadIdx.x >= 64) return;
    grid_combine<MODE>(rg, j, v, lv);
}

template <int DT, int MODE, bool NT>
__global__ void __launch_bounds__(NTHR) k_reduce_table(const Range *__restrict__ tab, int nr,
                                                     Levels lv) {
    table_chunk<DT, MODE, NT>(tab, nr, lv);
}

// A small batch passes its ranges inside the kernel arguments: no table
// upload (no host-to-device copy ahead of the kernel in the stream).
constexpr int INLINE_RANGES = 32;
struct RangePack {
    Range r[INLINE_RANGES];
};

template <int DT, int MODE, bool NT>
__global__ void __launch_bounds__(NTHR) k_reduce_table_inl(RangePack pk, int nr, Levels lv) {
    table_chunk<DT, MODE, NT>(pk.r, nr, lv);
}

// ---------------------------------------------------------------- segmented

// Segment geometry from its bounds [lo, hi) (a decreasing pair reads as
// empty here; k_seg_count flags it), identical to the host-side one of single
// ranges.
__device__ __forceinline__ Range seg_range_lh(const unsigned char *src, int64_t lo, int64_t hi,
                                              int64_t s, int eb, int64_t ch, unsigned char *out,
                                              int osz) {
    if (hi < lo) hi = lo;
    Range r;
    r.ptr = src + lo * eb;
    r.n = hi - lo;
    const int mis = (int)((uintptr_t)r.ptr & 15);
    int head = mis ? (16 - mis) / eb : 0;
    if (head > r.n) head = (int)r.n;
    r.head = head;
    const int64_t body = r.n - head;
    r.nchunks = body > 0 ? (body + ch - 1) / ch : 1;
    r.dst = out + s * osz;
    r.chunk_base = 0;
    r._pad = 0;
    return r;
}
__device__ __forceinline__ Range seg_range(const unsigned char *src, const int64_t *off, int64_t s,
                                           int eb, int64_t ch, unsigned char *out = nullptr,
                                           int osz = 8) {
    return seg_range_lh(src, off[s], off[s + 1], s, eb, ch, out, osz);
}

// Chunk j of segment s, whose elements are [lo, hi) of the source: one
// record per chunk of the chunked segments, so the reducing workgroup needs a
// single metadata load.
struct ChunkRec {
    int64_t lo, hi;
    int32_t s, j;
};

// Pass 1: chunk count of every segment, and per-block totals.
__global__ void __launch_bounds__(NTHR) k_seg_count(const unsigned char *src, const int64_t *off,
                                                  int64_t nseg, int eb, int64_t ch,
                                                  int64_t small, int64_t *counts,
                                                  int64_t *block_tot) {
    __shared__ int64_t sh[NW];
    const int64_t base = (int64_t)blockIdx.x * NTHR * 4;
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int64_t s = base + k * NTHR + threadIdx.x;
        if (s < nseg) {
            const Range r = seg_range(src, off, s, eb, ch);
            // small segments are reduced by one wave each and take no chunk slot
            int64_t c = (r.n - r.head <= small) ? 0 : r.nchunks;
            // a decreasing pair or a negative start poisons the total so that
            // the reduction kernel sees it exceed the chunk space (invalid table)
            if (off[s + 1] < off[s] || off[s] < 0) c = (int64_t)1 << 40;
            counts[s] = c;
            sum += c;
        }
    }
    uint64_t w = wave_reduce((uint64_t)sum);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = (int64_t)w;
    __syncthreads();
    if (threadIdx.x == 0) block_tot[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Pass 2: exclusive scan of the block totals by one workgroup (in place);
// also writes the grand total after the last block total.
__global__ void __launch_bounds__(NTHR) k_seg_scan_blocks(int64_t *block_tot, int64_t nblk) {
    __shared__ int64_t sh[NTHR];
    int64_t carry = 0;
    for (int64_t base = 0; base < nblk; base += NTHR) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nblk ? block_tot[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < NTHR; d <<= 1) {   // Hillis-Steele inclusive scan
            int64_t a = threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < nblk) block_tot[i] = carry + sh[threadIdx.x] - v;
        carry += sh[NTHR - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_tot[nblk] = carry;
}

// Pass 3: chunk_base of every segment and the chunk records.  The block's
// start in the chunk space is the sum of the block totals before it: read
// from the scanned totals (prefix = true: pass 2 ran), or summed here from
// the raw totals (a block sums at most MAX_DIRECT_BLOCKS of them, so for
// small tables the pass-2 launch is skipped).  The records of the block's
// chunks are written by all its threads together: slot q of the block's
// chunk range belongs to the segment whose range holds it (found by a
// binary search over the block's segment starts in LDS), so a segment of
// many chunks costs no thread more than a few stores.
constexpr int64_t MAX_DIRECT_BLOCKS = 4096;

__global__ void __launch_bounds__(NTHR) k_seg_place(const int64_t *counts, const int64_t *block_tot,
                                                  bool prefix, int64_t nblk,
                                                  const int64_t *off, int64_t nseg, int64_t cap,
                                                  int64_t *chunk_base, ChunkRec *recs) {
    __shared__ int64_t sh[NTHR];
    __shared__ int64_t start[NTHR * 4 + 1];   // chunk offset (within the block) of each segment
    __shared__ int64_t sh_base;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * NTHR * 4;
    const int64_t s0 = base + t * 4;   // this thread's 4 consecutive segments
    // the block's start in the chunk space
    if (prefix) {
        if (t == 0) sh_base = block_tot[blockIdx.x];
    } else {
        int64_t part = 0;
        for (int64_t i = t; i < (int64_t)blockIdx.x; i += NTHR) part += block_tot[i];
        uint64_t wsum = wave_reduce((uint64_t)part);
        if ((t & 63) == 0) sh[t >> 6] = (int64_t)wsum;
        __syncthreads();
        if (t == 0) sh_base = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    }
    int64_t c[4], tsum = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        c[k] = (s0 + k < nseg) ? counts[s0 + k] : 0;
        tsum += c[k];
    }
    __syncthreads();
    sh[t] = tsum;
    __syncthreads();
    for (int d = 1; d < NTHR; d <<= 1) {
        int64_t a = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    const int64_t blk_base = sh_base;
    const int64_t blk_total = sh[NTHR - 1];
    int64_t run = sh[t] - tsum;   // within the block
#pragma unroll
    for (int k = 0; k < 4; k++) {
        start[t * 4 + k] = run;
        if (s0 + k < nseg) chunk_base[s0 + k] = blk_base + run;
        run += c[k];
    }
    if (t == NTHR - 1) start[NTHR * 4] = run;   // = blk_total
    if (blockIdx.x == nblk - 1 && t == 0) chunk_base[nseg] = blk_base + blk_total;
    __syncthreads();
    // the records, every thread taking slots q = t, t + 256, ...
    const int nloc = (int)((nseg - base) < NTHR * 4 ? (nseg - base) : NTHR * 4);
    if (blk_base + blk_total > cap) return;   // invalid table (or no space): no records
    for (int64_t q = t; q < blk_total; q += NTHR) {
        // the last segment i with start[i] <= q (segments with no chunks have
        // start[i] == start[i + 1] and are passed over)
        int lo = 0, hi = nloc;   // start[lo] <= q < start[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (start[mid] <= q) lo = mid;
            else hi = mid;
        }
        const int64_t s = base + lo;
        recs[blk_base + q] = ChunkRec{off[s], off[s + 1], (int32_t)s, (int32_t)(q - start[lo])};
    }
}

// Pass 4a: small segments, one wave each: the waves of the grid stride over the
// segments (indices are wave-uniform, so the offsets come through scalar
// loads, one segment ahead).  A segment's loads are all issued before its
// value is computed from registers; the other waves of the SIMD cover the
// wait.
template <int DT, int MODE, bool NT>
__device__ __forceinline__ void small_segments(const unsigned char *src, const int64_t *off,
                                               int64_t nseg, void *out) {
    using P = typename PartT<MODE>::T;
    const int64_t nwaves = (int64_t)gridDim.x * NW;
    int64_t s = (int64_t)blockIdx.x * NW + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t lo = 0, hi = 0;
    if (s < nseg) lo = off[s], hi = off[s + 1];
    for (; s < nseg; s += nwaves) {
        const int64_t sn = s + nwaves;
        int64_t lo_n = 0, hi_n = 0;
        if (sn < nseg) lo_n = off[sn], hi_n = off[sn + 1];
        const Range rg = seg_range_lh(src, lo, hi, s, DTI<DT>::EB, chunk_elems<DT>(),
                                      (unsigned char *)out, (int)sizeof(P));
        if (rg.n - rg.head <= small_max<DT>()) {   // else a chunked segment (pass 4b)
            SmallRegs<2> r;
            small_load<DT, 2, NT>(rg, true, off, r);
            const P v = small_value<DT, MODE, 2>(rg, r);
            if ((threadIdx.x & 63) == 0) *reinterpret_cast<P *>(rg.dst) = v;
        }
        lo = lo_n;
        hi = hi_n;
    }
}

template <int DT, int MODE, bool NT>
__global__ void __launch_bounds__(NTHR) k_reduce_seg_small(const unsigned char *src,
                                                         const int64_t *off,
                                                         const int64_t *chunk_base, int64_t nseg,
                                                         int64_t cap, void *out) {
    if (chunk_base[nseg] > cap) return;   // invalid table: k_reduce_seg writes every output
    small_segments<DT, MODE, NT>(src, off, nseg, out);
}

// Pass 4b: the chunks of the other segments, workgroups striding over the
// chunk records (the next record is loaded before this chunk's data).  The
// first wave runs the grid combine of each chunk while the others go on to
// the next chunk (they meet again at its LDS barrier).
template <int DT, int MODE, bool NT>
__global__ void __launch_bounds__(NTHR) k_reduce_seg(const unsigned char *src,
                                                   const int64_t *chunk_base,
                                                   const ChunkRec *__restrict__ recs, int64_t nseg,
                                                   int64_t cap, Levels lv, void *out) {
    using P = typename PartT<MODE>::T;
    const int64_t total = chunk_base[nseg];
    if (total > cap) {   // invalid offsets table: defined outputs, no reads, no tickets
        for (int64_t s = (int64_t)blockIdx.x * NTHR + threadIdx.x; s < nseg;
             s += (int64_t)gridDim.x * NTHR) {
            if constexpr (MODE == INTM) reinterpret_cast<P *>(out)[s] = 0;
            else reinterpret_cast<P *>(out)[s] = (P)__builtin_nan("");
        }
        return;
    }
    int64_t b = blockIdx.x;
    ChunkRec cr{};
    if (b < total) cr = recs[b];
    for (; b < total; b += gridDim.x) {
        ChunkRec nx{};
        if (b + gridDim.x < total) nx = recs[b + gridDim.x];
        Range rg = seg_range_lh(src, cr.lo, cr.hi, cr.s, DTI<DT>::EB, chunk_elems<DT>(),
                                (unsigned char *)out, (int)sizeof(P));
        rg.chunk_base = b - cr.j;
        auto v = reduce_chunk<DT, MODE, NT>(rg, cr.j);
        if (threadIdx.x < 64) grid_combine<MODE>(rg, cr.j, v, lv);
        cr = nx;
    }
}

// Both passes in one launch: each workgroup reduces chunk records first
// (as k_reduce_seg), then its waves take small segments (as
// k_reduce_seg_small), so the fine-grained small segments fill the tail of
// the chunk work.  Same arithmetic, same results.
template <int DT, int MODE, bool NT>
__global__ void __launch_bounds__(NTHR) k_reduce_seg_all(const unsigned char *src,
                                                       const int64_t *off,
                                                       const int64_t *chunk_base,
                                                       const ChunkRec *__restrict__ recs,
                                                       int64_t nseg, int64_t cap, Levels lv,
                                                       void *out) {
    using P = typename PartT<MODE>::T;
    const int64_t total = chunk_base[nseg];
    if (total > cap) {   // invalid offsets table: defined outputs, no reads, no tickets
        for (int64_t s = (int64_t)blockIdx.x * NTHR + threadIdx.x; s < nseg;
             s += (int64_t)gridDim.x * NTHR) {
            if constexpr (MODE == INTM) reinterpret_cast<P *>(out)[s] = 0;
            else reinterpret_cast<P *>(out)[s] = (P)__builtin_nan("");
        }
        return;
    }
    int64_t b = blockIdx.x;
    ChunkRec cr{};
    if (b < total) cr = recs[b];
    for (; b < total; b += gridDim.x) {
        ChunkRec nx{};
        if (b + gridDim.x < total) nx = recs[b + gridDim.x];
        Range rg = seg_range_lh(src, cr.lo, cr.hi, cr.s, DTI<DT>::EB, chunk_elems<DT>(),
                                (unsigned char *)out, (int)sizeof(P));
        rg.chunk_base = b - cr.j;
        auto v = reduce_chunk<DT, MODE, NT>(rg, cr.j);
        if (threadIdx.x < 64) grid_combine<MODE>(rg, cr.j, v, lv);
        cr = nx;
    }
    small_segments<DT, MODE, NT>(src, off, nseg, out);
}

// ---------------------------------------------------------------- host side

int part_bytes(int mode) { return mode == PLAIN ? 4 : 8; }
size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// A reduction workspace is [tickets | data].  The ticket region is the first
// quarter of the workspace (rounded down to 256 bytes) whatever the call, so
// the tickets never move when calls of different sizes share one workspace;
// every call returns the tickets it used to zero.  Partials and the segmented
// tables live in the data region, which is always written before it is read.
struct WsView {
    uint32_t *tickets;
    size_t ticket_cap;      // entries
    unsigned char *data;
    size_t data_bytes;
};
WsView split_ws(void *ws, size_t bytes) {
    WsView v;
    const size_t c = (bytes / 4) / 256 * 256;
    v.tickets = reinterpret_cast<uint32_t *>(ws);
    v.ticket_cap = c / 4;
    v.data = reinterpret_cast<unsigned char *>(ws) + c;
    v.data_bytes = bytes - c;
    return v;
}
bool ws_fits(size_t bytes, int64_t slots, size_t data_bytes) {
    const WsView v = split_ws(nullptr, bytes);
    return v.ticket_cap >= (size_t)slots * MAXLEV && v.data_bytes >= data_bytes;
}
// smallest 256-byte multiple that holds `slots` ticket slots and `data_bytes`
size_t ws_size_for(int64_t slots, size_t data_bytes) {
    size_t w = al256(std::max((size_t)slots * MAXLEV * 4 * 4, data_bytes + data_bytes / 3) + 1024);
    while (!ws_fits(w, slots, data_bytes)) w += 256;
    return w;
}
// bytes of the per-level partial arrays for `slots` chunk slots
size_t parts_bytes(int64_t slots, int mode) { return al256((size_t)slots * part_bytes(mode)) * MAXLEV; }

Levels levels_at(const WsView &v, unsigned char *parts, int64_t slots, int mode) {
    Levels lv;
    const size_t pb = al256((size_t)slots * part_bytes(mode));
    for (int l = 0; l < MAXLEV; l++) lv.part[l] = parts + l * pb;
    lv.ctr = v.tickets;
    return lv;
}

// Get a workspace (caller's or the library's) for `slots` chunk slots and
// `data` bytes of data region; *view describes it.
int get_ws(void *ws, size_t ws_bytes, int64_t slots, size_t data, hipStream_t st,
           const char *who, WsView *view) {
    if (ws) {
        if (!ws_fits(ws_bytes, slots, data))
            return fail(XTR_EBUDGET, "%s: workspace %zu bytes < %zu needed", who, ws_bytes,
                        ws_size_for(slots, data));
    } else {
        int rc = workspace(WS_REDUCE, st, ws_size_for(slots, data), &ws, &ws_bytes);
        if (rc) return rc;
    }
    *view = split_ws(ws, ws_bytes);
    return XTR_OK;
}

Range host_range(const void *p, int64_t n, int dtype, void *dst) {
    const int eb = elem_bytes(dtype);
    const int64_t ch = chunk_elems_rt(dtype);
    Range r;
    r.ptr = (const unsigned char *)p;
    r.n = n;
    const int mis = (int)((uintptr_t)p & 15);
    int64_t head = mis ? (16 - mis) / eb : 0;
    if (head > n) head = n;
    r.head = (int32_t)head;
    const int64_t body = n - head;
    r.nchunks = body > 0 ? (body + ch - 1) / ch : 1;
    r.chunk_base = 0;
    r.dst = (unsigned char *)dst;
    r._pad = 0;
    return r;
}

int mode_for(int dtype, bool plain) {
    if (is_int_sum_dtype(dtype)) return INTM;
    return plain ? PLAIN : COMP;
}

int check_sum_args(const void *src, int64_t n, const void *out, int dtype, bool plain,
                   const char *who) {
    const int eb = elem_bytes(dtype);
    if (!is_float_sum_dtype(dtype) && !is_int_sum_dtype(dtype))
        return fail(XTR_EDTYPE, "%s: dtype %d is not summable", who, dtype);
    if (plain && !is_float_sum_dtype(dtype))
        return fail(XTR_EDTYPE, "%s: plain fp32 comparator takes float dtypes only", who);
    if (n < 0) return fail(XTR_EINVAL, "%s: negative n", who);
    if (!out) return fail(XTR_EINVAL, "%s: null out", who);
    if (n > 0 && !src) return fail(XTR_EINVAL, "%s: null src", who);
    if ((uintptr_t)src % eb) return fail(XTR_EALIGN, "%s: src not aligned to its element", who);
    if ((uintptr_t)out % (plain ? 4 : 8)) return fail(XTR_EALIGN, "%s: out misaligned", who);
    return XTR_OK;
}

#define XTR_DISPATCH_SUM(DTYPE, MODE, KERNEL, ...)                                           \
    switch ((DTYPE) * 4 + (MODE)) {                                                          \
    case XTR_F32 * 4 + COMP: KERNEL<XTR_F32, COMP> __VA_ARGS__; break;                       \
    case XTR_F16 * 4 + COMP: KERNEL<XTR_F16, COMP> __VA_ARGS__; break;                       \
    case XTR_BF16 * 4 + COMP: KERNEL<XTR_BF16, COMP> __VA_ARGS__; break;                     \
    case XTR_F8E4M3 * 4 + COMP: KERNEL<XTR_F8E4M3, COMP> __VA_ARGS__; break;                 \
    case XTR_F32 * 4 + PLAIN: KERNEL<XTR_F32, PLAIN> __VA_ARGS__; break;                     \
    case XTR_F16 * 4 + PLAIN: KERNEL<XTR_F16, PLAIN> __VA_ARGS__; break;                     \
    case XTR_BF16 * 4 + PLAIN: KERNEL<XTR_BF16, PLAIN> __VA_ARGS__; break;                   \
    case XTR_F8E4M3 * 4 + PLAIN: KERNEL<XTR_F8E4M3, PLAIN> __VA_ARGS__; break;               \
    case XTR_I32 * 4 + INTM: KERNEL<XTR_I32, INTM> __VA_ARGS__; break;                       \
    case XTR_I64 * 4 + INTM: KERNEL<XTR_I64, INTM> __VA_ARGS__; break;                       \
    default: return fail(XTR_EDTYPE, "internal: no kernel for dtype %d mode %d", DTYPE, MODE); \
    }

// Tuned settings per dtype (index = dtype code).
constexpr int SPLIT_DEFAULT = 1024;
// g_rcfg[XTR_SHAPE_SINGLE]: single ranges (reduce_sum, its _ws / no-allocation /
// host forms); g_rcfg[XTR_SHAPE_BATCHED]: batched and segmented launches.
xtr_reduce_config g_rcfg[2][XTR_U16 + 1] = {};
bool rcfg_init() {
    for (auto &cls : g_rcfg)
        for (auto &c : cls) {
            c.nt_load = 1;
            c.split_chunks = SPLIT_DEFAULT;
        }
    return true;
}
bool g_rcfg_ready = rcfg_init();

// In-kernel ticket combine: one workgroup per chunk of rg.
template <int DT, int MODE>
void launch_one_ticket(const Range &rg, const Levels &lv, hipStream_t st) {
    if (g_rcfg[XTR_SHAPE_SINGLE][DT].nt_load)
        hipLaunchKernelGGL((k_reduce_one<DT, MODE, true>), dim3((unsigned)rg.nchunks), dim3(NTHR), 0,
                           st, rg, lv);
    else
        hipLaunchKernelGGL((k_reduce_one<DT, MODE, false>), dim3((unsigned)rg.nchunks), dim3(NTHR),
                           0, st, rg, lv);
}

// A range of at least split_chunks chunks (and more than one) uses the split
// combine; the others combine in-kernel through tickets.  Same value either way.
// Plain partials of the chunks of rg (written at chunk_base + j of level 0).
template <int DT, int MODE>
void launch_parts(const Range &rg, const Levels &lv, hipStream_t st) {
    const dim3 g((unsigned)rg.nchunks);
    if (g_rcfg[XTR_SHAPE_SINGLE][DT].nt_load)
        hipLaunchKernelGGL((k_reduce_parts<DT, MODE, true>), g, dim3(NTHR), 0, st, rg, lv);
    else
        hipLaunchKernelGGL((k_reduce_parts<DT, MODE, false>), g, dim3(NTHR), 0, st, rg, lv);
}
// The combine levels over cnt > 1 level-0 partials; the last writes *dst.
template <int MODE>
void launch_combine(const Levels &lv, int64_t cnt, void *dst, hipStream_t st) {
    using P = typename PartT<MODE>::T;
    for (int level = 0; cnt > 1; level++) {
        const int64_t ng = (cnt + RADIX - 1) / RADIX;
        const dim3 gl((unsigned)((ng + NW - 1) / NW));
        hipLaunchKernelGGL((k_combine_level<P>), gl, dim3(NTHR), 0, st,
                           reinterpret_cast<const P *>(lv.part[level]), cnt,
                           reinterpret_cast<P *>(lv.part[level + 1]), reinterpret_cast<P *>(dst));
        cnt = ng;
    }
}

template <int DT, int MODE>
void launch_one(const Range &rg, const Levels &lv, hipStream_t st) {
    const xtr_reduce_config &c = g_rcfg[XTR_SHAPE_SINGLE][DT];
    if (c.split_chunks > 0 && rg.nchunks >= c.split_chunks && rg.nchunks > 1) {
        launch_parts<DT, MODE>(rg, lv, st);
        launch_combine<MODE>(lv, rg.nchunks, rg.dst, st);
        return;
    }
    launch_one_ticket<DT, MODE>(rg, lv, st);
}
template <int DT, int MODE>
void launch_table_inl(const RangePack &pk, int nr, int64_t nchunks, const Levels &lv,
                      hipStream_t st) {
    if (g_rcfg[XTR_SHAPE_BATCHED][DT].nt_load)
        hipLaunchKernelGGL((k_reduce_table_inl<DT, MODE, true>), dim3((unsigned)nchunks),
                           dim3(NTHR), 0, st, pk, nr, lv);
    else
        hipLaunchKernelGGL((k_reduce_table_inl<DT, MODE, false>), dim3((unsigned)nchunks),
                           dim3(NTHR), 0, st, pk, nr, lv);
}
template <int DT, int MODE>
void launch_table(const Range *tab, int nr, int64_t nchunks, const Levels &lv, hipStream_t st) {
    if (g_rcfg[XTR_SHAPE_BATCHED][DT].nt_load)
        hipLaunchKernelGGL((k_reduce_table<DT, MODE, true>), dim3((unsigned)nchunks), dim3(NTHR), 0,
                           st, tab, nr, lv);
    else
        hipLaunchKernelGGL((k_reduce_table<DT, MODE, false>), dim3((unsigned)nchunks), dim3(NTHR), 0,
                           st, tab, nr, lv);
}
// Both passes run as grids that stride over their segments / chunks (the
// chunk space is only known on the device): the resident workgroups (8 per CU
// at most), or seg_over times as many, the later ones starting as earlier
// ones finish (measured: 4x the resident grid, 130 -> 120 us for 100k fp32
// segments).
// side: a second stream for the small segments (their launch then overlaps
// the chunks'), or nullptr.
template <int DT, int MODE>
void launch_seg(const unsigned char *src, const int64_t *off, const int64_t *cb, const ChunkRec *cs,
                int64_t nseg, int64_t cap, const Levels &lv, void *out, hipStream_t st,
                hipStream_t side) {
    const xtr_reduce_config &c = g_rcfg[XTR_SHAPE_BATCHED][DT];
    const bool nt = c.nt_load != 0;
    const int64_t gs_n = (nseg + NW - 1) / NW;                 // workgroups, one wave per segment
    const int64_t gc_n = cap > nseg ? cap : nseg;
    const int64_t over = c.seg_over > 1 ? c.seg_over : 1;      // grids beyond the resident ones
    hipStream_t ss = side ? side : st;
#define XTR_SEG(NTV)                                                                             \
    do {                                                                                         \
        const int64_t o1 = over * resident_blocks(                                               \
                                      (const void *)&k_reduce_seg_small<DT, MODE, NTV>, NTHR,    \
                                      c.seg_small_per_cu);                                       \
        const int64_t o2 = over * resident_blocks((const void *)&k_reduce_seg<DT, MODE, NTV>,    \
                                                  NTHR, c.seg_chunk_per_cu);                     \
        hipLaunchKernelGGL((k_reduce_seg_small<DT, MODE, NTV>),                                 \
                           dim3((unsigned)(gs_n < o1 ? gs_n : o1)), dim3(NTHR), 0, ss, src, off, \
                           cb, nseg, cap, out);                                                  \
        hipLaunchKernelGGL((k_reduce_seg<DT, MODE, NTV>),                                       \
                           dim3((unsigned)(gc_n < o2 ? gc_n : o2)), dim3(NTHR), 0, st, src, cb,  \
                           cs, nseg, cap, lv, out);                                              \
    } while (0)
#define XTR_SEG_ALL(NTV)                                                                         \
    do {                                                                                         \
        const int64_t o =                                                                        \
            over * resident_blocks((const void *)&k_reduce_seg_all<DT, MODE, NTV>, NTHR);         \
        const int64_t g = gc_n > gs_n ? gc_n : gs_n;                                             \
        hipLaunchKernelGGL((k_reduce_seg_all<DT, MODE, NTV>), dim3((unsigned)(g < o ? g : o)),   \
                           dim3(NTHR), 0, st, src, off, cb, cs, nseg, cap, lv, out);             \
    } while (0)
    if (c.seg_fused && !side) {
        if (nt) XTR_SEG_ALL(true);
        else XTR_SEG_ALL(false);
    } else {
        if (nt) XTR_SEG(true);
        else XTR_SEG(false);
    }
#undef XTR_SEG_ALL
#undef XTR_SEG
}

int sum_one(const void *src, int64_t n, void *out, int dtype, bool plain, void *ws,
            size_t ws_bytes, hipStream_t st, const char *who) {
    int rc = check_sum_args(src, n, out, dtype, plain, who);
    if (rc) return rc;
    const int mode = mode_for(dtype, plain);
    Range rg = host_range(src, n, dtype, out);
    if (rg.nchunks > 0x7fffffffLL) return fail(XTR_EINVAL, "%s: n too large", who);
    WsView v;
    rc = get_ws(ws, ws_bytes, rg.nchunks, parts_bytes(rg.nchunks, mode), st, who, &v);
    if (rc) return rc;
    Levels lv = levels_at(v, v.data, rg.nchunks, mode);
    XTR_DISPATCH_SUM(dtype, mode, launch_one, (rg, lv, st));
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

// Panels of the host-buffer sum hold this many chunks (32 MiB).
constexpr int64_t HOST_PANEL_CHUNKS = 1024;

template <int DT, int MODE>
void launch_host_panel(const Range &rg, const Levels &lv, bool single, hipStream_t st) {
    if (single) launch_one_ticket<DT, MODE>(rg, lv, st);
    else launch_parts<DT, MODE>(rg, lv, st);
}
template <int DT, int MODE>
void launch_host_combine(const Levels &lv, int64_t cnt, void *dst, hipStream_t st) {
    launch_combine<MODE>(lv, cnt, dst, st);
}

// Sum of a host array through the device, panel by panel (the copy in of
// panel k+1 overlaps the reduction of panel k).  The chunking is that of the
// same n values at a 16-byte-aligned device address (no head): each panel's
// chunks write their partials at their global chunk index, and the combine
// levels then run over all of them, so the result equals reduce_sum of an
// aligned device copy bit for bit.
int sum_host_impl(const void *src, int64_t n, void *out, int dtype) {
    const char *who = "xtr_reduce_sum_host";
    int rc = check_sum_args(src, n, out, dtype, false, who);
    if (rc) return rc;
    const int mode = mode_for(dtype, false);
    const int64_t eb = elem_bytes(dtype), ch = chunk_elems_rt(dtype);
    const int64_t nchunks = n > 0 ? (n + ch - 1) / ch : 1;
    if (nchunks > 0x7fffffffLL) return fail(XTR_EINVAL, "%s: n too large", who);
    HostPipe *p = nullptr;
    rc = host_pipe(&p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(p->mu);
    if ((rc = pipe_sync(p))) return rc;
    const bool spin = host_pinned(src);
    const int64_t pc = nchunks < HOST_PANEL_CHUNKS ? nchunks : HOST_PANEL_CHUNKS;
    const size_t pbytes = (size_t)(pc * ch * eb);
    void *din[2], *sin[2] = {nullptr, nullptr}, *dres = nullptr;
    for (int b = 0; b < 2; b++) {
        if ((rc = pipe_dev(p, b, pbytes, &din[b]))) return rc;
        if (!spin && (rc = pipe_pin(p, b, pbytes, &sin[b]))) return rc;
    }
    if ((rc = pipe_dev(p, 2, 256, &dres))) return rc;
    WsView v;
    if ((rc = get_ws(nullptr, 0, nchunks, parts_bytes(nchunks, mode), p->comp, who, &v))) return rc;
    const Levels lv = levels_at(v, v.data, nchunks, mode);
    const unsigned char *hs = static_cast<const unsigned char *>(src);
    const int64_t np = (nchunks + pc - 1) / pc;
    for (int64_t k = 0; k < np; k++) {
        const int b = (int)(k & 1);
        const int64_t c0 = k * pc, ck = (nchunks - c0) < pc ? (nchunks - c0) : pc;
        const int64_t e0 = c0 * ch, nk = (n - e0) < ck * ch ? (n - e0) : ck * ch;
        if (k >= 2) XTR_HIP(hipStreamWaitEvent(p->in, p->k_done[b], 0));
        if (nk > 0) {
            if (spin) {
                XTR_HIP(hipMemcpyAsync(din[b], hs + e0 * eb, (size_t)(nk * eb),
                                       hipMemcpyHostToDevice, p->in));
            } else {
                if (k >= 2) XTR_HIP(hipEventSynchronize(p->in_done[b]));
                memcpy(sin[b], hs + e0 * eb, (size_t)(nk * eb));
                XTR_HIP(hipMemcpyAsync(din[b], sin[b], (size_t)(nk * eb), hipMemcpyHostToDevice,
                                       p->in));
            }
        }
        XTR_HIP(hipEventRecord(p->in_done[b], p->in));
        XTR_HIP(hipStreamWaitEvent(p->comp, p->in_done[b], 0));
        Range rg;
        rg.ptr = static_cast<const unsigned char *>(din[b]);
        rg.n = nk;
        rg.chunk_base = c0;
        rg.nchunks = ck;
        rg.dst = static_cast<unsigned char *>(dres);
        rg.head = 0;
        rg._pad = 0;
        XTR_DISPATCH_SUM(dtype, mode, launch_host_panel, (rg, lv, nchunks == 1, p->comp));
        XTR_HIP(hipEventRecord(p->k_done[b], p->comp));
    }
    if (nchunks > 1) XTR_DISPATCH_SUM(dtype, mode, launch_host_combine, (lv, nchunks, dres, p->comp));
    XTR_HIP(hipGetLastError());
    XTR_HIP(hipMemcpyAsync(out, dres, 8, hipMemcpyDeviceToHost, p->comp));
    return pipe_sync(p);
}

}  // namespace

size_t reduce_ws_bytes(int64_t n, int dtype, bool plain) {
    if (!is_float_sum_dtype(dtype) && !is_int_sum_dtype(dtype)) return 0;
    if (n < 0) return 0;
    Range rg = host_range((const void *)0, n, dtype, nullptr);
    return ws_size_for(rg.nchunks, parts_bytes(rg.nchunks, mode_for(dtype, plain)));
}

// Host table of a batch of ranges; returns the total chunk count in *total.
// outs == nullptr: range i writes out + i * (result size); else it writes outs[i].
int build_ranges(const void *const *srcs, const int64_t *ns, int64_t count, void *out,
                 void *const *outs, int dtype, const char *who, std::vector<Range> &tab,
                 int64_t *total) {
    if (count < 0) return fail(XTR_EINVAL, "%s: negative count", who);
    if (count > 0 && (!srcs || !ns)) return fail(XTR_EINVAL, "%s: null host array", who);
    if (count > 0x7fffffffLL) return fail(XTR_EINVAL, "%s: too many jobs", who);
    tab.resize((size_t)count);
    *total = 0;
    if (count > 0 && outs == nullptr && out == nullptr) return fail(XTR_EINVAL, "%s: null out", who);
    for (int64_t i = 0; i < count; i++) {
        void *dst = outs ? outs[i] : (void *)((unsigned char *)out + i * 8);
        int rc = check_sum_args(srcs[i], ns[i], dst, dtype, false, who);
        if (rc) {
            set_error("%s: job %lld: %s", who, (long long)i, xtr_last_error());
            return rc;
        }
        tab[i] = host_range(srcs[i], ns[i], dtype, dst);
        tab[i].chunk_base = *total;
        *total += tab[i].nchunks;
    }
    if (*total > 0x7fffffffLL) return fail(XTR_EINVAL, "%s: too many chunks", who);
    return XTR_OK;
}

int sum_batched_impl(const void *const *srcs, const int64_t *ns, int64_t count, void *out,
                     void *const *outs, int dtype, hipStream_t st, const char *who) {
    std::vector<Range> tab;
    int64_t total = 0;
    if (count == 0) return XTR_OK;
    int rc0 = build_ranges(srcs, ns, count, out, outs, dtype, who, tab, &total);
    if (rc0) return rc0;
    const int mode = mode_for(dtype, false);
    void *tw = nullptr;
    WsView v;
    int rc = get_ws(nullptr, 0, total, parts_bytes(total, mode), st, who, &v);
    if (rc) return rc;
    if (count <= INLINE_RANGES) {
        RangePack pk;
        for (int64_t i = 0; i < count; i++) pk.r[i] = tab[i];
        Levels lv = levels_at(v, v.data, total, mode);
        XTR_DISPATCH_SUM(dtype, mode, launch_table_inl, (pk, (int)count, total, lv, st));
        XTR_HIP(hipGetLastError());
        return XTR_OK;
    }
    rc = workspace(WS_TABLE, st, tab.size() * sizeof(Range), &tw);
    if (rc) return rc;
    rc = upload(tab.data(), tab.size() * sizeof(Range), tw, st);
    if (rc) return rc;
    Levels lv = levels_at(v, v.data, total, mode);
    XTR_DISPATCH_SUM(dtype, mode, launch_table, ((const Range *)tw, (int)count, total, lv, st));
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

// Segmented data region: counts, chunk_base (nseg+1), block totals, chunk map,
// level partials.
struct SegLayout {
    size_t counts, cbase, btot, cmap, parts, total;
};
SegLayout seg_layout(int64_t nseg, int64_t cap, int mode) {
    const int64_t nblk = (nseg + NTHR * 4 - 1) / (NTHR * 4);
    SegLayout L;
    L.counts = 0;
    L.cbase = L.counts + al256((size_t)nseg * 8);
    L.btot = L.cbase + al256((size_t)(nseg + 1) * 8);
    L.cmap = L.btot + al256((size_t)(nblk + 1) * 8);
    L.parts = L.cmap + al256((size_t)cap * sizeof(ChunkRec));
    L.total = L.parts + parts_bytes(cap, mode);
    return L;
}

size_t seg_ws_bytes(int64_t nseg, int64_t total_elems, int dtype) {
    if (!is_float_sum_dtype(dtype) && !is_int_sum_dtype(dtype)) return 0;
    if (nseg < 0 || total_elems < 0) return 0;
    const int64_t cap = nseg + (total_elems + chunk_elems_rt(dtype) - 1) / chunk_elems_rt(dtype);
    return ws_size_for(cap, seg_layout(nseg, cap, mode_for(dtype, false)).total);
}

// Largest chunk space a caller workspace of ws_bytes holds for nseg segments
// (at least nseg + 1 slots), or -1 when it holds less.
int64_t seg_cap_of(size_t ws_bytes, int64_t nseg, int mode) {
    auto fits = [&](int64_t cap) { return ws_fits(ws_bytes, cap, seg_layout(nseg, cap, mode).total); };
    constexpr int64_t LIM = 0x7fffffffLL;
    int64_t lo = nseg + 1;
    if (lo > LIM || !fits(lo)) return -1;
    int64_t top;                       // the first doubling that does not fit
    for (;;) {
        const int64_t nxt = 2 * lo > LIM ? LIM : 2 * lo;
        if (nxt == lo) return lo;      // LIM fits
        if (!fits(nxt)) {
            top = nxt;
            break;
        }
        lo = nxt;
    }
    while (top - lo > 1) {             // fits(lo), !fits(top)
        const int64_t mid = lo + (top - lo) / 2;
        if (fits(mid)) lo = mid;
        else top = mid;
    }
    return lo;
}

// total_elems >= 0: the chunk space is sized from it; -1: offsets[nseg] is
// read back; -2: the chunk space is what the caller workspace holds.
int sum_segmented_impl(const void *src, const int64_t *offsets, int64_t nseg, void *out,
                       int dtype, void *ws, size_t ws_bytes, int64_t total_elems,
                       hipStream_t st) {
    const char *who = "reduce_sum_segmented";
    if (nseg < 0) return fail(XTR_EINVAL, "%s: negative nseg", who);
    if (nseg == 0) return XTR_OK;
    if (!offsets || !out) return fail(XTR_EINVAL, "%s: null offsets or out", who);
    int rc = check_sum_args(src, 0, out, dtype, false, who);
    if (rc) return rc;
    if (!src) return fail(XTR_EINVAL, "%s: null src", who);
    if ((uintptr_t)offsets % 8) return fail(XTR_EALIGN, "%s: offsets misaligned", who);
    if (nseg > 0x7fffffffLL) return fail(XTR_EINVAL, "%s: too many segments", who);
    const int mode = mode_for(dtype, false);
    const int eb = elem_bytes(dtype);
    const int64_t ch = chunk_elems_rt(dtype);
    int64_t cap;
    if (total_elems == -2) {   // as much chunk space as the caller's workspace holds
        cap = seg_cap_of(ws_bytes, nseg, mode);
        if (cap < 0)
            return fail(XTR_EBUDGET, "%s: workspace %zu bytes holds fewer than nseg + 1 chunks",
                        who, ws_bytes);
    } else {
        if (total_elems < 0) {   // read offsets[nseg] back to size the chunk space
            XTR_HIP(hipMemcpyAsync(&total_elems, offsets + nseg, 8, hipMemcpyDeviceToHost, st));
            XTR_HIP(hipStreamSynchronize(st));
            if (total_elems < 0) return fail(XTR_EINVAL, "%s: offsets[nseg] < 0", who);
        }
        // Each segment has max(1, ceil(body / ch)) chunks, body <= its length, and
        // lengths (after clamping decreasing pairs to 0) sum to at most offsets[nseg]
        // minus offsets[0]; so nseg + ceil(total / ch) bounds the chunk space.
        cap = nseg + (total_elems + ch - 1) / ch;
        if (cap > 0x7fffffffLL) return fail(XTR_EINVAL, "%s: chunk space too large", who);
    }
    const SegLayout L = seg_layout(nseg, cap, mode);
    WsView v;
    rc = get_ws(ws, ws_bytes, cap, L.total, st, who, &v);
    if (rc) return rc;
    unsigned char *w = v.data;
    int64_t *counts = (int64_t *)(w + L.counts), *cbase = (int64_t *)(w + L.cbase);
    int64_t *btot = (int64_t *)(w + L.btot);
    ChunkRec *cmap = (ChunkRec *)(w + L.cmap);
    const int64_t nblk = (nseg + NTHR * 4 - 1) / (NTHR * 4);
    const int64_t small = (int64_t)2 * NTHR * (16 / eb);   // small_max<DT>() of the kernels
    hipLaunchKernelGGL(k_seg_count, dim3((unsigned)nblk), dim3(NTHR), 0, st,
                       (const unsigned char *)src, offsets, nseg, eb, ch, small, counts, btot);
    const bool scanned = nblk > MAX_DIRECT_BLOCKS;   // else each block sums the totals before it
    if (scanned) hipLaunchKernelGGL(k_seg_scan_blocks, dim3(1), dim3(NTHR), 0, st, btot, nblk);
    hipLaunchKernelGGL(k_seg_place, dim3((unsigned)nblk), dim3(NTHR), 0, st, (const int64_t *)counts,
                       (const int64_t *)btot, scanned, nblk, offsets, nseg, cap, cbase, cmap);
    XTR_HIP(hipGetLastError());
    Levels lv = levels_at(v, w + L.parts, cap, mode);
    const xtr_reduce_config &c = g_rcfg[XTR_SHAPE_BATCHED][dtype];
    if (c.seg_streams && !c.seg_fused) {
        // the small segments on the side stream, the chunks on st: fork after
        // the planning passes, join before returning
        SideStream *side = nullptr;
        rc = side_stream(&side);
        if (rc) return rc;
        std::lock_guard<std::mutex> lk(side->mu);
        rc = side_fork(side, st);
        if (rc) return rc;
        XTR_DISPATCH_SUM(dtype, mode, launch_seg,
                         ((const unsigned char *)src, offsets, (const int64_t *)cbase,
                          (const ChunkRec *)cmap, nseg, cap, lv, out, st, side->s));
        XTR_HIP(hipGetLastError());
        return side_join(side, st);
    }
    XTR_DISPATCH_SUM(dtype, mode, launch_seg,
                     ((const unsigned char *)src, offsets, (const int64_t *)cbase,
                      (const ChunkRec *)cmap, nseg, cap, lv, out, st, nullptr));
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

int sum_one_impl(const void *src, int64_t n, void *out, int dtype, bool plain, void *ws,
                 size_t ws_bytes, hipStream_t st, const char *who) {
    return sum_one(src, n, out, dtype, plain, ws, ws_bytes, st, who);
}

// ---------------------------------------------------------------- no allocation

// The workspace of reduce_sum_noalloc: a fixed device array, one copy per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): it passes the
// device address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[XTR_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current).
int scratch_ptr(void **p, const char *who) {
    int dev = 0;
    XTR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(XTR_EINVAL, "%s: device %d out of range", who, dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!q) return fail(XTR_EHIP, "%s: hipGetSymbolAddress(scratch) gave a null address", who);
        g_scratch_ptr[dev] = q;
    }
    *p = g_scratch_ptr[dev];
    return XTR_OK;
}

int sum_noalloc(const void *src, int64_t n, void *out, int dtype, hipStream_t st) {
    const char *who = "reduce_sum_noalloc";
    int rc = check_sum_args(src, n, out, dtype, false, who);
    if (rc) return rc;
    const int mode = mode_for(dtype, false);
    const Range rg = host_range(src, n, dtype, out);
    if (!ws_fits(XTR_NOALLOC_SCRATCH_BYTES, rg.nchunks, parts_bytes(rg.nchunks, mode)))
        return fail(XTR_EBUDGET, "%s: n = %lld needs %zu bytes of scratch, more than the "
                    "fixed %zu", who, (long long)n, ws_size_for(rg.nchunks, parts_bytes(rg.nchunks, mode)),
                    (size_t)XTR_NOALLOC_SCRATCH_BYTES);
    void *p = nullptr;
    if ((rc = scratch_ptr(&p, who))) return rc;
    // The array keeps the previous call's contents: clear the tickets this call
    // may use (a fill kernel; the partial arrays are written before they are read).
    const WsView v = split_ws(p, XTR_NOALLOC_SCRATCH_BYTES);
    if ((rc = zero_fill(v.tickets, (size_t)rg.nchunks * MAXLEV * 4, st))) return rc;
    return sum_one(src, n, out, dtype, false, p, XTR_NOALLOC_SCRATCH_BYTES, st, who);
}

}  // namespace xtr

extern "C" {

int reduce_sum(const void *src, int64_t n, void *out, int dtype, void *stream) {
    return xtr::sum_one_impl(src, n, out, dtype, false, nullptr, 0, (hipStream_t)stream,
                             "reduce_sum");
}

struct xtr_sum_plan {
    xtr::Range *tab = nullptr;     // device table
    int nr = 0;
    int64_t total = 0;             // chunks
    int dtype = 0, mode = 0;
    void *ws = nullptr;            // plan-owned workspace
    size_t ws_bytes = 0;
    void *out = nullptr;
};

int xtr_sum_plan_create(const void *const *srcs, const int64_t *ns, int64_t count, int dtype,
                        void *out, void *stream, xtr_sum_plan **plan) {
    using namespace xtr;
    if (!plan) return fail(XTR_EINVAL, "xtr_sum_plan_create: null plan");
    *plan = nullptr;
    std::vector<Range> tab;
    int64_t total = 0;
    if (count > 0 && !out) return fail(XTR_EINVAL, "xtr_sum_plan_create: null out");
    int rc = build_ranges(srcs, ns, count, out, nullptr, dtype, "xtr_sum_plan_create", tab, &total);
    if (rc) return rc;
    auto *p = new (std::nothrow) xtr_sum_plan();
    if (!p) return fail(XTR_ENOMEM, "xtr_sum_plan_create: out of host memory");
    p->nr = (int)count;
    p->total = total;
    p->dtype = dtype;
    p->mode = mode_for(dtype, false);
    p->out = out;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (count > 0) {
        p->ws_bytes = ws_size_for(total, parts_bytes(total, p->mode));
        e = hipMalloc(&p->ws, p->ws_bytes);
        if (e == hipSuccess) e = hipMalloc(&p->tab, tab.size() * sizeof(Range));
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->tab, tab.data(), tab.size() * sizeof(Range),
                               hipMemcpyHostToDevice, st);
        if (e == hipSuccess) rc = zero_fill(p->ws, p->ws_bytes, st);
        if (e == hipSuccess && !rc) e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess || rc) {
        if (!rc) rc = hip_fail(e, "xtr_sum_plan_create");
        if (p->ws) (void)hipFree(p->ws);
        if (p->tab) (void)hipFree(p->tab);
        delete p;
        return rc;
    }
    *plan = p;
    return XTR_OK;
}

int xtr_sum_plan_run(const xtr_sum_plan *p, void *stream) {
    using namespace xtr;
    if (!p) return fail(XTR_EINVAL, "xtr_sum_plan_run: null plan");
    if (p->nr == 0) return XTR_OK;
    const WsView v = split_ws(p->ws, p->ws_bytes);
    Levels lv = levels_at(v, v.data, p->total, p->mode);
    hipStream_t st = (hipStream_t)stream;
    XTR_DISPATCH_SUM(p->dtype, p->mode, launch_table, (p->tab, p->nr, p->total, lv, st));
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

int xtr_sum_plan_destroy(xtr_sum_plan *p) {
    if (!p) return XTR_OK;
    if (p->ws) (void)hipFree(p->ws);
    if (p->tab) (void)hipFree(p->tab);
    delete p;
    return XTR_OK;
}

int xtr_reduce_get_class_config(int dtype, int shape_class, xtr_reduce_config *cfg) {
    if (!cfg || !(xtr::is_float_sum_dtype(dtype) || xtr::is_int_sum_dtype(dtype)) ||
        (shape_class != XTR_SHAPE_SINGLE && shape_class != XTR_SHAPE_BATCHED))
        return xtr::fail(XTR_EINVAL, "xtr_reduce_get_class_config: bad arguments");
    *cfg = xtr::g_rcfg[shape_class][dtype];
    return XTR_OK;
}

int xtr_reduce_set_class_config(int dtype, int shape_class, const xtr_reduce_config *cfg) {
    if (!cfg || !(xtr::is_float_sum_dtype(dtype) || xtr::is_int_sum_dtype(dtype)) ||
        (shape_class != XTR_SHAPE_SINGLE && shape_class != XTR_SHAPE_BATCHED))
        return xtr::fail(XTR_EINVAL, "xtr_reduce_set_class_config: bad arguments");
    if (cfg->split_chunks < 0 || cfg->seg_small_per_cu < 0 || cfg->seg_small_per_cu > 64 ||
        cfg->seg_chunk_per_cu < 0 || cfg->seg_chunk_per_cu > 64 || cfg->seg_over < 0 ||
        cfg->seg_over > 16)
        return xtr::fail(XTR_EINVAL, "xtr_reduce_set_class_config: split_chunks >= 0, "
                                     "seg_*_per_cu in [0, 64], seg_over in [0, 16]");
    xtr::g_rcfg[shape_class][dtype] = *cfg;
    return XTR_OK;
}

int xtr_reduce_get_config(int dtype, xtr_reduce_config *cfg) {
    return xtr_reduce_get_class_config(dtype, XTR_SHAPE_SINGLE, cfg);
}

int xtr_reduce_set_config(int dtype, const xtr_reduce_config *cfg) {
    int rc = xtr_reduce_set_class_config(dtype, XTR_SHAPE_SINGLE, cfg);
    if (rc == XTR_OK) rc = xtr_reduce_set_class_config(dtype, XTR_SHAPE_BATCHED, cfg);
    return rc;
}

int xtr_reduce_sum_host(const void *src, int64_t n, void *out, int dtype) {
    return xtr::sum_host_impl(src, n, out, dtype);
}

int reduce_sum_plain_f32(const void *src, int64_t n, float *out, int dtype, void *stream) {
    return xtr::sum_one_impl(src, n, out, dtype, true, nullptr, 0, (hipStream_t)stream,
                             "reduce_sum_plain_f32");
}

size_t xtr_reduce_workspace_bytes(int64_t n, int dtype) {
    return xtr::reduce_ws_bytes(n, dtype, false);
}

int reduce_sum_noalloc(const void *src, int64_t n, void *out, int dtype, void *stream) {
    return xtr::sum_noalloc(src, n, out, dtype, (hipStream_t)stream);
}

int reduce_sum_ws(const void *src, int64_t n, void *out, int dtype, void *ws, size_t ws_bytes,
                  void *stream) {
    if (!ws) return xtr::fail(XTR_EINVAL, "reduce_sum_ws: null workspace");
    return xtr::sum_one_impl(src, n, out, dtype, false, ws, ws_bytes, (hipStream_t)stream,
                             "reduce_sum_ws");
}

int reduce_sum_batched(const void *const *srcs, const int64_t *ns, int64_t count, void *out,
                       int dtype, void *stream) {
    return xtr::sum_batched_impl(srcs, ns, count, out, nullptr, dtype, (hipStream_t)stream,
                                 "reduce_sum_batched");
}

int reduce_sum_batched_scatter(const void *const *srcs, const int64_t *ns, void *const *outs,
                               int64_t count, int dtype, void *stream) {
    if (count > 0 && !outs) return xtr::fail(XTR_EINVAL, "reduce_sum_batched_scatter: null outs");
    return xtr::sum_batched_impl(srcs, ns, count, nullptr, outs, dtype, (hipStream_t)stream,
                                 "reduce_sum_batched_scatter");
}

size_t xtr_segmented_workspace_bytes(int64_t nseg, int64_t total_elems, int dtype) {
    return xtr::seg_ws_bytes(nseg, total_elems, dtype);
}

int reduce_sum_segmented(const void *src, const int64_t *offsets, int64_t nseg, void *out,
                         int dtype, void *stream) {
    return xtr::sum_segmented_impl(src, offsets, nseg, out, dtype, nullptr, 0, -1,
                                   (hipStream_t)stream);
}

int reduce_sum_segmented_ws(const void *src, const int64_t *offsets, int64_t nseg, void *out,
                            int dtype, void *ws, size_t ws_bytes, void *stream) {
    if (!ws) return xtr::fail(XTR_EINVAL, "reduce_sum_segmented_ws: null workspace");
    return xtr::sum_segmented_impl(src, offsets, nseg, out, dtype, ws, ws_bytes, -2,
                                   (hipStream_t)stream);
}

int reduce_sum_segmented_ws_total(const void *src, const int64_t *offsets, int64_t nseg,
                                  int64_t total_elems, void *out, int dtype, void *ws,
                                  size_t ws_bytes, void *stream) {
    if (!ws) return xtr::fail(XTR_EINVAL, "reduce_sum_segmented_ws_total: null workspace");
    if (total_elems < 0) return xtr::fail(XTR_EINVAL, "reduce_sum_segmented_ws_total: total < 0");
    return xtr::sum_segmented_impl(src, offsets, nseg, out, dtype, ws, ws_bytes, total_elems,
                                   (hipStream_t)stream);
}

}  // extern "C"
