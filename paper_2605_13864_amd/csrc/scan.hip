// Prefix sums (scan) for gfx950: the parallel prefix sum that the thesis's
// conclusion names as the next case study after the tree reduction.
//
// What is computed: the inclusive scan out[i] = x[0] + ... + x[i], or the
// exclusive scan out[i] = x[0] + ... + x[i-1] (out[0] = 0), i.e. reduce_sum
// (Section 2.1) of every prefix.  Integers (int32 / int64) accumulate in
// 64-bit wrap-around arithmetic (exact; modulo 2^64 for int64); floats (fp32,
// bf16, fp16, fp8-e4m3fn) are decoded exactly and accumulated in fp64 in a
// fixed order, so the result is deterministic.
//
// How: reduce, then scan (four launches, no workgroup ever waits on
// another):
//   1. k_scan_tiles: one wave per tile of 64 lanes x V elements x SROWS rows
//      (16 KiB of input) sums its tile: lane-local running sums over the rows,
//      then a 64-lane butterfly.
//   2. k_scan_blocks / k_scan_offsets: the tile sums are scanned (exclusive)
//      in blocks of 1024 by many workgroups, then the block totals by one.
//   3. k_scan_apply: one wave per tile rescans it row by row: lane-local
//      prefixes of its V elements, an exclusive 64-lane scan of the lane totals
//      (shuffles), plus the carry of the rows before and the tile's offset;
//      the outputs of a row go out through LDS as whole-line stores.
// The input is read twice and the 8-byte outputs written once.
// Integer scans of 16-byte aligned inputs take one pass instead (k_scan_lookback,
// below): integer sums do not depend on their order, so a tile may add up the
// totals its predecessors publish in whatever state it finds them.
#include "common.hpp"

#pragma clang fp contract(off)

namespace xtr {
namespace {

constexpr int SNT = 256;            // threads per workgroup (4 waves = 4 tiles)
constexpr int SROWS = 16;           // 16-byte vectors per lane per tile
constexpr int OFF_NT = 1024;        // threads of the offset scan

template <int DT> struct ScanT;
template <> struct ScanT<XTR_F32> { static constexpr int EB = 4; using T = double; };
template <> struct ScanT<XTR_F16> { static constexpr int EB = 2; using T = double; };
template <> struct ScanT<XTR_BF16> { static constexpr int EB = 2; using T = double; };
template <> struct ScanT<XTR_F8E4M3> { static constexpr int EB = 1; using T = double; };
template <> struct ScanT<XTR_I32> { static constexpr int EB = 4; using T = uint64_t; };
template <> struct ScanT<XTR_I64> { static constexpr int EB = 8; using T = uint64_t; };

template <int DT> constexpr int svec() { return 16 / ScanT<DT>::EB; }
template <int DT> constexpr int64_t tile_elems() { return (int64_t)64 * svec<DT>() * SROWS; }

// element i (compile-time) of a 16-byte vector, decoded exactly
template <int DT> __device__ __forceinline__ typename ScanT<DT>::T sdecode(const uint4 &v, int i) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    if constexpr (DT == XTR_F32) {
        return (double)__uint_as_float(w[i]);
    } else if constexpr (DT == XTR_BF16) {
        const uint32_t h = (w[i >> 1] >> (16 * (i & 1))) & 0xffffu;
        return (double)__uint_as_float(h << 16);
    } else if constexpr (DT == XTR_F16) {
        const uint16_t h = (uint16_t)((w[i >> 1] >> (16 * (i & 1))) & 0xffffu);
        return (double)(float)__builtin_bit_cast(_Float16, h);
    } else if constexpr (DT == XTR_F8E4M3) {
        const uint32_t b = (w[i >> 2] >> (8 * (i & 3))) & 0xffu;
        return (double)__builtin_amdgcn_cvt_pk_f32_fp8((int)b, false)[0];
    } else if constexpr (DT == XTR_I32) {
        return (uint64_t)(int64_t)(int32_t)w[i];
    } else {
        return (i == 0) ? ((uint64_t)w[0] | ((uint64_t)w[1] << 32))
                        : ((uint64_t)w[2] | ((uint64_t)w[3] << 32));
    }
}

// an element at byte address p (edge loads)
template <int DT> __device__ __forceinline__ typename ScanT<DT>::T sdecode_at(const unsigned char *p) {
    if constexpr (DT == XTR_F32) {
        return (double)*reinterpret_cast<const float *>(p);
    } else if constexpr (DT == XTR_BF16) {
        return (double)__uint_as_float((uint32_t)*reinterpret_cast<const uint16_t *>(p) << 16);
    } else if constexpr (DT == XTR_F16) {
        return (double)(float)__builtin_bit_cast(_Float16, *reinterpret_cast<const uint16_t *>(p));
    } else if constexpr (DT == XTR_F8E4M3) {
        return (double)__builtin_amdgcn_cvt_pk_f32_fp8((int)(uint32_t)*p, false)[0];
    } else if constexpr (DT == XTR_I32) {
        return (uint64_t)(int64_t)*reinterpret_cast<const int32_t *>(p);
    } else {
        return *reinterpret_cast<const uint64_t *>(p);
    }
}

template <typename T> __device__ __forceinline__ T shfl_up64(T v, int d) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t o = (uint64_t)(uint32_t)__shfl_up((int)(uint32_t)b, d, 64) |
                       ((uint64_t)(uint32_t)__shfl_up((int)(uint32_t)(b >> 32), d, 64) << 32);
    return __builtin_bit_cast(T, o);
}
template <typename T> __device__ __forceinline__ T shfl_xor64(T v, int m) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t o = (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)b, m, 64) |
                       ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(b >> 32), m, 64) << 32);
    return __builtin_bit_cast(T, o);
}
template <typename T> __device__ __forceinline__ T shfl64(T v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t o = (uint64_t)(uint32_t)__shfl((int)(uint32_t)b, lane, 64) |
                       ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(b >> 32), lane, 64) << 32);
    return __builtin_bit_cast(T, o);
}

// The V elements lane l holds in row r of tile t: elements
// t * TILE + r * 64V + l * V + i.  Elements at or past n read as 0.  With VEC
// (16-byte aligned src) rows are read as 16-byte vectors, RG rows at a time,
// all RG issued before any is used.
typedef uint32_t su32x4 __attribute__((ext_vector_type(4)));

template <int DT, bool VEC, int RG> struct RowGroup {
    uint4 raw[RG];
    __device__ __forceinline__ void load(const unsigned char *src, int64_t n, int64_t base, int l,
                                         int r0) {
        constexpr int EB = ScanT<DT>::EB, V = svec<DT>();
        if constexpr (VEC) {
#pragma unroll
            for (int k = 0; k < RG; k++) {
                const int64_t e0 = base + (int64_t)(r0 + k) * 64 * V + (int64_t)l * V;
                raw[k] = make_uint4(0, 0, 0, 0);
                if (e0 + V <= n) raw[k] = *reinterpret_cast<const uint4 *>(src + e0 * EB);
            }
        }
    }
    // decoded elements of row r0 + k
    __device__ __forceinline__ void row(const unsigned char *src, int64_t n, int64_t base, int l,
                                        int r0, int k, typename ScanT<DT>::T *x) const {
        constexpr int EB = ScanT<DT>::EB, V = svec<DT>();
        using T = typename ScanT<DT>::T;
        const int64_t e0 = base + (int64_t)(r0 + k) * 64 * V + (int64_t)l * V;
        if (VEC && e0 + V <= n) {
#pragma unroll
            for (int i = 0; i < V; i++) x[i] = sdecode<DT>(raw[k], i);
        } else {
#pragma unroll
            for (int i = 0; i < V; i++)
                x[i] = (e0 + i < n) ? sdecode_at<DT>(src + (e0 + i) * EB) : T(0);
        }
    }
};

// Pass 1: the sum of every tile.
template <int DT, bool VEC>
__global__ void __launch_bounds__(SNT) k_scan_tiles(const unsigned char *__restrict__ src, int64_t n,
                                                    int64_t ntiles,
                                                    typename ScanT<DT>::T *__restrict__ sums) {
    using T = typename ScanT<DT>::T;
    constexpr int V = svec<DT>();
    const int64_t t = (int64_t)blockIdx.x * (SNT / 64) + (threadIdx.x >> 6);
    if (t >= ntiles) return;
    const int l = threadIdx.x & 63;
    const int64_t base = t * tile_elems<DT>();
    constexpr int EB = ScanT<DT>::EB;
    T acc = T(0);
    if (VEC && base + tile_elems<DT>() <= n) {        // whole tile: every row in flight at once
        su32x4 raw[SROWS];
#pragma unroll
        for (int r = 0; r < SROWS; r++)
            raw[r] = __builtin_nontemporal_load(reinterpret_cast<const su32x4 *>(
                src + (base + (int64_t)r * 64 * V + (int64_t)l * V) * EB));
#pragma unroll
        for (int r = 0; r < SROWS; r++) {
            const uint4 v = make_uint4(raw[r].x, raw[r].y, raw[r].z, raw[r].w);
#pragma unroll
            for (int i = 0; i < V; i++) acc = acc + sdecode<DT>(v, i);
        }
    } else {                                          // last tile, or unaligned src
#pragma unroll 1
        for (int r = 0; r < SROWS; r++) {
            const int64_t e0 = base + (int64_t)r * 64 * V + (int64_t)l * V;
#pragma unroll 1
            for (int i = 0; i < V; i++)
                if (e0 + i < n) acc = acc + sdecode_at<DT>(src + (e0 + i) * EB);
        }
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) acc = acc + shfl_xor64(acc, m);
    if (l == 0) sums[t] = acc;
}

// Pass 2a: exclusive scan of the tile sums inside blocks of OFF_NT (in
// place, one value per thread, Hillis-Steele in LDS); block totals to btot.
template <typename T>
__global__ void __launch_bounds__(OFF_NT) k_scan_blocks(T *__restrict__ v, int64_t m,
                                                        T *__restrict__ btot) {
    __shared__ T sh[OFF_NT];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * OFF_NT + t;
    const T x = i < m ? v[i] : T(0);
    sh[t] = x;
    __syncthreads();
    for (int d = 1; d < OFF_NT; d <<= 1) {
        const T a = t >= d ? sh[t - d] : T(0);
        __syncthreads();
        sh[t] = sh[t] + a;
        __syncthreads();
    }
    if (i < m) v[i] = t > 0 ? sh[t - 1] : T(0);
    if (t == OFF_NT - 1) btot[blockIdx.x] = sh[t];
}

// Pass 2b: exclusive scan of the block totals, in place, by one workgroup
// (each thread a contiguous run, then the run totals through LDS).
template <typename T>
__global__ void __launch_bounds__(OFF_NT) k_scan_offsets(T *__restrict__ v, int64_t m) {
    __shared__ T sh[OFF_NT];
    const int t = threadIdx.x;
    const int64_t per = (m + OFF_NT - 1) / OFF_NT;
    const int64_t lo = t * per, hi = (lo + per) < m ? (lo + per) : m;
    T tot = T(0);
    for (int64_t i = lo; i < hi; i++) tot = tot + v[i];
    sh[t] = tot;
    __syncthreads();
    for (int d = 1; d < OFF_NT; d <<= 1) {   // inclusive Hillis-Steele scan of the totals
        const T a = t >= d ? sh[t - d] : T(0);
        __syncthreads();
        sh[t] = sh[t] + a;
        __syncthreads();
    }
    T run = t > 0 ? sh[t - 1] : T(0);
    for (int64_t i = lo; i < hi; i++) {
        const T x = v[i];
        v[i] = run;
        run = run + x;
    }
}

// Rescans one row of a wave tile (lane l holds elements x[0..V-1] at
// rb + l V + i) on top of `carry`, writes the outputs through the wave's LDS
// slice `sw` as 16-byte pieces that consecutive lanes place side by side
// (whole lines per instruction, streamed past the caches: every output is
// written once), and returns the row total.
template <int DT, bool EXCL, bool OUTV>
__device__ __forceinline__ typename ScanT<DT>::T apply_row(const typename ScanT<DT>::T *x,
                                                           typename ScanT<DT>::T carry,
                                                           typename ScanT<DT>::T *sw, int l,
                                                           int64_t rb, int64_t n,
                                                           typename ScanT<DT>::T *out) {
    using T = typename ScanT<DT>::T;
    constexpr int V = svec<DT>();
    constexpr int ROW = 64 * V;
    T p[V];
    p[0] = x[0];
#pragma unroll
    for (int i = 1; i < V; i++) p[i] = p[i - 1] + x[i];
    // exclusive scan of the lane totals over the wave (Hillis-Steele)
    T inc = p[V - 1];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T o = shfl_up64(inc, d);
        if (l >= d) inc = inc + o;
    }
    T ex = shfl_up64(inc, 1);
    if (l == 0) ex = T(0);
    const T rowbase = carry + ex;
    const T rowtot = shfl64(inc, 63);
#pragma unroll
    for (int i = 0; i < V; i++) {
        T y;
        if constexpr (EXCL) y = (i == 0) ? rowbase : rowbase + p[i - 1];
        else y = rowbase + p[i];
        sw[l * V + i] = y;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (OUTV && rb + ROW <= n) {
#pragma unroll
        for (int q = 0; q < V / 2; q++) {            // 16 bytes = 2 outputs per lane
            const int j = (q * 64 + l) * 2;
            const uint64_t a = __builtin_bit_cast(uint64_t, sw[j]);
            const uint64_t b = __builtin_bit_cast(uint64_t, sw[j + 1]);
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            const u32x4 w = {(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
            __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(out + rb + j));
        }
    } else {
        for (int j = l; j < ROW; j += 64)
            if (rb + j < n) out[rb + j] = sw[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();   // the slice is rewritten by the next row
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return rowtot;
}

// Pass 3: every tile rescanned row by row, plus its offset (the block
// offset plus the tile's offset inside its block).
template <int DT, bool VEC, bool EXCL, bool OUTV>
__global__ void __launch_bounds__(SNT) k_scan_apply(const unsigned char *__restrict__ src, int64_t n,
                                                    int64_t ntiles,
                                                    const typename ScanT<DT>::T *__restrict__ offs,
                                                    const typename ScanT<DT>::T *__restrict__ boffs,
                                                    typename ScanT<DT>::T *__restrict__ out) {
    using T = typename ScanT<DT>::T;
    constexpr int V = svec<DT>();
    constexpr int ROW = 64 * V;                       // elements (outputs) of a row
    __shared__ T stage[SNT / 64][ROW];
    const int64_t t = (int64_t)blockIdx.x * (SNT / 64) + (threadIdx.x >> 6);
    if (t >= ntiles) return;
    const int l = threadIdx.x & 63;
    T *sw = stage[threadIdx.x >> 6];
    const int64_t base = t * tile_elems<DT>();
    T carry = boffs[t / OFF_NT] + offs[t];
    constexpr int RG = 4;                             // rows in flight per group
#pragma unroll 1
    for (int r0 = 0; r0 < SROWS; r0 += RG) {
        if (base + (int64_t)r0 * ROW >= n) break;     // uniform: past the end
        RowGroup<DT, VEC, RG> g;
        g.load(src, n, base, l, r0);
#pragma unroll
        for (int k = 0; k < RG; k++) {
            const int64_t rb = base + (int64_t)(r0 + k) * ROW;   // first element of the row
            if (rb >= n) break;                                   // uniform
            T x[V];
            g.row(src, n, base, l, r0, k, x);
            carry = carry + apply_row<DT, EXCL, OUTV>(x, carry, sw, l, rb, n, out);
        }
    }
}

// ---------------------------------------------------------------- one pass
// Integer scans (exact, so any order of additions gives the same result) in
// one pass over the input with a decoupled look-back (Merrill and Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016): a
// workgroup takes the next tile of 4 wave tiles from a ticket counter, keeps
// its input in registers, publishes the tile's total (flag 1), finds the sum
// of all earlier tiles from their published totals and inclusive prefixes
// (64 predecessors per step, one per lane), publishes its own inclusive
// prefix (flag 2), and only then rescans and writes its elements.  A
// workgroup waits only on tiles whose tickets were taken earlier, i.e. by
// workgroups already running, so every wait ends.  Each wait is bounded all
// the same: once a window of 64 predecessors has been polled `spin_limit`
// times while a nearer tile in it has still published nothing, the waiting
// wave computes that tile's total from the input itself (a tile's total is a
// function of its elements alone, and integer sums are exact, so the result
// is the same bit for bit).  Floats keep the three-pass form: their fixed
// summation order is part of the result.
constexpr int LB_WAVES = SNT / 64;
constexpr uint32_t LB_SPIN_DEFAULT = 1u << 18;   // polls per window before computing

template <int DT> constexpr int64_t lb_tile_elems() { return LB_WAVES * tile_elems<DT>(); }

// Total of look-back tile `tile` (every element in range: it precedes another
// tile), summed by one wave; every lane returns it.
template <int DT> __device__ __noinline__ uint64_t lb_tile_total(const unsigned char *src, int64_t n,
                                                                int64_t tile) {
    constexpr int V = svec<DT>(), EB = ScanT<DT>::EB;
    const int l = threadIdx.x & 63;
    uint64_t acc = 0;
    for (int w = 0; w < LB_WAVES; w++) {
        const int64_t base = tile * lb_tile_elems<DT>() + (int64_t)w * tile_elems<DT>();
#pragma unroll 4
        for (int r = 0; r < SROWS; r++) {
            const int64_t e0 = base + (int64_t)r * 64 * V + (int64_t)l * V;
#pragma unroll
            for (int i = 0; i < V; i++)
                if (e0 + i < n) acc += sdecode_at<DT>(src + (e0 + i) * EB);
        }
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) acc += shfl_xor64(acc, m);
    return acc;
}

// Publication without cache-wide fences: the totals, prefixes and flags are
// written and read only with device-scope relaxed atomics, which go past the
// XCD-private L2s to the coherent level.  A writer waits until its value store
// has completed (s_waitcnt vmcnt(0)) before it stores the flag, and a reader
// loads a value only after it has seen the flag, so a flag is never seen
// before its value.  (Release/acquire fences would write back and invalidate
// the whole L2 of the XCD on every publication.)
__device__ __forceinline__ uint32_t lb_flag(const uint32_t *f) {
    return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_value(const uint64_t *v) {
    return __hip_atomic_load(v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_publish(uint64_t *v, uint64_t x, uint32_t *f, uint32_t state) {
    __hip_atomic_store(v, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(f, state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int DT, bool EXCL, bool OUTV>
__global__ void __launch_bounds__(SNT) k_scan_lookback(const unsigned char *__restrict__ src,
                                                       int64_t n, int64_t ntiles,
                                                       uint32_t *__restrict__ ticket,
                                                       uint32_t *__restrict__ flag,
                                                       uint64_t *__restrict__ agg,
                                                       uint64_t *__restrict__ incl,
                                                       uint64_t *__restrict__ out,
                                                       uint32_t spin_limit) {
    using T = uint64_t;
    constexpr int V = svec<DT>(), EB = ScanT<DT>::EB;
    constexpr int ROW = 64 * V;
    __shared__ T stage[LB_WAVES][ROW];
    __shared__ T wsum[LB_WAVES];
    __shared__ T sh_excl;
    __shared__ uint32_t sh_tile;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (threadIdx.x == 0) sh_tile = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t tile = sh_tile;
    if (tile >= ntiles) return;                      // (the grid has exactly ntiles workgroups)
    const int64_t base = tile * lb_tile_elems<DT>() + (int64_t)w * tile_elems<DT>();
    // this wave's 16 rows, all in flight, kept for the rescan
    su32x4 raw[SROWS];
#pragma unroll
    for (int r = 0; r < SROWS; r++) {
        const int64_t e0 = base + (int64_t)r * ROW + (int64_t)l * V;
        raw[r] = su32x4{0, 0, 0, 0};
        if (e0 + V <= n)
            raw[r] = __builtin_nontemporal_load(reinterpret_cast<const su32x4 *>(src + e0 * EB));
        else
            for (int i = 0; i < V; i++)
                if (e0 + i < n) {
                    const T v = sdecode_at<DT>(src + (e0 + i) * EB);
                    if constexpr (EB == 4) raw[r][i] = (uint32_t)v;
                    else { raw[r][2 * i] = (uint32_t)v; raw[r][2 * i + 1] = (uint32_t)(v >> 32); }
                }
    }
    T acc = 0;
#pragma unroll
    for (int r = 0; r < SROWS; r++) {
        const uint4 v = make_uint4(raw[r].x, raw[r].y, raw[r].z, raw[r].w);
#pragma unroll
        for (int i = 0; i < V; i++) acc += sdecode<DT>(v, i);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) acc += shfl_xor64(acc, m);
    if (l == 0) wsum[w] = acc;
    __syncthreads();
    if (w == 0) {
        T tot = 0;
#pragma unroll
        for (int k = 0; k < LB_WAVES; k++) tot += wsum[k];
        // publish the tile total (its inclusive prefix at once for tile 0)
        if (l == 0) {
            if (tile == 0) lb_publish(incl, tot, flag, 2u);
            else lb_publish(agg + tile, tot, flag + tile, 1u);
        }
        // look back: lane i examines tile j - i
        T excl = 0;
        int64_t j = tile - 1;
        uint32_t spins = 0;                          // polls of the current window
        while (j >= 0) {
            const int64_t jj = j - l;
            const uint32_t f = jj >= 0 ? lb_flag(flag + jj) : 2u;   // before tile 0: prefix 0
            const uint64_t has_incl = __ballot(f == 2u);
            const uint64_t none = __ballot(f == 0u);
            const int s = has_incl ? __builtin_ctzll(has_incl) : 64;   // nearest inclusive prefix
            const uint64_t before = s == 64 ? ~0ull : ((1ull << s) - 1);
            uint64_t silent = none & before;         // nearer tiles that published nothing
            if (silent && ++spins < spin_limit) continue;
            T v = 0;
            if (jj >= 0 && l < s && !((silent >> l) & 1)) v = lb_value(agg + jj);
            else if (jj >= 0 && l == s) v = lb_value(incl + jj);
            while (silent) {                         // bound reached: sum those tiles here
                const int i = __builtin_ctzll(silent);
                silent &= silent - 1;
                const T tot = lb_tile_total<DT>(src, n, j - i);
                if (l == i) v = tot;
            }
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) v += shfl_xor64(v, m);
            excl += v;
            if (s < 64) break;
            j -= 64;
            spins = 0;
        }
        if (l == 0) {
            if (tile > 0) lb_publish(incl + tile, excl + tot, flag + tile, 2u);
            sh_excl = excl;
        }
    }
    __syncthreads();
    // rescan this wave's rows on top of the tile's prefix and the waves before
    T carry = sh_excl;
    for (int k = 0; k < w; k++) carry += wsum[k];
    T *sw = stage[w];
#pragma unroll
    for (int r = 0; r < SROWS; r++) {
        const int64_t rb = base + (int64_t)r * ROW;
        if (rb >= n) break;                                    // uniform
        const uint4 v = make_uint4(raw[r].x, raw[r].y, raw[r].z, raw[r].w);
        T x[V];
#pragma unroll
        for (int i = 0; i < V; i++) x[i] = sdecode<DT>(v, i);
        carry += apply_row<DT, EXCL, OUTV>(x, carry, sw, l, rb, n, out);
    }
}

uint32_t g_lb_spin = LB_SPIN_DEFAULT;

template <int DT>
int launch_lookback(const void *src, int64_t n, void *out, bool excl, hipStream_t st) {
    const int64_t ntiles = (n + lb_tile_elems<DT>() - 1) / lb_tile_elems<DT>();
    if (ntiles > 0x7fffffff) return fail(XTR_EINVAL, "scan_sum: input too large");
    // ticket and flags (zeroed by a fill kernel every call), totals, prefixes
    const size_t fbytes = ((size_t)(ntiles + 1) * 4 + 255) / 256 * 256;
    const size_t vbytes = (size_t)ntiles * 8;
    void *ws = nullptr;
    int rc = workspace(WS_SCAN, st, fbytes + 2 * vbytes, &ws);
    if (rc) return rc;
    unsigned char *wb = static_cast<unsigned char *>(ws);
    uint32_t *ticket = reinterpret_cast<uint32_t *>(wb);
    uint32_t *flag = ticket + 1;
    uint64_t *agg = reinterpret_cast<uint64_t *>(wb + fbytes);
    uint64_t *incl = reinterpret_cast<uint64_t *>(wb + fbytes + vbytes);
    rc = zero_fill(wb, fbytes, st);
    if (rc) return rc;
    const unsigned char *s = static_cast<const unsigned char *>(src);
    uint64_t *o = static_cast<uint64_t *>(out);
    const bool outv = ((uintptr_t)out % 16) == 0;
    const uint32_t spin = __atomic_load_n(&g_lb_spin, __ATOMIC_RELAXED);
#define XTR_LB(EE, OO)                                                                        \
    hipLaunchKernelGGL((k_scan_lookback<DT, EE, OO>), dim3((unsigned)ntiles), dim3(SNT), 0, st, s, \
                       n, ntiles, ticket, flag, agg, incl, o, spin)
    if (outv) {
        if (excl) XTR_LB(true, true);
        else XTR_LB(false, true);
    } else {
        if (excl) XTR_LB(true, false);
        else XTR_LB(false, false);
    }
#undef XTR_LB
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

template <int DT>
int launch_scan(const void *src, int64_t n, void *out, bool excl, hipStream_t st) {
    using T = typename ScanT<DT>::T;
    if constexpr (DT == XTR_I32 || DT == XTR_I64)
        if ((uintptr_t)src % 16 == 0) return launch_lookback<DT>(src, n, out, excl, st);
    const int64_t ntiles = (n + tile_elems<DT>() - 1) / tile_elems<DT>();
    const int64_t nblk = (ntiles + OFF_NT - 1) / OFF_NT;
    const size_t sums_bytes = ((size_t)ntiles * sizeof(T) + 255) / 256 * 256;
    void *ws = nullptr;
    int rc = workspace(WS_SCAN, st, sums_bytes + (size_t)nblk * sizeof(T), &ws);
    if (rc) return rc;
    T *sums = static_cast<T *>(ws);
    T *btot = reinterpret_cast<T *>(static_cast<unsigned char *>(ws) + sums_bytes);
    const bool vec = ((uintptr_t)src % 16) == 0;
    const bool outv = ((uintptr_t)out % 16) == 0;
    const dim3 grid((unsigned)((ntiles + SNT / 64 - 1) / (SNT / 64)));
    const unsigned char *s = static_cast<const unsigned char *>(src);
    if (vec) hipLaunchKernelGGL((k_scan_tiles<DT, true>), grid, dim3(SNT), 0, st, s, n, ntiles, sums);
    else hipLaunchKernelGGL((k_scan_tiles<DT, false>), grid, dim3(SNT), 0, st, s, n, ntiles, sums);
    hipLaunchKernelGGL((k_scan_blocks<T>), dim3((unsigned)nblk), dim3(OFF_NT), 0, st, sums, ntiles,
                       btot);
    hipLaunchKernelGGL((k_scan_offsets<T>), dim3(1), dim3(OFF_NT), 0, st, btot, nblk);
    T *o = static_cast<T *>(out);
#define XTR_SA(VV, EE, OO)                                                                    \
    hipLaunchKernelGGL((k_scan_apply<DT, VV, EE, OO>), grid, dim3(SNT), 0, st, s, n, ntiles, sums, \
                       btot, o)
    if (outv) {
        if (vec && excl) XTR_SA(true, true, true);
        else if (vec) XTR_SA(true, false, true);
        else if (excl) XTR_SA(false, true, true);
        else XTR_SA(false, false, true);
    } else {
        if (vec && excl) XTR_SA(true, true, false);
        else if (vec) XTR_SA(true, false, false);
        else if (excl) XTR_SA(false, true, false);
        else XTR_SA(false, false, false);
    }
#undef XTR_SA
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

}  // namespace

int scan_impl(const void *src, int64_t n, void *out, int dtype, int exclusive, hipStream_t st) {
    const char *who = "scan_sum";
    if (!is_float_sum_dtype(dtype) && !is_int_sum_dtype(dtype))
        return fail(XTR_EDTYPE, "%s: dtype %d is not summable", who, dtype);
    if (n < 0) return fail(XTR_EINVAL, "%s: negative n", who);
    if (n == 0) return XTR_OK;
    if (!src || !out) return fail(XTR_EINVAL, "%s: null pointer", who);
    const int eb = elem_bytes(dtype);
    if ((uintptr_t)src % eb) return fail(XTR_EALIGN, "%s: src not aligned to its element", who);
    if ((uintptr_t)out % 8) return fail(XTR_EALIGN, "%s: out not 8-byte aligned", who);
    const uintptr_t s0 = (uintptr_t)src, s1 = s0 + (uintptr_t)n * eb;
    const uintptr_t d0 = (uintptr_t)out, d1 = d0 + (uintptr_t)n * 8;
    if (s0 < d1 && d0 < s1) return fail(XTR_EOVERLAP, "%s: src and out overlap", who);
    const bool ex = exclusive != 0;
    switch (dtype) {
    case XTR_F32: return launch_scan<XTR_F32>(src, n, out, ex, st);
    case XTR_F16: return launch_scan<XTR_F16>(src, n, out, ex, st);
    case XTR_BF16: return launch_scan<XTR_BF16>(src, n, out, ex, st);
    case XTR_F8E4M3: return launch_scan<XTR_F8E4M3>(src, n, out, ex, st);
    case XTR_I32: return launch_scan<XTR_I32>(src, n, out, ex, st);
    default: return launch_scan<XTR_I64>(src, n, out, ex, st);
    }
}

}  // namespace xtr

extern "C" int scan_sum(const void *src, int64_t n, void *out, int dtype, int exclusive,
                        void *stream) {
    return xtr::scan_impl(src, n, out, dtype, exclusive, (hipStream_t)stream);
}

extern "C" uint32_t xtr_scan_lookback_bound(uint32_t polls) {
    uint32_t old = __atomic_exchange_n(&xtr::g_lb_spin, polls, __ATOMIC_RELAXED);
    return old;
}
