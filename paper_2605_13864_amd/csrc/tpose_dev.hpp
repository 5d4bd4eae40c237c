// Device side of the transpose (tile routine, kernels) and its launch
// templates, shared by the translation units tpose_s<EB>.hip (single
// launches) and tpose_b<EB>.hip (batched launches) for EB = 1, 2, 4, 8 (each
// instantiates the kernels of one element size and form, so they compile in
// parallel) and by the host side in tpose.hip.  What the kernels compute and how is described in tpose.hip.
#pragma once

#include "common.hpp"
#include "tile_map.h"

#include <type_traits>

namespace xtr {
namespace tpk {

constexpr int NT = 256;   // threads per workgroup

// Tile geometry: SC 16-byte chunks per src row segment and DC per dst row
// segment (16 = 256 bytes, the default on both sides; 32 = 512 bytes).
template <int EB, int SC = 16, int DC = 16> struct Geo {
    static constexpr int V = 16 / EB;     // elements per 16-byte vector
    static constexpr int TC = SC * V;     // tile columns (src) = 16 * SC bytes of a src row
    static constexpr int TR = DC * V;     // tile rows (src) = 16 * DC bytes of a dst row
    static constexpr int CHUNKS = SC;     // 16-byte chunks per LDS tile row
    static constexpr int LDS_VECS = TR * SC;
};

template <int EB> struct Elem;
template <> struct Elem<1> { using T = uint8_t; };
template <> struct Elem<2> { using T = uint16_t; };
template <> struct Elem<4> { using T = uint32_t; };
template <> struct Elem<8> { using T = uint64_t; };

// LDS swizzle of the tile rows (tile_map.h).
using tmap::swz;

// ---------------------------------------------------------------- register
// transposes of one V x V element block: a[i] holds src row i (V elements),
// out[j] receives dst row j = (a[0][j], a[1][j], ..., a[V-1][j]).

__device__ __forceinline__ uint32_t dw(const uint4 &v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

template <int EB> __device__ __forceinline__ void block_transpose(const uint4 *a, uint4 *out);

template <> __device__ __forceinline__ void block_transpose<8>(const uint4 *a, uint4 *out) {
    out[0] = make_uint4(a[0].x, a[0].y, a[1].x, a[1].y);
    out[1] = make_uint4(a[0].z, a[0].w, a[1].z, a[1].w);
}

template <> __device__ __forceinline__ void block_transpose<4>(const uint4 *a, uint4 *out) {
    out[0] = make_uint4(a[0].x, a[1].x, a[2].x, a[3].x);
    out[1] = make_uint4(a[0].y, a[1].y, a[2].y, a[3].y);
    out[2] = make_uint4(a[0].z, a[1].z, a[2].z, a[3].z);
    out[3] = make_uint4(a[0].w, a[1].w, a[2].w, a[3].w);
}

// 16-bit elements: dword m of dst row j packs rows 2m (low half) and 2m+1.
template <> __device__ __forceinline__ void block_transpose<2>(const uint4 *a, uint4 *out) {
#pragma unroll
    for (int j = 0; j < 8; j++) {
        uint32_t d[4];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            uint32_t A = dw(a[2 * m], j >> 1), B = dw(a[2 * m + 1], j >> 1);
            d[m] = (j & 1) ? ((A >> 16) | (B & 0xffff0000u)) : ((A & 0xffffu) | (B << 16));
        }
        out[j] = make_uint4(d[0], d[1], d[2], d[3]);
    }
}

// 8-bit elements: byte k of dword m of dst row j is byte (j & 3) of dword
// (j >> 2) of src row 4m + k -- a 4 x 4 byte transpose per (m, j >> 2).
__device__ __forceinline__ void byte4x4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                        uint32_t *y) {
    // t0 = [x0.b0 x1.b0 x0.b2 x1.b2], t1 = [x0.b1 x1.b1 x0.b3 x1.b3], same for t2/t3 on x2/x3
    uint32_t t0 = (x0 & 0x00ff00ffu) | ((x1 & 0x00ff00ffu) << 8);
    uint32_t t1 = ((x0 >> 8) & 0x00ff00ffu) | (x1 & 0xff00ff00u);
    uint32_t t2 = (x2 & 0x00ff00ffu) | ((x3 & 0x00ff00ffu) << 8);
    uint32_t t3 = ((x2 >> 8) & 0x00ff00ffu) | (x3 & 0xff00ff00u);
    y[0] = (t0 & 0x0000ffffu) | (t2 << 16);
    y[1] = (t1 & 0x0000ffffu) | (t3 << 16);
    y[2] = (t0 >> 16) | (t2 & 0xffff0000u);
    y[3] = (t1 >> 16) | (t3 & 0xffff0000u);
}

template <> __device__ __forceinline__ void block_transpose<1>(const uint4 *a, uint4 *out) {
#pragma unroll
    for (int q = 0; q < 4; q++) {          // src dword column -> dst rows 4q .. 4q+3
        uint32_t y[4][4];                   // y[m][r]: dword m of dst row 4q + r
#pragma unroll
        for (int m = 0; m < 4; m++)
            byte4x4(dw(a[4 * m], q), dw(a[4 * m + 1], q), dw(a[4 * m + 2], q),
                    dw(a[4 * m + 3], q), y[m]);
#pragma unroll
        for (int r = 0; r < 4; r++) out[4 * q + r] = make_uint4(y[0][r], y[1][r], y[2][r], y[3][r]);
    }
}

// ---------------------------------------------------------------- 16-byte I/O

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Nontemporal (streaming) accesses do not keep the line in the caches; every
// byte of a transpose is touched once, so they save cache capacity for the
// partial lines that neighbouring tiles share.
template <bool NT> __device__ __forceinline__ uint4 ld16(const unsigned char *p) {
    u32x4 v;
    if constexpr (NT) v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    else v = *reinterpret_cast<const u32x4 *>(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <bool NT> __device__ __forceinline__ void st16(unsigned char *p, const uint4 &o) {
    u32x4 v = {o.x, o.y, o.z, o.w};
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
    else *reinterpret_cast<u32x4 *>(p) = v;
}

// ---------------------------------------------------------------- tile order

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  xcd_remap gives each XCD a contiguous range of the launch's
// linear order, so neighbouring tiles -- which share the cache lines at their
// edges when rows are not 128-byte aligned -- meet in the same L2.
// Tile counts fit in 32 bits (the host checks it), so the index arithmetic
// of a tile's position is 32-bit.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G) {
    const uint32_t x = b & 7, k = b >> 3, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + k;
}

// Tile (tr, tc) at position L of the launch order: bands of `group` tile rows,
// column-major inside a band (group = 1 is plain row-major), so that the tiles
// in flight together write longer runs of each dst row.
__device__ __forceinline__ void band_order(uint32_t L, uint32_t tiles_r, uint32_t tiles_c,
                                           uint32_t group, uint32_t &tr, uint32_t &tc) {
    const uint32_t per = group * tiles_c;
    const uint32_t band = L / per, w = L - band * per;
    const uint32_t left = tiles_r - band * group;
    const uint32_t rib = left < group ? left : group;
    tc = w / rib;
    tr = band * group + (w - tc * rib);
}

// Largest tile count of one launch (single call or batch group).
constexpr int64_t MAX_TILES = (int64_t)1 << 31;

// ---------------------------------------------------------------- W-byte pieces

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Global accesses move W-byte pieces, W in {4, 8, 16}: the largest power of
// two that divides both base pointers and both row pitches (in bytes).  A
// 16-byte vector is split into 16 / W pieces on the store side.
template <int W> struct PieceT;
template <> struct PieceT<1> { using T = uint32_t; };   // 4-byte pieces at any alignment
template <> struct PieceT<4> { using T = uint32_t; };
template <> struct PieceT<8> { using T = u32x2; };
template <> struct PieceT<16> { using T = u32x4; };

template <int W, bool NT> __device__ __forceinline__ typename PieceT<W>::T ldw(const unsigned char *p) {
    using T = typename PieceT<W>::T;
    if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const T *>(p));
    else return *reinterpret_cast<const T *>(p);
}
template <int W, bool NT> __device__ __forceinline__ void stw(unsigned char *p, typename PieceT<W>::T v) {
    using T = typename PieceT<W>::T;
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<T *>(p));
    else *reinterpret_cast<T *>(p) = v;
}
// Element i of a 16-byte vector of EB-byte elements (i known at compile time).
template <int EB> __device__ __forceinline__ uint64_t elem_at(const uint4 &v, int i) {
    if constexpr (EB == 8) return i == 0 ? ((uint64_t)v.y << 32 | v.x) : ((uint64_t)v.w << 32 | v.z);
    else if constexpr (EB == 4) return dw(v, i);
    else if constexpr (EB == 2) return (dw(v, i >> 1) >> (16 * (i & 1))) & 0xffffu;
    else return (dw(v, i >> 2) >> (8 * (i & 3))) & 0xffu;
}

// Narrow-piece transpose: a[e] holds V elements of tile row e (e < E = W / EB
// rows); out[i] is the W-byte piece (a[0][i], a[1][i], ..., a[E-1][i]), i.e.
// E consecutive elements of dst row i.  W = 16 is block_transpose.
template <int EB, int W>
__device__ __forceinline__ void piece_transpose(const uint4 *a, typename PieceT<W>::T *out) {
    constexpr int V = 16 / EB, E = W / EB;
    if constexpr (W == 16) {
        uint4 o[V];
        block_transpose<EB>(a, o);
#pragma unroll
        for (int i = 0; i < V; i++) out[i] = u32x4{o[i].x, o[i].y, o[i].z, o[i].w};
    } else {
#pragma unroll
        for (int i = 0; i < V; i++) {
            uint64_t r = 0;
#pragma unroll
            for (int e = 0; e < E; e++) r |= elem_at<EB>(a[e], i) << (8 * EB * e);
            if constexpr (W == 8) out[i] = u32x2{(uint32_t)r, (uint32_t)(r >> 32)};
            else out[i] = (uint32_t)r;
        }
    }
}

// Rows of 1- and 2-byte elements whose addresses are not 4-byte aligned
// (odd pitches): a wave moves one 256-byte row segment as 64 4-byte pieces,
// each built from aligned dwords.  Reading, lane k loads the aligned dword that
// holds the first byte of its piece and funnel-shifts it with its right
// neighbour's (lane 63 loads that one itself; it still holds a byte of the
// segment, so it lies on a page the segment touches).  Writing, lane k stores
// the aligned dword that ends inside its piece, funnel-shifted from its left
// neighbour's piece and its own; the segment's partial first and last dwords
// are written byte by byte, so no byte outside the segment is touched.
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t bytes) {
    return __builtin_amdgcn_alignbyte(hi, lo, bytes);   // (hi:lo) >> 8 * bytes
}
// Lane k receives lane k - 1's value (lane 0: 0), and lane k + 1's (lane 63:
// 0): whole-wave DPP shifts, no LDS traffic.
__device__ __forceinline__ uint32_t from_left(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}
__device__ __forceinline__ uint32_t from_right(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}
template <bool NT>
__device__ __forceinline__ void st_funnel(unsigned char *pp, uint32_t piece, int k) {
    const uint32_t md = (uint32_t)(uintptr_t)pp & 3;     // the same in every lane
    const uint32_t prev = from_left(piece);
    if (md == 0) {
        stw<4, NT>(pp, piece);
        return;
    }
    if (k > 0) stw<4, NT>(pp - md, funnel(piece, prev, 4 - md));
    // The partial dwords: lane 0 writes bytes [0, 4 - md) of its piece (they
    // end on a dword edge), lane 63 bytes [4 - md, 4) (they start on one).
    // Each writes at most one naturally aligned 16-bit half and one byte, and
    // the two lanes share the store instructions.
    if (k == 0 || k == 63) {
        const uint32_t b0 = k == 0 ? 0u : 4 - md, n = k == 0 ? 4 - md : md;
        unsigned char *q = pp + b0;
        const uint32_t v = piece >> (8 * b0);
        const bool odd = ((uintptr_t)q & 1) != 0;
        const bool has_b = odd || (n & 1);          // the byte: at q if q is odd,
        const uint32_t bo = odd ? 0u : n - 1;       // else the last of an odd count
        const uint32_t so = odd ? 1u : 0u;          // the half: after an odd q, else first
        if (n > 1) *reinterpret_cast<uint16_t *>(q + so) = (uint16_t)(v >> (8 * so));
        if (has_b) q[bo] = (unsigned char)(v >> (8 * bo));
    }
}

// The same on an edge tile: only logical bytes [0, vb) of the segment exist.
// Whole dwords inside them as above; a dword the end cuts, and the head when
// it is cut, byte by byte.
template <bool NT>
__device__ __forceinline__ void st_funnel_edge(unsigned char *pp, uint32_t piece, int k, int vb) {
    const int md = (int)((uintptr_t)pp & 3);
    const uint32_t prev = from_left(piece);
    if (md == 0) {
        if (4 * k + 4 <= vb) stw<4, NT>(pp, piece);
        else
            for (int b = 0; b < 4; b++)
                if (4 * k + b < vb) pp[b] = (unsigned char)(piece >> (8 * b));
        return;
    }
    if (k > 0) {
        const int lo = 4 * k - md;                      // logical byte at pp - md
        const uint32_t v = funnel(piece, prev, 4 - md);
        if (lo + 4 <= vb) stw<4, NT>(pp - md, v);
        else
            for (int b = 0; b < 4; b++)
                if (lo + b < vb) pp[b - md] = (unsigned char)(v >> (8 * b));
    } else {
        for (int b = 0; b < 4 - md; b++)
            if (b < vb) pp[b] = (unsigned char)(piece >> (8 * b));
    }
    if (k == 63)
        for (int b = 4 - md; b < 4; b++)
            if (4 * k + b < vb) pp[b] = (unsigned char)(piece >> (8 * b));
}

// ---------------------------------------------------------------- one tile

// Moves the TR x TC tile at (R0, C0), in two phases with a block barrier
// between them (tile_phase<1>: src -> LDS; tile_phase<2>: LDS -> dst).
// Interior tiles run without any bounds test; tiles on the right or bottom
// edge mask whole pieces and fall back to single elements only for the one
// piece a matrix edge cuts.
template <int PH, int EB, int W, bool NTL, bool NTS, bool OFF32, int SC = 16, int DC = 16>
__device__ __forceinline__ void tile_phase(const unsigned char *__restrict__ src,
                                        unsigned char *__restrict__ dst, int64_t rows,
                                        int64_t cols, int64_t ld_src, int64_t ld_dst, int64_t R0,
                                        int64_t C0, uint4 *lds) {
    using G = Geo<EB, SC, DC>;
    using T = typename Elem<EB>::T;
    using PT = typename PieceT<W>::T;
    // per-lane part of an address: 32 bits when the host guarantees it fits
    using LaneOff = typename std::conditional<OFF32, uint32_t, int64_t>::type;
    // W = 1: 4-byte pieces of rows at any alignment (interior tiles only)
    constexpr bool UA = W == 1;
    constexpr int WP = UA ? 4 : W;      // piece bytes
    static_assert(!UA || (SC == 16 && DC == 16 && EB <= 2), "unaligned rows: default tiles");
    using M = tmap::TileMap<EB, WP, SC, DC, NT>;   // the tile's index maps
    static_assert(M::TR == G::TR && M::TC == G::TC, "tile geometry");
    constexpr int V = G::V;
    constexpr int P = M::P;             // pieces per src row segment
    constexpr int RP = M::RP;           // tile rows per pass of the workgroup
    constexpr int PASSES = M::PASSES;
    constexpr int EPW = M::EPW;         // elements per piece
    const int t = threadIdx.x;
    const bool full = (R0 + G::TR <= rows) && (C0 + G::TC <= cols);
    unsigned char *ldsb = reinterpret_cast<unsigned char *>(lds);

    // Addresses are (uniform tile base + uniform per-pass offset) + lane offset:
    // the first two live in scalar registers, the lane offset is computed once.

    // phase 1: P lanes per src row segment, rows RP apart per pass
    if constexpr (PH == 1) {
        const int k = t % P, r0 = M::p1_row(t, 0);
        const int64_t ldsrc = ld_src * EB;
        const unsigned char *tb = src + (R0 * ld_src + C0) * EB;           // uniform
        const LaneOff lane = (LaneOff)r0 * (LaneOff)ldsrc + (LaneOff)M::p1_byte(t);
        if constexpr (UA) {
            // Cached accesses whatever the settings: neighbouring lanes and tiles
            // read and write the same dwords and lines.
            // In batches of PB passes: the aligned dwords first (all in flight),
            // then the funnel shifts and the LDS writes.  On an edge tile only
            // bytes [0, vb) of a row exist: a lane whose piece they cut reads its
            // bytes one by one (and shifts by 0), and a lane whose right
            // neighbour does so loads that neighbour's dword itself.
            constexpr int PB = PASSES < 16 ? PASSES : 16;
            const int vb = full ? 256 : (int)(cols - C0 < G::TC ? (cols - C0) * EB : 256);
            const bool whole = 4 * k + 4 <= vb, cut = !whole && 4 * k < vb;
            const bool own_next = k == P - 1 || 4 * k + 8 > vb;
            for (int p0 = 0; p0 < PASSES; p0 += PB) {
                uint32_t d[PB], x[PB];
                if (full) {
#pragma unroll
                    for (int j = 0; j < PB; j++) {
                        const unsigned char *pp = (tb + (int64_t)(RP * (p0 + j)) * ldsrc) + lane;
                        const uint32_t m = (uint32_t)(uintptr_t)pp & 3;
                        d[j] = ldw<4, false>(pp - m);
                        x[j] = (k == P - 1 && m != 0) ? ldw<4, false>(pp - m + 4) : 0u;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < PB; j++) {
                        const unsigned char *pp = (tb + (int64_t)(RP * (p0 + j)) * ldsrc) + lane;
                        const uint32_t m = (uint32_t)(uintptr_t)pp & 3;
                        const bool rowok = R0 + r0 + RP * (p0 + j) < rows;
                        d[j] = 0u;
                        x[j] = 0u;
                        if (rowok && whole) {
                            d[j] = ldw<4, false>(pp - m);
                            if (own_next && m != 0) x[j] = ldw<4, false>(pp - m + 4);
                        } else if (rowok && cut) {
                            for (int b = 0; b < 4; b++)
                                if (4 * k + b < vb) d[j] |= (uint32_t)pp[b] << (8 * b);
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < PB; j++) {
                    const int row = M::p1_row(t, p0 + j);
                    const unsigned char *pp = (tb + (int64_t)(RP * (p0 + j)) * ldsrc) + lane;
                    const uint32_t m = cut ? 0u : (uint32_t)(uintptr_t)pp & 3;
                    uint32_t nxt = from_right(d[j]);
                    if (own_next) nxt = x[j];
                    if (full || (R0 + row < rows && 4 * k < vb))
                        *reinterpret_cast<uint32_t *>(ldsb + M::lds_byte(row, M::p1_byte(t))) =
                            funnel(nxt, d[j], m);
                }
            }
        } else if (full) {
            // all loads first (PASSES pieces in flight per lane), then the LDS writes
            PT v[PASSES];
#pragma unroll
            for (int p = 0; p < PASSES; p++) v[p] = ldw<W, NTL>((tb + (int64_t)(RP * p) * ldsrc) + lane);
#pragma unroll
            for (int p = 0; p < PASSES; p++) {
                const int row = M::p1_row(t, p);
                *reinterpret_cast<PT *>(ldsb + M::lds_byte(row, M::p1_byte(t))) = v[p];
            }
        } else {
            // Edge tile: every whole piece in range is loaded first, all in
            // flight (a piece out of range, or the one a matrix edge cuts,
            // loads the tile's first piece instead -- it always exists -- and
            // that value is never used); then the LDS writes, with the cut
            // piece read element by element.  LDS rows and columns outside
            // the matrix are left as they are: phase 2 never stores them.
            const int64_t c = C0 + (int64_t)k * EPW;
            const bool cin = c < cols, cwhole = c + EPW <= cols;
            PT v[PASSES];
#pragma unroll
            for (int p = 0; p < PASSES; p++) {
                const bool use = cwhole && R0 + M::p1_row(t, p) < rows;
                v[p] = ldw<W, NTL>(use ? (tb + (int64_t)(RP * p) * ldsrc) + lane : tb);
            }
#pragma unroll
            for (int p = 0; p < PASSES; p++) {
                const int row = M::p1_row(t, p);
                if (R0 + row >= rows || !cin) continue;   // never stored: LDS left as is
                PT pv = v[p];
                if (!cwhole) {
                    const unsigned char *a = (tb + (int64_t)(RP * p) * ldsrc) + lane;
                    union { PT pt; T e[EPW]; } u;
                    u.pt = PT{};
#pragma unroll
                    for (int i = 0; i < EPW; i++)
                        if (c + i < cols) u.e[i] = reinterpret_cast<const T *>(a)[i];
                    pv = u.pt;
                }
                *reinterpret_cast<PT *>(ldsb + M::lds_byte(row, M::p1_byte(t))) = pv;
            }
        }
    }

    // (between the phases: a block barrier -- ownership of the LDS tile moves
    // from loaders to storers)

    // phase 2: P2 lanes per dst row segment.  Lane k stores piece k,
    // i.e. src rows k*E .. k*E+E-1 of one src column, so the lanes of a store
    // instruction write consecutive W-byte pieces of a dst row (whole lines
    // per instruction whatever W is).  The lane reads E 16-byte row chunks
    // from LDS and transposes them in registers into V pieces, one per dst
    // row of the chunk.  With W = 16 this is the V x V block transpose.
    if constexpr (PH == 2) {
        constexpr int RP2 = M::RP2;                  // column chunks per pass
        constexpr int CPT = M::CPT;                  // 16-byte column chunks per lane
        const int k = M::p2_piece(t), g = M::p2_chunk(t, 0);
        const int64_t lddst = ld_dst * EB;
        unsigned char *tb = dst + (C0 * ld_dst + R0) * EB;                  // uniform
        const LaneOff lane = (LaneOff)(g * V) * (LaneOff)lddst + (LaneOff)(k * WP);
        const int64_t rk = R0 + (int64_t)k * EPW;    // first src row of the piece
#pragma unroll
        for (int cc = 0; cc < CPT; cc++) {
            const int m = M::p2_chunk(t, cc);        // src cols m*V .. m*V+V-1
            uint4 a[EPW];
#pragma unroll
            for (int e = 0; e < EPW; e++) a[e] = lds[M::p2_lds_vec(k, e, m)];
            PT o[V];
            piece_transpose<EB, WP>(a, o);
            unsigned char *cb = tb + (int64_t)(RP2 * cc * V) * lddst;       // uniform
            if constexpr (UA) {
                if (full) {
#pragma unroll
                    for (int i = 0; i < V; i++)
                        st_funnel<false>((cb + (int64_t)i * lddst) + lane, o[i], k);
                } else {
                    const int vb = (int)(rows - R0 < G::TR ? (rows - R0) * EB : 256);
#pragma unroll
                    for (int i = 0; i < V; i++)
                        if (C0 + m * V + i < cols)
                            st_funnel_edge<false>((cb + (int64_t)i * lddst) + lane, o[i], k, vb);
                }
            } else if (full) {
#pragma unroll
                for (int i = 0; i < V; i++) stw<W, NTS>((cb + (int64_t)i * lddst) + lane, o[i]);
            } else {
                if (rk >= rows) continue;
#pragma unroll
                for (int i = 0; i < V; i++) {
                    if (C0 + m * V + i >= cols) continue;
                    unsigned char *a2 = (cb + (int64_t)i * lddst) + lane;
                    if (rk + EPW <= rows) {
                        stw<W, NTS>(a2, o[i]);
                    } else {
                        union { PT pt; T e[EPW]; } u;
                        u.pt = o[i];
#pragma unroll
                        for (int e = 0; e < EPW; e++)
                            if (rk + e < rows) reinterpret_cast<T *>(a2)[e] = u.e[e];
                    }
                }
            }
        }
    }
}

// W = 0 selects the form for rows that are not 4-byte aligned (funnel-shifted
// 4-byte pieces, default geometry).  OFF32: every per-lane offset inside a
// tile fits in 32 bits (the host checks the pitches), so addresses are a
// uniform 64-bit tile base plus a 32-bit lane offset.
template <int PH, int EB, int W, bool NTL, bool NTS, bool OFF32, int SC = 16, int DC = 16>
__device__ __forceinline__ void phase_any(const unsigned char *src, unsigned char *dst, int64_t rows,
                                          int64_t cols, int64_t ld_src, int64_t ld_dst, int64_t R0,
                                          int64_t C0, uint4 *lds) {
    if constexpr (W == 0) {
        static_assert(SC == 16 && DC == 16, "unaligned rows use the default geometry");
        tile_phase<PH, EB, 1, NTL, NTS, OFF32, 16, 16>(src, dst, rows, cols, ld_src, ld_dst, R0,
                                                       C0, lds);
    } else {
        tile_phase<PH, EB, W, NTL, NTS, OFF32, SC, DC>(src, dst, rows, cols, ld_src, ld_dst, R0,
                                                       C0, lds);
    }
}

template <int EB, int W, bool NTL, bool NTS, bool OFF32, int SC = 16, int DC = 16>
__device__ __forceinline__ void tile_any(const unsigned char *src, unsigned char *dst, int64_t rows,
                                         int64_t cols, int64_t ld_src, int64_t ld_dst, int64_t R0,
                                         int64_t C0, uint4 *lds) {
    phase_any<1, EB, W, NTL, NTS, OFF32, SC, DC>(src, dst, rows, cols, ld_src, ld_dst, R0, C0, lds);
    __syncthreads();   // ownership of the LDS tile moves from loaders to storers
    phase_any<2, EB, W, NTL, NTS, OFF32, SC, DC>(src, dst, rows, cols, ld_src, ld_dst, R0, C0, lds);
}

// ---------------------------------------------------------------- kernels

template <int EB, int W, bool NTL, bool NTS, bool OFF32, int SC = 16, int DC = 16>
__global__ void __launch_bounds__(NT) k_tpose(const unsigned char *__restrict__ src,
                                              unsigned char *__restrict__ dst, int64_t rows,
                                              int64_t cols, int64_t ld_src, int64_t ld_dst,
                                              int64_t tiles_r, int64_t tiles_c, int xcd,
                                              int group, int skew) {
    using G = Geo<EB, SC, DC>;
    __shared__ uint4 lds[G::LDS_VECS];
    const uint32_t ntiles = (uint32_t)(tiles_r * tiles_c), Gd = gridDim.x, bx = blockIdx.x;
    for (uint32_t b = bx; b < ntiles; b += Gd) {
        // position in the launch order: XCD-contiguous within each wave of Gd tiles
        const uint32_t wave0 = b - bx;
        const uint32_t inwave = (ntiles - wave0) < Gd ? (ntiles - wave0) : Gd;
        const uint32_t L = xcd ? wave0 + xcd_remap(bx, inwave) : b;
        uint32_t tr, tc;
        band_order(L, (uint32_t)tiles_r, (uint32_t)tiles_c, (uint32_t)group, tr, tc);
        // skewed band: tile row i of a band starts i tile columns further on
        // (a permutation of each tile row), so that tiles dispatched together
        // differ in both coordinates and, with power-of-two pitches, read and
        // write rows that fall on different memory channels
        if (skew) tc = (tc + tr % (uint32_t)group) % (uint32_t)tiles_c;
        tile_any<EB, W, NTL, NTS, OFF32, SC, DC>(src, dst, rows, cols, ld_src, ld_dst,
                                                 (int64_t)tr * G::TR, (int64_t)tc * G::TC, lds);
        __syncthreads();   // LDS is reused by the next tile of this workgroup
    }
}

// Device-side job of a batched launch.
struct Job {
    const unsigned char *src;
    unsigned char *dst;
    int64_t rows, cols, ld_src, ld_dst;
    int64_t tiles_c;
    int64_t tile_base;   // first global tile id of this job
    int32_t w, _pad;     // piece width in bytes (4, 8, 16), 0 = rows not 4-byte aligned
};
constexpr int JOB_DWORDS = (int)(sizeof(Job) / 4);
static_assert(sizeof(Job) % 4 == 0 && JOB_DWORDS <= 64, "a Job is loaded one dword per lane");

// Job of linear tile L within a group: the last j with bases[j] <= L
// (bases[0] = 0, increasing; bases[j] = first tile of job j).  Every lane of
// a wave probes one candidate per step, so both searches cost one memory
// round trip per step and give the same j in every lane.
__device__ __forceinline__ int job_search(const int64_t *bases, int nj, int64_t L) {
    const int l = threadIdx.x & 63;
    int lo = 0, hi = nj;   // bases[lo] <= L, and L < bases[hi] (bases[nj] is past the end)
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) / 64;
        const int c = lo + l * step;
        const bool le = c < hi && bases[c] <= L;
        lo += (__popcll(__ballot(le)) - 1) * step;   // lane 0 probes lo itself
        hi = (lo + step) < hi ? (lo + step) : hi;
    }
    return lo;
}
__device__ __forceinline__ int job_forward(const int64_t *bases, int nj, int j, int64_t L) {
    const int l = threadIdx.x & 63;
    for (;;) {
        const int c = j + 1 + l;
        const int k = __popcll(__ballot(c < nj && bases[c] <= L));
        j += k;
        if (k < 64) return j;
    }
}

// A job's record, dword i held by lane i (one vector load per lane, so the
// wave can wait for it together with its other vector loads), and the record
// gathered from the lanes.
__device__ __forceinline__ uint32_t job_dword(const Job *jobs, int j) {
    const int l = threadIdx.x & 63;
    const uint32_t *p = reinterpret_cast<const uint32_t *>(jobs + j);
    return p[l < JOB_DWORDS ? l : 0];   // lanes past the record reload dword 0
}
__device__ __forceinline__ Job job_gather(uint32_t v) {
    uint32_t d[JOB_DWORDS];
#pragma unroll
    for (int i = 0; i < JOB_DWORDS; i++) d[i] = (uint32_t)__builtin_amdgcn_readlane((int)v, i);
    Job jb;
    __builtin_memcpy(&jb, d, sizeof(Job));
    return jb;
}

// Persistent over the concatenated tile space of a group of jobs, in slots
// of K consecutive positions of the launch order (K = run, the tiles a
// workgroup takes one after another).  xcd 0 / 1: round r of the grid covers
// positions [r G K, r G K + G K) in G slots; with xcd = 1 each XCD takes a
// contiguous range of the round's slots (xcd_remap).  xcd = 2: each XCD
// sweeps a contiguous eighth of the whole order.  Within a job tiles follow
// the band order, so tiles that share cache lines at their edges (rows of a
// job whose pitch is not a multiple of the line) meet in one L2, and with
// K > 1 in one CU.
// The next tile's job is found while the current tile moves: its search
// probe is loaded before the tile's loads, and its record after the tile is
// staged in LDS, ahead of the tile's stores; neither waits on the tile's
// memory traffic.
template <int EB, int W, bool NTL, bool NTS, bool OFF32, int SC, int DC>
__device__ __forceinline__ void batched_tiles(const Job *jobs, const int64_t *bases, int njobs,
                                              int64_t ntiles64, int xcd, int group, int run,
                                              uint32_t *ctr, uint4 *lds, uint32_t *slot) {
    using Gm = Geo<EB, SC, DC>;
    const uint32_t ntiles = (uint32_t)ntiles64, G = gridDim.x, bx = blockIdx.x;
    const uint32_t K = run > 1 ? (uint32_t)run : 1u;
    const int l = threadIdx.x & 63;
    // xcd == 2 (with at least 8 workgroups): XCD x = bx % 8 sweeps its own
    // eighth [lo_x, hi_x) of the launch order, its Gx workgroups taking slots
    // of K positions round-robin, as a launch of one workgroup per tile
    // places them; so the tiles that share edge lines meet in one L2 close
    // together in time.  Slot s of region x goes to workgroup 8 (s % Gx) + x,
    // and 8 (Gx - 1) + x < G, so every position is taken exactly once.
    // xcd == 3 (with a counter block): the order is cut into chunks of
    // CS slots, chunk k belonging to "XCD" k % 8, and a workgroup takes the
    // next free slot of its XCD's chunks from that XCD's counter, as the
    // dispatcher hands out the workgroups of a launch of one workgroup per
    // tile: the tiles in flight stay a window of the order however the
    // workgroups' speeds drift apart, and the eight XCDs work on adjacent
    // chunks (far-apart windows that advance in step can meet the same HBM
    // channels).  Each counter value is taken once, and the values of XCD x
    // map to increasing positions, so its workgroups, which take values in
    // increasing order until one lies past the end, take every position of
    // x's chunks; every class bx % 8 has a workgroup (G >= 8).
    constexpr uint32_t CS = 128;
    const bool dyn = xcd == 3 && ctr != nullptr && G >= 8;
    const bool reg = xcd == 2 && G >= 8;
    const uint32_t xr = bx & 7, kx = bx >> 3;
    const uint32_t Gx = (G >> 3) + (xr < (G & 7) ? 1u : 0u);
    const uint32_t share = (ntiles + 7) >> 3;
    const uint32_t lo_x = xr * share < ntiles ? xr * share : ntiles;
    const uint32_t hi_x = ntiles - lo_x < share ? ntiles : lo_x + share;
    // this workgroup's positions: visit R, its first position, count, index
    uint32_t R = 0, first = 0, count = 0, i = 0;
    auto visit = [&](uint32_t r) {   // this workgroup's r-th slot; false: none left
        uint64_t f;
        uint32_t end;
        if (reg) {
            f = (uint64_t)lo_x + ((uint64_t)kx + (uint64_t)r * Gx) * K;
            end = hi_x;
        } else {
            const uint64_t r0 = (uint64_t)r * G * K;   // rounds of G slots
            if (r0 >= ntiles) return false;
            const uint32_t rem = ntiles - (uint32_t)r0;
            const uint32_t slots = (rem + K - 1) / K < G ? (rem + K - 1) / K : G;
            if (bx >= slots) return false;
            f = r0 + (uint64_t)(xcd ? xcd_remap(bx, slots) : bx) * K;
            end = ntiles;
        }
        if (f >= end) return false;
        R = r;
        first = (uint32_t)f;
        count = end - first < K ? end - first : K;
        i = 0;
        return true;
    };
    // dynamic slots: value s of XCD x is slot s % CS of x's chunk s / CS,
    // i.e. chunk 8 (s / CS) + x of the order (CS K positions per chunk)
    auto take = [&](uint32_t s) {
        const uint64_t chunk = (uint64_t)(s / CS) * 8 + xr;
        const uint64_t f = (chunk * CS + s % CS) * K;
        if (f >= ntiles) return false;
        first = (uint32_t)f;
        count = ntiles - first < K ? ntiles - first : K;
        i = 0;
        return true;
    };
    bool live;
    if (dyn) {
        if (threadIdx.x == 0)
            slot[0] = __hip_atomic_fetch_add(&ctr[xr], 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        live = take(slot[0]);
    } else {
        live = visit(0);
    }
    if (live) {
        uint32_t L = first;
        int j = job_search(bases, njobs, L);
        Job jb = job_gather(job_dword(jobs, j));
        for (;;) {
            // the next position of this workgroup: the next one of its slot, or
            // the first of its next slot (a dynamic slot is known after the
            // barrier below: its counter is read while the tile loads fly)
            bool more = false, ask = false;
            uint32_t got = 0;
            if (i + 1 < count) {
                i++;
                more = true;
            } else if (dyn) {
                ask = true;
                if (threadIdx.x == 0)
                    got = __hip_atomic_fetch_add(&ctr[xr], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            } else {
                more = visit(R + 1);
            }
            uint32_t Ln = more ? first + i : 0;
            int c = 0;
            int64_t probe = 0;
            if (more) {
                c = j + 1 + l;
                probe = bases[c < njobs ? c : njobs - 1];   // (unconditional load; c checked below)
            }
            const uint32_t tiles_r = (uint32_t)((jb.rows + Gm::TR - 1) / Gm::TR);
            uint32_t tr, tc;
            band_order(L - (uint32_t)jb.tile_base, tiles_r, (uint32_t)jb.tiles_c, (uint32_t)group,
                       tr, tc);
            const int64_t R0 = (int64_t)tr * Gm::TR, C0 = (int64_t)tc * Gm::TC;
            phase_any<1, EB, W, NTL, NTS, OFF32, SC, DC>(jb.src, jb.dst, jb.rows, jb.cols,
                                                         jb.ld_src, jb.ld_dst, R0, C0, lds);
            if (ask && threadIdx.x == 0) slot[1] = got;
            __syncthreads();   // ownership of the LDS tile moves from loaders to storers
            if (ask) {
                more = take(slot[1]);
                Ln = more ? first : 0;
                if (more) {
                    c = j + 1 + l;
                    probe = bases[c < njobs ? c : njobs - 1];
                }
            }
            uint32_t next = 0;
            if (more) {
                const int k = __popcll(__ballot(c < njobs && probe <= (int64_t)Ln));
                j += k;
                if (k == 64) j = job_forward(bases, njobs, j, Ln);   // more than 64 jobs ahead
                next = job_dword(jobs, j);
            }
            phase_any<2, EB, W, NTL, NTS, OFF32, SC, DC>(jb.src, jb.dst, jb.rows, jb.cols,
                                                         jb.ld_src, jb.ld_dst, R0, C0, lds);
            __syncthreads();   // LDS is reused by the next tile of this workgroup
            if (!more) break;
            jb = job_gather(next);
            L = Ln;
        }
    }
    if (dyn && threadIdx.x == 0) {
        // the last workgroup to leave sets the counters back to zero for the
        // next launch: every workgroup takes its last slot before it counts
        // itself out (release), and the last one sees all of them (acquire)
        const uint32_t done = __hip_atomic_fetch_add(&ctr[8], 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (done == G - 1) {
#pragma unroll
            for (int k = 0; k < 9; k++)
                __hip_atomic_store(&ctr[k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Tile geometry of a batch group: SC / DC 16-byte chunks per src / dst row
// segment (SC = 32: 512-byte src row segments, DC = 32: 512-byte dst ones).
template <int EB, int W, bool NTL, bool NTS, bool OFF32, int SC = 16, int DC = 16>
__global__ void __launch_bounds__(NT) k_tpose_batched(const Job *__restrict__ jobs,
                                                      const int64_t *__restrict__ bases, int njobs,
                                                      int64_t ntiles, int xcd, int group, int run,
                                                      uint32_t *ctr) {
    __shared__ uint4 lds[Geo<EB, SC, DC>::LDS_VECS];
    __shared__ uint32_t slot[2];
    batched_tiles<EB, W, NTL, NTS, OFF32, SC, DC>(jobs, bases, njobs, ntiles, xcd, group, run, ctr,
                                                  lds, slot);
}

// A small group passes its jobs inside the kernel arguments: no table upload
// (no host-to-device copy ahead of the kernel in the stream).
constexpr int INLINE_JOBS = 24;
struct JobPack {
    Job jobs[INLINE_JOBS];
    int64_t bases[INLINE_JOBS];
};

template <int EB, int W, bool NTL, bool NTS, bool OFF32, int SC = 16, int DC = 16>
__global__ void __launch_bounds__(NT) k_tpose_batched_inl(JobPack pk, int njobs, int64_t ntiles,
                                                          int xcd, int group, int run) {
    __shared__ uint4 lds[Geo<EB, SC, DC>::LDS_VECS];
    batched_tiles<EB, W, NTL, NTS, OFF32, SC, DC>(pk.jobs, pk.bases, njobs, ntiles, xcd, group, run,
                                                  nullptr, lds, nullptr);
}

// ---------------------------------------------------------------- host side


// Per-lane offsets inside a tile stay below 2^31 (so the 32-bit addressing of
// tile_phase is exact): tile rows x row pitch on either side, plus one row.
template <int EB, int SC = 16, int DC = 16> bool off32_ok(int64_t ld_src, int64_t ld_dst) {
    using G = Geo<EB, SC, DC>;
    const int64_t lim = (int64_t)1 << 31;
    return (int64_t)G::TR * ld_src * EB + 16 * SC < lim &&
           (int64_t)G::TC * ld_dst * EB + 16 * DC < lim;
}
inline bool off32_rt(int eb, int64_t ld_src, int64_t ld_dst) {
    switch (eb) {
    case 1: return off32_ok<1>(ld_src, ld_dst);
    case 2: return off32_ok<2>(ld_src, ld_dst);
    case 4: return off32_ok<4>(ld_src, ld_dst);
    default: return off32_ok<8>(ld_src, ld_dst);
    }
}

// Widest piece (16, 8 or 4 bytes, and >= the element) that divides both base
// pointers and both row pitches; 0 = none (1- or 2-byte elements only): rows
// not 4-byte aligned, moved as funnel-shifted 4-byte pieces.
inline int piece_width(const void *src, const void *dst, int64_t ld_src, int64_t ld_dst, int eb) {
    const uint64_t a = (uint64_t)(uintptr_t)src | (uint64_t)(uintptr_t)dst |
                       (uint64_t)(ld_src * eb) | (uint64_t)(ld_dst * eb);
    for (int w = 16; w >= 4; w >>= 1)
        if (w >= eb && (a % w) == 0) return w;
    return 0;
}

template <int EB, int SC = 16, int DC = 16>
int64_t tiles_of(int64_t rows, int64_t cols, int64_t *tiles_c) {
    using G = Geo<EB, SC, DC>;
    const int64_t tr = (rows + G::TR - 1) / G::TR;
    const int64_t tc = (cols + G::TC - 1) / G::TC;
    if (tiles_c) *tiles_c = tc;
    return tr * tc;
}

// Tile geometries of 2- to 8-byte elements: 0 = 256 x 256 bytes, 1 = 512-byte
// src row segments (SC = 32), 2 = 512-byte dst row segments (DC = 32), 3 =
// both (4- and 8-byte elements only: 64 KiB of LDS for fp32).  Wider row
// segments leave fewer partial cache lines at segment ends, which neighbouring
// tiles share when rows do not start on lines.
template <int EB, int GEO> struct GeoOf;
template <int EB> struct GeoOf<EB, 0> { static constexpr int SC = 16, DC = 16; };
template <int EB> struct GeoOf<EB, 1> { static constexpr int SC = 32, DC = 16; };
template <int EB> struct GeoOf<EB, 2> { static constexpr int SC = 16, DC = 32; };
template <int EB> struct GeoOf<EB, 3> { static constexpr int SC = 32, DC = 32; };
template <int EB> struct GeoOf<EB, 4> { static constexpr int SC = 16, DC = 64; };

inline int64_t tiles_for(int eb, int64_t rows, int64_t cols, int64_t *tiles_c, int geo = 0) {
#define XTR_TF(E)                                                                              \
    return geo == 1 ? tiles_of<E, 32, 16>(rows, cols, tiles_c)                                \
         : geo == 2 ? tiles_of<E, 16, 32>(rows, cols, tiles_c)                                \
         : geo == 3 && E >= 4 ? tiles_of<E, 32, 32>(rows, cols, tiles_c)                      \
         : geo == 4 && E >= 4 ? tiles_of<E, 16, 64>(rows, cols, tiles_c)                      \
                              : tiles_of<E>(rows, cols, tiles_c)
    switch (eb) {
    case 1: return tiles_of<1>(rows, cols, tiles_c);
    case 2: XTR_TF(2);
    case 4: XTR_TF(4);
    default: XTR_TF(8);
    }
#undef XTR_TF
}

inline bool off32_geo(int eb, int geo, int64_t ld_src, int64_t ld_dst) {
#define XTR_OG(E)                                                                              \
    return geo == 1 ? off32_ok<E, 32, 16>(ld_src, ld_dst)                                     \
         : geo == 2 ? off32_ok<E, 16, 32>(ld_src, ld_dst)                                     \
         : geo == 3 && E >= 4 ? off32_ok<E, 32, 32>(ld_src, ld_dst)                           \
         : geo == 4 && E >= 4 ? off32_ok<E, 16, 64>(ld_src, ld_dst) : off32_ok<E>(ld_src, ld_dst)
    switch (eb) {
    case 1: return off32_ok<1>(ld_src, ld_dst);
    case 2: XTR_OG(2);
    case 4: XTR_OG(4);
    default: XTR_OG(8);
    }
#undef XTR_OG
}

constexpr int64_t MAX_GRID = 1 << 20;   // workgroups per launch; larger jobs loop

// Tuned launch configuration per element size (slot cfg_slot(elem bytes));
// defined in tpose.hip, set through xtr_tpose_set_config.
// g_cfg[XTR_SHAPE_SINGLE] serves single transposes, g_cfg[XTR_SHAPE_BATCHED]
// the groups of batched launches.
extern xtr_tpose_config g_cfg[2][4];
inline int cfg_slot(int eb) { return eb == 1 ? 0 : eb == 2 ? 1 : eb == 4 ? 2 : 3; }

template <int EB, int W, bool NTL, bool NTS, int SC, int DC>
void launch_k(dim3 grid, hipStream_t st, const void *src, void *dst, int64_t rows, int64_t cols,
              int64_t ld_src, int64_t ld_dst, int64_t tiles_r, int64_t tiles_c, int xcd,
              int group, int skew) {
    if (off32_ok<EB, SC, DC>(ld_src, ld_dst))
        hipLaunchKernelGGL((k_tpose<EB, W, NTL, NTS, true, SC, DC>), grid, dim3(NT), 0, st,
                           (const unsigned char *)src, (unsigned char *)dst, rows, cols, ld_src,
                           ld_dst, tiles_r, tiles_c, xcd, group, skew);
    else
        hipLaunchKernelGGL((k_tpose<EB, W, NTL, NTS, false, SC, DC>), grid, dim3(NT), 0, st,
                           (const unsigned char *)src, (unsigned char *)dst, rows, cols, ld_src,
                           ld_dst, tiles_r, tiles_c, xcd, group, skew);
}

// Rows of a matrix start on 128-byte cache lines (base and pitch), so no
// line is shared by two tiles.  Streaming (nontemporal) accesses suit such
// rows; where tiles share the lines at their edges, the neighbour tile wants
// those lines to stay cached, and the *_shared settings apply.
inline bool lines_ok(const void *p, int64_t ld, int eb) {
    return (((uint64_t)(uintptr_t)p | (uint64_t)(ld * eb)) & 127) == 0;
}

template <int EB, int W, int SC = 16, int DC = 16>
void launch_w(const xtr_tpose_config &c, hipStream_t st, const void *src, void *dst,
              int64_t rows, int64_t cols, int64_t ld_src, int64_t ld_dst) {
    using G = Geo<EB, SC, DC>;
    const int64_t tiles_r = (rows + G::TR - 1) / G::TR;
    const int64_t tiles_c = (cols + G::TC - 1) / G::TC;
    const int64_t ntiles = tiles_r * tiles_c;
    int64_t grid = ntiles < MAX_GRID ? ntiles : MAX_GRID;
    if (c.blocks_per_cu > 0) {
        const int64_t g = (int64_t)cu_count() * c.blocks_per_cu;
        if (g < grid) grid = g;
    }
    const int group = c.group < 1 ? 1 : c.group;
    // 512 x 512-byte tiles and both byte pitches powers of two: tiles of one
    // tile column share memory channels, so the band is skewed (fp32 16384 x
    // 16384 +2%, 8192 x 8192 +4%; other pitches gain nothing, and other
    // geometries lose: fp64 16384 x 8192 in 512-byte src segments -3%)
    const uint64_t ps = (uint64_t)(ld_src * EB), pd = (uint64_t)(ld_dst * EB);
    const int skew = (SC == 32 && DC == 32 && (ps & (ps - 1)) == 0 && (pd & (pd - 1)) == 0) ? 1 : 0;
    const dim3 gd((unsigned)grid);
    const bool ntl = lines_ok(src, ld_src, EB) ? c.nt_load != 0 : c.nt_load_shared != 0;
    const bool nts = lines_ok(dst, ld_dst, EB) ? c.nt_store != 0 : c.nt_store_shared != 0;
#define XTR_K(NL, NS)                                                                        \
    launch_k<EB, W, NL, NS, SC, DC>(gd, st, src, dst, rows, cols, ld_src, ld_dst, tiles_r,    \
                                    tiles_c, c.xcd, group, skew)
    if (ntl && nts) XTR_K(true, true);
    else if (ntl) XTR_K(true, false);
    else if (nts) XTR_K(false, true);
    else XTR_K(false, false);
#undef XTR_K
}

// Tile geometry of a single transpose (`tile` for line-aligned rows,
// `tile_shared` otherwise): 1 = 512-byte src row segments, 2 = 512-byte dst
// row segments, 3 = both, 4 = 1 KiB dst row segments of 256-byte src ones (3
// and 4: 4- and 8-byte elements), else 256 x 256 bytes.  Wider segments halve
// the share of edge lines that neighbouring tiles split.  2- to 8-byte
// elements only.
// A matrix of fewer default tiles than c.wide_min per CU keeps the default
// geometry: there wide tiles leave CUs idle and tie or lose; from fp32 8192 x
// 8192 up they win, halving the edge lines that tiles of power-of-two strides
// split.
template <int EB>
int launch_one(const void *src, void *dst, int64_t rows, int64_t cols, int64_t ld_src,
               int64_t ld_dst, hipStream_t stream) {
    const xtr_tpose_config &c = g_cfg[XTR_SHAPE_SINGLE][cfg_slot(EB)];
    const bool lines = lines_ok(src, ld_src, EB) && lines_ok(dst, ld_dst, EB);
    const int64_t ntiles = ((rows + Geo<EB>::TR - 1) / Geo<EB>::TR) *
                           ((cols + Geo<EB>::TC - 1) / Geo<EB>::TC);
    if (ntiles >= MAX_TILES) return fail(XTR_EINVAL, "tpose: %lld tiles (limit 2^31)", (long long)ntiles);
    const int tile = ntiles < (int64_t)c.wide_min * cu_count() ? 0
                   : lines ? c.tile : c.tile_shared;
    switch (piece_width(src, dst, ld_src, ld_dst, EB)) {
    case 16:
        if constexpr (EB >= 4) {
            if (tile == 3) {
                launch_w<EB, 16, 32, 32>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
            if (tile == 4) {
                launch_w<EB, 16, 16, 64>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
        }
        if constexpr (EB >= 2) {
            if (tile == 1) {
                launch_w<EB, 16, 32, 16>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
            if (tile == 2) {
                launch_w<EB, 16, 16, 32>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
        }
        launch_w<EB, 16>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
        break;
    case 8:
        if constexpr (EB >= 4 && EB <= 8) {
            if (tile == 3) {
                launch_w<EB, 8, 32, 32>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
            if (tile == 4) {
                launch_w<EB, 8, 16, 64>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
        }
        if constexpr (EB >= 2 && EB <= 8) {
            if (tile == 1) {
                launch_w<EB, 8, 32, 16>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
            if (tile == 2) {
                launch_w<EB, 8, 16, 32>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
        }
        if constexpr (EB <= 8) launch_w<EB, 8>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
        break;
    case 4:
        if constexpr (EB == 4) {
            if (tile == 3) {
                launch_w<EB, 4, 32, 32>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
            if (tile == 4) {
                launch_w<EB, 4, 16, 64>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
        }
        if constexpr (EB >= 2 && EB <= 4) {
            if (tile == 1) {
                launch_w<EB, 4, 32, 16>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
            if (tile == 2) {
                launch_w<EB, 4, 16, 32>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
                break;
            }
        }
        if constexpr (EB <= 4) launch_w<EB, 4>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
        break;
    default:
        if constexpr (EB <= 2) launch_w<EB, 0>(c, stream, src, dst, rows, cols, ld_src, ld_dst);
        break;
    }
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

// `lines`: every job of the group has line-aligned src and dst rows.  `pk`
// (host) non-null: the group's jobs travel in the kernel arguments.
template <int EB, int W, bool OFF32, int SC = 16, int DC = 16>
void launch_batched_w(bool lines, int64_t grid, hipStream_t st, const Job *jobs,
                      const int64_t *bases, int nj, int64_t ntiles, const JobPack *pk,
                      uint32_t *ctr) {
    const xtr_tpose_config &c = g_cfg[XTR_SHAPE_BATCHED][cfg_slot(EB)];
    const bool ntl = lines ? c.nt_load != 0 : c.nt_load_shared != 0;
    const bool nts = lines ? c.nt_store != 0 : c.nt_store_shared != 0;
    const int group = c.group < 1 ? 1 : c.group;
    // persistent grid: the resident capacity, or blocks_per_cu workgroups per CU
    const int cap = c.blocks_per_cu;
#define XTR_KB(NL, NS)                                                                      \
    do {                                                                                    \
        if (pk) {                                                                           \
            const int64_t occ = resident_blocks(                                            \
                (const void *)&k_tpose_batched_inl<EB, W, NL, NS, OFF32, SC, DC>, NT, cap);  \
            hipLaunchKernelGGL((k_tpose_batched_inl<EB, W, NL, NS, OFF32, SC, DC>),         \
                               dim3((unsigned)(grid < occ ? grid : occ)), dim3(NT), 0, st,   \
                               *pk, nj, ntiles, c.xcd, group, c.run);                       \
        } else {                                                                            \
            const int64_t occ = resident_blocks(                                            \
                (const void *)&k_tpose_batched<EB, W, NL, NS, OFF32, SC, DC>, NT, cap);      \
            hipLaunchKernelGGL((k_tpose_batched<EB, W, NL, NS, OFF32, SC, DC>),             \
                               dim3((unsigned)(grid < occ ? grid : occ)), dim3(NT), 0, st,   \
                               jobs, bases, nj, ntiles, c.xcd, group, c.run, ctr);          \
        }                                                                                   \
    } while (0)
    if (ntl && nts) XTR_KB(true, true);
    else if (ntl) XTR_KB(true, false);
    else if (nts) XTR_KB(false, true);
    else XTR_KB(false, false);
#undef XTR_KB
}

// geo: the group's tile geometry (0 to 4, as `tile`); the wider ones need
// 32-bit lane offsets (the host groups jobs accordingly).
template <int EB>
void launch_batched(int w, bool off32, bool lines, int geo, int64_t grid, hipStream_t st,
                    const Job *jobs, const int64_t *bases, int nj, int64_t ntiles,
                    const JobPack *pk, uint32_t *ctr) {
#define XTR_BW(WW)                                                                             \
    if constexpr (EB >= 2 && WW >= 4) {                                                        \
        if (geo == 1) {                                                                        \
            launch_batched_w<EB, WW, true, 32, 16>(lines, grid, st, jobs, bases, nj, ntiles, pk, ctr); \
            return;                                                                            \
        }                                                                                      \
        if (geo == 2) {                                                                        \
            launch_batched_w<EB, WW, true, 16, 32>(lines, grid, st, jobs, bases, nj, ntiles, pk, ctr); \
            return;                                                                            \
        }                                                                                      \
    }                                                                                          \
    if constexpr (EB >= 4 && WW >= 4) {                                                        \
        if (geo == 3) {                                                                        \
            launch_batched_w<EB, WW, true, 32, 32>(lines, grid, st, jobs, bases, nj, ntiles, pk, ctr); \
            return;                                                                            \
        }                                                                                      \
        if (geo == 4) {                                                                        \
            launch_batched_w<EB, WW, true, 16, 64>(lines, grid, st, jobs, bases, nj, ntiles, pk, ctr); \
            return;                                                                            \
        }                                                                                      \
    }                                                                                          \
    if (off32) launch_batched_w<EB, WW, true>(lines, grid, st, jobs, bases, nj, ntiles, pk, ctr);   \
    else launch_batched_w<EB, WW, false>(lines, grid, st, jobs, bases, nj, ntiles, pk, ctr);
    switch (w) {
    case 16: XTR_BW(16) break;
    case 8:
        if constexpr (EB <= 8) { XTR_BW(8) }
        break;
    case 4:
        if constexpr (EB <= 4) { XTR_BW(4) }
        break;
    default:
        if constexpr (EB <= 2) { XTR_BW(0) }
        break;
    }
#undef XTR_BW
}


// Per element size EB (1, 2, 4, 8): a single transpose (launch_one<EB>,
// defined in tpose_s<EB>.hip) and one group launch of a batch
// (launch_batched<EB>, defined in tpose_b<EB>.hip).
#define XTR_TPOSE_EB_DECL(EB)                                                               \
    int launch_single_e##EB(const void *src, void *dst, int64_t rows, int64_t cols,          \
                            int64_t ld_src, int64_t ld_dst, hipStream_t stream);             \
    void launch_group_e##EB(int w, bool off32, bool lines, int geo, int64_t grid,            \
                            hipStream_t st, const Job *jobs, const int64_t *bases, int nj,   \
                            int64_t ntiles, const JobPack *pk, uint32_t *ctr);
XTR_TPOSE_EB_DECL(1)
XTR_TPOSE_EB_DECL(2)
XTR_TPOSE_EB_DECL(4)
XTR_TPOSE_EB_DECL(8)
#undef XTR_TPOSE_EB_DECL

}  // namespace tpk
}  // namespace xtr
