// Index maps of the transpose tile (plain constexpr integer arithmetic, so the
// same functions serve the HIP kernels and a host-side checker that
// enumerates every thread of every tile geometry).
//
// A tile is TR x TC elements: TR tile rows of 16 * SC bytes (the src row
// segment), staged in LDS as TR rows of SC 16-byte chunks.  Phase 1: thread t
// loads the W-byte piece (t % P) of tile rows t / P + RP * p (p < PASSES) and
// writes it to LDS.  A block barrier follows (ownership of the LDS tile moves
// from the loading threads to the storing threads, Section 3.3).  Phase 2:
// thread t owns piece k = t % P2 of the dst row segments of the 16-byte
// column chunks m = t / P2 + RP2 * cc (cc < CPT); it reads the EPW tile rows
// k * EPW + e (e < EPW) of chunk m and writes, for each of the V columns i of
// the chunk, the piece (row k * EPW + e of column m * V + i, e < EPW) to dst
// row m * V + i at byte k * W of the dst row segment.
#pragma once

namespace xtr {
namespace tmap {

// Physical 16-byte chunk of logical chunk k in tile row `row`: XOR with a
// per-row key, so each row holds a permutation of its chunks.  The key
// (row / V) ^ (row % V) * (16 / V) takes 16 distinct values both over the rows
// {b * V + i : b = 0..15} (fixed i) that a 16-lane group reads in the V x V
// block layout, and over the rows that 8 consecutive lanes read in the narrow
// piece layout (rows k * E + e for k = 0..7, E = 1, 2, 4 or 8 elements per
// piece), so neither read pattern serialises on LDS banks.
template <int EB> constexpr int swz(int row, int k) {
    constexpr int V = 16 / EB;
    return k ^ (((row / V) ^ ((row % V) * (16 / V))) & 15);
}

// EB: element bytes; WP: piece bytes (4, 8, 16); SC / DC: 16-byte chunks per
// src / dst row segment; NT: threads per workgroup.
template <int EB, int WP, int SC, int DC, int NT> struct TileMap {
    static constexpr int V = 16 / EB;            // elements per 16-byte chunk
    static constexpr int TC = SC * V;            // tile columns
    static constexpr int TR = DC * V;            // tile rows
    static constexpr int P = 16 * SC / WP;       // pieces per src row segment
    static constexpr int RP = NT / P;            // tile rows per phase-1 pass
    static constexpr int PASSES = TR / RP;
    static constexpr int EPW = WP / EB;          // elements per piece
    static constexpr int P2 = 16 * DC / WP;      // pieces per dst row segment
    static constexpr int RP2 = NT / P2;          // column chunks per phase-2 pass
    static constexpr int CPT = SC / RP2;         // column chunks per thread
    static_assert(RP >= 1 && PASSES >= 1 && TR % RP == 0, "phase-1 lane layout");
    static_assert(RP2 >= 1 && CPT >= 1 && SC % RP2 == 0, "phase-2 lane layout");

    // phase 1: tile row and byte (within the src row segment) of thread t, pass p
    static constexpr int p1_row(int t, int p) { return t / P + RP * p; }
    static constexpr int p1_byte(int t) { return (t % P) * WP; }
    // LDS byte address of byte `byte` of tile row `row`
    static constexpr int lds_byte(int row, int byte) {
        return (row * SC + swz<EB>(row, byte >> 4)) * 16 + (byte & 15);
    }
    // phase 2: piece index, column chunk, and the LDS 16-byte chunk it reads
    static constexpr int p2_piece(int t) { return t % P2; }
    static constexpr int p2_chunk(int t, int cc) { return t / P2 + RP2 * cc; }
    static constexpr int p2_lds_vec(int k, int e, int m) {
        return (k * EPW + e) * SC + swz<EB>(k * EPW + e, m);
    }
};

}  // namespace tmap
}  // namespace xtr
