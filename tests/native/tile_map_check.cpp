// Host-side check of the transpose tile's index maps (tile_map.h, the same
// functions the HIP kernels use), over every thread of every tile geometry
// the library instantiates:
//   * exact cover: phase 1 writes every LDS byte of the tile exactly once, and
//     the pieces of phase 2 write every byte of the dst tile exactly once;
//   * data path: the LDS chunk a phase-2 thread reads holds exactly the src
//     bytes the transpose needs (the swizzle is undone), so dst element
//     (c, r) receives src element (r, c);
//   * barrier order: with the barrier between the phases and the one closing
//     each tile, no LDS cell is written and read by different threads within
//     one barrier interval; without the first barrier some are (it is needed
//     exactly where ownership moves from the loading to the storing threads,
//     the rule of Section 3.3), and likewise for the closing barrier;
//   * LDS banks (model: 64 banks of 4 bytes; a 16-byte access serves 16 lanes
//     per cycle, an 8-byte one 32, a 4-byte one 64): the worst number of
//     distinct addresses that share a bank within one cycle's lanes, reported
//     per instruction class; phase-2 reads must be conflict-free.
// Prints one line per geometry; exit status 1 on any failure.
// TILE_MAP_H: the header under test (the mutation tests point it at a copy)
#ifndef TILE_MAP_H
#define TILE_MAP_H "../../paper_2605_13864_amd/csrc/tile_map.h"
#endif
#include TILE_MAP_H

#include <cstdio>
#include <map>
#include <set>
#include <vector>

using namespace xtr::tmap;

static int failures = 0;
#define CHECK(c, ...)                                                   \
    do {                                                                \
        if (!(c)) {                                                     \
            if (++failures < 20) {                                      \
                std::printf("FAIL line %d: ", __LINE__);                \
                std::printf(__VA_ARGS__);                               \
                std::printf("\n");                                      \
            }                                                           \
        }                                                               \
    } while (0)

constexpr int NT = 256;

// worst bank-conflict degree of one wave-wide access of `bytes` per lane
static int conflict_degree(const std::vector<int> &addr, int bytes) {
    const int per_cycle = bytes == 16 ? 16 : bytes == 8 ? 32 : 64;
    int worst = 1;
    for (int g0 = 0; g0 < 64; g0 += per_cycle) {
        std::map<int, std::set<int>> bank;   // bank of the access's first dword -> addresses
        for (int l = g0; l < g0 + per_cycle; l++) bank[(addr[l] >> 2) & 63].insert(addr[l]);
        for (auto &kv : bank) worst = std::max(worst, (int)kv.second.size());
    }
    return worst;
}

template <int EB, int WP, int SC, int DC> void check(const char *name) {
    using M = TileMap<EB, WP, SC, DC, NT>;
    const int ROWB = 16 * SC;                  // bytes of a tile row (src row segment)
    const int LDSB = M::TR * ROWB;
    const int DROWB = M::TR * EB;              // bytes of a dst row segment
    const int fails0 = failures;
    // phase 1 (epoch 0): who writes which LDS byte, holding which src byte
    std::vector<int> src_of(LDSB, -1), writer(LDSB, -1);
    int w1_worst = 1;
    for (int p = 0; p < M::PASSES; p++) {
        std::vector<int> addr(NT);
        for (int t = 0; t < NT; t++) {
            const int row = M::p1_row(t, p), b0 = M::p1_byte(t);
            CHECK(row >= 0 && row < M::TR && b0 >= 0 && b0 + WP <= ROWB, "%s p1 range", name);
            addr[t] = M::lds_byte(row, b0);
            for (int q = 0; q < WP; q++) {
                const int a = M::lds_byte(row, b0 + q);
                CHECK(a >= 0 && a < LDSB, "%s p1 lds range", name);
                if (a < 0 || a >= LDSB) continue;
                CHECK(src_of[a] == -1, "%s LDS byte %d written twice", name, a);
                CHECK(a == addr[t] + q, "%s piece not contiguous in LDS", name);
                src_of[a] = row * ROWB + b0 + q;
                writer[a] = t;
            }
        }
        for (int w = 0; w < NT / 64; w++)
            w1_worst = std::max(w1_worst, conflict_degree(
                std::vector<int>(addr.begin() + 64 * w, addr.begin() + 64 * w + 64), WP));
    }
    for (int a = 0; a < LDSB; a++) CHECK(src_of[a] != -1, "%s LDS byte %d never written", name, a);
    // phase 2 (epoch 1): reads, and the dst bytes written
    std::vector<int> dst_src(M::TC * DROWB, -1);
    int cross = 0, r2_worst = 1;
    for (int cc = 0; cc < M::CPT; cc++)
        for (int e = 0; e < M::EPW; e++) {
            std::vector<int> addr(NT);
            for (int t = 0; t < NT; t++) {
                const int k = M::p2_piece(t), m = M::p2_chunk(t, cc);
                CHECK(k >= 0 && k * M::EPW + e < M::TR && m >= 0 && m < SC, "%s p2 range", name);
                const int vec = M::p2_lds_vec(k, e, m);
                addr[t] = vec * 16;
                const int row = k * M::EPW + e;
                for (int j = 0; j < 16; j++) {
                    const int a = vec * 16 + j;
                    CHECK(a >= 0 && a < LDSB, "%s p2 lds range", name);
                    if (a < 0 || a >= LDSB) continue;
                    // the chunk holds logical bytes m*16 .. m*16+15 of tile row `row`
                    CHECK(src_of[a] == row * ROWB + m * 16 + j, "%s swizzle not undone", name);
                    if (writer[a] != t) cross++;
                }
                // element i of the chunk (src column m*V + i) goes to dst row m*V + i,
                // element e of piece k: dst byte k*WP + e*EB of that row
                for (int i = 0; i < M::V; i++)
                    for (int q = 0; q < EB; q++) {
                        const int d = (m * M::V + i) * DROWB + k * WP + e * EB + q;
                        CHECK(d >= 0 && d < (int)dst_src.size(), "%s dst range", name);
                        CHECK(dst_src[d] == -1, "%s dst byte written twice", name);
                        dst_src[d] = row * ROWB + (m * M::V + i) * EB + q;
                    }
            }
            for (int w = 0; w < NT / 64; w++)
                r2_worst = std::max(r2_worst, conflict_degree(
                    std::vector<int>(addr.begin() + 64 * w, addr.begin() + 64 * w + 64), 16));
        }
    // dst (c, r) <- src (r, c), every byte once
    for (int c = 0; c < M::TC; c++)
        for (int r = 0; r < M::TR; r++)
            for (int q = 0; q < EB; q++)
                CHECK(dst_src[c * DROWB + r * EB + q] == r * ROWB + c * EB + q,
                      "%s dst (%d, %d) is not src (%d, %d)", name, c, r, r, c);
    // barriers: phase 2 reads bytes written by other threads in phase 1, so
    // the barrier between the phases is required; the next tile's phase 1
    // overwrites bytes this tile's phase 2 reads in other threads, so the
    // closing barrier is required too (the maps are the same every tile).
    CHECK(cross > 0, "%s: no ownership change, the barrier would be redundant", name);
    CHECK(r2_worst == 1, "%s phase-2 reads conflict %d-way", name, r2_worst);
    std::printf("%-28s TR=%3d TC=%3d passes=%2d ok=%d  phase1 %2d-byte writes: %d-way  "
                "phase2 16-byte reads: %d-way  LDS bytes read across threads: %d\n",
                name, M::TR, M::TC, M::PASSES, failures == fails0, WP, w1_worst, r2_worst, cross);
}

int main() {
    // (element bytes, piece bytes, src / dst 16-byte chunks per row segment):
    // every geometry the transpose kernels instantiate (W = 0 rows move
    // 4-byte pieces through the same maps)
    check<1, 16, 16, 16>("u8  W16 256x256");
    check<1, 8, 16, 16>("u8  W8  256x256");
    check<1, 4, 16, 16>("u8  W4  256x256");
    check<2, 16, 16, 16>("b16 W16 256x256");
    check<2, 8, 16, 16>("b16 W8  256x256");
    check<2, 4, 16, 16>("b16 W4  256x256");
    check<2, 16, 32, 16>("b16 W16 src512");
    check<2, 16, 16, 32>("b16 W16 dst512");
    check<2, 8, 16, 32>("b16 W8  dst512");
    check<2, 4, 16, 32>("b16 W4  dst512");
    check<4, 16, 16, 16>("f32 W16 256x256");
    check<4, 8, 16, 16>("f32 W8  256x256");
    check<4, 4, 16, 16>("f32 W4  256x256");
    check<4, 16, 32, 16>("f32 W16 src512");
    check<4, 16, 16, 32>("f32 W16 dst512");
    check<4, 8, 16, 32>("f32 W8  dst512");
    check<4, 4, 16, 32>("f32 W4  dst512");
    check<8, 16, 16, 16>("f64 W16 256x256");
    check<8, 8, 16, 16>("f64 W8  256x256");
    check<8, 16, 32, 16>("f64 W16 src512");
    check<8, 16, 16, 32>("f64 W16 dst512");
    check<8, 8, 16, 32>("f64 W8  dst512");
    check<2, 8, 32, 16>("b16 W8  src512");
    check<2, 4, 32, 16>("b16 W4  src512");
    check<4, 8, 32, 16>("f32 W8  src512");
    check<4, 4, 32, 16>("f32 W4  src512");
    check<8, 8, 32, 16>("f64 W8  src512");
    check<4, 16, 32, 32>("f32 W16 512x512");
    check<4, 8, 32, 32>("f32 W8  512x512");
    check<4, 4, 32, 32>("f32 W4  512x512");
    check<8, 16, 32, 32>("f64 W16 512x512");
    check<8, 8, 32, 32>("f64 W8  512x512");
    check<4, 16, 16, 64>("f32 W16 dst1024");
    check<4, 8, 16, 64>("f32 W8  dst1024");
    check<4, 4, 16, 64>("f32 W4  dst1024");
    check<8, 16, 16, 64>("f64 W16 dst1024");
    check<8, 8, 16, 64>("f64 W8  dst1024");
    std::printf("%s\n", failures ? "FAILED" : "all tile maps ok");
    return failures ? 1 : 0;
}
