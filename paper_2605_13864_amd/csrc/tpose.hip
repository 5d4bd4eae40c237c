// Out-of-place transpose for gfx950 (single, batched and host-buffer forms).
//
// What is computed: the sequential transpose of Listing 3.5,
//     dst[c*ld_dst + r] = src[r*ld_src + c],  0 <= r < rows, 0 <= c < cols,
// as a copy of element bits.
//
// How (tiled form of Listings 3.8 / 3.10): one workgroup of 256 threads moves
// one TR x TC tile.  Phase 1 loads the tile from HBM in W-byte pieces (W = 16,
// 8 or 4: the widest piece that divides both pointers and both row pitches),
// 256 / W lanes per 256-byte row segment so that every wave-level load covers
// whole cache lines, and writes the pieces to LDS.  A block barrier then hands
// ownership of the LDS tile from the loading threads to the storing threads:
// Section 3.3 places the barrier exactly where tile ownership changes.  Phase 2
// gives lane k of a dst row segment the piece k of that segment: it reads the
// tile rows its piece covers from LDS with 16-byte reads, transposes them in
// registers, and stores consecutive pieces across consecutive lanes.
//
// Differences from the paper's kernels (Listings 3.6 and 6.21), made for CDNA4:
//  - the tile is 256 x 256 BYTES whatever the element size (fp32 64 x 64,
//    bf16 128 x 128, fp8 256 x 256, fp64 32 x 32), or 512-byte row segments on
//    one side (tuned), so both HBM sides move whole cache lines;
//  - each lane moves W-byte pieces and transposes in registers (the paper's
//    kernel moves 2 elements per thread, Section 7.2);
//  - LDS 16-byte chunks are XOR-swizzled per row so that both the row writes
//    and the transposed reads hit distinct bank groups (the paper's 32 x 32
//    tile is unpadded);
//  - tile coordinates come from one division per tile, not per element (the
//    paper attributes its transpose gap to per-thread index arithmetic,
//    Section 7.2 / Chapter 6);
//  - the launch order is XCD-aware and banded, so tiles that share cache lines
//    at their edges meet in one L2.
// Tiles on the right or bottom edge mask whole pieces (elements only where an
// edge cuts a piece).  1- and 2-byte matrices whose rows are not 4-byte
// aligned (odd pitches or offsets) move 4-byte pieces too: each is built from
// aligned dwords by a funnel shift with the neighbouring lane's, over the
// same LDS layout.
#include "tpose_dev.hpp"

#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

namespace xtr {
using namespace tpk;

// Tuned launch configuration per shape class and element size (slot
// cfg_slot(elem bytes)).  wide_min as measured on rotating buffers: 2-byte
// elements keep wide tiles from 8 default tiles per CU (bf16 8192 x 8192 runs
// 2% faster in them), 4- and 8-byte ones from 32 (fp32 4096 x 4096: 15% faster
// in default tiles).
xtr_tpose_config tpk::g_cfg[2][4] = {
    {{1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 32}, {1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 8},
     {1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 32}, {1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 32}},
    {{1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 32}, {1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 8},
     {1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 32}, {1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 32}},
};

namespace {

int check_one(const void *src, const void *dst, int64_t rows, int64_t cols, int64_t ld_src,
              int64_t ld_dst, int dtype, const char *who) {
    const int eb = elem_bytes(dtype);
    if (!eb) return fail(XTR_EDTYPE, "%s: unknown dtype %d", who, dtype);
    if (rows < 0 || cols < 0) return fail(XTR_EINVAL, "%s: negative size %lld x %lld", who,
                                          (long long)rows, (long long)cols);
    if (rows == 0 || cols == 0) return XTR_OK;
    if (!src || !dst) return fail(XTR_EINVAL, "%s: null pointer", who);
    if (ld_src < cols || ld_dst < rows)
        return fail(XTR_EINVAL, "%s: ld_src=%lld < cols=%lld or ld_dst=%lld < rows=%lld", who,
                    (long long)ld_src, (long long)cols, (long long)ld_dst, (long long)rows);
    if (((uintptr_t)src | (uintptr_t)dst) % eb)
        return fail(XTR_EALIGN, "%s: pointer not aligned to the %d-byte element", who, eb);
    // byte extents of the two operands
    const uintptr_t s0 = (uintptr_t)src, s1 = s0 + ((rows - 1) * ld_src + cols) * eb;
    const uintptr_t d0 = (uintptr_t)dst, d1 = d0 + ((cols - 1) * ld_dst + rows) * eb;
    if (s0 < d1 && d0 < s1) return fail(XTR_EOVERLAP, "%s: src and dst overlap", who);
    return XTR_OK;
}

}  // namespace

int tpose_impl(const void *src, void *dst, int64_t rows, int64_t cols, int64_t ld_src,
               int64_t ld_dst, int dtype, hipStream_t stream) {
    int rc = check_one(src, dst, rows, cols, ld_src, ld_dst, dtype, "tpose");
    if (rc || rows == 0 || cols == 0) return rc;
    switch (elem_bytes(dtype)) {
    case 1: return launch_single_e1(src, dst, rows, cols, ld_src, ld_dst, stream);
    case 2: return launch_single_e2(src, dst, rows, cols, ld_src, ld_dst, stream);
    case 4: return launch_single_e4(src, dst, rows, cols, ld_src, ld_dst, stream);
    default: return launch_single_e8(src, dst, rows, cols, ld_src, ld_dst, stream);
    }
}

// ---------------------------------------------------------------- host buffers

// Row panels of the host-buffer transpose hold about this many bytes.
constexpr size_t HOST_PANEL_BYTES = size_t(32) << 20;

// Transposes host src into host dst through the device, one row panel at a
// time: the copy in of panel k+1, the transpose of panel k and the copy out
// of panel k-1 overlap on the pipe's three streams.  A src row panel
// [r0, r0 + R) becomes the dst column panel [r0, r0 + R): a strided copy out.
// Page-locked host buffers are copied by DMA directly; pageable ones pass
// through the pipe's pinned staging (a host memcpy per panel).
int tpose_host_impl(const void *src, void *dst, int64_t rows, int64_t cols, int64_t ld_src,
                    int64_t ld_dst, int dtype) {
    const char *who = "xtr_tpose_host";
    int rc = check_one(src, dst, rows, cols, ld_src, ld_dst, dtype, who);
    if (rc || rows == 0 || cols == 0) return rc;
    const int64_t eb = elem_bytes(dtype);
    HostPipe *p = nullptr;
    rc = host_pipe(&p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(p->mu);
    if ((rc = pipe_sync(p))) return rc;   // a failed earlier call may have left work queued
    const bool spin = host_pinned(src), dpin = host_pinned(dst);
    const int64_t tr = 256 / eb;                       // tile rows of the default geometry
    int64_t R = (int64_t)(HOST_PANEL_BYTES / (size_t)(cols * eb));
    R = R < tr ? tr : R / tr * tr;
    if (R > rows) R = rows;
    const size_t pbytes = (size_t)(R * cols * eb);
    void *din[2], *dout[2], *sin[2] = {nullptr, nullptr}, *sout[2] = {nullptr, nullptr};
    for (int b = 0; b < 2; b++) {
        if ((rc = pipe_dev(p, b, pbytes, &din[b]))) return rc;
        if ((rc = pipe_dev(p, 2 + b, pbytes, &dout[b]))) return rc;
        if (!spin && (rc = pipe_pin(p, b, pbytes, &sin[b]))) return rc;
        if (!dpin && (rc = pipe_pin(p, 2 + b, pbytes, &sout[b]))) return rc;
    }
    const unsigned char *hs = static_cast<const unsigned char *>(src);
    unsigned char *hd = static_cast<unsigned char *>(dst);
    auto scatter = [&](int64_t k) {   // pageable dst: staged panel k -> its dst columns
        const int b = (int)(k & 1);
        const int64_t r0 = k * R, Rk = (rows - r0) < R ? (rows - r0) : R;
        const unsigned char *st = static_cast<const unsigned char *>(sout[b]);
        for (int64_t c = 0; c < cols; c++)
            memcpy(hd + (c * ld_dst + r0) * eb, st + c * Rk * eb, (size_t)(Rk * eb));
    };
    const int64_t np = (rows + R - 1) / R;
    for (int64_t k = 0; k < np; k++) {
        const int b = (int)(k & 1);
        const int64_t r0 = k * R, Rk = (rows - r0) < R ? (rows - r0) : R;
        // copy in (waits until the kernel of panel k-2 has read din[b])
        if (k >= 2) XTR_HIP(hipStreamWaitEvent(p->in, p->k_done[b], 0));
        if (spin) {
            XTR_HIP(hipMemcpy2DAsync(din[b], (size_t)(cols * eb), hs + r0 * ld_src * eb,
                                     (size_t)(ld_src * eb), (size_t)(cols * eb), (size_t)Rk,
                                     hipMemcpyHostToDevice, p->in));
        } else {
            if (k >= 2) XTR_HIP(hipEventSynchronize(p->in_done[b]));   // sin[b] is free again
            unsigned char *st = static_cast<unsigned char *>(sin[b]);
            if (ld_src == cols) {
                memcpy(st, hs + r0 * cols * eb, (size_t)(Rk * cols * eb));
            } else {
                for (int64_t r = 0; r < Rk; r++)
                    memcpy(st + r * cols * eb, hs + (r0 + r) * ld_src * eb, (size_t)(cols * eb));
            }
            XTR_HIP(hipMemcpyAsync(din[b], st, (size_t)(Rk * cols * eb), hipMemcpyHostToDevice,
                                   p->in));
        }
        XTR_HIP(hipEventRecord(p->in_done[b], p->in));
        // transpose (waits for its input, and for the copy out of panel k-2 from dout[b])
        XTR_HIP(hipStreamWaitEvent(p->comp, p->in_done[b], 0));
        if (k >= 2) XTR_HIP(hipStreamWaitEvent(p->comp, p->out_done[b], 0));
        rc = tpose_impl(din[b], dout[b], Rk, cols, cols, Rk, dtype, p->comp);
        if (rc) {
            (void)pipe_sync(p);
            return rc;
        }
        XTR_HIP(hipEventRecord(p->k_done[b], p->comp));
        // copy out
        XTR_HIP(hipStreamWaitEvent(p->out, p->k_done[b], 0));
        if (dpin) {
            XTR_HIP(hipMemcpy2DAsync(hd + r0 * eb, (size_t)(ld_dst * eb), dout[b], (size_t)(Rk * eb),
                                     (size_t)(Rk * eb), (size_t)cols, hipMemcpyDeviceToHost, p->out));
        } else {
            XTR_HIP(hipMemcpyAsync(sout[b], dout[b], (size_t)(cols * Rk * eb),
                                   hipMemcpyDeviceToHost, p->out));
        }
        XTR_HIP(hipEventRecord(p->out_done[b], p->out));
        if (!dpin && k >= 1) {   // the previous panel is staged: place it while this one runs
            XTR_HIP(hipEventSynchronize(p->out_done[(k - 1) & 1]));
            scatter(k - 1);
        }
    }
    if (!dpin) {
        XTR_HIP(hipEventSynchronize(p->out_done[(np - 1) & 1]));
        scatter(np - 1);
    }
    return pipe_sync(p);
}

// Host-side form of a batch: jobs grouped by (element size, piece width,
// 32-bit offsets); each group has its own slice of the device table, its own
// concatenated tile space and one persistent launch.
// eb slot x piece class (16, 8, 4, elem) x off32 x line-aligned rows x tile
// geometry (0: 256 x 256 bytes, 1: 512-byte src row segments, 2: 512-byte dst
// row segments, 3: both, 4: 1 KiB dst row segments)
constexpr int NGEO = 5;
constexpr int NGROUPS = 4 * 4 * 2 * 2 * NGEO;
// jobs of at least this many default tiles may take a wider geometry
constexpr int64_t WIDE_MIN_TILES = 16;
int wclass(int w) { return w == 16 ? 0 : w == 8 ? 1 : w == 4 ? 2 : 3; }
int wof(int wc) { return wc == 0 ? 16 : wc == 1 ? 8 : wc == 2 ? 4 : 0; }

// Slot counters of a group launch (order xcd = 3): one per XCD and an exit
// count, zero before every launch (uploaded as zeros; the last
// workgroup of a launch sets them back to zero).
constexpr int CTR_WORDS = 16;

struct BatchTable {
    std::vector<Job> all;                // groups concatenated
    std::vector<int64_t> bases;          // tile_base of every job of `all` (same order)
    size_t at[NGROUPS] = {};             // first job of each group in `all` / `bases`
    int nj[NGROUPS] = {};
    int64_t ntiles[NGROUPS] = {};
    // device image: the Job array, then (at a 256-byte boundary) `tail`: for
    // each non-empty group its bases, then its CTR_WORDS zero counter words
    std::vector<int64_t> tail;
    size_t tail_at[NGROUPS] = {};        // a group's bases in `tail`; counters follow
    size_t jobs_bytes() const { return (all.size() * sizeof(Job) + 255) / 256 * 256; }
    size_t bytes() const { return jobs_bytes() + tail.size() * sizeof(int64_t); }
};

int build_batch(const xtr_tpose_desc *descs, int64_t count, const char *who, BatchTable &bt) {
    if (count < 0) return fail(XTR_EINVAL, "%s: negative count", who);
    if (count > 0 && !descs) return fail(XTR_EINVAL, "%s: null descriptor array", who);
    if (count > 0x7fffffffLL) return fail(XTR_EINVAL, "%s: too many descriptors", who);
    for (int64_t i = 0; i < count; i++) {
        const xtr_tpose_desc &d = descs[i];
        int rc = check_one(d.src, d.dst, d.rows, d.cols, d.ld_src, d.ld_dst, d.dtype, who);
        if (rc) {
            set_error("%s: descriptor %lld: %s", who, (long long)i, xtr_last_error());
            return rc;
        }
    }
    std::vector<Job> groups[NGROUPS];
    for (int64_t i = 0; i < count; i++) {
        const xtr_tpose_desc &d = descs[i];
        if (d.rows == 0 || d.cols == 0) continue;
        const int eb = elem_bytes(d.dtype);
        Job j;
        j.src = (const unsigned char *)d.src;
        j.dst = (unsigned char *)d.dst;
        j.rows = d.rows; j.cols = d.cols; j.ld_src = d.ld_src; j.ld_dst = d.ld_dst;
        j.w = piece_width(d.src, d.dst, d.ld_src, d.ld_dst, eb);
        const xtr_tpose_config &cb = g_cfg[XTR_SHAPE_BATCHED][cfg_slot(eb)];
        if (cb.narrow && j.w > 4) j.w = eb >= 8 ? 8 : 4;   // one launch per element size
        j._pad = 0;
        const bool lines = lines_ok(d.src, d.ld_src, eb) && lines_ok(d.dst, d.ld_dst, eb);
        const xtr_tpose_config &c = g_cfg[XTR_SHAPE_BATCHED][cfg_slot(eb)];
        const int want = lines ? c.tile : c.tile_shared;
        const int geo = eb >= 2 && j.w >= 4 &&
                                (want == 1 || want == 2 || (want >= 3 && eb >= 4)) &&
                                tiles_for(eb, d.rows, d.cols, nullptr) >= WIDE_MIN_TILES &&
                                off32_geo(eb, want, d.ld_src, d.ld_dst)
                            ? want
                            : 0;
        const int g = (((cfg_slot(eb) * 4 + wclass(j.w)) * 2 +
                        (off32_rt(eb, d.ld_src, d.ld_dst) ? 1 : 0)) * 2 + (lines ? 1 : 0)) * NGEO +
                      geo;
        j.tile_base = bt.ntiles[g];
        bt.ntiles[g] += tiles_for(eb, d.rows, d.cols, &j.tiles_c, geo);
        groups[g].push_back(j);
    }
    for (int g = 0; g < NGROUPS; g++) {
        if (bt.ntiles[g] >= MAX_TILES)
            return fail(XTR_EINVAL, "%s: %lld tiles in one launch group (limit 2^31)", who,
                        (long long)bt.ntiles[g]);
        bt.at[g] = bt.all.size();
        bt.nj[g] = (int)groups[g].size();
        bt.all.insert(bt.all.end(), groups[g].begin(), groups[g].end());
    }
    bt.bases.resize(bt.all.size());
    for (size_t i = 0; i < bt.all.size(); i++) bt.bases[i] = bt.all[i].tile_base;
    for (int g = 0; g < NGROUPS; g++) {
        if (!bt.nj[g]) continue;
        bt.tail_at[g] = bt.tail.size();
        bt.tail.insert(bt.tail.end(), bt.bases.begin() + bt.at[g],
                       bt.bases.begin() + bt.at[g] + bt.nj[g]);
        bt.tail.insert(bt.tail.end(), CTR_WORDS / 2, 0);   // counters, 8-byte aligned
    }
    return XTR_OK;
}

// Copies the device image of bt (jobs, then bases and zero counters) to dev
// with upload().
int upload_batch(const BatchTable &bt, void *dev, hipStream_t stream) {
    int rc = upload(bt.all.data(), bt.all.size() * sizeof(Job), dev, stream);
    if (rc) return rc;
    return upload(bt.tail.data(), bt.tail.size() * sizeof(int64_t),
                  static_cast<unsigned char *>(dev) + bt.jobs_bytes(), stream);
}

// Every group has at most INLINE_JOBS jobs (the batch can run without a table).
bool batch_inline(const BatchTable &bt) {
    for (int g = 0; g < NGROUPS; g++)
        if (bt.nj[g] > INLINE_JOBS) return false;
    return true;
}

// One persistent launch per non-empty group; `dev` is the device image of bt,
// or nullptr when batch_inline(bt) (jobs in the kernel arguments).
int launch_batch(const BatchTable &bt, const void *dev, hipStream_t stream) {
    const Job *djobs = static_cast<const Job *>(dev);
    int64_t *dtail = dev ? reinterpret_cast<int64_t *>(
                               static_cast<unsigned char *>(const_cast<void *>(dev)) +
                               bt.jobs_bytes())
                         : nullptr;
    JobPack pack;
    for (int g = 0; g < NGROUPS; g++) {
        if (!bt.nj[g]) continue;
        const JobPack *pk = nullptr;
        if (!dev) {
            for (int i = 0; i < bt.nj[g]; i++) {
                pack.jobs[i] = bt.all[bt.at[g] + i];
                pack.bases[i] = bt.bases[bt.at[g] + i];
            }
            pk = &pack;
        }
        const int geo = g % NGEO, h = g / NGEO;
        const int slot = h / 16, w = wof((h / 4) % 4);
        const bool off32 = ((h / 2) & 1) != 0, lines = (h & 1) != 0;
        // at most the resident capacity of the group's kernel (clamped at launch)
        int64_t grid = bt.ntiles[g] < 0x7fffffff ? bt.ntiles[g] : 0x7fffffff;
        if (grid < 1) grid = 1;
        const Job *jobs = dev ? djobs + bt.at[g] : nullptr;
        const int64_t *bases = dev ? dtail + bt.tail_at[g] : nullptr;
        uint32_t *ctr = dev ? reinterpret_cast<uint32_t *>(dtail + bt.tail_at[g] + bt.nj[g])
                            : nullptr;
        const int64_t nt = bt.ntiles[g];
        const int nj = bt.nj[g];
        switch (slot) {
        case 0: launch_group_e1(w, off32, lines, geo, grid, stream, jobs, bases, nj, nt, pk, ctr); break;
        case 1: launch_group_e2(w, off32, lines, geo, grid, stream, jobs, bases, nj, nt, pk, ctr); break;
        case 2: launch_group_e4(w, off32, lines, geo, grid, stream, jobs, bases, nj, nt, pk, ctr); break;
        default: launch_group_e8(w, off32, lines, geo, grid, stream, jobs, bases, nj, nt, pk, ctr); break;
        }
        XTR_HIP(hipGetLastError());
    }
    return XTR_OK;
}

int tpose_batched_impl(const xtr_tpose_desc *descs, int64_t count, hipStream_t stream) {
    BatchTable bt;
    int rc = build_batch(descs, count, "tpose_batched", bt);
    if (rc || bt.all.empty()) return rc;
    if (batch_inline(bt)) return launch_batch(bt, nullptr, stream);
    void *wsp = nullptr;
    rc = workspace(WS_TABLE, stream, bt.bytes(), &wsp);
    if (rc) return rc;
    rc = upload_batch(bt, wsp, stream);
    if (rc) return rc;
    return launch_batch(bt, wsp, stream);
}

}  // namespace xtr

extern "C" {

int tpose(const void *src, void *dst, int64_t rows, int64_t cols, int64_t ld_src, int64_t ld_dst,
          int dtype, void *stream) {
    return xtr::tpose_impl(src, dst, rows, cols, ld_src, ld_dst, dtype, (hipStream_t)stream);
}

int tpose_batched(const xtr_tpose_desc *descs, int64_t count, void *stream) {
    return xtr::tpose_batched_impl(descs, count, (hipStream_t)stream);
}

int xtr_tpose_host(const void *src, void *dst, int64_t rows, int64_t cols, int64_t ld_src,
                   int64_t ld_dst, int dtype) {
    return xtr::tpose_host_impl(src, dst, rows, cols, ld_src, ld_dst, dtype);
}

struct xtr_tpose_plan {
    xtr::BatchTable bt;
    void *dev = nullptr;    // device image of bt
    int device = 0;
};

int xtr_tpose_plan_create(const xtr_tpose_desc *descs, int64_t count, void *stream,
                          xtr_tpose_plan **plan) {
    if (!plan) return xtr::fail(XTR_EINVAL, "xtr_tpose_plan_create: null plan");
    *plan = nullptr;
    auto *p = new (std::nothrow) xtr_tpose_plan();
    if (!p) return xtr::fail(XTR_ENOMEM, "xtr_tpose_plan_create: out of host memory");
    int rc = xtr::build_batch(descs, count, "xtr_tpose_plan_create", p->bt);
    if (!rc && hipGetDevice(&p->device) != hipSuccess) rc = xtr::fail(XTR_EHIP, "hipGetDevice");
    if (!rc && !p->bt.all.empty()) {
        const size_t bytes = p->bt.bytes();
        hipError_t e = hipMalloc(&p->dev, bytes);
        if (e != hipSuccess) {
            p->dev = nullptr;
            rc = xtr::fail(XTR_ENOMEM, "xtr_tpose_plan_create: hipMalloc(%zu): %s", bytes,
                           hipGetErrorString(e));
        } else {
            hipStream_t st = (hipStream_t)stream;
            e = hipMemcpyAsync(p->dev, p->bt.all.data(), p->bt.all.size() * sizeof(xtr::Job),
                               hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(static_cast<unsigned char *>(p->dev) + p->bt.jobs_bytes(),
                                   p->bt.tail.data(), p->bt.tail.size() * sizeof(int64_t),
                                   hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = xtr::hip_fail(e, "xtr_tpose_plan_create: table upload");
        }
    }
    if (rc) {
        if (p->dev) (void)hipFree(p->dev);
        delete p;
        return rc;
    }
    *plan = p;
    return XTR_OK;
}

int xtr_tpose_plan_run(const xtr_tpose_plan *plan, void *stream) {
    if (!plan) return xtr::fail(XTR_EINVAL, "xtr_tpose_plan_run: null plan");
    if (plan->bt.all.empty()) return XTR_OK;
    return xtr::launch_batch(plan->bt, plan->dev, (hipStream_t)stream);
}

int xtr_tpose_plan_destroy(xtr_tpose_plan *plan) {
    if (!plan) return XTR_OK;
    if (plan->dev) (void)hipFree(plan->dev);
    delete plan;
    return XTR_OK;
}

int xtr_tpose_get_class_config(int elem_bytes, int shape_class, xtr_tpose_config *cfg) {
    if (!cfg || (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) ||
        (shape_class != XTR_SHAPE_SINGLE && shape_class != XTR_SHAPE_BATCHED))
        return xtr::fail(XTR_EINVAL, "xtr_tpose_get_class_config: bad arguments");
    *cfg = xtr::g_cfg[shape_class][xtr::cfg_slot(elem_bytes)];
    return XTR_OK;
}

int xtr_tpose_set_class_config(int elem_bytes, int shape_class, const xtr_tpose_config *cfg) {
    if (!cfg || (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) ||
        (shape_class != XTR_SHAPE_SINGLE && shape_class != XTR_SHAPE_BATCHED))
        return xtr::fail(XTR_EINVAL, "xtr_tpose_set_class_config: bad arguments");
    if (cfg->xcd < 0 || cfg->xcd > 3 ||
        cfg->group < 1 || cfg->group > 64 || cfg->blocks_per_cu < 0 || cfg->blocks_per_cu > 64 ||
        cfg->tile < 0 || cfg->tile > 4 || cfg->tile_shared < 0 || cfg->tile_shared > 4 ||
        cfg->run < 0 || cfg->run > 64 || cfg->narrow < 0 || cfg->narrow > 1 ||
        cfg->wide_min < 0 || cfg->wide_min > 1024)
        return xtr::fail(XTR_EINVAL, "xtr_tpose_set_class_config: xcd in [0, 3], group in "
                                     "[1, 64], blocks_per_cu in [0, 64], tile and tile_shared in "
                                     "[0, 4], run in [0, 64], narrow in [0, 1], wide_min in "
                                     "[0, 1024]");
    xtr::g_cfg[shape_class][xtr::cfg_slot(elem_bytes)] = *cfg;
    return XTR_OK;
}

int xtr_tpose_get_config(int elem_bytes, xtr_tpose_config *cfg) {
    return xtr_tpose_get_class_config(elem_bytes, XTR_SHAPE_SINGLE, cfg);
}

int xtr_tpose_set_config(int elem_bytes, const xtr_tpose_config *cfg) {
    int rc = xtr_tpose_set_class_config(elem_bytes, XTR_SHAPE_SINGLE, cfg);
    if (rc == XTR_OK) rc = xtr_tpose_set_class_config(elem_bytes, XTR_SHAPE_BATCHED, cfg);
    return rc;
}

}  // extern "C"
