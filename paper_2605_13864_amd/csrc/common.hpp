// Internal helpers shared by the HIP translation units of libxtr.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <mutex>

#include "../../include/xtr.h"

namespace xtr {

// ------------------------------------------------------------------ errors
// Thread-local message for the last nonzero return (xtr_last_error).
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);          // set_error + return code
int hip_fail(hipError_t e, const char *what);      // XTR_EHIP with HIP's message

#define XTR_HIP(call)                                           \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return ::xtr::hip_fail(e_, #call); \
    } while (0)

inline int elem_bytes(int dtype) {
    switch (dtype) {
    case XTR_F32: case XTR_I32: return 4;
    case XTR_F16: case XTR_BF16: case XTR_U16: return 2;
    case XTR_F8E4M3: case XTR_U8: return 1;
    case XTR_I64: case XTR_F64: return 8;
    default: return 0;
    }
}

inline bool is_float_sum_dtype(int d) {
    return d == XTR_F32 || d == XTR_F16 || d == XTR_BF16 || d == XTR_F8E4M3;
}
inline bool is_int_sum_dtype(int d) { return d == XTR_I32 || d == XTR_I64; }

// ------------------------------------------------------------------ workspace
// Library-owned device workspace, one buffer per (kind, device, stream).
//   WS_REDUCE: zero-filled when (re)allocated; the reduction kernels leave it
//              zeroed again when they finish (counters, partials).
//   WS_TABLE:  job/descriptor tables uploaded by the batched entry points.
// Returns XTR_OK and sets *ptr, or an error code.  Growing a buffer retires
// the old one without freeing it (enqueued work or a captured graph may still
// use it); retired buffers are freed by xtr_release.
//   WS_SCAN:   tile sums / offsets of the prefix sums (written before read).
//   WS_HIST:   per-workgroup partial histograms (written before read).
//   WS_MM:     the transposed B operand of a matrix product (written before read).
enum { WS_REDUCE = 0, WS_TABLE = 1, WS_SCAN = 2, WS_HIST = 3, WS_MM = 4, WS_KINDS = 5 };
int workspace(int kind, hipStream_t stream, size_t bytes, void **ptr, size_t *actual = nullptr);

// Asynchronous host -> device copy of `bytes` from pageable `host` memory:
// the bytes are first copied into a ring of pinned staging buffers owned by
// the library (so the caller may reuse `host` at once and the copy does not
// block on earlier work in the stream), then copied with hipMemcpyAsync.
int upload(const void *host, size_t bytes, void *dev, hipStream_t stream);

// Zero-fill `bytes` (multiple of 4) at device pointer p on stream (a fill
// kernel, not a memset node, so the sequence is safe to capture in graphs).
int zero_fill(void *p, size_t bytes, hipStream_t stream);

// Number of compute units of the current device (cached).
int cu_count();

// A second stream of default priority on the current device, owned by the
// library (created on first use, kept until the process ends), for work that one
// call splits over two streams: fork(st) makes the side stream wait for
// everything enqueued on st so far, join(st) makes st wait for everything
// enqueued on the side stream so far.  The pattern is capturable in a graph
// (the side stream joins the capture through the fork event).  A mutex held
// from fork to join keeps concurrent callers' forks and joins apart.
struct SideStream {
    std::mutex mu;
    int device = 0;
    hipStream_t s = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
};
int side_stream(SideStream **side);
int side_fork(SideStream *side, hipStream_t st);
int side_join(SideStream *side, hipStream_t st);

// ------------------------------------------------------------------ host buffers
// Resources of the entry points that take host buffers, one set per device
// (created on first use, kept until xtr_release): copies in, kernels and
// copies out run on three streams of default priority, so the copy of one
// panel overlaps the kernel of the previous one and the copy out of the one
// before.  Panels are double-buffered: slot b = panel index % 2.  A call holds
// `mu` from start to end (the calls are synchronous).
struct HostPipe {
    std::mutex mu;
    int device = 0;
    hipStream_t in = nullptr, comp = nullptr, out = nullptr;
    hipEvent_t in_done[2] = {}, k_done[2] = {}, out_done[2] = {};
    void *dev[4] = {};         // device panels: 0/1 input, 2/3 output
    size_t dev_bytes[4] = {};
    void *pin[4] = {};         // pinned staging for pageable host buffers: 0/1 in, 2/3 out
    size_t pin_bytes[4] = {};
};
// The current device's pipe (created on first use).
int host_pipe(HostPipe **pipe);
// Device panel / pinned staging buffer i of at least `bytes` (grown as needed;
// the caller has synchronized every stream of the pipe that used it).
int pipe_dev(HostPipe *p, int i, size_t bytes, void **ptr);
int pipe_pin(HostPipe *p, int i, size_t bytes, void **ptr);
// Whether host pointer p lies in page-locked memory the GPU can reach by DMA.
bool host_pinned(const void *p);
// Waits for every stream of the pipe.
int pipe_sync(HostPipe *p);

// Workgroups of `kernel` (block_threads threads, static LDS only) that are
// resident on the current device at once: the occupancy per CU (at most
// cap_per_cu when > 0) times the CU count.  A persistent grid of exactly this
// size has no workgroup that starts only after others finish.  Cached.
int resident_blocks(const void *kernel, int block_threads, int cap_per_cu = 0);

}  // namespace xtr
