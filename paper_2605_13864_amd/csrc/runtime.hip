// Runtime support of libxtr.so: error strings, the per-(device, stream)
// workspace pool, the zero-fill kernel and the small informational entry
// points of the C ABI.
#include "common.hpp"

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <mutex>
#include <utility>
#include <vector>

namespace xtr {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return XTR_EHIP;
}

// ------------------------------------------------------------------ zero fill

__global__ void __launch_bounds__(256) k_zero_fill(uint32_t *p, size_t words) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    size_t stride = (size_t)gridDim.x * 256;
    for (; i < words; i += stride) p[i] = 0u;
}

int zero_fill(void *p, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return XTR_OK;
    size_t words = (bytes + 3) / 4;
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_fill, dim3((unsigned)blocks), dim3(256), 0, stream,
                       (uint32_t *)p, words);
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

// ------------------------------------------------------------------ plain copy
// Streaming device-to-device copy: 16-byte vectors, 4 per thread in flight,
// grid-stride.  It is the reference kernel for the achievable HBM bandwidth
// and for scaling the HBM byte counters (FETCH_SIZE / WRITE_SIZE).

// One 16 KiB chunk per workgroup (4 vectors per thread, all in flight),
// streaming loads and stores: the fastest plain copy shape measured on gfx950.
typedef uint32_t cu32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy16(const cu32x4 *__restrict__ src,
                                                cu32x4 *__restrict__ dst, size_t nvec) {
    const size_t base = (size_t)blockIdx.x * 256 * 4 + threadIdx.x;
    cu32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const size_t i = base + (size_t)k * 256;
        if (i < nvec) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const size_t i = base + (size_t)k * 256;
        if (i < nvec) __builtin_nontemporal_store(v[k], dst + i);
    }
}

__global__ void __launch_bounds__(256) k_copy1(const unsigned char *__restrict__ src,
                                               unsigned char *__restrict__ dst, size_t n) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------ workspace

namespace {
struct Buf {
    void *ptr = nullptr;
    size_t bytes = 0;
};
struct Key {
    int kind, dev;
    hipStream_t stream;
    bool operator<(const Key &o) const {
        if (kind != o.kind) return kind < o.kind;
        if (dev != o.dev) return dev < o.dev;
        return (uintptr_t)stream < (uintptr_t)o.stream;
    }
};
std::mutex g_mu;
std::map<Key, Buf> g_ws;
// Buffers replaced by a larger one.  They are kept until xtr_release: a graph
// captured while one of them was current still holds its address.
struct Retired {
    int dev;
    void *ptr;
};
std::vector<Retired> g_retired;

// pinned host staging ring for upload(): RING slots per (device, stream), each
// guarded by the event recorded after the copy that last read it
constexpr int RING = 8;
struct Stage {
    void *host[RING] = {};
    size_t bytes[RING] = {};
    hipEvent_t done[RING] = {};
    int next = 0;
};
std::map<Key, Stage> g_stage;
}  // namespace

int workspace(int kind, hipStream_t stream, size_t bytes, void **ptr, size_t *actual) {
    int dev = 0;
    XTR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    Buf &b = g_ws[Key{kind, dev, stream}];
    if (b.bytes >= bytes && b.ptr) {
        *ptr = b.ptr;
        if (actual) *actual = b.bytes;
        return XTR_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    XTR_HIP(hipStreamIsCapturing(stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
        return fail(XTR_ENOMEM, "workspace must grow to %zu bytes while the stream is being "
                    "captured; use the *_ws entry points with a caller-owned workspace", bytes);
    if (b.ptr) {
        // The old buffer may be in use by queued work, or be held by a graph
        // captured earlier: it is retired, not freed, until xtr_release.
        g_retired.push_back(Retired{dev, b.ptr});
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes + bytes / 4;   // headroom
    want = (want + 255) & ~size_t(255);
    hipError_t e = hipMalloc(&b.ptr, want);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return fail(XTR_ENOMEM, "hipMalloc(%zu) for workspace: %s", want, hipGetErrorString(e));
    }
    b.bytes = want;
    if (kind == WS_REDUCE) {
        int rc = zero_fill(b.ptr, want, stream);
        if (rc) return rc;
    }
    *ptr = b.ptr;
    if (actual) *actual = b.bytes;
    return XTR_OK;
}

int upload(const void *host, size_t bytes, void *dev_dst, hipStream_t stream) {
    if (!bytes) return XTR_OK;
    int dev = 0;
    XTR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    Stage &st = g_stage[Key{0, dev, stream}];
    const int slot = st.next;
    st.next = (st.next + 1) % RING;
    if (st.done[slot]) XTR_HIP(hipEventSynchronize(st.done[slot]));   // previous reader finished
    else XTR_HIP(hipEventCreateWithFlags(&st.done[slot], hipEventDisableTiming));
    if (st.bytes[slot] < bytes) {
        if (st.host[slot]) XTR_HIP(hipHostFree(st.host[slot]));
        st.host[slot] = nullptr;
        size_t want = bytes < 65536 ? 65536 : bytes * 2;
        hipError_t e = hipHostMalloc(&st.host[slot], want, hipHostMallocDefault);
        if (e != hipSuccess) {
            st.host[slot] = nullptr;
            st.bytes[slot] = 0;
            return fail(XTR_ENOMEM, "hipHostMalloc(%zu) for staging: %s", want,
                        hipGetErrorString(e));
        }
        st.bytes[slot] = want;
    }
    memcpy(st.host[slot], host, bytes);
    XTR_HIP(hipMemcpyAsync(dev_dst, st.host[slot], bytes, hipMemcpyHostToDevice, stream));
    XTR_HIP(hipEventRecord(st.done[slot], stream));
    return XTR_OK;
}

namespace {
std::mutex g_side_mu;
std::map<int, SideStream *> g_side;   // by device; never moved once created
}  // namespace

int side_stream(SideStream **side) {
    int dev = 0;
    XTR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_side_mu);
    SideStream *&p = g_side[dev];
    if (!p) {
        SideStream *q = new (std::nothrow) SideStream();
        if (!q) return fail(XTR_ENOMEM, "side stream: out of host memory");
        q->device = dev;
        hipError_t e = hipStreamCreateWithFlags(&q->s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&q->fork_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&q->join_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (q->s) (void)hipStreamDestroy(q->s);
            if (q->fork_ev) (void)hipEventDestroy(q->fork_ev);
            delete q;
            return hip_fail(e, "side stream");
        }
        p = q;
    }
    *side = p;
    return XTR_OK;
}

int side_fork(SideStream *side, hipStream_t st) {
    XTR_HIP(hipEventRecord(side->fork_ev, st));
    XTR_HIP(hipStreamWaitEvent(side->s, side->fork_ev, 0));
    return XTR_OK;
}

int side_join(SideStream *side, hipStream_t st) {
    XTR_HIP(hipEventRecord(side->join_ev, side->s));
    XTR_HIP(hipStreamWaitEvent(st, side->join_ev, 0));
    return XTR_OK;
}

int cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

// ------------------------------------------------------------------ host buffers

namespace {
std::mutex g_pipe_mu;
std::map<int, HostPipe *> g_pipes;   // by device; never moved once created
}  // namespace

int host_pipe(HostPipe **pipe) {
    int dev = 0;
    XTR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_pipe_mu);
    HostPipe *&p = g_pipes[dev];
    if (!p) {
        HostPipe *q = new (std::nothrow) HostPipe();
        if (!q) return fail(XTR_ENOMEM, "host buffers: out of host memory");
        q->device = dev;
        hipError_t e = hipStreamCreateWithFlags(&q->in, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->comp, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->out, hipStreamNonBlocking);
        for (int b = 0; b < 2 && e == hipSuccess; b++) {
            e = hipEventCreateWithFlags(&q->in_done[b], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&q->k_done[b], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&q->out_done[b], hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            delete q;   // streams / events already made are reclaimed at exit
            return hip_fail(e, "host buffers: stream or event creation");
        }
        p = q;
    }
    *pipe = p;
    return XTR_OK;
}

int pipe_dev(HostPipe *p, int i, size_t bytes, void **ptr) {
    if (p->dev_bytes[i] < bytes) {
        if (p->dev[i]) XTR_HIP(hipFree(p->dev[i]));
        p->dev[i] = nullptr;
        p->dev_bytes[i] = 0;
        const size_t want = (bytes + 255) & ~size_t(255);
        hipError_t e = hipMalloc(&p->dev[i], want);
        if (e != hipSuccess) {
            p->dev[i] = nullptr;
            return fail(XTR_ENOMEM, "hipMalloc(%zu) for a host-buffer panel: %s", want,
                        hipGetErrorString(e));
        }
        p->dev_bytes[i] = want;
    }
    *ptr = p->dev[i];
    return XTR_OK;
}

int pipe_pin(HostPipe *p, int i, size_t bytes, void **ptr) {
    if (p->pin_bytes[i] < bytes) {
        if (p->pin[i]) XTR_HIP(hipHostFree(p->pin[i]));
        p->pin[i] = nullptr;
        p->pin_bytes[i] = 0;
        hipError_t e = hipHostMalloc(&p->pin[i], bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            p->pin[i] = nullptr;
            return fail(XTR_ENOMEM, "hipHostMalloc(%zu) for host-buffer staging: %s", bytes,
                        hipGetErrorString(e));
        }
        p->pin_bytes[i] = bytes;
    }
    *ptr = p->pin[i];
    return XTR_OK;
}

bool host_pinned(const void *ptr) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();   // pageable memory is not an error here
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

int pipe_sync(HostPipe *p) {
    XTR_HIP(hipStreamSynchronize(p->in));
    XTR_HIP(hipStreamSynchronize(p->comp));
    XTR_HIP(hipStreamSynchronize(p->out));
    return XTR_OK;
}

int resident_blocks(const void *kernel, int block_threads, int cap_per_cu) {
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int> cache;   // (kernel, device) -> per CU
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find({kernel, dev});
        if (it != cache.end()) per_cu = it->second;
    }
    if (per_cu == 0) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block_threads, 0) != hipSuccess ||
            n <= 0)
            n = 1;
        per_cu = n;
        std::lock_guard<std::mutex> lk(mu);
        cache[{kernel, dev}] = per_cu;
    }
    if (cap_per_cu > 0 && per_cu > cap_per_cu) per_cu = cap_per_cu;
    return per_cu * cu_count();
}

}  // namespace xtr

extern "C" {

int xtr_copy(void *dst, const void *src, size_t nbytes, void *stream) {
    if (nbytes == 0) return XTR_OK;
    if (!dst || !src) return xtr::fail(XTR_EINVAL, "xtr_copy: null pointer");
    const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
    if (s0 < d0 + nbytes && d0 < s0 + nbytes) return xtr::fail(XTR_EOVERLAP, "xtr_copy: overlap");
    hipStream_t st = (hipStream_t)stream;
    if (((s0 | d0 | nbytes) & 15) == 0) {
        const size_t nvec = nbytes / 16;
        const size_t blocks = (nvec + 1023) / 1024;
        if (blocks > 0xffffffffull) return xtr::fail(XTR_EINVAL, "xtr_copy: too large");
        hipLaunchKernelGGL(xtr::k_copy16, dim3((unsigned)blocks), dim3(256), 0, st,
                           (const xtr::cu32x4 *)src, (xtr::cu32x4 *)dst, nvec);
    } else {
        hipLaunchKernelGGL(xtr::k_copy1, dim3((unsigned)((nbytes + 255) / 256)), dim3(256), 0, st,
                           (const unsigned char *)src, (unsigned char *)dst, nbytes);
    }
    XTR_HIP(hipGetLastError());
    return XTR_OK;
}

const char *xtr_last_error(void) { return xtr::g_err; }

int xtr_elem_bytes(int dtype) { return xtr::elem_bytes(dtype); }

int xtr_version(void) { return (0 << 16) | 2; }

int xtr_release(void) {
    std::lock_guard<std::mutex> lk(xtr::g_mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) cur = 0;
    for (auto &kv : xtr::g_ws) {
        if (kv.second.ptr) {
            (void)hipSetDevice(kv.first.dev);
            (void)hipFree(kv.second.ptr);
        }
    }
    xtr::g_ws.clear();
    for (const auto &r : xtr::g_retired) {
        (void)hipSetDevice(r.dev);
        (void)hipFree(r.ptr);
    }
    xtr::g_retired.clear();
    for (auto &kv : xtr::g_stage) {
        (void)hipSetDevice(kv.first.dev);
        for (int i = 0; i < xtr::RING; i++) {
            if (kv.second.done[i]) {
                (void)hipEventSynchronize(kv.second.done[i]);
                (void)hipEventDestroy(kv.second.done[i]);
            }
            if (kv.second.host[i]) (void)hipHostFree(kv.second.host[i]);
        }
    }
    xtr::g_stage.clear();
    {
        std::lock_guard<std::mutex> pk(xtr::g_pipe_mu);
        for (auto &kv : xtr::g_pipes) {
            xtr::HostPipe *p = kv.second;
            std::lock_guard<std::mutex> pl(p->mu);
            (void)hipSetDevice(p->device);
            (void)xtr::pipe_sync(p);
            for (int i = 0; i < 4; i++) {
                if (p->dev[i]) (void)hipFree(p->dev[i]);
                if (p->pin[i]) (void)hipHostFree(p->pin[i]);
                p->dev[i] = p->pin[i] = nullptr;
                p->dev_bytes[i] = p->pin_bytes[i] = 0;
            }
        }
        // streams and events stay (a pipe may be in use again); buffers regrow
    }
    (void)hipSetDevice(cur);
    return XTR_OK;
}

}  // extern "C"
