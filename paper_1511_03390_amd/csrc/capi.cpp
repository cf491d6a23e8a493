// Diagnostics, validation and library-owned scratch for libqld.
#include <cstdarg>
#include <map>
#include <mutex>
#include <utility>

#include "qld_internal.hpp"

namespace qld {

static thread_local char g_err[512];
static thread_local hipEvent_t g_t0 = nullptr, g_t1 = nullptr;

void take_kernel_timer(hipEvent_t *start, hipEvent_t *stop) {
    *start = g_t0;
    *stop = g_t1;
    g_t0 = g_t1 = nullptr;
}

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

qld_status check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return QLD_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? QLD_E_NOMEM : QLD_E_DEVICE;
}

namespace {
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
std::mutex g_cu_mu;
std::map<int, int> g_cus;
}  // namespace

void *stream_workspace(hipStream_t stream, size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[{dev, stream}];
    if (w.bytes >= bytes && w.ptr) return w.ptr;
    if (w.ptr) {
        // Work already enqueued on this stream may still read the old buffer.
        if (hipStreamSynchronize(stream) != hipSuccess || hipFree(w.ptr) != hipSuccess) {
            set_error("releasing the old workspace failed");
            w.ptr = nullptr;
            w.bytes = 0;
            return nullptr;
        }
        w.ptr = nullptr;
        w.bytes = 0;
    }
    size_t want = bytes + bytes / 2 + 4096;
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        set_error("workspace allocation of %zu bytes failed", want);
        return nullptr;
    }
    w.ptr = p;
    w.bytes = want;
    return p;
}

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(g_cu_mu);
    auto it = g_cus.find(dev);
    if (it != g_cus.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        n = 256;
    g_cus[dev] = n;
    return n;
}

qld_status check_desc(const qld_frame_desc *d, int *elem_bytes) {
    if (!d) {
        set_error("frame descriptor is NULL");
        return QLD_E_INVAL;
    }
    int eb;
    if (d->dtype == QLD_U8) eb = 1;
    else if (d->dtype == QLD_U16) eb = 2;
    else {
        set_error("dtype %d is neither QLD_U8 nor QLD_U16", (int)d->dtype);
        return QLD_E_DTYPE;
    }
    if (d->bits < 1 || d->bits > 8 * eb) {
        set_error("bits=%d outside 1..%d for this dtype", d->bits, 8 * eb);
        return QLD_E_DTYPE;
    }
    if (d->H < 0 || d->W < 0) {
        set_error("negative frame size %dx%d", d->H, d->W);
        return QLD_E_SHAPE;
    }
    if (d->H > 0 && d->W > 0) {
        if (d->row_pitch < d->W) {
            set_error("row_pitch %lld < W %d", (long long)d->row_pitch, d->W);
            return QLD_E_SHAPE;
        }
        int64_t span = (int64_t)(d->H - 1) * d->row_pitch + d->W;
        if (d->frame_stride < span) {
            set_error("frame_stride %lld < frame extent %lld", (long long)d->frame_stride, (long long)span);
            return QLD_E_SHAPE;
        }
    }
    if (elem_bytes) *elem_bytes = eb;
    return QLD_OK;
}

}  // namespace qld

extern "C" {

const char *qld_status_str(qld_status st) {
    switch (st) {
        case QLD_OK: return "QLD_OK";
        case QLD_E_INVAL: return "QLD_E_INVAL: invalid argument";
        case QLD_E_DTYPE: return "QLD_E_DTYPE: unsupported sample format";
        case QLD_E_SHAPE: return "QLD_E_SHAPE: inconsistent shape or strides";
        case QLD_E_ALIGN: return "QLD_E_ALIGN: misaligned buffer";
        case QLD_E_OVERFLOW: return "QLD_E_OVERFLOW: int32 accumulators could overflow";
        case QLD_E_NOMEM: return "QLD_E_NOMEM: allocation failed";
        case QLD_E_BUDGET: return "QLD_E_BUDGET: exceeds the HBM budget";
        case QLD_E_AGAIN: return "QLD_E_AGAIN: not now, retry later";
        case QLD_E_STATE: return "QLD_E_STATE: invalid in the current state";
        case QLD_E_GAP: return "QLD_E_GAP: frame index gap, window reset";
        case QLD_E_DEVICE: return "QLD_E_DEVICE: HIP runtime or kernel failure";
        case QLD_E_IO: return "QLD_E_IO: file error";
    }
    return "unknown qld_status";
}

const char *qld_last_error(void) { return qld::g_err; }

qld_status qld_time_next_kernel(void *start_event, void *stop_event) {
    qld::g_t0 = static_cast<hipEvent_t>(start_event);
    qld::g_t1 = static_cast<hipEvent_t>(stop_event);
    if ((start_event == nullptr) != (stop_event == nullptr)) {
        qld::g_t0 = qld::g_t1 = nullptr;
        qld::set_error("start and stop events must be both set or both NULL");
        return QLD_E_INVAL;
    }
    return QLD_OK;
}

int64_t qld_frame_stride_hint(int32_t H, int32_t W, int64_t row_pitch, qld_dtype dtype) {
    const int64_t eb = dtype == QLD_U16 ? 2 : (dtype == QLD_U8 ? 1 : 0);
    if (eb == 0 || H < 0 || W < 0 || row_pitch < W) return 0;
    int64_t bytes = (int64_t)H * row_pitch * eb;
    bytes = (bytes + 255) / 256 * 256;
    // Frames whose size is a multiple of 64 KiB put the same pixel of
    // consecutive frames on the same HBM bank; a gap moves them apart: 4 KiB
    // for frames of 2 MiB and more, 256 bytes below that (measured best).
    if (bytes > 0 && bytes % 65536 == 0) bytes += bytes >= (2 << 20) ? 4096 : 256;
    return bytes / eb;
}

const char *qld_version(void) {
    return "libqld 0.1 (HIP, gfx950, " __VERSION__ ")";
}

}  // extern "C"
