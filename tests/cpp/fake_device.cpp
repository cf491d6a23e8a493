// Host stand-ins for the device side of the serving runtime, so that
// server.cpp and capi.cpp run unchanged on a machine without a GPU, under the
// sanitizers.  TEST INFRASTRUCTURE ONLY.
//
// "Device" memory is host memory; every asynchronous HIP call completes before
// it returns, so an event is complete once recorded.  The batched window
// update is computed here on the host from its job table (the definition:
// after window cycle c, I/Q are the sums over the last min(c + 1, M) cycles of
// (S0 - S2, S1 - S3), kept with a ring of per-cycle differences), so the
// driver can check every image the server publishes.  LEARNED streams are not
// supported here (their calls fail).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <new>

#include "serve_learned.hpp"
#include "window.hpp"

struct ihipStream_t {
    unsigned flags;
};
struct ihipEvent_t {
    std::atomic<int> recorded{0};
};

hipError_t hipMalloc(void **p, size_t bytes) {
    *p = std::calloc(1, bytes ? bytes : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
    std::free(p);
    return hipSuccess;
}
namespace {
std::mutex g_host_mu;
std::map<uintptr_t, size_t> g_host;        // page-locked allocations: start -> bytes
thread_local hipError_t g_last = hipSuccess;
}  // namespace

hipError_t hipHostMalloc(void **p, size_t bytes, unsigned) {
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_host_mu);
        g_host[reinterpret_cast<uintptr_t>(*p)] = bytes;
    }
    return e;
}
hipError_t hipHostFree(void *p) {
    {
        std::lock_guard<std::mutex> lk(g_host_mu);
        g_host.erase(reinterpret_cast<uintptr_t>(p));
    }
    return hipFree(p);
}
hipError_t hipPointerGetAttributes(hipPointerAttribute_t *attr, const void *p) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    std::lock_guard<std::mutex> lk(g_host_mu);
    auto it = g_host.upper_bound(a);
    if (it != g_host.begin()) {
        --it;
        if (a < it->first + it->second) {
            *attr = hipPointerAttribute_t{};
            attr->type = hipMemoryTypeHost;
            attr->hostPointer = const_cast<void *>(p);
            return hipSuccess;
        }
    }
    g_last = hipErrorInvalidValue;
    return hipErrorInvalidValue;
}
hipError_t hipMemset(void *p, int v, size_t bytes) {
    std::memset(p, v, bytes);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t) {
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind, hipStream_t) {
    for (size_t r = 0; r < height; ++r)
        std::memcpy(static_cast<char *>(dst) + r * dpitch, static_cast<const char *>(src) + r * spitch, width);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
    *e = new (std::nothrow) ihipEvent_t();
    return *e ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    if (!e) return hipErrorInvalidValue;
    e->recorded.store(1);
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) { return e ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags) {
    *s = new (std::nothrow) ihipStream_t{flags};
    return *s ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) {
    return e && e->recorded.load() ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *dev) {
    *dev = 0;
    return hipSuccess;
}
hipError_t hipGetLastError() {
    const hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake device error"; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) {
    *v = 256;
    return hipSuccess;
}

namespace qld {

namespace {
int padded(int W, int eb) { return (W + window_vpx(eb) - 1) / window_vpx(eb) * window_vpx(eb); }
}  // namespace

size_t window_bytes(const qld_frame_desc *d, int32_t M, int32_t Ms) {
    int eb = 0;
    if (check_desc(d, &eb) != QLD_OK || M < 1) return 0;
    const size_t px = (size_t)d->H * padded(d->W, eb);
    return (size_t)M * px * 8 + px * 8 + (Ms > 0 ? px * 8 : 0);
}

// Ring of int32 (dI, dQ) pairs [M][H][Wp]; state [H][Wp].
qld_status window_alloc(const qld_frame_desc *d, int32_t M, int32_t Ms, qld_window **out) {
    int eb = 0;
    QLD_TRY(check_desc(d, &eb));
    auto *w = new (std::nothrow) qld_window();
    if (!w) return QLD_E_NOMEM;
    w->d = *d;
    w->eb = eb;
    w->M = M;
    w->Ms = Ms;
    w->wide = 1;
    w->Wp = padded(d->W, eb);
    const size_t px = (size_t)d->H * w->Wp;
    w->ring = std::calloc((size_t)M * px * 2 + 1, sizeof(int32_t));
    w->I = static_cast<int32_t *>(std::calloc(px * 4 + 1, sizeof(int32_t)));
    if (!w->ring || !w->I) {
        std::free(w->ring);
        std::free(w->I);
        delete w;
        return QLD_E_NOMEM;
    }
    w->Q = w->I + px;
    w->Is = w->I + 2 * px;
    w->Qs = w->I + 3 * px;
    *out = w;
    return QLD_OK;
}

hipError_t launch_window_batch(const WinBatch &b, int elem, bool, bool, hipStream_t) {
    for (int j = 0; j < b.n_jobs; ++j) {
        const WinJob &J = b.job[j];
        int32_t *ring = static_cast<int32_t *>(J.ring);
        const int64_t px = (int64_t)J.H * J.Wp;
        for (int k = 0; k < J.n_cycles; ++k) {
            const int64_t c = J.c0 + k;
            const uint8_t *slot = J.stage + (int64_t)((J.stage0 + k) % J.n_stage) * J.slot_b;
            if (k == 0 && J.fresh) {
                std::memset(J.I, 0, px * 4);
                std::memset(J.Q, 0, px * 4);
                if (J.Ms > 0) {
                    std::memset(J.Is, 0, px * 4);
                    std::memset(J.Qs, 0, px * 4);
                }
            }
            const int o = (J.out0 + k) % J.out_slots;
            for (int y = 0; y < J.H; ++y)
                for (int x = 0; x < J.W; ++x) {
                    int32_t s[4];
                    for (int f = 0; f < 4; ++f) {
                        const uint8_t *p = slot + f * J.fs_b + y * J.rp_b + (int64_t)x * elem;
                        uint16_t v16;
                        std::memcpy(&v16, p, sizeof v16);
                        s[f] = elem == 2 ? (int32_t)v16 : (int32_t)*p;
                    }
                    const int32_t di = s[0] - s[2], dq = s[1] - s[3];
                    const int64_t q = (int64_t)y * J.Wp + x;
                    int32_t *now = ring + 2 * ((c % J.M) * px + q);
                    if (c >= J.M) {
                        J.I[q] -= now[0];
                        J.Q[q] -= now[1];
                    }
                    if (J.Ms > 0 && c >= J.Ms) {
                        const int32_t *old = ring + 2 * (((c - J.Ms) % J.M) * px + q);
                        J.Is[q] -= old[0];
                        J.Qs[q] -= old[1];
                    }
                    now[0] = di;
                    now[1] = dq;
                    J.I[q] += di;
                    J.Q[q] += dq;
                    if (J.Ms > 0) {
                        J.Is[q] += di;
                        J.Qs[q] += dq;
                    }
                    const int64_t oo = (int64_t)o * J.H * J.W + (int64_t)y * J.W + x;
                    if (J.amp) {
                        const int64_t a = J.I[q], bq = J.Q[q];
                        J.amp[oo] = (float)std::sqrt((double)(uint64_t)(a * a + bq * bq));
                    }
                    if (J.Io) {
                        J.Io[oo] = J.I[q];
                        J.Qo[oo] = J.Q[q];
                    }
                    if (J.Iso) {
                        J.Iso[oo] = J.Is[q];
                        J.Qso[oo] = J.Qs[q];
                    }
                }
        }
    }
    return hipSuccess;
}

hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t) {
    std::memset(p, 0, n * 4);
    return hipSuccess;
}

hipError_t launch_cycle_sums(const uint8_t *, int64_t, int, int, int, int, uint64_t *, int, int64_t, int,
                             hipStream_t) {
    return hipErrorLaunchFailure;
}
hipError_t launch_window_sum(const uint64_t *, int, int, int64_t, int, uint64_t *, hipStream_t) {
    return hipErrorLaunchFailure;
}
hipError_t launch_pixel_cycle_sums(const uint8_t *, int64_t, int64_t, int64_t, int, int, int, int, int, int,
                                   uint32_t *, int, int64_t, hipStream_t) {
    return hipErrorLaunchFailure;
}
hipError_t launch_pixel_window_sum(const uint32_t *, int, int64_t, int64_t, int, uint32_t *, hipStream_t) {
    return hipErrorLaunchFailure;
}
hipError_t launch_serve(const float *, const float *, const float *, const float *, int64_t, float, float, float *,
                        float *, hipStream_t) {
    return hipErrorLaunchFailure;
}

}  // namespace qld

extern "C" {

qld_status qld_window_destroy(qld_window *w) {
    if (!w) return QLD_E_INVAL;
    std::free(w->ring);
    std::free(w->I);
    delete w;
    return QLD_OK;
}

qld_status qld_denoise_prepare(const int32_t *, const int32_t *, const uint32_t *, const uint64_t *, int32_t, int32_t,
                               int32_t, int32_t, float *, float *, qld_hip_stream) {
    return QLD_E_STATE;
}
qld_status qld_denoiser_forward(qld_denoiser *, const float *, int32_t, float *, float *, qld_hip_stream) {
    return QLD_E_STATE;
}
qld_status qld_denoiser_info(const qld_denoiser *, int32_t *, int32_t *, int32_t *) { return QLD_E_STATE; }
qld_status qld_denoiser_tensor(qld_denoiser *, int32_t, void **, int64_t *) { return QLD_E_STATE; }

}  // extern "C"
