// Per-frame sliding window: an image at the camera frame rate.
//
// The paper's display refreshes the lock-in image as each new frame arrives,
// over the last N frames (Supplementary, sliding sequence).  With four samples
// per period and a window of 4M frames, frame t enters with the reference
// values c(t) = {1, 0, -1, 0} and s(t) = {0, 1, 0, -1} at its phase
// (phase0 + t) mod 4, and the frame that leaves (t - 4M) has the same phase,
// so one update is
//     I += c(t) (S_t - S_{t-4M}),   Q += s(t) (S_t - S_{t-4M})
// exact in int32.  The ring keeps the last 4M raw frames (the difference needs
// the sample that leaves); before the window is full the leaving sample is 0.
// The quadratures are in the absolute phase of the frame counter, so the image
// R = (I^2 + Q^2)^(1/2) does not rotate from frame to frame.
//
// Layout: ring [4M][H][W] samples (uint8 / uint16), I/Q state [H][W] int32.
// One lane per pixel; per frame and pixel 2 B read (new), 2 B read + 2 B
// written (ring), 8 B read + 8 B written (I/Q), optional I/Q/amplitude out.
#include <new>

#include "qld_internal.hpp"

struct qld_fwindow {
    qld_frame_desc d;
    int eb;
    int M;               // cycles; the window holds 4 M frames
    int phase0;          // phase of frame 0 after creation / the last reset
    int64_t t;           // frames since creation / reset
    void *ring;
    int32_t *I, *Q;
    hipStream_t last_stream;
};

namespace qld {
namespace {

constexpr int kFBlock = 256;

template <typename T>
__global__ __launch_bounds__(kFBlock) void fwindow_kernel(const T *__restrict__ frame, int64_t row_pitch, int H, int W,
                                                          T *__restrict__ ring_slot, int use_old, int ci, int cq,
                                                          int fresh, int32_t *__restrict__ I, int32_t *__restrict__ Q,
                                                          int32_t *__restrict__ I_out, int32_t *__restrict__ Q_out,
                                                          float *__restrict__ amp_out) {
    const int64_t npx = (int64_t)H * W;
    for (int64_t p = (int64_t)blockIdx.x * kFBlock + threadIdx.x; p < npx; p += (int64_t)gridDim.x * kFBlock) {
        const int64_t y = p / W, x = p % W;
        const int32_t s = (int32_t)frame[y * row_pitch + x];
        const int32_t old = use_old ? (int32_t)ring_slot[p] : 0;
        ring_slot[p] = (T)s;
        const int32_t d = s - old;
        const int32_t i = (fresh ? 0 : I[p]) + ci * d;
        const int32_t q = (fresh ? 0 : Q[p]) + cq * d;
        I[p] = i;
        Q[p] = q;
        if (I_out) {
            I_out[p] = i;
            Q_out[p] = q;
        }
        if (amp_out) {
            const int64_t a = i, b = q;
            amp_out[p] = (float)__builtin_sqrt((double)((uint64_t)(a * a) + (uint64_t)(b * b)));
        }
    }
}

}  // namespace
}  // namespace qld

using namespace qld;

extern "C" size_t qld_fwindow_bytes(const qld_frame_desc *d, int32_t M_cycles) {
    int eb = 0;
    if (check_desc(d, &eb) != QLD_OK || M_cycles < 1) return 0;
    const size_t npx = (size_t)d->H * (size_t)d->W;
    return (size_t)4 * M_cycles * npx * eb + npx * 8;
}

extern "C" qld_status qld_fwindow_create(const qld_frame_desc *d, int32_t M_cycles, int32_t phase0,
                                         qld_fwindow **out) {
    clear_error();
    int eb = 0;
    QLD_TRY(check_desc(d, &eb));
    if (!out || M_cycles < 1) {
        set_error("out must be non-NULL and M_cycles >= 1 (got %d)", M_cycles);
        return QLD_E_INVAL;
    }
    if ((uint64_t)M_cycles * ((1ull << d->bits) - 1) >= (1ull << 31)) {
        set_error("M=%d cycles of %d-bit data could overflow int32", M_cycles, d->bits);
        return QLD_E_OVERFLOW;
    }
    auto *w = new (std::nothrow) qld_fwindow();
    if (!w) {
        set_error("host allocation failed");
        return QLD_E_NOMEM;
    }
    w->d = *d;
    w->eb = eb;
    w->M = M_cycles;
    w->phase0 = ((phase0 % 4) + 4) % 4;
    w->t = 0;
    const size_t npx = (size_t)d->H * (size_t)d->W;
    if (npx > 0) {
        const size_t ring_b = (size_t)4 * M_cycles * npx * eb;
        if (hipMalloc(&w->ring, ring_b) != hipSuccess || hipMalloc(&w->I, npx * 8) != hipSuccess) {
            (void)hipGetLastError();
            if (w->ring) (void)hipFree(w->ring);
            delete w;
            set_error("frame window allocation of %zu bytes failed", ring_b + npx * 8);
            return QLD_E_NOMEM;
        }
        w->Q = w->I + npx;
    }
    *out = w;
    return QLD_OK;
}

extern "C" qld_status qld_fwindow_update(qld_fwindow *w, const void *frame, int32_t *I_out, int32_t *Q_out,
                                         float *amp_out, int32_t *warm_out, qld_hip_stream stream) {
    clear_error();
    if (!w) {
        set_error("frame window is NULL");
        return QLD_E_INVAL;
    }
    if ((I_out == nullptr) != (Q_out == nullptr)) {
        set_error("I_out and Q_out must be both NULL or both set");
        return QLD_E_INVAL;
    }
    const qld_frame_desc &d = w->d;
    const int64_t npx = (int64_t)d.H * d.W;
    if (npx > 0 && !frame) {
        set_error("frame is NULL");
        return QLD_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n_ring = 4 * (int64_t)w->M;
    if (npx > 0) {
        static const int kC[4] = {1, 0, -1, 0}, kS[4] = {0, 1, 0, -1};
        const int ph = (int)((w->phase0 + w->t) & 3);
        const int slot = (int)(w->t % n_ring);
        const int use_old = w->t >= n_ring ? 1 : 0;
        const int fresh = w->t == 0 ? 1 : 0;
        const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(npx, kFBlock), 8192);
        if (w->eb == 2) {
            hipLaunchKernelGGL(fwindow_kernel<uint16_t>, dim3(grid), dim3(kFBlock), 0, s,
                               static_cast<const uint16_t *>(frame), d.row_pitch, d.H, d.W,
                               static_cast<uint16_t *>(w->ring) + slot * npx, use_old, kC[ph], kS[ph], fresh, w->I,
                               w->Q, I_out, Q_out, amp_out);
        } else {
            hipLaunchKernelGGL(fwindow_kernel<uint8_t>, dim3(grid), dim3(kFBlock), 0, s,
                               static_cast<const uint8_t *>(frame), d.row_pitch, d.H, d.W,
                               static_cast<uint8_t *>(w->ring) + slot * npx, use_old, kC[ph], kS[ph], fresh, w->I,
                               w->Q, I_out, Q_out, amp_out);
        }
        QLD_TRY(check_hip(hipGetLastError(), "fwindow_kernel launch"));
    }
    w->t += 1;
    w->last_stream = s;
    if (warm_out) *warm_out = w->t >= n_ring ? 1 : 0;
    return QLD_OK;
}

extern "C" qld_status qld_fwindow_reset(qld_fwindow *w, int32_t phase0) {
    clear_error();
    if (!w) {
        set_error("frame window is NULL");
        return QLD_E_INVAL;
    }
    // The next update starts from an empty window: its kernel ignores the old
    // state, and ring slots are not read before they are rewritten.
    w->t = 0;
    w->phase0 = ((phase0 % 4) + 4) % 4;
    return QLD_OK;
}

extern "C" qld_status qld_fwindow_info(const qld_fwindow *w, int32_t *n_in_window, int64_t *n_frames) {
    clear_error();
    if (!w) {
        set_error("frame window is NULL");
        return QLD_E_INVAL;
    }
    if (n_in_window) *n_in_window = (int32_t)std::min<int64_t>(w->t, 4 * (int64_t)w->M);
    if (n_frames) *n_frames = w->t;
    return QLD_OK;
}

extern "C" qld_status qld_fwindow_destroy(qld_fwindow *w) {
    clear_error();
    if (!w) return QLD_OK;
    qld_status st = QLD_OK;
    if (w->last_stream) st = check_hip(hipStreamSynchronize(w->last_stream), "frame window stream sync");
    if (w->ring) (void)hipFree(w->ring);
    if (w->I) (void)hipFree(w->I);
    delete w;
    return st;
}
