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
// Exactly one of c(t), s(t) is non-zero, so a frame changes only one of I, Q:
// the other is read only when the amplitude or the I/Q outputs need it.
// Vector kernel (W, row pitch and base in whole groups of 4 pixels): a lane
// owns 4 pixels, with 4- or 8-byte sample accesses and 16-byte I/Q and
// amplitude accesses; per frame and pixel (uint16, amplitude out) 2 B read
// (new), 2 + 2 B (ring), 8 B read + 4 B written (I/Q), 4 B written
// (amplitude).  Otherwise one lane per pixel.
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

template <typename T>
struct Vec4;
template <>
struct Vec4<uint16_t> {
    typedef uint32_t raw __attribute__((ext_vector_type(2)));
    __device__ static void unpack(raw r, int32_t (&v)[4]) {
        v[0] = (int32_t)(r[0] & 0xffffu);
        v[1] = (int32_t)(r[0] >> 16);
        v[2] = (int32_t)(r[1] & 0xffffu);
        v[3] = (int32_t)(r[1] >> 16);
    }
    __device__ static raw pack(const int32_t (&v)[4]) {
        return raw{((uint32_t)v[0] & 0xffffu) | ((uint32_t)v[1] << 16), ((uint32_t)v[2] & 0xffffu) | ((uint32_t)v[3] << 16)};
    }
};
template <>
struct Vec4<uint8_t> {
    typedef uint32_t raw;
    __device__ static void unpack(raw r, int32_t (&v)[4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = (int32_t)((r >> (8 * k)) & 0xffu);
    }
    __device__ static raw pack(const int32_t (&v)[4]) {
        return ((uint32_t)v[0] & 0xffu) | (((uint32_t)v[1] & 0xffu) << 8) | (((uint32_t)v[2] & 0xffu) << 16) |
               ((uint32_t)v[3] << 24);
    }
};

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4w __attribute__((ext_vector_type(4)));

// The vector kernel: W % 4 == 0, row pitch % 4 == 0, frame base aligned to 4
// samples, outputs 16-byte aligned (checked on the host).
template <typename T>
__global__ __launch_bounds__(kFBlock) void fwindow_vec_kernel(const T *__restrict__ frame, int64_t row_pitch, int H,
                                                              int W, T *__restrict__ ring_slot, int use_old, int ci,
                                                              int cq, int fresh, int32_t *__restrict__ I,
                                                              int32_t *__restrict__ Q, int32_t *__restrict__ I_out,
                                                              int32_t *__restrict__ Q_out,
                                                              float *__restrict__ amp_out) {
    typedef typename Vec4<T>::raw raw;
    const int64_t n4 = (int64_t)H * W / 4;
    const bool need_both = amp_out || I_out;
    for (int64_t g = (int64_t)blockIdx.x * kFBlock + threadIdx.x; g < n4; g += (int64_t)gridDim.x * kFBlock) {
        const int64_t p = 4 * g, y = p / W, x = p % W;
        int32_t sv[4], ov[4] = {0, 0, 0, 0};
        Vec4<T>::unpack(__builtin_nontemporal_load(reinterpret_cast<const raw *>(frame + y * row_pitch + x)), sv);
        raw *rp = reinterpret_cast<raw *>(ring_slot) + g;
        if (use_old) Vec4<T>::unpack(*rp, ov);
        *rp = Vec4<T>::pack(sv);
        i32x4 d, iv, qv;
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = sv[k] - ov[k];
        i32x4 *Ip = reinterpret_cast<i32x4 *>(I) + g;
        i32x4 *Qp = reinterpret_cast<i32x4 *>(Q) + g;
        if (fresh) {
            iv = ci * d;
            qv = cq * d;
            *Ip = iv;
            *Qp = qv;
        } else if (ci != 0) {
            iv = *Ip + ci * d;
            *Ip = iv;
            if (need_both) qv = *Qp;
        } else {
            qv = *Qp + cq * d;
            *Qp = qv;
            if (need_both) iv = *Ip;
        }
        if (I_out) {
            reinterpret_cast<i32x4 *>(I_out)[g] = iv;
            reinterpret_cast<i32x4 *>(Q_out)[g] = qv;
        }
        if (amp_out) {
            f32x4w a;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t u = iv[k], v = qv[k];
                a[k] = (float)__builtin_sqrt((double)((uint64_t)(u * u) + (uint64_t)(v * v)));
            }
            reinterpret_cast<f32x4w *>(amp_out)[g] = a;
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
        hipEvent_t ev0, ev1;
        take_kernel_timer(&ev0, &ev1);
        if (ev0) QLD_TRY(check_hip(hipEventRecord(ev0, s), "timer start"));
        auto al = [](const void *q, uintptr_t a) { return q == nullptr || reinterpret_cast<uintptr_t>(q) % a == 0; };
        const bool vec = d.W % 4 == 0 && d.row_pitch % 4 == 0 && al(frame, 4 * (uintptr_t)w->eb) && al(I_out, 16) &&
                         al(Q_out, 16) && al(amp_out, 16);
        if (vec) {
            const unsigned g4 = (unsigned)std::min<int64_t>(ceil_div(npx / 4, kFBlock), 8192);
            if (w->eb == 2)
                hipLaunchKernelGGL(fwindow_vec_kernel<uint16_t>, dim3(g4), dim3(kFBlock), 0, s,
                                   static_cast<const uint16_t *>(frame), d.row_pitch, d.H, d.W,
                                   static_cast<uint16_t *>(w->ring) + slot * npx, use_old, kC[ph], kS[ph], fresh, w->I,
                                   w->Q, I_out, Q_out, amp_out);
            else
                hipLaunchKernelGGL(fwindow_vec_kernel<uint8_t>, dim3(g4), dim3(kFBlock), 0, s,
                                   static_cast<const uint8_t *>(frame), d.row_pitch, d.H, d.W,
                                   static_cast<uint8_t *>(w->ring) + slot * npx, use_old, kC[ph], kS[ph], fresh, w->I,
                                   w->Q, I_out, Q_out, amp_out);
        } else if (w->eb == 2) {
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
        if (ev1) QLD_TRY(check_hip(hipEventRecord(ev1, s), "timer stop"));
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
