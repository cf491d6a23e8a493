// Sliding-window quadrature lock-in (paper: Supplementary, the sliding
// sequence that refreshes the processed image at the camera rate, and the
// buffer of N frames it needs; section "Quadrature Lock-in Discrimination",
// processing that begins with the first frame).
//
// Instead of N raw frames the window keeps, per pixel, a ring of the per-cycle
// differences D_c = (S0 - S2, S1 - S3) -- int16 pairs for data of up to 15
// bits (4 bytes per pixel per cycle, half of one 16-bit frame per cycle) --
// and the running sums.  A new cycle adds D_c and, once M cycles are in,
// subtracts D_{c-M}, which it then overwrites in the ring:
//     (I, Q) += D_c - D_{c-M}.
// Integer arithmetic, so the window equals the batch sums of its last M
// cycles exactly.  An optional short window Ms <= M shares the same ring.
//
// One launch serves many streams of different sizes (continuous batching):
// a job table in the kernel arguments maps work-group ranges to streams; the
// cycles of one stream in a launch are applied in order by the same lanes.
#include <cstdio>
#include <cstring>
#include <new>

#include "window.hpp"

namespace qld {
namespace {

constexpr int kBlock = 256;

// One 16-byte group of a frame unpacked into VPX samples.
template <int ELEM, int VPX>
__device__ __forceinline__ void unpack_frame(const u32x4 &q, int32_t (&v)[VPX]) {
    const uint32_t w[4] = {q[0], q[1], q[2], q[3]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if constexpr (ELEM == 2) {
            v[2 * k] = (int32_t)(w[k] & 0xffffu);
            v[2 * k + 1] = (int32_t)(w[k] >> 16);
        } else {
            v[4 * k] = (int32_t)(w[k] & 0xffu);
            v[4 * k + 1] = (int32_t)((w[k] >> 8) & 0xffu);
            v[4 * k + 2] = (int32_t)((w[k] >> 16) & 0xffu);
            v[4 * k + 3] = (int32_t)(w[k] >> 24);
        }
    }
}

template <int ELEM, int VPX, bool VEC>
__device__ __forceinline__ void load_frame(const uint8_t *p, bool full, int nvalid, int32_t (&v)[VPX]) {
    if constexpr (VEC) {
        if (full) {
            const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
            const uint32_t w[4] = {q[0], q[1], q[2], q[3]};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if constexpr (ELEM == 2) {
                    v[2 * k] = (int32_t)(w[k] & 0xffffu);
                    v[2 * k + 1] = (int32_t)(w[k] >> 16);
                } else {
                    v[4 * k] = (int32_t)(w[k] & 0xffu);
                    v[4 * k + 1] = (int32_t)((w[k] >> 8) & 0xffu);
                    v[4 * k + 2] = (int32_t)((w[k] >> 16) & 0xffu);
                    v[4 * k + 3] = (int32_t)(w[k] >> 24);
                }
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < VPX; ++k) {
        if (k < nvalid) {
            if constexpr (ELEM == 2) v[k] = reinterpret_cast<const uint16_t *>(p)[k];
            else v[k] = p[k];
        } else {
            v[k] = 0;
        }
    }
}

// Ring entries of VPX pixels: RT pairs (i, q) interleaved, 16-byte aligned.
template <typename RT, int VPX>
__device__ __forceinline__ void ring_load(const RT *r, int32_t (&di)[VPX], int32_t (&dq)[VPX]) {
    constexpr int n32 = (int)(2 * VPX * sizeof(RT)) / 4;
    uint32_t w[n32];
#pragma unroll
    for (int k = 0; k < n32; k += 4) {
        const u32x4 q = *reinterpret_cast<const u32x4 *>(reinterpret_cast<const uint32_t *>(r) + k);
        w[k] = q[0];
        w[k + 1] = q[1];
        w[k + 2] = q[2];
        w[k + 3] = q[3];
    }
#pragma unroll
    for (int j = 0; j < VPX; ++j) {
        if constexpr (sizeof(RT) == 2) {
            di[j] = (int32_t)(int16_t)(w[j] & 0xffffu);
            dq[j] = (int32_t)(int16_t)(w[j] >> 16);
        } else {
            di[j] = (int32_t)w[2 * j];
            dq[j] = (int32_t)w[2 * j + 1];
        }
    }
}

template <typename RT, int VPX>
__device__ __forceinline__ void ring_store(RT *r, const int32_t (&di)[VPX], const int32_t (&dq)[VPX]) {
    constexpr int n32 = (int)(2 * VPX * sizeof(RT)) / 4;
    uint32_t w[n32];
#pragma unroll
    for (int j = 0; j < VPX; ++j) {
        if constexpr (sizeof(RT) == 2) {
            w[j] = ((uint32_t)di[j] & 0xffffu) | ((uint32_t)dq[j] << 16);
        } else {
            w[2 * j] = (uint32_t)di[j];
            w[2 * j + 1] = (uint32_t)dq[j];
        }
    }
#pragma unroll
    for (int k = 0; k < n32; k += 4) {
        u32x4 q;
        q[0] = w[k];
        q[1] = w[k + 1];
        q[2] = w[k + 2];
        q[3] = w[k + 3];
        *reinterpret_cast<u32x4 *>(reinterpret_cast<uint32_t *>(r) + k) = q;
    }
}

template <int VPX>
__device__ __forceinline__ void state_load(const int32_t *p, int32_t (&v)[VPX]) {
#pragma unroll
    for (int k = 0; k < VPX; k += 4) {
        const u32x4 q = *reinterpret_cast<const u32x4 *>(p + k);
        v[k] = (int32_t)q[0];
        v[k + 1] = (int32_t)q[1];
        v[k + 2] = (int32_t)q[2];
        v[k + 3] = (int32_t)q[3];
    }
}

template <int VPX>
__device__ __forceinline__ void state_store(int32_t *p, const int32_t (&v)[VPX]) {
#pragma unroll
    for (int k = 0; k < VPX; k += 4) {
        u32x4 q;
        q[0] = (uint32_t)v[k];
        q[1] = (uint32_t)v[k + 1];
        q[2] = (uint32_t)v[k + 2];
        q[3] = (uint32_t)v[k + 3];
        *reinterpret_cast<u32x4 *>(p + k) = q;
    }
}

__device__ __forceinline__ bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// VPX 4-byte values to a 16-byte aligned address.
template <typename T, int VPX>
__device__ __forceinline__ void store16(T *p, const T (&v)[VPX]) {
    static_assert(sizeof(T) == 4 && VPX % 4 == 0, "4-byte values, whole 16-byte groups");
#pragma unroll
    for (int k = 0; k < VPX; k += 4) {
        u32x4 q;
        q[0] = __builtin_bit_cast(uint32_t, v[k]);
        q[1] = __builtin_bit_cast(uint32_t, v[k + 1]);
        q[2] = __builtin_bit_cast(uint32_t, v[k + 2]);
        q[3] = __builtin_bit_cast(uint32_t, v[k + 3]);
        *reinterpret_cast<u32x4 *>(p + k) = q;
    }
}

template <int VPX>
__device__ __forceinline__ void out_iq(int32_t *io, int32_t *qo, const int32_t (&I)[VPX], const int32_t (&Q)[VPX],
                                       bool full, int nvalid) {
    if (full && aligned16(io) && aligned16(qo)) {
        store16<int32_t, VPX>(io, I);
        store16<int32_t, VPX>(qo, Q);
    } else {
#pragma unroll
        for (int k = 0; k < VPX; ++k) {
            if (k < nvalid) {
                io[k] = I[k];
                qo[k] = Q[k];
            }
        }
    }
}

__device__ __forceinline__ float amp_of(int32_t i, int32_t q) {
    const int64_t a = i, b = q;
    return (float)__builtin_sqrt((double)((uint64_t)(a * a) + (uint64_t)(b * b)));
}

template <int ELEM, int VPX, bool VEC, typename RT>
__global__ __launch_bounds__(kBlock) void window_batch_kernel(WinBatch bt) {
    const int b = blockIdx.x;
    int j = 0;
    while (j + 1 < bt.n_jobs && b >= bt.tile_start[j + 1]) ++j;
    const WinJob &J = bt.job[j];
    const int64_t g = (int64_t)(b - bt.tile_start[j]) * kBlock + threadIdx.x;
    const int nvx = J.Wp / VPX;
    const int64_t y = g / nvx;
    if (y >= J.H) return;
    const int x0 = (int)(g % nvx) * VPX;
    const int nvalid = min(VPX, J.W - x0);
    if (nvalid <= 0) return;              // padding lanes past the row end
    const bool full = nvalid == VPX;

    const int64_t sidx = y * J.Wp + x0;   // ring / state index (padded rows)
    const int64_t npx_p = (int64_t)J.H * J.Wp;
    const int64_t npx = (int64_t)J.H * J.W;
    RT *ring = static_cast<RT *>(J.ring);

    int32_t I[VPX], Q[VPX], Is[VPX], Qs[VPX];
    if (J.fresh) {
#pragma unroll
        for (int k = 0; k < VPX; ++k) I[k] = Q[k] = Is[k] = Qs[k] = 0;
    } else {
        state_load<VPX>(J.I + sidx, I);
        state_load<VPX>(J.Q + sidx, Q);
        if (J.Ms > 0) {
            state_load<VPX>(J.Is + sidx, Is);
            state_load<VPX>(J.Qs + sidx, Qs);
        }
    }

    for (int ci = 0; ci < J.n_cycles; ++ci) {
        const int64_t c = J.c0 + ci;
        const uint8_t *f = J.stage + (int64_t)((J.stage0 + ci) % J.n_stage) * J.slot_b + y * J.rp_b +
                           (int64_t)x0 * ELEM;
        int32_t s0[VPX], s1[VPX], s2[VPX], s3[VPX];
        const int64_t slot = c % J.M;
        RT *rs = ring + (slot * npx_p + sidx) * 2;
        const bool old = c >= J.M;
        int32_t oi[VPX], oq[VPX];
        if (VEC && full) {
            // Whole lane: the four frames' loads and the oldest ring entry are
            // issued together, then unpacked (a branch between the loads had
            // made each wait for the one before).
            u32x4 q[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                q[i] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(f + i * J.fs_b));
            if (old) ring_load<RT, VPX>(rs, oi, oq);
            __builtin_amdgcn_sched_barrier(0);
            unpack_frame<ELEM, VPX>(q[0], s0);
            unpack_frame<ELEM, VPX>(q[1], s1);
            unpack_frame<ELEM, VPX>(q[2], s2);
            unpack_frame<ELEM, VPX>(q[3], s3);
        } else {
            load_frame<ELEM, VPX, false>(f, full, nvalid, s0);
            load_frame<ELEM, VPX, false>(f + J.fs_b, full, nvalid, s1);
            load_frame<ELEM, VPX, false>(f + 2 * J.fs_b, full, nvalid, s2);
            load_frame<ELEM, VPX, false>(f + 3 * J.fs_b, full, nvalid, s3);
            if (old) ring_load<RT, VPX>(rs, oi, oq);
        }
        int32_t di[VPX], dq[VPX];
#pragma unroll
        for (int k = 0; k < VPX; ++k) {
            di[k] = s0[k] - s2[k];
            dq[k] = s1[k] - s3[k];
        }
        if (old) {
#pragma unroll
            for (int k = 0; k < VPX; ++k) {
                I[k] -= oi[k];
                Q[k] -= oq[k];
            }
        }
        if (J.Ms > 0) {
            if (c >= J.Ms) {
                int32_t oi[VPX], oq[VPX];
                ring_load<RT, VPX>(ring + (((c - J.Ms) % J.M) * npx_p + sidx) * 2, oi, oq);
#pragma unroll
                for (int k = 0; k < VPX; ++k) {
                    Is[k] -= oi[k];
                    Qs[k] -= oq[k];
                }
            }
#pragma unroll
            for (int k = 0; k < VPX; ++k) {
                Is[k] += di[k];
                Qs[k] += dq[k];
            }
        }
#pragma unroll
        for (int k = 0; k < VPX; ++k) {
            I[k] += di[k];
            Q[k] += dq[k];
        }
        ring_store<RT, VPX>(rs, di, dq);

        const int64_t oslot = (int64_t)((J.out0 + ci) % J.out_slots) * npx + y * J.W + x0;
        // Outputs: 16-byte stores where the lane's pixels are all in the row and
        // that output's address is 16-byte aligned, else element by element.
        if (J.amp) {
            if (full && aligned16(J.amp + oslot)) {
                float av[VPX];
#pragma unroll
                for (int k = 0; k < VPX; ++k) av[k] = amp_of(I[k], Q[k]);
                store16<float, VPX>(J.amp + oslot, av);
            } else {
#pragma unroll
                for (int k = 0; k < VPX; ++k)
                    if (k < nvalid) J.amp[oslot + k] = amp_of(I[k], Q[k]);
            }
        }
        if (J.Io) out_iq<VPX>(J.Io + oslot, J.Qo + oslot, I, Q, full, nvalid);
        if (J.Iso) out_iq<VPX>(J.Iso + oslot, J.Qso + oslot, Is, Qs, full, nvalid);
    }
    state_store<VPX>(J.I + sidx, I);
    state_store<VPX>(J.Q + sidx, Q);
    if (J.Ms > 0) {
        state_store<VPX>(J.Is + sidx, Is);
        state_store<VPX>(J.Qs + sidx, Qs);
    }
}

__global__ __launch_bounds__(256) void zero_i32_kernel(int32_t *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

template <int ELEM, bool VEC, typename RT>
hipError_t launch_t(const WinBatch &b, hipStream_t s) {
    constexpr int VPX = 16 / ELEM;   // lane width is fixed by the ring layout; VEC only selects frame loads
    hipLaunchKernelGGL((window_batch_kernel<ELEM, VPX, VEC, RT>), dim3(b.tile_start[b.n_jobs]), dim3(kBlock), 0,
                       s, b);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_window_batch(const WinBatch &b, int elem, bool wide, bool vec, hipStream_t s) {
    if (b.n_jobs <= 0 || b.tile_start[b.n_jobs] <= 0) return hipSuccess;
    if (elem == 2) {
        if (wide) return vec ? launch_t<2, true, int32_t>(b, s) : launch_t<2, false, int32_t>(b, s);
        return vec ? launch_t<2, true, int16_t>(b, s) : launch_t<2, false, int16_t>(b, s);
    }
    return vec ? launch_t<1, true, int16_t>(b, s) : launch_t<1, false, int16_t>(b, s);
}

hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), 4096);
    hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// The window kernel's lane width is fixed by the vector path (16 bytes of
// samples per lane); ring and state rows are padded to a multiple of it so
// every lane's ring/state access is one aligned 16-byte group.
static int padded_width(int W, int eb) {
    const int v = window_vpx(eb);
    return (int)(ceil_div(W, v) * v);
}

size_t window_bytes(const qld_frame_desc *d, int32_t M, int32_t Ms) {
    int eb = 0;
    if (check_desc(d, &eb) != QLD_OK || M < 1 || Ms < 0 || Ms > M) return 0;
    const int wide = d->bits > 15;
    const size_t npx_p = (size_t)d->H * (size_t)padded_width(d->W, eb);
    const size_t ring = (size_t)M * npx_p * (wide ? 8 : 4);
    const size_t state = npx_p * 4 * (Ms > 0 ? 4 : 2);
    return ring + state;
}

qld_status window_alloc(const qld_frame_desc *d, int32_t M, int32_t Ms, qld_window **out) {
    int eb = 0;
    QLD_TRY(check_desc(d, &eb));
    if (!out) {
        set_error("out is NULL");
        return QLD_E_INVAL;
    }
    if (M < 1 || Ms < 0 || Ms > M) {
        set_error("window length M=%d (short %d) invalid", M, Ms);
        return QLD_E_INVAL;
    }
    if ((uint64_t)M * ((1ull << d->bits) - 1) >= (1ull << 31)) {
        set_error("M=%d cycles of %d-bit data could overflow int32", M, d->bits);
        return QLD_E_OVERFLOW;
    }
    qld_window *w = new (std::nothrow) qld_window();
    if (!w) {
        set_error("host allocation failed");
        return QLD_E_NOMEM;
    }
    w->d = *d;
    w->eb = eb;
    w->M = M;
    w->Ms = Ms;
    w->wide = d->bits > 15;
    w->Wp = padded_width(d->W, eb);
    (void)hipGetDevice(&w->device);
    const size_t npx_p = (size_t)d->H * (size_t)w->Wp;
    const size_t ring_b = (size_t)M * npx_p * (w->wide ? 8 : 4);
    const size_t nstate = Ms > 0 ? 4 : 2;
    void *ring = nullptr, *state = nullptr;
    if (npx_p > 0) {
        if (hipMalloc(&ring, ring_b) != hipSuccess || hipMalloc(&state, npx_p * 4 * nstate) != hipSuccess) {
            (void)hipGetLastError();
            if (ring) (void)hipFree(ring);
            delete w;
            set_error("window allocation of %zu bytes failed", ring_b + npx_p * 4 * nstate);
            return QLD_E_NOMEM;
        }
        if (hipMemset(state, 0, npx_p * 4 * nstate) != hipSuccess) {
            (void)hipFree(ring);
            (void)hipFree(state);
            delete w;
            set_error("window state clear failed");
            return QLD_E_DEVICE;
        }
    }
    w->ring = ring;
    w->I = static_cast<int32_t *>(state);
    w->Q = w->I ? w->I + npx_p : nullptr;
    w->Is = (Ms > 0 && w->I) ? w->I + 2 * npx_p : nullptr;
    w->Qs = (Ms > 0 && w->I) ? w->I + 3 * npx_p : nullptr;
    w->c = 0;
    w->last_stream = nullptr;
    *out = w;
    return QLD_OK;
}

}  // namespace qld

using namespace qld;

extern "C" size_t qld_window_bytes(const qld_frame_desc *d, int32_t M_cycles) {
    return window_bytes(d, M_cycles, 0);
}

extern "C" qld_status qld_window_create(const qld_frame_desc *d, int32_t M_cycles, qld_window **out) {
    clear_error();
    return window_alloc(d, M_cycles, 0, out);
}

extern "C" qld_status qld_window_update(qld_window *w, const void *cycle_frames, int32_t *I_out, int32_t *Q_out,
                                        float *amp_out, int32_t *warm_out, qld_hip_stream stream) {
    clear_error();
    if (!w) {
        set_error("window is NULL");
        return QLD_E_INVAL;
    }
    const qld_frame_desc &d = w->d;
    const int64_t npx = (int64_t)d.H * d.W;
    if (npx > 0 && !cycle_frames) {
        set_error("cycle_frames is NULL");
        return QLD_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (npx > 0) {
        const int64_t rp_b = d.row_pitch * w->eb, fs_b = d.frame_stride * w->eb;
        const bool vec = (reinterpret_cast<uintptr_t>(cycle_frames) % 16 == 0) && rp_b % 16 == 0 && fs_b % 16 == 0;
        WinBatch b{};
        b.n_jobs = 1;
        WinJob &J = b.job[0];
        J.stage = static_cast<const uint8_t *>(cycle_frames);
        J.rp_b = rp_b;
        J.fs_b = fs_b;
        J.slot_b = 4 * fs_b;
        J.n_stage = 1;
        J.stage0 = 0;
        J.H = d.H;
        J.W = d.W;
        J.Wp = w->Wp;
        J.M = w->M;
        J.Ms = w->Ms;
        J.c0 = w->c;
        J.n_cycles = 1;
        J.fresh = w->c == 0;
        J.ring = w->ring;
        J.I = w->I;
        J.Q = w->Q;
        J.Is = w->Is;
        J.Qs = w->Qs;
        J.amp = amp_out;
        J.Io = (I_out && Q_out) ? I_out : nullptr;
        J.Qo = (I_out && Q_out) ? Q_out : nullptr;
        J.out_slots = 1;
        J.out0 = 0;
        // Lanes cover window_vpx pixels (the ring layout) whatever the frame
        // alignment; unaligned frames are read element by element.
        J.tiles = (int32_t)ceil_div((int64_t)d.H * (w->Wp / window_vpx(w->eb)), 256);
        b.tile_start[0] = 0;
        b.tile_start[1] = J.tiles;
        if (I_out && !Q_out) {
            set_error("I_out and Q_out must be both NULL or both set");
            return QLD_E_INVAL;
        }
        hipEvent_t ev0, ev1;
        take_kernel_timer(&ev0, &ev1);
        if (ev0) QLD_TRY(check_hip(hipEventRecord(ev0, s), "timer start"));
        QLD_TRY(check_hip(launch_window_batch(b, w->eb, w->wide, vec, s), "window_batch_kernel launch"));
        if (ev1) QLD_TRY(check_hip(hipEventRecord(ev1, s), "timer stop"));
    }
    w->c += 1;
    w->last_stream = s;
    if (warm_out) *warm_out = w->c >= w->M ? 1 : 0;
    return QLD_OK;
}

extern "C" qld_status qld_window_reset(qld_window *w) {
    clear_error();
    if (!w) {
        set_error("window is NULL");
        return QLD_E_INVAL;
    }
    // The next update starts from an empty window (its kernel ignores the old
    // state and the ring slots are rewritten before they are read again).
    w->c = 0;
    return QLD_OK;
}

extern "C" qld_status qld_window_destroy(qld_window *w) {
    clear_error();
    if (!w) return QLD_OK;
    qld_status st = QLD_OK;
    if (w->last_stream) st = check_hip(hipStreamSynchronize(w->last_stream), "window stream sync");
    if (w->ring) (void)hipFree(w->ring);
    if (w->I) (void)hipFree(w->I);
    delete w;
    return st;
}

extern "C" qld_status qld_window_info(const qld_window *w, int32_t *n_in_window, int64_t *n_cycles) {
    clear_error();
    if (!w) {
        set_error("window is NULL");
        return QLD_E_INVAL;
    }
    if (n_in_window) *n_in_window = (int32_t)std::min<int64_t>(w->c, w->M);
    if (n_cycles) *n_cycles = w->c;
    return QLD_OK;
}

namespace {
struct CkptHeader {
    char magic[8];
    int32_t version;
    int32_t H, W, dtype, bits, M, Ms, Wp;
    int64_t c;
    int64_t ring_bytes, state_bytes;
};
}  // namespace

extern "C" qld_status qld_window_save(const qld_window *w, const char *path) {
    clear_error();
    if (!w || !path) {
        set_error("window and path must be non-NULL");
        return QLD_E_INVAL;
    }
    const size_t npx_p = (size_t)w->d.H * w->Wp;
    CkptHeader h{};
    memcpy(h.magic, "QLDWIN1", 8);
    h.version = 1;
    h.H = w->d.H;
    h.W = w->d.W;
    h.dtype = (int32_t)w->d.dtype;
    h.bits = w->d.bits;
    h.M = w->M;
    h.Ms = w->Ms;
    h.Wp = w->Wp;
    h.c = w->c;
    h.ring_bytes = (int64_t)((size_t)w->M * npx_p * (w->wide ? 8 : 4));
    h.state_bytes = (int64_t)(npx_p * 4 * (w->Ms > 0 ? 4 : 2));
    char *buf = static_cast<char *>(malloc((size_t)(h.ring_bytes + h.state_bytes) + 1));
    if (!buf) {
        set_error("host allocation failed");
        return QLD_E_NOMEM;
    }
    if (w->last_stream) QLD_TRY(check_hip(hipStreamSynchronize(w->last_stream), "window stream sync"));
    qld_status st = QLD_OK;
    if (npx_p > 0) {
        st = check_hip(hipMemcpy(buf, w->ring, (size_t)h.ring_bytes, hipMemcpyDeviceToHost), "ring copy");
        if (st == QLD_OK)
            st = check_hip(hipMemcpy(buf + h.ring_bytes, w->I, (size_t)h.state_bytes, hipMemcpyDeviceToHost),
                           "state copy");
    }
    if (st == QLD_OK) {
        FILE *f = fopen(path, "wb");
        if (!f || fwrite(&h, sizeof(h), 1, f) != 1 ||
            fwrite(buf, 1, (size_t)(h.ring_bytes + h.state_bytes), f) != (size_t)(h.ring_bytes + h.state_bytes)) {
            set_error("writing %s failed", path);
            st = QLD_E_IO;
        }
        if (f && fclose(f) != 0 && st == QLD_OK) {
            set_error("closing %s failed", path);
            st = QLD_E_IO;
        }
    }
    free(buf);
    return st;
}

extern "C" qld_status qld_window_load(qld_window *w, const char *path) {
    clear_error();
    if (!w || !path) {
        set_error("window and path must be non-NULL");
        return QLD_E_INVAL;
    }
    FILE *f = fopen(path, "rb");
    if (!f) {
        set_error("cannot open %s", path);
        return QLD_E_IO;
    }
    CkptHeader h{};
    if (fread(&h, sizeof(h), 1, f) != 1 || memcmp(h.magic, "QLDWIN1", 8) != 0 || h.version != 1) {
        fclose(f);
        set_error("%s is not a window checkpoint", path);
        return QLD_E_IO;
    }
    const size_t npx_p = (size_t)w->d.H * w->Wp;
    if (h.H != w->d.H || h.W != w->d.W || h.dtype != (int32_t)w->d.dtype || h.bits != w->d.bits || h.M != w->M ||
        h.Ms != w->Ms || h.Wp != w->Wp || h.ring_bytes != (int64_t)((size_t)w->M * npx_p * (w->wide ? 8 : 4)) ||
        h.state_bytes != (int64_t)(npx_p * 4 * (w->Ms > 0 ? 4 : 2))) {
        fclose(f);
        set_error("checkpoint %s does not match this window's shape", path);
        return QLD_E_STATE;
    }
    char *buf = static_cast<char *>(malloc((size_t)(h.ring_bytes + h.state_bytes) + 1));
    if (!buf) {
        fclose(f);
        set_error("host allocation failed");
        return QLD_E_NOMEM;
    }
    const size_t want = (size_t)(h.ring_bytes + h.state_bytes);
    const bool ok = fread(buf, 1, want, f) == want;
    fclose(f);
    if (!ok) {
        free(buf);
        set_error("%s is truncated", path);
        return QLD_E_IO;
    }
    qld_status st = QLD_OK;
    if (w->last_stream) st = check_hip(hipStreamSynchronize(w->last_stream), "window stream sync");
    if (st == QLD_OK && npx_p > 0) {
        st = check_hip(hipMemcpy(w->ring, buf, (size_t)h.ring_bytes, hipMemcpyHostToDevice), "ring copy");
        if (st == QLD_OK)
            st = check_hip(hipMemcpy(w->I, buf + h.ring_bytes, (size_t)h.state_bytes, hipMemcpyHostToDevice),
                           "state copy");
    }
    free(buf);
    if (st == QLD_OK) w->c = h.c;
    return st;
}
