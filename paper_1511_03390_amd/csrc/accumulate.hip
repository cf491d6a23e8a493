// Batch quadrature lock-in: I/Q accumulation with fused per-frame statistics,
// and the amplitude image.
//
// Paper: Methods, formula for R(j,k) (sums of the series times sin and cos of
// the lock-in phase, then the root of the sum of squares); Supplementary,
// "Timing sequence" (each frame multiplied by sin and cos and accumulated into
// two 2-D arrays, then squared and added).  With four samples per period the
// sin/cos arrays take the values {0, +1, -1}, so the products reduce to
// I += S0 - S2 and Q += S1 - S3 per cycle: exact integer adds, no multiplies.
//
// Layout and mapping (gfx950, wave64):
//   * one lane owns VPX adjacent pixels of one row: 16 uint8 or 8 uint16, read
//     with one 16-byte load per frame (global_load_dwordx4), so a wave reads
//     1 KiB per frame, fully coalesced;
//   * int32 accumulators stay in VGPRs across the whole frame loop;
//   * the frame axis can be split into chunks handled by different work-groups
//     (for small images); chunk partials are combined with int32 atomics,
//     which are exact and order-free.  The chunks of one pixel tile are placed
//     on the same XCD (work-group ids are dealt round-robin over the 8 XCDs),
//     so their atomics meet in one L2;
//   * per-frame statistics (sum, saturated count) are reduced across the wave
//     with DPP row shifts/broadcasts and a ballot popcount, buffered one value
//     per lane for 64 frames, and written as per-wave partials that a second
//     small kernel folds into frame_sum / frame_sat.
#include "qld_internal.hpp"

namespace qld {
namespace {

constexpr int kBlock = 256;            // lanes per work-group (4 waves)
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kXcds = 8;

struct AccumArgs {
    const uint8_t *frames;
    int64_t rp_b;          // row pitch, bytes
    int64_t fs_b;          // frame stride, bytes
    int32_t H, W;
    int32_t n_frames;
    int32_t chunk;         // frames per split (multiple of 4)
    int32_t n_split;
    int32_t rot;           // phase of frame 0, mod 4
    int32_t nvx;           // lane vectors per row
    int32_t n_tiles;       // work-group tiles over pixels
    uint32_t top;          // 2^bits - 1
    int32_t *I;
    int32_t *Q;
    uint32_t *part_sum;    // [n_tiles * 4 waves][n_frames]
    uint32_t *part_sat;
};

template <int ELEM, int VPX, bool VEC>
__device__ __forceinline__ void load_px(const uint8_t *p, bool full, int nvalid, uint32_t (&v)[VPX]) {
    if constexpr (VEC) {
        if (full) {
            const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
            const uint32_t w[4] = {q[0], q[1], q[2], q[3]};
            if constexpr (ELEM == 2) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    v[2 * k] = w[k] & 0xffffu;
                    v[2 * k + 1] = w[k] >> 16;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    v[4 * k] = w[k] & 0xffu;
                    v[4 * k + 1] = (w[k] >> 8) & 0xffu;
                    v[4 * k + 2] = (w[k] >> 16) & 0xffu;
                    v[4 * k + 3] = w[k] >> 24;
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

// Sum of a 32-bit value over the 64 lanes of the wave, valid in lane 63.
// Inclusive shifts inside each 16-lane row, then row broadcasts 15 and 31.
__device__ __forceinline__ uint32_t wave_sum_lane63(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, true);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, true);  // row_bcast:31
    return v;
}

template <int VPX>
struct FrameStats {
    uint32_t buf_sum = 0, buf_sat = 0;   // lane j holds the value of frame (group base + j)
    int slot = 0;                        // frames buffered in the current 64-frame group
    int64_t base = 0;                    // chunk-relative index of the group's first frame

    __device__ __forceinline__ void add(const uint32_t (&v)[VPX], uint32_t top, int lane) {
        uint32_t s = 0, c = 0;
#pragma unroll
        for (int k = 0; k < VPX; ++k) {
            s += v[k];
            c += (uint32_t)__popcll(__ballot(v[k] == top));
        }
        uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)wave_sum_lane63(s), 63);
        if (lane == slot) {
            buf_sum = tot;
            buf_sat = c;
        }
        ++slot;
    }

    __device__ __forceinline__ void flush(uint32_t *ps, uint32_t *pc, int64_t row, int lane) {
        if (lane < slot) {
            ps[row + base + lane] = buf_sum;
            pc[row + base + lane] = buf_sat;
        }
        base += slot;
        slot = 0;
    }
};

template <int ELEM, int VPX, bool VEC, bool STATS>
__global__ __launch_bounds__(kBlock) void qld_accum_kernel(AccumArgs a) {
    // Work-group id -> (pixel tile, frame chunk), chunks of a tile on one XCD.
    const int b = blockIdx.x;
    const int xcd = b % kXcds;
    const int q = b / kXcds;
    const int split = q % a.n_split;
    const int tile = (q / a.n_split) * kXcds + xcd;
    if (tile >= a.n_tiles) return;

    const int lane = threadIdx.x & 63;
    const int64_t g = (int64_t)tile * kBlock + threadIdx.x;
    const int64_t y = g / a.nvx;
    const int x0 = (int)(g % a.nvx) * VPX;
    const bool row_ok = y < a.H;
    const int nvalid = row_ok ? min(VPX, a.W - x0) : 0;
    const bool full = nvalid == VPX;

    const int64_t t0 = (int64_t)split * a.chunk;
    const int64_t t1 = min((int64_t)a.n_frames, t0 + a.chunk);
    const int64_t len = t1 - t0;
    const uint8_t *p = a.frames + (row_ok ? (y * a.rp_b + (int64_t)x0 * ELEM + t0 * a.fs_b) : 0);
    const int64_t fs = a.fs_b;

    int32_t accI[VPX], accQ[VPX];
#pragma unroll
    for (int k = 0; k < VPX; ++k) accI[k] = accQ[k] = 0;

    FrameStats<VPX> st;
    const int64_t wave_row = ((int64_t)tile * kWavesPerBlock + (threadIdx.x >> 6)) * a.n_frames + t0;

    const int64_t n_cyc = len >> 2;
    for (int64_t c = 0; c < n_cyc; ++c) {
        uint32_t s0[VPX], s1[VPX], s2[VPX], s3[VPX];
        load_px<ELEM, VPX, VEC>(p, full, nvalid, s0);
        load_px<ELEM, VPX, VEC>(p + fs, full, nvalid, s1);
        load_px<ELEM, VPX, VEC>(p + 2 * fs, full, nvalid, s2);
        load_px<ELEM, VPX, VEC>(p + 3 * fs, full, nvalid, s3);
        p += 4 * fs;
#pragma unroll
        for (int k = 0; k < VPX; ++k) {
            accI[k] += (int32_t)s0[k] - (int32_t)s2[k];
            accQ[k] += (int32_t)s1[k] - (int32_t)s3[k];
        }
        if constexpr (STATS) {
            st.add(s0, a.top, lane);
            st.add(s1, a.top, lane);
            st.add(s2, a.top, lane);
            st.add(s3, a.top, lane);
            if (st.slot == 64) st.flush(a.part_sum, a.part_sat, wave_row, lane);
        }
    }
    // Partial cycle at the end of the stack (only the last chunk has one).
    const int rem = (int)(len & 3);
    for (int j = 0; j < rem; ++j) {
        uint32_t s[VPX];
        load_px<ELEM, VPX, VEC>(p, full, nvalid, s);
        p += fs;
#pragma unroll
        for (int k = 0; k < VPX; ++k) {
            if (j == 0) accI[k] += (int32_t)s[k];
            else if (j == 1) accQ[k] += (int32_t)s[k];
            else accI[k] -= (int32_t)s[k];
        }
        if constexpr (STATS) {
            st.add(s, a.top, lane);
            if (st.slot == 64) st.flush(a.part_sum, a.part_sat, wave_row, lane);
        }
    }
    if constexpr (STATS) {
        if (st.slot) st.flush(a.part_sum, a.part_sat, wave_row, lane);
    }

    if (!row_ok) return;
    int32_t *Ip = a.I + y * a.W + x0;
    int32_t *Qp = a.Q + y * a.W + x0;
#pragma unroll
    for (int k = 0; k < VPX; ++k) {
        if (k < nvalid) {
            int32_t oi, oq;
            rotate_iq(a.rot, accI[k], accQ[k], oi, oq);
            if (a.n_split > 1) {
                atomicAdd(Ip + k, oi);
                atomicAdd(Qp + k, oq);
            } else {
                Ip[k] += oi;
                Qp[k] += oq;
            }
        }
    }
}

// frame_sum[t] += sum over waves of part_sum[w][t] (and the same for counts).
// Grid: (ceil(T/64), ceil(n_waves/kRowsPerBlock)), one wave per work-group.
constexpr int kRowsPerBlock = 32;

__global__ __launch_bounds__(64) void qld_stats_reduce_kernel(const uint32_t *ps, const uint32_t *pc,
                                                              int64_t n_waves, int32_t T,
                                                              uint64_t *frame_sum, uint32_t *frame_sat) {
    const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (t >= T) return;
    const int64_t w0 = (int64_t)blockIdx.y * kRowsPerBlock;
    const int64_t w1 = min(n_waves, w0 + kRowsPerBlock);
    uint64_t s = 0;
    uint32_t c = 0;
    for (int64_t w = w0; w < w1; ++w) {
        s += ps[w * T + t];
        c += pc[w * T + t];
    }
    if (frame_sum) atomicAdd(reinterpret_cast<unsigned long long *>(frame_sum + t), (unsigned long long)s);
    if (frame_sat) atomicAdd(frame_sat + t, c);
}

__global__ __launch_bounds__(256) void qld_amplitude_kernel(const int32_t *__restrict__ I,
                                                            const int32_t *__restrict__ Q, int64_t n,
                                                            float *__restrict__ amp) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t a = I[i], q = Q[i];
        const uint64_t ss = (uint64_t)(a * a) + (uint64_t)(q * q);   // exact: |I|, |Q| < 2^31
        amp[i] = (float)__builtin_sqrt((double)ss);
    }
}

template <int ELEM, int VPX, bool VEC, bool STATS>
hipError_t launch_accum(const AccumArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((qld_accum_kernel<ELEM, VPX, VEC, STATS>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace
}  // namespace qld

using namespace qld;

extern "C" qld_status qld_accumulate(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                                     int32_t phase0, int32_t *I, int32_t *Q, uint64_t *frame_sum,
                                     uint32_t *frame_sat, qld_hip_stream stream) {
    clear_error();
    int eb = 0;
    QLD_TRY(check_desc(d, &eb));
    if (n_frames < 0) {
        set_error("n_frames %d < 0", n_frames);
        return QLD_E_INVAL;
    }
    const int64_t npx = (int64_t)d->H * d->W;
    if (n_frames == 0 || npx == 0) return QLD_OK;
    if (!frames || !I || !Q) {
        set_error("frames, I and Q must be non-NULL");
        return QLD_E_INVAL;
    }
    const uint64_t top = (1ull << d->bits) - 1;
    if ((uint64_t)ceil_div(n_frames, 4) * top >= (1ull << 31)) {
        set_error("ceil(%d/4) * %llu >= 2^31: int32 I/Q could overflow", n_frames, (unsigned long long)top);
        return QLD_E_OVERFLOW;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    const uintptr_t base = reinterpret_cast<uintptr_t>(frames);
    const int64_t rp_b = d->row_pitch * eb, fs_b = d->frame_stride * eb;
    const bool vec = (base % 16 == 0) && (rp_b % 16 == 0) && (fs_b % 16 == 0);
    const int vpx = vec ? 16 / eb : 1;

    AccumArgs a{};
    a.frames = static_cast<const uint8_t *>(frames);
    a.rp_b = rp_b;
    a.fs_b = fs_b;
    a.H = d->H;
    a.W = d->W;
    a.n_frames = n_frames;
    a.rot = ((phase0 % 4) + 4) % 4;
    a.nvx = (int32_t)ceil_div(d->W, vpx);
    const int64_t n_vec = (int64_t)a.nvx * d->H;
    const int64_t n_tiles = ceil_div(n_vec, kBlock);
    if (n_tiles > (1ll << 24)) {
        set_error("image too large (%lld tiles)", (long long)n_tiles);
        return QLD_E_SHAPE;
    }
    a.n_tiles = (int32_t)n_tiles;
    a.top = (uint32_t)top;
    a.I = I;
    a.Q = Q;

    // Split the frame axis until the grid holds ~8 work-groups per CU, keeping
    // chunks of at least 64 frames.
    const int64_t want_blocks = 8ll * device_cu_count();
    int64_t n_split = 1;
    if (n_tiles < want_blocks) n_split = ceil_div(want_blocks, n_tiles);
    n_split = std::max<int64_t>(1, std::min<int64_t>(n_split, n_frames / 64));
    int64_t chunk = ceil_div(ceil_div(n_frames, n_split), 4) * 4;
    n_split = ceil_div(n_frames, chunk);
    a.chunk = (int32_t)chunk;
    a.n_split = (int32_t)n_split;

    const bool stats = frame_sum || frame_sat;
    const int64_t n_waves = n_tiles * kWavesPerBlock;
    if (stats) {
        size_t need = sizeof(uint32_t) * 2 * (size_t)n_waves * (size_t)n_frames;
        void *ws = stream_workspace(s, need);
        if (!ws) return QLD_E_NOMEM;
        a.part_sum = static_cast<uint32_t *>(ws);
        a.part_sat = a.part_sum + (size_t)n_waves * n_frames;
    }
    const int64_t grid = ceil_div(n_tiles, kXcds) * kXcds * n_split;
    if (grid > 0x7fffffff) {
        set_error("grid too large");
        return QLD_E_SHAPE;
    }

    hipEvent_t ev0, ev1;
    take_kernel_timer(&ev0, &ev1);
    if (ev0) QLD_TRY(check_hip(hipEventRecord(ev0, s), "timer start"));
    hipError_t e;
    if (eb == 2) {
        if (vec) e = stats ? launch_accum<2, 8, true, true>(a, (int)grid, s) : launch_accum<2, 8, true, false>(a, (int)grid, s);
        else e = stats ? launch_accum<2, 1, false, true>(a, (int)grid, s) : launch_accum<2, 1, false, false>(a, (int)grid, s);
    } else {
        if (vec) e = stats ? launch_accum<1, 16, true, true>(a, (int)grid, s) : launch_accum<1, 16, true, false>(a, (int)grid, s);
        else e = stats ? launch_accum<1, 1, false, true>(a, (int)grid, s) : launch_accum<1, 1, false, false>(a, (int)grid, s);
    }
    QLD_TRY(check_hip(e, "qld_accum_kernel launch"));
    if (ev1) QLD_TRY(check_hip(hipEventRecord(ev1, s), "timer stop"));
    if (stats) {
        dim3 g2((unsigned)ceil_div(n_frames, 64), (unsigned)ceil_div(n_waves, kRowsPerBlock));
        hipLaunchKernelGGL(qld_stats_reduce_kernel, g2, dim3(64), 0, s, a.part_sum, a.part_sat, n_waves,
                           n_frames, frame_sum, frame_sat);
        QLD_TRY(check_hip(hipGetLastError(), "qld_stats_reduce_kernel launch"));
    }
    return QLD_OK;
}

extern "C" qld_status qld_amplitude(const int32_t *I, const int32_t *Q, int64_t n_pixels, float *amp,
                                    qld_hip_stream stream) {
    clear_error();
    if (n_pixels < 0) {
        set_error("n_pixels < 0");
        return QLD_E_INVAL;
    }
    if (n_pixels == 0) return QLD_OK;
    if (!I || !Q || !amp) {
        set_error("I, Q and amp must be non-NULL");
        return QLD_E_INVAL;
    }
    const int64_t blocks = std::min<int64_t>(ceil_div(n_pixels, 256), 16ll * device_cu_count());
    hipLaunchKernelGGL(qld_amplitude_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), I, Q, n_pixels, amp);
    return check_hip(hipGetLastError(), "qld_amplitude_kernel launch");
}
