// Single-bin DFT of every pixel's series: the Fourier discrimination that QLD
// replaces (paper: Methods, the map of |F(j,k,omega)|^2 at the frequency of
// interest; section "Processing Time and Speedup", Fourier decomposition as a
// series of lock-ins at different frequencies).
//
//     X_k(y,x) = sum_{n<N} S_n(y,x) exp(-2 pi i ((k n) mod N) / N),  N = n_frames
//
// Same memory layout and lane mapping as the QLD accumulation (one 16-byte
// load per lane per frame), but with multiply-adds against a twiddle table
// instead of integer adds.  The table is built per call by a small kernel in
// double precision from the exact integer angle (k n) mod N (sincospi, so
// quarter turns are exact) and rounded to the accumulation type: float, or
// double for the FP64 variant (the paper computes in double).  Frame chunks
// write partials that a second kernel sums in fixed chunk order, so the
// result is deterministic.
#include "qld_internal.hpp"

namespace qld {
namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;
// With four frames in flight per wave, two work-groups per CU stream best
// (measured at 1024 frames of 1024 x 1024 uint16: 75-79% of HBM peak versus
// 67-68% at three or four).
#ifndef QLD_DFT_BLOCKS_PER_CU
#define QLD_DFT_BLOCKS_PER_CU 2
#endif

// R = float or double: the twiddle and accumulation type.
template <typename R>
struct alignas(2 * sizeof(R)) Tw2 {
    R c, s;
};

template <typename R>
struct DftArgs {
    const uint8_t *frames;
    int64_t rp_b, fs_b;
    int32_t H, W;
    int32_t n_frames;
    int32_t chunk, n_split;
    int32_t nvx, n_tiles;
    const Tw2<R> *tw;       // [N] (cos, sin)
    R *re, *im;             // final outputs [H][W] (n_split == 1)
    R *part;                // [n_split][2][H*W] (n_split > 1)
};

__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// tw[n] = (cos, sin)(2 pi r / period), r = (k (t0 + n)) mod period, n < n_frames.
template <typename R>
__global__ __launch_bounds__(256) void dft_twiddle_kernel(int32_t n_frames, int32_t period, int32_t k, int32_t t0,
                                                          Tw2<R> *tw) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_frames) return;
    const int64_t r = (((int64_t)k * ((int64_t)t0 + n)) % period + period) % period;
    double s, c;
    sincospi(2.0 * (double)r / (double)period, &s, &c);
    tw[n] = Tw2<R>{(R)c, (R)s};
}

// A lane's VPX samples of one frame: one 16-byte load (VECLOAD), or element
// by element for the row-tail lane and unaligned stacks.
template <int ELEM, int VPX, bool VECLOAD, typename R>
__device__ __forceinline__ void load_f(const uint8_t *p, int nvalid, R (&v)[VPX]) {
    if constexpr (VECLOAD) {
        const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        const uint32_t w[4] = {q[0], q[1], q[2], q[3]};
        if constexpr (ELEM == 2) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[2 * j] = (R)(w[j] & 0xffffu);
                v[2 * j + 1] = (R)(w[j] >> 16);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[4 * j] = (R)(w[j] & 0xffu);
                v[4 * j + 1] = (R)((w[j] >> 8) & 0xffu);
                v[4 * j + 2] = (R)((w[j] >> 16) & 0xffu);
                v[4 * j + 3] = (R)(w[j] >> 24);
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < VPX; ++j) {
            if (j < nvalid) {
                if constexpr (ELEM == 2) v[j] = (R)reinterpret_cast<const uint16_t *>(p)[j];
                else v[j] = (R)p[j];
            } else {
                v[j] = (R)0;
            }
        }
    }
}

// Frames t0 .. t1-1 of one lane into (re, im) += S_t (cos, sin).  With vector
// loads the four loads of an iteration are kept together ahead of the
// arithmetic, so a wave has four frames in flight.
template <int ELEM, int VPX, bool VECLOAD, typename R>
__device__ __forceinline__ void dft_frames(const Tw2<R> *__restrict__ tw, const uint8_t *p, int64_t fs, int64_t t0,
                                           int64_t t1, int nvalid, R (&re)[VPX], R (&im)[VPX]) {
    int64_t t = t0;
    for (; t + 4 <= t1; t += 4) {
        R v0[VPX], v1[VPX], v2[VPX], v3[VPX];
        load_f<ELEM, VPX, VECLOAD>(p, nvalid, v0);
        load_f<ELEM, VPX, VECLOAD>(p + fs, nvalid, v1);
        load_f<ELEM, VPX, VECLOAD>(p + 2 * fs, nvalid, v2);
        load_f<ELEM, VPX, VECLOAD>(p + 3 * fs, nvalid, v3);
        if constexpr (VECLOAD) __builtin_amdgcn_sched_barrier(0);
        p += 4 * fs;
        const Tw2<R> w0 = tw[t], w1 = tw[t + 1], w2 = tw[t + 2], w3 = tw[t + 3];
#pragma unroll
        for (int j = 0; j < VPX; ++j) {
            re[j] = fma_r(v0[j], w0.c, re[j]);
            im[j] = fma_r(v0[j], w0.s, im[j]);
            re[j] = fma_r(v1[j], w1.c, re[j]);
            im[j] = fma_r(v1[j], w1.s, im[j]);
            re[j] = fma_r(v2[j], w2.c, re[j]);
            im[j] = fma_r(v2[j], w2.s, im[j]);
            re[j] = fma_r(v3[j], w3.c, re[j]);
            im[j] = fma_r(v3[j], w3.s, im[j]);
        }
    }
    for (; t < t1; ++t) {
        R v[VPX];
        load_f<ELEM, VPX, VECLOAD>(p, nvalid, v);
        p += fs;
        const Tw2<R> w = tw[t];
#pragma unroll
        for (int j = 0; j < VPX; ++j) {
            re[j] = fma_r(v[j], w.c, re[j]);
            im[j] = fma_r(v[j], w.s, im[j]);
        }
    }
}

template <int ELEM, int VPX, bool VEC, typename R>
__global__ __launch_bounds__(kBlock) void dft_bin_kernel(DftArgs<R> a) {
    const int b = blockIdx.x;
    const int xcd = b % kXcds;
    const int q = b / kXcds;
    const int split = q % a.n_split;
    const int tile = (q / a.n_split) * kXcds + xcd;
    if (tile >= a.n_tiles) return;

    const int64_t g = (int64_t)tile * kBlock + threadIdx.x;
    const int64_t y = g / a.nvx;
    const int x0 = (int)(g % a.nvx) * VPX;
    if (y >= a.H) return;
    const int nvalid = min(VPX, a.W - x0);
    const bool full = nvalid == VPX;

    const int64_t t0 = (int64_t)split * a.chunk;
    const int64_t t1 = min((int64_t)a.n_frames, t0 + a.chunk);
    const uint8_t *p = a.frames + y * a.rp_b + (int64_t)x0 * ELEM + t0 * a.fs_b;
    const int64_t fs = a.fs_b;

    R re[VPX], im[VPX];
#pragma unroll
    for (int j = 0; j < VPX; ++j) re[j] = im[j] = (R)0;

    // Full lanes stream with vector loads; only the lane at a row's ragged end
    // (or an unaligned stack) reads element by element.
    if constexpr (VEC) {
        if (full) dft_frames<ELEM, VPX, true>(a.tw, p, fs, t0, t1, nvalid, re, im);
        else dft_frames<ELEM, VPX, false>(a.tw, p, fs, t0, t1, nvalid, re, im);
    } else {
        dft_frames<ELEM, VPX, false>(a.tw, p, fs, t0, t1, nvalid, re, im);
    }

    const int64_t npx = (int64_t)a.H * a.W;
    const int64_t o = y * a.W + x0;
    R *dre = a.n_split > 1 ? a.part + (int64_t)split * 2 * npx : a.re;
    R *dim = a.n_split > 1 ? a.part + (int64_t)split * 2 * npx + npx : a.im;
#pragma unroll
    for (int j = 0; j < VPX; ++j) {
        if (j < nvalid) {
            dre[o + j] = re[j];
            dim[o + j] = -im[j];   // exp(-i theta) = cos - i sin
        }
    }
}

template <typename R>
__global__ __launch_bounds__(256) void dft_split_reduce_kernel(const R *__restrict__ part, int32_t n_split,
                                                               int64_t npx, R *__restrict__ re,
                                                               R *__restrict__ im) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npx; i += stride) {
        R r = (R)0, m = (R)0;
        for (int s = 0; s < n_split; ++s) {
            r += part[(int64_t)s * 2 * npx + i];
            m += part[(int64_t)s * 2 * npx + npx + i];
        }
        re[i] = r;
        im[i] = m;
    }
}

template <int ELEM, int VPX, bool VEC, typename R>
hipError_t launch_dft(const DftArgs<R> &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((dft_bin_kernel<ELEM, VPX, VEC, R>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace
}  // namespace qld

using namespace qld;

namespace {

// X = sum_{n < n_frames} S_n exp(-2 pi i ((k (t0 + n)) mod period) / period), in R.
template <typename R>
qld_status single_frequency(const void *frames, const qld_frame_desc *d, int32_t n_frames, int32_t k,
                            int32_t period, int32_t t0, R *re, R *im, qld_hip_stream stream) {
    int eb = 0;
    QLD_TRY(check_desc(d, &eb));
    const int64_t npx = (int64_t)d->H * d->W;
    if (npx == 0) return QLD_OK;
    if (!frames || !re || !im) {
        set_error("frames, re and im must be non-NULL");
        return QLD_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uintptr_t base = reinterpret_cast<uintptr_t>(frames);
    const int64_t rp_b = d->row_pitch * eb, fs_b = d->frame_stride * eb;
    const bool vec = (base % 16 == 0) && (rp_b % 16 == 0) && (fs_b % 16 == 0);
    const int vpx = vec ? 16 / eb : 1;

    DftArgs<R> a{};
    a.frames = static_cast<const uint8_t *>(frames);
    a.rp_b = rp_b;
    a.fs_b = fs_b;
    a.H = d->H;
    a.W = d->W;
    a.n_frames = n_frames;
    a.nvx = (int32_t)ceil_div(d->W, vpx);
    const int64_t n_tiles = ceil_div((int64_t)a.nvx * d->H, kBlock);
    if (n_tiles > (1ll << 24)) {
        set_error("image too large");
        return QLD_E_SHAPE;
    }
    a.n_tiles = (int32_t)n_tiles;
    // Same grid policy as the lock-in accumulation: split the frame axis only
    // until the grid holds QLD_DFT_BLOCKS_PER_CU work-groups per CU.
    const int64_t want_blocks = (int64_t)QLD_DFT_BLOCKS_PER_CU * device_cu_count();
    int64_t n_split = 1;
    if (n_tiles < want_blocks) n_split = ceil_div(want_blocks, n_tiles);
    n_split = std::max<int64_t>(1, std::min<int64_t>(n_split, n_frames / 64));
    int64_t chunk = ceil_div(n_frames, n_split);
    n_split = ceil_div(n_frames, chunk);
    a.chunk = (int32_t)chunk;
    a.n_split = (int32_t)n_split;

    size_t tw_bytes = sizeof(Tw2<R>) * (size_t)n_frames;
    size_t part_bytes = n_split > 1 ? sizeof(R) * 2 * (size_t)n_split * (size_t)npx : 0;
    char *ws = static_cast<char *>(stream_workspace(s, tw_bytes + 256 + part_bytes));
    if (!ws) return QLD_E_NOMEM;
    Tw2<R> *tw = reinterpret_cast<Tw2<R> *>(ws);
    a.tw = tw;
    a.part = n_split > 1 ? reinterpret_cast<R *>(ws + ((tw_bytes + 255) / 256) * 256) : nullptr;
    a.re = re;
    a.im = im;

    hipLaunchKernelGGL(dft_twiddle_kernel<R>, dim3((unsigned)ceil_div(n_frames, 256)), dim3(256), 0, s, n_frames,
                       period, k, t0, tw);
    QLD_TRY(check_hip(hipGetLastError(), "dft_twiddle_kernel launch"));
    const int64_t grid = ceil_div(n_tiles, kXcds) * kXcds * n_split;
    hipEvent_t ev0, ev1;
    take_kernel_timer(&ev0, &ev1);
    if (ev0) QLD_TRY(check_hip(hipEventRecord(ev0, s), "timer start"));
    hipError_t e;
    if (eb == 2) e = vec ? launch_dft<2, 8, true>(a, (int)grid, s) : launch_dft<2, 1, false>(a, (int)grid, s);
    else e = vec ? launch_dft<1, 16, true>(a, (int)grid, s) : launch_dft<1, 1, false>(a, (int)grid, s);
    QLD_TRY(check_hip(e, "dft_bin_kernel launch"));
    if (ev1) QLD_TRY(check_hip(hipEventRecord(ev1, s), "timer stop"));
    if (n_split > 1) {
        const int64_t blocks = std::min<int64_t>(ceil_div(npx, 256), 16ll * device_cu_count());
        hipLaunchKernelGGL(dft_split_reduce_kernel<R>, dim3((unsigned)blocks), dim3(256), 0, s, a.part,
                           (int32_t)n_split, npx, re, im);
        QLD_TRY(check_hip(hipGetLastError(), "dft_split_reduce_kernel launch"));
    }
    return QLD_OK;
}

}  // namespace

extern "C" qld_status dft_bin_baseline(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                                       int32_t k_bin, float *re, float *im, qld_hip_stream stream) {
    clear_error();
    if (n_frames < 1) {
        set_error("dft_bin_baseline needs n_frames >= 1 (got %d)", n_frames);
        return QLD_E_SHAPE;
    }
    return single_frequency(frames, d, n_frames, k_bin, n_frames, 0, re, im, stream);
}

extern "C" qld_status dft_bin_baseline_f64(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                                           int32_t k_bin, double *re, double *im, qld_hip_stream stream) {
    clear_error();
    if (n_frames < 1) {
        set_error("dft_bin_baseline_f64 needs n_frames >= 1 (got %d)", n_frames);
        return QLD_E_SHAPE;
    }
    return single_frequency(frames, d, n_frames, k_bin, n_frames, 0, re, im, stream);
}

extern "C" qld_status qld_lockin_ratio(const void *frames, const qld_frame_desc *d, int32_t n_frames, int32_t p,
                                       int32_t q, int32_t t0, float *re, float *im, qld_hip_stream stream) {
    clear_error();
    if (n_frames < 1) {
        set_error("qld_lockin_ratio needs n_frames >= 1 (got %d)", n_frames);
        return QLD_E_SHAPE;
    }
    if (q < 1 || t0 < 0) {
        set_error("qld_lockin_ratio needs q >= 1 and t0 >= 0 (got q=%d, t0=%d)", q, t0);
        return QLD_E_INVAL;
    }
    return single_frequency(frames, d, n_frames, p, q, t0, re, im, stream);
}
