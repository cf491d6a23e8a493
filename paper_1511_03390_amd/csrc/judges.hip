// Judges and the learned path's input/target preparation.
//
// CNR follows the paper's Eq. CNR (Methods, "Estimation of contrast-to-noise
// ratio"): (mean over the source - mean over the surround) divided by the RMS
// of the surround about its own mean.  NRMSE(x) = RMS(x - ref) / RMS(ref) per
// tile.  Both reduce in double precision with a fixed order (chunks of a tile
// reduced by work-group trees, then the chunks added in order), so results are
// deterministic.
//
// Learned-path preparation (not in the paper):
//   b      = mean sample level of a window = sum / (H W 4 M)
//   x      = (I_S, Q_S) / (sqrt(2 b_S) sqrt(M_S))     network input
//   scale  = sqrt(2 b_S) / sqrt(M_S)                   per-cycle amplitude per network unit
//   t      = sqrt(max(I_L^2 + Q_L^2 - 4 M_L b_L, 0)) / M_L / scale
//            (the long-window amplitude with its noise power removed)
//   a*     = |(lambda_0 - lambda_2, lambda_1 - lambda_3)|, the per-cycle lock-in
//            amplitude of the noise-free rates
#include "qld_internal.hpp"

namespace qld {
namespace {

// x = (I, Q) / sqrt(P / 2) per pixel (0 where P = 0); scale = sigma / sqrt(M),
// sigma^2 = 2 * the tile's mean sample level.
__global__ void prepare_kernel(const int32_t *__restrict__ I, const int32_t *__restrict__ Q,
                               const uint32_t *__restrict__ psum, const unsigned long long *__restrict__ sum,
                               int32_t M, int64_t npx, float *__restrict__ x, float *__restrict__ scale) {
    const int b = blockIdx.y;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double mean = (double)sum[b] / (double)(npx * 4 * (int64_t)M);
        scale[b] = (float)(sqrt(2.0 * mean) / sqrt((double)M));
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += stride) {
        const int64_t o = (int64_t)b * npx + p;
        const double den = sqrt((double)psum[o] * 0.5);
        const bool ok = den > 0.0;
        x[2 * o] = ok ? (float)((double)I[o] / den) : 0.0f;
        x[2 * o + 1] = ok ? (float)((double)Q[o] / den) : 0.0f;
    }
}

// t = sqrt(max(I^2 + Q^2 - P, 0)) / M / scale per pixel, P the pixel's sample sum.
__global__ void target_kernel(const int32_t *__restrict__ I, const int32_t *__restrict__ Q,
                              const uint32_t *__restrict__ psum, int32_t M, const float *__restrict__ scale,
                              int64_t npx, float *__restrict__ t) {
    const int b = blockIdx.y;
    const double sc = (double)scale[b];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += stride) {
        const int64_t o = (int64_t)b * npx + p;
        const double i = I[o], q = Q[o];
        const double r2 = i * i + q * q - (double)psum[o];
        t[o] = (float)(sqrt(r2 > 0.0 ? r2 : 0.0) / (double)M / sc);
    }
}

__global__ void clean_kernel(const uint8_t *__restrict__ mask, const double *__restrict__ rates, int64_t npx,
                             float *__restrict__ a) {
    const int b = blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += stride) {
        const int64_t o = (int64_t)b * npx + p;
        const double *r = rates + (int64_t)b * 8 + (mask[o] ? 4 : 0);
        const double i = r[0] - r[2], q = r[1] - r[3];
        a[o] = (float)sqrt(i * i + q * q);
    }
}

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double (*red)[256]) {
#pragma unroll
    for (int k = 0; k < N; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
#pragma unroll
            for (int k = 0; k < N; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = red[k][0];
}

// Two-stage fixed-order reductions: stage 1 splits each tile into `chunks`
// contiguous pieces (enough work-groups to fill the GPU for any batch), each
// reduced by a work-group tree into double partials; stage 2 adds a tile's
// partials in chunk order.  The result depends only on (B, n), never on timing.
constexpr int kJudgeBlocks = 1024;   // target work-groups of stage 1
constexpr int kMaxChunks = 256;

int judge_chunks(int B, int64_t n) {
    const int64_t want = std::min<int64_t>(std::max<int64_t>(1, ceil_div(kJudgeBlocks, B)), kMaxChunks);
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, ceil_div(n, 1024)));
}

__global__ __launch_bounds__(256) void nrmse_part_kernel(const float *__restrict__ x, const float *__restrict__ scale,
                                                         const float *__restrict__ ref, int64_t n, int chunks,
                                                         double *__restrict__ part) {
    __shared__ double red[2][256];
    const int b = blockIdx.y, ch = blockIdx.x;
    const int64_t per = ceil_div(n, (int64_t)chunks);
    const int64_t p0 = ch * per, p1 = std::min<int64_t>(n, p0 + per);
    const double sc = scale ? (double)scale[b] : 1.0;
    const float *xb = x + (int64_t)b * n, *rb = ref + (int64_t)b * n;
    double v[2] = {0.0, 0.0};
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
        const double r = rb[p];
        const double d = (double)xb[p] * sc - r;
        v[0] += d * d;
        v[1] += r * r;
    }
    block_sum<2>(v, red);
    if (threadIdx.x == 0) {
        part[((int64_t)b * chunks + ch) * 2] = v[0];
        part[((int64_t)b * chunks + ch) * 2 + 1] = v[1];
    }
}

__global__ void nrmse_final_kernel(const double *__restrict__ part, int chunks, int B, float *__restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    // Chunks in order; loads issued 16 chunks at a time.
    const double *pb = part + (int64_t)b * chunks * 2;
    double e = 0.0, r = 0.0;
    int c = 0;
    for (; c + 16 <= chunks; c += 16) {
        double ve[16], vr[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            ve[i] = pb[(int64_t)(c + i) * 2];
            vr[i] = pb[(int64_t)(c + i) * 2 + 1];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            e += ve[i];
            r += vr[i];
        }
    }
    for (; c < chunks; ++c) {
        e += pb[(int64_t)c * 2];
        r += pb[(int64_t)c * 2 + 1];
    }
    out[b] = r > 0.0 ? (float)sqrt(e / r) : 0.0f;
}

__global__ __launch_bounds__(256) void cnr_part_kernel(const float *__restrict__ img, const uint8_t *__restrict__ lab,
                                                       int64_t n, int chunks, double *__restrict__ part) {
    __shared__ double red[5][256];
    const int b = blockIdx.y, ch = blockIdx.x;
    const int64_t per = ceil_div(n, (int64_t)chunks);
    const int64_t p0 = ch * per, p1 = std::min<int64_t>(n, p0 + per);
    const float *ib = img + (int64_t)b * n;
    const uint8_t *lb = lab + (int64_t)b * n;
    double v[5] = {0, 0, 0, 0, 0};   // sum_src, n_src, sum_surr, sum_surr^2, n_surr
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
        const uint8_t l = lb[p];
        const double z = ib[p];
        if (l == 1) {
            v[0] += z;
            v[1] += 1.0;
        } else if (l == 2) {
            v[2] += z;
            v[3] += z * z;
            v[4] += 1.0;
        }
    }
    block_sum<5>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < 5; ++k) part[((int64_t)b * chunks + ch) * 5 + k] = v[k];
}

__global__ void cnr_final_kernel(const double *__restrict__ part, int chunks, int B, float *__restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double v[5] = {0, 0, 0, 0, 0};
    for (int c = 0; c < chunks; ++c)
#pragma unroll
        for (int k = 0; k < 5; ++k) v[k] += part[((int64_t)b * chunks + c) * 5 + k];
    const double ms = v[0] / v[1], mr = v[2] / v[4];
    const double var = v[3] / v[4] - mr * mr;
    out[b] = (v[1] > 0 && v[4] > 0 && var > 0) ? (float)((ms - mr) / sqrt(var)) : 0.0f;
}

dim3 pix_grid(int64_t npx, int B) { return dim3((unsigned)std::min<int64_t>(ceil_div(npx, 256), 1024), (unsigned)B); }

}  // namespace
}  // namespace qld

using namespace qld;

extern "C" qld_status qld_denoise_prepare(const int32_t *I_S, const int32_t *Q_S, const uint32_t *psum_S,
                                          const uint64_t *sum_S, int32_t M_S, int32_t B, int32_t H, int32_t W,
                                          float *x, float *scale, qld_hip_stream stream) {
    clear_error();
    if (!I_S || !Q_S || !psum_S || !sum_S || !x || !scale || M_S < 1 || B < 1 || B > 65535 || H < 1 || W < 1) {
        set_error("prepare: bad arguments");
        return QLD_E_INVAL;
    }
    const int64_t npx = (int64_t)H * W;
    hipLaunchKernelGGL(prepare_kernel, pix_grid(npx, B), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), I_S, Q_S,
                       psum_S, reinterpret_cast<const unsigned long long *>(sum_S), M_S, npx, x, scale);
    return check_hip(hipGetLastError(), "prepare_kernel launch");
}

extern "C" qld_status qld_denoise_target(const int32_t *I_L, const int32_t *Q_L, const uint32_t *psum_L, int32_t M_L,
                                         const float *scale, int32_t B, int32_t H, int32_t W, float *t,
                                         qld_hip_stream stream) {
    clear_error();
    if (!I_L || !Q_L || !psum_L || !scale || !t || M_L < 1 || B < 1 || B > 65535 || H < 1 || W < 1) {
        set_error("target: bad arguments");
        return QLD_E_INVAL;
    }
    const int64_t npx = (int64_t)H * W;
    hipLaunchKernelGGL(target_kernel, pix_grid(npx, B), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), I_L, Q_L,
                       psum_L, M_L, scale, npx, t);
    return check_hip(hipGetLastError(), "target_kernel launch");
}

extern "C" qld_status qld_clean_amplitude(const uint8_t *mask, const double *rates_host, int32_t B, int32_t H,
                                          int32_t W, float *a, qld_hip_stream stream) {
    clear_error();
    if (!mask || !rates_host || !a || B < 1 || B > 65535 || H < 1 || W < 1) {
        set_error("clean amplitude: bad arguments");
        return QLD_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double *r = static_cast<double *>(stream_workspace(s, sizeof(double) * 8 * (size_t)B));
    if (!r) return QLD_E_NOMEM;
    QLD_TRY(check_hip(hipMemcpyAsync(r, rates_host, sizeof(double) * 8 * (size_t)B, hipMemcpyHostToDevice, s),
                      "rates upload"));
    const int64_t npx = (int64_t)H * W;
    hipLaunchKernelGGL(clean_kernel, pix_grid(npx, B), dim3(256), 0, s, mask, r, npx, a);
    return check_hip(hipGetLastError(), "clean_kernel launch");
}

extern "C" qld_status qld_judge_nrmse(const float *x, const float *scale, const float *ref, int32_t B, int64_t n,
                                      float *out, qld_hip_stream stream) {
    clear_error();
    if (!x || !ref || !out || B < 0 || B > 65535 || n < 0) {
        set_error("nrmse: bad arguments");
        return QLD_E_INVAL;
    }
    if (B == 0) return QLD_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int chunks = judge_chunks(B, n);
    double *part = static_cast<double *>(stream_workspace(s, sizeof(double) * 2 * (size_t)B * chunks));
    if (!part) return QLD_E_NOMEM;
    hipLaunchKernelGGL(nrmse_part_kernel, dim3(chunks, B), dim3(256), 0, s, x, scale, ref, n, chunks, part);
    hipLaunchKernelGGL(nrmse_final_kernel, dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, s, part, chunks, B, out);
    return check_hip(hipGetLastError(), "nrmse launch");
}

extern "C" qld_status qld_judge_cnr(const float *img, const uint8_t *labels, int32_t B, int64_t n, float *out,
                                    qld_hip_stream stream) {
    clear_error();
    if (!img || !labels || !out || B < 0 || B > 65535 || n < 0) {
        set_error("cnr: bad arguments");
        return QLD_E_INVAL;
    }
    if (B == 0) return QLD_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int chunks = judge_chunks(B, n);
    double *part = static_cast<double *>(stream_workspace(s, sizeof(double) * 5 * (size_t)B * chunks));
    if (!part) return QLD_E_NOMEM;
    hipLaunchKernelGGL(cnr_part_kernel, dim3(chunks, B), dim3(256), 0, s, img, labels, n, chunks, part);
    hipLaunchKernelGGL(cnr_final_kernel, dim3((unsigned)ceil_div(B, 64)), dim3(64), 0, s, part, chunks, B, out);
    return check_hip(hipGetLastError(), "cnr launch");
}
