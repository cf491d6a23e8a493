// Per-cycle kernels of a LEARNED serving stream (not in the paper): the
// sample sums that normalise the denoiser's input, and the gate's choice
// between the denoiser's image and the plain long-window amplitude.
//
// The denoiser's input divides each pixel's short-window I/Q by that pixel's
// noise level, estimated from its sample sum over the last M_short cycles;
// the output scale uses the frame's mean level over the same cycles.  Each
// cycle's four staged frames are summed once per pixel into a ring of
// per-pixel cycle sums, and once per work-group into a ring of partials; a
// window's sums are then exact integer sums over M_short ring entries (the
// frame's in a fixed order), so the results do not depend on scheduling.
#include "serve_learned.hpp"

namespace qld {
namespace {

typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    return lds[0];
}

// Grid (nblk, n_cycles).  Cycle i of the job is staged in slot (stage0 + i) %
// n_stage: 4 frames of slot_b / 4 bytes each, rows zero-padded to 16 bytes, so
// the whole slot is summed as 16-byte words (padding adds nothing).
__global__ __launch_bounds__(kThreads) void cycle_sum_kernel(const uint8_t *__restrict__ stage, int64_t slot_b,
                                                             int n_stage, int stage0, int eb, uint64_t *csum,
                                                             int ring, int64_t c0, int nblk) {
    __shared__ uint64_t lds[kThreads];
    const int i = blockIdx.y;
    const u32x4v *src = reinterpret_cast<const u32x4v *>(stage + (int64_t)((stage0 + i) % n_stage) * slot_b);
    const int64_t nwords = slot_b / 16;
    uint64_t acc = 0;
    for (int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x; w < nwords; w += (int64_t)nblk * kThreads) {
        const u32x4v v = src[w];
        uint32_t part = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t x = v[k];
            part += eb == 2 ? (x & 0xFFFFu) + (x >> 16)
                            : (x & 0xFFu) + ((x >> 8) & 0xFFu) + ((x >> 16) & 0xFFu) + (x >> 24);
        }
        acc += part;
    }
    const uint64_t tot = block_sum_u64(acc, lds);
    if (threadIdx.x == 0) csum[((c0 + i) % ring) * nblk + blockIdx.x] = tot;
}

// One work-group: sumS = partials of cycles c_last - Ms + 1 .. c_last, in order.
__global__ __launch_bounds__(kThreads) void window_sum_kernel(const uint64_t *__restrict__ csum, int ring, int nblk,
                                                              int64_t c_last, int Ms, uint64_t *sumS) {
    __shared__ uint64_t lds[kThreads];
    const int64_t n = (int64_t)Ms * nblk;
    uint64_t acc = 0;
    for (int64_t k = threadIdx.x; k < n; k += kThreads) {
        const int64_t c = c_last - Ms + 1 + k / nblk;
        acc += csum[(c % ring) * nblk + k % nblk];
    }
    const uint64_t tot = block_sum_u64(acc, lds);
    if (threadIdx.x == 0) sumS[0] = tot;
}

// Grid (ceil(H * W / 256), n_cycles): one lane per pixel, the four frames of
// its cycle added in uint32.
__global__ __launch_bounds__(kThreads) void pixel_cycle_sum_kernel(const uint8_t *__restrict__ stage, int64_t slot_b,
                                                                   int64_t fs_b, int64_t rp_b, int n_stage,
                                                                   int stage0, int eb, int H, int W,
                                                                   uint32_t *__restrict__ pcs, int ring, int64_t c0) {
    const int i = blockIdx.y;
    const int64_t npx = (int64_t)H * W;
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= npx) return;
    const int64_t y = p / W, x = p % W;
    const uint8_t *src = stage + (int64_t)((stage0 + i) % n_stage) * slot_b + y * rp_b + x * eb;
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        acc += eb == 2 ? (uint32_t)*reinterpret_cast<const uint16_t *>(src + j * fs_b) : (uint32_t)src[j * fs_b];
    pcs[((c0 + i) % ring) * npx + p] = acc;
}

// psum[p] = pcs[c][p] summed over window cycles c = c_last - Ms + 1 .. c_last.
__global__ __launch_bounds__(kThreads) void pixel_window_sum_kernel(const uint32_t *__restrict__ pcs, int ring,
                                                                    int64_t npx, int64_t c_last, int Ms,
                                                                    uint32_t *__restrict__ psum) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < npx; p += stride) {
        uint32_t acc = 0;
        for (int k = 0; k < Ms; ++k) acc += pcs[((c_last - Ms + 1 + k) % ring) * npx + p];
        psum[p] = acc;
    }
}

// served = gate <= thr ? y * scale : plain * inv_n.  gate NULL: the denoiser
// did not run (short window not full): plain, gate recorded as NaN.
__global__ __launch_bounds__(kThreads) void serve_kernel(const float *__restrict__ y, const float *__restrict__ scale,
                                                         const float *__restrict__ gate,
                                                         const float *__restrict__ plain, int64_t npx, float thr,
                                                         float inv_n, float *__restrict__ served, float *gate_slot) {
    const float g = gate ? gate[0] : __builtin_nanf("");
    const bool use = gate && g <= thr;
    const float sc = use ? scale[0] : 0.0f;
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < npx; p += (int64_t)gridDim.x * kThreads)
        served[p] = use ? y[p] * sc : plain[p] * inv_n;
    if (blockIdx.x == 0 && threadIdx.x == 0) gate_slot[0] = g;
}

}  // namespace

hipError_t launch_cycle_sums(const uint8_t *stage, int64_t slot_b, int n_stage, int stage0, int n_cycles, int eb,
                             uint64_t *csum, int ring, int64_t c0, int nblk, hipStream_t s) {
    if (n_cycles < 1) return hipSuccess;
    hipLaunchKernelGGL(cycle_sum_kernel, dim3(nblk, n_cycles), dim3(kThreads), 0, s, stage, slot_b, n_stage, stage0,
                       eb, csum, ring, c0, nblk);
    return hipGetLastError();
}

hipError_t launch_window_sum(const uint64_t *csum, int ring, int nblk, int64_t c_last, int Ms, uint64_t *sumS,
                             hipStream_t s) {
    hipLaunchKernelGGL(window_sum_kernel, dim3(1), dim3(kThreads), 0, s, csum, ring, nblk, c_last, Ms, sumS);
    return hipGetLastError();
}

hipError_t launch_pixel_cycle_sums(const uint8_t *stage, int64_t slot_b, int64_t fs_b, int64_t rp_b, int n_stage,
                                   int stage0, int n_cycles, int eb, int H, int W, uint32_t *pcs, int ring,
                                   int64_t c0, hipStream_t s) {
    const int64_t npx = (int64_t)H * W;
    if (n_cycles < 1 || npx == 0) return hipSuccess;
    hipLaunchKernelGGL(pixel_cycle_sum_kernel, dim3((unsigned)ceil_div(npx, kThreads), n_cycles), dim3(kThreads), 0,
                       s, stage, slot_b, fs_b, rp_b, n_stage, stage0, eb, H, W, pcs, ring, c0);
    return hipGetLastError();
}

hipError_t launch_pixel_window_sum(const uint32_t *pcs, int ring, int64_t npx, int64_t c_last, int Ms, uint32_t *psum,
                                   hipStream_t s) {
    if (npx == 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(npx, kThreads), 4096);
    hipLaunchKernelGGL(pixel_window_sum_kernel, dim3(g), dim3(kThreads), 0, s, pcs, ring, npx, c_last, Ms, psum);
    return hipGetLastError();
}

hipError_t launch_serve(const float *y, const float *scale, const float *gate, const float *plain, int64_t npx,
                        float thr, float inv_n, float *served, float *gate_slot, hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(npx, kThreads), 2048);
    hipLaunchKernelGGL(serve_kernel, dim3(g), dim3(kThreads), 0, s, y, scale, gate, plain, npx, thr, inv_n, served,
                       gate_slot);
    return hipGetLastError();
}

}  // namespace qld
