// Learned short-window denoiser: 4 conv3x3 layers (2 -> 32 -> 32 -> 32 -> 1),
// bias and ReLU between layers, zero "same" padding, trained on pairs the
// lock-in itself generates (short-window I/Q in, long-window amplitude out).
// Not in the paper: it lets fewer frames reach the image quality of a longer
// plain lock-in, with plain QLD as its fallback (gate) and its judge.
//
// Layout: activations NHWC bfloat16 [B][H][W][32]; weights fp32 master copy in
// a canonical order, packed to bfloat16 operand layouts after every update.
// Convolutions are implicit GEMMs on the matrix cores
// (v_mfma_f32_16x16x32_bf16, fp32 accumulation): a work-group stages its
// input tile in LDS once and each lane keeps its weight fragments of all nine
// taps in registers.  The same kernel, with the tap offsets negated and the
// weights transposed, computes the gradient with respect to the input; the
// 1-channel output layer is the same kernel with one zero-padded 16-column
// weight block.  Weight gradients are MFMA reductions over pixels (K = 32
// pixels per step; operands staged transposed in LDS, the bias gradients
// summed from the same staged tiles) into per-work-group partials that a
// second kernel sums in a fixed order, so training is deterministic.  The
// 2-channel input layer packs its 18 (tap, channel) products into one K = 32
// MFMA; the output layer's weight gradient and the pooling use the VALU.
#include <cstring>
#include <new>
#include <vector>

#include "qld_internal.hpp"

namespace qld {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4c __attribute__((ext_vector_type(4)));

// Canonical parameter order (fp32): W[3][3][Cin][Cout] then b[Cout], per layer; then the gate.
constexpr int64_t OFF_W1 = 0, OFF_B1 = 576, OFF_W2 = 608, OFF_B2 = 9824, OFF_W3 = 9856, OFF_B3 = 19072,
                  OFF_W4 = 19104, OFF_B4 = 19392, OFF_WG = 19393, OFF_BG = 19425, N_ALL = 19426;

constexpr int kRows = 4;        // output rows per work-group (one per wave)
constexpr int kCols = 64;       // output pixels per row and work-group

__device__ __forceinline__ int tap_dy(int t) { return t / 3 - 1; }
__device__ __forceinline__ int tap_dx(int t) { return t % 3 - 1; }

__device__ __forceinline__ f32x4 mfma16(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

// ---------------------------------------------------------------------------
// Weight packing: fp32 canonical -> bf16 operand layouts.
//   w1f [32 co][32 k], k = tap*2 + ch (k < 18), zero elsewhere
//   wNf [9][32 co][32 ci]   forward B operand (K = ci contiguous)
//   wNb [9][32 ci][32 co]   input-gradient B operand (K = co contiguous)
//   w4  [9][32]
//   w4f [9][16][32]  output-layer B operand: row 0 = w4[tap], rows 1..15 zero
// ---------------------------------------------------------------------------
__global__ void pack_kernel(const float *__restrict__ p, __bf16 *w1f, __bf16 *w2f, __bf16 *w2b, __bf16 *w3f,
                            __bf16 *w3b, __bf16 *w4, __bf16 *w4f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 1024) {
        const int co = i / 32, k = i % 32;
        w1f[i] = (__bf16)(k < 18 ? p[OFF_W1 + (k / 2 * 2 + k % 2) * 32 + co] : 0.0f);
    }
    if (i < 9 * 1024) {
        const int t = i / 1024, r = i % 1024;
        const int a = r / 32, b = r % 32;
        // forward: [t][co = a][ci = b]  <- W[t][ci][co]
        w2f[i] = (__bf16)p[OFF_W2 + (t * 32 + b) * 32 + a];
        w3f[i] = (__bf16)p[OFF_W3 + (t * 32 + b) * 32 + a];
        // input gradient: [t][ci = a][co = b] <- W[t][ci][co]
        w2b[i] = (__bf16)p[OFF_W2 + (t * 32 + a) * 32 + b];
        w3b[i] = (__bf16)p[OFF_W3 + (t * 32 + a) * 32 + b];
    }
    if (i < 288) w4[i] = (__bf16)p[OFF_W4 + i];
    if (i < 9 * 512) {
        const int t = i / 512, co = (i / 32) % 16, ci = i % 32;
        w4f[i] = (__bf16)(co == 0 ? p[OFF_W4 + t * 32 + ci] : 0.0f);
    }
}

// Four values per step with a 16-byte load and an 8-byte store when the
// caller's x is 16-byte aligned (y is the denoiser's own buffer), then the
// rest one by one.
__global__ void to_bf16_kernel(const float *__restrict__ x, __bf16 *__restrict__ y, int64_t n) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = (reinterpret_cast<uintptr_t>(x) & 15) == 0 ? n / 4 : 0;
    for (int64_t i = gid; i < n4; i += stride) {
        const f32x4 v = reinterpret_cast<const f32x4 *>(x)[i];
        bf16x4 o;
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = (__bf16)v[k];
        reinterpret_cast<bf16x4 *>(y)[i] = o;
    }
    for (int64_t i = 4 * n4 + gid; i < n; i += stride) y[i] = (__bf16)x[i];
}

// Work-group tile -> (image, first row, first column).
__device__ __forceinline__ bool tile_of(int H, int W, int &b, int &y, int &x0) {
    const int tx = (W + kCols - 1) / kCols, ty = (H + kRows - 1) / kRows;
    int id = blockIdx.x;
    x0 = (id % tx) * kCols;
    id /= tx;
    y = (id % ty) * kRows + (int)(threadIdx.x >> 6);
    b = id / ty;
    return y < H;
}

// ---------------------------------------------------------------------------
// 3x3 convolutions with 32 input channels on the matrix cores (implicit GEMM).
// A tile is 4 output rows x 64 pixels: its input (rows y0-1 .. y0+4, pixels
// x0-1 .. x0+64, 32 channels, zero outside the image; 25 KB) is staged in LDS
// once, each lane keeps its B-operand fragments of all 9 taps in registers,
// and wave w computes output row y0 + w: per tap and group of 16 pixels one
// 16-byte LDS read (a lane's 8 input channels of one pixel; the 64 lanes read
// 1 KiB contiguous) and one MFMA per 16 output channels.
// The grid is persistent: a work-group loads its weights once and walks tiles
// blockIdx.x, + gridDim.x, ...; the next tile's input (7 16-byte loads per
// lane, all issued before any is waited for) is in flight while the current
// tile's products run, so the HBM latency is covered by the loop itself
// rather than by other resident work-groups.
// MODE 0 (forward):        out = bf16(relu(sum_tap in[p + tap] W[tap] + bias))
// MODE 1 (input gradient): out = bf16((sum_tap in[p - tap] W^T[tap]) * (act[p] > 0))
// MODE 2 (output layer):   y   = sum_tap in[p + tap] . w4[tap] + b4 (fp32; the
//                          weights form one 16-column block with column 0 used);
//                          with pool_part, also each wave's channel sums of its
//                          row of the input (the gate's pooling, read from the
//                          LDS tile instead of a second pass over a3):
//                          pool_part[tile][wave][32], 64 pixels each, zeros
//                          past the image's edge included.
// ---------------------------------------------------------------------------
constexpr int kTileItems = (kRows + 2) * (kCols + 2) * 4;   // 16-byte items of an input tile
constexpr int kTilePer = (kTileItems + 255) / 256;          // per lane

// Work-groups per CU of the output layer's persistent grid (it needs fewer
// registers than the 32-channel layers, so more groups fit).
#ifndef QLD_OUT_LAYER_GROUPS_PER_CU
#define QLD_OUT_LAYER_GROUPS_PER_CU 3
#endif
#ifndef QLD_CONV_GROUPS_PER_CU
#define QLD_CONV_GROUPS_PER_CU 3
#endif
template <int MODE>
__global__ __launch_bounds__(256, MODE == 2 ? QLD_OUT_LAYER_GROUPS_PER_CU : QLD_CONV_GROUPS_PER_CU) void conv_tile_kernel(const __bf16 *__restrict__ in, const __bf16 *__restrict__ wt,
                                                        const float *__restrict__ bias, const __bf16 *__restrict__ act,
                                                        void *__restrict__ out, int H, int W, int n_tiles,
                                                        float *__restrict__ pool_part) {
    constexpr int NCB = MODE == 2 ? 1 : 2;          // 16-channel output blocks
    // The 32-channel layers keep their weights in LDS (18 KB, read per tap),
    // which leaves registers for three work-groups per CU; the output layer's
    // fit in registers.
    constexpr bool kWLds = MODE != 2;
    __shared__ __align__(16) __bf16 tile[kRows + 2][kCols + 2][32];
    __shared__ __align__(16) __bf16 wS[kWLds ? 9 * 16 * NCB * 32 : 8];
    const int tx = (W + kCols - 1) / kCols, ty = (H + kRows - 1) / kRows;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, m = lane & 15, kb = lane >> 4;
    bf16x8 w[kWLds ? 1 : 9][NCB];
    if constexpr (kWLds) {
        // Visible to every wave after the first tile's barriers.
        for (int i = t; i < 9 * 16 * NCB * 4; i += 256)
            reinterpret_cast<bf16x8 *>(wS)[i] = reinterpret_cast<const bf16x8 *>(wt)[i];
    } else {
#pragma unroll
        for (int k = 0; k < 9; ++k)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
                w[k][cb] = *reinterpret_cast<const bf16x8 *>(wt + ((k * 16 * NCB + cb * 16 + m) * 32 + kb * 8));
    }
    float bco[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) bco[cb] = MODE == 1 ? 0.f : bias[MODE == 2 ? 0 : 16 * cb + m];

    bf16x8 v[kTilePer];
    auto fetch = [&](int tl) {
        const int x0 = (tl % tx) * kCols, y0 = ((tl / tx) % ty) * kRows;
        const int64_t img = (int64_t)(tl / (tx * ty)) * H;
#pragma unroll
        for (int j = 0; j < kTilePer; ++j) {
            const int item = t + 256 * j;
            const int cg = item & 3, q = item >> 2, px = q % (kCols + 2), r = q / (kCols + 2);
            const int iy = y0 - 1 + r, ix = x0 - 1 + px;
            const bool ok = item < kTileItems && iy >= 0 && iy < H && ix >= 0 && ix < W;
            v[j] = ok ? *reinterpret_cast<const bf16x8 *>(in + ((img + iy) * W + ix) * 32 + cg * 8) : zero8();
        }
    };
    if (blockIdx.x < (unsigned)n_tiles) fetch(blockIdx.x);
    for (int tl = blockIdx.x; tl < n_tiles; tl += gridDim.x) {
        const int x0 = (tl % tx) * kCols, y0 = ((tl / tx) % ty) * kRows;
        const int64_t img = (int64_t)(tl / (tx * ty)) * H;
        const int y = y0 + wave;
        __syncthreads();                              // the previous tile's LDS readers are done
        // Item i is the 16 bytes at offset 16 i of the tile (row, pixel, channel group).
#pragma unroll
        for (int j = 0; j < kTilePer; ++j) {
            const int item = t + 256 * j;
            if (item < kTileItems) reinterpret_cast<bf16x8 *>(&tile[0][0][0])[item] = v[j];
        }
        __syncthreads();
        if (tl + (int)gridDim.x < n_tiles) fetch(tl + gridDim.x);
        if constexpr (MODE == 2) {
            if (pool_part) {
                // Lane (channel pair c2, quarter q): channels 2 c2, 2 c2 + 1 over
                // pixels 16 q .. 16 q + 15 of the wave's row (one 4-byte LDS read
                // per pixel), in order; the quarters added pairwise, one store
                // per channel.
                const int c2 = lane & 15, q = lane >> 4;
                float p0 = 0.f, p1 = 0.f;
#pragma unroll 8
                for (int p = 0; p < 16; ++p) {
                    const uint32_t u = *reinterpret_cast<const uint32_t *>(&tile[wave + 1][1 + 16 * q + p][2 * c2]);
                    p0 += __uint_as_float(u << 16);
                    p1 += __uint_as_float(u & 0xffff0000u);
                }
                p0 += __shfl_xor(p0, 16);
                p1 += __shfl_xor(p1, 16);
                p0 += __shfl_xor(p0, 32);
                p1 += __shfl_xor(p1, 32);
                if (q == 0) {
                    float *dst = pool_part + ((int64_t)tl * kRows + wave) * 32 + 2 * c2;
                    dst[0] = p0;
                    dst[1] = p1;
                }
            }
        }
        // MODE 1: the ReLU mask of this wave's outputs, loaded ahead of the products.
        bf16x8 am[4];
        if constexpr (MODE == 1) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const int j = lane + 64 * jj, pl = j >> 2, cg = j & 3;
                const int px = x0 + pl;
                am[jj] = y < H && px < W ? *reinterpret_cast<const bf16x8 *>(act + ((img + y) * W + px) * 32 + cg * 8)
                                         : zero8();
            }
        }
        f32x4 acc[4][NCB];
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[g][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int sy = MODE == 1 ? -tap_dy(k) : tap_dy(k);
            const int sx = MODE == 1 ? -tap_dx(k) : tap_dx(k);
            bf16x8 a[4];
#pragma unroll
            for (int g = 0; g < 4; ++g)
                a[g] = *reinterpret_cast<const bf16x8 *>(&tile[wave + 1 + sy][16 * g + m + 1 + sx][kb * 8]);
            bf16x8 wk[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
                wk[cb] = kWLds ? *reinterpret_cast<const bf16x8 *>(&wS[(k * 16 * NCB + cb * 16 + m) * 32 + kb * 8])
                               : w[k][cb];
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[g][cb] = mfma16(a[g], wk[cb], acc[g][cb]);
        }
        if constexpr (MODE == 2) {
            if (y < H && m == 0) {
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int px = x0 + 16 * g + 4 * kb + i;
                        if (px < W) static_cast<float *>(out)[(img + y) * W + px] = acc[g][0][i] + bco[0];
                    }
            }
        } else {
            // The wave's 64 pixels x 32 channels go out through LDS (the input
            // tile is no longer read): each lane writes its bf16 results (MODE 0:
            // bias and ReLU applied first), then moves four 16-byte chunks, so the
            // global stores are 1 KiB contiguous per instruction.  Rounding before
            // masking equals masking first (the mask is 0 or 1).  Rows of 40
            // channels keep the writes conflict-free.
            constexpr int kORow = 40;
            __bf16(*ot)[kORow] = reinterpret_cast<__bf16(*)[kORow]>(&tile[0][0][0]) + wave * 64;
            static_assert(4 * 64 * kORow * sizeof(__bf16) <= sizeof(tile), "output staging fits in the tile");
            __syncthreads();                              // every wave is done reading the input tile
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        const int co = 16 * cb + m;
                        float vv = acc[g][cb][i];
                        if (MODE == 0) vv = fmaxf(vv + bco[cb], 0.0f);
                        ot[16 * g + 4 * kb + i][co] = (__bf16)vv;
                    }
            // Only this wave reads back what it wrote.
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (y < H) {
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int j = lane + 64 * jj, pl = j >> 2, cg = j & 3;
                    const int px = x0 + pl;
                    if (px >= W) continue;
                    const int64_t idx = ((img + y) * W + px) * 32 + cg * 8;
                    bf16x8 o = *reinterpret_cast<const bf16x8 *>(&ot[pl][cg * 8]);
                    if constexpr (MODE == 1) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) o[e] = (float)am[jj][e] > 0.0f ? o[e] : (__bf16)0.0f;
                    }
                    *reinterpret_cast<bf16x8 *>(static_cast<__bf16 *>(out) + idx) = o;
                }
            }
        }
    }
}

// 2 -> 32 input layer: the 18 (tap, channel) products form one K = 32 MFMA.
// The work-group's input (rows y0-1 .. y0+4, pixels xs-1 .. xs+64, both
// channels of a pixel as one 4-byte word, zero outside the image) is staged
// in LDS once; a lane's operand dword e is then tap 4 kb + e's word.
__global__ __launch_bounds__(256) void conv1_kernel(const __bf16 *__restrict__ x0, const __bf16 *__restrict__ w1f,
                                                    const float *__restrict__ bias, __bf16 *__restrict__ out, int H,
                                                    int W) {
    __shared__ uint32_t xt[kRows + 2][kCols + 2];
    int b, y, xs;
    const bool row_ok = tile_of(H, W, b, y, xs);
    const int wave = threadIdx.x >> 6, y0 = y - wave;
    const int64_t img = (int64_t)b * H;
    for (int i = threadIdx.x; i < (kRows + 2) * (kCols + 2); i += 256) {
        const int r = i / (kCols + 2), c = i % (kCols + 2);
        const int iy = y0 - 1 + r, ix = xs - 1 + c;
        xt[r][c] = iy >= 0 && iy < H && ix >= 0 && ix < W
                       ? *reinterpret_cast<const uint32_t *>(x0 + ((img + iy) * W + ix) * 2)
                       : 0u;
    }
    __syncthreads();
    if (!row_ok) return;
    const int lane = threadIdx.x & 63, m = lane & 15, kb = lane >> 4;
    const bf16x8 w0 = *reinterpret_cast<const bf16x8 *>(w1f + (m * 32 + kb * 8));
    const bf16x8 w1 = *reinterpret_cast<const bf16x8 *>(w1f + ((16 + m) * 32 + kb * 8));
    f32x4 acc[4][2];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        u32x4c aw;
#pragma unroll
        for (int e = 0; e < 4; ++e) {          // k = 8 kb + 2 e + ch: tap 4 kb + e
            const int t = 4 * kb + e;
            aw[e] = t < 9 ? xt[wave + 1 + tap_dy(t)][16 * g + m + 1 + tap_dx(t)] : 0u;
        }
        const bf16x8 a = __builtin_bit_cast(bf16x8, aw);
        acc[g][0] = mfma16(a, w0, f32x4{0.f, 0.f, 0.f, 0.f});
        acc[g][1] = mfma16(a, w1, f32x4{0.f, 0.f, 0.f, 0.f});
    }
    // Out through a per-wave LDS tile (64 pixels x 32 channels, rows of 40):
    // 16-byte global stores, 1 KiB contiguous per instruction.  Only this
    // wave reads what it wrote, so a wave-level scheduling barrier suffices.
    __shared__ __align__(16) __bf16 ot_all[4][64][40];
    __bf16(*ot)[40] = ot_all[threadIdx.x >> 6];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = 16 * cb + m;
                ot[16 * g + 4 * kb + i][co] = (__bf16)fmaxf(acc[g][cb][i] + bias[co], 0.0f);
            }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int j = lane + 64 * jj, pl = j >> 2, cg = j & 3;
        const int px = xs + pl;
        if (px >= W) continue;
        *reinterpret_cast<bf16x8 *>(out + ((img + y) * W + px) * 32 + cg * 8) =
            *reinterpret_cast<const bf16x8 *>(&ot[pl][cg * 8]);
    }
}

// dy = 2 (y - t) / N; per-block partial sums of (y - t)^2.
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ y, const float *__restrict__ t,
                                                   float *__restrict__ dy, int64_t n, double *__restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const float sc = (float)(2.0 / (double)n);
    // Groups of four pixels with 16-byte accesses (y and dy are the
    // denoiser's own 16-byte aligned buffers; the caller's t may not be,
    // and then every pixel takes the loop below), then the rest one by one.
    const int64_t n4 = (reinterpret_cast<uintptr_t>(t) & 15) == 0 ? n / 4 : 0;
    for (int64_t i = gid; i < n4; i += stride) {
        const f32x4 yv = reinterpret_cast<const f32x4 *>(y)[i];
        const f32x4 tv = reinterpret_cast<const f32x4 *>(t)[i];
        f32x4 o;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float d = yv[k] - tv[k];
            o[k] = sc * d;
            s += (double)d * d;
        }
        reinterpret_cast<f32x4 *>(dy)[i] = o;
    }
    for (int64_t i = 4 * n4 + gid; i < n; i += stride) {
        const float d = y[i] - t[i];
        dy[i] = sc * d;
        s += (double)d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// 32x32 weight gradient on the matrix cores: D[tap][ci][co] = sum_px a[px + tap][ci] dz[px][co]
// (v_mfma_f32_16x16x32_bf16: M = co, N = ci, K = 32 pixels).  An MFMA operand
// lane holds 8 consecutive pixels of one channel, so a work-group stages each
// 64-pixel row segment transposed in LDS: dT[co][px] from dz, and aT[slot][ci][px]
// from the input rows around it (pixels x0-1 .. x0+64, zero outside the
// image).  A lane then reads its 8 pixels with one 16-byte LDS read; the taps
// at dx = -1 / +1 combine two aligned reads with a 16-bit funnel shift.  Wave w
// owns the 16x16 block (co block w & 1, ci block w >> 1) for all 9 taps; waves
// 0 and 1 also sum their dz operands for the bias gradient.
// Work units are vertical runs of `rows` rows of one 64-pixel strip, walked
// top to bottom: the input rows y-1, y, y+1 sit in a three-slot ring (row r
// in slot (r + 3) % 3), so each row of `a` is loaded and transposed once per
// unit instead of three times, and rows y+2, y+3 of `a` and y+1, y+2 of dz
// are in flight while row y's products run.  Units are dealt round-robin to
// work-groups; each writes one row of partial sums part[block][tap][ci][co]
// followed by the 32 bias sums (the canonical order of W and b), summed later
// in a fixed order.
constexpr int kSegPx = 64;
constexpr int kAStride = 88;   // bf16 per aT row: pixels x0-8 .. x0+71 (+8 pad); 176 B, 16-B multiple
constexpr int kDStride = 72;   // bf16 per dT row: 64 pixels (+8 pad); 144 B
constexpr int kW32Row = 9 * 1024 + 32;   // partial row: weights then bias
constexpr int kARowItems = 4 * 66;       // 16-byte items of one row of `a` (4 channel groups x 66 pixels)

typedef uint32_t u32x4w __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int ring_slot(int r) { return (r + 3) % 3; }

__global__ __launch_bounds__(256) void dw32_kernel(const __bf16 *__restrict__ a, const __bf16 *__restrict__ dz, int B,
                                                   int H, int W, int rows, float *__restrict__ part) {
    __shared__ __align__(16) __bf16 aT[3][32][kAStride];
    __shared__ __align__(16) __bf16 dT[32][kDStride];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, m = lane & 15, kb = lane >> 4;
    const int cb = wave & 1, cib = wave >> 1;
    const int segs_x = (W + kSegPx - 1) / kSegPx, runs_y = (H + rows - 1) / rows;
    const int64_t n_units = (int64_t)B * segs_x * runs_y;
    f32x4 acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    const bf16x8 zero = zero8();
    // Row iy of `a` (item t + 256 i: pixel x0 - 1 + item % 66, channels
    // 8 (item / 66) .. +8), and row y of dz (pixel x0 + (t & 63), channels
    // 8 (t >> 6) .. +8); rows outside the image read as zero.
    // Register buffers: P holds the rows at an even distance from the unit's
    // first row, Q those at an odd one; with the loop unrolled by two rows the
    // buffer of every row is known at compile time, and two rows of each input
    // are in flight while a row is worked.
    struct Buf {
        bf16x8 va[2], vd;
    } P, Q;
    auto fetch_a = [&](Buf &bf, int64_t img, int x0, int iy) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int item = t + 256 * i;
            const int px = item % 66, cg = item / 66;
            const int xa = x0 - 1 + px;
            const bool ok = item < kARowItems && xa >= 0 && xa < W && iy >= 0 && iy < H;
            bf.va[i] = ok ? *reinterpret_cast<const bf16x8 *>(a + ((img + iy) * W + xa) * 32 + cg * 8) : zero;
        }
    };
    auto store_a = [&](const Buf &bf, int slot) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int item = t + 256 * i;
            if (item < kARowItems) {
                const int px = item % 66, cg = item / 66;
#pragma unroll
                for (int e = 0; e < 8; ++e) aT[slot][cg * 8 + e][px + 7] = bf.va[i][e];
            }
        }
    };
    auto fetch_d = [&](Buf &bf, int64_t img, int x0, int y) {
        const int x = x0 + (t & 63);
        bf.vd = x < W ? *reinterpret_cast<const bf16x8 *>(dz + ((img + y) * W + x) * 32 + (t >> 6) * 8) : zero;
    };
    auto store_d = [&](const Buf &bf) {
        const int px = t & 63, cg = t >> 6;
#pragma unroll
        for (int i = 0; i < 8; ++i) dT[cg * 8 + i][px] = bf.vd[i];
    };
    auto products = [&](int y) {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int pxb = kk * 32 + kb * 8;       // this lane's 8 pixels: x0 + pxb .. +8
            const bf16x8 A = *reinterpret_cast<const bf16x8 *>(&dT[cb * 16 + m][pxb]);
            if (cib == 0) {
                float sb = 0.f;
#pragma unroll
                for (int e = 0; e < 8; ++e) sb += (float)A[e];
                bacc += sb;
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const __bf16 *rp = &aT[ring_slot(y - 1 + r)][cib * 16 + m][0];
                const u32x4w pv = *reinterpret_cast<const u32x4w *>(rp + pxb);        // pixels pxb-8 ..
                const u32x4w c = *reinterpret_cast<const u32x4w *>(rp + pxb + 8);     // pixels pxb ..
                const u32x4w nx = *reinterpret_cast<const u32x4w *>(rp + pxb + 16);   // pixels pxb+8 ..
                u32x4w lft, rgt;                                                      // shifted by -1 / +1
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    lft[k] = __builtin_amdgcn_alignbit(c[k], k ? c[k - 1] : pv[3], 16);
                    rgt[k] = __builtin_amdgcn_alignbit(k < 3 ? c[k + 1] : nx[0], c[k], 16);
                }
                acc[3 * r + 0] = mfma16(A, __builtin_bit_cast(bf16x8, lft), acc[3 * r + 0]);
                acc[3 * r + 1] = mfma16(A, __builtin_bit_cast(bf16x8, c), acc[3 * r + 1]);
                acc[3 * r + 2] = mfma16(A, __builtin_bit_cast(bf16x8, rgt), acc[3 * r + 2]);
            }
        }
    };
    // Row y (k = y - y_begin): a-row y+1 comes from the buffer of parity k+1,
    // d-row y from that of parity k; a-row y+3 and d-row y+2 are then fetched
    // into the buffers just emptied.
    auto step = [&](Buf &even, Buf &odd, int64_t img, int x0, int y, int y_end) {
        __syncthreads();                            // readers of row y-2's slot and of dT are done
        store_a(odd, ring_slot(y + 1));
        store_d(even);
        __syncthreads();
        if (y + 2 < y_end) {
            fetch_a(odd, img, x0, y + 3);
            fetch_d(even, img, x0, y + 2);
        }
        products(y);
    };
    for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        const int x0 = (int)(u % segs_x) * kSegPx;
        const int64_t q = u / segs_x;
        const int y_begin = (int)(q % runs_y) * rows, y_end = min(H, y_begin + rows);
        const int64_t img = (q / runs_y) * H;
        __syncthreads();                            // the previous unit's readers are done
        fetch_a(P, img, x0, y_begin - 1);
        store_a(P, ring_slot(y_begin - 1));
        fetch_a(P, img, x0, y_begin);
        store_a(P, ring_slot(y_begin));
        fetch_a(Q, img, x0, y_begin + 1);           // a-rows y_begin+1 (odd), y_begin+2 (even)
        fetch_a(P, img, x0, y_begin + 2);
        fetch_d(P, img, x0, y_begin);               // d-rows y_begin (even), y_begin+1 (odd)
        if (y_begin + 1 < y_end) fetch_d(Q, img, x0, y_begin + 1);
        for (int y = y_begin; y < y_end; y += 2) {
            step(P, Q, img, x0, y, y_end);
            if (y + 1 < y_end) step(Q, P, img, x0, y + 1, y_end);
        }
    }
    float *pb = part + (int64_t)blockIdx.x * kW32Row;
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = 16 * cb + 4 * kb + i, ci = 16 * cib + m;
            pb[(k * 32 + ci) * 32 + co] = acc[k][i];
        }
    if (cib == 0) {
        bacc += __shfl_xor(bacc, 16);
        bacc += __shfl_xor(bacc, 32);
        if (kb == 0) pb[9 * 1024 + cb * 16 + m] = bacc;
    }
}

// Input layer (2 -> 32) weight and bias gradients on the matrix cores:
// dW1[tap][ci][co] = sum_px x0[px + tap][ci] dz1[px][co] with M = co, N = the
// 18 (tap, ci) pairs in two 16-column blocks, K = 32 pixels; db1[co] = sum_px
// dz1[px][co].  Staged like dw32_kernel (vertical strips, a three-slot ring of
// input rows, two rows of each input in flight): dz1 transposed dT[co][px]
// and the input rows transposed xT[slot][ci][px].  Wave w: co block w & 1,
// column block w >> 1; each lane's column (tap, ci) picks the shifted pixel
// window of its tap.  Partial rows part[block][608]: W1 then b1 (the
// canonical order).
constexpr int kW1Row = 576 + 32;

__global__ __launch_bounds__(256) void dw1_kernel(const __bf16 *__restrict__ x, const __bf16 *__restrict__ dz, int B,
                                                  int H, int W, int rows, float *__restrict__ part) {
    __shared__ __align__(16) __bf16 xT[3][2][kAStride];
    __shared__ __align__(16) __bf16 dT[32][kDStride];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, m = lane & 15, kb = lane >> 4;
    const int cb = wave & 1, nb = wave >> 1;
    const int n = nb * 16 + m;                       // column: tap n / 2, input channel n % 2
    const bool col_ok = n < 18;
    const int tap = col_ok ? n >> 1 : 0, ch = n & 1;
    const int tr = tap / 3, dx = tap % 3 - 1;
    const int segs_x = (W + kSegPx - 1) / kSegPx, runs_y = (H + rows - 1) / rows;
    const int64_t n_units = (int64_t)B * segs_x * runs_y;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    const bf16x8 zero = zero8();
    // Row iy of x (lanes t < 66: both channels of pixel x0 - 1 + t, one bf16
    // pair) and row y of dz1 (pixel x0 + (t & 63), channels 8 (t >> 6) .. +8).
    struct Buf {
        uint32_t vx;
        bf16x8 vd;
    } P, Q;
    auto fetch_x = [&](Buf &bf, int64_t img, int x0, int iy) {
        const int xi = x0 - 1 + t;
        const bool ok = t < 66 && xi >= 0 && xi < W && iy >= 0 && iy < H;
        bf.vx = ok ? *reinterpret_cast<const uint32_t *>(x + ((img + iy) * W + xi) * 2) : 0u;
    };
    auto store_x = [&](const Buf &bf, int slot) {
        if (t < 66) {
            xT[slot][0][t + 7] = __builtin_bit_cast(__bf16, (uint16_t)(bf.vx & 0xffffu));
            xT[slot][1][t + 7] = __builtin_bit_cast(__bf16, (uint16_t)(bf.vx >> 16));
        }
    };
    auto fetch_d = [&](Buf &bf, int64_t img, int x0, int y) {
        const int xx = x0 + (t & 63);
        bf.vd = xx < W ? *reinterpret_cast<const bf16x8 *>(dz + ((img + y) * W + xx) * 32 + (t >> 6) * 8) : zero;
    };
    auto store_d = [&](const Buf &bf) {
        const int px = t & 63, cg = t >> 6;
#pragma unroll
        for (int i = 0; i < 8; ++i) dT[cg * 8 + i][px] = bf.vd[i];
    };
    auto products = [&](int y) {
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const int pxb = kk * 32 + kb * 8;
            const bf16x8 A = *reinterpret_cast<const bf16x8 *>(&dT[cb * 16 + m][pxb]);
            if (nb == 0) {
                float sb = 0.f;
#pragma unroll
                for (int e = 0; e < 8; ++e) sb += (float)A[e];
                bacc += sb;
            }
            const __bf16 *rp = &xT[ring_slot(y - 1 + tr)][ch][0];
            const u32x4w pv = *reinterpret_cast<const u32x4w *>(rp + pxb);
            const u32x4w c = *reinterpret_cast<const u32x4w *>(rp + pxb + 8);
            const u32x4w nx = *reinterpret_cast<const u32x4w *>(rp + pxb + 16);
            u32x4w bv;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t lft = __builtin_amdgcn_alignbit(c[k], k ? c[k - 1] : pv[3], 16);
                const uint32_t rgt = __builtin_amdgcn_alignbit(k < 3 ? c[k + 1] : nx[0], c[k], 16);
                bv[k] = !col_ok ? 0u : (dx < 0 ? lft : (dx > 0 ? rgt : c[k]));
            }
            acc = mfma16(A, __builtin_bit_cast(bf16x8, bv), acc);
        }
    };
    // Buffers by parity of the distance from the unit's first row, as in dw32_kernel.
    auto step = [&](Buf &even, Buf &odd, int64_t img, int x0, int y, int y_end) {
        __syncthreads();
        store_x(odd, ring_slot(y + 1));
        store_d(even);
        __syncthreads();
        if (y + 2 < y_end) {
            fetch_x(odd, img, x0, y + 3);
            fetch_d(even, img, x0, y + 2);
        }
        products(y);
    };
    for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        const int x0 = (int)(u % segs_x) * kSegPx;
        const int64_t q = u / segs_x;
        const int y_begin = (int)(q % runs_y) * rows, y_end = min(H, y_begin + rows);
        const int64_t img = (q / runs_y) * H;
        __syncthreads();
        fetch_x(P, img, x0, y_begin - 1);
        store_x(P, ring_slot(y_begin - 1));
        fetch_x(P, img, x0, y_begin);
        store_x(P, ring_slot(y_begin));
        fetch_x(Q, img, x0, y_begin + 1);
        fetch_x(P, img, x0, y_begin + 2);
        fetch_d(P, img, x0, y_begin);
        if (y_begin + 1 < y_end) fetch_d(Q, img, x0, y_begin + 1);
        for (int y = y_begin; y < y_end; y += 2) {
            step(P, Q, img, x0, y, y_end);
            if (y + 1 < y_end) step(Q, P, img, x0, y + 1, y_end);
        }
    }
    float *pb = part + (int64_t)blockIdx.x * kW1Row;
    if (col_ok)
#pragma unroll
        for (int i = 0; i < 4; ++i) pb[(tap * 2 + ch) * 32 + 16 * cb + 4 * kb + i] = acc[i];
    if (nb == 0) {
        bacc += __shfl_xor(bacc, 16);
        bacc += __shfl_xor(bacc, 32);
        if (kb == 0) pb[576 + cb * 16 + m] = bacc;
    }
}

// Output layer (32 -> 1) backward in one pass over a3 and dy:
//   dW4[tap][ci] = sum_px a3[px + tap][ci] dy[px],  db4 = sum_px dy[px]
//   dz3[q][c] = bf16((sum_tap dy[q - tap] w4[tap][c]) * (a3[q][c] > 0))
// Both contractions run on the matrix cores in bf16.  dy is split exactly
// into three bf16 parts, dy = hi + mid + lo (its top 8 significant bits, the
// next 8, the last 8), so every product is exact and only the fp32
// accumulation rounds.  Work units are vertical runs of `rows` rows of one
// 64-pixel strip, walked top to bottom like dw32_kernel: a three-slot ring
// holds rows y-1, y, y+1 of a3 (transposed, aT[slot][ci][px]) and of dy (fp32
// dyS[slot][px] and its parts dyP[slot][part][px], in aT's column order), and
// two rows of each are in flight while row y is worked.  For row y:
//  * dW4: wave w takes channel block w & 1 (M = 16 channels) and pixels
//    32 (w >> 1) .. +32 of the strip (K); N = the three parts of dy at those
//    pixels (one 16-byte read), A = a3 of row y-1+r at the pixels shifted by
//    the tap's dx (16-bit funnel shifts of aligned chunks, the strip's halo
//    columns included); one product per (r, dx), the parts added at the end.
//  * dz3: wave w takes pixels 16w .. +16 of the strip (M), the channels in
//    two blocks (N) and K = 16 with lane group kb holding dy row y+1-kb at
//    the three column offsets (taps 3 kb .. 3 kb + 2; kb = 3 empty); one
//    16x16x16 product per part.  The ReLU mask comes from a3 in the ring, and
//    the results pass through a per-wave LDS tile so each lane stores 16
//    contiguous bytes of a pixel.
//  * db4: the lanes of wave 0 add dy of row y, one pixel each.
// Each work-group writes partial rows part[2 block + half][289] (dW4 in
// canonical order, then db4 in row 2 block), summed later in a fixed order.
constexpr int kOutRow = 289;
constexpr int kStgRow = 40;    // bf16 per row of the per-wave dz3 tile (32 channels + 8 pad)

typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16k16(const s16x4 &a, const s16x4 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// x = hi + mid + lo exactly, each part a bf16 value (returned as its bits):
// hi is x cut to its top 16 bits, mid the rest x - hi (exact) cut the same
// way, lo = x - hi - mid (exact, at most 8 significant bits).
__device__ __forceinline__ void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l) {
    const uint32_t xb = __float_as_uint(x);
    const float r1 = x - __uint_as_float(xb & 0xffff0000u);
    const uint32_t rb = __float_as_uint(r1);
    const float lo = r1 - __uint_as_float(rb & 0xffff0000u);
    h = (uint16_t)(xb >> 16);
    m = (uint16_t)(rb >> 16);
    l = (uint16_t)(__float_as_uint(lo) >> 16);
}

#ifndef QLD_OUT_GRAD_BLOCKS_PER_CU
#define QLD_OUT_GRAD_BLOCKS_PER_CU 4
#endif
__global__ __launch_bounds__(256, QLD_OUT_GRAD_BLOCKS_PER_CU) void out_grad_kernel(const __bf16 *__restrict__ a, const float *__restrict__ dy,
                                                       const __bf16 *__restrict__ w4, int B, int H, int W, int rows,
                                                       __bf16 *__restrict__ dz, float *__restrict__ part) {
    __shared__ __align__(16) __bf16 aT[3][32][kAStride];
    __shared__ __align__(16) uint16_t dyP[4][3][kAStride];   // slot 3: zeros
    // The same parts interleaved per column (hi | mid << 16, lo) for dz3's
    // operand gathers: one 8-byte read per column; slot 3: zeros.
    __shared__ __align__(16) uint32_t dyQ[4][kAStride][2];
    __shared__ __align__(16) float dyS[3][72];               // pixels x0-1 .. x0+64 at 3 .. 68
    __shared__ __align__(16) __bf16 stg[4][16][kStgRow];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, m = lane & 15, kb = lane >> 4;
    const int cib = wave & 1, kk = wave >> 1;
    const int segs_x = (W + kSegPx - 1) / kSegPx, runs_y = (H + rows - 1) / rows;
    const int64_t n_units = (int64_t)B * segs_x * runs_y;
    const bf16x8 zero = zero8();
    for (int i = t; i < 3 * kAStride; i += 256) dyP[3][i / kAStride][i % kAStride] = 0;
    for (int i = t; i < 2 * kAStride; i += 256) dyQ[3][i / 2][i % 2] = 0u;
    // dz3's B operand: lane (channel n = m, kb) holds w4[3 kb + i][16 cb + m]
    // for i < 3 and kb < 3 (K slot 4 kb + i), zero elsewhere.
    s16x4 bw[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            bw[cb][i] = kb < 3 && i < 3 ? __builtin_bit_cast(short, w4[(3 * kb + i) * 32 + 16 * cb + m]) : (short)0;
    f32x4 acc[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[r][d] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    // Register buffers by parity of the distance from the unit's first row
    // (as in dw32_kernel): two rows of a3 and dy in flight while a row is worked.
    struct Buf {
        bf16x8 va[2];
        float vdy;
    } P, Q;
    auto fetch = [&](Buf &bf, int64_t img, int x0, int iy) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int item = t + 256 * i;
            const int px = item % 66, g = item / 66;
            const int xa = x0 - 1 + px;
            const bool ok = item < kARowItems && xa >= 0 && xa < W && iy >= 0 && iy < H;
            bf.va[i] = ok ? *reinterpret_cast<const bf16x8 *>(a + ((img + iy) * W + xa) * 32 + g * 8) : zero;
        }
        const int xd = x0 - 1 + t;
        bf.vdy = t < 66 && xd >= 0 && xd < W && iy >= 0 && iy < H ? dy[(img + iy) * W + xd] : 0.f;
    };
    auto store = [&](const Buf &bf, int slot) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int item = t + 256 * i;
            if (item < kARowItems) {
                const int px = item % 66, g = item / 66;
#pragma unroll
                for (int e = 0; e < 8; ++e) aT[slot][g * 8 + e][px + 7] = bf.va[i][e];
            }
        }
        if (t < 66) {
            dyS[slot][t + 3] = bf.vdy;
            uint16_t h, md, l;
            split3(bf.vdy, h, md, l);
            dyP[slot][0][t + 7] = h;
            dyP[slot][1][t + 7] = md;
            dyP[slot][2][t + 7] = l;
            dyQ[slot][t + 7][0] = (uint32_t)h | ((uint32_t)md << 16);
            dyQ[slot][t + 7][1] = l;
        }
    };
    auto work = [&](int64_t img, int x0, int y) {
        // dW4: B = the parts of dy (row y) at this lane's 8 pixels.
        const int col0 = 32 * kk + 8 * kb + 8;                  // aT / dyP column of pixel x0 + 32 kk + 8 kb
        const uint16_t *bp = m < 3 ? &dyP[ring_slot(y)][m][col0] : &dyP[3][0][col0];
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(bp);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const __bf16 *rp = &aT[ring_slot(y - 1 + r)][16 * cib + m][0];
            const u32x4w pv = *reinterpret_cast<const u32x4w *>(rp + col0 - 8);
            const u32x4w c = *reinterpret_cast<const u32x4w *>(rp + col0);
            const u32x4w nx = *reinterpret_cast<const u32x4w *>(rp + col0 + 8);
            u32x4w lft, rgt;                                     // a3 at the pixels shifted by -1 / +1
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                lft[k] = __builtin_amdgcn_alignbit(c[k], k ? c[k - 1] : pv[3], 16);
                rgt[k] = __builtin_amdgcn_alignbit(k < 3 ? c[k + 1] : nx[0], c[k], 16);
            }
            acc[r][0] = mfma16(__builtin_bit_cast(bf16x8, lft), bv, acc[r][0]);
            acc[r][1] = mfma16(__builtin_bit_cast(bf16x8, c), bv, acc[r][1]);
            acc[r][2] = mfma16(__builtin_bit_cast(bf16x8, rgt), bv, acc[r][2]);
        }
        // db4: pixel x0 + lane of row y.
        if (wave == 0) bacc += dyS[ring_slot(y)][lane + 4];
        // dz3 of pixel x0 + 16 wave + m: K slot 4 kb + i holds the parts of dy
        // at (y + 1 - kb, x + 1 - i), i < 3.
        s16x4 ap[3];
        {
            typedef uint32_t u32x2q __attribute__((ext_vector_type(2)));
            const int sl = kb < 3 ? ring_slot(y + 1 - kb) : 3;
            const int cq = 16 * wave + m + 9;                    // dyQ column of pixel x + 1
            const u32x2q q0 = *reinterpret_cast<const u32x2q *>(&dyQ[sl][cq][0]);
            const u32x2q q1 = *reinterpret_cast<const u32x2q *>(&dyQ[sl][cq - 1][0]);
            const u32x2q q2 = *reinterpret_cast<const u32x2q *>(&dyQ[sl][cq - 2][0]);
            // Part s of columns cq, cq - 1, cq - 2 in K slots 0, 1, 2; slot 3 zero.
            const u32x2q hi = {(q0[0] & 0xffffu) | (q1[0] << 16), q2[0] & 0xffffu};
            const u32x2q mid = {(q0[0] >> 16) | (q1[0] & 0xffff0000u), q2[0] >> 16};
            const u32x2q lo = {(q0[1] & 0xffffu) | (q1[1] << 16), q2[1] & 0xffffu};
            ap[0] = __builtin_bit_cast(s16x4, hi);
            ap[1] = __builtin_bit_cast(s16x4, mid);
            ap[2] = __builtin_bit_cast(s16x4, lo);
        }
        f32x4 dv[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            dv[cb] = mfma16k16(ap[0], bw[cb], f32x4{0.f, 0.f, 0.f, 0.f});
            dv[cb] = mfma16k16(ap[1], bw[cb], dv[cb]);
            dv[cb] = mfma16k16(ap[2], bw[cb], dv[cb]);
        }
        // Lane (channel m, kb) holds pixels 16 wave + 4 kb + i of channels m
        // and 16 + m: mask them with a3 > 0, round to bf16 into the wave's tile.
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const uint32_t *mp =
                reinterpret_cast<const uint32_t *>(&aT[ring_slot(y)][16 * cb + m][16 * wave + 4 * kb + 8]);
            const uint32_t mk[2] = {mp[0], mp[1]};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t mb = (mk[i >> 1] >> (16 * (i & 1))) & 0xffffu;
                const bool pos = (mb & 0x8000u) == 0 && mb != 0;   // bf16 > 0 (a3 is never NaN)
                stg[wave][4 * kb + i][16 * cb + m] = (__bf16)(pos ? dv[cb][i] : 0.f);
            }
        }
        const int px = lane >> 2, g = lane & 3;
        const int x = x0 + 16 * wave + px;
        const bf16x8 ov = *reinterpret_cast<const bf16x8 *>(&stg[wave][px][8 * g]);
        if (x < W) *reinterpret_cast<bf16x8 *>(dz + ((img + y) * W + x) * 32 + 8 * g) = ov;
    };
    auto step = [&](Buf &even, Buf &odd, int64_t img, int x0, int y, int y_end) {
        __syncthreads();                            // readers of row y-2's slot are done
        store(odd, ring_slot(y + 1));
        __syncthreads();
        if (y + 2 < y_end) fetch(odd, img, x0, y + 3);
        work(img, x0, y);
    };
    for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        const int x0 = (int)(u % segs_x) * kSegPx;
        const int64_t q = u / segs_x;
        const int y_begin = (int)(q % runs_y) * rows, y_end = min(H, y_begin + rows);
        const int64_t img = (q / runs_y) * H;
        __syncthreads();                            // the previous unit's readers are done
        fetch(P, img, x0, y_begin - 1);
        store(P, ring_slot(y_begin - 1));
        fetch(P, img, x0, y_begin);
        store(P, ring_slot(y_begin));
        fetch(Q, img, x0, y_begin + 1);
        fetch(P, img, x0, y_begin + 2);
        for (int y = y_begin; y < y_end; y += 2) {
            step(P, Q, img, x0, y, y_end);
            if (y + 1 < y_end) step(Q, P, img, x0, y + 1, y_end);
        }
    }
    // Add the three parts (D columns 0, 1, 2) in order and write the
    // partial row of this wave's pixel half: lane (0, kb) holds channels
    // 16 cib + 4 kb + i.
    float *pb = part + ((int64_t)blockIdx.x * 2 + kk) * kOutRow;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[r][d][i];
                const float s = (v + __shfl_down(v, 1)) + __shfl_down(v, 2);
                if (m == 0) pb[(3 * r + d) * 32 + 16 * cib + 4 * kb + i] = s;
            }
    if (wave == 0) {
        float s = bacc;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) pb[288] = s;
    } else if (wave == 2 && lane == 0) {
        pb[288] = 0.f;
    }
}

// Column sums of several arrays part[R][n] in one launch, in a fixed order.
// Segment i covers blocks b0 .. b0 + bx * by - 1 of the 1-D grid (bx column
// blocks of 64, by slabs of 64 rows); block (cx, slab) of a segment takes 64
// columns x 4 row groups: group g adds rows slab*64 + g, +4, ... (their loads
// issued 16 at a time), and the four groups are combined in order into row
// `slab` of out[slabs][n].
constexpr int kMaxRedSegs = 4;
struct RedSeg {
    const float *in;
    float *out;
    int R, n, bx, b0;
};
// The loss's last stage, taken by one more block of a reduction launch:
// lane j < 64 adds partials j*c .. j*c+c-1 in order (c = n_blocks / 64,
// n_blocks a multiple of 64), then lane 0 adds the 64 sums in lane order;
// zero_n floats at zero_out (the gate's gradient when the step has no gate
// loss) are cleared.
struct LossFinish {
    const double *part;
    int n_blocks;
    int64_t n;
    float *loss, *zero_out;
    int zero_n;
};
struct RedJob {
    int n_seg;
    RedSeg seg[kMaxRedSegs];
    int b_end;          // blocks of the segments; block b_end takes lf (if lf.part)
    LossFinish lf;
};

__device__ void loss_finish_block(const LossFinish &f) {
    __shared__ double lane_sum[64];
    const int j = threadIdx.x, c = f.n_blocks / 64;
    for (int i = j; i < f.zero_n; i += blockDim.x) f.zero_out[i] = 0.f;
    if (j < 64) {
        double s = 0.0;
        for (int b = j * c; b < (j + 1) * c; ++b) s += f.part[b];
        lane_sum[j] = s;
    }
    __syncthreads();
    if (j == 0) {
        double tot = 0.0;
        for (int i = 0; i < 64; ++i) tot += lane_sum[i];
        f.loss[0] = (float)(tot / (double)f.n);
    }
}

__global__ __launch_bounds__(256) void reduce_segs_kernel(RedJob job) {
    if ((int)blockIdx.x == job.b_end) {
        if (job.lf.part) loss_finish_block(job.lf);
        return;
    }
    int si = 0;
    while (si + 1 < job.n_seg && (int)blockIdx.x >= job.seg[si + 1].b0) ++si;
    const RedSeg &S = job.seg[si];
    const int lb = (int)blockIdx.x - S.b0, bx = lb % S.bx, by = lb / S.bx;
    const int n = S.n;
    __shared__ float red[4][64];
    const int c = bx * 64 + (threadIdx.x & 63);
    const int g = threadIdx.x >> 6;
    const int r0 = by * 64, r1 = min(S.R, r0 + 64);
    float s = 0.f;
    if (c < n) {
        int r = r0 + g;
        for (; r + 4 * 15 < r1; r += 4 * 16) {
            float v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = S.in[(int64_t)(r + 4 * i) * n + c];
#pragma unroll
            for (int i = 0; i < 16; ++i) s += v[i];
        }
        for (; r < r1; r += 4) s += S.in[(int64_t)r * n + c];
    }
    red[g][threadIdx.x & 63] = s;
    __syncthreads();
    if (g == 0 && c < n) S.out[(int64_t)by * n + c] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                                       red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// Gate: pool[b][c] = mean_p a3[b][p][c]; gate[b] = pool[b] . Wg + bg.
// The output layer's kernel leaves one row of 32 channel sums per tile row
// (a few thousand per image); gate_fwd_kernel adds an image's rows in a fixed
// order, so the pooled values do not depend on timing.
// First stage of the gate's pooling: work-group (s, b) adds rows s*64 ..
// s*64 + 63 of image b's rows[b][rows][32] in order (4 groups of 16 rows,
// combined in order) into slab[b][s][32].
__global__ __launch_bounds__(256) void pool_rows_kernel(const float *__restrict__ rows, int n_rows,
                                                        float *__restrict__ slab) {
    __shared__ float red[8][32];
    const int s = blockIdx.x, b = blockIdx.y, c = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int r0 = s * 64 + g * 8, r1 = min(n_rows, r0 + 8);
    const float *src = rows + (int64_t)b * n_rows * 32 + c;
    float v = 0.f;
    for (int r = r0; r < r1; ++r) v += src[(int64_t)r * 32];
    red[g][c] = v;
    __syncthreads();
    if (threadIdx.x < 32) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) t += red[k][c];
        slab[((int64_t)b * gridDim.x + s) * 32 + c] = t;
    }
}

__global__ __launch_bounds__(256) void gate_fwd_kernel(const float *__restrict__ part, int chunks, int64_t npx,
                                                       const float *__restrict__ p, float *__restrict__ pool,
                                                       float *__restrict__ gate) {
    __shared__ float red[8][32];
    __shared__ float pooled[32];
    const int b = blockIdx.x, c = threadIdx.x & 31, r = threadIdx.x >> 5;
    // Chunks r, r + 8, ... added in that order; their loads issued 16 at a
    // time (one at a time, each add waited for its load: ~20 us).
    const float *pc = part + (int64_t)b * chunks * 32 + c;
    float s = 0.f;
    int k = r;
    for (; k + 8 * 15 < chunks; k += 8 * 16) {
        float v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = pc[(int64_t)(k + 8 * i) * 32];
#pragma unroll
        for (int i = 0; i < 16; ++i) s += v[i];
    }
    for (; k < chunks; k += 8) s += pc[(int64_t)k * 32];
    red[r][c] = s;
    __syncthreads();
    if (threadIdx.x < 32) {
        float t = 0.f;
        for (int k = 0; k < 8; ++k) t += red[k][c];
        const float v = t / (float)npx;
        pool[b * 32 + c] = v;
        pooled[c] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float g = p[OFF_BG];
        for (int k = 0; k < 32; ++k) g = fmaf(pooled[k], p[OFF_WG + k], g);
        gate[b] = g;
    }
}

// Gate gradient (its own loss, w * mean_b (gate - e)^2; e = ea - eb), one work-group.
__global__ void gate_back_kernel(const float *__restrict__ pool, const float *__restrict__ gate,
                                 const float *__restrict__ ea, const float *__restrict__ eb, float w, int B,
                                 float *__restrict__ grads, float *__restrict__ loss) {
    const int c = threadIdx.x;
    float gw = 0.f, gb = 0.f, l = 0.f;
    for (int b = 0; b < B; ++b) {
        const float e = ea[b] - (eb ? eb[b] : 0.f);
        const float d = gate[b] - e;
        const float de = w * 2.0f / (float)B * d;
        if (c < 32) gw = fmaf(pool[b * 32 + c], de, gw);
        gb += de;
        l += d * d;
    }
    if (c < 32) grads[OFF_WG + c] = gw;
    if (c == 0) {
        grads[OFF_BG] = gb;
        if (loss) loss[1] = w * l / (float)B;
    }
}


// One Adam step with the weights' bf16 copies refreshed in the same launch:
// thread j updates parameter j (m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / c1) / (sqrt(v / c2) + eps), c1 and c2 the bias corrections) and
// writes its bf16 copy into each operand layout of pack_kernel it has an
// entry in (the layouts' zero entries, written by the full pack when the
// parameters are set, never change).
__global__ void adam_pack_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                 float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2,
                                 __bf16 *w1f, __bf16 *w2f, __bf16 *w2b, __bf16 *w3f, __bf16 *w3b, __bf16 *w4,
                                 __bf16 *w4f) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N_ALL) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.f - b1) * gj;
    const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    float pj = p[j];
    pj -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    p[j] = pj;
    const __bf16 h = (__bf16)pj;
    if (j < OFF_B1) {                                   // W1[tap][ci][co] -> w1f[co][2 tap + ci]
        const int r = j - OFF_W1;
        w1f[(r % 32) * 32 + r / 32] = h;
    } else if (j >= OFF_W2 && j < OFF_B2) {             // W[t][ci][co] -> wf[t][co][ci], wb[t][ci][co]
        const int r = j - OFF_W2, t = r / 1024, ci = (r / 32) % 32, co = r % 32;
        w2f[t * 1024 + co * 32 + ci] = h;
        w2b[r] = h;
    } else if (j >= OFF_W3 && j < OFF_B3) {
        const int r = j - OFF_W3, t = r / 1024, ci = (r / 32) % 32, co = r % 32;
        w3f[t * 1024 + co * 32 + ci] = h;
        w3b[r] = h;
    } else if (j >= OFF_W4 && j < OFF_B4) {             // W4[t][ci] -> w4[t][ci], w4f[t][0][ci]
        const int r = j - OFF_W4;
        w4[r] = h;
        w4f[(r / 32) * 512 + r % 32] = h;
    }
}

}  // namespace
}  // namespace qld

// ---------------------------------------------------------------------------
// Object and entry points
// ---------------------------------------------------------------------------
struct qld_denoiser {
    int H, W, max_batch;
    int64_t step;
    float *params, *grads, *m, *v;
    __bf16 *w1f, *w2f, *w2b, *w3f, *w3b, *w4, *w4f;
    __bf16 *x0, *a1, *a2, *a3, *dzA, *dzB, *dzC;   // dz3, dz2, dz1
    float *y, *dy, *pool, *gate, *part, *part2, *loss;
    double *lpart;
    int64_t part_floats;
    // Weight-gradient partial rows of the backward (W4, W3, W2, W1), each
    // summed at the end of the backward: rows, columns, and the slab sums.
    float *gpart[4], *gslab;
    int gpart_R[4], gpart_n[4];
    int64_t gslab_off[4];
    int last_B;
    std::vector<void *> allocs;
};

namespace qld {
namespace {

constexpr int kW32Blocks = 1024;     // work-groups of dw32_kernel (four resident per CU)
constexpr int kW1Blocks = 2048;      // work-groups of dw1_kernel (eight resident per CU)

// Rows per work unit of dw32_kernel: enough units for every work-group, at
// least 4 rows (each unit loads two halo rows of `a` beyond its own).
int dw32_rows(int B, int H, int W, int blocks = kW32Blocks) {
    const int64_t strips = (int64_t)B * ceil_div(W, kSegPx);
    const int64_t want = ceil_div(strips * H, blocks);
    return (int)std::min<int64_t>(H, std::max<int64_t>(4, want));
}

// out_grad_kernel: QLD_OUT_GRAD_BLOCKS_PER_CU work-groups per CU (its launch
// bound keeps that many resident), one unit each.
int out_grad_blocks() { return std::max(8, QLD_OUT_GRAD_BLOCKS_PER_CU * device_cu_count() / 8 * 8); }
constexpr int kLossBlocks = 1024;   // a multiple of 64 (loss_finish_block)

template <typename T>
qld_status dalloc(qld_denoiser *d, T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, count * sizeof(T) + 64) != hipSuccess) {
        (void)hipGetLastError();
        set_error("denoiser allocation of %zu bytes failed", count * sizeof(T));
        return QLD_E_NOMEM;
    }
    d->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return QLD_OK;
}

int conv_grid(int B, int H, int W) {
    return (int)((int64_t)B * ceil_div(H, kRows) * ceil_div(W, kCols));
}

// Persistent grid of conv_tile_kernel: at most kConvGroupsPerCU work-groups
// per CU (a multiple of 8), looping over the tiles.
constexpr int kConvGroupsPerCU = QLD_CONV_GROUPS_PER_CU;
int conv_persistent_grid(int n_tiles, int per_cu = kConvGroupsPerCU) {
    const int64_t cap = std::max<int64_t>(8, (int64_t)per_cu * device_cu_count() / 8 * 8);
    return (int)std::min<int64_t>(n_tiles, cap);
}

qld_status pack(qld_denoiser *d, hipStream_t s) {
    hipLaunchKernelGGL(pack_kernel, dim3(36), dim3(256), 0, s, d->params, d->w1f, d->w2f, d->w2b, d->w3f, d->w3b,
                       d->w4, d->w4f);
    return check_hip(hipGetLastError(), "pack_kernel launch");
}

// Weights and bias of a 32 -> 32 layer (the bias follows the weights in the
// canonical order) into partial rows gpart[gi], summed by reduce_grads.
qld_status dw32(qld_denoiser *d, const __bf16 *a, const __bf16 *dz, int B, int gi, hipStream_t s) {
    hipLaunchKernelGGL(dw32_kernel, dim3(kW32Blocks), dim3(256), 0, s, a, dz, B, d->H, d->W, dw32_rows(B, d->H, d->W),
                       d->gpart[gi]);
    return check_hip(hipGetLastError(), "dw32 launch");
}

// Weights and bias of the input layer, into gpart[3].
qld_status dw1(qld_denoiser *d, int B, hipStream_t s) {
    hipLaunchKernelGGL(dw1_kernel, dim3(kW1Blocks), dim3(256), 0, s, d->x0, d->dzC, B, d->H, d->W,
                       dw32_rows(B, d->H, d->W, kW1Blocks), d->gpart[3]);
    return check_hip(hipGetLastError(), "dw1 launch");
}

// Output layer backward: dW4, db4 (into gpart[0]) and dz3 (into dzA) in one pass.
qld_status out_grad(qld_denoiser *d, int B, hipStream_t s) {
    const int blocks = out_grad_blocks();
    hipLaunchKernelGGL(out_grad_kernel, dim3(blocks), dim3(256), 0, s, d->a3, d->dy, d->w4, B, d->H, d->W,
                       dw32_rows(B, d->H, d->W, blocks), d->dzA, d->gpart[0]);
    return check_hip(hipGetLastError(), "out_grad launch");
}

// The four weight gradients from their partial rows, in two launches: the
// first adds each array's rows in slabs of 64 (or all of them, for at most 64
// rows, straight into the gradient), the second adds the slabs in order.
qld_status reduce_grads(qld_denoiser *d, const LossFinish &lf, hipStream_t s) {
    static const int64_t kOff[4] = {OFF_W4, OFF_W3, OFF_W2, OFF_W1};
    RedJob j1{}, j2{};
    int b1 = 0, b2 = 0;
    for (int i = 0; i < 4; ++i) {
        const int R = d->gpart_R[i], n = d->gpart_n[i], bx = (int)ceil_div(n, 64);
        const int slabs = (int)ceil_div(R, 64);
        float *dst = d->grads + kOff[i];
        if (slabs > 64) {
            set_error("reduction too large");
            return QLD_E_INVAL;
        }
        RedSeg &a = j1.seg[j1.n_seg++];
        a = RedSeg{d->gpart[i], slabs > 1 ? d->gslab + d->gslab_off[i] : dst, R, n, bx, b1};
        b1 += bx * slabs;
        if (slabs > 1) {
            RedSeg &c = j2.seg[j2.n_seg++];
            c = RedSeg{d->gslab + d->gslab_off[i], dst, slabs, n, bx, b2};
            b2 += bx;
        }
    }
    j1.b_end = b1;
    j1.lf = lf;
    j2.b_end = b2;
    hipLaunchKernelGGL(reduce_segs_kernel, dim3((unsigned)b1 + 1), dim3(256), 0, s, j1);
    if (j2.n_seg > 0) hipLaunchKernelGGL(reduce_segs_kernel, dim3((unsigned)b2), dim3(256), 0, s, j2);
    return check_hip(hipGetLastError(), "reduce_grads launch");
}

}  // namespace
}  // namespace qld

using namespace qld;

extern "C" qld_status qld_denoiser_create(int32_t H, int32_t W, int32_t max_batch, qld_denoiser **out) {
    clear_error();
    if (!out || H < 1 || W < 1 || max_batch < 1 || max_batch > 65535) {
        set_error("invalid denoiser shape %dx%d, batch %d", H, W, max_batch);
        return QLD_E_INVAL;
    }
    auto *d = new (std::nothrow) qld_denoiser();
    if (!d) return QLD_E_NOMEM;
    d->H = H;
    d->W = W;
    d->max_batch = max_batch;
    const size_t npx = (size_t)max_batch * H * W;
    // The forward's partials: the gate's row sums (one row of 32 channel sums
    // per tile row).
    d->part_floats = (int64_t)conv_grid(max_batch, H, W) * kRows * 32;
    // The backward's weight-gradient partial rows (W4, W3, W2, W1).
    const int gR[4] = {2 * out_grad_blocks(), kW32Blocks, kW32Blocks, kW1Blocks};
    const int gn[4] = {kOutRow, kW32Row, kW32Row, kW1Row};
    int64_t slab_floats = 0;
    for (int i = 0; i < 4; ++i) {
        d->gpart_R[i] = gR[i];
        d->gpart_n[i] = gn[i];
        d->gslab_off[i] = slab_floats;
        slab_floats += ceil_div(gR[i], 64) * (int64_t)gn[i];
    }
    qld_status st = QLD_OK;
    if (st == QLD_OK) st = dalloc(d, &d->params, N_ALL);
    if (st == QLD_OK) st = dalloc(d, &d->grads, N_ALL);
    if (st == QLD_OK) st = dalloc(d, &d->m, N_ALL);
    if (st == QLD_OK) st = dalloc(d, &d->v, N_ALL);
    if (st == QLD_OK) st = dalloc(d, &d->w1f, 1024);
    if (st == QLD_OK) st = dalloc(d, &d->w2f, 9 * 1024);
    if (st == QLD_OK) st = dalloc(d, &d->w2b, 9 * 1024);
    if (st == QLD_OK) st = dalloc(d, &d->w3f, 9 * 1024);
    if (st == QLD_OK) st = dalloc(d, &d->w3b, 9 * 1024);
    if (st == QLD_OK) st = dalloc(d, &d->w4, 288);
    if (st == QLD_OK) st = dalloc(d, &d->w4f, 9 * 512);
    if (st == QLD_OK) st = dalloc(d, &d->x0, npx * 2);
    if (st == QLD_OK) st = dalloc(d, &d->a1, npx * 32);
    if (st == QLD_OK) st = dalloc(d, &d->a2, npx * 32);
    if (st == QLD_OK) st = dalloc(d, &d->a3, npx * 32);
    if (st == QLD_OK) st = dalloc(d, &d->dzA, npx * 32);
    if (st == QLD_OK) st = dalloc(d, &d->dzB, npx * 32);
    if (st == QLD_OK) st = dalloc(d, &d->dzC, npx * 32);
    if (st == QLD_OK) st = dalloc(d, &d->y, npx);
    if (st == QLD_OK) st = dalloc(d, &d->dy, npx);
    if (st == QLD_OK) st = dalloc(d, &d->pool, (size_t)max_batch * 32);
    if (st == QLD_OK) st = dalloc(d, &d->gate, (size_t)max_batch);
    if (st == QLD_OK) st = dalloc(d, &d->part, (size_t)d->part_floats);
    if (st == QLD_OK) st = dalloc(d, &d->part2, (size_t)d->part_floats / 16 + 65536);
    for (int i = 0; i < 4 && st == QLD_OK; ++i) st = dalloc(d, &d->gpart[i], (size_t)gR[i] * gn[i]);
    if (st == QLD_OK) st = dalloc(d, &d->gslab, (size_t)slab_floats);
    if (st == QLD_OK) st = dalloc(d, &d->loss, 2);
    if (st == QLD_OK) st = dalloc(d, &d->lpart, kLossBlocks);
    if (st == QLD_OK) {
        for (void *p : d->allocs)
            if (hipMemset(p, 0, 64) != hipSuccess) st = QLD_E_DEVICE;
        const size_t zero_n = N_ALL * sizeof(float);
        if (hipMemset(d->params, 0, zero_n) != hipSuccess || hipMemset(d->grads, 0, zero_n) != hipSuccess ||
            hipMemset(d->m, 0, zero_n) != hipSuccess || hipMemset(d->v, 0, zero_n) != hipSuccess ||
            hipMemset(d->loss, 0, 8) != hipSuccess)
            st = QLD_E_DEVICE;
    }
    if (st != QLD_OK) {
        for (void *p : d->allocs) (void)hipFree(p);
        delete d;
        return st;
    }
    d->step = 0;
    d->last_B = 0;
    *out = d;
    return QLD_OK;
}

extern "C" qld_status qld_denoiser_info(const qld_denoiser *d, int32_t *H, int32_t *W, int32_t *max_batch) {
    clear_error();
    if (!d) {
        set_error("denoiser is NULL");
        return QLD_E_INVAL;
    }
    if (H) *H = d->H;
    if (W) *W = d->W;
    if (max_batch) *max_batch = d->max_batch;
    return QLD_OK;
}

extern "C" qld_status qld_denoiser_destroy(qld_denoiser *d) {
    clear_error();
    if (!d) return QLD_OK;
    (void)hipDeviceSynchronize();
    for (void *p : d->allocs) (void)hipFree(p);
    delete d;
    return QLD_OK;
}

extern "C" int32_t qld_denoiser_param_count(void) { return (int32_t)N_ALL; }

extern "C" qld_status qld_denoiser_set_params(qld_denoiser *d, const float *host, int32_t n) {
    clear_error();
    if (!d || !host || n != N_ALL) {
        set_error("set_params needs %lld floats", (long long)N_ALL);
        return QLD_E_INVAL;
    }
    QLD_TRY(check_hip(hipDeviceSynchronize(), "sync"));
    QLD_TRY(check_hip(hipMemcpy(d->params, host, N_ALL * sizeof(float), hipMemcpyHostToDevice), "params upload"));
    QLD_TRY(check_hip(hipMemset(d->m, 0, N_ALL * sizeof(float)), "adam reset"));
    QLD_TRY(check_hip(hipMemset(d->v, 0, N_ALL * sizeof(float)), "adam reset"));
    d->step = 0;
    QLD_TRY(pack(d, nullptr));
    return check_hip(hipDeviceSynchronize(), "pack sync");
}

extern "C" qld_status qld_denoiser_get_params(qld_denoiser *d, float *host, int32_t n) {
    clear_error();
    if (!d || !host || n != N_ALL) return QLD_E_INVAL;
    QLD_TRY(check_hip(hipDeviceSynchronize(), "sync"));
    return check_hip(hipMemcpy(host, d->params, N_ALL * sizeof(float), hipMemcpyDeviceToHost), "params download");
}

extern "C" qld_status qld_denoiser_get_grads(qld_denoiser *d, float *host, int32_t n) {
    clear_error();
    if (!d || !host || n != N_ALL) return QLD_E_INVAL;
    QLD_TRY(check_hip(hipDeviceSynchronize(), "sync"));
    return check_hip(hipMemcpy(host, d->grads, N_ALL * sizeof(float), hipMemcpyDeviceToHost), "grads download");
}

extern "C" qld_status qld_denoiser_tensor(qld_denoiser *d, int32_t which, void **ptr, int64_t *count) {
    clear_error();
    if (!d || !ptr) return QLD_E_INVAL;
    const int64_t npx = (int64_t)d->max_batch * d->H * d->W;
    void *p = nullptr;
    int64_t c = 0;
    switch (which) {
        case 0: p = d->x0; c = npx * 2; break;     // bf16 input
        case 1: p = d->a1; c = npx * 32; break;    // bf16 activations
        case 2: p = d->a2; c = npx * 32; break;
        case 3: p = d->a3; c = npx * 32; break;
        case 4: p = d->y; c = npx; break;          // f32 output
        case 5: p = d->dzA; c = npx * 32; break;   // bf16 gradient dz3
        case 6: p = d->dzB; c = npx * 32; break;   // bf16 gradient dz2
        case 7: p = d->pool; c = (int64_t)d->max_batch * 32; break;
        case 8: p = d->gate; c = d->max_batch; break;
        case 9: p = d->loss; c = 2; break;
        case 10: p = d->dzC; c = npx * 32; break;  // bf16 gradient dz1
        default: set_error("unknown tensor %d", which); return QLD_E_INVAL;
    }
    *ptr = p;
    if (count) *count = c;
    return QLD_OK;
}

extern "C" qld_status qld_denoiser_forward(qld_denoiser *d, const float *x, int32_t B, float *y_out,
                                           float *gate_out, qld_hip_stream stream) {
    clear_error();
    if (!d || !x || B < 1 || B > d->max_batch) {
        set_error("forward: bad arguments (batch %d, max %d)", B, d ? d->max_batch : 0);
        return QLD_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int H = d->H, W = d->W;
    const int64_t npx = (int64_t)B * H * W;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(npx * 2, 1024), 8192)), dim3(256), 0,
                       s, x, d->x0, npx * 2);
    const int g = conv_grid(B, H, W);
    hipEvent_t ev0, ev1;
    take_kernel_timer(&ev0, &ev1);
    if (ev0) QLD_TRY(check_hip(hipEventRecord(ev0, s), "timer start"));
    hipLaunchKernelGGL(conv1_kernel, dim3(g), dim3(256), 0, s, d->x0, d->w1f, d->params + OFF_B1, d->a1, H, W);
    const int gp = conv_persistent_grid(g);
    hipLaunchKernelGGL((conv_tile_kernel<0>), dim3(gp), dim3(256), 0, s, d->a1, d->w2f, d->params + OFF_B2, nullptr,
                       d->a2, H, W, g, nullptr);
    hipLaunchKernelGGL((conv_tile_kernel<0>), dim3(gp), dim3(256), 0, s, d->a2, d->w3f, d->params + OFF_B3, nullptr,
                       d->a3, H, W, g, nullptr);
    // The output layer also leaves the gate's per-row channel sums of a3.
    hipLaunchKernelGGL((conv_tile_kernel<2>), dim3(conv_persistent_grid(g, QLD_OUT_LAYER_GROUPS_PER_CU)), dim3(256), 0,
                       s, d->a3, d->w4f, d->params + OFF_B4, nullptr, d->y, H, W, g, d->part);
    if (ev1) QLD_TRY(check_hip(hipEventRecord(ev1, s), "timer stop"));
    // Per image: its tiles' row sums in tile order, added in slabs of 64, then the slabs.
    const int rows = (g / B) * kRows, slabs = (int)ceil_div(rows, 64);
    hipLaunchKernelGGL(pool_rows_kernel, dim3(slabs, B), dim3(256), 0, s, d->part, rows, d->part2);
    hipLaunchKernelGGL(gate_fwd_kernel, dim3(B), dim3(256), 0, s, d->part2, slabs, (int64_t)H * W, d->params, d->pool,
                       d->gate);
    QLD_TRY(check_hip(hipGetLastError(), "forward launch"));
    if (y_out) QLD_TRY(check_hip(hipMemcpyAsync(y_out, d->y, npx * sizeof(float), hipMemcpyDeviceToDevice, s), "y copy"));
    if (gate_out)
        QLD_TRY(check_hip(hipMemcpyAsync(gate_out, d->gate, B * sizeof(float), hipMemcpyDeviceToDevice, s), "gate copy"));
    d->last_B = B;
    return QLD_OK;
}

extern "C" qld_status qld_denoiser_backward(qld_denoiser *d, const float *t, const float *e_a, const float *e_b,
                                            float gate_weight, int32_t B, float *loss_out, qld_hip_stream stream) {
    clear_error();
    if (!d || !t || B < 1 || B != d->last_B) {
        set_error("backward: bad arguments or no matching forward (batch %d, last forward %d)", B, d ? d->last_B : 0);
        return QLD_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int H = d->H, W = d->W;
    const int64_t npx = (int64_t)B * H * W;
    hipLaunchKernelGGL(loss_kernel, dim3(kLossBlocks), dim3(256), 0, s, d->y, t, d->dy, npx, d->lpart);
    // Output layer: dW4, db4, and dz3 = bf16(d a3 * (a3 > 0)).
    QLD_TRY(out_grad(d, B, s));
    const int g = conv_grid(B, H, W), gp = conv_persistent_grid(g);
    // Layer 3: dW3 from (a2, dz3); dz2 = bf16(conv^T(dz3, W3) * (a2 > 0)).
    QLD_TRY(dw32(d, d->a2, d->dzA, B, 1, s));   // and b3
    hipLaunchKernelGGL((conv_tile_kernel<1>), dim3(gp), dim3(256), 0, s, d->dzA, d->w3b, nullptr, d->a2, d->dzB, H, W,
                       g, nullptr);
    // Layer 2: dW2 from (a1, dz2); dz1 = bf16(conv^T(dz2, W2) * (a1 > 0)).
    QLD_TRY(dw32(d, d->a1, d->dzB, B, 2, s));   // and b2
    hipLaunchKernelGGL((conv_tile_kernel<1>), dim3(gp), dim3(256), 0, s, d->dzB, d->w2b, nullptr, d->a1, d->dzC, H, W,
                       g, nullptr);
    // Layer 1: dW1 from (x0, dz1).
    QLD_TRY(dw1(d, B, s));   // and b1
    // The weight gradients' sums, and the loss's last stage in the same launch
    // (without a gate loss the gate's gradient is zero, cleared there too).
    const LossFinish lf{d->lpart, kLossBlocks, npx, d->loss, e_a ? nullptr : d->grads + OFF_WG, e_a ? 0 : 33};
    QLD_TRY(reduce_grads(d, lf, s));
    // Gate (its own loss; its gradient reaches only Wg, bg).
    if (e_a) {
        hipLaunchKernelGGL(gate_back_kernel, dim3(1), dim3(64), 0, s, d->pool, d->gate, e_a, e_b, gate_weight, B,
                           d->grads, d->loss);
    }
    QLD_TRY(check_hip(hipGetLastError(), "backward launch"));
    if (loss_out) QLD_TRY(check_hip(hipMemcpyAsync(loss_out, d->loss, 8, hipMemcpyDeviceToDevice, s), "loss copy"));
    return QLD_OK;
}

extern "C" qld_status qld_denoiser_adam(qld_denoiser *d, float lr, float beta1, float beta2, float eps,
                                        qld_hip_stream stream) {
    clear_error();
    if (!d || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
        set_error("adam: bad hyper-parameters");
        return QLD_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    d->step += 1;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)d->step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)d->step));
    hipLaunchKernelGGL(adam_pack_kernel, dim3((unsigned)ceil_div(N_ALL, 256)), dim3(256), 0, s, d->params, d->grads,
                       d->m, d->v, lr, beta1, beta2, eps, c1, c2, d->w1f, d->w2f, d->w2b, d->w3f, d->w3b, d->w4,
                       d->w4f);
    return check_hip(hipGetLastError(), "adam launch");
}
