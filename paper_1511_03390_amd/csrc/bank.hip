// Multi-frequency lock-in bank: F lock-ins of every pixel's series at once.
//
// The paper obtains its multi-source images (Fig. 1: sources at 20, 23, 26
// and 29 Hz) by running the lock-in at each frequency, and compares the
// lock-in against a full Fourier transform of the series (Methods, Fourier
// map; "Processing Time and Speedup").  For F frequencies p_f / q of the frame
// rate the bank is one contraction
//     X[f][px] = sum_t S_t[px] (cos th_ft - i sin th_ft),
//     th_ft = 2 pi ((p_f (t0 + t)) mod q) / q,
// i.e. C[px][2F] = S^T[px][T] . B[T][2F] with B[t][2f] = cos, B[t][2f+1] = -sin.
// It runs on the matrix cores in fp32 (v_mfma_f32_16x16x4_f32: fp32 products
// and accumulation, the arithmetic of the single-frequency float path):
//   * A operand (16 pixels x 4 frames): lane (m, kb) holds sample (frame kb,
//     pixel m), read straight from the time-major stack (16 consecutive
//     pixels of a frame per 16 lanes);
//   * B operand (4 frames x 16 columns): from the table, staged in LDS in
//     chunks of 32 frames and shared by the work-group's four waves;
//   * a wave owns 64 pixels (4 row blocks) x all 2F columns (F <= 32 per
//     launch; larger banks are split into groups of 32 frequencies).
// Frame operand, fast path (uint16, 16-byte aligned, W, row pitch and frame
// stride multiples of 8): a wave loads its 64 pixels x 32 frames per chunk
// with four 16-byte loads per lane (a 4 KiB tile), issued one chunk ahead,
// converts them to float into a padded per-wave LDS tile and the MFMAs read
// the A operand from there.  Otherwise each lane gathers its samples with
// 2-byte loads.  Measured on MI355X: the gathers bound the kernel (with the
// frame loads taken out it ran twice as fast).
// The table is built per call in double from the exact integer angle and
// rounded to float, like the single-frequency path.
#include <vector>

#include "qld_internal.hpp"

namespace qld {
namespace {

typedef float f32x4b __attribute__((ext_vector_type(4)));

constexpr int kBankBlock = 256;     // 4 waves x 64 pixels
constexpr int kMaxF = 32;           // frequencies per launch
constexpr int kTChunk = 32;         // frames per staged table chunk
constexpr int kTabStride = 80;      // floats per staged table row: the 4 rows a wave reads fall in different banks

// tab[t][2f] = cos, tab[t][2f+1] = -sin of 2 pi r / q, r = (p_f (t0 + t)) mod q; columns padded to ncol.
__global__ __launch_bounds__(256) void bank_table_kernel(const int32_t *__restrict__ p, int32_t F, int32_t q,
                                                         int32_t t0, int32_t T, int32_t ncol, float *__restrict__ tab) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)T * ncol) return;
    const int64_t t = i / ncol;
    const int n = (int)(i % ncol), f = n >> 1;
    float v = 0.f;
    if (f < F) {
        const int64_t r = (((int64_t)p[f] * ((int64_t)t0 + t)) % q + q) % q;
        double s, c;
        sincospi(2.0 * (double)r / (double)q, &s, &c);
        v = (n & 1) ? (float)(-s) : (float)c;
    }
    tab[i] = v;
}

template <typename T, int NCB>
__global__ __launch_bounds__(kBankBlock) void bank_kernel(const T *__restrict__ frames, int64_t row_pitch,
                                                          int64_t frame_stride, int H, int W, int n_frames,
                                                          const float *__restrict__ tab, int F,
                                                          float *__restrict__ re, float *__restrict__ im) {
    constexpr int NCOL = NCB * 16;
    __shared__ float tl[kTChunk][kTabStride];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, m = lane & 15, kb = lane >> 4;
    const int64_t npx = (int64_t)H * W;
    const int64_t px0 = (int64_t)blockIdx.x * kBankBlock + wave * 64;
    // The four pixels this lane loads (one per 16-row block) and their offsets.
    int64_t off[4];
    bool ok[4];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) {
        const int64_t p = px0 + pb * 16 + m;
        ok[pb] = p < npx;
        const int64_t pc = ok[pb] ? p : 0;
        off[pb] = (pc / W) * row_pitch + pc % W;
    }
    f32x4b acc[4][NCB];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[pb][cb] = f32x4b{0.f, 0.f, 0.f, 0.f};

    for (int tc = 0; tc < n_frames; tc += kTChunk) {
        __syncthreads();                                  // the previous chunk's readers are done
        for (int i = t; i < kTChunk * NCOL; i += kBankBlock) {
            const int tt = i / NCOL, n = i % NCOL;
            tl[tt][n] = tc + tt < n_frames ? tab[(int64_t)(tc + tt) * NCOL + n] : 0.f;
        }
        __syncthreads();
#pragma unroll 2   // measured: deeper unrolling (8) is slower at 32 frequencies
        for (int ks = 0; ks < kTChunk; ks += 4) {
            const int tf = tc + ks + kb;                  // this lane's frame
            const bool in_t = tf < n_frames;
            const T *fp = frames + (int64_t)(in_t ? tf : 0) * frame_stride;
            float a[4];
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) a[pb] = (in_t && ok[pb]) ? (float)fp[off[pb]] : 0.f;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const float b = tl[ks + kb][cb * 16 + m];
#pragma unroll
                for (int pb = 0; pb < 4; ++pb)
                    acc[pb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[pb], b, acc[pb][cb], 0, 0, 0);
            }
        }
    }
    // D[row = 4 kb + i][col = m]: pixel px0 + 16 pb + 4 kb + i, column 16 cb + m.
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int n = cb * 16 + m, f = n >> 1;
            if (f >= F) continue;
            float *dst = (n & 1) ? im : re;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t p = px0 + pb * 16 + 4 * kb + i;
                if (p < npx) dst[(int64_t)f * npx + p] = acc[pb][cb][i];
            }
        }
}

constexpr int kXStride = 80;        // floats per staged frame row of a wave's tile (64 pixels + padding)

typedef uint32_t u32x4b __attribute__((ext_vector_type(4)));
typedef float f32x4s __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8b __attribute__((ext_vector_type(8)));

template <int NCB>
__global__ __launch_bounds__(kBankBlock) void bank_vec_kernel(const uint16_t *__restrict__ frames, int64_t row_pitch,
                                                              int64_t frame_stride, int H, int W, int n_frames,
                                                              const float *__restrict__ tab, int F,
                                                              float *__restrict__ re, float *__restrict__ im) {
    constexpr int NCOL = NCB * 16;
    __shared__ __attribute__((aligned(16))) float tl[kTChunk][kTabStride];
    __shared__ __attribute__((aligned(16))) float xa[kBankBlock / 64][kTChunk][kXStride];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, m = lane & 15, kb = lane >> 4;
    const int64_t npx = (int64_t)H * W;
    const int64_t px0 = (int64_t)blockIdx.x * kBankBlock + wave * 64;
    // Tile loads: lane (fr, c) reads pixels px0 + 8c .. +7 of frames fr, fr + 8, fr + 16, fr + 24 of
    // the chunk.  W is a multiple of 8, so a group of 8 never crosses a row and is all in or all out.
    const int c = lane & 7, fr = lane >> 3;
    const int64_t pc = px0 + 8 * c;
    const bool okc = pc < npx;
    const int64_t offc = okc ? (pc / W) * row_pitch + pc % W : 0;
    float(*tile)[kXStride] = xa[wave];

    u32x4b v[4];
    auto load_chunk = [&](int tc) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = tc + fr + 8 * i;
            const bool ok = okc && f < n_frames;
            const uint16_t *src = frames + (int64_t)(ok ? f : 0) * frame_stride + offc;
            u32x4b d = __builtin_nontemporal_load(reinterpret_cast<const u32x4b *>(src));
            v[i] = ok ? d : u32x4b{0u, 0u, 0u, 0u};
        }
    };
    f32x4b acc[4][NCB];
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[pb][cb] = f32x4b{0.f, 0.f, 0.f, 0.f};

    // The chunk's table rows, also fetched one chunk ahead: element t + 256 j of the chunk.
    constexpr int kTabPer = kTChunk * NCOL / kBankBlock;
    float tv[kTabPer];
    auto load_tab = [&](int tc) {
#pragma unroll
        for (int j = 0; j < kTabPer; ++j) {
            const int i = t + kBankBlock * j, tt = i / NCOL;
            tv[j] = tc + tt < n_frames ? tab[(int64_t)(tc + tt) * NCOL + i % NCOL] : 0.f;
        }
    };

    load_chunk(0);
    load_tab(0);
    for (int tc = 0; tc < n_frames; tc += kTChunk) {
        __syncthreads();                                  // the previous chunk's readers are done
#pragma unroll
        for (int j = 0; j < kTabPer; ++j) {
            const int i = t + kBankBlock * j;
            tl[i / NCOL][i % NCOL] = tv[j];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f32x4s lo, hi;
            lo[0] = (float)(v[i][0] & 0xffffu);
            lo[1] = (float)(v[i][0] >> 16);
            lo[2] = (float)(v[i][1] & 0xffffu);
            lo[3] = (float)(v[i][1] >> 16);
            hi[0] = (float)(v[i][2] & 0xffffu);
            hi[1] = (float)(v[i][2] >> 16);
            hi[2] = (float)(v[i][3] & 0xffffu);
            hi[3] = (float)(v[i][3] >> 16);
            *reinterpret_cast<f32x4s *>(&tile[fr + 8 * i][8 * c]) = lo;
            *reinterpret_cast<f32x4s *>(&tile[fr + 8 * i][8 * c + 4]) = hi;
        }
        if (tc + kTChunk < n_frames) {                    // next chunk in flight during the MFMAs
            load_chunk(tc + kTChunk);
            load_tab(tc + kTChunk);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kTChunk; ks += 4) {
            float a[4];
#pragma unroll
            for (int pb = 0; pb < 4; ++pb) a[pb] = tile[ks + kb][pb * 16 + m];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const float b = tl[ks + kb][cb * 16 + m];
#pragma unroll
                for (int pb = 0; pb < 4; ++pb)
                    acc[pb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[pb], b, acc[pb][cb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int pb = 0; pb < 4; ++pb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int n = cb * 16 + m, f = n >> 1;
            if (f >= F) continue;
            float *dst = (n & 1) ? im : re;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t p = px0 + pb * 16 + 4 * kb + i;
                if (p < npx) dst[(int64_t)f * npx + p] = acc[pb][cb][i];
            }
        }
}

// ---------------------------------------------------------------------------
// bf16 matrix-core path with exact operand splitting (uint16 fast path).
//   * a sample x < 2^16 is x = xh + xl with xh = x & 0xff00, xl = x & 0xff:
//     8 significant bits each, so both are exact in bf16;
//   * a twiddle (the float table value Bf) is b1 + b2 + b3, b_i = bf16 of the
//     remaining residual (round to nearest even): 24 significant bits in all;
//   * products of bf16 values are exact in fp32, so every MFMA term xh b_i and
//     xl b_i is exact; all six per frame are accumulated in fp32.
// v_mfma_f32_16x16x32_bf16: A = 16 pixels x 32 frames (lane (m, kb) holds
// pixel m, frames 8 kb .. 8 kb + 7), B = 32 frames x 16 columns; one chunk of
// 32 frames is one k-step.  LDS rows are 32 frames + 8 padding (80 bytes).
// ---------------------------------------------------------------------------
constexpr int kBRow = 40;           // uint16 per LDS row: 32 frames + padding

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// tab3[chunk][part][ncol][32]: part i of the split of the float twiddle of frame 32 chunk + tt, column n.
__global__ __launch_bounds__(256) void bank_table3_kernel(const int32_t *__restrict__ p, int32_t F, int32_t q,
                                                          int32_t t0, int32_t T, int32_t ncol, int32_t n_chunks,
                                                          uint16_t *__restrict__ tab3) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_chunks * 32 * ncol) return;
    const int64_t t = i / ncol;
    const int n = (int)(i % ncol), f = n >> 1;
    float bf = 0.f;
    if (f < F && t < T) {
        const int64_t r = (((int64_t)p[f] * ((int64_t)t0 + t)) % q + q) % q;
        double s, c;
        sincospi(2.0 * (double)r / (double)q, &s, &c);
        bf = (n & 1) ? (float)(-s) : (float)c;
    }
    const uint16_t b1 = bf16_rne(bf);
    const float r1 = bf - bf16_val(b1);
    const uint16_t b2 = bf16_rne(r1);
    const uint16_t b3 = bf16_rne(r1 - bf16_val(b2));
    const int64_t ch = t / 32, tt = t % 32;
    uint16_t *dst = tab3 + ch * 3 * ncol * 32 + (int64_t)n * 32 + tt;
    dst[0] = b1;
    dst[(int64_t)ncol * 32] = b2;
    dst[(int64_t)2 * ncol * 32] = b3;
}

// Frames are not staged: lane (m, kb) of a wave loads pixels px0 + 8m .. +7
// (16 bytes) of frames 8 kb .. 8 kb + 7 of the chunk and splits them in
// registers, which is the A operand of eight MFMAs at once (A block i, row m:
// pixel px0 + 8m + i; a wave owns 128 pixels).  Only the split table goes
// through LDS, shared by the work-group's four waves and double-buffered (one
// barrier per chunk); a wave holds the chunk's twelve table fragments while
// it walks its eight blocks.  The next chunk's frames are requested behind
// the chunk's products (holding them beside the current ones takes more
// registers than two waves per SIMD have); the SIMD's other wave covers them.
// Measured at 1024 x 1024 x 1024, 32 frequencies: 1.12 -> 0.92 ms per call
// against the first version, which staged the frames transposed in LDS (its
// stores conflicted across banks for about half the kernel's time).  Frames
// one or two chunks ahead at 64 pixels per wave, or the table read straight
// from memory with no barrier, measured 0.92-1.1 ms: the kernel is held about
// equally by the VALU split, the MFMA products and the frame stream, which
// overlap only in part.
constexpr int kBf16Px = 128;                     // pixels per wave
constexpr int kBf16Block = 4 * kBf16Px;          // pixels per work-group

template <int NCB>
__global__ __launch_bounds__(256, 2) void bank_bf16_kernel(const uint16_t *__restrict__ frames, int64_t row_pitch,
                                                           int64_t frame_stride, int H, int W, int n_frames,
                                                           const uint16_t *__restrict__ tab3, int F,
                                                           float *__restrict__ re, float *__restrict__ im) {
    constexpr int NCOL = NCB * 16;
    constexpr int kPieces = 3 * NCOL * 4;                    // 16-byte pieces of a chunk's table
    constexpr int kPiecesPer = (kPieces + 255) / 256;
    __shared__ __attribute__((aligned(16))) uint16_t tb[2][3][NCOL][kBRow];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, m = lane & 15, kb = lane >> 4;
    const int64_t npx = (int64_t)H * W;
    const int64_t px0 = (int64_t)blockIdx.x * kBf16Block + wave * kBf16Px;
    // W is a multiple of 8, so the lane's 8 pixels never cross a row and are all in or all out.
    const int64_t pc = px0 + 8 * m;
    const bool okc = pc < npx;
    const int64_t offc = okc ? (pc / W) * row_pitch + pc % W : 0;
    const int n_chunks = (n_frames + kTChunk - 1) / kTChunk;

    u32x4b v[8], tv[kPiecesPer];
    auto load = [&](int ch) {
        const int tc = ch * kTChunk + 8 * kb;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int f = tc + e;
            const bool ok = okc && f < n_frames;
            const uint16_t *src = frames + (int64_t)(ok ? f : 0) * frame_stride + offc;
            const u32x4b d = __builtin_nontemporal_load(reinterpret_cast<const u32x4b *>(src));
            v[e] = ok ? d : u32x4b{0u, 0u, 0u, 0u};
        }
        const u32x4b *src = reinterpret_cast<const u32x4b *>(tab3 + (int64_t)ch * 3 * NCOL * 32);
#pragma unroll
        for (int j = 0; j < kPiecesPer; ++j) {
            const int i = t + 256 * j;
            if (i < kPieces) tv[j] = src[i];
        }
    };
    f32x4b acc[8][NCB];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[i][cb] = f32x4b{0.f, 0.f, 0.f, 0.f};

    load(0);
    for (int ch = 0; ch < n_chunks; ++ch) {
        const int buf = ch & 1;
#pragma unroll
        for (int j = 0; j < kPiecesPer; ++j) {
            const int i = t + 256 * j;
            if (i < kPieces) {
                const int part = i / (NCOL * 4), col = (i / 4) % NCOL, qq = i % 4;
                *reinterpret_cast<u32x4b *>(&tb[buf][part][col][8 * qq]) = tv[j];
            }
        }
        __syncthreads();                                  // this chunk's table is in LDS
        bf16x8b b[3][NCB];
#pragma unroll
        for (int bi = 0; bi < 3; ++bi)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
                b[bi][cb] = __builtin_bit_cast(bf16x8b, *reinterpret_cast<const u32x4b *>(&tb[buf][bi][16 * cb + m][8 * kb]));
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            // Pixel i of the lane's eight over frames 8 kb .. +7: x = (x & 0xff00) + (x & 0xff), each
            // exact in bf16; two frames per word.
            const int w = i >> 1, sh = (i & 1) * 16;
            u32x4b ah, al;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const uint32_t x0 = v[2 * d][w] >> sh, x1 = v[2 * d + 1][w] >> sh;
                const uint32_t l0 = __float_as_uint((float)(x0 & 0xffu)), l1 = __float_as_uint((float)(x1 & 0xffu));
                const uint32_t h0 = __float_as_uint((float)(x0 & 0xff00u)),
                               h1 = __float_as_uint((float)(x1 & 0xff00u));
                al[d] = (l0 >> 16) | (l1 & 0xffff0000u);
                ah[d] = (h0 >> 16) | (h1 & 0xffff0000u);
            }
#pragma unroll
            for (int bi = 0; bi < 3; ++bi)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    acc[i][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8b, ah), b[bi][cb],
                                                                         acc[i][cb], 0, 0, 0);
                    acc[i][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8b, al), b[bi][cb],
                                                                         acc[i][cb], 0, 0, 0);
                }
        }
        if (ch + 1 < n_chunks) load(ch + 1);             // next chunk requested behind the products
    }
    // D[row = 4 kb + r][col = m] of block i: pixel px0 + 8 (4 kb + r) + i, column 16 cb + m; the
    // lane's 32 values of a column are pixels px0 + 32 kb .. +31 (16-byte stores where aligned).
    const bool vec_out = ((reinterpret_cast<uintptr_t>(re) | reinterpret_cast<uintptr_t>(im)) & 15) == 0 &&
                         npx % 4 == 0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int n = cb * 16 + m, f = n >> 1;
        if (f >= F) continue;
        float *dst = ((n & 1) ? im : re) + (int64_t)f * npx + px0 + 32 * kb;
        const int64_t left = npx - (px0 + 32 * kb);
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int hq = 0; hq < 2; ++hq) {
                const int o0 = 8 * r + 4 * hq;
                const f32x4b o = {acc[4 * hq][cb][r], acc[4 * hq + 1][cb][r], acc[4 * hq + 2][cb][r],
                                  acc[4 * hq + 3][cb][r]};
                if (vec_out && left >= o0 + 4) *reinterpret_cast<f32x4b *>(dst + o0) = o;
                else
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (o0 + i < left) dst[o0 + i] = o[i];
            }
    }
}

hipError_t launch_bank_bf16(int ncb, const uint16_t *frames, int64_t rp, int64_t fs, int H, int W, int n,
                            const uint16_t *tab3, int F, float *re, float *im, hipStream_t s) {
    const int64_t npx = (int64_t)H * W;
    const dim3 grid((unsigned)ceil_div(npx, kBf16Block));
    switch (ncb) {
        case 1: hipLaunchKernelGGL((bank_bf16_kernel<1>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab3, F, re, im); break;
        case 2: hipLaunchKernelGGL((bank_bf16_kernel<2>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab3, F, re, im); break;
        case 3: hipLaunchKernelGGL((bank_bf16_kernel<3>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab3, F, re, im); break;
        default: hipLaunchKernelGGL((bank_bf16_kernel<4>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab3, F, re, im); break;
    }
    return hipGetLastError();
}

hipError_t launch_bank_vec(int ncb, const uint16_t *frames, int64_t rp, int64_t fs, int H, int W, int n,
                           const float *tab, int F, float *re, float *im, hipStream_t s) {
    const int64_t npx = (int64_t)H * W;
    const dim3 grid((unsigned)ceil_div(npx, kBankBlock));
    switch (ncb) {
        case 1: hipLaunchKernelGGL((bank_vec_kernel<1>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab, F, re, im); break;
        case 2: hipLaunchKernelGGL((bank_vec_kernel<2>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab, F, re, im); break;
        case 3: hipLaunchKernelGGL((bank_vec_kernel<3>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab, F, re, im); break;
        default: hipLaunchKernelGGL((bank_vec_kernel<4>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab, F, re, im); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bank(int ncb, const T *frames, int64_t rp, int64_t fs, int H, int W, int n, const float *tab, int F,
                       float *re, float *im, hipStream_t s) {
    const int64_t npx = (int64_t)H * W;
    const dim3 grid((unsigned)ceil_div(npx, kBankBlock));
    switch (ncb) {
        case 1: hipLaunchKernelGGL((bank_kernel<T, 1>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab, F, re, im); break;
        case 2: hipLaunchKernelGGL((bank_kernel<T, 2>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab, F, re, im); break;
        case 3: hipLaunchKernelGGL((bank_kernel<T, 3>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab, F, re, im); break;
        default: hipLaunchKernelGGL((bank_kernel<T, 4>), grid, dim3(kBankBlock), 0, s, frames, rp, fs, H, W, n, tab, F, re, im); break;
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace qld

using namespace qld;

extern "C" qld_status qld_lockin_bank(const void *frames, const qld_frame_desc *d, int32_t n_frames, int32_t n_freq,
                                      const int32_t *p_host, int32_t q, int32_t t0, float *re, float *im,
                                      qld_hip_stream stream) {
    clear_error();
    int eb = 0;
    QLD_TRY(check_desc(d, &eb));
    if (n_frames < 1 || n_freq < 0) {
        set_error("qld_lockin_bank needs n_frames >= 1 and n_freq >= 0 (got %d, %d)", n_frames, n_freq);
        return QLD_E_SHAPE;
    }
    if (q < 1 || t0 < 0 || (n_freq > 0 && !p_host)) {
        set_error("qld_lockin_bank needs q >= 1, t0 >= 0 and the frequencies (got q=%d, t0=%d)", q, t0);
        return QLD_E_INVAL;
    }
    const int64_t npx = (int64_t)d->H * d->W;
    if (npx == 0 || n_freq == 0) return QLD_OK;
    if (!frames || !re || !im) {
        set_error("frames, re and im must be non-NULL");
        return QLD_E_INVAL;
    }
    if (ceil_div(npx, kBankBlock) > 0x7fffffff) {
        set_error("image too large");
        return QLD_E_SHAPE;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool vec = eb == 2 && reinterpret_cast<uintptr_t>(frames) % 16 == 0 && d->W % 8 == 0 &&
                     d->row_pitch % 8 == 0 && d->frame_stride % 8 == 0;
    for (int32_t f0 = 0; f0 < n_freq; f0 += kMaxF) {
        const int F = std::min<int32_t>(kMaxF, n_freq - f0);
        const int ncb = (int)ceil_div(2 * F, 16);
        const int ncol = ncb * 16;
        const int64_t n_chunks = ceil_div(n_frames, kTChunk);
        // Groups of more than 8 frequencies take the bf16 path; at 8 or fewer the frame staging
        // bounds both fast kernels and the fp32 one measured faster.
        const bool bf16 = vec && F > 8;
        // Float table [T][ncol], or the bf16 split table [chunk][3][ncol][32].
        const size_t tab_raw = bf16 ? sizeof(uint16_t) * (size_t)n_chunks * 3 * ncol * kTChunk
                                    : sizeof(float) * (size_t)n_frames * ncol;
        const size_t tab_b = ((tab_raw + 255) / 256) * 256;
        char *ws = static_cast<char *>(stream_workspace(s, tab_b + 256));
        if (!ws) return QLD_E_NOMEM;
        int32_t *pd = reinterpret_cast<int32_t *>(ws + tab_b);
        QLD_TRY(check_hip(hipMemcpyAsync(pd, p_host + f0, sizeof(int32_t) * F, hipMemcpyHostToDevice, s),
                          "frequency upload"));
        float *tab = reinterpret_cast<float *>(ws);
        uint16_t *tab3 = reinterpret_cast<uint16_t *>(ws);
        if (bf16)
            hipLaunchKernelGGL(bank_table3_kernel, dim3((unsigned)ceil_div(n_chunks * kTChunk * ncol, 256)), dim3(256),
                               0, s, pd, F, q, t0, n_frames, ncol, (int32_t)n_chunks, tab3);
        else
            hipLaunchKernelGGL(bank_table_kernel, dim3((unsigned)ceil_div((int64_t)n_frames * ncol, 256)), dim3(256),
                               0, s, pd, F, q, t0, n_frames, ncol, tab);
        QLD_TRY(check_hip(hipGetLastError(), "bank table kernel launch"));
        hipEvent_t ev0, ev1;
        take_kernel_timer(&ev0, &ev1);
        if (ev0) QLD_TRY(check_hip(hipEventRecord(ev0, s), "timer start"));
        hipError_t e;
        if (bf16)
            e = launch_bank_bf16(ncb, static_cast<const uint16_t *>(frames), d->row_pitch, d->frame_stride, d->H,
                                 d->W, n_frames, tab3, F, re + (int64_t)f0 * npx, im + (int64_t)f0 * npx, s);
        else if (vec)
            e = launch_bank_vec(ncb, static_cast<const uint16_t *>(frames), d->row_pitch, d->frame_stride, d->H,
                                d->W, n_frames, tab, F, re + (int64_t)f0 * npx, im + (int64_t)f0 * npx, s);
        else if (eb == 2)
            e = launch_bank(ncb, static_cast<const uint16_t *>(frames), d->row_pitch, d->frame_stride, d->H, d->W,
                            n_frames, tab, F, re + (int64_t)f0 * npx, im + (int64_t)f0 * npx, s);
        else
            e = launch_bank(ncb, static_cast<const uint8_t *>(frames), d->row_pitch, d->frame_stride, d->H, d->W,
                            n_frames, tab, F, re + (int64_t)f0 * npx, im + (int64_t)f0 * npx, s);
        QLD_TRY(check_hip(e, "bank_kernel launch"));
        if (ev1) QLD_TRY(check_hip(hipEventRecord(ev1, s), "timer stop"));
    }
    return QLD_OK;
}
