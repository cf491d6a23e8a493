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
//   * vector kernel: one lane owns 16 bytes of one row (8 uint16 or 16 uint8
//     pixels) and reads them with one global_load_dwordx4 per frame, so a wave
//     reads 1 KiB per frame, fully coalesced; rows are covered by whole 16-byte
//     lanes only, and the ragged end of each row (W mod lane width pixels) goes
//     to a scalar kernel (one lane per pixel), as do unaligned stacks;
//   * the inner loop is branch-free; the I/Q differences are accumulated in
//     packed 16-bit halves (v_pk_sub/v_pk_add) for up to 8 cycles of 12-bit
//     data (128 cycles of 8-bit data) and then folded into int32 registers,
//     which stay in VGPRs across the whole frame loop;
//   * when the image alone does not fill the GPU, the cycles are dealt
//     round-robin to S work-groups per pixel tile (cycle c to split c mod S),
//     so the whole grid still sweeps the stack as one front.  Each split
//     stores its I/Q partial with plain coalesced stores and a small kernel
//     adds the S partials of a pixel in split order (int32, exact).  Measured
//     on MI355X: int32 atomics into I/Q from the splits cost 20-30% of the
//     kernel's bandwidth at 256x256 and 512x512;
//   * per-frame statistics: each lane's sum of its samples (v_dot2_u32_u16 /
//     v_sad_u8) goes to LDS, one row per frame; every 64 frames lane j adds up
//     row j, which transposes the cross-lane reduction into plain adds, the
//     four waves' sums are added in LDS and the work-group partial stored; a
//     small kernel folds the partials into frame_sum.  Clipped samples are rare: a packed max per frame detects
//     whether any sample reaches 2^bits - 1 and only then are they counted
//     with ballots.  (The scalar kernel reduces with DPP row shifts instead.)
#include <mutex>

#include "qld_internal.hpp"

namespace qld {
namespace {


constexpr int kBlock = 256;            // lanes per work-group (4 waves)
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kXcds = 8;

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

// Reinterpret a 32-bit word as two 16-bit halves.  Takes the word by value:
// a bit_cast applied directly to an element of a vector lvalue reads element
// 0 with this compiler.
__device__ __forceinline__ u16x2 h2(uint32_t w) { return __builtin_bit_cast(u16x2, w); }

struct AccumArgs {
    const uint8_t *frames;
    int64_t rp_b;          // row pitch, bytes
    int64_t fs_b;          // frame stride, bytes
    int32_t H, W;
    int32_t n_frames;
    int32_t n_split;       // work-groups per split tile; split s takes cycles s, s+n_split, ...
    int32_t n_full;        // vector kernel: tiles 0 .. n_full-1 are not split (a multiple of kXcds)
    int32_t rot;           // phase of frame 0, mod 4
    int32_t x_begin;       // first column this kernel covers
    int32_t ncols;         // columns it covers (vector kernel: whole lanes only)
    int32_t n_tiles;       // work-group tiles over its lanes (vector kernel: wide tiles of tk tiles)
    int32_t tk;            // vector kernel: 256-lane tiles per wide tile (1, 2 or 4)
    int32_t n_units;       // (tile, split) work units, tiles rounded up to a multiple of kXcds
    int32_t row_base;      // first stats-partial row of this kernel (vector: one per wide tile, scalar: per wave)
    uint32_t top;          // 2^bits - 1
    int32_t *I;
    int32_t *Q;
    int32_t *part_iq;      // n_split > 1: [n_split][2][part_n] I/Q partials of pixels part_p0 .. part_p0+part_n-1
    int64_t part_p0, part_n;  //   (the pixels of the split tiles, in I/Q order)
    uint32_t *part_sum;    // [waves][n_frames]
    uint32_t *part_sat;
    // One-shot image (qld_lockin_image): I/Q written, not added (single pass
    // over the frames only), the amplitude written from the final sums, and
    // the frame statistics cleared by work-group 0 before the reduction adds.
    int32_t overwrite;
    float *amp;
    uint64_t *clear_sum;
    uint32_t *clear_sat;
    int32_t clear_n;
};

// x + y in two's complement, wrapping like the hardware add (no signed
// overflow in C++): the caller's running sums plus a stack's sums.
__device__ __forceinline__ int32_t add_wrap(int32_t x, int32_t y) { return (int32_t)((uint32_t)x + (uint32_t)y); }

// R = (I^2 + Q^2)^(1/2): the sum of squares exact in uint64 (|I|, |Q| < 2^31),
// one double square root, rounded to float.
__device__ __forceinline__ float amp_exact(int32_t i, int32_t q) {
    const int64_t a = i, b = q;
    return (float)__builtin_sqrt((double)((uint64_t)(a * a) + (uint64_t)(b * b)));
}

// Work-group 0 of the launch clears the statistics a one-shot image reports.
__device__ __forceinline__ void clear_stats_once(const AccumArgs &a) {
    if (a.clear_n == 0 || blockIdx.x != 0) return;
    for (int t = threadIdx.x; t < a.clear_n; t += blockDim.x) {
        if (a.clear_sum) a.clear_sum[t] = 0;
        if (a.clear_sat) a.clear_sat[t] = 0;
    }
}

// Sum of a 32-bit value over the 64 lanes of the wave, valid in lane 63:
// inclusive shifts inside each 16-lane row, then row broadcasts 15 and 31.
__device__ __forceinline__ uint32_t wave_sum_lane63(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, true);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, true);  // row_bcast:31
    return v;
}

// Per-wave, per-frame statistics buffered one frame per lane.
struct Stats {
    uint32_t buf_sum = 0, buf_sat = 0;   // lane j: values of the j-th buffered frame
    uint32_t buf_t = 0;                  // lane j: that frame's index
    int slot = 0;                        // frames buffered (uniform)
    int64_t row;                         // partial index of frame 0 for this wave

    __device__ __forceinline__ void put(uint32_t lane_sum, uint32_t wave_sat, uint32_t t) {
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)wave_sum_lane63(lane_sum), 63);
        // Lane `slot` of the buffer registers takes the (uniform) values.
        const bool mine = (int)(threadIdx.x & 63) == slot;
        buf_sum = mine ? tot : buf_sum;
        buf_sat = mine ? wave_sat : buf_sat;
        buf_t = mine ? t : buf_t;
        if (++slot == 64) flush();
    }

    __device__ __forceinline__ void flush() {
        const int lane = (int)(threadIdx.x & 63);
        if (lane < slot) {
            part_sum[row + buf_t] = buf_sum;
            part_sat[row + buf_t] = buf_sat;
        }
        slot = 0;
    }

    uint32_t *part_sum, *part_sat;
};

// Per-frame statistics of the vector kernel, transposed through LDS: each
// lane writes its lane sum of frame slot j into row j of its wave's
// [kStatsSlots][65]-word buffer (one store per frame, consecutive banks); at a
// flush lane j adds up row j (the padding column puts the lanes' reads in
// different banks), the four waves' sums meet in LDS after a work-group
// barrier (every wave of a group flushes at the same frame counts), and wave 0
// stores the work-group partial of each frame: a quarter of the partials, and
// of the reduction's reads, of one row per wave.  Slots follow the
// wave's frames in order (cycle k0 + j/4, phase j%4), so a slot's frame index
// is computed at the flush instead of being carried.  The saturation count is
// wave-uniform; it is written into lane j's register only for frames that have
// a clipped sample (rare), else stays 0.
constexpr int kStatsRow = 65;
constexpr int kStatsSlots = 64;   // frames buffered per wave between flushes (multiple of 4)

struct StatsLds {
    uint32_t buf_sat = 0;
    int slot = 0;
    int64_t k0 = 0;                      // wave cycle index of slot 0
    int64_t split = 0, S = 1;            // frame of (cycle k, phase j) = 4 (split + k S) + j
    int64_t row;
    uint32_t *lds;                       // this wave's [kStatsSlots][kStatsRow] words
    uint32_t *comb;                      // the work-group's [2][kWavesPerBlock][2][64] words
    int parity = 0;                      // comb half of this flush (the halves alternate)
    uint32_t *part_sum, *part_sat;

    __device__ __forceinline__ void put(uint32_t lane_sum) {
        lds[slot * kStatsRow + (int)(threadIdx.x & 63)] = lane_sum;
        ++slot;
    }
    __device__ __forceinline__ void sat(int j, uint32_t wave_sat) {   // slot j's clipped count
        buf_sat = (int)(threadIdx.x & 63) == j ? wave_sat : buf_sat;
    }

    __device__ __forceinline__ void flush() {
        const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
        __builtin_amdgcn_wave_barrier();
        uint32_t sum = 0;
        if (lane < slot) {
            const uint32_t *r = lds + lane * kStatsRow;
            uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
            for (int i = 0; i < 64; i += 4) {
                s0 += r[i];
                s1 += r[i + 1];
                s2 += r[i + 2];
                s3 += r[i + 3];
            }
            sum = (s0 + s1) + (s2 + s3);
        }
        uint32_t *c = comb + parity * (kWavesPerBlock * 2 * 64);
        c[(wave * 2 + 0) * 64 + lane] = sum;
        c[(wave * 2 + 1) * 64 + lane] = buf_sat;
        // A half is rewritten two flushes later, after the next flush's
        // barrier, which wave 0 reaches only once it has read this one.
        __syncthreads();
        if (wave == 0 && lane < slot) {
            uint32_t gs = 0, gc = 0;
#pragma unroll
            for (int w = 0; w < kWavesPerBlock; ++w) {
                gs += c[(w * 2 + 0) * 64 + lane];
                gc += c[(w * 2 + 1) * 64 + lane];
            }
            const int64_t t = 4 * (split + (k0 + lane / 4) * S) + lane % 4;
            part_sum[row + t] = gs;
            part_sat[row + t] = gc;
        }
        parity ^= 1;
        k0 += slot / 4;
        slot = 0;
        buf_sat = 0;
    }
};

// Lane sum of one 16-byte group of samples.
template <int ELEM>
__device__ __forceinline__ uint32_t lane_sum16(const u32x4 &d) {
    if constexpr (ELEM == 2) {
        const u16x2 one = {1, 1};
        uint32_t s = __builtin_amdgcn_udot2(h2(d[0]), one, 0u, false);
        s = __builtin_amdgcn_udot2(h2(d[1]), one, s, false);
        s = __builtin_amdgcn_udot2(h2(d[2]), one, s, false);
        return __builtin_amdgcn_udot2(h2(d[3]), one, s, false);
    } else {
        uint32_t s = __builtin_amdgcn_sad_u8(d[0], 0u, 0u);
        s = __builtin_amdgcn_sad_u8(d[1], 0u, s);
        s = __builtin_amdgcn_sad_u8(d[2], 0u, s);
        return __builtin_amdgcn_sad_u8(d[3], 0u, s);
    }
}

// Largest sample of a lane's 16-byte group, as packed 16-bit halves.
template <int ELEM>
__device__ __forceinline__ u16x2 lane_max16(const u32x4 &d) {
    if constexpr (ELEM == 2) {
        return __builtin_elementwise_max(__builtin_elementwise_max(h2(d[0]), h2(d[1])),
                                         __builtin_elementwise_max(h2(d[2]), h2(d[3])));
    } else {
        // Even and odd bytes widened to 16-bit halves.
        const uint32_t b = 0x00ff00ffu;
        u16x2 mx = h2(d[0] & b);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k) mx = __builtin_elementwise_max(mx, h2(d[k] & b));
            mx = __builtin_elementwise_max(mx, h2((d[k] >> 8) & b));
        }
        return mx;
    }
}

// ---------------------------------------------------------------------------
// Vector kernel: 16 bytes per lane.
// ---------------------------------------------------------------------------
template <int ELEM>
struct Lane16 {
    static constexpr int kPx = 16 / ELEM;
};

// Counts samples equal to top in one 16-byte group (exact; wave total).
template <int ELEM>
__device__ __forceinline__ uint32_t count_top(const u32x4 &d, uint32_t top) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if constexpr (ELEM == 2) {
            c += (uint32_t)__popcll(__ballot((d[k] & 0xffffu) == top));
            c += (uint32_t)__popcll(__ballot((d[k] >> 16) == top));
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b) c += (uint32_t)__popcll(__ballot(((d[k] >> (8 * b)) & 0xffu) == top));
        }
    }
    return c;
}

// Accumulators of one lane: int32 I/Q per pixel plus packed 16-bit partials.
template <int ELEM>
struct Acc {
    static constexpr int kPx = 16 / ELEM;
    int32_t I[kPx], Q[kPx];
    // ELEM == 2: 4 words, word k = pixels (2k, 2k+1).
    // ELEM == 1: 8 words, word k<4 = pixels (4k, 4k+2), word 4+k = (4k+1, 4k+3).
    u16x2 pi[ELEM == 2 ? 4 : 8], pq[ELEM == 2 ? 4 : 8];

    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < kPx; ++k) I[k] = Q[k] = 0;
        clear_packed();
    }
    __device__ __forceinline__ void clear_packed() {
#pragma unroll
        for (int k = 0; k < (ELEM == 2 ? 4 : 8); ++k) pi[k] = pq[k] = u16x2{0, 0};
    }
    // Fold the packed 16-bit partials (two's complement) into int32.
    __device__ __forceinline__ void fold() {
#pragma unroll
        for (int k = 0; k < (ELEM == 2 ? 4 : 8); ++k) {
            const int32_t i0 = (int16_t)pi[k][0], i1 = (int16_t)pi[k][1];
            const int32_t q0 = (int16_t)pq[k][0], q1 = (int16_t)pq[k][1];
            int a, b;
            if constexpr (ELEM == 2) {
                a = 2 * k;
                b = 2 * k + 1;
            } else {
                a = k < 4 ? 4 * k : 4 * (k - 4) + 1;
                b = a + 2;
            }
            I[a] += i0;
            I[b] += i1;
            Q[a] += q0;
            Q[b] += q1;
        }
        clear_packed();
    }
    // One cycle S0..S3 of packed words: I += S0 - S2, Q += S1 - S3 (mod 2^16 per half).
    __device__ __forceinline__ void cycle(const u32x4 &s0, const u32x4 &s1, const u32x4 &s2, const u32x4 &s3) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if constexpr (ELEM == 2) {
                pi[k] += h2(s0[k]) - h2(s2[k]);
                pq[k] += h2(s1[k]) - h2(s3[k]);
            } else {
                const uint32_t m = 0x00ff00ffu;
                pi[k] += h2(s0[k] & m) - h2(s2[k] & m);
                pq[k] += h2(s1[k] & m) - h2(s3[k] & m);
                pi[4 + k] += h2((s0[k] >> 8) & m) - h2((s2[k] >> 8) & m);
                pq[4 + k] += h2((s1[k] >> 8) & m) - h2((s3[k] >> 8) & m);
            }
        }
    }
    // Unpacked update of one frame with coefficient +1 into I (ci=1), Q (cq=1), or -1.
    __device__ __forceinline__ void frame32(const u32x4 &d, int ci, int cq) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if constexpr (ELEM == 2) {
                const int32_t lo = (int32_t)(d[k] & 0xffffu), hi = (int32_t)(d[k] >> 16);
                I[2 * k] += ci * lo;
                I[2 * k + 1] += ci * hi;
                Q[2 * k] += cq * lo;
                Q[2 * k + 1] += cq * hi;
            } else {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int32_t v = (int32_t)((d[k] >> (8 * b)) & 0xffu);
                    I[4 * k + b] += ci * v;
                    Q[4 * k + b] += cq * v;
                }
            }
        }
    }
};

__device__ __forceinline__ u32x4 ld16(const uint8_t *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
}

// Statistics of one frame of a lane's TK 16-byte groups: their lane sum into
// the LDS buffer; a packed max tells whether any sample is clipped, and only
// then are they counted with ballots.
template <int ELEM, int TK>
__device__ __forceinline__ void frame_stats_k(const u32x4 (&d)[TK], uint32_t top, StatsLds &st) {
    const int j = st.slot;
    uint32_t sum = lane_sum16<ELEM>(d[0]);
    u16x2 mx = lane_max16<ELEM>(d[0]);
#pragma unroll
    for (int k = 1; k < TK; ++k) {
        sum += lane_sum16<ELEM>(d[k]);
        mx = __builtin_elementwise_max(mx, lane_max16<ELEM>(d[k]));
    }
    st.put(sum);
    if (__ballot(max((uint32_t)mx[0], (uint32_t)mx[1]) >= top)) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < TK; ++k) c += count_top<ELEM>(d[k], top);
        st.sat(j, c);
    }
}

// PACKED: 16-bit partials hold `fold_every` cycles without overflow
// (fold_every * (2^bits - 1) <= 32767); otherwise every cycle goes to int32.
// MASKED: some lanes of this work-group are past the last vector; they read
// a valid address and zero what they read.
// TK: the work-group's unit is a wide tile of TK adjacent 256-lane tiles; a
// lane owns one 16-byte group in each (TK loads per frame).  Large images
// then fit the persistent grid in one round: every work-group sweeps the
// frames from the first to the last once, together, where several rounds of
// one tile per unit let the work-groups drift apart in the stack (2048 x
// 2048 x 256: 4 rounds at 68-72% of 8 TB/s against 82-85% for one round at
// the same frame stride).
// stats_parity: the comb half of the work-group's next statistics flush.  It
// is carried from one persistent-grid unit to the next (every wave of the
// work-group flushes equally often, so it is uniform): a unit that ends on an
// odd number of flushes must not start the next unit on the half whose read
// by wave 0 only the next flush's barrier orders.
template <int ELEM, bool STATS, bool PACKED, bool MASKED, int TK>
__device__ __forceinline__ void vec_body(const AccumArgs &a, int tile, int split, int S, uint32_t *stats_lds,
                                         uint32_t *stats_comb, int &stats_parity) {
    constexpr int kPx = 16 / ELEM;
    const int nvx = a.ncols / kPx;
    const int64_t n_vec = (int64_t)nvx * a.H;
    // This work-group owns cycles split, split + S, split + 2S, ... of its
    // tiles, so all work-groups sweep the stack together.
    const int64_t n_cyc_all = a.n_frames >> 2;
    const int64_t my = split < n_cyc_all ? (n_cyc_all - split + S - 1) / S : 0;
    const int64_t fs = a.fs_b;
    const int64_t step = 4 * S * fs;

    // Group k of the lane: its vector (row y, first column x0), recomputed
    // where needed rather than kept live through the frame loop.  A lane past
    // the last vector reads one that exists and zeroes what it reads.
    auto coords = [&](int k, int64_t &y, int &x0) {
        const int64_t t0 = ((int64_t)tile * TK + k) * kBlock;          // first vector of 256-lane tile k
        const int64_t g = t0 + threadIdx.x;
        const bool ok = !MASKED || g < n_vec;
        const int64_t gc = ok ? g : (t0 < n_vec ? t0 : 0);
        y = gc / nvx;
        x0 = a.x_begin + (int)(gc % nvx) * kPx;
        return ok;
    };
    uint32_t vmask[TK];
    const uint8_t *p[TK];
#pragma unroll
    for (int k = 0; k < TK; ++k) {
        int64_t y;
        int x0;
        vmask[k] = coords(k, y, x0) ? 0xffffffffu : 0u;
        p[k] = a.frames + y * a.rp_b + (int64_t)x0 * ELEM + 4 * (int64_t)split * fs;
    }

    Acc<ELEM> acc[TK];
#pragma unroll
    for (int k = 0; k < TK; ++k) acc[k].zero();
    StatsLds st;
    if constexpr (STATS) {
        st.part_sum = a.part_sum;
        st.part_sat = a.part_sat;
        st.row = ((int64_t)a.row_base + tile) * a.n_frames;
        st.lds = stats_lds + (threadIdx.x >> 6) * kStatsSlots * kStatsRow;
        st.comb = stats_comb;
        st.parity = stats_parity;
        st.split = split;
        st.S = S;
    }
    auto load = [&](int k, const uint8_t *q) {
        u32x4 d = ld16(q);
        if constexpr (MASKED) d &= vmask[k];
        return d;
    };
    const int fold_every = ELEM == 2 ? (int)(32767u / max(a.top, 1u)) : 128;

    int since_fold = 0;
    // One cycle (four frames, 4 x TK x 16 B per lane) per iteration.  The
    // loads are kept together ahead of the arithmetic (left to itself the
    // compiler issued three, waited, then the fourth).  Measured on MI355X:
    // four frames in flight per wave stream faster than deeper software
    // pipelining with two register sets.
    for (int64_t c = 0; c < my; ++c) {
        u32x4 s[4][TK];
#pragma unroll
        for (int k = 0; k < TK; ++k) {
            s[0][k] = load(k, p[k]);
            s[1][k] = load(k, p[k] + fs);
            s[2][k] = load(k, p[k] + 2 * fs);
            s[3][k] = load(k, p[k] + 3 * fs);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < TK; ++k) {
            p[k] += step;
            if constexpr (PACKED) {
                acc[k].cycle(s[0][k], s[1][k], s[2][k], s[3][k]);
            } else {
                acc[k].frame32(s[0][k], 1, 0);
                acc[k].frame32(s[1][k], 0, 1);
                acc[k].frame32(s[2][k], -1, 0);
                acc[k].frame32(s[3][k], 0, -1);
            }
        }
        if constexpr (PACKED) {
            if (++since_fold == fold_every) {
#pragma unroll
                for (int k = 0; k < TK; ++k) acc[k].fold();
                since_fold = 0;
            }
        }
        if constexpr (STATS) {
#pragma unroll
            for (int j = 0; j < 4; ++j) frame_stats_k<ELEM, TK>(s[j], a.top, st);
            if (st.slot == kStatsSlots) st.flush();
        }
    }
    if constexpr (PACKED) {
#pragma unroll
        for (int k = 0; k < TK; ++k) acc[k].fold();
    }
    // Partial cycle at the end of the stack: taken by the split next in turn.
    const int rem = (int)(a.n_frames & 3);
    if (rem && split == (int)(n_cyc_all % S)) {
        for (int j = 0; j < rem; ++j) {
            u32x4 sj[TK];
#pragma unroll
            for (int k = 0; k < TK; ++k) {
                int64_t y;
                int x0;
                coords(k, y, x0);
                const uint8_t *q = a.frames + y * a.rp_b + (int64_t)x0 * ELEM + (4 * n_cyc_all + j) * fs;
                sj[k] = load(k, q);
                acc[k].frame32(sj[k], j == 0 ? 1 : (j == 2 ? -1 : 0), j == 1 ? 1 : 0);
            }
            if constexpr (STATS) frame_stats_k<ELEM, TK>(sj, a.top, st);
        }
    }
    if constexpr (STATS) {
        if (st.slot) st.flush();
        stats_parity = st.parity;
    }

#pragma unroll
    for (int k = 0; k < TK; ++k) {
        int64_t y;
        int x0;
        if (!coords(k, y, x0)) continue;
        int32_t *Ip = S > 1 ? a.part_iq + 2 * a.part_n * split + (y * a.W + x0 - a.part_p0) : a.I + y * a.W + x0;
        int32_t *Qp = S > 1 ? Ip + a.part_n : a.Q + y * a.W + x0;
#pragma unroll
        for (int i = 0; i < kPx; ++i) {
            int32_t oi, oq;
            rotate_iq(a.rot, acc[k].I[i], acc[k].Q[i], oi, oq);
            if (S > 1) {
                Ip[i] = oi;
                Qp[i] = oq;
            } else {
                const int32_t ni = a.overwrite ? oi : add_wrap(Ip[i], oi), nq = a.overwrite ? oq : add_wrap(Qp[i], oq);
                Ip[i] = ni;
                Qp[i] = nq;
                if (a.amp) a.amp[y * a.W + x0 + i] = amp_exact(ni, nq);
            }
        }
    }
}

__device__ __forceinline__ void tile_and_split(const AccumArgs &a, int b, int &tile, int &split, int &S) {
    // Work unit -> (pixel tile, frame chunk), chunks of a tile on one XCD:
    // units below n_full are whole tiles; after them each tile is split S ways.
    if (b < a.n_full) {
        tile = b;
        split = 0;
        S = 1;
        return;
    }
    const int r = b - a.n_full;
    const int xcd = r % kXcds;
    const int q = r / kXcds;
    S = a.n_split;
    split = q % S;
    tile = a.n_full + (q / S) * kXcds + xcd;
}

template <int ELEM, bool STATS, bool PACKED, int TK>
__global__ __launch_bounds__(kBlock, 2) void qld_accum_kernel(AccumArgs a) {
    clear_stats_once(a);
    const int64_t n_vec = (int64_t)(a.ncols / (16 / ELEM)) * a.H;
    uint32_t *lds = nullptr, *comb = nullptr;
    if constexpr (STATS) {
        __shared__ uint32_t stats_lds[kWavesPerBlock * kStatsSlots * kStatsRow];
        __shared__ uint32_t stats_comb[2 * kWavesPerBlock * 2 * 64];
        lds = stats_lds;
        comb = stats_comb;
    }
    // Persistent grid (a multiple of kXcds work-groups): work-group b takes
    // units b, b + gridDim.x, ..., all on its own XCD.
    int parity = 0;
    for (int u = blockIdx.x; u < a.n_units; u += gridDim.x) {
        int tile, split, S;
        tile_and_split(a, u, tile, split, S);
        if (tile >= a.n_tiles) continue;
        if ((int64_t)(tile + 1) * TK * kBlock <= n_vec)
            vec_body<ELEM, STATS, PACKED, false, TK>(a, tile, split, S, lds, comb, parity);
        else vec_body<ELEM, STATS, PACKED, true, TK>(a, tile, split, S, lds, comb, parity);
    }
}

// ---------------------------------------------------------------------------
// Scalar kernel: one pixel per lane (row tails and unaligned stacks).
// ---------------------------------------------------------------------------
template <int ELEM, bool STATS>
__global__ __launch_bounds__(kBlock) void qld_accum_scalar_kernel(AccumArgs a) {
    clear_stats_once(a);
    int tile, split, S_unit;
    tile_and_split(a, blockIdx.x, tile, split, S_unit);   // n_full = 0 here: S_unit = n_split
    if (tile >= a.n_tiles) return;
    const int64_t n_px = (int64_t)a.ncols * a.H;
    const int64_t g = (int64_t)tile * kBlock + threadIdx.x;
    const bool valid = g < n_px;
    const int64_t gc = valid ? g : 0;
    const int64_t y = gc / a.ncols;
    const int x = a.x_begin + (int)(gc % a.ncols);
    const int64_t S = a.n_split;
    const int64_t n_cyc_all = a.n_frames >> 2;
    const int64_t fs = a.fs_b;
    const uint8_t *base = a.frames + y * a.rp_b + (int64_t)x * ELEM;
    const uint32_t vmask = valid ? 0xffffffffu : 0u;
    auto load = [&](int64_t t) {
        const uint8_t *q = base + t * fs;
        return (ELEM == 2 ? (uint32_t)*reinterpret_cast<const uint16_t *>(q) : (uint32_t)*q) & vmask;
    };

    Stats st;
    if constexpr (STATS) {
        st.part_sum = a.part_sum;
        st.part_sat = a.part_sat;
        st.row = ((int64_t)a.row_base + (int64_t)tile * kWavesPerBlock + (threadIdx.x >> 6)) * a.n_frames;
    }
    int32_t I = 0, Q = 0;
    // Cycles split, split + S, ... (all work-groups sweep the stack together).
    for (int64_t c = split; c < n_cyc_all; c += S) {
        const uint32_t v0 = load(4 * c), v1 = load(4 * c + 1), v2 = load(4 * c + 2), v3 = load(4 * c + 3);
        I += (int32_t)v0 - (int32_t)v2;
        Q += (int32_t)v1 - (int32_t)v3;
        if constexpr (STATS) {
            st.put(v0, (uint32_t)__popcll(__ballot(valid && v0 == a.top)), (uint32_t)(4 * c));
            st.put(v1, (uint32_t)__popcll(__ballot(valid && v1 == a.top)), (uint32_t)(4 * c + 1));
            st.put(v2, (uint32_t)__popcll(__ballot(valid && v2 == a.top)), (uint32_t)(4 * c + 2));
            st.put(v3, (uint32_t)__popcll(__ballot(valid && v3 == a.top)), (uint32_t)(4 * c + 3));
        }
    }
    const int rem = (int)(a.n_frames & 3);
    if (rem && split == (int)(n_cyc_all % S)) {
        for (int j = 0; j < rem; ++j) {
            const int64_t t = 4 * n_cyc_all + j;
            const uint32_t v = load(t);
            if (j == 0) I += (int32_t)v;
            else if (j == 1) Q += (int32_t)v;
            else I -= (int32_t)v;
            if constexpr (STATS) st.put(v, (uint32_t)__popcll(__ballot(valid && v == a.top)), (uint32_t)t);
        }
    }
    if constexpr (STATS) {
        if (st.slot) st.flush();
    }
    if (!valid) return;
    int32_t oi, oq;
    rotate_iq(a.rot, I, Q, oi, oq);
    if (a.n_split > 1) {
        int32_t *Ip = a.part_iq + 2 * a.part_n * split + (y * a.W + x - a.part_p0);
        Ip[0] = oi;
        Ip[a.part_n] = oq;
    } else {
        const int64_t o = y * a.W + x;
        const int32_t ni = a.overwrite ? oi : add_wrap(a.I[o], oi), nq = a.overwrite ? oq : add_wrap(a.Q[o], oq);
        a.I[o] = ni;
        a.Q[o] = nq;
        if (a.amp) a.amp[o] = amp_exact(ni, nq);
    }
}

// frame_sum[t] += sum over waves of part_sum[w][t] (and the same for counts).
// Grid: (ceil(T/256), ceil(n_rows/kRowsPerBlock)), 256 lanes per work-group.
constexpr int kRowsPerBlock = 16;

// Folds the partial rows: work-group (frames 256 bx .. +256, rows
// kRowsPerBlock by .. +kRowsPerBlock); the rows are read with many loads in
// flight per lane, and the integer sums combined with order-free atomics.
__global__ __launch_bounds__(256) void qld_stats_reduce_kernel(const uint32_t *ps, const uint32_t *pc,
                                                               int64_t n_rows, int32_t T,
                                                               uint64_t *frame_sum, uint32_t *frame_sat) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= T) return;
    const int64_t w0 = (int64_t)blockIdx.y * kRowsPerBlock;
    const int64_t w1 = min(n_rows, w0 + kRowsPerBlock);
    uint64_t s = 0;
    uint32_t c = 0;
#pragma unroll 16
    for (int64_t w = w0; w < w1; ++w) {
        s += ps[w * T + t];
        c += pc[w * T + t];
    }
    if (frame_sum) atomicAdd(reinterpret_cast<unsigned long long *>(frame_sum + t), (unsigned long long)s);
    if (frame_sat) atomicAdd(frame_sat + t, c);
}

// Frame-split images: per pixel, the S split partials added in split order,
// then I/Q replaced (overwrite) or added to, and the amplitude written when
// amp is non-NULL, for pixels p0 .. npx-1 (those of the split tiles).
// part: [S][2][npx - p0].
__global__ __launch_bounds__(256) void qld_iq_reduce_kernel(const int32_t *__restrict__ part, int32_t S, int64_t p0,
                                                            int64_t npx, int32_t overwrite, int32_t *__restrict__ I,
                                                            int32_t *__restrict__ Q, float *__restrict__ amp) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n = npx - p0;
    for (int64_t p = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += stride) {
        int32_t si = 0, sq = 0;
        for (int32_t k = 0; k < S; ++k) {
            si += part[2 * n * k + (p - p0)];
            sq += part[2 * n * k + n + (p - p0)];
        }
        if (!overwrite) {
            si = add_wrap(si, I[p]);
            sq = add_wrap(sq, Q[p]);
        }
        I[p] = si;
        Q[p] = sq;
        if (amp) amp[p] = amp_exact(si, sq);
    }
}

__global__ __launch_bounds__(256) void qld_amplitude_kernel(const int32_t *__restrict__ I,
                                                            const int32_t *__restrict__ Q, int64_t n,
                                                            float *__restrict__ amp) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) amp[i] = amp_exact(I[i], Q[i]);
}

template <int ELEM, bool STATS, bool PACKED>
hipError_t launch_vec_p(const AccumArgs &a, int grid, hipStream_t s) {
    // Four tiles per unit only for 16-bit packed data (the other variants
    // would not fit two waves per SIMD); the host chooses tk accordingly.
    if constexpr (ELEM == 2 && PACKED)
        if (a.tk == 4) {
            hipLaunchKernelGGL((qld_accum_kernel<ELEM, STATS, PACKED, 4>), dim3(grid), dim3(kBlock), 0, s, a);
            return hipGetLastError();
        }
    if (a.tk == 2) hipLaunchKernelGGL((qld_accum_kernel<ELEM, STATS, PACKED, 2>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((qld_accum_kernel<ELEM, STATS, PACKED, 1>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int ELEM, bool STATS>
hipError_t launch_vec(const AccumArgs &a, bool packed, int grid, hipStream_t s) {
    return packed ? launch_vec_p<ELEM, STATS, true>(a, grid, s) : launch_vec_p<ELEM, STATS, false>(a, grid, s);
}

template <int ELEM, bool STATS>
hipError_t launch_scalar(const AccumArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((qld_accum_scalar_kernel<ELEM, STATS>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Grid and frame-axis split of the vector kernel.  The grid is persistent:
// at most QLD_ACCUM_BLOCKS_PER_CU work-groups per CU, looping over (tile,
// split) units.  Measured on MI355X: one pass over the frames at 1-2
// work-groups per CU streams fastest (the whole grid sweeps the stack as one
// front); at 2160 x 2160 x 800 without statistics (2279 tiles, up to 8 groups
// per CU resident when each tile had its own group) the cap gains 3%.  With
// fewer tiles than work-groups a frame split fills the grid (at least 16
// cycles per unit).  Splitting every tile of a larger image to even out the
// rounds (2279 tiles on 512 groups: 5 rounds, the last 45% full; 9 half
// rounds split in two) measured no faster, the partials' reduction costing
// what the tail did; splitting only the tiles of the last round (see
// accumulate_impl) gains 2-4% at 2160 x 2160 x 800.
#ifndef QLD_ACCUM_BLOCKS_PER_CU
#define QLD_ACCUM_BLOCKS_PER_CU 2
#endif
int64_t accum_grid_cap() {
    return std::max<int64_t>(kXcds, ((int64_t)QLD_ACCUM_BLOCKS_PER_CU * device_cu_count()) / kXcds * kXcds);
}

int32_t choose_split(int64_t n_tiles, int32_t n_frames) {
    const int64_t G = accum_grid_cap();
    const int64_t smax = std::max<int64_t>(1, (n_frames / 4) / 16);
    if (n_tiles >= G) return 1;
    return (int32_t)std::min<int64_t>(ceil_div(G, n_tiles), smax);
}

}  // namespace
}  // namespace qld

using namespace qld;

// Scratch of qld_lockin_image_noalloc: a fixed array in device memory, one
// copy per device (loaded with this file's code object).  Host code never
// uses the array's name as an address: on the host it is only a stand-in for
// the symbol, so the device address of each device's copy is looked up with
// hipGetSymbolAddress (with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[QLD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, or nullptr (error set).
char *noalloc_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        set_error("qld_lockin_image_noalloc: no usable current device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            set_error("qld_lockin_image_noalloc: hipGetSymbolAddress of the scratch array failed (%s)",
                      hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    return g_scratch_ptr[dev];
}

// overwrite = false: (I, Q) += the stack's sums, frame statistics added.
// overwrite = true: one image: I/Q and the statistics replaced, amp (may be
// NULL) written.  Without a frame split all of it happens in the accumulation
// kernel's epilogue; with one, qld_iq_reduce_kernel adds the splits' partials
// into I/Q (or replaces them) and writes the amplitude.
// noalloc: the scratch comes from the fixed device array (noalloc_scratch)
// instead of the per-stream workspace, and a call that needs more than it
// holds is refused before anything is launched.
qld_status accumulate_impl(const void *frames, const qld_frame_desc *d, int32_t n_frames, int32_t phase0,
                           int32_t *I, int32_t *Q, float *amp, uint64_t *frame_sum, uint32_t *frame_sat,
                           bool overwrite, bool noalloc, qld_hip_stream stream) {
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
    const int lw = 16 / eb;                                 // pixels per vector lane
    const int vcols = vec ? (d->W / lw) * lw : 0;           // columns of the vector kernel
    const int scols = d->W - vcols;                         // columns of the scalar kernel

    AccumArgs a{};
    a.frames = static_cast<const uint8_t *>(frames);
    a.rp_b = rp_b;
    a.fs_b = fs_b;
    a.H = d->H;
    a.W = d->W;
    a.n_frames = n_frames;
    a.rot = ((phase0 % 4) + 4) % 4;
    a.top = (uint32_t)top;
    a.I = I;
    a.Q = Q;
    a.overwrite = overwrite ? 1 : 0;
    if (overwrite) {
        a.clear_sum = frame_sum;
        a.clear_sat = frame_sat;
    }

    AccumArgs av = a, as = a;
    const int64_t vt = vcols ? ceil_div((int64_t)(vcols / lw) * d->H, kBlock) : 0;
    const int64_t st = scols ? ceil_div((int64_t)scols * d->H, kBlock) : 0;
    if (vt > (1ll << 24) || st > (1ll << 24)) {
        set_error("image too large");
        return QLD_E_SHAPE;
    }
    // Wide tiles: with more 256-lane tiles than the persistent grid holds,
    // each work-group unit takes 2 or 4 adjacent tiles, so that one round
    // covers the image (or as much of it as 4 tiles per unit reach).
    const int64_t G = accum_grid_cap();
    // 16-bit partial sums hold at least two cycles for data of up to 14 bits.
    const bool packed = eb == 1 || top <= 16383;
    // Four tiles per unit only for packed 16-bit data (registers).
    const int tk = vt <= G ? 1 : (vt <= 2 * G || eb == 1 || !packed ? 2 : 4);
    const int64_t vw = ceil_div(vt, (int64_t)tk);          // wide tiles of the vector kernel
    av.x_begin = 0;
    av.ncols = vcols;
    av.n_tiles = (int32_t)vw;
    av.tk = tk;
    av.row_base = 0;
    as.x_begin = vcols;
    as.ncols = scols;
    as.n_tiles = (int32_t)st;
    as.tk = 1;
    as.row_base = (int32_t)vw;
    // A frame split fills the grid when an image has fewer tiles than
    // work-groups; wide tiles (tk > 1) keep as many bytes in flight as tk
    // times as many work-groups would, so they are left unsplit.
    av.n_split = tk == 1 ? choose_split(vw + st, n_frames) : 1;
    as.n_split = av.n_split;
    // Tail of the persistent grid: with more wide tiles than work-groups and
    // no scalar columns (the vector lanes then cover the pixels in flat
    // order), the wide tiles past the last whole round are split over the
    // frames so that round ends sooner; only their pixels take the partials'
    // reduction.  2160 x 2160: 2279 tiles = 570 wide tiles of 4 on 512
    // work-groups: one round, then 58 wide tiles split 8 ways.
    int64_t p_split = 0;                    // first pixel of the split tiles
    if (st == 0 && av.n_split == 1) {
        const int64_t full = (vw / G) * G, rest = vw - full;
        const int64_t s2 = rest > 0 ? std::min<int64_t>(G / rest, std::max<int64_t>(1, (n_frames / 4) / 16)) : 1;
        if (full > 0 && s2 >= 2) {
            av.n_full = (int32_t)full;
            av.n_split = (int32_t)s2;
            p_split = full * tk * kBlock * lw;
        }
    }
    // With a frame split the splits store I/Q partials and
    // qld_iq_reduce_kernel adds them (and writes amp); without one the
    // accumulation kernel's epilogue does both (for the whole tiles of a
    // split tail too).
    const bool split = av.n_split > 1;
    av.amp = as.amp = amp;
    // Only the first kernel launched clears the statistics.
    if (overwrite && (frame_sum || frame_sat)) {
        if (vt > 0) av.clear_n = n_frames;
        else as.clear_n = n_frames;
    }

    const bool stats = frame_sum || frame_sat;
    // Statistics partial rows: one per wide vector tile, one per scalar-kernel wave.
    const int64_t n_rows = vw + st * kWavesPerBlock;
    const size_t stats_b = stats ? ((sizeof(uint32_t) * 2 * (size_t)n_rows * (size_t)n_frames + 255) / 256) * 256 : 0;
    av.part_p0 = as.part_p0 = p_split;
    av.part_n = as.part_n = npx - p_split;
    const size_t iq_b = split ? sizeof(int32_t) * 2 * (size_t)av.n_split * (size_t)(npx - p_split) : 0;
    if (stats_b + iq_b > 0) {
        char *ws = nullptr;
        if (noalloc) {
            if (stats_b + iq_b > (size_t)QLD_NOALLOC_SCRATCH_BYTES) {
                set_error("qld_lockin_image_noalloc: this call needs %zu bytes of scratch, the fixed array holds %zu",
                          stats_b + iq_b, (size_t)QLD_NOALLOC_SCRATCH_BYTES);
                return QLD_E_NOMEM;
            }
            ws = noalloc_scratch();
        } else {
            ws = static_cast<char *>(stream_workspace(s, stats_b + iq_b));
        }
        if (!ws) return QLD_E_NOMEM;
        if (stats) {
            uint32_t *ps = reinterpret_cast<uint32_t *>(ws);
            av.part_sum = as.part_sum = ps;
            av.part_sat = as.part_sat = ps + (size_t)n_rows * n_frames;
        }
        if (split) av.part_iq = as.part_iq = reinterpret_cast<int32_t *>(ws + stats_b);
    }
    const int64_t uv = av.n_full + ceil_div(vw - av.n_full, kXcds) * kXcds * av.n_split;
    const int64_t gs = ceil_div(st, kXcds) * kXcds * as.n_split;
    if (uv > 0x7fffffff || gs > 0x7fffffff) {
        set_error("grid too large");
        return QLD_E_SHAPE;
    }
    av.n_units = (int32_t)uv;
    const int64_t gv = std::min<int64_t>(uv, accum_grid_cap());

    hipEvent_t ev0, ev1;
    take_kernel_timer(&ev0, &ev1);
    if (ev0) QLD_TRY(check_hip(hipEventRecord(ev0, s), "timer start"));
    hipError_t e = hipSuccess;
    if (vt > 0) {
        if (eb == 2) e = stats ? launch_vec<2, true>(av, packed, (int)gv, s) : launch_vec<2, false>(av, packed, (int)gv, s);
        else e = stats ? launch_vec<1, true>(av, packed, (int)gv, s) : launch_vec<1, false>(av, packed, (int)gv, s);
        QLD_TRY(check_hip(e, "qld_accum_kernel launch"));
    }
    if (ev1) QLD_TRY(check_hip(hipEventRecord(ev1, s), "timer stop"));
    if (st > 0) {
        if (eb == 2) e = stats ? launch_scalar<2, true>(as, (int)gs, s) : launch_scalar<2, false>(as, (int)gs, s);
        else e = stats ? launch_scalar<1, true>(as, (int)gs, s) : launch_scalar<1, false>(as, (int)gs, s);
        QLD_TRY(check_hip(e, "qld_accum_scalar_kernel launch"));
    }
    if (stats) {
        dim3 g2((unsigned)ceil_div(n_frames, 256), (unsigned)ceil_div(n_rows, kRowsPerBlock));
        hipLaunchKernelGGL(qld_stats_reduce_kernel, g2, dim3(256), 0, s, av.part_sum, av.part_sat, n_rows,
                           n_frames, frame_sum, frame_sat);
        QLD_TRY(check_hip(hipGetLastError(), "qld_stats_reduce_kernel launch"));
    }
    if (split) {
        const int64_t blocks = std::min<int64_t>(ceil_div(npx - p_split, 256), 16ll * device_cu_count());
        hipLaunchKernelGGL(qld_iq_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, av.part_iq, av.n_split,
                           p_split, npx, overwrite ? 1 : 0, I, Q, overwrite ? amp : nullptr);
        QLD_TRY(check_hip(hipGetLastError(), "qld_iq_reduce_kernel launch"));
    }
    return QLD_OK;
}

}  // namespace

extern "C" qld_status qld_accumulate(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                                     int32_t phase0, int32_t *I, int32_t *Q, uint64_t *frame_sum,
                                     uint32_t *frame_sat, qld_hip_stream stream) {
    clear_error();
    return accumulate_impl(frames, d, n_frames, phase0, I, Q, nullptr, frame_sum, frame_sat, false, false, stream);
}

extern "C" qld_status qld_lockin_image(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                                       int32_t phase0, int32_t *I, int32_t *Q, float *amp, uint64_t *frame_sum,
                                       uint32_t *frame_sat, qld_hip_stream stream) {
    clear_error();
    if (n_frames < 1) {
        set_error("qld_lockin_image needs n_frames >= 1 (got %d)", n_frames);
        return QLD_E_SHAPE;
    }
    return accumulate_impl(frames, d, n_frames, phase0, I, Q, amp, frame_sum, frame_sat, true, false, stream);
}

extern "C" qld_status qld_lockin_image_noalloc(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                                               int32_t phase0, int32_t *I, int32_t *Q, float *amp,
                                               uint64_t *frame_sum, uint32_t *frame_sat, qld_hip_stream stream) {
    clear_error();
    if (n_frames < 1) {
        set_error("qld_lockin_image_noalloc needs n_frames >= 1 (got %d)", n_frames);
        return QLD_E_SHAPE;
    }
    return accumulate_impl(frames, d, n_frames, phase0, I, Q, amp, frame_sum, frame_sat, true, true, stream);
}

namespace {

// XOR of every 8-byte word of a buffer: a plain streaming read.  Work-group b
// reads its own contiguous range, eight 16-byte nontemporal loads per lane in
// flight (32 KiB per iteration), one work-group per CU; one 64-bit atomic XOR
// per wave.  Measured on MI355X over 2 GiB: this layout reads at 7.1-7.25 TB/s,
// a grid-stride loop at 5.4-5.8 TB/s.
__global__ __launch_bounds__(256) void read_probe_kernel(const uint8_t *__restrict__ p, int64_t n16, int64_t per,
                                                         unsigned long long *out) {
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    const v4 *q = reinterpret_cast<const v4 *>(p);
    const int64_t lo = (int64_t)blockIdx.x * per, hi = lo + per < n16 ? lo + per : n16;
    v4 acc = {0u, 0u, 0u, 0u};
    int64_t i = lo + threadIdx.x;
    for (; i + 7 * 256 < hi; i += 8 * 256) {
        v4 d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) d[u] = __builtin_nontemporal_load(q + i + u * 256);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= d[u];
    }
    for (; i < hi; i += 256) acc ^= __builtin_nontemporal_load(q + i);
    unsigned long long x = ((unsigned long long)(acc[1] ^ acc[3]) << 32) | (acc[0] ^ acc[2]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x ^= __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicXor(out, x);
}

__global__ void clear_u64_kernel(unsigned long long *out) { *out = 0ull; }

}  // namespace

extern "C" qld_status qld_read_probe(const void *p, int64_t n_bytes, uint64_t *out, qld_hip_stream stream) {
    clear_error();
    if (n_bytes < 0 || n_bytes % 16 != 0 || reinterpret_cast<uintptr_t>(p) % 16 != 0) {
        set_error("qld_read_probe needs a 16-byte aligned buffer and a size in whole 16-byte units");
        return QLD_E_ALIGN;
    }
    if (!out || (n_bytes > 0 && !p)) {
        set_error("qld_read_probe: NULL buffer or output");
        return QLD_E_INVAL;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(clear_u64_kernel, dim3(1), dim3(1), 0, s, reinterpret_cast<unsigned long long *>(out));
    QLD_TRY(check_hip(hipGetLastError(), "qld_read_probe clear"));
    if (n_bytes == 0) return QLD_OK;
    const int64_t n16 = n_bytes / 16;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n16, 8 * 256), device_cu_count()));
    const int64_t per = ceil_div(n16, blocks);
    hipEvent_t ev0, ev1;
    take_kernel_timer(&ev0, &ev1);
    if (ev0) QLD_TRY(check_hip(hipEventRecord(ev0, s), "timer start"));
    hipLaunchKernelGGL(read_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint8_t *>(p),
                       n16, per, reinterpret_cast<unsigned long long *>(out));
    QLD_TRY(check_hip(hipGetLastError(), "read_probe_kernel launch"));
    if (ev1) QLD_TRY(check_hip(hipEventRecord(ev1, s), "timer stop"));
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
