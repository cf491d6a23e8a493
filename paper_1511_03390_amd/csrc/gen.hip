// Method-generated training pairs for the learned short-window path.
//
// Each training tile is a synthetic camera stack (Poisson light, four samples
// per modulation period) that is never written to memory: a lane draws the
// samples of one pixel frame by frame and feeds them straight into the
// lock-in sums I += S0 - S2, Q += S1 - S3 (Methods, R(j,k)), recording the
// short-window sums after M_S cycles and the long-window sums after M_L.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011), one
// call per pixel and cycle: counter (pixel, cycle, tile, 0), key = seed;
// word j drives the frame of phase j.
// Poisson variates by inversion against a 32-bit fixed-point CDF table per
// rate (Devroye 1986), built here on the device from the ratios
// p(k+1)/p(k) = lambda/(k+1) with explicitly rounded double operations in a
// fixed order, so the table is reproducible bit for bit:
//   m = floor(lambda); W = ceil(12 sqrt(lambda)) + 10; lo = max(0, m-W); hi = m+W
//   w[m] = 1; w[k] = (w[k-1] lambda)/k (k > m); w[k] = (w[k+1] (k+1))/lambda (k < m)
//   total = sum w (ascending k); thr[k] = min(floor(cum_k/total * 2^32), 2^32-1), k < hi
//   X(u) = lo + #{k : thr[k] <= u}
// The count #{k : thr[k] <= u} is read from a two-level index built with the
// table, so that almost every sample costs two LDS reads and one compare:
//   level 1, 512 buckets of width 2^23 (u >> 23): per bucket the count at its
//     start and the resolution 2^kb (1 <= kb <= 8) of its level-2 part;
//   level 2, per bucket 2^kb equal sub-buckets: per sub-bucket its count at
//     the start relative to the bucket's and, if one threshold falls inside,
//     that threshold's low 23 bits, so the count is the start count plus one
//     comparison of u's low 23 bits.
// kb is the least resolution at which every sub-bucket of the bucket holds at
// most one threshold (the largest allowed, 8, where none does, and lower
// everywhere when the level-2 parts would overflow their LDS budget).  The
// sub-buckets that still hold several thresholds (in the far tails, where
// thresholds crowd at 0 and 2^32 - 1; a few per 10^5 samples) carry their
// count range instead, searched in the threshold array in global memory.
//
// Where no sample can reach the clamp (lo + n <= 2^bits - 1 for all eight
// rates of a tile), the per-sample sums are taken over the counts alone and
// each rate's lo is added once per window at the end (M lo per phase), which
// is the same integer.
#include <algorithm>
#include <cmath>
#include <cstddef>

#include "qld_internal.hpp"

namespace qld {
namespace {

constexpr int kTableMax = 2048;     // thresholds per rate (lambda up to ~6900)
constexpr int kBucketShift = 23;    // level 1: bucket u >> 23
constexpr int kBuckets = 1 << (32 - kBucketShift);
constexpr int kSubBitsMax = 8;      // level 2: at most 2^8 sub-buckets per bucket
constexpr int kL2Max = 1984;        // level-2 entries per table (eight tables' two levels in 78 KB of LDS)
constexpr uint32_t kLowMask = (1u << kBucketShift) - 1;
constexpr uint32_t kSlow = 511u;    // level-2 delta marking a sub-bucket that is searched
constexpr int kBlock = 1024;        // 16 waves; two work-groups per CU
constexpr double kRateMax = 6000.0;  // tables of at most kTableMax thresholds

// Level-1 entry: bits 0-4 = 32 - kb (the right shift that takes u << 9 to the
// sub-bucket index), bits 5-16 = (count at the bucket start) - 1 as a 12-bit
// two's complement, bits 17-31 = word offset of the bucket's level-2 part
// (within the table's level 2 in memory; within LDS in the kernel).
// Level-2 entry: bits 23-31 = d, bits 0-22 = off, with
//   count(u) = (count at bucket start) - 1 + d + [u & kLowMask >= off]:
//   no threshold in the sub-bucket: d = c_s - base, off = 0;
//   one threshold t in it:          d = c_s - base + 1, off = t & kLowMask;
// (c_s the count at the sub-bucket's start, base the bucket's).  d = kSlow:
// several thresholds; bits 0-11 = c_s, bits 12-22 = their number (2047: up to
// the end of the table), searched in thr.
struct Table {
    int32_t lo, n;                  // n thresholds
    int32_t l2n, pad;               // level-2 entries used
    uint32_t l1[kBuckets];
    uint32_t l2[kL2Max];
    uint32_t thr[kTableMax];
};

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4]) {
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u, kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
    // Each round's two 32 x 32 -> 64-bit products are taken whole (one
    // v_mad_u64_u32 each instead of separate low and high multiplies).
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kM0 * c0, p1 = (uint64_t)kM1 * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kW0;
        k1 += kW1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// One work-group builds one table.  The sequential parts run exactly in the
// order the definition fixes: the ratio recurrence upward from m on lane 0
// and downward on lane 1 (the two chains are independent), then the
// ascending partial sums on lane 0, whose last one plus the final weight is
// the ascending total.  All threads then form the thresholds and the index.
constexpr int kBuildThreads = 256;

__global__ __launch_bounds__(kBuildThreads) void build_tables_kernel(const double *__restrict__ rates,
                                                                     int32_t n_rates, Table *__restrict__ tables) {
    __shared__ double wk[kTableMax + 1];
    __shared__ uint32_t sthr[kTableMax];
    __shared__ uint16_t cb[kBuckets], ce[kBuckets];   // counts at each bucket's start and end
    __shared__ uint16_t l2off[kBuckets];
    __shared__ uint8_t kb[kBuckets];
    __shared__ int32_t scan[kBuildThreads];
    __shared__ double tot;
    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    if (t >= n_rates) return;
    const double lam = rates[t];
    Table &T = tables[t];
    const int32_t m = (int32_t)floor(lam);
    const int32_t w = (int32_t)ceil(__dmul_rn(12.0, __dsqrt_rn(lam))) + 10;
    const int32_t lo = m - w < 0 ? 0 : m - w;
    const int32_t hi = m + w;
    const int32_t n = hi - lo;                       // thresholds k = lo .. hi-1
    if (tid < 2) {
        // Lane 0: w[k] = (w[k-1] lam) / k, k = m+1 .. hi; lane 1: w[k] = (w[k+1] (k+1)) / lam, k = m-1 .. lo.
        const bool up = tid == 0;
        const int32_t steps = up ? hi - m : m - lo;
        double prev = 1.0;
        if (up) wk[m - lo] = 1.0;
        for (int32_t st = 1; st <= steps; ++st) {
            const int32_t k = up ? m + st : m - st;
            const double mul = up ? lam : (double)(k + 1), div = up ? (double)k : lam;
            prev = __ddiv_rn(__dmul_rn(prev, mul), div);
            wk[k - lo] = prev;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double cum = 0.0;
#pragma unroll 8
        for (int32_t i = 0; i < n; ++i) {
            cum = __dadd_rn(cum, wk[i]);
            wk[i] = cum;                              // wk now holds the partial sums
        }
        tot = __dadd_rn(cum, wk[n]);
        T.lo = lo;
        T.n = n;
    }
    __syncthreads();
    const double total = tot;
    for (int32_t i = tid; i < n; i += kBuildThreads) {
        const double f = floor(__dmul_rn(__ddiv_rn(wk[i], total), 4294967296.0));
        const uint32_t v = f >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)f;
        sthr[i] = v;
        T.thr[i] = v;
    }
    __syncthreads();
    auto count_le = [&](uint32_t v, int32_t a, int32_t b) {   // #{thr <= v}, known to lie in [a, b]
        while (a < b) {
            const int32_t mid = (a + b) >> 1;
            if (sthr[mid] <= v) a = mid + 1;
            else b = mid;
        }
        return a;
    };
    // Per bucket: the counts at its ends, and the least resolution at which
    // no two distinct thresholds inside share a sub-bucket (sub-bucket of t:
    // (t - 1 - start) >> (23 - kb); a threshold at a sub-bucket's start is
    // counted there, so this can only overstate what is needed).
    for (int g = tid; g < kBuckets; g += kBuildThreads) {
        const uint32_t b0 = (uint32_t)g << kBucketShift;
        const int32_t c0 = count_le(b0, 0, n), c1 = count_le(b0 + kLowMask, c0, n);
        cb[g] = (uint16_t)c0;
        ce[g] = (uint16_t)c1;
        int k = 1;
        for (int32_t i = c0; i + 1 < c1; ++i) {
            const uint32_t y1 = sthr[i] - 1u - b0, y2 = sthr[i + 1] - 1u - b0;
            if (y1 != y2) k = max(k, kBucketShift - (31 - __clz((int)(y1 ^ y2))));
        }
        kb[g] = (uint8_t)min(k, kSubBitsMax);
    }
    __syncthreads();
    // Level-2 layout: exclusive scan of the part sizes (two buckets per
    // thread), lowering the resolution cap until the parts fit the budget.
    int32_t size = 0;
    for (int cap = kSubBitsMax;; --cap) {
        const int g0 = 2 * tid;
        const int32_t s0 = 1 << min((int)kb[g0], cap), s1 = 1 << min((int)kb[g0 + 1], cap);
        scan[tid] = s0 + s1;
        __syncthreads();
        for (int o = 1; o < kBuildThreads; o <<= 1) {
            const int32_t v = tid >= o ? scan[tid - o] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        size = scan[kBuildThreads - 1];
        const int32_t excl = scan[tid] - s0 - s1;
        if (size <= kL2Max || cap == 1) {
            l2off[g0] = (uint16_t)excl;
            l2off[g0 + 1] = (uint16_t)(excl + s0);
            kb[g0] = (uint8_t)min((int)kb[g0], cap);
            kb[g0 + 1] = (uint8_t)min((int)kb[g0 + 1], cap);
            break;
        }
        __syncthreads();
    }
    if (tid == 0) T.l2n = size;
    __syncthreads();
    for (int32_t e = tid; e < size; e += kBuildThreads) {
        int32_t ga = 0, gb = kBuckets;                // last bucket whose part starts at or before e
        while (gb - ga > 1) {
            const int32_t mid = (ga + gb) >> 1;
            if ((int32_t)l2off[mid] <= e) ga = mid;
            else gb = mid;
        }
        const int g = ga;
        const uint32_t sw = 1u << (kBucketShift - kb[g]);
        const uint32_t s0 = ((uint32_t)g << kBucketShift) + (uint32_t)(e - l2off[g]) * sw;
        const int32_t base = cb[g];
        const int32_t cs = count_le(s0, base, ce[g]), span = count_le(s0 + (sw - 1), cs, ce[g]) - cs;
        const int32_t d = cs - base + span;
        T.l2[e] = span <= 1 && d < (int32_t)kSlow
                      ? ((uint32_t)d << kBucketShift) | (span ? sthr[cs] & kLowMask : 0u)
                      : (kSlow << kBucketShift) | ((uint32_t)min(span, 2047) << 12) | (uint32_t)cs;
    }
    for (int g = tid; g < kBuckets; g += kBuildThreads)
        T.l1[g] = ((uint32_t)l2off[g] << 17) | (((uint32_t)cb[g] - 1u) & 0xFFFu) << 5 | (uint32_t)(32 - kb[g]);
}

struct GenArgs {
    const uint8_t *mask;      // [n][H][W]
    const Table *tables;      // [n][8]: (mask state, phase)
    int32_t n_tiles, H, W, M_S, M_L;
    int32_t blocks_per_tile;
    uint32_t tile0, key0, key1;
    uint32_t top;
    int32_t *I_S, *Q_S, *I_L, *Q_L;
    unsigned long long *sum_S, *sum_L;
    uint32_t *psum_S, *psum_L;        // per-pixel sample sums (may be NULL)
};

// LDS of gen_pairs_kernel: the eight level-2 arrays at a stride of kL2Max
// words, then the eight level-1 arrays.
constexpr int kL1Words = 8 * kL2Max;
constexpr size_t kGenLds = (size_t)8 * (kL2Max + kBuckets) * 4;
static_assert(kL1Words < (1 << 15), "level-2 word offsets must fit 15 bits");

// Count in a sub-bucket that holds several thresholds: binary search of thr
// between the entry's start count and its end (rare; global memory).
__device__ __forceinline__ int32_t count_searched(const Table *__restrict__ T, uint32_t e2, uint32_t u) {
    int32_t a = (int32_t)(e2 & 0xFFFu);
    const uint32_t sp = (e2 >> 12) & 0x7FFu;
    int32_t b = sp == 0x7FFu ? T->n : a + (int32_t)sp;
    while (a < b) {
        const int32_t mid = (a + b) >> 1;
        if (T->thr[mid] <= u) a = mid + 1;
        else b = mid;
    }
    return a;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// The M_L cycles of one pixel: per phase j the sum over cycles of the count
// (CLAMP false: the sample minus its rate's lo) or of the clamped sample
// (CLAMP true), A after M_L cycles, AS after M_S.
template <bool CLAMP>
__device__ __forceinline__ void draw_pixel(const GenArgs &a, const uint32_t *__restrict__ lds, const Table *__restrict__ tt,
                                           int j0, uint32_t p, uint32_t tile_ctr, const int32_t lo[4], uint32_t A[4],
                                           uint32_t AS[4]) {
    const uint32_t *l1 = lds + kL1Words + j0 * kBuckets;
    for (int c = 0; c < a.M_L; ++c) {
        uint32_t r[4];
        philox4x32_10(p, (uint32_t)c, tile_ctr, 0u, a.key0, a.key1, r);
        uint32_t e2[4];
        int32_t x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t u = r[j];
            const uint32_t e1 = l1[j * kBuckets + (u >> kBucketShift)];
            const uint32_t sub = (u << (32 - kBucketShift)) >> (e1 & 31u);
            e2[j] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(lds) +
                                                        (((e1 >> 17) + sub) << 2));
            const int32_t base_m1 = (int32_t)(e1 << 15) >> 20;
            const uint32_t tcmp = (e2[j] & ~kLowMask) | (u & kLowMask);
            x[j] = base_m1 + (int32_t)(e2[j] >> kBucketShift) + (tcmp >= e2[j] ? 1 : 0);
        }
        if (max(max(e2[0], e2[1]), max(e2[2], e2[3])) >= (kSlow << kBucketShift)) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((e2[j] >> kBucketShift) == kSlow) x[j] = count_searched(tt + j0 + j, e2[j], r[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) A[j] += CLAMP ? (uint32_t)min(lo[j] + x[j], (int32_t)a.top) : (uint32_t)x[j];
        if (c + 1 == a.M_S) {
#pragma unroll
            for (int j = 0; j < 4; ++j) AS[j] = A[j];
        }
    }
}

// Work-group: a run of pixels of one tile; the two levels of the tile's eight
// tables are copied to LDS first.
__global__ __launch_bounds__(kBlock) void gen_pairs_kernel(GenArgs a) {
    __shared__ uint32_t lds[kGenLds / 4];
    const int tile = blockIdx.x / a.blocks_per_tile;
    const int part = blockIdx.x % a.blocks_per_tile;
    if (tile >= a.n_tiles) return;
    const Table *tt = a.tables + (int64_t)tile * 8;
    bool clamp = false;
    for (int t = 0; t < 8; ++t) {
        const int32_t l2n = tt[t].l2n;
        for (int i = threadIdx.x; i < l2n; i += kBlock) lds[t * kL2Max + i] = tt[t].l2[i];
        for (int i = threadIdx.x; i < kBuckets; i += kBlock)
            lds[kL1Words + t * kBuckets + i] = tt[t].l1[i] + ((uint32_t)(t * kL2Max) << 17);
        clamp |= (int64_t)tt[t].lo + tt[t].n > (int64_t)a.top;
    }
    __syncthreads();
    const int64_t npx = (int64_t)a.H * a.W;
    const int64_t per = ceil_div(npx, a.blocks_per_tile);
    const int64_t p0 = (int64_t)part * per, p1 = min(npx, p0 + per);
    unsigned long long sS = 0, sL = 0;
    for (int64_t pb = p0; pb < p1; pb += kBlock) {
        const int64_t p = pb + threadIdx.x;
        if (p < p1) {
            const int j0 = a.mask[(int64_t)tile * npx + p] ? 4 : 0;
            int32_t lo[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) lo[j] = tt[j0 + j].lo;
            uint32_t A[4] = {0, 0, 0, 0}, AS[4] = {0, 0, 0, 0};
            if (clamp) draw_pixel<true>(a, lds, tt, j0, (uint32_t)p, a.tile0 + (uint32_t)tile, lo, A, AS);
            else draw_pixel<false>(a, lds, tt, j0, (uint32_t)p, a.tile0 + (uint32_t)tile, lo, A, AS);
            // Without the clamp each sample is lo + count: add M lo per phase.
            const uint32_t mL = clamp ? 0u : (uint32_t)a.M_L, mS = clamp ? 0u : (uint32_t)a.M_S;
            uint32_t L[4], S[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                L[j] = A[j] + mL * (uint32_t)lo[j];
                S[j] = AS[j] + mS * (uint32_t)lo[j];
            }
            const uint32_t s32 = L[0] + L[1] + L[2] + L[3], s32S = S[0] + S[1] + S[2] + S[3];
            sS += s32S;
            sL += s32;
            const int64_t o = (int64_t)tile * npx + p;
            a.I_S[o] = (int32_t)(S[0] - S[2]);
            a.Q_S[o] = (int32_t)(S[1] - S[3]);
            a.I_L[o] = (int32_t)(L[0] - L[2]);
            a.Q_L[o] = (int32_t)(L[1] - L[3]);
            if (a.psum_S) a.psum_S[o] = s32S;
            if (a.psum_L) a.psum_L[o] = s32;
        }
    }
    sS = wave_sum_u64(sS);
    sL = wave_sum_u64(sL);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(a.sum_S + tile, sS);
        atomicAdd(a.sum_L + tile, sL);
    }
}

__global__ void zero_u64_kernel(unsigned long long *p, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace
}  // namespace qld

using namespace qld;

extern "C" qld_status qld_gen_pairs(const uint8_t *mask, const double *rates_host, int32_t n_tiles, int32_t H, int32_t W,
                                    int32_t M_short, int32_t M_long, uint32_t tile0, uint64_t seed, int32_t bits,
                                    int32_t *I_S, int32_t *Q_S, int32_t *I_L, int32_t *Q_L, uint64_t *sum_S,
                                    uint64_t *sum_L, uint32_t *psum_S, uint32_t *psum_L, qld_hip_stream stream) {
    clear_error();
    if (n_tiles < 0 || H < 0 || W < 0 || M_short < 1 || M_long < M_short || bits < 1 || bits > 16) {
        set_error("invalid generator arguments");
        return QLD_E_INVAL;
    }
    if ((int64_t)n_tiles * H * W == 0) return QLD_OK;
    if (!mask || !rates_host || !I_S || !Q_S || !I_L || !Q_L || !sum_S || !sum_L) {
        set_error("all pointers must be non-NULL");
        return QLD_E_INVAL;
    }
    for (int64_t i = 0; i < (int64_t)n_tiles * 8; ++i) {
        const double lam = rates_host[i];
        if (!(lam > 0.0 && lam <= kRateMax)) {
            set_error("rate %g at index %lld outside (0, %g]", lam, (long long)i, kRateMax);
            return QLD_E_INVAL;
        }
    }
    if ((uint64_t)M_long * ((1ull << bits) - 1) >= (1ull << 31) ||
        (uint64_t)M_long * 4 * ((1ull << bits) - 1) >= (1ull << 32)) {
        set_error("M_long=%d too long for %d-bit samples", M_long, bits);
        return QLD_E_OVERFLOW;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int32_t n_rates = n_tiles * 8;
    const size_t tab_b = ((sizeof(Table) * (size_t)n_rates + 255) / 256) * 256;
    const size_t r_b = sizeof(double) * (size_t)n_rates;
    char *ws = static_cast<char *>(stream_workspace(s, tab_b + r_b));
    if (!ws) return QLD_E_NOMEM;
    Table *tables = reinterpret_cast<Table *>(ws);
    double *rates = reinterpret_cast<double *>(ws + tab_b);
    QLD_TRY(check_hip(hipMemcpyAsync(rates, rates_host, r_b, hipMemcpyHostToDevice, s), "rates upload"));
    hipLaunchKernelGGL(build_tables_kernel, dim3((unsigned)n_rates), dim3(kBuildThreads), 0, s, rates, n_rates, tables);
    QLD_TRY(check_hip(hipGetLastError(), "build_tables_kernel launch"));
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)ceil_div(n_tiles, 256)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long *>(sum_S), n_tiles);
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)ceil_div(n_tiles, 256)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long *>(sum_L), n_tiles);
    QLD_TRY(check_hip(hipGetLastError(), "zero kernel launch"));

    GenArgs a{};
    a.mask = mask;
    a.tables = tables;
    a.n_tiles = n_tiles;
    a.H = H;
    a.W = W;
    a.M_S = M_short;
    a.M_L = M_long;
    const int64_t npx = (int64_t)H * W;
    const int64_t want = std::max<int64_t>(1, (4ll * device_cu_count() + n_tiles - 1) / n_tiles);
    a.blocks_per_tile = (int32_t)std::min<int64_t>(want, ceil_div(npx, kBlock));
    a.tile0 = tile0;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.top = (uint32_t)((1u << bits) - 1);
    a.I_S = I_S;
    a.Q_S = Q_S;
    a.I_L = I_L;
    a.Q_L = Q_L;
    a.sum_S = reinterpret_cast<unsigned long long *>(sum_S);
    a.sum_L = reinterpret_cast<unsigned long long *>(sum_L);
    a.psum_S = psum_S;
    a.psum_L = psum_L;
    const int64_t grid = (int64_t)n_tiles * a.blocks_per_tile;
    hipLaunchKernelGGL(gen_pairs_kernel, dim3((unsigned)grid), dim3(kBlock), 0, s, a);
    return check_hip(hipGetLastError(), "gen_pairs_kernel launch");
}
