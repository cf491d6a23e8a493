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
// A 1024-entry guide table (Chen and Asau, 1974) brackets the answer for each
// u >> 22, with two 256-entry sub-guides of 2^16-wide buckets over the first
// and the last 2^24 values of u, where one main bucket would span hundreds of
// thresholds; a binary search inside the bracket finishes it.  Brackets hold
// at most a few thresholds except in the outermost sub-buckets (probability
// 2^-16 each), so the lanes of a wave rarely wait on a long search.
#include <algorithm>
#include <cmath>
#include <cstddef>

#include "qld_internal.hpp"

namespace qld {
namespace {

constexpr int kTableMax = 2048;     // thresholds per rate (lambda up to ~6900)
constexpr int kGuide = 1024;
constexpr int kSub = 256;           // sub-guide entries over [0, 2^24) and [2^32 - 2^24, 2^32)
constexpr uint32_t kHighStart = 0xFF000000u;
constexpr int kBlock = 1024;     // 16 waves; two work-groups per CU where the tables fit twice in LDS
constexpr double kRateMax = 6000.0;  // tables of at most kTableMax thresholds

struct Table {
    int32_t lo, n;                  // n thresholds
    uint16_t guide[kGuide];         // #{thr <= g 2^22}
    uint16_t lguide[kSub];          // #{thr <= i 2^16}
    uint16_t hguide[kSub];          // #{thr <= 2^32 - 2^24 + i 2^16}
    uint32_t thr[kTableMax];
};
// The part of a table before its thresholds; in LDS the eight headers come
// first, then the eight threshold arrays at a stride of the launch's largest n.
constexpr int kHeadBytes = (int)offsetof(Table, thr);
static_assert(kHeadBytes % 4 == 0, "header copied in words");

// Thresholds of a rate's table: the table size of build_tables_kernel.
int32_t table_size(double lam) {
    const int32_t m = (int32_t)std::floor(lam);
    const int32_t w = (int32_t)std::ceil(12.0 * std::sqrt(lam)) + 10;
    const int32_t lo = m - w < 0 ? 0 : m - w;
    return m + w - lo;
}

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

// One work-group builds one table: lane 0 runs the sequential parts exactly
// in the order the definition fixes (the ratio recurrence and the two
// ascending sums, in LDS), then all lanes form the thresholds and the guide.
__global__ __launch_bounds__(64) void build_tables_kernel(const double *__restrict__ rates, int32_t n_rates,
                                                          Table *__restrict__ tables) {
    __shared__ double wk[kTableMax + 1];
    __shared__ double tot;
    const int t = blockIdx.x;
    if (t >= n_rates) return;
    const double lam = rates[t];
    Table &T = tables[t];
    const int32_t m = (int32_t)floor(lam);
    const int32_t w = (int32_t)ceil(__dmul_rn(12.0, __dsqrt_rn(lam))) + 10;
    const int32_t lo = m - w < 0 ? 0 : m - w;
    const int32_t hi = m + w;
    const int32_t n = hi - lo;                       // thresholds k = lo .. hi-1
    if (threadIdx.x == 0) {
        wk[m - lo] = 1.0;
        for (int32_t k = m + 1; k <= hi; ++k) wk[k - lo] = __ddiv_rn(__dmul_rn(wk[k - 1 - lo], lam), (double)k);
        for (int32_t k = m - 1; k >= lo; --k) wk[k - lo] = __ddiv_rn(__dmul_rn(wk[k + 1 - lo], (double)(k + 1)), lam);
        double total = 0.0;
        for (int32_t i = 0; i <= n; ++i) total = __dadd_rn(total, wk[i]);
        double cum = 0.0;
        for (int32_t i = 0; i < n; ++i) {
            cum = __dadd_rn(cum, wk[i]);
            wk[i] = cum;                              // wk now holds the partial sums
        }
        tot = total;
        T.lo = lo;
        T.n = n;
    }
    __syncthreads();
    const double total = tot;
    for (int32_t i = threadIdx.x; i < n; i += 64) {
        const double f = floor(__dmul_rn(__ddiv_rn(wk[i], total), 4294967296.0));
        T.thr[i] = f >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)f;
    }
    __syncthreads();
    // Guide entries: #{thr <= v} by binary search, one entry per lane.
    auto count_le = [&](uint32_t v) {
        int32_t a = 0, b = n;
        while (a < b) {
            const int32_t mid = (a + b) >> 1;
            if (T.thr[mid] <= v) a = mid + 1;
            else b = mid;
        }
        return (uint16_t)a;
    };
    for (int g = threadIdx.x; g < kGuide; g += 64) T.guide[g] = count_le((uint32_t)g << 22);
    for (int i = threadIdx.x; i < kSub; i += 64) {
        T.lguide[i] = count_le((uint32_t)i << 16);
        T.hguide[i] = count_le(kHighStart + ((uint32_t)i << 16));
    }
}

struct GenArgs {
    const uint8_t *mask;      // [n][H][W]
    const Table *tables;      // [n][8]: (mask state, phase)
    int32_t n_tiles, H, W, M_S, M_L;
    int32_t blocks_per_tile;
    int32_t thr_stride;       // LDS words per threshold array (>= every table's n)
    uint32_t tile0, key0, key1;
    uint32_t top;
    int32_t *I_S, *Q_S, *I_L, *Q_L;
    unsigned long long *sum_S, *sum_L;
    uint32_t *psum_S, *psum_L;        // per-pixel sample sums (may be NULL)
};

// X(u) = lo + #{k : thr[k] <= u}.  The count lies between the guide entries of
// u's bucket and of the next bucket (thresholds are non-decreasing); a binary
// search between them finishes it.
__device__ __forceinline__ int32_t invert(const Table *__restrict__ T, const uint32_t *__restrict__ thr, uint32_t u) {
    int32_t a, b;
    if (u < (1u << 24)) {
        const uint32_t i = u >> 16;
        a = T->lguide[i];
        b = i + 1 < (uint32_t)kSub ? (int32_t)T->lguide[i + 1] : (int32_t)T->guide[4];
    } else if (u >= kHighStart) {
        const uint32_t i = (u - kHighStart) >> 16;
        a = T->hguide[i];
        b = i + 1 < (uint32_t)kSub ? (int32_t)T->hguide[i + 1] : T->n;
    } else {
        const uint32_t g = u >> 22;
        a = T->guide[g];
        b = T->guide[g + 1];                        // g + 1 <= 1020 < kGuide here
    }
    while (a < b) {
        const int32_t mid = (a + b) >> 1;
        if (thr[mid] <= u) a = mid + 1;
        else b = mid;
    }
    return T->lo + a;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Work-group: a run of pixels of one tile; the tile's eight tables are
// copied to LDS first.
__global__ __launch_bounds__(kBlock) void gen_pairs_kernel(GenArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tile = blockIdx.x / a.blocks_per_tile;
    const int part = blockIdx.x % a.blocks_per_tile;
    if (tile >= a.n_tiles) return;
    // LDS: eight table headers (lo, n, guides), then eight threshold arrays.
    uint32_t *lthr = reinterpret_cast<uint32_t *>(smem + 8 * kHeadBytes);
    {
        const Table *src = a.tables + (int64_t)tile * 8;
        constexpr int hw = kHeadBytes / 4;
        for (int i = threadIdx.x; i < 8 * hw; i += kBlock)
            reinterpret_cast<uint32_t *>(smem)[i] = reinterpret_cast<const uint32_t *>(src + i / hw)[i % hw];
        for (int i = threadIdx.x; i < 8 * a.thr_stride; i += kBlock) {
            const int j = i / a.thr_stride, k = i % a.thr_stride;
            lthr[i] = k < src[j].n ? src[j].thr[k] : 0xFFFFFFFFu;
        }
    }
    __syncthreads();
    // Table j's header (only lo, n and the guides are read through it).
    auto head = [&](int j) { return reinterpret_cast<const Table *>(smem + j * kHeadBytes); };
    const int64_t npx = (int64_t)a.H * a.W;
    const int64_t per = ceil_div(npx, a.blocks_per_tile);
    const int64_t p0 = (int64_t)part * per, p1 = min(npx, p0 + per);
    unsigned long long sS = 0, sL = 0;
    for (int64_t pb = p0; pb < p1; pb += kBlock) {
        const int64_t p = pb + threadIdx.x;
        const bool valid = p < p1;
        const int mk = valid ? (a.mask[(int64_t)tile * npx + p] ? 1 : 0) : 0;
        const int j0 = mk * 4;
        int32_t I = 0, Q = 0, Is = 0, Qs = 0;
        uint32_t s32 = 0, s32S = 0;
        if (valid) {
            for (int c = 0; c < a.M_L; ++c) {
                uint32_t r[4];
                philox4x32_10((uint32_t)p, (uint32_t)c, a.tile0 + (uint32_t)tile, 0u, a.key0, a.key1, r);
                int32_t x[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    x[j] = min(invert(head(j0 + j), lthr + (j0 + j) * a.thr_stride, r[j]), (int32_t)a.top);
                I += x[0] - x[2];
                Q += x[1] - x[3];
                s32 += (uint32_t)(x[0] + x[1] + x[2] + x[3]);
                if (c + 1 == a.M_S) {
                    Is = I;
                    Qs = Q;
                    s32S = s32;
                    sS += s32;
                }
            }
            sL += s32;
            const int64_t o = (int64_t)tile * npx + p;
            a.I_S[o] = Is;
            a.Q_S[o] = Qs;
            a.I_L[o] = I;
            a.Q_L[o] = Q;
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
    hipLaunchKernelGGL(build_tables_kernel, dim3((unsigned)n_rates), dim3(64), 0, s, rates, n_rates, tables);
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
    int32_t max_n = 1;
    for (int64_t i = 0; i < (int64_t)n_tiles * 8; ++i) max_n = std::max(max_n, table_size(rates_host[i]));
    a.thr_stride = std::min(kTableMax, max_n + 4);   // + 4: margin over the host's recomputation of n
    const size_t lds = (size_t)8 * kHeadBytes + (size_t)8 * a.thr_stride * 4;
    const int64_t grid = (int64_t)n_tiles * a.blocks_per_tile;
    hipLaunchKernelGGL(gen_pairs_kernel, dim3((unsigned)grid), dim3(kBlock), lds, s, a);
    return check_hip(hipGetLastError(), "gen_pairs_kernel launch");
}
