/*
 * CPU oracle for the method-generated training pairs of the learned
 * short-window path.
 *
 * TEST INFRASTRUCTURE ONLY (see qld_oracle.c).  Shares no code with the HIP
 * library: the counter-based generator and the Poisson sampler are written
 * here from their published definitions, independently of the GPU side.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64-bit
 * multiplications with a Weyl-sequence key schedule.
 *
 * Poisson variates by inversion (Devroye, "Non-Uniform Random Variate
 * Generation", 1986, ch. III.2 and X.3): X = the smallest k whose cumulative
 * probability exceeds a uniform u.  The cumulative table is a 32-bit fixed-point
 * version of the Poisson CDF on [lo, hi], built from the probability ratios
 * p(k+1)/p(k) = lambda/(k+1) in double precision with a fixed order of
 * correctly rounded operations (so any IEEE-754 implementation that follows
 * the same steps builds the same table):
 *   m = floor(lambda); W = ceil(12 sqrt(lambda)) + 10; lo = max(0, m - W); hi = m + W
 *   w[m] = 1; w[k] = (w[k-1] * lambda) / k        for k = m+1..hi
 *             w[k] = (w[k+1] * (k+1)) / lambda    for k = m-1..lo
 *   total = w[lo] + w[lo+1] + ... + w[hi]             (ascending order)
 *   cum_k = w[lo] + ... + w[k]                       (ascending order)
 *   thr[k] = min(floor((cum_k / total) * 2^32), 2^32 - 1),   k = lo..hi-1
 *   X(u) = lo + #{k in [lo, hi-1] : thr[k] <= u}
 * The mass outside [lo, hi] is below 1e-20 for lambda >= 1, far below the 2^-32
 * resolution of the table.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint32_t mulhilo32(uint32_t a, uint32_t b, uint32_t *hi) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    return (uint32_t)p;
}

/* Philox4x32 with R rounds: out = f(ctr, key). */
void oracle_philox4x32(const uint32_t ctr_in[4], const uint32_t key_in[2], int rounds, uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   /* key increments (golden ratio, sqrt 3 - 1) */
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < rounds; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint32_t hi0, hi1;
        uint32_t lo0 = mulhilo32(M0, c0, &hi0);
        uint32_t lo1 = mulhilo32(M1, c2, &hi1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Table bounds for rate lambda; returns hi - lo + 1. */
int oracle_poisson_bounds(double lambda, int32_t *lo, int32_t *hi) {
    int32_t m = (int32_t)floor(lambda);
    int32_t w = (int32_t)ceil(12.0 * sqrt(lambda)) + 10;
    *lo = m - w < 0 ? 0 : m - w;
    *hi = m + w;
    return *hi - *lo + 1;
}

/* thr[0 .. hi-lo-1] as defined above.  Returns the table length hi-lo. */
int oracle_poisson_table(double lambda, uint32_t *thr, int32_t *lo_out, int32_t *hi_out) {
    int32_t lo, hi;
    int n = oracle_poisson_bounds(lambda, &lo, &hi);
    int32_t m = (int32_t)floor(lambda);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!w) return -1;
    w[m - lo] = 1.0;
    for (int32_t k = m + 1; k <= hi; ++k) w[k - lo] = (w[k - 1 - lo] * lambda) / (double)k;
    for (int32_t k = m - 1; k >= lo; --k) w[k - lo] = (w[k + 1 - lo] * (double)(k + 1)) / lambda;
    double total = 0.0;
    for (int i = 0; i < n; ++i) total += w[i];
    double cum = 0.0;
    for (int i = 0; i < n - 1; ++i) {
        cum += w[i];
        double f = floor(ldexp(cum / total, 32));
        thr[i] = f >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)f;
    }
    free(w);
    *lo_out = lo;
    *hi_out = hi;
    return n - 1;
}

/* X(u) by the definition: count of thresholds <= u. */
int32_t oracle_poisson_invert(const uint32_t *thr, int n_thr, int32_t lo, uint32_t u) {
    int32_t c = 0;
    for (int i = 0; i < n_thr; ++i) c += thr[i] <= u;
    return lo + c;
}

/*
 * Frames of training tiles.  Tile i (global index tile0 + i) has a mask
 * [H][W] (0/1) and per-phase rates rates[i][mask][phase] (double).  Sample
 * (t, y, x) of tile i: cycle c = t / 4, phase j = t % 4, uniform
 * u = word j of Philox4x32-10(ctr = (y*W + x, c, tile0 + i, 0), key = (seed_lo, seed_hi)),
 * value = min(X_{lambda}(u), 2^bits - 1) with lambda = rates[i][mask][j].
 * Writes frames[i][t][y][x] (uint16) for t < 4*n_cycles.
 */
int oracle_gen_frames(const uint8_t *mask, const double *rates, int n_tiles, int H, int W, int n_cycles,
                      uint32_t tile0, uint32_t seed_lo, uint32_t seed_hi, int bits, uint16_t *frames) {
    const int32_t top = (1 << bits) - 1;
    for (int i = 0; i < n_tiles; ++i) {
        uint32_t *thr[8];
        int nthr[8];
        int32_t lo[8], hi[8];
        for (int s = 0; s < 8; ++s) {
            double lam = rates[(size_t)i * 8 + s];
            int32_t l, h;
            oracle_poisson_bounds(lam, &l, &h);
            thr[s] = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(h - l + 1));
            if (!thr[s]) return 1;
            nthr[s] = oracle_poisson_table(lam, thr[s], &lo[s], &hi[s]);
        }
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int mk = mask[((size_t)i * H + y) * W + x] ? 1 : 0;
                for (int c = 0; c < n_cycles; ++c) {
                    uint32_t ctr[4] = {(uint32_t)(y * W + x), (uint32_t)c, tile0 + (uint32_t)i, 0u};
                    uint32_t key[2] = {seed_lo, seed_hi};
                    uint32_t r[4];
                    oracle_philox4x32(ctr, key, 10, r);
                    for (int j = 0; j < 4; ++j) {
                        int s = mk * 4 + j;
                        int32_t v = oracle_poisson_invert(thr[s], nthr[s], lo[s], r[j]);
                        if (v > top) v = top;
                        frames[(((size_t)i * 4 * n_cycles + (size_t)(4 * c + j)) * H + y) * W + x] = (uint16_t)v;
                    }
                }
            }
        for (int s = 0; s < 8; ++s) free(thr[s]);
    }
    return 0;
}

/*
 * Series of selected pixels of one tile (same definition as above): for each
 * k, pixel index pix[k] = y*W + x of a tile of width W, mask state mk[k];
 * writes series[k][t] for t < 4*n_cycles.
 */
int oracle_gen_pixels(const int64_t *pix, const uint8_t *mk, int n_px, const double *rates, int n_cycles,
                      uint32_t tile, uint32_t seed_lo, uint32_t seed_hi, int bits, uint16_t *series) {
    const int32_t top = (1 << bits) - 1;
    uint32_t *thr[8];
    int nthr[8];
    int32_t lo[8], hi[8];
    for (int s = 0; s < 8; ++s) {
        int32_t l, h;
        oracle_poisson_bounds(rates[s], &l, &h);
        thr[s] = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(h - l + 1));
        if (!thr[s]) return 1;
        nthr[s] = oracle_poisson_table(rates[s], thr[s], &lo[s], &hi[s]);
    }
    for (int k = 0; k < n_px; ++k) {
        for (int c = 0; c < n_cycles; ++c) {
            uint32_t ctr[4] = {(uint32_t)pix[k], (uint32_t)c, tile, 0u};
            uint32_t key[2] = {seed_lo, seed_hi};
            uint32_t r[4];
            oracle_philox4x32(ctr, key, 10, r);
            for (int j = 0; j < 4; ++j) {
                int s = (mk[k] ? 1 : 0) * 4 + j;
                int32_t v = oracle_poisson_invert(thr[s], nthr[s], lo[s], r[j]);
                if (v > top) v = top;
                series[(size_t)k * 4 * n_cycles + (size_t)(4 * c + j)] = (uint16_t)v;
            }
        }
    }
    for (int s = 0; s < 8; ++s) free(thr[s]);
    return 0;
}
