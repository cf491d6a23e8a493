/*
 * CPU oracle for quadrature lock-in discrimination (QLD).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call this file:
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header, table or constant with the HIP library.
 *
 * Plain, slow and obviously correct: each function writes out the definition
 * it follows, in 64-bit integers or double precision, frame by frame, with no
 * blocking or fusion.  OpenMP only splits independent pixel rows.
 *
 * Conventions (the paper's readings are listed in the design notes):
 *   frames   [T][H][W] samples, element (t, y, x) at
 *            base + t*frame_stride + y*row_pitch + x      (strides in elements)
 *   elem     1 = uint8, 2 = uint16
 *   phase    frame t is sampled at lock-in phase (phase0 + t) mod 4, i.e. at
 *            omega * t_s = 2*pi*(phase0 + t)/4 (four samples per period)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double ORACLE_PI = 3.14159265358979323846264338327950288;

static inline int64_t sample_at(const void *frames, int elem, int64_t off)
{
    if (elem == 1) return (int64_t)((const uint8_t *)frames)[off];
    return (int64_t)((const uint16_t *)frames)[off];
}

static inline int mod4(int64_t v) { return (int)(((v % 4) + 4) % 4); }

/*
 * Reference arrays of the lock-in (Methods, formula for R(j,k); Supplementary,
 * "Timing sequence": sin and cos tables prepared for the chosen lock-in and
 * sampling frequencies).  With four samples per period the arrays hold
 * cos(2*pi*j/4) and sin(2*pi*j/4), j = 0..3, whose exact values are integers.
 * They are evaluated here from the definition and rounded to those integers;
 * the rounding moves each value by less than 1e-15.  Returns 0 on success.
 */
int oracle_reference_tables(int64_t cos_tab[4], int64_t sin_tab[4])
{
    for (int j = 0; j < 4; ++j) {
        double th = 2.0 * ORACLE_PI * (double)j / 4.0;
        double c = cos(th), s = sin(th);
        cos_tab[j] = (int64_t)llround(c);
        sin_tab[j] = (int64_t)llround(s);
        if (fabs(c - (double)cos_tab[j]) > 1e-12 || fabs(s - (double)sin_tab[j]) > 1e-12)
            return 1;
    }
    return 0;
}

/*
 * Quadrature sums of every pixel (Methods, R(j,k); Supplementary, "Timing
 * sequence": each frame is multiplied by sin and by cos and the products are
 * accumulated into two 2-D arrays):
 *     I(y,x) = sum_t S_t(y,x) * cos(2*pi*(phase0+t)/4)
 *     Q(y,x) = sum_t S_t(y,x) * sin(2*pi*(phase0+t)/4)
 * I and Q are overwritten ([H][W], int64).
 */
int oracle_qld(const void *frames, int elem, int H, int W, int64_t row_pitch,
               int64_t frame_stride, int T, int phase0, int64_t *I, int64_t *Q,
               int n_threads)
{
    int64_t ct[4], st[4];
    if (oracle_reference_tables(ct, st)) return 1;
    if (elem != 1 && elem != 2) return 2;
    memset(I, 0, sizeof(int64_t) * (size_t)H * (size_t)W);
    memset(Q, 0, sizeof(int64_t) * (size_t)H * (size_t)W);
    if (n_threads < 1) n_threads = 1;
    for (int t = 0; t < T; ++t) {
        const int64_t c = ct[mod4((int64_t)phase0 + t)];
        const int64_t s = st[mod4((int64_t)phase0 + t)];
#pragma omp parallel for num_threads(n_threads) schedule(static)
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                int64_t v = sample_at(frames, elem, (int64_t)t * frame_stride + (int64_t)y * row_pitch + x);
                I[(int64_t)y * W + x] += v * c;
                Q[(int64_t)y * W + x] += v * s;
            }
        }
    }
    return 0;
}

/*
 * Per-frame statistics: sum of all samples of frame t and the number of
 * samples equal to the largest code 2^bits - 1 (clipped pixels).
 * Overwrites frame_sum[T] and frame_sat[T].
 */
int oracle_frame_stats(const void *frames, int elem, int H, int W, int64_t row_pitch,
                       int64_t frame_stride, int T, int bits, uint64_t *frame_sum,
                       uint32_t *frame_sat)
{
    if (elem != 1 && elem != 2) return 2;
    const int64_t top = ((int64_t)1 << bits) - 1;
    for (int t = 0; t < T; ++t) {
        uint64_t s = 0;
        uint32_t n = 0;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t v = sample_at(frames, elem, (int64_t)t * frame_stride + (int64_t)y * row_pitch + x);
                s += (uint64_t)v;
                n += (v == top);
            }
        frame_sum[t] = s;
        frame_sat[t] = n;
    }
    return 0;
}

/*
 * Lock-in amplitude R = (I^2 + Q^2)^(1/2) (Methods, R(j,k)), in double.
 * I^2 + Q^2 is formed exactly in 64-bit integers (|I|, |Q| < 2^31) and the
 * square root is taken in long double, whose 64-bit significand holds that
 * sum exactly, then rounded once more to double.
 */
void oracle_amplitude(const int64_t *I, const int64_t *Q, int64_t n, double *amp)
{
    for (int64_t p = 0; p < n; ++p) {
        uint64_t ss = (uint64_t)(I[p] * I[p]) + (uint64_t)(Q[p] * Q[p]);
        amp[p] = (double)sqrtl((long double)ss);
    }
}

/*
 * Single-bin discrete Fourier transform of every pixel's series (Methods:
 * Fourier discrimination evaluates F(j,k,omega_q) of I(j,k,t_p) and maps
 * |F|^2 at the frequency of interest):
 *     X_k(y,x) = sum_{n<N} S_n(y,x) * exp(-2*pi*i*((k*n) mod N)/N)
 * The angle is reduced in exact integers before the double-precision cos/sin.
 * re, im overwritten ([H][W]).  N = T.
 */
int oracle_dft_bin(const void *frames, int elem, int H, int W, int64_t row_pitch,
                   int64_t frame_stride, int T, int k, double *re, double *im, int n_threads)
{
    if (elem != 1 && elem != 2) return 2;
    if (T <= 0) return 3;
    memset(re, 0, sizeof(double) * (size_t)H * (size_t)W);
    memset(im, 0, sizeof(double) * (size_t)H * (size_t)W);
    if (n_threads < 1) n_threads = 1;
    for (int n = 0; n < T; ++n) {
        int64_t r = (((int64_t)k * n) % T + T) % T;
        double th = 2.0 * ORACLE_PI * (double)r / (double)T;
        double c = cos(th), s = sin(th);
#pragma omp parallel for num_threads(n_threads) schedule(static)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double v = (double)sample_at(frames, elem, (int64_t)n * frame_stride + (int64_t)y * row_pitch + x);
                re[(int64_t)y * W + x] += v * c;
                im[(int64_t)y * W + x] -= v * s;
            }
    }
    return 0;
}

/*
 * Lock-in at a general ratio f_mod / f_s = p / q (Methods, R(j,k) with the
 * reference tables of that frequency): X = sum_n S_n (cos th_n - i sin th_n),
 * th_n = 2 pi ((p (t0 + n)) mod q) / q, the angle reduced in exact integers
 * first.  In double.
 */
int oracle_lockin_ratio(const void *frames, int elem, int H, int W, int64_t row_pitch, int64_t frame_stride,
                        int T, int p, int q, int t0, double *re, double *im, int n_threads)
{
    if (elem != 1 && elem != 2) return 2;
    if (T <= 0 || q <= 0 || t0 < 0) return 3;
    memset(re, 0, sizeof(double) * (size_t)H * (size_t)W);
    memset(im, 0, sizeof(double) * (size_t)H * (size_t)W);
    if (n_threads < 1) n_threads = 1;
    for (int n = 0; n < T; ++n) {
        int64_t r = (((int64_t)p * ((int64_t)t0 + n)) % q + q) % q;
        double th = 2.0 * ORACLE_PI * (double)r / (double)q;
        double c = cos(th), s = sin(th);
#pragma omp parallel for num_threads(n_threads) schedule(static)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double v = (double)sample_at(frames, elem, (int64_t)n * frame_stride + (int64_t)y * row_pitch + x);
                re[(int64_t)y * W + x] += v * c;
                im[(int64_t)y * W + x] -= v * s;
            }
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
