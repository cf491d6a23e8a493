/*
 * libqld: quadrature lock-in discrimination (QLD) imaging on AMD Instinct MI355X
 * (gfx950).  C ABI.
 *
 * The operation (paper: Methods, the formula for R(j,k); Supplementary
 * Information, "Timing sequence for hybrid parallelisation"): every pixel's
 * intensity series S_t, sampled four times per modulation period, is
 * multiplied by the cosine and the sine of the lock-in phase and summed,
 *     I = sum_t S_t cos(2 pi (phase0 + t)/4) = sum over cycles (S0 - S2)
 *     Q = sum_t S_t sin(2 pi (phase0 + t)/4) = sum over cycles (S1 - S3)
 * and the image is the amplitude R = (I^2 + Q^2)^(1/2).  Accumulation starts
 * with the first frame and proceeds frame by frame (section "Quadrature
 * Lock-in Discrimination", on-the-fly processing); a sliding window of N
 * frames refreshes the image at the camera rate (Supplementary, sliding
 * sequence and buffer requirement).  The conventional alternative, a Fourier
 * transform of the series evaluated at the lock-in frequency (Methods,
 * Fourier map), is provided as the single-bin baseline dft_bin_baseline.
 *
 * General conventions
 *   - Pointers are DEVICE pointers (hipMalloc or torch CUDA tensors on the
 *     current device) unless the comment says "host".
 *   - Frame stacks are [T][H][W] with element (t, y, x) at
 *         base + t*frame_stride + y*row_pitch + x       (strides in ELEMENTS).
 *     Frame t is sampled at lock-in phase (phase0 + t) mod 4.
 *   - The caller owns every buffer it passes; libqld owns the handles it
 *     creates (qld_window, qld_server) and the device memory behind them.
 *   - Batch calls that need scratch memory (frame statistics partials, the
 *     I/Q partials of a frame-split grid, twiddle and reference tables) take
 *     it from a device workspace that libqld keeps per (device, stream) and
 *     grows on demand (hipMalloc; a grow first synchronises that stream).
 *     Calls on one stream therefore run in order over one workspace; calls on
 *     different streams never share it.  It lives until the process ends.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the legacy default
 *     stream) and is asynchronous: outputs are valid once the stream reaches
 *     the call.  Argument errors are detected synchronously, before anything
 *     is enqueued, and leave every output untouched.
 *   - A launch or runtime failure returns QLD_E_DEVICE; a fault inside a
 *     kernel surfaces as QLD_E_DEVICE from a later call.  qld_last_error()
 *     gives a thread-local message for the most recent failure.
 *   - No C++ exception crosses this interface.
 */
#ifndef QLD_H
#define QLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same type as hipStream_t, declared here so the header needs no HIP include. */
typedef struct ihipStream_t *qld_hip_stream;

typedef enum {
    QLD_OK = 0,
    QLD_E_INVAL = 1,     /* null pointer, negative count, bad enum */
    QLD_E_DTYPE = 2,     /* dtype/bits combination not supported */
    QLD_E_SHAPE = 3,     /* H, W, pitches or frame count inconsistent */
    QLD_E_ALIGN = 4,     /* alignment required by this entry point not met */
    QLD_E_OVERFLOW = 5,  /* int32 accumulators could overflow for this input */
    QLD_E_NOMEM = 6,     /* device or pinned host allocation failed */
    QLD_E_BUDGET = 7,    /* request can never fit in the server's HBM budget */
    QLD_E_AGAIN = 8,     /* not now: queued for admission, or no slot free yet */
    QLD_E_STATE = 9,     /* call not valid in the handle's current state */
    QLD_E_GAP = 10,      /* frame index skipped: the window was reset */
    QLD_E_DEVICE = 11,   /* HIP runtime or kernel failure */
    QLD_E_IO = 12        /* checkpoint file could not be read or written */
} qld_status;

typedef enum { QLD_U8 = 1, QLD_U16 = 2 } qld_dtype;

/* Geometry and sample format of one frame (and of a stack of frames). */
typedef struct {
    int32_t H, W;            /* rows, columns (>= 0) */
    int64_t row_pitch;       /* elements between rows, >= W */
    int64_t frame_stride;    /* elements between frames, >= (H-1)*row_pitch + W */
    qld_dtype dtype;         /* QLD_U8 or QLD_U16 */
    int32_t bits;            /* significant bits per sample: 1..8 (U8) or 1..16 (U16) */
} qld_frame_desc;

/* ------------------------------------------------------------------------ */
/* Batch lock-in                                                            */
/* ------------------------------------------------------------------------ */

/*
 * qld_frame_stride_hint -- host-side helper: the frame stride (in ELEMENTS)
 * to allocate a [T][H][row_pitch] stack with, for frames of H rows of
 * row_pitch elements of `dtype`.  It is the frame size rounded up to 256
 * bytes, plus a gap when that size is a multiple of 64 KiB: with such sizes
 * (1024 x 1024 uint16 frames are 2 MiB) the same pixel of consecutive frames
 * falls on the same HBM bank, and the batch kernels, which read four
 * consecutive frames of a pixel at once, measured 2-7% slower on MI355X.
 * The gap is 4 KiB for frames of 2 MiB and more, 256 bytes for smaller ones
 * (the faster of the two measured at each size).
 * Any stride >= the frame size works with every call; this one is faster.
 * Returns 0 for invalid arguments (H or W < 0, row_pitch < W, unknown dtype)
 * and for empty frames (H = 0 or row_pitch = 0), which need no stride.
 * Touches no device.
 */
int64_t qld_frame_stride_hint(int32_t H, int32_t W, int64_t row_pitch, qld_dtype dtype);

/*
 * qld_accumulate -- quadrature sums of a frame stack (Methods, R(j,k);
 * Supplementary, each frame multiplied by sin and cos and accumulated into
 * two 2-D arrays).
 *
 *   frames     device, [n_frames][H][W] in the layout of `d`
 *   n_frames   >= 0; frame t has phase (phase0 + t) mod 4, phase0 any int
 *   I, Q       device int32 [H][W] (dense, row pitch W).  ACCUMULATED: the
 *              call adds this stack's sums to the values already there, so a
 *              stack can be fed in chunks (pass phase0 + frames done so far)
 *   frame_sum  device uint64 [n_frames] or NULL: frame_sum[t] += sum of frame t
 *   frame_sat  device uint32 [n_frames] or NULL: frame_sat[t] += number of
 *              samples equal to 2^bits - 1 (clipped pixels break the exact
 *              cancellation of the unmodulated light)
 * Precondition: every sample is <= 2^bits - 1 (d->bits states the range of
 * the data, not only of the dtype).  The overflow check below and the 16-bit
 * partial sums of the fast path rely on it; a larger sample gives undefined
 * I/Q (and is not counted in frame_sat).  Data of unknown range must be
 * described with bits = 8 (U8) or 16 (U16).
 * Errors: QLD_E_OVERFLOW if ceil(n_frames/4) * (2^bits - 1) >= 2^31 (the
 * caller must split longer stacks into separate accumulators).  Inputs need
 * no particular alignment; 16-byte aligned base and pitches take the fast
 * path.  Integer arithmetic throughout: the result is exact.
 */
qld_status qld_accumulate(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                          int32_t phase0, int32_t *I, int32_t *Q, uint64_t *frame_sum,
                          uint32_t *frame_sat, qld_hip_stream stream);

/*
 * qld_amplitude -- R = (I^2 + Q^2)^(1/2) (Methods, R(j,k)).
 *   I, Q       device int32 [n_pixels];  amp  device float [n_pixels] (overwritten)
 * I^2 + Q^2 is formed exactly in 64-bit integers, its square root taken in
 * double precision and rounded once to float.
 */
qld_status qld_amplitude(const int32_t *I, const int32_t *Q, int64_t n_pixels, float *amp,
                         qld_hip_stream stream);

/*
 * qld_lockin_image -- one image from a stack in a single pass over it:
 * I, Q = the stack's quadrature sums (overwritten, not added), amp =
 * (I^2 + Q^2)^(1/2) as qld_amplitude computes it (may be NULL), frame_sum /
 * frame_sat the per-frame statistics (each may be NULL; overwritten).  The
 * same as clearing the outputs, qld_accumulate and qld_amplitude, without
 * the separate clears and the second pass over I/Q.  Arguments and errors as
 * qld_accumulate, plus QLD_E_SHAPE for n_frames < 1.
 */
qld_status qld_lockin_image(const void *frames, const qld_frame_desc *d, int32_t n_frames, int32_t phase0,
                            int32_t *I, int32_t *Q, float *amp, uint64_t *frame_sum, uint32_t *frame_sat,
                            qld_hip_stream stream);

/*
 * qld_lockin_image_noalloc -- qld_lockin_image for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * qld_lockin_image (the same kernels run), but the scratch the kernels need
 * (per-work-group frame-statistics partials when frame_sum or frame_sat is
 * given; per-split I/Q partials when a small image's frames are split over
 * several work-groups) lives in a fixed device array of
 * QLD_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends.  The call makes no hipMalloc/hipFree and no
 * allocating library call.  The array's device address is looked up once
 * per device, on the first call with that device current.
 * Errors: as qld_lockin_image, plus QLD_E_NOMEM (nothing launched) when the
 * call would need more scratch than the array holds: about
 * 8 * n_frames * (H*W / 2048 for aligned 16-bit stacks, / 4096 for 8-bit,
 * / 64 for unaligned ones) bytes with statistics, plus 8 bytes per pixel per
 * frame split of images too small to fill the GPU.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (two host threads, or two streams whose work is not
 * ordered) race on it and give undefined results.  Calls ordered on one
 * stream are safe; the array keeps the last call's partials, and every call
 * writes all of the scratch it reads, so nothing needs clearing.
 */
#define QLD_NOALLOC_SCRATCH_BYTES (32u << 20)
qld_status qld_lockin_image_noalloc(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                                    int32_t phase0, int32_t *I, int32_t *Q, float *amp, uint64_t *frame_sum,
                                    uint32_t *frame_sat, qld_hip_stream stream);

/*
 * dft_bin_baseline -- the Fourier alternative at one frequency (Methods,
 * Fourier map |F(omega)|^2 of each pixel's series):
 *     X_k = sum_{n < N} S_n exp(-2 pi i ((k n) mod N) / N),   N = n_frames
 *   re, im     device float [H][W] (dense, overwritten)
 * Twiddles are a float table built in double from the exact integer angle
 * (k n) mod N; accumulation is float.  At k = N/4 with N = 4M, X = I - iQ up
 * to rounding.  Reports QLD_E_SHAPE for n_frames < 1.
 */
qld_status dft_bin_baseline(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                            int32_t k_bin, float *re, float *im, qld_hip_stream stream);

/*
 * dft_bin_baseline_f64 -- the same single-bin DFT in double precision, the
 * precision the paper computes in (Supplementary Information, "Details of
 * apparatus": every computation in double precision): twiddles
 * from the exact integer angle rounded to double, multiply-adds in double.
 *   re, im     device double [H][W] (dense, overwritten)
 * Error <= (N + 2) * 2^-53 * sum_n |S_n| per component.  The sample read is
 * the same as the float path's, so on MI355X it streams at the same rate.
 * Arguments and errors as dft_bin_baseline.
 */
qld_status dft_bin_baseline_f64(const void *frames, const qld_frame_desc *d, int32_t n_frames,
                                int32_t k_bin, double *re, double *im, qld_hip_stream stream);

/*
 * qld_lockin_ratio -- lock-in at a general frequency ratio f_mod / f_s = p / q
 * (Methods, R(j,k) with reference tables of any frequency, precomputed once):
 *     X = sum_{t < n} S_t exp(-2 pi i ((p (t0 + t)) mod q) / q) = I - iQ,
 * I and Q the sums of the series times the cos and sin tables of the lock-in
 * phase 2 pi p (t0 + t) / q; the image is R = |X|.  t0 >= 0 is the time index
 * of frame 0.  With p / q = 1/4 and t0 = phase0 this is the four-sample QLD in
 * float; with q = n_frames it is dft_bin_baseline at bin p.  A source at
 * another frequency cancels over whole beat periods (the wrong-frequency
 * rejection of the method).  Same tables, precision and layout as
 * dft_bin_baseline.  QLD_E_INVAL for q < 1 or t0 < 0, QLD_E_SHAPE for
 * n_frames < 1.
 *   re, im  device float [H][W] (dense, overwritten)
 */
qld_status qld_lockin_ratio(const void *frames, const qld_frame_desc *d, int32_t n_frames, int32_t p,
                            int32_t q, int32_t t0, float *re, float *im, qld_hip_stream stream);

/*
 * qld_lockin_bank -- a bank of n_freq lock-ins at once (the paper's
 * multi-frequency images, Fig. 1, sources at several modulation frequencies;
 * Methods, Fourier map as a series of lock-ins): for f < n_freq
 *     X_f = sum_{t < n} S_t exp(-2 pi i ((p_f (t0 + t)) mod q) / q) = I_f - i Q_f,
 * each equal to qld_lockin_ratio(p_f, q, t0), computed as one contraction on
 * the matrix cores, frequencies in groups of 32.  Arithmetic by path:
 *   - uint16 stacks with a 16-byte aligned base and W, row pitch and frame
 *     stride multiples of 8, groups of more than 8 frequencies: bf16 MFMA with
 *     exact operand splitting (sample = (x & 0xff00) + (x & 0xff), twiddle =
 *     3 bf16 terms of the float table value; 6 exact products per frame,
 *     fp32 accumulation): error <= (6 N + 2) * 1.01 * 2^-24 * sum_t |S_t|;
 *   - otherwise fp32 MFMA on the float table: error <= (N + 2) * 2^-24 *
 *     sum_t |S_t|, the single-frequency path's bound.
 *   p_host  HOST int32 [n_freq], any integers (reduced mod q)
 *   re, im  device float [n_freq][H][W] (dense, overwritten)
 * QLD_E_INVAL for q < 1, t0 < 0 or a NULL p_host; QLD_E_SHAPE for n_frames < 1.
 */
qld_status qld_lockin_bank(const void *frames, const qld_frame_desc *d, int32_t n_frames, int32_t n_freq,
                           const int32_t *p_host, int32_t q, int32_t t0, float *re, float *im,
                           qld_hip_stream stream);

/* ------------------------------------------------------------------------ */
/* Sliding window (Supplementary: sliding sequence of N frames, buffer N n^2) */
/* ------------------------------------------------------------------------ */

typedef struct qld_window qld_window;

/* Device bytes a window of M_cycles cycles needs for frames described by d:
 * ring of per-cycle differences (4 B/px per cycle for bits <= 15, 8 B/px for
 * 16-bit data) + I/Q state (8 B/px).  0 for invalid arguments. */
size_t qld_window_bytes(const qld_frame_desc *d, int32_t M_cycles);

/* Create a window on the current device.  M_cycles >= 1 and
 * M_cycles * (2^bits - 1) < 2^31. */
qld_status qld_window_create(const qld_frame_desc *d, int32_t M_cycles, qld_window **out);

/*
 * Feed one cycle (four frames, phases 0..3, in the layout of d starting at
 * cycle_frames) and refresh the window:
 *     D = (S0 - S2, S1 - S3);   (I, Q) += D - D_oldest  (once M cycles are in)
 * I_out, Q_out (int32 [H][W]) and amp_out (float [H][W]) are device, each may
 * be NULL.  warm_out (host, may be NULL) receives 1 once the window holds M
 * cycles (0 before: the image then covers the cycles received so far).
 */
qld_status qld_window_update(qld_window *w, const void *cycle_frames, int32_t *I_out,
                             int32_t *Q_out, float *amp_out, int32_t *warm_out,
                             qld_hip_stream stream);

/* Forget every cycle (the next update starts a new window).  Enqueued on the
 * window's last stream. */
qld_status qld_window_reset(qld_window *w);
qld_status qld_window_destroy(qld_window *w);
/* Cycles currently in the window (0..M) and cycles fed since creation/reset. */
qld_status qld_window_info(const qld_window *w, int32_t *n_in_window, int64_t *n_cycles);
/* Checkpoint: ring, I/Q state and counters to a file; load restores them into
 * a window created with the same desc and M (QLD_E_STATE otherwise).  Both
 * synchronise with the device. */
qld_status qld_window_save(const qld_window *w, const char *path);
qld_status qld_window_load(qld_window *w, const char *path);

/* ------------------------------------------------------------------------ */
/* Per-frame sliding window: an image for every camera frame                */
/* (Supplementary, sliding sequence: the display refreshes on each frame)  */
/* ------------------------------------------------------------------------ */

typedef struct qld_fwindow qld_fwindow;

/* Device bytes of a per-frame window: a ring of 4*M_cycles raw frames plus
 * int32 I/Q state (0 for an invalid desc). */
size_t qld_fwindow_bytes(const qld_frame_desc *d, int32_t M_cycles);

/* Create a per-frame window of the last 4*M_cycles frames on the current
 * device.  Frame n (counted from creation or the last reset) has lock-in
 * phase (phase0 + n) mod 4.  M_cycles >= 1 and M_cycles * (2^bits - 1) < 2^31
 * (else QLD_E_OVERFLOW). */
qld_status qld_fwindow_create(const qld_frame_desc *d, int32_t M_cycles, int32_t phase0, qld_fwindow **out);

/*
 * Feed one frame (device, layout of d: rows row_pitch elements apart) and
 * refresh the window: with c, s the reference values of the frame's phase and
 * S_old the frame 4*M_cycles earlier (0 while the window is filling),
 *     I += c (S - S_old),   Q += s (S - S_old).
 * I_out, Q_out (int32 [H][W], both or neither) and amp_out (float [H][W]) are
 * device outputs, each may be NULL; warm_out (host, may be NULL) receives 1
 * once the window holds 4*M_cycles frames.  The quadratures use the absolute
 * phase of the frame counter, so the amplitude does not rotate between frames.
 */
qld_status qld_fwindow_update(qld_fwindow *w, const void *frame, int32_t *I_out, int32_t *Q_out,
                              float *amp_out, int32_t *warm_out, qld_hip_stream stream);

/* Forget every frame; the next frame has phase phase0 (e.g. after a gap). */
qld_status qld_fwindow_reset(qld_fwindow *w, int32_t phase0);
/* Frames currently in the window (0..4M) and frames fed since creation/reset. */
qld_status qld_fwindow_info(const qld_fwindow *w, int32_t *n_in_window, int64_t *n_frames);
qld_status qld_fwindow_destroy(qld_fwindow *w);

/* ------------------------------------------------------------------------ */
/* Serving: many camera streams, one GPU, continuous batching               */
/* ------------------------------------------------------------------------ */
/*
 * The paper's real-time loop (Supplementary Information, "Timing sequence for
 * hybrid parallelisation", which also displays a sliding sequence at the
 * camera rate) hands every camera frame on as it arrives: one thread
 * takes it from the camera, another copies it to the GPU, a kernel adds it to
 * the lock-in sums, and the image is refreshed from a sliding window.  The
 * server below does the same for many cameras at once: submits copy frames to
 * the device as they arrive, and a scheduler applies every complete cycle of
 * every stream that is ready in one batched launch.
 */

typedef struct qld_server qld_server;

/* PLAIN: the image is the window's amplitude R (Methods, R(j,k)).
 * LEARNED (not in the paper): every cycle the stream's denoiser maps the
 * short window's I/Q to a per-cycle amplitude; its gate decides whether that
 * image or the plain long-window amplitude per cycle is served (see
 * qld_stream_set_denoiser). */
typedef enum { QLD_MODE_PLAIN = 0, QLD_MODE_LEARNED = 1 } qld_mode;

/* Server flags. */
enum { QLD_SERVER_KEEP_IQ = 1 };   /* also keep per-cycle I/Q output slots */

typedef enum {
    QLD_STREAM_PENDING = 1,   /* waiting for HBM budget */
    QLD_STREAM_ACTIVE = 2,
    QLD_STREAM_CLOSED = 3
} qld_stream_state_t;

/* One processed image (one per complete cycle of a stream). */
typedef struct {
    int32_t stream_id;
    int32_t warm;              /* 1 once the window holds M cycles */
    int64_t cycle;             /* camera cycle index: frame_index / 4 of its frames */
    uint64_t t_arrival_ns;     /* arrival time of the cycle's last frame (caller's clock) */
    uint64_t t_done_ns;        /* CLOCK_MONOTONIC when the image was complete on the device */
    const float *amp;          /* device [H][W]; valid until out_slots more cycles of
                                  the stream complete, or the stream closes.
                                  PLAIN: R of the window.  LEARNED: the served
                                  image, amplitude per cycle (counts) */
    int32_t H, W;
    const float *amp_plain;    /* device [H][W], same lifetime: R of the (long)
                                  window; equals amp for a PLAIN stream */
    float gate;                /* LEARNED: the gate's predicted excess NRMSE, NaN
                                  while the short window is not yet full; PLAIN: 0 */
    int32_t learned;           /* 1 if amp is the denoiser's output */
    int64_t seq;               /* the stream's cycle count when this cycle was
                                  taken (0, 1, 2, ... over the stream's life);
                                  see qld_stream_result_valid */
} qld_result;

/*
 * Create a server on the current device.
 *   hbm_budget_bytes  device memory the server may hold for stream state
 *                     (window ring + I/Q state + frame staging + output slots)
 *   out_slots         images kept per stream (ring of output slots), 1..1024
 *   flags             QLD_SERVER_KEEP_IQ to also keep per-cycle I/Q
 * Starts a scheduler thread (batches every ready cycle of every stream into
 * one launch) and a completion thread (stamps t_done_ns, publishes results).
 * At most one launch round is on the device at a time (see
 * qld_server_set_max_inflight): cycles that complete while it runs are
 * gathered into the next round, so a launch carries the ready cycles of all
 * streams.  (Supplementary Information, "Timing sequence for hybrid
 * parallelisation": frames are processed as they arrive.)
 */
qld_status qld_server_create(size_t hbm_budget_bytes, int32_t out_slots, int32_t flags,
                             qld_server **out);

/* Device bytes one stream of this shape, window and mode costs under the
 * server's policy (what admission charges against the budget; a LEARNED
 * stream's denoiser is the caller's and is not counted). */
size_t qld_server_stream_bytes(const qld_server *s, const qld_frame_desc *d, int32_t M_cycles,
                               int32_t M_short, int32_t mode);

/* Open a stream of dense host frames (d->row_pitch/frame_stride are ignored)
 * (Supplementary Information, "Timing sequence for hybrid parallelisation":
 * one camera's frames handed to the GPU; admission by HBM budget is this
 * library's own)
 * with a window of M_cycles cycles and optionally a short window of M_short
 * (0 = none) cycles sharing the same ring.  mode: QLD_MODE_PLAIN, or
 * QLD_MODE_LEARNED (needs 1 <= M_short <= M_cycles, and a denoiser set with
 * qld_stream_set_denoiser before the first frame).  QLD_OK: admitted now.
 * QLD_E_AGAIN: queued (state PENDING); admitted in FIFO order once closes
 * free enough budget.  QLD_E_BUDGET: can never fit.  *stream_id is set in
 * the first two cases. */
qld_status qld_stream_open(qld_server *s, const qld_frame_desc *d, int32_t M_cycles,
                           int32_t M_short, int32_t mode, int32_t *stream_id);

qld_status qld_stream_state(qld_server *s, int32_t stream_id, int32_t *state);

typedef struct qld_denoiser qld_denoiser;

/*
 * Denoiser of a LEARNED stream (created by the caller for the stream's H x W,
 * any max_batch; it must outlive the stream or be replaced after
 * qld_server_drain, and the caller must not use it while the server may).
 * For each cycle c of the window (c = 0 after a reset) the server, on its
 * compute stream after the window update:
 *   - if c + 1 >= M_short: x = qld_denoise_prepare(short-window I/Q, each
 *     pixel's and the frame's sample sums over the short window), runs the
 *     forward (batch 1) and serves y * scale when gate <= gate_threshold;
 *   - otherwise, or when the gate is above the threshold, serves the plain
 *     long-window amplitude per cycle, R / min(c + 1, M_cycles).
 * Submissions to a LEARNED stream without a denoiser fail with QLD_E_STATE.
 * QLD_E_SHAPE if the denoiser's H x W differ from the stream's.
 */
qld_status qld_stream_set_denoiser(qld_server *s, int32_t stream_id, qld_denoiser *dn, float gate_threshold);

/*
 * Submit one frame (host pointer, dense [H][W] of the stream's dtype)
 * (Supplementary Information, "Timing sequence for hybrid parallelisation":
 * each camera frame is copied to the GPU as it arrives; here the hand-over
 * returns a status and no ticket -- the cycle's image is identified by its
 * stream and camera cycle in qld_stream_poll).  Frame
 * index f has lock-in phase f mod 4; a cycle is the four frames 4m..4m+3.
 * The frame is copied into pinned staging before the call returns, so the
 * caller may reuse its buffer at once; a frame already in page-locked host
 * memory (hipHostMalloc) is copied to the device straight from the caller's
 * buffer instead, and the call returns once that copy is done.  frame_index must be the previous
 * index + 1: a larger index resets the window (the partial cycle is dropped,
 * frames are skipped until the next index that is a multiple of 4) and the
 * call returns QLD_E_GAP; a smaller one is rejected (QLD_E_INVAL).  A pending
 * stream returns QLD_E_AGAIN.  Blocks while all staging slots of the stream
 * are in flight (back-pressure); while the server is held (qld_server_hold)
 * it returns QLD_E_AGAIN instead, having taken nothing (submit the same frame
 * again later).  Thread-safe: one submitting thread per stream.
 */
qld_status qld_stream_submit(qld_server *s, int32_t stream_id, const void *host_frame,
                             int64_t frame_index, uint64_t t_arrival_ns);

/*
 * Submit a whole cycle: the four frames first_frame_index .. +3 (host,
 * dense [4][H][W]), first_frame_index a multiple of 4 (else QLD_E_INVAL).
 * The same as four qld_stream_submit calls, with one copy into pinned
 * staging and one host-to-device copy instead of four.  A first_frame_index
 * beyond the next expected frame resets the window (a partial cycle from
 * single-frame submits is dropped) and returns QLD_E_GAP, the cycle itself
 * being taken as the first of the new window.  Back-pressure, hold and
 * threading as qld_stream_submit.  (Same passage as qld_stream_submit.)
 */
qld_status qld_stream_submit_cycle(qld_server *s, int32_t stream_id, const void *host_frames,
                                   int64_t first_frame_index, uint64_t t_arrival_ns);

/*
 * Hold (on != 0) or release (on = 0) the scheduler.  While held nothing is
 * launched; submits still copy frames into free staging slots.  Releasing
 * launches every staged cycle of every stream together (one launch per
 * sample format).  qld_server_drain, qld_stream_close and qld_server_destroy
 * release a hold.  For callers that gather a known set of cycles into one
 * launch (and for tests of batching).
 */
qld_status qld_server_hold(qld_server *s, int32_t on);

/*
 * Launch rounds the scheduler may have on the device at once, 1..64
 * (default 1).  With 1 every cycle that lands while a round runs waits for
 * the next round, which then carries them all; larger values launch sooner
 * and batch less.  QLD_E_INVAL outside the range.
 */
qld_status qld_server_set_max_inflight(qld_server *s, int32_t n);

/* Completed images, oldest first, at most max; *n_out set.  Non-blocking.
 * Returns QLD_E_DEVICE if a launch has failed.  (Supplementary Information,
 * "Timing sequence for hybrid parallelisation": the processed image is handed
 * on for display as soon as it is formed.) */
qld_status qld_stream_poll(qld_server *s, qld_result *out, int32_t max, int32_t *n_out);

/*
 * *valid = 1 while the output slot of a polled result still holds that
 * cycle's image (and I/Q), 0 once a later cycle of the stream has been
 * launched into the slot or the stream has closed.  A result's slot is
 * reused out_slots cycles later, so a slow reader can find a newer image
 * there: copy the image, then call this; 1 means the copy is this cycle's.
 */
qld_status qld_stream_result_valid(qld_server *s, const qld_result *res, int32_t *valid);

/* Device I/Q and short-window I/Q of a polled result, each NULL when not
 * kept: the long window's with QLD_SERVER_KEEP_IQ, the short window's with
 * QLD_SERVER_KEEP_IQ or in a LEARNED stream.  QLD_E_STATE if the stream keeps
 * neither.  Same lifetime as res->amp. */
qld_status qld_stream_result_iq(qld_server *s, const qld_result *res, const int32_t **I,
                                const int32_t **Q, const int32_t **Is, const int32_t **Qs);

/* Block until every submitted complete cycle has been processed. */
qld_status qld_server_drain(qld_server *s);

/* Close a stream: its pending cycles are finished, its unpolled results
 * dropped, its memory released, and queued streams admitted if they now fit. */
qld_status qld_stream_close(qld_server *s, int32_t stream_id);
qld_status qld_server_destroy(qld_server *s);

/* Counters: launches, cycles processed, most streams in one launch, budget bytes in use. */
qld_status qld_server_stats(const qld_server *s, int64_t *batches, int64_t *cycles,
                            int32_t *max_streams_in_batch, size_t *bytes_in_use);

/* ------------------------------------------------------------------------ */
/* Learned short-window path (not in the paper): training pairs, denoiser,  */
/* gate, judges.  Plain QLD is the fallback and the judge.                  */
/* ------------------------------------------------------------------------ */

/*
 * qld_gen_pairs -- training pairs generated by the lock-in itself.  Tile i is
 * a synthetic stack of Poisson frames (four samples per modulation period)
 * that is never stored: sample (t, y, x) = min(X_lambda(u), 2^bits - 1) with
 * lambda = rates_host[i][mask(y,x)][t mod 4] and u = word (t mod 4) of
 * Philox4x32-10(counter = (y*W + x, t / 4, tile0 + i, 0), key = seed), X the
 * Poisson inversion defined in the library source.  The lock-in sums of its
 * first M_short cycles go to I_S, Q_S and of its first M_long cycles to
 * I_L, Q_L (Methods, R(j,k)); sum_S / sum_L receive the tile's sample sums
 * over the same windows, and psum_S / psum_L (each may be NULL) each pixel's.
 *   mask       device uint8 [n_tiles][H][W] (0 or 1)
 *   rates_host HOST double [n_tiles][2][4], each in (0, 6000]
 *   outputs    device int32 [n_tiles][H][W]; uint64 [n_tiles]; uint32
 *              [n_tiles][H][W] (overwritten)
 * QLD_E_OVERFLOW if M_long * 4 * (2^bits - 1) >= 2^32.
 */
qld_status qld_gen_pairs(const uint8_t *mask, const double *rates_host, int32_t n_tiles, int32_t H,
                         int32_t W, int32_t M_short, int32_t M_long, uint32_t tile0, uint64_t seed,
                         int32_t bits, int32_t *I_S, int32_t *Q_S, int32_t *I_L, int32_t *Q_L,
                         uint64_t *sum_S, uint64_t *sum_L, uint32_t *psum_S, uint32_t *psum_L,
                         qld_hip_stream stream);

/*
 * Network input of the denoiser from a short window of M cycles: each
 * pixel's (I, Q) over the noise standard deviation of its own quadrature
 * sums, x = (I, Q) / sqrt(P / 2), P = psum_S the pixel's sample sum over the
 * window (for Poisson light of rate lam, Var(I) = Var(Q) = 2 M lam and P
 * estimates 4 M lam); x = 0 where P = 0.  scale[i] = sigma / sqrt(M), sigma^2 =
 * 2 b, b = sum_S / (H W 4 M) the tile's mean sample level, converts the
 * network output to counts per cycle.
 *   I_S, Q_S device int32 [B][H][W]; psum_S device uint32 [B][H][W];
 *   sum_S device uint64 [B]; x device float [B][H][W][2]; scale device float [B]
 *   (overwritten)
 */
qld_status qld_denoise_prepare(const int32_t *I_S, const int32_t *Q_S, const uint32_t *psum_S,
                               const uint64_t *sum_S, int32_t M_S, int32_t B, int32_t H, int32_t W, float *x,
                               float *scale, qld_hip_stream stream);

/* Training target: long-window amplitude per cycle with each pixel's noise
 * power removed, in network units: t = sqrt(max(I^2 + Q^2 - P, 0)) / M / scale,
 * P = psum_L the pixel's sample sum over the long window (E[I^2 + Q^2] is
 * 4 M lam without signal).
 *   psum_L device uint32 [B][H][W]; t device float [B][H][W] (overwritten) */
qld_status qld_denoise_target(const int32_t *I_L, const int32_t *Q_L, const uint32_t *psum_L,
                              int32_t M_L, const float *scale, int32_t B, int32_t H, int32_t W,
                              float *t, qld_hip_stream stream);

/* Per-cycle lock-in amplitude of the noise-free rates of each tile,
 * |(lambda_0 - lambda_2, lambda_1 - lambda_3)|: the reference of the NRMSE judge.
 *   mask device uint8 [B][H][W]; rates_host HOST double [B][2][4]; a device float [B][H][W] */
qld_status qld_clean_amplitude(const uint8_t *mask, const double *rates_host, int32_t B, int32_t H,
                               int32_t W, float *a, qld_hip_stream stream);

/* Judges, per tile, double-precision fixed-order reductions:
 *   qld_judge_nrmse: out[b] = RMS(x[b]*scale[b] - ref[b]) / RMS(ref[b]); scale may be NULL (1).
 *   qld_judge_cnr:   Eq. CNR of the paper (Methods): labels 1 = source, 2 = surround,
 *                    out[b] = (mean_src - mean_surr) / RMS(surr - mean_surr).
 * x, ref, img device float [B][n]; labels device uint8 [B][n]; out device float [B]. */
qld_status qld_judge_nrmse(const float *x, const float *scale, const float *ref, int32_t B, int64_t n,
                           float *out, qld_hip_stream stream);
qld_status qld_judge_cnr(const float *img, const uint8_t *labels, int32_t B, int64_t n, float *out,
                         qld_hip_stream stream);

/*
 * The denoiser: 3x3 convolutions 2 -> 32 -> 32 -> 32 -> 1 with bias, ReLU
 * between layers and zero "same" padding, NHWC bfloat16 activations, fp32
 * accumulation (matrix cores), fp32 master weights; plus a gate
 * gate[b] = mean_pixels(a3[b]) . Wg + bg predicting the tile's excess error.
 * Parameters (qld_denoiser_param_count() = 19426 floats, in this order):
 * W1[3][3][2][32] b1[32] W2[3][3][32][32] b2[32] W3[3][3][32][32] b3[32]
 * W4[3][3][32][1] b4[1] Wg[32] bg[1].  Work is enqueued on `stream`; the
 * object keeps the activations of its last forward for the backward.
 * Device memory: about 400 bytes per pixel of max_batch x H x W (bf16
 * activations and their gradients, fp32 output and its gradient) plus about
 * 85 MB whatever the size (the weight gradients' partial rows).
 */
int32_t qld_denoiser_param_count(void);
qld_status qld_denoiser_create(int32_t H, int32_t W, int32_t max_batch, qld_denoiser **out);
/* Shape the denoiser was created for. */
qld_status qld_denoiser_info(const qld_denoiser *d, int32_t *H, int32_t *W, int32_t *max_batch);
qld_status qld_denoiser_destroy(qld_denoiser *d);
/* Host copies (synchronous).  set_params also resets the optimizer state. */
qld_status qld_denoiser_set_params(qld_denoiser *d, const float *host, int32_t n);
qld_status qld_denoiser_get_params(qld_denoiser *d, float *host, int32_t n);
qld_status qld_denoiser_get_grads(qld_denoiser *d, float *host, int32_t n);
/* Device pointer to an internal tensor (0 x0 bf16 [B][H][W][2], 1..3 a1..a3
 * bf16 [B][H][W][32], 4 y f32, 5 dz3, 6 dz2, 10 dz1 (bf16 [B][H][W][32], the
 * ReLU-masked gradients of the hidden pre-activations), 7 pool f32 [B][32],
 * 8 gate f32 [B], 9 loss f32 [2]); sized for max_batch. */
qld_status qld_denoiser_tensor(qld_denoiser *d, int32_t which, void **ptr, int64_t *count);
/* x device float [B][H][W][2]; y_out device float [B][H][W] or NULL; gate_out device float [B] or NULL. */
qld_status qld_denoiser_forward(qld_denoiser *d, const float *x, int32_t B, float *y_out,
                                float *gate_out, qld_hip_stream stream);
/* Gradients of mean (y - t)^2 (weights W1..b4) and of the gate's own loss
 * gate_weight * mean (gate - (e_a - e_b))^2 (Wg, bg only; e_a NULL: none;
 * e_b may be NULL).  loss_out device float [2] or NULL. */
qld_status qld_denoiser_backward(qld_denoiser *d, const float *t, const float *e_a, const float *e_b,
                                 float gate_weight, int32_t B, float *loss_out, qld_hip_stream stream);
/* One Adam step (Kingma and Ba, 2015, bias-corrected) on all parameters. */
qld_status qld_denoiser_adam(qld_denoiser *d, float lr, float beta1, float beta2, float eps,
                             qld_hip_stream stream);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                              */
/* ------------------------------------------------------------------------ */
const char *qld_status_str(qld_status st);
const char *qld_last_error(void);
/* Device timing of the main kernel alone: start_event / stop_event are
 * hipEvent_t handles created by the caller.  The next qld_accumulate,
 * qld_lockin_image, dft_bin_baseline(_f64), qld_lockin_ratio,
 * qld_lockin_bank, qld_window_update, qld_fwindow_update, qld_read_probe or
 * qld_denoiser_forward call made by this thread records start_event on its
 * stream right before its main kernel (qld_accum_kernel / dft_bin_kernel /
 * the first bank kernel / window_batch_kernel / the frame-window kernel /
 * read_probe_kernel / the four convolution kernels) and stop_event right
 * after it, excluding the helper kernels (statistics and frame-split
 * reductions, twiddle tables, input conversion, pooling).  Both NULL
 * cancels. */
qld_status qld_time_next_kernel(void *start_event, void *stop_event);
/*
 * qld_read_probe -- measurement helper, not part of the method: a plain
 * streaming read of n_bytes of device memory at p (16-byte nontemporal loads),
 * the yardstick for the HBM fraction the batch kernels reach on a given
 * device.  *out (device uint64) = XOR of every 8-byte word of the buffer, so
 * the read cannot be optimised away and its result can be checked.  Timed by
 * qld_time_next_kernel like the batch calls.  QLD_E_ALIGN unless p is 16-byte
 * aligned and n_bytes a multiple of 16; QLD_E_INVAL for a NULL out (or p with
 * n_bytes > 0).
 */
qld_status qld_read_probe(const void *p, int64_t n_bytes, uint64_t *out, qld_hip_stream stream);
/* Library build string (compiler, target). */
const char *qld_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QLD_H */
