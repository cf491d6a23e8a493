// Sliding-window lock-in: the batched update kernel's job table and the window
// object shared by qld_window_* and the server (internal, not part of the ABI).
#pragma once

#include "qld_internal.hpp"

namespace qld {

constexpr int kMaxJobs = 12;   // jobs per launch (kernel-argument table)

// One stream's share of a launch: n_cycles consecutive cycles, applied in order.
struct WinJob {
    const uint8_t *stage;    // frames of staged cycle slot 0
    int64_t rp_b, fs_b;      // row pitch / frame stride of the staged frames, bytes
    int64_t slot_b;          // bytes between staged cycle slots
    int32_t n_stage;         // staged cycle slots (cycle k of the job uses slot (stage0 + k) % n_stage)
    int32_t stage0;
    int32_t H, W, Wp;        // Wp: padded row length of ring/state (multiple of the lane width)
    int32_t M, Ms;           // window length; short window (0 = none), Ms <= M
    int64_t c0;              // window cycle index of the job's first cycle (0 after a reset)
    int32_t n_cycles;
    int32_t fresh;           // 1: start from an empty window (I = Q = 0)
    void *ring;              // [M][H][Wp] pairs (int16 or int32)
    int32_t *I, *Q;          // long-window state [H][Wp]
    int32_t *Is, *Qs;        // short-window state [H][Wp] (Ms > 0)
    float *amp;              // output slots [out_slots][H][W] or NULL
    int32_t *Io, *Qo;        // output slots for I/Q or NULL
    int32_t *Iso, *Qso;      // output slots for the short-window I/Q or NULL
    int32_t out_slots, out0; // cycle k of the job writes output slot (out0 + k) % out_slots
    int32_t tiles;           // work-groups this job uses
    int32_t _pad;
};

struct WinBatch {
    int32_t n_jobs;
    int32_t tile_start[kMaxJobs + 1];
    WinJob job[kMaxJobs];
};

// Launch the batched update.  elem = 1 or 2 bytes per sample; wide_ring: int32
// pairs (16-bit data) instead of int16 pairs; vec: every job's staged frames
// are 16-byte aligned with 16-byte multiple pitches.
hipError_t launch_window_batch(const WinBatch &b, int elem, bool wide_ring, bool vec, hipStream_t s);

// Enqueue a fill of n int32 with zero (a kernel, not a memset node).
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s);

// Lane width (pixels per lane) of the window kernel for this sample size.
inline int window_vpx(int elem) { return 16 / elem; }

}  // namespace qld

struct qld_window {
    qld_frame_desc d;
    int eb;
    int M, Ms;
    int wide;            // ring holds int32 pairs
    int Wp;
    void *ring;
    int32_t *I, *Q, *Is, *Qs;
    int64_t c;           // cycles since creation / reset
    int device;
    hipStream_t last_stream;
};

namespace qld {
// Allocate a window's device memory (ring + state) on the current device.
qld_status window_alloc(const qld_frame_desc *d, int32_t M, int32_t Ms, qld_window **out);
size_t window_bytes(const qld_frame_desc *d, int32_t M, int32_t Ms);
}  // namespace qld
