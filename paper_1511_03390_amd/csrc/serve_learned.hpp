// Kernels of a LEARNED serving stream (internal, not part of the ABI).
#pragma once

#include "qld_internal.hpp"

namespace qld {

// Work-groups of the per-cycle sample sum (partials per cycle).
constexpr int kCycleSumBlocks = 128;

// Per-work-group sums of the samples of n_cycles staged cycles; cycle i of the
// job (window cycle c0 + i) is in staging slot (stage0 + i) % n_stage and its
// partials go to csum[((c0 + i) % ring) * nblk + block].
hipError_t launch_cycle_sums(const uint8_t *stage, int64_t slot_b, int n_stage, int stage0, int n_cycles, int eb,
                             uint64_t *csum, int ring, int64_t c0, int nblk, hipStream_t s);

// sumS[0] = sum of the partials of window cycles c_last - Ms + 1 .. c_last (fixed order).
hipError_t launch_window_sum(const uint64_t *csum, int ring, int nblk, int64_t c_last, int Ms, uint64_t *sumS,
                             hipStream_t s);

// Per-pixel sample sums of n_cycles staged cycles: pixel (y, x) of cycle i of
// the job (window cycle c0 + i, staging slot (stage0 + i) % n_stage, frames of
// fs_b bytes with rows of rp_b bytes) -> pcs[((c0 + i) % ring) * H * W + y * W + x].
hipError_t launch_pixel_cycle_sums(const uint8_t *stage, int64_t slot_b, int64_t fs_b, int64_t rp_b, int n_stage,
                                   int stage0, int n_cycles, int eb, int H, int W, uint32_t *pcs, int ring,
                                   int64_t c0, hipStream_t s);

// psum[p] = sum of pcs over window cycles c_last - Ms + 1 .. c_last (exact, uint32).
hipError_t launch_pixel_window_sum(const uint32_t *pcs, int ring, int64_t npx, int64_t c_last, int Ms, uint32_t *psum,
                                   hipStream_t s);

// served = (gate && gate[0] <= thr) ? y * scale[0] : plain * inv_n; gate_slot[0] = gate[0] (NaN if gate is NULL).
hipError_t launch_serve(const float *y, const float *scale, const float *gate, const float *plain, int64_t npx,
                        float thr, float inv_n, float *served, float *gate_slot, hipStream_t s);

}  // namespace qld
