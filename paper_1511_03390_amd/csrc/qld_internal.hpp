// Internal helpers shared by the libqld translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/qld.h"

namespace qld {

// Native 128-bit vector (one global_load_dwordx4).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Thread-local message of the most recent failure (qld_last_error()).
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

// Returns QLD_E_DEVICE (with a message) if `e` is an error.
qld_status check_hip(hipError_t e, const char *what);

// Events set by qld_time_next_kernel for this thread (consumed by the next
// main-kernel launch: records `start` before it and `stop` after it).
void take_kernel_timer(hipEvent_t *start, hipEvent_t *stop);

// Device scratch owned by the library, one buffer per (device, stream) so
// calls on different streams never share it.  Grows on demand; never shrinks.
// Returns nullptr (and sets the error) if the allocation fails.
void *stream_workspace(hipStream_t stream, size_t bytes);

// Number of compute units of the current device (cached per device).
int device_cu_count();

// Validation shared by the entry points.  Returns QLD_OK or an error status
// (with the message set).  elem_bytes receives 1 or 2.
qld_status check_desc(const qld_frame_desc *d, int *elem_bytes);

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Rotation of the local quadratures by the lock-in phase of the first frame:
// one step of phase maps (I, Q) to (-Q, I).
__host__ __device__ inline void rotate_iq(int rot, int32_t i, int32_t q, int32_t &oi, int32_t &oq) {
    switch (rot & 3) {
        case 0: oi = i;  oq = q;  break;
        case 1: oi = -q; oq = i;  break;
        case 2: oi = -i; oq = -q; break;
        default: oi = q; oq = -i; break;
    }
}

}  // namespace qld

#define QLD_TRY(...)                               \
    do {                                           \
        qld_status _st = (__VA_ARGS__);            \
        if (_st != QLD_OK) return _st;             \
    } while (0)
