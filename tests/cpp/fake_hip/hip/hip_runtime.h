// Host-only stand-in for the parts of the HIP runtime API that the serving
// runtime (server.cpp) and the library's host helpers (capi.cpp) call, so
// that they can be built with a host compiler and run under the thread,
// address and undefined-behaviour sanitizers on a machine without a GPU.
// TEST INFRASTRUCTURE ONLY: "device" memory is host memory and every
// asynchronous operation completes before the call returns (fake_device.cpp).
#pragma once

#include <cstddef>
#include <cstdint>

#define __host__
#define __device__
#define __forceinline__ inline

struct ihipStream_t;
struct ihipEvent_t;
typedef ihipStream_t *hipStream_t;
typedef ihipEvent_t *hipEvent_t;

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorLaunchFailure = 719,
} hipError_t;

typedef enum {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
} hipMemcpyKind;

typedef enum { hipDeviceAttributeMultiprocessorCount = 63 } hipDeviceAttribute_t;

typedef enum hipMemoryType {
    hipMemoryTypeUnregistered = 0,
    hipMemoryTypeHost = 1,
    hipMemoryTypeDevice = 2,
} hipMemoryType;

typedef struct hipPointerAttribute_t {
    enum hipMemoryType type;
    int device;
    void *devicePointer;
    void *hostPointer;
    int isManaged;
    unsigned allocationFlags;
} hipPointerAttribute_t;

constexpr unsigned hipEventDisableTiming = 0x2;
constexpr unsigned hipStreamNonBlocking = 0x1;
constexpr unsigned hipHostMallocDefault = 0x0;

hipError_t hipMalloc(void **p, size_t bytes);
template <typename T>
inline hipError_t hipMalloc(T **p, size_t bytes) {
    return hipMalloc(reinterpret_cast<void **>(p), bytes);
}
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned flags);
template <typename T>
inline hipError_t hipHostMalloc(T **p, size_t bytes, unsigned flags) {
    return hipHostMalloc(reinterpret_cast<void **>(p), bytes, flags);
}
hipError_t hipHostFree(void *p);
hipError_t hipMemset(void *p, int v, size_t bytes);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind kind, hipStream_t s);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipSetDevice(int dev);
hipError_t hipGetDevice(int *dev);
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t attr, int dev);
// hipMemoryTypeHost inside a hipHostMalloc allocation; hipErrorInvalidValue
// (and a sticky last error, as the runtime leaves) for any other host pointer.
hipError_t hipPointerGetAttributes(hipPointerAttribute_t *attr, const void *p);
