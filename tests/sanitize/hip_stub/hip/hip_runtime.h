// Host-only stand-in for the HIP runtime, for a CPU build of libtri's API
// layer (tri_api.hip) under AddressSanitizer/UndefinedBehaviorSanitizer.
// "Device" memory is host memory, streams and events are tokens, graph
// capture records nothing; kernel launchers are stubbed in api_stubs.cpp.
// Only what tri_api.hip and tri_internal.h use is declared.
#pragma once
#include <cstddef>
#include <cstdint>

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNoDevice = 100,
} hipError_t;
typedef enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4,
} hipMemcpyKind;
typedef enum hipStreamCaptureMode {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2,
} hipStreamCaptureMode;
struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph;
struct hipGraphExec;
struct hipGraphNode;
typedef ihipStream_t *hipStream_t;
typedef ihipEvent_t *hipEvent_t;
typedef ihipGraph *hipGraph_t;
typedef hipGraphExec *hipGraphExec_t;
typedef hipGraphNode *hipGraphNode_t;
#define hipStreamNonBlocking 0x01

// device-side qualifiers compile away in the host-only build
#define __device__
#define __host__
#define __align__(n) alignas(n)
#define HIP_SYMBOL(s) (&(s))

hipError_t hipGetDeviceCount(int *count);
hipError_t hipSetDevice(int device);
hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemset(void *dst, int value, size_t bytes);
hipError_t hipMemsetAsync(void *dst, int value, size_t bytes, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *err_node, char *log, size_t n);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetSymbolAddress(void **p, const void *symbol);
const char *hipGetErrorString(hipError_t e);
