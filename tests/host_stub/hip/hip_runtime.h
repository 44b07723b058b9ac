// A CPU stand-in for the HIP runtime, for building the engine's host driver
// (api.cpp) without a GPU so that its threading (batches, servers, the hub)
// can run under ThreadSanitizer and AddressSanitizer.  Device memory is host
// memory, streams run their work on the calling thread at once (or record it
// while a graph is captured), and events carry no time.  Test support only.
#pragma once

#include <cstddef>
#include <cstdint>

typedef enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidDevice = 101,
} hipError_t;

typedef struct StubStream* hipStream_t;
typedef struct StubEvent* hipEvent_t;
typedef struct StubGraph* hipGraph_t;
typedef struct StubGraph* hipGraphExec_t;
typedef struct StubGraphNode* hipGraphNode_t;

struct hipDeviceProp_t {
  int multiProcessorCount;
};

enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
};

#define hipStreamNonBlocking 1u
#define hipHostMallocDefault 0u
#define hipEventDisableTiming 2u
#define HIP_SYMBOL(x) (&(x))

hipError_t hipSetDevice(int device);
hipError_t hipGetDeviceCount(int* count);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int device);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipMallocBytes(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMallocBytes(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s);
hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, hipGraphNode_t* err_node, char* log, size_t len);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphDestroy(hipGraph_t g);

template <typename T>
inline hipError_t hipMalloc(T** p, size_t bytes) {
  return hipMallocBytes(reinterpret_cast<void**>(p), bytes);
}
template <typename T>
inline hipError_t hipHostMalloc(T** p, size_t bytes, unsigned flags) {
  return hipHostMallocBytes(reinterpret_cast<void**>(p), bytes, flags);
}
