// The CPU stand-in for the HIP runtime (see hip/hip_runtime.h).  Test support only.
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <vector>

#include "hip/hip_runtime.h"
#include "host_stub.h"

struct StubStream {
  bool capturing = false;
  std::vector<std::function<void()>> rec;
};
struct StubEvent {
  int dummy = 0;
};
struct StubGraph {
  std::vector<std::function<void()>> ops;
};

void stub_submit(hipStream_t s, std::function<void()> fn) {
  if (s && s->capturing) s->rec.push_back(std::move(fn));
  else fn();
}

hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDeviceCount(int* count) {
  *count = 1;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int) {
  prop->multiProcessorCount = 8;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new StubStream();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new StubEvent();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipMallocBytes(void** p, size_t bytes) {
  *p = calloc(1, bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipHostMallocBytes(void** p, size_t bytes, unsigned) { return hipMallocBytes(p, bytes); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  stub_submit(s, [=] { memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s) {
  stub_submit(s, [=] { memset(dst, value, bytes); });
  return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes) {
  *free_bytes = (size_t)8 << 30;
  *total_bytes = (size_t)16 << 30;
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub error"; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  s->capturing = true;
  s->rec.clear();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  StubGraph* gr = new StubGraph();
  gr->ops.swap(s->rec);
  s->capturing = false;
  *g = gr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  StubGraph* e = new StubGraph();
  e->ops = g->ops;
  *exec = e;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s) {
  for (auto& op : exec->ops) stub_submit(s, op);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
  delete exec;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
