// Host-only stand-in for the HIP runtime, for one purpose: compiling the HIP
// backend's host code (backend_hip.hip) with g++ -fsanitize=thread, so that
// ThreadSanitizer sees every access its threads make to the backend's own
// bookkeeping and to the runtime objects it shares between threads.
//
// It is never part of libset.so.  Semantics kept from the real runtime:
//  - a stream is an in-order queue, drained by a thread of its own;
//  - an event completes when its stream reaches it; a wait on an event made
//    by another stream holds that stream back until then;
//  - a graph executable keeps its own copy of every node's parameters; an
//    update rewrites that copy, and a launch reads it when the stream
//    executes the node (as the device reads a graph's kernel arguments from
//    memory the executable owns), so an update that overlaps a launch of the
//    same executable is a data race ThreadSanitizer reports;
//  - stream capture records kernel launches and copies as a linear chain;
//  - "device" memory is host memory, so kernels (host functions here, run on
//    stream threads) and host code touch the same bytes, as on the device.
// Kernels are looked up by address in a registry the stub's own kernel
// definitions fill; launching an unregistered address fails.
#pragma once

#include <cstddef>
#include <cstdint>

#define __global__
#define __device__
#define __host__
#define __shared__
#define __launch_bounds__(...)
#define __forceinline__ inline

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorNotReady = 600,
  hipErrorNotSupported = 801,
  hipErrorUnknown = 999
} hipError_t;

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned x_ = 1, unsigned y_ = 1, unsigned z_ = 1) : x(x_), y(y_), z(z_) {}
};

typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph* hipGraph_t;
typedef struct hipGraphNode* hipGraphNode_t;
typedef struct hipGraphExec* hipGraphExec_t;
typedef void (*hipHostFn_t)(void* userData);

typedef enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipGraphNodeType {
  hipGraphNodeTypeKernel = 0,
  hipGraphNodeTypeMemcpy = 1,
  hipGraphNodeTypeMemset = 2,
  hipGraphNodeTypeHost = 3
} hipGraphNodeType;

typedef enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;

struct hipKernelNodeParams {
  dim3 blockDim;
  void** extra;
  void* func;
  dim3 gridDim;
  void** kernelParams;
  unsigned int sharedMemBytes;
};

#define hipStreamDefault 0x0
#define hipStreamNonBlocking 0x1
#define hipEventDefault 0x0
#define hipEventBlockingSync 0x1
#define hipEventDisableTiming 0x2
#define hipHostMallocDefault 0x0

const char* hipGetErrorString(hipError_t e);
typedef enum hipDeviceAttribute_t { hipDeviceAttributeWallClockRate = 1 } hipDeviceAttribute_t;
hipError_t hipGetDeviceCount(int* n);
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t attr, int dev);
hipError_t hipSetDevice(int dev);
hipError_t hipGetDevice(int* dev);
hipError_t hipDeviceSynchronize();

hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemset(void* dst, int value, size_t bytes);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void* user);
hipError_t hipLaunchKernel(const void* func, dim3 grid, dim3 block, void** args, size_t shmem, hipStream_t s);

hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);

hipError_t hipGraphCreate(hipGraph_t* g, unsigned flags);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphAddKernelNode(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* p);
hipError_t hipGraphAddMemcpyNode1D(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                   void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipGraphGetNodes(hipGraph_t g, hipGraphNode_t* nodes, size_t* n);
hipError_t hipGraphNodeGetDependencies(hipGraphNode_t node, hipGraphNode_t* deps, size_t* n);
hipError_t hipGraphNodeGetDependentNodes(hipGraphNode_t node, hipGraphNode_t* deps, size_t* n);
hipError_t hipGraphNodeGetType(hipGraphNode_t node, hipGraphNodeType* t);
hipError_t hipGraphKernelNodeGetParams(hipGraphNode_t node, hipKernelNodeParams* p);
hipError_t hipGraphInstantiateWithFlags(hipGraphExec_t* ex, hipGraph_t g, unsigned long long flags);
hipError_t hipGraphExecDestroy(hipGraphExec_t ex);
hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t ex, hipGraphNode_t node, const hipKernelNodeParams* p);
hipError_t hipGraphExecMemcpyNodeSetParams1D(hipGraphExec_t ex, hipGraphNode_t node, void* dst, const void* src,
                                             size_t bytes, hipMemcpyKind kind);
hipError_t hipGraphUpload(hipGraphExec_t ex, hipStream_t s);
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);

// Registry of the stub's kernels: a kernel's address maps to the size of its
// single argument struct and a function that runs it on a copy of that struct.
namespace hipstub {
typedef void (*Invoke)(const void* func, const void* args);
void register_kernel(const void* func, size_t arg_bytes, Invoke run);
template <class A>
void register_kernel(void (*f)(A)) {
  register_kernel((const void*)f, sizeof(A), [](const void* fn, const void* args) {
    reinterpret_cast<void (*)(A)>(const_cast<void*>(fn))(*static_cast<const A*>(args));
  });
}
// Counters the stress driver reads.
uint64_t launches();
uint64_t updates_while_in_flight();
}  // namespace hipstub
