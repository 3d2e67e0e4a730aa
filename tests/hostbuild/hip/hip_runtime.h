// Host-only stand-in for the HIP runtime header, used to build the library's
// host code (argument checks, workspace planning, weight packing, the entry
// points' control flow) with a plain C++ compiler on a machine without a GPU,
// under the host sanitizers.  "Device" memory is host memory; streams and
// events are opaque tokens; there are no kernels: the library's launchers are
// replaced by counting stubs (fake_device.cpp).  Test infrastructure only.
#pragma once
#include <cstddef>
#include <cstdint>

typedef int hipError_t;
enum : int { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorNoDevice = 100,
             hipErrorLaunchFailure = 719 };
typedef struct fake_stream* hipStream_t;
typedef struct fake_event* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
struct hipDeviceProp_t {
  int multiProcessorCount;
  char gcnArchName[256];
};
struct int2 {
  int x, y;
};
inline int2 make_int2(int x, int y) { return int2{x, y}; }

#define __host__
#define __device__
#define __global__
#define __shared__
#define __forceinline__ inline
#define __align__(n) alignas(n)
#define __launch_bounds__(...)
#define HIP_SYMBOL(s) (static_cast<const void*>(&(s)))

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
