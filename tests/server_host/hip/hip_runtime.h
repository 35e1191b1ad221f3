// CPU stand-in for the HIP runtime, for the served mode's host-code harness
// (tests/test_server_host.py): the types and the few calls that code makes.
// Not part of the library; nothing here runs on a GPU.
#pragma once
#include <cstddef>
#include <cstdint>

#define __host__
#define __device__
#define __global__
#define __shared__
#define __forceinline__ inline

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
enum { hipStreamNonBlocking = 1 };

hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int *d);
