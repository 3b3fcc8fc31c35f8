// Shared definitions for the ufalcon HIP sources.
// The device helpers are also compilable as plain host C++ (UFX_HOST_BUILD) so
// that their logic can be exercised on a machine without a GPU.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__) && !defined(UFX_HOST_BUILD)
#include <hip/hip_runtime.h>
#define UFX_FN __device__ __forceinline__
#define UFX_NOINLINE __device__ __noinline__
#define UFX_HD __host__ __device__ inline
#else
#include <cmath>
using std::fabs;
using std::floor;
using std::fmax;
using std::fmin;
using std::fma;
using std::sqrt;
using std::atan2;
#define UFX_FN inline
#define UFX_NOINLINE __attribute__((noinline))
#define UFX_HD inline
#endif
