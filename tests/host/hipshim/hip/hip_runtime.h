// Host stand-in for the few HIP runtime names that the in-LDS FFT header
// (csrc/fft_core.h) and its includes use, so that the FFT stages compile
// for the CPU: each GPU thread of a block becomes a std::thread, threadIdx
// is thread-local and __syncthreads() is a std::barrier over the block
// (fft_emulate.cpp).  Only for the CPU check of the transforms.
#pragma once

#include <cstddef>

#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)

struct double2 {
  double x, y;
};
struct float2 {
  float x, y;
};

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2 };
inline const char* hipGetErrorString(hipError_t) { return "host emulation"; }
typedef struct ihipStream_t* hipStream_t;

struct EmuDim3 {
  unsigned x = 0, y = 0, z = 0;
};
extern thread_local EmuDim3 threadIdx;
void __syncthreads();
