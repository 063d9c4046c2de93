// Host stand-in for the HIP runtime header, so that the FFT and pair-stage
// device bodies can be compiled by a host compiler and run by one thread
// (every pass reads all its inputs before its barrier and writes after it,
// so a single thread executes a workgroup's bodies exactly).
#pragma once
#include <cmath>
#define __device__
#define __host__
#define __forceinline__ inline
#define __syncthreads() ((void)0)
struct double2 { double x, y; };
struct float2 { float x, y; };
typedef int hipError_t;
typedef void* hipStream_t;
struct cpu_dim3 { unsigned x = 0, y = 0, z = 0; };
static cpu_dim3 threadIdx, blockIdx, blockDim, gridDim;
template <typename X> X __shfl_down(X v, int, int) { return v; }
using std::expm1;
using std::fma;
