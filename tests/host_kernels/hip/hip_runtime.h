// Host execution model of the few HIP constructs the adjoint kernel
// templates use, for running those templates on the CPU under sanitizers
// (test infrastructure only: never part of the library build).  One block at
// a time, one OS thread per lane; __syncthreads and the wavefront barrier are
// a block-wide pthread barrier (stronger than a wave barrier); the hardware
// reciprocal estimate is an exact division.  Warp intrinsics and atomics the
// adjoint kernels do not call abort.
#pragma once
#include <pthread.h>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
using std::fma; using std::fmax; using std::fmin; using std::sqrt; using std::fabs; using std::isfinite;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__
struct dim3s { unsigned x, y, z; };
extern thread_local dim3s threadIdx, blockIdx;
extern dim3s gridDim, blockDim;
extern pthread_barrier_t g_block_barrier;
inline void __syncthreads() { pthread_barrier_wait(&g_block_barrier); }
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_fence(a, b) ((void)0)
#define __builtin_amdgcn_wave_barrier() __syncthreads()
struct double2 { double x, y; };
inline double2 make_double2(double a, double b) { return double2{a, b}; }
typedef int hipError_t;
typedef void* hipStream_t;
#define hipSuccess 0
inline int __lane_id() { return (int)(threadIdx.x & 63); }
template <class T> T __shfl_xor(T, int) { std::abort(); }
template <class T> T __shfl_up(T, int) { std::abort(); }
inline unsigned long long __ballot(int) { std::abort(); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
template <class T> T atomicAdd(T*, T) { std::abort(); }
template <class T> T atomicOr(T*, T) { std::abort(); }
template <class T> T atomicMax(T*, T) { std::abort(); }
inline long long __double_as_longlong(double) { std::abort(); }
#include <algorithm>
using std::min;
using std::max;
inline int hipGetDevice(int* d) { *d = 0; return 0; }
enum { hipDeviceAttributeMultiprocessorCount = 0 };
inline int hipDeviceGetAttribute(int* n, int, int) { *n = 256; return 0; }
template <class K> int hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, K, int, int) { *n = 1; return 0; }
