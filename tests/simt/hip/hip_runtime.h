// CPU stand-in for the parts of the HIP device API that the LDS-resident
// kernels use, so that their device source runs on the host: one workgroup
// is a set of std::threads; __syncthreads is a barrier over all of them,
// the wavefront barrier one over the 64 threads of a wavefront, and
// __shfl_xor / __ballot / readlane exchange values through memory between
// barriers.
// Threads run freely between barriers, which is stricter than lock-step
// wavefronts: a kernel that relied on lock-step without a barrier shows a
// race here.  Every __shared__ object lands in one section that the driver
// fills with NaN bytes before each workgroup, so a read of LDS that the
// kernel never wrote surfaces as a NaN in its output.
#pragma once
#include <math.h>
#include <cmath>
#include <stdint.h>
#include <stddef.h>
#include <string.h>
using std::isfinite;
#define __device__
#define __global__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static __attribute__((section("simt_lds")))
typedef void* hipStream_t;
typedef int hipError_t;
struct simt_dim3 {
  unsigned x, y, z;
};
extern thread_local simt_dim3 threadIdx;
extern thread_local simt_dim3 blockIdx;
extern simt_dim3 blockDim;
void __syncthreads();
double __shfl_xor(double x, int o, int w);
unsigned long long __ballot(int p);
int simt_readlane(int v, int src);
void simt_wave_barrier();
#define __builtin_amdgcn_wave_barrier() simt_wave_barrier()
#define __builtin_amdgcn_fence(a, b) ((void)0)
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_readlane(v, l) simt_readlane((v), (l))
#define __builtin_amdgcn_readfirstlane(v) simt_readlane((v), 0)
