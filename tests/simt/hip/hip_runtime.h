// CPU stand-in for the parts of the HIP device API that the LDS-resident
// kernels use, so that their device source runs on the host: one workgroup
// is a set of std::threads; __syncthreads is a barrier over all of them,
// the wavefront barrier one over the 64 threads of a wavefront, and
// __shfl_xor / __shfl / __ballot / readlane / the FP64 MFMA exchange values through
// memory between wavefront barriers.
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
double __shfl(double x, int src, int w);
unsigned long long __ballot(int p);
int simt_readlane(int v, int src);
void simt_wave_barrier();
#define __builtin_amdgcn_wave_barrier() simt_wave_barrier()
#define __builtin_amdgcn_fence(a, b) ((void)0)
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_readlane(v, l) simt_readlane((v), (l))
#define __builtin_amdgcn_readfirstlane(v) simt_readlane((v), 0)
#define __builtin_amdgcn_s_waitcnt(x) ((void)0)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __noinline__ __attribute__((noinline))
using std::max;
using std::min;
// FP64 MFMA 16x16x4 of one wavefront (lanes exchange operands through memory)
typedef double simt_d4 __attribute__((ext_vector_type(4)));
simt_d4 simt_mfma_f64_16x16x4(double a, double b, simt_d4 c);
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) simt_mfma_f64_16x16x4((a), (b), (c))
// Raw buffer descriptors: base and byte range.  A load at an offset past
// the range returns 0 and such a store is dropped, as on the GPU; an access
// that straddles the end of the range is a kernel bug and aborts.
struct simt_rsrc {
  char* base;
  unsigned nrec;
};
typedef simt_rsrc __amdgpu_buffer_rsrc_t;
typedef unsigned simt_u2 __attribute__((ext_vector_type(2)));
inline simt_rsrc __builtin_amdgcn_make_buffer_rsrc(void* p, short stride, int nrec, int flags) {
  if (stride != 0 || flags != 0x00020000) __builtin_trap();
  return simt_rsrc{(char*)p, (unsigned)nrec};
}
inline simt_u2 __builtin_amdgcn_raw_buffer_load_b64(simt_rsrc r, int off, int soff, int aux) {
  const unsigned o = (unsigned)off + (unsigned)soff;
  simt_u2 v = {0u, 0u};
  if (o >= r.nrec) return v;
  if (o + 8u > r.nrec || aux != 0) __builtin_trap();
  memcpy(&v, r.base + o, 8);
  return v;
}
inline void __builtin_amdgcn_raw_buffer_store_b64(simt_u2 v, simt_rsrc r, int off, int soff, int aux) {
  const unsigned o = (unsigned)off + (unsigned)soff;
  if (o >= r.nrec) return;
  if (o + 8u > r.nrec || aux != 0) __builtin_trap();
  memcpy(r.base + o, &v, 8);
}
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline unsigned atomicOr(unsigned* p, unsigned v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
