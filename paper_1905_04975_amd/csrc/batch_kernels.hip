// batch_kernels.hip -- the persistent batched kernel: a grid of one
// workgroup per CU takes matrices from a queue (sorted by cost, largest
// first) and runs each whole Schur reduction on the device (batch_solve.h),
// so a batch of matrices of uneven orders is one launch.
#define SCHUR_SOLVER_WAVE_SYNC 1
#include "batch_solve.h"

namespace schur {

static_assert(PB_LDS_D * sizeof(double) + sizeof(PShared) + 64 <= 163840, "160 KiB of LDS");

// next: queue counter (zero before the launch); order: job indices in the
// order they are taken; every workgroup leaves once the queue is empty.
__global__ __launch_bounds__(PB_THREADS, 1) void k_batch_persistent(const PJob* jobs,
                                                                   const int* order, int count,
                                                                   int* next, PScratch* scratch) {
  __shared__ double lds[PB_LDS_D];
  __shared__ PShared sh;
  PScratch* X = scratch + blockIdx.x;
  while (true) {
    if (threadIdx.x == 0) sh.job = atomicAdd(next, 1);
    __syncthreads();
    const int q = sh.job;
    if (q >= count) break;
    pb_solve(jobs[order[q]], lds, sh, X);
    __syncthreads();
  }
}

__global__ void k_pb_reset(int* next) {
  if (threadIdx.x == 0) *next = 0;
}

void launch_batch_persistent(const PJob* jobs, const int* order, int count, int* next,
                             PScratch* scratch, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_pb_reset, dim3(1), dim3(64), 0, s, next);
  if (count > 0 && grid > 0)
    hipLaunchKernelGGL(k_batch_persistent, dim3(grid), dim3(PB_THREADS), 0, s, jobs, order, count,
                       next, scratch);
}

}  // namespace schur
