// split_kernels.hip -- the window kernel of the parallel early-deflation
// passes: one window per workgroup of four wavefronts.  The Francis
// iteration of the window runs as chains of up to four bulges, one per
// wavefront (small_iter_mw); the reorderings, the spike reductions and the
// write-back that follow are wavefront 0's, so the solvers' barrier is the
// wavefront-local one here.
#define SCHUR_SOLVER_WAVE_SYNC 1
#include "schur_internal.h"
#include "device_common.h"
#include "kernels.h"
#include "wave_solvers.h"

namespace schur {

constexpr int SPLIT_WAVES = 4;

template <int MAXM>
__global__ __launch_bounds__(64 * SPLIT_WAVES) void k_split(const SplitTask* tasks) {
  const SplitTask T = tasks[blockIdx.x];
  constexpr int LD = SmallSmem<MAXM>::LD;
  static_assert(7 * MAXM >= SMALL_MW_AUX, "the iteration's scratch lives in pbuf");
  __shared__ double S[LD * MAXM];
  __shared__ double Z[LD * MAXM];
  __shared__ double vv[MAXM];
  __shared__ int ibuf[6 * MAXM];
  __shared__ double pbuf[7 * MAXM];
  split_window<MAXM, SPLIT_WAVES>(T, S, Z, vv, ibuf, pbuf);
}

void launch_split(const SplitTask* tasks, int count, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL((k_split<SMALL_Z_MAX>), dim3(count), dim3(64 * SPLIT_WAVES), 0, s, tasks);
}

}  // namespace schur
