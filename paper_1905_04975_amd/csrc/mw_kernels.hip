// mw_kernels.hip -- kernels whose Francis iteration runs on a workgroup of
// four wavefronts, as chains of up to four bulges, one per wavefront
// (small_iter_mw): the windows of the parallel early-deflation passes, the
// bottom early-deflation windows, the whole small blocks with Schur vectors
// and the eigenvalue problems that give a sweep its shifts.  Their reorderings, spike reductions and V^T products are shared
// by the four wavefronts too; the one-wavefront parts around them (loading,
// flips, standardisation) are wavefront 0's, so the solvers' barrier is the
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

// Whole small block with Schur vectors, one per workgroup.
template <int MAXM>
__global__ __launch_bounds__(64 * SPLIT_WAVES) void k_small_z(SmallTask t0, const SmallTask* tasks) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  __shared__ double S[LD * MAXM];
  __shared__ double Z[LD * MAXM];
  __shared__ double aux[SMALL_MW_AUX];
  const SmallTask T = tasks ? tasks[blockIdx.x] : t0;
  if (T.m <= 0 || T.m > MAXM) return;
  small_qr<true, MAXM, SPLIT_WAVES>(T, S, Z, aux);
}

void launch_small_z(const SmallTask& t, const SmallTask* tasks, int count, int maxm,
                    hipStream_t s) {
  const dim3 g(count), b(64 * SPLIT_WAVES);
  if (maxm <= 32)
    hipLaunchKernelGGL((k_small_z<32>), g, b, 0, s, t, tasks);
  else if (maxm <= 64)
    hipLaunchKernelGGL((k_small_z<64>), g, b, 0, s, t, tasks);
  else
    hipLaunchKernelGGL((k_small_z<SMALL_Z_MAX>), g, b, 0, s, t, tasks);
}

// Eigenvalues of a small block (the shifts of a sweep), one per workgroup.
template <int MAXM>
__global__ __launch_bounds__(64 * SPLIT_WAVES) void k_small_eig(SmallTask t0, const SmallTask* tasks) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  __shared__ double S[LD * MAXM];
  __shared__ double aux[SMALL_MW_AUX];
  const SmallTask T = tasks ? tasks[blockIdx.x] : t0;
  if (T.m <= 0 || T.m > MAXM) return;
  small_qr<false, MAXM, SPLIT_WAVES>(T, S, nullptr, aux);
}

void launch_small_eig(const SmallTask& t, hipStream_t s) {
  const dim3 b(64 * SPLIT_WAVES);
  const SmallTask* none = nullptr;
  if (t.m <= 32)
    hipLaunchKernelGGL((k_small_eig<32>), dim3(1), b, 0, s, t, none);
  else if (t.m <= 64)
    hipLaunchKernelGGL((k_small_eig<64>), dim3(1), b, 0, s, t, none);
  else
    hipLaunchKernelGGL((k_small_eig<SMALL_EIG_MAX>), dim3(1), b, 0, s, t, none);
}

void launch_small_eig_b(const SmallTask* tasks, int count, int maxm, hipStream_t s) {
  if (count <= 0) return;
  const dim3 g(count), b(64 * SPLIT_WAVES);
  SmallTask none{};
  if (maxm <= 32)
    hipLaunchKernelGGL((k_small_eig<32>), g, b, 0, s, none, tasks);
  else if (maxm <= 64)
    hipLaunchKernelGGL((k_small_eig<64>), g, b, 0, s, none, tasks);
  else
    hipLaunchKernelGGL((k_small_eig<SMALL_EIG_MAX>), g, b, 0, s, none, tasks);
}

// One bottom early-deflation window per workgroup.
template <int MAXM>
__global__ __launch_bounds__(64 * SPLIT_WAVES) void k_aed(AedTask t0, const AedTask* tasks) {
  const AedTask T = tasks ? tasks[blockIdx.x] : t0;
  constexpr int LD = SmallSmem<MAXM>::LD;
  static_assert(7 * MAXM >= SMALL_MW_AUX, "the iteration's scratch lives in stdbuf");
  __shared__ double S[LD * MAXM];
  __shared__ double Z[LD * MAXM];
  __shared__ double vv[MAXM];
  __shared__ int ibuf[6 * MAXM];
  __shared__ double stdbuf[7 * MAXM];
  aed_window<MAXM, SPLIT_WAVES>(T, S, Z, vv, ibuf, stdbuf);
}

void launch_aed(const AedTask& t, hipStream_t s) {
  hipLaunchKernelGGL((k_aed<SMALL_Z_MAX>), dim3(1), dim3(64 * SPLIT_WAVES), 0, s, t,
                     (const AedTask*)nullptr);
}

void launch_aed_b(const AedTask* tasks, int count, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL((k_aed<SMALL_Z_MAX>), dim3(count), dim3(64 * SPLIT_WAVES), 0, s, AedTask{},
                       tasks);
}

void launch_split(const SplitTask* tasks, int count, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL((k_split<SMALL_Z_MAX>), dim3(count), dim3(64 * SPLIT_WAVES), 0, s, tasks);
}

}  // namespace schur
