// batch.h -- host view of the persistent batched kernel (batch_kernels.hip):
// the job and scratch layouts shared by the host driver and the device code.
#pragma once
#include <hip/hip_runtime.h>

#include "schur_internal.h"

namespace schur {

constexpr int PB_THREADS = 256;
constexpr int PB_NBMAX = PB_THREADS / 32;   // bulges per window chain (window chase)
constexpr int PB_NMAX = 8192;               // largest order (deflation bitmap in LDS)

// One matrix of a persistent batched launch (device array, read-only).
struct PJob {
  double* H; double* Q; double* wr; double* wi;   // Q may be null
  int ldh, ldq, n;
  int ns, nb, step, nw, nibble, nmin, exc_period, max_sweeps;   // resolved, in range
  int* info;          // out: 0, > 0 (no convergence: rows 1..info not in Schur form) or < 0
  double* counters;   // out (optional): PB_COUNTERS values, see below
};

// counters of one matrix (counts, and flops counted as the host solver
// counts them: panel products from their shapes, 20 ws nb per chain step
// and window, 25 m^3 per small block with Z, 10 m^3 per shift solve,
// 25 nw^3 + 10/3 nu^3 per early-deflation window)
enum {
  PB_SWEEPS = 0, PB_WINDOWS, PB_CHAIN_STEPS, PB_AED_WINDOWS, PB_AED_DEFLATED, PB_SMALL,
  PB_SHIFTS, PB_GEMM_FLOPS, PB_CHASE_FLOPS, PB_SMALL_FLOPS, PB_AED_FLOPS, PB_COUNTERS
};

// Per-workgroup global scratch.
struct PScratch {
  double U[UPAD * UPAD];                           // a window's U^T (zero padded)
  double ewr[SMALL_EIG_MAX], ewi[SMALL_EIG_MAX];   // eigenvalues of a trailing block
  double sr[SMALL_Z_MAX], si[SMALL_Z_MAX];         // undeflated early-deflation eigenvalues
  double st[SMALL_EIG_MAX];                        // shift pairs (sum, product)
};

// Zero the queue counter, then launch `grid` workgroups of the persistent
// kernel over `count` jobs taken in `order` (device arrays; scratch: grid
// PScratch blocks).
void launch_batch_persistent(const PJob* jobs, const int* order, int count, int* next,
                             PScratch* scratch, int grid, hipStream_t s);

}  // namespace schur
