// evec.h -- shared definitions of the eigenvector kernels (paper Sec. 2,
// Eqs. (5) and (6)).
#pragma once
#include <hip/hip_runtime.h>

namespace schur {

constexpr int EVT = 64;      // eigenvector columns per workgroup of the tile solve
constexpr int EVTMAX = 66;   // largest tile row (64, moved so that no 2x2 block is split)

// S: the real Schur form (lds); Y: the eigenvectors being computed (ldy,
// n x n, upper quasi-triangular); colmax[r] = max_{i < r} |S(i, r)|;
// bound[j]: upper bound of the pending entries of eigenvector j.
struct EvArgs {
  const double* S; int lds;
  double* Y; int ldy;
  int n;
  double* colmax;
  double* bound;
};

void launch_ev_prep(const EvArgs& g, hipStream_t s);
void launch_ev_diag(const EvArgs& g, int r0, int r1, hipStream_t s);
void launch_ev_normalise(double* X, int ldx, const double* S, int lds, int n, hipStream_t s);

}  // namespace schur
