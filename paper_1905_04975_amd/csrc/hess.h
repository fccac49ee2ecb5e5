// hess.h -- shared definitions of the Hessenberg-reduction kernels
// (paper Sec. 2, Eq. (3)) and the general FP64 product.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace schur {

constexpr int NBH = 32;      // panel width (reflectors per panel)
constexpr int HROWS = 256;   // rows per workgroup of the column kernels
constexpr int HPART = NBH;   // doubles per workgroup partial

// Everything the column kernels of one panel touch.  V, Y: n x NBH (ld n);
// T: NBH x NBH (ld NBH), upper triangular, I - V T V^T = P_0 P_1 ...;
// part, part3: per-workgroup partial sums (HPART each); part2: per-workgroup
// (scale, scaled sum of squares); ypart: n x csplit partial products; tau:
// NBH reflector factors; sc[0]: the pivot entry of the current column.
struct HessArgs {
  double* A; int lda; int n;
  double* V; double* Y; double* T;
  double* part; double* part2; double* part3;
  double* ypart; double* tau; double* sc;
};

// C = alpha op(A) op(B) + beta C (beta 0: C is not read), column-major
void launch_gemm(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                 const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s);
void launch_hess_zero(double* p, size_t count, hipStream_t s);
// column c = K + i of the panel starting at K: update, reflector, Y column
void launch_hess_column(const HessArgs& g, int K, int i, int csplit, hipStream_t s);

}  // namespace schur
