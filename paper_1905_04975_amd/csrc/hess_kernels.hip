// hess_kernels.hip -- kernels of the Hessenberg reduction A = Q1 H Q1^T
// (paper Sec. 2, Eq. (3)) and the general FP64 matrix product they use.
//
// The reduction is the blocked Householder method: panels of NBH columns;
// inside a panel each column is brought up to date with the panel's earlier
// reflectors (from the right through Y = A V T, from the left through
// I - V T V^T), its reflector is generated, and Y gains a column from one
// product of the trailing matrix with the new reflector (a matrix-vector
// product, the part of the method that streams the whole trailing matrix
// from HBM for every column).  After the panel the trailing matrix and Q
// receive the panel's transformation as matrix-matrix products (FP64 MFMA).
//
// Every kernel here is written for gfx950 (64-wide wavefronts); the
// reductions over rows run in a fixed order (per-workgroup partials combined
// by every consumer in the same order), so results are bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hess.h"

namespace schur {

typedef double d4h __attribute__((ext_vector_type(4)));

// ============================================================================
// General FP64 product C = alpha op(A) op(B) + beta C (beta 0 or 1), column-
// major, on the 16x16x4 FP64 MFMA.  A workgroup (4 wavefronts) owns a 128 x BN
// tile of C; wavefront w owns rows 32w..32w+31 of it.  K advances in chunks
// of 16 staged through double-buffered LDS, the next chunk's loads issued
// before the current chunk's products.  MFMA operand layout (16x16x4 f64):
// lane l holds A(l & 15, l >> 4) and B(l >> 4, l & 15); result element e of
// lane l is C(l >> 4 + 4 e, l & 15).
// ============================================================================
constexpr int GBM = 128;
constexpr int GBK = 16;

template <int BN, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, double alpha,
                                              const double* __restrict__ A, int lda,
                                              const double* __restrict__ B, int ldb, double beta,
                                              double* __restrict__ C, int ldc) {
  constexpr int LA = GBM + 1;   // padded LDS rows (conflict-free transposed stores)
  constexpr int LB = BN + 1;
  constexpr int NA = GBM * GBK / 256;   // A elements per thread and chunk
  constexpr int NB = BN * GBK / 256;    // B elements per thread and chunk
  constexpr int JB = BN / 16;
  __shared__ double As[2][GBK * LA];
  __shared__ double Bs[2][GBK * LB];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * BN;
  const int i0 = wave * 32;

  // element e of this thread's chunk loads: (row of op(A), k) and (k, column of op(B))
  auto a_idx = [&](int e, int& i, int& k) {
    if (TA) { k = tid & 15; i = (tid >> 4) + 16 * e; }
    else { i = tid & 127; k = (tid >> 7) + 2 * e; }
  };
  auto b_idx = [&](int e, int& k, int& j) {
    if (TB) { j = tid % BN; k = tid / BN + (256 / BN) * e; }
    else { k = tid & 15; j = (tid >> 4) + 16 * e; }
  };
  double ra[NA], rb[NB];
  auto load = [&](int kc) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      int i, k;
      a_idx(e, i, k);
      const int gi = m0 + i, gk = kc + k;
      ra[e] = (gi < M && gk < K) ? (TA ? A[(size_t)gk + (size_t)gi * lda]
                                       : A[(size_t)gi + (size_t)gk * lda]) : 0.0;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      int k, j;
      b_idx(e, k, j);
      const int gj = n0 + j, gk = kc + k;
      rb[e] = (gj < N && gk < K) ? (TB ? B[(size_t)gj + (size_t)gk * ldb]
                                       : B[(size_t)gk + (size_t)gj * ldb]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      int i, k;
      a_idx(e, i, k);
      As[buf][k * LA + i] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      int k, j;
      b_idx(e, k, j);
      Bs[buf][k * LB + j] = rb[e];
    }
  };

  d4h acc[2][JB];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) acc[ib][jb] = d4h{0.0, 0.0, 0.0, 0.0};

  const int nchunks = (K + GBK - 1) / GBK;
  if (nchunks > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    const bool more = c + 1 < nchunks;
    if (more) load((c + 1) * GBK);
    const double* as = As[buf];
    const double* bs = Bs[buf];
#pragma unroll
    for (int ks = 0; ks < GBK / 4; ++ks) {
      const int k = 4 * ks + lk;
      const double a0 = as[k * LA + i0 + li];
      const double a1 = as[k * LA + i0 + 16 + li];
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const double b = bs[k * LB + jb * 16 + li];
        acc[0][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc[0][jb], 0, 0, 0);
        acc[1][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc[1][jb], 0, 0, 0);
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = m0 + i0 + 16 * ib + lk + 4 * e;
        const int gj = n0 + 16 * jb + li;
        if (gi < M && gj < N) {
          double* cp = C + (size_t)gi + (size_t)gj * ldc;
          const double v = alpha * acc[ib][jb][e];
          *cp = (beta != 0.0) ? v + beta * *cp : v;
        }
      }
}

template <int BN, bool TA, bool TB>
static void gemm_launch(int M, int N, int K, double alpha, const double* A, int lda,
                        const double* B, int ldb, double beta, double* C, int ldc,
                        hipStream_t s) {
  dim3 grid((M + GBM - 1) / GBM, (N + BN - 1) / BN);
  hipLaunchKernelGGL((k_gemm<BN, TA, TB>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, B,
                     ldb, beta, C, ldc);
}

template <int BN>
static void gemm_bn(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                    const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s) {
  if (!ta && !tb) gemm_launch<BN, false, false>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
  else if (!ta && tb) gemm_launch<BN, false, true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
  else if (ta && !tb) gemm_launch<BN, true, false>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
  else gemm_launch<BN, true, true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

void launch_gemm(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                 const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  if (N <= 32) gemm_bn<32>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
  else if (N <= 64) gemm_bn<64>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
  else gemm_bn<128>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

// ============================================================================
// Panel factorisation, one column c = K + i of the panel starting at column K.
// Rows handled: K+1 .. n-1, HROWS per workgroup (one row per thread).
// Workspace (HessWs): V and Y (n x NBH, ld n), T (NBH x NBH, ld NBH), and
// per-workgroup partials.
// ============================================================================

// sum over the 64 lanes of a wavefront (butterfly: every lane gets the sum)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// per-workgroup sums of x_l over the workgroup's rows for l < cnt, written to
// out[l]; `red` is LDS of at least 4 * NBH doubles (x stays in registers:
// every index is a constant after unrolling, cnt only masks)
__device__ __forceinline__ void block_sums(const double (&x)[NBH], int cnt, double* red,
                                           double* out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int l = 0; l < NBH; ++l) {
    if (l < cnt) {
      const double s = wave_sum(x[l]);
      if (lane == 0) red[wave * NBH + l] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    const int l = threadIdx.x;
    out[l] = ((red[l] + red[NBH + l]) + red[2 * NBH + l]) + red[3 * NBH + l];
  }
}

// (a) right and left updates of column c by the panel's first i reflectors:
//     a <- a - Y(:, 0:i) V(c, 0:i)^T, then partial sums of V(:, 0:i)^T a.
__global__ __launch_bounds__(HROWS) void k_hcol_a(HessArgs g, int K, int i) {
  __shared__ double red[4 * NBH];
  const int n = g.n, c = K + i;
  const int r = K + 1 + blockIdx.x * HROWS + threadIdx.x;
  const bool ok = r < n;
  double a = ok ? g.A[(size_t)r + (size_t)c * g.lda] : 0.0;
  if (ok) {
    for (int l = 0; l < i; ++l) a -= g.Y[(size_t)r + (size_t)l * n] * g.V[(size_t)c + (size_t)l * n];
    g.A[(size_t)r + (size_t)c * g.lda] = a;
  }
  double x[NBH];
#pragma unroll
  for (int l = 0; l < NBH; ++l) x[l] = (ok && l < i) ? g.V[(size_t)r + (size_t)l * n] * a : 0.0;
  block_sums(x, i, red, g.part + (size_t)blockIdx.x * HPART);
}

// (b) a <- a - V(:, 0:i) T(0:i, 0:i)^T w with w the sum of the partials of
//     (a); then per workgroup the scale and scaled sum of squares of the
//     column below row K+i+1 (the reflector's tail).
__global__ __launch_bounds__(HROWS) void k_hcol_b(HessArgs g, int K, int i, int nwg) {
  __shared__ double wt[NBH];
  __shared__ double red[4];
  const int n = g.n, c = K + i;
  const int r = K + 1 + blockIdx.x * HROWS + threadIdx.x;
  const bool ok = r < n;
  const int l = threadIdx.x;
  if (l < i) {
    double wl = 0.0;
    for (int b = 0; b < nwg; ++b) wl += g.part[(size_t)b * HPART + l];
    wt[l] = wl;
  }
  __syncthreads();
  double tw = 0.0;   // (T^T w)_l = sum_{k <= l} T(k, l) w_k
  if (l < i)
    for (int k = 0; k <= l; ++k) tw += g.T[k + l * NBH] * wt[k];
  __syncthreads();
  if (l < i) wt[l] = tw;
  __syncthreads();
  double a = ok ? g.A[(size_t)r + (size_t)c * g.lda] : 0.0;
  if (ok && i > 0) {
    for (int k = 0; k < i; ++k) a -= g.V[(size_t)r + (size_t)k * n] * wt[k];
    g.A[(size_t)r + (size_t)c * g.lda] = a;
  }
  if (r == K + i + 1) g.sc[0] = a;   // the pivot entry, read by (c)
  // tail of the reflector: rows K+i+2 .. n-1
  const bool tail = ok && r >= K + i + 2;
  const double m = wave_max(tail ? fabs(a) : 0.0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[wave] = m;
  __syncthreads();
  const double mb = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  const double t = (tail && mb > 0.0) ? a / mb : 0.0;
  const double ss = wave_sum(t * t);
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double* p = g.part2 + 2 * (size_t)blockIdx.x;
    p[0] = mb;
    p[1] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// scale-safe norm of the reflector's tail from the per-workgroup (scale,
// scaled sum of squares) pairs; every caller combines them in the same order
__device__ double tail_norm(const double* part2, int nwg) {
  double mx = 0.0;
  for (int b = 0; b < nwg; ++b) mx = fmax(mx, part2[2 * b]);
  if (mx == 0.0) return 0.0;
  double ss = 0.0;
  for (int b = 0; b < nwg; ++b) {
    const double f = part2[2 * b] / mx;
    ss += part2[2 * b + 1] * f * f;
  }
  return mx * sqrt(ss);
}

// (c) the reflector of column c: beta = -sign(alpha) ||(alpha, tail)||,
//     tau = (beta - alpha) / beta, v = (1, tail / (alpha - beta)); v goes to
//     V(:, i), the column of A gets beta and exact zeros below it; partial
//     sums of V(:, 0:i)^T v.
__global__ __launch_bounds__(HROWS) void k_hcol_c(HessArgs g, int K, int i, int nwg) {
  __shared__ double red[4 * NBH];
  const int n = g.n, c = K + i;
  const int r = K + 1 + blockIdx.x * HROWS + threadIdx.x;
  const bool ok = r < n;
  const int rp = K + i + 1;   // pivot row
  const double alpha = g.sc[0];   // the pivot row's workgroup overwrites A(rp, c) below
  const double xn = tail_norm(g.part2, nwg);
  double beta = alpha, tau = 0.0, scal = 0.0;
  if (xn != 0.0) {
    const double h = hypot(alpha, xn);
    beta = alpha >= 0.0 ? -h : h;
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  double v = 0.0;
  if (ok) {
    if (r == rp) v = 1.0;
    else if (r > rp) v = g.A[(size_t)r + (size_t)c * g.lda] * scal;
    g.V[(size_t)r + (size_t)i * n] = v;
    if (r == rp) g.A[(size_t)r + (size_t)c * g.lda] = beta;
    else if (r > rp) g.A[(size_t)r + (size_t)c * g.lda] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) g.tau[i] = tau;
  double x[NBH];
#pragma unroll
  for (int l = 0; l < NBH; ++l) x[l] = (ok && l < i) ? g.V[(size_t)r + (size_t)l * n] * v : 0.0;
  block_sums(x, i, red, g.part3 + (size_t)blockIdx.x * HPART);
}

// (d) y = A(K+1:n, K+i+1:n) v over a slice of columns: grid (row blocks,
//     column splits); split s writes its partial to ypart(:, s).
__global__ __launch_bounds__(HROWS) void k_hgemv(HessArgs g, int K, int i, int csplit) {
  const int n = g.n;
  const int r = K + 1 + blockIdx.x * HROWS + threadIdx.x;
  const int j0 = K + i + 1;
  const int cols = n - j0;
  const int per = (cols + csplit - 1) / csplit;
  const int ja = j0 + blockIdx.y * per;
  const int jb = min(n, ja + per);
  const double* vv = g.V + (size_t)i * n;
  if (r >= n) return;
  const double* col = g.A + (size_t)r;
  double s[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = 0.0;
  int j = ja;
  for (; j + 8 <= jb; j += 8) {   // eight loads in flight per thread
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = col[(size_t)(j + u) * g.lda];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += a[u] * vv[j + u];
  }
  for (; j < jb; ++j) s[0] += col[(size_t)j * g.lda] * vv[j];
  g.ypart[(size_t)r + (size_t)blockIdx.y * n] =
      ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// (e) Y(:, i) = tau (y - Y(:, 0:i) q) with q = V(:, 0:i)^T v (sum of the
//     partials of (c)); the first workgroup also writes T's column i:
//     T(0:i, i) = -tau T(0:i, 0:i) q, T(i, i) = tau.
__global__ __launch_bounds__(HROWS) void k_hy(HessArgs g, int K, int i, int nwg, int csplit) {
  __shared__ double q[NBH];
  const int n = g.n;
  const int r = K + 1 + blockIdx.x * HROWS + threadIdx.x;
  if (threadIdx.x < i) {
    const int l = threadIdx.x;
    double s = 0.0;
    for (int b = 0; b < nwg; ++b) s += g.part3[(size_t)b * HPART + l];
    q[l] = s;
  }
  __syncthreads();
  const double tau = g.tau[i];
  if (r < n) {
    double y = 0.0;
    for (int s = 0; s < csplit; ++s) y += g.ypart[(size_t)r + (size_t)s * n];
    for (int l = 0; l < i; ++l) y -= g.Y[(size_t)r + (size_t)l * n] * q[l];
    g.Y[(size_t)r + (size_t)i * n] = tau * y;
  }
  if (blockIdx.x == 0 && threadIdx.x <= i) {
    const int k = threadIdx.x;
    double t;
    if (k == i) {
      t = tau;
    } else {   // -tau (T q)_k, T upper triangular
      double s = 0.0;
      for (int l = k; l < i; ++l) s += g.T[k + l * NBH] * q[l];
      t = -tau * s;
    }
    g.T[k + i * NBH] = t;
  }
}

// zero the panel's V and T (and Y's columns) before a panel
__global__ void k_hzero(double* p, size_t count) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < count;
       k += (size_t)gridDim.x * blockDim.x)
    p[k] = 0.0;
}

void launch_hess_zero(double* p, size_t count, hipStream_t s) {
  const int blocks = (int)std::min<size_t>(4096, (count + 255) / 256);
  if (blocks > 0) hipLaunchKernelGGL(k_hzero, dim3(blocks), dim3(256), 0, s, p, count);
}

void launch_hess_column(const HessArgs& g, int K, int i, int csplit, hipStream_t s) {
  const int rows = g.n - K - 1;
  const int nwg = (rows + HROWS - 1) / HROWS;
  if (i > 0) hipLaunchKernelGGL(k_hcol_a, dim3(nwg), dim3(HROWS), 0, s, g, K, i);
  hipLaunchKernelGGL(k_hcol_b, dim3(nwg), dim3(HROWS), 0, s, g, K, i, nwg);
  hipLaunchKernelGGL(k_hcol_c, dim3(nwg), dim3(HROWS), 0, s, g, K, i, nwg);
  hipLaunchKernelGGL(k_hgemv, dim3(nwg, csplit), dim3(HROWS), 0, s, g, K, i, csplit);
  hipLaunchKernelGGL(k_hy, dim3(nwg), dim3(HROWS), 0, s, g, K, i, nwg, csplit);
}

}  // namespace schur
