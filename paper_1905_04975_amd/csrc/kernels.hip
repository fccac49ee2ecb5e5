// kernels.hip -- CDNA4 (gfx950) device kernels of the Schur engine.
//
// Kernel families (paper Sec. 3.2; the window / right-update / left-update
// task types of Sec. 3.2 become kernel roles here):
//   k_small_*     whole Francis double-shift QR of a small block in LDS, used
//                 for the shifts (eigenvalues of a trailing block), for the
//                 last small active blocks and for whole small matrices
//   k_chase       the window task: bulge introduction and chasing with
//                 overlapping 3x3 Householder reflectors inside an LDS window,
//                 then accumulation of the window's orthogonal factor U
//   k_panel_row   left update of the row panel  H(win, right) <- U^T H(win, right)
//   k_panel_colq  right update of the column panel and of Q  X <- X U
//                 (both as FP64 MFMA matrix products)
//   k_deflate     negligible-subdiagonal scan and bottom deflation
//   k_std_*       2x2 standardisation of the converged blocks and (wr, wi)
#include "schur_internal.h"
#include "device_common.h"
#include "kernels.h"

namespace schur {

typedef double d4 __attribute__((ext_vector_type(4)));

// ============================================================================
// Small-block Francis double-shift QR (one wavefront, block in LDS)
// ============================================================================

// Column-major LDS block with odd leading dimension (spreads banks).
template <int MAXM>
struct SmallSmem {
  static constexpr int LD = MAXM | 1;
};

// Francis double-shift iteration on the m x m block already in LDS (S, and Z
// when WANTZ), one wavefront.  Writes T.wr / T.wi of converged blocks when
// given; returns 0 or the 1-based end of a block that did not converge.
template <bool WANTZ, int MAXM>
__device__ int small_iter(const SmallTask& T, double* S, double* Zs) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = T.m;
  const int lane = threadIdx.x;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };

  int i = m - 1, its = 0, info = 0;
  const int itmax = T.itmax > 0 ? T.itmax : 30;
  while (i >= 0) {
    // ---- deflation search: largest k in [1, i] with a negligible subdiagonal
    int l = 0;
    for (int top = i; top >= 1; top -= 64) {
      const int k = top - lane;
      bool neg = false;
      if (k >= 1) {
        const double sub = fabs(Sx(k, k - 1));
        double tst = fabs(Sx(k - 1, k - 1)) + fabs(Sx(k, k));
        if (tst == 0.0) {
          tst = fabs(Sx(k - 1, k));
          if (k >= 2) tst += fabs(Sx(k - 1, k - 2));
          if (k + 1 <= i) tst += fabs(Sx(k + 1, k));
        }
        neg = (sub <= kUlp * tst);
      }
      const unsigned long long mask = __ballot(neg);
      if (mask) {
        l = top - __builtin_ctzll(mask);
        break;
      }
    }
    __syncthreads();
    if (l > 0 && lane == 0) Sx(l, l - 1) = 0.0;
    __syncthreads();

    if (l == i) {
      if (lane == 0 && T.wr) { T.wr[i] = Sx(i, i); T.wi[i] = 0.0; }
      i -= 1; its = 0;
      continue;
    }
    if (l == i - 1) {
      const Std2 o = standardize2(Sx(i - 1, i - 1), Sx(i - 1, i), Sx(i, i - 1), Sx(i, i));
      __syncthreads();
      if (WANTZ && !(o.cs == 1.0 && o.sn == 0.0)) {
        for (int c = i + 1 + lane; c < m; c += 64) {
          const double x = Sx(i - 1, c), y = Sx(i, c);
          Sx(i - 1, c) = o.cs * x + o.sn * y;
          Sx(i, c) = o.cs * y - o.sn * x;
        }
        for (int r = lane; r < i - 1; r += 64) {
          const double x = Sx(r, i - 1), y = Sx(r, i);
          Sx(r, i - 1) = o.cs * x + o.sn * y;
          Sx(r, i) = o.cs * y - o.sn * x;
        }
        for (int r = lane; r < m; r += 64) {
          const double x = Zx(r, i - 1), y = Zx(r, i);
          Zx(r, i - 1) = o.cs * x + o.sn * y;
          Zx(r, i) = o.cs * y - o.sn * x;
        }
      }
      if (lane == 0) {
        if (WANTZ) {
          Sx(i - 1, i - 1) = o.a; Sx(i - 1, i) = o.b;
          Sx(i, i - 1) = o.c;     Sx(i, i) = o.d;
        }
        if (T.wr) {
          T.wr[i - 1] = o.wr1; T.wi[i - 1] = o.wi1;
          T.wr[i] = o.wr2;     T.wi[i] = o.wi2;
        }
      }
      __syncthreads();
      i -= 2; its = 0;
      continue;
    }
    its += 1;
    if (its > itmax) { info = i + 1; break; }

    // ---- shifts: trailing 2x2 (Francis) or the ad-hoc exceptional pair
    double s, t;
    if (its == 10 || its == 20) {
      double w, e;
      if (its == 10) {
        w = fabs(Sx(i, i - 1)) + fabs(Sx(i - 1, i - 2));
        e = Sx(i, i) + 0.75 * w;
      } else {
        w = fabs(Sx(l + 1, l)) + fabs(Sx(l + 2, l + 1));
        e = Sx(l, l) + 0.75 * w;
      }
      s = e + e;
      t = e * e + 0.4375 * w * w;
    } else {
      const double a = Sx(i - 1, i - 1), b = Sx(i - 1, i), c = Sx(i, i - 1), d = Sx(i, i);
      s = a + d;
      t = a * d - b * c;
    }

    // ---- one double-shift step on rows/cols l..i
    const int cend = WANTZ ? m - 1 : i;    // last column of left updates
    const int rbeg = WANTZ ? 0 : l;        // first row of right updates
    double x, y, z;
    first_column(Sx(l, l), Sx(l, l + 1), Sx(l + 1, l), Sx(l + 1, l + 1), Sx(l + 2, l + 1), s, t,
                 x, y, z);
    for (int r = l; r <= i - 1; ++r) {
      const int nr = (r <= i - 2) ? 3 : 2;
      if (r > l) {
        x = Sx(r, r - 1);
        y = Sx(r + 1, r - 1);
        z = (nr == 3) ? Sx(r + 2, r - 1) : 0.0;
      }
      const Refl h = make_reflector(nr, x, y, z);
      __syncthreads();
      if (h.tau == 0.0) continue;
      const double tv2 = h.tau * h.v2, tv3 = h.tau * h.v3;
      for (int c = r + lane; c <= cend; c += 64) {
        const double a1 = Sx(r, c), a2 = Sx(r + 1, c);
        const double a3 = (nr == 3) ? Sx(r + 2, c) : 0.0;
        const double w = a1 + h.v2 * a2 + h.v3 * a3;
        Sx(r, c) = a1 - h.tau * w;
        Sx(r + 1, c) = a2 - tv2 * w;
        if (nr == 3) Sx(r + 2, c) = a3 - tv3 * w;
      }
      if (r > l && lane == 0) {
        Sx(r, r - 1) = h.beta;
        Sx(r + 1, r - 1) = 0.0;
        if (nr == 3) Sx(r + 2, r - 1) = 0.0;
      }
      __syncthreads();
      const int rlast = (r + 3 < i) ? r + 3 : i;
      for (int q = rbeg + lane; q <= rlast; q += 64) {
        const double a1 = Sx(q, r), a2 = Sx(q, r + 1);
        const double a3 = (nr == 3) ? Sx(q, r + 2) : 0.0;
        const double w = a1 + h.v2 * a2 + h.v3 * a3;
        Sx(q, r) = a1 - h.tau * w;
        Sx(q, r + 1) = a2 - tv2 * w;
        if (nr == 3) Sx(q, r + 2) = a3 - tv3 * w;
      }
      if (WANTZ) {
        for (int q = lane; q < m; q += 64) {
          const double a1 = Zx(q, r), a2 = Zx(q, r + 1);
          const double a3 = (nr == 3) ? Zx(q, r + 2) : 0.0;
          const double w = a1 + h.v2 * a2 + h.v3 * a3;
          Zx(q, r) = a1 - h.tau * w;
          Zx(q, r + 1) = a2 - tv2 * w;
          if (nr == 3) Zx(q, r + 2) = a3 - tv3 * w;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  return info;
}

template <bool WANTZ, int MAXM>
__device__ void small_load(const SmallTask& T, double* S, double* Zs) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = T.m;
  const int lane = threadIdx.x;
  for (int c = 0; c < m; ++c)
    for (int r = lane; r < m; r += 64)
      S[r + c * LD] = (r <= c + 1) ? T.A[r + (size_t)c * T.lda] : 0.0;
  if (WANTZ)
    for (int c = 0; c < m; ++c)
      for (int r = lane; r < m; r += 64) Zs[r + c * LD] = (r == c) ? 1.0 : 0.0;
  __syncthreads();
}

template <bool WANTZ, int MAXM>
__device__ void small_qr(const SmallTask& T, double* S, double* Zs) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = T.m;
  const int lane = threadIdx.x;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };
  small_load<WANTZ, MAXM>(T, S, Zs);
  const int info = small_iter<WANTZ, MAXM>(T, S, Zs);
  if (lane == 0 && T.info) *T.info = info;
  if (WANTZ) {
    // Schur form of the block back to global memory, Z^T into the U slot layout
    for (int c = 0; c < m; ++c)
      for (int r = lane; r < m; r += 64) T.A[r + (size_t)c * T.lda] = Sx(r, c);
    if (T.Zt) {
      for (int c = 0; c < T.ldzt; ++c)
        for (int r = lane; r < T.ldzt; r += 64)
          T.Zt[r + (size_t)c * T.ldzt] = (r < m && c < m) ? Zx(c, r) : 0.0;
    }
    if (T.Z) {
      for (int c = 0; c < m; ++c)
        for (int r = lane; r < m; r += 64) T.Z[r + (size_t)c * T.ldz] = Zx(r, c);
    }
    if (T.Qacc) {
      // Qacc <- Qacc Z, rows by lanes, 16 columns at a time; the block's LDS
      // copy (already written back) is the staging area
      __syncthreads();
      for (int r = lane; r < m; r += 64) {
        for (int c0 = 0; c0 < m; c0 += 16) {
          double acc[16];
#pragma unroll
          for (int j = 0; j < 16; ++j) acc[j] = 0.0;
          for (int k = 0; k < m; ++k) {
            const double q = T.Qacc[r + (size_t)k * T.ldqacc];
#pragma unroll
            for (int j = 0; j < 16; ++j)
              if (c0 + j < m) acc[j] += q * Zx(k, c0 + j);
          }
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (c0 + j < m) Sx(r, c0 + j) = acc[j];
        }
      }
      __syncthreads();
      for (int c = 0; c < m; ++c)
        for (int r = lane; r < m; r += 64) T.Qacc[r + (size_t)c * T.ldqacc] = Sx(r, c);
    }
  }
}

template <int MAXM>
__global__ __launch_bounds__(64) void k_small_z(SmallTask t0, const SmallTask* tasks) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  __shared__ double S[LD * MAXM];
  __shared__ double Z[LD * MAXM];
  const SmallTask T = tasks ? tasks[blockIdx.x] : t0;
  if (T.m <= 0 || T.m > MAXM) return;
  small_qr<true, MAXM>(T, S, Z);
}

template <int MAXM>
__global__ __launch_bounds__(64) void k_small_eig(SmallTask t0, const SmallTask* tasks) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  __shared__ double S[LD * MAXM];
  const SmallTask T = tasks ? tasks[blockIdx.x] : t0;
  if (T.m <= 0 || T.m > MAXM) return;
  small_qr<false, MAXM>(T, S, nullptr);
}

// ============================================================================
// Aggressive early deflation (paper Sec. 3.2: the algorithm alternates AED
// steps with bulge-chasing sweeps).  One wavefront owns a bottom window
// W = H(kwtop:kbot, kwtop:kbot) of order nw <= SMALL_Z_MAX and its spike
// s = H(kwtop, kwtop-1):
//   1. real Schur form W = V T V^T in LDS (the small Francis iteration);
//   2. from the bottom of T, a diagonal block whose spike entries s V(0, .)
//      are negligible next to it is deflated; a block that is not is moved
//      to the top of the unchecked part by orthogonal swaps of adjacent
//      diagonal blocks (direct swapping: a Sylvester equation for the
//      invariant subspace, then its QR factor);
//   3. the spike of the undeflated part is reflected onto its first entry
//      and the undeflated part is brought back to Hessenberg form;
//   4. T goes back into H, V^T into a panel slot; the caller applies V to
//      the rows right of the window, the rows above it and to Q.
// The eigenvalues of the undeflated blocks are the next sweep's shifts.
// ============================================================================

// 64-lane sums and maxima (all lanes receive the result)
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Solve M x = b (N <= 4) by Givens QR; a diagonal entry of R below smin in
// magnitude is replaced by +-smin.  b is overwritten by x.
template <int N>
__device__ inline void tiny_solve(double (&M)[N][N], double (&b)[N], double smin) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const double a = M[j][j], c = M[i][j];
      const double r = hypot(a, c);
      const double cs = (r == 0.0) ? 1.0 : a / r;
      const double sn = (r == 0.0) ? 0.0 : c / r;
#pragma unroll
      for (int k = j; k < N; ++k) {
        const double x = M[j][k], y = M[i][k];
        M[j][k] = cs * x + sn * y;
        M[i][k] = cs * y - sn * x;
      }
      const double x = b[j], y = b[i];
      b[j] = cs * x + sn * y;
      b[i] = cs * y - sn * x;
    }
  }
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    double acc = b[j];
#pragma unroll
    for (int k = j + 1; k < N; ++k) acc -= M[j][k] * b[k];
    double d = M[j][j];
    if (fabs(d) < smin) d = (d < 0.0) ? -smin : smin;
    b[j] = acc / d;
  }
}

// Householder reflectors of one swap: reflector h is I - tau[h] v[h] v[h]^T
// on rows/columns k .. k+N-1 (v[h][i] = 0 for i < h, v[h][h] = 1).
struct SwapPlan {
  double v[2][4];
  double tau[2];
};

// Plan the swap of the adjacent diagonal blocks A (P x P, at k) and
// B (R x R, at k + P) of the quasi-triangular T (LDS, leading dimension LD).
// With A X - X B = -C (C the coupling block) the columns of [X; I] span the
// invariant subspace of B; the orthogonal factor of their QR factorisation
// moves B to the top.  Returns false when the transformed block fails the
// backward-stability test (the swap is then not done).
template <int P, int R>
__device__ bool plan_swap(const double* S, int LD, int k, SwapPlan& pl) {
  constexpr int N = P + R;
  constexpr int M = P * R;
  double T[N][N];
  double dnorm = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T[i][j] = (i <= j + 1) ? S[(k + i) + (k + j) * LD] : 0.0;
      dnorm = fmax(dnorm, fabs(T[i][j]));
    }
  const double tiny = 2.2250738585072014e-308;
  const double smin = fmax(kUlp * dnorm, tiny);
  // Kronecker form of A X - X B = -C, unknown x[i + P j] = X(i, j)
  double K[M][M], x[M];
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int i = 0; i < P; ++i) {
#pragma unroll
      for (int jj = 0; jj < R; ++jj)
#pragma unroll
        for (int ii = 0; ii < P; ++ii)
          K[i + P * j][ii + P * jj] = (jj == j ? T[i][ii] : 0.0) - (ii == i ? T[P + jj][P + j] : 0.0);
      x[i + P * j] = -T[i][P + j];
    }
  tiny_solve<M>(K, x, smin);
  // W = [X; I] (N x R), QR by R Householder reflectors
  double W[N][R];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) W[i][j] = (i < P) ? x[i + P * j] : (i - P == j ? 1.0 : 0.0);
#pragma unroll
  for (int h = 0; h < R; ++h) {
    double tail = 0.0;
#pragma unroll
    for (int i = h + 1; i < N; ++i) tail = fmax(tail, fabs(W[i][h]));
    const double alpha = W[h][h];
#pragma unroll
    for (int i = 0; i < 4; ++i) pl.v[h][i] = 0.0;
    pl.v[h][h] = 1.0;
    pl.tau[h] = 0.0;
    if (tail == 0.0 || !isfinite(tail) || !isfinite(alpha)) {
      if (!(tail == 0.0)) return false;
      continue;
    }
    const int e = ilogb(fmax(fabs(alpha), tail));
    double ss = 0.0;
#pragma unroll
    for (int i = h + 1; i < N; ++i) {
      const double t = ldexp(W[i][h], -e);
      ss += t * t;
    }
    const double as = ldexp(alpha, -e);
    const double nrm = sqrt(as * as + ss);
    const double bs = (as < 0.0) ? nrm : -nrm;
    const double ds = as - bs;
    const double r = 1.0 / (bs * ds);
    pl.tau[h] = -ds * (ds * r);
#pragma unroll
    for (int i = h + 1; i < N; ++i) pl.v[h][i] = ldexp(W[i][h], -e) * (bs * r);
    // apply to the remaining columns of W
#pragma unroll
    for (int j = h + 1; j < R; ++j) {
      double w = 0.0;
#pragma unroll
      for (int i = h; i < N; ++i) w += pl.v[h][i] * W[i][j];
#pragma unroll
      for (int i = h; i < N; ++i) W[i][j] -= pl.tau[h] * pl.v[h][i] * w;
    }
  }
  // T' = Q^T T Q with Q = H_0 H_1 ...; accept if its lower-left block is tiny
#pragma unroll
  for (int h = 0; h < R; ++h) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double w = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) w += pl.v[h][i] * T[i][j];
#pragma unroll
      for (int i = 0; i < N; ++i) T[i][j] -= pl.tau[h] * pl.v[h][i] * w;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double w = 0.0;
#pragma unroll
      for (int j = 0; j < N; ++j) w += T[i][j] * pl.v[h][j];
#pragma unroll
      for (int j = 0; j < N; ++j) T[i][j] -= pl.tau[h] * w * pl.v[h][j];
    }
  }
  double low = 0.0;
#pragma unroll
  for (int i = R; i < N; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) low = fmax(low, fabs(T[i][j]));
  const double thresh = fmax(20.0 * kUlp * dnorm, tiny);
  return low <= thresh;   // false for NaN as well
}

// Rotate rows/columns i, i+1 of the m x m quasi-triangular S (and columns of
// Z) so that the 2x2 block at i is in standard form.  Returns whether the
// block stayed a complex pair.
__device__ bool aed_std_block(double* S, double* Zs, int LD, int m, int i) {
  const int lane = threadIdx.x;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };
  const Std2 o = standardize2(Sx(i, i), Sx(i, i + 1), Sx(i + 1, i), Sx(i + 1, i + 1));
  __syncthreads();
  if (!(o.cs == 1.0 && o.sn == 0.0)) {
    for (int c = i + 2 + lane; c < m; c += 64) {
      const double x = Sx(i, c), y = Sx(i + 1, c);
      Sx(i, c) = o.cs * x + o.sn * y;
      Sx(i + 1, c) = o.cs * y - o.sn * x;
    }
    for (int r = lane; r < i; r += 64) {
      const double x = Sx(r, i), y = Sx(r, i + 1);
      Sx(r, i) = o.cs * x + o.sn * y;
      Sx(r, i + 1) = o.cs * y - o.sn * x;
    }
    for (int r = lane; r < m; r += 64) {
      const double x = Zx(r, i), y = Zx(r, i + 1);
      Zx(r, i) = o.cs * x + o.sn * y;
      Zx(r, i + 1) = o.cs * y - o.sn * x;
    }
  }
  if (lane == 0) {
    Sx(i, i) = o.a; Sx(i, i + 1) = o.b;
    Sx(i + 1, i) = o.c; Sx(i + 1, i + 1) = o.d;
  }
  __syncthreads();
  return o.c != 0.0;
}

// Swap the adjacent diagonal blocks of orders p (at k) and r (at k + p) of
// the m x m quasi-triangular S, updating the columns of Z.  Returns 0 when
// done, 1 when the swap was rejected (nothing changed), 2 when the moved
// block (now at k) split into two real eigenvalues.
__device__ int aed_swap(double* S, double* Zs, int LD, int m, int k, int p, int r,
                        SwapPlan* plds) {
  const int lane = threadIdx.x;
  auto Sx = [&](int rr, int c) -> double& { return S[rr + c * LD]; };
  __shared__ int ok_lds;
  __shared__ double dA, dB;
  if (lane == 0) {
    SwapPlan pl;
    bool ok;
    if (p == 1 && r == 1) ok = plan_swap<1, 1>(S, LD, k, pl);
    else if (p == 1) ok = plan_swap<1, 2>(S, LD, k, pl);
    else if (r == 1) ok = plan_swap<2, 1>(S, LD, k, pl);
    else ok = plan_swap<2, 2>(S, LD, k, pl);
    *plds = pl;
    ok_lds = ok ? 1 : 0;
    dA = Sx(k, k);           // the 1x1 eigenvalues are restored exactly
    dB = Sx(k + p + r - 1, k + p + r - 1);
  }
  __syncthreads();
  if (!ok_lds) return 1;
  const int N = p + r;
  // left: rows k .. k+N-1, columns k .. m-1
  for (int c = k + lane; c < m; c += 64) {
    double a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = (i < N) ? Sx(k + i, c) : 0.0;
    for (int h = 0; h < r; ++h) {
      double w = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) w += plds->v[h][i] * a[i];
      w *= plds->tau[h];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] -= plds->v[h][i] * w;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < N) Sx(k + i, c) = a[i];
  }
  __syncthreads();
  // right: columns k .. k+N-1 of rows 0 .. k+N-1 of S and all rows of Z
  for (int q = lane; q < m + k + N; q += 64) {
    const bool inS = q < k + N;
    double* base = inS ? S : Zs;
    const int row = inS ? q : q - (k + N);
    double a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = (i < N) ? base[row + (k + i) * LD] : 0.0;
    for (int h = 0; h < r; ++h) {
      double w = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) w += a[i] * plds->v[h][i];
      w *= plds->tau[h];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] -= w * plds->v[h][i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < N) base[row + (k + i) * LD] = a[i];
  }
  __syncthreads();
  if (lane == 0) {
    for (int i = r; i < N; ++i)
      for (int j = 0; j < r; ++j) Sx(k + i, k + j) = 0.0;
    if (r == 1) Sx(k, k) = dB;
    if (p == 1) Sx(k + r, k + r) = dA;
  }
  __syncthreads();
  int ret = 0;
  if (r == 2 && !aed_std_block(S, Zs, LD, m, k)) ret = 2;
  if (p == 2) (void)aed_std_block(S, Zs, LD, m, k + r);
  return ret;
}

// Householder reflector from a column held one entry per lane-slot:
// x0 = alpha (scalar), tail entries x[i] for i in [1, L) at LDS vv[i].
// On return vv[0] = 1, vv[1..L) = v, and the function yields (tau, beta).
// tau = 0 (identity) when the tail is zero.
__device__ void aed_reflector(double alpha, double* vv, int L, double& tau, double& beta) {
  const int lane = threadIdx.x;
  double tmax = 0.0;
  for (int i = 1 + lane; i < L; i += 64) tmax = fmax(tmax, fabs(vv[i]));
  tmax = wave_max(tmax);
  if (tmax == 0.0) {
    tau = 0.0;
    beta = alpha;
    __syncthreads();
    if (lane == 0) vv[0] = 1.0;
    __syncthreads();
    return;
  }
  const int e = ilogb(fmax(fabs(alpha), tmax));
  double ss = 0.0;
  for (int i = 1 + lane; i < L; i += 64) {
    const double t = ldexp(vv[i], -e);
    ss += t * t;
  }
  ss = wave_sum(ss);
  const double as = ldexp(alpha, -e);
  const double nrm = sqrt(as * as + ss);
  const double bs = (as < 0.0) ? nrm : -nrm;
  const double ds = as - bs;
  const double r = 1.0 / (bs * ds);
  tau = -ds * (ds * r);
  beta = ldexp(bs, e);
  const double f = bs * r;
  __syncthreads();
  for (int i = 1 + lane; i < L; i += 64) vv[i] = ldexp(vv[i], -e) * f;
  if (lane == 0) vv[0] = 1.0;
  __syncthreads();
}

template <int MAXM>
__global__ __launch_bounds__(64) void k_aed(AedTask t0, const AedTask* tasks) {
  const AedTask T = tasks ? tasks[blockIdx.x] : t0;
  constexpr int LD = SmallSmem<MAXM>::LD;
  __shared__ double S[LD * MAXM];
  __shared__ double Z[LD * MAXM];
  __shared__ double vv[MAXM];
  __shared__ SwapPlan plan;
  const int lane = threadIdx.x;
  const int nw = T.nw;
  const int kwtop = T.kbot - nw + 1;
  if (nw < 1 || nw > MAXM || kwtop < T.ktop) return;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Z[r + c * LD]; };
  double* Hw = T.H + kwtop + (size_t)kwtop * T.ldh;
  const double s = (kwtop > T.ktop) ? T.H[kwtop + (size_t)(kwtop - 1) * T.ldh] : 0.0;

  SmallTask st{};
  st.A = Hw; st.lda = T.ldh; st.m = nw; st.itmax = T.itmax;
  small_load<true, MAXM>(st, S, Z);
  const int info = small_iter<true, MAXM>(st, S, Z);
  if (info != 0) {   // window not in Schur form: no deflation, no shifts
    if (lane == 0) { T.ctrl->aed_nd = 0; T.ctrl->aed_nu = 0; }
    return;
  }

  // ---- deflation checks from the bottom, undeflatable blocks moved up
  const double tiny = 2.2250738585072014e-308;
  const double smlnum = tiny * ((double)nw / kUlp);
  int bot = nw - 1, ilst = 0;
  bool stop = false;
  while (!stop && ilst <= bot) {
    const int bs = (bot > ilst && Sx(bot, bot - 1) != 0.0) ? 2 : 1;
    double foo, spk;
    if (bs == 1) {
      foo = fabs(Sx(bot, bot));
      spk = fabs(s * Zx(0, bot));
    } else {
      foo = fabs(Sx(bot, bot)) + sqrt(fabs(Sx(bot, bot - 1))) * sqrt(fabs(Sx(bot - 1, bot)));
      spk = fmax(fabs(s * Zx(0, bot)), fabs(s * Zx(0, bot - 1)));
    }
    if (foo == 0.0) foo = fabs(s);
    __syncthreads();
    if (spk <= fmax(smlnum, kUlp * foo)) {
      bot -= bs;
      continue;
    }
    int pos = bot - bs + 1;
    while (pos > ilst) {
      const int above = (pos - 2 >= ilst && Sx(pos - 1, pos - 2) != 0.0) ? 2 : 1;
      __syncthreads();
      const int k = pos - above;
      if (aed_swap(S, Z, LD, nw, k, above, bs, &plan) != 0) { stop = true; break; }
      pos = k;
    }
    if (!stop) ilst += bs;
  }
  const int nu = bot + 1;
  const int nd = nw - nu;

  // ---- eigenvalues: undeflated blocks give the next shifts, deflated ones
  // are final (written when the caller asks for them)
  for (int e = lane; e < nw; e += 64) {
    const bool first = (e + 1 < nw) && Sx(e + 1, e) != 0.0;
    const bool second = (e >= 1) && Sx(e, e - 1) != 0.0;
    double wr = Sx(e, e), wi = 0.0;
    if (first) wi = sqrt(fabs(Sx(e, e + 1))) * sqrt(fabs(Sx(e + 1, e)));
    if (second) wi = -sqrt(fabs(Sx(e - 1, e))) * sqrt(fabs(Sx(e, e - 1)));
    if (e < nu) {
      T.sr[e] = wr;
      T.si[e] = wi;
    } else if (T.wr) {
      T.wr[e] = wr;
      T.wi[e] = wi;
    }
  }
  if (lane == 0) { T.ctrl->aed_nd = nd; T.ctrl->aed_nu = nu; }
  if (nd == 0) return;   // nothing deflated: H stays as it was

  // ---- reflect the spike of the undeflated part onto its first entry
  double spike = 0.0;
  if (nu == 1) {
    spike = s * Zx(0, 0);
  } else if (nu > 1) {
    for (int i = lane; i < nu; i += 64) vv[i] = s * Zx(0, i);
    __syncthreads();
    const double alpha = vv[0];
    double tau, beta;
    aed_reflector(alpha, vv, nu, tau, beta);
    spike = beta;
    if (tau != 0.0) {
      for (int c = lane; c < nw; c += 64) {          // rows 0..nu-1, all columns
        double w = 0.0;
        for (int i = 0; i < nu; ++i) w += vv[i] * Sx(i, c);
        w *= tau;
        for (int i = 0; i < nu; ++i) Sx(i, c) -= vv[i] * w;
      }
      __syncthreads();
      for (int q = lane; q < nu + nw; q += 64) {     // columns 0..nu-1 of S rows < nu, and of Z
        double* base = (q < nu) ? S : Z;
        const int row = (q < nu) ? q : q - nu;
        double w = 0.0;
        for (int j = 0; j < nu; ++j) w += base[row + j * LD] * vv[j];
        w *= tau;
        for (int j = 0; j < nu; ++j) base[row + j * LD] -= w * vv[j];
      }
      __syncthreads();
    }
    // ---- Hessenberg form of the undeflated part
    for (int j = 0; j + 2 < nu; ++j) {
      const int L = nu - j - 1;                       // rows j+1 .. nu-1
      const double a0 = Sx(j + 1, j);
      for (int i = 1 + lane; i < L; i += 64) vv[i] = Sx(j + 1 + i, j);
      __syncthreads();
      double tj, bj;
      aed_reflector(a0, vv, L, tj, bj);
      if (tj == 0.0) continue;
      if (lane == 0) Sx(j + 1, j) = bj;
      for (int i = 2 + lane; i <= L; i += 64) Sx(j + i, j) = 0.0;
      for (int c = j + 1 + lane; c < nw; c += 64) {  // left: rows j+1..nu-1
        double w = 0.0;
        for (int i = 0; i < L; ++i) w += vv[i] * Sx(j + 1 + i, c);
        w *= tj;
        for (int i = 0; i < L; ++i) Sx(j + 1 + i, c) -= vv[i] * w;
      }
      __syncthreads();
      for (int q = lane; q < nu + nw; q += 64) {     // right: columns j+1..nu-1
        double* base = (q < nu) ? S : Z;
        const int row = (q < nu) ? q : q - nu;
        double w = 0.0;
        for (int i = 0; i < L; ++i) w += base[row + (j + 1 + i) * LD] * vv[i];
        w *= tj;
        for (int i = 0; i < L; ++i) base[row + (j + 1 + i) * LD] -= w * vv[i];
      }
      __syncthreads();
    }
  }

  // ---- write back: the window, its spike, and V^T into the panel slot
  for (int c = 0; c < nw; ++c)
    for (int r = lane; r <= c + 1 && r < nw; r += 64) Hw[r + (size_t)c * T.ldh] = Sx(r, c);
  if (lane == 0 && kwtop > T.ktop) T.H[kwtop + (size_t)(kwtop - 1) * T.ldh] = spike;
  for (int c = 0; c < T.ldut; ++c)
    for (int r = lane; r < T.ldut; r += 64)
      T.Ut[r + (size_t)c * T.ldut] = (r < nw && c < nw) ? Zx(c, r) : 0.0;
}

// ============================================================================
// Shift preparation: sort the trailing-block eigenvalues by decreasing
// modulus (conjugate pairs stay together), pair the real ones, and emit one
// (sum, product) pair per bulge.  Missing pairs (if the small solve did not
// converge) are filled with ad-hoc shifts from the bottom of the block.
// ============================================================================
__device__ void shift_prep(const double* wr, const double* wi, int ns, const int* small_info,
                           int exceptional, const double* H, int ldh, int ktop, int kbot,
                           double* st) {
  __shared__ double key[512];
  __shared__ int kind[512];   // 0 real, 1 first of a conjugate pair, 2 second (skipped)
  __shared__ int rank[512];
  __shared__ int order[512];
  const int tid = threadIdx.x;
  const int npair = ns / 2;
  int valid0 = 0;  // eigenvalues [valid0, ns) converged
  if (!exceptional && small_info) {
    const int inf = *small_info;
    valid0 = inf;  // 1-based end of the failed block -> entries >= inf are valid
  }
  if (exceptional) valid0 = ns;
  for (int e = tid; e < ns; e += blockDim.x) {
    const bool ok = e >= valid0;
    key[e] = ok ? hypot(wr[e], wi[e]) : -1.0;
    int kd = 0;
    if (ok && wi[e] > 0.0) kd = 1;
    else if (ok && wi[e] < 0.0) kd = 2;
    else if (!ok) kd = 3;
    kind[e] = kd;
  }
  __syncthreads();
  // rank of each unit (real or first-of-pair) by decreasing modulus, stable
  for (int e = tid; e < ns; e += blockDim.x) {
    int rk = 0;
    if (kind[e] <= 1) {
      for (int f = 0; f < ns; ++f) {
        if (kind[f] > 1) continue;
        if (key[f] > key[e] || (key[f] == key[e] && f < e)) ++rk;
      }
      rank[e] = rk;
    } else {
      rank[e] = -1;
    }
  }
  __syncthreads();
  for (int e = tid; e < ns; e += blockDim.x)
    if (rank[e] >= 0) order[rank[e]] = e;
  __syncthreads();
  if (tid == 0) {
    int nunits = 0;
    for (int e = 0; e < ns; ++e) nunits += (rank[e] >= 0);
    int np = 0;
    int pend = -1;
    for (int u = 0; u < nunits && np < npair; ++u) {
      const int e = order[u];
      if (kind[e] == 1) {
        st[2 * np] = 2.0 * wr[e];
        st[2 * np + 1] = wr[e] * wr[e] + wi[e] * wi[e];
        ++np;
      } else if (pend < 0) {
        pend = e;
      } else {
        st[2 * np] = wr[pend] + wr[e];
        st[2 * np + 1] = wr[pend] * wr[e];
        ++np;
        pend = -1;
      }
    }
    // fill: ad-hoc pairs from 2x2 windows at the bottom of the block
    int row = kbot;
    while (np < npair) {
      if (row - 2 < ktop) row = kbot;
      const double w = fabs(H[row + (size_t)(row - 1) * ldh]) +
                       fabs(H[(row - 1) + (size_t)(row - 2) * ldh]);
      const double e = H[row + (size_t)row * ldh] + 0.75 * w;
      st[2 * np] = e + e;
      st[2 * np + 1] = e * e + 0.4375 * w * w;
      ++np;
      row -= 2;
    }
  }
}

__global__ __launch_bounds__(256) void k_shift_prep(const double* wr, const double* wi, int ns,
                                                    const int* small_info, int exceptional,
                                                    const double* H, int ldh, int ktop, int kbot,
                                                    double* st) {
  shift_prep(wr, wi, ns, small_info, exceptional, H, ldh, ktop, kbot, st);
}

__global__ __launch_bounds__(256) void k_shift_prep_b(const ShiftB* tasks) {
  const ShiftB T = tasks[blockIdx.x];
  shift_prep(T.wr, T.wi, T.ns, T.info, T.exceptional, T.H, T.ldh, T.ktop, T.kbot, T.st);
}

// ============================================================================
// Window chase (the window task).  One workgroup per diagonal window.
//
// Thread layout: 1024 threads; group b (TPB = 64 or 32 consecutive threads,
// inside one wavefront) owns bulge b of the window's chain.  One chain step
// advances every bulge by one row:
//   B  left update of rows K+1..K+3 from the bulge column to the window end;
//   C  right update of columns K+1..K+3 from the window top to row K+4;
//   A  the group forms bulge b's reflector for the next step from column
//      K+1, rows K+2..K+4, which only its own B and C of this step touched,
//      so no workgroup barrier is needed before it.  A bulge entering the
//      block takes its reflector from the shift pair after the barrier.
// Bulges sit three rows apart, so all left updates of a step precede all
// right updates (B, barrier, C, barrier).  Each thread issues all loads of
// a phase before its stores.  The reflectors are logged in LDS; after the
// window is written back, U is accumulated in the freed LDS with eight
// lanes of one wavefront per row (rows are independent).
// ============================================================================
constexpr int CHASE_THREADS = 1024;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ WinCtx ctx_of(const SweepArgs& a, const Win& w) {
  WinCtx c;
  c.H = a.H; c.Q = a.Q; c.U = a.U + (size_t)w.slot * UPAD * UPAD;
  c.st = a.st + 2 * w.shift0;
  c.ldh = a.ldh; c.ldq = a.ldq; c.n = a.n;
  c.ktop = a.ktop; c.kbot = a.kbot; c.rtop = a.rtop; c.cend = a.cend;
  c.p = w.p; c.ws = w.ws; c.tau0 = w.tau0; c.tau1 = w.tau1; c.nb = w.nb;
  return c;
}

__device__ void chase_window(const WinCtx& d) {
  __shared__ double W[LDW * WMAX];
  __shared__ double R[REFL_LDS * 3];
  const int tid = threadIdx.x;
  const int p = d.p, ws = d.ws, nb = d.nb;
  const int ktop = d.ktop, kbot = d.kbot;
  const WinCtx& a = d;   // matrix fields
  auto Wx = [&](int r, int c) -> double& { return W[r + c * LDW]; };

  // load the window: 8 columns per pass, all loads issued before the stores
  {
    const int r = tid & 127, c0 = tid >> 7;
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = c0 + 8 * q;
      v[q] = (r < ws && c < ws) ? a.H[(size_t)(p + r) + (size_t)(p + c) * a.ldh] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = c0 + 8 * q;
      if (r < ws && c < ws) Wx(r, c) = v[q];
    }
  }
  const int lgt = (nb <= 16) ? 6 : 5;
  const int tpb = 1 << lgt;
  const int b = tid >> lgt;
  const int t = tid & (tpb - 1);
  const bool mine = b < nb;
  const double s_sum = mine ? d.st[2 * b] : 0.0;
  const double s_prod = mine ? d.st[2 * b + 1] : 0.0;
  __syncthreads();

  // reflector of bulge b at chain step tau (reads column K, or the shifts)
  auto form = [&](int tau, int& K, int& nr, bool& act, Refl& h) {
    K = ktop - 1 + tau - 3 * b;
    act = mine && K >= ktop - 1 && K <= kbot - 2;
    nr = (K <= kbot - 3) ? 3 : 2;
    h = Refl{0.0, 0.0, 0.0, 0.0};
    if (act) {
      double x, y, z;
      if (K == ktop - 1) {
        const int o = ktop - p;
        first_column(Wx(o, o), Wx(o, o + 1), Wx(o + 1, o), Wx(o + 1, o + 1),
                     (nr == 3) ? Wx(o + 2, o + 1) : 0.0, s_sum, s_prod, x, y, z);
      } else {
        const int k = K - p;
        x = Wx(k + 1, k);
        y = Wx(k + 2, k);
        z = (nr == 3) ? Wx(k + 3, k) : 0.0;
      }
      h = make_reflector(nr, x, y, z);
      if (h.tau == 0.0) act = false;
    }
  };

  int K, nr;
  bool act;
  Refl h;
  form(d.tau0, K, nr, act, h);
  for (int tau = d.tau0; tau < d.tau1; ++tau) {
    if (K == ktop - 1) form(tau, K, nr, act, h);   // entering bulge: after the barrier
    const int k = K - p;
    if (mine && t == 0) {
      double* rr = &R[3 * ((tau - d.tau0) * nb + b)];
      rr[0] = h.v2;
      rr[1] = (nr == 3) ? h.v3 : 0.0;
      rr[2] = act ? h.tau : 0.0;
    }
    // ---- B: left update (at most 2 columns per thread with TPB = 64)
    if (act) {
      const int c0 = (k < 0) ? 0 : k;
      double x1[4], x2[4], x3[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = c0 + t + q * tpb;
        if (c < ws && c != k) {
          const double* col = &Wx(k + 1, c);
          x1[q] = col[0]; x2[q] = col[1]; x3[q] = (nr == 3) ? col[2] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = c0 + t + q * tpb;
        if (c >= ws) continue;
        if (c == k) {
          Wx(k + 1, k) = h.beta;
          Wx(k + 2, k) = 0.0;
          if (nr == 3) Wx(k + 3, k) = 0.0;
          continue;
        }
        const double w = h.tau * (x1[q] + h.v2 * x2[q] + h.v3 * x3[q]);
        double* col = &Wx(k + 1, c);
        col[0] = x1[q] - w;
        col[1] = x2[q] - w * h.v2;
        if (nr == 3) col[2] = x3[q] - w * h.v3;
      }
    }
    __syncthreads();
    // ---- C: right update, then the next reflector of this bulge
    if (act) {
      const int rl = ((K + 4 < kbot) ? K + 4 : kbot) - p;
      double y1[2], y2[2], y3[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int r = t + q * tpb;
        if (r <= rl) {
          y1[q] = Wx(r, k + 1); y2[q] = Wx(r, k + 2); y3[q] = (nr == 3) ? Wx(r, k + 3) : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int r = t + q * tpb;
        if (r > rl) continue;
        const double w = h.tau * (y1[q] + h.v2 * y2[q] + h.v3 * y3[q]);
        Wx(r, k + 1) = y1[q] - w;
        Wx(r, k + 2) = y2[q] - w * h.v2;
        if (nr == 3) Wx(r, k + 3) = y3[q] - w * h.v3;
      }
      // rows beyond two per thread (TPB = 32 only)
      for (int r = t + 2 * tpb; r <= rl; r += tpb) {
        const double a1 = Wx(r, k + 1), a2 = Wx(r, k + 2);
        const double a3 = (nr == 3) ? Wx(r, k + 3) : 0.0;
        const double w = h.tau * (a1 + h.v2 * a2 + h.v3 * a3);
        Wx(r, k + 1) = a1 - w;
        Wx(r, k + 2) = a2 - w * h.v2;
        if (nr == 3) Wx(r, k + 3) = a3 - w * h.v3;
      }
    }
    wave_sync();
    if (tau + 1 < d.tau1 && K + 1 != ktop - 1) form(tau + 1, K, nr, act, h);
    else { K = ktop - 1 + tau + 1 - 3 * b; }
    __syncthreads();
  }

  // window back to HBM
  {
    const int r = tid & 127, c0 = tid >> 7;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = c0 + 8 * q;
      if (r < ws && c < ws) a.H[(size_t)(p + r) + (size_t)(p + c) * a.ldh] = Wx(r, c);
    }
  }
  __syncthreads();

  // ---- accumulate U = P_1 P_2 ... ; row r by lanes j = 0..7 of its wave,
  // lane j applying the reflectors of bulges j, j+8, j+16 of each chain step
  {
    const int r = tid >> 3, j = tid & 7;
    if (r < ws)
      for (int c = j; c < ws; c += 8) Wx(r, c) = (r == c) ? 1.0 : 0.0;
    wave_sync();
    for (int tau = d.tau0; tau < d.tau1; ++tau) {
      int klead = ktop - 1 + tau;
      if (klead > kbot - 2) klead = kbot - 2;
      const bool rowact = (r < ws) && (r <= klead + 3 - p);
      const double* rt = &R[3 * (tau - d.tau0) * nb];
      if (rowact) {
        double u1[3], u2[3], u3[3], tv[3], v2[3], v3[3];
        int kk[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const int bb = j + 8 * q;
          tv[q] = (bb < nb) ? rt[3 * bb + 2] : 0.0;
          if (tv[q] != 0.0) {
            v2[q] = rt[3 * bb];
            v3[q] = rt[3 * bb + 1];
            kk[q] = ktop - 1 + tau - 3 * bb - p;
            const double* row = &Wx(r, kk[q] + 1);
            u1[q] = row[0]; u2[q] = row[LDW]; u3[q] = row[2 * LDW];
          }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (tv[q] == 0.0) continue;
          const double w = tv[q] * (u1[q] + v2[q] * u2[q] + v3[q] * u3[q]);
          double* row = &Wx(r, kk[q] + 1);
          row[0] = u1[q] - w;
          row[LDW] = u2[q] - w * v2[q];
          row[2 * LDW] = u3[q] - w * v3[q];
        }
      }
      wave_sync();
    }
  }
  __syncthreads();
  // U^T (column-major, ld UPAD, zero padded) -> the slot read by the panel kernels
  double* Ut = d.U;
  {
    const int r = tid & 127, c0 = tid >> 7;
#pragma unroll
    for (int q = 0; q < 16; ++q) {   // Ut(r, c) = U(c, r)
      const int c = c0 + 8 * q;
      Ut[r + (size_t)c * UPAD] = (r < ws && c < ws) ? Wx(c, r) : 0.0;
    }
  }
}

__global__ __launch_bounds__(CHASE_THREADS) void k_chase(SweepArgs a) {
  chase_window(ctx_of(a, a.win[blockIdx.x]));
}

__global__ __launch_bounds__(CHASE_THREADS) void k_chase_b(const WinB* wins) {
  chase_window(wins[blockIdx.x].c);
}

// ============================================================================
// Panel updates with FP64 MFMA (v_mfma_f64_16x16x4f64).
// Fragment layout of the 16x16x4 FP64 MFMA (wave64), measured on gfx950:
//   A(i, k): lane = i + 16 k      B(k, j): lane = j + 16 k
//   D(i, j): lane = j + 16 (i % 4), element i / 4
// ============================================================================
constexpr int PT = GEMM_T;       // 64
constexpr int LDT = PT + 4;      // padded LDS leading dimension of panel tiles

__device__ __forceinline__ int find_window(const SweepArgs& a, int bid, bool row) {
  int w = 0;
  if (row) {
    while (w + 1 < a.nwin && a.win[w + 1].base_r <= bid) ++w;
  } else {
    while (w + 1 < a.nwin && a.win[w + 1].base_cq <= bid) ++w;
  }
  return w;
}

// last window whose prefix is <= bid (zero-tile windows share the next prefix)
__device__ __forceinline__ int find_window_b(const WinB* wins, int nwin, int bid, bool row) {
  int lo = 0, hi = nwin - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int base = row ? wins[mid].base_r : wins[mid].base_cq;
    if (base <= bid) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Y(ws x 64) = U^T X for one 64-column tile of a window's row panel, in place.
__device__ void panel_row_tile(const WinCtx& d, int tile) {
  __shared__ double Xs[WMAX * LDT];   // row-major tile: Xs[c + r*LDT]
  const int p = d.p, ws = d.ws;
  const int c0 = p + ws + tile * PT;
  const int nc = min(PT, d.cend - c0);
  const int kpad = (ws + 3) & ~3;
  const double* Ut = d.U;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = wave * 32;
  // this wave's A operands (rows i0..i0+31 of U^T, all k) go to registers
  // before the tile load so that their latency hides behind it; the slot is
  // zero padded to UPAD x UPAD, so the full K = UPAD is read
  double ua[UPAD / 4][2];
  if (i0 < ws) {
#pragma unroll
    for (int ks = 0; ks < UPAD / 4; ++ks) {
      const int k = 4 * ks + lk;
      ua[ks][0] = Ut[(i0 + li) + (size_t)k * UPAD];
      ua[ks][1] = Ut[(i0 + 16 + li) + (size_t)k * UPAD];
    }
  }

  for (int idx = tid; idx < kpad * PT; idx += 256) {
    const int c = idx / kpad, r = idx - c * kpad;
    double v = 0.0;
    if (r < ws && c < nc) v = d.H[(size_t)(p + r) + (size_t)(c0 + c) * d.ldh];
    Xs[c + r * LDT] = v;
  }
  __syncthreads();

  if (i0 >= ws) return;
  d4 acc[2][4];
  for (int ib = 0; ib < 2; ++ib)
    for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < UPAD / 4; ++ks) {
    if (4 * ks >= kpad) break;
    const int k = 4 * ks + lk;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      const double b = Xs[(jb * 16 + li) + k * LDT];
      acc[0][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[ks][0], b, acc[0][jb], 0, 0, 0);
      acc[1][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[ks][1], b, acc[1][jb], 0, 0, 0);
    }
  }
  for (int ib = 0; ib < 2; ++ib)
    for (int jb = 0; jb < 4; ++jb) {
      const int col = jb * 16 + li;
      if (col >= nc) continue;
      for (int e = 0; e < 4; ++e) {
        const int row = i0 + ib * 16 + lk + 4 * e;
        if (row < ws) d.H[(size_t)(p + row) + (size_t)(c0 + col) * d.ldh] = acc[ib][jb][e];
      }
    }
}

// Y(64 x ws) = X U for one 64-row tile of a window's column panel (tile <
// tiles_c) or of Q (the remaining tiles).
__device__ void panel_colq_tile(const WinCtx& d, int tile, int tiles_c) {
  __shared__ double Xs[WMAX * LDT];   // column-major tile: Xs[r + c*LDT]
  const int p = d.p, ws = d.ws;
  double* M;
  int ld, r0, rend;
  if (tile < tiles_c) {
    M = d.H; ld = d.ldh; r0 = d.rtop + tile * PT; rend = p;
  } else {
    tile -= tiles_c;
    M = d.Q; ld = d.ldq; r0 = tile * PT; rend = d.n;
  }
  const int nr = min(PT, rend - r0);
  const int kpad = (ws + 3) & ~3;
  const double* Ut = d.U;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int j0 = wave * 32;
  // this wave's B operands (columns j0..j0+31 of U, all k) go to registers
  // before the tile load (zero-padded slot, full K = UPAD)
  double ub[UPAD / 4][2];
  if (j0 < ws) {
#pragma unroll
    for (int ks = 0; ks < UPAD / 4; ++ks) {
      const int k = 4 * ks + lk;
      ub[ks][0] = Ut[(j0 + li) + (size_t)k * UPAD];
      ub[ks][1] = Ut[(j0 + 16 + li) + (size_t)k * UPAD];
    }
  }

  for (int idx = tid; idx < kpad * PT; idx += 256) {
    const int c = idx / PT, r = idx - c * PT;
    double v = 0.0;
    if (r < nr && c < ws) v = M[(size_t)(r0 + r) + (size_t)(p + c) * ld];
    Xs[r + c * LDT] = v;
  }
  __syncthreads();

  if (j0 >= ws) return;
  d4 acc[4][2];
  for (int ib = 0; ib < 4; ++ib)
    for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < UPAD / 4; ++ks) {
    if (4 * ks >= kpad) break;
    const int k = 4 * ks + lk;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
      const double av = Xs[(ib * 16 + li) + k * LDT];
      acc[ib][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, ub[ks][0], acc[ib][0], 0, 0, 0);
      acc[ib][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, ub[ks][1], acc[ib][1], 0, 0, 0);
    }
  }
  for (int ib = 0; ib < 4; ++ib)
    for (int jb = 0; jb < 2; ++jb) {
      const int col = j0 + jb * 16 + li;
      if (col >= ws) continue;
      for (int e = 0; e < 4; ++e) {
        const int row = ib * 16 + lk + 4 * e;
        if (row < nr) M[(size_t)(r0 + row) + (size_t)(p + col) * ld] = acc[ib][jb][e];
      }
    }
}

__global__ __launch_bounds__(256, 2) void k_panel_row(SweepArgs a) {
  const int w = find_window(a, blockIdx.x, true);
  panel_row_tile(ctx_of(a, a.win[w]), blockIdx.x - a.win[w].base_r);
}

__global__ __launch_bounds__(256, 2) void k_panel_colq(SweepArgs a) {
  const int w = find_window(a, blockIdx.x, false);
  panel_colq_tile(ctx_of(a, a.win[w]), blockIdx.x - a.win[w].base_cq, a.win[w].tiles_c);
}

__global__ __launch_bounds__(256, 2) void k_panel_row_b(const WinB* wins, int nwin) {
  const int w = find_window_b(wins, nwin, blockIdx.x, true);
  panel_row_tile(wins[w].c, blockIdx.x - wins[w].base_r);
}

__global__ __launch_bounds__(256, 2) void k_panel_colq_b(const WinB* wins, int nwin) {
  const int w = find_window_b(wins, nwin, blockIdx.x, false);
  panel_colq_tile(wins[w].c, blockIdx.x - wins[w].base_cq, wins[w].tiles_c);
}

// ============================================================================
// Input check and clean-up: flag non-finite entries of the Hessenberg part,
// then (separate launch) zero everything below the first subdiagonal.
// ============================================================================
__global__ void k_check_finite(const double* H, int ldh, int n, Ctrl* ctrl) {
  const size_t total = (size_t)n * n;
  int bad = 0;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / n), r = (int)(idx - (size_t)c * n);
    if (r <= c + 1) {
      const double v = H[r + (size_t)c * ldh];
      if (!isfinite(v)) bad = 1;
    }
  }
  if (bad) atomicOr(&ctrl->bad, 1);
}

__global__ void k_zero_lower(double* H, int ldh, int n) {
  const size_t total = (size_t)n * n;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / n), r = (int)(idx - (size_t)c * n);
    if (r > c + 1) H[r + (size_t)c * ldh] = 0.0;
  }
}

__global__ void k_set_identity(double* Q, int ldq, int n) {
  const size_t total = (size_t)n * n;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(idx / n), r = (int)(idx - (size_t)c * n);
    Q[r + (size_t)c * ldq] = (r == c) ? 1.0 : 0.0;
  }
}

__global__ void k_ctrl_reset(Ctrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->bad = 0;
    ctrl->small_info = 0;
    ctrl->ndefl = 0;
  }
}

// ============================================================================
// Deflation scan of the bottom unreduced block (one workgroup).
// Negligible subdiagonal entries of rows 1..kbot are set to exactly zero;
// converged 1x1 / 2x2 blocks at the bottom are peeled off.
// ============================================================================
constexpr int DEFL_THREADS = 1024;
constexpr int DEFL_WORDS = 16384;   // bitmap words: n <= 524288

__global__ __launch_bounds__(DEFL_THREADS) void k_deflate(double* H, int ldh, int kbot, int klo,
                                                          Ctrl* ctrl) {
  __shared__ unsigned bits[DEFL_WORDS];
  const int tid = threadIdx.x;
  const int nwords = (kbot >> 5) + 1;
  for (int wv = tid; wv < nwords; wv += DEFL_THREADS) bits[wv] = 0u;
  __syncthreads();
  for (int k = klo + 1 + tid; k <= kbot; k += DEFL_THREADS) {
    const double sub = fabs(H[k + (size_t)(k - 1) * ldh]);
    double tst = fabs(H[(k - 1) + (size_t)(k - 1) * ldh]) + fabs(H[k + (size_t)k * ldh]);
    if (tst == 0.0) {
      tst = fabs(H[(k - 1) + (size_t)k * ldh]);
      if (k >= 2) tst += fabs(H[(k - 1) + (size_t)(k - 2) * ldh]);
      if (k + 1 <= kbot) tst += fabs(H[(k + 1) + (size_t)k * ldh]);
    }
    if (sub <= kUlp * tst) {
      if (sub != 0.0) H[k + (size_t)(k - 1) * ldh] = 0.0;
      atomicOr(&bits[k >> 5], 1u << (k & 31));
    }
  }
  __syncthreads();
  if (tid < 64) {
    const int lane = tid;
    int kb = kbot, kt = 0, peeled = 0;
    while (kb >= 0) {
      // largest flagged k <= kb (k >= klo+1), else klo
      kt = klo;
      const int wtop = kb >> 5;
      for (int wbase = wtop; wbase >= 0; wbase -= 64) {
        const int wv = wbase - lane;
        unsigned word = 0u;
        if (wv >= 0) {
          word = bits[wv];
          if (wv == wtop) {
            const int sh = kb & 31;
            word &= (sh == 31) ? 0xffffffffu : ((2u << sh) - 1u);
          }
        }
        const unsigned long long mask = __ballot(word != 0u);
        if (mask) {
          const int src = __builtin_ctzll(mask);
          const unsigned wsel = __shfl(word, src);
          const int wi = wbase - src;
          kt = wi * 32 + 31 - __builtin_clz(wsel);
          break;
        }
      }
      if (kt < klo) kt = klo;
      if (kb - kt + 1 <= 2) {
        peeled += kb - kt + 1;
        kb = kt - 1;
        if (kb < klo) { kb = klo - 1; break; }
        continue;
      }
      break;
    }
    if (lane == 0) {
      ctrl->kbot = kb;
      ctrl->ktop = (kb < klo) ? klo : kt;
      ctrl->ndefl = peeled;
    }
  }
}

// ============================================================================
// Batched deflation scan: one workgroup per matrix.  Negligible subdiagonal
// entries of rows 1..kbot are set to zero; converged 1x1 and 2x2 blocks at
// the bottom are peeled off at once: (wr, wi) are written, and each 2x2
// block is standardised with its rotation applied to the rest of H and to Q.
// ============================================================================
constexpr int DB_WORDS = 2048;   // n <= 65536

__global__ __launch_bounds__(256) void k_deflate_b(const DeflB* tasks) {
  const DeflB T = tasks[blockIdx.x];
  __shared__ unsigned bits[DB_WORDS];
  __shared__ int s_kt;
  const int tid = threadIdx.x;
  double* H = T.H;
  const int ldh = T.ldh, n = T.n;
  int kbot = T.kbot;
  if (kbot < 0) {
    if (tid == 0) { T.out->kbot = -1; T.out->ktop = 0; }
    return;
  }
  for (int wv = tid; wv <= (kbot >> 5); wv += 256) bits[wv] = 0u;
  __syncthreads();
  for (int k = 1 + tid; k <= kbot; k += 256) {
    const double sub = fabs(H[k + (size_t)(k - 1) * ldh]);
    double tst = fabs(H[(k - 1) + (size_t)(k - 1) * ldh]) + fabs(H[k + (size_t)k * ldh]);
    if (tst == 0.0) {
      tst = fabs(H[(k - 1) + (size_t)k * ldh]);
      if (k >= 2) tst += fabs(H[(k - 1) + (size_t)(k - 2) * ldh]);
      if (k + 1 <= kbot) tst += fabs(H[(k + 1) + (size_t)k * ldh]);
    }
    if (sub <= kUlp * tst) {
      if (sub != 0.0) H[k + (size_t)(k - 1) * ldh] = 0.0;
      atomicOr(&bits[k >> 5], 1u << (k & 31));
    }
  }
  __syncthreads();
  int kt = 0;
  while (kbot >= 0) {
    if (tid == 0) {
      int f = 0;
      for (int wv = kbot >> 5; wv >= 0; --wv) {
        unsigned word = bits[wv];
        if (wv == (kbot >> 5)) {
          const int sh = kbot & 31;
          word &= (sh == 31) ? 0xffffffffu : ((2u << sh) - 1u);
        }
        if (word) { f = wv * 32 + 31 - __builtin_clz(word); break; }
      }
      s_kt = f;
    }
    __syncthreads();
    kt = s_kt;
    const int m = kbot - kt + 1;
    if (m == 1) {
      if (tid == 0) { T.wr[kbot] = H[kbot + (size_t)kbot * ldh]; T.wi[kbot] = 0.0; }
      kbot -= 1;
    } else if (m == 2) {
      const int i = kbot;
      const Std2 o = standardize2(H[(i - 1) + (size_t)(i - 1) * ldh], H[(i - 1) + (size_t)i * ldh],
                                  H[i + (size_t)(i - 1) * ldh], H[i + (size_t)i * ldh]);
      if (!(o.cs == 1.0 && o.sn == 0.0)) {
        for (int c = i + 1 + tid; c < n; c += 256) {
          const double x = H[(i - 1) + (size_t)c * ldh], y = H[i + (size_t)c * ldh];
          H[(i - 1) + (size_t)c * ldh] = o.cs * x + o.sn * y;
          H[i + (size_t)c * ldh] = o.cs * y - o.sn * x;
        }
        for (int r = tid; r < i - 1; r += 256) {
          const double x = H[r + (size_t)(i - 1) * ldh], y = H[r + (size_t)i * ldh];
          H[r + (size_t)(i - 1) * ldh] = o.cs * x + o.sn * y;
          H[r + (size_t)i * ldh] = o.cs * y - o.sn * x;
        }
        if (T.Q) {
          for (int r = tid; r < n; r += 256) {
            const double x = T.Q[r + (size_t)(i - 1) * T.ldq], y = T.Q[r + (size_t)i * T.ldq];
            T.Q[r + (size_t)(i - 1) * T.ldq] = o.cs * x + o.sn * y;
            T.Q[r + (size_t)i * T.ldq] = o.cs * y - o.sn * x;
          }
        }
      }
      __syncthreads();
      if (tid == 0) {
        H[(i - 1) + (size_t)(i - 1) * ldh] = o.a; H[(i - 1) + (size_t)i * ldh] = o.b;
        H[i + (size_t)(i - 1) * ldh] = o.c;       H[i + (size_t)i * ldh] = o.d;
        T.wr[i - 1] = o.wr1; T.wi[i - 1] = o.wi1;
        T.wr[i] = o.wr2;     T.wi[i] = o.wi2;
      }
      kbot -= 2;
    } else {
      break;
    }
    __syncthreads();
  }
  if (tid == 0) {
    T.out->kbot = kbot;
    T.out->ktop = (kbot < 0) ? 0 : kt;
  }
}

// ============================================================================
// Final standardisation of the 2x2 blocks and eigenvalue extraction.
// Blocks are found as nonzero subdiagonal entries; each block's rotation is
// recomputed from its four (untouched) entries by every thread that needs it.
// Phase 1 rotates block rows (columns to the right), phase 2 block columns
// (rows above) and Q, phase 3 writes the standard blocks and (wr, wi).
// ============================================================================
__global__ void k_find_blocks(const double* H, int ldh, int n, int kmin, int* list, int* count,
                              int cap) {
  for (int k = kmin + blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    if (H[k + (size_t)(k - 1) * ldh] != 0.0) {
      const int pos = atomicAdd(count, 1);
      if (pos < cap) list[pos] = k;
    }
  }
}

__global__ void k_clamp_count(int* count, int cap) {
  if (threadIdx.x == 0 && *count > cap) *count = cap;
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

__global__ void k_std_rows(double* H, int ldh, int n, const int* list, const int* count) {
  const int nbk = *count;
  for (int e = blockIdx.x; e < nbk; e += gridDim.x) {
    const int k = list[e];
    const Std2 o = standardize2(H[(k - 1) + (size_t)(k - 1) * ldh], H[(k - 1) + (size_t)k * ldh],
                                H[k + (size_t)(k - 1) * ldh], H[k + (size_t)k * ldh]);
    if (o.cs == 1.0 && o.sn == 0.0) continue;
    for (int c = k + 1 + threadIdx.x; c < n; c += blockDim.x) {
      const double x = H[(k - 1) + (size_t)c * ldh], y = H[k + (size_t)c * ldh];
      H[(k - 1) + (size_t)c * ldh] = o.cs * x + o.sn * y;
      H[k + (size_t)c * ldh] = o.cs * y - o.sn * x;
    }
  }
}

__global__ void k_std_cols(double* H, int ldh, double* Q, int ldq, int n, const int* list,
                           const int* count) {
  const int nbk = *count;
  for (int e = blockIdx.x; e < nbk; e += gridDim.x) {
    const int k = list[e];
    const Std2 o = standardize2(H[(k - 1) + (size_t)(k - 1) * ldh], H[(k - 1) + (size_t)k * ldh],
                                H[k + (size_t)(k - 1) * ldh], H[k + (size_t)k * ldh]);
    if (o.cs == 1.0 && o.sn == 0.0) continue;
    for (int r = threadIdx.x; r < k - 1; r += blockDim.x) {
      const double x = H[r + (size_t)(k - 1) * ldh], y = H[r + (size_t)k * ldh];
      H[r + (size_t)(k - 1) * ldh] = o.cs * x + o.sn * y;
      H[r + (size_t)k * ldh] = o.cs * y - o.sn * x;
    }
    if (Q) {
      for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const double x = Q[r + (size_t)(k - 1) * ldq], y = Q[r + (size_t)k * ldq];
        Q[r + (size_t)(k - 1) * ldq] = o.cs * x + o.sn * y;
        Q[r + (size_t)k * ldq] = o.cs * y - o.sn * x;
      }
    }
  }
}

__global__ void k_std_finish(double* H, int ldh, int n, double* wr, double* wi) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const bool top = (k + 1 < n) && H[(k + 1) + (size_t)k * ldh] != 0.0;   // k is first of a block
    const bool bottom = (k >= 1) && H[k + (size_t)(k - 1) * ldh] != 0.0;   // k is second
    if (!top && !bottom) {
      wr[k] = H[k + (size_t)k * ldh];
      wi[k] = 0.0;
    }
  }
}

__global__ void k_std_blocks(double* H, int ldh, int n, const int* list, const int* count,
                             double* wr, double* wi) {
  const int nbk = *count;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nbk; e += gridDim.x * blockDim.x) {
    const int k = list[e];
    const Std2 o = standardize2(H[(k - 1) + (size_t)(k - 1) * ldh], H[(k - 1) + (size_t)k * ldh],
                                H[k + (size_t)(k - 1) * ldh], H[k + (size_t)k * ldh]);
    H[(k - 1) + (size_t)(k - 1) * ldh] = o.a;
    H[(k - 1) + (size_t)k * ldh] = o.b;
    H[k + (size_t)(k - 1) * ldh] = o.c;
    H[k + (size_t)k * ldh] = o.d;
    wr[k - 1] = o.wr1; wi[k - 1] = o.wi1;
    wr[k] = o.wr2;     wi[k] = o.wi2;
  }
}

// ============================================================================
// Host-side launch wrappers
// ============================================================================
void launch_small_z(const SmallTask& t, const SmallTask* tasks, int count, int maxm,
                    hipStream_t s) {
  if (maxm <= 32)
    hipLaunchKernelGGL((k_small_z<32>), dim3(count), dim3(64), 0, s, t, tasks);
  else if (maxm <= 64)
    hipLaunchKernelGGL((k_small_z<64>), dim3(count), dim3(64), 0, s, t, tasks);
  else
    hipLaunchKernelGGL((k_small_z<SMALL_Z_MAX>), dim3(count), dim3(64), 0, s, t, tasks);
}

void launch_small_eig(const SmallTask& t, hipStream_t s) {
  if (t.m <= 32)
    hipLaunchKernelGGL((k_small_eig<32>), dim3(1), dim3(64), 0, s, t, (const SmallTask*)nullptr);
  else if (t.m <= 64)
    hipLaunchKernelGGL((k_small_eig<64>), dim3(1), dim3(64), 0, s, t, (const SmallTask*)nullptr);
  else
    hipLaunchKernelGGL((k_small_eig<SMALL_EIG_MAX>), dim3(1), dim3(64), 0, s, t,
                       (const SmallTask*)nullptr);
}

void launch_aed(const AedTask& t, hipStream_t s) {
  hipLaunchKernelGGL((k_aed<SMALL_Z_MAX>), dim3(1), dim3(64), 0, s, t,
                     (const AedTask*)nullptr);
}

void launch_aed_b(const AedTask* tasks, int count, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL((k_aed<SMALL_Z_MAX>), dim3(count), dim3(64), 0, s, AedTask{}, tasks);
}

void launch_shift_prep(const double* wr, const double* wi, int ns, const int* small_info,
                       int exceptional, const double* H, int ldh, int ktop, int kbot, double* st,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_shift_prep, dim3(1), dim3(256), 0, s, wr, wi, ns, small_info, exceptional,
                     H, ldh, ktop, kbot, st);
}

void launch_chase(const SweepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_chase, dim3(a.nwin), dim3(CHASE_THREADS), 0, s, a);
}

void launch_panel_row(const SweepArgs& a, int tiles, hipStream_t s) {
  if (tiles > 0) hipLaunchKernelGGL(k_panel_row, dim3(tiles), dim3(256), 0, s, a);
}

void launch_panel_colq(const SweepArgs& a, int tiles, hipStream_t s) {
  if (tiles > 0) hipLaunchKernelGGL(k_panel_colq, dim3(tiles), dim3(256), 0, s, a);
}

void launch_small_tasks(const SmallTask* tasks, int count, int maxm, bool wantz, hipStream_t s) {
  if (count <= 0) return;
  SmallTask none{};
  if (wantz) {
    launch_small_z(none, tasks, count, maxm, s);
  } else if (maxm <= 32) {
    hipLaunchKernelGGL((k_small_eig<32>), dim3(count), dim3(64), 0, s, none, tasks);
  } else if (maxm <= 64) {
    hipLaunchKernelGGL((k_small_eig<64>), dim3(count), dim3(64), 0, s, none, tasks);
  } else {
    hipLaunchKernelGGL((k_small_eig<SMALL_EIG_MAX>), dim3(count), dim3(64), 0, s, none, tasks);
  }
}

void launch_chase_b(const WinB* wins, int nwin, hipStream_t s) {
  if (nwin > 0) hipLaunchKernelGGL(k_chase_b, dim3(nwin), dim3(CHASE_THREADS), 0, s, wins);
}

void launch_panel_row_b(const WinB* wins, int nwin, int tiles, hipStream_t s) {
  if (tiles > 0) hipLaunchKernelGGL(k_panel_row_b, dim3(tiles), dim3(256), 0, s, wins, nwin);
}

void launch_panel_colq_b(const WinB* wins, int nwin, int tiles, hipStream_t s) {
  if (tiles > 0) hipLaunchKernelGGL(k_panel_colq_b, dim3(tiles), dim3(256), 0, s, wins, nwin);
}

void launch_deflate_b(const DeflB* tasks, int count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_deflate_b, dim3(count), dim3(256), 0, s, tasks);
}

void launch_shift_prep_b(const ShiftB* tasks, int count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_shift_prep_b, dim3(count), dim3(256), 0, s, tasks);
}

void launch_check_finite(const double* H, int ldh, int n, Ctrl* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, s, H, ldh, n, ctrl);
}

void launch_zero_lower(double* H, int ldh, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_lower, dim3(2048), dim3(256), 0, s, H, ldh, n);
}

void launch_set_identity(double* Q, int ldq, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_set_identity, dim3(1024), dim3(256), 0, s, Q, ldq, n);
}

void launch_ctrl_reset(Ctrl* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, s, ctrl);
}

void launch_deflate(double* H, int ldh, int kbot, int klo, Ctrl* ctrl, hipStream_t s) {
  hipLaunchKernelGGL(k_deflate, dim3(1), dim3(DEFL_THREADS), 0, s, H, ldh, kbot, klo, ctrl);
}

void launch_standardize(double* H, int ldh, double* Q, int ldq, int n, int kmin, double* wr,
                        double* wi, int* list, int* count, int cap, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, count);
  if (kmin < 1) kmin = 1;
  hipLaunchKernelGGL(k_find_blocks, dim3(64), dim3(256), 0, s, H, ldh, n, kmin, list, count, cap);
  hipLaunchKernelGGL(k_clamp_count, dim3(1), dim3(64), 0, s, count, cap);
  hipLaunchKernelGGL(k_std_rows, dim3(1024), dim3(256), 0, s, H, ldh, n, list, count);
  hipLaunchKernelGGL(k_std_cols, dim3(1024), dim3(256), 0, s, H, ldh, Q, ldq, n, list, count);
  hipLaunchKernelGGL(k_std_finish, dim3(64), dim3(256), 0, s, H, ldh, n, wr, wi);
  hipLaunchKernelGGL(k_std_blocks, dim3(64), dim3(256), 0, s, H, ldh, n, list, count, wr, wi);
}

}  // namespace schur
