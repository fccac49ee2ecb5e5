// evec_kernels.hip -- eigenvectors of a real Schur form (paper Sec. 2,
// Eq. (5)) with protection against overflow, and their normalisation.
//
// All eigenvectors are computed together, tile row by tile row from the
// bottom of S (right-looking): for tile row t,
//   1. every eigenvector with entries in the tile solves the tile's rows of
//      (S - lambda I) y = 0 by back substitution inside the tile (one thread
//      per eigenvalue, the tile of S and the tile of Y in LDS), its pending
//      right-hand side already holding the contributions of every tile
//      below;
//   2. one FP64 MFMA product brings those contributions to every row above
//      the tile: Y(above, cols) -= S(above, tile) Y(tile, cols).
// Overflow protection follows the bound-tracking idea of robust triangular
// solvers: each eigenvector keeps an upper bound of its pending entries;
// before a division or an update could push an entry past a threshold the
// whole vector (all of its rows, wherever they are) is scaled down.  Since
// the vectors are normalised at the end, a scaling only has to be applied
// consistently to the whole vector.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "evec.h"

namespace schur {

namespace {

constexpr double EV_ULP = 2.220446049250313e-16;   // 2^-52
constexpr double EV_TINY = 2.2250738585072014e-308;
constexpr double EV_BIG = 0x1p960;                  // scaling threshold (~1e289)

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ double cabs1(cplx a) { return fabs(a.re) + fabs(a.im); }
// a / b (Smith's method: no intermediate overflow for finite results)
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.im + b.re * r;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
// a pivot of modulus at least smin (same direction when nonzero)
__device__ __forceinline__ cplx pivot(cplx d, double smin) {
  if (cabs1(d) >= smin) return d;
  const double m = hypot(d.re, d.im);
  if (m > 0.0) return {d.re * (smin / m), d.im * (smin / m)};
  return {smin, 0.0};
}

// Factor f <= 1 such that f (bound + c x) <= EV_BIG, evaluated without
// forming c x when that product could overflow (bound <= EV_BIG holds on
// entry); 1 when no scaling is needed.
__device__ __forceinline__ double guard(double bound, double c, double x) {
  if (c <= 0.0 || x <= (EV_BIG - bound) / c) return 1.0;
  return (EV_BIG / c) / (bound / c + x);
}

}  // namespace

// The eigenvalue owning column j and its block: kind 1 = real (block row p =
// j), 2 = first column of a complex pair (block rows j, j+1; lambda with
// positive imaginary part), 0 = second column of a pair (handled by j-1).
__device__ __forceinline__ int column_kind(const double* S, int lds, int n, int j) {
  if (j + 1 < n && S[(size_t)(j + 1) + (size_t)j * lds] != 0.0) return 2;
  if (j >= 1 && S[(size_t)j + (size_t)(j - 1) * lds] != 0.0) return 0;
  return 1;
}

// Tile row [r0, r1) of every eigenvector with columns in [c0, n): one
// thread per column, EVT columns per workgroup.
__global__ __launch_bounds__(EVT) void k_ev_diag(EvArgs g, int r0, int r1) {
  // S(r0:r1, r0:r1) and Y(r0:r1, c0 .. c0+EVT): the workgroup's columns
  // plus one, the imaginary part of a pair whose real part is its last
  constexpr int LS = EVTMAX + 1, LY = EVTMAX + 1;
  __shared__ double St[EVTMAX * LS];
  __shared__ double Yt[LY * (EVT + 1)];
  const int n = g.n;
  const int m = r1 - r0;
  const int c0 = r0 + blockIdx.x * EVT;   // first column of this workgroup
  const int tid = threadIdx.x;
  const int j = c0 + tid;
  for (int e = tid; e < m * m; e += EVT) {
    const int r = e % m, c = e / m;
    St[r + c * LS] = g.S[(size_t)(r0 + r) + (size_t)(r0 + c) * g.lds];
  }
  for (int e = tid; e < m * (EVT + 1); e += EVT) {
    const int r = e % m, c = e / m;
    const int jj = c0 + c;
    Yt[r + c * LY] = (jj < n) ? g.Y[(size_t)(r0 + r) + (size_t)jj * g.ldy] : 0.0;
  }
  __syncthreads();
  const int kind = (j < n) ? column_kind(g.S, g.lds, n, j) : 0;
  if (kind != 0) {
    const bool cx = kind == 2;
    const int p = j, s = cx ? 2 : 1;
    // lambda
    cplx lam = {g.S[(size_t)p + (size_t)p * g.lds], 0.0};
    double bq = 0.0, cq = 0.0;
    if (cx) {
      bq = g.S[(size_t)p + (size_t)(p + 1) * g.lds];
      cq = g.S[(size_t)(p + 1) + (size_t)p * g.lds];
      lam.im = sqrt(fabs(bq)) * sqrt(fabs(cq));
    }
    const double smin = fmax(EV_ULP * cabs1(lam), EV_TINY);
    double bound = g.bound[j];   // bound of this vector's pending entries
    const int yc = j - c0;       // LDS column (the imaginary part at yc + 1)
    auto yget = [&](int r) -> cplx {
      return {Yt[r + yc * LY], cx ? Yt[r + (yc + 1) * LY] : 0.0};
    };
    auto yset = [&](int r, cplx v) {
      Yt[r + yc * LY] = v.re;
      if (cx) Yt[r + (yc + 1) * LY] = v.im;
    };
    // scale the whole vector (rows 0 .. p+s-1): global rows outside the
    // tile, LDS rows inside it
    auto scale_all = [&](double f) {
      for (int r = 0; r < p + s; ++r) {
        if (r >= r0 && r < r1) continue;
        g.Y[(size_t)r + (size_t)j * g.ldy] *= f;
        if (cx) g.Y[(size_t)r + (size_t)(j + 1) * g.ldy] *= f;
      }
      for (int r = 0; r < m; ++r) {
        Yt[r + yc * LY] *= f;
        if (cx) Yt[r + (yc + 1) * LY] *= f;
      }
      bound *= f;
    };
    int top;   // the next row to solve (descending); rows > top are known
    if (p >= r1) {
      top = r1 - 1;
    } else {
      // the block lies in this tile: its entries, by the LAPACK convention
      if (!cx) {
        yset(p - r0, {1.0, 0.0});
      } else if (fabs(bq) >= fabs(cq)) {
        yset(p - r0, {1.0, 0.0});
        yset(p + 1 - r0, {0.0, lam.im / bq});
      } else {
        yset(p - r0, {-lam.im / cq, 0.0});
        yset(p + 1 - r0, {0.0, 1.0});
      }
      // the block's contribution to the rows above it inside the tile
      {
        double x = 0.0, c = 0.0;
        for (int q = 0; q < s; ++q) {
          x += cabs1(yget(p + q - r0));
          c = fmax(c, g.colmax[p + q]);
        }
        const double f = guard(bound, c, x);
        if (f < 1.0) scale_all(f);
      }
      for (int q = 0; q < s; ++q) {
        const cplx y = yget(p + q - r0);
        for (int rr = 0; rr < p - r0; ++rr) {
          const double sv = St[rr + (p + q - r0) * LS];
          yset(rr, csub(yget(rr), {sv * y.re, sv * y.im}));
        }
        bound += g.colmax[p + q] * cabs1(y);
      }
      top = p - 1;
    }
    int r = top;
    while (r >= r0) {
      const bool two = (r - 1 >= r0) && St[(r - r0) + (r - 1 - r0) * LS] != 0.0;
      const int rt = two ? r - 1 : r;
      const int a = rt - r0, b = r - r0;
      cplx u1, u2;
      if (!two) {
        const cplx d = pivot({St[b + b * LS] - lam.re, -lam.im}, smin);
        cplx f = yget(b);
        const double fm = cabs1(f);
        if (fm > EV_BIG * cabs1(d)) {   // the quotient would pass the threshold
          scale_all(EV_BIG * cabs1(d) / fm);
          f = yget(b);
        }
        u2 = cdiv(f, d);
        yset(b, u2);
      } else {
        cplx a11 = {St[a + a * LS] - lam.re, -lam.im}, a12 = {St[a + b * LS], 0.0};
        cplx a21 = {St[b + a * LS], 0.0}, a22 = {St[b + b * LS] - lam.re, -lam.im};
        cplx f0 = yget(a), f1 = yget(b);
        if (cabs1(a21) > cabs1(a11)) {   // partial pivoting
          cplx t = a11; a11 = a21; a21 = t;
          t = a12; a12 = a22; a22 = t;
          t = f0; f0 = f1; f1 = t;
        }
        a11 = pivot(a11, smin);
        const cplx mlt = cdiv(a21, a11);
        const cplx p22 = pivot(csub(a22, cmul(mlt, a12)), smin);
        f1 = csub(f1, cmul(mlt, f0));
        const double fm = fmax(cabs1(f0), cabs1(f1));
        const double dm = fmin(cabs1(a11), cabs1(p22)) / (1.0 + cabs1(a12));
        if (fm > EV_BIG * dm) {
          const double f = EV_BIG * dm / fm;
          scale_all(f);
          f0 = {f0.re * f, f0.im * f};
          f1 = {f1.re * f, f1.im * f};
        }
        u2 = cdiv(f1, p22);
        u1 = cdiv(csub(f0, cmul(a12, u2)), a11);
        yset(a, u1);
        yset(b, u2);
      }
      // updates of every pending row (in the tile now, above it through the
      // product): keep the bound below the threshold
      {
        const double x = cabs1(u2) + (two ? cabs1(u1) : 0.0);
        const double c = two ? fmax(g.colmax[r], g.colmax[rt]) : g.colmax[r];
        const double f = guard(bound, c, x);
        if (f < 1.0) {
          scale_all(f);
          u2 = yget(b);
          if (two) u1 = yget(a);
        }
      }
      for (int rr = 0; rr < a; ++rr) {
        cplx v = yget(rr);
        const double s2 = St[rr + b * LS];
        v = csub(v, {s2 * u2.re, s2 * u2.im});
        if (two) {
          const double s1 = St[rr + a * LS];
          v = csub(v, {s1 * u1.re, s1 * u1.im});
        }
        yset(rr, v);
      }
      bound += cabs1(u2) * g.colmax[r] + (two ? cabs1(u1) * g.colmax[rt] : 0.0);
      r = rt - 1;
    }
    g.bound[j] = bound;
  }
  __syncthreads();
  // write back the columns this workgroup owns: its real columns and pairs
  // whose first column is one of its EVT (the imaginary part may be column
  // c0 + EVT); column c0 is skipped when it is a pair's second column
  for (int e = tid; e < m * (EVT + 1); e += EVT) {
    const int r = e % m, c = e / m;
    const int jj = c0 + c;
    if (jj >= n) continue;
    const int own = column_kind(g.S, g.lds, n, jj) == 0 ? jj - 1 : jj;
    if (own >= c0 && own < c0 + EVT) g.Y[(size_t)(r0 + r) + (size_t)jj * g.ldy] = Yt[r + c * LY];
  }
}

// colmax[r] = max over rows i < r of |S(i, r)| (0 for r = 0); bound = 0
__global__ void k_ev_prep(EvArgs g) {
  const int r = blockIdx.x;
  double m = 0.0;
  for (int i = threadIdx.x; i < r; i += blockDim.x)
    m = fmax(m, fabs(g.S[(size_t)i + (size_t)r * g.lds]));
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    g.colmax[r] = red[0];
    g.bound[r] = 0.0;
  }
}

// Each eigenvector (real column, or the two columns of a pair) scaled so
// that its largest |Re| + |Im| is 1.  One workgroup per column.
__global__ void k_ev_normalise(double* X, int ldx, const double* S, int lds, int n) {
  const int j = blockIdx.x;
  const int kind = column_kind(S, lds, n, j);
  if (kind == 0) return;
  const bool cx = kind == 2;
  const double* re = X + (size_t)j * ldx;
  const double* im = cx ? X + (size_t)(j + 1) * ldx : nullptr;
  double m = 0.0;
  for (int r = threadIdx.x; r < n; r += blockDim.x)
    m = fmax(m, fabs(re[r]) + (cx ? fabs(im[r]) : 0.0));
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  const double emax = red[0];
  if (emax <= 0.0) return;
  const double f = 1.0 / emax;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    X[(size_t)r + (size_t)j * ldx] *= f;
    if (cx) X[(size_t)r + (size_t)(j + 1) * ldx] *= f;
  }
}

__global__ void k_ev_zero(double* Y, int ldy, int n) {
  const size_t total = (size_t)n * n;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total;
       k += (size_t)gridDim.x * blockDim.x)
    Y[(size_t)(k % n) + (size_t)(k / n) * ldy] = 0.0;
}

void launch_ev_prep(const EvArgs& g, hipStream_t s) {
  hipLaunchKernelGGL(k_ev_zero, dim3(std::min<size_t>(8192, ((size_t)g.n * g.n + 255) / 256)),
                     dim3(256), 0, s, g.Y, g.ldy, g.n);
  hipLaunchKernelGGL(k_ev_prep, dim3(g.n), dim3(256), 0, s, g);
}

void launch_ev_diag(const EvArgs& g, int r0, int r1, hipStream_t s) {
  const int cols = g.n - r0;
  const int blocks = (cols + EVT - 1) / EVT;
  hipLaunchKernelGGL(k_ev_diag, dim3(blocks), dim3(EVT), 0, s, g, r0, r1);
}

void launch_ev_normalise(double* X, int ldx, const double* S, int lds, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_ev_normalise, dim3(n), dim3(256), 0, s, X, ldx, S, lds, n);
}

}  // namespace schur
