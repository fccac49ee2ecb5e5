// device_common.h -- small FP64 device helpers of the Schur engine.
#pragma once
#include <hip/hip_runtime.h>

namespace schur {

constexpr double kUlp = 2.220446049250313080847263336181640625e-16;  // 2^-52

// Householder reflector P = I - tau v v^T, v = (1, v2, v3), mapping the
// column (x, y, z) to (beta, 0, 0); nr = 2 ignores z.  A zero tail leaves
// P = I (tau = 0).  beta carries the opposite sign of x (x = 0 counts as +).
struct Refl {
  double v2, v3, tau, beta;
};

__device__ __forceinline__ Refl make_reflector(int nr, double x, double y, double z) {
  Refl h;
  if (nr == 2) z = 0.0;
  const double tail = fabs(y) + fabs(z);
  if (tail == 0.0) {
    h.v2 = 0.0; h.v3 = 0.0; h.tau = 0.0; h.beta = x;
    return h;
  }
  // exact power-of-two scaling (no division) keeps every square and product
  // below in range; the scaled quantities are O(1)
  const int e = ilogb(fabs(x) + tail);
  const double xs = ldexp(x, -e), ys = ldexp(y, -e), zs = ldexp(z, -e);
  const double ls = sqrt(xs * xs + ys * ys + zs * zs);
  const double bs = (xs < 0.0) ? ls : -ls;     // beta / 2^e
  const double ds = xs - bs;                   // (x - beta) / 2^e
  // one reciprocal r = 1 / (bs ds) gives 1/beta and 1/(x - beta)
  const double r = 1.0 / (bs * ds);
  h.beta = ldexp(bs, e);
  h.tau = -ds * (ds * r);                      // (beta - x) / beta
  h.v2 = ys * (bs * r);                        // y / (x - beta)
  h.v3 = zs * (bs * r);
  return h;
}

// 1 / d for a normal, finite d: the hardware reciprocal estimate refined by
// two Newton steps (each doubles the correct bits), fewer dependent
// instructions than the correctly rounded division sequence.
__device__ __forceinline__ double fast_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Orders the LDS accesses of the lanes of one wavefront before and after it.
// The hardware executes a wavefront's LDS instructions in order, so only the
// compiler must be kept from moving memory accesses across (a signal fence:
// no instruction, and no wait for outstanding LDS operations); the wave
// barrier makes the CPU emulation of the lanes, which run freely, wait for
// each other.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Barrier of the one-wavefront solvers (small-block QR, early-deflation and
// reordering windows).  Their own kernels run one wavefront per workgroup,
// where it is __syncthreads().  A kernel that runs them on the first
// wavefront of a larger workgroup defines SCHUR_SOLVER_WAVE_SYNC before the
// includes: then it drains the wavefront's outstanding memory operations
// (what the barrier's fence does for a lone wavefront) and orders the lanes,
// without waiting for the other wavefronts.
#ifdef SCHUR_SOLVER_WAVE_SYNC
__device__ __forceinline__ void solver_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
#else
__device__ __forceinline__ void solver_sync() { __syncthreads(); }
#endif

// Value of v held by lane src of the wavefront (src uniform, 0..63): two
// v_readlane_b32 into scalar registers, no LDS round trip.
__device__ __forceinline__ double lane_read(double v, int src) {
  unsigned long long b;
  __builtin_memcpy(&b, &v, sizeof(b));
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  const unsigned long long r = ((unsigned long long)hi << 32) | lo;
  double d;
  __builtin_memcpy(&d, &r, sizeof(d));
  return d;
}

// make_reflector with a short critical path: when x^2 + y^2 + z^2 is far
// from overflow and underflow (the normal case) no scaling is needed; the
// scaled construction covers the rest.  Same reflector up to rounding.
__device__ __forceinline__ Refl make_reflector_fast(int nr, double x, double y, double z) {
  if (nr == 2) z = 0.0;
  const double t2 = y * y + z * z;
  const double s2 = x * x + t2;
  if (!(t2 > 0x1p-900 && s2 < 0x1p+900)) return make_reflector(nr, x, y, z);
  Refl h;
  const double l = sqrt(s2);
  const double b = (x < 0.0) ? l : -l;   // beta
  const double d = x - b;                // x - beta
  const double r = fast_rcp(b * d);
  h.beta = b;
  h.tau = -d * (d * r);                  // (beta - x) / beta
  h.v2 = y * (b * r);                    // y / (x - beta)
  h.v3 = z * (b * r);
  return h;
}

// Shift pair as (sum, product) of the first column polynomial
// (H - s1)(H - s2) e1 restricted to its three nonzeros.
__device__ __forceinline__ void first_column(double h00, double h01, double h10, double h11,
                                             double h21, double s, double t,
                                             double& x, double& y, double& z) {
  x = h00 * h00 + h01 * h10 - s * h00 + t;
  y = h10 * (h00 + h11 - s);
  z = h10 * h21;
}

// Standard form of one 2x2 diagonal block [[a, b], [c, d]] of S.
// The block is an orthogonal similarity G^T B G away from:
//   complex pair: equal diagonal entries and b' c' < 0,
//   real pair   : c' = 0 (two 1x1 blocks).
// G = [[cs, -sn], [sn, cs]].  Writing the block as p I + al Z + be X + ga J
// (Z = diag(1,-1), X = [[0,1],[1,0]], J = [[0,1],[-1,0]]) a rotation by theta
// keeps p and ga and turns the vector (al, be) by 2 theta; the eigenvalues
// are p +- sqrt(al^2 + b c).
struct Std2 {
  double a, b, c, d, cs, sn;
  double wr1, wi1, wr2, wi2;
};

__device__ __forceinline__ void rotate_block(double a, double b, double c, double d,
                                             double cs, double sn, Std2& o) {
  const double p11 = a * cs + b * sn, p12 = b * cs - a * sn;
  const double p21 = c * cs + d * sn, p22 = d * cs - c * sn;
  o.a = cs * p11 + sn * p21;
  o.b = cs * p12 + sn * p22;
  o.c = cs * p21 - sn * p11;
  o.d = cs * p22 - sn * p12;
}

__device__ inline Std2 standardize2(double a, double b, double c, double d) {
  Std2 o;
  o.a = a; o.b = b; o.c = c; o.d = d; o.cs = 1.0; o.sn = 0.0;
  bool split = true;
  const double al = 0.5 * (a - d);
  const double disc = al * al + b * c;
  if (c != 0.0) {
    if (disc < 0.0) {
      // complex pair: choose 2 theta with al cos(2t) + be sin(2t) = 0, cos(2t) >= 0
      const double be = 0.5 * (b + c);
      const double r = hypot(al, be);
      double cs = 1.0, sn = 0.0;
      if (r != 0.0) {
        double c2 = be / r, s2 = -al / r;
        if (c2 < 0.0) { c2 = -c2; s2 = -s2; }
        cs = sqrt(0.5 * (1.0 + c2));
        sn = s2 / (2.0 * cs);
      }
      rotate_block(a, b, c, d, cs, sn, o);
      const double m = 0.5 * (o.a + o.d);
      o.a = m; o.d = m;
      o.cs = cs; o.sn = sn;
      split = !(o.b * o.c < 0.0);   // rounding may leave a (nearly) real pair
      if (split) { o.a = a; o.b = b; o.c = c; o.d = d; }
    }
    if (split) {
      // real pair: the rotation's first column is an eigenvector (l1 - d, c)
      const double r = (disc > 0.0) ? sqrt(disc) : 0.0;
      const double e1 = (al >= 0.0) ? al + r : al - r;
      const double nv = hypot(e1, c);
      const double cs = e1 / nv, sn = c / nv;
      rotate_block(a, b, c, d, cs, sn, o);
      o.c = 0.0;
      o.cs = cs; o.sn = sn;
    }
  }
  if (o.c == 0.0) {
    o.wr1 = o.a; o.wi1 = 0.0; o.wr2 = o.d; o.wi2 = 0.0;
  } else {
    const double im = sqrt(fabs(o.b)) * sqrt(fabs(o.c));
    o.wr1 = o.a; o.wi1 = im; o.wr2 = o.d; o.wi2 = -im;
  }
  return o;
}

}  // namespace schur
