// window_chase.h -- the window task of a sweep: bulge chains chased
// through one diagonal window held in LDS, and the window's accumulated
// orthogonal factor.  Included by kernels.hip; written against the HIP
// device API only, so the same source also runs under a CPU emulation of a
// workgroup in the tests.
#pragma once
#include "schur_internal.h"
#include "device_common.h"

namespace schur {

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
    // entering bulge: formed after the barrier (at tau0 the form above is it)
    if (tau > d.tau0 && K == ktop - 1) form(tau, K, nr, act, h);
    wave_sync();   // all lanes of a bulge have read its column before any lane updates
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
            u1[q] = row[0]; u2[q] = row[LDW];
            // a 2-row reflector (v3 = 0, at the block bottom) must not touch
            // the third column: it can lie past the window's last column
            u3[q] = (v3[q] != 0.0) ? row[2 * LDW] : 0.0;
          }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (tv[q] == 0.0) continue;
          const double w = tv[q] * (u1[q] + v2[q] * u2[q] + v3[q] * u3[q]);
          double* row = &Wx(r, kk[q] + 1);
          row[0] = u1[q] - w;
          row[LDW] = u2[q] - w * v2[q];
          if (v3[q] != 0.0) row[2 * LDW] = u3[q] - w * v3[q];
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

}  // namespace schur
