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
// Thread layout: NT = 1024 threads (the sweep kernels) or 256 (the
// persistent batched kernel); group b (TPB = 64 or 32 consecutive threads,
// inside one wavefront) owns bulge b of the window's chain, so a window
// carries at most NBMAX (1024 threads) or 8 (256 threads) bulges.  One chain step
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
// window is written back, U is accumulated in the freed LDS with NT / 128
// lanes of one wavefront per row (rows are independent).
// ============================================================================
constexpr int CHASE_THREADS = 1024;

// W: LDW x WMAX doubles of LDS, R: 3 REFL_LDS doubles of LDS.
template <int NT, bool REORTH = true>
__device__ void chase_window_t(const WinCtx& d, double* W, double* R) {
  static_assert(NT == 1024 || NT == 256, "1024 or 256 threads");
  constexpr int CG = NT / 128;       // column groups of the window load / store
  constexpr int QL = WMAX / CG;      // columns per thread in them
  constexpr int QB = QL < 16 ? QL : 16;   // loads in flight per batch
  constexpr int J = NT / 128;        // lanes per row of the U accumulation
  constexpr int NBT = NT == 1024 ? NBMAX : NT / 32;   // most bulges per window
  constexpr int QU = (NBT + J - 1) / J;   // bulges per lane and chain step in it
  const int tid = threadIdx.x;
  const int p = d.p, ws = d.ws, nb = d.nb;
  const int ktop = d.ktop, kbot = d.kbot;
  const WinCtx& a = d;   // matrix fields
  auto Wx = [&](int r, int c) -> double& { return W[r + c * LDW]; };

  // load the window: CG columns per pass, a batch of loads issued before
  // its stores
  {
    const int r = tid & 127, c0 = tid >> 7;
    for (int qb = 0; qb < QL; qb += QB) {
      double v[QB];
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int c = c0 + CG * (qb + q);
        v[q] = (r < ws && c < ws) ? a.H[(size_t)(p + r) + (size_t)(p + c) * a.ldh] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int c = c0 + CG * (qb + q);
        if (r < ws && c < ws) Wx(r, c) = v[q];
      }
    }
  }
  const int lgt = (nb <= NT / 64) ? 6 : 5;
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
    for (int q = 0; q < QL; ++q) {
      const int c = c0 + CG * q;
      if (r < ws && c < ws) a.H[(size_t)(p + r) + (size_t)(p + c) * a.ldh] = Wx(r, c);
    }
  }
  __syncthreads();

  // ---- accumulate U = P_1 P_2 ... ; row r by lanes j = 0..J-1 of its wave,
  // lane j applying the reflectors of bulges j, j+J, j+2J, ... of each chain
  // step (they touch disjoint columns)
  {
    const int r = tid / J, j = tid % J;
    if (r < ws)
      for (int c = j; c < ws; c += J) Wx(r, c) = (r == c) ? 1.0 : 0.0;
    wave_sync();
    for (int tau = d.tau0; tau < d.tau1; ++tau) {
      int klead = ktop - 1 + tau;
      if (klead > kbot - 2) klead = kbot - 2;
      const bool rowact = (r < ws) && (r <= klead + 3 - p);
      const double* rt = &R[3 * (tau - d.tau0) * nb];
      if (rowact) {
        double u1[QU], u2[QU], u3[QU], tv[QU], v2[QU], v3[QU];
        int kk[QU];
#pragma unroll
        for (int q = 0; q < QU; ++q) {
          const int bb = j + J * q;
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
        for (int q = 0; q < QU; ++q) {
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
    for (int q = 0; q < QL; ++q) {   // Ut(r, c) = U(c, r)
      const int c = c0 + CG * q;
      Ut[r + (size_t)c * UPAD] = (r < ws && c < ws) ? Wx(c, r) : 0.0;
    }
  }
  // ---- one first-order re-orthogonalisation, U^T <- (I - E / 2) U^T with
  // E = U^T U - I, before U reaches the panels and Q: U collected every
  // reflector of the window, and its departure from orthogonality would
  // otherwise add up in Q over the sweep's windows.  The persistent kernel's
  // matrices (order <= 1024) put few window products into Q; it skips it.  Both products as FP64
  // MFMA 16 x 16 tiles over the workgroup's wavefronts.  E is symmetric:
  // its upper tiles from U in LDS, then E (both triangles) replaces U in
  // LDS (U^T is in the slot).  The new U^T by column blocks of 16 in two
  // halves of row tiles, one wavefront per half: a half's tiles read only
  // its column block of the slot (held in registers, read by every half
  // before any writes).
  if constexpr (REORTH) {
    typedef double cw_d4 __attribute__((ext_vector_type(4)));
    constexpr int NW = NT / 64;                     // wavefronts
    constexpr int NTM = WMAX / 16;                  // tiles per side at most
    constexpr int TPW = (NTM * (NTM + 1) / 2 + NW - 1) / NW;   // upper tiles per wavefront
    const int wv = tid >> 6, lane = tid & 63, kr = lane >> 4, kc = lane & 15;
    const int nt = (ws + 15) >> 4;
    const int npair = nt * (nt + 1) / 2;
    auto pair_of = [&](int q, int& I, int& J) {   // q = J (J + 1) / 2 + I, I <= J
      J = 0;
      while ((J + 1) * (J + 2) / 2 <= q) ++J;
      I = q - J * (J + 1) / 2;
    };
    // the wavefront's tiles side by side in each k step: independent
    // accumulation chains keep the MFMA pipeline busy
    cw_d4 acc[TPW];
    int ia[TPW], jb[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      acc[u] = cw_d4{0.0, 0.0, 0.0, 0.0};
      const int q = wv + NW * u;
      int I = 0, J = 0;
      if (q < npair) pair_of(q, I, J);
      ia[u] = q < npair ? 16 * I + kc : ws;   // out of the window: zero operands
      jb[u] = q < npair ? 16 * J + kc : ws;
    }
#pragma unroll 4
    for (int s4 = 0; s4 < WMAX / 4; ++s4) {
      const int k = 4 * s4 + kr;
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        if (wv + NW * u >= npair) continue;   // uniform over the wavefront
        const double a = (k < ws && ia[u] < ws) ? Wx(k, ia[u]) : 0.0;   // A(i, k) = U(k, i)
        const double b = (k < ws && jb[u] < ws) ? Wx(k, jb[u]) : 0.0;   // B(k, j) = U(k, j)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
      }
    }
    __syncthreads();   // every read of U in LDS is done, and U^T is in the slot
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const int q = wv + NW * u;
      if (q >= npair) continue;
      int I, J;
      pair_of(q, I, J);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = 16 * I + 4 * e + kr, col = 16 * J + kc;
        if (row < ws && col < ws) {
          const double v = acc[u][e] - (row == col ? 1.0 : 0.0);
          Wx(row, col) = v;
          Wx(col, row) = v;
        }
      }
    }
    __syncthreads();   // E in LDS
    // jobs: (column block R, half h of its row tiles), h = 0: tiles 0..3,
    // h = 1: tiles 4..7; each wavefront owns whole jobs, and a job reads
    // only its own column block of the slot (rows of other jobs of the same
    // block are written by another wavefront but never read by this one:
    // bv holds the block's column, read before the barrier below)
    const int nj = 2 * nt;
    for (int jb0 = 0; jb0 < 2 * NTM; jb0 += NW) {
      const int job = jb0 + wv;
      const bool act = job < nj;
      const int R = act ? job >> 1 : 0, h = job & 1;
      const int rb = 16 * R + kc;
      // the block's column of U^T in registers, every load in flight at once:
      // bv[s] = U^T(4 s + kr, R0 + kc), the B operand of step s and, for
      // s = 4 J + e, the old value of this lane's result entry (e) of tile J
      double bv[WMAX / 4];
#pragma unroll
      for (int s4 = 0; s4 < WMAX / 4; ++s4) {
        const int k = 4 * s4 + kr;
        bv[s4] = (act && k < ws && rb < ws) ? Ut[k + (size_t)rb * UPAD] : 0.0;
      }
      __syncthreads();   // every job has read its column before any writes
      if (act && 4 * h < nt) {
        // the half's four row tiles, their accumulation chains interleaved
        cw_d4 c[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) c[g] = cw_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < WMAX / 4; ++s4) {
          const int k = 4 * s4 + kr;
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int ja = 16 * (4 * h + g) + kc;
            const double av = (k < ws && ja < ws) ? Wx(ja, k) : 0.0;   // E(16 J + i, k)
            c[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[s4], c[g], 0, 0, 0);
          }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int J = 4 * h + g;
            const int jr = 16 * J + 4 * e + kr;
            const double old = h ? bv[16 + 4 * g + e] : bv[4 * g + e];
            if (jr < ws && rb < ws) Ut[jr + (size_t)rb * UPAD] = old - 0.5 * c[g][e];
          }
        }
      }
    }
  }
}

__device__ void chase_window(const WinCtx& d) {
  __shared__ double W[LDW * WMAX];
  __shared__ double R[REFL_LDS * 3];
  chase_window_t<CHASE_THREADS>(d, W, R);
}

}  // namespace schur
