// batch_solve.h -- one whole Schur reduction inside one workgroup of 256
// threads: the device-side driver of the persistent batched kernel
// (batch_kernels.hip).  The same steps as a single solve (paper Sec. 2,
// Eq. (4); Sec. 3.2: early deflation at the bottom of the active block,
// shifts from its undeflated eigenvalues, chains of 3x3 bulges chased
// through diagonal windows whose orthogonal factors go to the off-diagonal
// panels and to Q as FP64 MFMA products), with every decision taken on the
// device, so a batch of matrices needs no host round trip at all: each
// workgroup takes whole matrices from a queue and finishes them.
//
// Written against the HIP device API only, so the same source also runs
// under a CPU emulation of the workgroup in the tests.  The including file
// defines SCHUR_SOLVER_WAVE_SYNC: the one-wavefront solvers run on wavefront
// 0 while the other three wait at the next workgroup barrier.
#pragma once
#include "schur_internal.h"
#include "device_common.h"
#include "kernels.h"
#include "wave_solvers.h"
#include "window_chase.h"
#include "wg_ops.h"
#include "batch.h"

namespace schur {

// LDS of the driver, in doubles: the largest of the window chase (window and
// reflector log), the early-deflation window (S, Z and its buffers), the
// shift solve (S of order 128), the panel products (two tiles) and the
// shift preparation; the deflation scan's bitmap (PB_NMAX / 32 words) also
// lives there while the scan runs.
constexpr int PB_LD96 = SmallSmem<SMALL_Z_MAX>::LD;
constexpr int PB_AED_D = 2 * PB_LD96 * SMALL_Z_MAX + SMALL_Z_MAX + 3 * SMALL_Z_MAX + 7 * SMALL_Z_MAX;
constexpr int PB_CHASE_D = LDW * WMAX + 3 * REFL_LDS;
constexpr int PB_EIG_D = SmallSmem<SMALL_EIG_MAX>::LD * SMALL_EIG_MAX;
constexpr int PB_PANEL_D = 2 * WMAX * LDT;
constexpr int PB_SHIFT_D = (int)(sizeof(ShiftLds) / sizeof(double));
constexpr int pb_max(int a, int b) { return a > b ? a : b; }
constexpr int PB_LDS_D =
    pb_max(pb_max(pb_max(PB_AED_D, PB_CHASE_D), pb_max(PB_EIG_D, PB_PANEL_D)), PB_SHIFT_D);

// small shared state of the driver
struct PShared {
  Ctrl ctrl;                     // deflation scan, early deflation, small solves
  int kt;                        // deflation scan broadcast
  int flag;                      // input check
  int job;                       // queue position of the workgroup's matrix
};

// The window's U (U^T in X->U) to the row panel right of it, the column panel
// above it and Q (one workgroup, all tiles).
__device__ __noinline__ void pb_panels(const WinCtx& c, double* lds, double* cnt) {
  const int pe = c.p + c.ws - 1;
  const double ws2 = 2.0 * c.ws * (double)c.ws;
  cnt[PB_GEMM_FLOPS] += ws2 * ((double)max(0, c.cend - pe - 1) + (double)(c.p - c.rtop) +
                               (c.Q ? (double)c.n : 0.0));
  const int tiles_r = (c.cend - pe - 1 + GEMM_T - 1) / GEMM_T;
  const int tiles_c = (c.p - c.rtop + GEMM_T - 1) / GEMM_T;
  const int tiles_q = c.Q ? (c.n + GEMM_T - 1) / GEMM_T : 0;
  __syncthreads();   // U^T is in X->U; LDS is free
  if (tiles_r > 0) panel_row_tiles(c, 0, tiles_r, lds);
  __syncthreads();
  if (tiles_c + tiles_q > 0) panel_colq_tiles(c, 0, tiles_c + tiles_q, tiles_c, lds);
  __syncthreads();
}

// Solve one matrix.  All 256 threads call it; every branch below is taken
// by all of them (it depends only on LDS or on values every thread read
// after the same barrier).
__device__ inline void pb_solve(const PJob& J, double* lds, PShared& sh, PScratch* X) {
  const int tid = threadIdx.x;
  const int n = J.n;
  double* const H = J.H;
  const int ldh = J.ldh;
  double cnt[PB_COUNTERS];
  for (int i = 0; i < PB_COUNTERS; ++i) cnt[i] = 0.0;
  int info = 0;
  auto finish = [&]() {
    __syncthreads();
    if (tid == 0) {
      *J.info = info;
      if (J.counters)
        for (int i = 0; i < PB_COUNTERS; ++i) J.counters[i] = cnt[i];
    }
  };
  if (n <= 0 || n > PB_NMAX) {
    info = n == 0 ? 0 : -1;
    finish();
    return;
  }
  // ---- input check: the Hessenberg part must be finite; zeros below it
  if (tid == 0) { sh.flag = 0; sh.ctrl = Ctrl{}; }
  __syncthreads();
  {
    int bad = 0;
    for (int c = 0; c < n; ++c)
      for (int r = tid; r < n && r <= c + 1; r += PB_THREADS)
        if (!isfinite(H[r + (size_t)c * ldh])) bad = 1;
    if (bad) atomicOr(&sh.flag, 1);
  }
  __syncthreads();
  if (sh.flag) {
    info = -2;
    finish();
    return;
  }
  for (int c = 0; c + 2 < n; ++c)
    for (int r = c + 2 + tid; r < n; r += PB_THREADS) H[r + (size_t)c * ldh] = 0.0;
  __syncthreads();

  constexpr int LD96 = PB_LD96;
  double* const S96 = lds;
  double* const Z96 = lds + LD96 * SMALL_Z_MAX;
  int kbot = n - 1;
  int nodefl = 0, sweeps = 0;
  while (true) {
    // ---- deflation scan: zeros, converged bottom blocks peeled and
    // standardised (rotations on H and Q), eigenvalues written
    {
      DeflB T{H, J.Q, J.wr, J.wi, ldh, J.ldq, n, kbot, &sh.ctrl};
      deflate_b_wg(T, (unsigned*)lds, sh.kt);
    }
    __syncthreads();
    if (sh.ctrl.bad) { info = -105; break; }
    if (sh.ctrl.kbot < kbot) nodefl = 0;
    kbot = sh.ctrl.kbot;
    if (kbot < 0) break;
    const int ktop = sh.ctrl.ktop;
    const int len = kbot - ktop + 1;
    // ---- a small active block: the workgroup solves it with its Z (bulge
    // chains on the four wavefronts)
    if (len <= J.nmin) {
      const bool whole = ktop == 0 && kbot == n - 1;
      {
        SmallTask t{};
        t.A = H + ktop + (size_t)ktop * ldh;
        t.lda = ldh;
        t.m = len;
        t.wr = J.wr + ktop;
        t.wi = J.wi + ktop;
        t.info = &sh.ctrl.small_info;
        t.itmax = 0;
        if (whole) {
          t.Qacc = J.Q;
          t.ldqacc = J.ldq;
        } else {
          t.Zt = X->U;
          t.ldzt = UPAD;
        }
        small_qr<true, SMALL_Z_MAX, PB_THREADS / 64>(t, S96, Z96, lds + 2 * LD96 * SMALL_Z_MAX);
      }
      __syncthreads();
      cnt[PB_SMALL] += 1;
      cnt[PB_SMALL_FLOPS] += 25.0 * len * (double)len * len;
      if (sh.ctrl.small_info != 0) { info = ktop + sh.ctrl.small_info; break; }
      if (!whole) {
        WinCtx c{};
        c.H = H; c.Q = J.Q; c.U = X->U; c.st = nullptr;
        c.ldh = ldh; c.ldq = J.ldq; c.n = n;
        c.ktop = ktop; c.kbot = kbot; c.rtop = 0; c.cend = n;
        c.p = ktop; c.ws = len;
        pb_panels(c, lds, cnt);
      }
      kbot = ktop - 1;
      if (kbot < 0) break;
      continue;
    }
    if (++sweeps > J.max_sweeps) { info = kbot + 1; break; }
    int ns = min(J.ns, 2 * ((len - 2) / 6));
    if (ns < 2) ns = 2;
    const bool exc = nodefl > 0 && nodefl % J.exc_period == 0;
    // ---- early deflation on the bottom window
    int nu = 0;
    bool aed_shifts = false;
    const int nw = min(J.nw, len - 1);
    if (nw >= 4) {
      {
        AedTask t{};
        t.H = H; t.ldh = ldh;
        t.ktop = ktop; t.kbot = kbot; t.nw = nw;
        t.Ut = X->U; t.ldut = UPAD;
        t.sr = X->sr; t.si = X->si;
        t.wr = J.wr + (kbot - nw + 1); t.wi = J.wi + (kbot - nw + 1);
        t.ctrl = &sh.ctrl;
        t.itmax = 0;
        aed_window<SMALL_Z_MAX, PB_THREADS / 64>(t, S96, Z96, lds + 2 * LD96 * SMALL_Z_MAX,
                                (int*)(lds + 2 * LD96 * SMALL_Z_MAX + SMALL_Z_MAX),
                                lds + 2 * LD96 * SMALL_Z_MAX + 4 * SMALL_Z_MAX);
      }
      __syncthreads();
      const int nd = sh.ctrl.aed_nd;
      nu = sh.ctrl.aed_nu;
      cnt[PB_AED_WINDOWS] += 1;
      cnt[PB_AED_FLOPS] += 25.0 * nw * (double)nw * nw +
                           (nd > 0 ? (10.0 / 3.0) * nu * (double)nu * nu : 0.0);
      if (nd > 0) {
        WinCtx c{};
        c.H = H; c.Q = J.Q; c.U = X->U; c.st = nullptr;
        c.ldh = ldh; c.ldq = J.ldq; c.n = n;
        c.ktop = ktop; c.kbot = kbot; c.rtop = 0; c.cend = n;
        c.p = kbot - nw + 1; c.ws = nw;
        pb_panels(c, lds, cnt);
        cnt[PB_AED_DEFLATED] += nd;
        kbot -= nd;
        nodefl = 0;
        // many deflations: look again before spending a sweep
        if ((J.nibble >= 0 && 100 * nd > J.nibble * nw) || kbot - ktop + 1 <= J.nmin) continue;
      }
      const int m2 = kbot - ktop + 1;
      ns = max(2, min(J.ns, 2 * ((m2 - 2) / 6)));
      if (!exc && nu >= 2 && 2 * nu >= ns) {
        ns = min(ns, nu) & ~1;
        aed_shifts = true;
      }
    }
    // ---- shifts: the undeflated window eigenvalues nearest the deflated
    // part, else the eigenvalues of the trailing block, else ad-hoc pairs
    if (aed_shifts) {
      shift_prep(X->sr + (nu - ns), X->si + (nu - ns), ns, nullptr, 0, H, ldh, ktop, kbot, X->st,
                 *(ShiftLds*)lds);
    } else {
      if (!exc) {
        if (tid < 64) {
          SmallTask t{};
          const int b0 = kbot - ns + 1;
          t.A = H + b0 + (size_t)b0 * ldh;
          t.lda = ldh;
          t.m = ns;
          t.wr = X->ewr;
          t.wi = X->ewi;
          t.info = &sh.ctrl.nshift;
          t.itmax = 0;
          small_qr<false, SMALL_EIG_MAX>(t, lds, nullptr);
        }
        __syncthreads();
        cnt[PB_SMALL_FLOPS] += 10.0 * ns * (double)ns * ns;
      }
      shift_prep(X->ewr, X->ewi, ns, exc ? nullptr : &sh.ctrl.nshift, exc ? 1 : 0, H, ldh, ktop,
                 kbot, X->st, *(ShiftLds*)lds);
    }
    __syncthreads();
    // ---- the sweep: groups of at most PB_NBMAX bulges, each chased down
    // the whole block window by window (a group after the previous one)
    const int npair = ns / 2;
    const int G = (npair + PB_NBMAX - 1) / PB_NBMAX;
    const int nb0 = npair / G + (npair % G ? 1 : 0);
    int step = WMAX - 3 * nb0 - 1;
    step = min(step, REFL_LDS / nb0);
    if (J.step > 0) step = min(step, J.step);
    if (step < 3) step = 3;
    int sh0 = 0;
    bool bad_plan = false;
    for (int g = 0; g < G && !bad_plan; ++g) {
      const int nbg = npair / G + (g < npair % G ? 1 : 0);
      const int tend = kbot - ktop + 3 * nbg - 3;
      const int nwin = (tend + step - 1) / step;
      for (int i = 0; i < nwin; ++i) {
        WinCtx c{};
        c.tau0 = i * step;
        c.tau1 = min(c.tau0 + step, tend);
        c.nb = nbg;
        const int bhi = min(nbg - 1, (c.tau1 - 1) / 3);
        const int kmin = ktop - 1 + max(0, c.tau0 - 3 * bhi);
        const int kmax = min(kbot - 2, ktop - 1 + c.tau1 - 1);
        c.p = max(ktop, kmin);
        c.ws = min(kbot, kmax + 4) - c.p + 1;
        if (c.ws > WMAX || c.ws < 3 || c.p + c.ws - 1 > kbot || nbg > PB_NBMAX ||
            (c.tau1 - c.tau0) * nbg > REFL_LDS) {
          bad_plan = true;   // cannot happen for ns <= 128; never chase out of range
          break;
        }
        c.H = H; c.Q = J.Q; c.U = X->U; c.st = X->st + 2 * sh0;
        c.ldh = ldh; c.ldq = J.ldq; c.n = n;
        c.ktop = ktop; c.kbot = kbot; c.rtop = 0; c.cend = n;
        chase_window_t<PB_THREADS, false>(c, lds, lds + LDW * WMAX);
        pb_panels(c, lds, cnt);
        cnt[PB_WINDOWS] += 1;
        cnt[PB_CHAIN_STEPS] += c.tau1 - c.tau0;
        cnt[PB_CHASE_FLOPS] += 20.0 * c.ws * (double)nbg * (c.tau1 - c.tau0);
      }
      sh0 += nbg;
    }
    if (bad_plan) { info = -3; break; }
    cnt[PB_SWEEPS] += 1;
    cnt[PB_SHIFTS] += ns;
    ++nodefl;
  }
  finish();
}

}  // namespace schur
