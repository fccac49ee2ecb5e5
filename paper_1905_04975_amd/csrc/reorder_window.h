// reorder_window.h -- the window task of eigenvalue reordering (paper
// Sec. 2, Eq. (7); Sec. 3.2: overlapping Givens rotations and 3x3
// Householder reflectors applied inside a diagonal window and accumulated).
// Included by kernels.hip; written against the HIP device API only.
#pragma once
#include "wave_solvers.h"

namespace schur {

// Rounds of parallel swaps: every selected block whose upper neighbour is
// an unselected block swaps with it (such pairs never overlap, so the
// round's swaps are independent: plans first, one lane each, then all left
// transforms, then all right transforms, as in a sweep).  Selected blocks
// never pass each other, so their order is kept.  Returns 0, or 1 when a
// swap failed the stability test of its plan (the reordering of this
// window stops there; the window is still an orthogonal similarity of the
// input).  status: w ints of LDS (1 = selected row); ibuf: 4 (w / 2 + 1)
// ints; pbuf: 12 (w / 2 + 1) doubles.
__device__ int select_reorder(double* S, double* Zs, int LD, int w, int* status, int* ibuf,
                              double* pbuf) {
  const int lane = threadIdx.x;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  const int maxsw = w / 2 + 1;
  int* sw_k = ibuf;              // first row of the swapped pair of blocks
  int* sw_p = ibuf + maxsw;      // order of the upper (unselected) block
  int* sw_r = ibuf + 2 * maxsw;  // order of the lower (selected) block
  int* sw_ok = ibuf + 3 * maxsw;
  double* pl_v = pbuf;               // 8 per swap
  double* pl_t = pbuf + 8 * maxsw;   // 2 per swap
  double* pl_d = pbuf + 10 * maxsw;  // 2 per swap (restored 1x1 diagonals)
  int rounds = 0;
  int failed = 0;
  while (true) {
    if (++rounds > 4 * w + 16) break;   // never reached: each round moves a block up
    // ---- this round's swaps: a selected block start r whose upper
    // neighbour (ending at r - 1) is unselected
    int nsw = 0;
    for (int base = 0; base < w; base += 64) {
      const int r = base + lane;
      bool go = false;
      int pp = 1, rr = 1;
      if (r >= 1 && r < w && status[r] == 1 && status[r - 1] == 0 && Sx(r, r - 1) == 0.0) {
        rr = (r + 1 < w && Sx(r + 1, r) != 0.0) ? 2 : 1;
        pp = (r >= 2 && Sx(r - 1, r - 2) != 0.0) ? 2 : 1;
        go = true;
      }
      const unsigned long long mask = __ballot(go);
      if (go) {
        const int idx = nsw + __builtin_popcountll(mask & ((1ull << lane) - 1ull));
        sw_k[idx] = r - pp;
        sw_p[idx] = pp;
        sw_r[idx] = rr;
      }
      nsw += __builtin_popcountll(mask);
    }
    __syncthreads();
    if (nsw == 0) break;
    // ---- plans, one lane per swap
    for (int q = lane; q < nsw; q += 64) {
      const int k = sw_k[q], pp = sw_p[q], rr = sw_r[q];
      SwapPlan pl;
      bool ok;
      if (pp == 1 && rr == 1) ok = plan_swap<1, 1>(S, LD, k, pl);
      else if (pp == 1) ok = plan_swap<1, 2>(S, LD, k, pl);
      else if (rr == 1) ok = plan_swap<2, 1>(S, LD, k, pl);
      else ok = plan_swap<2, 2>(S, LD, k, pl);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        pl_t[2 * q + h] = (h < rr) ? pl.tau[h] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) pl_v[8 * q + 4 * h + i] = (h < rr) ? pl.v[h][i] : 0.0;
      }
      pl_d[2 * q] = Sx(k, k);                                   // upper block's 1x1 eigenvalue
      pl_d[2 * q + 1] = Sx(k + pp + rr - 1, k + pp + rr - 1);   // lower block's
      sw_ok[q] = ok ? 1 : 0;
    }
    __syncthreads();
    bool bad = false;
    for (int q = lane; q < nsw; q += 64) bad = bad || sw_ok[q] == 0;
    if (__ballot(bad) != 0ull) {   // uniform: nothing of this round is applied
      failed = 1;
      break;
    }
    // ---- transforms: lanes in groups of G per swap (swaps beyond 64 lanes
    // take further passes)
    for (int s0 = 0; s0 < nsw; s0 += 64) {
      const int cnt = min(64, nsw - s0);
      const int G = 64 / cnt;
      const int t = lane / G, sub = lane - t * G;
      const bool mine = t < cnt;
      const int q = s0 + (mine ? t : 0);
      const int k = sw_k[q], pp = sw_p[q], rr = sw_r[q], N = pp + rr;
      double v[8], tau[2];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = mine ? pl_v[8 * q + i] : 0.0;
      tau[0] = mine ? pl_t[2 * q] : 0.0;
      tau[1] = mine ? pl_t[2 * q + 1] : 0.0;
      // left: rows k..k+N-1, columns k..w-1
      if (mine) {
        for (int c = k + sub; c < w; c += G) {
          double a4[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) a4[i] = Sx((i < N) ? k + i : k, c);
          swap_apply(a4, v, tau, N);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (i < N) Sx(k + i, c) = a4[i];
        }
      }
      __syncthreads();
      // right: columns k..k+N-1 of S rows 0..k+N-1, then of every row of Z
      if (mine) {
        const int ns = k + N;
        const int tot = ns + w;
        const double dA = pl_d[2 * q], dB = pl_d[2 * q + 1];
        for (int e = sub; e < tot; e += G) {
          double* base = (e < ns) ? S : Zs;
          const int row = (e < ns) ? e : e - ns;
          double a4[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) a4[i] = base[row + ((i < N) ? k + i : k) * LD];
          swap_apply(a4, v, tau, N);
          if (e < ns) {   // exact zeros below the moved blocks, 1x1 eigenvalues restored
            if (row >= k + rr) { a4[0] = 0.0; if (rr == 2) a4[1] = 0.0; }
            if (rr == 1 && row == k) a4[0] = dB;
            if (pp == 1 && row == k + rr) a4[rr] = dA;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (i < N) base[row + (k + i) * LD] = a4[i];
        }
      }
      __syncthreads();
    }
    // ---- bookkeeping: the selected block now leads its pair
    for (int q = lane; q < nsw; q += 64) {
      const int k = sw_k[q], pp = sw_p[q], rr = sw_r[q];
      for (int i = 0; i < rr; ++i) status[k + i] = 1;
      for (int i = 0; i < pp; ++i) status[k + rr + i] = 0;
    }
    __syncthreads();
  }
  __syncthreads();
  return failed;
}

template <int MAXM>
__device__ void reorder_window(const ReorderTask& T, double* S, double* Z, int* status, int* ibuf,
                               double* pbuf) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int lane = threadIdx.x;
  const int w = T.w;
  if (w < 1 || w > MAXM) return;
  double* Sw = T.S + T.a + (size_t)T.a * T.lds;
  SmallTask st{};
  st.A = Sw; st.lda = T.lds; st.m = w;
  small_load<true, MAXM>(st, S, Z);   // the window (zeros below the subdiagonal) and Z = I
  for (int r = lane; r < w; r += 64) status[r] = T.sel[T.a + r];
  __syncthreads();
  const int failed = select_reorder(S, Z, LD, w, status, ibuf, pbuf);
  // moved 2x2 blocks back to standard form (rotations on S and Z)
  aed_std_all(S, Z, LD, w, 0, pbuf);
  __syncthreads();
  for (int c = 0; c < w; ++c)
    for (int r = lane; r < w; r += 64) Sw[r + (size_t)c * T.lds] = S[r + c * LD];
  for (int r = lane; r < w; r += 64) T.sel[T.a + r] = (unsigned char)status[r];
  if (lane == 0 && failed && T.info) *T.info = 1;
  __syncthreads();
  aed_write_vt(S, Z, LD, w, T.Ut, T.ldut);
}

}  // namespace schur
