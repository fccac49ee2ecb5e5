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
#include "wave_solvers.h"
#include "window_chase.h"
#include "reorder_window.h"

namespace schur {

typedef double d4 __attribute__((ext_vector_type(4)));

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

template <int MAXM>
__global__ __launch_bounds__(64) void k_aed(AedTask t0, const AedTask* tasks) {
  const AedTask T = tasks ? tasks[blockIdx.x] : t0;
  constexpr int LD = SmallSmem<MAXM>::LD;
  __shared__ double S[LD * MAXM];
  __shared__ double Z[LD * MAXM];
  __shared__ double vv[MAXM];
  __shared__ int ibuf[6 * MAXM];
  __shared__ double stdbuf[7 * MAXM];
  aed_window<MAXM>(T, S, Z, vv, ibuf, stdbuf);
}

// One window of eigenvalue reordering per workgroup (one wavefront, window
// and its accumulated orthogonal factor in LDS).
template <int MAXM>
__global__ __launch_bounds__(64) void k_reorder(const ReorderTask* tasks) {
  const ReorderTask T = tasks[blockIdx.x];
  constexpr int LD = SmallSmem<MAXM>::LD;
  __shared__ double S[LD * MAXM];
  __shared__ double Z[LD * MAXM];
  __shared__ int status[MAXM];
  __shared__ int ibuf[4 * (MAXM / 2 + 1)];
  __shared__ double pbuf[7 * MAXM + 16];   // swap plans, then the standardisation
  reorder_window<MAXM>(T, S, Z, status, ibuf, pbuf);
}

// One window of a parallel early-deflation pass per workgroup (one wavefront,
// window and Schur vectors in LDS).
template <int MAXM>
__global__ __launch_bounds__(64) void k_split(const SplitTask* tasks) {
  const SplitTask T = tasks[blockIdx.x];
  constexpr int LD = SmallSmem<MAXM>::LD;
  __shared__ double S[LD * MAXM];
  __shared__ double Z[LD * MAXM];
  __shared__ double vv[MAXM];
  __shared__ int ibuf[6 * MAXM];
  __shared__ double pbuf[7 * MAXM];
  split_window<MAXM>(T, S, Z, vv, ibuf, pbuf);
}

// Chosen windows of a pass (disjoint) written from their output slots into
// H (the Hessenberg part), and the coupling entries at their ends scaled:
// above by this window's and the committed neighbour's factors, below by
// this window's alone when no committed window starts there.  One
// workgroup per window.
__global__ void k_split_commit(const SplitCommit* cm, const SplitTask* tasks) {
  const SplitCommit c = cm[blockIdx.x];
  const SplitTask t = tasks[c.task];
  const int nw = t.nw;
  for (int idx = threadIdx.x; idx < nw * nw; idx += blockDim.x) {
    const int r = idx % nw, col = idx / nw;
    if (r <= col + 1) t.H[(t.a + r) + (size_t)(t.a + col) * t.ldh] = t.Wo[r + (size_t)col * t.ldwo];
  }
  if (threadIdx.x == 0) {
    const SplitRes r = *t.res;
    if (c.fix_top) {
      const double f = r.ftop * (c.above >= 0 ? tasks[c.above].res->fbot : 1.0);
      t.H[t.a + (size_t)(t.a - 1) * t.ldh] *= f;
    }
    if (c.fix_below) t.H[(t.a + nw) + (size_t)(t.a + nw - 1) * t.ldh] *= r.fbot;
  }
}

// Negligible subdiagonal entries (same test as the deflation scan) over the
// whole matrix: zero[k] = 1 where row k starts a block.  Read-only on H, so
// every test sees the original neighbours; k_split_zero writes the zeros.
__global__ void k_split_scan(const double* H, int ldh, int n, unsigned char* zero) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    if (k == 0) {
      zero[0] = 1;
      continue;
    }
    const double sub = fabs(H[k + (size_t)(k - 1) * ldh]);
    double tst = fabs(H[(k - 1) + (size_t)(k - 1) * ldh]) + fabs(H[k + (size_t)k * ldh]);
    if (tst == 0.0) {
      tst = fabs(H[(k - 1) + (size_t)k * ldh]);
      if (k >= 2) tst += fabs(H[(k - 1) + (size_t)(k - 2) * ldh]);
      if (k + 1 < n) tst += fabs(H[(k + 1) + (size_t)k * ldh]);
    }
    zero[k] = (sub <= kUlp * tst) ? 1 : 0;
  }
}

// The entries flagged by k_split_scan set to exactly zero.
__global__ void k_split_zero(double* H, int ldh, int n, const unsigned char* zero) {
  for (int k = 1 + blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    if (zero[k]) H[k + (size_t)(k - 1) * ldh] = 0.0;
}

// Identity of order sizes[b] in the leading corner of UPAD x UPAD slot b,
// zero elsewhere (grid.y = slots).
__global__ void k_slot_ident(double* U, const int* sizes) {
  const int b = blockIdx.y;
  const int m = sizes[b];
  double* u = U + (size_t)b * UPAD * UPAD;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < UPAD * UPAD;
       idx += gridDim.x * blockDim.x) {
    const int r = idx % UPAD, c = idx / UPAD;
    u[idx] = (r == c && r < m) ? 1.0 : 0.0;
  }
}

// Slot b of dst = transpose of slot b of src (grid.y = slots).
__global__ void k_slot_transpose(const double* src, double* dst) {
  const size_t off = (size_t)blockIdx.y * UPAD * UPAD;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < UPAD * UPAD;
       idx += gridDim.x * blockDim.x) {
    const int r = idx % UPAD, c = idx / UPAD;
    dst[off + c + (size_t)r * UPAD] = src[off + idx];
  }
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
    // non-finite candidates are dropped: the ranking below needs a strict
    // order of the keys (ties broken by index)
    const bool ok = e >= valid0 && isfinite(wr[e]) && isfinite(wi[e]);
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

__device__ __forceinline__ WinCtx ctx_of(const SweepArgs& a, const Win& w) {
  WinCtx c;
  c.H = a.H; c.Q = a.Q; c.U = a.U + (size_t)w.slot * UPAD * UPAD;
  c.st = a.st + 2 * w.shift0;
  c.ldh = a.ldh; c.ldq = a.ldq; c.n = a.n;
  c.ktop = a.ktop; c.kbot = a.kbot; c.rtop = a.rtop; c.cend = a.cend;
  c.p = w.p; c.ws = w.ws; c.tau0 = w.tau0; c.tau1 = w.tau1; c.nb = w.nb;
  return c;
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

// Panel tiles are processed up to PANEL_TPB at a time by one workgroup of
// four waves, one workgroup per CU (two 128 x 68 FP64 LDS buffers, 136 KiB):
//  * the window's U (or U^T) is read into registers once;
//  * while tile t is multiplied from LDS, the wave issues, one per k step,
//    the global loads of tile t+1 (into registers) and the global stores of
//    the results of tile t-1 (kept in a second set of accumulators), so that
//    HBM traffic and the FP64 MFMA work overlap instead of alternating;
//  * the operands of the next k step are read from LDS before the products
//    of the current one are issued.
// Each pass: tile t -> LDS, barrier, then the interleaved k loop.  One pass
// more than there are tiles stores the last results.

// Row panel: Y(ws x 64) = U^T X for 64-column tiles of H(p:p+ws-1, right of
// the window).  Wave w owns rows 32w..32w+31 of U^T (A operand, registers)
// and all 64 tile columns (B operand from LDS, row-major tile Xs[c + r*LDT]).
// Element e of a thread's tile load: window row r = lane + 64 (e & 1), tile
// column c = wave + 4 (e >> 1).  Element s of a thread's results: acc[s >> 4]
// [(s >> 2) & 3][s & 3], row i0 + 16 (s >> 4) + lk + 4 (s & 3), column
// 16 ((s >> 2) & 3) + li.
__device__ void panel_row_tiles(const WinCtx& d, int t0, int t1) {
  __shared__ double Xs[2][WMAX * LDT];
  const int p = d.p, ws = d.ws;
  const int kpad = (ws + 3) & ~3;
  const double* Ut = d.U;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = wave * 32;
  const bool active = i0 < ws;
  double ua[UPAD / 4][2];
  if (active) {
#pragma unroll
    for (int ks = 0; ks < UPAD / 4; ++ks) {
      const int k = 4 * ks + lk;
      ua[ks][0] = Ut[(i0 + li) + (size_t)k * UPAD];
      ua[ks][1] = Ut[(i0 + 16 + li) + (size_t)k * UPAD];
    }
  }
  double* const H = d.H;
  const size_t ldh = d.ldh;
  // first column of tile t and its width
  auto col0 = [&](int t) { return p + ws + t * PT; };
  auto ncols = [&](int t) { return min(PT, d.cend - col0(t)); };
  // rows past the window read row ws-1 and are zeroed on the way to LDS;
  // columns past the panel are not read (uniform test per wave)
  auto load_one = [&](double& dst, int c0, int nc, int e) {
    const int r = lane + 64 * (e & 1), c = wave + 4 * (e >> 1);
    dst = (c < nc) ? H[(size_t)(p + min(r, ws - 1)) + (size_t)(c0 + c) * ldh] : 0.0;
  };
  auto store_one = [&](const d4 (&res)[2][4], int c0, int nc, int s) {
    const int ib = s >> 4, jb = (s >> 2) & 3, e = s & 3;
    const int row = i0 + ib * 16 + lk + 4 * e, col = jb * 16 + li;
    if (row < ws && col < nc) H[(size_t)(p + row) + (size_t)(c0 + col) * ldh] = res[ib][jb][e];
  };
  double pre[32];
  {
    const int c0 = col0(t0), nc = ncols(t0);
#pragma unroll
    for (int e = 0; e < 32; ++e) load_one(pre[e], c0, nc, e);
  }
  __builtin_amdgcn_s_waitcnt(0);   // U and the first tile are in registers
  d4 acc[2][4], accp[2][4];
  for (int t = t0; t <= t1; ++t) {
    const bool cur = t < t1, prev = t > t0 && active, next = t + 1 < t1;
    double* X = Xs[(t - t0) & 1];
    if (cur) {
#pragma unroll
      for (int e = 0; e < 32; ++e) {
        const int r = lane + 64 * (e & 1), c = wave + 4 * (e >> 1);
        X[c + r * LDT] = r < ws ? pre[e] : 0.0;   // r < 128, c < 64: inside the buffer
      }
      __syncthreads();
    }
    const int cn0 = col0(t + 1), nnc = ncols(t + 1);
    const int cp0 = col0(t - 1), npc = ncols(t - 1);
    const bool mm = active && cur;
    if (mm) {
      for (int ib = 0; ib < 2; ++ib)
        for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
    }
    double bn[4];
    if (mm) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) bn[jb] = X[(jb * 16 + li) + lk * LDT];
    }
#pragma unroll
    for (int ks = 0; ks < UPAD / 4; ++ks) {
      if (next) load_one(pre[ks], cn0, nnc, ks);
      if (prev) store_one(accp, cp0, npc, ks);
      if (mm && 4 * ks < kpad) {
        double b[4];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) b[jb] = bn[jb];
        const int kn = min(4 * ks + 4, kpad - 4) + lk;   // the last step re-reads a valid row
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) bn[jb] = X[(jb * 16 + li) + kn * LDT];
        __builtin_amdgcn_sched_barrier(0);   // keep these reads ahead of the products below
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
          acc[0][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[ks][0], b[jb], acc[0][jb], 0, 0, 0);
          acc[1][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[ks][1], b[jb], acc[1][jb], 0, 0, 0);
        }
      }
    }
    if (mm) {
      for (int ib = 0; ib < 2; ++ib)
        for (int jb = 0; jb < 4; ++jb) accp[ib][jb] = acc[ib][jb];
    }
  }
}

// Column panel and Q: Y(64 x ws) = X U for 64-row tiles; tile < tiles_c is
// a tile of H(rtop:p-1, p:p+ws-1), the others are tiles of Q(:, p:p+ws-1).
// Wave w owns columns 32w..32w+31 of U (B operand, registers) and all 64
// tile rows (A operand from LDS, column-major tile Xs[r + c*LDT]).  Element
// e of a thread's tile load: tile row lane, window column wave + 4 e.
// Element s of a thread's results: acc[s >> 3][(s >> 2) & 1][s & 3], row
// 16 (s >> 3) + lk + 4 (s & 3), column j0 + 16 ((s >> 2) & 1) + li.
__device__ void panel_colq_tiles(const WinCtx& d, int t0, int t1, int tiles_c) {
  __shared__ double Xs[2][WMAX * LDT];
  const int p = d.p, ws = d.ws;
  const int kpad = (ws + 3) & ~3;
  const double* Ut = d.U;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int j0 = wave * 32;
  const bool active = j0 < ws;
  double ub[UPAD / 4][2];
  if (active) {
#pragma unroll
    for (int ks = 0; ks < UPAD / 4; ++ks) {
      const int k = 4 * ks + lk;
      ub[ks][0] = Ut[(j0 + li) + (size_t)k * UPAD];
      ub[ks][1] = Ut[(j0 + 16 + li) + (size_t)k * UPAD];
    }
  }
  // tile t: first element (row r0, column p) and number of rows
  struct Tile { double* base; size_t ld; int nr; };
  auto tile = [&](int t) {
    Tile T;
    if (t < tiles_c) {
      const int r0 = d.rtop + t * PT;
      T.base = d.H + (size_t)r0 + (size_t)p * d.ldh; T.ld = d.ldh; T.nr = min(PT, p - r0);
    } else {
      const int r0 = (t - tiles_c) * PT;
      T.base = d.Q + (size_t)r0 + (size_t)p * d.ldq; T.ld = d.ldq; T.nr = min(PT, d.n - r0);
    }
    return T;
  };
  // rows past the tile read its last row and are zeroed on the way to LDS;
  // columns past the window are not read (uniform test per wave)
  auto load_one = [&](double& dst, const Tile& T, int e) {
    const int c = wave + 4 * e;
    dst = (c < ws) ? T.base[(size_t)min(lane, T.nr - 1) + (size_t)c * T.ld] : 0.0;
  };
  auto store_one = [&](const d4 (&res)[4][2], const Tile& T, int s) {
    const int ib = s >> 3, jb = (s >> 2) & 1, e = s & 3;
    const int row = ib * 16 + lk + 4 * e, col = j0 + jb * 16 + li;
    if (row < T.nr && col < ws) T.base[(size_t)row + (size_t)col * T.ld] = res[ib][jb][e];
  };
  double pre[32];
  {
    const Tile T = tile(t0);
#pragma unroll
    for (int e = 0; e < 32; ++e) load_one(pre[e], T, e);
  }
  __builtin_amdgcn_s_waitcnt(0);   // U and the first tile are in registers
  d4 acc[4][2], accp[4][2];
  for (int t = t0; t <= t1; ++t) {
    const bool cur = t < t1, prev = t > t0 && active, next = t + 1 < t1;
    double* X = Xs[(t - t0) & 1];
    if (cur) {
      const int nr_t = tile(t).nr;
#pragma unroll
      for (int e = 0; e < 32; ++e)   // inside the buffer
        X[lane + (wave + 4 * e) * LDT] = lane < nr_t ? pre[e] : 0.0;
      __syncthreads();
    }
    const Tile TN = tile(next ? t + 1 : t0), TP = tile(prev ? t - 1 : t0);
    const bool mm = active && cur;
    if (mm) {
      for (int ib = 0; ib < 4; ++ib)
        for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
    }
    double an[4];
    if (mm) {
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) an[ib] = X[(ib * 16 + li) + lk * LDT];
    }
#pragma unroll
    for (int ks = 0; ks < UPAD / 4; ++ks) {
      if (next) load_one(pre[ks], TN, ks);
      if (prev) store_one(accp, TP, ks);
      if (mm && 4 * ks < kpad) {
        double av[4];
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) av[ib] = an[ib];
        const int kn = min(4 * ks + 4, kpad - 4) + lk;   // the last step re-reads a valid row
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) an[ib] = X[(ib * 16 + li) + kn * LDT];
        __builtin_amdgcn_sched_barrier(0);   // keep these reads ahead of the products below
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) {
          acc[ib][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ib], ub[ks][0], acc[ib][0], 0, 0, 0);
          acc[ib][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ib], ub[ks][1], acc[ib][1], 0, 0, 0);
        }
      }
    }
    if (mm) {
      for (int ib = 0; ib < 4; ++ib)
        for (int jb = 0; jb < 2; ++jb) accp[ib][jb] = acc[ib][jb];
    }
  }
}

// tiles [t0, t1) of the window whose workgroup prefix is `base`
__device__ __forceinline__ void block_tiles(int bid, int base, int tiles, int tpb, int& t0,
                                            int& t1) {
  t0 = (bid - base) * tpb;
  t1 = min(tiles, t0 + tpb);
}

__global__ __launch_bounds__(256, 1) void k_panel_row(SweepArgs a) {
  const int w = find_window(a, blockIdx.x, true);
  int t0, t1;
  block_tiles(blockIdx.x, a.win[w].base_r, a.win[w].tiles_r, a.tpb_r, t0, t1);
  panel_row_tiles(ctx_of(a, a.win[w]), t0, t1);
}

__global__ __launch_bounds__(256, 1) void k_panel_colq(SweepArgs a) {
  const int w = find_window(a, blockIdx.x, false);
  int t0, t1;
  block_tiles(blockIdx.x, a.win[w].base_cq, a.win[w].tiles_c + a.win[w].tiles_q, a.tpb_cq, t0,
              t1);
  panel_colq_tiles(ctx_of(a, a.win[w]), t0, t1, a.win[w].tiles_c);
}

__global__ __launch_bounds__(256, 1) void k_panel_row_b(const WinB* wins, int nwin) {
  const int w = find_window_b(wins, nwin, blockIdx.x, true);
  int t0, t1;
  block_tiles(blockIdx.x, wins[w].base_r, wins[w].tiles_r, PANEL_TPB_BATCH, t0, t1);
  panel_row_tiles(wins[w].c, t0, t1);
}

__global__ __launch_bounds__(256, 1) void k_panel_colq_b(const WinB* wins, int nwin) {
  const int w = find_window_b(wins, nwin, blockIdx.x, false);
  int t0, t1;
  block_tiles(blockIdx.x, wins[w].base_cq, wins[w].tiles_c + wins[w].tiles_q, PANEL_TPB_BATCH,
              t0, t1);
  panel_colq_tiles(wins[w].c, t0, t1, wins[w].tiles_c);
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
  if (threadIdx.x == 0) *ctrl = Ctrl{};   // every field of a solve starts at zero
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
    if (!isfinite(sub) || !isfinite(tst)) atomicOr(&ctrl->bad, 1);
    if (sub <= kUlp * tst) atomicOr(&bits[k >> 5], 1u << (k & 31));
  }
  __syncthreads();
  // zeros written only after every test has read the original neighbours
  for (int k = klo + 1 + tid; k <= kbot; k += DEFL_THREADS)
    if (bits[k >> 5] & (1u << (k & 31))) H[k + (size_t)(k - 1) * ldh] = 0.0;
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
    if (!isfinite(sub) || !isfinite(tst)) atomicOr(&T.out->bad, 1);
    if (sub <= kUlp * tst) atomicOr(&bits[k >> 5], 1u << (k & 31));
  }
  __syncthreads();
  // zeros written only after every test has read the original neighbours
  for (int k = 1 + tid; k <= kbot; k += 256)
    if (bits[k >> 5] & (1u << (k & 31))) H[k + (size_t)(k - 1) * ldh] = 0.0;
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

void launch_reorder(const ReorderTask* tasks, int count, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL((k_reorder<SMALL_Z_MAX>), dim3(count), dim3(64), 0, s, tasks);
}

void launch_split(const SplitTask* tasks, int count, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL((k_split<SMALL_Z_MAX>), dim3(count), dim3(64), 0, s, tasks);
}

void launch_split_commit(const SplitCommit* cm, int count, const SplitTask* tasks, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_split_commit, dim3(count), dim3(256), 0, s, cm, tasks);
}

void launch_split_scan(double* H, int ldh, int n, unsigned char* zero, hipStream_t s) {
  if (n > 0) {
    const int blocks = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_split_scan, dim3(blocks), dim3(256), 0, s, (const double*)H, ldh, n,
                       zero);
    hipLaunchKernelGGL(k_split_zero, dim3(blocks), dim3(256), 0, s, H, ldh, n,
                       (const unsigned char*)zero);
  }
}

void launch_slot_ident(double* U, const int* sizes, int count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_slot_ident, dim3(16, count), dim3(256), 0, s, U, sizes);
}

void launch_slot_transpose(const double* src, double* dst, int count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_slot_transpose, dim3(16, count), dim3(256), 0, s, src, dst);
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

void launch_panel_row(const SweepArgs& a, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_panel_row, dim3(blocks), dim3(256), 0, s, a);
}

void launch_panel_colq(const SweepArgs& a, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_panel_colq, dim3(blocks), dim3(256), 0, s, a);
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

void launch_panel_row_b(const WinB* wins, int nwin, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_panel_row_b, dim3(blocks), dim3(256), 0, s, wins, nwin);
}

void launch_panel_colq_b(const WinB* wins, int nwin, int blocks, hipStream_t s) {
  if (blocks > 0) hipLaunchKernelGGL(k_panel_colq_b, dim3(blocks), dim3(256), 0, s, wins, nwin);
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
