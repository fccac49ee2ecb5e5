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
#include "wg_ops.h"

namespace schur {

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

__global__ __launch_bounds__(256) void k_shift_prep(const double* wr, const double* wi, int ns,
                                                    const int* small_info, int exceptional,
                                                    const double* H, int ldh, int ktop, int kbot,
                                                    double* st) {
  __shared__ ShiftLds lds;
  shift_prep(wr, wi, ns, small_info, exceptional, H, ldh, ktop, kbot, st, lds);
}

__global__ __launch_bounds__(256) void k_shift_prep_b(const ShiftB* tasks) {
  const ShiftB T = tasks[blockIdx.x];
  __shared__ ShiftLds lds;
  shift_prep(T.wr, T.wi, T.ns, T.info, T.exceptional, T.H, T.ldh, T.ktop, T.kbot, T.st, lds);
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
// Panel launches (the products themselves are panel_row_tiles and
// panel_colq_tiles): workgroup bid finds its window by the prefix counts.
// ============================================================================
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
  __shared__ double Xs[2 * WMAX * LDT];
  panel_row_tiles(ctx_of(a, a.win[w]), t0, t1, Xs);
}

__global__ __launch_bounds__(256, 1) void k_panel_colq(SweepArgs a) {
  const int w = find_window(a, blockIdx.x, false);
  int t0, t1;
  block_tiles(blockIdx.x, a.win[w].base_cq, a.win[w].tiles_c + a.win[w].tiles_q, a.tpb_cq, t0,
              t1);
  __shared__ double Xs[2 * WMAX * LDT];
  panel_colq_tiles(ctx_of(a, a.win[w]), t0, t1, a.win[w].tiles_c, Xs);
}

// Row panels of H and Q products of one time step in one launch (they touch
// different matrices): blocks [0, nrb) as k_panel_row over a, the rest as
// k_panel_colq over aq (Q tiles only).
__global__ __launch_bounds__(256, 1) void k_panel_rowq(SweepArgs a, SweepArgs aq, int nrb) {
  __shared__ double Xs[2 * WMAX * LDT];
  const int b = blockIdx.x;
  if (b < nrb) {
    const int w = find_window(a, b, true);
    int t0, t1;
    block_tiles(b, a.win[w].base_r, a.win[w].tiles_r, a.tpb_r, t0, t1);
    panel_row_tiles(ctx_of(a, a.win[w]), t0, t1, Xs);
  } else {
    const int bq = b - nrb;
    const int w = find_window(aq, bq, false);
    int t0, t1;
    block_tiles(bq, aq.win[w].base_cq, aq.win[w].tiles_c + aq.win[w].tiles_q, aq.tpb_cq, t0, t1);
    panel_colq_tiles(ctx_of(aq, aq.win[w]), t0, t1, aq.win[w].tiles_c, Xs);
  }
}

__global__ __launch_bounds__(256, 1) void k_panel_row_b(const WinB* wins, int nwin) {
  const int w = find_window_b(wins, nwin, blockIdx.x, true);
  int t0, t1;
  block_tiles(blockIdx.x, wins[w].base_r, wins[w].tiles_r, wins[w].tpb, t0, t1);
  __shared__ double Xs[2 * WMAX * LDT];
  panel_row_tiles(wins[w].c, t0, t1, Xs);
}

__global__ __launch_bounds__(256, 1) void k_panel_colq_b(const WinB* wins, int nwin) {
  const int w = find_window_b(wins, nwin, blockIdx.x, false);
  int t0, t1;
  block_tiles(blockIdx.x, wins[w].base_cq, wins[w].tiles_c + wins[w].tiles_q, wins[w].tpb, t0,
              t1);
  __shared__ double Xs[2 * WMAX * LDT];
  panel_colq_tiles(wins[w].c, t0, t1, wins[w].tiles_c, Xs);
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

// Batched deflation scan (the operation is deflate_b_wg): one workgroup of
// 256 threads per matrix.
__global__ __launch_bounds__(256) void k_deflate_b(const DeflB* tasks) {
  __shared__ unsigned bits[DB_WORDS];
  __shared__ int s_kt;
  deflate_b_wg(tasks[blockIdx.x], bits, s_kt);
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
void launch_reorder(const ReorderTask* tasks, int count, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL((k_reorder<SMALL_Z_MAX>), dim3(count), dim3(64), 0, s, tasks);
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

void launch_panel_rowq(const SweepArgs& a, int row_blocks, const SweepArgs& aq, int q_blocks,
                       hipStream_t s) {
  if (row_blocks + q_blocks > 0)
    hipLaunchKernelGGL(k_panel_rowq, dim3(row_blocks + q_blocks), dim3(256), 0, s, a, aq,
                       row_blocks);
}

void launch_small_tasks(const SmallTask* tasks, int count, int maxm, bool wantz, hipStream_t s) {
  if (count <= 0) return;
  SmallTask none{};
  if (wantz) {
    launch_small_z(none, tasks, count, maxm, s);
  } else {
    launch_small_eig_b(tasks, count, maxm, s);
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
