// kernels.h -- host-visible launch wrappers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "schur_internal.h"

namespace schur {

// One small block solved inside a single workgroup (LDS resident).
struct SmallTask {
  double* A; int lda; int m;   // block, overwritten by its Schur form (Z mode)
  double* Z; int ldz;          // optional: Z (m x m) written column-major
  double* Zt; int ldzt;        // optional: Z^T written into a ldzt x ldzt slot, zero padded
  double* wr; double* wi;      // optional: eigenvalues of the block
  int* info;                   // optional: 0, or 1-based end of a non-converged block
  int itmax;                   // Francis steps per deflation (<= 0: 30 max(10, m))
  double* Qacc; int ldqacc;    // optional: Qacc(0:m, 0:m) <- Qacc(0:m, 0:m) Z
};

// Aggressive early deflation on the window H(kbot-nw+1:kbot, same) of the
// active block [ktop, kbot]; nw <= SMALL_Z_MAX.
struct AedTask {
  double* H; int ldh;
  int ktop, kbot, nw;
  double* Ut; int ldut;        // V^T of the window, zero padded to ldut x ldut
  double* sr; double* si;      // eigenvalues of the undeflated part (nu entries)
  double* wr; double* wi;      // optional: final eigenvalues, indexed from the window top
  Ctrl* ctrl;                  // aed_nd, aed_nu
  int itmax;
};

// Outcome of one window of a parallel early-deflation pass.
struct SplitRes {
  int split;                   // 1: the window was transformed (V^T in its slot)
  int nu, nf, nb;              // rows coupled upward, free (deflated), coupled downward
  double ftop, fbot;           // factors of the new coupling entries above / below
};

// One window H(a:a+nw, a:a+nw) of a parallel early-deflation pass over the
// unreduced blocks of H; nw <= SMALL_Z_MAX.  Windows of one pass tile the
// unreduced blocks without overlap.
struct SplitTask {
  double* H; int ldh;
  int a, nw;
  int above;                   // >= 0: the block continues above the window (coupling H(a, a-1))
  int below;                   // 1: the block continues below the window
  int itmax;
  int pad;
  double* Ut; int ldut;        // V^T of the window, zero padded to ldut x ldut
  SplitRes* res;               // this window's outcome
  double* Wo; int ldwo;        // optional: the new window goes here instead of into H
  int pad2;
};

// A window of a pass whose result is written into H (windows of one commit
// launch are disjoint).
struct SplitCommit {
  int task;                    // index into the pass's SplitTask array
  int above;                   // committed window ending at row a-1 (-1: none)
  int fix_top;                 // 1: scale H(a, a-1) (coupling above the window)
  int fix_below;               // 1: scale H(a+nw, a+nw-1) (no committed window below)
};

// One diagonal window S(a:a+w, a:a+w) of a real Schur form (standardised
// 1x1 / 2x2 blocks; the window starts and ends at block boundaries) in
// eigenvalue reordering.  The selected rows (flag 1 in sel[a .. a+w)) form
// whole blocks; the window task moves them to the top of the window,
// keeping their order, by swaps of adjacent diagonal blocks, and writes the
// window's orthogonal factor (transposed) to Ut.  w <= SMALL_Z_MAX.
struct ReorderTask {
  double* S; int lds;
  int a, w;
  unsigned char* sel;          // per row of S: 1 = selected (updated in place)
  double* Ut; int ldut;        // U^T of the window, zero padded to ldut x ldut
  int* info;                   // set to 1 when a swap is rejected
  int pad;
};

// One matrix of a batched deflation scan.
struct DeflB {
  double* H; double* Q; double* wr; double* wi;
  int ldh, ldq, n, kbot;       // kbot: current bottom of the unreduced part
  Ctrl* out;                   // kbot / ktop after the converged bottom blocks are peeled
};

// One matrix of a batched shift preparation.
struct ShiftB {
  const double* wr; const double* wi;   // eigenvalues of the trailing block
  const int* info;                      // its small-solve info (may be null)
  const double* H; double* st;
  int ns, exceptional, ldh, ktop, kbot, pad;
};

void launch_small_z(const SmallTask& t, const SmallTask* tasks, int count, int maxm,
                    hipStream_t s);
void launch_small_eig(const SmallTask& t, hipStream_t s);
void launch_small_eig_b(const SmallTask* tasks, int count, int maxm, hipStream_t s);
void launch_aed(const AedTask& t, hipStream_t s);
void launch_aed_b(const AedTask* tasks, int count, hipStream_t s);
void launch_split(const SplitTask* tasks, int count, hipStream_t s);
void launch_reorder(const ReorderTask* tasks, int count, hipStream_t s);
void launch_split_commit(const SplitCommit* cm, int count, const SplitTask* tasks, hipStream_t s);
void launch_split_scan(double* H, int ldh, int n, unsigned char* zero, hipStream_t s);
void launch_slot_ident(double* U, const int* sizes, int count, hipStream_t s);
void launch_slot_transpose(const double* src, double* dst, int count, hipStream_t s);
void launch_shift_prep(const double* wr, const double* wi, int ns, const int* small_info,
                       int exceptional, const double* H, int ldh, int ktop, int kbot, double* st,
                       hipStream_t s);
void launch_chase(const SweepArgs& a, hipStream_t s);
void launch_panel_row(const SweepArgs& a, int blocks, hipStream_t s);
void launch_panel_colq(const SweepArgs& a, int blocks, hipStream_t s);
void launch_panel_rowq(const SweepArgs& a, int row_blocks, const SweepArgs& aq, int q_blocks,
                       hipStream_t s);
void launch_check_finite(const double* H, int ldh, int n, Ctrl* ctrl, hipStream_t s);
void launch_zero_lower(double* H, int ldh, int n, hipStream_t s);
void launch_ctrl_reset(Ctrl* ctrl, hipStream_t s);
void launch_set_identity(double* Q, int ldq, int n, hipStream_t s);
void launch_deflate(double* H, int ldh, int kbot, int klo, Ctrl* ctrl, hipStream_t s);
void launch_standardize(double* H, int ldh, double* Q, int ldq, int n, int kmin, double* wr,
                        double* wi, int* list, int* count, int cap, hipStream_t s);

// batched (descriptor arrays in device memory)
void launch_small_tasks(const SmallTask* tasks, int count, int maxm, bool wantz, hipStream_t s);
void launch_chase_b(const WinB* wins, int nwin, hipStream_t s);
void launch_panel_row_b(const WinB* wins, int nwin, int blocks, hipStream_t s);
void launch_panel_colq_b(const WinB* wins, int nwin, int blocks, hipStream_t s);
void launch_deflate_b(const DeflB* tasks, int count, hipStream_t s);
void launch_shift_prep_b(const ShiftB* tasks, int count, hipStream_t s);

}  // namespace schur
