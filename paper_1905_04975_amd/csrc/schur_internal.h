// schur_internal.h -- device/host shared definitions of the MI355X Schur engine.
//
// The engine computes the real Schur form H = Q S Q^T of an upper Hessenberg
// matrix (paper Sec. 2, Eq. (4)) with small-bulge multishift QR sweeps: shifts
// from a trailing block start chains of 3x3 bulges that are chased down the
// diagonal with overlapping 3x3 Householder reflectors (Sec. 3.2); the
// reflectors are first applied inside small diagonal windows, accumulated into
// an orthogonal factor U per window, and U is then applied to the off-diagonal
// panels and to Q as level-3 (matrix-matrix) updates (Sec. 3.2, Fig. 1(b)).
// Several diagonal windows are processed at once (Sec. 3.2, Fig. 1(d)).
//
// All matrices are FP64 and column-major with a leading dimension.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace schur {

// ---- limits ---------------------------------------------------------------
constexpr int WMAX = 128;          // largest diagonal window (rows = cols)
constexpr int LDW = WMAX + 1;      // padded LDS leading dimension of a window
constexpr int NBMAX = 24;          // bulges per group (one window chain)
constexpr int MAXWIN = 32;         // windows processed by one launch
constexpr int UPAD = WMAX;         // leading dimension of the U slots
constexpr int SMALL_Z_MAX = 96;    // block order solved in LDS with its Z
constexpr int SMALL_EIG_MAX = 128; // block order solved in LDS, eigenvalues only
constexpr int GEMM_T = 64;         // panel tile edge (rows or columns)
constexpr int LD_MAX = 1 << 20;    // largest leading dimension (a panel tile's byte range)
constexpr int PANEL_TPB = 8;       // most panel tiles per workgroup (one load of U)
constexpr int PANEL_TPB_BATCH = 4; // panel tiles per workgroup: launches of the round engine
constexpr int PANEL_TPB_WIDE = 8;  // ... launches of many windows (passes, finish, reordering)
constexpr int REFL_LDS = 1280;     // reflectors (chain step x bulge) logged in LDS per window

// ---- one diagonal window of a sweep (a "window task") -----------------------
struct Win {
  int p, ws;          // window rows/cols [p, p+ws)
  int tau0, tau1;     // chain steps covered by this window
  int nb;             // bulges in this window's group
  int shift0;         // first bulge shift pair of the group (index into st)
  int slot;           // U / reflector slot
  int tiles_r;        // row-panel tiles  (columns pe+1 .. ncol-1)
  int tiles_c;        // column-panel tiles (rows rtop .. p-1)
  int tiles_q;        // Q tiles (rows 0 .. n-1)
  int base_r;         // prefix of panel_blocks(tiles_r, tpb_r) over the windows
  int base_cq;        // prefix of panel_blocks(tiles_c + tiles_q, tpb_cq) over the windows
};

struct SweepArgs {
  double* H; int ldh;
  double* Q; int ldq;       // Q may be null
  int n;                    // matrix order
  int ktop, kbot;           // active unreduced block (0-based, inclusive)
  int rtop;                 // first row of column-panel updates (0 for Schur form)
  int cend;                 // one past the last column of row-panel updates (n)
  const double* st;         // shift pairs: st[2b] = s1 + s2, st[2b+1] = s1 * s2
  double* U;                // U slots, each UPAD x UPAD, zero padded
  double* refl;             // reflector slots (v2, v3, tau) per chain step & bulge
  int refl_stride;          // doubles per reflector slot
  int nwin;
  int tpb_r, tpb_cq;        // panel tiles per workgroup of the row and column/Q launches
  Win win[MAXWIN];
};

// ---- everything one window task (and its panel tiles) needs ----------------
struct WinCtx {
  double* H;                // matrix, column-major
  double* Q;                // Schur vectors or null
  double* U;                // this window's U^T slot (UPAD x UPAD, zero padded)
  const double* st;         // shift pairs of the window's group, first pair
  int ldh, ldq, n;
  int ktop, kbot;           // active block of the sweep
  int rtop, cend;           // column-panel first row, row-panel end column
  int p, ws, tau0, tau1, nb;
};

// ---- batched form: windows of many matrices in one launch ------------------
struct WinB {
  WinCtx c;
  int tiles_r, tiles_c, tiles_q;
  int base_r, base_cq;      // workgroup prefixes over the launch's windows (ascending)
  int tpb;                  // panel tiles per workgroup of this window
};

// workgroups of a panel launch that cover `tiles` tiles of one window, tpb
// tiles per workgroup
__host__ __device__ inline int panel_blocks(int tiles, int tpb) {
  return (tiles + tpb - 1) / tpb;
}

// ---- small control block kept in device memory ----------------------------
struct Ctrl {
  int kbot;        // bottom of the active block after bottom deflation (-1: done)
  int ktop;        // top of the unreduced block ending at kbot
  int ndefl;       // number of eigenvalues peeled off at the bottom this scan
  int bad;         // non-finite entry seen in the input scan
  int small_info;  // convergence failure in a small-block solve (1-based), 0 ok
  int nshift;      // shifts produced for the next sweep
  int aed_nd;      // eigenvalues deflated by the last early-deflation window
  int aed_nu;      // undeflated eigenvalues of that window (shift candidates)
};

}  // namespace schur
