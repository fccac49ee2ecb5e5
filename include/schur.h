/*
 * schur.h -- C ABI of the MI355X (gfx950) Schur-reduction engine.
 *
 * The library reduces an upper Hessenberg matrix H to real Schur form
 *
 *     H = Q2 S Q2^T,
 *
 * with Q2 orthogonal and S upper quasi-triangular with 1x1 and 2x2 diagonal
 * blocks; the eigenvalues are read from the diagonal blocks (paper Sec. 2,
 * Eq. (4), "Schur reduction").  The eigenvector step backtransforms with the
 * product Q1 Q2 (Sec. 2, Eq. (6)), so Q is accumulated: Q <- Q_in Q2.
 *
 * Method (Sec. 3.2): multishift QR sweeps with small bulges.  Shifts are the
 * eigenvalues of a trailing block; chains of 3x3 bulges are chased down the
 * diagonal with overlapping 3x3 Householder reflectors, first inside small
 * diagonal windows whose orthogonal factors are accumulated, then applied to
 * the off-diagonal panels and to Q as matrix-matrix products.  All arithmetic
 * is IEEE binary64.
 *
 * Conventions (LAPACK/ScaLAPACK style, which the paper keeps compatibility
 * with, Sec. 4.2):
 *   - matrices are column-major with a leading dimension: element (i, j) of
 *     H is H[i + j*ldh], 0-based;
 *   - pointers named H, Q, wr, wi are DEVICE pointers (memory of the current
 *     HIP device, e.g. a torch tensor's data_ptr()), unless stated otherwise;
 *   - streams are passed as `void*` holding a hipStream_t; NULL is the null
 *     (default) stream itself, so work the caller queued there (for example
 *     on PyTorch's default stream) is ordered before the call's work;
 *   - return value `info`:
 *         0      success
 *        -i      argument i is illegal (1-based position in the argument
 *                list of schur_reduce: n -> -1, H -> -2, ldh -> -3, Q -> -4,
 *                ldq -> -5, wr -> -6, wi -> -7).  A non-finite entry in the
 *                Hessenberg part of H is reported as -2 and nothing is
 *                modified.
 *        >0      the QR iteration did not converge within the sweep limit;
 *                info is the 1-based last row of the unreduced block that
 *                failed.  wr/wi rows info+1..n hold the eigenvalues that
 *                converged, and H_in = Q S Q^T still holds for the returned
 *                (non-triangular) S.
 *       <=-100   runtime failure: -101 out of device memory, -102 HIP error,
 *                -103 pointer is not device memory, -104 bad handle,
 *                -105 a non-finite value appeared during the iteration
 *                (an internal failure; H and Q are then unspecified),
 *                -106 n above the maximum of schur_reduce_noalloc.
 *   - entries of H below the first subdiagonal are ignored on input and are
 *     exactly zero on output; S's 2x2 blocks are standardised (equal diagonal
 *     entries, off-diagonal entries of opposite sign, i.e. a complex pair);
 *     real eigenvalue pairs always appear as two 1x1 blocks;
 *   - wr/wi are in the diagonal order of S; a conjugate pair is adjacent with
 *     the positive imaginary part first.
 *   - ownership: the caller owns every buffer passed in; the library never
 *     frees or keeps them beyond the call (async calls: until the stream
 *     reaches the end of the enqueued work).  A handle owns its workspace.
 *   - threading: a handle must not be used by two threads at once.
 */
#ifndef SCHUR_MI355X_H
#define SCHUR_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct schur_handle_s* schur_handle_t;

/* Tuning options; zero fields take the built-in defaults (per-n table). */
typedef struct schur_opts {
  int ns;          /* shifts per sweep (even, <= 256); 0 = by table. Above 128 */
                   /* the trailing block that supplies them is reduced by a    */
                   /* nested solve of this engine (no Schur vectors)           */
  int nb;          /* bulges per window chain (group), 1..24; 0 = by table     */
  int step;        /* chain steps per window; 0 = largest that fits 128 rows   */
  int nmin;        /* active blocks of order <= nmin are solved in one kernel  */
  int max_sweeps;  /* sweep limit per solve; 0 = 30 * max(10, n)/max(2, ns)    */
  int exc_period;  /* sweeps without deflation before ad-hoc shifts; 0 = 6     */
  int flags;       /* SCHUR_FLAG_*                                             */
  int aed_window;  /* early-deflation window order (<= 96); 0 = from ns,       */
                   /* < 0 = no early deflation (shifts from the trailing block) */
  int aed_nibble;  /* a window that deflated more than this percentage of its  */
                   /* rows is followed by another window instead of a sweep;   */
                   /* 0 = by table, < 0 = always sweep                        */
  int split_window; /* parallel early deflation: window order (<= 96) of the   */
                    /* passes that deflate on windows tiling every unreduced   */
                    /* block at once before the sweeps (the early-deflation    */
                    /* step of paper Sec. 3.2 applied to interior windows);    */
                    /* 0 = 96, < 0 = off.  Single solves and members of        */
                    /* batched calls use them; the server does not             */
  int split_min_n;  /* smallest order that starts with those passes;          */
                    /* 0 = 2048                                                */
  int panel_tile;   /* panel products of the sweeps: tiles (64 columns or rows of */
                    /* the panel) per workgroup, i.e. the workgroup's output   */
                    /* tile is ws x 64*panel_tile; 1..8, 0 = by table, else a  */
                    /* per-launch cost model                                   */
} schur_opts;

#define SCHUR_FLAG_TIME_KERNELS 1   /* time each kernel family with HIP events */
#define SCHUR_FLAG_BATCH_ROUNDS 2   /* schur_reduce_batched and the server: every      */
                                    /* matrix through the round engine (no persistent  */
                                    /* kernel)                                         */
#define SCHUR_FLAG_ONE_STREAM 4     /* single solves: the Q products on the solve      */
                                    /* stream too (no overlap with the window chase),  */
                                    /* so each kernel's timed duration is its own; a   */
                                    /* time step's Q products share one launch with    */
                                    /* its row-panel products (same result bit for     */
                                    /* bit)                                            */

/* Counters of the last solve on a handle. */
typedef struct schur_stats {
  int64_t sweeps;           /* multishift sweeps                               */
  int64_t windows;          /* diagonal windows chased                         */
  int64_t chain_steps;      /* window chain steps (all windows)                */
  int64_t small_solves;     /* blocks finished by the single-kernel solver      */
  int64_t launches;         /* kernel launches                                 */
  double gemm_flops;        /* flops of the panel matrix products               */
  double gemm_ms;           /* summed duration of the panel kernels (TIME flag) */
  int64_t gemm_launches;    /* number of panel kernel launches                 */
  double chase_ms;          /* summed duration of the window kernels (TIME)    */
  int64_t chase_launches;
  double shift_ms;          /* summed duration of the shift kernels (TIME)     */
  double other_ms;          /* deflation, standardisation, small solves (TIME) */
  int64_t shifts_applied;   /* total shifts used in sweeps                     */
  double row_flops;         /* flops of the row-panel (left) products          */
  double row_ms;            /* summed duration of k_panel_row launches (TIME)  */
  int64_t row_launches;
  double colq_flops;        /* flops of the column-panel and Q (right) products */
  double colq_ms;           /* summed duration of k_panel_colq launches (TIME) */
  int64_t colq_launches;
  double aed_ms;            /* summed duration of the early-deflation kernels   */
  int64_t aed_windows;      /* early-deflation windows processed               */
  int64_t aed_deflated;     /* eigenvalues deflated by them                    */
  double aed_flops;         /* nominal work of those windows: 25 nw^3 (Schur   */
                            /* form with vectors) + 10/3 nu^3 (reduction back) */
  int64_t split_passes;     /* parallel early-deflation passes                  */
  int64_t split_windows;    /* windows of those passes                          */
  int64_t split_accepted;   /* windows that split their block (V applied)       */
  int64_t split_converged;  /* rows in converged 1x1 / 2x2 blocks after them    */
  double split_ms;          /* summed duration of their window kernels (TIME)  */
  double split_flops;       /* nominal work of their windows (as aed_flops)    */
  double small_ms;          /* summed duration of the small-block solves (TIME) */
  double small_flops;       /* their nominal work: 25 m^3 per block of order m  */
                            /* with Schur vectors, 10 m^3 for eigenvalues only  */
                            /* (shift solves)                                   */
  double chase_flops;       /* counted work of the window chases: 10 flops per  */
                            /* touched row or column and reflector, for the    */
                            /* left and right updates in the window and the    */
                            /* accumulation of U                                */
  int64_t small_launches;   /* launches of the small-block solver (each may     */
                            /* carry many blocks)                               */
  int64_t aed_launches;     /* launches of the early-deflation kernels          */
  /* schur_hessenberg */
  double hess_panel_ms;     /* summed duration of the panels' column kernels    */
                            /* (TIME)                                           */
  double hess_gemv_bytes;   /* bytes of the trailing matrix streamed by the     */
                            /* matrix-vector products (8 per entry and column)  */
  double hess_gemm_ms;      /* summed duration of the panels' products (TIME)   */
  double hess_gemm_flops;   /* flops of those products                          */
  /* schur_eigenvectors */
  double ev_solve_ms;       /* summed duration of the tile solves (TIME)        */
  double ev_gemm_ms;        /* summed duration of the tile-row updates (TIME)   */
  double ev_gemm_flops;     /* flops of those updates                           */
  double ev_back_ms;        /* duration of the backtransform product (TIME)     */
  double ev_back_flops;     /* its flops (2 n^3)                                */
  /* schur_reorder */
  double reorder_ms;        /* summed duration of the window tasks (TIME)       */
  int64_t reorder_windows;  /* windows processed                                */
  int64_t reorder_steps;    /* time steps (launches of window tasks)            */
  double chase_bytes;       /* algorithmic HBM bytes of the window chases: the  */
                            /* window read and written back and its factor U   */
                            /* written, 24 ws^2 per window of order ws         */
  /* schur_reduce_batched */
  double persist_ms;        /* duration of the persistent kernel (TIME)         */
  int64_t persist_jobs;     /* matrices it solved                               */
} schur_stats;

/* --------------------------------------------------------------------------
 * schur_reduce -- synchronous Schur reduction (paper Sec. 2, Eq. (4)).
 *   n        order, n >= 0
 *   H        device, ldh x n; in: upper Hessenberg; out: S
 *   ldh      max(1, n) <= ldh <= 1048576 (2^20: a panel tile of up to 128
 *            columns is addressed through one buffer descriptor of under
 *            2^30 bytes)
 *   Q        device, ldq x n or NULL; in: Q_in; out: Q_in Q2 (NULL: no
 *            Schur vectors, the Q products are skipped)
 *   ldq      max(1, n) <= ldq <= 1048576 when Q != NULL
 *   wr, wi   device, n doubles each
 * Uses a per-device default handle; runs on the null stream after the
 * work already there and blocks until done.
 * ------------------------------------------------------------------------ */
int schur_reduce(int n, double* H, int ldh, double* Q, int ldq, double* wr, double* wi);

/* Handle with its own stream and workspace on `device` (opts may be NULL). */
int schur_create(schur_handle_t* h, int device, const schur_opts* opts);
int schur_destroy(schur_handle_t h);
int schur_set_opts(schur_handle_t h, const schur_opts* opts);
int schur_get_stats(schur_handle_t h, schur_stats* out);

/* --------------------------------------------------------------------------
 * schur_reduce_async -- stream-ordered Schur reduction.
 * All device work is enqueued on `stream` after the work already there and
 * nothing else is synchronised; the host thread drives the sweep loop and
 * waits on `stream` for the few control integers each sweep needs, so the
 * call returns once the last kernel has been enqueued.  The results (and
 * *info_out, a HOST int) are final when the call returns; the output buffers
 * are written by work on `stream`.
 * ------------------------------------------------------------------------ */
int schur_reduce_async(schur_handle_t h, void* stream, int n, double* H, int ldh, double* Q,
                       int ldq, double* wr, double* wi, int* info_out);

/* --------------------------------------------------------------------------
 * schur_hessenberg -- Hessenberg reduction A = Q1 H Q1^T (paper Sec. 2,
 * Eq. (3)), the step before the Schur reduction: H = schur_hessenberg(A),
 * then schur_reduce(H, Q) with the same Q gives A = (Q1 Q2) S (Q1 Q2)^T.
 *   h        handle (its workspace; stream NULL = the null stream)
 *   n        order, n >= 0
 *   A        device, lda x n; in: dense A; out: H (upper Hessenberg, exact
 *            zeros below the first subdiagonal)
 *   lda      >= max(1, n)
 *   Q        device, ldq x n or NULL; in: Q_in; out: Q_in Q1 (pass the
 *            identity to get Q1; Q1 e_1 = e_1)
 *   ldq      >= max(1, n) when Q != NULL
 * Blocked Householder reflectors, panels of 32 columns; the new subdiagonal
 * entry of a column is -sign(x_1) ||x|| (the LAPACK convention).  All work is
 * enqueued on the stream in order and the call returns without waiting for
 * it (workspace growth aside); results are final when the stream reaches
 * them.  Returns 0, -1 (n), -2 (A), -3 (lda), -5 (ldq), -101 (device
 * memory), -102 (HIP error), -103 (not device memory), -104 (handle).
 * ------------------------------------------------------------------------ */
int schur_hessenberg(schur_handle_t h, void* stream, int n, double* A, int lda, double* Q,
                     int ldq);

/* --------------------------------------------------------------------------
 * schur_eigenvectors -- eigenvectors of a real Schur form and their
 * backtransform (paper Sec. 2, Eqs. (5) and (6)), the step after the Schur
 * reduction: with S and Q = Q1 Q2 from schur_hessenberg and schur_reduce,
 * X holds the eigenvectors of A.
 *   h        handle (its workspace; stream NULL = the null stream)
 *   n        order, n >= 0
 *   S        device, lds x n, read only: a standardised real Schur form (as
 *            schur_reduce returns it: 2x2 blocks with equal diagonal and
 *            off-diagonal entries of opposite sign, exact zeros elsewhere
 *            below the diagonal)
 *   lds      >= max(1, n)
 *   Q        device, ldq x n or NULL, read only: X = Q Y (NULL: X = Y, the
 *            eigenvectors of S)
 *   ldq      >= max(1, n) when Q != NULL
 *   X        device, ldx x n, output (must not overlap S or Q): LAPACK's
 *            real layout -- column k a real eigenvector, columns k and k+1
 *            the real and imaginary parts of the eigenvector of the
 *            eigenvalue with positive imaginary part of the 2x2 block at
 *            rows k, k+1; each eigenvector scaled to largest |Re| + |Im| = 1
 *   ldx      >= max(1, n)
 * Conventions (LAPACK's): y(p) = 1 at the row p of a real eigenvalue,
 * zeros below; for a pair (y(p), y(p+1)) = (1, i wi / S(p,p+1)) when
 * |S(p,p+1)| >= |S(p+1,p)|, else (-wi / S(p+1,p), i); pivots smaller than
 * max(ulp |lambda|, tiny) are raised to that.  Overflow protection: every
 * vector is scaled down before a division or update could pass ~2^960.
 * Work is enqueued on the stream after one read of S's subdiagonal (a
 * synchronisation) that places the tiles; results are final when the stream
 * reaches them.  With Q the handle keeps an n x n workspace.  Returns 0,
 * -1 (n), -2 (S), -3 (lds), -5 (ldq), -6 (X), -7 (ldx), -101, -102, -103,
 * -104.
 * ------------------------------------------------------------------------ */
int schur_eigenvectors(schur_handle_t h, void* stream, int n, const double* S, int lds,
                       const double* Q, int ldq, double* X, int ldx);

/* --------------------------------------------------------------------------
 * schur_reorder -- eigenvalue reordering (paper Sec. 2, Eq. (7)): an
 * orthogonal Q3 with S = Q3 S' Q3^T, S' a standardised real Schur form whose
 * leading m x m block carries exactly the selected eigenvalues, keeping
 * their diagonal order; Q <- Q Q3.  With S and Q = Q1 Q2 from the previous
 * steps, the first m columns of Q span the invariant subspace of A for the
 * selected eigenvalues.
 *   h        handle (its workspace; stream NULL = the null stream)
 *   n        order, n >= 0
 *   S        device, lds x n; in: a standardised real Schur form (as
 *            schur_reduce returns it); out: S'
 *   lds      max(1, n) <= lds <= 1048576 (as ldh of schur_reduce)
 *   Q        device, ldq x n or NULL; in: Q_in; out: Q_in Q3
 *   ldq      max(1, n) <= ldq <= 1048576 when Q != NULL
 *   select   HOST, n ints: select[k] != 0 selects eigenvalue k (either row
 *            of a 2x2 block selects the pair)
 *   wr, wi   device, n doubles each: the eigenvalues of S' (diagonal order)
 *   m        HOST int or NULL: the number of selected eigenvalues
 * Method (Sec. 3.2): chunks of at most 32 selected rows travel to the top
 * through chains of diagonal windows (at most 96 rows, in LDS) in which
 * adjacent blocks are swapped (2x2 and 3x3 / 4x4 Householder reflectors from
 * the Sylvester equation of the two blocks), each window's factor applied
 * to the rest of S and to Q as FP64 MFMA products; chains of later chunks
 * follow a few time steps behind.  Returns 0; 1 when a swap was rejected as
 * unstable (eigenvalues too close to separate, LAPACK's convention: S and Q
 * are then a valid but only partly reordered pair); -1 (n), -2 (S),
 * -3 (lds), -5 (ldq), -6 (select), -7 (wr), -8 (wi), -101, -102, -103, -104.
 * Synchronises at the start (S's subdiagonal, for the plan) and at the end.
 * ------------------------------------------------------------------------ */
int schur_reorder(schur_handle_t h, void* stream, int n, double* S, int lds, double* Q, int ldq,
                  const int* select, double* wr, double* wi, int* m);

/* --------------------------------------------------------------------------
 * Reordering schedule (host-only diagnostic of the library's planner, no
 * device work): for blocks of orders bsize[i] (1 or 2, summing to n) with
 * selection flags bsel[i], the window chains of schur_reorder.  Writes up
 * to `cap` records of 4 ints (chain, time step, first row, order) to `out`;
 * returns the number of windows (which may exceed cap) or -1.
 * ------------------------------------------------------------------------ */
int schur_plan_reorder(int n, const int* bsize, const int* bsel, int nblocks, int* out, int cap);

/* --------------------------------------------------------------------------
 * schur_reduce_noalloc -- the Schur reduction of schur_reduce for callers
 * that cannot allocate memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  It calls no hipMalloc, hipFree,
 * hipHostMalloc or other allocating device routine, creates no stream or
 * event, and takes its workspace from a static device array of
 * SCHUR_NOALLOC_SCRATCH_BYTES (about 6.6 MB) that each GPU it runs on holds
 * until the process ends.  Host-side planning uses ordinary C++ containers.
 *   stream   hipStream_t as void* (NULL = the null stream); all device work
 *            runs on it, in order
 *   n        0 <= n <= SCHUR_NOALLOC_MAX_N; larger orders return -106
 *            (the workspace holds the block list of at most that order)
 *   H, ldh, Q, ldq, wr, wi   as in schur_reduce (device pointers of the
 *            current device; the caller passes inputs and outputs)
 * Differences from schur_reduce: no parallel early-deflation passes (their
 * per-window workspace is not in the array), at most 128 shifts per sweep
 * (no nested shift solve), one stream (the Q products are not overlapped
 * with the window chase).  Returns like schur_reduce; the results are final
 * when it returns.  Every call on a device shares that device's array, which
 * keeps the last call's contents (the control block is cleared at the start
 * of each call); calls from several host threads on one device are
 * serialised by the library, calls from several processes use separate
 * arrays.
 * ------------------------------------------------------------------------ */
#define SCHUR_NOALLOC_MAX_N 32768
#define SCHUR_NOALLOC_SCRATCH_BYTES 6632192
int schur_reduce_noalloc(void* stream, int n, double* H, int ldh, double* Q, int ldq,
                         double* wr, double* wi);

/* --------------------------------------------------------------------------
 * schur_reduce_begin / schur_reduce_end -- the Schur reduction of
 * schur_reduce_async (paper Sec. 2, Eq. (4)) without holding the caller's
 * thread.  schur_reduce_begin checks the arguments (host-side), marks the
 * current point of `stream` and returns at once; a thread owned by the
 * handle then runs the solve on the handle's own stream after that point
 * (the sweep loop needs the host between sweeps, so it cannot be captured
 * into one stream submission) and finally writes the info code to
 * *info_dev (a DEVICE int, may be NULL) on that stream.  schur_reduce_end
 * waits for that thread, makes `stream` wait for the solve's device work
 * (an event wait: work enqueued on `stream` afterwards sees S, Q, wr, wi
 * and *info_dev) and returns the info code.
 *   arguments as schur_reduce_async; info_dev: device int or NULL
 * Between the two calls the handle and the buffers must not be used
 * otherwise (the handle is busy: a second begin returns -104).  begin
 * returns 0 or an argument error (nothing started then); end returns the
 * solve's info, or -104 when no solve was begun.
 * ------------------------------------------------------------------------ */
int schur_reduce_begin(schur_handle_t h, void* stream, int n, double* H, int ldh, double* Q,
                       int ldq, double* wr, double* wi, int* info_dev);
int schur_reduce_end(schur_handle_t h, void* stream);

/* --------------------------------------------------------------------------
 * schur_reduce_batched -- many independent Hessenberg matrices of uneven
 * orders in one call.  n, ldh, ldq are HOST arrays of `count` ints; H, Q,
 * wr, wi are HOST arrays of `count` DEVICE pointers (Q[i] may be NULL,
 * or Q itself NULL for no Schur vectors).  info is a HOST array of `count`
 * ints receiving each matrix's info.  Matrices of order <= 1024 are solved by
 * one persistent launch: a grid of one workgroup per CU takes them from a
 * queue, largest first, and each workgroup runs a whole Schur reduction on
 * the device (early deflation, shifts, bulge chains chased through LDS
 * windows, FP64 MFMA panel products; paper Sec. 3.2) with no host round
 * trip.  Larger matrices (or all of them, with SCHUR_FLAG_BATCH_ROUNDS) are
 * advanced sweep by sweep with the windows and panel tiles of all of them in
 * shared launches (matrices of order <= 96 one per workgroup).
 * Returns 0 when every matrix succeeded, else the first nonzero info.
 * ------------------------------------------------------------------------ */
int schur_reduce_batched(schur_handle_t h, void* stream, int count, const int* n,
                         double* const* H, const int* ldh, double* const* Q, const int* ldq,
                         double* const* wr, double* const* wi, int* info);

/* --------------------------------------------------------------------------
 * Tuning table (written by the autotuner).  For a matrix (or active block)
 * of order n, the first entry with n <= nmax[i] supplies the shifts per
 * sweep, bulges per window chain, chain steps per window (0 = largest that
 * fits; with the bulges it sets the diagonal window's order), the
 * early-deflation window (nw: 0 = from ns, < 0 = off, else 4..96), its
 * sweep-skip percentage (nibble: 0 = 14, < 0 = always sweep, else 1..100)
 * and the panel products' tiles per workgroup (tile: 0 = cost model, else
 * 1..8) whenever the handle's options leave them 0; nw, nibble and tile may
 * be NULL for all 0.  Arrays of `count` entries, nmax strictly ascending;
 * host memory, read during the call.  Process-wide; count = 0 restores the
 * built-in table.  Returns 0, -1 (count < 0) or -2 (an entry out of range).
 * Host-only, no device work.
 * ------------------------------------------------------------------------ */
int schur_set_tuning(int count, const int* nmax, const int* ns, const int* nb, const int* step,
                     const int* nw, const int* nibble, const int* tile);

/* --------------------------------------------------------------------------
 * Sweep schedule (host-only diagnostic of the planner, no device work):
 * the lock-step window plan of one sweep over the active block
 * [ktop, kbot] (0-based) with npair bulges in groups of at most nb and at
 * most `step` chain steps per window (0 = largest that fits).  Writes up to
 * `cap` records of 7 ints (time step, group, first row p, order ws, first
 * and one-past-last chain step, bulges) to `out`; returns the number of
 * windows (which may exceed cap), or a negative value on bad arguments.
 * ------------------------------------------------------------------------ */
int schur_plan_sweep(int ktop, int kbot, int npair, int nb, int step, int* out, int cap);

/* --------------------------------------------------------------------------
 * Window tiling of the parallel early-deflation passes (host-only
 * diagnostic of the solver's own code, no device work; the passes apply the
 * early-deflation step of paper Sec. 3.2 to windows inside the matrix): the
 * windows laid over the unreduced block [lo, hi] (0-based) with a bottom
 * window of `first` rows (1 <= first <= nw) and the others of nw rows; a top
 * window shorter than 16 rows and the one below it become two halves.
 * Writes up to `cap` (start, order) pairs, top to bottom, to `out`; returns
 * the number of windows (which may exceed cap) or -1 on bad arguments.
 * ------------------------------------------------------------------------ */
int schur_plan_split(int lo, int hi, int nw, int first, int* out, int cap);

/* --------------------------------------------------------------------------
 * Window selection of a pass (host-only diagnostic of the solver's own
 * code): among `count` candidate windows of one block (start a[i], order
 * w[i] >= 1, weight wt[i] > 0; host arrays) the disjoint set of largest total
 * weight.  Writes the chosen indices in increasing start order to `picked`
 * (room for `count` entries); returns how many were chosen, or -1 on bad
 * arguments.
 * ------------------------------------------------------------------------ */
int schur_select_windows(int count, const int* a, const int* w, const double* wt, int* picked);

/* --------------------------------------------------------------------------
 * Candidate weight of a window of a pass (host-only diagnostic of the
 * solver's own code): split = the window passed its tests, nf = rows it
 * deflated, top / below = 1 when its block continues above / below it.
 * Returns 1 + nf, or 0 when the window is no candidate: it failed its tests,
 * or it sits at an end of its block and deflated nothing (it would neither
 * deflate nor split).  An interior window that deflated nothing still splits
 * its block (weight 1).
 * ------------------------------------------------------------------------ */
double schur_split_weight(int split, int nf, int top, int below);

/* --------------------------------------------------------------------------
 * Serving loop (continuous batching).  A server owns a device handle and a
 * background thread.  Requests (HOST matrices) queue FIFO; between rounds of
 * the batched engine (one sweep per resident matrix per round) the thread
 * admits queued requests while the device bytes of the resident ones (H, Q,
 * wr, wi) stay within `hbm_budget_bytes`, so requests that arrive while
 * others are on the GPU join the next round.  Requests of order <= 256 (all
 * of them go to the round engine with SCHUR_FLAG_BATCH_ROUNDS in the
 * options) are instead solved by a persistent launch per group admitted
 * together, on one of two streams of the server: each by one workgroup from
 * start to end, so its result is the one it gets alone, bit for bit.
 * Finished results are copied to pinned host memory (blocks reused from
 * request to request); latency = submit to results on the host.
 * ------------------------------------------------------------------------ */
typedef struct schur_server_s* schur_server_t;

typedef struct schur_server_stats {
  int64_t submitted, completed, rounds;
  int64_t resident, queued, peak_resident;
  double bytes_in_use, peak_bytes;
  double reserved[4];
} schur_server_stats;

/* opts may be NULL; budget 0 = 64 GiB. */
int schur_server_create(schur_server_t* srv, int device, size_t hbm_budget_bytes,
                        const schur_opts* opts);
/* Finishes queued and resident requests, then stops the thread and frees. */
int schur_server_destroy(schur_server_t srv);
/* H_host: HOST, column-major ldh x n (copied before return).  want_q != 0
 * returns Schur vectors.  *ticket identifies the request.  A request whose
 * device bytes exceed the whole budget completes with info -101. */
int schur_submit(schur_server_t srv, int n, const double* H_host, int ldh, int want_q,
                 uint64_t* ticket);
/* Returns 1 while the request is not done.  When done (return 0) copies S
 * (HOST, lds >= n), Q (HOST, ldq >= n; ignored when NULL or not requested),
 * wr/wi (HOST, n each; may be NULL), *info and *latency_s (may be NULL),
 * and forgets the ticket.  Unknown ticket: -2. */
int schur_poll(schur_server_t srv, uint64_t ticket, double* S_host, int lds, double* Q_host,
               int ldq, double* wr, double* wi, int* info, double* latency_s);
int schur_server_get_stats(schur_server_t srv, schur_server_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* SCHUR_MI355X_H */
