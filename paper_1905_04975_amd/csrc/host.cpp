// host.cpp -- sweep driver and C ABI of the MI355X Schur engine.
//
// One solve (paper Sec. 2, Eq. (4)) is a host-driven loop over sweeps of the
// multishift QR algorithm with small bulges (Sec. 3.2):
//   1. deflation scan of the bottom unreduced block (k_deflate), one small
//      device-to-host read of the control block;
//   2. if the block is small, one single-workgroup solve (k_small_z) whose
//      orthogonal factor is applied to the rest of H and to Q as panel
//      products; otherwise
//   3. shifts = eigenvalues of a trailing block (k_small_eig + k_shift_prep),
//      and one sweep: bulge groups chased through diagonal windows in
//      lock-step time steps.  Each time step launches the window tasks of
//      all groups at once (k_chase, disjoint windows), then the left
//      (row-panel) products, then the right (column-panel and Q) products.
//      Stream order gives the sequentially consistent order of window,
//      right-update and left-update tasks (Sec. 3.2, Fig. 2) without any
//      global synchronisation inside a sweep.
//   4. at the end, 2x2 standardisation and (wr, wi) (k_std_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/schur.h"
#include "batch.h"
#include "evec.h"
#include "hess.h"
#include "kernels.h"
#include "schur_internal.h"

using namespace schur;

namespace {

constexpr int NSMAX = 512;             // shifts buffer capacity
constexpr int NS_MAX = 256;            // shifts per sweep; above SMALL_EIG_MAX the trailing
                                       // block is reduced by a nested solve of this engine
constexpr int REFL_STRIDE = WMAX * NBMAX * 3;

struct HipErr {
  hipError_t e;
};

#define HCHECK(x)                          \
  do {                                     \
    hipError_t _e = (x);                   \
    if (_e != hipSuccess) throw HipErr{_e}; \
  } while (0)

// Event-pair timer for kernel families (optional, flag SCHUR_FLAG_TIME_KERNELS).
struct Timer {
  std::vector<hipEvent_t> pool;
  struct Rec { hipEvent_t a, b; double* acc; };
  std::vector<Rec> pending;
  hipEvent_t get() {
    if (pool.empty()) {
      hipEvent_t e;
      HCHECK(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  void begin(hipStream_t s, hipEvent_t& a) {
    a = get();
    HCHECK(hipEventRecord(a, s));
  }
  void end(hipStream_t s, hipEvent_t a, double* acc) {
    hipEvent_t b = get();
    HCHECK(hipEventRecord(b, s));
    pending.push_back({a, b, acc});
  }
  // stream must be synchronised
  void harvest() {
    for (auto& r : pending) {
      float ms = 0.f;
      HCHECK(hipEventElapsedTime(&ms, r.a, r.b));
      *r.acc += ms;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  ~Timer() {
    for (auto& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

constexpr int NBUF = 4;   // ring of U-slot buffers shared by the two streams

struct schur_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;     // Q products run here, overlapping the window chase
  hipEvent_t ev_u[NBUF] = {};    // U slots of a buffer written (main stream)
  hipEvent_t ev_q[NBUF] = {};    // U slots of a buffer read by the Q products (aux stream)
  hipEvent_t ev_join = nullptr;
  schur_opts opts{};
  double* U = nullptr;
  double* refl = nullptr;
  double* st = nullptr;
  double* ewr = nullptr;
  double* ewi = nullptr;
  Ctrl* ctrl = nullptr;
  Ctrl* ctrl_h = nullptr;
  int* blist = nullptr;
  int blist_cap = 0;
  int* bcount = nullptr;
  schur_stats stats{};
  Timer timer;
  // batched workspace (grow-only)
  struct Grow {
    void* dev = nullptr;
    void* host = nullptr;   // pinned staging
    size_t cap = 0;
  };
  Grow b_ctrl, b_defl, b_small, b_shift, b_win, b_u, b_sh, b_aedt, b_aedw;
  // parallel early-deflation passes: tasks, outcomes, V^T slots, block
  // starts, panel descriptors
  Grow b_splt, b_splr, b_splu, b_splz, b_splw;
  Grow b_splq, b_splb;   // batched finish: per-block Z slots, block orders
  // Hessenberg reduction: V and Y of a panel, T / tau / pivot, per-workgroup
  // partials, partial matrix-vector products, product scratch
  Grow b_hvy, b_ht, b_hp, b_hy, b_hw;
  // eigenvectors: Y when they are backtransformed, per-column bounds
  Grow b_evy, b_evb;
  // reordering: row flags + info, window tasks, panel descriptors, U slots
  Grow b_rsel, b_rtask, b_rwin, b_ru;
  // persistent batched kernel: jobs, queue order, results (info, counters),
  // per-workgroup scratch and the queue counter
  Grow b_pjob, b_pord, b_pres, b_pscr;
  // nested solve of a trailing block larger than SMALL_EIG_MAX (shifts only)
  schur_handle_s* sub = nullptr;
  // buffers of the parallel early-deflation passes that the batched engine
  // runs on its large matrices (kept apart from the engine's own)
  schur_handle_s* side = nullptr;
  double* shm = nullptr;         // NS_MAX x NS_MAX copy of the trailing block
  // schur_reduce_begin / _end: the thread that drives a solve begun on the
  // handle, the caller's stream point it starts after, its completion on
  // the handle's stream, its info code (and a pinned copy for the device)
  std::thread* job = nullptr;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  int job_rc = 0;
  int* job_info_h = nullptr;
};

namespace {

std::mutex g_mu;
schur_handle_s* g_default[64] = {nullptr};

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// ---- defaults and the tuning table -----------------------------------------
struct TuneRow {
  int nmax, ns, nb, step, nw;   // nw: early-deflation window (0: from ns, < 0: off)
  int nibble;                   // sweep-skip percentage after a window (0: default)
  int tile;                     // panel tiles (64 columns or rows) per workgroup (0: model)
};
// built-in table: plain double-shift sweeps for small orders, then more
// shifts per sweep as the order grows; early-deflation windows of 64 rows
// for large orders, followed by another window rather than a sweep once it
// deflates more than 7 % (measured at n = 16384: 64 rows beat 48 and 96;
// 7 % needs no sweep, 14 % a few)
const TuneRow kBuiltinTune[] = {{299, 2, 1, 0, 0, 0, 0},
                                {2999, 32, 16, 0, 0, 0, 0},
                                {5999, 64, 16, 0, 64, 7, 0},
                                {1 << 30, 128, 16, 0, 64, 7, 0}};
std::mutex g_tune_mu;
std::vector<TuneRow> g_tune(std::begin(kBuiltinTune), std::end(kBuiltinTune));

TuneRow tune_for(int n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const TuneRow& r : g_tune)
    if (n <= r.nmax) return r;
  return g_tune.back();
}

struct Params {
  int ns, nb, step, nmin, max_sweeps, exc_period;
  int nw;      // early-deflation window order (0: none)
  int nibble;  // skip the sweep after a window that deflated > nibble % of nw (-1: never)
  int split_nw;     // window order of the parallel early-deflation passes (0: none)
  int split_min_n;  // smallest order that runs them
  int tile;         // panel tiles per workgroup of the sweep's products (0: cost model)
  bool time;
};

// nominal flops of one early-deflation window: the Schur form with vectors
// (25 nw^3, the usual count of the double-shift QR with Schur vectors) and
// the reduction of the undeflated part back to Hessenberg form with V
double aed_work(int nw, int nu) {
  return 25.0 * nw * (double)nw * nw + (10.0 / 3.0) * nu * (double)nu * nu;
}

// counted flops of one window chase: per chain step and bulge, 10 flops for
// each row or column of the window its reflector touches in the left and
// right updates together (about ws of them), and 10 per row of U
double chase_work(int ws, int nb, int steps) { return 20.0 * ws * (double)nb * steps; }

// info code of a solve in which a non-finite value appeared (never for
// finite input; reported instead of a Schur form)
constexpr int kErrNonFinite = -105;

// early deflation: by default the next sweep is skipped when a window
// deflated more than this percentage of its order
constexpr int kAedSkipPct = 14;

// parallel early deflation: default smallest order, and the most passes
constexpr int kSplitMinN = 2048;
constexpr int kSplitMaxPasses = 64;

Params resolve(const schur_opts& o, int n) {
  Params p;
  const TuneRow tr = tune_for(n);
  p.ns = o.ns > 0 ? (o.ns & ~1) : tr.ns;
  if (p.ns < 2) p.ns = 2;
  if (p.ns > NS_MAX) p.ns = NS_MAX;
  p.nb = o.nb > 0 ? o.nb : (tr.nb > 0 ? tr.nb : 16);
  if (p.nb > NBMAX) p.nb = NBMAX;
  p.step = o.step > 0 ? o.step : tr.step;
  p.nmin = o.nmin > 0 ? std::min(o.nmin, SMALL_Z_MAX) : SMALL_Z_MAX;
  p.max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 30 * std::max(10, n) / std::max(2, p.ns) + 100;
  p.exc_period = o.exc_period > 0 ? o.exc_period : 6;
  p.time = (o.flags & SCHUR_FLAG_TIME_KERNELS) != 0;
  const int aw = o.aed_window != 0 ? o.aed_window : tr.nw;
  const int nib = o.aed_nibble != 0 ? o.aed_nibble : tr.nibble;
  p.nibble = nib < 0 ? -1 : (nib > 0 ? nib : kAedSkipPct);
  p.split_nw = o.split_window < 0 ? 0 : (o.split_window > 0 ? std::min(o.split_window, SMALL_Z_MAX)
                                                              : SMALL_Z_MAX);
  if (p.split_nw < 3) p.split_nw = 0;
  p.split_min_n = o.split_min_n > 0 ? o.split_min_n : kSplitMinN;
  const int tl = o.panel_tile != 0 ? o.panel_tile : tr.tile;
  p.tile = tl > 0 ? std::min(tl, PANEL_TPB) : 0;
  if (aw < 0) p.nw = 0;
  else if (aw > 0) p.nw = std::min(aw, SMALL_Z_MAX);
  else p.nw = std::min(SMALL_Z_MAX, std::max(16, p.ns + p.ns / 2));
  return p;
}

int alloc_ws(schur_handle_s* h, int n) {
  if (!h->U) {
    if (hipMalloc(&h->U, sizeof(double) * (size_t)NBUF * MAXWIN * UPAD * UPAD) != hipSuccess)
      return -101;
    if (hipMalloc(&h->refl, sizeof(double) * (size_t)MAXWIN * REFL_STRIDE) != hipSuccess) return -101;
    if (hipMalloc(&h->st, sizeof(double) * NSMAX) != hipSuccess) return -101;
    if (hipMalloc(&h->ewr, sizeof(double) * NSMAX) != hipSuccess) return -101;
    if (hipMalloc(&h->ewi, sizeof(double) * NSMAX) != hipSuccess) return -101;
    if (hipMalloc(&h->ctrl, sizeof(Ctrl)) != hipSuccess) return -101;
    if (hipHostMalloc(&h->ctrl_h, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess) return -101;
    if (hipMalloc(&h->bcount, sizeof(int)) != hipSuccess) return -101;
    HCHECK(hipMemset(h->ctrl, 0, sizeof(Ctrl)));
  }
  const int need = n / 2 + 2;
  if (h->blist_cap < need) {
    if (h->blist) HCHECK(hipFree(h->blist));
    h->blist = nullptr;
    if (hipMalloc(&h->blist, sizeof(int) * (size_t)need) != hipSuccess) return -101;
    h->blist_cap = need;
  }
  return 0;
}

// grow-only device buffer with a pinned host mirror
void* grow(schur_handle_s::Grow& g, size_t bytes, bool staging) {
  if (g.cap < bytes) {
    if (g.dev) HCHECK(hipFree(g.dev));
    if (g.host) HCHECK(hipHostFree(g.host));
    g.dev = nullptr;
    g.host = nullptr;
    g.cap = 0;
    const size_t cap = bytes + bytes / 2 + 4096;
    HCHECK(hipMalloc(&g.dev, cap));
    if (staging) HCHECK(hipHostMalloc(&g.host, cap, hipHostMallocDefault));
    g.cap = cap;
  }
  if (staging && !g.host) HCHECK(hipHostMalloc(&g.host, g.cap, hipHostMallocDefault));
  return g.dev;
}

void free_grow(schur_handle_s::Grow& g) {
  if (g.dev) (void)hipFree(g.dev);
  if (g.host) (void)hipHostFree(g.host);
  g.dev = nullptr;
  g.host = nullptr;
  g.cap = 0;
}

void free_ws(schur_handle_s* h) {
  free_grow(h->b_ctrl); free_grow(h->b_defl); free_grow(h->b_small);
  free_grow(h->b_shift); free_grow(h->b_win); free_grow(h->b_u); free_grow(h->b_sh);
  free_grow(h->b_aedt); free_grow(h->b_aedw);
  free_grow(h->b_splt); free_grow(h->b_splr); free_grow(h->b_splu); free_grow(h->b_splz);
  free_grow(h->b_splw); free_grow(h->b_splq); free_grow(h->b_splb);
  free_grow(h->b_hvy); free_grow(h->b_ht); free_grow(h->b_hp); free_grow(h->b_hy);
  free_grow(h->b_hw); free_grow(h->b_evy); free_grow(h->b_evb);
  free_grow(h->b_rsel); free_grow(h->b_rtask); free_grow(h->b_rwin); free_grow(h->b_ru);
  free_grow(h->b_pjob); free_grow(h->b_pord); free_grow(h->b_pres); free_grow(h->b_pscr);
  if (h->U) (void)hipFree(h->U);
  if (h->refl) (void)hipFree(h->refl);
  if (h->st) (void)hipFree(h->st);
  if (h->ewr) (void)hipFree(h->ewr);
  if (h->ewi) (void)hipFree(h->ewi);
  if (h->ctrl) (void)hipFree(h->ctrl);
  if (h->ctrl_h) (void)hipHostFree(h->ctrl_h);
  if (h->blist) (void)hipFree(h->blist);
  if (h->bcount) (void)hipFree(h->bcount);
  h->U = h->refl = h->st = h->ewr = h->ewi = nullptr;
  h->ctrl = nullptr; h->ctrl_h = nullptr; h->blist = nullptr; h->bcount = nullptr;
  h->blist_cap = 0;
}

// Panel tiles of one window of a batched panel launch (tpb tiles per
// workgroup: PANEL_TPB_WIDE where a launch carries many windows, so that each
// workgroup reads its U once for more tiles; PANEL_TPB_BATCH in the round
// engine, whose launches can hold only a few windows), appended after the
// workgroups counted so far.
void fill_tiles_b(WinB& w, int& tr, int& tcq, schur_stats& st, int tpb) {
  const int pe = w.c.p + w.c.ws - 1;
  w.tiles_r = std::max(0, (w.c.cend - pe - 1 + GEMM_T - 1) / GEMM_T);
  w.tiles_c = std::max(0, (w.c.p - w.c.rtop + GEMM_T - 1) / GEMM_T);
  w.tiles_q = w.c.Q ? (w.c.n + GEMM_T - 1) / GEMM_T : 0;
  w.base_r = tr;
  w.base_cq = tcq;
  w.tpb = tpb;
  tr += panel_blocks(w.tiles_r, tpb);
  tcq += panel_blocks(w.tiles_c + w.tiles_q, tpb);
  const double ws = w.c.ws;
  const double fr = 2.0 * ws * ws * (double)std::max(0, w.c.cend - pe - 1);
  const double fc = 2.0 * ws * ws * ((double)(w.c.p - w.c.rtop) + (w.c.Q ? (double)w.c.n : 0.0));
  st.row_flops += fr;
  st.colq_flops += fc;
  st.gemm_flops += fr + fc;
}

// ---- sweep schedule ---------------------------------------------------------
struct WinPlan {
  int p, ws, tau0, tau1, nb, shift0;
};

// Lock-step schedule of one sweep over the active block [ktop, kbot] with
// `npair` bulges split into groups of at most nbmax.  Group j starts L time
// steps after group j-1 so that the windows of one time step are disjoint and
// ordered top (later groups) to bottom (earlier groups).
void plan_sweep(int ktop, int kbot, int npair, int nbmax, int step_opt,
                std::vector<std::vector<WinPlan>>& steps, int& step_out) {
  steps.clear();
  const int G = (npair + nbmax - 1) / nbmax;
  std::vector<int> nbj(G), sh0(G);
  int acc = 0;
  for (int j = 0; j < G; ++j) {
    nbj[j] = npair / G + (j < npair % G ? 1 : 0);
    sh0[j] = acc;
    acc += nbj[j];
  }
  const int nbm = nbj[0];
  int step = WMAX - 3 * nbm - 1;
  step = std::min(step, REFL_LDS / nbm);   // reflector log of one window fits LDS
  if (step_opt > 0) step = std::min(step, step_opt);
  if (step < 3) step = 3;
  step_out = step;
  int L = 1;
  while ((L - 1) * step <= 3 * nbm) ++L;
  std::vector<int> nw(G), tend(G);
  int T = 0;
  for (int j = 0; j < G; ++j) {
    tend[j] = kbot - ktop + 3 * nbj[j] - 3;
    nw[j] = (tend[j] + step - 1) / step;
    T = std::max(T, j * L + nw[j]);
  }
  steps.resize(T);
  for (int t = 0; t < T; ++t) {
    // earlier groups are lower in the matrix: list bottom window last
    for (int j = G - 1; j >= 0; --j) {
      const int i = t - j * L;
      if (i < 0 || i >= nw[j]) continue;
      WinPlan w;
      w.tau0 = i * step;
      w.tau1 = std::min(w.tau0 + step, tend[j]);
      w.nb = nbj[j];
      w.shift0 = sh0[j];
      const int bhi = std::min(w.nb - 1, (w.tau1 - 1) / 3);
      const int kmin = ktop - 1 + std::max(0, w.tau0 - 3 * bhi);
      const int kmax = std::min(kbot - 2, ktop - 1 + w.tau1 - 1);
      w.p = std::max(ktop, kmin);
      const int pe = std::min(kbot, kmax + 4);
      w.ws = pe - w.p + 1;
      steps[t].push_back(w);
    }
  }
}

// ---- parallel early deflation: window tiling and selection (host) ---------
// Windows over the unreduced block [lo, hi], bottom-aligned: the bottom one
// has `first` rows (at most nw), the others nw, the top one what is left; a
// top window shorter than 16 rows and the one below it become two halves.
// Writes (start, order) pairs bottom to top.
void split_tile(int lo, int hi, int first, int nw, std::vector<std::pair<int, int>>& ws) {
  ws.clear();
  for (int b = hi + 1; b > lo;) {
    const int a = std::max(lo, b - (ws.empty() ? first : nw));
    ws.push_back({a, b - a});
    b = a;
  }
  if (ws.size() >= 2 && ws.back().second < 16) {
    const int tot = ws.back().second + ws[ws.size() - 2].second;
    const int top = ws.back().first;
    ws.pop_back();
    ws.pop_back();
    ws.push_back({top + tot / 2, tot - tot / 2});
    ws.push_back({top, tot / 2});
  }
}

// Among candidate windows (start a[c], order w[c], weight wt[c]) of one
// block, the disjoint set of largest total weight (weighted interval
// scheduling over the window ends).  Appends the chosen indices of `cand`.
void split_select(const std::vector<int>& cand, const int* a, const int* w, const double* wt,
                  std::vector<int>& pick) {
  std::vector<int> order(cand);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return a[x] + w[x] < a[y] + w[y]; });
  const int k = (int)order.size();
  std::vector<double> best(k + 1, 0.0);
  std::vector<int> prev(k + 1, -1);
  for (int j = 1; j <= k; ++j) {
    const int c = order[j - 1];
    int p = j - 1;   // windows ending at or above this one's start
    while (p > 0 && a[order[p - 1]] + w[order[p - 1]] > a[c]) --p;
    const double take = best[p] + wt[c];
    if (take > best[j - 1]) {
      best[j] = take;
      prev[j] = p;
    } else {
      best[j] = best[j - 1];
      prev[j] = -1;   // not taken
    }
  }
  for (int j = k; j > 0;) {
    if (prev[j] >= 0) {
      pick.push_back(order[j - 1]);
      j = prev[j];
    } else {
      --j;
    }
  }
}

// Weight of a window of a pass as a candidate for the selection: 1 + rows
// deflated for a window that passed its tests, 0 (not a candidate) when it
// failed them, or when it sits at an end of its block (no coupling above or
// none below, so its one-sided test cannot fail) and deflated nothing: such
// a window neither deflates nor splits, and committing it would only cost
// panel products and rounding.  An interior window that deflated nothing
// still splits its block between its up- and down-coupled parts.
double split_weight(int split, int nf, int top, int below) {
  if (!split) return 0.0;
  if (nf <= 0 && !(top && below)) return 0.0;
  return 1.0 + (double)std::max(0, nf);
}

int create_handle(schur_handle_s** out, int device, const schur_opts* opts);
bool batch_blocks(schur_handle_s* h, hipStream_t s, const std::vector<std::pair<int, int>>& blocks,
                  int n, double* H, int ldh, double* Q, int ldq, double* wr, double* wi,
                  bool time);

struct Solver {
  schur_handle_s* h;
  hipStream_t s;
  Params P;
  int n;
  double* H; int ldh;
  double* Q; int ldq;
  double* wr; double* wi;

  int64_t tslot = 0;   // time steps issued so far (ring position of the U slots)
  // everything on stream s, one U-slot buffer, no events (the handle has no
  // aux stream): the entry point that allocates nothing
  bool one_stream = false;

  // Workgroup counts of the row panel and column panel (main stream) in `a`, and
  // of the Q products (aux stream) in `aq`, a copy of `a`.
  // Tiles per workgroup of one panel launch (one workgroup per CU at a
  // time): the count that minimises rounds of workgroups x (tiles per
  // workgroup + the fixed cost of a workgroup, about half a tile), so that
  // the windows' ragged tile counts leave few CUs idle in the last round.
  template <typename TilesOf>
  int tiles_per_block(int nwin, TilesOf tiles_of) const {
    if (P.tile > 0) return P.tile;   // fixed by the options or the tuning table
    constexpr int kCUs = 256;
    int best = 1;
    double best_cost = 1e300;
    for (int tpb = 1; tpb <= PANEL_TPB; ++tpb) {
      long blocks = 0;
      for (int w = 0; w < nwin; ++w) blocks += panel_blocks(tiles_of(w), tpb);
      if (blocks == 0) return 1;
      const long rounds = (blocks + kCUs - 1) / kCUs;
      const double cost = (double)rounds * (tpb + 0.5);
      if (cost < best_cost - 1e-9) { best_cost = cost; best = tpb; }
    }
    return best;
  }

  void fill_gemm(SweepArgs& a, SweepArgs& aq, int& tr, int& tc, int& tq) {
    for (int w = 0; w < a.nwin; ++w) {
      Win& d = a.win[w];
      const int pe = d.p + d.ws - 1;
      d.tiles_r = std::max(0, (a.cend - pe - 1 + GEMM_T - 1) / GEMM_T);
      d.tiles_c = std::max(0, (d.p - a.rtop + GEMM_T - 1) / GEMM_T);
      d.tiles_q = 0;
      const double ws = d.ws;
      const double fr = 2.0 * ws * ws * (double)std::max(0, a.cend - pe - 1);
      const double fc = 2.0 * ws * ws * ((double)(d.p - a.rtop) + (a.Q ? (double)n : 0.0));
      h->stats.row_flops += fr;
      h->stats.colq_flops += fc;
      h->stats.gemm_flops += fr + fc;
    }
    a.tpb_r = tiles_per_block(a.nwin, [&](int w) { return a.win[w].tiles_r; });
    a.tpb_cq = tiles_per_block(a.nwin, [&](int w) { return a.win[w].tiles_c; });
    tr = 0;
    tc = 0;
    for (int w = 0; w < a.nwin; ++w) {
      Win& d = a.win[w];
      d.base_r = tr;
      d.base_cq = tc;
      tr += panel_blocks(d.tiles_r, a.tpb_r);
      tc += panel_blocks(d.tiles_c, a.tpb_cq);
    }
    aq = a;
    const int tiles_q = a.Q ? (n + GEMM_T - 1) / GEMM_T : 0;
    aq.tpb_r = 1;
    aq.tpb_cq = tiles_per_block(aq.nwin, [&](int) { return tiles_q; });
    tq = 0;
    for (int w = 0; w < aq.nwin; ++w) {
      Win& d = aq.win[w];
      d.tiles_r = 0;
      d.tiles_c = 0;
      d.tiles_q = tiles_q;
      d.base_cq = tq;
      tq += panel_blocks(d.tiles_q, aq.tpb_cq);
    }
  }

  // ring buffer of U slots for the next time step: wait until the Q products
  // that last read this buffer are done
  int acquire_buffer() {
    if (one_stream) {   // stream order: the last time step's readers are done
      ++tslot;
      return 0;
    }
    const int buf = (int)(tslot % NBUF);
    if (tslot >= NBUF) HCHECK(hipStreamWaitEvent(s, h->ev_q[buf], 0));
    ++tslot;
    return buf;
  }

  // Q products of one time step on the aux stream, after the U slots are ready
  void launch_q(const SweepArgs& aq, int tq, int buf) {
    if (one_stream) {
      if (tq > 0) {
        hipEvent_t e0 = nullptr;
        if (P.time) h->timer.begin(s, e0);
        launch_panel_colq(aq, tq, s);
        HCHECK(hipGetLastError());
        if (P.time) h->timer.end(s, e0, &h->stats.colq_ms);
        h->stats.colq_launches += 1;
        h->stats.gemm_launches += 1;
        h->stats.launches += 1;
      }
      return;
    }
    HCHECK(hipEventRecord(h->ev_u[buf], s));
    if (tq > 0) {
      HCHECK(hipStreamWaitEvent(h->aux, h->ev_u[buf], 0));
      hipEvent_t e0 = nullptr;
      if (P.time) h->timer.begin(h->aux, e0);
      launch_panel_colq(aq, tq, h->aux);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(h->aux, e0, &h->stats.colq_ms);
      h->stats.colq_launches += 1;
      h->stats.gemm_launches += 1;
      h->stats.launches += 1;
    }
    HCHECK(hipEventRecord(h->ev_q[buf], h->aux));
  }

  // main stream waits for everything issued on the aux stream
  void join_aux() {
    if (one_stream) return;
    HCHECK(hipEventRecord(h->ev_join, h->aux));
    HCHECK(hipStreamWaitEvent(s, h->ev_join, 0));
  }

  void base_args(SweepArgs& a, int ktop, int kbot) {
    std::memset(&a, 0, sizeof(a));
    a.H = H; a.ldh = ldh; a.Q = Q; a.ldq = ldq; a.n = n;
    a.ktop = ktop; a.kbot = kbot;
    a.rtop = 0; a.cend = n;
    a.st = h->st;
    a.U = h->U;
    a.refl = h->refl;
    a.refl_stride = REFL_STRIDE;
  }

  void launch_gemms(const SweepArgs& a, int tr, int tcq) {
    hipEvent_t e0 = nullptr;
    if (tr > 0) {
      if (P.time) h->timer.begin(s, e0);
      launch_panel_row(a, tr, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.row_ms);
      h->stats.row_launches += 1;
    }
    if (tcq > 0) {
      if (P.time) h->timer.begin(s, e0);
      launch_panel_colq(a, tcq, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.colq_ms);
      h->stats.colq_launches += 1;
    }
    h->stats.gemm_launches += (tr > 0) + (tcq > 0);
    h->stats.launches += (tr > 0) + (tcq > 0);
  }

  // The panel products of one time step.  Two streams: Q on the aux stream,
  // rows then columns of H on the main one.  One stream: two launches, the
  // rows of H with Q (different matrices, no order between them), then the
  // columns of H.  (The rows and the columns of H meet in the blocks
  // rows(A) x cols(B) of two windows A above B, so they stay in two
  // launches in stream order.  Splitting Q between the two launches so that
  // they carry equal tile counts measured slower.)
  void launch_panels(const SweepArgs& a, const SweepArgs& aq, int tr, int tc, int tq, int buf) {
    if (!one_stream) {
      launch_q(aq, tq, buf);
      launch_gemms(a, tr, tc);
      return;
    }
    (void)buf;
    // the Q products are timed with the rows of H
    for (int w = 0; w < aq.nwin; ++w) {
      const double fq = 2.0 * (double)aq.win[w].ws * (double)aq.win[w].ws * (a.Q ? (double)n : 0.0);
      h->stats.row_flops += fq;
      h->stats.colq_flops -= fq;
    }
    hipEvent_t e0 = nullptr;
    if (tr + tq > 0) {
      if (P.time) h->timer.begin(s, e0);
      launch_panel_rowq(a, tr, aq, tq, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.row_ms);
      h->stats.row_launches += 1;
    }
    if (tc > 0) {
      if (P.time) h->timer.begin(s, e0);
      launch_panel_colq(a, tc, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.colq_ms);
      h->stats.colq_launches += 1;
    }
    h->stats.gemm_launches += (tr + tq > 0) + (tc > 0);
    h->stats.launches += (tr + tq > 0) + (tc > 0);
  }

  void sync_ctrl() {
    HCHECK(hipMemcpyAsync(h->ctrl_h, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    if (P.time) {
      HCHECK(hipStreamSynchronize(h->aux));
      h->timer.harvest();
    }
  }

  // finish a small active block [ktop, kbot] in one kernel, then apply its
  // Z to the row panel, the column panel and Q
  void small_block(int ktop, int kbot) {
    const int m = kbot - ktop + 1;
    const int buf = acquire_buffer();
    SmallTask t{};
    t.A = H + ktop + (size_t)ktop * ldh;
    t.lda = ldh;
    t.m = m;
    t.Zt = h->U + (size_t)buf * MAXWIN * UPAD * UPAD;
    t.ldzt = UPAD;
    t.info = &h->ctrl->small_info;
    t.itmax = 0;   // default budget
    hipEvent_t e0 = nullptr;
    if (P.time) h->timer.begin(s, e0);
    launch_small_z(t, nullptr, 1, m, s);
    HCHECK(hipGetLastError());
    if (P.time) h->timer.end(s, e0, &h->stats.small_ms);
    h->stats.small_solves += 1;
    h->stats.small_launches += 1;
    h->stats.small_flops += 25.0 * m * (double)m * m;
    h->stats.launches += 1;
    SweepArgs a, aq;
    base_args(a, ktop, kbot);
    a.nwin = 1;
    a.win[0].p = ktop;
    a.win[0].ws = m;
    a.win[0].slot = buf * MAXWIN;
    int tr, tc, tq;
    fill_gemm(a, aq, tr, tc, tq);
    launch_panels(a, aq, tr, tc, tq, buf);
  }

  // Early deflation on the bottom nw rows of [ktop, kbot]; applies the
  // window's orthogonal factor to the rest of H and to Q when something
  // deflated.  Returns the number deflated; *nu receives the number of
  // undeflated window eigenvalues left in ewr/ewi (0 if the window's Schur
  // form did not converge).
  int aed(int ktop, int kbot, int nw, int* nu) {
    const int buf = acquire_buffer();
    AedTask t{};
    t.H = H; t.ldh = ldh;
    t.ktop = ktop; t.kbot = kbot; t.nw = nw;
    t.Ut = h->U + (size_t)buf * MAXWIN * UPAD * UPAD;
    t.ldut = UPAD;
    t.sr = h->ewr; t.si = h->ewi;
    t.wr = wr + (kbot - nw + 1); t.wi = wi + (kbot - nw + 1);
    t.ctrl = h->ctrl;
    t.itmax = 0;   // default budget
    hipEvent_t e0 = nullptr;
    if (P.time) h->timer.begin(s, e0);
    launch_aed(t, s);
    HCHECK(hipGetLastError());
    if (P.time) h->timer.end(s, e0, &h->stats.aed_ms);
    h->stats.launches += 1;
    h->stats.aed_windows += 1;
    h->stats.aed_launches += 1;
    sync_ctrl();
    const int nd = h->ctrl_h->aed_nd;
    *nu = h->ctrl_h->aed_nu;
    SweepArgs a, aq;
    base_args(a, ktop, kbot);
    int tr = 0, tc = 0, tq = 0;
    if (nd > 0) {
      a.nwin = 1;
      a.win[0].p = kbot - nw + 1;
      a.win[0].ws = nw;
      a.win[0].slot = buf * MAXWIN;
      fill_gemm(a, aq, tr, tc, tq);
    } else {
      a.nwin = 0;
      aq = a;
    }
    launch_panels(a, aq, tr, tc, tq, buf);   // records the slot's events even when idle
    h->stats.aed_deflated += nd;
    h->stats.aed_flops += aed_work(nw, nd > 0 ? *nu : 0);
    return nd;
  }

  // Eigenvalues of the trailing ns x ns block (H(kbot-ns+1:kbot, same)) by a
  // nested solve of this engine on a copy, without Schur vectors; returns its
  // info (0: ewr/ewi hold all ns eigenvalues).
  int nested_shift_solve(int kbot, int ns) {
    if (!h->sub) {
      schur_handle_s* sub = nullptr;
      if (create_handle(&sub, h->device, nullptr) != 0) throw HipErr{hipErrorOutOfMemory};
      h->sub = sub;
    }
    if (!h->shm && hipMalloc(&h->shm, sizeof(double) * NS_MAX * NS_MAX) != hipSuccess)
      throw HipErr{hipErrorOutOfMemory};
    const int b0 = kbot - ns + 1;
    HCHECK(hipMemcpy2DAsync(h->shm, sizeof(double) * ns, H + b0 + (size_t)b0 * ldh,
                            sizeof(double) * ldh, sizeof(double) * ns, ns,
                            hipMemcpyDeviceToDevice, s));
    if (alloc_ws(h->sub, ns) != 0) throw HipErr{hipErrorOutOfMemory};
    std::memset(&h->sub->stats, 0, sizeof(h->sub->stats));
    schur_opts so{};
    Solver sv{h->sub, s, resolve(so, ns), ns, h->shm, ns, nullptr, ns, h->ewr, h->ewi};
    const int info = sv.run();
    h->stats.launches += h->sub->stats.launches;
    const schur_stats& ss = h->sub->stats;
    h->stats.small_flops += ss.gemm_flops + ss.chase_flops + ss.small_flops + ss.aed_flops +
                            ss.split_flops;
    return info;
  }

  void compute_shifts(int ktop, int kbot, int ns, bool exceptional) {
    hipEvent_t e0 = nullptr;
    if (P.time) h->timer.begin(s, e0);
    if (!exceptional && ns > SMALL_EIG_MAX) {
      // a failed nested solve (or a non-finite block) falls back to the ad-hoc pair
      const int info = nested_shift_solve(kbot, ns);
      launch_shift_prep(h->ewr, h->ewi, ns, nullptr, info != 0 ? 1 : 0, H, ldh, ktop, kbot, h->st,
                        s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.shift_ms);
      h->stats.launches += 1;
      return;
    }
    if (!exceptional) {
      SmallTask t{};
      const int b0 = kbot - ns + 1;
      t.A = H + b0 + (size_t)b0 * ldh;
      t.lda = ldh;
      t.m = ns;
      t.wr = h->ewr;
      t.wi = h->ewi;
      // a shift solve that does not converge only costs shifts: its own
      // status slot, read by the shift preparation
      t.info = &h->ctrl->nshift;
      t.itmax = 0;   // default budget
      launch_small_eig(t, s);
      h->stats.small_flops += 10.0 * ns * (double)ns * ns;
    }
    launch_shift_prep(h->ewr, h->ewi, ns, &h->ctrl->nshift, exceptional ? 1 : 0, H, ldh, ktop,
                      kbot, h->st, s);
    HCHECK(hipGetLastError());
    if (P.time) h->timer.end(s, e0, &h->stats.shift_ms);
    h->stats.launches += exceptional ? 1 : 2;
  }

  void sweep(int ktop, int kbot, int ns) {
    std::vector<std::vector<WinPlan>> steps;
    int step = 0;
    const int npair = ns / 2;
    plan_sweep(ktop, kbot, npair, P.nb, P.step, steps, step);
    h->stats.sweeps += 1;
    h->stats.shifts_applied += ns;
    for (const auto& ws : steps) {
      if (ws.empty()) continue;   // gap between groups on short blocks
      SweepArgs a, aq;
      base_args(a, ktop, kbot);
      a.nwin = (int)ws.size();
      if (a.nwin > MAXWIN) throw HipErr{hipErrorInvalidValue};
      const int buf = acquire_buffer();
      int prev_end = -1;
      for (int w = 0; w < a.nwin; ++w) {
        const WinPlan& pl = ws[w];
        if (pl.ws > WMAX || pl.ws < 3 || pl.p <= prev_end || pl.p < ktop ||
            pl.p + pl.ws - 1 > kbot || pl.nb > NBMAX || pl.tau1 - pl.tau0 > WMAX ||
            (pl.tau1 - pl.tau0) * pl.nb > REFL_LDS)
          throw HipErr{hipErrorInvalidValue};
        prev_end = pl.p + pl.ws - 1;
        Win& d = a.win[w];
        d.p = pl.p; d.ws = pl.ws; d.tau0 = pl.tau0; d.tau1 = pl.tau1;
        d.nb = pl.nb; d.shift0 = pl.shift0; d.slot = buf * MAXWIN + w;
        h->stats.windows += 1;
        h->stats.chain_steps += pl.tau1 - pl.tau0;
        h->stats.chase_flops += chase_work(pl.ws, pl.nb, pl.tau1 - pl.tau0);
        h->stats.chase_bytes += 24.0 * (double)pl.ws * (double)pl.ws;
      }
      hipEvent_t e0 = nullptr;
      if (P.time) h->timer.begin(s, e0);
      launch_chase(a, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.chase_ms);
      h->stats.chase_launches += 1;
      h->stats.launches += 1;
      int tr, tc, tq;
      fill_gemm(a, aq, tr, tc, tq);
      launch_panels(a, aq, tr, tc, tq, buf);
    }
  }

  // Parallel early deflation (split_window): passes of windows over every
  // unreduced block at once.  A pass scans the subdiagonal for the
  // unreduced blocks and lays two tilings of windows over each of them, the
  // second with its boundaries half a window further up (as long as the
  // launch fits the CUs).  One launch solves and tests every window, each
  // writing its result to its own slot.  Per block, the host keeps the set of
  // disjoint windows that split with the most rows deflated (weighted
  // interval scheduling); one launch writes those into H and scales their
  // coupling entries, and their V go to the row panels (one launch) and to
  // the column panels and Q (one launch; disjoint windows, so each launch
  // updates disjoint rows or columns).  Once the unreduced blocks all have
  // order <= UPAD, or a pass neither shrinks the largest block by a tenth
  // nor reduces the unreduced rows by 1 %, the blocks of order <= UPAD are
  // finished together by the batched engine; sweeps and bottom windows
  // finish what is left.
  bool split_phase() {
    constexpr int kCUs = 256;
    const int nw = P.split_nw;
    grow(h->b_splz, (size_t)n, true);
    unsigned char* zd = (unsigned char*)h->b_splz.dev;
    unsigned char* zh = (unsigned char*)h->b_splz.host;
    struct Wn { int a, nw, top, below; };
    std::vector<Wn> wins;
    std::vector<std::pair<int, int>> regs, ws;
    std::vector<int> order, pick;
    int64_t prev_active = -1;
    int prev_max = -1;
    int interior = 0;   // committed windows with blocks both above and below
    for (int pass = 0; pass < kSplitMaxPasses; ++pass) {
      launch_split_scan(H, ldh, n, zd, s);
      HCHECK(hipGetLastError());
      h->stats.launches += 1;
      HCHECK(hipMemcpyAsync(zh, zd, (size_t)n, hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));
      regs.clear();
      int64_t active = 0;
      int mx = 0;
      for (int k = 0; k < n;) {
        int e = k + 1;
        while (e < n && !zh[e]) ++e;
        const int m = e - k;
        if (m >= 3) {
          regs.push_back({k, e - 1});
          active += m;
          mx = std::max(mx, m);
        }
        k = e;
      }
      h->stats.split_converged = n - active;
      if (active == 0) return true;
      const bool stuck = prev_active >= 0 && 100 * (prev_active - active) < prev_active &&
                         10 * (int64_t)mx > 9 * (int64_t)prev_max;
      if (stuck || mx <= UPAD) {
        std::vector<std::pair<int, int>> fin;
        for (const auto& r : regs)
          if (r.second - r.first + 1 <= UPAD) fin.push_back(r);
        const bool ok = batch_blocks(h, s, fin, n, H, ldh, Q, ldq, wr, wi, P.time);
        if (ok && fin.size() == regs.size()) h->stats.split_converged = n;
        return ok && fin.size() == regs.size();
      }
      prev_active = active;
      prev_max = mx;
      // ---- candidate windows: per block, tiling 0 (bottom window of nw or
      // nw / 2 rows, alternating between passes) for every block, tiling 1
      // (the other offset) for the largest blocks while the launch fits
      auto tile = [&](int lo, int hi, int first) { split_tile(lo, hi, first, nw, ws); };
      const int f0 = (pass & 1) ? nw / 2 : nw, f1 = (pass & 1) ? nw : nw / 2;
      std::vector<int> tilings(regs.size(), 1);
      int total = 0;
      for (const auto& r : regs) total += (r.second - r.first + 1 + nw - 1) / nw + 1;
      order.resize(regs.size());
      for (size_t i = 0; i < regs.size(); ++i) order[i] = (int)i;
      std::sort(order.begin(), order.end(), [&](int x, int y) {
        return regs[x].second - regs[x].first > regs[y].second - regs[y].first;
      });
      for (int i : order) {
        const int m = regs[i].second - regs[i].first + 1;
        const int extra = (m + nw - 1) / nw + 1;
        if (m > nw && total + extra <= kCUs) {
          tilings[i] = 2;
          total += extra;
        }
      }
      wins.clear();
      std::vector<std::pair<int, int>> span(regs.size());   // candidate range per block
      for (size_t i = 0; i < regs.size(); ++i) {
        const int lo = regs[i].first, hi = regs[i].second;
        span[i].first = (int)wins.size();
        for (int t = 0; t < tilings[i]; ++t) {
          tile(lo, hi, (hi - lo + 1 > nw) ? (t == 0 ? f0 : f1) : nw);
          for (int j = (int)ws.size() - 1; j >= 0; --j) {
            Wn w;
            w.a = ws[j].first;
            w.nw = ws[j].second;
            w.top = w.a > lo ? 1 : 0;
            w.below = (w.a + w.nw <= hi) ? 1 : 0;
            if (w.nw < 1 || w.nw > SMALL_Z_MAX) throw HipErr{hipErrorInvalidValue};
            wins.push_back(w);
          }
        }
        span[i].second = (int)wins.size();
      }
      const int cnt = (int)wins.size();
      const size_t wslot = (size_t)SMALL_Z_MAX * SMALL_Z_MAX;
      grow(h->b_splt, sizeof(SplitTask) * cnt, true);
      grow(h->b_splr, sizeof(SplitRes) * cnt, true);
      grow(h->b_splu, sizeof(double) * (size_t)UPAD * UPAD * cnt, false);
      grow(h->b_splq, sizeof(double) * wslot * cnt, false);
      SplitTask* th = (SplitTask*)h->b_splt.host;
      SplitRes* rd = (SplitRes*)h->b_splr.dev;
      double* ud = (double*)h->b_splu.dev;
      double* wo = (double*)h->b_splq.dev;
      for (int i = 0; i < cnt; ++i) {
        SplitTask& t = th[i];
        std::memset(&t, 0, sizeof(t));
        t.H = H; t.ldh = ldh;
        t.a = wins[i].a; t.nw = wins[i].nw;
        t.above = wins[i].top ? 0 : -1;   // read as a flag by the window kernel
        t.below = wins[i].below;
        t.itmax = 0;   // default budget
        t.Ut = ud + (size_t)i * UPAD * UPAD; t.ldut = UPAD;
        t.res = rd + i;
        t.Wo = wo + (size_t)i * wslot; t.ldwo = SMALL_Z_MAX;
      }
      SplitTask* td = (SplitTask*)h->b_splt.dev;
      HCHECK(hipMemcpyAsync(td, th, sizeof(SplitTask) * cnt, hipMemcpyHostToDevice, s));
      hipEvent_t e0 = nullptr;
      if (P.time) h->timer.begin(s, e0);
      launch_split(td, cnt, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.split_ms);
      h->stats.launches += 1;
      h->stats.split_passes += 1;
      h->stats.split_windows += cnt;
      SplitRes* rh = (SplitRes*)h->b_splr.host;
      HCHECK(hipMemcpyAsync(rh, rd, sizeof(SplitRes) * cnt, hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));
      if (P.time) h->timer.harvest();
      // ---- per block: disjoint splitting windows of most weight (1 + rows
      // deflated), by weighted interval scheduling over the window ends
      pick.clear();
      std::vector<int> ca(cnt), cw(cnt);
      std::vector<double> cwt(cnt);
      for (int c = 0; c < cnt; ++c) {
        ca[c] = wins[c].a;
        cw[c] = wins[c].nw;
        cwt[c] = split_weight(rh[c].split, rh[c].nf, wins[c].top, wins[c].below);
        h->stats.split_flops += aed_work(wins[c].nw, rh[c].split ? rh[c].nu : 0) +
                                (10.0 / 3.0) * rh[c].nb * (double)rh[c].nb * rh[c].nb;
      }
      for (size_t i = 0; i < regs.size(); ++i) {
        order.clear();
        for (int c = span[i].first; c < span[i].second; ++c)
          if (cwt[c] > 0.0) order.push_back(c);
        split_select(order, ca.data(), cw.data(), cwt.data(), pick);
      }
      std::sort(pick.begin(), pick.end(), [&](int x, int y) { return wins[x].a < wins[y].a; });
      const int ncm = (int)pick.size();
      for (int j : pick) interior += (wins[j].top && wins[j].below) ? 1 : 0;
      // no window split inside a block in the first two passes (both
      // offsets): the eigenvectors are not localised, the sweeps are the
      // better tool (windows at the block ends are still committed)
      const bool give_up = pass == 1 && interior == 0;
      if (ncm == 0) {
        if (give_up) return false;
        continue;
      }
      grow(h->b_splb, sizeof(SplitCommit) * ncm, true);
      SplitCommit* ch = (SplitCommit*)h->b_splb.host;
      for (int j = 0; j < ncm; ++j) {
        const Wn& w = wins[pick[j]];
        SplitCommit& c = ch[j];
        c.task = pick[j];
        c.above = (j > 0 && wins[pick[j - 1]].a + wins[pick[j - 1]].nw == w.a) ? pick[j - 1] : -1;
        c.fix_top = w.top;
        const bool next_adj = j + 1 < ncm && wins[pick[j + 1]].a == w.a + w.nw;
        c.fix_below = (w.below && !next_adj) ? 1 : 0;
      }
      SplitCommit* cd = (SplitCommit*)h->b_splb.dev;
      HCHECK(hipMemcpyAsync(cd, ch, sizeof(SplitCommit) * ncm, hipMemcpyHostToDevice, s));
      launch_split_commit(cd, ncm, td, s);
      HCHECK(hipGetLastError());
      h->stats.launches += 1;
      h->stats.split_accepted += ncm;
      grow(h->b_splw, sizeof(WinB) * ncm, true);
      WinB* wh = (WinB*)h->b_splw.host;
      int tr = 0, tcq = 0;
      for (int j = 0; j < ncm; ++j) {
        const int i = pick[j];
        WinB& w = wh[j];
        std::memset(&w, 0, sizeof(w));
        w.c.H = H; w.c.Q = Q; w.c.U = ud + (size_t)i * UPAD * UPAD; w.c.st = nullptr;
        w.c.ldh = ldh; w.c.ldq = ldq; w.c.n = n;
        w.c.ktop = 0; w.c.kbot = n - 1; w.c.rtop = 0; w.c.cend = n;
        w.c.p = wins[i].a; w.c.ws = wins[i].nw;
        fill_tiles_b(w, tr, tcq, h->stats, PANEL_TPB_WIDE);
      }
      WinB* wd = (WinB*)h->b_splw.dev;
      HCHECK(hipMemcpyAsync(wd, wh, sizeof(WinB) * ncm, hipMemcpyHostToDevice, s));
      if (tr > 0) {
        if (P.time) h->timer.begin(s, e0);
        launch_panel_row_b(wd, ncm, tr, s);
        HCHECK(hipGetLastError());
        if (P.time) h->timer.end(s, e0, &h->stats.row_ms);
        h->stats.row_launches += 1;
        h->stats.gemm_launches += 1;
        h->stats.launches += 1;
      }
      if (tcq > 0) {
        if (P.time) h->timer.begin(s, e0);
        launch_panel_colq_b(wd, ncm, tcq, s);
        HCHECK(hipGetLastError());
        if (P.time) h->timer.end(s, e0, &h->stats.colq_ms);
        h->stats.colq_launches += 1;
        h->stats.gemm_launches += 1;
        h->stats.launches += 1;
      }
      if (give_up) return false;
    }
    return false;
  }

  int run() {
    // the aux stream starts after the work already queued on the solve stream
    if (!one_stream) {
      HCHECK(hipEventRecord(h->ev_join, s));
      HCHECK(hipStreamWaitEvent(h->aux, h->ev_join, 0));
    }
    launch_ctrl_reset(h->ctrl, s);
    launch_check_finite(H, ldh, n, h->ctrl, s);
    sync_ctrl();
    if (h->ctrl_h->bad) return -2;
    launch_zero_lower(H, ldh, n, s);
    // nothing left after the parallel passes: straight to the standardisation
    const bool done = P.split_nw > 0 && n >= P.split_min_n && split_phase();
    int info = 0;
    int kbot = n - 1;
    int nodefl = 0;
    int64_t sweeps = 0;
    while (!done) {
      hipEvent_t e0 = nullptr;
      if (P.time) h->timer.begin(s, e0);
      launch_deflate(H, ldh, kbot, 0, h->ctrl, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.other_ms);
      h->stats.launches += 1;
      sync_ctrl();
      if (h->ctrl_h->bad) {   // a non-finite value appeared during the iteration
        info = kErrNonFinite;
        break;
      }
      const int nk = h->ctrl_h->kbot;
      if (nk < kbot) nodefl = 0;
      kbot = nk;
      if (kbot < 0) break;
      const int ktop = h->ctrl_h->ktop;
      const int m = kbot - ktop + 1;
      if (m <= P.nmin) {
        // a failure is reported as the global end of the non-converged block
        small_block(ktop, kbot);
        sync_ctrl();
        if (h->ctrl_h->small_info != 0) {
          info = ktop + h->ctrl_h->small_info;
          break;
        }
        kbot = ktop - 1;
        if (kbot < 0) break;
        continue;
      }
      if (++sweeps > P.max_sweeps) {
        info = kbot + 1;
        break;
      }
      int ns = std::min(P.ns, 2 * ((m - 2) / 6));
      if (ns < 2) ns = 2;
      const bool exc = (nodefl > 0 && nodefl % P.exc_period == 0);
      const int nw = std::min(P.nw, m - 1);
      if (nw >= 4) {
        int nu = 0;
        const int nd = aed(ktop, kbot, nw, &nu);
        if (nd > 0) {
          kbot -= nd;
          nodefl = 0;
          // many deflations: look again before spending a sweep; a block
          // that became small goes to the single-kernel solver
          if ((P.nibble >= 0 && 100 * nd > P.nibble * nw) || kbot - ktop + 1 <= P.nmin) continue;
        }
        const int m2 = kbot - ktop + 1;
        ns = std::max(2, std::min(P.ns, 2 * ((m2 - 2) / 6)));
        if (!exc && nu >= 2 && 2 * nu >= ns) {
          // the undeflated window eigenvalues closest to the deflated part
          const int use = std::min(ns, nu) & ~1;
          hipEvent_t e0 = nullptr;
          if (P.time) h->timer.begin(s, e0);
          launch_shift_prep(h->ewr + (nu - use), h->ewi + (nu - use), use, nullptr, 0, H, ldh,
                            ktop, kbot, h->st, s);
          HCHECK(hipGetLastError());
          if (P.time) h->timer.end(s, e0, &h->stats.shift_ms);
          h->stats.launches += 1;
          sweep(ktop, kbot, use);
          ++nodefl;
          continue;
        }
      }
      compute_shifts(ktop, kbot, ns, exc);
      sweep(ktop, kbot, ns);
      ++nodefl;
    }
    join_aux();   // the standardisation rotates columns of Q
    if (info < 0) {
      HCHECK(hipStreamSynchronize(s));
      return info;
    }
    const int kmin = info > 0 ? info + 1 : 1;
    hipEvent_t e0 = nullptr;
    if (P.time) h->timer.begin(s, e0);
    launch_standardize(H, ldh, Q, ldq, n, kmin, wr, wi, h->blist, h->bcount, h->blist_cap, s);
    HCHECK(hipGetLastError());
    if (P.time) h->timer.end(s, e0, &h->stats.other_ms);
    h->stats.launches += 6;
    HCHECK(hipStreamSynchronize(s));
    if (P.time) h->timer.harvest();
    h->stats.gemm_ms = h->stats.row_ms + h->stats.colq_ms;
    return info;
  }
};

int check_args(int n, double* H, int ldh, double* Q, int ldq, double* wr, double* wi) {
  if (n < 0 || n > 524288) return -1;
  if (n == 0) return 0;
  if (!H) return -2;
  if (ldh < std::max(1, n) || ldh > LD_MAX) return -3;
  if (Q && (ldq < std::max(1, n) || ldq > LD_MAX)) return -5;
  if (!wr) return -6;
  if (!wi) return -7;
  if (!is_device_ptr(H) || (Q && !is_device_ptr(Q)) || !is_device_ptr(wr) || !is_device_ptr(wi))
    return -103;
  return 0;
}

int solve(schur_handle_s* h, hipStream_t s, int n, double* H, int ldh, double* Q, int ldq,
          double* wr, double* wi) {
  int rc = check_args(n, H, ldh, Q, ldq, wr, wi);
  if (rc != 0 || n == 0) return rc;
  try {
    HCHECK(hipSetDevice(h->device));
    rc = alloc_ws(h, n);
    if (rc) return rc;
    std::memset(&h->stats, 0, sizeof(h->stats));
    Solver sv{h, s, resolve(h->opts, n), n, H, ldh, Q, ldq, wr, wi};
    sv.one_stream = (h->opts.flags & SCHUR_FLAG_ONE_STREAM) != 0;
    return sv.run();
  } catch (const HipErr& e) {
    (void)hipGetLastError();
    return e.e == hipErrorOutOfMemory ? -101 : -102;
  }
}

// ---------------------------------------------------------------------------
// Hessenberg reduction A = Q1 H Q1^T (paper Sec. 2, Eq. (3)): blocked
// Householder reduction in panels of NBH columns.  Per column of a panel five
// launches (update of the column by the panel's earlier reflectors, its
// reflector, one matrix-vector product with the trailing matrix, the new
// column of Y = A V T and of T); per panel the top rows of Y, the right
// update of the trailing columns, the top rows of the panel's columns, the
// left update of the trailing block and Q <- Q (I - V T V^T) as FP64 MFMA
// products.  No host synchronisation: every launch is stream-ordered.
// ---------------------------------------------------------------------------
int hess_reduce(schur_handle_s* h, hipStream_t s, int n, double* A, int lda, double* Q, int ldq) {
  if (n < 0 || n > 524288) return -1;
  if (n == 0) return 0;
  if (!A) return -2;
  if (lda < std::max(1, n)) return -3;
  if (Q && ldq < std::max(1, n)) return -5;
  if (!is_device_ptr(A) || (Q && !is_device_ptr(Q))) return -103;
  try {
    HCHECK(hipSetDevice(h->device));
    std::memset(&h->stats, 0, sizeof(h->stats));
    if (n <= 2) return 0;
    const int rows_max = n - 1;
    const int nwg_max = (rows_max + HROWS - 1) / HROWS;
    constexpr int kSplitMax = 64;
    double* vy = (double*)grow(h->b_hvy, sizeof(double) * 2 * (size_t)n * NBH, false);
    double* tt = (double*)grow(h->b_ht, sizeof(double) * (NBH * NBH + NBH + 8), false);
    double* pp = (double*)grow(h->b_hp, sizeof(double) * (size_t)nwg_max * (2 * HPART + 2), false);
    double* yp = (double*)grow(h->b_hy, sizeof(double) * (size_t)n * kSplitMax, false);
    double* ww = (double*)grow(h->b_hw, sizeof(double) * 2 * (size_t)n * NBH, false);
    HessArgs g{};
    g.A = A; g.lda = lda; g.n = n;
    g.V = vy; g.Y = vy + (size_t)n * NBH;
    g.T = tt; g.tau = tt + NBH * NBH; g.sc = tt + NBH * NBH + NBH;
    g.part = pp; g.part3 = pp + (size_t)nwg_max * HPART; g.part2 = pp + (size_t)nwg_max * 2 * HPART;
    g.ypart = yp;
    double* W = ww;
    double* W2 = ww + (size_t)n * NBH;
    const bool time = (h->opts.flags & SCHUR_FLAG_TIME_KERNELS) != 0;
    hipEvent_t e0 = nullptr;
    for (int K = 0; K < n - 2; K += NBH) {
      const int ib = std::min(NBH, n - 2 - K);
      const int m1 = n - K - 1;
      const int nwg = (m1 + HROWS - 1) / HROWS;
      launch_hess_zero(g.V, (size_t)n * NBH, s);
      launch_hess_zero(g.T, (size_t)NBH * NBH, s);
      if (time) h->timer.begin(s, e0);
      for (int i = 0; i < ib; ++i) {
        // column splits of the matrix-vector product: about 1024 workgroups,
        // at least 32 columns each
        const int cols = n - (K + i + 1);
        int cs = std::max(1, 1024 / nwg);
        cs = std::min(std::min(cs, kSplitMax), std::max(1, cols / 32));
        launch_hess_column(g, K, i, cs, s);
        HCHECK(hipGetLastError());
        h->stats.launches += (i > 0) + 4;
        h->stats.hess_gemv_bytes += 8.0 * (double)m1 * cols;
      }
      if (time) h->timer.end(s, e0, &h->stats.hess_panel_ms);
      if (time) h->timer.begin(s, e0);
      const int nt = n - K - ib;   // trailing columns K+ib .. n-1
      // top rows of Y: Y(0:K+1, :) = A(0:K+1, K+1:n) V(K+1:n, :) T
      launch_gemm(false, false, K + 1, ib, m1, 1.0, A + (size_t)(K + 1) * lda, lda, g.V + (K + 1), n,
                  0.0, W, n, s);
      launch_gemm(false, false, K + 1, ib, ib, 1.0, W, n, g.T, NBH, 0.0, g.Y, n, s);
      // right update of the trailing columns, all rows: A -= Y V(K+ib:n, :)^T
      launch_gemm(false, true, n, nt, ib, -1.0, g.Y, n, g.V + (K + ib), n, 1.0,
                  A + (size_t)(K + ib) * lda, lda, s);
      // top rows of the panel's columns K+1 .. K+ib-1
      launch_gemm(false, true, K + 1, ib - 1, ib, -1.0, g.Y, n, g.V + (K + 1), n, 1.0,
                  A + (size_t)(K + 1) * lda, lda, s);
      // left update of the trailing block: A -= V (A^T V T)^T
      double* At = A + (K + 1) + (size_t)(K + ib) * lda;
      launch_gemm(true, false, nt, ib, m1, 1.0, At, lda, g.V + (K + 1), n, 0.0, W, n, s);
      launch_gemm(false, false, nt, ib, ib, 1.0, W, n, g.T, NBH, 0.0, W2, n, s);
      launch_gemm(false, true, m1, nt, ib, -1.0, g.V + (K + 1), n, W2, n, 1.0, At, lda, s);
      double fl = 2.0 * (K + 1) * (double)ib * (m1 + ib) + 2.0 * n * (double)nt * ib +
                  2.0 * (K + 1) * (double)(ib - 1) * ib + 2.0 * nt * (double)ib * (m1 + ib) +
                  2.0 * m1 * (double)nt * ib;
      int launches = 7;
      if (Q) {   // Q(:, K+1:n) <- Q (I - V T V^T)
        launch_gemm(false, false, n, ib, m1, 1.0, Q + (size_t)(K + 1) * ldq, ldq, g.V + (K + 1), n,
                    0.0, W, n, s);
        launch_gemm(false, false, n, ib, ib, 1.0, W, n, g.T, NBH, 0.0, W2, n, s);
        launch_gemm(false, true, n, m1, ib, -1.0, W2, n, g.V + (K + 1), n, 1.0,
                    Q + (size_t)(K + 1) * ldq, ldq, s);
        fl += 2.0 * n * (double)ib * (m1 + ib) + 2.0 * n * (double)m1 * ib;
        launches += 3;
      }
      HCHECK(hipGetLastError());
      if (time) h->timer.end(s, e0, &h->stats.hess_gemm_ms);
      h->stats.hess_gemm_flops += fl;
      h->stats.launches += launches + 2;
    }
    if (time) {
      HCHECK(hipStreamSynchronize(s));
      h->timer.harvest();
    }
    return 0;
  } catch (const HipErr& e) {
    (void)hipGetLastError();
    return e.e == hipErrorOutOfMemory ? -101 : -102;
  }
}

// ---------------------------------------------------------------------------
// Eigenvectors of a real Schur form (paper Sec. 2, Eqs. (5) and (6)): tile
// rows of about 64 (never splitting a 2x2 block) from the bottom; per tile
// row one launch solves the tile's rows of every eigenvector with entries
// there (overflow-protected back substitution, one thread per eigenvalue)
// and one FP64 MFMA product updates every row above; then the backtransform
// X = Q Y as one product and the normalisation.  The only host
// synchronisation is the read of S's subdiagonal that places the tiles.
// ---------------------------------------------------------------------------
int evec_compute(schur_handle_s* h, hipStream_t s, int n, const double* S, int lds,
                 const double* Q, int ldq, double* X, int ldx) {
  if (n < 0 || n > 524288) return -1;
  if (n == 0) return 0;
  if (!S) return -2;
  if (lds < std::max(1, n)) return -3;
  if (Q && ldq < std::max(1, n)) return -5;
  if (!X) return -6;
  if (ldx < std::max(1, n)) return -7;
  if (!is_device_ptr(S) || (Q && !is_device_ptr(Q)) || !is_device_ptr(X)) return -103;
  try {
    HCHECK(hipSetDevice(h->device));
    std::memset(&h->stats, 0, sizeof(h->stats));
    // tile rows: about 64 rows, extended by one where a 2x2 block would be split
    std::vector<double> sub(std::max(1, n - 1), 0.0);
    if (n > 1) {
      HCHECK(hipMemcpy2DAsync(sub.data(), sizeof(double), S + 1, sizeof(double) * (lds + 1),
                              sizeof(double), n - 1, hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));
    }
    std::vector<int> bnd{0};
    while (bnd.back() < n) {
      int e = std::min(n, bnd.back() + 64);
      if (e < n && sub[e - 1] != 0.0) ++e;   // S(e, e-1) != 0: rows e-1, e form a block
      if (e - bnd.back() > EVTMAX) throw HipErr{hipErrorInvalidValue};
      bnd.push_back(e);
    }
    double* Y = X;
    int ldy = ldx;
    if (Q) {
      Y = (double*)grow(h->b_evy, sizeof(double) * (size_t)n * n, false);
      ldy = n;
    }
    double* wb = (double*)grow(h->b_evb, sizeof(double) * 2 * (size_t)n, false);
    EvArgs g{S, lds, Y, ldy, n, wb, wb + n};
    const bool time = (h->opts.flags & SCHUR_FLAG_TIME_KERNELS) != 0;
    hipEvent_t e0 = nullptr;
    launch_ev_prep(g, s);
    HCHECK(hipGetLastError());
    for (int t = (int)bnd.size() - 2; t >= 0; --t) {
      const int r0 = bnd[t], r1 = bnd[t + 1];
      if (time) h->timer.begin(s, e0);
      launch_ev_diag(g, r0, r1, s);
      HCHECK(hipGetLastError());
      if (time) h->timer.end(s, e0, &h->stats.ev_solve_ms);
      if (r0 > 0) {
        if (time) h->timer.begin(s, e0);
        launch_gemm(false, false, r0, n - r0, r1 - r0, -1.0, S + (size_t)r0 * lds, lds,
                    Y + r0 + (size_t)r0 * ldy, ldy, 1.0, Y + (size_t)r0 * ldy, ldy, s);
        HCHECK(hipGetLastError());
        if (time) h->timer.end(s, e0, &h->stats.ev_gemm_ms);
        h->stats.ev_gemm_flops += 2.0 * r0 * (double)(n - r0) * (r1 - r0);
      }
      h->stats.launches += 1 + (r0 > 0);
    }
    if (Q) {
      if (time) h->timer.begin(s, e0);
      launch_gemm(false, false, n, n, n, 1.0, Q, ldq, Y, ldy, 0.0, X, ldx, s);
      HCHECK(hipGetLastError());
      if (time) h->timer.end(s, e0, &h->stats.ev_back_ms);
      h->stats.ev_back_flops += 2.0 * n * (double)n * n;
      h->stats.launches += 1;
    }
    launch_ev_normalise(X, ldx, S, lds, n, s);
    HCHECK(hipGetLastError());
    h->stats.launches += 3;
    if (time) {
      HCHECK(hipStreamSynchronize(s));
      h->timer.harvest();
    }
    return 0;
  } catch (const HipErr& e) {
    (void)hipGetLastError();
    return e.e == hipErrorOutOfMemory ? -101 : -102;
  }
}

// ---------------------------------------------------------------------------
// Eigenvalue reordering (paper Sec. 2, Eq. (7); Sec. 3.2): the selected
// blocks move to the top in chunks of at most kReorderChunk rows, in
// diagonal order.  A chunk travels up through a chain of diagonal windows
// of at most SMALL_Z_MAX rows: each window holds the chunk's blocks gathered
// so far at its bottom (plus any further blocks of the chunk it covers) and
// moves them to its top; the window's orthogonal factor goes to the row
// panel right of it, the column panel above it and Q.  Chains of later
// chunks follow in lock-step a few time steps behind, each window strictly
// below the windows of earlier chunks at the same time step, so every time
// step is one launch of window tasks and one launch each of left and right
// updates, in a sequentially consistent order (the window / right / left
// update task structure of Sec. 3.2).  The whole schedule is planned on the
// host from the block structure and the selection before anything runs.
// ---------------------------------------------------------------------------
constexpr int kReorderChunk = 32;

struct RWin { int a, w; };

// Plan: per chain (chunk) its windows, per chain its start time step.
// blocks: sizes in diagonal order; sel: selected flags per block.
void plan_reorder(int n, std::vector<int> bsz, std::vector<char> bsel, int W,
                  std::vector<std::vector<RWin>>& chains, std::vector<int>& start) {
  chains.clear();
  start.clear();
  const int nb = (int)bsz.size();
  // row of each block start in the current (simulated) layout
  int ilst = 0, i = 0;
  while (i < nb && bsel[i]) ilst += bsz[i++];   // already leading
  while (true) {
    // the next chunk: selected blocks in order, at most kReorderChunk rows
    // (a block larger than that still forms a chunk of its own)
    int pos = ilst, j = i, kc = 0, last_end = -1, jl = -1;
    std::vector<int> pick;
    for (; j < nb; ++j) {
      if (bsel[j]) {
        if (kc > 0 && kc + bsz[j] > kReorderChunk) break;
        kc += bsz[j];
        last_end = pos + bsz[j];
        jl = j;
        pick.push_back(j);
      }
      pos += bsz[j];
    }
    if (kc == 0) break;
    // blocks i .. jl cover rows [ilst, last_end): simulate the chain on them
    std::vector<int> lsz(bsz.begin() + i, bsz.begin() + jl + 1);
    std::vector<char> lsel(bsel.begin() + i, bsel.begin() + jl + 1);
    std::vector<RWin> chain;
    int bot = last_end;
    while (true) {
      int top = std::max(ilst, bot - W);
      // align top to a block start (never split a 2x2 block)
      int r = ilst;
      size_t b = 0;
      while (b < lsz.size() && r + lsz[b] <= top) r += lsz[b++];
      if (r < top) { r += lsz[b]; ++b; }
      top = r;
      const size_t b0 = b;
      size_t b1 = b0;
      int rr = top;
      while (b1 < lsz.size() && rr < bot) rr += lsz[b1++];
      // stable partition of the window's blocks: the chunk's first
      std::vector<int> s1, s2;
      std::vector<char> f1, f2;
      int kin = 0;
      for (size_t q = b0; q < b1; ++q) {
        if (lsel[q]) { s1.push_back(lsz[q]); f1.push_back(1); kin += lsz[q]; }
        else { s2.push_back(lsz[q]); f2.push_back(0); }
      }
      size_t q = b0;
      for (size_t u = 0; u < s1.size(); ++u, ++q) { lsz[q] = s1[u]; lsel[q] = 1; }
      for (size_t u = 0; u < s2.size(); ++u, ++q) { lsz[q] = s2[u]; lsel[q] = 0; }
      chain.push_back({top, bot - top});
      if (top <= ilst) break;
      bot = top + kin;
    }
    chains.push_back(chain);
    // the global layout after the chunk: its blocks first, the rest in order
    for (size_t q = 0; q < lsz.size(); ++q) { bsz[i + q] = lsz[q]; bsel[i + q] = lsel[q]; }
    // blocks moved to the top are done; mark them unselected for later chunks
    int moved = 0;
    while (moved < kc) { moved += bsz[i]; bsel[i] = 0; ++i; }
    ilst += kc;
  }
  // start times: each chain a time step after the previous one at least, and
  // at every time step strictly below the windows of all earlier chains
  for (size_t c = 0; c < chains.size(); ++c) {
    int s0 = c == 0 ? 0 : start[c - 1] + 1;
    for (;; ++s0) {
      bool ok = true;
      for (size_t d = 0; d < c && ok; ++d) {
        for (size_t t = 0; t < chains[c].size() && ok; ++t) {
          const int tt = s0 + (int)t - start[d];
          if (tt < 0 || tt >= (int)chains[d].size()) continue;
          const RWin& x = chains[c][t];
          const RWin& y = chains[d][tt];
          if (x.a < y.a + y.w) ok = false;
        }
      }
      if (ok) break;
    }
    start.push_back(s0);
  }
}

int reorder_run(schur_handle_s* h, hipStream_t s, int n, double* S, int lds, double* Q, int ldq,
                const int* select, double* wr, double* wi, int* m_out) {
  if (n < 0 || n > 524288) return -1;
  if (n == 0) { if (m_out) *m_out = 0; return 0; }
  if (!S) return -2;
  if (lds < std::max(1, n) || lds > LD_MAX) return -3;
  if (Q && (ldq < std::max(1, n) || ldq > LD_MAX)) return -5;
  if (!select) return -6;
  if (!wr) return -7;
  if (!wi) return -8;
  if (!is_device_ptr(S) || (Q && !is_device_ptr(Q)) || !is_device_ptr(wr) || !is_device_ptr(wi))
    return -103;
  try {
    HCHECK(hipSetDevice(h->device));
    std::memset(&h->stats, 0, sizeof(h->stats));
    int rc = alloc_ws(h, n);
    if (rc) return rc;
    // block structure from S's subdiagonal
    std::vector<double> sub(std::max(1, n - 1), 0.0);
    if (n > 1) {
      HCHECK(hipMemcpy2DAsync(sub.data(), sizeof(double), S + 1, sizeof(double) * (lds + 1),
                              sizeof(double), n - 1, hipMemcpyDeviceToHost, s));
      HCHECK(hipStreamSynchronize(s));
    }
    std::vector<int> bsz;
    std::vector<char> bsel;
    std::vector<unsigned char> rows(n, 0);
    int m = 0;
    for (int k = 0; k < n;) {
      const int sz = (k + 1 < n && sub[k] != 0.0) ? 2 : 1;
      const bool on = select[k] != 0 || (sz == 2 && select[k + 1] != 0);
      bsz.push_back(sz);
      bsel.push_back(on ? 1 : 0);
      for (int q = 0; q < sz; ++q) rows[k + q] = on ? 1 : 0;
      if (on) m += sz;
      k += sz;
    }
    if (m_out) *m_out = m;
    std::vector<std::vector<RWin>> chains;
    std::vector<int> start;
    plan_reorder(n, bsz, bsel, SMALL_Z_MAX, chains, start);
    int T = 0;
    for (size_t c = 0; c < chains.size(); ++c) T = std::max(T, start[c] + (int)chains[c].size());
    // windows per time step (top to bottom = chains in order)
    std::vector<std::vector<RWin>> steps(T);
    for (size_t c = 0; c < chains.size(); ++c)
      for (size_t t = 0; t < chains[c].size(); ++t) steps[start[c] + t].push_back(chains[c][t]);
    size_t total = 0, maxw = 1;
    for (const auto& st : steps) { total += st.size(); maxw = std::max(maxw, st.size()); }
    // device buffers: row flags (+ info), tasks and panel descriptors of the
    // whole schedule, U slots for the widest time step
    unsigned char* seld = (unsigned char*)grow(h->b_rsel, (size_t)n + 64, true);
    int* infod = (int*)(seld + (((size_t)n + 15) & ~(size_t)15));
    std::memcpy(h->b_rsel.host, rows.data(), (size_t)n);
    std::memset((unsigned char*)h->b_rsel.host + (((size_t)n + 15) & ~(size_t)15), 0, sizeof(int));
    HCHECK(hipMemcpyAsync(seld, h->b_rsel.host, (((size_t)n + 15) & ~(size_t)15) + sizeof(int),
                          hipMemcpyHostToDevice, s));
    double* uslots =
        (double*)grow(h->b_ru, sizeof(double) * (size_t)UPAD * UPAD * maxw, false);
    ReorderTask* td = (ReorderTask*)grow(h->b_rtask, sizeof(ReorderTask) * std::max<size_t>(1, total), true);
    WinB* wd = (WinB*)grow(h->b_rwin, sizeof(WinB) * std::max<size_t>(1, total), true);
    ReorderTask* th = (ReorderTask*)h->b_rtask.host;
    WinB* wh = (WinB*)h->b_rwin.host;
    std::vector<int> tr_t(T, 0), tcq_t(T, 0);
    std::vector<size_t> off(T + 1, 0);
    for (int t = 0; t < T; ++t) {
      off[t + 1] = off[t] + steps[t].size();
      int tr = 0, tcq = 0;
      for (size_t q = 0; q < steps[t].size(); ++q) {
        const RWin& rw = steps[t][q];
        if (rw.w < 1 || rw.w > SMALL_Z_MAX || rw.a < 0 || rw.a + rw.w > n)
          throw HipErr{hipErrorInvalidValue};
        const size_t k = off[t] + q;
        double* slot = uslots + q * (size_t)UPAD * UPAD;
        ReorderTask& rt = th[k];
        std::memset(&rt, 0, sizeof(rt));
        rt.S = S; rt.lds = lds; rt.a = rw.a; rt.w = rw.w; rt.sel = seld;
        rt.Ut = slot; rt.ldut = UPAD; rt.info = infod;
        WinB& w = wh[k];
        std::memset(&w, 0, sizeof(w));
        w.c.H = S; w.c.Q = Q; w.c.U = slot; w.c.st = nullptr;
        w.c.ldh = lds; w.c.ldq = ldq; w.c.n = n;
        w.c.ktop = 0; w.c.kbot = n - 1; w.c.rtop = 0; w.c.cend = n;
        w.c.p = rw.a; w.c.ws = rw.w;
        fill_tiles_b(w, tr, tcq, h->stats, PANEL_TPB_WIDE);
      }
      tr_t[t] = tr;
      tcq_t[t] = tcq;
    }
    if (total > 0) {
      HCHECK(hipMemcpyAsync(td, th, sizeof(ReorderTask) * total, hipMemcpyHostToDevice, s));
      HCHECK(hipMemcpyAsync(wd, wh, sizeof(WinB) * total, hipMemcpyHostToDevice, s));
    }
    const bool time = (h->opts.flags & SCHUR_FLAG_TIME_KERNELS) != 0;
    hipEvent_t e0 = nullptr;
    for (int t = 0; t < T; ++t) {
      const int nw = (int)steps[t].size();
      if (nw == 0) continue;
      if (time) h->timer.begin(s, e0);
      launch_reorder(td + off[t], nw, s);
      HCHECK(hipGetLastError());
      if (time) h->timer.end(s, e0, &h->stats.reorder_ms);
      if (tr_t[t] > 0) {
        if (time) h->timer.begin(s, e0);
        launch_panel_row_b(wd + off[t], nw, tr_t[t], s);
        HCHECK(hipGetLastError());
        if (time) h->timer.end(s, e0, &h->stats.row_ms);
        h->stats.row_launches += 1;
      }
      if (tcq_t[t] > 0) {
        if (time) h->timer.begin(s, e0);
        launch_panel_colq_b(wd + off[t], nw, tcq_t[t], s);
        HCHECK(hipGetLastError());
        if (time) h->timer.end(s, e0, &h->stats.colq_ms);
        h->stats.colq_launches += 1;
      }
      h->stats.launches += 1 + (tr_t[t] > 0) + (tcq_t[t] > 0);
      h->stats.reorder_windows += nw;
    }
    h->stats.reorder_steps = T;
    // eigenvalues in the new diagonal order (the blocks are standard already)
    launch_standardize(S, lds, Q, ldq, n, 1, wr, wi, h->blist, h->bcount, h->blist_cap, s);
    HCHECK(hipGetLastError());
    int info = 0;
    HCHECK(hipMemcpyAsync(&info, infod, sizeof(int), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    if (time) h->timer.harvest();
    h->stats.gemm_ms = h->stats.row_ms + h->stats.colq_ms;
    return info ? 1 : 0;
  } catch (const HipErr& e) {
    (void)hipGetLastError();
    return e.e == hipErrorOutOfMemory ? -101 : -102;
  }
}

// ---------------------------------------------------------------------------
// Entry point that allocates nothing (schur_reduce_noalloc).  Its workspace
// lives in one static device array per GPU, carved as below: U slots of one
// time step (a single stream needs no ring of buffers), the reflector log,
// shift and eigenvalue buffers, the control block and the block list of the
// standardisation for orders up to SCHUR_NOALLOC_MAX_N.  The array's name is
// a host-side stand-in in host code: kernels get the address
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNaU = align256(sizeof(double) * (size_t)MAXWIN * UPAD * UPAD);
constexpr size_t kNaRefl = align256(sizeof(double) * (size_t)MAXWIN * REFL_STRIDE);
constexpr size_t kNaVec = align256(sizeof(double) * NSMAX);
constexpr size_t kNaCtrl = align256(sizeof(Ctrl));
constexpr size_t kNaCount = 256;
constexpr int kNaBlist = SCHUR_NOALLOC_MAX_N / 2 + 2;
constexpr size_t kNaBytes =
    kNaU + kNaRefl + 3 * kNaVec + kNaCtrl + kNaCount + align256(sizeof(int) * (size_t)kNaBlist);

static_assert(kNaBytes == SCHUR_NOALLOC_SCRATCH_BYTES, "workspace size stated in schur.h");
static __device__ __align__(256) unsigned char scratch[kNaBytes];

struct NoAllocDev {
  schur_handle_s* h = nullptr;   // host-side state; its buffers point into scratch
  Ctrl ctrl_host{};              // host mirror of the control block
  std::mutex mu;                 // calls on one device run one at a time
};
NoAllocDev g_na[64];
std::mutex g_na_setup;

// once per device, with that device current: the device address of its copy
// of the array, carved into the handle's buffers
int noalloc_setup(int dev) {
  std::lock_guard<std::mutex> lk(g_na_setup);
  NoAllocDev& d = g_na[dev];
  if (d.h) return 0;
  void* base = nullptr;
  if (hipGetSymbolAddress(&base, HIP_SYMBOL(scratch)) != hipSuccess || !base) {
    (void)hipGetLastError();
    return -102;
  }
  unsigned char* b = (unsigned char*)base;
  schur_handle_s* h = new schur_handle_s();
  h->device = dev;
  h->U = (double*)b;      b += kNaU;
  h->refl = (double*)b;   b += kNaRefl;
  h->st = (double*)b;     b += kNaVec;
  h->ewr = (double*)b;    b += kNaVec;
  h->ewi = (double*)b;    b += kNaVec;
  h->ctrl = (Ctrl*)b;     b += kNaCtrl;
  h->bcount = (int*)b;    b += kNaCount;
  h->blist = (int*)b;
  h->blist_cap = kNaBlist;
  h->ctrl_h = &d.ctrl_host;
  d.h = h;
  return 0;
}

int solve_noalloc(hipStream_t s, int n, double* H, int ldh, double* Q, int ldq, double* wr,
                  double* wi) {
  int rc = check_args(n, H, ldh, Q, ldq, wr, wi);
  if (rc != 0) return rc;
  if (n > SCHUR_NOALLOC_MAX_N) return -106;
  if (n == 0) return 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -102;
  rc = noalloc_setup(dev);
  if (rc) return rc;
  NoAllocDev& d = g_na[dev];
  std::lock_guard<std::mutex> lk(d.mu);
  schur_handle_s* h = d.h;
  try {
    std::memset(&h->stats, 0, sizeof(h->stats));
    Params P = resolve(schur_opts{}, n);
    P.split_nw = 0;                        // the passes need per-window workspace
    P.ns = std::min(P.ns, SMALL_EIG_MAX);  // shifts without a nested solve
    P.time = false;                        // timing needs events
    Solver sv{h, s, P, n, H, ldh, Q, ldq, wr, wi};
    sv.one_stream = true;
    return sv.run();
  } catch (const HipErr& e) {
    (void)hipGetLastError();
    return -102;
  }
}

// ---------------------------------------------------------------------------
// Batched engine: independent matrices advance in rounds.  A round is one
// batched deflation scan (one workgroup per matrix, with converged bottom
// blocks peeled and standardised at once), one batched small-block solve
// for the matrices whose active block is small, one batched shift solve, and
// one sweep for every other matrix -- the sweeps' time steps are merged so
// that each launch carries the windows (or panel tiles) of all matrices.
// Matrices can be added between rounds (continuous batching); each matrix
// owns a fixed slot (control block and shift buffers) until it retires.
// ---------------------------------------------------------------------------
struct BatchEngine {
  schur_handle_s* h = nullptr;
  hipStream_t s = nullptr;
  int cap = 0;                       // slots
  struct Mat {
    int n = 0, ldh = 1, ldq = 1;
    double *H = nullptr, *Q = nullptr, *wr = nullptr, *wi = nullptr;
    int kbot = -1, ktop = 0, info = 0, nodefl = 0;
    int last_small_top = -1;         // ktop of the last small-block solve (-1: none)
    int64_t sweeps = 0;
    bool used = false, active = false, checked = false;
    Params P{};
    uint64_t tag = 0;
  };
  std::vector<Mat> M;
  Ctrl* ctrl_d = nullptr;
  Ctrl* ctrl_h = nullptr;
  double* shbuf = nullptr;
  int64_t rounds = 0;
  // hold small active blocks back while any matrix still sweeps, so that
  // they are solved by one launch (for blocks of one matrix that must all
  // finish before anything else runs)
  bool defer_small = false;
  // run the parallel early-deflation passes on large matrices (off for the
  // engine that finishes the blocks those passes leave)
  bool allow_split = true;
  // time the kernel families with HIP events into the handle's counters
  bool time = false;
  hipEvent_t e0 = nullptr;
  void tbeg() { if (time) h->timer.begin(s, e0); }
  void tend(double* acc) { if (time) h->timer.end(s, e0, acc); }
  void sync() {
    HCHECK(hipStreamSynchronize(s));
    if (time) h->timer.harvest();
  }

  template <class T>
  T* dev_of(schur_handle_s::Grow& g) { return (T*)g.dev; }
  template <class T>
  T* host_of(schur_handle_s::Grow& g) { return (T*)g.host; }

  void upload(schur_handle_s::Grow& g, size_t bytes) {
    if (bytes) HCHECK(hipMemcpyAsync(g.dev, g.host, bytes, hipMemcpyHostToDevice, s));
  }

  void init(schur_handle_s* hh, hipStream_t ss, int slots) {
    h = hh;
    s = ss;
    cap = slots;
    M.assign(slots, Mat{});
    grow(h->b_ctrl, sizeof(Ctrl) * slots, true);
    grow(h->b_defl, sizeof(DeflB) * slots, true);
    grow(h->b_sh, sizeof(double) * 3 * SMALL_EIG_MAX * (size_t)slots, false);
    ctrl_d = dev_of<Ctrl>(h->b_ctrl);
    ctrl_h = host_of<Ctrl>(h->b_ctrl);
    shbuf = dev_of<double>(h->b_sh);
    HCHECK(hipMemsetAsync(ctrl_d, 0, sizeof(Ctrl) * slots, s));
    rounds = 0;
  }

  int free_slot() const {
    for (int i = 0; i < cap; ++i) if (!M[i].used) return i;
    return -1;
  }

  // Register a matrix in slot i (device buffers owned by the caller).  The
  // input check runs with the next round.
  void add(int i, int n, double* H, int ldh, double* Q, int ldq, double* wr, double* wi,
           uint64_t tag) {
    Mat& m = M[i];
    m = Mat{};
    m.used = true;
    m.n = n; m.H = H; m.ldh = ldh; m.Q = Q; m.ldq = Q ? ldq : 1; m.wr = wr; m.wi = wi;
    m.tag = tag;
    m.info = 0;
    m.active = n > 0;
    m.kbot = n - 1;
    m.P = resolve(h->opts, std::max(1, n));
    HCHECK(hipMemsetAsync(ctrl_d + i, 0, sizeof(Ctrl), s));
  }

  void release(int i) { M[i] = Mat{}; }

  bool any_active() const {
    for (const Mat& m : M) if (m.used && m.active) return true;
    return false;
  }

  // input check (non-finite entries -> info -2) and zeroing below the
  // subdiagonal for matrices added since the last round
  void check_new() {
    bool any = false;
    for (int i = 0; i < cap; ++i) {
      Mat& m = M[i];
      if (!m.used || !m.active || m.checked) continue;
      launch_check_finite(m.H, m.ldh, m.n, ctrl_d + i, s);
      any = true;
    }
    if (!any) return;
    HCHECK(hipMemcpyAsync(ctrl_h, ctrl_d, sizeof(Ctrl) * cap, hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    for (int i = 0; i < cap; ++i) {
      Mat& m = M[i];
      if (!m.used || !m.active || m.checked) continue;
      m.checked = true;
      if (ctrl_h[i].bad) { m.info = -2; m.active = false; continue; }
      launch_zero_lower(m.H, m.ldh, m.n, s);
      if (allow_split && m.P.split_nw > 0 && m.n >= m.P.split_min_n) split_passes(m);
    }
  }

  // the parallel early-deflation passes of a single solve on one large
  // matrix (on a side handle's buffers), before its rounds start
  void split_passes(Mat& m) {
    if (!h->side) {
      schur_handle_s* side = nullptr;
      if (create_handle(&side, h->device, &h->opts) != 0) throw HipErr{hipErrorOutOfMemory};
      h->side = side;
    }
    Solver sv{h->side, s, m.P, m.n, m.H, m.ldh, m.Q, m.ldq, m.wr, m.wi};
    sv.P.time = false;
    sv.split_phase();
    h->stats.split_passes += h->side->stats.split_passes;
    h->stats.split_windows += h->side->stats.split_windows;
    h->stats.split_accepted += h->side->stats.split_accepted;
    std::memset(&h->side->stats, 0, sizeof(h->side->stats));
  }

  // One round.  Afterwards, matrices with used && !active are finished
  // (info set) once the stream has drained; the caller retires them.
  void round() {
    check_new();
    if (++rounds > (int64_t)1 << 40) throw HipErr{hipErrorUnknown};
    std::vector<int> idx;
    for (int i = 0; i < cap; ++i) if (M[i].used && M[i].active) idx.push_back(i);
    if (idx.empty()) return;
    // ---- deflation scan of every active matrix
    DeflB* dh = host_of<DeflB>(h->b_defl);
    for (size_t q = 0; q < idx.size(); ++q) {
      Mat& m = M[idx[q]];
      dh[q] = DeflB{m.H, m.Q, m.wr, m.wi, m.ldh, m.ldq, m.n, m.kbot, ctrl_d + idx[q]};
    }
    upload(h->b_defl, sizeof(DeflB) * idx.size());
    tbeg();
    launch_deflate_b(dev_of<DeflB>(h->b_defl), (int)idx.size(), s);
    HCHECK(hipGetLastError());
    tend(&h->stats.other_ms);
    h->stats.launches += 1;
    HCHECK(hipMemcpyAsync(ctrl_h, ctrl_d, sizeof(Ctrl) * cap, hipMemcpyDeviceToHost, s));
    sync();
    // ---- classify
    std::vector<int> small, big;
    for (int i : idx) {
      Mat& m = M[i];
      if (ctrl_h[i].bad) {                   // a non-finite value appeared
        m.info = kErrNonFinite;
        m.active = false;
        continue;
      }
      if (ctrl_h[i].small_info != 0) {       // the last small-block solve failed
        m.info = m.last_small_top + ctrl_h[i].small_info;
        m.active = false;
        continue;
      }
      const int nk = ctrl_h[i].kbot;
      if (nk < m.kbot) m.nodefl = 0;
      m.kbot = nk;
      m.ktop = ctrl_h[i].ktop;
      if (m.kbot < 0) { m.active = false; continue; }
      const int len = m.kbot - m.ktop + 1;
      if (len <= m.P.nmin) small.push_back(i);
      else if (++m.sweeps > m.P.max_sweeps) { m.info = m.kbot + 1; m.active = false; }
      else big.push_back(i);
    }
    if (defer_small && !big.empty()) small.clear();
    if (small.empty() && big.empty()) return;
    // U slots: one per small block, per early-deflation window, and per
    // window of the widest sweep time step (at most one per bulge group)
    size_t gsum = 0;
    for (int i : big) {
      const Mat& m = M[i];
      const int len = m.kbot - m.ktop + 1;
      const int ns = std::max(2, std::min(std::min(m.P.ns, SMALL_EIG_MAX), 2 * ((len - 2) / 6)));
      gsum += (size_t)((ns / 2 + m.P.nb - 1) / m.P.nb);
    }
    const size_t nslots = std::max(std::max(gsum, small.size()), big.size());
    double* Ubase =
        (double*)grow(h->b_u, sizeof(double) * UPAD * UPAD * std::max<size_t>(1, nslots), false);
    // ---- small blocks: one workgroup each; whole small matrices accumulate Q
    // in the kernel, blocks of larger matrices apply Z as panel products
    if (!small.empty()) {
      grow(h->b_small, sizeof(SmallTask) * small.size(), true);
      grow(h->b_win, sizeof(WinB) * small.size(), true);
      SmallTask* th = host_of<SmallTask>(h->b_small);
      WinB* wh = host_of<WinB>(h->b_win);
      int nwin = 0, tr = 0, tcq = 0;
      int maxm = 0;
      for (size_t q = 0; q < small.size(); ++q) {
        Mat& m = M[small[q]];
        const int len = m.kbot - m.ktop + 1;
        maxm = std::max(maxm, len);
        const bool whole = (m.ktop == 0 && m.kbot == m.n - 1);
        m.last_small_top = m.ktop;
        SmallTask t{};
        t.A = m.H + m.ktop + (size_t)m.ktop * m.ldh;
        t.lda = m.ldh;
        t.m = len;
        t.wr = m.wr + m.ktop;
        t.wi = m.wi + m.ktop;
        t.info = &ctrl_d[small[q]].small_info;
        t.itmax = 0;   // default budget
        double* slot = Ubase + (size_t)q * UPAD * UPAD;
        if (whole) {
          t.Qacc = m.Q;
          t.ldqacc = m.ldq;
        } else {
          t.Zt = slot;
          t.ldzt = UPAD;
          WinB& w = wh[nwin++];
          std::memset(&w, 0, sizeof(w));
          w.c.H = m.H; w.c.Q = m.Q; w.c.U = slot; w.c.st = nullptr;
          w.c.ldh = m.ldh; w.c.ldq = m.ldq; w.c.n = m.n;
          w.c.ktop = m.ktop; w.c.kbot = m.kbot; w.c.rtop = 0; w.c.cend = m.n;
          w.c.p = m.ktop; w.c.ws = len;
          fill_tiles(w, tr, tcq);
        }
        th[q] = t;
        m.kbot = m.ktop - 1;     // the block is finished by this round's launches
        if (m.kbot < 0) m.active = false;   // a failure is read from its ctrl later
        h->stats.small_solves += 1;
        h->stats.small_flops += 25.0 * len * (double)len * len;
      }
      upload(h->b_small, sizeof(SmallTask) * small.size());
      tbeg();
      launch_small_tasks(dev_of<SmallTask>(h->b_small), (int)small.size(), maxm, true, s);
      HCHECK(hipGetLastError());
      tend(&h->stats.small_ms);
      h->stats.launches += 1;
      h->stats.small_launches += 1;
      if (nwin > 0) {
        upload(h->b_win, sizeof(WinB) * nwin);
        panels(dev_of<WinB>(h->b_win), nwin, tr, tcq);
      }
      if (!big.empty()) sync();   // slots and staging reused below
    }
    if (big.empty()) return;
    // ---- early deflation: one workgroup per matrix, then V applied to the
    // rest of each matrix and to its Q by the panel kernels
    std::vector<int> aed_nu(big.size(), 0), sweep_it(big.size(), 1);
    {
      std::vector<int> who;
      grow(h->b_aedt, sizeof(AedTask) * big.size(), true);
      AedTask* ah = host_of<AedTask>(h->b_aedt);
      std::vector<int> nwv(big.size(), 0);
      for (size_t q = 0; q < big.size(); ++q) {
        Mat& m = M[big[q]];
        const int len = m.kbot - m.ktop + 1;
        const int nw = std::min(m.P.nw, len - 1);
        if (nw < 4) continue;
        nwv[q] = nw;
        double* base = shbuf + (size_t)big[q] * 3 * SMALL_EIG_MAX;
        AedTask t{};
        t.H = m.H; t.ldh = m.ldh;
        t.ktop = m.ktop; t.kbot = m.kbot; t.nw = nw;
        t.Ut = Ubase + who.size() * (size_t)UPAD * UPAD;
        t.ldut = UPAD;
        t.sr = base; t.si = base + SMALL_EIG_MAX;
        t.wr = m.wr + (m.kbot - nw + 1); t.wi = m.wi + (m.kbot - nw + 1);
        t.ctrl = ctrl_d + big[q];
        t.itmax = 0;   // default budget
        ah[who.size()] = t;
        who.push_back((int)q);
      }
      if (!who.empty()) {
        upload(h->b_aedt, sizeof(AedTask) * who.size());
        tbeg();
        launch_aed_b(dev_of<AedTask>(h->b_aedt), (int)who.size(), s);
        HCHECK(hipGetLastError());
        tend(&h->stats.aed_ms);
        h->stats.launches += 1;
        h->stats.aed_launches += 1;
        h->stats.aed_windows += (int64_t)who.size();
        HCHECK(hipMemcpyAsync(ctrl_h, ctrl_d, sizeof(Ctrl) * cap, hipMemcpyDeviceToHost, s));
        sync();
        grow(h->b_aedw, sizeof(WinB) * who.size(), true);
        WinB* wh = host_of<WinB>(h->b_aedw);
        int nwin = 0, tr = 0, tcq = 0;
        for (size_t j = 0; j < who.size(); ++j) {
          const int q = who[j];
          Mat& m = M[big[q]];
          const int nd = ctrl_h[big[q]].aed_nd;
          aed_nu[q] = ctrl_h[big[q]].aed_nu;
          h->stats.aed_flops += aed_work(nwv[q], nd > 0 ? aed_nu[q] : 0);
          if (nd <= 0) continue;
          WinB& w = wh[nwin++];
          std::memset(&w, 0, sizeof(w));
          w.c.H = m.H; w.c.Q = m.Q; w.c.U = Ubase + j * (size_t)UPAD * UPAD; w.c.st = nullptr;
          w.c.ldh = m.ldh; w.c.ldq = m.ldq; w.c.n = m.n;
          w.c.ktop = m.ktop; w.c.kbot = m.kbot; w.c.rtop = 0; w.c.cend = m.n;
          w.c.p = m.kbot - nwv[q] + 1; w.c.ws = nwv[q];
          fill_tiles(w, tr, tcq);
          m.kbot -= nd;
          m.nodefl = 0;
          h->stats.aed_deflated += nd;
          if ((m.P.nibble >= 0 && 100 * nd > m.P.nibble * nwv[q]) || m.kbot - m.ktop + 1 <= m.P.nmin)
            sweep_it[q] = 0;
        }
        if (nwin > 0) {
          upload(h->b_aedw, sizeof(WinB) * nwin);
          panels(dev_of<WinB>(h->b_aedw), nwin, tr, tcq);
        }
      }
    }
    // ---- sweep plans with the (possibly shrunk) active blocks
    std::vector<std::vector<std::vector<WinPlan>>> plans(big.size());
    std::vector<int> nsv(big.size(), 0), use_aed(big.size(), 0);
    size_t maxw = 0, tmax = 0;
    for (size_t q = 0; q < big.size(); ++q) {
      if (!sweep_it[q]) continue;
      Mat& m = M[big[q]];
      const int len = m.kbot - m.ktop + 1;
      int ns = std::min(std::min(m.P.ns, SMALL_EIG_MAX), 2 * ((len - 2) / 6));
      if (ns < 2) ns = 2;
      const bool exc = (m.nodefl > 0 && m.nodefl % m.P.exc_period == 0);
      if (!exc && aed_nu[q] >= 2 && 2 * aed_nu[q] >= ns) {
        ns = std::min(ns, aed_nu[q]) & ~1;
        use_aed[q] = 1;
      }
      nsv[q] = ns;
      int step = 0;
      plan_sweep(m.ktop, m.kbot, ns / 2, m.P.nb, m.P.step, plans[q], step);
      tmax = std::max(tmax, plans[q].size());
    }
    std::vector<size_t> per_t(tmax, 0);
    for (size_t q = 0; q < big.size(); ++q)
      for (size_t t = 0; t < plans[q].size(); ++t) per_t[t] += plans[q][t].size();
    for (size_t t = 0; t < tmax; ++t) maxw = std::max(maxw, per_t[t]);
    if (maxw > nslots) throw HipErr{hipErrorInvalidValue};
    if (tmax == 0) return;
    // ---- shifts: undeflated window eigenvalues, else eigenvalues of the
    // trailing blocks (or ad-hoc pairs)
    {
      grow(h->b_small, sizeof(SmallTask) * big.size(), true);
      grow(h->b_shift, sizeof(ShiftB) * big.size(), true);
      SmallTask* th = host_of<SmallTask>(h->b_small);
      ShiftB* sh = host_of<ShiftB>(h->b_shift);
      int ne = 0, maxns = 0, nsh = 0;
      for (size_t q = 0; q < big.size(); ++q) {
        if (!sweep_it[q]) continue;
        Mat& m = M[big[q]];
        const int ns = nsv[q];
        double* base = shbuf + (size_t)big[q] * 3 * SMALL_EIG_MAX;
        const bool exc = (m.nodefl > 0 && m.nodefl % m.P.exc_period == 0);
        if (use_aed[q]) {
          const int off = aed_nu[q] - ns;
          sh[nsh++] = ShiftB{base + off, base + SMALL_EIG_MAX + off, nullptr, m.H,
                             base + 2 * SMALL_EIG_MAX, ns, 0, m.ldh, m.ktop, m.kbot, 0};
        } else {
          if (!exc) {
            SmallTask t{};
            const int b0 = m.kbot - ns + 1;
            t.A = m.H + b0 + (size_t)b0 * m.ldh;
            t.lda = m.ldh;
            t.m = ns;
            t.wr = base;
            t.wi = base + SMALL_EIG_MAX;
            t.info = &ctrl_d[big[q]].nshift;   // per-matrix scratch for the shift solve
            t.itmax = 0;   // default budget
            th[ne++] = t;
            maxns = std::max(maxns, ns);
            h->stats.small_flops += 10.0 * ns * (double)ns * ns;
          }
          sh[nsh++] = ShiftB{base, base + SMALL_EIG_MAX, exc ? nullptr : &ctrl_d[big[q]].nshift,
                             m.H, base + 2 * SMALL_EIG_MAX, ns, exc ? 1 : 0, m.ldh, m.ktop, m.kbot,
                             0};
        }
        ++m.nodefl;
        h->stats.sweeps += 1;
        h->stats.shifts_applied += ns;
      }
      upload(h->b_small, sizeof(SmallTask) * ne);
      upload(h->b_shift, sizeof(ShiftB) * nsh);
      tbeg();
      if (ne > 0) launch_small_tasks(dev_of<SmallTask>(h->b_small), ne, maxns, false, s);
      launch_shift_prep_b(dev_of<ShiftB>(h->b_shift), nsh, s);
      HCHECK(hipGetLastError());
      tend(&h->stats.shift_ms);
      h->stats.launches += 1 + (ne > 0);
    }
    // ---- merged sweeps: time step t carries the windows of every matrix
    {
      size_t total = 0;
      for (size_t t = 0; t < tmax; ++t) total += per_t[t];
      grow(h->b_win, sizeof(WinB) * std::max<size_t>(1, total), true);
      WinB* wh = host_of<WinB>(h->b_win);
      std::vector<size_t> off(tmax + 1, 0);
      std::vector<int> tr_t(tmax, 0), tcq_t(tmax, 0);
      for (size_t t = 0; t < tmax; ++t) {
        off[t + 1] = off[t] + per_t[t];
        size_t k = off[t];
        int tr = 0, tcq = 0;
        for (size_t q = 0; q < big.size(); ++q) {
          if (t >= plans[q].size()) continue;
          Mat& m = M[big[q]];
          const double* st = shbuf + (size_t)big[q] * 3 * SMALL_EIG_MAX + 2 * SMALL_EIG_MAX;
          for (const WinPlan& pl : plans[q][t]) {
            if (pl.ws > WMAX || pl.ws < 3 || pl.p < m.ktop || pl.p + pl.ws - 1 > m.kbot ||
                (pl.tau1 - pl.tau0) * pl.nb > REFL_LDS || pl.nb > NBMAX)
              throw HipErr{hipErrorInvalidValue};
            WinB& w = wh[k];
            std::memset(&w, 0, sizeof(w));
            w.c.H = m.H; w.c.Q = m.Q;
            w.c.U = Ubase + (k - off[t]) * (size_t)UPAD * UPAD;
            w.c.st = st + 2 * pl.shift0;
            w.c.ldh = m.ldh; w.c.ldq = m.ldq; w.c.n = m.n;
            w.c.ktop = m.ktop; w.c.kbot = m.kbot; w.c.rtop = 0; w.c.cend = m.n;
            w.c.p = pl.p; w.c.ws = pl.ws; w.c.tau0 = pl.tau0; w.c.tau1 = pl.tau1;
            w.c.nb = pl.nb;
            fill_tiles(w, tr, tcq);
            ++k;
            h->stats.windows += 1;
            h->stats.chain_steps += pl.tau1 - pl.tau0;
            h->stats.chase_flops += chase_work(pl.ws, pl.nb, pl.tau1 - pl.tau0);
            h->stats.chase_bytes += 24.0 * (double)pl.ws * (double)pl.ws;
          }
        }
        tr_t[t] = tr;
        tcq_t[t] = tcq;
      }
      upload(h->b_win, sizeof(WinB) * total);
      WinB* wd = dev_of<WinB>(h->b_win);
      for (size_t t = 0; t < tmax; ++t) {
        const int nw = (int)per_t[t];
        if (nw == 0) continue;
        tbeg();
        launch_chase_b(wd + off[t], nw, s);
        HCHECK(hipGetLastError());
        tend(&h->stats.chase_ms);
        h->stats.chase_launches += 1;
        h->stats.launches += 1;
        panels(wd + off[t], nw, tr_t[t], tcq_t[t]);
      }
    }
  }

  // Wait for the stream, then report small-block failures of matrices that
  // finished inside the last launches.
  void settle() {
    HCHECK(hipMemcpyAsync(ctrl_h, ctrl_d, sizeof(Ctrl) * cap, hipMemcpyDeviceToHost, s));
    sync();
    for (int i = 0; i < cap; ++i) {
      Mat& m = M[i];
      if (m.used && !m.active && m.info == 0 && m.last_small_top >= 0 && ctrl_h[i].small_info != 0)
        m.info = m.last_small_top + ctrl_h[i].small_info;
    }
  }

  void fill_tiles(WinB& w, int& tr, int& tcq) {
    fill_tiles_b(w, tr, tcq, h->stats, PANEL_TPB_BATCH);
  }

  // row-panel and column-panel/Q products of `nwin` windows (descriptors on
  // the device)
  void panels(const WinB* wd, int nwin, int tr, int tcq) {
    if (tr > 0) {
      tbeg();
      launch_panel_row_b(wd, nwin, tr, s);
      HCHECK(hipGetLastError());
      tend(&h->stats.row_ms);
      h->stats.row_launches += 1;
    }
    if (tcq > 0) {
      tbeg();
      launch_panel_colq_b(wd, nwin, tcq, s);
      HCHECK(hipGetLastError());
      tend(&h->stats.colq_ms);
      h->stats.colq_launches += 1;
    }
    h->stats.gemm_launches += (tr > 0) + (tcq > 0);
    h->stats.launches += (tr > 0) + (tcq > 0);
  }
};

// Independent unreduced blocks [lo, hi] of one matrix (order <= UPAD each)
// solved together by the batched engine, in place in H, each with its own Z
// accumulated in a slot; then Z^T X for the rows right of each block, X Z for
// the rows above it and for Q, in one row-panel and one column-panel launch.
// Returns true when every block reached Schur form.
bool batch_blocks(schur_handle_s* h, hipStream_t s, const std::vector<std::pair<int, int>>& blocks,
                  int n, double* H, int ldh, double* Q, int ldq, double* wr, double* wi,
                  bool time) {
  const int cnt = (int)blocks.size();
  if (cnt == 0) return true;
  const size_t slot = (size_t)UPAD * UPAD;
  grow(h->b_splq, sizeof(double) * slot * cnt, false);
  grow(h->b_splu, sizeof(double) * slot * cnt, false);
  grow(h->b_splb, sizeof(int) * cnt, true);
  double* zq = (double*)h->b_splq.dev;
  double* ut = (double*)h->b_splu.dev;
  int* sz = (int*)h->b_splb.host;
  for (int i = 0; i < cnt; ++i) {
    sz[i] = blocks[i].second - blocks[i].first + 1;
    if (sz[i] < 1 || sz[i] > UPAD) throw HipErr{hipErrorInvalidValue};
  }
  HCHECK(hipMemcpyAsync(h->b_splb.dev, sz, sizeof(int) * cnt, hipMemcpyHostToDevice, s));
  launch_slot_ident(zq, (const int*)h->b_splb.dev, cnt, s);
  HCHECK(hipGetLastError());
  BatchEngine b;
  b.init(h, s, cnt);
  b.defer_small = true;
  b.allow_split = false;
  b.time = time;
  for (int i = 0; i < cnt; ++i) {
    const int lo = blocks[i].first;
    b.add(i, sz[i], H + lo + (size_t)lo * ldh, ldh, zq + (size_t)i * slot, UPAD, wr + lo, wi + lo,
          (uint64_t)i);
  }
  int64_t guard = 0;
  while (b.any_active()) {
    b.round();
    if (++guard > (int64_t)4 * 1000 * 1000) throw HipErr{hipErrorUnknown};
  }
  b.settle();
  bool ok = true;
  for (int i = 0; i < cnt; ++i) ok = ok && b.M[i].info == 0;
  launch_slot_transpose(zq, ut, cnt, s);
  HCHECK(hipGetLastError());
  grow(h->b_splw, sizeof(WinB) * cnt, true);
  WinB* wh = (WinB*)h->b_splw.host;
  int tr = 0, tcq = 0;
  for (int i = 0; i < cnt; ++i) {
    WinB& w = wh[i];
    std::memset(&w, 0, sizeof(w));
    w.c.H = H; w.c.Q = Q; w.c.U = ut + (size_t)i * slot; w.c.st = nullptr;
    w.c.ldh = ldh; w.c.ldq = ldq; w.c.n = n;
    w.c.ktop = 0; w.c.kbot = n - 1; w.c.rtop = 0; w.c.cend = n;
    w.c.p = blocks[i].first; w.c.ws = sz[i];
    fill_tiles_b(w, tr, tcq, h->stats, PANEL_TPB_WIDE);
  }
  WinB* wd = (WinB*)h->b_splw.dev;
  HCHECK(hipMemcpyAsync(wd, wh, sizeof(WinB) * cnt, hipMemcpyHostToDevice, s));
  hipEvent_t e0 = nullptr;
  if (tr > 0) {
    if (time) h->timer.begin(s, e0);
    launch_panel_row_b(wd, cnt, tr, s);
    HCHECK(hipGetLastError());
    if (time) h->timer.end(s, e0, &h->stats.row_ms);
    h->stats.row_launches += 1;
  }
  if (tcq > 0) {
    if (time) h->timer.begin(s, e0);
    launch_panel_colq_b(wd, cnt, tcq, s);
    HCHECK(hipGetLastError());
    if (time) h->timer.end(s, e0, &h->stats.colq_ms);
    h->stats.colq_launches += 1;
  }
  h->stats.gemm_launches += (tr > 0) + (tcq > 0);
  h->stats.launches += 2 + (tr > 0) + (tcq > 0);
  // the staging buffers are rewritten by the next call: wait for the copies
  HCHECK(hipStreamSynchronize(s));
  return ok;
}

// Matrices of order up to this go to the persistent kernel (one workgroup
// per matrix, the whole solve on the device); larger ones to the round
// engine, which spreads one matrix's windows and panel tiles over the GPU.
constexpr int kPersistMaxN = 1024;

// One job of the persistent kernel: the options resolved for order n, in the
// kernel's ranges (at most 128 shifts, 8 bulges per window chain).
void fill_job(PJob& J, const schur_opts& o, int n, double* H, int ldh, double* Q, int ldq,
              double* wr, double* wi, int* info, double* counters) {
  const Params P = resolve(o, std::max(1, n));
  std::memset(&J, 0, sizeof(J));
  J.H = H; J.Q = Q; J.wr = wr; J.wi = wi;
  J.ldh = ldh; J.ldq = Q ? ldq : 1; J.n = n;
  J.ns = std::max(2, std::min(P.ns, SMALL_EIG_MAX) & ~1);
  J.nb = std::max(1, std::min(P.nb, PB_NBMAX));
  J.step = P.step;
  J.nw = P.nw;
  J.nibble = P.nibble;
  J.nmin = P.nmin;
  J.exc_period = P.exc_period;
  J.max_sweeps = P.max_sweeps;
  J.info = info;
  J.counters = counters;
}

// queue order: largest first, so that the last workgroups to finish hold
// small matrices
void order_jobs(const PJob* jobs, int* order, int cnt) {
  for (int j = 0; j < cnt; ++j) order[j] = j;
  std::stable_sort(order, order + cnt, [&](int a, int b) { return jobs[a].n > jobs[b].n; });
}

int device_cus(int device) {
  int cus = 0;
  HCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  return std::max(1, cus);
}

// The persistent batched kernel over the matrices idx[] of a batched call:
// one launch, taken largest first; writes their info codes to info[idx[j]].
void solve_persistent(schur_handle_s* h, hipStream_t s, const std::vector<int>& idx,
                      const int* n, double* const* H, const int* ldh, double* const* Q,
                      const int* ldq, double* const* wr, double* const* wi, int* info) {
  const int cnt = (int)idx.size();
  if (cnt == 0) return;
  const int grid = std::min(cnt, device_cus(h->device));
  grow(h->b_pjob, sizeof(PJob) * cnt, true);
  grow(h->b_pord, sizeof(int) * cnt, true);
  const size_t res_bytes = sizeof(double) * PB_COUNTERS * cnt + sizeof(int) * cnt;
  grow(h->b_pres, res_bytes, true);
  grow(h->b_pscr, sizeof(PScratch) * grid + 256, false);
  PJob* jh = (PJob*)h->b_pjob.host;
  int* oh = (int*)h->b_pord.host;
  double* cnt_d = (double*)h->b_pres.dev;
  int* info_d = (int*)(cnt_d + (size_t)PB_COUNTERS * cnt);
  for (int j = 0; j < cnt; ++j) {
    const int i = idx[j];
    double* qi = Q ? Q[i] : nullptr;
    fill_job(jh[j], h->opts, n[i], H[i], ldh[i], qi, (qi && ldq) ? ldq[i] : 1, wr[i], wi[i],
             info_d + j, cnt_d + (size_t)PB_COUNTERS * j);
  }
  order_jobs(jh, oh, cnt);
  HCHECK(hipMemcpyAsync(h->b_pjob.dev, jh, sizeof(PJob) * cnt, hipMemcpyHostToDevice, s));
  HCHECK(hipMemcpyAsync(h->b_pord.dev, oh, sizeof(int) * cnt, hipMemcpyHostToDevice, s));
  PScratch* scr = (PScratch*)h->b_pscr.dev;
  int* next = (int*)((char*)h->b_pscr.dev + sizeof(PScratch) * grid);
  const bool time = (h->opts.flags & SCHUR_FLAG_TIME_KERNELS) != 0;
  hipEvent_t e0 = nullptr;
  if (time) h->timer.begin(s, e0);
  launch_batch_persistent((const PJob*)h->b_pjob.dev, (const int*)h->b_pord.dev, cnt, next, scr,
                          grid, s);
  HCHECK(hipGetLastError());
  if (time) h->timer.end(s, e0, &h->stats.persist_ms);
  HCHECK(hipMemcpyAsync(h->b_pres.host, h->b_pres.dev, res_bytes, hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  if (time) h->timer.harvest();
  const double* ch = (const double*)h->b_pres.host;
  const int* ih = (const int*)(ch + (size_t)PB_COUNTERS * cnt);
  schur_stats& st = h->stats;
  for (int j = 0; j < cnt; ++j) {
    info[idx[j]] = ih[j];
    const double* c = ch + (size_t)PB_COUNTERS * j;
    st.sweeps += (int64_t)c[PB_SWEEPS];
    st.windows += (int64_t)c[PB_WINDOWS];
    st.chain_steps += (int64_t)c[PB_CHAIN_STEPS];
    st.aed_windows += (int64_t)c[PB_AED_WINDOWS];
    st.aed_deflated += (int64_t)c[PB_AED_DEFLATED];
    st.small_solves += (int64_t)c[PB_SMALL];
    st.shifts_applied += (int64_t)c[PB_SHIFTS];
    st.gemm_flops += c[PB_GEMM_FLOPS];
    st.chase_flops += c[PB_CHASE_FLOPS];
    st.small_flops += c[PB_SMALL_FLOPS];
    st.aed_flops += c[PB_AED_FLOPS];
  }
  st.persist_jobs += cnt;
  st.launches += 2;
}

int solve_batched(schur_handle_s* h, hipStream_t s, int count, const int* n, double* const* H,
                  const int* ldh, double* const* Q, const int* ldq, double* const* wr,
                  double* const* wi, int* info) {
  try {
    HCHECK(hipSetDevice(h->device));
    const int rc = alloc_ws(h, 2);
    if (rc) return rc;
    std::memset(&h->stats, 0, sizeof(h->stats));
    BatchEngine b;
    b.init(h, s, count);
    b.time = (h->opts.flags & SCHUR_FLAG_TIME_KERNELS) != 0;
    std::vector<int> pre(count, 0), pinfo(count, 0), pidx;
    const bool rounds_only = (h->opts.flags & SCHUR_FLAG_BATCH_ROUNDS) != 0;
    for (int i = 0; i < count; ++i) {
      double* qi = Q ? Q[i] : nullptr;
      const int lq = (qi && ldq) ? ldq[i] : 1;
      pre[i] = check_args(n[i], H[i], ldh[i], qi, lq, wr[i], wi[i]);
      if (pre[i] == 0 && n[i] > 65536) pre[i] = -1;
      if (pre[i] != 0 || n[i] == 0) continue;
      if (!rounds_only && n[i] <= kPersistMaxN) pidx.push_back(i);
      else b.add(i, n[i], H[i], ldh[i], qi, lq, wr[i], wi[i], (uint64_t)i);
    }
    solve_persistent(h, b.s, pidx, n, H, ldh, Q, ldq, wr, wi, pinfo.data());
    int64_t guard = 0;
    while (b.any_active()) {
      b.round();
      if (++guard > (int64_t)4 * 1000 * 1000) throw HipErr{hipErrorUnknown};
    }
    b.settle();
    int first = 0;
    for (int i = 0; i < count; ++i) {
      const int r = pre[i] != 0 ? pre[i] : (b.M[i].used ? b.M[i].info : pinfo[i]);
      if (info) info[i] = r;
      if (r != 0 && first == 0) first = r;
    }
    return first;
  } catch (const HipErr& e) {
    (void)hipGetLastError();
    return e.e == hipErrorOutOfMemory ? -101 : -102;
  }
}

int create_handle(schur_handle_s** out, int device, const schur_opts* opts) {
  schur_handle_s* h = new schur_handle_s();
  h->device = device;
  if (opts) h->opts = *opts;
  if (hipSetDevice(device) != hipSuccess) { delete h; return -102; }
  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) != hipSuccess) {
    delete h;
    return -102;
  }
  for (int i = 0; i < NBUF; ++i) {
    if (hipEventCreateWithFlags(&h->ev_u[i], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_q[i], hipEventDisableTiming) != hipSuccess) {
      delete h;
      return -102;
    }
  }
  if (hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
    delete h;
    return -102;
  }
  *out = h;
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Serving loop
// ---------------------------------------------------------------------------
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  int n = 0;
  bool want_q = false;
  double* hH = nullptr;     // pinned: the input, then S
  double* hQ = nullptr;     // pinned: Q
  double* hw = nullptr;     // pinned: wr (n), wi (n)
  Ctrl* hctrl = nullptr;    // pinned: the slot's control block at retirement
  double *dH = nullptr, *dQ = nullptr, *dw = nullptr;
  size_t bytes = 0;
  int slot = -1;
  int info = 0;
  int last_small_top = -1;
  double t_submit = 0, t_done = 0;
  hipEvent_t ev = nullptr;
  void* hblock = nullptr;   // the pinned block holding hH, hQ, hw, hctrl
  size_t hcap = 0;
  enum State { QUEUED, RESIDENT, DRAINING, DONE } state = QUEUED;
};

}  // namespace

struct schur_server_s {
  schur_handle_s* h = nullptr;
  size_t budget = 0, in_use = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> all;
  std::vector<Request*> resident;     // by engine slot
  std::vector<Request*> draining;
  std::thread th;
  bool stop = false;
  int error = 0;
  BatchEngine eng;
  int slots = 1024;
  uint64_t next_ticket = 1;
  schur_server_stats st{};
  // requests of order <= kServePersistMaxN: one persistent launch per group of
  // requests admitted together, on a small pool of streams, so that groups
  // admitted while others run overlap with them on the device
  // (groups on one stream run in stream order; each group's pinned staging
  // comes from the pool below and its completion event from a free list, so
  // no host allocation or free, which can wait for the device, happens per
  // group).  Two streams: with the round engine's stream and its second
  // stream they need four hardware queues, the runtime's default, so a long
  // persistent launch never sits in front of the round engine's kernels.
  static constexpr int kLanes = 2;
  hipStream_t lane[kLanes] = {};
  int lane_next = 0;
  std::vector<hipEvent_t> free_events;
  struct Group {
    std::vector<Request*> reqs;
    void* host = nullptr;   // pinned (pool): jobs and queue order, then the info codes
    size_t host_cap = 0;
    size_t off_info = 0;
    hipEvent_t ev = nullptr;
  };
  std::vector<Group> groups;
  // pinned host blocks of finished requests, reused by later ones of the
  // same size class (a pinned allocation or free can wait for the device)
  std::mutex pool_mu;
  std::map<size_t, std::vector<void*>> pool;
  size_t pooled = 0;
  static constexpr size_t kPoolMax = (size_t)8 << 30;
};

namespace {

size_t request_bytes(int n, bool want_q) {
  const size_t nn = (size_t)n * n;
  return sizeof(double) * (nn + (want_q ? nn : 0) + 2 * (size_t)n) + sizeof(Ctrl);
}

// size class of a pinned block: the next power of two from 4 KiB
size_t pin_class(size_t bytes) {
  size_t c = 4096;
  while (c < bytes) c <<= 1;
  return c;
}

void* pin_get(schur_server_s* S, size_t bytes, size_t* cap) {
  *cap = pin_class(bytes);
  {
    std::lock_guard<std::mutex> lk(S->pool_mu);
    auto it = S->pool.find(*cap);
    if (it != S->pool.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      S->pooled -= *cap;
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, *cap, hipHostMallocDefault) != hipSuccess) return nullptr;
  return p;
}

void pin_put(schur_server_s* S, void* p, size_t cap) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(S->pool_mu);
    if (S->pooled + cap <= schur_server_s::kPoolMax) {
      S->pool[cap].push_back(p);
      S->pooled += cap;
      return;
    }
  }
  (void)hipHostFree(p);
}

void free_request_host(schur_server_s* S, Request* r) {
  pin_put(S, r->hblock, r->hcap);
  if (r->ev) (void)hipEventDestroy(r->ev);
  r->hblock = nullptr;
  r->hH = r->hQ = r->hw = nullptr;
  r->hctrl = nullptr;
  r->ev = nullptr;
}

// Served requests up to this order go to persistent launches, larger ones to
// the round engine.  Lower than kPersistMaxN: a request alone on one CU
// finishes later than in the round engine once its order is in the hundreds,
// and a served mix has few such requests at once to fill the CUs (measured
// on the serving bench, orders log-uniform in [64, 4096]: saturation 12.9
// solves/s with 256, 10.2 with 1024, 12.8 with every request in the round
// engine).
constexpr int kServePersistMaxN = 256;

// One persistent launch for the requests of order <= kServePersistMaxN admitted
// together: their device buffers, input copies, the launch, result copies
// to pinned memory and the frees, all in order on one stream of the pool;
// an event marks the group's completion.
void launch_group(schur_server_s* S, const std::vector<Request*>& reqs) {
  schur_server_s::Group G;
  G.reqs = reqs;
  hipStream_t gs = S->lane[S->lane_next++ % schur_server_s::kLanes];
  const int cnt = (int)reqs.size();
  const int grid = std::min(cnt, device_cus(S->h->device));
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t off_ord = up(sizeof(PJob) * cnt);
  G.off_info = up(off_ord + sizeof(int) * cnt);
  const size_t off_scr = up(G.off_info + sizeof(int) * cnt);
  const size_t off_next = off_scr + sizeof(PScratch) * grid;
  char* dev = nullptr;
  HCHECK(hipMallocAsync((void**)&dev, off_next + 256, gs));
  char* host = (char*)pin_get(S, off_scr, &G.host_cap);
  if (!host) throw HipErr{hipErrorOutOfMemory};
  G.host = host;
  PJob* jh = (PJob*)host;
  int* oh = (int*)(host + off_ord);
  for (int j = 0; j < cnt; ++j) {
    Request* r = reqs[j];
    const int n = r->n;
    const size_t nn = (size_t)n * n;
    HCHECK(hipMallocAsync((void**)&r->dH, sizeof(double) * std::max<size_t>(1, nn), gs));
    if (r->want_q)
      HCHECK(hipMallocAsync((void**)&r->dQ, sizeof(double) * std::max<size_t>(1, nn), gs));
    HCHECK(hipMallocAsync((void**)&r->dw, sizeof(double) * 2 * std::max(1, n), gs));
    HCHECK(hipMemcpyAsync(r->dH, r->hH, sizeof(double) * nn, hipMemcpyHostToDevice, gs));
    if (r->want_q) launch_set_identity(r->dQ, n, n, gs);
    fill_job(jh[j], S->h->opts, n, r->dH, std::max(1, n), r->dQ, std::max(1, n), r->dw,
             r->dw + std::max(1, n), (int*)(dev + G.off_info) + j, nullptr);
  }
  order_jobs(jh, oh, cnt);
  HCHECK(hipMemcpyAsync(dev, host, G.off_info, hipMemcpyHostToDevice, gs));
  launch_batch_persistent((const PJob*)dev, (const int*)(dev + off_ord), cnt,
                          (int*)(dev + off_next), (PScratch*)(dev + off_scr), grid, gs);
  HCHECK(hipGetLastError());
  HCHECK(hipMemcpyAsync(host + G.off_info, dev + G.off_info, sizeof(int) * cnt,
                        hipMemcpyDeviceToHost, gs));
  for (Request* r : reqs) {
    const int n = r->n;
    const size_t nn = (size_t)n * n;
    HCHECK(hipMemcpyAsync(r->hH, r->dH, sizeof(double) * nn, hipMemcpyDeviceToHost, gs));
    if (r->want_q)
      HCHECK(hipMemcpyAsync(r->hQ, r->dQ, sizeof(double) * nn, hipMemcpyDeviceToHost, gs));
    HCHECK(hipMemcpyAsync(r->hw, r->dw, sizeof(double) * 2 * std::max(1, n),
                          hipMemcpyDeviceToHost, gs));
    HCHECK(hipFreeAsync(r->dH, gs));
    if (r->dQ) HCHECK(hipFreeAsync(r->dQ, gs));
    HCHECK(hipFreeAsync(r->dw, gs));
    r->dH = r->dQ = r->dw = nullptr;
  }
  HCHECK(hipFreeAsync(dev, gs));
  if (S->free_events.empty()) {
    hipEvent_t e = nullptr;
    HCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    S->free_events.push_back(e);
  }
  G.ev = S->free_events.back();
  S->free_events.pop_back();
  HCHECK(hipEventRecord(G.ev, gs));
  S->groups.push_back(G);
}

void server_loop(schur_server_s* S) {
  hipStream_t s = S->h->stream;
  try {
    HCHECK(hipSetDevice(S->h->device));
    while (true) {
      std::vector<Request*> admitted;
      {
        std::unique_lock<std::mutex> lk(S->mu);
        const bool idle = S->queue.empty() && !S->eng.any_active() && S->draining.empty() &&
                          S->groups.empty();
        if (idle) {
          if (S->stop) break;
          S->cv.wait_for(lk, std::chrono::milliseconds(2));
          continue;
        }
        // FIFO admission by device-memory budget, as slots free up
        while (!S->queue.empty()) {
          Request* r = S->queue.front();
          const bool empty_gpu = S->in_use == 0;
          if (r->bytes > S->budget) {          // can never fit
            S->queue.pop_front();
            r->info = -101;
            r->state = Request::DONE;
            r->t_done = now_s();
            S->st.completed += 1;
            continue;
          }
          if (S->in_use + r->bytes > S->budget && !empty_gpu) break;
          const bool small = r->n <= kServePersistMaxN &&
                             (S->h->opts.flags & SCHUR_FLAG_BATCH_ROUNDS) == 0;
          const int slot = small ? -1 : S->eng.free_slot();
          if (!small && slot < 0) break;
          S->queue.pop_front();
          r->slot = slot;
          if (!small) S->eng.M[slot].used = true;   // reserve; filled below
          S->in_use += r->bytes;
          r->state = Request::RESIDENT;
          admitted.push_back(r);
        }
      }
      // device state of the admitted requests (stream-ordered allocations);
      // the small ones go out as one persistent launch
      std::vector<Request*> group;
      for (Request* r : admitted) {
        if (r->slot < 0) { group.push_back(r); continue; }
        const int n = r->n;
        const size_t nn = (size_t)n * n;
        HCHECK(hipMallocAsync((void**)&r->dH, sizeof(double) * std::max<size_t>(1, nn), s));
        if (r->want_q)
          HCHECK(hipMallocAsync((void**)&r->dQ, sizeof(double) * std::max<size_t>(1, nn), s));
        HCHECK(hipMallocAsync((void**)&r->dw, sizeof(double) * 2 * std::max(1, n), s));
        HCHECK(hipMemcpyAsync(r->dH, r->hH, sizeof(double) * nn, hipMemcpyHostToDevice, s));
        if (r->want_q) launch_set_identity(r->dQ, n, n, s);
        S->eng.add(r->slot, n, r->dH, std::max(1, n), r->dQ, std::max(1, n), r->dw,
                   r->dw + std::max(1, n), r->ticket);
        S->resident[r->slot] = r;
      }
      if (!group.empty()) launch_group(S, group);
      {
        std::lock_guard<std::mutex> lk(S->mu);
        int64_t res = (int64_t)std::count_if(S->resident.begin(), S->resident.end(),
                                             [](Request* r) { return r != nullptr; });
        for (const auto& G : S->groups) res += (int64_t)G.reqs.size();
        S->st.resident = res;
        S->st.peak_resident = std::max(S->st.peak_resident, res);
        S->st.bytes_in_use = (double)S->in_use;
        S->st.peak_bytes = std::max(S->st.peak_bytes, (double)S->in_use);
      }
      if (S->eng.any_active()) {
        S->eng.round();
        S->st.rounds += 1;
      }
      // retire finished requests: results to pinned host memory, free device memory
      for (int i = 0; i < S->eng.cap; ++i) {
        Request* r = S->resident[i];
        if (!r || S->eng.M[i].active) continue;
        const int n = r->n;
        const size_t nn = (size_t)n * n;
        r->info = S->eng.M[i].info;
        r->last_small_top = S->eng.M[i].last_small_top;
        HCHECK(hipMemcpyAsync(r->hH, r->dH, sizeof(double) * nn, hipMemcpyDeviceToHost, s));
        if (r->want_q)
          HCHECK(hipMemcpyAsync(r->hQ, r->dQ, sizeof(double) * nn, hipMemcpyDeviceToHost, s));
        HCHECK(hipMemcpyAsync(r->hw, r->dw, sizeof(double) * 2 * std::max(1, n),
                              hipMemcpyDeviceToHost, s));
        HCHECK(hipMemcpyAsync(r->hctrl, S->eng.ctrl_d + i, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        HCHECK(hipEventRecord(r->ev, s));
        HCHECK(hipFreeAsync(r->dH, s));
        if (r->dQ) HCHECK(hipFreeAsync(r->dQ, s));
        HCHECK(hipFreeAsync(r->dw, s));
        r->dH = r->dQ = r->dw = nullptr;
        S->eng.release(i);
        S->resident[i] = nullptr;
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_use -= r->bytes;
        r->state = Request::DRAINING;
        S->draining.push_back(r);
      }
      // completions
      std::vector<Request*> keep;
      for (Request* r : S->draining) {
        const hipError_t q = hipEventQuery(r->ev);
        if (q == hipErrorNotReady) { keep.push_back(r); continue; }
        HCHECK(q);
        std::lock_guard<std::mutex> lk(S->mu);
        if (r->info == 0 && r->last_small_top >= 0 && r->hctrl->small_info != 0)
          r->info = r->last_small_top + r->hctrl->small_info;
        r->t_done = now_s();
        r->state = Request::DONE;
        S->st.completed += 1;
      }
      S->draining.swap(keep);
      // finished persistent groups
      std::vector<schur_server_s::Group> running;
      for (auto& G : S->groups) {
        const hipError_t q = hipEventQuery(G.ev);
        if (q == hipErrorNotReady) { running.push_back(G); continue; }
        HCHECK(q);
        const int* infos = (const int*)((char*)G.host + G.off_info);
        {
          std::lock_guard<std::mutex> lk(S->mu);
          for (size_t j = 0; j < G.reqs.size(); ++j) {
            Request* r = G.reqs[j];
            r->info = infos[j];
            r->t_done = now_s();
            r->state = Request::DONE;
            S->in_use -= r->bytes;
            S->st.completed += 1;
          }
        }
        pin_put(S, G.host, G.host_cap);
        S->free_events.push_back(G.ev);
      }
      S->groups.swap(running);
      if ((!S->draining.empty() || !S->groups.empty()) && !S->eng.any_active()) {
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->queue.empty()) S->cv.wait_for(lk, std::chrono::microseconds(200));
      }
      S->cv.notify_all();
    }
  } catch (const HipErr& e) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->error = e.e == hipErrorOutOfMemory ? -101 : -102;
    for (auto& kv : S->all) {
      Request* r = kv.second;
      if (r->state != Request::DONE) { r->state = Request::DONE; r->info = S->error; r->t_done = now_s(); }
    }
  }
  S->cv.notify_all();
}

}  // namespace


extern "C" {

int schur_create(schur_handle_t* h, int device, const schur_opts* opts) {
  if (!h) return -1;
  return create_handle(h, device, opts);
}

int schur_destroy(schur_handle_t h) {
  if (!h) return -104;
  if (h->job) {   // a begun solve that was never ended
    h->job->join();
    delete h->job;
    h->job = nullptr;
  }
  (void)hipSetDevice(h->device);
  if (h->ev_begin) (void)hipEventDestroy(h->ev_begin);
  if (h->ev_end) (void)hipEventDestroy(h->ev_end);
  if (h->job_info_h) (void)hipHostFree(h->job_info_h);
  if (h->stream) {
    (void)hipStreamSynchronize(h->stream);
    (void)hipStreamDestroy(h->stream);
  }
  if (h->aux) {
    (void)hipStreamSynchronize(h->aux);
    (void)hipStreamDestroy(h->aux);
  }
  for (int i = 0; i < NBUF; ++i) {
    if (h->ev_u[i]) (void)hipEventDestroy(h->ev_u[i]);
    if (h->ev_q[i]) (void)hipEventDestroy(h->ev_q[i]);
  }
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->sub) (void)schur_destroy(h->sub);
  if (h->side) (void)schur_destroy(h->side);
  if (h->shm) (void)hipFree(h->shm);
  free_ws(h);
  delete h;
  return 0;
}

int schur_set_opts(schur_handle_t h, const schur_opts* opts) {
  if (!h) return -104;
  if (opts) h->opts = *opts; else h->opts = schur_opts{};
  return 0;
}

int schur_get_stats(schur_handle_t h, schur_stats* out) {
  if (!h || !out) return -104;
  *out = h->stats;
  return 0;
}

int schur_reduce(int n, double* H, int ldh, double* Q, int ldq, double* wr, double* wi) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -102;
  schur_handle_s* h;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_default[dev]) {
      if (create_handle(&g_default[dev], dev, nullptr) != 0) return -102;
    }
    h = g_default[dev];
  }
  std::lock_guard<std::mutex> lk(g_mu);
  // on the null stream: after whatever the caller queued there
  return solve(h, nullptr, n, H, ldh, Q, ldq, wr, wi);
}

int schur_reduce_noalloc(void* stream, int n, double* H, int ldh, double* Q, int ldq,
                         double* wr, double* wi) {
  return solve_noalloc((hipStream_t)stream, n, H, ldh, Q, ldq, wr, wi);
}

int schur_hessenberg(schur_handle_t h, void* stream, int n, double* A, int lda, double* Q,
                     int ldq) {
  if (!h) return -104;
  return hess_reduce(h, (hipStream_t)stream, n, A, lda, Q, ldq);
}

int schur_eigenvectors(schur_handle_t h, void* stream, int n, const double* S, int lds,
                       const double* Q, int ldq, double* X, int ldx) {
  if (!h) return -104;
  return evec_compute(h, (hipStream_t)stream, n, S, lds, Q, ldq, X, ldx);
}

int schur_reorder(schur_handle_t h, void* stream, int n, double* S, int lds, double* Q, int ldq,
                  const int* select, double* wr, double* wi, int* m) {
  if (!h) return -104;
  return reorder_run(h, (hipStream_t)stream, n, S, lds, Q, ldq, select, wr,
                     wi, m);
}

int schur_plan_reorder(int n, const int* bsize, const int* bsel, int nblocks, int* out, int cap) {
  if (n < 0 || nblocks < 0 || (nblocks > 0 && (!bsize || !bsel))) return -1;
  std::vector<int> bs(bsize, bsize + nblocks);
  std::vector<char> sl(nblocks);
  int tot = 0;
  for (int i = 0; i < nblocks; ++i) {
    if (bs[i] != 1 && bs[i] != 2) return -1;
    sl[i] = bsel[i] ? 1 : 0;
    tot += bs[i];
  }
  if (tot != n) return -1;
  std::vector<std::vector<RWin>> chains;
  std::vector<int> start;
  plan_reorder(n, bs, sl, SMALL_Z_MAX, chains, start);
  int k = 0;
  for (size_t c = 0; c < chains.size(); ++c)
    for (size_t t = 0; t < chains[c].size(); ++t, ++k)
      if (out && k < cap) {
        out[4 * k] = (int)c;
        out[4 * k + 1] = start[c] + (int)t;
        out[4 * k + 2] = chains[c][t].a;
        out[4 * k + 3] = chains[c][t].w;
      }
  return k;
}

int schur_reduce_begin(schur_handle_t h, void* stream, int n, double* H, int ldh, double* Q,
                       int ldq, double* wr, double* wi, int* info_dev) {
  if (!h) return -104;
  if (h->job) return -104;   // a solve begun on this handle has not been ended
  const int rc = check_args(n, H, ldh, Q, ldq, wr, wi);
  if (rc != 0) return rc;
  if (info_dev && !is_device_ptr(info_dev)) return -103;
  try {
    HCHECK(hipSetDevice(h->device));
    if (!h->ev_begin) HCHECK(hipEventCreateWithFlags(&h->ev_begin, hipEventDisableTiming));
    if (!h->ev_end) HCHECK(hipEventCreateWithFlags(&h->ev_end, hipEventDisableTiming));
    if (!h->job_info_h &&
        hipHostMalloc((void**)&h->job_info_h, sizeof(int), hipHostMallocDefault) != hipSuccess)
      return -101;
    // the solve starts after the work already on the caller's stream
    HCHECK(hipEventRecord(h->ev_begin, (hipStream_t)stream));
  } catch (const HipErr& e) {
    (void)hipGetLastError();
    return -102;
  }
  h->job_rc = 0;
  h->job = new std::thread([h, n, H, ldh, Q, ldq, wr, wi, info_dev]() {
    int r = -102;
    if (hipSetDevice(h->device) == hipSuccess &&
        hipStreamWaitEvent(h->stream, h->ev_begin, 0) == hipSuccess)
      r = solve(h, h->stream, n, H, ldh, Q, ldq, wr, wi);
    if (info_dev) {   // info on the device, ordered before the completion event
      *h->job_info_h = r;
      if (hipMemcpyAsync(info_dev, h->job_info_h, sizeof(int), hipMemcpyHostToDevice,
                         h->stream) != hipSuccess)
        r = -102;
    }
    if (hipEventRecord(h->ev_end, h->stream) != hipSuccess) r = -102;
    (void)hipStreamSynchronize(h->stream);   // the pinned info copy has been read
    h->job_rc = r;
  });
  return 0;
}

int schur_reduce_end(schur_handle_t h, void* stream) {
  if (!h) return -104;
  if (!h->job) return -104;
  h->job->join();
  delete h->job;
  h->job = nullptr;
  if (hipStreamWaitEvent((hipStream_t)stream, h->ev_end, 0) != hipSuccess) {
    (void)hipGetLastError();
    return -102;
  }
  return h->job_rc;
}

int schur_reduce_async(schur_handle_t h, void* stream, int n, double* H, int ldh, double* Q,
                       int ldq, double* wr, double* wi, int* info_out) {
  if (!h) return -104;
  const int rc = solve(h, (hipStream_t)stream, n, H, ldh, Q, ldq, wr, wi);
  if (info_out) *info_out = rc;
  return rc;
}

int schur_reduce_batched(schur_handle_t h, void* stream, int count, const int* n,
                         double* const* H, const int* ldh, double* const* Q, const int* ldq,
                         double* const* wr, double* const* wi, int* info) {
  if (!h) return -104;
  if (count < 0) return -3;
  if (count == 0) return 0;
  if (!n || !H || !ldh || !wr || !wi) return -4;
  return solve_batched(h, (hipStream_t)stream, count, n, H, ldh, Q, ldq, wr, wi, info);
}

int schur_server_create(schur_server_t* out, int device, size_t hbm_budget_bytes,
                        const schur_opts* opts) {
  if (!out) return -1;
  schur_server_s* S = new schur_server_s();
  if (create_handle(&S->h, device, opts) != 0) { delete S; return -102; }
  S->budget = hbm_budget_bytes ? hbm_budget_bytes : ((size_t)64 << 30);
  try {
    HCHECK(hipSetDevice(device));
    if (alloc_ws(S->h, 2) != 0) throw HipErr{hipErrorOutOfMemory};
    S->eng.init(S->h, S->h->stream, S->slots);
    for (int k = 0; k < schur_server_s::kLanes; ++k)
      HCHECK(hipStreamCreateWithFlags(&S->lane[k], hipStreamNonBlocking));
    // the passes run on the host thread that drives the rounds: they would
    // stall every other resident request for their duration
    S->eng.allow_split = false;
    S->resident.assign(S->slots, nullptr);
    HCHECK(hipStreamSynchronize(S->h->stream));
  } catch (const HipErr&) {
    for (int k = 0; k < schur_server_s::kLanes; ++k)
      if (S->lane[k]) (void)hipStreamDestroy(S->lane[k]);
    schur_destroy(S->h);
    delete S;
    return -101;
  }
  S->th = std::thread(server_loop, S);
  *out = S;
  return 0;
}

int schur_server_destroy(schur_server_t S) {
  if (!S) return -104;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  (void)hipSetDevice(S->h->device);
  for (int k = 0; k < schur_server_s::kLanes; ++k) {
    if (!S->lane[k]) continue;
    (void)hipStreamSynchronize(S->lane[k]);
    (void)hipStreamDestroy(S->lane[k]);
  }
  for (auto& G : S->groups) {   // left by a failed loop: their streams are drained
    pin_put(S, G.host, G.host_cap);
    if (G.ev) (void)hipEventDestroy(G.ev);
  }
  S->groups.clear();
  for (hipEvent_t e : S->free_events) (void)hipEventDestroy(e);
  S->free_events.clear();
  for (auto& kv : S->all) { free_request_host(S, kv.second); delete kv.second; }
  for (auto& kv : S->pool)
    for (void* p : kv.second) (void)hipHostFree(p);
  S->pool.clear();
  S->all.clear();
  schur_destroy(S->h);
  delete S;
  return 0;
}

int schur_submit(schur_server_t S, int n, const double* H_host, int ldh, int want_q,
                 uint64_t* ticket) {
  if (!S) return -104;
  if (n < 0 || n > 65536) return -2;
  if (n > 0 && !H_host) return -3;
  if (ldh < std::max(1, n)) return -4;
  if (!ticket) return -6;
  Request* r = new Request();
  r->n = n;
  r->want_q = want_q != 0;
  r->bytes = request_bytes(n, r->want_q);
  const size_t nn = (size_t)n * n;
  // one pinned block: S (or H), Q, (wr, wi), the control block
  const size_t dh = std::max<size_t>(1, nn), dq = r->want_q ? dh : 0,
               dw = 2 * (size_t)std::max(1, n);
  r->hblock = pin_get(S, sizeof(double) * (dh + dq + dw) + sizeof(Ctrl), &r->hcap);
  if (!r->hblock || hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
    free_request_host(S, r);
    delete r;
    return -101;
  }
  r->hH = (double*)r->hblock;
  r->hQ = r->want_q ? r->hH + dh : nullptr;
  r->hw = r->hH + dh + dq;
  r->hctrl = (Ctrl*)(r->hw + dw);
  std::memset(r->hctrl, 0, sizeof(Ctrl));
  for (int c = 0; c < n; ++c)
    std::memcpy(r->hH + (size_t)c * n, H_host + (size_t)c * ldh, sizeof(double) * n);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error) { free_request_host(S, r); delete r; return S->error; }
    r->ticket = S->next_ticket++;
    r->t_submit = now_s();
    if (n == 0) { r->state = Request::DONE; r->t_done = r->t_submit; S->st.completed += 1; }
    else S->queue.push_back(r);
    S->all[r->ticket] = r;
    S->st.submitted += 1;
    S->st.queued = (int64_t)S->queue.size();
    *ticket = r->ticket;
  }
  S->cv.notify_all();
  return 0;
}

int schur_poll(schur_server_t S, uint64_t ticket, double* S_host, int lds, double* Q_host, int ldq,
               double* wr, double* wi, int* info, double* latency_s) {
  if (!S) return -104;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return -2;
    r = it->second;
    if (r->state != Request::DONE) return 1;
    S->all.erase(it);
  }
  const int n = r->n;
  if (r->info >= 0 && r->hH) {
    if (S_host && lds >= n)
      for (int c = 0; c < n; ++c)
        std::memcpy(S_host + (size_t)c * lds, r->hH + (size_t)c * n, sizeof(double) * n);
    if (Q_host && r->want_q && ldq >= n)
      for (int c = 0; c < n; ++c)
        std::memcpy(Q_host + (size_t)c * ldq, r->hQ + (size_t)c * n, sizeof(double) * n);
    if (wr) std::memcpy(wr, r->hw, sizeof(double) * n);
    if (wi) std::memcpy(wi, r->hw + std::max(1, n), sizeof(double) * n);
  }
  if (info) *info = r->info;
  if (latency_s) *latency_s = r->t_done - r->t_submit;
  free_request_host(S, r);
  delete r;
  return 0;
}

int schur_server_get_stats(schur_server_t S, schur_server_stats* out) {
  if (!S || !out) return -104;
  std::lock_guard<std::mutex> lk(S->mu);
  S->st.queued = (int64_t)S->queue.size();
  *out = S->st;
  return 0;
}

int schur_set_tuning(int count, const int* nmax, const int* ns, const int* nb, const int* step,
                     const int* nw, const int* nibble, const int* tile) {
  if (count < 0) return -1;
  std::vector<TuneRow> t;
  if (count == 0) {
    t.assign(std::begin(kBuiltinTune), std::end(kBuiltinTune));
  } else {
    if (!nmax || !ns || !nb || !step) return -2;
    for (int i = 0; i < count; ++i) {
      const int w = nw ? nw[i] : 0;
      const int nib = nibble ? nibble[i] : 0;
      if (ns[i] < 2 || ns[i] > NS_MAX || nb[i] < 1 || nb[i] > NBMAX || step[i] < 0 ||
          w > SMALL_Z_MAX || (w > 0 && w < 4) || nib > 100 || (i > 0 && nmax[i] <= nmax[i - 1]))
        return -2;
      const int tl = tile ? tile[i] : 0;
      if (tl < 0 || tl > PANEL_TPB) return -2;
      t.push_back(TuneRow{nmax[i], ns[i] & ~1, nb[i], step[i], w, nib, tl});
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.swap(t);
  return 0;
}

int schur_plan_split(int lo, int hi, int nw, int first, int* out, int cap) {
  if (lo < 0 || hi < lo || nw < 1 || nw > SMALL_Z_MAX || first < 1 || first > nw || cap < 0 ||
      (cap > 0 && !out))
    return -1;
  std::vector<std::pair<int, int>> ws;
  split_tile(lo, hi, first, nw, ws);
  const int k = (int)ws.size();
  for (int j = 0; j < k && j < cap; ++j) {   // top to bottom
    out[2 * j] = ws[k - 1 - j].first;
    out[2 * j + 1] = ws[k - 1 - j].second;
  }
  return k;
}

int schur_select_windows(int count, const int* a, const int* w, const double* wt, int* picked) {
  if (count < 0 || (count > 0 && (!a || !w || !wt || !picked))) return -1;
  for (int i = 0; i < count; ++i)
    if (a[i] < 0 || w[i] < 1 || !(wt[i] > 0.0)) return -1;
  std::vector<int> cand(count), pick;
  for (int i = 0; i < count; ++i) cand[i] = i;
  split_select(cand, a, w, wt, pick);
  std::sort(pick.begin(), pick.end(), [&](int x, int y) { return a[x] < a[y]; });
  for (size_t j = 0; j < pick.size(); ++j) picked[j] = pick[j];
  return (int)pick.size();
}

double schur_split_weight(int split, int nf, int top, int below) {
  return split_weight(split, nf, top, below);
}

int schur_plan_sweep(int ktop, int kbot, int npair, int nb, int step, int* out, int cap) {
  if (ktop < 0 || kbot - ktop + 1 < 3 || npair < 1 || nb < 1 || nb > NBMAX || step < 0 ||
      cap < 0 || (cap > 0 && !out))
    return -1;
  std::vector<std::vector<WinPlan>> steps;
  int st = 0;
  plan_sweep(ktop, kbot, npair, nb, step, steps, st);
  int k = 0;
  for (size_t t = 0; t < steps.size(); ++t) {
    for (const WinPlan& w : steps[t]) {
      if (k < cap) {
        int* o = out + 7 * k;
        o[0] = (int)t;
        o[1] = w.shift0;   // groups are identified by their first bulge
        o[2] = w.p;
        o[3] = w.ws;
        o[4] = w.tau0;
        o[5] = w.tau1;
        o[6] = w.nb;
      }
      ++k;
    }
  }
  return k;
}

}  // extern "C"
