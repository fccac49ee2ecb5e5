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
#include <mutex>
#include <vector>

#include "../../include/schur.h"
#include "kernels.h"
#include "schur_internal.h"

using namespace schur;

namespace {

constexpr int NSMAX = 512;             // shifts buffer capacity
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

struct schur_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
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

// ---- defaults ------------------------------------------------------------
int default_ns(int n) {
  if (n < 300) return 2;       // plain Francis double-shift steps
  if (n < 3000) return 32;
  if (n < 6000) return 64;
  return 128;
}

struct Params {
  int ns, nb, step, nmin, max_sweeps, exc_period;
  bool time;
};

Params resolve(const schur_opts& o, int n) {
  Params p;
  p.ns = o.ns > 0 ? (o.ns & ~1) : default_ns(n);
  if (p.ns < 2) p.ns = 2;
  if (p.ns > SMALL_EIG_MAX) p.ns = SMALL_EIG_MAX;
  p.nb = o.nb > 0 ? o.nb : 16;
  if (p.nb > NBMAX) p.nb = NBMAX;
  p.step = o.step;
  p.nmin = o.nmin > 0 ? std::min(o.nmin, SMALL_Z_MAX) : SMALL_Z_MAX;
  p.max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 30 * std::max(10, n) / std::max(2, p.ns) + 100;
  p.exc_period = o.exc_period > 0 ? o.exc_period : 6;
  p.time = (o.flags & SCHUR_FLAG_TIME_KERNELS) != 0;
  return p;
}

int alloc_ws(schur_handle_s* h, int n) {
  if (!h->U) {
    if (hipMalloc(&h->U, sizeof(double) * (size_t)MAXWIN * UPAD * UPAD) != hipSuccess) return -101;
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

void free_ws(schur_handle_s* h) {
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

struct Solver {
  schur_handle_s* h;
  hipStream_t s;
  Params P;
  int n;
  double* H; int ldh;
  double* Q; int ldq;
  double* wr; double* wi;

  void fill_gemm(SweepArgs& a, int& tr, int& tcq) {
    tr = 0;
    tcq = 0;
    for (int w = 0; w < a.nwin; ++w) {
      Win& d = a.win[w];
      const int pe = d.p + d.ws - 1;
      d.tiles_r = std::max(0, (a.cend - pe - 1 + GEMM_T - 1) / GEMM_T);
      d.tiles_c = std::max(0, (d.p - a.rtop + GEMM_T - 1) / GEMM_T);
      d.tiles_q = a.Q ? (n + GEMM_T - 1) / GEMM_T : 0;
      d.base_r = tr;
      d.base_cq = tcq;
      tr += d.tiles_r;
      tcq += d.tiles_c + d.tiles_q;
      const double ws = d.ws;
      const double fr = 2.0 * ws * ws * (double)std::max(0, a.cend - pe - 1);
      const double fc = 2.0 * ws * ws * ((double)(d.p - a.rtop) + (a.Q ? (double)n : 0.0));
      h->stats.row_flops += fr;
      h->stats.colq_flops += fc;
      h->stats.gemm_flops += fr + fc;
    }
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

  void sync_ctrl() {
    HCHECK(hipMemcpyAsync(h->ctrl_h, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    if (P.time) h->timer.harvest();
  }

  // finish a small active block [ktop, kbot] in one kernel, then apply its
  // Z to the row panel, the column panel and Q
  void small_block(int ktop, int kbot) {
    const int m = kbot - ktop + 1;
    SmallTask t{};
    t.A = H + ktop + (size_t)ktop * ldh;
    t.lda = ldh;
    t.m = m;
    t.Zt = h->U;
    t.ldzt = UPAD;
    t.info = &h->ctrl->small_info;
    t.itmax = 30;
    hipEvent_t e0 = nullptr;
    if (P.time) h->timer.begin(s, e0);
    launch_small_z(t, nullptr, 1, m, s);
    HCHECK(hipGetLastError());
    if (P.time) h->timer.end(s, e0, &h->stats.other_ms);
    h->stats.small_solves += 1;
    h->stats.launches += 1;
    SweepArgs a;
    base_args(a, ktop, kbot);
    a.nwin = 1;
    a.win[0].p = ktop;
    a.win[0].ws = m;
    a.win[0].slot = 0;
    int tr, tcq;
    fill_gemm(a, tr, tcq);
    launch_gemms(a, tr, tcq);
  }

  void compute_shifts(int ktop, int kbot, int ns, bool exceptional) {
    hipEvent_t e0 = nullptr;
    if (P.time) h->timer.begin(s, e0);
    if (!exceptional) {
      SmallTask t{};
      const int b0 = kbot - ns + 1;
      t.A = H + b0 + (size_t)b0 * ldh;
      t.lda = ldh;
      t.m = ns;
      t.wr = h->ewr;
      t.wi = h->ewi;
      t.info = &h->ctrl->small_info;
      t.itmax = 30;
      launch_small_eig(t, s);
    }
    launch_shift_prep(h->ewr, h->ewi, ns, &h->ctrl->small_info, exceptional ? 1 : 0, H, ldh, ktop,
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
      SweepArgs a;
      base_args(a, ktop, kbot);
      a.nwin = (int)ws.size();
      if (a.nwin > MAXWIN) throw HipErr{hipErrorInvalidValue};
      int prev_end = -1;
      for (int w = 0; w < a.nwin; ++w) {
        const WinPlan& pl = ws[w];
        if (pl.ws > WMAX || pl.ws < 3 || pl.p <= prev_end || pl.p < ktop ||
            pl.p + pl.ws - 1 > kbot || pl.nb > NBMAX || pl.tau1 - pl.tau0 > WMAX)
          throw HipErr{hipErrorInvalidValue};
        prev_end = pl.p + pl.ws - 1;
        Win& d = a.win[w];
        d.p = pl.p; d.ws = pl.ws; d.tau0 = pl.tau0; d.tau1 = pl.tau1;
        d.nb = pl.nb; d.shift0 = pl.shift0; d.slot = w;
        h->stats.windows += 1;
        h->stats.chain_steps += pl.tau1 - pl.tau0;
      }
      hipEvent_t e0 = nullptr;
      if (P.time) h->timer.begin(s, e0);
      launch_chase(a, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.chase_ms);
      h->stats.chase_launches += 1;
      h->stats.launches += 1;
      int tr, tcq;
      fill_gemm(a, tr, tcq);
      launch_gemms(a, tr, tcq);
    }
  }

  int run() {
    launch_ctrl_reset(h->ctrl, s);
    launch_check_finite(H, ldh, n, h->ctrl, s);
    sync_ctrl();
    if (h->ctrl_h->bad) return -2;
    launch_zero_lower(H, ldh, n, s);
    int info = 0;
    int kbot = n - 1;
    int nodefl = 0;
    int64_t sweeps = 0;
    while (true) {
      hipEvent_t e0 = nullptr;
      if (P.time) h->timer.begin(s, e0);
      launch_deflate(H, ldh, kbot, 0, h->ctrl, s);
      HCHECK(hipGetLastError());
      if (P.time) h->timer.end(s, e0, &h->stats.other_ms);
      h->stats.launches += 1;
      sync_ctrl();
      if (h->ctrl_h->small_info != 0) {
        // a single-kernel block solve failed: report its block end
        info = h->ctrl_h->small_info;
        break;
      }
      const int nk = h->ctrl_h->kbot;
      if (nk < kbot) nodefl = 0;
      kbot = nk;
      if (kbot < 0) break;
      const int ktop = h->ctrl_h->ktop;
      const int m = kbot - ktop + 1;
      if (m <= P.nmin) {
        // small_info is rebased to the global row by the next check
        small_block(ktop, kbot);
        HCHECK(hipMemcpyAsync(h->ctrl_h, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        HCHECK(hipStreamSynchronize(s));
        if (P.time) h->timer.harvest();
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
      compute_shifts(ktop, kbot, ns, exc);
      sweep(ktop, kbot, ns);
      ++nodefl;
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
  if (ldh < std::max(1, n)) return -3;
  if (Q && ldq < std::max(1, n)) return -5;
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
    Solver sv{h, s ? s : h->stream, resolve(h->opts, n), n, H, ldh, Q, ldq, wr, wi};
    return sv.run();
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
  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
    delete h;
    return -102;
  }
  *out = h;
  return 0;
}

}  // namespace

extern "C" {

int schur_create(schur_handle_t* h, int device, const schur_opts* opts) {
  if (!h) return -1;
  return create_handle(h, device, opts);
}

int schur_destroy(schur_handle_t h) {
  if (!h) return -104;
  (void)hipSetDevice(h->device);
  if (h->stream) {
    (void)hipStreamSynchronize(h->stream);
    (void)hipStreamDestroy(h->stream);
  }
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
  return solve(h, h->stream, n, H, ldh, Q, ldq, wr, wi);
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
  int first = 0;
  for (int i = 0; i < count; ++i) {
    const int rc = solve(h, (hipStream_t)stream, n[i], H[i], ldh[i], Q ? Q[i] : nullptr,
                         ldq ? ldq[i] : 1, wr[i], wi[i]);
    if (info) info[i] = rc;
    if (rc != 0 && first == 0) first = rc;
  }
  return first;
}

}  // extern "C"
