// wg_ops.h -- workgroup-level device operations shared by the sweep
// kernels (kernels.hip) and the persistent batched kernel
// (batch_kernels.hip): shift preparation, the FP64 MFMA panel products of a
// window's orthogonal factor, and the batched deflation scan.  Each takes its
// LDS from the caller, so one kernel can run several of them over the same
// LDS.
#pragma once
#include <type_traits>
#include "schur_internal.h"
#include "device_common.h"
#include "kernels.h"

namespace schur {

typedef double d4 __attribute__((ext_vector_type(4)));

// ============================================================================
// Shift preparation: sort the trailing-block eigenvalues by decreasing
// modulus (conjugate pairs stay together), pair the real ones, and emit one
// (sum, product) pair per bulge.  Missing pairs (if the small solve did not
// converge) are filled with ad-hoc shifts from the bottom of the block.
// ============================================================================
// LDS of the shift preparation (ns <= 512).
struct ShiftLds {
  double key[512];
  int kind[512];   // 0 real, 1 first of a conjugate pair, 2 second (skipped)
  int rank[512];
  int order[512];
};

__device__ void shift_prep(const double* wr, const double* wi, int ns, const int* small_info,
                           int exceptional, const double* H, int ldh, int ktop, int kbot,
                           double* st, ShiftLds& lds) {
  double* key = lds.key;
  int* kind = lds.kind;
  int* rank = lds.rank;
  int* order = lds.order;
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

// ============================================================================
// Panel updates with FP64 MFMA (v_mfma_f64_16x16x4f64).
// Fragment layout of the 16x16x4 FP64 MFMA (wave64), measured on gfx950:
//   A(i, k): lane = i + 16 k      B(k, j): lane = j + 16 k
//   D(i, j): lane = j + 16 (i % 4), element i / 4
// ============================================================================
constexpr int PT = GEMM_T;       // 64
// s_waitcnt operand for vmcnt(32) alone (expcnt and lgkmcnt at their
// maxima; vmcnt in bits 3:0 and 15:14)
constexpr int PANEL_VMCNT32 = 0x8F70;

// Tile accesses go through buffer instructions: one descriptor per tile
// (base at the tile's first element, byte range PANEL_NREC) and a 32-bit
// byte offset per lane.  A lane outside the tile gets an offset of at least
// PANEL_OOB: its load returns 0 and its store is dropped, so the k loop
// needs no exec masks, branches or 64-bit address arithmetic around its
// loads and stores.  A valid offset is at most 127 ld 8 + 127 8 bytes (a
// column-panel tile spans up to 128 window columns), under PANEL_NREC for
// ld <= LD_MAX; the sum of two invalid parts, 2 PANEL_OOB, does not wrap.
constexpr unsigned PANEL_OOB = 0x40000000u;
constexpr int PANEL_NREC = 0x3FFFFFFF;
static_assert(127ull * LD_MAX * 8 + 128 * 8 <= (unsigned long long)PANEL_NREC, "tile range");
typedef unsigned panel_u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t panel_rsrc(const double* base) {
  // dword 3: 32-bit data format (needed for untyped loads and stores on gfx9)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, PANEL_NREC,
                                           0x00020000);
}
__device__ __forceinline__ double panel_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void panel_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(panel_u2, v), r, (int)off, 0, 0);
}
static_assert(UPAD / 4 == 32, "32 k steps of 4 carry a tile's 32 loads and 32 stores");
constexpr int LDT = PT + 4;      // padded LDS leading dimension of panel tiles

// Panel tiles are processed up to PANEL_TPB at a time by one workgroup of
// four waves, one workgroup per CU (two 128 x 68 FP64 LDS buffers, 136 KiB,
// passed in as Xs: 2 WMAX LDT doubles):
//  * the window's U (or U^T) is read into registers once;
//  * while tile t is multiplied from LDS, the wave issues the loads of tile
//    t+1 (into registers) in the first half of the k loop and the stores of
//    the results of tile t-1 (kept in a second set of accumulators) in the
//    second half, two per k step, and in the last quarter writes tile t+1
//    from its registers into the other LDS buffer: HBM traffic at an even
//    rate, the LDS writes and the FP64 MFMA work overlap instead of
//    alternating (measured: memory operations bunched into part of the loop,
//    or the tile written to LDS between passes, are slower);
//  * the operands of the next k step are read from LDS before the products
//    of the current one are issued.
// Each pass: barrier (tile t is in LDS; every wave has finished reading tile
// t-1, whose buffer takes tile t+1), then the interleaved k loop.  One pass
// more than there are tiles stores the last results.

// Row panel: Y(ws x 64) = U^T X for 64-column tiles of H(p:p+ws-1, right of
// the window).  Wave w owns rows 32w..32w+31 of U^T (A operand, registers)
// and all 64 tile columns (B operand from LDS, row-major tile Xs[c + r*LDT]).
// Element e of a thread's tile load: window row r = lane + 64 (e & 1), tile
// column c = wave + 4 (e >> 1).  Element s of a thread's results: acc[s >> 4]
// [(s >> 2) & 3][s & 3], row i0 + 16 (s >> 4) + lk + 4 (s & 3), column
// 16 ((s >> 2) & 3) + li.
__device__ void panel_row_tiles(const WinCtx& d, int t0, int t1, double* Xs) {
  const int p = d.p, ws = d.ws;
  const int kpad = (ws + 3) & ~3;
  const double* Ut = d.U;
  const int tid = threadIdx.x;
  // wave index in a scalar register: the tests on it below are uniform branches
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
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
  const unsigned ldb = (unsigned)ldh * 8u;   // bytes per column
  // first column of tile t and its width
  auto col0 = [&](int t) { return p + ws + t * PT; };
  auto ncols = [&](int t) { return min(PT, d.cend - col0(t)); };
  auto rsrc = [&](int t) { return panel_rsrc(H + (size_t)p + (size_t)col0(t) * ldh); };
  // lane parts of the load offsets (window rows lane and lane + 64)
  const unsigned rl0 = lane < ws ? lane * 8u : PANEL_OOB;
  const unsigned rl1 = lane + 64 < ws ? (lane + 64) * 8u : PANEL_OOB;
  auto load_one = [&](double& dst, __amdgpu_buffer_rsrc_t R, int nc, int e) {
    const int c = wave + 4 * (e >> 1);
    dst = panel_load(R, (c < nc ? (unsigned)c * ldb : PANEL_OOB) + ((e & 1) ? rl1 : rl0));
  };
  auto store_one = [&](const d4 (&res)[2][4], __amdgpu_buffer_rsrc_t R, int nc, int s) {
    const int ib = s >> 4, jb = (s >> 2) & 3, e = s & 3;
    const int row = i0 + ib * 16 + lk + 4 * e, col = jb * 16 + li;
    const unsigned off = (row < ws && col < nc) ? (unsigned)row * 8u + (unsigned)col * ldb
                                                : PANEL_OOB;
    panel_store(R, off, res[ib][jb][e]);
  };
  double pre[32];
  // element e of the registers into tile buffer X (entries outside the tile
  // were loaded as 0)
  auto lds_one = [&](double* X, int e) {
    const int r = lane + 64 * (e & 1), c = wave + 4 * (e >> 1);
    X[c + r * LDT] = pre[e];   // r < 128, c < 64: inside the buffer
  };
  {
    const __amdgpu_buffer_rsrc_t R = rsrc(t0);
    const int nc = ncols(t0);
#pragma unroll
    for (int e = 0; e < 32; ++e) load_one(pre[e], R, nc, e);
  }
  __builtin_amdgcn_s_waitcnt(0);   // U and the first tile are in registers
#pragma unroll
  for (int e = 0; e < 32; ++e) lds_one(Xs, e);
  d4 acc[2][4], accp[2][4];
  for (int ib = 0; ib < 2; ++ib)   // stored (as dropped stores) before the first results exist
    for (int jb = 0; jb < 4; ++jb) accp[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
  for (int t = t0; t <= t1; ++t) {
    const bool cur = t < t1, prev = t > t0 && active, next = t + 1 < t1;
    double* X = Xs + ((t - t0) & 1) * (WMAX * LDT);
    double* XN = Xs + ((t - t0 + 1) & 1) * (WMAX * LDT);
    // the loads of the last pass were written to LDS inside it; its stores
    // (the last 32 memory operations) may still be in flight
    __builtin_amdgcn_s_waitcnt(PANEL_VMCNT32);
    __syncthreads();
    // neighbouring tiles; a width of 0 drops every access to one (no next
    // tile to load, no results of a previous tile to store)
    const __amdgpu_buffer_rsrc_t RN = rsrc(next ? t + 1 : t), RP = rsrc(prev ? t - 1 : t);
    const int nnc = next ? ncols(t + 1) : 0, npc = prev ? ncols(t - 1) : 0;
    const bool mm = active && cur;
    // the k loop: MODE 0 loads and stores only, 1 products for the k steps
    // below kpad, 2 products for all 32 steps, 3 for the first 24 (kpad =
    // 96: the order-96 early-deflation and AED windows).  Modes 2 and 3
    // have no test inside: the loop is one block in which the compiler
    // interleaves memory operations with the products.
    auto kloop = [&](auto mode) {
      constexpr int MODE = decltype(mode)::value;
      double bn[4];
      if constexpr (MODE > 0) {
        for (int ib = 0; ib < 2; ++ib)
          for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) bn[jb] = X[(jb * 16 + li) + lk * LDT];
      }
#pragma unroll
      for (int ks = 0; ks < UPAD / 4; ++ks) {
        if (ks < 16) {   // loads of tile t+1, then stores of tile t-1
          load_one(pre[2 * ks], RN, nnc, 2 * ks);
          load_one(pre[2 * ks + 1], RN, nnc, 2 * ks + 1);
        } else {
          store_one(accp, RP, npc, 2 * ks - 32);
          store_one(accp, RP, npc, 2 * ks - 31);
        }
        if (ks >= 24) {   // tile t+1 into the other buffer
#pragma unroll
          for (int q = 0; q < 4; ++q) lds_one(XN, 4 * (ks - 24) + q);
        }
        if constexpr (MODE > 0) {
          if (MODE == 2 || (MODE == 3 && ks < 24) || (MODE == 1 && 4 * ks < kpad)) {
            double b[4];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) b[jb] = bn[jb];
            const int kp = MODE == 2 ? UPAD : (MODE == 3 ? 96 : kpad);
            const int kn = min(4 * ks + 4, kp - 4) + lk;   // the last step re-reads a valid row
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
      }
    };
    if (mm && kpad == UPAD) kloop(std::integral_constant<int, 2>());
    else if (mm && kpad == 96) kloop(std::integral_constant<int, 3>());
    else if (mm) kloop(std::integral_constant<int, 1>());
    else kloop(std::integral_constant<int, 0>());
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
__device__ void panel_colq_tiles(const WinCtx& d, int t0, int t1, int tiles_c, double* Xs) {
  const int p = d.p, ws = d.ws;
  const int kpad = (ws + 3) & ~3;
  const double* Ut = d.U;
  const int tid = threadIdx.x;
  // wave index in a scalar register: the tests on it below are uniform branches
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
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
  // tile t: first element (row r0, column p), leading dimension in bytes
  // and number of rows
  struct Tile { __amdgpu_buffer_rsrc_t R; unsigned ldb; int nr; };
  auto tile = [&](int t) {
    Tile T;
    if (t < tiles_c) {
      const int r0 = d.rtop + t * PT;
      T.R = panel_rsrc(d.H + (size_t)r0 + (size_t)p * d.ldh);
      T.ldb = (unsigned)d.ldh * 8u; T.nr = min(PT, p - r0);
    } else {
      const int r0 = (t - tiles_c) * PT;
      T.R = panel_rsrc(d.Q + (size_t)r0 + (size_t)p * d.ldq);
      T.ldb = (unsigned)d.ldq * 8u; T.nr = min(PT, d.n - r0);
    }
    return T;
  };
  auto load_one = [&](double& dst, const Tile& T, int e) {
    const int c = wave + 4 * e;
    dst = panel_load(T.R, (lane < T.nr ? lane * 8u : PANEL_OOB) +
                              (c < ws ? (unsigned)c * T.ldb : PANEL_OOB));
  };
  auto store_one = [&](const d4 (&res)[4][2], const Tile& T, int s) {
    const int ib = s >> 3, jb = (s >> 2) & 1, e = s & 3;
    const int row = ib * 16 + lk + 4 * e, col = j0 + jb * 16 + li;
    const unsigned off = (row < T.nr && col < ws) ? (unsigned)row * 8u + (unsigned)col * T.ldb
                                                  : PANEL_OOB;
    panel_store(T.R, off, res[ib][jb][e]);
  };
  double pre[32];
  // as in the row panel (inside the buffer)
  auto lds_one = [&](double* X, int e) { X[lane + (wave + 4 * e) * LDT] = pre[e]; };
  {
    const Tile T = tile(t0);
#pragma unroll
    for (int e = 0; e < 32; ++e) load_one(pre[e], T, e);
  }
  __builtin_amdgcn_s_waitcnt(0);   // U and the first tile are in registers
#pragma unroll
  for (int e = 0; e < 32; ++e) lds_one(Xs, e);
  d4 acc[4][2], accp[4][2];
  for (int ib = 0; ib < 4; ++ib)   // as in the row panel
    for (int jb = 0; jb < 2; ++jb) accp[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
  for (int t = t0; t <= t1; ++t) {
    const bool cur = t < t1, prev = t > t0 && active, next = t + 1 < t1;
    double* X = Xs + ((t - t0) & 1) * (WMAX * LDT);
    double* XN = Xs + ((t - t0 + 1) & 1) * (WMAX * LDT);
    __builtin_amdgcn_s_waitcnt(PANEL_VMCNT32);   // as in the row panel
    __syncthreads();
    // neighbouring tiles; 0 rows drop every access to one
    Tile TN = tile(next ? t + 1 : t0), TP = tile(prev ? t - 1 : t0);
    if (!next) TN.nr = 0;
    if (!prev) TP.nr = 0;
    const bool mm = active && cur;
    // the k loop, MODE as in the row panel
    auto kloop = [&](auto mode) {
      constexpr int MODE = decltype(mode)::value;
      double an[4];
      if constexpr (MODE > 0) {
        for (int ib = 0; ib < 4; ++ib)
          for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ib = 0; ib < 4; ++ib) an[ib] = X[(ib * 16 + li) + lk * LDT];
      }
#pragma unroll
      for (int ks = 0; ks < UPAD / 4; ++ks) {
        if (ks < 16) {   // as in the row panel
          load_one(pre[2 * ks], TN, 2 * ks);
          load_one(pre[2 * ks + 1], TN, 2 * ks + 1);
        } else {
          store_one(accp, TP, 2 * ks - 32);
          store_one(accp, TP, 2 * ks - 31);
        }
        if (ks >= 24) {
#pragma unroll
          for (int q = 0; q < 4; ++q) lds_one(XN, 4 * (ks - 24) + q);
        }
        if constexpr (MODE > 0) {
          if (MODE == 2 || (MODE == 3 && ks < 24) || (MODE == 1 && 4 * ks < kpad)) {
            double av[4];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) av[ib] = an[ib];
            const int kp = MODE == 2 ? UPAD : (MODE == 3 ? 96 : kpad);
            const int kn = min(4 * ks + 4, kp - 4) + lk;   // the last step re-reads a valid row
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
      }
    };
    if (mm && kpad == UPAD) kloop(std::integral_constant<int, 2>());
    else if (mm && kpad == 96) kloop(std::integral_constant<int, 3>());
    else if (mm) kloop(std::integral_constant<int, 1>());
    else kloop(std::integral_constant<int, 0>());
    if (mm) {
      for (int ib = 0; ib < 4; ++ib)
        for (int jb = 0; jb < 2; ++jb) accp[ib][jb] = acc[ib][jb];
    }
  }
}

// ============================================================================
// Batched deflation scan: one workgroup of 256 threads per matrix.  Negligible subdiagonal
// entries of rows 1..kbot are set to zero; converged 1x1 and 2x2 blocks at
// the bottom are peeled off at once: (wr, wi) are written, and each 2x2
// block is standardised with its rotation applied to the rest of H and to Q.
// ============================================================================
constexpr int DB_WORDS = 2048;   // n <= 65536

// bits: (T.kbot >> 5) + 1 words of LDS; s_kt: one int of LDS.
__device__ void deflate_b_wg(const DeflB& T, unsigned* bits, int& s_kt) {
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

}  // namespace schur
