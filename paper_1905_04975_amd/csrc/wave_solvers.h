// wave_solvers.h -- one-wavefront LDS solvers of the Schur engine: the
// small-block Francis double-shift QR and the aggressive-early-deflation
// window step.  Included by kernels.hip and batch_kernels.hip; written
// against the HIP device API only (threadIdx, __syncthreads through
// solver_sync, __shfl_xor, __ballot), so the same source also runs under a
// CPU emulation of one wavefront in the tests.
#pragma once
#include "schur_internal.h"
#include "device_common.h"
#include "kernels.h"

namespace schur {

// ============================================================================
// Small-block Francis double-shift QR (one wavefront, block in LDS)
// ============================================================================

// Column-major LDS block with odd leading dimension (spreads banks).
template <int MAXM>
struct SmallSmem {
  static constexpr int LD = MAXM | 1;
};

// One double-shift bulge chase over rows/cols l..i of the m x m block in
// LDS with Schur vectors (whole-block updates: left to column m-1, right from
// row 0, all rows of Z), for m <= 64.  Lane q owns column q in the left
// updates and row q (of S and of Z) in the right updates.  Per position r
// the wavefront waits for LDS once instead of three times:
//  * the bulge column S(r..r+2, r-1) was just computed by the right update
//    of position r-1 in row lanes r..r+2 and is taken from their registers
//    (lane_read);
//  * the left update's operands S(r..r+2, q) were loaded at the end of
//    position r-1, right after its stores, so the load overlaps the
//    reflector of position r;
//  * the right update's operands S(q, r..r+2) are loaded after the left
//    stores of this position (the one wait); Z's columns r, r+1 come from
//    this lane's previous Z update and column r+2, untouched so far in this
//    step, was loaded a position ahead.
// Every updated value is stored to LDS at once, so the block in LDS is exact
// after every position (the lanes of a wavefront access LDS in order;
// wave_sync orders the accesses that read another lane's stores).
// x, y, z: first column of the shift polynomial (position l).
template <int MAXM>
__device__ void chase_reg(double* S, double* Zs, int m_in, int l_in, int i_in, double x,
                          double y, double z) {
  static_assert((MAXM & 1) == 0, "row MAXM of the LDS block is padding");
  constexpr int LD = SmallSmem<MAXM>::LD;
  // the bounds are the same in every lane: in scalar registers, the position
  // loop and the lane numbers of lane_read are scalar too
  const int m = __builtin_amdgcn_readfirstlane(m_in);
  const int l = __builtin_amdgcn_readfirstlane(l_in);
  const int i = __builtin_amdgcn_readfirstlane(i_in);
  const int q = threadIdx.x;
  const bool inm = q < m;
  const int qc = inm ? q : m - 1;   // clamped: every lane issues valid loads
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };
  // left operands S(r..r+2, q) and Z(q, r..r+2) of the first position; the
  // first two rows are kept as loaded (lA, lB) beside this lane's previous
  // left-update results (pA, pB) and chosen only where the left update uses
  // them, so that the wait for the loads falls after the reflector
  double lA = Sx(l, qc), lB = Sx(l + 1, qc), cC = Sx(l + 2, qc);
  double pA = 0.0, pB = 0.0;
  bool far = false;
  double zA = Zx(qc, l), zB = Zx(qc, l + 1), zC = Zx(qc, l + 2);
  double o1 = 0.0;   // S(q, r-1) from this row's last right update
  wave_sync();       // every lane has read its operands before any lane stores
  for (int r = l; r <= i - 1; ++r) {
    const bool three = r <= i - 2;
    const int r2 = three ? r + 2 : r + 1;   // the third row / column, or a valid stand-in
    if (r > l) {
      x = lane_read(o1, r);
      y = lane_read(o1, r + 1);
      z = three ? lane_read(o1, r + 2) : 0.0;
    }
    const Refl h = make_reflector_fast(three ? 3 : 2, x, y, z);
    const double tv2 = h.tau * h.v2, tv3 = h.tau * h.v3;

    // ---- left update: rows r..r+2 of every column (column lane q).  No
    // branches: columns left of the bulge hold exact zeros in these rows (the
    // block is Hessenberg and the bulge column is set below), so updating
    // them rewrites zeros; lanes past the block store to the padding row
    // MAXM (never read); a 2-row reflector stores its second row twice.
    // Each position is then one straight-line block, and each wait for LDS
    // sits where a loaded value is used.
    const double cA = far ? pA : lA, cB = far ? pB : lB;
    const double a3 = three ? cC : 0.0;
    const double wl = cA + h.v2 * cB + h.v3 * a3;
    const double n2 = cB - tv2 * wl, n3 = a3 - tv3 * wl;
    {
      const bool bc = r > l && q == r - 1;   // the bulge column: beta above two zeros
      Sx(inm ? r : MAXM, qc) = bc ? h.beta : cA - h.tau * wl;
      Sx(inm ? r + 1 : MAXM, qc) = bc ? 0.0 : n2;
      Sx(inm ? r2 : MAXM, qc) = bc ? 0.0 : (three ? n3 : n2);
    }
    wave_sync();   // the left stores precede the right update's loads

    // ---- right update: columns r..r+2 of every row (rows below min(r+3, i)
    // hold zeros there and rewrite them), all rows of Z
    const double s1 = Sx(qc, r), s2 = Sx(qc, r + 1), t3 = Sx(qc, r2);
    const double s3 = three ? t3 : 0.0;
    const double z3 = three ? zC : 0.0;
    const double wr = s1 + h.v2 * s2 + h.v3 * s3;
    const double wz = zA + h.v2 * zB + h.v3 * z3;
    const double e1 = s1 - h.tau * wr;
    const double e2 = s2 - tv2 * wr;
    const int qs = inm ? q : MAXM;   // lanes past the block: the padding row
    Sx(qs, r) = e1;
    Sx(qs, r + 1) = e2;
    Sx(qs, r2) = three ? s3 - tv3 * wr : e2;
    o1 = e1;
    const double f2 = zB - tv2 * wz, f3 = z3 - tv3 * wz;
    Zx(qs, r) = zA - h.tau * wz;
    Zx(qs, r + 1) = f2;
    Zx(qs, r2) = three ? f3 : f2;
    zA = f2;
    zB = f3;
    wave_sync();   // this position's stores precede the loads below
    // operands of position r+1: S(r+1..r+3, q) as just stored, Z(q, r+3)
    // untouched so far (indices clamped to the block)
    const int r3 = (r + 3 < m - 1) ? r + 3 : m - 1;
    lA = Sx(r + 1, qc);
    lB = Sx((r + 2 < m - 1) ? r + 2 : m - 1, qc);
    cC = Sx(r3, qc);
    zC = Zx(qc, r3);
    // columns right of the next bulge were changed by this left update only:
    // its results (equal to the loaded values) stay in the registers that
    // were stored from, which the compiler then does not reuse early
    far = q >= r + 3;
    pA = n2;
    pB = n3;
  }
  solver_sync();
}

// The same chase for 64 < m <= 128: lane q owns columns q and q + 64 in the
// left updates and rows q and q + 64 (of S and of Z) in the right updates;
// the bulge column comes from the slot of the lanes that computed it.
template <int MAXM>
__device__ void chase_reg2(double* S, double* Zs, int m_in, int l_in, int i_in, double x,
                           double y, double z) {
  static_assert((MAXM & 1) == 0, "row MAXM of the LDS block is padding");
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = __builtin_amdgcn_readfirstlane(m_in);
  const int l = __builtin_amdgcn_readfirstlane(l_in);
  const int i = __builtin_amdgcn_readfirstlane(i_in);
  const int q = threadIdx.x;        // slot 0: q < 64 < m
  const int qb = q + 64;            // slot 1
  const bool inb = qb < m;
  const int qbc = inb ? qb : m - 1;   // clamped: every lane issues valid loads
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };
  // value of row `row` of the last right update, from the lane that owns it
  auto bulge = [&](double o0, double o1, int row) -> double {
    return (row < 64) ? lane_read(o0, row) : lane_read(o1, row - 64);
  };
  // first two rows as loaded (l*) and this lane's previous left-update
  // results (p*), chosen where the left update uses them (see chase_reg)
  double lA0 = Sx(l, q), lB0 = Sx(l + 1, q), cC0 = Sx(l + 2, q);
  double lA1 = Sx(l, qbc), lB1 = Sx(l + 1, qbc), cC1 = Sx(l + 2, qbc);
  double pA0 = 0.0, pB0 = 0.0, pA1 = 0.0, pB1 = 0.0;
  bool far0 = false, far1 = false;
  double zA0 = Zx(q, l), zB0 = Zx(q, l + 1), zC0 = Zx(q, l + 2);
  double zA1 = Zx(qbc, l), zB1 = Zx(qbc, l + 1), zC1 = Zx(qbc, l + 2);
  double o0 = 0.0, o1 = 0.0;   // S(q, r-1), S(q+64, r-1) from the last right update
  wave_sync();
  for (int r = l; r <= i - 1; ++r) {
    const bool three = r <= i - 2;
    const int r2 = three ? r + 2 : r + 1;
    if (r > l) {
      x = bulge(o0, o1, r);
      y = bulge(o0, o1, r + 1);
      z = three ? bulge(o0, o1, r + 2) : 0.0;
    }
    const Refl h = make_reflector_fast(three ? 3 : 2, x, y, z);
    const double tv2 = h.tau * h.v2, tv3 = h.tau * h.v3;

    // ---- left update: rows r..r+2, columns q and q+64 (from r on)
    const double cA0 = far0 ? pA0 : lA0, cB0 = far0 ? pB0 : lB0;
    const double cA1 = far1 ? pA1 : lA1, cB1 = far1 ? pB1 : lB1;
    const double a30 = three ? cC0 : 0.0, a31 = three ? cC1 : 0.0;
    const double wl0 = cA0 + h.v2 * cB0 + h.v3 * a30;
    const double wl1 = cA1 + h.v2 * cB1 + h.v3 * a31;
    const double n20 = cB0 - tv2 * wl0, n30 = a30 - tv3 * wl0;
    const double n21 = cB1 - tv2 * wl1, n31 = a31 - tv3 * wl1;
    // every lane stores every entry, without branches (see chase_reg); the
    // second slot of lanes past the block stores to the padding row MAXM
    {
      const bool bc0 = r > l && q == r - 1, bc1 = r > l && qb == r - 1;   // bulge column
      Sx(r, q) = bc0 ? h.beta : cA0 - h.tau * wl0;
      Sx(r + 1, q) = bc0 ? 0.0 : n20;
      Sx(r2, q) = bc0 ? 0.0 : (three ? n30 : n20);
      Sx(inb ? r : MAXM, qbc) = bc1 ? h.beta : cA1 - h.tau * wl1;
      Sx(inb ? r + 1 : MAXM, qbc) = bc1 ? 0.0 : n21;
      Sx(inb ? r2 : MAXM, qbc) = bc1 ? 0.0 : (three ? n31 : n21);
    }
    wave_sync();   // the left stores precede the right update's loads

    // ---- right update: columns r..r+2 of rows q, q+64 (rows below
    // min(r+3, i) hold zeros there and rewrite them), and of rows q, q+64
    // of Z
    const double s10 = Sx(q, r), s20 = Sx(q, r + 1), t30 = Sx(q, r2);
    const double s11 = Sx(qbc, r), s21 = Sx(qbc, r + 1), t31 = Sx(qbc, r2);
    const double s30 = three ? t30 : 0.0, s31 = three ? t31 : 0.0;
    const double z30 = three ? zC0 : 0.0, z31 = three ? zC1 : 0.0;
    const double wr0 = s10 + h.v2 * s20 + h.v3 * s30;
    const double wr1 = s11 + h.v2 * s21 + h.v3 * s31;
    const double wz0 = zA0 + h.v2 * zB0 + h.v3 * z30;
    const double wz1 = zA1 + h.v2 * zB1 + h.v3 * z31;
    const double e10 = s10 - h.tau * wr0, e11 = s11 - h.tau * wr1;
    const double e20 = s20 - tv2 * wr0, e21 = s21 - tv2 * wr1;
    Sx(q, r) = e10;
    Sx(q, r + 1) = e20;
    Sx(q, r2) = three ? s30 - tv3 * wr0 : e20;
    const int qs1 = inb ? qb : MAXM;   // second slot past the block: the padding row
    Sx(qs1, r) = e11;
    Sx(qs1, r + 1) = e21;
    Sx(qs1, r2) = three ? s31 - tv3 * wr1 : e21;
    o0 = e10;
    o1 = e11;
    const double f20 = zB0 - tv2 * wz0, f30 = z30 - tv3 * wz0;
    const double f21 = zB1 - tv2 * wz1, f31 = z31 - tv3 * wz1;
    Zx(q, r) = zA0 - h.tau * wz0;
    Zx(q, r + 1) = f20;
    Zx(q, r2) = three ? f30 : f20;
    Zx(qs1, r) = zA1 - h.tau * wz1;
    Zx(qs1, r + 1) = f21;
    Zx(qs1, r2) = three ? f31 : f21;
    zA0 = f20;
    zB0 = f30;
    zA1 = f21;
    zB1 = f31;
    wave_sync();   // this position's stores precede the loads below
    // operands of position r+1 (indices clamped to the block); columns right
    // of the next bulge keep this left update's results from the registers
    const int r3 = (r + 3 < m - 1) ? r + 3 : m - 1;
    const int rb = (r + 2 < m - 1) ? r + 2 : m - 1;
    lA0 = Sx(r + 1, q);
    lB0 = Sx(rb, q);
    lA1 = Sx(r + 1, qbc);
    lB1 = Sx(rb, qbc);
    cC0 = Sx(r3, q);
    cC1 = Sx(r3, qbc);
    zC0 = Zx(q, r3);
    zC1 = Zx(qbc, r3);
    far0 = q >= r + 3;
    far1 = qb >= r + 3;
    pA0 = n20;
    pB0 = n30;
    pA1 = n21;
    pB1 = n31;
  }
  solver_sync();
}

// Chain of kb double-shift bulges over rows/cols l..i of the m x m block in
// LDS with Schur vectors, one bulge per wavefront of the workgroup (kb <= the
// wavefronts; the others idle through the barriers).  Bulge b, chased by
// wavefront b, enters at the top three positions after bulge b-1, so at step
// k it is at position p = l + k - 3b; (s, t) is this wavefront's shift pair
// as (sum, product).  A step is two phases, each closed by a workgroup
// barrier: every bulge's reflector from the left (rows p..p+2, lane q owning
// columns q and q + 64), then from the right (columns p..p+2 of S and of Z,
// lane q owning rows q and q + 64).  In a phase the bulges touch disjoint
// rows (left) or disjoint columns (right); where the left update of one
// bulge meets the right update of the bulge ahead (rows p-3..p-1 of columns
// p..p+2) the two commute, and a bulge's own column, read before its left
// update, is untouched by the others since its last right update.  So the
// result is that of kb single-bulge sweeps one after the other with the
// shift pairs fixed beforehand (the multishift sweep of the paper, Sec. 2,
// at the scale of one workgroup): no step waits for the chase of another
// bulge.  NS = 1 for m <= 64, 2 for 64 < m <= 128.  Updates run over every
// column and row of the block without branches, as in chase_reg (entries
// outside a bulge's reach hold exact zeros and are rewritten as zeros);
// lanes past the block store to the padding row MAXM.  WZ = false: no Schur
// vectors (Zs unused), for eigenvalues only.
template <int NS, int MAXM, bool WZ = true>
__device__ void chase_multi(double* S, double* Zs, int m_in, int l_in, int i_in, int kb_in,
                            double s, double t) {
  static_assert((MAXM & 1) == 0, "row MAXM of the LDS block is padding");
  static_assert(NS == 1 || NS == 2, "one or two columns per lane");
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = __builtin_amdgcn_readfirstlane(m_in);
  const int l = __builtin_amdgcn_readfirstlane(l_in);
  const int i = __builtin_amdgcn_readfirstlane(i_in);
  const int kb = __builtin_amdgcn_readfirstlane(kb_in);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int q = threadIdx.x & 63;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };
  int cc[NS], cs[NS];   // this lane's columns (rows), clamped; store index
  bool in[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int c = q + 64 * k;
    in[k] = c < m;
    cc[k] = in[k] ? c : m - 1;
    cs[k] = in[k] ? c : MAXM;
  }
  auto bulge = [](double o0, double o1, int row) -> double {
    if (NS == 1 || row < 64) return lane_read(o0, row);
    return lane_read(o1, row - 64);
  };
  double o[NS], zA[NS], zB[NS], zc[NS];   // S(q, p-1); Z(q, p), Z(q, p+1), Z(q, p+2)
#pragma unroll
  for (int k = 0; k < NS; ++k) { o[k] = 0.0; zA[k] = 0.0; zB[k] = 0.0; zc[k] = 0.0; }
  Refl hn{};   // the reflector of the next position, formed before the step's last barrier
  const int nsteps = (i - l) + 3 * (kb - 1);
  for (int stp = 0; stp < nsteps; ++stp) {
    const int p = l + stp - 3 * w;
    const bool act = w < kb && p >= l && p <= i - 1;   // uniform over the wavefront
    const bool three = p <= i - 2;
    const int p2 = three ? p + 2 : p + 1;   // the third row / column, or a valid stand-in
    Refl h{};
    double tv2 = 0.0, tv3 = 0.0;
    if (act) {
      // operands first (the bulge ahead changed them in the last step)
      double a1[NS], a2[NS], a3[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        a1[k] = Sx(p, cc[k]);
        a2[k] = Sx(p + 1, cc[k]);
        a3[k] = Sx(p2, cc[k]);
        if constexpr (WZ) zc[k] = Zx(cc[k], p2);
      }
      if (p == l) {
        if constexpr (WZ) {
#pragma unroll
          for (int k = 0; k < NS; ++k) {
            zA[k] = Zx(cc[k], l);
            zB[k] = Zx(cc[k], l + 1);
          }
        }
        double x, y, z;
        first_column(Sx(l, l), Sx(l, l + 1), Sx(l + 1, l), Sx(l + 1, l + 1), Sx(l + 2, l + 1), s,
                     t, x, y, z);
        wave_sync();   // the corner (other lanes' columns) is read before the left stores
        h = make_reflector_fast(three ? 3 : 2, x, y, z);
      } else {
        h = hn;
      }
      tv2 = h.tau * h.v2;
      tv3 = h.tau * h.v3;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const double c3 = three ? a3[k] : 0.0;
        const double wl = a1[k] + h.v2 * a2[k] + h.v3 * c3;
        const double n2 = a2[k] - tv2 * wl, n3 = c3 - tv3 * wl;
        const bool bc = p > l && q + 64 * k == p - 1;   // the bulge column: beta above two zeros
        Sx(in[k] ? p : MAXM, cc[k]) = bc ? h.beta : a1[k] - h.tau * wl;
        Sx(in[k] ? p + 1 : MAXM, cc[k]) = bc ? 0.0 : n2;
        Sx(in[k] ? p2 : MAXM, cc[k]) = bc ? 0.0 : (three ? n3 : n2);
      }
    }
    __syncthreads();
    if (act) {
      // every slot's operands before any store (one LDS round trip)
      double s1[NS], s2[NS], t3[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        s1[k] = Sx(cc[k], p);
        s2[k] = Sx(cc[k], p + 1);
        t3[k] = Sx(cc[k], p2);
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const double s3 = three ? t3[k] : 0.0, z3 = three ? zc[k] : 0.0;
        const double wr = s1[k] + h.v2 * s2[k] + h.v3 * s3;
        const double wz = zA[k] + h.v2 * zB[k] + h.v3 * z3;
        const double e1 = s1[k] - h.tau * wr, e2 = s2[k] - tv2 * wr;
        Sx(cs[k], p) = e1;
        Sx(cs[k], p + 1) = e2;
        Sx(cs[k], p2) = three ? s3 - tv3 * wr : e2;
        o[k] = e1;
        if constexpr (WZ) {
          const double f2 = zB[k] - tv2 * wz, f3 = z3 - tv3 * wz;
          Zx(cs[k], p) = zA[k] - h.tau * wz;
          Zx(cs[k], p + 1) = f2;
          Zx(cs[k], p2) = three ? f3 : f2;
          zA[k] = f2;
          zB[k] = f3;
        }
      }
      // the next position's reflector from this wavefront's own results
      // (column p, rows p+1..p+3, which no other bulge touches before it is
      // used), while the stores drain ahead of the barrier
      if (p + 1 <= i - 1) {
        const bool three1 = p + 1 <= i - 2;
        const double x = bulge(o[0], o[NS - 1], p + 1);
        const double y = bulge(o[0], o[NS - 1], p + 2);
        const double z = three1 ? bulge(o[0], o[NS - 1], p + 3) : 0.0;
        hn = make_reflector_fast(three1 ? 3 : 2, x, y, z);
      }
    }
    __syncthreads();
  }
}

// Francis double-shift iteration on the m x m block already in LDS (S, and Z
// when WANTZ), one wavefront.  Writes T.wr / T.wi of converged blocks when
// given; returns 0 or the 1-based end of a block that did not converge.
// With WANTZ the whole Schur form is kept: the left updates run to the last
// column and the right updates from row 0, and Z is updated (with 64 lanes
// and m <= 64 these cost no extra step latency).
template <bool WANTZ, int MAXM>
__device__ int small_iter(const SmallTask& T, double* S, double* Zs) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = T.m;
  const int lane = threadIdx.x;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };

  int i = m - 1, its = 0, info = 0;
  // steps allowed per deflation (the budget of the LAPACK-style iteration)
  const int itmax = T.itmax > 0 ? T.itmax : 30 * (m > 10 ? m : 10);
  while (i >= 0) {
    // ---- deflation search: largest k in [1, i] with a negligible subdiagonal
    int l = 0;
    for (int top = i; top >= 1; top -= 64) {
      const int k = top - lane;
      bool neg = false;
      if (k >= 1) {
        const double sub = fabs(Sx(k, k - 1));
        double tst = fabs(Sx(k - 1, k - 1)) + fabs(Sx(k, k));
        if (tst == 0.0) {
          tst = fabs(Sx(k - 1, k));
          if (k >= 2) tst += fabs(Sx(k - 1, k - 2));
          if (k + 1 <= i) tst += fabs(Sx(k + 1, k));
        }
        neg = (sub <= kUlp * tst);
      }
      const unsigned long long mask = __ballot(neg);
      if (mask) {
        l = top - __builtin_ctzll(mask);
        break;
      }
    }
    solver_sync();
    if (l > 0 && lane == 0) Sx(l, l - 1) = 0.0;
    solver_sync();

    if (l == i) {
      if (lane == 0 && T.wr) { T.wr[i] = Sx(i, i); T.wi[i] = 0.0; }
      i -= 1; its = 0;
      continue;
    }
    if (l == i - 1) {
      const Std2 o = standardize2(Sx(i - 1, i - 1), Sx(i - 1, i), Sx(i, i - 1), Sx(i, i));
      solver_sync();
      if (WANTZ && !(o.cs == 1.0 && o.sn == 0.0)) {
        for (int c = i + 1 + lane; c < m; c += 64) {
          const double x = Sx(i - 1, c), y = Sx(i, c);
          Sx(i - 1, c) = o.cs * x + o.sn * y;
          Sx(i, c) = o.cs * y - o.sn * x;
        }
        for (int r = lane; r < i - 1; r += 64) {
          const double x = Sx(r, i - 1), y = Sx(r, i);
          Sx(r, i - 1) = o.cs * x + o.sn * y;
          Sx(r, i) = o.cs * y - o.sn * x;
        }
        for (int r = lane; r < m; r += 64) {
          const double x = Zx(r, i - 1), y = Zx(r, i);
          Zx(r, i - 1) = o.cs * x + o.sn * y;
          Zx(r, i) = o.cs * y - o.sn * x;
        }
      }
      if (lane == 0) {
        if (WANTZ) {
          Sx(i - 1, i - 1) = o.a; Sx(i - 1, i) = o.b;
          Sx(i, i - 1) = o.c;     Sx(i, i) = o.d;
        }
        if (T.wr) {
          T.wr[i - 1] = o.wr1; T.wi[i - 1] = o.wi1;
          T.wr[i] = o.wr2;     T.wi[i] = o.wi2;
        }
      }
      solver_sync();
      i -= 2; its = 0;
      continue;
    }
    its += 1;
    if (its > itmax) { info = i + 1; break; }

    // ---- shifts: trailing 2x2 (Francis) or the ad-hoc exceptional pair
    double s, t;
    if (its % 10 == 0) {   // ad-hoc pair every 10 steps without deflation
      double w, e;
      if ((its / 10) % 2 == 1) {
        w = fabs(Sx(i, i - 1)) + fabs(Sx(i - 1, i - 2));
        e = Sx(i, i) + 0.75 * w;
      } else {
        w = fabs(Sx(l + 1, l)) + fabs(Sx(l + 2, l + 1));
        e = Sx(l, l) + 0.75 * w;
      }
      s = e + e;
      t = e * e + 0.4375 * w * w;
    } else {
      const double a = Sx(i - 1, i - 1), b = Sx(i - 1, i), c = Sx(i, i - 1), d = Sx(i, i);
      s = a + d;
      t = a * d - b * c;
    }

    // ---- one double-shift step on rows/cols l..i
    const int cend = WANTZ ? m - 1 : i;    // last column of left updates
    const int rbeg = WANTZ ? 0 : l;        // first row of right updates
    double x, y, z;
    first_column(Sx(l, l), Sx(l, l + 1), Sx(l + 1, l), Sx(l + 1, l + 1), Sx(l + 2, l + 1), s, t,
                 x, y, z);
    solver_sync();   // every lane has read the corner before the first left update
    if (WANTZ && m <= 64) {
      chase_reg<MAXM>(S, Zs, m, l, i, x, y, z);
      continue;
    }
    if (WANTZ && MAXM > 64 && m <= 128) {
      chase_reg2<MAXM>(S, Zs, m, l, i, x, y, z);
      continue;
    }
    for (int r = l; r <= i - 1; ++r) {
      const int nr = (r <= i - 2) ? 3 : 2;
      // the third row / column of a 2-row reflector is replaced by a valid
      // neighbour and the value selected away: every phase issues all its
      // loads at once, without a branch, and never reads outside the block
      const int r3 = (nr == 3) ? r + 2 : r + 1;
      if (r > l) {
        x = Sx(r, r - 1);
        y = Sx(r + 1, r - 1);
        const double zz = Sx(r3, r - 1);
        z = (nr == 3) ? zz : 0.0;
      }
      const Refl h = make_reflector_fast(nr, x, y, z);
      if (h.tau == 0.0) continue;   // uniform: every lane formed the same reflector
      const double tv2 = h.tau * h.v2, tv3 = h.tau * h.v3;
      // left: rows r..r+2, columns r..cend (column r-1 is written after the
      // barrier, as every lane has read it above)
      for (int c = r + lane; c <= cend; c += 64) {
        const double a1 = Sx(r, c), a2 = Sx(r + 1, c), t3 = Sx(r3, c);
        const double a3 = (nr == 3) ? t3 : 0.0;
        const double w = a1 + h.v2 * a2 + h.v3 * a3;
        Sx(r, c) = a1 - h.tau * w;
        Sx(r + 1, c) = a2 - tv2 * w;
        Sx(r3, c) = (nr == 3) ? a3 - tv3 * w : a2 - tv2 * w;   // r3 = r + 1 for two rows
      }
      solver_sync();
      if (r > l && lane == 0) {
        Sx(r, r - 1) = h.beta;
        Sx(r + 1, r - 1) = 0.0;
        if (nr == 3) Sx(r + 2, r - 1) = 0.0;
      }
      // right: columns r..r+2 of rows rbeg..rlast, and of every row of Z,
      // in one pass (one lane: one row of each)
      const int rlast = (r + 3 < i) ? r + 3 : i;
      const int nzr = WANTZ ? m : 0;
      const int nsr = rlast - rbeg + 1;
      const int ntask = nsr > nzr ? nsr : nzr;
      for (int q = lane; q < ntask; q += 64) {
        // clamped rows: all loads are issued together, stores are predicated
        const int qs = (rbeg + q <= rlast) ? rbeg + q : rlast;
        const int qz = (q < m) ? q : m - 1;
        const double s1 = Sx(qs, r), s2 = Sx(qs, r + 1), ts3 = Sx(qs, r3);
        double z1 = 0.0, z2 = 0.0, tz3 = 0.0;
        if (WANTZ) {
          z1 = Zx(qz, r);
          z2 = Zx(qz, r + 1);
          tz3 = Zx(qz, r3);
        }
        const double s3 = (nr == 3) ? ts3 : 0.0;
        const double z3 = (nr == 3) ? tz3 : 0.0;
        const double ws = s1 + h.v2 * s2 + h.v3 * s3;
        const double wz = z1 + h.v2 * z2 + h.v3 * z3;
        if (q < nsr) {
          Sx(qs, r) = s1 - h.tau * ws;
          Sx(qs, r + 1) = s2 - tv2 * ws;
          if (nr == 3) Sx(qs, r + 2) = s3 - tv3 * ws;
        }
        if (WANTZ && q < nzr) {
          Zx(qz, r) = z1 - h.tau * wz;
          Zx(qz, r + 1) = z2 - tv2 * wz;
          if (nr == 3) Zx(qz, r + 2) = z3 - tv3 * wz;
        }
      }
      solver_sync();
    }
  }
  solver_sync();
  return info;
}

// LDS scratch of the multi-wavefront iteration: the eigenvalues of the
// trailing block (order <= 8), the shift pairs and their count.
constexpr int SMALL_MW_AUX = 16 + 2 * 4 + 1;

// Eigenvalues of an n x n upper Hessenberg block (n <= 8) held one entry per
// lane (entry (r, c) in lane r + 8c; zeros outside the block): the Francis
// double-shift iteration of small_iter without Schur vectors (the same
// deflation test, Francis and exceptional shifts, 2x2 standardisation).
// A position's reflector comes from three lanes' entries (readlane); the
// left update gathers each column's rows p..p+2 and the right update each
// row's columns p..p+2 by lane permutes, so the whole iteration stays in
// registers (no LDS round trip, no barrier).  Updates span the whole block
// (entries outside a reflector's reach are zero or off the active block,
// as in chase_reg).  er/ei written by lane 0; returns 0 or the 1-based end
// of a block that did not converge.  One wavefront.
__device__ int tiny_eigs8(double h, int n, double* er, double* ei) {
  const int lane = threadIdx.x & 63;
  const int row = lane & 7, col = lane >> 3;
  auto at = [&](int r, int c) -> double { return lane_read(h, r + 8 * c); };
  auto gather = [&](int src) -> double { return __shfl(h, src & 63, 64); };
  int i = n - 1, its = 0, info = 0;
  const int itmax = 30 * 10;
  while (i >= 0) {
    // ---- deflation: lane (k, k-1) tests subdiagonal entry k, 1 <= k <= i
    {
      const double dkm = gather(lane - 1), dk = gather(lane + 8);   // H(k-1,k-1), H(k,k)
      const double up = gather(lane + 7), lft = gather(lane - 9), dn = gather(lane + 9);
      const bool sub = row == col + 1 && row <= i;
      double tst = fabs(dkm) + fabs(dk);
      if (tst == 0.0) {
        tst = fabs(up);
        if (row >= 2) tst += fabs(lft);
        if (row + 1 <= i) tst += fabs(dn);
      }
      const bool neg = sub && fabs(h) <= kUlp * tst;
      const unsigned long long mask = __ballot(neg);
      const int l = mask ? (63 - __builtin_clzll(mask) + 8) / 9 : 0;   // lane 9k - 8 -> k
      if (l > 0 && row == l && col == l - 1) h = 0.0;
      if (l == i) {
        const double v = at(i, i);
        if (lane == 0) { er[i] = v; ei[i] = 0.0; }
        i -= 1; its = 0;
        continue;
      }
      if (l == i - 1) {
        const Std2 o = standardize2(at(i - 1, i - 1), at(i - 1, i), at(i, i - 1), at(i, i));
        if (lane == 0) {
          er[i - 1] = o.wr1; ei[i - 1] = o.wi1;
          er[i] = o.wr2;     ei[i] = o.wi2;
        }
        i -= 2; its = 0;
        continue;
      }
      its += 1;
      if (its > itmax) { info = i + 1; break; }
      // ---- shifts: trailing 2x2 (Francis) or the ad-hoc pair
      double s, t;
      if (its % 10 == 0) {
        double wv, e;
        if ((its / 10) % 2 == 1) {
          wv = fabs(at(i, i - 1)) + fabs(at(i - 1, i - 2));
          e = at(i, i) + 0.75 * wv;
        } else {
          wv = fabs(at(l + 1, l)) + fabs(at(l + 2, l + 1));
          e = at(l, l) + 0.75 * wv;
        }
        s = e + e;
        t = e * e + 0.4375 * wv * wv;
      } else {
        const double a = at(i - 1, i - 1), b = at(i - 1, i), c = at(i, i - 1), d = at(i, i);
        s = a + d;
        t = a * d - b * c;
      }
      double x, y, z;
      first_column(at(l, l), at(l, l + 1), at(l + 1, l), at(l + 1, l + 1), at(l + 2, l + 1), s, t,
                   x, y, z);
      // ---- one double-shift step on rows/cols l..i
      for (int p = l; p <= i - 1; ++p) {
        const bool three = p <= i - 2;
        const int p2 = three ? p + 2 : p + 1;
        if (p > l) {
          x = at(p, p - 1);
          y = at(p + 1, p - 1);
          z = three ? at(p2, p - 1) : 0.0;
        }
        const Refl r = make_reflector_fast(three ? 3 : 2, x, y, z);
        const double tv2 = r.tau * r.v2, tv3 = r.tau * r.v3;
        {   // left: rows p..p+2 of this lane's column
          const double a1 = gather(p + 8 * col), a2 = gather(p + 1 + 8 * col), a3 = gather(p2 + 8 * col);
          const double wl = a1 + r.v2 * a2 + r.v3 * (three ? a3 : 0.0);
          const double cf = row == p ? r.tau : row == p + 1 ? tv2 : (three && row == p + 2) ? tv3 : 0.0;
          h -= cf * wl;
          if (p > l && col == p - 1 && row >= p && row <= p2) h = row == p ? r.beta : 0.0;
        }
        {   // right: columns p..p+2 of this lane's row
          const double b1 = gather(row + 8 * p), b2 = gather(row + 8 * (p + 1)), b3 = gather(row + 8 * p2);
          const double wr = b1 + r.v2 * b2 + r.v3 * (three ? b3 : 0.0);
          const double cf = col == p ? r.tau : col == p + 1 ? tv2 : (three && col == p + 2) ? tv3 : 0.0;
          h -= cf * wr;
        }
      }
    }
  }
  return info;
}

// Shift pairs for a chain of nsh / 2 bulges (nsh <= 8): the eigenvalues of
// the trailing nsh x nsh block S(i-nsh+1..i, i-nsh+1..i) (tiny_eigs8) as
// (sum, product) pairs in aux[SMALL_MW_SH + 2b], aux[SMALL_MW_SH + 2b + 1]:
// complex conjugate pairs first, then the real eigenvalues two at a time,
// each group by decreasing modulus; the number of pairs goes to
// aux[SMALL_MW_SH + 8] (0 when the iteration did not converge).  One
// wavefront.
constexpr int SMALL_MW_SH = 16;
template <int MAXM>
__device__ void trailing_shifts(const double* S, int i, int nsh, double* aux) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  double* const er = aux;
  double* const ei = aux + 8;
  double* const sh = aux + SMALL_MW_SH;
  const int lane = threadIdx.x & 63;
  const int i0 = i - nsh + 1;
  const int r = lane & 7, c = lane >> 3;
  const double h = (r < nsh && c < nsh && r <= c + 1) ? S[(i0 + r) + (i0 + c) * LD] : 0.0;
  const int info = tiny_eigs8(h, nsh, er, ei);
  wave_sync();
  if (lane == 0) {
    int np = 0;
    unsigned used = 0;
    if (info == 0) {
      for (int it = 0; it < nsh; ++it) {   // complex pairs (positive imaginary parts)
        int best = -1;
        double bm = -1.0;
        for (int k = 0; k < nsh; ++k) {
          const double md = er[k] * er[k] + ei[k] * ei[k];
          if (!((used >> k) & 1u) && ei[k] > 0.0 && md > bm) { bm = md; best = k; }
        }
        if (best < 0) break;
        used |= 1u << best;
        sh[2 * np] = er[best] + er[best];
        sh[2 * np + 1] = bm;
        ++np;
      }
      bool half = false;
      double first = 0.0;
      for (int it = 0; it < nsh; ++it) {   // real ones, two at a time
        int best = -1;
        double bm = -1.0;
        for (int k = 0; k < nsh; ++k)
          if (!((used >> k) & 1u) && ei[k] == 0.0 && fabs(er[k]) > bm) { bm = fabs(er[k]); best = k; }
        if (best < 0) break;
        used |= 1u << best;
        if (!half) {
          first = er[best];
        } else {
          sh[2 * np] = first + er[best];
          sh[2 * np + 1] = first * er[best];
          ++np;
        }
        half = !half;
      }
    }
    sh[8] = (double)np;
  }
  wave_sync();
}

// The Francis iteration of small_iter (with Schur vectors) by a workgroup of
// K wavefronts: the deflation checks and 2x2 standardisations as there, each
// step a chain of up to K bulges (chase_multi) with shifts from the trailing
// 2kb x 2kb block (trailing_shifts); kb = K while the active block has at
// least 6 K rows, halved below, and one bulge (wavefront 0 alone, Francis or
// exceptional shifts as in small_iter) for small active blocks and every
// tenth step without deflation.  Needs the wavefront-local solver_sync
// (SCHUR_SOLVER_WAVE_SYNC): the one-wavefront parts run on wavefront 0 while
// the others wait at the workgroup barrier.  aux: SMALL_MW_AUX doubles of
// LDS.  Every wavefront returns the same info.  WZ = false: eigenvalues only
// (no Schur vectors, converged 2x2 blocks not standardised in place, single
// bulges as chains of one).
template <int MAXM, int K, bool WZ = true>
__device__ int small_iter_mw(const SmallTask& T, double* S, double* Zs, double* aux) {
#ifndef SCHUR_SOLVER_WAVE_SYNC
  static_assert(K < 0, "the multi-wavefront iteration needs the wavefront-local solver_sync");
#endif
  static_assert(K == 2 || K == 4, "two or four wavefronts");
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = T.m;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };
  const double* const sh = aux + SMALL_MW_SH;

  int i = m - 1, its = 0, info = 0;
  const int itmax = T.itmax > 0 ? T.itmax : 30 * (m > 10 ? m : 10);
  while (i >= 0) {
    // ---- deflation search (every wavefront the same, reads only)
    int l = 0;
    for (int top = i; top >= 1; top -= 64) {
      const int k = top - lane;
      bool neg = false;
      if (k >= 1) {
        const double sub = fabs(Sx(k, k - 1));
        double tst = fabs(Sx(k - 1, k - 1)) + fabs(Sx(k, k));
        if (tst == 0.0) {
          tst = fabs(Sx(k - 1, k));
          if (k >= 2) tst += fabs(Sx(k - 1, k - 2));
          if (k + 1 <= i) tst += fabs(Sx(k + 1, k));
        }
        neg = (sub <= kUlp * tst);
      }
      const unsigned long long mask = __ballot(neg);
      if (mask) {
        l = top - __builtin_ctzll(mask);
        break;
      }
    }
    __syncthreads();
    if (w == 0 && l > 0 && lane == 0) Sx(l, l - 1) = 0.0;
    __syncthreads();

    if (l == i) {
      if (w == 0 && lane == 0 && T.wr) { T.wr[i] = Sx(i, i); T.wi[i] = 0.0; }
      i -= 1; its = 0;
      continue;
    }
    if (l == i - 1) {
      const Std2 o = standardize2(Sx(i - 1, i - 1), Sx(i - 1, i), Sx(i, i - 1), Sx(i, i));
      __syncthreads();
      if (WZ && w == 0) {
        if (!(o.cs == 1.0 && o.sn == 0.0)) {
          for (int c = i + 1 + lane; c < m; c += 64) {
            const double x = Sx(i - 1, c), y = Sx(i, c);
            Sx(i - 1, c) = o.cs * x + o.sn * y;
            Sx(i, c) = o.cs * y - o.sn * x;
          }
          for (int r = lane; r < i - 1; r += 64) {
            const double x = Sx(r, i - 1), y = Sx(r, i);
            Sx(r, i - 1) = o.cs * x + o.sn * y;
            Sx(r, i) = o.cs * y - o.sn * x;
          }
          for (int r = lane; r < m; r += 64) {
            const double x = Zx(r, i - 1), y = Zx(r, i);
            Zx(r, i - 1) = o.cs * x + o.sn * y;
            Zx(r, i) = o.cs * y - o.sn * x;
          }
        }
        if (lane == 0) {
          Sx(i - 1, i - 1) = o.a; Sx(i - 1, i) = o.b;
          Sx(i, i - 1) = o.c;     Sx(i, i) = o.d;
          if (T.wr) {
            T.wr[i - 1] = o.wr1; T.wi[i - 1] = o.wi1;
            T.wr[i] = o.wr2;     T.wi[i] = o.wi2;
          }
        }
      }
      if (!WZ && w == 0 && lane == 0 && T.wr) {
        T.wr[i - 1] = o.wr1; T.wi[i - 1] = o.wi1;
        T.wr[i] = o.wr2;     T.wi[i] = o.wi2;
      }
      __syncthreads();
      i -= 2; its = 0;
      continue;
    }
    its += 1;
    if (its > itmax) { info = i + 1; break; }

    // ---- shifts: a chain of kb bulges, or one (Francis or exceptional)
    int kb = K;
    while (kb > 1 && i - l + 1 < 6 * kb) kb >>= 1;
    if (its % 10 == 0) kb = 1;
    double s = 0.0, t = 0.0;
    if (kb > 1) {
      if (w == 0) trailing_shifts<MAXM>(S, i, 2 * kb, aux);
      __syncthreads();
      const int np = (int)sh[8];
      kb = np < kb ? np : kb;
      if (w < kb) { s = sh[2 * w]; t = sh[2 * w + 1]; }
    }
    if (kb >= 2) {
      if (m <= 64) chase_multi<1, MAXM, WZ>(S, Zs, m, l, i, kb, s, t);
      else         chase_multi<2, MAXM, WZ>(S, Zs, m, l, i, kb, s, t);
      continue;
    }
    if (WZ ? w == 0 : true) {
      if (its % 10 == 0) {   // ad-hoc pair every 10 steps without deflation
        double wv, e;
        if ((its / 10) % 2 == 1) {
          wv = fabs(Sx(i, i - 1)) + fabs(Sx(i - 1, i - 2));
          e = Sx(i, i) + 0.75 * wv;
        } else {
          wv = fabs(Sx(l + 1, l)) + fabs(Sx(l + 2, l + 1));
          e = Sx(l, l) + 0.75 * wv;
        }
        s = e + e;
        t = e * e + 0.4375 * wv * wv;
      } else {
        const double a = Sx(i - 1, i - 1), b = Sx(i - 1, i), c = Sx(i, i - 1), d = Sx(i, i);
        s = a + d;
        t = a * d - b * c;
      }
      if constexpr (WZ) {
        double x, y, z;
        first_column(Sx(l, l), Sx(l, l + 1), Sx(l + 1, l), Sx(l + 1, l + 1), Sx(l + 2, l + 1), s,
                     t, x, y, z);
        solver_sync();   // every lane has read the corner before the first left update
        if (m <= 64) chase_reg<MAXM>(S, Zs, m, l, i, x, y, z);
        else         chase_reg2<MAXM>(S, Zs, m, l, i, x, y, z);
      }
    }
    if constexpr (!WZ) {   // one bulge on wavefront 0, the others through the barriers
      __syncthreads();     // every wavefront has read the shift inputs
      if (m <= 64) chase_multi<1, MAXM, false>(S, Zs, m, l, i, 1, s, t);
      else         chase_multi<2, MAXM, false>(S, Zs, m, l, i, 1, s, t);
      continue;
    }
    __syncthreads();
  }
  __syncthreads();
  return info;
}

template <bool WANTZ, int MAXM>
__device__ void small_load(const SmallTask& T, double* S, double* Zs) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = T.m;
  const int lane = threadIdx.x;
  for (int c = 0; c < m; ++c)
    for (int r = lane; r < m; r += 64)
      S[r + c * LD] = (r <= c + 1) ? T.A[r + (size_t)c * T.lda] : 0.0;
  if (WANTZ)
    for (int c = 0; c < m; ++c)
      for (int r = lane; r < m; r += 64) Zs[r + c * LD] = (r == c) ? 1.0 : 0.0;
  solver_sync();
}

// Whole small-block solve: load, iterate, then the Schur form back in place
// and Z (or Z^T, or Qacc Z) out.  K > 1: a workgroup of K wavefronts
// iterates (small_iter_mw, aux: SMALL_MW_AUX doubles of LDS); loading and
// writing back are done by wavefront 0, from which the others return.
template <bool WANTZ, int MAXM, int K = 1>
__device__ void small_qr(const SmallTask& T, double* S, double* Zs, double* aux = nullptr) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int m = T.m;
  const int lane = threadIdx.x;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };
  int info;
  if constexpr (K > 1) {
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (w == 0) small_load<WANTZ, MAXM>(T, S, Zs);
    __syncthreads();
    info = small_iter_mw<MAXM, K, WANTZ>(T, S, Zs, aux);
    if (w != 0) return;
  } else {
    small_load<WANTZ, MAXM>(T, S, Zs);
    info = small_iter<WANTZ, MAXM>(T, S, Zs);
  }
  if (lane == 0 && T.info) *T.info = info;
  if (WANTZ) {
    // Schur form of the block back to global memory, Z^T into the U slot layout
    for (int c = 0; c < m; ++c)
      for (int r = lane; r < m; r += 64) T.A[r + (size_t)c * T.lda] = Sx(r, c);
    if (T.Zt) {
      for (int c = 0; c < T.ldzt; ++c)
        for (int r = lane; r < T.ldzt; r += 64)
          T.Zt[r + (size_t)c * T.ldzt] = (r < m && c < m) ? Zx(c, r) : 0.0;
    }
    if (T.Z) {
      for (int c = 0; c < m; ++c)
        for (int r = lane; r < m; r += 64) T.Z[r + (size_t)c * T.ldz] = Zx(r, c);
    }
    if (T.Qacc) {
      // Qacc <- Qacc Z, rows by lanes, 16 columns at a time; the block's LDS
      // copy (already written back) is the staging area
      solver_sync();
      for (int r = lane; r < m; r += 64) {
        for (int c0 = 0; c0 < m; c0 += 16) {
          double acc[16];
#pragma unroll
          for (int j = 0; j < 16; ++j) acc[j] = 0.0;
          for (int k = 0; k < m; ++k) {
            const double q = T.Qacc[r + (size_t)k * T.ldqacc];
#pragma unroll
            for (int j = 0; j < 16; ++j)
              if (c0 + j < m) acc[j] += q * Zx(k, c0 + j);
          }
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (c0 + j < m) Sx(r, c0 + j) = acc[j];
        }
      }
      solver_sync();
      for (int c = 0; c < m; ++c)
        for (int r = lane; r < m; r += 64) T.Qacc[r + (size_t)c * T.ldqacc] = Sx(r, c);
    }
  }
}

// ============================================================================
// Aggressive early deflation (paper Sec. 3.2: the algorithm alternates AED
// steps with bulge-chasing sweeps).  One wavefront owns a bottom window
// W = H(kwtop:kbot, kwtop:kbot) of order nw <= SMALL_Z_MAX and its spike
// s = H(kwtop, kwtop-1):
//   1. real Schur form W = V T V^T in LDS (the small Francis iteration);
//   2. from the bottom of T, a diagonal block whose spike entries s V(0, .)
//      are negligible next to it is deflated; a block that is not is moved
//      to the top of the unchecked part by orthogonal swaps of adjacent
//      diagonal blocks (direct swapping: a Sylvester equation for the
//      invariant subspace, then its QR factor);
//   3. the spike of the undeflated part is reflected onto its first entry
//      and the undeflated part is brought back to Hessenberg form;
//   4. T goes back into H, V^T into a panel slot; the caller applies V to
//      the rows right of the window, the rows above it and to Q.
// The eigenvalues of the undeflated blocks are the next sweep's shifts.
// ============================================================================

// 64-lane sums and maxima (all lanes receive the result)
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Solve M x = b (N <= 4) by Gaussian elimination with partial pivoting,
// fully unrolled (row exchanges as selects, so everything stays in
// registers); a pivot below smin in magnitude is replaced by +-smin.  b is
// overwritten by x.  The swap that uses x is checked for backward stability
// afterwards, so a poor solve only rejects the swap.
template <int N>
__device__ inline void tiny_solve(double (&M)[N][N], double (&b)[N], double smin) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    // pivot: largest |M[i][j]|, i >= j, swapped into row j
    int piv = j;
    double best = fabs(M[j][j]);
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const double v = fabs(M[i][j]);
      if (v > best) { best = v; piv = i; }
    }
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const bool sw = (piv == i);
#pragma unroll
      for (int k = j; k < N; ++k) {
        const double t = M[j][k];
        M[j][k] = sw ? M[i][k] : t;
        M[i][k] = sw ? t : M[i][k];
      }
      const double t = b[j];
      b[j] = sw ? b[i] : t;
      b[i] = sw ? t : b[i];
    }
    double d = M[j][j];
    if (fabs(d) < smin) d = (d < 0.0) ? -smin : smin;
    M[j][j] = d;
    const double rd = 1.0 / d;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const double f = M[i][j] * rd;
#pragma unroll
      for (int k = j + 1; k < N; ++k) M[i][k] -= f * M[j][k];
      b[i] -= f * b[j];
    }
  }
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    double acc = b[j];
#pragma unroll
    for (int k = j + 1; k < N; ++k) acc -= M[j][k] * b[k];
    b[j] = acc / M[j][j];
  }
}

// Householder reflectors of one swap: reflector h is I - tau[h] v[h] v[h]^T
// on rows/columns k .. k+N-1 (v[h][i] = 0 for i < h, v[h][h] = 1).
struct SwapPlan {
  double v[2][4];
  double tau[2];
};

// Plan the swap of the adjacent diagonal blocks A (P x P, at k) and
// B (R x R, at k + P) of the quasi-triangular T (LDS, leading dimension LD).
// With A X - X B = -C (C the coupling block) the columns of [X; I] span the
// invariant subspace of B; the orthogonal factor of their QR factorisation
// moves B to the top.  Returns false when the transformed block fails the
// backward-stability test (the swap is then not done).
template <int P, int R>
__device__ bool plan_swap(const double* S, int LD, int k, SwapPlan& pl) {
  constexpr int N = P + R;
  constexpr int M = P * R;
  double T[N][N];
  double dnorm = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T[i][j] = (i <= j + 1) ? S[(k + i) + (k + j) * LD] : 0.0;
      dnorm = fmax(dnorm, fabs(T[i][j]));
    }
  const double tiny = 2.2250738585072014e-308;
  const double smin = fmax(kUlp * dnorm, tiny);
  // Kronecker form of A X - X B = -C, unknown x[i + P j] = X(i, j)
  double K[M][M], x[M];
#pragma unroll
  for (int j = 0; j < R; ++j)
#pragma unroll
    for (int i = 0; i < P; ++i) {
#pragma unroll
      for (int jj = 0; jj < R; ++jj)
#pragma unroll
        for (int ii = 0; ii < P; ++ii)
          K[i + P * j][ii + P * jj] = (jj == j ? T[i][ii] : 0.0) - (ii == i ? T[P + jj][P + j] : 0.0);
      x[i + P * j] = -T[i][P + j];
    }
  tiny_solve<M>(K, x, smin);
#pragma unroll
  for (int h = 0; h < 2; ++h) {   // every entry of the plan defined
    pl.tau[h] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) pl.v[h][i] = 0.0;
  }
  // W = [X; I] (N x R), QR by R Householder reflectors
  double W[N][R];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) W[i][j] = (i < P) ? x[i + P * j] : (i - P == j ? 1.0 : 0.0);
#pragma unroll
  for (int h = 0; h < R; ++h) {
    double tail = 0.0;
#pragma unroll
    for (int i = h + 1; i < N; ++i) tail = fmax(tail, fabs(W[i][h]));
    const double alpha = W[h][h];
#pragma unroll
    for (int i = 0; i < 4; ++i) pl.v[h][i] = 0.0;
    pl.v[h][h] = 1.0;
    pl.tau[h] = 0.0;
    if (tail == 0.0 || !isfinite(tail) || !isfinite(alpha)) {
      if (!(tail == 0.0)) return false;
      continue;
    }
    const int e = ilogb(fmax(fabs(alpha), tail));
    double ss = 0.0;
#pragma unroll
    for (int i = h + 1; i < N; ++i) {
      const double t = ldexp(W[i][h], -e);
      ss += t * t;
    }
    const double as = ldexp(alpha, -e);
    const double nrm = sqrt(as * as + ss);
    const double bs = (as < 0.0) ? nrm : -nrm;
    const double ds = as - bs;
    const double r = 1.0 / (bs * ds);
    pl.tau[h] = -ds * (ds * r);
#pragma unroll
    for (int i = h + 1; i < N; ++i) pl.v[h][i] = ldexp(W[i][h], -e) * (bs * r);
    // apply to the remaining columns of W
#pragma unroll
    for (int j = h + 1; j < R; ++j) {
      double w = 0.0;
#pragma unroll
      for (int i = h; i < N; ++i) w += pl.v[h][i] * W[i][j];
#pragma unroll
      for (int i = h; i < N; ++i) W[i][j] -= pl.tau[h] * pl.v[h][i] * w;
    }
  }
  // T' = Q^T T Q with Q = H_0 H_1 ...; accept if its lower-left block is tiny
#pragma unroll
  for (int h = 0; h < R; ++h) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double w = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) w += pl.v[h][i] * T[i][j];
#pragma unroll
      for (int i = 0; i < N; ++i) T[i][j] -= pl.tau[h] * pl.v[h][i] * w;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double w = 0.0;
#pragma unroll
      for (int j = 0; j < N; ++j) w += T[i][j] * pl.v[h][j];
#pragma unroll
      for (int j = 0; j < N; ++j) T[i][j] -= pl.tau[h] * w * pl.v[h][j];
    }
  }
  double low = 0.0;
#pragma unroll
  for (int i = R; i < N; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) low = fmax(low, fabs(T[i][j]));
  const double thresh = fmax(20.0 * kUlp * dnorm, tiny);
  return low <= thresh;   // false for NaN as well
}

// Standardise every 2x2 block of the quasi-triangular S whose first row is
// in [lo, m), updating Z.  The rotations of different blocks commute (each
// turns its own pair of rows and its own pair of columns), so all are
// computed first and then applied together.  buf: 7 m doubles of LDS.
__device__ void aed_std_all(double* S, double* Zs, int LD, int m, int lo, double* buf) {
  const int lane = threadIdx.x;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  double* cs_l = buf;
  double* sn_l = buf + m;
  double* isblk = buf + 2 * m;
  double* blk = buf + 3 * m;   // the standard block, 4 entries per start row
  for (int i = lo + lane; i < m; i += 64) {
    cs_l[i] = 1.0;
    sn_l[i] = 0.0;
    isblk[i] = 0.0;
    if (i + 1 < m && Sx(i + 1, i) != 0.0) {
      isblk[i] = 1.0;
      const Std2 o = standardize2(Sx(i, i), Sx(i, i + 1), Sx(i + 1, i), Sx(i + 1, i + 1));
      cs_l[i] = o.cs;
      sn_l[i] = o.sn;
      blk[4 * (i - lo) + 0] = o.a;
      blk[4 * (i - lo) + 1] = o.b;
      blk[4 * (i - lo) + 2] = o.c;
      blk[4 * (i - lo) + 3] = o.d;
    }
  }
  solver_sync();
  // row pairs: column c meets the blocks starting at i <= c
  for (int c = lo + lane; c < m; c += 64) {
    for (int i = lo; i + 1 < m && i <= c; ++i) {
      const double cs = cs_l[i], sn = sn_l[i];
      if (cs == 1.0 && sn == 0.0) continue;
      const double x = Sx(i, c), y = Sx(i + 1, c);
      Sx(i, c) = cs * x + sn * y;
      Sx(i + 1, c) = cs * y - sn * x;
    }
  }
  solver_sync();
  // column pairs: row r of S meets the blocks with i + 1 >= r; all rows of Z
  for (int q = lane; q < 2 * m; q += 64) {
    const bool inS = q < m;
    const int r = inS ? q : q - m;
    double* base = inS ? S : Zs;
    for (int i = lo; i + 1 < m; ++i) {
      if (inS && r > i + 1) continue;
      const double cs = cs_l[i], sn = sn_l[i];
      if (cs == 1.0 && sn == 0.0) continue;
      const double x = base[r + i * LD], y = base[r + (i + 1) * LD];
      base[r + i * LD] = cs * x + sn * y;
      base[r + (i + 1) * LD] = cs * y - sn * x;
    }
  }
  solver_sync();
  // the blocks exactly in standard form (a complex pair with equal diagonal,
  // or two real eigenvalues with a zero subdiagonal)
  for (int i = lo + lane; i + 1 < m; i += 64) {
    if (isblk[i] == 0.0) continue;
    Sx(i, i) = blk[4 * (i - lo) + 0];
    Sx(i, i + 1) = blk[4 * (i - lo) + 1];
    Sx(i + 1, i) = blk[4 * (i - lo) + 2];
    Sx(i + 1, i + 1) = blk[4 * (i - lo) + 3];
  }
  solver_sync();
}

// Householder reflector from a column held one entry per lane-slot:
// x0 = alpha (scalar), tail entries x[i] for i in [1, L) at LDS vv[i].
// On return vv[0] = 1, vv[1..L) = v, and the function yields (tau, beta).
// tau = 0 (identity) when the tail is zero.
__device__ void aed_reflector(double alpha, double* vv, int L, double& tau, double& beta) {
  const int lane = threadIdx.x;
  double tmax = 0.0;
  for (int i = 1 + lane; i < L; i += 64) tmax = fmax(tmax, fabs(vv[i]));
  tmax = wave_max(tmax);
  if (tmax == 0.0) {
    tau = 0.0;
    beta = alpha;
    solver_sync();
    if (lane == 0) vv[0] = 1.0;
    solver_sync();
    return;
  }
  const int e = ilogb(fmax(fabs(alpha), tmax));
  double ss = 0.0;
  for (int i = 1 + lane; i < L; i += 64) {
    const double t = ldexp(vv[i], -e);
    ss += t * t;
  }
  ss = wave_sum(ss);
  const double as = ldexp(alpha, -e);
  const double nrm = sqrt(as * as + ss);
  const double bs = (as < 0.0) ? nrm : -nrm;
  const double ds = as - bs;
  const double r = 1.0 / (bs * ds);
  tau = -ds * (ds * r);
  beta = ldexp(bs, e);
  const double f = bs * r;
  solver_sync();
  for (int i = 1 + lane; i < L; i += 64) vv[i] = ldexp(vv[i], -e) * f;
  if (lane == 0) vv[0] = 1.0;
  solver_sync();
}

// The whole early-deflation step on one window; S, Z (LD x MAXM each), vv
// (MAXM), ibuf (6 MAXM ints) and stdbuf (7 MAXM) live in LDS and belong to
// the calling wavefront.
// 2x2 block [[a, b], [c, d]]: eigenvalues (re +- sqrt(disc)) or re +- i im,
// without assuming standard form
__device__ __forceinline__ void block_eigs(double a, double b, double c, double d, double& re,
                                           double& im, double& r1, double& r2) {
  const double h = 0.5 * (a - d);
  const double disc = h * h + b * c;
  re = 0.5 * (a + d);
  if (disc < 0.0) {
    im = sqrt(-disc);
    r1 = r2 = re;
  } else {
    im = 0.0;
    const double sq = sqrt(disc);
    r1 = re + sq;
    r2 = re - sq;
  }
}

// Pipelined reordering for early deflation.  The sequential rule (test the
// bottom block; deflate it, or move it above every block not tested yet) is
// kept, but the moves of several undeflatable blocks run concurrently: each
// round, every moving block whose upper neighbour is untested swaps with it
// (the windows of one round are disjoint, so all left updates precede all
// right updates, as in a sweep), while the bottom block, which no swap of
// the round touches, is tested.  Untested blocks thus flow down through the
// moving ones to the bottom; every block meets the same swaps and the same
// test as in the sequential order.  Returns nu: rows [0, nu) hold the
// undeflated blocks, [nu, m) the deflated ones.  A rejected swap stops the
// reordering with everything not yet deflated counted as undeflated.
//   ibuf: 6 m ints of LDS; pbuf: 12 (m / 2 + 1) doubles of LDS.

// One swap's left transform on column c (rows k..k+N-1) or right transform
// on a row (columns k..k+N-1): a[] holds the N entries, v/tau the plan.
__device__ __forceinline__ void swap_apply(double (&a)[4], const double* v, const double* tau,
                                           int N) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double w = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) w += v[4 * h + i] * ((i < N) ? a[i] : 0.0);
    w *= tau[h];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] -= v[4 * h + i] * w;
  }
}

//   xr: rows above the block (rows -xr..-1 of S, same columns) that take the
//   right transforms too; zrows: rows of Zs that take them; srow: the row of
//   Zs whose entries, times s, form the spike (0 for a bottom window).
// K > 1: a workgroup of K wavefronts (every one calls it): wavefront 0 keeps
// the round's bookkeeping (swap list, bottom test, plans), all K apply the
// swaps, with workgroup barriers between the phases.
template <int K = 1>
__device__ int aed_reorder(double* S, double* Zs, int LD, int m, double s, int* ibuf,
                           double* pbuf, int xr = 0, int zrows = -1, int srow = 0) {
  if (zrows < 0) zrows = m;
  const int lane = threadIdx.x & 63;
  const int w = K > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
  auto sync = [&]() {
    if constexpr (K > 1) __syncthreads();
    else solver_sync();
  };
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Zs[r + c * LD]; };
  int* status = ibuf;            // per row: 0 untested, 1 undeflatable
  int* mv_pos = ibuf + m;        // moving blocks, top to bottom
  int* mv_sz = ibuf + 2 * m;
  int* mv_tgt = ibuf + 3 * m;
  int* sw_k = ibuf + 4 * m;      // this round's swaps (at most m / 2)
  int* sw_p = sw_k + m / 2;
  int* sw_j = ibuf + 5 * m;
  int* sw_ok = sw_j + m / 2;
  const int maxsw = m / 2 + 1;
  double* pl_v = pbuf;               // 8 per swap
  double* pl_t = pbuf + 8 * maxsw;   // 2 per swap
  double* pl_d = pbuf + 10 * maxsw;  // 2 per swap (restored 1x1 diagonals)
  __shared__ int sh_nmv, sh_bot, sh_left, sh_tgt, sh_nsw;
  if (w == 0) {
    for (int i = lane; i < m; i += 64) status[i] = 0;
    if (lane == 0) {
      sh_nmv = 0; sh_bot = m - 1; sh_left = m; sh_tgt = 0;
    }
  }
  sync();
  const double tiny = 2.2250738585072014e-308;
  const double smlnum = tiny * ((double)m / kUlp);
  int rounds = 0;
  while (true) {
    const int nmv = sh_nmv, bot = sh_bot, left = sh_left;
    if (left == 0 || ++rounds > 4 * m + 16) break;   // the bound is never reached
    // ---- this round's swaps: moving blocks with an untested upper neighbour
    // (wavefront 0)
    int nsw = 0;
    for (int base = 0; w == 0 && base < nmv; base += 64) {
      const int j = base + lane;
      bool go = false;
      int k = 0, as = 1;
      if (j < nmv) {
        const int pos = mv_pos[j];
        if (pos > mv_tgt[j] && status[pos - 1] == 0) {
          as = (pos - 2 >= 0 && status[pos - 2] == 0 && Sx(pos - 1, pos - 2) != 0.0) ? 2 : 1;
          k = pos - as;
          go = true;
        }
      }
      const unsigned long long mask = __ballot(go);
      if (go) {
        const int idx = nsw + __builtin_popcountll(mask & ((1ull << lane) - 1ull));
        sw_k[idx] = k;
        sw_p[idx] = as;
        sw_j[idx] = j;
      }
      nsw += __builtin_popcountll(mask);
    }
    if (w == 0 && lane == 0) sh_nsw = nsw;
    // ---- bottom block test (it meets no swap window of this round)
    const bool test = w == 0 && status[bot] == 0;
    const int bs = (test && bot >= 1 && status[bot - 1] == 0 && Sx(bot, bot - 1) != 0.0) ? 2 : 1;
    bool defl = false;
    if (test) {
      double foo, spk;
      if (bs == 1) {
        foo = fabs(Sx(bot, bot));
        spk = fabs(s * Zx(srow, bot));
      } else {
        double re, im, r1, r2;
        block_eigs(Sx(bot - 1, bot - 1), Sx(bot - 1, bot), Sx(bot, bot - 1), Sx(bot, bot), re, im,
                   r1, r2);
        foo = (im != 0.0) ? fabs(re) + im : fmax(fabs(r1), fabs(r2));
        spk = fmax(fabs(s * Zx(srow, bot)), fabs(s * Zx(srow, bot - 1)));
      }
      if (foo == 0.0) foo = fabs(s);
      defl = spk <= fmax(smlnum, kUlp * foo);
    }
    sync();
    nsw = sh_nsw;
    // ---- plans, one lane of wavefront 0 per swap
    if (w == 0 && lane < nsw) {
      const int k = sw_k[lane], pp = sw_p[lane], rr = mv_sz[sw_j[lane]];
      SwapPlan pl;
      bool ok;
      if (pp == 1 && rr == 1) ok = plan_swap<1, 1>(S, LD, k, pl);
      else if (pp == 1) ok = plan_swap<1, 2>(S, LD, k, pl);
      else if (rr == 1) ok = plan_swap<2, 1>(S, LD, k, pl);
      else ok = plan_swap<2, 2>(S, LD, k, pl);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        pl_t[2 * lane + h] = (h < rr) ? pl.tau[h] : 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) pl_v[8 * lane + 4 * h + i] = (h < rr) ? pl.v[h][i] : 0.0;
      }
      pl_d[2 * lane] = Sx(k, k);                                   // A's 1x1 eigenvalue
      pl_d[2 * lane + 1] = Sx(k + pp + rr - 1, k + pp + rr - 1);   // B's
      sw_ok[lane] = ok ? 1 : 0;
    }
    sync();
    const bool bad = lane < nsw && sw_ok[lane] == 0;
    if (__ballot(bad) != 0ull) break;   // uniform: nothing of this round is applied
    if (nsw > 0) {
      // threads in groups of G per swap; a group walks its swap's columns
      // (left) and rows (right) two at a time
      const int tid = w * 64 + lane;
      const int G = 64 * K / nsw;
      const int t = tid / G, sub = tid - t * G;
      const bool mine = t < nsw;
      int k = 0, pp = 1, rr = 1, N = 2;
      double v[8], tau[2];
      if (mine) {
        k = sw_k[t]; pp = sw_p[t]; rr = mv_sz[sw_j[t]]; N = pp + rr;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = pl_v[8 * t + i];
        tau[0] = pl_t[2 * t]; tau[1] = pl_t[2 * t + 1];
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = 0.0;
        tau[0] = tau[1] = 0.0;
      }
      // left: columns k..m-1, rows k..k+N-1
      if (mine) {
        for (int c = k + sub; c < m; c += 2 * G) {
          const int c2 = c + G;
          const bool two = c2 < m;
          double a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = Sx((i < N) ? k + i : k, c);
#pragma unroll
          for (int i = 0; i < 4; ++i) b[i] = Sx((i < N) ? k + i : k, two ? c2 : c);
          swap_apply(a, v, tau, N);
          swap_apply(b, v, tau, N);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (i < N) Sx(k + i, c) = a[i];
          if (two) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (i < N) Sx(k + i, c2) = b[i];
          }
        }
      }
      sync();
      // right: rows -xr..k+N-1 of S, then rows 0..zrows-1 of Z (one index
      // space; ra below is the S row relative to the block)
      if (mine) {
        const int ns = xr + k + N;
        const int tot = ns + zrows;
        const double dA = pl_d[2 * t], dB = pl_d[2 * t + 1];
        for (int q = sub; q < tot; q += 2 * G) {
          const int q2 = q + G;
          const bool two = q2 < tot;
          double* ba = (q < ns) ? S : Zs;
          const int ra = (q < ns) ? q - xr : q - ns;
          double* bb = (two && q2 < ns) ? S : Zs;
          const int rb = two ? ((q2 < ns) ? q2 - xr : q2 - ns) : ra;
          double* bbx = two ? bb : ba;
          double a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = ba[ra + ((i < N) ? k + i : k) * LD];
#pragma unroll
          for (int i = 0; i < 4; ++i) b[i] = bbx[rb + ((i < N) ? k + i : k) * LD];
          swap_apply(a, v, tau, N);
          swap_apply(b, v, tau, N);
          // rows of S inside the window: exact zeros below the moved block and
          // the 1x1 eigenvalues restored
          if (q < ns) {
            if (ra >= k + rr) { a[0] = 0.0; if (rr == 2) a[1] = 0.0; }
            if (rr == 1 && ra == k) a[0] = dB;
            if (pp == 1 && ra == k + rr) a[rr] = dA;
          }
          if (two && q2 < ns) {
            if (rb >= k + rr) { b[0] = 0.0; if (rr == 2) b[1] = 0.0; }
            if (rr == 1 && rb == k) b[0] = dB;
            if (pp == 1 && rb == k + rr) b[rr] = dA;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (i < N) ba[ra + (k + i) * LD] = a[i];
          if (two) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (i < N) bb[rb + (k + i) * LD] = b[i];
          }
        }
      }
    }
    sync();
    // ---- bookkeeping (wavefront 0): each swap's lane moves its block; the
    // last lane records the bottom test (disjoint rows and entries)
    if (w == 0 && lane < nsw) {
      const int j = sw_j[lane], k = sw_k[lane], pp = sw_p[lane], rr = mv_sz[j];
      mv_pos[j] = k;
      for (int i = 0; i < rr; ++i) status[k + i] = 1;
      for (int i = 0; i < pp; ++i) status[k + rr + i] = 0;
    }
    if (lane == 63 && test) {
      if (defl) {
        sh_bot = bot - bs;
      } else {
        const int j = nmv;
        mv_pos[j] = bot - bs + 1;
        mv_sz[j] = bs;
        mv_tgt[j] = sh_tgt;
        sh_tgt += bs;
        for (int i = 0; i < bs; ++i) status[bot - bs + 1 + i] = 1;
        sh_nmv = nmv + 1;
      }
      sh_left = left - bs;
    }
    sync();
  }
  sync();
  return sh_bot + 1;
}

// V^T of a window into its panel slot (ldut x ldut, zero padded), after one
// first-order re-orthogonalisation V <- V (I - E / 2), E = V^T V - I: V's
// own rounding (it collected every rotation of the window) would otherwise
// reach Q.  S (free once the window is written back) holds E.  Both
// products as FP64 MFMA 16 x 16 tiles (16x16x4 steps, operands straight
// from LDS, zero outside the window), the tiles shared by the K wavefronts
// of the workgroup (K = 1: the calling wavefront).
typedef double wv_d4 __attribute__((ext_vector_type(4)));
template <int K = 1>
__device__ void aed_write_vt(double* S, const double* Z, int LD, int nw, double* Ut, int ldut) {
  const int lane = threadIdx.x & 63;
  const int w = K > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
  const int kr = lane >> 4, kc = lane & 15;   // operand (k, i) / result (i % 4, j) of a lane
  const int nt = (nw + 15) >> 4;
  auto Zx = [&](int r, int c) -> double { return Z[r + c * LD]; };
  auto sync = [&]() {
    if constexpr (K > 1) __syncthreads();
    else solver_sync();
  };
  // ---- E = V^T V - I: E(i, j) = sum_r V(r, i) V(r, j)
  for (int tix = w; tix < nt * nt; tix += K) {
    const int I0 = (tix % nt) * 16, J0 = (tix / nt) * 16;
    const int ia = I0 + kc, jb = J0 + kc;
    const int iac = ia < nw ? ia : nw - 1, jbc = jb < nw ? jb : nw - 1;
    wv_d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nw; k0 += 4) {
      const int r = k0 + kr;
      const int rc = r < nw ? r : nw - 1;
      const double av = Zx(rc, iac), bv = Zx(rc, jbc);
      const double a = (r < nw && ia < nw) ? av : 0.0;   // A(i, k) = V(k, i)
      const double b = (r < nw && jb < nw) ? bv : 0.0;   // B(k, j) = V(k, j)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I0 + 4 * e + kr, col = J0 + kc;
      if (row < nw && col < nw) S[row + col * LD] = acc[e] - (row == col ? 1.0 : 0.0);
    }
  }
  sync();
  // ---- Ut(j, r) = (V - V E / 2)(r, j)
  for (int tix = w; tix < nt * nt; tix += K) {
    const int R0 = (tix % nt) * 16, J0 = (tix / nt) * 16;
    const int ra = R0 + kc, jb = J0 + kc;
    const int rac = ra < nw ? ra : nw - 1, jbc = jb < nw ? jb : nw - 1;
    wv_d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nw; k0 += 4) {
      const int k = k0 + kr;
      const int kk = k < nw ? k : nw - 1;
      const double av = Zx(rac, kk), bv = S[kk + jbc * LD];
      const double a = (k < nw && ra < nw) ? av : 0.0;   // A(i, k) = V(R0 + i, k)
      const double b = (k < nw && jb < nw) ? bv : 0.0;   // B(k, j) = E(k, J0 + j)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = R0 + 4 * e + kr, j = J0 + kc;
      const double v = (r < nw && j < nw) ? Zx(r, j) - 0.5 * acc[e] : 0.0;
      if (r < ldut && j < ldut) Ut[j + (size_t)r * ldut] = v;
    }
  }
  // ---- zeros of the slot outside the tiles (ldut >= nw)
  const int nt16 = nt * 16 < ldut ? nt * 16 : ldut;
  const int wide = (ldut - nt16) * ldut;          // columns j >= nt16 of every row r
  const int rest = (ldut - nt16) * nt16;          // rows r >= nt16, columns j < nt16
  for (int x = w * 64 + lane; x < wide + rest; x += 64 * K) {
    int j, r;
    if (x < wide) { r = x / (ldut - nt16); j = nt16 + x % (ldut - nt16); }
    else { const int y = x - wide; r = nt16 + y / nt16; j = y % nt16; }
    Ut[j + (size_t)r * ldut] = 0.0;
  }
}

// Anti-transpose of the trailing block T = S(lo:nw, lo:nw) in place
// (T(r, c) <-> T(d-1-c, d-1-r), d = nw - lo), with the columns lo..nw-1 of
// the rows above it (S(0:lo, .)) and of Z (all nw rows) put in reverse
// order.  J T^T J is quasi-triangular when T is; a similarity by Y of the
// flipped block is a similarity by J Y J of T, and the reversed columns take
// it as their right transform.  The map is its own inverse.
__device__ void flip_tail(double* S, double* Z, int LD, int nw, int lo) {
  const int lane = threadIdx.x;
  const int d = nw - lo;
  solver_sync();
  if (d <= 1) return;
  for (int idx = lane; idx < d * d; idx += 64) {
    const int r = idx % d, c = idx / d;
    if (r + c < d - 1) {
      double* p = S + (lo + r) + (lo + c) * LD;
      double* q = S + (lo + d - 1 - c) + (lo + d - 1 - r) * LD;
      const double t = *p;
      *p = *q;
      *q = t;
    }
  }
  const int rows = lo + nw;
  const int half = d / 2;
  for (int idx = lane; idx < rows * half; idx += 64) {
    const int q = idx % rows, j = idx / rows;
    double* base = (q < lo) ? S + q : Z + (q - lo);
    double* p1 = base + (lo + j) * LD;
    double* p2 = base + (nw - 1 - j) * LD;
    const double t = *p1;
    *p1 = *p2;
    *p2 = t;
  }
  solver_sync();
}

// Reflector I - tau vv vv^T (vv[0] = 1, L entries) applied to rows
// r0..r0+L-1 of S over columns c0..ncols-1 (left), then to columns
// r0..r0+L-1 over rows -xr..rend-1 of S and rows 0..zrows-1 of Z (right).
// K > 1: by the K wavefronts of the workgroup (columns, then rows, split
// over all threads, a workgroup barrier after each phase).
template <int K = 1>
__device__ void refl_apply(double* S, double* Z, int LD, const double* vv, double tau, int r0,
                           int L, int c0, int ncols, int xr, int rend, int zrows) {
  const int tid = K > 1 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  auto sync = [&]() {
    if constexpr (K > 1) __syncthreads();
    else solver_sync();
  };
  for (int c = c0 + tid; c < ncols; c += 64 * K) {
    double w = 0.0;
    for (int i = 0; i < L; ++i) w += vv[i] * S[(r0 + i) + c * LD];
    w *= tau;
    for (int i = 0; i < L; ++i) S[(r0 + i) + c * LD] -= vv[i] * w;
  }
  sync();
  const int ns = xr + rend;
  for (int q = tid; q < ns + zrows; q += 64 * K) {
    double* base = (q < ns) ? S + (q - xr) : Z + (q - ns);
    double w = 0.0;
    for (int j = 0; j < L; ++j) w += base[(r0 + j) * LD] * vv[j];
    w *= tau;
    for (int j = 0; j < L; ++j) base[(r0 + j) * LD] -= w * vv[j];
  }
  sync();
}

// The m x m quasi-triangular block B = S(0:m, 0:m) is coupled to the rest of
// the matrix through the row Z(srow, 0:m) (times a scalar): reflect that row
// onto its first entry, then bring B back to Hessenberg form with reflectors
// that leave row and column 0 alone.  Left transforms run over columns
// 0..ncols-1, right transforms over rows -xr..m-1 of S and rows 0..zrows-1
// of Z.  Returns the first entry of the reflected row.  K > 1: every
// wavefront of the workgroup calls it; wavefront 0 forms the reflectors
// (published through LDS), all apply them.
template <int K = 1>
__device__ double spike_reduce(double* S, double* Z, int LD, int m, int ncols, int xr, int zrows,
                               int srow, double* vv) {
  const int lane = threadIdx.x & 63;
  const int w = K > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto sync = [&]() {
    if constexpr (K > 1) __syncthreads();
    else solver_sync();
  };
  // a reflector's (tau, beta) for the other wavefronts, two buffers used in
  // turn: a buffer is rewritten only after every wavefront passed the barrier
  // that follows its last read
  __shared__ double sh_tb[2][2];
  int par = 0;
  sync();
  if (m <= 0) return 0.0;
  if (m == 1) return Z[srow];
  if (w == 0) {
    for (int i = lane; i < m; i += 64) vv[i] = Z[srow + i * LD];
    solver_sync();
    const double alpha = vv[0];
    double t0, b0;
    aed_reflector(alpha, vv, m, t0, b0);
    if (lane == 0) { sh_tb[par][0] = t0; sh_tb[par][1] = b0; }
  }
  sync();
  const double tau = sh_tb[par][0], beta = sh_tb[par][1];
  par ^= 1;
  if (tau != 0.0) refl_apply<K>(S, Z, LD, vv, tau, 0, m, 0, ncols, xr, m, zrows);
  for (int j = 0; j + 2 < m; ++j) {
    const int L = m - j - 1;   // rows j+1 .. m-1
    if (w == 0) {
      const double a0 = Sx(j + 1, j);
      for (int i = 1 + lane; i < L; i += 64) vv[i] = Sx(j + 1 + i, j);
      solver_sync();
      double tj, bj;
      aed_reflector(a0, vv, L, tj, bj);
      if (lane == 0) { sh_tb[par][0] = tj; sh_tb[par][1] = bj; }
      if (tj != 0.0) {
        if (lane == 0) Sx(j + 1, j) = bj;
        for (int i = 2 + lane; i <= L; i += 64) Sx(j + i, j) = 0.0;
      }
    }
    sync();
    const double tj = sh_tb[par][0];
    par ^= 1;
    if (tj == 0.0) continue;
    refl_apply<K>(S, Z, LD, vv, tj, j + 1, L, j + 1, ncols, xr, m, zrows);
  }
  sync();
  return beta;
}

// K > 1: every wavefront of a workgroup of K calls it: the iteration, the
// reordering, the spike reduction and the write of V^T are the K
// wavefronts', the standardisation and the eigenvalue output wavefront 0's
// (the solvers' barrier must then be the wavefront-local one).
template <int MAXM, int K = 1>
__device__ void aed_window(const AedTask& T, double* S, double* Z, double* vv, int* ibuf,
                           double* stdbuf) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int lane = threadIdx.x & 63;
  const int w = K > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
  const int nw = T.nw;
  const int kwtop = T.kbot - nw + 1;
  if (nw < 1 || nw > MAXM || kwtop < T.ktop) return;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto sync = [&]() {
    if constexpr (K > 1) __syncthreads();
    else solver_sync();
  };
  double* Hw = T.H + kwtop + (size_t)kwtop * T.ldh;
  const double s = (kwtop > T.ktop) ? T.H[kwtop + (size_t)(kwtop - 1) * T.ldh] : 0.0;

  SmallTask st{};
  st.A = Hw; st.lda = T.ldh; st.m = nw; st.itmax = T.itmax;
  int info;
  if constexpr (K > 1) {
    if (w == 0) small_load<true, MAXM>(st, S, Z);
    __syncthreads();
    info = small_iter_mw<MAXM, K>(st, S, Z, stdbuf);   // stdbuf is free until the reordering
  } else {
    small_load<true, MAXM>(st, S, Z);
    info = small_iter<true, MAXM>(st, S, Z);
  }
  if (info != 0) {   // window not in Schur form: no deflation, no shifts
    if (threadIdx.x == 0) { T.ctrl->aed_nd = 0; T.ctrl->aed_nu = 0; }
    return;
  }

  // ---- deflation checks from the bottom, undeflatable blocks moved up
  const int nu = aed_reorder<K>(S, Z, LD, nw, s, ibuf, stdbuf);
  const int nd = nw - nu;
  if (w == 0) {
    // the deflated blocks are final: standard form now
    if (nd > 0) aed_std_all(S, Z, LD, nw, nu, stdbuf);

    // ---- eigenvalues: undeflated blocks give the next shifts, deflated
    // ones are final (written when the caller asks for them)
    for (int e = lane; e < nw; e += 64) {
      const bool first = (e + 1 < nw) && Sx(e + 1, e) != 0.0;
      const bool second = (e >= 1) && Sx(e, e - 1) != 0.0;
      double wr = Sx(e, e), wi = 0.0;
      if (first || second) {
        const int b0 = first ? e : e - 1;
        double re, im, r1, r2;
        block_eigs(Sx(b0, b0), Sx(b0, b0 + 1), Sx(b0 + 1, b0), Sx(b0 + 1, b0 + 1), re, im, r1, r2);
        if (e >= nu) {   // standard form: read off the block as the final S shows it
          wr = Sx(e, e);
          wi = sqrt(fabs(Sx(b0, b0 + 1))) * sqrt(fabs(Sx(b0 + 1, b0)));
          if (second) wi = -wi;
        } else if (im != 0.0) {
          wr = re;
          wi = first ? im : -im;
        } else {
          wr = first ? r1 : r2;
        }
      }
      if (e < nu) {
        T.sr[e] = wr;
        T.si[e] = wi;
      } else if (T.wr) {
        T.wr[e] = wr;
        T.wi[e] = wi;
      }
    }
    if (lane == 0) { T.ctrl->aed_nd = nd; T.ctrl->aed_nu = nu; }
  }
  if (nd == 0) return;   // nothing deflated: H stays as it was

  // ---- the spike s V(0, 0:nu) reflected onto its first entry and the
  // undeflated part back to Hessenberg form (the reflector of V(0, .) is
  // that of s V(0, .), whose first entry is s times V(0, .)'s)
  const double spike = nu >= 1 ? s * spike_reduce<K>(S, Z, LD, nu, nw, 0, nw, 0, vv) : 0.0;
  sync();

  // ---- write back: the window and its spike
  for (int c = w; c < nw; c += K)
    for (int r = lane; r <= c + 1 && r < nw; r += 64) Hw[r + (size_t)c * T.ldh] = Sx(r, c);
  if (threadIdx.x == 0 && kwtop > T.ktop) T.H[kwtop + (size_t)(kwtop - 1) * T.ldh] = spike;
  sync();
  aed_write_vt<K>(S, Z, LD, nw, T.Ut, T.ldut);
}


// ============================================================================
// Early deflation on many windows at once.  Windows tile the unreduced
// blocks of H; each window W (order nw <= SMALL_Z_MAX) is coupled to the
// rest of its block by one subdiagonal entry above it (st, row 0 of W) and
// one below it (sb, last column of W).  With W = V T V^T in real Schur form
// the couplings become st V(0, .) on the left and sb V(nw-1, .) below.
//   1. blocks whose entries of st V(0, .) are not negligible move to the top
//      of T (the bottom-window reordering, rows [0, nu));
//   2. if every one of them has negligible entries in sb V(nw-1, .), the
//      window splits its block: among the remaining blocks, those with
//      negligible sb V(nw-1, .) entries stay on top (free: deflated), the
//      others move to the bottom (rows [bs, nw)); this is the same
//      reordering on the flipped block J T^T J, whose spike is the last row
//      of V;
//   3. each coupled part is brought back to Hessenberg form with its
//      coupling reflected onto one entry (the upper part as after a bottom
//      window, the lower one flipped), so that H stays Hessenberg with zero
//      subdiagonal entries around the free part;
//   4. the window and V^T go out; the caller applies V to the panels and to
//      Q and scales the coupling entries by the reflected first entries.
// A window that does not split is left untouched (V = I).  Every dropped
// entry is below the early-deflation threshold, so each pass is a backward
// stable orthogonal similarity, as a bottom window is (paper Sec. 3.2, AED).
// ============================================================================

template <int MAXM, int K = 1>
__device__ void split_window(const SplitTask& T, double* S, double* Z, double* vv, int* ibuf,
                             double* pbuf) {
  constexpr int LD = SmallSmem<MAXM>::LD;
  const int lane = threadIdx.x & 63;
  const int w = K > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
  const int nw = T.nw, a = T.a;
  auto Sx = [&](int r, int c) -> double& { return S[r + c * LD]; };
  auto Zx = [&](int r, int c) -> double& { return Z[r + c * LD]; };
  auto sync = [&]() {
    if constexpr (K > 1) __syncthreads();
    else solver_sync();
  };
  SplitRes out;
  out.split = 0; out.nu = nw; out.nf = 0; out.nb = 0; out.ftop = 1.0; out.fbot = 1.0;
  bool ok = false;
  // every exit below is uniform over the workgroup; with K > 1 the
  // iteration, the reorderings and the spike reductions are the K
  // wavefronts', the flips wavefront 0's
  do {
    if (nw < 1 || nw > MAXM) break;
    double* Hw = T.H + a + (size_t)a * T.ldh;
    const double st = (T.above >= 0) ? T.H[a + (size_t)(a - 1) * T.ldh] : 0.0;
    const double sb = T.below ? T.H[(a + nw) + (size_t)(a + nw - 1) * T.ldh] : 0.0;
    SmallTask t{};
    t.A = Hw; t.lda = T.ldh; t.m = nw; t.itmax = T.itmax;
    int info;
    if constexpr (K > 1) {
      if (w == 0) small_load<true, MAXM>(t, S, Z);
      __syncthreads();
      info = small_iter_mw<MAXM, K>(t, S, Z, pbuf);   // pbuf is free until the reorderings
    } else {
      small_load<true, MAXM>(t, S, Z);
      info = small_iter<true, MAXM>(t, S, Z);
    }
    if (info != 0) break;
    // ---- 1. blocks coupled upward to the top
    const int nu = (st != 0.0) ? aed_reorder<K>(S, Z, LD, nw, st, ibuf, pbuf) : 0;
    // ---- 2. they must not reach the coupling below (read only: every
    // wavefront reaches the same verdict)
    if (nu > 0 && sb != 0.0) {
      const double smlnum = 2.2250738585072014e-308 * ((double)nw / kUlp);
      bool bad = false;
      for (int e = lane; e < nu; e += 64) {
        if (e >= 1 && Sx(e, e - 1) != 0.0) continue;   // second row of a 2x2 block
        const bool two = e + 1 < nu && Sx(e + 1, e) != 0.0;
        double foo, spk;
        if (!two) {
          foo = fabs(Sx(e, e));
          spk = fabs(sb * Zx(nw - 1, e));
        } else {
          double re, im, r1, r2;
          block_eigs(Sx(e, e), Sx(e, e + 1), Sx(e + 1, e), Sx(e + 1, e + 1), re, im, r1, r2);
          foo = (im != 0.0) ? fabs(re) + im : fmax(fabs(r1), fabs(r2));
          spk = fmax(fabs(sb * Zx(nw - 1, e)), fabs(sb * Zx(nw - 1, e + 1)));
        }
        if (foo == 0.0) foo = fabs(sb);
        if (!(spk <= fmax(smlnum, kUlp * foo))) bad = true;
      }
      if (__ballot(bad) != 0ull) break;
    }
    // ---- the rest against the coupling below: free blocks stay on top,
    // coupled ones go to the bottom (a bottom-window reordering of the
    // flipped block, whose spike row is the last row of Z)
    int nb = 0;
    if (sb != 0.0 && nu < nw) {
      if (w == 0) flip_tail(S, Z, LD, nw, nu);
      sync();
      nb = aed_reorder<K>(S + nu + nu * LD, Z + nu * LD, LD, nw - nu, sb, ibuf, pbuf, nu, nw,
                          nw - 1);
      if (w == 0) flip_tail(S, Z, LD, nw, nu);
    }
    const int bs = nw - nb;
    // ---- 3. coupled parts back to Hessenberg form
    double ftop = 0.0, fbot = 0.0;
    if (nu > 0) ftop = spike_reduce<K>(S, Z, LD, nu, nw, 0, nw, 0, vv);
    if (nb > 0) {
      if (w == 0) flip_tail(S, Z, LD, nw, bs);
      fbot = spike_reduce<K>(S + bs + bs * LD, Z + bs * LD, LD, nb, nb, bs, nw, nw - 1, vv);
      if (w == 0) flip_tail(S, Z, LD, nw, bs);
    }
    out.split = 1;
    out.nu = nu;
    out.nb = nb;
    out.nf = nw - nu - nb;
    out.ftop = ftop;
    out.fbot = fbot;
    ok = true;
  } while (false);
  sync();
  if (ok) {
    // ---- 4. the window back into H (or its output slot), V^T into its slot
    double* Wd = T.Wo ? T.Wo : T.H + a + (size_t)a * T.ldh;
    const int ldw = T.Wo ? T.ldwo : T.ldh;
    for (int c = w; c < nw; c += K)
      for (int r = lane; r <= c + 1 && r < nw; r += 64) Wd[r + (size_t)c * ldw] = Sx(r, c);
    sync();
    aed_write_vt<K>(S, Z, LD, nw, T.Ut, T.ldut);
  }
  if (threadIdx.x == 0) *T.res = out;   // wavefront 0's results
}

}  // namespace schur
