// Host driver that runs the device source of the LDS kernels on the CPU
// (see hip/hip_runtime.h): the window chase of a sweep time step (1024 or
// 256 threads), the small-block solver, the early-deflation window step and
// the whole-matrix driver of the persistent batched kernel.  Test
// infrastructure.
//
//   simt_kernels chase|chase256 in.bin out.bin
//     in : int n, ktop, kbot, nst, nwin; double H[n*n] (column-major);
//          double st[nst]; nwin x int (p, ws, tau0, tau1, nb, shift0)
//     out: double H[n*n]; nwin x double Ut[128*128]
//   simt_kernels small|small2|small4 in.bin out.bin   (1, 2 or 4 wavefronts)
//     in : int m; double A[m*m] (upper Hessenberg, m <= 96)
//     out: int info; double S[m*m]; double Z[m*m]; double wr[m], wi[m]
//   simt_kernels eig|eig4 in.bin out.bin   (eigenvalues only, 1 or 4 wavefronts)
//     in : int m; double A[m*m] (upper Hessenberg, m <= 128)
//     out: int info; double wr[m], wi[m]
//   simt_kernels tiny in.bin out.bin   (eigenvalues of a block of order <= 8)
//     in : int n; double A[n*n] (upper Hessenberg)
//     out: int info; double wr[n], wi[n]
//   simt_kernels split|split4 in.bin out.bin   (1 or 4 wavefronts)
//     in : int n, a, nw, above, below; double H[n*n]
//     out: int split, nu, nf, nb; double ftop, fbot; double H[n*n];
//          double Ut[128*128]
//   simt_kernels aed|aed4 in.bin out.bin   (1 or 4 wavefronts)
//     in : int n, ktop, kbot, nw; double H[n*n]
//     out: int nd, nu; double H[n*n]; double Ut[128*128]; double sr[96], si[96];
//          double wr[n], wi[n]
// The one-wavefront solvers use the wavefront-level barrier here, as in the
// persistent batched kernel (for a workgroup of one wavefront it is the same
// as the workgroup barrier).
#define SCHUR_SOLVER_WAVE_SYNC 1
#include "hip/hip_runtime.h"
#include "wave_solvers.h"
#include "window_chase.h"
#include "batch_solve.h"

#include <atomic>

#include <cstdio>
#include <string>
#include <thread>
#include <vector>

thread_local simt_dim3 threadIdx;
thread_local simt_dim3 blockIdx;
simt_dim3 blockDim{64, 1, 1};

namespace {
// Barrier of n threads: arrival count plus a generation number; waiters spin
// briefly, then yield (the lanes outnumber the host cores, and the kernels
// cross a barrier every few instructions, where a sleeping barrier would
// spend most of the time in the kernel's scheduler).
struct SpinBarrier {
  std::atomic<int> count{0};
  std::atomic<unsigned> gen{0};
  int n = 0;
  void init(int threads) {
    n = threads;
    count.store(0);
  }
  void wait() {
    const unsigned g = gen.load(std::memory_order_acquire);
    if (count.fetch_add(1, std::memory_order_acq_rel) == n - 1) {
      count.store(0, std::memory_order_relaxed);
      gen.fetch_add(1, std::memory_order_acq_rel);
      return;
    }
    int spins = 0;
    while (gen.load(std::memory_order_acquire) == g)
      if (++spins > 32) std::this_thread::yield();
  }
};
SpinBarrier g_all, g_wave[16];
int g_threads = 64;
double g_shfl[1024];
int g_ball[1024];
}  // namespace

void __syncthreads() { g_all.wait(); }
void simt_wave_barrier() { g_wave[threadIdx.x >> 6].wait(); }

// exchanges within the calling thread's wavefront
double __shfl_xor(double x, int o, int) {
  const int l = threadIdx.x;
  g_shfl[l] = x;
  simt_wave_barrier();
  const double r = g_shfl[l ^ o];
  simt_wave_barrier();
  return r;
}

double __shfl(double x, int src, int) {
  const int l = threadIdx.x;
  g_shfl[l] = x;
  simt_wave_barrier();
  const double r = g_shfl[(l & ~63) + (src & 63)];
  simt_wave_barrier();
  return r;
}

// readlane: two slot sets used alternately, so one barrier per call is
// enough (a lane can write call k+2's slot only after every lane has passed
// call k+1's barrier, i.e. has read call k's value)
int g_rdl[2][1024];
thread_local unsigned g_rdl_calls = 0;
int simt_readlane(int v, int src) {
  const int l = threadIdx.x;
  const unsigned k = g_rdl_calls++ & 1u;
  g_rdl[k][l] = v;
  simt_wave_barrier();
  return g_rdl[k][(l & ~63) + src];
}

unsigned long long __ballot(int p) {
  const int l = threadIdx.x, base = l & ~63;
  g_ball[l] = p != 0;
  simt_wave_barrier();
  unsigned long long m = 0;
  for (int i = 0; i < 64; ++i)
    if (g_ball[base + i]) m |= 1ull << i;
  simt_wave_barrier();
  return m;
}

// D = C + A B of the wavefront: A(i, k) in lane i + 16 k, B(k, j) in lane
// j + 16 k, D(i, j) in lane j + 16 (i % 4), element i / 4
double g_ma[1024], g_mb[1024];
simt_d4 simt_mfma_f64_16x16x4(double a, double b, simt_d4 c) {
  const int t = threadIdx.x, base = t & ~63, l = t & 63;
  g_ma[t] = a;
  g_mb[t] = b;
  simt_wave_barrier();
  simt_d4 d;
  for (int e = 0; e < 4; ++e) {
    const int i = (l >> 4) + 4 * e, j = l & 15;
    double acc = c[e];
    for (int k = 0; k < 4; ++k) acc += g_ma[base + i + 16 * k] * g_mb[base + j + 16 * k];
    d[e] = acc;
  }
  simt_wave_barrier();
  return d;
}

extern char __start_simt_lds[], __stop_simt_lds[];

template <class F>
void run_workgroup(int threads, int block, F f) {
  memset(__start_simt_lds, 0xff, (size_t)(__stop_simt_lds - __start_simt_lds));   // NaN
  g_threads = threads;
  blockDim = simt_dim3{(unsigned)threads, 1, 1};
  g_all.init(threads);
  for (int w = 0; w < threads / 64; ++w) g_wave[w].init(64);
  std::vector<std::thread> th;
  for (int l = 0; l < threads; ++l)
    th.emplace_back([=] {
      threadIdx = simt_dim3{(unsigned)l, 0, 0};
      blockIdx = simt_dim3{(unsigned)block, 0, 0};
      f();
    });
  for (auto& t : th) t.join();
}

template <class T>
bool rd(FILE* f, T* p, size_t n) { return fread(p, sizeof(T), n, f) == n; }

using namespace schur;

// LDS of the 256-thread window chase and of the persistent driver
__shared__ double g_cw[LDW * WMAX];
__shared__ double g_cr[3 * REFL_LDS];
__shared__ double g_pb_lds[PB_LDS_D];
__shared__ PShared g_pb_sh;

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  const std::string mode = argv[1];
  FILE* f = fopen(argv[2], "rb");
  if (!f) return 2;
  if (mode == "chase" || mode == "chase256") {
    int hdr[5];
    if (!rd(f, hdr, 5)) return 2;
    const int n = hdr[0], ktop = hdr[1], kbot = hdr[2], nst = hdr[3], nwin = hdr[4];
    std::vector<double> H((size_t)n * n), st(nst);
    std::vector<int> wd(6 * (size_t)nwin);
    if (!rd(f, H.data(), H.size()) || !rd(f, st.data(), st.size()) || !rd(f, wd.data(), wd.size()))
      return 2;
    fclose(f);
    std::vector<double> U((size_t)nwin * UPAD * UPAD, NAN);
    for (int w = 0; w < nwin; ++w) {
      WinCtx c{};
      c.H = H.data(); c.Q = nullptr; c.U = U.data() + (size_t)w * UPAD * UPAD;
      c.st = st.data() + 2 * wd[6 * w + 5];
      c.ldh = n; c.ldq = n; c.n = n; c.ktop = ktop; c.kbot = kbot; c.rtop = 0; c.cend = n;
      c.p = wd[6 * w]; c.ws = wd[6 * w + 1]; c.tau0 = wd[6 * w + 2]; c.tau1 = wd[6 * w + 3];
      c.nb = wd[6 * w + 4];
      if (mode == "chase")
        run_workgroup(CHASE_THREADS, w, [c] { chase_window(c); });
      else
        run_workgroup(PB_THREADS, w, [c] { chase_window_t<PB_THREADS>(c, g_cw, g_cr); });
    }
    FILE* g = fopen(argv[3], "wb");
    fwrite(H.data(), sizeof(double), H.size(), g);
    fwrite(U.data(), sizeof(double), U.size(), g);
    fclose(g);
    return 0;
  }
  if (mode == "aed" || mode == "aed4") {
    constexpr int MAXM = SMALL_Z_MAX;
    constexpr int LD = SmallSmem<MAXM>::LD;
    int hdr[4];
    if (!rd(f, hdr, 4)) return 2;
    const int n = hdr[0];
    std::vector<double> H((size_t)n * n), Ut(UPAD * UPAD, NAN), sr(MAXM, NAN), si(MAXM, NAN),
        wr(n, NAN), wi(n, NAN);
    if (!rd(f, H.data(), H.size())) return 2;
    fclose(f);
    static std::vector<double> S(LD * MAXM), Z(LD * MAXM), vv(MAXM), sb(7 * MAXM);
    static std::vector<int> ib(6 * MAXM);
    for (auto* v : {&S, &Z, &vv, &sb})
      for (double& x : *v) x = NAN;
    for (int& x : ib) x = -12345;
    Ctrl ctrl{};
    ctrl.aed_nd = -99;
    ctrl.aed_nu = -99;
    AedTask T{};
    T.H = H.data(); T.ldh = n; T.ktop = hdr[1]; T.kbot = hdr[2]; T.nw = hdr[3];
    T.Ut = Ut.data(); T.ldut = UPAD; T.sr = sr.data(); T.si = si.data();
    const int kwtop = T.kbot - T.nw + 1;
    T.wr = wr.data() + kwtop; T.wi = wi.data() + kwtop;
    T.ctrl = &ctrl; T.itmax = 30;
    if (mode == "aed")
      run_workgroup(64, 0, [T] {
        aed_window<MAXM>(T, S.data(), Z.data(), vv.data(), ib.data(), sb.data());
      });
    else
      run_workgroup(256, 0, [T] {
        aed_window<MAXM, 4>(T, S.data(), Z.data(), vv.data(), ib.data(), sb.data());
      });
    FILE* g = fopen(argv[3], "wb");
    const int o[2] = {ctrl.aed_nd, ctrl.aed_nu};
    fwrite(o, sizeof(int), 2, g);
    fwrite(H.data(), sizeof(double), H.size(), g);
    fwrite(Ut.data(), sizeof(double), Ut.size(), g);
    fwrite(sr.data(), sizeof(double), MAXM, g);
    fwrite(si.data(), sizeof(double), MAXM, g);
    fwrite(wr.data(), sizeof(double), n, g);
    fwrite(wi.data(), sizeof(double), n, g);
    fclose(g);
    return 0;
  }
  if (mode == "split" || mode == "split4") {
    constexpr int MAXM = SMALL_Z_MAX;
    constexpr int LD = SmallSmem<MAXM>::LD;
    int hdr[5];
    if (!rd(f, hdr, 5)) return 2;
    const int n = hdr[0];
    std::vector<double> H((size_t)n * n), Ut(UPAD * UPAD, NAN);
    if (!rd(f, H.data(), H.size())) return 2;
    fclose(f);
    static std::vector<double> S(LD * MAXM), Z(LD * MAXM), vv(MAXM), pb(7 * MAXM);
    static std::vector<int> ib(6 * MAXM);
    for (auto* v : {&S, &Z, &vv, &pb})
      for (double& x : *v) x = NAN;
    for (int& x : ib) x = -12345;
    SplitRes res{-9, -9, -9, -9, NAN, NAN};
    SplitTask T{};
    T.H = H.data(); T.ldh = n; T.a = hdr[1]; T.nw = hdr[2];
    T.above = hdr[3] ? 0 : -1; T.below = hdr[4]; T.itmax = 0;
    T.Ut = Ut.data(); T.ldut = UPAD; T.res = &res;
    if (mode == "split")
      run_workgroup(64, 0, [T] {
        split_window<MAXM>(T, S.data(), Z.data(), vv.data(), ib.data(), pb.data());
      });
    else
      run_workgroup(256, 0, [T] {
        split_window<MAXM, 4>(T, S.data(), Z.data(), vv.data(), ib.data(), pb.data());
      });
    FILE* g = fopen(argv[3], "wb");
    const int o[4] = {res.split, res.nu, res.nf, res.nb};
    fwrite(o, sizeof(int), 4, g);
    fwrite(&res.ftop, sizeof(double), 1, g);
    fwrite(&res.fbot, sizeof(double), 1, g);
    fwrite(H.data(), sizeof(double), H.size(), g);
    fwrite(Ut.data(), sizeof(double), Ut.size(), g);
    fclose(g);
    return 0;
  }
  if (mode == "small" || mode == "small2" || mode == "small4") {
    constexpr int MAXM = SMALL_Z_MAX;
    constexpr int LD = SmallSmem<MAXM>::LD;
    int hdr[1];
    if (!rd(f, hdr, 1)) return 2;
    const int m = hdr[0];
    std::vector<double> A((size_t)m * m), Zo((size_t)m * m, NAN), wr(m, NAN), wi(m, NAN);
    if (!rd(f, A.data(), A.size())) return 2;
    fclose(f);
    static std::vector<double> S(LD * MAXM), Z(LD * MAXM), aux(SMALL_MW_AUX);
    for (auto* v : {&S, &Z, &aux})
      for (double& x : *v) x = NAN;
    int info = -99;
    SmallTask T{};
    T.A = A.data(); T.lda = m; T.m = m; T.Z = Zo.data(); T.ldz = m;
    T.wr = wr.data(); T.wi = wi.data(); T.info = &info; T.itmax = 0;
    if (mode == "small")
      run_workgroup(64, 0, [T] { small_qr<true, MAXM>(T, S.data(), Z.data()); });
    else if (mode == "small2")
      run_workgroup(128, 0, [T] { small_qr<true, MAXM, 2>(T, S.data(), Z.data(), aux.data()); });
    else
      run_workgroup(256, 0, [T] { small_qr<true, MAXM, 4>(T, S.data(), Z.data(), aux.data()); });
    FILE* g = fopen(argv[3], "wb");
    fwrite(&info, sizeof(int), 1, g);
    fwrite(A.data(), sizeof(double), A.size(), g);
    fwrite(Zo.data(), sizeof(double), Zo.size(), g);
    fwrite(wr.data(), sizeof(double), m, g);
    fwrite(wi.data(), sizeof(double), m, g);
    fclose(g);
    return 0;
  }
  if (mode == "eig" || mode == "eig4") {
    // in : int m; double A[m*m] (upper Hessenberg, m <= 128)
    // out: int info; double wr[m], wi[m]
    constexpr int MAXM = SMALL_EIG_MAX;
    constexpr int LD = SmallSmem<MAXM>::LD;
    int hdr[1];
    if (!rd(f, hdr, 1)) return 2;
    const int m = hdr[0];
    std::vector<double> A((size_t)m * m), wr(m, NAN), wi(m, NAN);
    if (!rd(f, A.data(), A.size())) return 2;
    fclose(f);
    static std::vector<double> S(LD * MAXM), aux(SMALL_MW_AUX);
    for (auto* v : {&S, &aux})
      for (double& x : *v) x = NAN;
    int info = -99;
    SmallTask T{};
    T.A = A.data(); T.lda = m; T.m = m;
    T.wr = wr.data(); T.wi = wi.data(); T.info = &info; T.itmax = 0;
    if (mode == "eig")
      run_workgroup(64, 0, [T] { small_qr<false, MAXM>(T, S.data(), nullptr); });
    else
      run_workgroup(256, 0, [T] { small_qr<false, MAXM, 4>(T, S.data(), nullptr, aux.data()); });
    FILE* g = fopen(argv[3], "wb");
    fwrite(&info, sizeof(int), 1, g);
    fwrite(wr.data(), sizeof(double), m, g);
    fwrite(wi.data(), sizeof(double), m, g);
    fclose(g);
    return 0;
  }
  if (mode == "tiny") {
    // in : int n; double A[n*n] (upper Hessenberg, n <= 8)
    // out: int info; double wr[n], wi[n]
    int hdr[1];
    if (!rd(f, hdr, 1)) return 2;
    const int n = hdr[0];
    std::vector<double> A((size_t)n * n), er(8, NAN), ei(8, NAN);
    if (!rd(f, A.data(), A.size())) return 2;
    fclose(f);
    int info = -99;
    run_workgroup(64, 0, [&] {
      const int r = threadIdx.x & 7, c = threadIdx.x >> 3;
      const double h = (r < n && c < n && r <= c + 1) ? A[r + (size_t)c * n] : 0.0;
      const int o = tiny_eigs8(h, n, er.data(), ei.data());
      if (threadIdx.x == 0) info = o;
    });
    FILE* g = fopen(argv[3], "wb");
    fwrite(&info, sizeof(int), 1, g);
    fwrite(er.data(), sizeof(double), n, g);
    fwrite(ei.data(), sizeof(double), n, g);
    fclose(g);
    return 0;
  }
  if (mode == "pbsolve") {
    // in : int n, wantq, ns, nb, nw, nibble, nmin, max_sweeps; double H[n*n]
    // out: int info; double counters[PB_COUNTERS]; double H[n*n], Q[n*n], wr[n], wi[n]
    int hdr[8];
    if (!rd(f, hdr, 8)) return 2;
    const int n = hdr[0];
    std::vector<double> H((size_t)n * n), Q((size_t)n * n, 0.0), wr(n, NAN), wi(n, NAN);
    if (!rd(f, H.data(), H.size())) return 2;
    fclose(f);
    for (int i = 0; i < n; ++i) Q[i + (size_t)i * n] = 1.0;
    static std::vector<double> scratch(sizeof(PScratch) / sizeof(double), NAN);
    std::vector<double> cnt(PB_COUNTERS, NAN);
    int info = -99;
    PJob J{};
    J.H = H.data(); J.Q = hdr[1] ? Q.data() : nullptr; J.wr = wr.data(); J.wi = wi.data();
    J.ldh = n; J.ldq = n; J.n = n;
    J.ns = hdr[2]; J.nb = hdr[3]; J.step = 0; J.nw = hdr[4]; J.nibble = hdr[5]; J.nmin = hdr[6];
    J.exc_period = 6; J.max_sweeps = hdr[7];
    J.info = &info; J.counters = cnt.data();
    PScratch* X = (PScratch*)scratch.data();
    run_workgroup(PB_THREADS, 0, [J, X] { pb_solve(J, g_pb_lds, g_pb_sh, X); });
    FILE* g = fopen(argv[3], "wb");
    fwrite(&info, sizeof(int), 1, g);
    fwrite(cnt.data(), sizeof(double), cnt.size(), g);
    fwrite(H.data(), sizeof(double), H.size(), g);
    fwrite(Q.data(), sizeof(double), Q.size(), g);
    fwrite(wr.data(), sizeof(double), n, g);
    fwrite(wi.data(), sizeof(double), n, g);
    fclose(g);
    return 0;
  }
  return 2;
}
