"""Device source of the LDS kernels run on the CPU (no GPU needed).

``tests/simt/`` compiles the HIP source of the window chase and of the
early-deflation window step with g++ against a small stand-in for the
device API: a workgroup is a set of host threads with real barriers, LDS is
filled with NaN before every workgroup, uninitialised locals are filled with
a NaN pattern (clang), and AddressSanitizer watches every access.  So a read of LDS the kernel never wrote, an out-of-range index or a
missing barrier shows up here, on the CPU.

* window chase: whole sweeps (the sweep planner's windows, time step by time
  step, with the panel products done in numpy) must reproduce the oracle's
  sequential Francis double-shift steps with the same shifts (paper Sec. 3.2:
  the multishift sweep is that sequence, applied window by window);
* the window chase with 256 threads equals the 1024-thread one bit for bit;
* the whole-matrix driver of the persistent batched kernel gives a real
  Schur form with the oracle's spectrum;
* early deflation (paper Sec. 3.2): the returned V is orthogonal and
  V^T W V is the returned window; the undeflated part is Hessenberg, the
  deflated part quasi-triangular with no coupling back; the spike is
  reflected onto one entry; dropped spike entries are below the deflation
  threshold; the eigenvalues reported for both parts are those of their
  diagonal blocks and the window's spectrum is preserved.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1905_04975_amd import inputs, schur
from tests import checks

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
UPAD = 128
ULP = 2.0 ** -52


def _host_compiler():
    """ROCm's clang++ when present: it can fill every uninitialised local with
    a NaN pattern (-ftrivial-auto-var-init=pattern), so a register the kernel
    reads before writing shows up too; else g++."""
    clang = "/opt/rocm/lib/llvm/bin/clang++"
    if os.path.exists(clang):
        return [clang, "-ftrivial-auto-var-init=pattern"]
    if shutil.which("g++"):
        return ["g++"]
    pytest.skip("no host C++ compiler")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("simt") / "simt_kernels")
    cmd = _host_compiler() + ["-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined",
           "-I", os.path.join(HERE, "simt"), "-I", os.path.join(ROOT, "paper_1905_04975_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "simt", "simt_kernels.cpp"),
           "-o", out, "-lpthread"]
    subprocess.check_call(cmd)
    return out


def _call(driver, mode, payload, tmp_path):
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as f:
        for a in payload:
            a.tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([driver, mode, fin, fout], capture_output=True, text=True, timeout=600,
                       env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    return np.fromfile(fout, dtype=np.uint8).tobytes()


def _chase_step(driver, tmp_path, H, ktop, kbot, st, wins):
    n = H.shape[0]
    raw = _call(driver, "chase", [np.array([n, ktop, kbot, len(st), len(wins)], dtype=np.int32),
                                  np.asfortranarray(H).ravel(order="F"),
                                  np.asarray(st, dtype=np.float64),
                                  np.array([v for w in wins for v in w], dtype=np.int32)], tmp_path)
    x = np.frombuffer(raw, dtype=np.float64)
    H2 = x[:n * n].reshape(n, n, order="F").copy()
    Us = x[n * n:].reshape(len(wins), UPAD, UPAD)   # [w, i, j] = U(i, j) (slot holds U^T)
    return H2, Us


@pytest.mark.parametrize("n,ktop,kbot,npair,nb,seed", [
    (160, 0, 159, 1, 1, 3), (220, 0, 219, 6, 3, 4), (300, 10, 280, 8, 8, 5),
    (200, 0, 199, 16, 16, 6), (190, 0, 189, 20, 20, 7)])
def test_chase_sweep_equals_sequential_double_shift_steps(driver, tmp_path, n, ktop, kbot, npair,
                                                          nb, seed):
    H0 = inputs.hessenberg_normal(n, seed)
    if ktop > 0:
        H0[ktop, ktop - 1] = 0.0
    if kbot < n - 1:
        H0[kbot + 1, kbot] = 0.0
    rng = np.random.default_rng(seed)
    shifts = []
    for _ in range(npair):
        a, b = rng.uniform(-1, 1, 2)
        shifts.append((2 * a, a * a + b * b))
    st = [v for s in shifts for v in s]
    plan = schur.plan_sweep(ktop, kbot, npair, nb, 0)
    H = H0.copy()
    for t in sorted({r[0] for r in plan}):
        wins = [(p, ws, t0, t1, b, g) for (tt, g, p, ws, t0, t1, b) in plan if tt == t]
        H2, Us = _chase_step(driver, tmp_path, H, ktop, kbot, st, wins)
        assert not np.isnan(H2).any()
        for (p, ws, t0, t1, b, g), U in zip(wins, Us):
            assert not np.isnan(U).any(), "unwritten LDS reached the U slot"
            assert not U[ws:, :].any() and not U[:, ws:].any(), "slot not zero padded"
            U = U[:ws, :ws]
            assert np.linalg.norm(U.T @ U - np.eye(ws)) <= 1e-13 * ws
            H2[p:p + ws, p + ws:] = U.T @ H2[p:p + ws, p + ws:]
            H2[:p, p:p + ws] = H2[:p, p:p + ws] @ U
        H = H2
    Hs = np.asfortranarray(H0.copy())
    Qs = np.asfortranarray(np.eye(n))
    for (s, t) in shifts:
        oracle.francis_step_inplace(Hs, Qs, ktop, kbot, s, t)
    assert np.abs(np.abs(H) - np.abs(Hs)).max() <= 1e-11 * np.linalg.norm(H0)
    assert not np.tril(H, -2).any()


def _aed(driver, tmp_path, H, ktop, kbot, nw, waves=1):
    n = H.shape[0]
    raw = _call(driver, "aed" if waves == 1 else "aed4", [np.array([n, ktop, kbot, nw], dtype=np.int32),
                                np.asfortranarray(H).ravel(order="F")], tmp_path)
    nd, nu = np.frombuffer(raw[:8], dtype=np.int32)
    x = np.frombuffer(raw[8:], dtype=np.float64)
    H2 = x[:n * n].reshape(n, n, order="F"); x = x[n * n:]
    U = x[:UPAD * UPAD].reshape(UPAD, UPAD); x = x[UPAD * UPAD:]   # [i, j] = V(i, j)
    sr, si = x[:96], x[96:192]; x = x[192:]
    return int(nd), int(nu), H2, U, sr, si, x[:n], x[n:2 * n]


def _block_eigs(T):
    """Eigenvalues read from the diagonal blocks of a quasi-triangular T."""
    m = T.shape[0]
    out = np.zeros(m, dtype=complex)
    k = 0
    while k < m:
        if k + 1 < m and T[k + 1, k] != 0.0:
            out[k:k + 2] = np.linalg.eigvals(T[k:k + 2, k:k + 2])
            k += 2
        else:
            out[k] = T[k, k]
            k += 1
    return out


def _converging(n, seed, steps):
    """A random Hessenberg matrix after a few double-shift steps (oracle),
    so that its bottom is partly converged."""
    H = np.asfortranarray(inputs.hessenberg_normal(n, seed))
    Q = np.asfortranarray(np.eye(n))
    for _ in range(steps):
        a, b, c, d = H[n - 2, n - 2], H[n - 2, n - 1], H[n - 1, n - 2], H[n - 1, n - 1]
        oracle.francis_step_inplace(H, Q, 0, n - 1, a + d, a * d - b * c)
    return np.array(H)


def _graded(n, seed, m, lo):
    H = inputs.hessenberg_normal(n, seed)
    sub = np.ones(n - 1)
    sub[-m:] = np.logspace(-2, lo, m)
    H[np.arange(1, n), np.arange(n - 1)] *= sub
    return H


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("case", ["raw400", "conv256", "conv200", "graded", "all", "top"])
def test_aed_window(driver, tmp_path, case, waves):
    if case == "raw400":
        H, ktop, nw = inputs.hessenberg_normal(400, 5), 0, 48
    elif case == "conv256":
        H, ktop, nw = _converging(256, 1, 4), 0, 16
    elif case == "conv200":
        H, ktop, nw = _converging(200, 11, 6), 0, 24
    elif case == "graded":
        H, ktop, nw = _graded(300, 8, 120, -13), 0, 96
    elif case == "all":
        H, ktop, nw = _graded(160, 9, 100, -40), 0, 40
    else:   # window reaching up to the active block top (no spike)
        H, ktop, nw = _graded(120, 10, 50, -6), 40, 80
        H[40, 39] = 0.0
    n = H.shape[0]
    kbot = n - 1
    kw = kbot - nw + 1
    nd, nu, H2, Vfull, sr, si, wr, wi = _aed(driver, tmp_path, H, ktop, kbot, nw, waves)
    assert nd + nu == nw and nd >= 0
    W = H[kw:, kw:]
    if nd == 0:
        assert np.array_equal(H2, H), "nothing deflated: H must be unchanged"
        return
    assert not np.isnan(H2).any() and not np.isnan(Vfull).any()
    assert not Vfull[nw:, :].any() and not Vfull[:, nw:].any()
    V = Vfull[:nw, :nw]
    T = H2[kw:, kw:]
    assert np.linalg.norm(V.T @ V - np.eye(nw)) <= 1e-13 * nw
    assert np.linalg.norm(V.T @ W @ V - T) <= 1e-14 * nw * np.linalg.norm(W)
    assert not np.tril(T[:nu, :nu], -2).any()
    assert not np.tril(T[nu:, nu:], -2).any()
    assert not T[nu:, :nu].any()
    # spike: V^T s e1 = (beta, 0, ...) on the undeflated part, negligible below
    s = H[kw, kw - 1] if kw > ktop else 0.0
    spike = s * V[0, :]
    beta = H2[kw, kw - 1] if kw > ktop else 0.0
    if nu:
        assert abs(spike[0] - beta) <= 1e-13 * abs(s)
        assert np.linalg.norm(spike[1:nu]) <= 1e-13 * abs(s)
    teig = _block_eigs(T[nu:, nu:])
    thr = np.maximum(ULP * np.abs(teig), 1e-290)
    # each deflated block's spike entries are below ulp times its size
    k = 0
    Td = T[nu:, nu:]
    while k < nd:
        two = k + 1 < nd and Td[k + 1, k] != 0.0
        size = 2 if two else 1
        blk = Td[k:k + size, k:k + size]
        foo = abs(blk[-1, -1]) + (np.sqrt(abs(blk[1, 0])) * np.sqrt(abs(blk[0, 1])) if two else 0)
        assert np.abs(spike[nu + k:nu + k + size]).max() <= max(1e-290, ULP * (foo or abs(s))) * 1.0001
        k += size
    # reported eigenvalues: deflated part final (wr, wi), undeflated shifts (sr, si)
    got_d = wr[kw + nu:] + 1j * wi[kw + nu:]
    assert np.allclose(got_d, teig, rtol=1e-14, atol=1e-300)
    # the window's spectrum is preserved
    ev0 = np.linalg.eigvals(W)
    ev1 = np.concatenate([np.linalg.eigvals(T[:nu, :nu]) if nu else [], teig])
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(ev0[:, None] - ev1[None, :])
    r, c = linear_sum_assignment(cost)
    assert cost[r, c].max() <= 1e-9 * np.linalg.norm(W)
    if case == "graded":
        assert nd >= 40
    if case in ("all", "top"):
        assert nd == nw and H2[kw, kw - 1] == 0.0


@pytest.mark.parametrize("waves", [1, 2, 4])
@pytest.mark.parametrize("m,seed,kind", [(5, 1, "normal"), (33, 2, "normal"), (64, 3, "normal"),
                                         (96, 4, "normal"), (40, 5, "prescribed"),
                                         (60, 6, "graded"), (65, 7, "normal"),
                                         (80, 8, "prescribed"), (90, 9, "graded")])
def test_small_block_solver(driver, tmp_path, m, seed, kind, waves):
    """The small-block Francis solver with Z, on one wavefront (single
    double-shift bulges) or on two or four (chains of bulges, one per
    wavefront): a standardised real Schur form, H = Z S Z^T, and the
    eigenvalues of the oracle."""
    from tests import checks

    if kind == "prescribed":
        A, exact = inputs.prescribed(m, seed)
    elif kind == "graded":
        A = _graded(m, seed, m // 2, -10)
    else:
        A = inputs.hessenberg_normal(m, seed)
    mode = {1: "small", 2: "small2", 4: "small4"}[waves]
    raw = _call(driver, mode, [np.array([m], dtype=np.int32),
                                  np.asfortranarray(A).ravel(order="F")], tmp_path)
    info = int(np.frombuffer(raw[:4], dtype=np.int32)[0])
    x = np.frombuffer(raw[4:], dtype=np.float64)
    S = x[:m * m].reshape(m, m, order="F"); x = x[m * m:]
    Z = x[:m * m].reshape(m, m, order="F"); x = x[m * m:]
    wr, wi = x[:m], x[m:2 * m]
    assert info == 0
    assert not np.isnan(S).any() and not np.isnan(Z).any()
    assert checks.structure_errors(S, wr, wi) == []
    assert checks.residual(A, Z, S) <= 1e-14 * m
    assert checks.orthogonality(Z) <= 1e-14 * m
    _, _, owr, owi, oinfo, _ = oracle.schur(A)
    assert oinfo == 0
    lam, lam_o = wr + 1j * wi, owr + 1j * owi
    w, kappa = checks.eig_condition(np.triu(A, -1))
    k = kappa[np.argmin(np.abs(lam_o[:, None] - w[None, :]), axis=1)]
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(lam[:, None] - lam_o[None, :])
    r, c = linear_sum_assignment(cost)
    assert np.all(cost[r, c] <= checks.kappa_tolerance(A, lam_o[c], k[c], factor=200.0))


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("m,seed,kind", [(7, 1, "normal"), (40, 2, "normal"), (64, 3, "prescribed"),
                                         (100, 4, "normal"), (128, 5, "normal"),
                                         (128, 6, "prescribed"), (90, 7, "graded")])
def test_eigenvalue_solver(driver, tmp_path, m, seed, kind, waves):
    """The eigenvalues-only solver of a sweep's shift problem (orders up to
    128), one wavefront or bulge chains on four: every eigenvalue within a
    condition-weighted bound of numpy's (or of the known spectrum)."""
    from tests import checks

    exact = None
    if kind == "prescribed":
        A, exact = inputs.prescribed(m, seed)
    elif kind == "graded":
        A = _graded(m, seed, m // 2, -10)
    else:
        A = inputs.hessenberg_normal(m, seed)
    raw = _call(driver, "eig" if waves == 1 else "eig4",
                [np.array([m], dtype=np.int32), np.asfortranarray(A).ravel(order="F")], tmp_path)
    info = int(np.frombuffer(raw[:4], dtype=np.int32)[0])
    x = np.frombuffer(raw[4:], dtype=np.float64)
    lam = x[:m] + 1j * x[m:2 * m]
    assert info == 0 and not np.isnan(lam).any()
    ref = np.linalg.eigvals(A) if exact is None else np.asarray(exact)
    w, kappa = checks.eig_condition(np.triu(A, -1))
    kap = kappa[np.argmin(np.abs(ref[:, None] - w[None, :]), axis=1)]
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(lam[:, None] - ref[None, :])
    r, c = linear_sum_assignment(cost)
    assert np.all(cost[r, c] <= checks.kappa_tolerance(A, ref[c], kap[c], factor=200.0))


@pytest.mark.parametrize("n,seed,kind", [(1, 1, "normal"), (2, 2, "normal"), (3, 3, "normal"),
                                         (4, 4, "normal"), (5, 5, "prescribed"), (8, 6, "normal"),
                                         (8, 7, "prescribed"), (8, 8, "graded"), (6, 9, "zero_sub"),
                                         (8, 10, "companion")])
def test_tiny_eigenvalue_iteration(driver, tmp_path, n, seed, kind):
    """The register-resident eigenvalue iteration of blocks of order <= 8
    (the shifts of a bulge chain): every eigenvalue within a condition-
    weighted bound of numpy's, on random, prescribed-spectrum, graded,
    already split and companion (known roots) inputs."""
    from tests import checks

    exact = None
    if kind == "prescribed":
        A, exact = inputs.prescribed(n, seed)
    elif kind == "graded":
        A = _graded(n, seed, n // 2, -10)
    elif kind == "companion":
        roots = np.array([-3.0, -1.5, -0.5, 0.25, 1.0, 2.0, 2.5, 4.0])[:n]
        c = np.poly(roots)
        A = np.zeros((n, n))
        A[0, :] = -c[1:]
        A[np.arange(1, n), np.arange(n - 1)] = 1.0
        exact = roots.astype(complex)
    else:
        A = inputs.hessenberg_normal(n, seed)
        if kind == "zero_sub":
            A[3, 2] = 0.0
    raw = _call(driver, "tiny", [np.array([n], dtype=np.int32),
                                 np.asfortranarray(A).ravel(order="F")], tmp_path)
    info = int(np.frombuffer(raw[:4], dtype=np.int32)[0])
    x = np.frombuffer(raw[4:], dtype=np.float64)
    lam = x[:n] + 1j * x[n:2 * n]
    assert info == 0 and not np.isnan(lam).any()
    # conjugate pairs come as (re, +im), (re, -im)
    k = 0
    while k < n:
        if lam[k].imag != 0.0:
            assert lam[k].imag > 0 and lam[k + 1] == np.conj(lam[k])
            k += 2
        else:
            k += 1
    ref = np.linalg.eigvals(A) if exact is None else np.asarray(exact)
    w, kappa = checks.eig_condition(np.triu(A, -1))
    kap = kappa[np.argmin(np.abs(ref[:, None] - w[None, :]), axis=1)]
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(lam[:, None] - ref[None, :])
    r, c = linear_sum_assignment(cost)
    assert np.all(cost[r, c] <= checks.kappa_tolerance(A, ref[c], kap[c], factor=200.0))


def _split(driver, tmp_path, H, a, nw, above, below, waves=1):
    n = H.shape[0]
    raw = _call(driver, "split" if waves == 1 else "split4", [np.array([n, a, nw, int(above), int(below)], dtype=np.int32),
                                  np.asfortranarray(H).ravel(order="F")], tmp_path)
    split, nu, nf, nb = (int(v) for v in np.frombuffer(raw[:16], dtype=np.int32))
    ftop, fbot = np.frombuffer(raw[16:32], dtype=np.float64)
    x = np.frombuffer(raw[32:], dtype=np.float64)
    H2 = x[:n * n].reshape(n, n, order="F")
    U = x[n * n:n * n + UPAD * UPAD].reshape(UPAD, UPAD)   # [i, j] = V(i, j)
    return split, nu, nf, nb, float(ftop), float(fbot), H2, U


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("case", ["mid_split", "mid_nosplit", "bottom", "top", "whole"])
def test_split_window(driver, tmp_path, case, waves):
    """One window of a parallel early-deflation pass (paper Sec. 3.2, AED
    applied to windows inside the matrix): when it splits, V is orthogonal,
    V^T W V is the returned window with zero subdiagonal entries around the
    free part, the couplings above and below are reflected onto one entry
    each, every dropped coupling entry is below the deflation threshold, and
    the window's spectrum is preserved; otherwise H is untouched."""
    above = below = True
    if case == "mid_split":
        H, a, nw = inputs.hessenberg_normal(700, 3), 124, 96
    elif case == "mid_nosplit":
        H, a, nw = inputs.hessenberg_normal(700, 3), 100, 96
    elif case == "bottom":
        H, a, nw, below = inputs.hessenberg_normal(300, 4), 204, 96, False
    elif case == "top":
        H, a, nw, above = inputs.hessenberg_normal(300, 5), 0, 96, False
    else:
        H, a, nw, above, below = inputs.hessenberg_normal(80, 6), 0, 80, False, False
    n = H.shape[0]
    split, nu, nf, nb, ftop, fbot, H2, Vfull = _split(driver, tmp_path, H, a, nw, above, below,
                                                      waves)
    if case == "mid_nosplit":
        assert split == 0
    else:
        assert split == 1
    if not split:
        assert np.array_equal(H2, H), "a window that does not split leaves H unchanged"
        return
    assert nu + nf + nb == nw and min(nu, nf, nb) >= 0
    if not above:
        assert nu == 0
    if not below:
        assert nb == 0
    if case == "whole":
        assert nf == nw
    bs = nw - nb
    outside = np.ones((n, n), dtype=bool)
    outside[a:a + nw, a:a + nw] = False
    assert np.array_equal(H2[outside], H[outside]), "only the window itself is written"
    assert not np.isnan(Vfull).any()
    assert not Vfull[nw:, :].any() and not Vfull[:, nw:].any()
    V = Vfull[:nw, :nw]
    W = H[a:a + nw, a:a + nw]
    T = np.triu(H2[a:a + nw, a:a + nw], -1)
    assert np.linalg.norm(V.T @ V - np.eye(nw)) <= 1e-13 * nw
    assert np.linalg.norm(V.T @ W @ V - T) <= 1e-14 * nw * np.linalg.norm(W)
    # zero subdiagonal entries around the free part, free part quasi-triangular
    if nu and nu < nw:
        assert T[nu, nu - 1] == 0.0
    if nb and bs > 0:
        assert T[bs, bs - 1] == 0.0
    sub = np.diag(T, -1)[nu:bs - 1] if bs - nu >= 2 else np.zeros(0)
    assert not (np.logical_and(sub[:-1] != 0, sub[1:] != 0)).any()
    # couplings: reflected onto one entry, the dropped ones below the threshold
    st = H[a, a - 1] if above else 0.0
    sb = H[a + nw, a + nw - 1] if below else 0.0

    def blocks(lo, hi):
        k = lo
        while k < hi:
            two = k + 1 < hi and T[k + 1, k] != 0.0
            yield k, 2 if two else 1
            k += 2 if two else 1

    def dropped_ok(vrow, s, lo, hi):
        for k, size in blocks(lo, hi):
            blk = T[k:k + size, k:k + size]
            foo = (abs(np.linalg.eigvals(blk)).max() if size == 2 else abs(blk[0, 0])) or abs(s)
            assert np.abs(s * vrow[k:k + size]).max() <= max(1e-290, ULP * foo) * 4 + 1e-15 * abs(s) * 0

    if nu:
        assert abs(V[0, 0] - ftop) <= 1e-13
        assert np.linalg.norm(V[0, 1:nu]) <= 1e-13
    if above:
        dropped_ok(V[0, :], st, nu, nw)
    if nb:
        assert abs(V[nw - 1, nw - 1] - fbot) <= 1e-13
        assert np.linalg.norm(V[nw - 1, bs:nw - 1]) <= 1e-13
    if below:
        dropped_ok(V[nw - 1, :], sb, 0, bs)
    # the upward- and downward-coupled parts are Hessenberg (stored that way)
    # and the window's spectrum is preserved
    ev0 = np.linalg.eigvals(W)
    ev1 = np.linalg.eigvals(T)
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(ev0[:, None] - ev1[None, :])
    r, c = linear_sum_assignment(cost)
    assert cost[r, c].max() <= 1e-8 * np.linalg.norm(W)


@pytest.mark.parametrize("n,ktop,kbot,npair,nb,seed", [
    (160, 0, 159, 1, 1, 3), (220, 0, 219, 6, 3, 4), (300, 10, 280, 8, 8, 5), (150, 0, 149, 5, 5, 8)])
def test_chase_256_threads_equals_1024(driver, tmp_path, n, ktop, kbot, npair, nb, seed):
    """The window chase with 256 threads (the persistent batched kernel's
    layout: 32 lanes per bulge, two lanes per row of U) does exactly the
    arithmetic of the 1024-thread chase: the same H and U bit for bit."""
    H0 = inputs.hessenberg_normal(n, seed)
    rng = np.random.default_rng(seed)
    st = []
    for _ in range(npair):
        a, b = rng.uniform(-1, 1, 2)
        st += [2 * a, a * a + b * b]
    plan = schur.plan_sweep(ktop, kbot, npair, nb, 0)
    t0 = min(r[0] for r in plan)
    wins = [(p, ws, a0, a1, b, g) for (tt, g, p, ws, a0, a1, b) in plan if tt == t0]
    payload = [np.array([n, ktop, kbot, len(st), len(wins)], dtype=np.int32),
               np.asfortranarray(H0).ravel(order="F"), np.asarray(st, dtype=np.float64),
               np.array([v for w in wins for v in w], dtype=np.int32)]
    a = _call(driver, "chase", payload, tmp_path)
    b = _call(driver, "chase256", payload, tmp_path)
    assert a == b


def _pbsolve(driver, tmp_path, H, wantq=True, ns=16, nb=8, nw=24, nibble=14, nmin=96,
             max_sweeps=1000):
    n = H.shape[0]
    raw = _call(driver, "pbsolve",
                [np.array([n, int(wantq), ns, nb, nw, nibble, nmin, max_sweeps], dtype=np.int32),
                 np.asfortranarray(H).ravel(order="F")], tmp_path)
    info = int(np.frombuffer(raw[:4], dtype=np.int32)[0])
    x = np.frombuffer(raw[4:], dtype=np.float64)
    cnt, x = x[:11], x[11:]
    S = x[:n * n].reshape(n, n, order="F")
    Q = x[n * n:2 * n * n].reshape(n, n, order="F")
    w = x[2 * n * n:2 * n * n + n] + 1j * x[2 * n * n + n:]
    return info, cnt, S, Q, w


@pytest.mark.parametrize("n,ns,nb,nw,kind", [
    (60, 16, 8, 24, "normal"),      # whole matrix in the small solver
    (97, 16, 4, 24, "normal"),      # one sweep level above it
    (150, 16, 8, 24, "normal"),
    (180, 32, 8, 32, "prescribed"),  # two bulge groups per sweep
    (130, 12, 6, 0, "normal"),      # no early deflation: trailing-block shifts
])
def test_persistent_driver(driver, tmp_path, n, ns, nb, nw, kind):
    """The device-side driver of the persistent batched kernel (one
    workgroup, the whole solve: deflation scans, small-block solver, early
    deflation, shifts, bulge groups chased window by window, MFMA panel
    products) run on the CPU: a real Schur form with Q (backward error and
    orthogonality, standardised blocks, eigenvalues of the blocks), the
    oracle's spectrum (exact spectrum on the prescribed input), and the same
    S without Q."""
    if kind == "normal":
        H = inputs.hessenberg_normal(n, 300 + n)
        exact = None
    else:
        H, exact = inputs.prescribed(n, 300 + n)
    info, cnt, S, Q, w = _pbsolve(driver, tmp_path, H, True, ns, nb, nw)
    assert info == 0
    assert not np.isnan(S).any() and not np.isnan(Q).any()
    assert checks.structure_errors(S, w.real, w.imag) == []
    assert checks.residual(H, Q, S) <= 1e-13
    assert checks.orthogonality(Q) <= 1e-13
    if n > 96:
        assert cnt[0] > 0 and cnt[1] > 0   # sweeps, windows
    _, _, wr, wi, oinfo, _ = oracle.schur(H)
    assert oinfo == 0
    if exact is not None:
        assert np.all(checks.match_eigs(w, exact) <= checks.eig_rel_tol(exact, H, 1e-9))
    else:
        wref, kappa = checks.eig_condition(H)
        from scipy.optimize import linear_sum_assignment
        cost = np.abs((wr + 1j * wi)[:, None] - w[None, :])
        r, c = linear_sum_assignment(cost)
        ko = kappa[np.argmin(np.abs((wr + 1j * wi)[r][:, None] - wref[None, :]), axis=1)]
        assert np.all(cost[r, c] <= checks.kappa_tolerance(H, wref, ko, factor=200.0))
    info0, _, S0, _, w0 = _pbsolve(driver, tmp_path, H, False, ns, nb, nw)
    assert info0 == 0 and np.array_equal(S0, S) and np.array_equal(w0, w)


def test_persistent_driver_reports_non_finite_input(driver, tmp_path):
    H = inputs.hessenberg_normal(40, 5)
    H[3, 10] = np.nan
    info, cnt, S, Q, w = _pbsolve(driver, tmp_path, H)
    assert info == -2
