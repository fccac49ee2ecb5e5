"""GPU parity of the eigenvector step (paper Sec. 2, Eqs. (5) and (6))
against the oracle (MI355X only).

Both sides fix each eigenvector by the same convention (LAPACK's: unit entry
at the eigenvalue's row, the complex pair convention of the standardised
block, largest |Re| + |Im| = 1), so the vectors are compared element by
element; beside that every vector must satisfy the definition
(S y = lambda y, or A x = lambda x after the backtransform) to rounding
level.  Tile rows are 64 rows, moved where a 2x2 block would be split, so
the orders include 63..66 and blocks across tile boundaries.  Two
overflow cases need the protection (plain back substitution overflows).
"""
import numpy as np
import pytest

import oracle
from paper_1905_04975_amd import inputs
from tests.test_oracle_evec import _overflow_cases

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _dev(A):
    import torch

    return torch.from_numpy(np.asfortranarray(A)).to("cuda:0").t().contiguous().t()


def _gpu(schur, S, Q=None):
    import torch

    h = schur.Handle(0)
    X, rc = schur.eigenvectors(_dev(S), Q=None if Q is None else _dev(Q), handle=h)
    torch.cuda.synchronize()
    h.close()
    return X.cpu().numpy(), rc


def _residual(M, S, X):
    """max over eigenvectors of ||M v - lambda v|| / (||M|| ||v||)."""
    lam, V = oracle.complex_vectors(S, X)
    R = M @ V - V * lam[None, :]
    return (np.linalg.norm(R, axis=0) / (np.linalg.norm(M) * np.linalg.norm(V, axis=0))).max()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 66, 67, 129, 300, 700])
def test_eigenvectors_vs_oracle(gpu_lib, n):
    print("case evec n=%d" % n, flush=True)
    S = inputs.schur_form(n, 500 + n)
    X, rc = _gpu(gpu_lib, S)
    assert rc == 0
    Xo = oracle.eigenvectors(S)
    assert np.all(np.isfinite(X))
    assert _residual(S, S, X) <= 100 * max(n, 1) * U
    assert np.abs(X - Xo).max() <= 1e-10, np.abs(X - Xo).max()


def test_eigenvectors_of_computed_schur_forms(gpu_lib):
    """S and Q from the oracle's Schur reduction of random Hessenberg
    matrices (non-normal, blocks wherever they fall), with and without the
    backtransform."""
    for n, seed in ((97, 511), (260, 512)):
        print("case evec schur n=%d" % n, flush=True)
        H = inputs.hessenberg_normal(n, seed)
        S, Q, _, _, info, _ = oracle.schur(H)
        assert info == 0
        X, rc = _gpu(gpu_lib, S)
        XA, rcA = _gpu(gpu_lib, S, Q)
        assert rc == 0 and rcA == 0
        assert _residual(S, S, X) <= 100 * n * U
        assert _residual(H, S, XA) <= 1000 * n * U
        Xo = oracle.eigenvectors(S)
        XAo = oracle.eigenvectors(S, Q)
        # random Hessenberg eigenvectors can be ill-conditioned: the bound
        # follows the size of the oracle's own residual-scaled differences
        assert np.abs(X - Xo).max() <= 1e-7
        assert np.abs(XA - XAo).max() <= 1e-7


@pytest.mark.parametrize("case", [0, 1])
def test_eigenvectors_overflow_protection(gpu_lib, case):
    S = _overflow_cases()[case]
    X, rc = _gpu(gpu_lib, S)
    assert rc == 0
    assert np.all(np.isfinite(X))
    assert _residual(S, S, X) <= 1e-12
    Xo = oracle.eigenvectors(S)
    assert np.abs(X - Xo).max() <= 1e-10


def test_eigenvector_argument_errors(gpu_lib):
    import torch

    h = gpu_lib.Handle(0)
    A = torch.zeros(4, 4, dtype=torch.float64, device="cuda:0")
    p = A.data_ptr()
    assert h.eigenvectors_async(None, -1, p, 4, None, 1, p, 4) == -1
    assert h.eigenvectors_async(None, 4, None, 4, None, 1, p, 4) == -2
    assert h.eigenvectors_async(None, 4, p, 3, None, 1, p, 4) == -3
    assert h.eigenvectors_async(None, 4, p, 4, p, 2, p, 4) == -5
    assert h.eigenvectors_async(None, 4, p, 4, None, 1, None, 4) == -6
    assert h.eigenvectors_async(None, 4, p, 4, None, 1, p, 3) == -7
    assert h.eigenvectors_async(None, 0, None, 1, None, 1, None, 1) == 0
    h.close()


def test_pipeline_dense_to_eigenvectors(gpu_lib):
    """A dense -> Hessenberg -> Schur -> eigenvectors of A, all on the GPU:
    A x = lambda x for every returned vector (paper Sec. 2, Eqs. (3)-(6))."""
    import torch

    n = 500
    A = np.random.Generator(np.random.PCG64(513)).uniform(-1.0, 1.0, size=(n, n))
    dev = torch.device("cuda:0")
    h = gpu_lib.Handle(0)
    Ad = _dev(A)
    Q = _dev(np.eye(n))
    H, Q, rc = gpu_lib.hessenberg(Ad, Q=Q, handle=h)
    assert rc == 0
    S, Q, w, info = gpu_lib.reduce(H, Q=Q, handle=h)
    assert info == 0
    X, rc = gpu_lib.eigenvectors(S, Q=Q, handle=h)
    torch.cuda.synchronize(dev)
    h.close()
    assert rc == 0
    S = S.cpu().numpy()
    X = X.cpu().numpy()
    assert _residual(A, S, X) <= 1000 * n * U


def test_eigenvectors_full_size(gpu_lib):
    """n = 16384: eigenvectors of a standardised Schur form backtransformed
    with a dense orthogonal Q (one Householder reflector); checked by the
    definition A x = lambda x (A = Q S Q^T, torch FP64 products) and, on a
    sample of columns, against the oracle's vectors of S."""
    import torch

    n = 16384
    print("case evec full n=%d" % n, flush=True)
    dev = torch.device("cuda:0")
    S_np = inputs.schur_form(n, 16384)
    S = _dev(S_np)
    g = torch.Generator(dev).manual_seed(7)
    v = torch.randn(n, 1, dtype=torch.float64, device=dev, generator=g)
    Q = torch.eye(n, dtype=torch.float64, device=dev) - (2.0 / (v.t() @ v)) * (v @ v.t())
    Q = Q.t().contiguous().t()
    h = gpu_lib.Handle(0, flags=gpu_lib.FLAG_TIME_KERNELS)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    X, rc = gpu_lib.eigenvectors(S, Q=Q, handle=h)
    e1.record()
    torch.cuda.synchronize()
    st = h.stats()
    h.close()
    print("eigenvectors n=%d: %.3f s (tile solves %.3f s, updates %.3f s, backtransform %.3f s)"
          % (n, e0.elapsed_time(e1) / 1e3, st["ev_solve_ms"] / 1e3, st["ev_gemm_ms"] / 1e3,
             st["ev_back_ms"] / 1e3), flush=True)
    assert rc == 0
    assert torch.isfinite(X).all().item()
    # A X = X L, L block diagonal with [[a, b], [-b, a]] for the pairs
    sub = np.diag(S_np, -1)
    L = np.diag(np.diag(S_np)).astype(np.float64)
    for k in np.nonzero(sub)[0]:
        wi = np.sqrt(abs(S_np[k, k + 1])) * np.sqrt(abs(S_np[k + 1, k]))
        L[k, k + 1], L[k + 1, k] = wi, -wi
    Ld = torch.from_numpy(L).to(dev)
    A = Q @ (S @ Q.t())
    R = A @ X - X @ Ld
    res = (torch.linalg.norm(R, dim=0) / torch.linalg.norm(X, dim=0)).max().item() \
        / torch.linalg.norm(A).item()
    del R, A
    print("max relative residual %.3e" % res, flush=True)
    assert res <= 1e-13
    # a sample of eigenvectors of S against the oracle (columns 0..199 need
    # only the leading 200 x 200 block of S)
    m = 200
    if sub[m - 1] != 0.0:
        m += 1
    Y, rc = gpu_lib.eigenvectors(S)
    assert rc == 0
    Yo = oracle.eigenvectors(S_np[:m, :m])
    Ys = Y[:m, :m].cpu().numpy()
    assert np.abs(Ys - Yo).max() <= 1e-10
