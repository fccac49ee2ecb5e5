"""GPU parity of the Hessenberg reduction A = Q1 H Q1^T (paper Sec. 2,
Eq. (3)) against the oracle (MI355X only).

With Q1 e_1 = e_1 the Hessenberg form of a matrix with nonzero subdiagonal
is unique up to the signs of Q1's columns (implicit-Q theorem), and both
sides pick the sign -sign(x_1) ||x|| for each new subdiagonal entry, so H and
Q1 are compared with the oracle element by element (after matching column
signs, which must all agree).  Sizes span one panel (32 columns), several
panels and ragged tails.  At n = 16384 (the order of the Schur benchmark,
the paper's dense U(-1,1) test matrices of Sec. 5) the oracle is out of
reach: there the result is checked by properties that hold at any size
(backward error and orthogonality with torch FP64 products, exact zeros,
Q e_1 = e_1) and by the Arnoldi process, which fixes the first columns of Q1
and H from A and e_1 alone.
"""
import numpy as np
import pytest

import oracle
from paper_1905_04975_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _dense(n, seed):
    return np.random.Generator(np.random.PCG64(seed)).uniform(-1.0, 1.0, size=(n, n))


def _gpu(schur, A_np, want_q=True, Q_np=None):
    import torch

    dev = torch.device("cuda:0")
    n = A_np.shape[0]
    A = torch.from_numpy(np.asfortranarray(A_np)).to(dev).t().contiguous().t()
    Q = None
    if want_q:
        Qn = np.eye(n) if Q_np is None else Q_np
        Q = torch.from_numpy(np.asfortranarray(Qn)).to(dev).t().contiguous().t()
    h = schur.Handle(0)
    H, Qo, rc = schur.hessenberg(A, Q=Q, want_q=want_q, handle=h)
    torch.cuda.synchronize()
    h.close()
    return H.cpu().numpy(), (Qo.cpu().numpy() if want_q else None), rc


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 31, 32, 33, 34, 64, 100, 257, 700])
def test_hessenberg_vs_oracle(gpu_lib, n):
    print("case hess n=%d" % n, flush=True)
    A = _dense(n, 300 + n)
    H, Q, rc = _gpu(gpu_lib, A)
    assert rc == 0
    Ho, Qo = oracle.hessenberg(A)
    nrm = max(np.linalg.norm(A), 1e-300)
    if n > 2:
        assert np.count_nonzero(np.tril(H, -2)) == 0
    # column signs: both sides use -sign(x_1) ||x||
    d = np.sign(np.sum(Q * Qo, axis=0))
    d[d == 0] = 1.0
    assert np.all(d == 1.0), np.nonzero(d != 1.0)
    assert np.abs(H - Ho).max() <= 1e-12 * nrm, np.abs(H - Ho).max()
    assert np.abs(Q - Qo).max() <= 1e-12
    assert np.linalg.norm(A - Q @ H @ Q.T) <= 50 * max(n, 1) * U * nrm
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 50 * max(n, 1) * U
    if n:
        assert Q[0, 0] == 1.0 and not np.any(Q[0, 1:]) and not np.any(Q[1:, 0])


def test_hessenberg_accumulates_and_without_q(gpu_lib):
    n = 150
    A = _dense(n, 401)
    Qin = inputs.haar_orthogonal(n, np.random.Generator(np.random.PCG64(402)))
    H1, Q1, rc1 = _gpu(gpu_lib, A)
    H2, Q2, rc2 = _gpu(gpu_lib, A, Q_np=Qin)
    H3, _, rc3 = _gpu(gpu_lib, A, want_q=False)
    assert rc1 == rc2 == rc3 == 0
    assert np.array_equal(H1, H2) and np.array_equal(H1, H3)
    assert np.abs(Q2 - Qin @ Q1).max() <= 1e-12


def test_hessenberg_special_inputs(gpu_lib):
    # already Hessenberg: every reflector is the identity
    H0 = inputs.hessenberg_normal(70, 403)
    H, Q, rc = _gpu(gpu_lib, H0)
    assert rc == 0 and np.array_equal(H, H0) and np.array_equal(Q, np.eye(70))
    # symmetric: tridiagonal with the same eigenvalues
    S = _dense(90, 404)
    S = S + S.T
    H, Q, rc = _gpu(gpu_lib, S)
    Ho, _ = oracle.hessenberg(S)
    assert rc == 0 and np.abs(H - Ho).max() <= 1e-12 * np.linalg.norm(S)
    T = np.triu(np.tril(H, 1), -1)
    assert np.abs(np.linalg.eigvalsh(T) - np.linalg.eigvalsh(S)).max() <= 1e-12 * np.linalg.norm(S)
    # a zero column below the diagonal in the middle (reflector of a zero tail)
    A = _dense(80, 405)
    A[10:, 9] = 0.0
    H, Q, rc = _gpu(gpu_lib, A)
    Ho, Qo = oracle.hessenberg(A)
    assert rc == 0 and np.abs(H - Ho).max() <= 1e-12 * np.linalg.norm(A)


def test_hessenberg_argument_errors(gpu_lib):
    import torch

    h = gpu_lib.Handle(0)
    A = torch.zeros(4, 4, dtype=torch.float64, device="cuda:0")
    p = A.data_ptr()
    assert h.hessenberg_async(None, -1, p, 4, None, 1) == -1
    assert h.hessenberg_async(None, 4, None, 4, None, 1) == -2
    assert h.hessenberg_async(None, 4, p, 3, None, 1) == -3
    assert h.hessenberg_async(None, 4, p, 4, p, 3) == -5
    assert h.hessenberg_async(None, 0, None, 1, None, 1) == 0
    h.close()


def test_hessenberg_full_size(gpu_lib):
    """n = 16384, dense U(-1,1) (the paper's test matrices), with Q1."""
    import torch

    n = 16384
    print("case hess full n=%d" % n, flush=True)
    dev = torch.device("cuda:0")
    g = torch.Generator(dev).manual_seed(16384)
    A0 = torch.rand(n, n, dtype=torch.float64, device=dev, generator=g) * 2.0 - 1.0
    A = A0.t().contiguous().t()   # column-major copy of the same matrix
    assert A.stride(0) == 1
    Q = torch.eye(n, dtype=torch.float64, device=dev).t().contiguous().t()
    h = gpu_lib.Handle(0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    rc = h.hessenberg_async(torch.cuda.current_stream().cuda_stream, n, A.data_ptr(), A.stride(1),
                            Q.data_ptr(), Q.stride(1))
    e1.record()
    torch.cuda.synchronize()
    h.close()
    print("hessenberg n=%d: %.3f s" % (n, e0.elapsed_time(e1) / 1e3), flush=True)
    assert rc == 0
    H = A
    assert torch.count_nonzero(torch.tril(H, -2)).item() == 0
    assert Q[0, 0].item() == 1.0
    assert torch.count_nonzero(Q[0, 1:]).item() == 0 and torch.count_nonzero(Q[1:, 0]).item() == 0
    nrm = torch.linalg.norm(A0).item()
    R = A0 - Q @ (H @ Q.t())
    res = torch.linalg.norm(R).item() / nrm
    del R
    E = Q.t() @ Q
    E.diagonal().sub_(1.0)
    orth = torch.linalg.norm(E).item()
    del E
    print("residual %.3e orthogonality %.3e" % (res, orth), flush=True)
    assert res <= 1e-12
    assert orth <= 1e-11   # LAPACK's Hessenberg Q at this order: about 3e-12
    # Arnoldi with full re-orthogonalisation from e_1: the first k columns
    # of Q1 and the leading (k+1) x k block of H (signs of Q1 fixed)
    k = 8
    V = torch.zeros(n, k + 1, dtype=torch.float64, device=dev)
    Hk = torch.zeros(k + 1, k, dtype=torch.float64, device=dev)
    V[0, 0] = 1.0
    for j in range(k):
        w = A0 @ V[:, j]
        for _ in range(2):
            c = V[:, :j + 1].t() @ w
            w = w - V[:, :j + 1] @ c
            Hk[:j + 1, j] += c
        Hk[j + 1, j] = torch.linalg.norm(w)
        V[:, j + 1] = w / Hk[j + 1, j]
    # Arnoldi's subdiagonal entries are positive, ours -sign(x_1) ||x||
    sg = torch.sign(torch.sum(V * Q[:, :k + 1], dim=0))
    D = torch.diag(sg)
    errQ = (Q[:, :k + 1] @ D - V).abs().max().item()
    errH = (D @ H[:k + 1, :k] @ D[:k, :k] - Hk).abs().max().item()
    print("Arnoldi: max |dQ| %.3e max |dH| %.3e" % (errQ, errH), flush=True)
    assert errQ <= 1e-12 and errH <= 1e-10 * nrm / np.sqrt(n)
