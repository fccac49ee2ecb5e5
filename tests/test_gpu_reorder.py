"""GPU parity of eigenvalue reordering (paper Sec. 2, Eq. (7)) against the
oracle (MI355X only).

The reordered Schur form is not unique, but the invariant subspace of the
selected eigenvalues is: the span of the first m columns of Q3 is compared
with the oracle's through the sines of the principal angles.  Beside it:
similarity S = Q3 S' Q3^T, orthogonality, standardised structure, and the
eigenvalues of the leading m x m block equal to the selected ones.  Orders
span one window (96 rows), chains of many windows and several chains in
flight; selections cover none, all, the leading blocks, and random subsets.
"""
import numpy as np
import pytest

import oracle
from paper_1905_04975_amd import inputs
from tests import checks

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _dev(A):
    import torch

    return torch.from_numpy(np.asfortranarray(A)).to("cuda:0").t().contiguous().t()


def _gpu(schur, S, sel, Q=None):
    import torch

    n = S.shape[0]
    h = schur.Handle(0)
    Qd = _dev(np.eye(n) if Q is None else Q)
    Sd, Qd, w, m, rc = schur.reorder(_dev(S), sel, Q=Qd, handle=h)
    torch.cuda.synchronize()
    h.close()
    return Sd.cpu().numpy(), Qd.cpu().numpy(), w.cpu().numpy(), m, rc


def _selected_eigs(S, sel):
    lam, _ = oracle.complex_vectors(S, np.zeros_like(S))
    out, k, n = [], 0, S.shape[0]
    while k < n:
        s = 2 if (k + 1 < n and S[k + 1, k] != 0.0) else 1
        if sel[k] or (s == 2 and sel[k + 1]):
            out.extend(lam[k:k + s])
        k += s
    return np.array(out)


def _sine(Q1, Q2, m):
    """largest sine of the principal angles between span(Q1[:, :m]) and
    span(Q2[:, :m])."""
    A, B = Q1[:, :m], Q2[:, :m]
    return np.linalg.norm(B - A @ (A.T @ B), 2)


def _check(S, sel, S2, Q3, w, m, rc):
    n = S.shape[0]
    assert rc == 0
    assert checks.structure_errors(S2, w.real, w.imag) == []
    assert np.linalg.norm(Q3.T @ Q3 - np.eye(n)) <= 100 * n * U
    assert np.linalg.norm(S - Q3 @ S2 @ Q3.T) <= 100 * n * U * np.linalg.norm(S)
    want = _selected_eigs(S, sel)
    assert m == want.size
    if m:
        assert checks.match_eigs(w[:m], want).max() <= 1e-11 * np.linalg.norm(S)


@pytest.mark.parametrize("n,seed,frac", [(2, 1, 0.5), (5, 2, 0.5), (50, 3, 0.5), (96, 4, 0.4),
                                         (97, 5, 0.6), (200, 6, 0.5), (500, 7, 0.3),
                                         (1000, 8, 0.5), (1000, 9, 0.9)])
def test_reorder_vs_oracle(gpu_lib, n, seed, frac):
    print("case reorder n=%d seed=%d frac=%.1f" % (n, seed, frac), flush=True)
    S = inputs.schur_form(n, 700 + seed)
    sel = (np.random.Generator(np.random.PCG64(seed)).uniform(size=n) < frac).astype(int)
    S2, Q3, w, m, rc = _gpu(gpu_lib, S, sel)
    _check(S, sel, S2, Q3, w, m, rc)
    So, Qo, wro, wio, mo, info = oracle.reorder(S, sel)
    assert info == 0 and mo == m
    if m:
        assert _sine(Q3, Qo, m) <= 1e-10


def test_reorder_accumulates_q(gpu_lib):
    """Schur vectors of a random Hessenberg matrix (oracle) as Q_in: the
    first m columns of the result span the invariant subspace of H for the
    eigenvalues inside the unit disc."""
    n = 300
    H = inputs.hessenberg_normal(n, 710)
    S, Q, _, _, info, _ = oracle.schur(H)
    assert info == 0
    lam, _ = oracle.complex_vectors(S, np.zeros_like(S))
    sel = (np.abs(lam) < 1.0).astype(int)
    S2, Q2, w, m, rc = _gpu(gpu_lib, S, sel, Q=Q)
    assert rc == 0
    assert np.linalg.norm(H - Q2 @ S2 @ Q2.T) <= 1000 * n * U * np.linalg.norm(H)
    assert np.all(np.abs(w[:m]) < 1.0) and np.all(np.abs(w[m:]) >= 1.0)
    So, Qo, _, _, mo, info = oracle.reorder(S, sel, Q=Q)
    assert info == 0 and mo == m
    assert _sine(Q2, Qo, m) <= 1e-8   # subspace of a non-normal matrix: conditioning


def test_reorder_nothing_to_move(gpu_lib):
    S = inputs.schur_form(150, 711)
    blocks_lead = 0
    k = 0
    while k < 40:
        k += 2 if S[k + 1, k] != 0.0 else 1
    blocks_lead = k
    for sel in (np.zeros(150, int), np.ones(150, int),
                np.r_[np.ones(blocks_lead, int), np.zeros(150 - blocks_lead, int)]):
        S2, Q3, w, m, rc = _gpu(gpu_lib, S, sel)
        assert rc == 0
        assert np.array_equal(S2, S) and np.array_equal(Q3, np.eye(150))


def test_reorder_argument_errors(gpu_lib):
    import torch

    h = gpu_lib.Handle(0)
    A = torch.zeros(4, 4, dtype=torch.float64, device="cuda:0")
    p = A.data_ptr()
    sel = [1, 0, 0, 0]
    assert h.reorder_async(None, -1, p, 4, None, 1, sel, p, p)[0] == -1
    assert h.reorder_async(None, 4, None, 4, None, 1, sel, p, p)[0] == -2
    assert h.reorder_async(None, 4, p, 3, None, 1, sel, p, p)[0] == -3
    assert h.reorder_async(None, 4, p, 4, p, 3, sel, p, p)[0] == -5
    assert h.reorder_async(None, 4, p, (1 << 20) + 1, None, 1, sel, p, p)[0] == -3
    assert h.reorder_async(None, 4, p, 4, p, (1 << 20) + 1, sel, p, p)[0] == -5
    assert h.reorder_async(None, 4, p, 4, None, 1, sel, None, p)[0] == -7
    assert h.reorder_async(None, 4, p, 4, None, 1, sel, p, None)[0] == -8
    h.close()


def test_reorder_full_size(gpu_lib):
    """n = 16384, half of the eigenvalues selected at random, with Q."""
    import torch

    n = 16384
    print("case reorder full n=%d" % n, flush=True)
    S_np = inputs.schur_form(n, 16385)
    sel = (np.random.Generator(np.random.PCG64(16385)).uniform(size=n) < 0.5).astype(int)
    dev = torch.device("cuda:0")
    S = _dev(S_np)
    Q = torch.eye(n, dtype=torch.float64, device=dev).t().contiguous().t()
    h = gpu_lib.Handle(0, flags=gpu_lib.FLAG_TIME_KERNELS)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    S2, Q3, w, m, rc = gpu_lib.reorder(S, sel, Q=Q, handle=h)
    e1.record()
    torch.cuda.synchronize()
    st = h.stats()
    h.close()
    print("reorder n=%d: %.3f s, %d windows in %d steps, window tasks %.3f s, products %.3f s"
          % (n, e0.elapsed_time(e1) / 1e3, st["reorder_windows"], st["reorder_steps"],
             st["reorder_ms"] / 1e3, (st["row_ms"] + st["colq_ms"]) / 1e3), flush=True)
    assert rc == 0
    S0 = _dev(S_np)
    R = S0 - Q3 @ (S2 @ Q3.t())
    res = torch.linalg.norm(R).item() / torch.linalg.norm(S0).item()
    del R
    E = Q3.t() @ Q3
    E.diagonal().sub_(1.0)
    orth = torch.linalg.norm(E).item()
    del E
    print("residual %.3e orthogonality %.3e" % (res, orth), flush=True)
    assert res <= 1e-12 and orth <= 1e-11
    assert torch.count_nonzero(torch.tril(S2, -2)).item() == 0
    want = np.sort_complex(np.round(_selected_eigs(S_np, sel), 9))
    got = np.sort_complex(np.round(w[:m].cpu().numpy(), 9))
    assert m == want.size and np.abs(got - want).max() <= 2e-9
