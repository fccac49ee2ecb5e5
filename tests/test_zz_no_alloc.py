"""schur_reduce_noalloc: the Schur reduction with its workspace in a static
device array (no allocation), checked against the existing entry point
schur_reduce_async on a handle with the same options (no parallel passes;
at these orders at most 128 shifts per sweep, so no nested shift solve).

The two entry points run the same kernels on the same data in the same
order; the no-allocation one only keeps everything on one stream, so the
results must agree bit for bit.  Each result is also checked against the
definition of a real Schur form and the oracle's eigenvalues.  Two calls in
a row, the second on a smaller matrix, show that the array's leftover
contents from a previous call do not leak into the next."""
import numpy as np
import pytest

import oracle
from paper_1905_04975_amd import inputs
from tests import checks

pytestmark = pytest.mark.gpu


def _col(torch, A, dev):
    return torch.from_numpy(np.asfortranarray(A)).to(dev).t().contiguous().t()


def _existing(schur, torch, H_np, want_q, dev):
    n = H_np.shape[0]
    H = _col(torch, H_np, dev)
    Q = _col(torch, np.eye(n), dev) if want_q else None
    h = schur.Handle(0, split_window=-1)
    S, Qo, w, info = schur.reduce(H, Q=Q, want_q=want_q, handle=h)
    torch.cuda.synchronize()
    h.close()
    return S.cpu().numpy(), (Qo.cpu().numpy() if want_q else None), w.cpu().numpy(), info


def _noalloc(schur, torch, H_np, want_q, dev):
    n = H_np.shape[0]
    H = _col(torch, H_np, dev)
    Q = _col(torch, np.eye(n), dev) if want_q else None
    wr = torch.empty(n, dtype=torch.float64, device=dev)
    wi = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    info = schur.schur_reduce_noalloc(stream.cuda_stream, n, H.data_ptr(), H.stride(1),
                                      Q.data_ptr() if want_q else None,
                                      Q.stride(1) if want_q else 1, wr.data_ptr(), wi.data_ptr())
    torch.cuda.synchronize()
    w = wr.cpu().numpy() + 1j * wi.cpu().numpy()
    return H.cpu().numpy(), (Q.cpu().numpy() if want_q else None), w, info


def test_noalloc_equals_existing_entry_point(gpu_lib):
    import torch

    dev = torch.device("cuda:0")
    H1, truth1 = inputs.prescribed(700, 81)
    H2 = inputs.hessenberg_normal(300, 82)
    # two calls in a row, the second smaller; the first with Schur vectors,
    # then the second with and without them
    for label, H_np, want_q in (("prescribed n=700", H1, True), ("random n=300", H2, True),
                                ("random n=300 no Q", H2, False)):
        print("case noalloc %s" % label, flush=True)
        S, Q, w, info = _noalloc(gpu_lib, torch, H_np, want_q, dev)
        S0, Q0, w0, info0 = _existing(gpu_lib, torch, H_np, want_q, dev)
        assert info == 0 and info0 == 0
        assert np.array_equal(S, S0)
        assert np.array_equal(w, w0)
        if want_q:
            assert np.array_equal(Q, Q0)
            assert checks.residual(H_np, Q, S) <= 1e-12
            assert checks.orthogonality(Q) <= 1e-12
        assert checks.structure_errors(S, w.real, w.imag) == []
        _, _, wr, wi, oinfo, _ = oracle.schur(H_np)
        assert oinfo == 0
        nrm = np.linalg.norm(H_np)
        if H_np is H1:
            d = checks.match_eigs(w, truth1)
            assert np.all(d <= checks.eig_rel_tol(truth1, H_np)), d.max()
        else:
            assert checks.match_eigs(w, wr + 1j * wi).max() <= 1e-9 * max(1.0, nrm)


def test_noalloc_rejects_orders_above_its_maximum(gpu_lib):
    import torch

    dev = torch.device("cuda:0")
    big = 32769   # SCHUR_NOALLOC_MAX_N + 1; the check runs before any device work
    buf = torch.zeros(4, dtype=torch.float64, device=dev)
    p = buf.data_ptr()
    assert gpu_lib.schur_reduce_noalloc(None, big, p, big, None, 1, p, p) == -106
    assert gpu_lib.schur_reduce_noalloc(None, -1, p, 1, None, 1, p, p) == -1
    assert gpu_lib.schur_reduce_noalloc(None, 0, None, 1, None, 1, None, None) == 0
