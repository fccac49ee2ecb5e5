"""Parity at the full benchmark size (n = 16384, seed 3), in the launch
configuration bench.py times (default options).

The oracle cannot solve this size, so the result is checked through
properties that hold at any size: backward error and orthogonality computed
exactly on the GPU with torch FP64 matrix products (independent of the
library's kernels), exact quasi-triangular structure with standardised 2x2
blocks, and the similarity invariants trace(H) = sum(lambda) and
trace(H^2) = sum(lambda^2).
"""
import numpy as np
import pytest

from paper_1905_04975_amd import inputs

pytestmark = pytest.mark.gpu


def test_full_size_n16384(gpu_lib):
    import torch

    n = 16384
    print("case full n=%d seed=%d (default options)" % (n, inputs.SEED_N16384), flush=True)
    dev = torch.device("cuda:0")
    H0 = torch.from_numpy(inputs.hessenberg_normal(n, inputs.SEED_N16384)).to(dev)
    H = H0.clone()
    Q = torch.eye(n, dtype=torch.float64, device=dev).t().contiguous().t()
    h = gpu_lib.Handle(0)
    S, Qo, w, info = gpu_lib.reduce(H, Q=Q, handle=h)
    torch.cuda.synchronize()
    h.close()
    assert info == 0
    assert S.data_ptr() == H.data_ptr() and Qo.data_ptr() == Q.data_ptr()
    # structure: exact zeros below the subdiagonal, isolated standard 2x2 blocks
    assert torch.count_nonzero(torch.tril(S, -2)).item() == 0
    sub = torch.diagonal(S, -1)
    nz = (sub != 0)
    assert not torch.any(nz[1:] & nz[:-1]).item()
    k = torch.nonzero(nz).flatten()
    a = S[k, k]
    d = S[k + 1, k + 1]
    b = S[k, k + 1]
    c = S[k + 1, k]
    assert torch.equal(a, d)
    assert torch.all(b * c < 0).item()
    # eigenvalues read from the blocks
    assert torch.equal(w.real, torch.diagonal(S))
    assert torch.all(w.imag[k] > 0).item() and torch.equal(w.imag[k + 1], -w.imag[k])
    # backward error and orthogonality (exact Frobenius norms, torch FP64 GEMMs)
    Hh = torch.triu(H0, -1)
    nrm = torch.linalg.norm(Hh).item()
    R = Hh - Q @ (S @ Q.t())
    res = torch.linalg.norm(R).item() / nrm
    del R
    E = Q.t() @ Q
    E.diagonal().sub_(1.0)
    orth = torch.linalg.norm(E).item()
    del E
    print("residual %.3e orthogonality %.3e" % (res, orth), flush=True)
    assert res <= 1e-12
    assert orth <= 1e-12, orth
    # similarity invariants
    tr = torch.trace(Hh).item()
    assert abs(w.real.sum().item() - tr) <= 1e-10 * nrm
    tr2 = torch.sum(Hh * Hh.t()).item()
    lam2 = torch.sum(w * w).real.item()
    assert abs(lam2 - tr2) <= 1e-9 * nrm ** 2
