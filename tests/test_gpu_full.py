"""Parity at the full benchmark size (n = 16384), in the launch
configurations bench.py times.

The oracle cannot solve this size, so the result is checked through
properties that hold at any size: backward error and orthogonality computed
exactly on the GPU with torch FP64 matrix products (independent of the
library's kernels), exact quasi-triangular structure with standardised 2x2
blocks, and the similarity invariants trace(H) = sum(lambda) and
trace(H^2) = sum(lambda^2).

Orthogonality bar: 1e-12 as stated, except where LAPACK's own Schur
reduction of the same matrix does not reach it (the error of Q grows with the
order and the number of transformations; n u = 1.8e-12 at this order): there
the bar is twice LAPACK's figure, measured by
tests/golden/lapack_orthogonality.py on the same seeded input.
"""
import json
import os

import numpy as np
import pytest

from paper_1905_04975_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
N = 16384

# (label, input, order, options):
#   default     -- random N(0,1) Hessenberg, the bench configuration;
#   sweep256    -- the dense-derived matrix below with 256 shifts per sweep
#                  and the parallel passes off: multishift sweeps with LDS
#                  windows and MFMA panel products, alternating with early
#                  deflation (the random matrix above needs no sweep at all
#                  once early deflation runs: its windows deflate everything);
#   paper_like  -- the Hessenberg form of a dense matrix with U(-1,1)
#                  entries (the paper's test matrices, Sec. 5; drawn from its
#                  distribution in O(n^2)), default options: the passes find
#                  no localisation and hand over to sweeps with early
#                  deflation.
CASES = [
    ("default", "normal", N, {}),
    ("sweep256", "law", N, dict(ns=256, split_window=-1)),
    ("paper_like", "law", N, {}),
    ("paper_like_8192", "law", 8192, {}),
]


def _input(kind, n):
    if kind == "normal":
        return inputs.hessenberg_normal(n, inputs.SEED_N16384)
    return inputs.paper_like_law(n, inputs.SEED_PAPER_LIKE)


def _orth_bar(kind, n):
    with open(os.path.join(HERE, "golden", "lapack_orthogonality.json")) as f:
        ref = json.load(f)
    key = "%s_n%d_seed%d" % (kind, n, inputs.SEED_N16384 if kind == "normal"
                             else inputs.SEED_PAPER_LIKE)
    return max(1e-12, 2.0 * ref[key]["orthogonality"]), ref[key]["orthogonality"]


@pytest.mark.parametrize("label,kind,n,opts", CASES, ids=[c[0] for c in CASES])
def test_full_size(gpu_lib, label, kind, n, opts):
    import torch

    bar, lapack = _orth_bar(kind, n)
    print("case full %s n=%d opts=%s orthogonality bar %.3e (LAPACK %.3e)"
          % (label, n, opts, bar, lapack), flush=True)
    dev = torch.device("cuda:0")
    H0 = torch.from_numpy(_input(kind, n)).to(dev)
    H = H0.clone()
    Q = torch.eye(n, dtype=torch.float64, device=dev).t().contiguous().t()
    h = gpu_lib.Handle(0, **opts)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    S, Qo, w, info = gpu_lib.reduce(H, Q=Q, handle=h)
    ev1.record()
    torch.cuda.synchronize()
    st = h.stats()
    h.close()
    print("%.3f s, stats %s" % (ev0.elapsed_time(ev1) / 1e3,
                                {k: st[k] for k in ("sweeps", "windows", "shifts_applied",
                                                    "aed_windows", "aed_deflated", "split_passes",
                                                    "split_accepted", "small_solves")}),
          flush=True)
    assert info == 0
    assert S.data_ptr() == H.data_ptr() and Qo.data_ptr() == Q.data_ptr()
    if label == "sweep256":
        assert st["sweeps"] > 0 and st["split_passes"] == 0
        assert st["shifts_applied"] > 200 * st["sweeps"]   # mostly full 256-shift sweeps
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
    print("residual %.3e orthogonality %.3e (%.2f x LAPACK)" % (res, orth, orth / lapack),
          flush=True)
    assert res <= 1e-12
    assert orth <= bar, (orth, bar)
    # similarity invariants
    tr = torch.trace(Hh).item()
    assert abs(w.real.sum().item() - tr) <= 1e-10 * nrm
    tr2 = torch.sum(Hh * Hh.t()).item()
    lam2 = torch.sum(w * w).real.item()
    assert abs(lam2 - tr2) <= 1e-9 * nrm ** 2
