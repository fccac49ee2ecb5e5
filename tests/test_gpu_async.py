"""schur_reduce_begin / schur_reduce_end: the Schur reduction that returns
to the caller at once (MI355X only).  The begun solve must give the same
result, bit for bit, as the blocking call on the same handle options; the
begin call must return long before the solve is done; work enqueued on the
caller's stream after schur_reduce_end must see the result; the info code
reaches the device."""
import time

import numpy as np
import pytest

from paper_1905_04975_amd import inputs

pytestmark = pytest.mark.gpu


def _col(torch, A):
    return torch.from_numpy(np.asfortranarray(A)).to("cuda:0").t().contiguous().t()


@pytest.mark.parametrize("n,seed", [(600, 801), (3000, 802)])
def test_begin_end_equals_blocking_call(gpu_lib, n, seed):
    import torch

    print("case async n=%d" % n, flush=True)
    H_np = inputs.hessenberg_normal(n, seed)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    # the blocking call
    h0 = gpu_lib.Handle(0)
    S0, Q0, w0, info0 = gpu_lib.reduce(_col(torch, H_np), handle=h0)
    torch.cuda.synchronize()
    h0.close()
    assert info0 == 0
    # begin / end
    h = gpu_lib.Handle(0)
    H = _col(torch, H_np)
    Q = _col(torch, np.eye(n))
    wr = torch.empty(n, dtype=torch.float64, device=dev)
    wi = torch.empty(n, dtype=torch.float64, device=dev)
    info_dev = torch.full((1,), -7, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc = h.reduce_begin(stream.cuda_stream, n, H.data_ptr(), n, Q.data_ptr(), n, wr.data_ptr(),
                        wi.data_ptr(), info_dev.data_ptr())
    t1 = time.perf_counter()
    assert rc == 0
    assert h.reduce_begin(stream.cuda_stream, n, H.data_ptr(), n, Q.data_ptr(), n,
                          wr.data_ptr(), wi.data_ptr(), None) == -104   # busy
    info = h.reduce_end(stream.cuda_stream)
    t2 = time.perf_counter()
    # enqueued after end, on the caller's stream: sees the result
    Hc, Qc = H.clone(), Q.clone()
    wc = torch.complex(wr, wi).clone()
    ic = info_dev.clone()
    torch.cuda.synchronize()
    h.close()
    print("begin returned after %.4f s, solve done after %.4f s" % (t1 - t0, t2 - t0), flush=True)
    assert info == 0 and ic.item() == 0
    assert (t1 - t0) < 0.2 * (t2 - t0)
    assert torch.equal(Hc, S0) and torch.equal(Qc, Q0) and torch.equal(wc, w0)


def test_begin_end_errors(gpu_lib):
    import torch

    h = gpu_lib.Handle(0)
    dev = torch.device("cuda:0")
    A = torch.zeros(4, 4, dtype=torch.float64, device=dev)
    p = A.data_ptr()
    assert h.reduce_end(None) == -104               # nothing begun
    assert h.reduce_begin(None, -1, p, 4, None, 1, p, p) == -1
    assert h.reduce_begin(None, 4, p, 3, None, 1, p, p) == -3
    # a non-finite input is found by the solve: reported by end and on the device
    B = torch.eye(4, dtype=torch.float64, device=dev).t().contiguous().t()
    B[1, 0] = float("nan")
    info_dev = torch.zeros(1, dtype=torch.int32, device=dev)
    wr = torch.empty(4, dtype=torch.float64, device=dev)
    wi = torch.empty(4, dtype=torch.float64, device=dev)
    assert h.reduce_begin(None, 4, B.data_ptr(), 4, None, 1, wr.data_ptr(), wi.data_ptr(),
                          info_dev.data_ptr()) == 0
    assert h.reduce_end(None) == -2
    torch.cuda.synchronize()
    assert info_dev.item() == -2
    h.close()
