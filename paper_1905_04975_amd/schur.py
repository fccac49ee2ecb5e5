"""Python binding of the C ABI declared in ``include/schur.h``.

Argument marshalling only: every step of the Schur reduction runs in the
HIP library ``libschur_mi355x.so`` (built in-tree by ``build.py``).  PyTorch
supplies device memory and streams.  There is no CPU fallback: loading fails
loudly when the built library is missing.

Matrices are column-major.  A torch tensor ``T`` is used in place when
``T.stride(0) == 1`` (its memory is column-major with ``ld = T.stride(1)``);
otherwise ``reduce`` works on a column-major copy.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libschur_mi355x.so")

_lib = None


class SchurOpts(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("nb", ctypes.c_int), ("step", ctypes.c_int),
                ("nmin", ctypes.c_int), ("max_sweeps", ctypes.c_int),
                ("exc_period", ctypes.c_int), ("flags", ctypes.c_int),
                ("aed_window", ctypes.c_int), ("aed_nibble", ctypes.c_int),
                ("split_window", ctypes.c_int), ("split_min_n", ctypes.c_int),
                ("panel_tile", ctypes.c_int)]


class SchurStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int64), ("windows", ctypes.c_int64),
                ("chain_steps", ctypes.c_int64), ("small_solves", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("gemm_flops", ctypes.c_double),
                ("gemm_ms", ctypes.c_double), ("gemm_launches", ctypes.c_int64),
                ("chase_ms", ctypes.c_double), ("chase_launches", ctypes.c_int64),
                ("shift_ms", ctypes.c_double), ("other_ms", ctypes.c_double),
                ("shifts_applied", ctypes.c_int64),
                ("row_flops", ctypes.c_double), ("row_ms", ctypes.c_double),
                ("row_launches", ctypes.c_int64),
                ("colq_flops", ctypes.c_double), ("colq_ms", ctypes.c_double),
                ("colq_launches", ctypes.c_int64),
                ("aed_ms", ctypes.c_double), ("aed_windows", ctypes.c_int64),
                ("aed_deflated", ctypes.c_int64), ("aed_flops", ctypes.c_double),
                ("split_passes", ctypes.c_int64), ("split_windows", ctypes.c_int64),
                ("split_accepted", ctypes.c_int64), ("split_converged", ctypes.c_int64),
                ("split_ms", ctypes.c_double), ("split_flops", ctypes.c_double),
                ("small_ms", ctypes.c_double), ("small_flops", ctypes.c_double),
                ("chase_flops", ctypes.c_double), ("small_launches", ctypes.c_int64),
                ("aed_launches", ctypes.c_int64),
                ("hess_panel_ms", ctypes.c_double), ("hess_gemv_bytes", ctypes.c_double),
                ("hess_gemm_ms", ctypes.c_double), ("hess_gemm_flops", ctypes.c_double),
                ("ev_solve_ms", ctypes.c_double), ("ev_gemm_ms", ctypes.c_double),
                ("ev_gemm_flops", ctypes.c_double), ("ev_back_ms", ctypes.c_double),
                ("ev_back_flops", ctypes.c_double),
                ("reorder_ms", ctypes.c_double), ("reorder_windows", ctypes.c_int64),
                ("reorder_steps", ctypes.c_int64), ("chase_bytes", ctypes.c_double),
                ("persist_ms", ctypes.c_double), ("persist_jobs", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


FLAG_TIME_KERNELS = 1
FLAG_BATCH_ROUNDS = 2
FLAG_ONE_STREAM = 4

EXPORTS = ("schur_reduce", "schur_create", "schur_destroy", "schur_set_opts",
           "schur_get_stats", "schur_reduce_async", "schur_reduce_batched",
           "schur_server_create", "schur_server_destroy", "schur_submit", "schur_poll",
           "schur_server_get_stats", "schur_set_tuning", "schur_plan_sweep",
           "schur_plan_split", "schur_select_windows", "schur_split_weight",
           "schur_reduce_noalloc", "schur_hessenberg", "schur_eigenvectors",
           "schur_reorder", "schur_plan_reorder", "schur_reduce_begin", "schur_reduce_end")

TUNING_PATH = os.path.join(HERE, "tuning.json")


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("resident", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("peak_resident", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_double), ("peak_bytes", ctypes.c_double),
                ("reserved", ctypes.c_double * 4)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def load():
    """Load the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # the library binds to the HIP runtime already in the process (same
        # soname); load torch's first, so that one runtime serves both
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is missing: run `python -m paper_1905_04975_amd.build`"
                           % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p
    lib.schur_reduce.argtypes = [ip, dp, ip, dp, ip, dp, dp]
    lib.schur_reduce.restype = ctypes.c_int
    lib.schur_create.argtypes = [ctypes.POINTER(vp), ip, ctypes.POINTER(SchurOpts)]
    lib.schur_create.restype = ctypes.c_int
    lib.schur_destroy.argtypes = [vp]
    lib.schur_destroy.restype = ctypes.c_int
    lib.schur_set_opts.argtypes = [vp, ctypes.POINTER(SchurOpts)]
    lib.schur_set_opts.restype = ctypes.c_int
    lib.schur_get_stats.argtypes = [vp, ctypes.POINTER(SchurStats)]
    lib.schur_get_stats.restype = ctypes.c_int
    lib.schur_reduce_async.argtypes = [vp, vp, ip, dp, ip, dp, ip, dp, dp, ctypes.POINTER(ip)]
    lib.schur_reduce_async.restype = ctypes.c_int
    lib.schur_reduce_begin.argtypes = [vp, vp, ip, dp, ip, dp, ip, dp, dp, dp]
    lib.schur_reduce_begin.restype = ctypes.c_int
    lib.schur_reduce_end.argtypes = [vp, vp]
    lib.schur_reduce_end.restype = ctypes.c_int
    lib.schur_reorder.argtypes = [vp, vp, ip, dp, ip, dp, ip, ctypes.POINTER(ip), dp, dp,
                                  ctypes.POINTER(ip)]
    lib.schur_reorder.restype = ctypes.c_int
    lib.schur_plan_reorder.argtypes = [ip, ctypes.POINTER(ip), ctypes.POINTER(ip), ip,
                                       ctypes.POINTER(ip), ip]
    lib.schur_plan_reorder.restype = ctypes.c_int
    lib.schur_eigenvectors.argtypes = [vp, vp, ip, dp, ip, dp, ip, dp, ip]
    lib.schur_eigenvectors.restype = ctypes.c_int
    lib.schur_hessenberg.argtypes = [vp, vp, ip, dp, ip, dp, ip]
    lib.schur_hessenberg.restype = ctypes.c_int
    lib.schur_reduce_noalloc.argtypes = [vp, ip, dp, ip, dp, ip, dp, dp]
    lib.schur_reduce_noalloc.restype = ctypes.c_int
    pint = ctypes.POINTER(ctypes.c_int)
    pptr = ctypes.POINTER(ctypes.c_void_p)
    lib.schur_reduce_batched.argtypes = [vp, vp, ip, pint, pptr, pint, pptr, pint, pptr, pptr, pint]
    lib.schur_reduce_batched.restype = ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.schur_server_create.argtypes = [ctypes.POINTER(vp), ip, ctypes.c_size_t,
                                        ctypes.POINTER(SchurOpts)]
    lib.schur_server_create.restype = ctypes.c_int
    lib.schur_server_destroy.argtypes = [vp]
    lib.schur_server_destroy.restype = ctypes.c_int
    lib.schur_submit.argtypes = [vp, ip, dp, ip, ip, u64p]
    lib.schur_submit.restype = ctypes.c_int
    lib.schur_poll.argtypes = [vp, ctypes.c_uint64, dp, ip, dp, ip, dp, dp,
                               ctypes.POINTER(ip), ctypes.POINTER(ctypes.c_double)]
    lib.schur_poll.restype = ctypes.c_int
    lib.schur_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.schur_server_get_stats.restype = ctypes.c_int
    pi = ctypes.POINTER(ctypes.c_int)
    lib.schur_set_tuning.argtypes = [ip, pi, pi, pi, pi, pi, pi, pi]
    lib.schur_set_tuning.restype = ctypes.c_int
    lib.schur_plan_sweep.argtypes = [ip, ip, ip, ip, ip, pi, ip]
    lib.schur_plan_sweep.restype = ctypes.c_int
    lib.schur_plan_split.argtypes = [ip, ip, ip, ip, pi, ip]
    lib.schur_plan_split.restype = ctypes.c_int
    lib.schur_select_windows.argtypes = [ip, pi, pi, ctypes.POINTER(ctypes.c_double), pi]
    lib.schur_select_windows.restype = ctypes.c_int
    lib.schur_split_weight.argtypes = [ip, ip, ip, ip]
    lib.schur_split_weight.restype = ctypes.c_double
    _lib = lib
    path = os.environ.get("SCHUR_TUNE_TABLE", TUNING_PATH)
    if os.path.exists(path):
        load_tuning(path)
    return lib


def schur_reduce(n, H, ldh, Q, ldq, wr, wi):
    """C ``schur_reduce`` with raw device pointers (ints); returns info."""
    return load().schur_reduce(int(n), H, int(ldh), Q, int(ldq), wr, wi)


def schur_reduce_noalloc(stream, n, H, ldh, Q, ldq, wr, wi):
    """C ``schur_reduce_noalloc`` (workspace in a static device array, no
    allocation) with raw device pointers (ints) and a hipStream_t (int or
    None); returns info."""
    return load().schur_reduce_noalloc(stream, int(n), H, int(ldh), Q, int(ldq), wr, wi)


class Handle:
    """A library handle (its own HIP stream and workspace on one device)."""

    def __init__(self, device: int = 0, **opts):
        lib = load()
        self._h = ctypes.c_void_p()
        o = make_opts(**opts)
        rc = lib.schur_create(ctypes.byref(self._h), int(device), ctypes.byref(o))
        if rc != 0:
            raise RuntimeError("schur_create failed: %d" % rc)

    def set_opts(self, **opts):
        o = make_opts(**opts)
        load().schur_set_opts(self._h, ctypes.byref(o))

    def stats(self):
        st = SchurStats()
        load().schur_get_stats(self._h, ctypes.byref(st))
        return st.as_dict()

    def reduce_async(self, stream, n, H, ldh, Q, ldq, wr, wi):
        info = ctypes.c_int(0)
        rc = load().schur_reduce_async(self._h, stream, int(n), H, int(ldh), Q, int(ldq), wr, wi,
                                       ctypes.byref(info))
        return rc

    def hessenberg_async(self, stream, n, A, lda, Q, ldq):
        """C ``schur_hessenberg`` with raw device pointers; returns its code."""
        return load().schur_hessenberg(self._h, stream, int(n), A, int(lda), Q, int(ldq))

    def eigenvectors_async(self, stream, n, S, lds, Q, ldq, X, ldx):
        """C ``schur_eigenvectors`` with raw device pointers; returns its code."""
        return load().schur_eigenvectors(self._h, stream, int(n), S, int(lds), Q, int(ldq), X,
                                         int(ldx))

    def reduce_begin(self, stream, n, H, ldh, Q, ldq, wr, wi, info_dev=None):
        """C ``schur_reduce_begin`` (returns at once; raw device pointers)."""
        return load().schur_reduce_begin(self._h, stream, int(n), H, int(ldh), Q, int(ldq), wr,
                                         wi, info_dev)

    def reduce_end(self, stream):
        """C ``schur_reduce_end``: the stream waits for the begun solve; its info."""
        return load().schur_reduce_end(self._h, stream)

    def reorder_async(self, stream, n, S, lds, Q, ldq, select, wr, wi):
        """C ``schur_reorder`` with raw device pointers and a host selection
        (sequence of n ints); returns (code, m)."""
        vals = [int(x) for x in select]
        IA = ctypes.c_int * max(1, len(vals))
        sel = IA(*vals)
        m = ctypes.c_int(0)
        rc = load().schur_reorder(self._h, stream, int(n), S, int(lds), Q, int(ldq), sel, wr, wi,
                                  ctypes.byref(m))
        return rc, m.value

    def reduce_batched(self, stream, ns, Hs, ldhs, Qs, ldqs, wrs, wis):
        count = len(ns)
        IA = ctypes.c_int * count
        PA = ctypes.c_void_p * count
        info = IA()
        q_arr = PA(*[q or 0 for q in Qs]) if Qs is not None else None
        ldq_arr = IA(*ldqs) if ldqs is not None else None
        rc = load().schur_reduce_batched(self._h, stream, count, IA(*ns), PA(*Hs), IA(*ldhs),
                                         q_arr, ldq_arr, PA(*wrs), PA(*wis), info)
        return rc, list(info)

    def close(self):
        if self._h:
            load().schur_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_opts(ns=0, nb=0, step=0, nmin=0, max_sweeps=0, exc_period=0, flags=0, aed_window=0,
              aed_nibble=0, split_window=0, split_min_n=0, panel_tile=0):
    o = SchurOpts()
    o.ns, o.nb, o.step, o.nmin = int(ns), int(nb), int(step), int(nmin)
    o.max_sweeps, o.exc_period, o.flags = int(max_sweeps), int(exc_period), int(flags)
    o.aed_window = int(aed_window)
    o.aed_nibble = int(aed_nibble)
    o.split_window = int(split_window)
    o.split_min_n = int(split_min_n)
    o.panel_tile = int(panel_tile)
    return o


def _colmajor(T):
    """Column-major view (or copy) of a 2-D CUDA float64 tensor and its ld."""
    import torch

    if T.dtype != torch.float64:
        raise TypeError("FP64 tensors only")
    if T.stride(0) == 1 and T.stride(1) >= max(1, T.shape[0]):
        return T, T.stride(1)
    C = T.t().contiguous().t()
    return C, max(1, C.stride(1))


def reduce(H, Q=None, want_q=True, handle=None, stream=None):
    """Schur form of the upper Hessenberg CUDA/HIP tensor ``H`` (float64).

    Returns ``(S, Q, w, info)`` with ``w`` complex (torch complex128 on the
    device).  ``H`` is overwritten when it is already column-major; ``Q``
    (if given, column-major float64) is accumulated in place.
    """
    import torch

    n = H.shape[0]
    S, ldh = _colmajor(H)
    dev = S.device
    if want_q:
        if Q is None:
            Qm = torch.eye(n, dtype=torch.float64, device=dev).t()
        else:
            Qm = Q
        Qm, ldq = _colmajor(Qm)
        qptr = Qm.data_ptr()
    else:
        Qm, ldq, qptr = None, 1, None
    wr = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    wi = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    if handle is None:
        torch.cuda.synchronize(dev)
        info = schur_reduce(n, S.data_ptr(), ldh, qptr, ldq, wr.data_ptr(), wi.data_ptr())
    else:
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream
        info = handle.reduce_async(stream, n, S.data_ptr(), ldh, qptr, ldq, wr.data_ptr(),
                                   wi.data_ptr())
    w = torch.complex(wr[:n], wi[:n])
    return S, Qm, w, info


def hessenberg(A, Q=None, want_q=True, handle=None, stream=None):
    """Hessenberg form of the dense CUDA/HIP float64 tensor ``A`` (paper
    Sec. 2, Eq. (3)).  Returns ``(H, Q, rc)``; ``A`` is overwritten when it
    is already column-major, ``Q`` (default the identity) accumulates
    ``Q_in Q1``."""
    import torch

    n = A.shape[0]
    H, lda = _colmajor(A)
    dev = H.device
    if want_q:
        Qm = torch.eye(n, dtype=torch.float64, device=dev).t() if Q is None else Q
        Qm, ldq = _colmajor(Qm)
        qptr = Qm.data_ptr()
    else:
        Qm, ldq, qptr = None, 1, None
    own = handle is None
    if own:
        handle = Handle(dev.index or 0)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    rc = handle.hessenberg_async(stream, n, H.data_ptr(), lda, qptr, ldq)
    if own:
        torch.cuda.synchronize(dev)
        handle.close()
    return H, Qm, rc


def eigenvectors(S, Q=None, handle=None, stream=None):
    """Eigenvectors of the real Schur form ``S`` (CUDA/HIP float64), back-
    transformed with ``Q`` when given (paper Sec. 2, Eqs. (5)-(6)).  Returns
    ``(X, rc)`` with X in LAPACK's real layout (column-major tensor)."""
    import torch

    n = S.shape[0]
    Sm, lds = _colmajor(S)
    dev = Sm.device
    qptr, ldq = None, 1
    if Q is not None:
        Qm, ldq = _colmajor(Q)
        qptr = Qm.data_ptr()
    X = torch.empty(n, n, dtype=torch.float64, device=dev).t()
    own = handle is None
    if own:
        handle = Handle(dev.index or 0)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    rc = handle.eigenvectors_async(stream, n, Sm.data_ptr(), lds, qptr, ldq, X.data_ptr(),
                                   max(1, n))
    if own:
        torch.cuda.synchronize(dev)
        handle.close()
    return X, rc


def reorder(S, select, Q=None, handle=None, stream=None):
    """Reorder the real Schur form ``S`` (CUDA/HIP float64, column-major in
    place) so that the selected eigenvalues lead (paper Sec. 2, Eq. (7));
    ``Q`` accumulates.  Returns ``(S, Q, w, m, rc)``."""
    import torch

    n = S.shape[0]
    Sm, lds = _colmajor(S)
    dev = Sm.device
    qptr, ldq, Qm = None, 1, None
    if Q is not None:
        Qm, ldq = _colmajor(Q)
        qptr = Qm.data_ptr()
    wr = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    wi = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    own = handle is None
    if own:
        handle = Handle(dev.index or 0)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    rc, m = handle.reorder_async(stream, n, Sm.data_ptr(), lds, qptr, ldq, list(select),
                                 wr.data_ptr(), wi.data_ptr())
    if own:
        torch.cuda.synchronize(dev)
        handle.close()
    return Sm, Qm, torch.complex(wr[:n], wi[:n]), m, rc


def plan_reorder(bsize, bsel):
    """Host-only reordering schedule: list of (chain, time step, first row,
    order) for blocks of orders ``bsize`` with selection flags ``bsel``."""
    lib = load()
    nb = len(bsize)
    n = int(sum(bsize))
    IA = ctypes.c_int * max(nb, 1)
    k = lib.schur_plan_reorder(n, IA(*bsize), IA(*bsel), nb, None, 0)
    if k < 0:
        raise ValueError("bad reordering arguments")
    buf = (ctypes.c_int * (4 * max(k, 1)))()
    lib.schur_plan_reorder(n, IA(*bsize), IA(*bsel), nb, buf, k)
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(k)]


def reduce_batched(Hs, want_q=True, handle=None, stream=None):
    """Batched Schur reduction of a list of column-major float64 CUDA tensors.

    Each ``H`` is overwritten by its Schur form when it is column-major
    (otherwise a column-major copy is used).  Returns ``(Ss, Qs, ws, infos,
    rc)``.  Argument marshalling only: all matrices go to one
    ``schur_reduce_batched`` call.
    """
    import torch

    if handle is None:
        handle = Handle(Hs[0].device.index or 0) if Hs else Handle(0)
    Ss, lds, Qs, ldqs, wrs, wis = [], [], [], [], [], []
    for H in Hs:
        S, ld = _colmajor(H)
        n = S.shape[0]
        Ss.append(S)
        lds.append(max(1, ld))
        if want_q:
            Qm = torch.eye(n, dtype=torch.float64, device=S.device).t()
            Qm, ldq = _colmajor(Qm)
            Qs.append(Qm)
            ldqs.append(max(1, ldq))
        wrs.append(torch.empty(max(n, 1), dtype=torch.float64, device=S.device))
        wis.append(torch.empty(max(n, 1), dtype=torch.float64, device=S.device))
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    rc, infos = handle.reduce_batched(
        stream, [S.shape[0] for S in Ss], [S.data_ptr() for S in Ss], lds,
        [Q.data_ptr() for Q in Qs] if want_q else None, ldqs if want_q else None,
        [w.data_ptr() for w in wrs], [w.data_ptr() for w in wis])
    ws = [torch.complex(wr[:S.shape[0]], wi[:S.shape[0]]) for wr, wi, S in zip(wrs, wis, Ss)]
    return Ss, (Qs if want_q else None), ws, infos, rc


class Server:
    """Continuous-batching Schur server (C ``schur_server_*``), host arrays in/out."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, **opts):
        lib = load()
        self._s = ctypes.c_void_p()
        o = make_opts(**opts)
        rc = lib.schur_server_create(ctypes.byref(self._s), int(device), int(budget_bytes),
                                     ctypes.byref(o))
        if rc != 0:
            raise RuntimeError("schur_server_create failed: %d" % rc)

    def submit(self, H, want_q=True):
        """Queue a host numpy matrix (any layout; sent column-major)."""
        import numpy as np

        A = np.asfortranarray(H, dtype=np.float64)
        n = A.shape[0]
        t = ctypes.c_uint64(0)
        rc = load().schur_submit(self._s, n, A.ctypes.data if n else None, max(1, n),
                                 1 if want_q else 0, ctypes.byref(t))
        if rc != 0:
            raise RuntimeError("schur_submit failed: %d" % rc)
        return t.value, n

    def poll(self, ticket, n, want_q=True):
        """None while pending, else (S, Q, w, info, latency_s) as numpy arrays."""
        import numpy as np

        S = np.empty((n, n), order="F")
        Q = np.empty((n, n), order="F") if want_q else None
        wr = np.empty(max(n, 1))
        wi = np.empty(max(n, 1))
        info = ctypes.c_int(0)
        lat = ctypes.c_double(0.0)
        rc = load().schur_poll(self._s, ctypes.c_uint64(ticket),
                               S.ctypes.data if n else None, max(1, n),
                               Q.ctypes.data if (want_q and n) else None, max(1, n),
                               wr.ctypes.data, wi.ctypes.data, ctypes.byref(info),
                               ctypes.byref(lat))
        if rc == 1:
            return None
        if rc != 0:
            raise RuntimeError("schur_poll failed: %d" % rc)
        return S, Q, wr[:n] + 1j * wi[:n], info.value, lat.value

    def stats(self):
        st = ServerStats()
        load().schur_server_get_stats(self._s, ctypes.byref(st))
        return st.as_dict()

    def close(self):
        if self._s:
            load().schur_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_tuning(rows):
    """Install a tuning table: rows of dicts with nmax, ns, nb, step, the
    early-deflation window nw and its sweep-skip percentage nibble
    (ascending nmax)."""
    lib = load()
    k = len(rows)
    IA = ctypes.c_int * max(k, 1)
    rc = lib.schur_set_tuning(k, IA(*[r["nmax"] for r in rows]), IA(*[r["ns"] for r in rows]),
                              IA(*[r["nb"] for r in rows]), IA(*[r.get("step", 0) for r in rows]),
                              IA(*[r.get("nw", 0) for r in rows]),
                              IA(*[r.get("nibble", 0) for r in rows]),
                              IA(*[r.get("tile", 0) for r in rows]))
    if rc != 0:
        raise ValueError("invalid tuning table (rc=%d)" % rc)


def load_tuning(path):
    """Read a tuning table written by the autotuner and install it."""
    import json

    with open(path) as f:
        rows = json.load(f)["table"]
    set_tuning(rows)
    return rows


def plan_sweep(ktop, kbot, npair, nb, step=0):
    """Host-only window schedule of one sweep: list of (t, group, p, ws, tau0, tau1, nb)."""
    lib = load()
    k = lib.schur_plan_sweep(int(ktop), int(kbot), int(npair), int(nb), int(step), None, 0)
    if k < 0:
        raise ValueError("bad schedule arguments")
    buf = (ctypes.c_int * (7 * max(k, 1)))()
    lib.schur_plan_sweep(int(ktop), int(kbot), int(npair), int(nb), int(step), buf, k)
    return [tuple(buf[7 * i:7 * i + 7]) for i in range(k)]


def plan_split(lo, hi, nw, first):
    """Host-only window tiling of a parallel early-deflation pass over the
    block [lo, hi]: list of (start, order), top to bottom."""
    lib = load()
    k = lib.schur_plan_split(int(lo), int(hi), int(nw), int(first), None, 0)
    if k < 0:
        raise ValueError("bad tiling arguments")
    buf = (ctypes.c_int * (2 * max(k, 1)))()
    lib.schur_plan_split(int(lo), int(hi), int(nw), int(first), buf, k)
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(k)]


def select_windows(starts, orders, weights):
    """Host-only window selection of a pass: indices of the disjoint
    candidate windows of largest total weight, in increasing start order."""
    lib = load()
    c = len(starts)
    IA = ctypes.c_int * max(c, 1)
    DA = ctypes.c_double * max(c, 1)
    out = IA()
    k = lib.schur_select_windows(c, IA(*starts), IA(*orders), DA(*weights), out)
    if k < 0:
        raise ValueError("bad selection arguments")
    return [out[i] for i in range(k)]


def split_weight(split, nf, top, below):
    """Host-only candidate weight of a window of a pass (0: not a candidate)."""
    return load().schur_split_weight(int(split), int(nf), int(top), int(below))
