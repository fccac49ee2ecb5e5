"""Oracle: a plain, slow CPU reference for the Schur-reduction step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library never calls it, links it or shares code with it.

The arithmetic lives in plain C files (binary64, no BLAS):

* ``oracle_schur.c`` -- the practical Francis double-shift QR iteration that
  the paper points to for the theory of the Schur reduction (Sec. 2,
  Eq. (4); Golub & Van Loan, Sec. 7.5);
* ``oracle_hess.c`` -- the Householder reduction to Hessenberg form (Sec. 2,
  Eq. (3); Golub & Van Loan, Sec. 7.4.3);
* ``oracle_evec.c`` -- eigenvectors of a real Schur form by back
  substitution with overflow protection, and their backtransform (Sec. 2,
  Eqs. (5) and (6));
* ``oracle_reorder.c`` -- reordering of a real Schur form so that selected
  eigenvalues lead, by swaps of adjacent diagonal blocks (Sec. 2, Eq. (7)).

This module only builds those files with ``gcc`` and marshals numpy arrays
(column-major, Fortran order) through ``ctypes``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("oracle_schur.c", "oracle_hess.c",
                                                 "oracle_evec.c", "oracle_reorder.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle sources into ``liboracle.so`` (gcc -O2, no fast-math)."""
    stale = not os.path.exists(_LIB) or any(
        os.path.getmtime(_LIB) < os.path.getmtime(src) for src in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-shared", "-fPIC", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path):
    """Load a compiled oracle library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_schur.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int,
                                 dp, dp, ctypes.c_int, ip]
    lib.oracle_schur.restype = ctypes.c_int
    lib.oracle_std2x2.argtypes = [ctypes.c_double] * 4 + [dp]
    lib.oracle_std2x2.restype = None
    lib.oracle_francis_step.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double]
    lib.oracle_francis_step.restype = None
    lib.oracle_hessenberg.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int]
    lib.oracle_hessenberg.restype = ctypes.c_int
    lib.oracle_eigenvectors.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                        ctypes.c_int]
    lib.oracle_eigenvectors.restype = ctypes.c_int
    lib.oracle_reorder.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, ip, dp, dp,
                                   ip]
    lib.oracle_reorder.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _bind(_LIB)
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def schur(H, Q=None, want_q=True, itmax=30, lib=None):
    """Real Schur form of upper Hessenberg ``H`` (paper Sec. 2, Eq. (4)).

    Returns ``(S, Q, wr, wi, info, iters)`` with ``H = Q S Q^T`` (``Q`` is
    ``Q_in @ Q2``; ``Q_in`` defaults to the identity).  Entries of ``H``
    below the first subdiagonal are ignored.
    """
    lib = lib or _load()
    H = np.array(H, dtype=np.float64, order="F", copy=True)
    n = H.shape[0]
    assert H.shape == (n, n)
    if want_q:
        Qm = np.eye(n, order="F") if Q is None else np.array(Q, dtype=np.float64, order="F", copy=True)
        qptr, ldq = _dptr(Qm), max(1, n)
    else:
        Qm, qptr, ldq = None, None, 1
    wr = np.zeros(n)
    wi = np.zeros(n)
    iters = ctypes.c_int(0)
    info = lib.oracle_schur(n, _dptr(H) if n else None, max(1, n), qptr, ldq,
                            _dptr(wr), _dptr(wi), int(itmax), ctypes.byref(iters))
    return H, Qm, wr, wi, int(info), int(iters.value)


def std2x2(a, b, c, d, lib=None):
    """Standardise one 2x2 block; returns (a', b', c', d', cs, sn, wr1, wi1, wr2, wi2)."""
    lib = lib or _load()
    out = np.zeros(10)
    lib.oracle_std2x2(float(a), float(b), float(c), float(d), _dptr(out))
    return tuple(float(x) for x in out)


def francis_step(H, l, i, s, t, Q=None, lib=None):
    """One Francis double-shift step on block l..i (0-based) with shift sum
    ``s`` and product ``t``; returns the new (H, Q)."""
    lib = lib or _load()
    H = np.array(H, dtype=np.float64, order="F", copy=True)
    n = H.shape[0]
    Qm = np.eye(n, order="F") if Q is None else np.array(Q, dtype=np.float64, order="F", copy=True)
    lib.oracle_francis_step(n, _dptr(H), n, _dptr(Qm), n, int(l), int(i), float(s), float(t))
    return H, Qm


def eigenvalues(H, itmax=30):
    """Eigenvalues (complex array, diagonal order) of upper Hessenberg ``H``."""
    _, _, wr, wi, info, _ = schur(H, want_q=False, itmax=itmax)
    return wr + 1j * wi, info


def francis_step_inplace(H, Q, l, i, s, t, lib=None):
    """In-place variant of ``francis_step`` on Fortran-ordered float64 arrays
    (``Q`` may be None); used to time the oracle on large inputs."""
    lib = lib or _load()
    assert H.flags.f_contiguous and H.dtype == np.float64
    n = H.shape[0]
    if Q is not None:
        assert Q.flags.f_contiguous and Q.dtype == np.float64
    lib.oracle_francis_step(n, _dptr(H), n, _dptr(Q) if Q is not None else None, n,
                            int(l), int(i), float(s), float(t))


def hessenberg(A, Q=None, want_q=True, lib=None):
    """Householder reduction of the dense matrix ``A`` to upper Hessenberg
    form (paper Sec. 2, Eq. (3)).  Returns ``(H, Q)`` with ``A = Q H Q^T``
    (``Q`` is ``Q_in @ Q1``; ``Q_in`` defaults to the identity)."""
    lib = lib or _load()
    H = np.array(A, dtype=np.float64, order="F", copy=True)
    n = H.shape[0]
    assert H.shape == (n, n)
    if want_q:
        Qm = np.eye(n, order="F") if Q is None else np.array(Q, dtype=np.float64, order="F",
                                                               copy=True)
        qptr = _dptr(Qm)
    else:
        Qm, qptr = None, None
    rc = lib.oracle_hessenberg(n, _dptr(H) if n else None, max(1, n), qptr, max(1, n))
    if rc != 0:
        raise MemoryError("oracle_hessenberg: workspace")
    return H, Qm


def eigenvectors(S, Q=None, lib=None):
    """Eigenvectors of the real Schur form ``S`` (paper Sec. 2, Eq. (5)) in
    LAPACK's real layout (a complex pair's real and imaginary parts in two
    adjacent columns), backtransformed with ``Q`` when given (Eq. (6)), each
    scaled to largest |Re| + |Im| = 1."""
    lib = lib or _load()
    S = np.array(S, dtype=np.float64, order="F", copy=True)
    n = S.shape[0]
    X = np.zeros((n, n), order="F")
    qptr = None
    if Q is not None:
        Qm = np.array(Q, dtype=np.float64, order="F", copy=True)
        qptr = _dptr(Qm)
    rc = lib.oracle_eigenvectors(n, _dptr(S) if n else None, max(1, n), qptr, max(1, n),
                                 _dptr(X) if n else None, max(1, n))
    if rc != 0:
        raise MemoryError("oracle_eigenvectors: workspace")
    return X


def complex_vectors(S, X):
    """Columns of LAPACK's real layout as complex vectors, with eigenvalues."""
    n = S.shape[0]
    lam = np.zeros(n, dtype=complex)
    V = np.zeros((X.shape[0], n), dtype=complex)
    k = 0
    while k < n:
        if k + 1 < n and S[k + 1, k] != 0.0:
            wi = np.sqrt(abs(S[k, k + 1])) * np.sqrt(abs(S[k + 1, k]))
            lam[k], lam[k + 1] = S[k, k] + 1j * wi, S[k, k] - 1j * wi
            V[:, k] = X[:, k] + 1j * X[:, k + 1]
            V[:, k + 1] = X[:, k] - 1j * X[:, k + 1]
            k += 2
        else:
            lam[k] = S[k, k]
            V[:, k] = X[:, k]
            k += 1
    return lam, V


def reorder(S, select, Q=None, want_q=True, lib=None):
    """Reorder the real Schur form ``S`` so that the selected eigenvalues
    lead (paper Sec. 2, Eq. (7)).  Returns ``(S', Q, wr, wi, m, info)``
    with ``S = Q3 S' Q3^T`` (``Q`` is ``Q_in @ Q3``), ``m`` the number of
    selected eigenvalues, ``info`` 1 when a swap was rejected."""
    lib = lib or _load()
    S = np.array(S, dtype=np.float64, order="F", copy=True)
    n = S.shape[0]
    sel = np.ascontiguousarray(np.asarray(select, dtype=np.int32).reshape(n))
    if want_q:
        Qm = np.eye(n, order="F") if Q is None else np.array(Q, dtype=np.float64, order="F",
                                                               copy=True)
        qptr = _dptr(Qm)
    else:
        Qm, qptr = None, None
    wr = np.zeros(n)
    wi = np.zeros(n)
    m = ctypes.c_int(0)
    info = lib.oracle_reorder(n, _dptr(S) if n else None, max(1, n), qptr, max(1, n),
                              sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(wr),
                              _dptr(wi), ctypes.byref(m))
    return S, Qm, wr, wi, int(m.value), int(info)
