"""Checkers for Schur forms (test infrastructure, numpy float64).

The result of the Schur reduction is not unique (eigenvalue order on the
diagonal, signs of Q's columns, off-diagonal entries of S), so parity with
the oracle is judged on what is unique: backward error, orthogonality,
quasi-triangular structure with standardised 2x2 blocks, and the eigenvalue
multiset.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linear_sum_assignment

U = 2.0 ** -53


def residual(H, Q, S):
    H = np.triu(np.asarray(H), -1)
    return np.linalg.norm(H - Q @ S @ Q.T) / max(np.linalg.norm(H), np.finfo(float).tiny)


def orthogonality(Q):
    n = Q.shape[0]
    return np.linalg.norm(Q.T @ Q - np.eye(n))


def structure_errors(S, wr=None, wi=None):
    """List of violations of the standardised real Schur form."""
    S = np.asarray(S)
    n = S.shape[0]
    errs = []
    if n > 2 and np.any(np.tril(S, -2) != 0.0):
        errs.append("nonzero below the first subdiagonal")
    k = 0
    while k < n:
        if k + 1 < n and S[k + 1, k] != 0.0:
            if k + 2 < n and S[k + 2, k + 1] != 0.0:
                errs.append("overlapping 2x2 blocks at %d" % k)
            a, b, c, d = S[k, k], S[k, k + 1], S[k + 1, k], S[k + 1, k + 1]
            if a != d:
                errs.append("2x2 block at %d: unequal diagonal %r %r" % (k, a, d))
            if not (b * c < 0.0):
                errs.append("2x2 block at %d: b*c >= 0" % k)
            if wr is not None:
                if wr[k] != a or wr[k + 1] != d or not (wi[k] > 0 and wi[k + 1] == -wi[k]):
                    errs.append("2x2 block at %d: wr/wi mismatch" % k)
            k += 2
        else:
            if wr is not None and (wr[k] != S[k, k] or wi[k] != 0.0):
                errs.append("1x1 block at %d: wr/wi mismatch" % k)
            k += 1
    return errs


def match_eigs(a, b):
    """Optimal one-to-one matching of two eigenvalue multisets; returns the
    per-pair absolute distances (in the order of ``a``)."""
    a = np.asarray(a, dtype=complex)
    b = np.asarray(b, dtype=complex)
    assert a.shape == b.shape
    if a.size == 0:
        return np.zeros(0)
    cost = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(cost)
    out = np.empty(a.size)
    out[r] = cost[r, c]
    return out


def eig_condition(H):
    """Eigenvalue condition numbers 1/|y^H x| from scipy's left/right vectors."""
    import scipy.linalg as sla

    w, vl, vr = sla.eig(H, left=True, right=True)
    s = np.abs(np.sum(vl.conj() * vr, axis=0))
    s /= np.linalg.norm(vl, axis=0) * np.linalg.norm(vr, axis=0)
    return w, 1.0 / np.maximum(s, 1e-300)


def kappa_tolerance(H, w_ref, kappa, factor=10.0):
    """Per-eigenvalue bound factor * n * u * kappa_i * ||H||_F."""
    n = H.shape[0]
    return factor * n * U * kappa * np.linalg.norm(H)


def eig_rel_tol(lam, H, rel=1e-9):
    """|dl| <= rel * max(|l|, ||H||_F / sqrt(n)) for well-conditioned spectra."""
    n = H.shape[0]
    return rel * np.maximum(np.abs(lam), np.linalg.norm(H) / np.sqrt(max(n, 1)))
