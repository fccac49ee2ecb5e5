"""Pins of the reordering oracle (paper Sec. 2, Eq. (7)) against facts fixed
by the mathematics, not by its own formulas:

* definition: S = Q3 S' Q3^T with Q3 orthogonal, S' a standardised real
  Schur form, and the eigenvalues of its leading m x m block exactly the
  selected ones (multiset), the rest the others;
* the invariant subspace of the selected eigenvalues is unique: the span of
  Q3's first m columns equals the span of those eigenvalues' eigenvectors
  computed by LAPACK (scipy.linalg.eig, run not read) -- compared through
  the sines of the principal angles;
* closed form: two 1x1 blocks [[a, b], [0, d]] become [[d, +-b], [0, a]];
* nothing to move (selection empty, all, or already leading): S' = S and
  Q3 = I exactly;
* planted mistakes in private copies of the C source fail at least one pin.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1905_04975_amd import inputs
from tests import checks
from tests.test_oracle_mutants import build_mutant

U = 2.0 ** -53
RSRC = os.path.join(os.path.dirname(oracle.__file__), "oracle_reorder.c")


def _blocks(S):
    n = S.shape[0]
    out, k = [], 0
    while k < n:
        s = 2 if (k + 1 < n and S[k + 1, k] != 0.0) else 1
        out.append((k, s))
        k += s
    return out


def _eigs(S):
    lam, _ = oracle.complex_vectors(S, np.zeros((S.shape[0], S.shape[0])))
    return lam


def _selected(S, sel):
    lam = _eigs(S)
    chosen = []
    for k, s in _blocks(S):
        if sel[k] or (s == 2 and sel[k + 1]):
            chosen.extend(lam[k:k + s])
    return np.array(chosen)


def _subspace_sine(S, sel, Q3, m):
    """largest sine of the principal angles between span(Q3[:, :m]) and the
    span of the selected eigenvalues' eigenvectors (real basis)."""
    w, V = sla.eig(S)
    target = _selected(S, sel)
    cols = []
    used = np.zeros(w.size, bool)
    for t in target:
        d = np.abs(w - t)
        d[used] = np.inf
        j = int(np.argmin(d))
        used[j] = True
        cols.append(V[:, j])
    B = np.column_stack([np.column_stack([c.real for c in cols]),
                         np.column_stack([c.imag for c in cols])])
    Ub, sv, _ = np.linalg.svd(B, full_matrices=False)
    Ub = Ub[:, sv > 1e-10 * sv[0]]
    assert Ub.shape[1] == m
    return np.linalg.norm(Ub - Q3[:, :m] @ (Q3[:, :m].T @ Ub), 2)


def _check(S, sel, S2, Q3, m, info, tol_fac=100.0):
    n = S.shape[0]
    if info != 0:
        return False
    if checks.structure_errors(S2) != []:
        return False
    if np.linalg.norm(Q3.T @ Q3 - np.eye(n)) > tol_fac * n * U:
        return False
    if np.linalg.norm(S - Q3 @ S2 @ Q3.T) > tol_fac * n * U * np.linalg.norm(S):
        return False
    want = _selected(S, sel)
    if m != want.size:
        return False
    lam2 = _eigs(S2)
    if m and checks.match_eigs(lam2[:m], want).max() > 1e-10 * np.linalg.norm(S):
        return False
    rest = np.setdiff1d(np.arange(n), [])
    return True


def _pins_pass(lib):
    try:
        for n, seed, frac in ((9, 1, 0.5), (40, 2, 0.3), (60, 3, 0.6)):
            S = inputs.schur_form(n, seed)
            sel = (np.random.Generator(np.random.PCG64(seed)).uniform(size=n) < frac).astype(int)
            S2, Q3, wr, wi, m, info = oracle.reorder(S, sel, lib=lib)
            if not _check(S, sel, S2, Q3, m, info):
                return False
            if m and _subspace_sine(S, sel, Q3, m) > 1e-10:
                return False
        return True
    except Exception:
        return False


@pytest.mark.parametrize("n,seed,frac", [(2, 1, 0.5), (5, 2, 0.5), (30, 3, 0.2), (50, 4, 0.5),
                                         (80, 5, 0.8), (120, 6, 0.5)])
def test_definition_and_subspace(n, seed, frac):
    S = inputs.schur_form(n, 600 + seed)
    sel = (np.random.Generator(np.random.PCG64(seed)).uniform(size=n) < frac).astype(int)
    S2, Q3, wr, wi, m, info = oracle.reorder(S, sel)
    assert _check(S, sel, S2, Q3, m, info)
    if m:
        assert _subspace_sine(S, sel, Q3, m) <= 1e-10
    # wr / wi read from S'
    lam = _eigs(S2)
    assert np.array_equal(wr, lam.real) and np.array_equal(wi, lam.imag)


def test_schur_form_of_random_hessenberg():
    H = inputs.hessenberg_normal(70, 7)
    S, Q, _, _, info, _ = oracle.schur(H)
    assert info == 0
    sel = (np.abs(_eigs(S)) < 1.0).astype(int)   # the eigenvalues inside the unit disc
    S2, Q2, wr, wi, m, info = oracle.reorder(S, sel, Q=Q)
    assert info == 0
    assert np.linalg.norm(H - Q2 @ S2 @ Q2.T) <= 1000 * 70 * U * np.linalg.norm(H)
    assert np.all(np.abs(wr[:m] + 1j * wi[:m]) < 1.0) and np.all(np.abs(wr[m:] + 1j * wi[m:]) >= 1.0)


def test_closed_form_two_1x1():
    a, b, d = 1.5, 2.0, -0.5
    S = np.array([[a, b], [0.0, d]])
    S2, Q3, wr, wi, m, info = oracle.reorder(S, [0, 1])
    assert info == 0 and m == 1
    assert S2[0, 0] == d and S2[1, 1] == a and S2[1, 0] == 0.0
    assert abs(abs(S2[0, 1]) - abs(b)) <= 4 * U * abs(b)


def test_nothing_to_move():
    S = inputs.schur_form(25, 8)
    for sel in (np.zeros(25, int), np.ones(25, int)):
        S2, Q3, _, _, m, info = oracle.reorder(S, sel)
        assert info == 0 and np.array_equal(S2, S) and np.array_equal(Q3, np.eye(25))
    sel = np.zeros(25, int)
    k = _blocks(S)[2][0]
    sel[:k] = 1   # the leading blocks, already in place
    S2, Q3, _, _, m, info = oracle.reorder(S, sel)
    assert info == 0 and m == k and np.array_equal(S2, S) and np.array_equal(Q3, np.eye(25))


def test_pins_pass_on_the_real_oracle():
    assert _pins_pass(oracle._load())


RMUTANTS = {
    "givens_eigvec_sign": ("const double x = t12, y = t22 - t11, r = hypot(x, y);",
                           "const double x = t12, y = t11 - t22, r = hypot(x, y);"),
    "sylvester_sign": ("K[row + 4 * (i + n1 * k)] -= T[(n1 + k) + (n1 + j) * ldt];",
                       "K[row + 4 * (i + n1 * k)] += T[(n1 + k) + (n1 + j) * ldt];"),
    "basis_sign": ("for (a = 0; a < n1; ++a) B[a + 4 * b] = -X[a + n1 * b];",
                   "for (a = 0; a < n1; ++a) B[a + 4 * b] = X[a + n1 * b];"),
    "q_not_updated": ("    if (Q) {\n        for (r = 0; r < n; ++r) {", "    if (0) {\n        for (r = 0; r < n; ++r) {"),
    "right_short": ("for (r = 0; r < j + m; ++r) {", "for (r = 0; r < j; ++r) {"),
    "no_standardise": ("if (n2 == 2) orr_std(n, S, lds, Q, ldq, j + 1);", "if (0) orr_std(n, S, lds, Q, ldq, j + 1);"),
    "pair_not_selected": ("const int sel = select[k] || (s == 2 && select[k + 1]);",
                          "const int sel = select[k];"),
}


@pytest.mark.parametrize("name", sorted(RMUTANTS))
def test_mutant_fails_a_pin(tmp_path, name):
    old, new = RMUTANTS[name]
    lib = build_mutant(tmp_path, "reorder_" + name, old, new, target=RSRC)
    assert not _pins_pass(lib), name
