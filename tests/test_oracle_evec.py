"""Pins of the eigenvector oracle (paper Sec. 2, Eqs. (5) and (6)) against
facts fixed by the mathematics, not by its own formulas:

* definition: S y = lambda y for every returned vector (relative residual at
  rounding level), and after the backtransform A x = lambda x for
  A = Q S Q^T;
* closed forms: 2x2 triangular and standardised 2x2 blocks;
* LAPACK's eigenvectors (scipy.linalg.eig, run not read) agree up to a
  complex factor (length and phase are conventions);
* overflow protection: a triangular S whose eigenvectors grow by 1e39 per
  row still gives finite vectors that satisfy the definition (plain back
  substitution overflows);
* layout: real eigenvectors in one column, complex pairs as (Re, Im);
* planted mistakes in private copies of the C source fail at least one pin.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1905_04975_amd import inputs
from tests.test_oracle_mutants import build_mutant

U = 2.0 ** -53
ESRC = os.path.join(os.path.dirname(oracle.__file__), "oracle_evec.c")


def _schur(n, seed, prescribed=False):
    if prescribed:
        H, _ = inputs.prescribed(n, seed)
    else:
        H = inputs.hessenberg_normal(n, seed)
    S, Q, _, _, info, _ = oracle.schur(H)
    assert info == 0
    return H, S, Q


def _residual(M, lam, V):
    """max_k ||M v_k - lambda_k v_k|| / (||M|| ||v_k||)."""
    R = M @ V - V * lam[None, :]
    return (np.linalg.norm(R, axis=0) / (np.linalg.norm(M) * np.linalg.norm(V, axis=0))).max()


def _aligned(v, ref):
    """v times the complex factor that brings it closest to ref (the phase
    and length of an eigenvector are conventions; its direction is not)."""
    return v * (np.vdot(v, ref) / np.vdot(v, v))


def _overflow_cases(n=40):
    """Triangular S whose eigenvectors grow by about 1e39 per row (large
    off-diagonal entries over close eigenvalues), and one whose eigenvalues
    are distinct but all within 1e-298 of zero (tiny pivots)."""
    d = 1.0 + 1e-9 * np.arange(n)
    S1 = np.triu(np.full((n, n), 1e30), 1) + np.diag(d)
    S2 = np.triu(np.ones((n, n)), 1) + np.diag(1e-300 * (1.0 + np.arange(n)))
    return S1, S2


def _pins_pass(lib):
    try:
        for n, seed, pres in ((7, 1, False), (40, 2, False), (30, 3, True)):
            H, S, Q = _schur(n, seed, pres)
            X = oracle.eigenvectors(S, lib=lib)
            lam, V = oracle.complex_vectors(S, X)
            if not np.all(np.isfinite(X)) or _residual(S, lam, V) > 100 * n * U:
                return False
            XA = oracle.eigenvectors(S, Q=Q, lib=lib)
            lamA, VA = oracle.complex_vectors(S, XA)
            if _residual(H, lamA, VA) > 1000 * n * U:
                return False
        for S in _overflow_cases():
            X = oracle.eigenvectors(S, lib=lib)
            lam, V = oracle.complex_vectors(S, X)
            if not np.all(np.isfinite(X)) or _residual(S, lam, V) > 1e-12:
                return False
        return True
    except Exception:
        return False


@pytest.mark.parametrize("n,seed,pres", [(1, 1, False), (2, 2, False), (5, 3, False),
                                         (50, 4, False), (120, 5, False), (64, 6, True)])
def test_definition(n, seed, pres):
    H, S, Q = _schur(n, seed, pres)
    X = oracle.eigenvectors(S)
    lam, V = oracle.complex_vectors(S, X)
    assert _residual(S, lam, V) <= 100 * max(n, 1) * U
    # eigenvectors of S are zero below their block
    k = 0
    while k < n:
        s = 2 if (k + 1 < n and S[k + 1, k] != 0.0) else 1
        assert not np.any(X[k + s:, k:k + s])
        k += s
    XA = oracle.eigenvectors(S, Q=Q)
    lamA, VA = oracle.complex_vectors(S, XA)
    assert _residual(H, lamA, VA) <= 1000 * max(n, 1) * U
    # normalisation: the largest |Re| + |Im| of every vector is 1
    for V_ in (V, VA):
        m = np.max(np.abs(V_.real) + np.abs(V_.imag), axis=0)
        assert np.allclose(m, 1.0, rtol=0, atol=4 * U)


def test_closed_forms():
    # triangular 2x2: eigenvector of d is (b / (d - a), 1), scaled
    a, b, d = 2.0, 3.0, -1.0
    X = oracle.eigenvectors(np.array([[a, b], [0.0, d]]))
    v = np.array([b / (d - a), 1.0])
    v = v / np.max(np.abs(v))
    assert np.allclose(X[:, 0], [1.0, 0.0]) and np.allclose(X[:, 1], v, atol=4 * U)
    # standardised 2x2 block [[a, b], [c, a]], b c < 0: lambda = a + i sqrt(-b c)
    a, b, c = 0.5, 4.0, -1.0
    X = oracle.eigenvectors(np.array([[a, b], [c, a]]))
    wi = np.sqrt(-b * c)
    v = X[:, 0] + 1j * X[:, 1]
    M = np.array([[a, b], [c, a]])
    assert np.allclose(M @ v, (a + 1j * wi) * v, atol=1e-15)
    # |b| >= |c|: v = (1, i wi / b) scaled to largest |Re| + |Im| = 1
    w = np.array([1.0, 1j * wi / b])
    w = w / np.max(np.abs(w.real) + np.abs(w.imag))
    assert np.allclose(v, w, atol=4 * U)


@pytest.mark.parametrize("n,seed", [(20, 7), (90, 8)])
def test_lapack_eigenvectors_agree(n, seed):
    H, S, Q = _schur(n, seed, prescribed=True)   # well separated, normal: well conditioned
    X = oracle.eigenvectors(S, Q=Q)
    lam, V = oracle.complex_vectors(S, X)
    w, VL = sla.eig(H)
    for k in range(n):
        j = np.argmin(np.abs(w - lam[k]))
        assert abs(w[j] - lam[k]) <= 1e-10
        assert np.abs(_aligned(VL[:, j], V[:, k]) - V[:, k]).max() <= 1e-9


@pytest.mark.parametrize("case", [0, 1])
def test_overflow_protection(case):
    S = _overflow_cases()[case]
    n = S.shape[0]
    # plain back substitution overflows on this matrix
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        y = np.zeros(n)
        y[n - 1] = 1.0
        lam = S[n - 1, n - 1]
        for r in range(n - 2, -1, -1):
            y[r] = -(S[r, r + 1:] @ y[r + 1:]) / (S[r, r] - lam)
    assert not np.all(np.isfinite(y))
    X = oracle.eigenvectors(S)
    assert np.all(np.isfinite(X))
    lam, V = oracle.complex_vectors(S, X)
    assert _residual(S, lam, V) <= 1e-12


def test_pins_pass_on_the_real_oracle():
    assert _pins_pass(oracle._load())


EMUTANTS = {
    "pair_sign": ("y[p] = 1.0; y[p + 1] = I * (wi / b);", "y[p] = 1.0; y[p + 1] = -I * (wi / b);"),
    "pivot_sign": ("const double complex d = ore_pivot(SX(r, r) - lam, smin);",
                   "const double complex d = ore_pivot(SX(r, r) + lam, smin);"),
    "no_update_scaling": ("if (rb > 0.0 && ymax > ORE_BIG / rb) ore_scale",
                          "if (0) ore_scale"),
    "no_division_scaling": ("if (fm > ORE_BIG * ore_cabs1(d)) {", "if (0) {"),
    "back_transposed": ("for (l = 0; l < m; ++l) t += QX(r, l) * y[l];",
                        "for (l = 0; l < m; ++l) t += QX(l, r) * y[l];"),
    "two_by_two_ignored": ("const int two = (r >= 1 && SX(r, r - 1) != 0.0);", "const int two = 0;"),
    "update_skips_block": ("for (l = r + 1; l < top_known; ++l) {", "for (l = r + 2; l < top_known; ++l) {"),
}


@pytest.mark.parametrize("name", sorted(EMUTANTS))
def test_mutant_fails_a_pin(tmp_path, name):
    old, new = EMUTANTS[name]
    lib = build_mutant(tmp_path, "evec_" + name, old, new, target=ESRC)
    assert not _pins_pass(lib), name
