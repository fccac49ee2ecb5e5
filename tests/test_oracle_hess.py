"""Pins of the Hessenberg-reduction oracle (paper Sec. 2, Eq. (3)) against
facts fixed by the mathematics, not by its own formulas:

* definition: H upper Hessenberg (exact zeros), Q orthogonal, A = Q H Q^T,
  Q e_1 = e_1 (the reflectors act on rows and columns 1..n-1);
* implicit-Q theorem: the leading k columns of Q span the Krylov space
  K_k(A, e_1) = span{e_1, A e_1, ..., A^(k-1) e_1};
* special cases: an input already in Hessenberg form is a fixed point
  (Q = I exactly); a symmetric input gives a symmetric tridiagonal H with
  the same eigenvalues (numpy eigvalsh); n = 3 has a closed form;
* spectrum: a matrix with a prescribed normal spectrum keeps it;
* LAPACK's Householder reduction (scipy.linalg.hessenberg, run not read)
  uses the same sign convention, so H and Q agree elementwise to rounding;
* accumulation into a given Q;
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
HSRC = os.path.join(os.path.dirname(oracle.__file__), "oracle_hess.c")


def _dense(n, seed):
    return np.random.Generator(np.random.PCG64(seed)).uniform(-1.0, 1.0, size=(n, n))


def _definition_ok(A, H, Q, tol_fac=50.0):
    n = A.shape[0]
    nrm = np.linalg.norm(A)
    if n > 2 and np.any(np.tril(H, -2) != 0.0):
        return False
    if np.linalg.norm(Q.T @ Q - np.eye(n)) > tol_fac * n * U:
        return False
    if np.linalg.norm(A - Q @ H @ Q.T) > tol_fac * n * U * nrm:
        return False
    if n >= 1 and (Q[0, 0] != 1.0 or np.any(Q[0, 1:] != 0.0) or np.any(Q[1:, 0] != 0.0)):
        return False
    return True


def _krylov_ok(A, Q, kmax=6):
    """Q(:, :k) spans K_k(A, e_1): the residual of projecting each Krylov
    vector (normalised) onto the first k columns is at rounding level."""
    n = A.shape[0]
    x = np.zeros(n)
    x[0] = 1.0
    for k in range(1, min(kmax, n) + 1):
        Qk = Q[:, :k]
        r = x - Qk @ (Qk.T @ x)
        if np.linalg.norm(r) > 1e-10 * np.linalg.norm(x):
            return False
        x = A @ x
        x /= np.linalg.norm(x)
    return True


def _pins_pass(lib):
    try:
        for n, seed in ((3, 1), (17, 2), (40, 3)):
            A = _dense(n, seed)
            H, Q = oracle.hessenberg(A, lib=lib)
            if not _definition_ok(A, H, Q) or not _krylov_ok(A, Q):
                return False
            Hl, Ql = sla.hessenberg(A, calc_q=True)
            if np.abs(H - Hl).max() > 1e-12 * np.linalg.norm(A):
                return False
        S = _dense(12, 4)
        S = S + S.T
        H, Q = oracle.hessenberg(S, lib=lib)
        T = np.triu(np.tril(H, 1), -1)
        if np.abs(np.linalg.eigvalsh(T) - np.linalg.eigvalsh(S)).max() > 1e-12 * np.linalg.norm(S):
            return False
        return True
    except Exception:
        return False


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 9, 33, 64, 101])
def test_definition_and_krylov(n):
    A = _dense(n, 100 + n)
    H, Q = oracle.hessenberg(A)
    if n == 0:
        return
    assert _definition_ok(A, H, Q)
    assert _krylov_ok(A, Q)


def test_hessenberg_input_is_a_fixed_point():
    H0 = inputs.hessenberg_normal(30, 7)
    H, Q = oracle.hessenberg(H0)
    assert np.array_equal(H, H0)
    assert np.array_equal(Q, np.eye(30))


def test_n3_closed_form():
    A = np.array([[2.0, -1.0, 0.5], [3.0, 1.0, 4.0], [-4.0, 2.0, 1.0]])
    H, Q = oracle.hessenberg(A)
    # one reflector on rows/columns 1, 2 maps (3, -4) to -sign(3) * 5
    assert abs(H[1, 0] - (-5.0)) <= 4 * U * 5
    assert H[2, 0] == 0.0
    assert H[0, 0] == A[0, 0]
    # the reflector is the symmetric orthogonal matrix sending (3, -4)/5 to -e_1
    P = Q[1:, 1:]
    assert np.allclose(P, P.T, atol=1e-15) and np.allclose(P @ np.array([3.0, -4.0]), [-5.0, 0.0],
                                                             atol=1e-14)
    assert abs(np.trace(H) - np.trace(A)) <= 8 * U * np.linalg.norm(A)


def test_symmetric_gives_tridiagonal():
    S = _dense(60, 8)
    S = S + S.T
    H, Q = oracle.hessenberg(S)
    nrm = np.linalg.norm(S)
    assert np.abs(np.triu(H, 2)).max() <= 100 * 60 * U * nrm
    assert np.abs(np.diag(H, 1) - np.diag(H, -1)).max() <= 100 * 60 * U * nrm
    T = np.triu(np.tril(H, 1), -1)
    assert np.abs(np.linalg.eigvalsh(T) - np.linalg.eigvalsh(S)).max() <= 100 * 60 * U * nrm


def test_prescribed_spectrum_kept():
    n = 80
    rng = np.random.Generator(np.random.PCG64(9))
    d = rng.standard_normal(n)
    Z = inputs.haar_orthogonal(n, rng)
    A = Z @ np.diag(d) @ Z.T
    H, Q = oracle.hessenberg(A)
    ev = np.sort(np.linalg.eigvals(H).real)
    assert np.abs(ev - np.sort(d)).max() <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("n", [5, 48, 130])
def test_lapack_householder_agrees(n):
    A = _dense(n, 200 + n)
    H, Q = oracle.hessenberg(A)
    Hl, Ql = sla.hessenberg(A, calc_q=True)
    nrm = np.linalg.norm(A)
    assert np.abs(H - Hl).max() <= 50 * n * U * nrm
    assert np.abs(Q - Ql).max() <= 50 * n * U


def test_accumulates_into_given_q():
    n = 25
    A = _dense(n, 11)
    Qin = inputs.haar_orthogonal(n, np.random.Generator(np.random.PCG64(12)))
    H1, Q1 = oracle.hessenberg(A)
    H2, Q2 = oracle.hessenberg(A, Q=Qin)
    assert np.array_equal(H1, H2)
    assert np.abs(Q2 - Qin @ Q1).max() <= 50 * n * U


def test_pins_pass_on_the_real_oracle():
    assert _pins_pass(oracle._load())


HMUTANTS = {
    "alpha_sign": ("*alpha = (x[0] >= 0.0) ? -nrm : nrm;", "*alpha = (x[0] >= 0.0) ? nrm : -nrm;"),
    "beta_half": ("*beta = 2.0 / vv;", "*beta = 1.0 / vv;"),
    "right_skips_row0": ("            for (i = 0; i < n; ++i) {\n                double s = 0.0;\n"
                         "                for (j = 0; j < m; ++j) s += AX(i, k + 1 + j) * v[j];",
                         "            for (i = 1; i < n; ++i) {\n                double s = 0.0;\n"
                         "                for (j = 0; j < m; ++j) s += AX(i, k + 1 + j) * v[j];"),
    "v_index_shift": ("for (i = 1; i < m; ++i) v[i] = x[i] / d;",
                      "for (i = 1; i < m; ++i) v[i] = x[i - 1] / d;"),
    "q_transposed": ("for (j = 0; j < m; ++j) s += QX(i, k + 1 + j) * v[j];",
                     "for (j = 0; j < m; ++j) s += QX(k + 1 + j, i) * v[j];"),
    "short_last_column": ("for (k = 0; k + 2 < n; ++k) {", "for (k = 0; k + 3 < n; ++k) {"),
    "scale_dropped": ("nrm = scale * sqrt(t0 * t0 + ss);", "nrm = sqrt(t0 * t0 + ss);"),
}


@pytest.mark.parametrize("name", sorted(HMUTANTS))
def test_mutant_fails_a_pin(tmp_path, name):
    old, new = HMUTANTS[name]
    lib = build_mutant(tmp_path, "hess_" + name, old, new, target=HSRC)
    assert not _pins_pass(lib), name
