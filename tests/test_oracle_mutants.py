"""The oracle's pins are strong enough to catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle's C source
(a dropped term, a wrong sign or index, a shortened loop range), builds it
on the CPU and shows that at least one pin fails on it.  The real oracle
passes the same pins (see test_oracle.py).
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1905_04975_amd import inputs
from tests import checks
from tests.test_oracle import _cyclic, second_adhoc_step_error

U = 2.0 ** -53
ODIR = os.path.dirname(oracle.__file__)
SRC = os.path.join(ODIR, "oracle_schur.c")
SOURCES = [os.path.join(ODIR, f) for f in ("oracle_schur.c", "oracle_hess.c", "oracle_evec.c",
                                                  "oracle_reorder.c")]

MUTANTS = {
    "shift_product_sign": ("- s * h00 + t;", "- s * h00 - t;"),
    "dropped_h01h10": ("h00 * h00 + h01 * h10", "h00 * h00"),
    "wrong_index_y": ("h10 * (h00 + h11 - s)", "h10 * (h00 + h00 - s)"),
    "transposed_z": ("double z = h10 * h21;", "double z = h01 * h21;"),
    "short_right_update": ("rmax = (r + 3 < i) ? r + 3 : i;", "rmax = (r + 2 < i) ? r + 2 : i;"),
    "left_update_skips_col": ("orc_left(H, ldh, r, nr, r, n - 1", "orc_left(H, ldh, r, nr, r + 1, n - 1"),
    "tau_sign": ("*tau = (b - x) / b;", "*tau = (x - b) / b;"),
    "loose_deflation": ("if (sub <= ORC_ULP * tst) {", "if (sub <= 1e-6 * tst) {"),
    "rotation_sign": ("*nc = -sn * t11 + cs * t21;", "*nc = sn * t11 + cs * t21;"),
    "q_skips_last_reflector": ("if (Q) orc_right(Q, ldq, r, nr, 0, n - 1", "if (Q && nr == 3) orc_right(Q, ldq, r, nr, 0, n - 1"),
    "complex_wi": ("double wi = sqrt(fabs(nb)) * sqrt(fabs(nc));", "double wi = sqrt(fabs(nb)) * sqrt(fabs(nb));"),
    "householder_v3": ("*v3 = z / d;", "*v3 = z / b;"),
    # the second ad-hoc shift (top of the block, reading R7)
    "adhoc2_row_index": ("w = fabs(HX(l + 1, l)) + fabs(HX(l + 2, l + 1));",
                         "w = fabs(HX(l + 1, l)) + fabs(HX(l + 2, l));"),
    "adhoc2_dropped_term": ("w = fabs(HX(l + 1, l)) + fabs(HX(l + 2, l + 1));",
                            "w = fabs(HX(l + 1, l));"),
    "adhoc2_e_sign": ("e = HX(l, l) + 0.75 * w;", "e = HX(l, l) - 0.75 * w;"),
    "adhoc2_e_diag": ("e = HX(l, l) + 0.75 * w;", "e = HX(l + 1, l + 1) + 0.75 * w;"),
    "adhoc2_skipped": ("if (its == 10 || its == 20) {", "if (its == 10) {"),
}


def build_mutant(tmp_path, name, old, new, target=SRC):
    """The oracle library with one replacement planted in a private copy of
    the source `target` (the other sources unchanged)."""
    src = open(target).read()
    assert src.count(old) == 1, name
    path = tmp_path / ("m_%s.c" % name)
    path.write_text(src.replace(old, new))
    srcs = [str(path) if f == target else f for f in SOURCES]
    so = tmp_path / ("m_%s.so" % name)
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-o", str(so), *srcs, "-lm"])
    return oracle._bind(str(so))


def _build_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    return build_mutant(tmp_path, name, old, new)


def _pins_pass(lib):
    """A compact run of the pins; returns False as soon as one fails."""
    try:
        # 2x2 closed forms
        for (a, b, c, d) in [(4.0, 1.0, 2.0, 3.0), (1.0, 3.0, -2.0, 0.5), (0.3, -2.0, 1.5, -0.7)]:
            o = oracle.std2x2(a, b, c, d, lib=lib)
            G = np.array([[o[4], -o[5]], [o[5], o[4]]])
            Bp = G.T @ np.array([[a, b], [c, d]]) @ G
            if not np.allclose(Bp, [[o[0], o[1]], [o[2], o[3]]], atol=1e-14):
                return False
            ref = np.roots([1.0, -(a + d), a * d - b * c])
            if checks.match_eigs(np.array([o[6] + 1j * o[7], o[8] + 1j * o[9]]), ref).max() > 1e-13:
                return False
        # implicit Q
        n = 12
        H = inputs.hessenberg_normal(n, 5)
        H1, Q = oracle.francis_step(H, 0, n - 1, 0.7, 1.9, lib=lib)
        if np.linalg.norm(Q @ H1 @ Q.T - H) > 50 * n * U * np.linalg.norm(H):
            return False
        M = H @ H - 0.7 * H + 1.9 * np.eye(n)
        if abs(abs(M[:, 0] @ Q[:, 0]) / np.linalg.norm(M[:, 0]) - 1.0) > 100 * n * U:
            return False
        # whole run: residual, orthogonality, structure, eigenvalues
        for n, seed in [(9, 1), (40, 2)]:
            H = inputs.hessenberg_normal(n, seed)
            S, Q, wr, wi, info, it = oracle.schur(H, lib=lib, itmax=60)
            if info != 0 or checks.residual(H, Q, S) > 10 * n * U or checks.orthogonality(Q) > 10 * n * U:
                return False
            if checks.structure_errors(S, wr, wi):
                return False
            w = np.linalg.eigvals(H)
            if checks.match_eigs(wr + 1j * wi, w).max() > 1e-9 * np.linalg.norm(H):
                return False
        # the second ad-hoc shift: implicit-Q check of the 20th step
        err, _ = second_adhoc_step_error(_cyclic(19), lib=lib)
        if not err <= 100 * 19 * U:
            return False
        return True
    except Exception:
        return False


def test_real_oracle_passes_compact_pins():
    assert _pins_pass(oracle._load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    lib = _build_mutant(tmp_path, name)
    assert not _pins_pass(lib), "planted mistake %s was not detected" % name
