"""Orthogonality that LAPACK's own Schur reduction reaches on the full-size
inputs (tolerance reference for the large-order GPU tests; not an expected
value of any result).

The stated bar ||Q^T Q - I||_F <= 1e-12 is unscaled, while the rounding error
of any backward-stable QR algorithm's Q grows with the order: at n = 16384,
n u is already 1.8e-12.  This script runs LAPACK (``scipy.linalg.schur``,
i.e. xGEES; on an input that is already upper Hessenberg its Hessenberg
reduction is the identity, so the figure is that of xHSEQR with Schur vectors)
on the same seeded matrices the tests use and writes the Frobenius
orthogonality of its Schur vectors and its relative backward error to
``lapack_orthogonality.json``.  The GPU tests accept an orthogonality up to
``max(1e-12, 2 * LAPACK's)`` at the same order and input.

Run:  python tests/golden/lapack_orthogonality.py   (about 10 minutes on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_1905_04975_amd import inputs  # noqa: E402

CASES = [
    # (key, order, recipe)
    ("normal_n4096_seed3", 4096, "normal"),
    ("law_n4096_seed6", 4096, "law"),
    ("normal_n8192_seed3", 8192, "normal"),
    ("law_n8192_seed6", 8192, "law"),
    ("normal_n16384_seed3", 16384, "normal"),
    ("law_n16384_seed6", 16384, "law"),
]


def make(n, recipe):
    if recipe == "normal":
        return inputs.hessenberg_normal(n, inputs.SEED_N16384)
    return inputs.paper_like_law(n, inputs.SEED_PAPER_LIKE)


def main():
    out = {}
    for key, n, recipe in CASES:
        H = make(n, recipe)
        t0 = time.time()
        T, Z = sla.schur(H, output="real")
        dt = time.time() - t0
        E = Z.T @ Z
        E[np.diag_indices(n)] -= 1.0
        orth = float(np.linalg.norm(E))
        del E
        res = float(np.linalg.norm(H - Z @ T @ Z.T) / np.linalg.norm(H))
        out[key] = {"n": n, "recipe": recipe, "orthogonality": orth, "residual": res,
                    "seconds": round(dt, 1)}
        print(key, out[key], flush=True)
    out["_how"] = ("scipy.linalg.schur(H, output='real') (LAPACK xGEES via OpenBLAS) on "
                   "inputs.hessenberg_normal(n, 3) and inputs.paper_like_law(n, 6); "
                   "orthogonality = ||Z^T Z - I||_F, residual = ||H - Z T Z^T||_F / ||H||_F")
    with open(os.path.join(HERE, "lapack_orthogonality.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
