"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds only input generation: it contains none of the Schur
method's arithmetic, so both the HIP path and the oracle can consume it.

Recipes (all numpy ``Generator(PCG64(seed))``):

* ``hessenberg_normal(n, seed)`` -- upper Hessenberg with iid N(0,1) entries
  on and above the first subdiagonal, zero below.  A full n x n draw is
  taken and then masked, so the values do not depend on traversal order.
* ``prescribed(n, seed)`` -- Hessenberg matrix with a known, perfectly
  conditioned spectrum: a block-diagonal D of 1x1 blocks d ~ N(0,1) and 2x2
  blocks [[a, b], [-b, a]] with a, b ~ U(-2, 2) (half of the eigenvalues in
  complex pairs, blocks in shuffled order) is conjugated by a Haar-random
  orthogonal Z (QR of a Gaussian matrix with the signs of diag(R) fixed) and
  reduced to Hessenberg form with LAPACK's Householder reduction
  (``scipy.linalg.hessenberg``).  The ground-truth eigenvalues are returned.
* ``paper_like(n, seed)`` -- dense entries U(-1, 1) reduced to Hessenberg
  form, the test-matrix recipe of the paper's experiments (Sec. 5).
* ``paper_like_law(n, seed)`` -- a draw from the distribution of the
  Householder Hessenberg form of a dense matrix with iid N(0, 1/3) entries
  (1/3 is the variance of U(-1, 1)), sampled directly in O(n^2): entries on
  and above the diagonal iid N(0, 1/3), subdiagonal entry (k+1, k) equal to
  sqrt(chi^2_{n-1-k} / 3).  The law is exact for Gaussian entries (each
  Householder step maps the column below the diagonal to its norm and
  leaves the rest iid Gaussian, by orthogonal invariance); for U(-1, 1)
  entries it matches the first two moments of every entry of the reduced
  form.  It stands in for ``paper_like`` at orders where the dense CPU
  reduction takes minutes (n = 16384).
* ``schur_form(n, seed, offdiag=0.3)`` -- a standardised real Schur form:
  diagonal blocks 1x1 (d ~ U(-2, 2)) and 2x2 [[a, b], [c, a]] with
  a ~ U(-2, 2), b c < 0 (|b|, |c| ~ U(0.2, 2), half of the eigenvalues in
  complex pairs, blocks in random order), entries above the blocks
  offdiag * N(0, 1) / sqrt(n), zeros below.  Input of the eigenvector step.
* ``anderson(n, seed, W=24, g=0.2)`` -- a tridiagonal matrix with strongly
  localised, well-conditioned eigenvectors: diagonal U(-W/2, W/2),
  subdiagonal e^g, superdiagonal e^-g.  It is D T D^-1 with T the symmetric
  tridiagonal matrix of the same diagonal and unit off-diagonals and
  D = diag(e^(g k)), so its eigenvalues are exactly T's (real) while the
  matrix itself is not symmetric; for g below the inverse localisation
  length the eigenvalue condition numbers stay small (at most about 1.3 at
  the defaults, n = 1500).  At W = 24 a window of 96 rows typically has
  about half of its eigenvalues coupled to neither neighbour block (at
  W = 12 most windows have too few).
* ``batch_sizes(count, lo, hi, seed)`` -- matrix orders for batched runs.

All matrices are returned column-major (Fortran order), float64.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def hessenberg_normal(n: int, seed: int) -> np.ndarray:
    rng = _rng(seed)
    a = rng.standard_normal((n, n))
    return np.asfortranarray(np.triu(a, -1))


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def prescribed(n: int, seed: int, complex_fraction: float = 0.5):
    """Return ``(H, eigs)``: Hessenberg H with the known spectrum ``eigs``."""
    import scipy.linalg as sla

    rng = _rng(seed)
    npairs = int(round(n * complex_fraction / 2.0))
    nreal = n - 2 * npairs
    blocks = []
    for _ in range(npairs):
        a, b = rng.uniform(-2.0, 2.0, size=2)
        blocks.append(np.array([[a, b], [-b, a]]))
    for _ in range(nreal):
        blocks.append(np.array([[rng.standard_normal()]]))
    order = rng.permutation(len(blocks))
    d = np.zeros((n, n))
    eigs = []
    pos = 0
    for k in order:
        blk = blocks[k]
        m = blk.shape[0]
        d[pos:pos + m, pos:pos + m] = blk
        if m == 1:
            eigs.append(complex(blk[0, 0], 0.0))
        else:
            eigs.append(complex(blk[0, 0], abs(blk[0, 1])))
            eigs.append(complex(blk[0, 0], -abs(blk[0, 1])))
        pos += m
    z = haar_orthogonal(n, rng)
    a = z @ d @ z.T
    h = sla.hessenberg(a)
    h = np.triu(h, -1)
    return np.asfortranarray(h), np.array(eigs)


def paper_like(n: int, seed: int) -> np.ndarray:
    import scipy.linalg as sla

    rng = _rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(n, n))
    return np.asfortranarray(np.triu(sla.hessenberg(a), -1))


def paper_like_law(n: int, seed: int) -> np.ndarray:
    rng = _rng(seed)
    sd = 1.0 / np.sqrt(3.0)
    h = np.triu(rng.standard_normal((n, n)), 0) * sd
    if n > 1:
        df = np.arange(n - 1, 0, -1, dtype=np.float64)   # n-1, ..., 1
        h[np.arange(1, n), np.arange(n - 1)] = np.sqrt(rng.chisquare(df) / 3.0)
    return np.asfortranarray(h)


def schur_form(n: int, seed: int, offdiag: float = 0.3) -> np.ndarray:
    rng = _rng(seed)
    S = np.triu(rng.standard_normal((n, n)), 1) * (offdiag / np.sqrt(max(n, 1)))
    k = 0
    while k < n:
        if k + 1 < n and rng.uniform() < 0.5:
            a = rng.uniform(-2.0, 2.0)
            b = rng.uniform(0.2, 2.0) * (1.0 if rng.uniform() < 0.5 else -1.0)
            c = -np.sign(b) * rng.uniform(0.2, 2.0)
            S[k, k] = S[k + 1, k + 1] = a
            S[k, k + 1], S[k + 1, k] = b, c
            k += 2
        else:
            S[k, k] = rng.uniform(-2.0, 2.0)
            k += 1
    return np.asfortranarray(S)


def anderson(n: int, seed: int, W: float = 24.0, g: float = 0.2) -> np.ndarray:
    rng = _rng(seed)
    h = np.diag(rng.uniform(-W / 2.0, W / 2.0, size=n))
    if n > 1:
        k = np.arange(n - 1)
        h[k + 1, k] = np.exp(g)
        h[k, k + 1] = np.exp(-g)
    return np.asfortranarray(h)


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = _rng(seed)
    return rng.integers(lo, hi + 1, size=count)


# Seeds of the standard workloads.
SEED_N256 = 1          # N(0,1) Hessenberg, n = 256
SEED_N1024 = 2         # prescribed spectrum, n = 1024
SEED_N16384 = 3        # N(0,1) Hessenberg, n = 16384
SEED_PAPER_LIKE = 6    # dense-derived recipe (paper Sec. 5), n = 16384
SEED_BATCH_SIZES = 4   # batch of 2000, orders U{32..512}
SEED_BATCH_BASE = 40000
SEED_SERVE = 5
SEED_SERVE_BASE = 50000
