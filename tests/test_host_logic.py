"""Host logic of the library, on the CPU (no GPU calls).

The sweep planner (``schur_plan_sweep``, the same C++ code the solver uses)
is checked for the properties the windowed multishift sweep relies on:
windows of one time step are disjoint and ordered, each bulge group's chain
steps are tiled exactly once, every reflector (and the row below it that its
right update reaches) lies inside its window, and the reflector log fits.
A numpy model of the window chase driven by that schedule must reproduce
the oracle's sequential Francis double-shift steps with the same shifts
(the multishift sweep and the sequence of double-shift steps agree in exact
arithmetic; paper Sec. 3.2 describes the windowed, accumulated form).
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1905_04975_amd import inputs, schur

WMAX = 128
REFL_LDS = 1280


def _groups(npair, nb):
    g = (npair + nb - 1) // nb
    sizes = [npair // g + (1 if j < npair % g else 0) for j in range(g)]
    first = np.cumsum([0] + sizes[:-1])
    return dict(zip(first.tolist(), sizes))


@pytest.mark.parametrize("ktop,kbot,npair,nb,step", [
    (0, 299, 1, 1, 0), (0, 299, 8, 3, 0), (5, 1000, 64, 16, 0), (10, 140, 4, 2, 0),
    (0, 96, 15, 16, 0), (3, 700, 32, 5, 40), (0, 4095, 64, 24, 0), (0, 511, 16, 16, 30)])
def test_plan_invariants(ktop, kbot, npair, nb, step):
    plan = schur.plan_sweep(ktop, kbot, npair, nb, step)
    groups = _groups(npair, nb)
    by_t = {}
    for (t, g, p, ws, t0, t1, b) in plan:
        by_t.setdefault(t, []).append((p, ws))
        assert 3 <= ws <= WMAX and p >= ktop and p + ws - 1 <= kbot
        assert (t1 - t0) * b <= REFL_LDS and b == groups[g]
    for t, ws_ in by_t.items():
        ws_.sort()
        for (p0, w0), (p1, w1) in zip(ws_, ws_[1:]):
            assert p0 + w0 - 1 < p1, "windows of one time step overlap"
    for g, b in groups.items():
        mine = sorted((t0, t1, p, ws, t) for (t, gg, p, ws, t0, t1, bb) in plan if gg == g)
        tend = kbot - ktop + 3 * b - 3
        assert mine[0][0] == 0 and mine[-1][1] == tend
        for a, c in zip(mine, mine[1:]):
            assert a[1] == c[0] and c[4] == a[4] + 1
        # every active reflector of every bulge inside its window
        for (t0, t1, p, ws, _) in mine:
            for tau in range(t0, t1):
                for j in range(b):
                    K = ktop - 1 + tau - 3 * j
                    if K < ktop - 1 or K > kbot - 2:
                        continue
                    lo = max(K, ktop)
                    hi = min(K + 4, kbot)
                    assert p <= lo and hi <= p + ws - 1, (tau, j, K, p, ws)


def _house(nr, x, y, z):
    if nr == 2:
        z = 0.0
    tail = abs(y) + abs(z)
    if tail == 0:
        return None
    nrm = np.sqrt(x * x + y * y + z * z)
    beta = nrm if x < 0 else -nrm
    return np.array([1.0, y / (x - beta), z / (x - beta)])[:nr], (beta - x) / beta, beta


def _model_sweep(H, Q, ktop, kbot, shifts, nb):
    """Window chase + accumulated U + panel products, driven by the planner."""
    n = H.shape[0]
    npair = len(shifts)
    plan = schur.plan_sweep(ktop, kbot, npair, nb, 0)
    for t in sorted({r[0] for r in plan}):
        wins = [r for r in plan if r[0] == t]
        Us = []
        for (_, g, p, ws, t0, t1, b) in wins:
            W = H[p:p + ws, p:p + ws].copy()
            refl = []
            for tau in range(t0, t1):
                step_refl = []
                for j in range(b):
                    K = ktop - 1 + tau - 3 * j
                    if K < ktop - 1 or K > kbot - 2:
                        continue
                    nr = 3 if K <= kbot - 3 else 2
                    if K == ktop - 1:
                        o = ktop - p
                        s, tt = shifts[g + j]
                        x = W[o, o] ** 2 + W[o, o + 1] * W[o + 1, o] - s * W[o, o] + tt
                        y = W[o + 1, o] * (W[o, o] + W[o + 1, o + 1] - s)
                        z = W[o + 1, o] * W[o + 2, o + 1] if nr == 3 else 0.0
                    else:
                        k = K - p
                        x, y = W[k + 1, k], W[k + 2, k]
                        z = W[k + 3, k] if nr == 3 else 0.0
                    r = _house(nr, x, y, z)
                    if r is not None:
                        step_refl.append((K, nr) + r)
                for (K, nr, v, tv, beta) in step_refl:   # all left updates first
                    k = K - p
                    c0 = max(k, 0)
                    blk = W[k + 1:k + 1 + nr, c0:]
                    blk -= tv * np.outer(v, v @ blk)
                    if k >= 0:
                        W[k + 1:k + 1 + nr, k] = 0.0
                        W[k + 1, k] = beta
                for (K, nr, v, tv, beta) in step_refl:   # then the right updates
                    k = K - p
                    rl = min(K + 4, kbot) - p
                    blk = W[:rl + 1, k + 1:k + 1 + nr]
                    blk -= tv * np.outer(blk @ v, v)
                refl += step_refl
            H[p:p + ws, p:p + ws] = W
            U = np.eye(ws)
            for (K, nr, v, tv, beta) in refl:
                k = K - p
                blk = U[:, k + 1:k + 1 + nr]
                blk -= tv * np.outer(blk @ v, v)
            Us.append(U)
        for (_, g, p, ws, t0, t1, b), U in zip(wins, Us):   # left (row panel) first
            H[p:p + ws, p + ws:] = U.T @ H[p:p + ws, p + ws:]
        for (_, g, p, ws, t0, t1, b), U in zip(wins, Us):   # then right (column panel, Q)
            H[:p, p:p + ws] = H[:p, p:p + ws] @ U
            Q[:, p:p + ws] = Q[:, p:p + ws] @ U


@pytest.mark.parametrize("n,ktop,kbot,npair,nb", [(160, 0, 159, 1, 1), (220, 0, 219, 6, 3),
                                                 (260, 20, 240, 10, 4), (300, 0, 299, 8, 8)])
def test_planned_sweep_equals_sequential_double_shift_steps(n, ktop, kbot, npair, nb):
    H0 = inputs.hessenberg_normal(n, 9 + n)
    if ktop > 0:
        H0[ktop, ktop - 1] = 0.0
    if kbot < n - 1:
        H0[kbot + 1, kbot] = 0.0
    rng = np.random.default_rng(1)
    shifts = []
    for _ in range(npair):
        a, b = rng.uniform(-1, 1, 2)
        shifts.append((2 * a, a * a + b * b))
    H = H0.copy()
    Q = np.eye(n)
    _model_sweep(H, Q, ktop, kbot, shifts, nb)
    Hs = np.asfortranarray(H0.copy())
    Qs = np.asfortranarray(np.eye(n))
    for (s, t) in shifts:
        oracle.francis_step_inplace(Hs, Qs, ktop, kbot, s, t)
    # same similarity up to signs of the reflector columns
    assert np.abs(np.abs(H) - np.abs(Hs)).max() <= 1e-11 * np.linalg.norm(H0)
    assert np.linalg.norm(Q @ H @ Q.T - H0) <= 1e-13 * n * np.linalg.norm(H0)
    assert np.abs(np.tril(H, -2)).max() == 0.0


def test_tuning_table_roundtrip():
    rows = [{"nmax": 500, "ns": 8, "nb": 4, "step": 0, "nw": 24, "nibble": 5},
            {"nmax": 1 << 30, "ns": 64, "nb": 16, "step": 0, "nw": -1, "nibble": -1}]
    schur.set_tuning(rows)
    for bad in ({"nmax": 10, "ns": 1, "nb": 1, "step": 0},
                {"nmax": 10, "ns": 4, "nb": 2, "step": 0, "nw": 2},
                {"nmax": 10, "ns": 4, "nb": 2, "step": 0, "nw": 97},
                {"nmax": 10, "ns": 4, "nb": 25, "step": 0},
                {"nmax": 10, "ns": 4, "nb": 2, "step": 0, "nibble": 101}):
        with pytest.raises(ValueError):
            schur.set_tuning([bad])
    with pytest.raises(ValueError):   # nmax must ascend
        schur.set_tuning(rows[::-1])
    schur.set_tuning([])   # built-in table back


# ---- parallel early deflation: window tiling and selection (host code the
# solver uses, exported as diagnostics) ----

@pytest.mark.parametrize("lo,hi,nw,first", [
    (0, 299, 96, 96), (0, 299, 96, 48), (10, 120, 96, 48), (5, 5, 96, 96), (0, 2, 96, 48),
    (3, 98, 96, 96), (0, 96, 96, 96), (0, 111, 96, 96), (7, 16000, 96, 48), (0, 700, 80, 40),
    (0, 333, 33, 16), (0, 1000, 3, 1), (100, 100 + 96 + 15, 96, 96), (0, 127, 96, 48)])
def test_split_tiling(lo, hi, nw, first):
    ws = schur.plan_split(lo, hi, nw, first)
    m = hi - lo + 1
    assert ws[0][0] == lo and ws[-1][0] + ws[-1][1] == hi + 1
    for (a0, w0), (a1, w1) in zip(ws, ws[1:]):
        assert a0 + w0 == a1                      # contiguous, top to bottom
    assert all(1 <= w <= nw for _, w in ws)
    if m <= first:
        assert ws == [(lo, m)]                    # one window: the whole block
    elif len(ws) >= 3:
        assert ws[-1][1] == first                 # bottom window as asked
        assert all(w == nw for _, w in ws[2:-1])  # full windows in between
    if len(ws) >= 2:
        assert ws[0][1] >= min(16, (ws[0][1] + ws[1][1]) // 2)   # no short top window


def test_split_tiling_bad_arguments():
    for args in [(-1, 10, 96, 96), (10, 5, 96, 96), (0, 10, 0, 1), (0, 10, 97, 96),
                 (0, 10, 96, 0), (0, 10, 48, 96)]:
        with pytest.raises(ValueError):
            schur.plan_split(*args)


@pytest.mark.parametrize("seed", range(12))
def test_split_selection_is_optimal(seed):
    """Against brute force over every subset: the chosen windows are
    disjoint and of largest total weight."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 11))
    a = rng.integers(0, 300, size=k).tolist()
    w = rng.integers(1, 97, size=k).tolist()
    wt = (1 + rng.integers(0, 40, size=k)).astype(float).tolist()
    pick = schur.select_windows(a, w, wt)
    assert pick == sorted(pick, key=lambda i: a[i]) and len(set(pick)) == len(pick)
    for x, y in zip(pick, pick[1:]):
        assert a[x] + w[x] <= a[y]
    best = 0.0
    for mask in range(1 << k):
        idx = [i for i in range(k) if mask >> i & 1]
        idx.sort(key=lambda i: a[i])
        if all(a[x] + w[x] <= a[y] for x, y in zip(idx, idx[1:])):
            best = max(best, sum(wt[i] for i in idx))
    assert sum(wt[i] for i in pick) == best


def test_split_selection_edge_cases():
    assert schur.select_windows([], [], []) == []
    assert schur.select_windows([5], [10], [1.0]) == [0]
    # equal windows: one of them; touching windows: both
    assert len(schur.select_windows([0, 0], [10, 10], [1.0, 1.0])) == 1
    assert schur.select_windows([0, 10], [10, 10], [1.0, 1.0]) == [0, 1]
    with pytest.raises(ValueError):
        schur.select_windows([0], [0], [1.0])
    with pytest.raises(ValueError):
        schur.select_windows([0], [5], [0.0])


def test_split_candidate_weight():
    """A window that failed its tests is no candidate; one at an end of its
    block that deflated nothing neither deflates nor splits, so it is none
    either; an interior window that deflated nothing still splits its block
    (weight 1); otherwise the weight is 1 + rows deflated."""
    assert schur.split_weight(0, 5, 1, 1) == 0.0
    for top, below in ((0, 1), (1, 0), (0, 0)):
        assert schur.split_weight(1, 0, top, below) == 0.0
        assert schur.split_weight(1, 7, top, below) == 8.0
    assert schur.split_weight(1, 0, 1, 1) == 1.0
    assert schur.split_weight(1, 3, 1, 1) == 4.0


def _random_blocks(n, seed, frac):
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes, sel = [], []
    r = 0
    while r < n:
        s = 2 if (r + 1 < n and rng.uniform() < 0.4) else 1
        sizes.append(s)
        sel.append(1 if rng.uniform() < frac else 0)
        r += s
    return sizes, sel


@pytest.mark.parametrize("n,seed,frac", [(1, 1, 1.0), (7, 2, 0.5), (96, 3, 0.5), (97, 4, 0.3),
                                         (300, 5, 0.5), (1000, 6, 0.2), (1000, 7, 0.8),
                                         (2500, 8, 0.5)])
def test_reorder_schedule(n, seed, frac):
    """The reordering schedule, executed as the device does (time step by
    time step; in each window the flagged rows move to the top, stably),
    leaves every selected block at the top in diagonal order; windows of one
    time step are disjoint, none is larger than 96 rows, and every window
    starts and ends at block boundaries of the layout it meets."""
    sizes, sel = _random_blocks(n, seed, frac)
    plan = schur.plan_reorder(sizes, sel)
    # layout: list of blocks (id, size, selected) in diagonal order
    layout = [(i, s, f) for i, (s, f) in enumerate(zip(sizes, sel))]
    steps = {}
    for chain, t, a, w in plan:
        steps.setdefault(t, []).append((a, w, chain))
    for t in sorted(steps):
        wins = sorted(steps[t])
        for (a1, w1, _), (a2, _, _) in zip(wins, wins[1:]):
            assert a1 + w1 <= a2
        for a, w, _ in wins:
            assert 1 <= w <= 96
            starts, r = [], 0
            for b in layout:
                starts.append(r)
                r += b[1]
            assert a in starts and (a + w in starts or a + w == n)
            i0 = starts.index(a)
            i1 = starts.index(a + w) if a + w < n else len(layout)
            inside = layout[i0:i1]
            layout[i0:i1] = [b for b in inside if b[2]] + [b for b in inside if not b[2]]
    want = [i for i, f in enumerate(sel) if f]
    got = [b[0] for b in layout[:len(want)]]
    assert got == want
    assert all(not b[2] for b in layout[len(want):])


def test_reorder_schedule_bad_arguments():
    IA = ctypes.c_int * 2
    assert schur.load().schur_plan_reorder(3, IA(1, 3), IA(1, 0), 2, None, 0) == -1
    assert schur.load().schur_plan_reorder(4, IA(1, 2), IA(1, 0), 2, None, 0) == -1
