"""Autotuner: picks shifts per sweep, bulges per window chain, chain steps per
window (which sets the diagonal window's order), the early-deflation window
and its sweep-skip percentage for each matrix-order bucket, on the GPU it
runs on.

For every bucket order n it times complete Schur reductions for each
candidate, keeps only candidates whose result passes the accuracy checks
(info 0, backward-error and orthogonality probes, exact structure), and
writes the fastest into a table ``{"table": [{"nmax", "ns", "nb", "step",
"nw", "nibble"}, ...]}`` that the library applies to every solve, batched
solve and served request whose options leave these parameters unset.  The
choice depends on n only, so a matrix gets the same parameters alone, in a
batch or in a serving mix.

The input recipe per bucket follows where the parameters matter: up to
n = 1024 a random N(0,1) Hessenberg matrix; from n = 2048 on the Hessenberg
form of a dense U(-1,1) matrix (drawn from its distribution), because on
random Hessenberg matrices of these orders the parallel early-deflation
passes do the work and no sweep runs.  With ``--batched`` the buckets up to
512 are timed instead as batches (``schur_reduce_batched``, i.e. the
persistent kernel, which takes at most 8 bulges per window chain) of
matrices with orders spread around the bucket, by solves per second -- the
regime where such orders occur.  For single solves from n = 512 on, the
panel products' tiles per workgroup (64 columns or rows each; 0 keeps the
per-launch cost model) are tried last, with the best sweep parameters.

    python -m paper_1905_04975_amd.autotune [--quick] [--batched] [--out path]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

BUCKETS = [128, 256, 512, 1024, 2048, 4096, 8192, 16384]


def candidates(n, quick):
    """(ns, nb, step, nw, nibble) candidates for order n; nw is the
    early-deflation window (0: from ns, -1: none), step the chain steps per
    window (0: as many as fit a 128-row window)."""
    out = []
    for ns in (2, 4, 8, 16, 32, 64, 128, 256):
        if ns > max(2, n // 6):
            continue
        for nb in (1, 2, 4, 8, 12, 16, 20, 24):
            if nb > ns // 2:
                continue
            if ns > 2 and nb < 2:
                continue
            out.append({"ns": ns, "nb": nb, "step": 0})
    if n >= 8192:   # a complete solve takes seconds here: a short list
        keep = [(128, 16), (256, 16), (256, 24)]
        out = [c for c in out if (c["ns"], c["nb"]) in keep]
        out += [dict(c, step=48) for c in out if c["nb"] == 16]
    elif quick or n >= 2048:
        out = [c for c in out if c["nb"] in (1, 4, 8, 16) and c["ns"] >= max(2, n // 64)]
    else:
        out = [c for c in out if c["nb"] in (1, 2, 4, 8, 16)]
    windows = [-1, 0, 32, 48, 64, 80, 96] if n >= 512 else [-1, 0, 16, 24, 32, 48]
    nibbles = [0]
    if n >= 8192:
        windows = [64, 96]
        nibbles = [7, 14]
    if n >= 16384:   # about 12 s per solve: the short list measured first
        return [dict(ns=128, nb=16, step=0, nw=64, nibble=7),
                dict(ns=256, nb=16, step=0, nw=64, nibble=7),
                dict(ns=256, nb=16, step=0, nw=96, nibble=7),
                dict(ns=256, nb=16, step=0, nw=96, nibble=14),
                dict(ns=256, nb=24, step=0, nw=96, nibble=14),
                dict(ns=256, nb=16, step=48, nw=96, nibble=14)]
    elif n >= 2048:
        nibbles = [0, 7]
    full = []
    for c in out:
        for nw in windows:
            if nw > 0 and nw >= n // 2:
                continue
            for nib in nibbles:
                if nw < 0 and nib != nibbles[0]:
                    continue
                full.append(dict(c, nw=nw, nibble=nib))
    return full


def time_candidate(schur, torch, H0, c, reps):
    n = H0.shape[0]
    dev = H0.device
    h = schur.Handle(0, ns=c["ns"], nb=c["nb"], step=c["step"], aed_window=c["nw"],
                     aed_nibble=c["nibble"], panel_tile=c.get("tile", 0))
    best = math.inf
    ok = True
    for _ in range(reps):
        H = H0.clone()
        Q = torch.eye(n, dtype=torch.float64, device=dev).t().contiguous().t()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S, Q, w, info = schur.reduce(H, Q=Q, handle=h)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if info != 0:
            ok = False
            break
        g = torch.Generator(device=dev).manual_seed(1)
        x = torch.randn(n, 2, dtype=torch.float64, device=dev, generator=g)
        Hh = torch.triu(H0, -1)
        res = (torch.linalg.norm(Hh @ x - Q @ (S @ (Q.t() @ x))) /
               (torch.linalg.norm(Hh) * torch.linalg.norm(x))).item()
        orth = (torch.linalg.norm(Q.t() @ (Q @ x) - x) / torch.linalg.norm(x)).item()
        below = torch.count_nonzero(torch.tril(S, -2)).item()
        if not (res < 1e-14 and orth < 1e-13 and below == 0):
            ok = False
            break
        best = min(best, dt)
    h.close()
    return ok, best


def bucket_input(inputs, n):
    """(matrix, recipe) timed for bucket order n."""
    if n >= 2048:
        return inputs.paper_like_law(n, 7000 + n), "paper_like_law"
    return inputs.hessenberg_normal(n, 7000 + n), "hessenberg_normal"


def time_batched(schur, torch, mats, c, reps):
    """Solves per second of one schur_reduce_batched call over `mats`, and
    whether every result passed the checks."""
    dev = torch.device("cuda:0")
    h = schur.Handle(0, ns=c["ns"], nb=c["nb"], step=c["step"], aed_window=c["nw"],
                     aed_nibble=c["nibble"])
    best = 0.0
    ok = True
    for _ in range(reps):
        Hs = [torch.from_numpy(m).to(dev) for m in mats]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ss, Qs, ws, infos, rc = schur.reduce_batched(Hs, handle=h)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rc != 0:
            ok = False
            break
        for m, S, Q in zip(mats[:8], Ss, Qs):
            Hh = torch.triu(torch.from_numpy(m).to(dev), -1)
            res = (torch.linalg.norm(Hh - Q @ S @ Q.t()) / torch.linalg.norm(Hh)).item()
            if not res < 1e-13 or torch.count_nonzero(torch.tril(S, -2)).item() != 0:
                ok = False
        best = max(best, len(mats) / dt)
    h.close()
    return ok, best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="time the buckets up to 512 as batches (solves/s)")
    ap.add_argument("--max-n", type=int, default=16384)
    ap.add_argument("--min-n", type=int, default=0,
                    help="tune only buckets >= this; rows below come from the table in --out")
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    args = ap.parse_args()
    import torch

    from paper_1905_04975_amd import inputs, schur

    schur.set_tuning([])      # time the candidates, not a previous table
    dev = torch.device("cuda:0")
    rows, meas = [], {}
    buckets = [b for b in BUCKETS if b <= args.max_n]
    keep_rows, keep_meas, keep_rec = [], {}, {}
    if args.min_n > 0 and os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
        lo = [b for b in buckets if b < args.min_n]
        keep_rows = old["table"][:len(lo)]
        keep_meas = {k: v for k, v in old.get("measurements", {}).items() if int(k) < args.min_n}
        keep_rec = {k: v for k, v in old.get("recipes", {}).items() if int(k) < args.min_n}
    import numpy as np

    recipes = dict(keep_rec)
    rows.extend(keep_rows)
    meas.update(keep_meas)
    for i, n in enumerate(buckets):
        if n < args.min_n:
            continue
        batched = args.batched and n <= 512
        results = []
        if batched:
            rng = np.random.Generator(np.random.PCG64(9000 + n))
            orders = rng.integers(max(8, int(n / 1.41)), int(n * 1.41) + 1, size=200)
            mats = [inputs.hessenberg_normal(int(m), 9100 + n + k) for k, m in enumerate(orders)]
            recipes[str(n)] = "batch of 200 hessenberg_normal, orders U[n/1.41, 1.41 n]"
            for c in candidates(n, args.quick):
                if c["nb"] > 8:   # the persistent kernel caps the bulges per chain at 8
                    continue
                ok, rate = time_batched(schur, torch, mats, c, 2)
                t = 1.0 / rate if rate > 0 else math.inf
                results.append((c, ok, t))
                print("n=%d (batch) ns=%d nb=%d step=%d nw=%d nibble=%d -> %s %.1f solves/s"
                      % (n, c["ns"], c["nb"], c["step"], c["nw"], c["nibble"],
                         "ok" if ok else "FAIL", rate), flush=True)
        else:
            H_np, recipe = bucket_input(inputs, n)
            recipes[str(n)] = recipe
            H0 = torch.from_numpy(H_np).to(dev)
            reps = 3 if n <= 1024 else 1
            for c in candidates(n, args.quick):
                ok, t = time_candidate(schur, torch, H0, c, reps)
                results.append((c, ok, t))
                print("n=%d ns=%d nb=%d step=%d nw=%d nibble=%d -> %s %.4f s"
                      % (n, c["ns"], c["nb"], c["step"], c["nw"], c["nibble"],
                         "ok" if ok else "FAIL", t), flush=True)
        good = [(t, c) for c, ok, t in results if ok]
        if not good:
            raise RuntimeError("no candidate passed at n=%d" % n)
        t, c = min(good, key=lambda z: z[0])
        c = dict(c, tile=0)
        if not batched and n >= 512:
            # the panel products' tile (tiles per workgroup), with the best
            # sweep parameters; 0 keeps the per-launch cost model
            for tl in (2, 4, 8):
                c2 = dict(c, tile=tl)
                ok2, t2 = time_candidate(schur, torch, H0, c2, reps)
                results.append((c2, ok2, t2))
                print("n=%d tile=%d -> %s %.4f s" % (n, tl, "ok" if ok2 else "FAIL", t2), flush=True)
                if ok2 and t2 < t:
                    t, c = t2, c2
        nmax = (int(math.sqrt(n * buckets[i + 1])) if i + 1 < len(buckets) else (1 << 30))
        rows.append({"nmax": nmax, "ns": c["ns"], "nb": c["nb"], "step": c["step"], "nw": c["nw"],
                     "nibble": c["nibble"], "tile": c.get("tile", 0)})
        meas[str(n)] = [dict(c2, ok=ok, seconds=t2) for c2, ok, t2 in results]
    with open(args.out, "w") as f:
        json.dump({"table": rows, "measurements": meas, "recipes": recipes,
                   "device": torch.cuda.get_device_name(0)}, f, indent=1)
    print(json.dumps({"table": rows}), flush=True)


if __name__ == "__main__":
    main()
