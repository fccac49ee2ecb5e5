"""Autotuner: picks shifts per sweep, bulges per window chain, chain steps per
window, the early-deflation window and its sweep-skip percentage for each
matrix-order bucket, on the GPU it runs on.

For every bucket order n it times complete Schur reductions of a seeded
random N(0,1) Hessenberg matrix for each candidate, keeps only candidates
whose result passes the accuracy checks (info 0, backward-error and
orthogonality probes, exact structure), and writes the fastest into a table
``{"table": [{"nmax", "ns", "nb", "step", "nw", "nibble"}, ...]}`` that the library applies
to every solve, batched solve and served request whose options leave these
parameters unset.  The choice depends on n only, so a matrix gets the same
parameters alone, in a batch or in a serving mix.

    python -m paper_1905_04975_amd.autotune [--quick] [--out path]
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
    """(ns, nb, nw) candidates for order n; nw is the early-deflation window
    (0: from ns, -1: none)."""
    out = []
    for ns in (2, 4, 8, 16, 32, 64, 128):
        if ns > max(2, n // 6):
            continue
        for nb in (1, 2, 4, 8, 12, 16, 20, 24):
            if nb > ns // 2:
                continue
            if ns > 2 and nb < 2:
                continue
            out.append({"ns": ns, "nb": nb, "step": 0})
    if n >= 8192:   # a complete solve takes seconds here: a short list
        keep = [(64, 16), (128, 16)]
        out = [c for c in out if (c["ns"], c["nb"]) in keep]
    elif quick or n >= 2048:
        out = [c for c in out if c["nb"] in (1, 4, 8, 16) and c["ns"] >= max(2, n // 64)]
    else:
        out = [c for c in out if c["nb"] in (1, 2, 4, 8, 16)]
    windows = [-1, 0, 32, 48, 64, 80, 96] if n >= 512 else [-1, 0, 16, 24, 32, 48]
    nibbles = [0]
    if n >= 8192:
        windows = [56, 64, 72]
        nibbles = [7, 14]
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
                     aed_nibble=c["nibble"])
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--max-n", type=int, default=16384)
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    args = ap.parse_args()
    import torch

    from paper_1905_04975_amd import inputs, schur

    schur.set_tuning([])      # time the candidates, not a previous table
    dev = torch.device("cuda:0")
    rows, meas = [], {}
    buckets = [b for b in BUCKETS if b <= args.max_n]
    for i, n in enumerate(buckets):
        H0 = torch.from_numpy(inputs.hessenberg_normal(n, 7000 + n)).to(dev)
        reps = 3 if n <= 1024 else 1
        results = []
        for c in candidates(n, args.quick):
            ok, t = time_candidate(schur, torch, H0, c, reps)
            results.append((c, ok, t))
            print("n=%d ns=%d nb=%d nw=%d nibble=%d -> %s %.4f s"
                  % (n, c["ns"], c["nb"], c["nw"], c["nibble"], "ok" if ok else "FAIL", t),
                  flush=True)
        good = [(t, c) for c, ok, t in results if ok]
        if not good:
            raise RuntimeError("no candidate passed at n=%d" % n)
        t, c = min(good, key=lambda z: z[0])
        nmax = (int(math.sqrt(n * buckets[i + 1])) if i + 1 < len(buckets) else (1 << 30))
        rows.append({"nmax": nmax, "ns": c["ns"], "nb": c["nb"], "step": c["step"], "nw": c["nw"],
                     "nibble": c["nibble"]})
        meas[str(n)] = [dict(c2, ok=ok, seconds=t2) for c2, ok, t2 in results]
    with open(args.out, "w") as f:
        json.dump({"table": rows, "measurements": meas,
                   "device": torch.cuda.get_device_name(0)}, f, indent=1)
    print(json.dumps({"table": rows}), flush=True)


if __name__ == "__main__":
    main()
