#!/usr/bin/env python3
"""Benchmark of the Schur-reduction hot path on one MI355X.

One step = one complete Schur reduction (paper Sec. 2, Eq. (4)) of a random
N(0,1) upper Hessenberg matrix of order 16384 (seed 3) with Schur vectors:
the parallel early-deflation passes (windows tiling every unreduced block),
the batched finish of the small blocks they leave, every further iteration
(deflation scan, early deflation on a bottom window, shifts, bulge-chain
windows, panel products) and the 2x2 standardisation run inside the timed
region.  H and Q are resident in HBM
before timing starts; between steps they are reset from device copies
outside the timed region.

Prints one JSON line.  `value` is the measured seconds per Schur reduction
(lower is better).  Beside it, each labelled: `executed_tflops` (the flops
the executed schedule performed, counted per launch, divided by the time)
and `nominal_tflops` (the conventional 10 n^3 count divided by the time; not
a hardware rate, since early deflation removes most of that work on this
input).  `roofline` reports the dominant kernel family measured with HIP
events on the solve stream, `families` every family; `paper_like` times one
solve of the paper's own test-matrix recipe (Hessenberg form of a dense
U(-1,1) matrix, Sec. 5) at the same order; `sweep` times forced 256-shift
multishift sweeps; `cpu_baseline` times the oracle on a bounded sample of the
same workload on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
FP64_VECTOR_PEAK_TFLOPS = 78.6 # MI355X FP64 vector peak (256 CUs, 2.4 GHz)
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--ns", type=int, default=0, help="shifts per sweep (0: built-in table)")
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--step-len", type=int, default=0)
    ap.add_argument("--aed-window", type=int, default=0,
                    help="early-deflation window (0: from ns, <0: off)")
    ap.add_argument("--aed-nibble", type=int, default=0,
                    help="percent of the window deflated above which no sweep follows")
    ap.add_argument("--split-window", type=int, default=0,
                    help="window of the parallel early-deflation passes (0: 96, <0: off)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the oracle sample")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--sweep-ns", type=int, default=256,
                    help="shifts per sweep of the forced-sweep measurement (0: skip it)")
    ap.add_argument("--panel-tile", type=int, default=0,
                    help="panel tiles per workgroup of the sweep products (0: table/cost model)")
    ap.add_argument("--sweep-mode", choices=("both", "one"), default="both",
                    help="forced sweeps: both stream modes, or only the one-stream run (profiling)")
    ap.add_argument("--sweep-count", type=int, default=3,
                    help="sweeps timed by the forced-sweep measurement")
    ap.add_argument("--workload",
                    choices=["n16384", "paper_like", "pipeline", "batch", "serve", "sweep"],
                    default="n16384")
    ap.add_argument("--no-paper-like", action="store_true",
                    help="skip the solve of the paper's test-matrix recipe")
    ap.add_argument("--count", type=int, default=2000, help="batch: number of matrices")
    ap.add_argument("--plain-sample", type=int, default=200,
                    help="batch/serve: requests timed with per-matrix plain launches")
    ap.add_argument("--requests", type=int, default=240, help="serve: requests (first 10%% warm-up)")
    ap.add_argument("--rate", type=float, default=0.0, help="serve: arrivals/s (0: 0.7 x saturation)")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    return ap.parse_args()


def oracle_sample(H_np, budget_s):
    """Time the oracle's Francis double-shift step on the workload matrix.

    Sample: one oracle Francis step restricted to the leading rows 0..L-1 of
    the n x n input (L grows until the step takes about `budget_s`); every
    bulge step updates full rows and columns of H and Q exactly as in a
    full-size step, so the cost per bulge step is that of the n = 16384
    solve.  Scaling: a full solve takes about c * n / 2 double-shift steps
    over an active block shrinking from n to 0 (c = shifts per eigenvalue,
    measured by the oracle on the same recipe at n = 256), i.e.
    c * n^2 / 4 bulge steps.
    """
    import numpy as np

    import oracle
    from paper_1905_04975_amd import inputs

    n = H_np.shape[0]
    # shifts per eigenvalue of the oracle on the same recipe at a size it finishes quickly
    h256 = inputs.hessenberg_normal(256, 1)
    _, _, _, _, info, iters = oracle.schur(h256)
    c = 2.0 * iters / 256.0
    L = 64
    t = 0.0
    H = np.asfortranarray(H_np.copy())
    Q = np.asfortranarray(np.eye(n))
    while True:
        t0 = time.perf_counter()
        oracle.francis_step_inplace(H, Q, 0, L - 1, 0.5, 0.25)
        t = time.perf_counter() - t0
        if t >= budget_s / 4 or L >= n:
            break
        L = min(n, L * 2)
    per_bulge = t / max(1, L - 2)
    bulge_steps = c * n * n / 4.0
    t_solve = per_bulge * bulge_steps
    return {
        "value": t_solve,
        "unit": "s per Schur reduction (extrapolated from the sample)",
        "cores": 1,
        "kind": "oracle",
        "nominal_tflops": 10.0 * n ** 3 / t_solve / 1e12,
        "sample": ("one oracle Francis step on rows/cols 0..%d of the n=%d input with full-row "
                   "and full-column H and Q updates (%.2f s, %.3g s per bulge step), scaled to "
                   "c*n^2/4 bulge steps with c=%.2f shifts per eigenvalue measured by the oracle "
                   "on the n=256 instance" % (L - 1, n, t, per_bulge, c)),
    }


def bench_batch(args):
    """Batched solves: 2000 random Hessenberg matrices, orders U{32..512}."""
    import numpy as np
    import torch

    from paper_1905_04975_amd import inputs, schur

    dev = torch.device("cuda:0")
    torch.cuda.set_stream(torch.cuda.Stream(dev))   # as in the main bench
    sizes = inputs.batch_sizes(args.count, 32, 512, inputs.SEED_BATCH_SIZES)
    mats = [inputs.hessenberg_normal(int(n), inputs.SEED_BATCH_BASE + i) for i, n in enumerate(sizes)]
    H0 = [torch.from_numpy(H).to(dev) for H in mats]
    h = schur.Handle(0)

    def run_batch(hh=h):
        Hs = [H.clone() for H in H0]
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        Ss, Qs, ws, infos, rc = schur.reduce_batched(Hs, handle=hh)
        torch.cuda.synchronize(dev)
        t = time.perf_counter() - t0
        if rc != 0:
            raise RuntimeError("batched solve failed: %d" % rc)
        return t, Ss, Qs

    def worst(Ss, Qs):
        worst_res = worst_orth = 0.0
        for i in range(0, args.count, max(1, args.count // 50)):
            Hh = torch.triu(H0[i], -1)
            S, Q = Ss[i], Qs[i]
            n = Hh.shape[0]
            r = (torch.linalg.norm(Hh - Q @ S @ Q.t()) / torch.linalg.norm(Hh)).item()
            o = torch.linalg.norm(Q.t() @ Q - torch.eye(n, dtype=torch.float64, device=dev)).item()
            worst_res, worst_orth = max(worst_res, r), max(worst_orth, o)
        return worst_res, worst_orth

    for _ in range(args.warmup):
        run_batch()
    times = []
    for _ in range(args.steps):
        t, Ss, Qs = run_batch()
        times.append(t)
        print("batch step: %.3f s" % t, file=sys.stderr, flush=True)
    st = h.stats()
    # accuracy of a sample of the batch (checker)
    worst_res, worst_orth = worst(Ss, Qs)
    del Ss, Qs
    # the same batch through the round engine (every matrix advanced sweep by
    # sweep in shared launches, host-planned rounds), once after a warm-up
    hr = schur.Handle(0, flags=schur.FLAG_BATCH_ROUNDS)
    run_batch(hr)
    t_rounds, Sr, Qr = run_batch(hr)
    rounds_res, rounds_orth = worst(Sr, Qr)
    st_r = hr.stats()
    hr.close()
    del Sr, Qr
    print("batch rounds engine: %.3f s" % t_rounds, file=sys.stderr, flush=True)
    # the persistent kernel alone, timed with HIP events
    ht = schur.Handle(0, flags=schur.FLAG_TIME_KERNELS)
    run_batch(ht)
    stt = ht.stats()
    ht.close()
    # per-matrix plain launches (one schur_reduce per matrix): a stratified
    # sample (every k-th matrix in order of size), each timed alone; the
    # estimate for the whole batch sums the mean time of each size stratum
    # over its members (no model of the time against n)
    import numpy as np

    order = np.argsort(sizes, kind="stable")
    k = max(1, min(args.plain_sample, args.count))
    strata = np.array_split(order, k)
    plain_t, plain_res, plain_orth = [], 0.0, 0.0
    for stratum in strata:
        i = int(stratum[len(stratum) // 2])
        H = H0[i].clone()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        S, Q, w, info = schur.reduce(H, handle=h)
        torch.cuda.synchronize(dev)
        plain_t.append(time.perf_counter() - t0)
        Hh = torch.triu(H0[i], -1)
        n_i = Hh.shape[0]
        plain_res = max(plain_res, (torch.linalg.norm(Hh - Q @ S @ Q.t())
                                    / torch.linalg.norm(Hh)).item())
        plain_orth = max(plain_orth, torch.linalg.norm(
            Q.t() @ Q - torch.eye(n_i, dtype=torch.float64, device=dev)).item())
        if info != 0:
            raise RuntimeError("plain launch failed: %d" % info)
    est_total = sum(plain_t[j] * len(strata[j]) for j in range(k))
    plain_scaled = args.count / est_total
    t = sum(times) / len(times)
    out = {
        "metric": "batched solves/s (2000 random Hessenberg, orders U{32..512})",
        "value": args.count / t, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "schur_batched_random_hessenberg", "count": args.count,
                   "orders": "U{32..512}", "seed_sizes": inputs.SEED_BATCH_SIZES,
                   "schur_vectors": True},
        "plain_launches": {"sample": k, "sampling": "one matrix from the middle of each of "
                                                     "%d size strata" % k,
                           "solves_per_s_sample": k / sum(plain_t),
                           "solves_per_s_stratified_estimate": plain_scaled,
                           "speedup": (args.count / t) / plain_scaled,
                           "check": {"max_residual": plain_res, "max_orthogonality": plain_orth}},
        "check": {"max_residual": worst_res, "max_orthogonality": worst_orth},
        "persistent_kernel": {
            "matrices": stt["persist_jobs"], "launches": st["launches"],
            "kernel_ms_hip_events": stt["persist_ms"],
            "executed_tflops": (stt["gemm_flops"] + stt["chase_flops"] + stt["small_flops"]
                                + stt["aed_flops"]) / max(stt["persist_ms"] * 1e-3, 1e-30) / 1e12,
            "gemm_flops": stt["gemm_flops"]},
        "rounds_engine": {"solves_per_s": args.count / t_rounds, "seconds": t_rounds,
                          "launches": st_r["launches"],
                          "speedup_of_persistent": (args.count / t) / (args.count / t_rounds),
                          "check": {"max_residual": rounds_res, "max_orthogonality": rounds_orth}},
        "stats": {k2: st[k2] for k2 in ("sweeps", "windows", "launches", "small_solves",
                                        "aed_windows", "persist_jobs")},
    }
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Serving loop: Poisson arrivals, orders log-uniform in [64, 4096]."""
    import numpy as np

    from paper_1905_04975_amd import inputs, schur

    rng = np.random.Generator(np.random.PCG64(inputs.SEED_SERVE))
    pool = []
    for i in range(48):   # pre-generated request pool, reused round-robin
        r2 = np.random.Generator(np.random.PCG64(inputs.SEED_SERVE_BASE + i))
        n = int(round(np.exp(r2.uniform(np.log(64), np.log(4096)))))
        if i % 2 == 0:
            pool.append(inputs.hessenberg_normal(n, inputs.SEED_SERVE_BASE + i))
        else:
            pool.append(inputs.prescribed(n, inputs.SEED_SERVE_BASE + i)[0])
    budget = int(args.budget_gb * (1 << 30))
    srv = None

    def drain(pending, done, t_end=None):
        for tk in list(pending):
            r = srv.poll(tk, pending[tk][0])
            if r is not None:
                done[tk] = (pending[tk][1], r[3], r[4])
                del pending[tk]

    def saturation():
        # a block of 24 requests submitted at once: completions per second
        pending, done = {}, {}
        t0 = time.perf_counter()
        for i in range(24):
            tk, n = srv.submit(pool[i % len(pool)])
            pending[tk] = (n, i)
        while pending:
            drain(pending, done)
            time.sleep(0.001)
        return 24 / (time.perf_counter() - t0)

    # the same block through a server that sends every request to the round
    # engine (no persistent launches), for comparison
    srv = schur.Server(0, budget_bytes=budget, flags=schur.FLAG_BATCH_ROUNDS)
    saturation()
    mu_rounds = saturation()
    srv.close()
    srv = schur.Server(0, budget_bytes=budget)
    if args.rate <= 0:
        saturation()
        mu = saturation()
        rate = 0.7 * mu
    else:
        mu, rate = None, args.rate
    gaps = rng.exponential(1.0 / rate, size=args.requests)
    arrivals = np.cumsum(gaps)
    pending, done = {}, {}
    t0 = time.perf_counter()
    for i in range(args.requests):
        while time.perf_counter() - t0 < arrivals[i]:
            drain(pending, done)
            time.sleep(0.0005)
        tk, n = srv.submit(pool[i % len(pool)])
        pending[tk] = (n, i)
    while pending:
        drain(pending, done)
        time.sleep(0.001)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    warm = args.requests // 10
    lat = np.array(sorted(v[2] for v in done.values() if v[0] >= warm))
    by_order = {}
    for name, keep in (("n<=1024", lambda m: m <= 1024), ("n>1024", lambda m: m > 1024)):
        x = np.array([v[2] for v in done.values()
                      if v[0] >= warm and keep(pool[v[0] % len(pool)].shape[0])])
        if x.size:
            by_order[name] = {"requests": int(x.size), "p50": float(np.percentile(x, 50)),
                              "p99": float(np.percentile(x, 99))}
    infos = [v[1] for v in done.values()]
    # FIFO plain launches on the same arrivals (sample): one request at a time
    import torch

    k = min(args.plain_sample, args.requests, 60)
    h = schur.Handle(0)
    dev = torch.device("cuda:0")
    t_free = 0.0
    lat_plain = []
    tp0 = time.perf_counter()
    for i in range(k):
        H = pool[i % len(pool)]
        start = max(arrivals[i], t_free)
        s0 = time.perf_counter()
        Hd = torch.from_numpy(np.asfortranarray(H)).to(dev)
        S, Q, w, info = schur.reduce(Hd, handle=h)
        S.cpu(); Q.cpu(); w.cpu()
        svc = time.perf_counter() - s0
        t_free = start + svc
        lat_plain.append(t_free - arrivals[i])
    lat_plain = np.array(sorted(lat_plain))
    out = {
        "metric": "served solves/s and p50/p99 latency (Poisson arrivals, orders log-uniform [64, 4096])",
        "value": args.requests / wall, "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * wall, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "schur_serving_mix", "requests": args.requests,
                   "rate_per_s": rate, "saturation_per_s": mu,
                   "saturation_round_engine_only_per_s": mu_rounds, "budget_gb": args.budget_gb,
                   "mix": "half random N(0,1), half prescribed spectrum"},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean()), "by_order": by_order},
        "fifo_plain_launches": {"sample": k,
                                "p50": float(np.percentile(lat_plain, 50)),
                                "p99": float(np.percentile(lat_plain, 99)),
                                "solves_per_s": k / max(t_free, 1e-9)},
        "all_info_zero": all(i == 0 for i in infos),
        "server": st,
    }
    print(json.dumps(out), flush=True)


def table_row(n):
    """The tuning-table row the library uses for order n (options left at 0)."""
    from paper_1905_04975_amd import schur
    try:
        with open(schur.TUNING_PATH) as f:
            rows = json.load(f)["table"]
    except (OSError, ValueError, KeyError):
        return {}
    for r in sorted(rows, key=lambda r: r["nmax"]):
        if n <= r["nmax"]:
            return r
    return {}


def sweep_measure(args, hdl, H0, H, Q, eye, wr, wi, stream):
    """Forced multishift sweeps on the same matrix: `--sweep-ns` shifts per
    sweep (the trailing block of that order gives them), a sweep after every
    early-deflation window, stopped after `--sweep-count` sweeps.  Run twice:
    as the library runs them (the Q products on a second stream, overlapping
    the window chase; `seconds`), and with every kernel on the solve stream
    (`SCHUR_FLAG_ONE_STREAM`), where each kernel's HIP-event duration is its
    own, for the rates of the sweep kernels (window chase; the panel products
    of a time step, there two launches: rows of H with Q, then columns of
    H).  The partial reduction is still an orthogonal
    similarity, which the probe checks."""
    import torch
    from paper_1905_04975_amd import schur

    n = args.n
    dev = H0.device

    def run(flags):
        hs = schur.Handle(0, ns=args.sweep_ns, nb=args.nb, aed_nibble=-1, split_window=-1,
                          panel_tile=args.panel_tile, max_sweeps=args.sweep_count,
                          flags=schur.FLAG_TIME_KERNELS | flags)
        H.copy_(H0)
        Q.copy_(eye)
        torch.cuda.synchronize(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info = hs.reduce_async(stream.cuda_stream, n, H.data_ptr(), n, Q.data_ptr(), n,
                               wr.data_ptr(), wi.data_ptr())
        e1.record(stream)
        torch.cuda.synchronize(dev)
        st = hs.stats()
        hs.close()
        if info < 0:
            raise RuntimeError("forced-sweep run failed: info=%d" % info)
        return info, e0.elapsed_time(e1) / 1e3, st

    info1, sec1, st1 = run(schur.FLAG_ONE_STREAM)
    if args.sweep_mode == "one":
        info, sec, st = info1, sec1, st1
    else:
        info, sec, st = run(0)
    nsw = max(1, st1["sweeps"])

    def gl(name, key, ms, launches, flops):
        avg = ms / max(1, launches)
        ach = flops / max(1, launches) / max(avg * 1e-3, 1e-30) / 1e12
        out = {"kernel": name, "bound": "mfma", "achieved": ach, "peak": FP64_MFMA_PEAK_TFLOPS,
               "unit": "TFLOP/s", "frac": ach / FP64_MFMA_PEAK_TFLOPS, "avg_launch_ms": avg,
               "launches": launches, "flops_per_launch": flops / max(1, launches),
               "traffic": pmc_traffic(key, "sweep")}
        if out["traffic"] is not None:
            out["hbm_gbs_from_traffic"] = out["traffic"] / max(avg * 1e-3, 1e-30) / 1e9
        return out

    gemm_ms = st1["row_ms"] + st1["colq_ms"]
    res = None
    if not args.no_check:
        x = torch.randn(n, 2, dtype=torch.float64, device=dev,
                        generator=torch.Generator(dev).manual_seed(1))
        Hh = torch.triu(H0, -1)
        res = (torch.linalg.norm(Hh @ x - Q @ (H @ (Q.t() @ x)))
               / (torch.linalg.norm(Hh) * torch.linalg.norm(x))).item()
    out = {
        "shifts_per_sweep": args.sweep_ns, "sweeps": st["sweeps"],
        "shifts_applied": st["shifts_applied"], "stop_info": info,
        "seconds": sec,
        "seconds_one_stream": sec1,
        "ms_per_sweep_one_stream": {"chase": st1["chase_ms"] / nsw, "row_panel": st1["row_ms"] / nsw,
                                    "colq_panel": st1["colq_ms"] / nsw,
                                    "shifts": st1["shift_ms"] / nsw, "aed": st1["aed_ms"] / nsw},
        "gemm_tflops": st1["gemm_flops"] / max(gemm_ms * 1e-3, 1e-30) / 1e12,
        "gemm_frac_of_fp64_mfma_peak": st1["gemm_flops"] / max(gemm_ms * 1e-3, 1e-30) / 1e12
        / FP64_MFMA_PEAK_TFLOPS,
        # with every kernel on one stream a time step's panel products are two
        # launches: the rows of H with Q (k_panel_rowq), then the columns of H
        "k_panel_colq": gl("k_panel_colq (columns of H)", "k_panel_colq", st1["colq_ms"],
                           st1["colq_launches"], st1["colq_flops"]),
        "k_panel_row": gl("k_panel_rowq (rows of H and Q)", "k_panel_rowq", st1["row_ms"],
                          st1["row_launches"], st1["row_flops"]),
        "k_chase": family_lines(st1, "sweep").get("k_chase"),
        "residual_probe": res,
    }
    print("sweep: %d sweeps of %d shifts, %.3f s (%.3f s on one stream), GEMM %.2f TFLOP/s" %
          (st["sweeps"], args.sweep_ns, sec, sec1, out["gemm_tflops"]), file=sys.stderr,
          flush=True)
    return out


KERNEL_SOURCES = ("kernels.hip", "mw_kernels.hip", "wave_solvers.h", "window_chase.h",
                  "device_common.h", "wg_ops.h", "schur_internal.h")


def kernel_source_hash():
    """sha256 of the device sources: HBM traffic from PMC counters is only
    reported while the kernels are the ones the counters were taken on."""
    import hashlib

    hsh = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1905_04975_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            hsh.update(f.read())
    return hsh.hexdigest()


def pmc_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the calibration factors
    stated there), or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha256") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get("%s@%s" % (kernel, workload))
    return None if ent is None else ent.get("bytes_per_launch")


FAMILIES = (
    # name, stats keys (ms, launches, flops), bound
    ("k_panel_colq", ("colq_ms", "colq_launches", "colq_flops"), "mfma"),
    ("k_panel_row", ("row_ms", "row_launches", "row_flops"), "mfma"),
    ("k_chase", ("chase_ms", "chase_launches", "chase_flops"), "alu"),
    ("k_aed", ("aed_ms", "aed_launches", "aed_flops"), "alu"),
    ("k_split", ("split_ms", "split_passes", "split_flops"), "alu"),
    ("k_small", ("small_ms", "small_launches", "small_flops"), "alu"),
)


def counted_flops(st):
    """Flops the executed schedule performed (counted per launch from the
    shapes it ran; nominal per-window counts for the QR-in-a-workgroup
    kernels)."""
    return (st["gemm_flops"] + st["chase_flops"] + st["aed_flops"] + st["split_flops"]
            + st["small_flops"])


def family_lines(st, workload):
    """Per kernel family: summed HIP-event time, launches, counted flops and
    the rate against the FP64 peak of its bound."""
    out = {}
    for name, (kms, kl, kf), bound in FAMILIES:
        ms, launches, flops = st[kms], st[kl], st[kf]
        if launches <= 0 or ms <= 0:
            continue
        avg_ms = ms / launches
        achieved = flops / launches / (avg_ms * 1e-3) / 1e12
        peak = FP64_MFMA_PEAK_TFLOPS if bound == "mfma" else FP64_VECTOR_PEAK_TFLOPS
        traffic = pmc_traffic(name, workload)
        out[name] = {"kernel": name, "bound": bound, "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "avg_launch_ms": avg_ms, "launches": launches, "total_ms": ms,
                     "flops_per_launch": flops / launches}
        if traffic is not None:
            out[name]["hbm_gbs_from_traffic"] = traffic / (avg_ms * 1e-3) / 1e9
        if name == "k_chase":
            # the window task's own measures: chain steps per second and the
            # algorithmic HBM rate (window in and out, U out: 24 ws^2 bytes)
            out[name]["windows"] = st["windows"]
            out[name]["chain_steps"] = st["chain_steps"]
            out[name]["chain_steps_per_s"] = st["chain_steps"] / (ms * 1e-3)
            out[name]["algorithmic_bytes_per_launch"] = st["chase_bytes"] / launches
            out[name]["hbm_gbs_algorithmic"] = st["chase_bytes"] / (ms * 1e-3) / 1e9
            out[name]["hbm_frac_algorithmic"] = out[name]["hbm_gbs_algorithmic"] / HBM_PEAK_GBS
    return out


def roofline_of(fam, st):
    """The dominant kernel family by time.  A QR-in-a-workgroup kernel (one
    wavefront per window: chains of dependent small steps) is reported
    against the FP64 vector peak; `cus_per_launch` and `frac_used_cus` give
    the share of the peak of the CUs a launch occupies."""
    if not fam:
        return None
    name = max(fam, key=lambda k: fam[k]["total_ms"])
    r = dict(fam[name])
    if name == "k_split":
        cus = min(256.0, st["split_windows"] / max(1, st["split_passes"]))
        r["cus_per_launch"] = cus
        r["peak_used_cus"] = FP64_VECTOR_PEAK_TFLOPS * cus / 256
        r["frac_used_cus"] = r["achieved"] / r["peak_used_cus"]
    return r


def solve_timed(schur, dev, stream, hdl, H0, H, Q, eye, wr, wi):
    """One Schur reduction of H0 (reset from its device copy outside the
    timed region) bracketed by HIP events on the solve stream."""
    import torch

    n = H0.shape[0]
    H.copy_(H0)
    Q.copy_(eye)
    torch.cuda.synchronize(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    info = hdl.reduce_async(stream.cuda_stream, n, H.data_ptr(), n, Q.data_ptr(), n,
                            wr.data_ptr(), wi.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize(dev)
    w1 = time.perf_counter()
    if info != 0:
        raise RuntimeError("schur_reduce_async returned info=%d" % info)
    return e0.elapsed_time(e1) / 1e3, w1 - w0, hdl.stats()


def probe(H0, H, Q, wr, seed):
    """Freivalds-style probes of a result (checker, independent of the kernels)."""
    import torch

    n = H0.shape[0]
    dev = H0.device
    x = torch.randn(n, 2, dtype=torch.float64, device=dev,
                    generator=torch.Generator(dev).manual_seed(seed))
    Hh = torch.triu(H0, -1)
    r = torch.linalg.norm(Hh @ x - Q @ (H @ (Q.t() @ x))) / (torch.linalg.norm(Hh)
                                                             * torch.linalg.norm(x))
    o = torch.linalg.norm(Q.t() @ (Q @ x) - x) / torch.linalg.norm(x)
    below = torch.tril(H, -2).abs().max().item()
    return {"residual_probe": r.item(), "orthogonality_probe": o.item(),
            "max_below_subdiag": below,
            "trace_err": abs(wr.sum().item() - torch.trace(H0).item())
            / torch.linalg.norm(Hh).item()}


def block_matrix(S_np, m):
    """Real block-diagonal L with S's eigenvalues for the first m columns of
    an eigenvector matrix in LAPACK's layout: X L = S-image of X."""
    import numpy as np

    L = np.zeros((m, m))
    k = 0
    while k < m:
        if k + 1 < S_np.shape[0] and S_np[k + 1, k] != 0.0:
            wi = np.sqrt(abs(S_np[k, k + 1])) * np.sqrt(abs(S_np[k + 1, k]))
            L[k, k] = S_np[k, k]
            if k + 1 < m:
                L[k + 1, k + 1] = S_np[k, k]
                L[k, k + 1], L[k + 1, k] = wi, -wi
            k += 2
        else:
            L[k, k] = S_np[k, k]
            k += 1
    return L


def pipeline_measure(args, schur, inputs, dev, stream, H, Q, eye, wr, wi):
    """The paper's route on its own test matrices (Sec. 5) at the same
    order: a dense U(-1,1) matrix A (drawn on the device from a seeded
    generator) is reduced to Hessenberg form (Eq. (3)), then to real Schur
    form (Eq. (4)) with Q accumulating Q1 Q2, then the eigenvectors of A are
    computed (Eqs. (5)-(6)).  Each step is timed with HIP events on the
    stream and checked by probes (independent torch products)."""
    import torch

    n = args.n
    g = torch.Generator(dev).manual_seed(inputs.SEED_PAPER_LIKE)
    A0 = torch.rand(n, n, dtype=torch.float64, device=dev, generator=g).mul_(2.0).sub_(1.0)
    H.copy_(A0)   # column-major working copy
    Q.copy_(eye)
    h = schur.Handle(0, flags=schur.FLAG_TIME_KERNELS)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    torch.cuda.synchronize(dev)
    x = torch.randn(n, 2, dtype=torch.float64, device=dev,
                    generator=torch.Generator(dev).manual_seed(3))
    nA = torch.linalg.norm(A0).item()
    nx = torch.linalg.norm(x).item()
    # Hessenberg reduction
    w0 = time.perf_counter()
    ev[0].record(stream)
    rc = h.hessenberg_async(stream.cuda_stream, n, H.data_ptr(), n, Q.data_ptr(), n)
    ev[1].record(stream)
    torch.cuda.synchronize(dev)
    t_hess = time.perf_counter() - w0
    if rc != 0:
        raise RuntimeError("schur_hessenberg returned %d" % rc)
    sth = h.stats()
    r_hess = (torch.linalg.norm(A0 @ x - Q @ (H @ (Q.t() @ x))) / (nA * nx)).item()
    below = torch.count_nonzero(torch.tril(H, -2)).item()
    # Schur reduction of that Hessenberg form
    w0 = time.perf_counter()
    ev[2].record(stream)
    info = h.reduce_async(stream.cuda_stream, n, H.data_ptr(), n, Q.data_ptr(), n, wr.data_ptr(),
                          wi.data_ptr())
    ev[3].record(stream)
    torch.cuda.synchronize(dev)
    t_schur = time.perf_counter() - w0
    if info != 0:
        raise RuntimeError("schur_reduce_async returned info=%d" % info)
    sts = h.stats()
    r_schur = (torch.linalg.norm(A0 @ x - Q @ (H @ (Q.t() @ x))) / (nA * nx)).item()
    o_schur = (torch.linalg.norm(Q.t() @ (Q @ x) - x) / nx).item()
    # eigenvectors of A
    X = torch.empty(n, n, dtype=torch.float64, device=dev).t()
    w0 = time.perf_counter()
    ev[4].record(stream)
    rc = h.eigenvectors_async(stream.cuda_stream, n, H.data_ptr(), n, Q.data_ptr(), n,
                              X.data_ptr(), n)
    ev[5].record(stream)
    torch.cuda.synchronize(dev)
    t_ev = time.perf_counter() - w0
    if rc != 0:
        raise RuntimeError("schur_eigenvectors returned %d" % rc)
    ste = h.stats()
    m = 256   # eigenvector check on the first m columns (before S is reordered)
    S_lead = H[:m + 1, :m + 1].cpu().numpy()
    L = torch.from_numpy(block_matrix(S_lead, m)).to(dev)
    Xm = X[:, :m]
    R = A0 @ Xm - Xm @ L
    r_ev = (torch.linalg.norm(R, dim=0) / torch.linalg.norm(Xm, dim=0)).max().item() / nA
    del X, Xm, R
    # eigenvalue reordering (the paper's second Table 2 workload): a seeded
    # random half of the eigenvalues to the top, Q accumulating
    import numpy as np

    sel = (np.random.Generator(np.random.PCG64(inputs.SEED_PAPER_LIKE)).uniform(size=n)
           < 0.5).astype(int).tolist()
    w0 = time.perf_counter()
    rc, msel = h.reorder_async(stream.cuda_stream, n, H.data_ptr(), n, Q.data_ptr(), n, sel,
                               wr.data_ptr(), wi.data_ptr())
    torch.cuda.synchronize(dev)
    t_ro = time.perf_counter() - w0
    str_ = h.stats()
    h.close()
    if rc < 0:
        raise RuntimeError("schur_reorder returned %d" % rc)
    r_ro = (torch.linalg.norm(A0 @ x - Q @ (H @ (Q.t() @ x))) / (nA * nx)).item()
    below_ro = torch.count_nonzero(torch.tril(H, -2)).item()
    del A0
    fam = family_lines(sts, "paper_like_n%d" % n)
    gemv_s = sth["hess_panel_ms"] / 1e3
    hess = {
        "workload": "hessenberg_dense_uniform_n%d" % n, "seconds": t_hess,
        "seconds_hip_events": ev[0].elapsed_time(ev[1]) / 1e3,
        "panel_column_kernels_s": gemv_s,
        "panel_products_s": sth["hess_gemm_ms"] / 1e3,
        "roofline": {"kernel": "k_hgemv (+ the four column kernels of each column)",
                     "bound": "hbm", "achieved": sth["hess_gemv_bytes"] / gemv_s / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sth["hess_gemv_bytes"] / gemv_s / 1e9 / HBM_PEAK_GBS,
                     "traffic": pmc_traffic("k_hgemv", "hessenberg_n%d" % n),
                     "bytes_note": "8 bytes per trailing-matrix entry and column (the "
                                   "matrix-vector products' algorithmic reads)"},
        "products_tflops": sth["hess_gemm_flops"] / max(sth["hess_gemm_ms"], 1e-9) / 1e9,
        "nominal_tflops": (10.0 / 3.0 + 4.0 / 3.0) * n ** 3 / t_hess / 1e12,
        "check": {"residual_probe": r_hess, "nonzeros_below_subdiag": below},
    }
    paper = {
        "workload": "paper_like_n%d" % n, "seed": inputs.SEED_PAPER_LIKE,
        "input": ("Hessenberg form (computed above) of a dense U(-1,1) matrix drawn on the "
                  "device (torch generator, seed %d)" % inputs.SEED_PAPER_LIKE),
        "seconds_per_solve": t_schur, "seconds_hip_events": ev[2].elapsed_time(ev[3]) / 1e3,
        "executed_tflops": counted_flops(sts) / t_schur / 1e12,
        "nominal_tflops": 10.0 * n ** 3 / t_schur / 1e12,
        "roofline": roofline_of(fam, sts), "families": fam,
        "breakdown": breakdown_of(sts, t_schur),
        "check": {"residual_probe_of_A": r_schur, "orthogonality_probe": o_schur},
    }
    eig = {
        "workload": "eigenvectors_of_A_n%d" % n, "seconds": t_ev,
        "seconds_hip_events": ev[4].elapsed_time(ev[5]) / 1e3,
        "tile_solves_s": ste["ev_solve_ms"] / 1e3, "tile_updates_s": ste["ev_gemm_ms"] / 1e3,
        "backtransform_s": ste["ev_back_ms"] / 1e3,
        "update_tflops": ste["ev_gemm_flops"] / max(ste["ev_gemm_ms"], 1e-9) / 1e9,
        "backtransform_tflops": ste["ev_back_flops"] / max(ste["ev_back_ms"], 1e-9) / 1e9,
        "check": {"max_relative_residual_first_%d" % m: r_ev},
    }
    reo = {
        "workload": "reorder_half_of_eigenvalues_n%d" % n, "seconds": t_ro, "info": rc,
        "selected": msel, "windows": str_["reorder_windows"], "time_steps": str_["reorder_steps"],
        "window_tasks_s": str_["reorder_ms"] / 1e3,
        "products_s": (str_["row_ms"] + str_["colq_ms"]) / 1e3,
        "products_tflops": str_["gemm_flops"] / max(str_["row_ms"] + str_["colq_ms"], 1e-9) / 1e9,
        "check": {"residual_probe_of_A": r_ro, "nonzeros_below_subdiag": below_ro},
    }
    print("pipeline: hessenberg %.3f s, schur %.3f s, eigenvectors %.3f s, reorder %.3f s"
          % (t_hess, t_schur, t_ev, t_ro), file=sys.stderr, flush=True)
    return {"hessenberg": hess, "schur": paper, "eigenvectors": eig, "reorder": reo}


def breakdown_of(st, seconds):
    keys = ("sweeps", "windows", "launches", "shifts_applied", "aed_windows", "aed_deflated",
            "split_passes", "split_windows", "split_accepted", "split_converged",
            "small_solves", "chase_ms", "row_ms", "colq_ms", "shift_ms", "other_ms", "aed_ms",
            "split_ms", "small_ms")
    b = {k: st[k] for k in keys}
    b["executed_gemm_tflops"] = st["gemm_flops"] / seconds / 1e12
    return b


def main():
    args = parse()
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1905_04975_amd import inputs, schur

    dev = torch.device("cuda:0")
    # every step on one created stream (default priority): the library's
    # kernels, their HIP events and torch's own work are in one stream order
    # without the null stream's implicit synchronisation
    torch.cuda.set_stream(torch.cuda.Stream(dev))
    n = args.n
    t0 = time.time()
    paper_main = args.workload == "paper_like"
    if paper_main:
        H_np = inputs.paper_like_law(n, inputs.SEED_PAPER_LIKE)
    else:
        H_np = inputs.hessenberg_normal(n, args.seed)
    H0 = torch.from_numpy(H_np).to(dev)          # column-major storage (Fortran order)
    assert H0.stride(0) == 1
    H = torch.empty_like(H0)
    Q = torch.empty_like(H0)
    eye = torch.eye(n, dtype=torch.float64, device=dev).t()
    wr = torch.empty(n, dtype=torch.float64, device=dev)
    wi = torch.empty(n, dtype=torch.float64, device=dev)
    gen_s = time.time() - t0
    hdl = schur.Handle(0, ns=args.ns, nb=args.nb, step=args.step_len, aed_window=args.aed_window,
                       aed_nibble=args.aed_nibble, split_window=args.split_window,
                       panel_tile=args.panel_tile, flags=schur.FLAG_TIME_KERNELS)
    stream = torch.cuda.current_stream(dev)

    if args.workload == "pipeline":
        # only the paper's route on a dense U(-1,1) matrix (for profiling)
        del H0
        pl = pipeline_measure(args, schur, inputs, dev, stream, H, Q, eye, wr, wi)
        print(json.dumps({"metric": "paper route at n=%d: Hessenberg, Schur, eigenvectors, "
                                    "reordering (s)" % n,
                          "value": sum(pl[k]["seconds" if k != "schur" else "seconds_per_solve"]
                                       for k in pl),
                          "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
                          "data": "synthetic",
                          "config": {"workload": "paper_route_dense_uniform", "n": n}, **pl}),
              flush=True)
        return
    if args.workload == "sweep":
        # only the forced-sweep measurement (for profiling the sweep kernels)
        sw = sweep_measure(args, hdl, H0, H, Q, eye, wr, wi, stream)
        print(json.dumps({"metric": "forced multishift sweeps at n=%d: update-GEMM FP64 TFLOP/s" % n,
                          "value": sw["gemm_tflops"], "unit": "TFLOP/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "schur_forced_sweeps_random_hessenberg", "n": n,
                                     "seed": args.seed}, "sweep": sw}), flush=True)
        return
    workload = "paper_like_n%d" % n if paper_main else "random_hessenberg_n%d" % n
    for _ in range(args.warmup):
        solve_timed(schur, dev, stream, hdl, H0, H, Q, eye, wr, wi)
    torch.cuda.synchronize(dev)
    times, walls, stats = [], [], []
    for _ in range(args.steps):
        dt, wt, st = solve_timed(schur, dev, stream, hdl, H0, H, Q, eye, wr, wi)
        times.append(dt)
        walls.append(wt)
        stats.append(st)
        print("step: %.3f s (wall %.3f s) sweeps=%d" % (dt, wt, st["sweeps"]), file=sys.stderr,
              flush=True)
    total = sum(walls)
    sec = total / len(walls)
    st0 = stats[-1]
    fam = family_lines(st0, workload)
    roofline = roofline_of(fam, st0)
    check = None if args.no_check else probe(H0, H, Q, wr, 0)
    sweep = None
    if args.sweep_ns > 0 and not paper_main:
        sweep = sweep_measure(args, hdl, H0, H, Q, eye, wr, wi, stream)
    paper = None
    if not paper_main and not args.no_paper_like:
        del H0
        paper = pipeline_measure(args, schur, inputs, dev, stream, H, Q, eye, wr, wi)
    row = table_row(n)
    out = {
        "metric": "Schur-reduction s & FP64 TFLOP/s at n=16384; batched solves/s; p99 latency",
        "value": sec,
        "unit": "s per Schur reduction (H and Q, n=%d)" % n,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec,
        "seconds_per_solve": sec,
        "executed_tflops": counted_flops(st0) / sec / 1e12,
        "executed_tflops_note": ("flops the executed schedule performed (panel products counted "
                                 "from their shapes, window chases per reflector and row, the "
                                 "QR-in-a-workgroup kernels by the nominal 25 m^3 / 10 m^3 "
                                 "counts) divided by seconds per solve"),
        "nominal_tflops": 10.0 * n ** 3 / sec / 1e12,
        "nominal_tflops_note": ("10 n^3 / seconds: the conventional count of the QR algorithm "
                                "(about two shifts per eigenvalue); the early deflation of this "
                                "input removes most of that work, so this is no rate of the "
                                "hardware and can exceed its peak"),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n": n,
                   "seed": inputs.SEED_PAPER_LIKE if paper_main else args.seed,
                   "entries": ("Hessenberg form of dense U(-1,1)" if paper_main
                               else "iid N(0,1) on and above the subdiagonal"),
                   "shifts_per_sweep": args.ns or row.get("ns"),
                   "bulges_per_group": args.nb or row.get("nb"),
                   "chase_window_rows": 128,
                   "aed_window": args.aed_window or row.get("nw"),
                   "sweep_skip_pct": args.aed_nibble or row.get("nibble") or 14,
                   "split_window": args.split_window or 96,
                   "split_passes": st0["split_passes"],
                   "sweeps_executed": st0["sweeps"], "schur_vectors": True},
        "roofline": roofline,
        "families": fam,
        "breakdown": breakdown_of(st0, sec),
        "paper_like": paper["schur"] if paper else None,
        "hessenberg": paper["hessenberg"] if paper else None,
        "eigenvectors": paper["eigenvectors"] if paper else None,
        "reorder": paper["reorder"] if paper else None,
        "sweep": sweep,
        "check": check,
        "gen_seconds": gen_s,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = oracle_sample(H_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
