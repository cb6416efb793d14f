#!/usr/bin/env python
"""Benchmark: plain generalized-DWD solves on one MI355X.

A step is one whole solve of the HDLSS workload (d = 1e5, n = 1e3, FP32 data,
q = 1, C = 10, relative KKT 1e-5): set-up (scaling, Gram, inverse) plus the
sGS-ADMM iterations to convergence, with X already resident in HBM.  Prints
one JSON line; see the design doc for the roofline and baseline definitions.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solves/s at rel. KKT 1e-5 (d=1e5,n=1e3), batched vs plain; p50/p99 latency"


def pass_bytes(d, ld, n, elem):
    """Algorithmic HBM bytes of one Z~ [s, alpha] pass: the d x n data once,
    plus u, rho read and w, Z~alpha written (FP64, length ld), plus the two
    n-vectors."""
    return d * n * elem + 4 * ld * 8 + 2 * n * 8


def cpu_baseline(X, y, wl, iters_needed, sample_iters):
    """Time the FP64 oracle on the host: its set-up plus `sample_iters`
    iterations of Algorithm 1 on the same workload, extrapolated to the
    iteration count the solve needs."""
    import numpy as np
    from oracle import dwd_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = len(os.sched_getaffinity(0))
    Xd = np.asarray(X, dtype=np.float64)
    t0 = time.perf_counter()
    Zt, zs = O.scale_data(Xd, y)
    O.SMWFactor(Zt, y, 1.0)
    t1 = time.perf_counter()
    O.solve(Xd, y, wl.C, wl.q, tol=1e-300, max_iter=sample_iters)
    t2 = time.perf_counter()
    # solve() repeats the set-up; subtract it to get the iterations alone
    per_iter = max((t2 - t1) - (t1 - t0), 1e-9) / sample_iters
    setup_s = t1 - t0
    total = setup_s + per_iter * iters_needed
    return {"value": 1.0 / total, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"oracle set-up ({setup_s:.1f} s) + {sample_iters} iterations "
                       f"({per_iter:.2f} s each) on the same d=1e5 n=1e3 data, "
                       f"extrapolated to {iters_needed} iterations")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not part of this "
              "build (see DESIGN.md for how the path would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2305_12019_amd import dwd

    wl = synth.HDLSS_F32
    X, y = synth.two_class(wl.data)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    torch.cuda.synchronize()
    d, n = wl.data.d, wl.data.n
    ld = ((d + 1023) // 1024) * 1024

    def step(profile):
        t = time.perf_counter()
        P = dwd.Problem(Xd, y, storage="f32")
        r = P.solve(wl.C, wl.q, tol=wl.tol, want_state=False, profile=profile)
        P.close()
        return r, (time.perf_counter() - t) * 1e3

    for _ in range(args.warmup):
        step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(1) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    infos = [r["info"] for r, _ in runs]
    lat = np.array([ms for _, ms in runs])
    conv = all(i["converged"] == 1 for i in infos)
    launches = sum(i["stream_launches"] for i in infos)
    kern_ms = sum(i["stream_ms"] for i in infos)
    avg_us = kern_ms / max(launches, 1) * 1e3
    bpl = pass_bytes(d, ld, n, 4)
    achieved = bpl / (avg_us * 1e-6) / 1e9
    iters = int(np.median([i["iters"] for i in infos]))
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "d": d, "n": n, "q": wl.q, "C": wl.C, "tol": wl.tol,
                   "storage": "f32", "iters": iters,
                   "n_double": int(np.median([i["n_double"] for i in infos])),
                   "converged": conv,
                   "kkt_check_max": max(i["kkt_check"] for i in infos),
                   "setup_ms": float(np.median([i["setup_ms"] for i in infos])),
                   "solve_ms": float(np.median([i["solve_ms"] for i in infos]))},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "roofline": {"bound": "hbm", "kernel": "k_pass2<float,8> (Z~ [s, alpha] pass)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_us": avg_us, "launches": launches,
                     "bytes_per_launch": bpl},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, y, wl, iters, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
