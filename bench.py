#!/usr/bin/env python
"""Benchmark: generalized-DWD solves on one MI355X.

A step is one whole plain solve of the HDLSS workload (d = 1e5, n = 1e3,
FP32 data, q = 1, C = 10, relative KKT 1e-5): set-up (scaling, Gram,
inverse) plus the sGS-ADMM iterations to convergence, with X already resident
in HBM.  `value` is plain solves/s over the timed steps.

Beside it, on the same data and to the same tolerance, the line carries
  batched   the 64 (C, q) problems of the sweep grid solved by dwd_solve_batch
            against the same 64 problems solved one after another (set-up
            shared by both), solves/s and the gain;
  serving   the first 500 requests of the seeded request stream (mixed d,
            n, q, C, dense FP32/BF16 and CSR) replayed by dwd_serve at 0.75x
            the measured plain capacity and at 30 requests/s (p50/p99
            latency), and with every request queued at t = 0 (solves/s
            against the plain per-request solves);
  roofline  the Z~ [s, alpha] pass of the plain solve, timed live with HIP
            events on the solver's stream, against the HBM peak and against a
            measured device copy;
  large     the d=1e6 n=2000 q=2 workload (feature scales log-uniform in
            [0.1, 10]) solved with Z in BF16 (FP64 factors of the BF16 image,
            FP32 refinement, FP64 check) against Z in FP32, both to rel. KKT
            1e-5 (--no-large skips it);
  representer  the same HDLSS solves in the representer mode (the d-vectors
            carried as n-vector coefficients, so an iteration reads only the
            n x n matrices and Z is streamed once at the end and by the FP64
            check): a separate mode, since it bypasses the pass; the large
            leg runs it too;
  weighted  unbalanced classes (d = 1e5, n = 1e3, one positive in ten): the
            Section 4.1 choice of C on the device, then whole solves with the
            Section 4.5 class weights, pass and representer iterations
            (--no-weighted skips it);
  direct    the direct (d+1)^2 branch on d=300 n=5e4 and d=54 n=581012
            (--no-direct skips it);
  iterative the iterative branch (PSQMR, then the proximal term of eq-T;
            and eq-T from the start) on d=6000 n=70000 and d=20000 n=1e5
            (--no-iterative skips it);
  cpu_baseline  one whole solve of the FP64 oracle on the host cores;
  oracle_error  the last timed plain solve against that oracle solve.
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6
FP32_MFMA_PEAK_TFS = 157.3
METRIC = "solves/s at rel. KKT 1e-5 (d=1e5,n=1e3), batched vs plain; p50/p99 latency"
PASS_KERNEL_SRCS = [os.path.join(ROOT, "paper_2305_12019_amd", "csrc", f)
                    for f in ("kernels_iter.hip", "dwd_device.h", "dwd_internal.h")]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pmc_pass2_d1e5_n1e3_f32.md")


def pass_bytes(d, ld, n, elem):
    """Algorithmic HBM bytes of one Z~ [s, alpha] pass: the d x n data once,
    plus u, rho read and w, u, rho written (FP64, length ld), plus the two
    n-vectors.  (u and rho are read and written in place: 5 ld-vectors.)"""
    return d * n * elem + 5 * ld * 8 + 2 * n * 8


def recorded_traffic(bpl):
    """HBM bytes per pass launch from the committed rocprofv3 counter summary,
    provided it was taken on the pass kernel's current source (its hash is
    recorded there); else None."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    m = re.search(r"source sha256: ([0-9a-f]{64})", text)
    t = re.search(r"hbm bytes per launch: ([0-9.eE+]+)", text)
    if not m or not t:
        return None
    h = hashlib.sha256()
    for f in PASS_KERNEL_SRCS:
        h.update(open(f, "rb").read())
    if h.hexdigest() != m.group(1):
        return None
    val = float(t.group(1))
    return {"bytes_per_launch": val, "ratio_to_algorithmic": val / bpl}


def copy_bandwidth(torch, dev, nbytes=2 << 30, reps=10):
    """Achievable device-to-device copy rate (read + write bytes / time)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / s / 1e9


def cpu_baseline(X, y, wl, gpu):
    """One whole solve of the FP64 oracle on the host: set-up plus Algorithm 1
    to the same tolerance on the same data.  The same solve also states the
    error of the GPU's plain solve `gpu` (a dwd.Problem.solve result) against
    the FP64 oracle: the reduced objective of Section 2 at both (w, beta),
    ||w - w_o|| / ||w_o||, and both iteration counts."""
    import numpy as np
    from oracle import dwd_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = len(os.sched_getaffinity(0))
    Xd = np.asarray(X, dtype=np.float64)
    t0 = time.perf_counter()
    ref = O.solve(Xd, y, wl.C, wl.q, tol=wl.tol, max_iter=2000)
    s = time.perf_counter() - t0

    def obj(w, beta):
        w = np.asarray(w, np.float64)
        return float(O.reduced_objective(Xd, y, w / max(1.0, np.linalg.norm(w)), beta, wl.C, wl.q))

    f_gpu, f_ref = obj(gpu["w"], gpu["beta"]), obj(ref["w"], ref["beta"])
    err = {"reference": f"FP64 oracle, same data and tolerance ({wl.tol:g})",
           "rel_obj": abs(f_gpu - f_ref) / abs(f_ref),
           "rel_w": float(np.linalg.norm(gpu["w"] - ref["w"]) / np.linalg.norm(ref["w"])),
           "rel_beta": abs(gpu["beta"] - ref["beta"]) / max(1.0, abs(ref["beta"])),
           "iters_gpu": int(gpu["info"]["iters"]), "iters_oracle": int(ref["iters"]),
           "n_double_gpu": int(gpu["info"]["n_double"]), "n_double_oracle": int(ref["n_double"]),
           "kkt_check_gpu": gpu["info"]["kkt_check"]}
    return {"value": 1.0 / s, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"one whole oracle solve of the same d=1e5 n=1e3 problem to rel. KKT "
                       f"{wl.tol:g}: {ref['iters']} iterations, converged={bool(ref['converged'])}, "
                       f"{s:.1f} s")}, err


def batched_leg(dwd, Xd, y, tol, grid):
    """64 (C, q) problems on one X: dwd_solve_batch against plain solves.
    The timed batch runs as it would in use (graph-replayed chunks, no
    events); a second, profiled batch (every pass launch between HIP events,
    eager launches) gives the pass time behind the MFMA rate."""
    import numpy as np
    plist = [dict(C=C, q=q, tol=tol) for C, q in grid]
    P = dwd.Problem(Xd, y, storage="f32")
    P.solve_batch([dict(C=grid[0][0], q=grid[0][1], tol=tol, max_iter=20)])  # warm-up
    P.solve_batch(plist)  # (tile choice per slot count, cached for the timed run)
    t = time.perf_counter()
    rb = P.solve_batch(plist)
    t_batch = time.perf_counter() - t
    rprof = P.solve_batch([dict(q_, profile=1) for q_ in plist])
    t = time.perf_counter()
    plain = [P.solve(C, q, tol=tol, want_state=False) for C, q in grid]
    t_plain = time.perf_counter() - t
    d, n = P.d, P.n
    P.close()
    ib = rb["info"]
    it_total = sum(i["iters"] for i in ib)
    ip = rprof["info"]
    flops = 2.0 * d * n * sum(i["iters"] for i in ip)
    pass_s = ip[0]["stream_ms"] / 1e3
    achieved = flops / pass_s / 1e12 if pass_s > 0 else None
    # per-launch roofline: a launch at iteration t serves the problems still
    # running (b of them); its floor is the larger of the MFMA time of its
    # 2 d n b FLOP and the HBM time of X (once per 64 problems) plus the five
    # FP64 d-vectors per problem it reads or writes
    ld = ((d + 1023) // 1024) * 1024
    its = [i["iters"] for i in ip]
    floor_s = 0.0
    for t in range(max(its)):
        b = sum(1 for k in its if k > t)
        floor_s += max(2.0 * d * n * b / (FP32_MFMA_PEAK_TFS * 1e12),
                       (d * n * 4 * ((b + 63) // 64) + b * 5 * ld * 8) / (HBM_PEAK_GBS * 1e9))
    wdiff = max(np.linalg.norm(rb["W"][j] - plain[j]["w"]) / np.linalg.norm(plain[j]["w"])
                for j in range(len(grid)))
    # the same 64 problems in the representer mode, batched and one by one
    P = dwd.Problem(Xd, y, storage="f32")
    P.solve_batch([dict(C=grid[0][0], q=grid[0][1], tol=tol, max_iter=20, representer=1)])
    t = time.perf_counter()
    rr = P.solve_batch([dict(C=C, q=q, tol=tol, representer=1) for C, q in grid])
    t_rb = time.perf_counter() - t
    t = time.perf_counter()
    rp = [P.solve(C, q, tol=tol, want_state=False, representer=1) for C, q in grid]
    t_rp = time.perf_counter() - t
    P.close()
    rep = {"batched_solves_per_s": len(grid) / t_rb, "batched_s": t_rb,
           "plain_solves_per_s": len(grid) / t_rp, "plain_s": t_rp, "gain": t_rp / t_rb,
           "gain_vs_pass_plain": t_plain / t_rb,
           "converged_batched": sum(i["converged"] for i in rr["info"]),
           "converged_plain": sum(r["info"]["converged"] for r in rp),
           "kkt_check_max_batched": max(i["kkt_check"] for i in rr["info"]),
           "kkt_check_max_plain": max(r["info"]["kkt_check"] for r in rp)}
    return {
        "problems": len(grid), "grid": "C = 10^(-2+4a/15), a=0..15, x q in {0.5,1,2,4}",
        "batched_solves_per_s": len(grid) / t_batch, "batched_s": t_batch,
        "plain_solves_per_s": len(grid) / t_plain, "plain_s": t_plain,
        "gain": t_plain / t_batch,
        "converged_batched": sum(i["converged"] for i in ib),
        "converged_plain": sum(p["info"]["converged"] for p in plain),
        "kkt_check_max_batched": max(i["kkt_check"] for i in ib),
        "kkt_check_max_plain": max(p["info"]["kkt_check"] for p in plain),
        "max_rel_w_diff_batched_vs_plain": wdiff,
        "iters_max": max(i["iters"] for i in ib), "iters_sum": it_total,
        "resumed": sum(i["resumed"] for i in ib),
        "representer": rep,
        "mfma": {"kernel": "k_pass_b<float,float,NB> (Z~ [s_1..s_B], FP32 MFMA, FP64 sums over "
                           "K tiles; resumed problems continue on the FP64 MFMA variant)",
                 "achieved": achieved, "peak": FP32_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                 "frac": (achieved / FP32_MFMA_PEAK_TFS) if achieved else None,
                 "flops": flops, "pass_ms": ip[0]["stream_ms"],
                 "roofline_floor_ms": floor_s * 1e3,
                 "roofline_frac": (floor_s / pass_s) if pass_s > 0 else None,
                 "launches": ip[0]["stream_launches"],
                 "measured_on": "a second, profiled run of the same batch"},
        "graph_launches": ib[0]["graph_launches"],
    }


def serving_leg(dwd, torch, dev, count, tol, budget_gb=64.0, fixed_rate=30.0):
    """Replay the first `count` requests of the seeded request stream with
    dwd_serve (HBM budget `budget_gb`): at 0.75x the measured plain capacity
    and at a fixed rate (p50/p99 latency), and with every request queued at
    t = 0 (solves/s against the plain per-request solves), pass and
    representer iterations.  Dense data is drawn on the device
    (synth.request_dense_data_device), sparse data on the host."""
    import numpy as np
    import synth
    base = synth.request_stream(count, rate=1.0)
    reqs = []
    for r in base:
        if r.layout == "csr":
            ip, ix, val, y = synth.request_csr_data(r)
            reqs.append(dict(csr=(ip, ix, val, r.d), y=y))
        else:
            X, y = synth.request_dense_data_device(r, torch, dev)
            reqs.append(dict(X=X, y=y))
        reqs[-1]["params"] = dict(C=r.C, q=r.q, tol=tol, storage=r.storage)
    torch.cuda.synchronize()

    def plain(rep):
        """The requests solved one after another (set-up included)."""
        ts, conv, nrep = [], 0, 0
        for rq in reqs:
            p = rq["params"]
            t = time.perf_counter()
            if "csr" in rq:
                P = dwd.Problem(csr=rq["csr"], y=rq["y"], storage=p["storage"])
            else:
                P = dwd.Problem(rq["X"], rq["y"], storage=p["storage"])
            res = P.solve(p["C"], p["q"], tol=tol, want_state=False, representer=rep)
            P.close()
            ts.append(time.perf_counter() - t)
            conv += res["info"]["converged"]
            nrep += res["info"]["representer"]
        return len(reqs) / sum(ts), ts, conv, nrep

    cap, t_plain, conv_plain, _ = plain(0)
    cap_auto, t_plain_auto, conv_plain_auto, nrep_auto = plain(2)
    budget = budget_gb * (1 << 30)

    def replay(rate, rep=0):
        if rate is None:
            for rq in reqs:
                rq["t_arrival"] = 0.0
        else:  # the same requests, arrival gaps of a Poisson stream at `rate`
            for rq, r in zip(reqs, synth.request_stream(count, rate=rate)):
                rq["t_arrival"] = r.t_arrival
        for rq in reqs:
            rq["params"] = dict(rq["params"], representer=rep)
        t = time.perf_counter()
        out = dwd.serve(reqs, hbm_budget_bytes=budget)
        el = time.perf_counter() - t
        lat = np.array([o["latency"] for o in out]) * 1e3
        return {"solves_per_s": len(reqs) / el, "span_s": el,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "ok": sum(o["status"] == 0 for o in out),
                "kkt_check_max": max(o["info"]["kkt_check"] for o in out),
                "representer_requests": sum(o["info"]["representer"] for o in out)}

    # latency under load with the per-request iteration choice (representer = 2)
    lam = 0.75 * cap_auto
    at_075 = replay(lam, rep=2)
    at_fixed = replay(fixed_rate, rep=2)
    sat = replay(None)
    sat_rep = replay(None, rep=1)
    sat_auto = replay(None, rep=2)
    kinds = {"dense_f32": 0, "dense_bf16": 0, "csr": 0}
    for r in base:
        kinds["csr" if r.layout == "csr" else "dense_" + r.storage] += 1
    out = {
        "requests": len(reqs), "stream": "synth.request_stream(seed 5), first requests",
        "mix": kinds, "hbm_budget_gb": budget_gb,
        "plain_solves_per_s": cap,
        "plain_p50_ms": float(np.percentile(np.array(t_plain) * 1e3, 50)),
        "converged_plain": conv_plain,
        "plain_auto": {"solves_per_s": cap_auto, "converged": conv_plain_auto,
                       "representer_requests": nrep_auto,
                       "p50_ms": float(np.percentile(np.array(t_plain_auto) * 1e3, 50)),
                       "rule": "representer iteration when 8 n^2 < Z bytes + 5 FP64 d-vectors"},
        "latency_policy": "representer = 2 (per-request iteration form)",
        "arrival_rate_per_s": lam, "p50_ms": at_075["p50_ms"], "p99_ms": at_075["p99_ms"],
        "ok": at_075["ok"], "span_s": at_075["span_s"],
        "fixed_rate": dict(at_fixed, arrival_rate_per_s=fixed_rate),
        "saturated": dict(sat, gain_vs_plain=sat["solves_per_s"] / cap),
        "representer_saturated": dict(sat_rep, gain_vs_plain=sat_rep["solves_per_s"] / cap),
        "auto_saturated": dict(sat_auto, gain_vs_plain=sat_auto["solves_per_s"] / cap,
                               gain_vs_plain_auto=sat_auto["solves_per_s"] / cap_auto),
    }
    del reqs
    torch.cuda.empty_cache()
    return out


def weighted_leg(dwd, torch, dev, steps):
    """Unbalanced classes (d=1e5, n=1000, one positive in ten, FP32 storage):
    the Section 4.1 choice of C on the device, then whole solves with the
    Section 4.5 class weights (set-up included, like the plain leg), in the
    pass and the representer iteration."""
    import numpy as np
    import synth
    wl = synth.UNBALANCED_F32
    X, y = synth.two_class(wl.data)
    Xd = torch.from_numpy(X).to(dev)
    del X
    torch.cuda.synchronize()
    P = dwd.Problem(Xd, y, storage="f32")
    P.suggest_C(wl.q)
    t = time.perf_counter()
    C = P.suggest_C(wl.q)
    c_ms = (time.perf_counter() - t) * 1e3
    P.close()
    out = {"workload": wl.name, "d": wl.data.d, "n": wl.data.n, "n_pos": int((y > 0).sum()),
           "q": wl.q, "tol": wl.tol, "C_suggested": C, "suggest_C_ms": c_ms}

    def one(rep, cw):
        P = dwd.Problem(Xd, y, storage="f32")
        r = P.solve(C, wl.q, tol=wl.tol, want_state=False, class_weights=cw, representer=rep)
        P.close()
        return r["info"]

    for rep in (0, 1):
        one(rep, 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = [one(rep, 1) for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        out["representer" if rep else "pass"] = {
            "solves_per_s": steps / el, "ms_per_solve": el / steps * 1e3,
            "iters": int(np.median([i["iters"] for i in infos])),
            "converged": all(i["converged"] == 1 for i in infos),
            "kkt_check_max": max(i["kkt_check"] for i in infos),
            "eta_gap": infos[-1]["eta_gap"]}
    u = one(0, 0)
    out["unweighted_iters"] = u["iters"]
    del Xd
    torch.cuda.empty_cache()
    return out


def direct_leg(dwd, torch, dev, steps):
    """The direct (d+1)^2 branch (Section 3.3.1) on two d << n shapes of the
    paper's UCI/LIBSVM kind (d=300, n=5e4; d=54, n=581012, beyond the SMW
    factor's n <= 65536): whole solves with set-up, FP32 storage, q=1, C=1,
    tol 1e-5.  An iteration reads X twice (two fused sweeps); `sweep_gbs`
    counts the algorithmic bytes of both sweeps (X at d, not the padded
    leading dimension, plus the n-vectors each sweep reads and writes) per
    iteration over the whole iteration time, launches and small kernels
    included."""
    import numpy as np
    import synth
    out = {}
    for d, n, seed in [(300, 50000, 61), (54, 581012, 62)]:
        X, y = synth.random_two_class(d, n, seed=seed, mean=0.4, flip=0.1, pos_frac=0.3,
                                      dtype="f32")
        Xd = torch.from_numpy(X).to(dev)
        del X
        torch.cuda.synchronize()

        def one():
            P = dwd.Problem(Xd, y, storage="f32", solver="direct")
            r = P.solve(1.0, 1.0, tol=1e-5, want_state=False)
            P.close()
            return r["info"]

        one()
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = [one() for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        i = infos[-1]
        us_it = i["solve_ms"] * 1e3 / max(1, i["iters"])
        sweep_bytes = 2 * d * n * 4 + (7 + 8) * n * 8
        out[f"d{d}_n{n}"] = {
            "solves_per_s": steps / el, "ms_per_solve": el / steps * 1e3,
            "setup_ms": float(np.median([x["setup_ms"] for x in infos])),
            "iters": i["iters"], "us_per_iter": us_it,
            "converged": all(x["converged"] == 1 for x in infos),
            "kkt_check_max": max(x["kkt_check"] for x in infos),
            "sweep_gbs": sweep_bytes / (us_it * 1e-6) / 1e9}
        del Xd
        torch.cuda.empty_cache()
    return out


def iterative_leg(dwd, torch, dev):
    """The iterative branch (Section 3.3.3) where neither factor is built:
    d=6000 n=70000 and d=20000 n=1e5, FP32 storage, q=1, C=1, tol 1e-5, one
    whole solve each (set-up with the Lanczos eigenpairs included), with the
    paper's method (PSQMR with T = 0, the proximal term of eq-T after a solve
    of more than 50 steps) and with the proximal term from the first
    iteration.  `pass_gbs` counts the algorithmic bytes of X of every pass
    (two per PSQMR step; with T four per iteration, three when Step 1c keeps
    wbar) over the iteration time."""
    import synth
    out = {}
    for d, n in [(6000, 70000), (20000, 100000)]:
        X, y = synth.random_two_class(d, n, seed=63, mean=0.3, flip=0.05, dtype="f32")
        Xd = torch.from_numpy(X).to(dev)
        del X
        torch.cuda.synchronize()
        for mode, pmax in (("psqmr", 50), ("proximal_from_start", 0)):
            t = time.perf_counter()
            P = dwd.Problem(Xd, y, storage="f32", solver="iterative")
            ts = time.perf_counter() - t
            r = P.solve(1.0, 1.0, tol=1e-5, want_state=False, max_iter=20000, psqmr_max=pmax)
            P.close()
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            i = r["info"]
            # passes: with T from iteration `switch` on, as counted for the T
            # iterations; before it, the PSQMR steps plus Step 1b, Z~ dr and
            # the three-column pass (and Z~^T w after a re-solve)
            t_iters = i["iters"] - max(0, i["psqmr_switch"]) if i["psqmr_switch"] >= 0 else 0
            p_iters = i["iters"] - t_iters
            passes = 2 * i["psqmr_steps"] + 3 * p_iters + 4 * t_iters
            out.setdefault(f"d{d}_n{n}", {})[mode] = {
                "solve_s": el, "setup_s": ts, "iters": i["iters"], "n_double": i["n_double"],
                "psqmr_solves": i["psqmr_solves"], "psqmr_steps": i["psqmr_steps"],
                "psqmr_switch": i["psqmr_switch"],
                "ms_per_iter": i["solve_ms"] / max(1, i["iters"]), "converged": i["converged"],
                "kkt_check": i["kkt_check"],
                "pass_gbs_approx": passes * d * n * 4 / (i["solve_ms"] * 1e-3) / 1e9}
        del Xd
        torch.cuda.empty_cache()
    return out


def large_leg(dwd, torch, dev):
    """Mixed precision on one large problem: BF16 storage against FP32."""
    import synth
    wl = synth.LARGE_BF16
    X, y = synth.two_class(wl.data)
    Xd = torch.from_numpy(X).to(dev)
    del X
    torch.cuda.synchronize()
    out = {"workload": wl.name, "d": wl.data.d, "n": wl.data.n, "q": wl.q, "C": wl.C,
           "tol": wl.tol, "max_iter": 20000}
    for storage, rep in (("bf16", 0), ("f32", 0), ("f32", 1)):
        t = time.perf_counter()
        P = dwd.Problem(Xd, y, storage=storage)
        r = P.solve(wl.C, wl.q, tol=wl.tol, want_state=False, max_iter=20000, representer=rep)
        P.close()
        torch.cuda.synchronize()
        i = r["info"]
        out["representer" if rep else storage] = {
                        "solve_s": time.perf_counter() - t, "setup_ms": i["setup_ms"],
                        "iters": i["iters"], "iters_bf16": i["iters_lowp"],
                        "converged": i["converged"], "kkt_check": i["kkt_check"],
                        "eta_gap": i["eta_gap"], "primal_obj": i["primal_obj"]}
    out["gain_bf16_vs_f32"] = out["f32"]["solve_s"] / out["bf16"]["solve_s"]
    out["gain_representer_vs_f32"] = out["f32"]["solve_s"] / out["representer"]["solve_s"]
    del Xd
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=500, help="0 to skip the serving leg")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-weighted", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--no-iterative", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a 1 GiB device copy (counter calibration) and one solve")
    ap.add_argument("--batch-probe", action="store_true",
                    help="run only a 1 GiB device copy and the 64-problem sweep of the batched "
                         "leg for 24 iterations (counters of the batched pass)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this solver runs on one GPU; runs on several GPUs are not "
              "supported (the path would shard by rows of Z, one all-reduce of the pass "
              "partials per iteration)", file=sys.stderr)
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

    if args.copy_probe or args.batch_probe:
        # counter calibration: a plain copy of known size, then one solve (or
        # the batched sweep, every problem running for 24 iterations)
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        P = dwd.Problem(Xd, y, storage="f32")
        if args.batch_probe:
            r = P.solve_batch([dict(C=C, q=q, tol=wl.tol, max_iter=24)
                               for C, q in synth.sweep_grid()])
            iters = sum(i["iters"] for i in r["info"])
        else:
            iters = P.solve(wl.C, wl.q, tol=wl.tol, want_state=False)["info"]["iters"]
        P.close()
        print(json.dumps({"copy_bytes": 2 * a.numel() * 4, "iters": iters}), flush=True)
        return

    def step(profile, representer=0):
        t = time.perf_counter()
        P = dwd.Problem(Xd, y, storage="f32")
        r = P.solve(wl.C, wl.q, tol=wl.tol, want_state=False, profile=profile,
                    representer=representer)
        P.close()
        return r, (time.perf_counter() - t) * 1e3

    for _ in range(args.warmup):
        step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(0) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] plain: {args.steps} solves in {elapsed:.2f} s", file=sys.stderr, flush=True)
    # the pass timed with HIP events on the solver's stream, in separate
    # solves (the events stay out of the timed region above)
    prof = [step(1)[0]["info"] for _ in range(3)]

    infos = [r["info"] for r, _ in runs]
    lat = np.array([ms for _, ms in runs])
    conv = all(i["converged"] == 1 for i in infos)
    launches = sum(i["stream_launches"] for i in prof)
    kern_ms = sum(i["stream_ms"] for i in prof)
    avg_us = kern_ms / max(launches, 1) * 1e3
    bpl = pass_bytes(d, ld, n, 4)
    achieved = bpl / (avg_us * 1e-6) / 1e9
    iters = int(np.median([i["iters"] for i in infos]))
    # whole-iteration rate: the X bytes of the one pass per iteration over the
    # average time of an iteration of the solve loop (all kernels included)
    it_us = float(np.median([i["solve_ms"] / max(1, i["iters"]) for i in infos])) * 1e3
    it_gbs = d * n * 4 / (it_us * 1e-6) / 1e9
    copy_gbs = copy_bandwidth(torch, dev)
    traffic = recorded_traffic(bpl)
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
        "roofline": {"bound": "hbm", "kernel": "k_pass2<float,4> (Z~ [s, alpha] pass)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "traffic_ratio": traffic["ratio_to_algorithmic"] if traffic else None,
                     "avg_launch_us": avg_us, "launches": launches,
                     "measured_on": "HIP events around every pass on the solver's stream, "
                                    "3 solves after the timed ones",
                     "iteration_us": it_us, "iteration_gbs": it_gbs,
                     "iteration_frac": it_gbs / HBM_PEAK_GBS,
                     "bytes_per_launch": bpl,
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
    }
    # representer mode on the same workload (a separate mode: no pass per iteration)
    for _ in range(max(1, args.warmup)):
        step(0, 1)
    torch.cuda.synchronize()
    t0r = time.perf_counter()
    rruns = [step(0, 1) for _ in range(args.steps)]
    torch.cuda.synchronize()
    er = time.perf_counter() - t0r
    rinfo = [r["info"] for r, _ in rruns]
    out["representer"] = {
        "solves_per_s": args.steps / er, "ms_per_solve": er / args.steps * 1e3,
        "iters": int(np.median([i["iters"] for i in rinfo])),
        "converged": all(i["converged"] == 1 for i in rinfo),
        "kkt_check_max": max(i["kkt_check"] for i in rinfo),
        "gain_vs_pass": (args.steps / er) / out["value"],
        "latency_ms": {"p50": float(np.percentile([ms for _, ms in rruns], 50)),
                       "p99": float(np.percentile([ms for _, ms in rruns], 99))}}
    if not args.no_batched:
        out["batched"] = batched_leg(dwd, Xd, y, wl.tol, synth.sweep_grid())
        print(f"[bench] batched: gain {out['batched']['gain']:.2f}", file=sys.stderr, flush=True)
    if not args.no_weighted:
        out["weighted"] = weighted_leg(dwd, torch, dev, args.steps)
        print("[bench] weighted done", file=sys.stderr, flush=True)
    if not args.no_direct:
        out["direct"] = direct_leg(dwd, torch, dev, args.steps)
        print("[bench] direct done", file=sys.stderr, flush=True)
    if not args.no_iterative:
        out["iterative"] = iterative_leg(dwd, torch, dev)
        print("[bench] iterative done", file=sys.stderr, flush=True)
    if args.serve_requests > 0:
        del Xd
        torch.cuda.empty_cache()
        out["serving"] = serving_leg(dwd, torch, dev, args.serve_requests, wl.tol)
        print("[bench] serving done", file=sys.stderr, flush=True)
    if not args.no_large:
        if args.serve_requests <= 0:
            del Xd
            torch.cuda.empty_cache()
        out["large"] = large_leg(dwd, torch, dev)
        print("[bench] large done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["oracle_error"] = cpu_baseline(X, y, wl, runs[-1][0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
