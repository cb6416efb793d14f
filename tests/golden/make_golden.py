"""Write the stored expected values in tests/golden/ from the oracle alone.

Run from the repository root:  python tests/golden/make_golden.py
(and  python tests/golden/make_golden.py hdlss  for the d = 1e5 solution,
which takes minutes).

The paper prints no worked example with numbers (its result tables need the
UCI/LIBSVM data sets), so every stored value here is the oracle's, computed
by this script from seeded synthetic inputs (synth/, which holds no arithmetic
of the method).  tests/test_golden.py checks each value against mathematics
that does not go through the oracle, and checks that the oracle still
reproduces it; tests/test_gpu_parity.py compares the GPU solve with the stored
small solution.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import dwd_oracle as O  # noqa: E402


def _write(name, obj):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(obj, f, indent=1, sort_keys=True)
        f.write("\n")


def kappa_values():
    # Section 2 (dual problem): inf over r > 0 of r^-q + alpha r equals
    # kappa(q) alpha^(q/(q+1)).
    qs = [0.5, 1.0, 2.0, 4.0]
    _write("kappa_q.json", {
        "passage": "Section 2, the conjugate of theta_q in the dual problem",
        "call": "oracle.dwd_oracle.kappa(q)",
        "q": qs, "kappa": [float(O.kappa(q)) for q in qs]})


def prox_q1_values():
    # Section 3.2: the prox of theta_1, s = argmin s^-1 + sigma/2 (s - a)^2.
    a = [-1000.0, -10.0, -1.0, -1e-3, 0.0, 1e-3, 0.5, 1.0, 10.0, 1000.0]
    sig = [1e-3, 1.0, 1e4]
    rows = []
    for aa in a:
        for ss in sig:
            rows.append([aa, ss, float(O.prox_cubic_q1(np.array([aa]), ss)[0])])
    _write("prox_q1.json", {
        "passage": "Section 3.2, the proximal map of theta_q for q = 1",
        "call": "oracle.dwd_oracle.prox_cubic_q1(a, sigma)",
        "rows_a_sigma_s": rows})


def small_solution():
    # Algorithm 1 with the scaling, stopping and sigma rules of Sections
    # 4.2-4.4, on the small FP64 workload, to a tight tolerance.
    wl = synth.SMALL_F64
    X, y = synth.two_class(wl.data)
    ref = O.solve(X, y, wl.C, wl.q, tol=1e-9, max_iter=20000)
    w = np.asarray(ref["w"], np.float64)
    _write("small_f64_solution.json", {
        "passage": "Algorithm 1 (SMW branch) with Sections 4.2-4.4",
        "call": "oracle.dwd_oracle.solve(X, y, C, q, tol=1e-9, max_iter=20000)",
        "inputs": {"workload": wl.name, "d": wl.data.d, "n": wl.data.n, "seed": wl.data.seed,
                   "mean": wl.data.mean, "C": wl.C, "q": wl.q},
        "converged": bool(ref["converged"]), "iters": int(ref["iters"]),
        "w": [float(v) for v in w], "beta": float(ref["beta"]),
        "reduced_objective": float(O.reduced_objective(X, y, w / max(1.0, np.linalg.norm(w)),
                                                      ref["beta"], wl.C, wl.q))})


def _probe_directions(d, count=16, seed=20230519):
    """Fixed seeded unit directions on which a long w is pinned compactly."""
    V = np.random.default_rng(seed).standard_normal((count, d))
    return V / np.linalg.norm(V, axis=1)[:, None]


def hdlss_solution():
    # Algorithm 1 on the d = 1e5, n = 1e3 HDLSS workload (FP32 data of record,
    # computed in FP64) to a tight tolerance.  w has 1e5 entries, so the file
    # keeps its norm, its first 32 entries and its projections on 16 seeded
    # unit directions beside beta, the reduced objective and the multipliers
    # alpha (n values, from which w = Z alpha / ||Z alpha|| and a dual bound
    # follow without the oracle).
    wl = synth.HDLSS_F32
    X, y = synth.two_class(wl.data)
    Xd = X.astype(np.float64)
    ref = O.solve(Xd, y, wl.C, wl.q, tol=1e-9, max_iter=50000)
    w = np.asarray(ref["w"], np.float64)
    V = _probe_directions(w.size)
    _write("hdlss_f32_solution.json", {
        "passage": "Algorithm 1 (SMW branch) with Sections 4.2-4.4",
        "call": "oracle.dwd_oracle.solve(X, y, C, q, tol=1e-9, max_iter=50000)",
        "inputs": {"workload": wl.name, "d": wl.data.d, "n": wl.data.n, "seed": wl.data.seed,
                   "mean": wl.data.mean, "flip": wl.data.flip, "C": wl.C, "q": wl.q},
        "probe_directions": "tests/golden/make_golden.py _probe_directions(d, 16, 20230519)",
        "converged": bool(ref["converged"]), "iters": int(ref["iters"]),
        "beta": float(ref["beta"]), "w_norm": float(np.linalg.norm(w)),
        "w_head": [float(v) for v in w[:32]],
        "w_proj": [float(v) for v in V @ w],
        "alpha": [float(v) for v in ref["alpha"]],
        "reduced_objective": float(O.reduced_objective(Xd, y, w / max(1.0, np.linalg.norm(w)),
                                                      ref["beta"], wl.C, wl.q))})


if __name__ == "__main__":
    if "hdlss" in sys.argv[1:]:
        # (minutes of CPU time: written only on request)
        hdlss_solution()
        sys.exit(0)
    kappa_values()
    prox_q1_values()
    small_solution()
    print("wrote", sorted(f for f in os.listdir(HERE) if f.endswith(".json")))
