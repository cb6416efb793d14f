"""The stored values in tests/golden/ (written from the oracle by
tests/golden/make_golden.py) against mathematics that does not go through
the oracle, and the oracle against them (it must still reproduce them)."""
import json
import os

import numpy as np
import pytest
import scipy.optimize as sopt

import synth
from oracle import dwd_oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_kappa_is_the_infimum_of_the_conjugate():
    # Section 2: inf_{r>0} r^-q + r = kappa(q) (alpha = 1), by a bounded
    # scalar minimisation; the oracle reproduces the stored values.
    g = _load("kappa_q.json")
    for q, k in zip(g["q"], g["kappa"]):
        res = sopt.minimize_scalar(lambda r: r ** -q + r, bounds=(1e-3, 1e3), method="bounded",
                                   options={"xatol": 1e-12})
        assert abs(res.fun - k) <= 1e-9 * k, (q, res.fun, k)
        assert O.kappa(q) == k


def test_prox_q1_values_solve_the_cubic():
    # Section 3.2, q = 1: s > 0 is the prox of theta_1 iff
    # -1/s^2 + sigma (s - a) = 0, i.e. sigma s^2 (s - a) = 1.
    g = _load("prox_q1.json")
    for a, sigma, s in g["rows_a_sigma_s"]:
        assert s > 0
        lhs = sigma * s * s * (s - a)
        scale = max(1.0, sigma * s * s * (abs(s) + abs(a)))
        assert abs(lhs - 1.0) <= 1e-12 * scale, (a, sigma, s, lhs)
        assert float(O.prox_cubic_q1(np.array([a]), sigma)[0]) == s


def test_small_solution_is_the_optimum():
    # The stored tight solution: inside the ball, its reduced objective
    # matches a library solver of the reduced problem (Section 2, reading R3),
    # and the oracle still reproduces it.
    g = _load("small_f64_solution.json")
    wl = synth.SMALL_F64
    assert g["inputs"]["seed"] == wl.data.seed and g["inputs"]["d"] == wl.data.d
    X, y = synth.two_class(wl.data)
    w, beta = np.array(g["w"]), g["beta"]
    assert g["converged"] and np.linalg.norm(w) <= 1.0 + 1e-9
    C, q, d = wl.C, wl.q, X.shape[1]
    ts = (q / C) ** (1 / (q + 1))

    def f(v):
        m = y * (X @ v[:d] + v[d])
        hi = m >= ts
        mm = np.where(hi, m, 1.0)
        val = np.where(hi, mm ** -q, ts ** -q + C * (ts - m))
        dv = np.where(hi, -q * mm ** (-q - 1), -C) * y
        return val.sum(), np.concatenate([X.T @ dv, [dv.sum()]])

    cons = [{"type": "ineq", "fun": lambda v: 1.0 - v[:d] @ v[:d],
             "jac": lambda v: np.concatenate([-2 * v[:d], [0.0]])}]
    res = sopt.minimize(f, np.zeros(d + 1), jac=True, method="SLSQP", constraints=cons,
                        options={"ftol": 1e-15, "maxiter": 3000})
    assert abs(g["reduced_objective"] - res.fun) <= 1e-7 * abs(res.fun)
    assert f(np.concatenate([w / max(1.0, np.linalg.norm(w)), [beta]]))[0] == pytest.approx(
        g["reduced_objective"], rel=1e-12)
    ref = O.solve(X, y, C, q, tol=1e-9, max_iter=20000)
    assert ref["iters"] == g["iters"]
    assert np.allclose(ref["w"], w, rtol=0, atol=1e-13) and abs(ref["beta"] - beta) <= 1e-13


def _dual_feasible(alpha, y, C):
    """Euclidean projection of alpha onto {0 <= a <= C, y^T a = 0} (the dual
    feasible set of Section 2 with e = 1), by bisection on the multiplier of
    the equality."""
    f = lambda lam: y @ np.clip(alpha - lam * y, 0.0, C)
    lo, hi = -C - np.abs(alpha).max() - 1, C + np.abs(alpha).max() + 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 0 else (lo, mid)
    return np.clip(alpha - 0.5 * (lo + hi) * y, 0.0, C)


def test_hdlss_solution_is_certified_by_duality():
    # The stored tight solution at d = 1e5, n = 1e3, without the oracle:
    # from the stored multipliers, the optimality relation of Section 2
    # (w = Z alpha / ||Z alpha|| when Z alpha != 0) recovers w, whose stored
    # probes and reduced objective it must reproduce; and the dual objective
    # of Section 2 at a feasible projection of alpha bounds the optimum from
    # below (weak duality), within 1e-7 of the stored objective.
    g = _load("hdlss_f32_solution.json")
    wl = synth.HDLSS_F32
    assert g["inputs"]["seed"] == wl.data.seed and g["inputs"]["d"] == wl.data.d
    assert g["converged"]
    X, y = synth.two_class(wl.data)
    C, q = wl.C, wl.q
    alpha = np.array(g["alpha"])
    za = np.zeros(X.shape[1])
    for r0 in range(0, X.shape[0], 100):
        za += X[r0:r0 + 100].astype(np.float64).T @ (alpha[r0:r0 + 100] * y[r0:r0 + 100])
    w = za / np.linalg.norm(za)
    assert abs(np.linalg.norm(w) - g["w_norm"]) <= 1e-7
    assert np.max(np.abs(w[:32] - np.array(g["w_head"]))) <= 1e-7 * np.abs(w).max()
    V = np.random.default_rng(20230519).standard_normal((16, w.size))
    V /= np.linalg.norm(V, axis=1)[:, None]
    assert np.max(np.abs(V @ w - np.array(g["w_proj"]))) <= 1e-7
    # reduced objective (Section 2 with xi eliminated) at (w, beta)
    ts = (q / C) ** (1 / (q + 1))
    m = y * (np.concatenate([X[r0:r0 + 100].astype(np.float64) @ w
                             for r0 in range(0, X.shape[0], 100)]) + g["beta"])
    hi = m >= ts
    prim = float(np.sum(np.where(hi, np.where(hi, m, 1.0) ** -q, ts ** -q + C * (ts - m))))
    assert abs(prim - g["reduced_objective"]) <= 1e-7 * abs(prim), (prim, g["reduced_objective"])
    # weak duality: kappa sum a^(q/(q+1)) - ||Z a|| <= optimum <= prim
    a = _dual_feasible(alpha, y, C)
    zf = np.zeros(X.shape[1])
    for r0 in range(0, X.shape[0], 100):
        zf += X[r0:r0 + 100].astype(np.float64).T @ (a[r0:r0 + 100] * y[r0:r0 + 100])
    kappa = (q + 1.0) / q * q ** (1.0 / (q + 1.0))
    dual = kappa * float(np.sum(a ** (q / (q + 1.0)))) - float(np.linalg.norm(zf))
    assert dual <= g["reduced_objective"] * (1 + 1e-12)
    assert g["reduced_objective"] - dual <= 1e-7 * abs(g["reduced_objective"]), \
        (g["reduced_objective"], dual)
