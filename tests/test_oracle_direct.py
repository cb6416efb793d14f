"""Pins of the oracle's direct branch (Section 3.3.1): the Cholesky factor of
the whole (d+1) x (d+1) eq-linsys matrix, and the solver choice printed with
the paper's pseudo-code.  The SMW branch is pinned on its own in
test_oracle_pins.py; here the direct branch is checked against a dense solve
of the operator, against the SMW branch step by step, and against a library
convex solver on a d < n problem."""
import numpy as np
import pytest
import scipy.optimize as sopt

import synth
from oracle import dwd_oracle as O


def _dense_operator(Zt, y, mu):
    """eq-linsys matrix assembled column by column from linsys_matrix_apply."""
    d = Zt.shape[0]
    A = np.empty((d + 1, d + 1))
    for j in range(d + 1):
        e = np.zeros(d + 1)
        e[j] = 1.0
        top, bot = O.linsys_matrix_apply(Zt, y, mu, e[:d], e[d])
        A[:d, j] = top
        A[d, j] = bot
    return A


@pytest.mark.parametrize("d,n,mu", [(12, 40, 1.0), (30, 25, 2.5), (5, 200, 0.3)])
def test_direct_solve_matches_dense_solve_and_smw(d, n, mu):
    X, y = synth.random_two_class(d, n, seed=d + n)
    Zt, _ = O.scale_data(X, y)
    rng = np.random.default_rng(3)
    hw, hb = rng.standard_normal(d), float(rng.standard_normal())
    F = O.DirectFactor(Zt, y, mu)
    w, b = F.solve(hw, hb)
    A = _dense_operator(Zt, y, mu)
    x = np.linalg.solve(A, np.concatenate([hw, [hb]]))
    assert np.allclose(w, x[:d], rtol=1e-10, atol=1e-12)
    assert b == pytest.approx(x[d], rel=1e-10, abs=1e-12)
    ws, bs = O.SMWFactor(Zt, y, mu).solve(hw, hb)
    assert np.allclose(w, ws, rtol=1e-9, atol=1e-11)
    assert b == pytest.approx(bs, rel=1e-9, abs=1e-11)


@pytest.mark.parametrize("d,n", [(20, 150), (60, 30)])
def test_direct_iterates_equal_smw_iterates(d, n):
    X, y = synth.random_two_class(d, n, seed=7 * d + n, mean=0.6)
    e = synth.penalty_vector(n, seed=n)
    for k in (1, 2, 5, 20):
        a = O.solve(X, y, 2.0, 1.0, tol=1e-300, max_iter=k, solver="smw", weights=True, e=e)
        b = O.solve(X, y, 2.0, 1.0, tol=1e-300, max_iter=k, solver="direct", weights=True, e=e)
        for key in ("r", "xi", "alpha", "w", "u", "rho"):
            assert np.allclose(a[key], b[key], rtol=1e-9, atol=1e-12), (k, key)
        assert a["sigma"] == b["sigma"] and a["n_double"] == b["n_double"]


def test_direct_solve_matches_library_convex_solver():
    # d < n: the regime the direct branch is for
    X, y = synth.random_two_class(15, 120, seed=5, mean=0.5, flip=0.15)
    C, q = 1.0, 2.0
    sol = O.solve(X, y, C, q, tol=1e-9, max_iter=40000, solver="direct")
    assert sol["converged"]
    n, d = X.shape
    ts = (q / C) ** (1 / (q + 1))

    def f(v):
        w, b = v[:d], v[d]
        m = y * (X @ w + b)
        hi = m >= ts
        mm = np.where(hi, m, 1.0)
        val = np.where(hi, mm ** -q, ts ** -q + C * (ts - m))
        dv = np.where(hi, -q * mm ** (-q - 1), -C) * y
        return val.sum(), np.concatenate([X.T @ dv, [dv.sum()]])

    cons = [{"type": "ineq", "fun": lambda v: 1.0 - v[:d] @ v[:d],
             "jac": lambda v: np.concatenate([-2 * v[:d], [0.0]])}]
    res = sopt.minimize(f, np.zeros(d + 1), jac=True, method="SLSQP", constraints=cons,
                        options={"ftol": 1e-15, "maxiter": 3000})
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    fo = O.reduced_objective(X, y, w, sol["beta"], C, q)
    assert abs(fo - res.fun) <= 1e-7 * abs(res.fun)
    assert np.linalg.norm(w - res.x[:d]) <= 1e-4 * np.linalg.norm(res.x[:d])


@pytest.mark.parametrize("d,n,want", [(4000, 100, "direct"), (5000, 10**6, "direct"),
                                      (6000, 1000, "smw"), (6000, 1199, "smw"),
                                      (6000, 1200, "iterative"), (100000, 2500, "smw"),
                                      (100000, 2501, "iterative"), (5001, 100, "smw")])
def test_solver_choice_follows_the_printed_rule(d, n, want):
    assert O.select_solver(d, n) == want
