"""Pins of the oracle's iterative branch (Section 3.3.3): PSQMR, the Lanczos
eigenpairs, the proximal T of eq-T with its closed-form inverse and the Schur
complement of eq-schur, and whole solves that switch to T."""
import numpy as np
import pytest
import scipy.optimize as sopt

import synth
from oracle import dwd_oracle as O


@pytest.mark.parametrize("kind", ["spd", "indefinite"])
def test_psqmr_solves_symmetric_systems(kind):
    rng = np.random.default_rng(1)
    m = 40
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    ev = rng.uniform(0.5, 20.0, m)
    if kind == "indefinite":
        ev[::3] *= -1.0
    A = (Q * ev) @ Q.T
    b = rng.standard_normal(m)
    x, steps, ok = O.psqmr(lambda v: A @ v, b, np.zeros(m), lambda v: v, 1e-10, 500)
    assert ok and steps <= 3 * m
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)
    # an exact preconditioner: one step
    Ainv = np.linalg.inv(A) if kind == "spd" else None
    if Ainv is not None:
        x1, s1, ok1 = O.psqmr(lambda v: A @ v, b, np.zeros(m), lambda v: Ainv @ v, 1e-9, 5)
        assert ok1 and s1 == 1


def test_psqmr_warm_start_at_the_solution_takes_no_step():
    rng = np.random.default_rng(2)
    A = np.diag(rng.uniform(1, 3, 10))
    b = rng.standard_normal(10)
    x, steps, ok = O.psqmr(lambda v: A @ v, b, np.linalg.solve(A, b), lambda v: v, 1e-12, 10)
    assert ok and steps == 0


def test_lanczos_top_eigenpairs_match_a_dense_eigensolver():
    X, y = synth.random_two_class(60, 200, seed=3, log_scale=1.0)
    Zt, _ = O.scale_data(X, y)
    S = Zt @ Zt.T
    lam, V = O.top_eigenpairs(lambda v: S @ v, 60, 8)
    ref = np.sort(np.linalg.eigvalsh(S))[::-1][:8]
    assert np.allclose(lam, ref, rtol=1e-9)
    assert np.allclose(V.T @ V, np.eye(8), atol=1e-8)
    assert np.linalg.norm(S @ V - V * lam) <= 1e-7 * lam[0]


@pytest.fixture(scope="module")
def factor():
    X, y = synth.random_two_class(70, 50, seed=4, mean=0.6, log_scale=0.5)
    Zt, _ = O.scale_data(X, y)
    return Zt, y, O.IterativeFactor(Zt, y, mu=1.3, ell=6, psqmr_max=50)


def test_proximal_T_is_positive_semidefinite(factor):
    Zt, y, F = factor
    d = Zt.shape[0]
    T = np.column_stack([F.T_apply(e) for e in np.eye(d)])
    assert np.allclose(T, T.T, atol=1e-10)
    assert np.linalg.eigvalsh(T).min() >= -1e-9 * F.lam[0]


def test_closed_form_inverse_and_schur_solve(factor):
    Zt, y, F = factor
    d = Zt.shape[0]
    T = np.column_stack([F.T_apply(e) for e in np.eye(d)])
    Mw = Zt @ Zt.T + 1.3 * np.eye(d) + T
    rng = np.random.default_rng(5)
    x = rng.standard_normal(d)
    assert np.allclose(F.Mw_inv(x), np.linalg.solve(Mw, x), rtol=1e-9, atol=1e-11)
    AT = np.zeros((d + 1, d + 1))
    AT[:d, :d] = Mw
    AT[:d, d] = AT[d, :d] = Zt @ y
    AT[d, d] = y @ y
    hw, hb = rng.standard_normal(d), 0.7
    w, b = F.solve_T(hw, hb)
    ref = np.linalg.solve(AT, np.concatenate([hw, [hb]]))
    assert np.allclose(np.concatenate([w, [b]]), ref, rtol=1e-9, atol=1e-11)


def test_psqmr_solve_of_eq_linsys_meets_the_tolerance(factor):
    Zt, y, F = factor
    d = Zt.shape[0]
    rng = np.random.default_rng(6)
    hw, hb = rng.standard_normal(d), -0.3
    w, b, ok = F.solve_psqmr(hw, hb, np.zeros(d), 0.0, 1e-10)
    assert ok
    top, bot = O.linsys_matrix_apply(Zt, y, 1.3, w, b)
    assert np.sqrt(np.sum((top - hw) ** 2) + (bot - hb) ** 2) <= 1e-10
    ws, bs = O.SMWFactor(Zt, y, 1.3).solve(hw, hb)
    assert np.allclose(w, ws, rtol=1e-7, atol=1e-9)


def _slsqp(X, y, C, q):
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
    return sopt.minimize(f, np.zeros(d + 1), jac=True, method="SLSQP", constraints=cons,
                         options={"ftol": 1e-15, "maxiter": 3000})


@pytest.mark.parametrize("psqmr_max", [50, 3, 0])
def test_iterative_solves_reach_the_optimum(psqmr_max):
    # 50: PSQMR throughout (it converges within a few steps here); 3: the
    # switch to T happens during the solve; 0: T from the first iteration.
    X, y = synth.random_two_class(40, 30, seed=7, mean=0.7, log_scale=0.5)
    C, q = 2.0, 1.0
    sol = O.solve(X, y, C, q, tol=1e-9, max_iter=40000, solver="iterative", ell=6,
                  psqmr_max=psqmr_max)
    assert sol["converged"]
    if psqmr_max == 50:
        assert not sol["used_T"] and max(sol["psqmr_steps"]) <= 50
    else:
        assert sol["used_T"]
    res = _slsqp(X, y, C, q)
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    f = O.reduced_objective(X, y, w, sol["beta"], C, q)
    assert abs(f - res.fun) <= 1e-7 * abs(res.fun)
    assert np.linalg.norm(w - res.x[:-1]) <= 1e-4 * np.linalg.norm(res.x[:-1])


def test_iterative_without_switch_follows_the_smw_iterates():
    # With a tiny eps_k constant PSQMR solves each system to ~1e-13, so the
    # first iterates agree with those of the exact SMW solves.
    X, y = synth.random_two_class(40, 30, seed=8, mean=0.7)
    for k in (1, 2, 5, 20):
        a = O.solve(X, y, 1.0, 1.0, tol=1e-300, max_iter=k, solver="smw", eps_c=1e-12)
        b = O.solve(X, y, 1.0, 1.0, tol=1e-300, max_iter=k, solver="iterative", ell=6,
                    eps_c=1e-12, psqmr_max=200)
        assert not b["used_T"]
        for key in ("w", "alpha", "r", "xi"):
            assert np.allclose(a[key], b[key], rtol=1e-8, atol=1e-10), (k, key)
