"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, a library routine on a special case, an invariant of the problem, or a
brute-force search.  None of these needs a GPU.
"""
import math

import numpy as np
import pytest
import scipy.optimize as sopt

import synth
from oracle import dwd_oracle as O


def small_problem():
    X, y = synth.two_class(synth.SMALL_F64.data)
    return X, y, synth.SMALL_F64.C, synth.SMALL_F64.q


@pytest.fixture(scope="module")
def tight_small():
    """The small FP64 workload solved to relative KKT 1e-9."""
    X, y, C, q = small_problem()
    sol = O.solve(X, y, C, q, tol=1e-9, max_iter=20000)
    assert sol["converged"]
    return X, y, C, q, sol


# --------------------------------------------------------------------------
# Closed forms: the dual constant and the prox.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("q", [0.5, 1.0, 2.0, 4.0])
def test_kappa_is_the_inner_infimum(q):
    # inf_{r>0} r^-q + a r = kappa a^(q/(q+1)) (Lagrangian infimum, Section 2)
    for a in (0.05, 1.0, 7.3):
        res = sopt.minimize_scalar(lambda r: r ** -q + a * r, bounds=(1e-6, 1e4),
                                   method="bounded", options={"xatol": 1e-13})
        grid = np.geomspace(1e-4, 1e4, 400001)
        scan = np.min(grid ** -q + a * grid)
        expected = O.kappa(q) * a ** (q / (q + 1.0))
        assert abs(res.fun - expected) <= 1e-10 * expected
        assert abs(scan - expected) <= 1e-8 * expected


def _positive_real_roots(a, sigma):
    roots = np.roots([1.0, -a, 0.0, -1.0 / sigma])
    return [r.real for r in roots if abs(r.imag) <= 1e-7 * max(1.0, abs(r)) and r.real > 0]


def test_prox_q1_closed_form_matches_library_roots():
    # q = 1: s^3 - a s^2 - 1/sigma = 0 has exactly one positive root.
    for sigma in np.geomspace(1e-3, 1e4, 9):
        a_vals = np.concatenate([-np.geomspace(1e-3, 1e3, 15), [0.0], np.geomspace(1e-3, 1e3, 15)])
        s = O.prox_cubic_q1(a_vals, sigma)
        for a, si in zip(a_vals, s):
            pr = _positive_real_roots(a, sigma)
            assert len(pr) == 1
            assert abs(si - pr[0]) <= 1e-8 * pr[0], (a, sigma, si, pr)
            # residual of the cubic in extended precision
            sl, al = np.longdouble(si), np.longdouble(a)
            res = sl ** 3 - al * sl ** 2 - 1 / np.longdouble(sigma)
            scale = sl ** 3 + abs(al) * sl ** 2 + 1 / np.longdouble(sigma)
            assert abs(float(res / scale)) <= 1e-14


def test_prox_newton_matches_q1_closed_form():
    rng = np.random.default_rng(0)
    for sigma in np.geomspace(1e-3, 1e4, 8):
        a = np.concatenate([rng.uniform(-1e3, 1e3, 400), rng.uniform(-2, 2, 400)])
        s_cf = O.prox_cubic_q1(a, sigma)
        s_nt, steps = O.prox_newton(a, sigma, 1.0, np.ones_like(a), tol=0.0)
        assert np.all(np.abs(s_nt - s_cf) <= 1e-12 * s_cf)
        assert steps.max() <= O.MAX_NEWTON


@pytest.mark.parametrize("q", [0.5, 1.0, 2.0, 4.0, 1.7])
def test_prox_newton_optimality_and_bracket(q):
    rng = np.random.default_rng(1)
    for sigma in (1e-2, 1.0, 1e3):
        a = np.concatenate([rng.uniform(-50, 50, 1000), [-1e3, -1.0, 0.0, 1.0, 1e3]])
        s, _ = O.prox_newton(a, sigma, q, rng.uniform(0.01, 10, a.size), tol=0.0)
        # optimality condition of eq-varphi: s - a = q sigma^-1 / s^(q+1)
        F = sigma * s ** (q + 2) - sigma * a * s ** (q + 1) - q
        scale = sigma * s ** (q + 2) + sigma * np.abs(a) * s ** (q + 1) + q
        assert np.all(np.abs(F) <= 1e-13 * scale)
        lo, hi = O.prox_bracket(a, sigma, q)
        assert np.all(s > 0)
        assert np.all(s >= lo * (1 - 1e-14)) and np.all(s <= hi * (1 + 1e-14))


@pytest.mark.parametrize("q", [0.5, 1.0, 2.0, 4.0])
def test_prox_asymptotes(q):
    sigma = 2.0
    a = np.array([1e4])
    s, _ = O.prox_newton(a, sigma, q, np.ones(1), tol=0.0)
    approx = a + q / (sigma * a ** (q + 1))
    assert abs(s[0] - approx[0]) <= 1e-12 * a[0]
    a = np.array([-1e6])
    s, _ = O.prox_newton(a, sigma, q, np.ones(1), tol=0.0)
    approx = (q / (sigma * np.abs(a))) ** (1 / (q + 1))
    assert abs(s[0] - approx[0]) <= 1e-4 * approx[0]


def test_prox_newton_safeguard_from_far_right_start():
    # q=1, sigma=1, a=-10 from s=5: the raw Newton map leaves (0, inf).
    a = np.array([-10.0])
    raw = 5.0 * (3.0 + a[0] * 25.0) / (2.0 + 125.0)
    assert raw < 0
    s, steps = O.prox_newton(a, 1.0, 1.0, np.array([5.0]), tol=0.0)
    assert abs(s[0] - O.prox_cubic_q1(a, 1.0)[0]) <= 1e-12 * s[0]
    assert steps[0] < O.MAX_NEWTON


def test_prox_is_the_minimiser():
    # The Newton result minimises phi(s) = s^-q + sigma/2 (s-a)^2 over s > 0.
    for q, sigma, a in [(1.0, 3.0, -0.5), (2.0, 0.1, 4.0), (0.5, 40.0, 0.01), (4.0, 1.0, -3.0)]:
        s, _ = O.prox_newton(np.array([a]), sigma, q, np.ones(1), tol=0.0)
        res = sopt.minimize_scalar(lambda t: t ** -q + 0.5 * sigma * (t - a) ** 2,
                                   bounds=(1e-9, 1e3), method="bounded", options={"xatol": 1e-14})
        assert abs(s[0] - res.x) <= 1e-6 * max(1.0, res.x)


# --------------------------------------------------------------------------
# The Sherman-Morrison-Woodbury solve of eq-linsys.
# --------------------------------------------------------------------------

def _dense_A(Zt, y, mu):
    d = Zt.shape[0]
    Zy = Zt @ y
    A = np.zeros((d + 1, d + 1))
    A[:d, :d] = Zt @ Zt.T + mu * np.eye(d)
    A[:d, d] = Zy
    A[d, :d] = Zy
    A[d, d] = y @ y
    return A


@pytest.mark.parametrize("mu", [1.0, 0.3, 4.0])
def test_smw_solve_matches_dense_solve(mu):
    X, y, _, _ = small_problem()
    Zt, _ = O.scale_data(X, y)
    d = Zt.shape[0]
    F = O.SMWFactor(Zt, y, mu)
    A = _dense_A(Zt, y, mu)
    rng = np.random.default_rng(2)
    for _ in range(3):
        h = rng.standard_normal(d + 1)
        ref = np.linalg.solve(A, h)
        w, b = F.solve(h[:d], h[d])
        got = np.concatenate([w, [b]])
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


def test_smw_decomposition_of_A():
    # eq-Anew: A = Dhat + U E U^T with Dhat = diag(mu I, ||y||^2)
    X, y, _, _ = small_problem()
    Zt, _ = O.scale_data(X, y)
    d, n = Zt.shape
    mu = 0.7
    U = np.zeros((d + 1, n + 1))
    U[:d, :n] = Zt
    U[d, :n] = y
    U[d, n] = np.linalg.norm(y)
    E = np.diag(np.concatenate([np.ones(n), [-1.0]]))
    Dhat = np.diag(np.concatenate([mu * np.ones(d), [y @ y]]))
    assert np.allclose(Dhat + U @ E @ U.T, _dense_A(Zt, y, mu), rtol=0, atol=1e-12)


def test_H_inverse_rank_one_formula():
    # eq-H assembled densely against the rank-one update of J^-1
    X, y, _, _ = small_problem()
    Zt, _ = O.scale_data(X, y)
    n = Zt.shape[1]
    mu = 1.3
    F = O.SMWFactor(Zt, y, mu)
    ny = np.linalg.norm(y)
    H = np.zeros((n + 1, n + 1))
    H[:n, :n] = np.eye(n) + Zt.T @ Zt / mu + np.outer(y, y) / ny ** 2
    H[:n, n] = y / ny
    H[n, :n] = y / ny
    rng = np.random.default_rng(3)
    v = rng.standard_normal(n + 1)
    ref = np.linalg.solve(H, v)
    zn, zl = F.H_inv_apply(v[:n], v[n])
    got = np.concatenate([zn, [zl]])
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def _random_state(d, n, seed):
    rng = np.random.default_rng(seed)
    return dict(r=rng.uniform(0.5, 2, n), xi=rng.uniform(0, 1, n), u=rng.standard_normal(d) * 0.1,
                alpha=rng.uniform(0, 1, n), rho=rng.standard_normal(d) * 0.1)


def test_step1a_solution_is_the_argmin_of_the_augmented_lagrangian():
    # Finite differences of L_sigma in (w, beta) vanish at the eq-linsys solution.
    X, y, C, _ = small_problem()
    Zt, _ = O.scale_data(X, y)
    d, n = Zt.shape
    mu, sigma = 1.7, 3.0
    st = _random_state(d, n, 4)

    def L(w, beta):  # w,beta-dependent part of L_sigma (Section 3)
        a = Zt.T @ w + beta * y + st["xi"] - st["r"] - st["alpha"] / sigma
        b = math.sqrt(mu) * (w - st["u"]) - st["rho"] / sigma
        return 0.5 * sigma * (a @ a) + 0.5 * sigma * (b @ b)

    hw, hb = O.linsys_rhs(Zt, y, mu, sigma, st["r"], st["xi"], st["u"], st["alpha"], st["rho"])
    w, beta = O.SMWFactor(Zt, y, mu).solve(hw, hb)
    rng = np.random.default_rng(5)
    h = 1e-3
    for _ in range(5):
        e = rng.standard_normal(d + 1)
        e /= np.linalg.norm(e)
        g_opt = (L(w + h * e[:d], beta + h * e[d]) - L(w - h * e[:d], beta - h * e[d])) / (2 * h)
        w0, b0 = np.zeros(d), 0.0
        g_ref = (L(w0 + h * e[:d], b0 + h * e[d]) - L(w0 - h * e[:d], b0 - h * e[d])) / (2 * h)
        assert abs(g_opt) <= 1e-7 * max(1.0, abs(g_ref))


def test_step2_is_the_argmin_over_u_and_xi():
    rng = np.random.default_rng(6)
    d, n = 5, 4
    Zt = rng.standard_normal((d, n))
    y = np.array([1.0, -1.0, 1.0, -1.0])
    mu, sigma, C, R = 0.8, 2.5, 1.5, 0.7
    w = rng.standard_normal(d)
    beta = 0.3
    st = _random_state(d, n, 7)
    st["rho"] = rng.standard_normal(d)
    Ztw = Zt.T @ w
    u, xi = O.step2(w, beta, st["r"], st["alpha"], st["rho"], Ztw, y, C, sigma, mu, R)

    def Lu(uu):
        b = math.sqrt(mu) * (w - uu) - st["rho"] / sigma
        return 0.5 * sigma * b @ b

    ru = sopt.minimize(Lu, np.zeros(d), method="SLSQP",
                       constraints=[{"type": "ineq", "fun": lambda uu: R * R - uu @ uu}],
                       options={"ftol": 1e-14, "maxiter": 500})

    def Lxi(x):
        a = Ztw + beta * y + x - st["r"] - st["alpha"] / sigma
        return C * np.sum(x) + 0.5 * sigma * a @ a

    rx = sopt.minimize(Lxi, np.ones(n), method="L-BFGS-B", bounds=[(0, None)] * n,
                       options={"ftol": 1e-15, "gtol": 1e-12})
    assert np.linalg.norm(u - ru.x) <= 1e-5
    assert np.linalg.norm(xi - rx.x) <= 1e-5
    assert np.all(xi >= 0) and np.linalg.norm(u) <= R * (1 + 1e-15)


# --------------------------------------------------------------------------
# The whole solve: optimality, duality, boundedness, library and brute force.
# --------------------------------------------------------------------------

def _dual_feasible_projection(alpha, y, C):
    """Euclidean projection onto F_D = {0 <= a <= C, y^T a = 0} (bisection on
    the multiplier of y^T a = 0; y^T clip(a - lam y, 0, C) decreases in lam)."""
    f = lambda lam: y @ np.clip(alpha - lam * y, 0.0, C)
    lo, hi = -C - np.abs(alpha).max() - 1, C + np.abs(alpha).max() + 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            lo = mid
        else:
            hi = mid
    return np.clip(alpha - 0.5 * (lo + hi) * y, 0.0, C)


def _primal_value(X, y, w, beta, C, q):
    # eq-primal at (w, beta) with the best (r, xi): r = m + xi, xi = max(0, t* - m)
    m = y * (X @ w + beta)
    ts = (q / C) ** (1 / (q + 1))
    xi = np.maximum(0.0, ts - m)
    r = m + xi
    return np.sum(r ** -q) + C * np.sum(xi)


def _dual_value(X, y, a, q):
    k = (q + 1) / q * q ** (1 / (q + 1))
    return k * np.sum(a ** (q / (q + 1))) - np.linalg.norm(X.T @ (y * a))


def test_weak_duality_on_random_feasible_pairs():
    X, y, C, q = small_problem()
    rng = np.random.default_rng(8)
    for _ in range(20):
        w = rng.standard_normal(X.shape[1])
        w /= max(1.0, np.linalg.norm(w)) * rng.uniform(1, 3)
        beta = rng.uniform(-2, 2)
        a = _dual_feasible_projection(rng.uniform(0, C, X.shape[0]), y, C)
        assert _dual_value(X, y, a, q) <= _primal_value(X, y, w, beta, C, q)


def test_solution_closes_the_duality_gap(tight_small):
    X, y, C, q, sol = tight_small
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    P = _primal_value(X, y, w, sol["beta"], C, q)
    a = _dual_feasible_projection(sol["alpha"], y, C)
    D = _dual_value(X, y, a, q)
    assert D <= P
    assert (P - D) / (1 + abs(P)) <= 1e-7


def test_solution_satisfies_kkt(tight_small):
    X, y, C, q, sol = tight_small
    assert np.linalg.norm(sol["w"]) <= 1 + 1e-8
    assert np.all(sol["xi"] >= 0) and np.all(sol["r"] > 0)
    assert np.allclose(sol["alpha"], q / sol["r"] ** (q + 1), rtol=1e-4, atol=1e-6)
    Za = X.T @ (y * sol["alpha"])
    cosang = Za @ sol["w"] / (np.linalg.norm(Za) * np.linalg.norm(sol["w"]))
    assert cosang >= 1 - 1e-8
    assert abs(y @ sol["alpha"]) <= 1e-6 * (1 + C)
    assert np.all(sol["alpha"] >= -1e-9) and np.all(sol["alpha"] <= C + 1e-9)
    # complementarity <C - alpha, xi> = 0
    assert abs(sol["xi"] @ (C - sol["alpha"])) <= 1e-6 * (1 + C)


def test_boundedness_proposition(tight_small):
    # Section 2 proposition: 0 <= xi* <= varrho, |beta*| <= K + varrho,
    # r* <= 2(K + varrho), alpha* >= q / (2K + 2 varrho)^(q+1), with e = 1.
    X, y, C, q, sol = tight_small
    n = X.shape[0]
    varrho = (n + C * n) / C
    K = np.max(np.linalg.norm(X, axis=1))
    assert np.all(sol["xi"] >= 0) and np.all(sol["xi"] <= varrho)
    assert abs(sol["beta"]) <= K + varrho
    assert np.all(sol["r"] <= 2 * (K + varrho))
    assert np.all(sol["alpha"] >= q / (2 * K + 2 * varrho) ** (q + 1) * (1 - 1e-6))


def _scipy_reduced_solve(X, y, C, q):
    n, d = X.shape
    ts = (q / C) ** (1 / (q + 1))

    def f(v):
        w, b = v[:d], v[d]
        m = y * (X @ w + b)
        hi = m >= ts
        val = np.where(hi, np.abs(m) ** -q, ts ** -q + C * (ts - m))
        dv = np.where(hi, -q * np.abs(m) ** (-q - 1), -C) * y
        return val.sum(), np.concatenate([X.T @ dv, [dv.sum()]])

    v0 = np.zeros(d + 1)
    v0[d] = 0.0
    cons = [{"type": "ineq", "fun": lambda v: 1.0 - v[:d] @ v[:d],
             "jac": lambda v: np.concatenate([-2 * v[:d], [0.0]])}]
    res = sopt.minimize(f, v0, jac=True, method="SLSQP", constraints=cons,
                        options={"ftol": 1e-15, "maxiter": 2000})
    return res.x[:d], res.x[d], res.fun


def test_whole_solve_matches_library_convex_solver(tight_small):
    X, y, C, q, sol = tight_small
    w_ref, b_ref, f_ref = _scipy_reduced_solve(X, y, C, q)
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    f = O.reduced_objective(X, y, w, sol["beta"], C, q)
    assert abs(f - f_ref) <= 1e-7 * abs(f_ref)
    assert np.linalg.norm(w - w_ref) <= 1e-4 * np.linalg.norm(w_ref)
    assert abs(sol["beta"] - b_ref) <= 1e-4 * max(1.0, abs(b_ref))


@pytest.mark.parametrize("q,C", [(2.0, 3.0), (0.5, 0.2), (4.0, 10.0)])
def test_general_q_matches_library_convex_solver(q, C):
    X, y = synth.random_two_class(d=30, n=40, seed=9, mean=0.6)
    sol = O.solve(X, y, C, q, tol=1e-9, max_iter=20000)
    assert sol["converged"]
    w_ref, b_ref, f_ref = _scipy_reduced_solve(X, y, C, q)
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    f = O.reduced_objective(X, y, w, sol["beta"], C, q)
    assert abs(f - f_ref) <= 1e-7 * abs(f_ref)
    assert np.linalg.norm(w - w_ref) <= 1e-4 * np.linalg.norm(w_ref)


def test_two_dimensional_brute_force():
    X, y = synth.tiny_2d()
    C, q = 1.0, 1.0
    sol = O.solve(X, y, C, q, tol=1e-8, max_iter=50000)
    assert sol["converged"]
    n = X.shape[0]
    varrho = (n + C * n) / C
    K = np.max(np.linalg.norm(X, axis=1))
    phis = np.linspace(0, 2 * np.pi, 721)
    betas = np.linspace(-(K + varrho), K + varrho, 801)
    W = np.stack([np.cos(phis), np.sin(phis)], 1)
    best = (np.inf, 0, 0)
    for j, w in enumerate(W):
        m = y[None, :] * ((X @ w)[None, :] + betas[:, None])
        v = O.reduced_loss(m.ravel(), C, q).reshape(m.shape).sum(1)
        i = int(np.argmin(v))
        if v[i] < best[0]:
            best = (v[i], phis[j], betas[i])
    # refine the best grid cell with a bounded two-dimensional search
    f2 = lambda p: O.reduced_objective(X, y, np.array([math.cos(p[0]), math.sin(p[0])]), p[1], C, q)
    dphi, dbeta = phis[1] - phis[0], betas[1] - betas[0]
    res = sopt.minimize(f2, [best[1], best[2]], method="Nelder-Mead",
                        options={"xatol": 1e-12, "fatol": 1e-14, "maxiter": 20000})
    assert abs(res.x[0] - best[1]) <= 2 * dphi and abs(res.x[1] - best[2]) <= 2 * dbeta
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    f = O.reduced_objective(X, y, w, sol["beta"], C, q)
    assert abs(np.linalg.norm(sol["w"]) - 1) <= 1e-6
    assert abs(f - res.fun) <= 1e-6 * abs(res.fun)
    ang = math.atan2(w[1], w[0]) % (2 * np.pi)
    dang = abs((ang - res.x[0] + np.pi) % (2 * np.pi) - np.pi)
    assert dang <= 1e-4


# --------------------------------------------------------------------------
# Invariances of the problem.
# --------------------------------------------------------------------------

def test_label_flip_invariance(tight_small):
    X, y, C, q, sol = tight_small
    s2 = O.solve(X, -y, C, q, tol=1e-9, max_iter=20000)
    assert np.linalg.norm(s2["w"] + sol["w"]) <= 1e-5 * np.linalg.norm(sol["w"])
    assert abs(s2["beta"] + sol["beta"]) <= 1e-5


def test_sample_permutation_invariance(tight_small):
    X, y, C, q, sol = tight_small
    p = np.random.default_rng(10).permutation(X.shape[0])
    s2 = O.solve(X[p], y[p], C, q, tol=1e-9, max_iter=20000)
    assert np.linalg.norm(s2["w"] - sol["w"]) <= 1e-5 * np.linalg.norm(sol["w"])
    assert abs(s2["beta"] - sol["beta"]) <= 1e-5
    assert np.allclose(s2["alpha"], sol["alpha"][p], rtol=1e-4, atol=1e-7)


def test_rotation_invariance(tight_small):
    X, y, C, q, sol = tight_small
    Q, _ = np.linalg.qr(np.random.default_rng(11).standard_normal((X.shape[1], X.shape[1])))
    s2 = O.solve(X @ Q.T, y, C, q, tol=1e-9, max_iter=20000)  # x_i -> Q x_i
    assert np.linalg.norm(s2["w"] - Q @ sol["w"]) <= 1e-5 * np.linalg.norm(sol["w"])
    assert abs(s2["beta"] - sol["beta"]) <= 1e-5


# --------------------------------------------------------------------------
# Planted mistakes: each one, put into a copy of the oracle's arithmetic,
# must be caught by one of the pins above.
# --------------------------------------------------------------------------

def _solution_error(monkeypatch, target, replacement):
    X, y, C, q = small_problem()
    monkeypatch.setattr(O, target, replacement)
    try:
        with np.errstate(all="ignore"):
            sol = O.solve(X, y, C, q, tol=1e-9, max_iter=3000)
    except (OverflowError, FloatingPointError, ValueError, np.linalg.LinAlgError):
        return False, math.inf  # the planted mistake made the iteration diverge
    w_ref, b_ref, f_ref = _scipy_reduced_solve(X, y, C, q)
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    f = O.reduced_objective(X, y, w, sol["beta"], C, q)
    return sol["converged"], abs(f - f_ref) / abs(f_ref)


def test_planted_sign_error_in_rhs_is_caught(monkeypatch):
    orig = O.linsys_rhs

    def bad(Zt, y, mu, sigma, r, xi, u, alpha, rho):
        hw, hb = orig(Zt, y, mu, sigma, r, xi, u, alpha, -rho)  # wrong sign of rho
        return hw, hb

    conv, err = _solution_error(monkeypatch, "linsys_rhs", bad)
    assert (not conv) or err > 1e-7


def test_planted_wrong_kappa_is_caught(tight_small):
    X, y, C, q, sol = tight_small
    # a kappa off by 1% would leave a visible duality gap at the true optimum
    P = _primal_value(X, y, sol["w"] / max(1.0, np.linalg.norm(sol["w"])), sol["beta"], C, q)
    a = _dual_feasible_projection(sol["alpha"], y, C)
    k_bad = 1.01 * O.kappa(q)
    D_bad = k_bad * np.sum(a ** (q / (q + 1))) - np.linalg.norm(X.T @ (y * a))
    assert (P - D_bad) / (1 + abs(P)) > 1e-4 or D_bad > P
