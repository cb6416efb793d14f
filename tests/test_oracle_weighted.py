"""Pins of the oracle's weighted problem: the class weights of Section 4.5,
a general penalty vector e in eq-primal, and the choice of C of Section 4.1.

As in the other oracle pins, every check compares the oracle with something
other than itself: hand-computed values, a library minimiser, a duplicated
sample, an exact rescaling of the problem.  None of these needs a GPU.
"""
import math

import numpy as np
import pytest
import scipy.optimize as sopt

import synth
from oracle import dwd_oracle as O


# --------------------------------------------------------------------------
# Section 4.5 class weights and the Section 4.1 choice of C by hand.
# --------------------------------------------------------------------------

def test_class_weights_hand_values():
    # 3 positives, 7 negatives: tau_+ < tau_-, so the minority class keeps
    # weight 1 and the majority class gets (3/7)^(1/(1+q)), raised to q.
    y = np.array([1, -1, -1, 1, -1, -1, -1, 1, -1, -1], float)
    w1 = O.class_weights(y, 1.0)
    assert np.allclose(w1[y > 0], 1.0, rtol=0, atol=1e-15)
    assert np.allclose(w1[y < 0], 0.6546536707079771, rtol=1e-14)   # sqrt(3/7)
    w2 = O.class_weights(y, 2.0)
    assert np.allclose(w2[y < 0], 0.5684367439851988, rtol=1e-14)   # (3/7)^(2/3)
    wh = O.class_weights(y, 0.5)
    assert np.allclose(wh[y < 0], 0.7539474411291538, rtol=1e-14)   # (3/7)^(1/3)
    # labels swapped: the weights follow class size, not the sign
    assert np.array_equal(O.class_weights(-y, 1.0), w1)


def test_class_weights_balanced_are_one():
    y = np.array([1, -1] * 9, float)
    for q in (0.5, 1.0, 2.0, 4.0):
        assert np.array_equal(O.class_weights(y, q), np.ones(18))


def test_suggest_C_hand_example():
    # one feature; positives at 0 and 1, negatives at 3 and 5: the four
    # between-class distances are 3, 5, 2, 4, median 3.5; n = 4, d = 1.
    X = np.array([[0.0], [1.0], [3.0], [5.0]])
    y = np.array([1.0, 1.0, -1.0, -1.0])
    # q = 1: 100 * max(1, log(4) * 10 / 3.5^2) = 113.16...
    assert O.suggest_C(X, y, 1.0) == pytest.approx(113.1668866220319, rel=1e-13)
    # q = 2: 1000 * max(1, 10 * log(4) * 10 / 3.5^3)
    assert O.suggest_C(X, y, 2.0) == pytest.approx(3233.33961777234, rel=1e-13)
    # widely separated classes: the max picks 10^(q+1)
    assert O.suggest_C(X * 100.0, y, 1.0) == pytest.approx(100.0, rel=1e-15)


def test_suggest_C_median_by_pairwise_loops():
    X, y = synth.random_two_class(d=7, n=13, seed=21, pos_frac=0.3)
    dists = [math.dist(X[i], X[j]) for i in range(13) for j in range(13)
             if y[i] > 0 and y[j] < 0]
    dists.sort()
    k = len(dists)
    med = dists[k // 2] if k % 2 else 0.5 * (dists[k // 2 - 1] + dists[k // 2])
    q = 1.0
    want = 10 ** (q + 1) * max(1.0, 10 ** (q - 1) * math.log(13) * 1000 ** (1 / 3) / med ** (q + 1))
    assert O.suggest_C(X, y, q) == pytest.approx(want, rel=1e-12)


# --------------------------------------------------------------------------
# The weighted prox and the weighted dual term.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("q", [0.5, 1.0, 2.0, 4.0])
def test_weighted_prox_is_the_minimiser(q):
    rng = np.random.default_rng(31)
    a = rng.uniform(-3, 3, 12)
    wt = rng.uniform(0.05, 1.0, 12)
    sigma = 0.7
    s, _ = O.prox_weighted(a, sigma, q, wt, np.ones(12), 1e-13)
    for i in range(12):
        f = lambda t: wt[i] * t ** -q + 0.5 * sigma * (t - a[i]) ** 2
        res = sopt.minimize_scalar(f, bounds=(1e-6, 50.0), method="bounded",
                                   options={"xatol": 1e-12})
        assert s[i] == pytest.approx(res.x, rel=1e-6)
        # first-order condition of the weighted objective
        assert abs(-q * wt[i] * s[i] ** (-q - 1) + sigma * (s[i] - a[i])) <= 1e-10


def test_weighted_prox_q1_is_a_root_of_the_cubic():
    # q = 1: sigma s^2 (s - a) = wt, a cubic in s with one positive root
    a = np.array([-2.0, -0.3, 0.0, 0.4, 2.5])
    wt = np.array([0.2, 1.0, 0.5, 0.05, 0.9])
    sigma = 3.0
    s, _ = O.prox_weighted(a, sigma, 1.0, wt, np.ones(5), 1e-14)
    for i in range(5):
        roots = np.roots([sigma, -sigma * a[i], 0.0, -wt[i]])
        pos = [r.real for r in roots if abs(r.imag) < 1e-9 and r.real > 0]
        assert len(pos) == 1
        assert s[i] == pytest.approx(pos[0], rel=1e-12)


@pytest.mark.parametrize("q", [0.5, 1.0, 2.0])
def test_weighted_dual_term_is_the_inner_infimum(q):
    # inf_{r > 0} wt r^-q + a r = kappa(q) wt^(1/(q+1)) a^(q/(q+1)); kkt_residuals
    # must report that value as the dual objective of a weighted problem.
    for wt, a in [(0.3, 0.8), (1.0, 2.0), (0.05, 0.1)]:
        res = sopt.minimize_scalar(lambda r: wt * r ** -q + a * r, bounds=(1e-6, 1e3),
                                   method="bounded", options={"xatol": 1e-12})
        got = O.kappa(q) * wt ** (1 / (q + 1)) * a ** (q / (q + 1))
        assert got == pytest.approx(res.fun, rel=1e-9)
    # the same value through kkt_residuals (Z alpha = 0: one sample per class,
    # identical x, alpha equal)
    Zt = np.zeros((2, 2))
    e = O.kkt_residuals(Zt, 1.0, np.array([1.0, -1.0]), 5.0, q, 1.0, np.ones(2),
                        np.zeros(2), 0.0, np.zeros(2), np.zeros(2), np.array([0.8, 0.8]),
                        wt=np.array([0.3, 0.3]))
    assert e["dualobj"] == pytest.approx(2 * O.kappa(q) * 0.3 ** (1 / (q + 1))
                                         * 0.8 ** (q / (q + 1)), rel=1e-14)


# --------------------------------------------------------------------------
# Whole weighted solves.
# --------------------------------------------------------------------------

def _scipy_weighted_reduced_solve(X, y, C, q, wt, e):
    """min over ||w|| <= 1, beta of sum_i [wt_i theta_q(r_i) + C e_i xi_i] with
    the best xi for (w, beta), by SLSQP (independent of the ADMM)."""
    n, d = X.shape
    ce = C * e
    ts = (q * wt / ce) ** (1 / (q + 1))

    def f(v):
        w, b = v[:d], v[d]
        m = y * (X @ w + b)
        hi = m >= ts
        mm = np.where(hi, m, 1.0)
        val = np.where(hi, wt * mm ** -q, wt * ts ** -q + ce * (ts - m))
        dv = np.where(hi, -q * wt * mm ** (-q - 1), -ce) * y
        return val.sum(), np.concatenate([X.T @ dv, [dv.sum()]])

    cons = [{"type": "ineq", "fun": lambda v: 1.0 - v[:d] @ v[:d],
             "jac": lambda v: np.concatenate([-2 * v[:d], [0.0]])}]
    res = sopt.minimize(f, np.zeros(d + 1), jac=True, method="SLSQP", constraints=cons,
                        options={"ftol": 1e-15, "maxiter": 3000})
    return res.x[:d], res.x[d], res.fun


@pytest.fixture(scope="module")
def unbalanced_small():
    X, y = synth.random_two_class(d=40, n=30, seed=17, mean=0.7, flip=0.1, pos_frac=0.2)
    e = synth.penalty_vector(30, seed=18)
    return X, y, e


@pytest.mark.parametrize("q,C,use_e", [(1.0, 2.0, False), (1.0, 2.0, True), (2.0, 5.0, True),
                                       (0.5, 0.5, True)])
def test_weighted_solve_matches_library_convex_solver(unbalanced_small, q, C, use_e):
    X, y, e = unbalanced_small
    ev = e if use_e else None
    sol = O.solve(X, y, C, q, tol=1e-9, max_iter=40000, weights=True, e=ev)
    assert sol["converged"]
    wt = O.class_weights(y, q)
    assert len(np.unique(wt)) == 2
    w_ref, b_ref, f_ref = _scipy_weighted_reduced_solve(X, y, C, q, wt,
                                                        e if use_e else np.ones(30))
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    f = O.reduced_objective(X, y, w, sol["beta"], C, q, wt, ev)
    assert abs(f - f_ref) <= 1e-7 * abs(f_ref)
    assert np.linalg.norm(w - w_ref) <= 1e-4 * np.linalg.norm(w_ref)
    assert abs(sol["beta"] - b_ref) <= 1e-4 * max(1.0, abs(b_ref))
    # the weighted dual objective meets the weighted primal at the optimum
    assert sol["eta"]["gap"] <= 1e-6
    # alpha = q wt / r^(q+1) and 0 <= alpha <= C e
    # (eta_C3 is a squared norm: at tol 1e-9 the entries agree to ~1e-5)
    assert np.allclose(sol["alpha"], q * wt / sol["r"] ** (q + 1), rtol=1e-3, atol=5e-5)
    ce = C * (e if use_e else 1.0)
    assert np.all(sol["alpha"] <= ce + 1e-8)


def test_weighted_differs_from_unweighted(unbalanced_small):
    X, y, _ = unbalanced_small
    a = O.solve(X, y, 2.0, 1.0, tol=1e-8, max_iter=20000)
    b = O.solve(X, y, 2.0, 1.0, tol=1e-8, max_iter=20000, weights=True)
    assert np.linalg.norm(a["w"] - b["w"]) > 1e-3 * np.linalg.norm(a["w"])


def test_duplicated_sample_equals_doubled_weights():
    # sample 0 counted twice (wt = 2 and e = 2 on one copy) is the problem
    # with the sample duplicated (weights 1): the optimal (w, beta) agree.
    X, y = synth.random_two_class(d=25, n=16, seed=23, mean=0.8)
    X2 = np.vstack([X, X[:1]])
    y2 = np.concatenate([y, y[:1]])
    C, q = 3.0, 1.0
    wt = np.ones(16)
    wt[0] = 2.0
    a = O.solve(X, y, C, q, tol=1e-12, max_iter=40000, weights=wt, e=wt)
    b = O.solve(X2, y2, C, q, tol=1e-12, max_iter=40000)
    c = O.solve(X, y, C, q, tol=1e-12, max_iter=40000)
    assert a["converged"] and b["converged"]
    wa = a["w"] / max(1.0, np.linalg.norm(a["w"]))
    wb = b["w"] / max(1.0, np.linalg.norm(b["w"]))
    # (the unweighted single copy is ~5% away in w and 0.016 in beta)
    assert np.linalg.norm(c["w"] - b["w"]) > 1e-2 * np.linalg.norm(wb)
    assert np.linalg.norm(wa - wb) <= 1e-4 * np.linalg.norm(wb)
    assert a["beta"] == pytest.approx(b["beta"], abs=1e-5)


def test_uniform_loss_weight_is_a_rescaling():
    # wt = lam everywhere with C -> lam C multiplies the objective by lam: the
    # same (w, beta, r, xi), alpha scaled by lam.
    X, y = synth.random_two_class(d=30, n=20, seed=29, mean=0.6)
    C, q, lam = 1.5, 2.0, 0.25
    a = O.solve(X, y, C, q, tol=1e-10, max_iter=40000)
    b = O.solve(X, y, lam * C, q, tol=1e-10, max_iter=40000, weights=np.full(20, lam))
    assert a["converged"] and b["converged"]
    assert np.linalg.norm(a["w"] - b["w"]) <= 1e-5 * np.linalg.norm(a["w"])
    assert np.allclose(a["r"], b["r"], rtol=1e-5)
    assert np.allclose(lam * a["alpha"], b["alpha"], rtol=1e-4, atol=1e-8)


def test_penalty_vector_trades_with_C():
    # (C, e) and (C / lam, lam e) are the same problem (only C e appears)
    X, y = synth.random_two_class(d=30, n=20, seed=37, mean=0.6)
    e = synth.penalty_vector(20, seed=38)
    a = O.solve(X, y, 4.0, 1.0, tol=1e-10, max_iter=40000, e=e)
    b = O.solve(X, y, 2.0, 1.0, tol=1e-10, max_iter=40000, e=2.0 * e)
    assert a["converged"] and b["converged"]
    assert np.linalg.norm(a["w"] - b["w"]) <= 1e-5 * np.linalg.norm(a["w"])
    assert a["beta"] == pytest.approx(b["beta"], rel=1e-5, abs=1e-6)


def test_planted_weight_in_the_wrong_place_is_caught(monkeypatch, unbalanced_small):
    # a prox that multiplies sigma by the weight (instead of dividing) must
    # fail the library comparison
    X, y, _ = unbalanced_small
    real = O.prox_newton

    def wrong(a, sigma, q, s_init, tol, max_steps=O.MAX_NEWTON):
        return real(a, sigma, q, s_init, tol, max_steps)

    monkeypatch.setattr(O, "prox_weighted",
                        lambda a, sigma, q, wt, s_init, tol: wrong(a, sigma * np.asarray(wt), q,
                                                                   s_init, tol))
    sol = O.solve(X, y, 2.0, 1.0, tol=1e-9, max_iter=3000, weights=True)
    wt = O.class_weights(y, 1.0)
    w_ref, b_ref, f_ref = _scipy_weighted_reduced_solve(X, y, 2.0, 1.0, wt, np.ones(30))
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    f = O.reduced_objective(X, y, w, sol["beta"], 2.0, 1.0, wt)
    assert not (abs(f - f_ref) <= 1e-7 * abs(f_ref)
                and np.linalg.norm(w - w_ref) <= 1e-4 * np.linalg.norm(w_ref))
