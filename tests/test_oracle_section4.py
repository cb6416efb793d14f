"""Pins of the oracle's Section 4.3 residuals, stopping rule and Section 4.4
sigma rule against values worked out by hand.

Each residual below is evaluated on a tiny hand-built state whose numbers
were chosen so that every term has a short exact value; the expected values
are written out as literals (or as the short closed forms they reduce to),
never through the oracle's own functions.  A mistake in any single term (a
dropped square, a wrong exponent, a missing factor, the gap scaled, a
threshold swapped) changes at least one of them.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dwd_oracle as O


# ---------------------------------------------------------------------------
# Section 4.3 on hand-built states.
# ---------------------------------------------------------------------------

def _state_a(mu=1.0):
    """d = 2, n = 3, q = 1, C = 1 (so every residual is divided by 2),
    Z_scale = 2.

        Z~ = [[1, 0, 2], [0, 1, 1]],  y = (1, -1, 1),  w~ = (3, 4),
        u~ = (0, 4),  beta = 1,  xi = (0, 1, 0),  r = (1, 2, 4),
        alpha = (-1, 1/2, 2),  rho = (1, -1/2).
    """
    Zt = np.array([[1.0, 0.0, 2.0], [0.0, 1.0, 1.0]])
    return dict(Zt=Zt, zscale=2.0, y=np.array([1.0, -1.0, 1.0]), C=1.0, q=1.0, mu=mu,
                r=np.array([1.0, 2.0, 4.0]), w=np.array([3.0, 4.0]), beta=1.0,
                xi=np.array([0.0, 1.0, 0.0]), u=np.array([0.0, 4.0]),
                alpha=np.array([-1.0, 0.5, 2.0]), rho=np.array([1.0, -0.5]))


# Worked by hand for state A (mu = 1):
#   Z~^T w~ = (3, 4, 10); Z~^T w~ + beta y + xi - r = (3, 2, 7)     -> P1 = sqrt(62)/2
#   w~ - u~ = (3, 0)                                                 -> P2 = 3/2
#   ||w~|| = 5 > Z_scale = 2                                         -> P3 = 3/2
#   min(0, alpha) = (-1, 0, 0)                                       -> D1 = 1/2
#   max(0, alpha - C) = (0, 0, 1)                                    -> D2 = 1/2
#   Z~ alpha = (3, 5/2); Z~ alpha + rho = (4, 2)                     -> D3 = sqrt(20)/2
#   y^T alpha = -1 - 1/2 + 2 = 1/2                                   -> C1 = 1/4
#   xi^T (C - alpha) = 1 * (1 - 1/2) = 1/2                           -> C2 = 1/4
#   s = q / r^2 = (1, 1/4, 1/16); alpha - s = (-2, 1/4, 31/16);
#   ||alpha - s||^2 = 4 + 1/16 + 961/256 = 2001/256                  -> C3 = 2001/512
#   primal = 1 + 1/2 + 1/4 + C * 1 = 11/4
#   dual = kappa(1) (0 + sqrt(1/2) + sqrt(2)) - 2 sqrt(61/4)
#        = 2 * 3/sqrt(2) - sqrt(61) = 3 sqrt(2) - sqrt(61)
STATE_A = {
    "P1": math.sqrt(62.0) / 2, "P2": 1.5, "P3": 1.5, "D1": 0.5, "D2": 0.5,
    "D3": math.sqrt(20.0) / 2, "C1": 0.25, "C2": 0.25, "C3": 2001.0 / 512.0,
    "primobj": 2.75, "dualobj": 3.0 * math.sqrt(2.0) - math.sqrt(61.0),
}
STATE_A["gap"] = (abs(STATE_A["primobj"] - STATE_A["dualobj"])
                  / (1.0 + abs(STATE_A["primobj"]) + abs(STATE_A["dualobj"])))


def _state_b():
    """d = 1, n = 3, q = 2, C = 3 (divisor 4), Z_scale = 1, ||w~|| inside
    the ball.

        Z~ = [[1, 1, 1]],  y = (1, -1, -1),  w~ = u~ = (1/2),  beta = 0,
        xi = (1/2, 0, 0),  r = (1, 2, 1),  alpha = (8, 1, 0).
    """
    return dict(Zt=np.array([[1.0, 1.0, 1.0]]), zscale=1.0, y=np.array([1.0, -1.0, -1.0]),
                C=3.0, q=2.0, mu=1.0, r=np.array([1.0, 2.0, 1.0]), w=np.array([0.5]),
                beta=0.0, xi=np.array([0.5, 0.0, 0.0]), u=np.array([0.5]),
                alpha=np.array([8.0, 1.0, 0.0]), rho=None)


# Worked by hand for state B:
#   Z~^T w~ + xi - r = (0, -3/2, -1/2)                -> P1 = sqrt(5/2)/4
#   w~ = u~, ||w~|| = 1/2 < 1                          -> P2 = P3 = 0
#   alpha >= 0; max(0, alpha - 3) = (5, 0, 0)          -> D1 = 0, D2 = 5/4
#   y^T alpha = 8 - 1 = 7                              -> C1 = 7/4
#   xi^T (C - alpha) = 1/2 (3 - 8) = -5/2              -> C2 = 5/8
#   s = 2 / r^3 = (2, 1/4, 2); alpha - s = (6, 3/4, -2);
#   ||.||^2 = 36 + 9/16 + 4 = 649/16                   -> C3 = 649/64
#   primal = 1 + 1/4 + 1 + 3 * 1/2 = 15/4
#   kappa(2) = 3/2 * 2^(1/3); sum alpha^(2/3) = 4 + 1 + 0 = 5; Z~ alpha = 9
#   dual = 15/2 * 2^(1/3) - 9
STATE_B = {
    "P1": math.sqrt(2.5) / 4, "P2": 0.0, "P3": 0.0, "D1": 0.0, "D2": 1.25,
    "C1": 1.75, "C2": 0.625, "C3": 649.0 / 64.0,
    "primobj": 3.75, "dualobj": 7.5 * 2.0 ** (1.0 / 3.0) - 9.0,
}
STATE_B["gap"] = (abs(STATE_B["primobj"] - STATE_B["dualobj"])
                  / (1.0 + abs(STATE_B["primobj"]) + abs(STATE_B["dualobj"])))


def _eval(fn, s, **kw):
    return fn(s["Zt"], s["zscale"], s["y"], s["C"], s["q"], s["mu"], s["r"], s["w"], s["beta"],
              s["xi"], s["u"], s["alpha"], rho=s["rho"], **kw)


def _mismatches(got, expected, rtol=1e-14):
    return [k for k, v in expected.items()
            if not abs(got[k] - v) <= rtol * max(1.0, abs(v))]


def test_each_residual_of_state_a_matches_the_hand_value():
    got = _eval(O.kkt_residuals, _state_a())
    assert _mismatches(got, STATE_A) == []


def test_each_residual_of_state_b_matches_the_hand_value():
    got = _eval(O.kkt_residuals, _state_b())
    assert _mismatches(got, STATE_B) == []
    assert "D3" not in got          # no rho given: no multiplier residual


def test_maxima_of_the_groups():
    got = _eval(O.kkt_residuals, _state_a())
    assert got["P"] == pytest.approx(math.sqrt(62.0) / 2, rel=1e-15)
    assert got["C"] == pytest.approx(2001.0 / 512.0, rel=1e-15)
    # eta_D with the multiplier residual (reading R1), and the printed
    # two-term eta_D (rho_residual = False)
    assert got["D"] == pytest.approx(math.sqrt(20.0) / 2, rel=1e-15)
    lit = _eval(O.kkt_residuals, _state_a(), rho_residual=False)
    assert lit["D"] == 0.5
    got_b = _eval(O.kkt_residuals, _state_b())
    assert got_b["P"] == pytest.approx(math.sqrt(2.5) / 4, rel=1e-15)
    assert got_b["D"] == 1.25 and got_b["C"] == pytest.approx(649.0 / 64.0, rel=1e-15)


def test_mu_enters_as_sqrt_mu():
    # D = sqrt(mu) I: with mu = 4, P2 = 2 * 3 / 2 = 3 and
    # Z~ alpha + 2 rho = (5, 3/2), D3 = sqrt(25 + 9/4)/2 = sqrt(109)/4.
    got = _eval(O.kkt_residuals, _state_a(mu=4.0))
    assert got["P2"] == 3.0
    assert got["D3"] == pytest.approx(math.sqrt(109.0) / 4, rel=1e-15)
    assert got["P1"] == pytest.approx(math.sqrt(62.0) / 2, rel=1e-15)


def test_weighted_residuals_match_the_hand_values():
    # State A with C = 2 (divisor 3), loss weights v = (1/2, 1, 2) and
    # penalty vector e = (1, 1/2, 1/4), so C e = (2, 1, 1/2):
    #   max(0, alpha - C e) = (0, 0, 3/2)                 -> D2 = 1/2
    #   xi^T (C e - alpha) = 1 (1 - 1/2)                   -> C2 = 1/6
    #   s = q v / r^2 = (1/2, 1/4, 1/8); alpha - s = (-3/2, 1/4, 15/8);
    #   ||.||^2 = 9/4 + 1/16 + 225/64 = 373/64             -> C3 = 373/192
    #   primal = 1/2 + 1/4 * 1 ... = sum v / r + sum C e xi
    #          = 1/2 + 1/2 + 1/2 + 1 = 5/2
    #   dual = kappa(1) sum v^(1/2) alpha_+^(1/2) - Z_scale ||Z~ alpha||
    #        = 2 (sqrt(1/2) + sqrt(2) sqrt(2)) - sqrt(61) = sqrt(2) + 4 - sqrt(61)
    s = _state_a()
    s["C"] = 2.0
    got = _eval(O.kkt_residuals, s, wt=np.array([0.5, 1.0, 2.0]), e=np.array([1.0, 0.5, 0.25]))
    exp = {"D1": 1.0 / 3.0, "D2": 0.5, "C1": 0.5 / 3.0, "C2": 0.5 / 3.0,
           "C3": 373.0 / 192.0, "P1": math.sqrt(62.0) / 3, "primobj": 2.5,
           "dualobj": math.sqrt(2.0) + 4.0 - math.sqrt(61.0)}
    assert _mismatches(got, exp) == []


# Planted mistakes in a copy of the residual code: each must change a hand
# value above.

def _planted(kind):
    def fn(*a, **kw):
        e = O.kkt_residuals(*a, **kw)
        e = dict(e)
        if kind == "c3_unsquared":
            e["C3"] = math.sqrt(e["C3"] * (1.0 + a[3])) / (1.0 + a[3])
        elif kind == "gap_scaled":
            e["gap"] *= 0.01
        elif kind == "no_denominator_p1":
            e["P1"] *= 1.0 + a[3]
        elif kind == "dual_exponent":
            q = a[4]
            alpha = a[11]
            e["dualobj"] = (O.kappa(q) * float(np.sum(np.maximum(alpha, 0.0) ** (1.0 / (q + 1.0))))
                            - a[1] * float(np.linalg.norm(a[0] @ alpha)))
            pr, du = e["primobj"], e["dualobj"]
            e["gap"] = abs(pr - du) / (1.0 + abs(pr) + abs(du))
        elif kind == "xi_sign_in_c2":
            C, alpha, xi = a[3], a[11], a[9]
            e["C2"] = abs(float(xi @ (C + alpha))) / (1.0 + C)
        return e
    return fn


@pytest.mark.parametrize("kind", ["c3_unsquared", "gap_scaled", "no_denominator_p1",
                                  "dual_exponent", "xi_sign_in_c2"])
def test_planted_residual_mistakes_are_caught(kind):
    bad = _planted(kind)
    a = _mismatches(_eval(bad, _state_a()), STATE_A)
    b = _mismatches(_eval(bad, _state_b()), STATE_B)
    assert a or b, kind


# ---------------------------------------------------------------------------
# Section 4.3 stopping rule: a truth table.
# ---------------------------------------------------------------------------

TOL = 1e-4   # sqrt(TOL) = 1e-2

STOP_CASES = [
    # (eta_P, eta_D, eta_C, eta_gap, stop?)          what fails
    (5e-5, 5e-5, 1e-3, 4e-2, True),                  # nothing
    (2e-4, 5e-5, 1e-3, 4e-2, False),                 # eta_P >= tol
    (5e-5, 2e-4, 1e-3, 4e-2, False),                 # eta_D >= tol
    (1e-4, 5e-5, 1e-3, 4e-2, False),                 # eta_P == tol (strict)
    (5e-5, 5e-5, 2e-2, 3e-2, False),                 # min(eta_C, gap) >= sqrt(tol)
    (5e-5, 5e-5, 1e-2, 1e-2, False),                 # min == sqrt(tol) (strict)
    (5e-5, 5e-5, 1e-3, 6e-2, False),                 # max(eta_C, gap) >= 0.05 via gap
    (5e-5, 5e-5, 6e-2, 1e-3, False),                 # ... via eta_C
    (5e-5, 5e-5, 1e-3, 5e-2, False),                 # max == 0.05 (strict)
    (5e-5, 5e-5, 4e-2, 5e-3, True),                  # eta_C large but < 0.05, gap small
    (5e-5, 5e-5, 5e-3, 4.9e-2, True),                # gap large but < 0.05, eta_C small
    (0.0, 0.0, 0.0, 0.0, True),
]


@pytest.mark.parametrize("P,D,Cc,gap,expected", STOP_CASES)
def test_stop_rule_truth_table(P, D, Cc, gap, expected):
    assert O.stop_test(dict(P=P, D=D, C=Cc, gap=gap), TOL) is expected


# ---------------------------------------------------------------------------
# Section 4.4: sigma rule and sigma_0.
# ---------------------------------------------------------------------------

SIGMA_CASES = [
    # (eta_P, eta_D, new sigma for sigma = 10)
    (1.0, 1.0, 10.0),              # chi = 1: unchanged
    (4.9, 1.0, 10.0),              # chi below theta = 5
    (5.0, 1.0, 10.0),              # chi == theta (strict)
    (6.0, 1.0, 11.0),              # chi > 5: sigma * 1.1
    (50.0, 1.0, 11.0),             # max(chi, 1/chi) == 50: still 1.1
    (51.0, 1.0, 16.5),             # > 50: 1.65
    (500.0, 1.0, 16.5),            # == 500: 1.65
    (501.0, 1.0, 22.0),            # > 500: 2.2
    (1.0, 4.9, 10.0),              # 1/chi below theta
    (1.0, 5.0, 10.0),              # 1/chi == theta
    (1.0, 6.0, 10.0 / 1.1),        # 1/chi > 5: sigma / 1.1
    (1.0, 60.0, 10.0 / 1.65),
    (1.0, 600.0, 10.0 / 2.2),
    (0.0, 1.0, 10.0),              # eta_P = 0: no update
    (1.0, 0.0, 10.0),              # eta_D = 0: no update
]


@pytest.mark.parametrize("P,D,expected", SIGMA_CASES)
def test_sigma_rule_table(P, D, expected):
    assert O.sigma_update(10.0, P, D) == pytest.approx(expected, rel=1e-15)


@pytest.mark.parametrize("C,q,n,expected", [
    (1.0, 1.0, 50, 10.0),          # min(10, 50)^1
    (10.0, 1.0, 1000, 100.0),      # min(100, 1000)
    (100.0, 2.0, 50, 2500.0),      # min(1000, 50)^2
    (1.0, 2.0, 2000, 100.0),       # min(10, 2000)^2
    (0.01, 0.5, 50, math.sqrt(0.1)),
    (10.0, 4.0, 7, 2401.0),        # min(100, 7)^4
])
def test_sigma0_table(C, q, n, expected):
    assert O.default_sigma0(C, q, n) == pytest.approx(expected, rel=1e-15)


# ---------------------------------------------------------------------------
# The loop applies the two rules as stated: first sigma, the cadence, the
# printed two-term eta_D, the stopping point.
# ---------------------------------------------------------------------------

def _small():
    wl = synth.SMALL_F64
    X, y = synth.two_class(wl.data)
    return X, y, wl.C, wl.q


@pytest.mark.parametrize("every", [1, 2, 3])
def test_sigma_history_follows_the_rule_and_cadence(every):
    X, y, C, q = _small()
    sol = O.solve(X, y, C, q, tol=1e-300, max_iter=60, record=True, sigma_every=every)
    h = sol["history"]
    assert h[0]["sigma"] == min(10.0 * C, len(y)) ** q
    for k in range(len(h) - 1):
        want = h[k]["sigma"]
        if (k + 1) % every == 0:
            # the table-pinned rule on the recorded residuals
            want = O.sigma_update(want, h[k]["P"], h[k]["D"])
        assert h[k + 1]["sigma"] == want, k
    # the rule does move sigma on this problem
    assert len({x["sigma"] for x in h}) > 3


def test_literal_eta_d_has_only_the_box_terms():
    X, y, C, q = _small()
    sol = O.solve(X, y, C, q, tol=1e-300, max_iter=15, rho_residual=False)
    a = sol["alpha"]
    # eta_D = max(||min(0, alpha)||, ||max(0, alpha - C)||) / (1 + C)
    d1 = math.sqrt(sum(min(0.0, v) ** 2 for v in a)) / (1 + C)
    d2 = math.sqrt(sum(max(0.0, v - C) ** 2 for v in a)) / (1 + C)
    assert sol["eta"]["D"] == max(d1, d2)


def _reduced_optimum(X, y, C, q):
    from scipy.optimize import minimize
    n, d = X.shape

    def f(z):
        w, b = z[:d], z[d]
        return O.reduced_objective(X, y, w, b, C, q)

    cons = [{"type": "ineq", "fun": lambda z: 1.0 - z[:d] @ z[:d]}]
    best = None
    for seed in range(2):
        z0 = np.random.default_rng(seed).standard_normal(d + 1) * 0.01
        res = minimize(f, z0, method="SLSQP", constraints=cons,
                       options=dict(maxiter=2000, ftol=1e-14))
        if best is None or res.fun < best.fun:
            best = res
    return best.x[:d], best.x[d], best.fun


@pytest.fixture(scope="module")
def small_optimum():
    X, y, C, q = _small()
    return X, y, C, q, _reduced_optimum(X, y, C, q)


@pytest.mark.parametrize("kw", [dict(rho_residual=False), dict(sigma_every=1),
                                dict(rho_residual=False, sigma_every=1)])
def test_literal_modes_reach_the_library_optimum(small_optimum, kw):
    X, y, C, q, (w_ref, b_ref, f_ref) = small_optimum
    sol = O.solve(X, y, C, q, tol=1e-9, max_iter=20000, **kw)
    assert sol["converged"]
    w = sol["w"] / max(1.0, np.linalg.norm(sol["w"]))
    f = O.reduced_objective(X, y, w, sol["beta"], C, q)
    assert abs(f - f_ref) / abs(f_ref) <= 1e-7
    assert np.linalg.norm(sol["w"] - w_ref) / np.linalg.norm(w_ref) <= 1e-4


def test_loop_stops_at_the_first_iterate_that_passes_the_rule():
    X, y, C, q = _small()
    tol = 1e-6
    sol = O.solve(X, y, C, q, tol=tol, max_iter=5000, record=True)
    h = sol["history"]
    assert sol["converged"] and sol["iters"] == len(h)

    def passes(x):   # the rule, from the table-pinned stop_test
        return O.stop_test(x, tol)

    assert passes(h[-1]) and not any(passes(x) for x in h[:-1])
