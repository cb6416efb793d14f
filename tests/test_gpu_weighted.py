"""Parity of the weighted problem on the GPU with the FP64 oracle: the class
weights of Section 4.5, a general penalty vector e in eq-primal, and the
Section 4.1 choice of C (dwd_suggest_C).

Bar as in the unweighted parity tests: relative (weighted) objective error
<= 1e-6 and ||w - w*|| / ||w*|| <= 1e-4 against a tight oracle reference,
and the FP64 KKT residuals of the weighted problem recomputed by the oracle
from the returned state within the requested tolerance.
"""
import numpy as np
import pytest

import synth
from oracle import dwd_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dwd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_12019_amd import dwd as D
    return D


def _wobj(X, y, C, q, s, wt, e):
    w = np.asarray(s["w"], np.float64)
    return O.reduced_objective(X, y, w / max(1.0, np.linalg.norm(w)), s["beta"], C, q, wt, e)


def _compare(X, y, C, q, got, ref, wt, e, obj_tol=1e-6, w_tol=1e-4):
    f_got, f_ref = _wobj(X, y, C, q, got, wt, e), _wobj(X, y, C, q, ref, wt, e)
    rel_obj = abs(f_got - f_ref) / abs(f_ref)
    rel_w = np.linalg.norm(got["w"] - ref["w"]) / np.linalg.norm(ref["w"])
    assert rel_obj <= obj_tol, (rel_obj, f_got, f_ref)
    assert rel_w <= w_tol, rel_w


def _data(d, n, storage, seed, pos_frac=0.15):
    X, y = synth.random_two_class(d, n, seed=seed, mean=0.6, pos_frac=pos_frac,
                                  dtype="f64" if storage == "f64" else "f32")
    return X, y


def test_weighted_trajectory_follows_oracle(dwd):
    # a fixed number of iterations from the same start: the iterates agree
    X, y = _data(1500, 60, "f64", seed=51)
    e = synth.penalty_vector(60, seed=52)
    C, q = 2.0, 1.0
    P = dwd.Problem(X, y, storage="f64")
    for k in (1, 2, 5, 20):
        o = O.solve(X, y, C, q, tol=1e-300, max_iter=k, weights=True, e=e)
        for rep in (0, 1):
            g = P.solve(C, q, tol=1e-300, max_iter=k, class_weights=1, e=e, representer=rep)
            assert g["info"]["iters"] == k
            assert np.allclose(g["alpha"], o["alpha"], rtol=1e-9, atol=1e-12), (k, rep)
            assert np.allclose(g["r"], o["r"], rtol=1e-9, atol=1e-12), (k, rep)
            assert np.allclose(g["xi"], o["xi"], rtol=1e-9, atol=1e-12), (k, rep)
            assert np.allclose(g["w"], o["w"], rtol=1e-9,
                               atol=1e-12 * np.abs(o["w"]).max()), (k, rep)
            assert abs(g["info"]["sigma"] - o["sigma"]) <= 1e-12 * o["sigma"]
    P.close()


@pytest.mark.parametrize("q,C,d,n,storage,cw,use_e,rep", [
    (1.0, 2.0, 3000, 200, "f64", 1, False, 0),
    (2.0, 5.0, 5000, 123, "f32", 1, True, 0),
    (0.5, 0.5, 2500, 77, "f32", 0, True, 0),
    (1.0, 1.0, 2000, 1100, "f64", 1, True, 1),
    (4.0, 10.0, 1500, 90, "f32", 1, True, 1),
    (1.0, 1.0, 4000, 150, "bf16", 1, True, 0),
])
def test_weighted_solves_match_oracle(dwd, q, C, d, n, storage, cw, use_e, rep):
    X, y = _data(d, n, storage, seed=3 * d + n)
    e = synth.penalty_vector(n, seed=n) if use_e else None
    wt = O.loss_weights(y, q, bool(cw))
    ref = O.solve(X, y, C, q, tol=1e-9, max_iter=20000, weights=bool(cw), e=e)
    assert ref["converged"]
    P = dwd.Problem(X, y, storage=storage)
    got = P.solve(C, q, tol=1e-8, max_iter=20000, class_weights=cw, e=e, representer=rep)
    assert got["info"]["converged"] == 1, got["info"]
    _compare(X, y, C, q, got, ref, wt, e)
    k = O.kkt_of_solution(X, y, C, q, got, weights=bool(cw), e=e)
    assert max(k["P"], k["D"]) <= 2e-8, k
    assert got["info"]["kkt_check"] < 1e-8
    # the reported objectives are the weighted ones
    assert abs(got["info"]["primal_obj"] - k["primobj"]) <= 1e-6 * abs(k["primobj"])
    assert abs(got["info"]["dual_obj"] - k["dualobj"]) <= 1e-6 * abs(k["dualobj"])
    if storage != "bf16":
        # at a working tolerance: the oracle's stopping point
        same = O.solve(X, y, C, q, tol=1e-6, max_iter=2000, weights=bool(cw), e=e)
        got6 = P.solve(C, q, tol=1e-6, class_weights=cw, e=e, representer=rep)
        assert got6["info"]["converged"] == 1
        assert abs(got6["info"]["iters"] - same["iters"]) <= max(3, 0.1 * same["iters"])
    # the handle goes back to e = 1 and no weights when they are not passed
    plain = P.solve(C, q, tol=1e-6)
    ref0 = O.solve(X, y, C, q, tol=1e-6, max_iter=2000)
    assert abs(plain["info"]["iters"] - ref0["iters"]) <= max(3, 0.1 * ref0["iters"])
    P.close()


def test_unweighted_defaults_are_bit_identical(dwd):
    # class_weights = 0 and e = ones give the unweighted solve bit for bit
    X, y = _data(2000, 90, "f32", seed=61)
    P = dwd.Problem(X, y, storage="f32")
    a = P.solve(1.5, 2.0, tol=1e-6)
    b = P.solve(1.5, 2.0, tol=1e-6, class_weights=0, e=np.ones(90))
    P.close()
    for key in ("w", "alpha", "r", "xi", "rho"):
        assert np.array_equal(a[key], b[key]), key
    assert a["info"]["iters"] == b["info"]["iters"]


def test_balanced_class_weights_are_one(dwd):
    X, y = synth.random_two_class(1000, 64, seed=62, mean=0.6, flip=0.0, dtype="f32")
    assert (y > 0).sum() == 32
    P = dwd.Problem(X, y, storage="f32")
    a = P.solve(1.0, 1.0, tol=1e-6)
    b = P.solve(1.0, 1.0, tol=1e-6, class_weights=1)
    P.close()
    assert np.array_equal(a["w"], b["w"]) and a["info"]["iters"] == b["info"]["iters"]


def test_weighted_batch_matches_oracle_and_single_solves(dwd):
    X, y = _data(2500, 77, "f64", seed=71)
    e1, e2 = synth.penalty_vector(77, seed=72), synth.penalty_vector(77, seed=73, low=0.5)
    grid = [dict(C=1.0, q=1.0), dict(C=1.0, q=1.0, class_weights=1),
            dict(C=3.0, q=2.0, e=e1), dict(C=0.5, q=0.5, class_weights=1, e=e2),
            dict(C=10.0, q=4.0, class_weights=1)]
    P = dwd.Problem(X, y, storage="f64")
    res = P.solve_batch([dict(g, tol=1e-8, max_iter=20000) for g in grid])
    for j, g in enumerate(grid):
        info = res["info"][j]
        assert info["converged"] == 1 and info["kkt_check"] < 1e-8, (j, info)
        cw, e = bool(g.get("class_weights", 0)), g.get("e")
        ref = O.solve(X, y, g["C"], g["q"], tol=1e-9, max_iter=20000, weights=cw, e=e)
        got = dict(w=res["W"][j], beta=info["beta"])
        _compare(X, y, g["C"], g["q"], got, ref, O.loss_weights(y, g["q"], cw), e)
    # FP64 products on both sides at a working tolerance: same stopping points
    res7 = P.solve_batch([dict(g, tol=5e-7) for g in grid])
    for j, g in enumerate(grid):
        alone = P.solve(tol=5e-7, want_state=False, C_=g["C"], q=g["q"],
                        **{k: v for k, v in g.items() if k not in ("C", "q")})
        a, b = alone["info"], res7["info"][j]
        assert b["converged"] == 1
        assert abs(a["iters"] - b["iters"]) <= max(2, 0.05 * a["iters"]), (j, a, b)
        assert np.linalg.norm(alone["w"] - res7["W"][j]) <= 1e-4 * np.linalg.norm(alone["w"])
    P.close()


def test_weighted_serve_and_csr(dwd):
    req = synth.Request(0, 0.0, d=3000, n=140, q=1.0, C=1.0, layout="csr", storage="f32",
                        seed=81)
    ip, ix, val, yc = synth.request_csr_data(req, density=5e-3)
    Xd = synth.csr_to_dense(ip, ix, val, 3000, np.float64)
    e = synth.penalty_vector(len(yc), seed=82)
    ref = O.solve(Xd, yc, 1.0, 1.0, tol=1e-9, max_iter=20000, weights=True, e=e)
    P = dwd.Problem(csr=(ip, ix, val, 3000), y=yc, storage="f32")
    got = P.solve(1.0, 1.0, tol=1e-8, max_iter=20000, class_weights=1, e=e)
    P.close()
    assert got["info"]["converged"] == 1
    _compare(Xd, yc, 1.0, 1.0, got, ref, O.class_weights(yc, 1.0), e)
    X, y = _data(2000, 100, "f32", seed=83)
    e2 = synth.penalty_vector(100, seed=84)
    out = dwd.serve([dict(X=X, y=y, t_arrival=0.0,
                          params=dict(C=2.0, q=2.0, tol=1e-7, class_weights=1, e=e2,
                                      max_iter=20000)),
                     dict(X=X, y=y, t_arrival=0.0, params=dict(C=2.0, q=2.0, tol=1e-7,
                                                               max_iter=20000))])
    alone = dwd.solve(X, y, 2.0, 2.0, tol=1e-7, class_weights=1, e=e2, max_iter=20000)
    assert out[0]["status"] == 0 and out[1]["status"] == 0
    assert np.linalg.norm(out[0]["w"] - alone["w"]) <= 1e-6 * np.linalg.norm(alone["w"])
    assert np.linalg.norm(out[0]["w"] - out[1]["w"]) > 1e-3 * np.linalg.norm(alone["w"])


def test_invalid_penalty_vectors_are_rejected(dwd):
    X, y = _data(500, 20, "f64", seed=91)
    P = dwd.Problem(X, y, storage="f64")
    for bad in (np.zeros(20), -np.ones(20), np.full(20, np.inf)):
        with pytest.raises(dwd.DwdError) as ei:
            P.solve(1.0, 1.0, e=bad)
        assert ei.value.status == -1
    with pytest.raises(ValueError):
        P.solve(1.0, 1.0, e=np.ones(19))
    with pytest.raises(dwd.DwdError):
        P.solve(1.0, 1.0, class_weights=2)
    # the handle still solves afterwards
    assert P.solve(1.0, 1.0, tol=1e-6)["info"]["converged"] == 1
    P.close()


# ---------------------------------------------------------------------------
# Section 4.1: the choice of C.
# ---------------------------------------------------------------------------

def test_suggest_C_hand_example(dwd):
    # four points on a line (d = 1): between-class distances 3, 5, 2, 4
    X = np.array([[0.0], [1.0], [3.0], [5.0]])
    y = np.array([1.0, 1.0, -1.0, -1.0])
    P = dwd.Problem(X, y, storage="f64")
    assert P.suggest_C(1.0) == pytest.approx(113.1668866220319, rel=1e-12)
    assert P.suggest_C(2.0) == pytest.approx(3233.33961777234, rel=1e-12)
    P.close()
    P = dwd.Problem(X * 100.0, y, storage="f64")
    assert P.suggest_C(1.0) == pytest.approx(100.0, rel=1e-14)
    P.close()


@pytest.mark.parametrize("d,n,storage,pos_frac", [(700, 51, "f64", 0.3), (5000, 123, "f32", 0.5),
                                                   (3000, 400, "f32", 0.1), (64, 9, "f64", 0.5)])
def test_suggest_C_matches_oracle(dwd, d, n, storage, pos_frac):
    X, y = _data(d, n, storage, seed=d + 2 * n, pos_frac=pos_frac)
    P = dwd.Problem(X, y, storage=storage)
    for q in (0.5, 1.0, 2.0, 4.0):
        got = P.suggest_C(q)
        want = O.suggest_C(X, y, q)
        assert got == pytest.approx(want, rel=1e-9), (q, got, want)
    P.close()


def test_suggest_C_csr_matches_dense(dwd):
    req = synth.Request(0, 0.0, d=2000, n=90, q=1.0, C=1.0, layout="csr", storage="f32", seed=93)
    ip, ix, val, yc = synth.request_csr_data(req, density=1e-2)
    Xd = synth.csr_to_dense(ip, ix, val, 2000, np.float64)
    P = dwd.Problem(csr=(ip, ix, val, 2000), y=yc, storage="f32")
    got = P.suggest_C(1.0)
    P.close()
    assert got == pytest.approx(O.suggest_C(Xd, yc, 1.0), rel=1e-6)


def test_unbalanced_full_size(dwd):
    """The unbalanced workload at full size (d=1e5, n=1000, one positive in
    ten, FP32 storage) with the Section 4.5 weights and the Section 4.1 C:
    the C against the oracle's, the weighted KKT residuals recomputed in
    FP64 by the oracle, and a weighted duality-gap certificate."""
    wl = synth.UNBALANCED_F32
    X, y = synth.two_class(wl.data)
    assert (y > 0).sum() < 0.2 * len(y)
    P = dwd.Problem(X, y, storage="f32")
    C = P.suggest_C(wl.q)
    Xd = X.astype(np.float64)
    assert C == pytest.approx(O.suggest_C(Xd, y, wl.q), rel=1e-9)
    got = P.solve(C, wl.q, tol=wl.tol, class_weights=1)
    P.close()
    info = got["info"]
    print("unbalanced solve:", {k: info[k] for k in ("iters", "setup_ms", "solve_ms",
                                                       "kkt_check", "eta_gap")}, "C", C)
    assert info["converged"] == 1
    k = O.kkt_of_solution(Xd, y, C, wl.q, got, weights=True)
    assert max(k["P"], k["D"]) <= 1.5 * wl.tol, k
    wt = O.class_weights(y, wl.q)
    w = got["w"] / max(1.0, np.linalg.norm(got["w"]))
    Pv = O.reduced_objective(Xd, y, w, got["beta"], C, wl.q, wt)
    # a feasible alpha: projection onto {0 <= a <= C, y^T a = 0}
    a = got["alpha"]
    f = lambda lam: y @ np.clip(a - lam * y, 0.0, C)
    lo, hi = -C - np.abs(a).max() - 1, C + np.abs(a).max() + 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 0 else (lo, mid)
    af = np.clip(a - 0.5 * (lo + hi) * y, 0.0, C)
    Dv = O.dual_objective_unscaled(Xd, y, af, wl.q, wt)
    assert Dv <= Pv
    # the stopping rule of Section 4.3 bounds the relative gap by 0.05 (it asks
    # only min(eta_C, eta_gap) < sqrt(tol)); the certificate agrees with the
    # gap the solver reports
    gap = (Pv - Dv) / (1 + abs(Pv) + abs(Dv))
    assert gap <= 0.05
    assert abs(gap - info["eta_gap"]) <= 0.1 * info["eta_gap"] + 1e-6
