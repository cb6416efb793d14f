"""Parity of the HIP solver (through the C ABI) with the FP64 oracle.

Bar (from the stated target): relative objective error <= 1e-6 and
||w - w*|| / ||w*|| <= 1e-4 against a tight oracle reference, and the FP64
KKT residuals recomputed by the oracle from the returned state within the
requested tolerance.
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


def _obj(X, y, w, beta, C, q):
    w = np.asarray(w, np.float64)
    return O.reduced_objective(X, y, w / max(1.0, np.linalg.norm(w)), beta, C, q)


def _compare(X, y, C, q, got, ref, obj_tol=1e-6, w_tol=1e-4):
    f_got = _obj(X, y, got["w"], got["beta"], C, q)
    f_ref = _obj(X, y, ref["w"], ref["beta"], C, q)
    rel_obj = abs(f_got - f_ref) / abs(f_ref)
    rel_w = np.linalg.norm(got["w"] - ref["w"]) / np.linalg.norm(ref["w"])
    assert rel_obj <= obj_tol, (rel_obj, f_got, f_ref)
    assert rel_w <= w_tol, rel_w
    return rel_obj, rel_w


def _recomputed_kkt(X, y, C, q, got, mu=1.0):
    e = O.kkt_of_solution(X, y, C, q, got, mu=mu)
    return max(e["P"], e["D"]), e


# ---------------------------------------------------------------------------
# Set-up quantities: Z_scale, G~, M^-1, M^-1 y.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,storage", [((200, 50), "f64"), ((5000, 123), "f32"),
                                           ((3000, 257), "f64"), ((1, 3), "f64")])
def test_setup_matches_oracle(dwd, shape, storage):
    d, n = shape
    X, y = synth.random_two_class(d, n, seed=d + n, dtype="f64" if storage == "f64" else "f32")
    mu = 1.7
    P = dwd.Problem(X, y, storage=storage, mu=mu)
    Zt, zs = O.scale_data(X, y)  # X as stored (FP32 values are exact in FP64)
    assert abs(P.inspect("zscale")[0] - zs) <= 1e-14 * zs
    G = Zt.T @ Zt
    Gg = P.inspect("G")
    assert np.max(np.abs(Gg - G)) <= 1e-13 * np.max(np.abs(G))
    Minv = np.linalg.inv(np.eye(n) + G / mu)
    Mg = P.inspect("Minv")
    assert np.max(np.abs(Mg - Minv)) <= 1e-11 * np.max(np.abs(Minv))
    assert np.max(np.abs(P.inspect("my") - Minv @ y)) <= 1e-11 * np.max(np.abs(Minv @ y))
    P.close()


# ---------------------------------------------------------------------------
# Whole solves against the oracle.
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_ref():
    wl = synth.SMALL_F64
    X, y = synth.two_class(wl.data)
    ref = O.solve(X, y, wl.C, wl.q, tol=1e-9, max_iter=20000)
    same = O.solve(X, y, wl.C, wl.q, tol=wl.tol, max_iter=2000)
    return X, y, wl, ref, same


def test_small_f64_solve_matches_oracle(dwd, small_ref):
    X, y, wl, ref, same = small_ref
    got = dwd.solve(X, y, wl.C, wl.q, tol=wl.tol, storage="f64")
    assert got["status"] == 0 and got["info"]["converged"] == 1
    _compare(X, y, wl.C, wl.q, got, ref)
    kkt, e = _recomputed_kkt(X, y, wl.C, wl.q, got)
    assert kkt <= wl.tol * (1 + 1e-6), e
    assert got["info"]["kkt_check"] < wl.tol
    # Same parameters, same tolerance: the iteration count follows the oracle's.
    assert abs(got["info"]["iters"] - same["iters"]) <= max(3, 0.1 * same["iters"])
    assert np.linalg.norm(got["w"]) <= 1 + 1e-5
    assert np.all(got["xi"] >= 0) and np.all(got["r"] > 0)


def test_small_f64_solve_matches_stored_solution(dwd):
    # The stored tight oracle solution (tests/golden/small_f64_solution.json,
    # written by tests/golden/make_golden.py from the oracle alone).
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "small_f64_solution.json")) as f:
        g = json.load(f)
    wl = synth.SMALL_F64
    X, y = synth.two_class(wl.data)
    got = dwd.solve(X, y, wl.C, wl.q, tol=1e-8, storage="f64", max_iter=20000)
    assert got["info"]["converged"] == 1
    _compare(X, y, wl.C, wl.q, got, dict(w=np.array(g["w"]), beta=g["beta"]))


def test_small_f64_trajectory_follows_oracle(dwd, small_ref):
    # A fixed number of iterations from the same start: the iterates agree.
    X, y, wl, ref, same = small_ref
    for k in (1, 2, 5, 20):
        o = O.solve(X, y, wl.C, wl.q, tol=1e-300, max_iter=k)
        g = dwd.solve(X, y, wl.C, wl.q, tol=1e-300, storage="f64", max_iter=k)
        assert g["info"]["iters"] == k
        assert np.allclose(g["alpha"], o["alpha"], rtol=1e-9, atol=1e-12), k
        assert np.allclose(g["r"], o["r"], rtol=1e-9, atol=1e-12), k
        assert np.allclose(g["w"], o["w"], rtol=1e-9, atol=1e-12 * np.abs(o["w"]).max()), k
        assert abs(g["info"]["sigma"] - o["sigma"]) <= 1e-12 * o["sigma"]


def test_large_n_trajectory_follows_oracle(dwd):
    # n = 6001 (ragged) takes the paths that small n never reaches: several
    # 2048-sample panels in the pass, the pass's looped plan reduction, row
    # dots over six 1024-wide chunks, and several load rounds per lane in the
    # tail's sums.  Weighted, with a penalty vector, so both Step 1c outcomes
    # and every n-space sum are exercised.
    d, n = 2000, 6001
    X, y = synth.random_two_class(d, n, seed=61, mean=0.4, pos_frac=0.3, dtype="f32")
    e = synth.penalty_vector(n, seed=62)
    C, q = 2.0, 1.0
    P = dwd.Problem(X, y, storage="f32")
    for k in (1, 3, 8):
        o = O.solve(X, y, C, q, tol=1e-300, max_iter=k, weights=True, e=e)
        g = P.solve(C, q, tol=1e-300, max_iter=k, class_weights=1, e=e)
        assert g["info"]["iters"] == k
        for key in ("alpha", "r", "xi"):
            assert np.allclose(g[key], o[key], rtol=1e-9, atol=1e-12), (k, key)
        for key in ("w", "u", "rho"):
            assert np.allclose(g[key], o[key], rtol=1e-9,
                               atol=1e-12 * max(1e-300, np.abs(o[key]).max())), (k, key)
        assert abs(g["beta"] - o["beta"]) <= 1e-9 * max(1.0, abs(o["beta"])), k
        assert abs(g["info"]["sigma"] - o["sigma"]) <= 1e-12 * o["sigma"]
        assert g["info"]["n_double"] == o["n_double"], k
    P.close()


@pytest.mark.parametrize("q,C,d,n,storage", [
    (2.0, 3.0, 5000, 123, "f32"),
    (0.5, 0.2, 3000, 200, "f64"),
    (4.0, 10.0, 2500, 77, "f32"),
    (1.0, 1.0, 700, 50, "f32"),
])
def test_ragged_solves_match_oracle(dwd, q, C, d, n, storage):
    X, y = synth.random_two_class(d, n, seed=7 * d + n, mean=0.6,
                                  dtype="f64" if storage == "f64" else "f32")
    ref = O.solve(X, y, C, q, tol=1e-9, max_iter=20000)
    # Against the tight reference: solve to a tolerance at which the
    # objective is settled to the 1e-6 bar.
    got = dwd.solve(X, y, C, q, tol=1e-8, storage=storage, max_iter=20000)
    assert got["info"]["converged"] == 1, got["info"]
    _compare(X, y, C, q, got, ref)
    kkt, e = _recomputed_kkt(X, y, C, q, got)
    assert kkt <= 2e-8, e
    # At a working tolerance: the same stopping point as the oracle's.
    same = O.solve(X, y, C, q, tol=1e-6, max_iter=2000)
    got6 = dwd.solve(X, y, C, q, tol=1e-6, storage=storage)
    assert got6["info"]["converged"] == 1
    assert abs(got6["info"]["iters"] - same["iters"]) <= max(3, 0.1 * same["iters"])
    kkt, e = _recomputed_kkt(X, y, C, q, got6)
    assert kkt <= 2e-6, e


def test_mu_and_exact_sgs_modes(dwd, small_ref):
    X, y, wl, ref, same = small_ref
    for kw in (dict(mu=2.5), dict(eps_c=0.0), dict(resync=0), dict(resync=7)):
        got = dwd.solve(X, y, wl.C, wl.q, tol=1e-8, storage="f64", max_iter=20000, **kw)
        assert got["info"]["converged"] == 1, kw
        _compare(X, y, wl.C, wl.q, got, ref)
        if kw.get("eps_c") == 0.0:
            assert got["info"]["n_double"] >= got["info"]["iters"] - 1


@pytest.mark.parametrize("kw", [dict(rho_residual=0), dict(sigma_every=1),
                                dict(rho_residual=0, sigma_every=1)])
def test_paper_literal_modes_follow_oracle(dwd, small_ref, kw):
    """The printed two-term eta_D of Section 4.3 (rho_residual = 0) and the
    sigma rule of Section 4.4 after every iteration (sigma_every = 1): the
    first iterates agree with the oracle run in the same mode, a whole solve
    stops where the oracle's does, and a tight solve reaches the optimum."""
    X, y, wl, ref, _ = small_ref
    okw = dict(rho_residual=bool(kw.get("rho_residual", 1)), sigma_every=kw.get("sigma_every", 2))
    for k in (1, 2, 5, 20):
        o = O.solve(X, y, wl.C, wl.q, tol=1e-300, max_iter=k, **okw)
        g = dwd.solve(X, y, wl.C, wl.q, tol=1e-300, storage="f64", max_iter=k, **kw)
        assert g["info"]["iters"] == k
        for key in ("alpha", "r", "xi"):
            assert np.allclose(g[key], o[key], rtol=1e-9, atol=1e-12), (k, key)
        assert np.allclose(g["w"], o["w"], rtol=1e-9, atol=1e-12 * np.abs(o["w"]).max()), k
        assert abs(g["info"]["sigma"] - o["sigma"]) <= 1e-12 * o["sigma"], k
    same = O.solve(X, y, wl.C, wl.q, tol=wl.tol, max_iter=2000, **okw)
    got = dwd.solve(X, y, wl.C, wl.q, tol=wl.tol, storage="f64", **kw)
    assert got["status"] == 0 and got["info"]["converged"] == 1, got["info"]
    assert got["info"]["kkt_check"] < wl.tol
    assert abs(got["info"]["iters"] - same["iters"]) <= max(3, 0.1 * same["iters"]), \
        (got["info"]["iters"], same["iters"])
    tight = dwd.solve(X, y, wl.C, wl.q, tol=1e-8, storage="f64", max_iter=20000, **kw)
    assert tight["info"]["converged"] == 1
    _compare(X, y, wl.C, wl.q, tight, ref)


def test_paper_literal_modes_ragged_f32(dwd):
    """The literal modes on FP32 storage with a ragged shape (several tiles
    and a tail): first iterates and a whole solve against the oracle in the
    same mode.  On this case the printed two-term eta_D, which never measures
    w-stationarity (||Z~ alpha + D rho||, eta_D3), lets the stopping rule
    stop at tol 1e-8 about 0.5% above the optimal objective, with eta_D3
    near 1e-3; the oracle stops at the same point.  With the D3 term (the
    default) the same tolerance reaches the optimum."""
    d, n, q, C = 5000, 123, 2.0, 3.0
    X, y = synth.random_two_class(d, n, seed=7 * d + n, mean=0.6, dtype="f32")
    P = dwd.Problem(X, y, storage="f32")
    for k in (3, 8):
        o = O.solve(X, y, C, q, tol=1e-300, max_iter=k, rho_residual=False, sigma_every=1)
        g = P.solve(C, q, tol=1e-300, max_iter=k, rho_residual=0, sigma_every=1)
        for key in ("alpha", "r", "xi"):
            assert np.allclose(g[key], o[key], rtol=1e-9, atol=1e-12), (k, key)
        assert abs(g["info"]["sigma"] - o["sigma"]) <= 1e-12 * o["sigma"], k
    same = O.solve(X, y, C, q, tol=1e-8, max_iter=20000, rho_residual=False, sigma_every=1)
    got = P.solve(C, q, tol=1e-8, max_iter=20000, rho_residual=0, sigma_every=1)
    full = P.solve(C, q, tol=1e-8, max_iter=20000, sigma_every=1)
    P.close()
    assert got["info"]["converged"] == 1 and got["info"]["kkt_check"] < 1e-8, got["info"]
    assert abs(got["info"]["iters"] - same["iters"]) <= max(3, 0.1 * same["iters"]), \
        (got["info"]["iters"], same["iters"])
    _compare(X, y, C, q, got, same)  # the same stopping point
    ref = O.solve(X, y, C, q, tol=1e-9, max_iter=20000)
    f_got, f_ref = _obj(X, y, got["w"], got["beta"], C, q), _obj(X, y, ref["w"], ref["beta"], C, q)
    e = O.kkt_of_solution(X, y, C, q, got)
    print("printed eta_D: rel. objective above the optimum %.3e, eta_D3 %.3e" % (
        (f_got - f_ref) / f_ref, e["D3"]))
    assert f_got - f_ref > 1e-3 * f_ref and e["D3"] > 1e-4
    assert full["info"]["converged"] == 1
    _compare(X, y, C, q, full, ref)


def test_bf16_storage_with_fp32_refinement(dwd):
    X, y = synth.random_two_class(6000, 150, seed=31, mean=0.6, log_scale=1.0, dtype="f32")
    q, C = 2.0, 1.0
    ref = O.solve(X, y, C, q, tol=1e-9, max_iter=20000)
    got = dwd.solve(X, y, C, q, tol=1e-8, storage="bf16", max_iter=20000)
    assert got["info"]["converged"] == 1
    assert got["info"]["iters_lowp"] > 0
    _compare(X, y, C, q, got, ref)
    kkt, e = _recomputed_kkt(X, y, C, q, got)
    assert kkt <= 2e-8, e


def _bf16_round(X):
    """Round FP32 values to BF16 (nearest, ties to even), returned as FP32."""
    b = np.ascontiguousarray(X, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def test_bf16_phase_solves_the_bf16_problem(dwd):
    """With refinement off and a tight phase tolerance, the BF16 phase alone
    must reach the solution of the problem posed on the BF16-rounded data
    (its factor is the FP64 factor of that image)."""
    X, y = synth.random_two_class(5000, 120, seed=32, mean=0.6, log_scale=1.0, dtype="f32")
    Xb = _bf16_round(X)
    assert np.max(np.abs(Xb - X) / np.maximum(np.abs(X), 1e-30)) <= 2.0 ** -8
    for q, C in ((1.0, 1.0), (2.0, 0.3)):
        got = dwd.solve(X, y, C, q, tol=1e-8, storage="bf16", refine=0, lowp_tol=1e-8,
                        max_iter=20000)
        assert got["info"]["iters_lowp"] == got["info"]["iters"]
        ref = O.solve(Xb, y, C, q, tol=1e-9, max_iter=20000)
        f = _obj(Xb, y, got["w"], got["beta"], C, q)
        fr = _obj(Xb, y, ref["w"], ref["beta"], C, q)
        assert abs(f - fr) <= 1e-6 * abs(fr), (q, C, f, fr)
        assert np.linalg.norm(got["w"] - ref["w"]) <= 1e-4 * np.linalg.norm(ref["w"]), (q, C)


# ---------------------------------------------------------------------------
# Edge cases.
# ---------------------------------------------------------------------------

def test_degenerate_shapes(dwd):
    # one sample per class; d = 1; n > d
    for d, n, seed in ((1, 2, 1), (1, 7, 2), (3, 40, 3), (64, 2, 4)):
        X, y = synth.random_two_class(d, n, seed=seed, mean=1.0)
        got = dwd.solve(X, y, 1.0, 1.0, tol=1e-6, storage="f64", max_iter=5000)
        ref = O.solve(X, y, 1.0, 1.0, tol=1e-9, max_iter=50000)
        f_got = _obj(X, y, got["w"], got["beta"], 1.0, 1.0)
        f_ref = _obj(X, y, ref["w"], ref["beta"], 1.0, 1.0)
        assert abs(f_got - f_ref) <= 1e-5 * abs(f_ref), (d, n)


def test_iteration_cap_returns_valid_state(dwd, small_ref):
    X, y, wl, ref, same = small_ref
    got = dwd.solve(X, y, wl.C, wl.q, tol=wl.tol, storage="f64", max_iter=1)
    assert got["status"] == 1 and got["info"]["iters"] == 1 and got["info"]["converged"] == 0
    assert np.all(np.isfinite(got["w"])) and np.all(got["r"] > 0)


def test_host_stops_queueing_at_the_device_stop(dwd):
    # The tail kernel that sets the stop flag also sets a pinned host word,
    # which the host reads one chunk of queued iterations behind: a solve that
    # converges long before max_iter queues a chunk or two past the stop.  A
    # host that missed the word would queue 4e6 launches (seconds of work).
    X, y = synth.random_two_class(3000, 100, seed=9, dtype="f32")
    P = dwd.Problem(X, y, storage="f32")
    first = P.solve(1.0, 1.0, tol=1e-4)
    r = P.solve(1.0, 1.0, tol=1e-4, max_iter=1000000)
    P.close()
    i = r["info"]
    assert i["converged"] == 1 and i["iters"] == first["info"]["iters"]
    assert i["solve_ms"] < 1000.0, i["solve_ms"]
    assert np.array_equal(r["w"], first["w"])


def test_invalid_inputs_are_rejected(dwd):
    X, y = synth.random_two_class(100, 10, seed=5)
    Xn = X.copy()
    Xn[3, 7] = np.nan
    with pytest.raises(dwd.DwdError) as ei:
        dwd.Problem(Xn, y, storage="f64")
    assert ei.value.status == -1
    with pytest.raises(dwd.DwdError):
        dwd.Problem(np.zeros_like(X), y, storage="f64")
    P = dwd.Problem(X, y, storage="f64")
    for bad in (dict(C_=-1.0), dict(q=0.0), dict(tol=0.0), dict(tol=1.5), dict(max_iter=0),
                dict(tau=2.0)):
        with pytest.raises(dwd.DwdError):
            P.solve(**bad)
    P.close()


def test_repeated_solves_on_one_handle_are_identical(dwd):
    X, y = synth.random_two_class(3000, 100, seed=8, dtype="f32")
    P = dwd.Problem(X, y, storage="f32")
    a = P.solve(2.0, 1.0, tol=1e-6)
    b = P.solve(0.5, 2.0, tol=1e-6)
    c = P.solve(2.0, 1.0, tol=1e-6)
    assert np.array_equal(a["w"], c["w"]) and a["info"]["iters"] == c["info"]["iters"]
    assert not np.array_equal(a["w"], b["w"])
    P.close()


# ---------------------------------------------------------------------------
# The HDLSS workload at full size (d = 1e5, n = 1e3, FP32): properties that
# hold at any size, checked in FP64 by the oracle from the returned state.
# ---------------------------------------------------------------------------

def _dual_feasible(alpha, y, C):
    f = lambda lam: y @ np.clip(alpha - lam * y, 0.0, C)
    lo, hi = -C - np.abs(alpha).max() - 1, C + np.abs(alpha).max() + 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 0 else (lo, mid)
    return np.clip(alpha - 0.5 * (lo + hi) * y, 0.0, C)


def test_hdlss_full_size_properties(dwd):
    wl = synth.HDLSS_F32
    X, y = synth.two_class(wl.data)
    got = dwd.solve(X, y, wl.C, wl.q, tol=wl.tol, storage="f32")
    info = got["info"]
    print("HDLSS solve:", {k: info[k] for k in ("iters", "n_double", "setup_ms", "solve_ms",
                                                  "kkt_check", "eta_gap")})
    assert info["converged"] == 1 and info["kkt_check"] < wl.tol
    kkt, e = _recomputed_kkt(X, y, wl.C, wl.q, got)
    assert kkt <= wl.tol * (1 + 1e-6), e
    # Duality-gap certificate: the optimum lies between the dual value at a
    # feasible alpha and the primal value at the returned (w, beta).
    Xd = X.astype(np.float64)
    w = got["w"] / max(1.0, np.linalg.norm(got["w"]))
    P = O.reduced_objective(Xd, y, w, got["beta"], wl.C, wl.q)
    a = _dual_feasible(got["alpha"], y, wl.C)
    D = O.dual_objective_unscaled(Xd, y, a, wl.q)
    assert D <= P
    assert (P - D) / abs(P) <= 1e-3
    # sampled outputs: margins of 64 samples recomputed one by one in FP64
    idx = np.random.default_rng(0).choice(X.shape[0], 64, replace=False)
    m_gpu = got["r"][idx] - got["xi"][idx]
    m_ref = y[idx] * (Xd[idx] @ got["w"] + got["beta"])
    # r - xi = Z~^T w~ + beta y = y (x^T w + beta) for the unscaled w
    # (w~ = Z_scale w, Z~ = Z / Z_scale), up to the primal residual
    assert np.max(np.abs(m_gpu - m_ref)) <= 10 * wl.tol * (1 + wl.C)


def test_hdlss_full_size_against_oracle(dwd):
    """The HDLSS workload at full size (d = 1e5, n = 1e3, FP32 data) against
    the FP64 oracle.  At the working tolerance 1e-5 the GPU follows the
    oracle's own trajectory: the same iteration count and the same w and
    beta.  At 1e-6 it reaches the optimum stored in tests/golden (written by
    the oracle at 1e-9): w* = Z alpha* / ||Z alpha*||, objective within 1e-6,
    w within 1e-4.  (At 1e-5 the oracle's own w is about 4e-4 from w*, so
    the w bar is taken at 1e-6.)"""
    import json
    import os
    wl = synth.HDLSS_F32
    X, y = synth.two_class(wl.data)
    Xd = X.astype(np.float64)
    P = dwd.Problem(X, y, storage="f32")
    got = P.solve(wl.C, wl.q, tol=wl.tol, want_state=False)
    same = O.solve(Xd, y, wl.C, wl.q, tol=wl.tol, max_iter=2000)
    gi = got["info"]
    rel_w = np.linalg.norm(got["w"] - same["w"]) / np.linalg.norm(same["w"])
    print("HDLSS vs oracle: iters %d/%d n_double %d/%d rel_w %.2e beta %.12g/%.12g" % (
        gi["iters"], same["iters"], gi["n_double"], same["n_double"], rel_w, got["beta"],
        same["beta"]))
    assert gi["converged"] == 1 and gi["kkt_check"] < wl.tol, gi
    assert same["converged"]
    assert abs(gi["iters"] - same["iters"]) <= 2, (gi["iters"], same["iters"])
    f_got, f_same = _obj(Xd, y, got["w"], got["beta"], wl.C, wl.q), \
        _obj(Xd, y, same["w"], same["beta"], wl.C, wl.q)
    if gi["iters"] == same["iters"]:  # the same stopping point
        assert rel_w <= 1e-6, rel_w
        assert abs(got["beta"] - same["beta"]) <= 1e-6 * max(1.0, abs(same["beta"]))
        assert abs(f_got - f_same) <= 1e-9 * abs(f_same), (f_got, f_same)
    else:  # a neighbouring iterate of the same trajectory
        assert abs(f_got - f_same) <= 2e-6 * abs(f_same), (f_got, f_same)
    # the optimum
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "hdlss_f32_solution.json")) as f:
        g = json.load(f)
    za = _z_alpha_by_rows(X, y, np.array(g["alpha"]))
    w_star = za / np.linalg.norm(za)
    tight = P.solve(wl.C, wl.q, tol=1e-6, want_state=False, max_iter=20000)
    P.close()
    assert tight["info"]["converged"] == 1 and tight["info"]["kkt_check"] < 1e-6
    f_t = _obj(Xd, y, tight["w"], tight["beta"], wl.C, wl.q)
    rel_obj = abs(f_t - g["reduced_objective"]) / abs(g["reduced_objective"])
    rel_ws = np.linalg.norm(tight["w"] - w_star) / np.linalg.norm(w_star)
    print("HDLSS tol 1e-6 vs stored optimum: rel_obj %.2e rel_w %.2e" % (rel_obj, rel_ws))
    assert rel_obj <= 1e-6 and rel_ws <= 1e-4, (rel_obj, rel_ws)
    # and the working-tolerance solve is within 1e-6 of the optimal objective
    assert abs(f_got - g["reduced_objective"]) <= 1e-6 * abs(g["reduced_objective"])


def _margins_by_rows(X, y, w, beta, rows=64):
    """y_i (x_i^T w + beta) for every sample, in FP64, a block of rows at a time."""
    m = np.empty(X.shape[0])
    for r0 in range(0, X.shape[0], rows):
        r1 = min(X.shape[0], r0 + rows)
        m[r0:r1] = y[r0:r1] * (X[r0:r1].astype(np.float64) @ w + beta)
    return m


def _z_alpha_by_rows(X, y, a, rows=64):
    """Z alpha = sum_i a_i y_i x_i in FP64, a block of rows at a time."""
    acc = np.zeros(X.shape[1])
    for r0 in range(0, X.shape[0], rows):
        r1 = min(X.shape[0], r0 + rows)
        acc += X[r0:r1].astype(np.float64).T @ (y[r0:r1] * a[r0:r1])
    return acc


def _kkt_by_rows(X, y, C, got, mu=1.0, rows=64):
    """The Section 4.3 residuals eta_P and eta_D (with the D3 term) of a
    returned state, on the scaled problem, from X in row blocks in FP64: for
    data too large to scale whole on the host.  With w~ = Z_scale w,
    u~ = Z_scale u, Z~ = Z / Z_scale (Section 4.2):
      P1 = ||Z^T w + beta y + xi - r||, P2 = sqrt(mu) Z_scale ||w - u||,
      P3 = Z_scale max(||w|| - 1, 0), D1 = ||min(0, alpha)||,
      D2 = ||max(0, alpha - C)||, D3 = ||Z alpha / Z_scale + sqrt(mu) rho||,
    each over 1 + C."""
    fro2 = 0.0
    for r0 in range(0, X.shape[0], rows):
        b = X[r0:r0 + rows].astype(np.float64)
        fro2 += float(np.sum(b * b))
    zs = fro2 ** 0.25
    w, u, a = got["w"], got["u"], got["alpha"]
    m = _margins_by_rows(X, y, w, got["beta"], rows)
    den = 1.0 + C
    p1 = np.linalg.norm(m + got["xi"] - got["r"]) / den
    p2 = np.sqrt(mu) * zs * np.linalg.norm(w - u) / den
    p3 = zs * max(np.linalg.norm(w) - 1.0, 0.0) / den
    d1 = np.linalg.norm(np.minimum(0.0, a)) / den
    d2 = np.linalg.norm(np.maximum(0.0, a - C)) / den
    d3 = np.linalg.norm(_z_alpha_by_rows(X, y, a, rows) / zs + np.sqrt(mu) * got["rho"]) / den
    return max(p1, p2, p3), max(d1, d2, d3)


def test_large_bf16_full_size(dwd):
    """The large mixed-precision workload at full size (d=1e6, n=2000, q=2,
    C=1, BF16 storage of Z, FP64 factors, FP32 refinement): the FP64 check on
    the device, every sample's margin recomputed in FP64 on the host, a
    duality-gap certificate, and agreement with FP32 storage."""
    torch = pytest.importorskip("torch")
    # the host helper reproduces the oracle's residuals on a small solved state
    Xs, ys = synth.random_two_class(300, 40, seed=5, mean=0.6, dtype="f32")
    so = O.solve(Xs, ys, 1.0, 2.0, tol=1e-4)
    ek = O.kkt_of_solution(Xs, ys, 1.0, 2.0, so)
    hp, hd = _kkt_by_rows(Xs, ys, 1.0, so)
    assert abs(hp - ek["P"]) <= 1e-12 + 1e-9 * ek["P"] and abs(hd - ek["D"]) <= 1e-12 + 1e-9 * ek["D"]
    wl = synth.LARGE_BF16
    X, y = synth.two_class(wl.data)
    Xd = torch.from_numpy(X).to("cuda")
    got = dwd.solve(Xd, y, wl.C, wl.q, tol=wl.tol, storage="bf16", max_iter=20000)
    info = got["info"]
    print("large BF16 solve:", {k: info[k] for k in ("iters", "iters_lowp", "setup_ms",
                                                      "solve_ms", "kkt_check", "eta_gap")})
    assert info["converged"] == 1 and info["iters_lowp"] > 0
    assert info["kkt_check"] < wl.tol
    # the residuals recomputed on the host in FP64 from the returned state
    ep, ed = _kkt_by_rows(X, y, wl.C, got)
    print("large BF16 host residuals: eta_P %.3e (device %.3e) eta_D %.3e (device %.3e)" % (
        ep, info["eta_p_check"], ed, info["eta_d_check"]))
    assert max(ep, ed) < wl.tol, (ep, ed)
    assert abs(ep - info["eta_p_check"]) <= 1e-3 * wl.tol
    assert abs(ed - info["eta_d_check"]) <= 1e-3 * wl.tol
    # r - xi = y (x^T w + beta) for every sample, up to the primal residual
    m = _margins_by_rows(X, y, got["w"], got["beta"])
    assert np.max(np.abs((got["r"] - got["xi"]) - m)) <= 10 * wl.tol * (1 + wl.C)
    assert np.all(got["xi"] >= 0.0) and np.all(got["r"] > 0.0)
    assert np.linalg.norm(got["w"]) <= 1.0 + 1e-4
    # duality-gap certificate at a feasible alpha
    wn = got["w"] / max(1.0, np.linalg.norm(got["w"]))
    P = float(np.sum(O.reduced_loss(_margins_by_rows(X, y, wn, got["beta"]), wl.C, wl.q)))
    a = _dual_feasible(got["alpha"], y, wl.C)
    D = float(O.kappa(wl.q) * np.sum(a ** (wl.q / (wl.q + 1.0)))
              - np.linalg.norm(_z_alpha_by_rows(X, y, a)))
    assert D <= P
    assert (P - D) <= 0.06 * (1.0 + abs(P) + abs(D)), (P, D)
    # the same problem with FP32 storage reaches the same objective
    ref = dwd.solve(Xd, y, wl.C, wl.q, tol=wl.tol, storage="f32", max_iter=20000,
                    want_state=False)
    assert ref["info"]["converged"] == 1
    wr = ref["w"] / max(1.0, np.linalg.norm(ref["w"]))
    Pr = float(np.sum(O.reduced_loss(_margins_by_rows(X, y, wr, ref["beta"]), wl.C, wl.q)))
    print("primal objective bf16 %.9g f32 %.9g" % (P, Pr))
    assert abs(P - Pr) <= 1e-4 * abs(Pr)


# ---------------------------------------------------------------------------
# Representer iteration (params.representer = 1): no pass over Z per
# iteration; the same solution as the pass iteration and the oracle.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,n,q,C,storage", [(5000, 123, 2.0, 3.0, "f32"),
                                             (3000, 200, 0.5, 0.2, "f64"),
                                             (700, 50, 1.0, 1.0, "f32"),
                                             (800, 1100, 1.0, 0.5, "f64")])
def test_representer_matches_pass_iteration_and_oracle(dwd, d, n, q, C, storage):
    X, y = synth.random_two_class(d, n, seed=d + n + 7, mean=0.6,
                                  dtype="f64" if storage == "f64" else "f32")
    ref = O.solve(X, y, C, q, tol=1e-9, max_iter=20000)
    P = dwd.Problem(X, y, storage=storage)
    rep = P.solve(C, q, tol=1e-8, max_iter=20000, representer=1)
    assert rep["info"]["converged"] == 1 and rep["info"]["stream_launches"] == 0
    _compare(X, y, C, q, rep, ref)
    kkt, e = _recomputed_kkt(X, y, C, q, rep)
    assert kkt <= 2e-8, e
    # Same iteration as the pass form: at a working tolerance the counts agree
    # (near 1e-8 the sigma sequence is sensitive to rounding order, and the
    # counts of any two summation orders can differ by large factors: the
    # oracle itself needs 603 iterations at 1e-7 and 4196 at 1e-8 on one of
    # these cases).
    rep6 = P.solve(C, q, tol=1e-6, max_iter=20000, representer=1)
    pas6 = P.solve(C, q, tol=1e-6, max_iter=20000)
    P.close()
    a, b = rep6["info"]["iters"], pas6["info"]["iters"]
    assert abs(a - b) <= max(3, 0.10 * b), (a, b)
    assert np.linalg.norm(rep6["w"] - pas6["w"]) <= 1e-4 * np.linalg.norm(pas6["w"])


def test_representer_first_iterates_follow_the_pass_iteration(dwd):
    """The two forms are the same iteration: after k = 1, 2, 5, 20 iterations
    the states agree to rounding."""
    wl = synth.SMALL_F64
    X, y = synth.two_class(wl.data)
    P = dwd.Problem(X, y, storage="f64")
    for k in (1, 2, 5, 20):
        a = P.solve(wl.C, wl.q, tol=1e-12, max_iter=k, representer=1)
        b = P.solve(wl.C, wl.q, tol=1e-12, max_iter=k)
        for key in ("r", "xi", "alpha", "w", "u", "rho"):
            assert np.allclose(a[key], b[key], rtol=1e-9, atol=1e-12), (k, key)
        assert abs(a["beta"] - b["beta"]) <= 1e-9 * max(1.0, abs(b["beta"])), k
    P.close()


def test_representer_with_bf16_and_csr_inputs(dwd):
    # BF16 storage: the iteration never reads Z, so there is no BF16 phase
    X, y = synth.random_two_class(4000, 150, seed=41, mean=0.6, dtype="f32")
    r = dwd.solve(X, y, 1.0, 2.0, tol=1e-7, storage="bf16", representer=1, max_iter=20000)
    assert r["info"]["converged"] == 1 and r["info"]["iters_lowp"] == 0
    f = dwd.solve(X, y, 1.0, 2.0, tol=1e-7, storage="f32", representer=1, max_iter=20000)
    assert np.linalg.norm(r["w"] - f["w"]) <= 1e-9 * np.linalg.norm(f["w"])
    # CSR input
    req = synth.Request(0, 0.0, d=3000, n=140, q=1.0, C=1.0, layout="csr", storage="f32",
                        seed=42)
    ip, ix, val, yc = synth.request_csr_data(req, density=5e-3)
    Xd = synth.csr_to_dense(ip, ix, val, 3000, np.float64)
    ref = O.solve(Xd, yc, 1.0, 1.0, tol=1e-9, max_iter=20000)
    P = dwd.Problem(csr=(ip, ix, val, 3000), y=yc, storage="f32")
    got = P.solve(1.0, 1.0, tol=1e-8, max_iter=20000, representer=1)
    P.close()
    assert got["info"]["converged"] == 1
    _compare(Xd, yc, 1.0, 1.0, got, ref)
