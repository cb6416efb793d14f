"""Parity of the iterative branch (Section 3.3.3) with the oracle's, through
the C ABI: PSQMR solves of eq-linsys with T = 0 to the accuracy of
eq-linsys-tol, the switch to the proximal term of eq-T after a solve of more
than psqmr_max steps, and the eq-T iteration itself (T from the ell largest
eigenpairs of Z~ Z~^T, solved in closed form through eq-schur) from the
first iteration (psqmr_max = 0)."""
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


def _data(d, n, seed, storage="f32", log_scale=0.5):
    return synth.random_two_class(d, n, seed=seed, mean=0.6, log_scale=log_scale,
                                  dtype="f64" if storage == "f64" else "f32")


@pytest.mark.parametrize("d,n,ell,storage", [(400, 300, 10, "f32"), (1500, 120, 6, "f64"),
                                             (3000, 2100, 6, "f32"), (7000, 90, 12, "f32")])
def test_eigenpairs_match_the_oracle_lanczos_and_a_dense_solver(dwd, d, n, ell, storage):
    # (64 Lanczos steps resolve these top pairs; the flat spectrum of the
    # d = 3000, n = 2100 data is spread by feature scales over 1.5 decades)
    X, y = _data(d, n, seed=d + n, storage=storage, log_scale=1.5 if d == 3000 else 0.5)
    P = dwd.Problem(X, y, storage=storage, solver="iterative", ell=ell)
    assert P.inspect("solver")[0] == 3 and P.inspect("ell")[0] == ell
    lam = P.inspect("lam")
    P.close()
    Zt, _ = O.scale_data(X, y)
    lo, _ = O.top_eigenpairs(lambda v: Zt @ (Zt.T @ v), d, ell)
    assert np.allclose(lam, lo, rtol=1e-9)
    ev = np.linalg.eigvalsh(Zt.T @ Zt)[::-1][:ell]   # the same nonzero spectrum
    assert np.allclose(lam, ev, rtol=1e-7)


@pytest.mark.parametrize("d,n,storage", [(400, 300, "f32"), (900, 150, "f64")])
def test_iterative_trajectory_follows_oracle(dwd, d, n, storage):
    X, y = _data(d, n, seed=3 * d + n, storage=storage)
    e = synth.penalty_vector(n, seed=n + 3)
    C, q = 1.0, 1.0
    P = dwd.Problem(X, y, storage=storage, solver="iterative", ell=8)
    for k in (1, 2, 5, 20):
        o = O.solve(X, y, C, q, tol=1e-300, max_iter=k, solver="iterative", ell=8, psqmr_max=0,
                    weights=True, e=e)
        g = P.solve(C, q, tol=1e-300, max_iter=k, class_weights=1, e=e, psqmr_max=0)
        assert g["info"]["iters"] == k
        for key in ("alpha", "r", "xi"):
            assert np.allclose(g[key], o[key], rtol=1e-8, atol=1e-11), (k, key)
        for key in ("w", "u", "rho"):
            assert np.allclose(g[key], o[key], rtol=1e-8,
                               atol=1e-11 * max(1e-300, np.abs(o[key]).max())), (k, key)
        assert abs(g["beta"] - o["beta"]) <= 1e-8 * max(1.0, abs(o["beta"])), k
        assert g["info"]["n_double"] == o["n_double"], k
    P.close()


@pytest.mark.parametrize("d,n,q,C", [(400, 300, 1.0, 1.0), (800, 200, 2.0, 3.0),
                                     (300, 1000, 0.5, 0.5)])
def test_iterative_solves_match_oracle(dwd, d, n, q, C):
    X, y = _data(d, n, seed=d + n, log_scale=0.5 if d != 800 else 1.0)
    P = dwd.Problem(X, y, storage="f32", solver="iterative")
    for tol in (1e-6, 1e-7):
        ref = O.solve(X, y, C, q, tol=tol, max_iter=20000, solver="iterative", psqmr_max=0)
        assert ref["converged"]
        got = P.solve(C, q, tol=tol, max_iter=20000, psqmr_max=0)
        assert got["info"]["converged"] == 1, got["info"]
        assert abs(got["info"]["iters"] - ref["iters"]) <= max(3, 0.1 * ref["iters"]), tol
        w = got["w"] / max(1.0, np.linalg.norm(got["w"]))
        wr = ref["w"] / max(1.0, np.linalg.norm(ref["w"]))
        f = O.reduced_objective(X, y, w, got["beta"], C, q)
        fr = O.reduced_objective(X, y, wr, ref["beta"], C, q)
        assert abs(f - fr) <= 1e-6 * abs(fr), (tol, f, fr)
        assert np.linalg.norm(got["w"] - ref["w"]) <= 1e-4 * np.linalg.norm(ref["w"])
        k = O.kkt_of_solution(X, y, C, q, got)
        assert max(k["P"], k["D"]) <= 2 * tol, k
    # the same optimum as the exact SMW solves
    smw = dwd.solve(X, y, C, q, tol=1e-7, solver="smw", max_iter=20000)
    assert np.linalg.norm(got["w"] - smw["w"]) <= 1e-3 * np.linalg.norm(smw["w"])
    P.close()


@pytest.mark.parametrize("d,n,storage,pmax", [(400, 300, "f32", 50), (900, 150, "f64", 8),
                                              (600, 400, "f32", 2)])
def test_psqmr_trajectory_follows_oracle(dwd, d, n, storage, pmax):
    """PSQMR with T = 0 (warm started, to eps_k in Step 1a and 5 eps_k in the
    Step 1c re-solve): the first iterates, the step count of every solve and
    the iteration at which the proximal term takes over agree with the
    oracle.  psqmr_max = 50 never switches on these data; 8 switches inside
    a Step 1a solve (iteration 7 at d = 900), 2 inside the first Step 1c
    re-solve."""
    X, y = _data(d, n, seed=3 * d + n, storage=storage)
    e = synth.penalty_vector(n, seed=n + 3)
    C, q = 1.0, 1.0
    P = dwd.Problem(X, y, storage=storage, solver="iterative", ell=8)
    for k in (1, 2, 5, 12):
        o = O.solve(X, y, C, q, tol=1e-300, max_iter=k, solver="iterative", ell=8,
                    psqmr_max=pmax, weights=True, e=e)
        g = P.solve(C, q, tol=1e-300, max_iter=k, class_weights=1, e=e, psqmr_max=pmax)
        steps = P.inspect("psqmr_steps")
        info = g["info"]
        assert info["iters"] == k
        assert list(steps) == list(o["psqmr_steps"]), (k, list(steps), o["psqmr_steps"])
        assert info["psqmr_solves"] == len(o["psqmr_steps"])
        assert info["psqmr_steps"] == sum(o["psqmr_steps"])
        assert (info["psqmr_switch"] >= 0) == bool(o["used_T"]), k
        for key in ("alpha", "r", "xi"):
            assert np.allclose(g[key], o[key], rtol=1e-8, atol=1e-11), (k, key)
        for key in ("w", "u", "rho"):
            assert np.allclose(g[key], o[key], rtol=1e-8,
                               atol=1e-11 * max(1e-300, np.abs(o[key]).max())), (k, key)
        assert abs(g["beta"] - o["beta"]) <= 1e-8 * max(1.0, abs(o["beta"])), k
        assert info["n_double"] == o["n_double"], k
    P.close()


@pytest.mark.parametrize("d,n,q,C", [(400, 300, 1.0, 1.0), (800, 200, 2.0, 3.0)])
def test_psqmr_solves_match_oracle(dwd, d, n, q, C):
    """Whole solves with the paper's iterative method (PSQMR first, the
    proximal term after a solve of more than 50 steps): the same stopping
    point as the oracle, and the optimum of the exact SMW solve."""
    X, y = _data(d, n, seed=d + n, log_scale=0.5 if d != 800 else 1.0)
    P = dwd.Problem(X, y, storage="f32", solver="iterative")
    ref = O.solve(X, y, C, q, tol=1e-6, max_iter=20000, solver="iterative", psqmr_max=50)
    got = P.solve(C, q, tol=1e-6, max_iter=20000)
    tight = O.solve(X, y, C, q, tol=1e-9, max_iter=20000)
    P.close()
    info = got["info"]
    print("PSQMR solve d=%d n=%d: iters %d/%d, psqmr solves %d steps %d switch %d (oracle %s)" % (
        d, n, info["iters"], ref["iters"], info["psqmr_solves"], info["psqmr_steps"],
        info["psqmr_switch"], ref["used_T"]))
    assert ref["converged"] and info["converged"] == 1 and info["kkt_check"] < 1e-6, info
    assert abs(info["iters"] - ref["iters"]) <= max(3, 0.1 * ref["iters"])
    w = got["w"] / max(1.0, np.linalg.norm(got["w"]))
    f = O.reduced_objective(X, y, w, got["beta"], C, q)
    fr = O.reduced_objective(X, y, ref["w"] / max(1.0, np.linalg.norm(ref["w"])), ref["beta"], C, q)
    ft = O.reduced_objective(X, y, tight["w"] / max(1.0, np.linalg.norm(tight["w"])),
                             tight["beta"], C, q)
    assert abs(f - fr) <= 1e-6 * abs(fr), (f, fr)
    assert abs(f - ft) <= 1e-5 * abs(ft), (f, ft)
    k = O.kkt_of_solution(X, y, C, q, got)
    assert max(k["P"], k["D"]) <= 1e-6 * (1 + 1e-6), k


def test_iterative_beyond_both_limits(dwd):
    # d > 5120 and n > 65536: neither factor is built; AUTO picks this branch
    d, n = 6000, 70000
    X, y = synth.random_two_class(d, n, seed=91, mean=0.3, flip=0.05, dtype="f32")
    P = dwd.Problem(X, y, storage="f32", solver="auto")
    assert P.inspect("solver")[0] == 3
    got = P.solve(1.0, 1.0, tol=1e-4, max_iter=5000)
    P.close()
    info = got["info"]
    print("iterative d=6000 n=70000:", {k: info[k] for k in ("iters", "setup_ms", "solve_ms",
                                                          "kkt_check", "eta_gap")})
    assert info["converged"] == 1, info
    Xd = X.astype(np.float64)
    del X
    k = O.kkt_of_solution(Xd, y, 1.0, 1.0, got)
    assert max(k["P"], k["D"]) <= 1.5e-4, k


def test_iterative_rejections(dwd):
    X, y = _data(300, 100, seed=5)
    with pytest.raises(dwd.DwdError):
        dwd.Problem(X, y, storage="bf16", solver="iterative")
    with pytest.raises(dwd.DwdError):
        dwd.Problem(X, y, storage="f32", solver="iterative", ell=1)
    P = dwd.Problem(X, y, storage="f32", solver="iterative")
    with pytest.raises(dwd.DwdError):
        P.solve_batch([dict(C=1.0, q=1.0)])
    with pytest.raises(dwd.DwdError):
        P.solve(1.0, 1.0, representer=1)
    assert P.solve(1.0, 1.0, tol=1e-5)["info"]["converged"] == 1
    P.close()
    with pytest.raises(dwd.DwdError):
        dwd.serve([dict(X=X, y=y, t_arrival=0.0, params=dict(solver=3))])
    # CSR input: the iterative branch needs dense X
    req = synth.Request(0, 0.0, d=3000, n=140, q=1.0, C=1.0, layout="csr", storage="f32",
                        seed=42)
    ip, ix, val, yc = synth.request_csr_data(req, density=5e-3)
    with pytest.raises(dwd.DwdError):
        dwd.Problem(csr=(ip, ix, val, 3000), y=yc, storage="f32", solver="iterative")


@pytest.mark.parametrize("d,n", [(400, 300), (6000, 9000)])
def test_iterative_repeats_are_bit_identical(dwd, d, n):
    # The Z~ passes add their row-panel and sample shares in a fixed order:
    # two runs of the same solve give the same bits.
    X, y = _data(d, n, seed=7 * d + n)
    P = dwd.Problem(X, y, storage="f32", solver="iterative")
    for k in (3, 30):
        a = P.solve(1.5, 1.0, tol=1e-300, max_iter=k)
        b = P.solve(1.5, 1.0, tol=1e-300, max_iter=k)
        for key in ("w", "alpha", "r", "xi", "u", "rho"):
            assert np.array_equal(a[key], b[key]), (k, key)
    P.close()
