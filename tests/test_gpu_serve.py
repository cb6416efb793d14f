"""Sparse (CSR) data and the serving loop (dwd_serve) on the GPU."""
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


def _csr_request(d, n, seed, density):
    req = synth.Request(0, 0.0, d=d, n=n, q=1.0, C=1.0, layout="csr", storage="f32", seed=seed)
    return synth.request_csr_data(req, density=density)


def test_csr_setup_and_solve_match_oracle(dwd):
    ip, ix, val, y = _csr_request(4000, 150, 77, 5e-3)
    Xd = synth.csr_to_dense(ip, ix, val, 4000, np.float64)
    P = dwd.Problem(csr=(ip, ix, val, 4000), y=y, storage="f32")
    Zt, zs = O.scale_data(Xd, y)
    assert abs(P.inspect("zscale")[0] - zs) <= 1e-12 * zs
    G = Zt.T @ Zt
    assert np.max(np.abs(P.inspect("G") - G)) <= 1e-12 * np.max(np.abs(G))
    for C, q in ((1.0, 2.0), (0.3, 1.0)):
        ref = O.solve(Xd, y, C, q, tol=1e-9, max_iter=20000)
        got = P.solve(C, q, tol=1e-8, max_iter=20000)
        assert got["info"]["converged"] == 1
        f, fr = _obj(Xd, y, got["w"], got["beta"], C, q), _obj(Xd, y, ref["w"], ref["beta"], C, q)
        assert abs(f - fr) <= 1e-6 * abs(fr)
        assert np.linalg.norm(got["w"] - ref["w"]) <= 1e-4 * np.linalg.norm(ref["w"])
        e = O.kkt_of_solution(Xd, y, C, q, got)
        assert max(e["P"], e["D"]) <= 2e-8, e
    P.close()


def test_csr_matches_dense_storage(dwd):
    ip, ix, val, y = _csr_request(3000, 120, 78, 4e-3)
    Xd = synth.csr_to_dense(ip, ix, val, 3000, np.float32)
    Pc = dwd.Problem(csr=(ip, ix, val, 3000), y=y, storage="f32")
    Pd = dwd.Problem(Xd, y, storage="f32")
    rc, rd = Pc.solve(1.0, 1.0, tol=1e-6), Pd.solve(1.0, 1.0, tol=1e-6)
    assert abs(rc["info"]["iters"] - rd["info"]["iters"]) <= 2
    assert np.linalg.norm(rc["w"] - rd["w"]) <= 1e-6 * np.linalg.norm(rd["w"])
    Pc.close()
    Pd.close()


def test_csr_rejects_bad_structure(dwd):
    ip = np.array([0, 2, 3], np.int64)
    y = np.array([1.0, -1.0])
    with pytest.raises(dwd.DwdError):
        dwd.Problem(csr=(ip, np.array([1, 1, 0], np.int32), np.ones(3, np.float32), 5), y=y)
    with pytest.raises(dwd.DwdError):
        dwd.Problem(csr=(ip, np.array([0, 7, 0], np.int32), np.ones(3, np.float32), 5), y=y)


def _mixed_requests():
    reqs = []
    specs = [  # (d, n, q, C, kind, storage)
        (3000, 200, 1.0, 1.0, "dense", "f32"),
        (8000, 120, 2.0, 0.5, "dense", "bf16"),
        (5000, 300, 1.0, 3.0, "csr", "f32"),
        (1500, 400, 2.0, 1.0, "dense", "f32"),
        (12000, 90, 1.0, 0.2, "dense", "f32"),
        (2000, 64, 2.0, 2.0, "csr", "f32"),
    ]
    for j, (d, n, q, C, kind, storage) in enumerate(specs):
        seed = 500 + j
        if kind == "csr":
            ip, ix, val, y = _csr_request(d, n, seed, 5e-3)
            rq = dict(csr=(ip, ix, val, d), y=y)
        else:
            X, y = synth.random_two_class(d, n, seed=seed, mean=0.5, dtype="f32")
            rq = dict(X=X, y=y)
        rq["params"] = dict(C=C, q=q, tol=1e-5, storage=storage)
        reqs.append(rq)
    return reqs


def test_serve_result_is_the_same_alone_and_in_the_mix(dwd):
    reqs = _mixed_requests()
    for j, r in enumerate(reqs):  # staggered arrivals
        r["t_arrival"] = 0.002 * j
    mix = dwd.serve(reqs, iters_per_round=8)
    for j, r in enumerate(reqs):
        alone = dwd.serve([dict(r, t_arrival=0.0)], iters_per_round=8)[0]
        m = mix[j]
        assert m["status"] == 0 and alone["status"] == 0, (j, m["status"], alone["status"])
        assert m["info"]["iters"] == alone["info"]["iters"], j
        assert np.array_equal(m["w"], alone["w"]), j
        assert m["info"]["kkt_check"] < 1e-5, (j, m["info"])
    # some requests shared the device
    iv = [(m["t_admit"], m["t_done"]) for m in mix]
    assert any(a2 < d1 and a1 < d2 for j, (a1, d1) in enumerate(iv) for (a2, d2) in iv[j + 1:])


def test_serve_representer_mix_is_the_same_alone(dwd):
    """The representer step reads every coefficient of its problem in every
    block while each block updates its own rows; in a multi-problem launch a
    small problem's blocks can run far apart, so the step must not read a
    coefficient another block of the same launch already replaced.  A
    small-n problem among large-n ones must follow exactly its lone
    trajectory (and the plain representer solve)."""
    specs = [  # (d, n, q, C, storage)
        (20000, 60, 1.0, 0.25, "bf16"),
        (4000, 1800, 2.0, 1.0, "f32"),
        (3000, 2000, 1.0, 3.0, "f32"),
        (6000, 1500, 2.0, 0.5, "bf16"),
        (9000, 75, 1.0, 0.3, "f32"),
    ]
    reqs = []
    for j, (d, n, q, C, storage) in enumerate(specs):
        X, y = synth.random_two_class(d, n, seed=700 + j, mean=0.5, dtype="f32")
        reqs.append(dict(X=X, y=y, t_arrival=0.0,
                         params=dict(C=C, q=q, tol=1e-5, storage=storage, representer=1)))
    mix = dwd.serve(reqs, iters_per_round=8)
    for j, r in enumerate(reqs):
        alone = dwd.serve([r], iters_per_round=8)[0]
        m = mix[j]
        assert m["status"] == 0 and alone["status"] == 0, (j, m["info"], alone["info"])
        assert m["info"]["iters"] == alone["info"]["iters"], j
        assert np.array_equal(m["w"], alone["w"]), j
        p = r["params"]
        P = dwd.Problem(r["X"], r["y"], storage=p["storage"])
        single = P.solve(p["C"], p["q"], tol=p["tol"], want_state=False, representer=1)
        P.close()
        assert np.array_equal(single["w"], m["w"]), j


def test_auto_iteration_form_follows_the_byte_rule(dwd):
    """representer = 2 picks the representer iteration when one more read of
    the n x n G~ (8 n^2 bytes) costs less than the pass it replaces (Z in its
    storage type plus five FP64 d-vectors), and then runs exactly the chosen
    form, in dwd_solve and in dwd_serve."""
    cases = [(20000, 100, "f32"), (1500, 1400, "f32"), (3000, 700, "bf16")]
    reqs = []
    for j, (d, n, storage) in enumerate(cases):
        ld = (d + 1023) // 1024 * 1024
        es = {"f32": 4, "bf16": 2}[storage]
        want = 1 if 8 * n * n < ld * n * es + 40 * ld else 0
        X, y = synth.random_two_class(d, n, seed=900 + j, mean=0.5, dtype="f32")
        P = dwd.Problem(X, y, storage=storage)
        auto = P.solve(1.0, 1.0, tol=1e-5, want_state=False, representer=2)
        same = P.solve(1.0, 1.0, tol=1e-5, want_state=False, representer=want)
        P.close()
        assert auto["info"]["representer"] == want, (d, n, storage)
        assert auto["info"]["converged"] == 1
        assert np.array_equal(auto["w"], same["w"]), (d, n, storage)
        reqs.append(dict(X=X, y=y, t_arrival=0.0,
                         params=dict(C=1.0, q=1.0, tol=1e-5, storage=storage, representer=2),
                         want=want, w=same["w"]))
    assert {r["want"] for r in reqs} == {0, 1}
    out = dwd.serve(reqs, iters_per_round=8)
    for r, o in zip(reqs, out):
        assert o["status"] == 0 and o["info"]["representer"] == r["want"]
        assert np.array_equal(o["w"], r["w"])


def test_serve_matches_single_solves_and_oracle(dwd):
    reqs = _mixed_requests()[:3]
    res = dwd.serve(reqs)
    for r, out in zip(reqs, res):
        p = r["params"]
        if "csr" in r:
            ip, ix, val, d = r["csr"]
            X = synth.csr_to_dense(ip, ix, val, d, np.float64)
            single = dwd.Problem(csr=r["csr"], y=r["y"], storage=p["storage"]).solve(
                p["C"], p["q"], tol=p["tol"], want_state=False)
        else:
            X = r["X"].astype(np.float64)
            single = dwd.Problem(r["X"], r["y"], storage=p["storage"]).solve(
                p["C"], p["q"], tol=p["tol"], want_state=False)
        assert np.array_equal(single["w"], out["w"])
        ref = O.solve(X, r["y"], p["C"], p["q"], tol=1e-9, max_iter=20000)
        same = O.solve(X, r["y"], p["C"], p["q"], tol=p["tol"], max_iter=2000)
        fr = _obj(X, r["y"], ref["w"], ref["beta"], p["C"], p["q"])
        err = abs(_obj(X, r["y"], out["w"], out["beta"], p["C"], p["q"]) - fr) / abs(fr)
        err_o = abs(_obj(X, r["y"], same["w"], same["beta"], p["C"], p["q"]) - fr) / abs(fr)
        assert err <= max(5 * err_o, 1e-6), (err, err_o)


def test_serve_admission_by_memory_budget(dwd):
    reqs = _mixed_requests()[:4]
    fps = []
    for r in reqs:
        if "X" in r:
            fps.append(dwd.footprint(r["X"].shape[1], r["X"].shape[0], r["params"]["storage"]))
        else:
            ip, _, val, d = r["csr"]
            fps.append(dwd.footprint(d, len(ip) - 1, r["params"]["storage"], dwd.CSR, len(val)))
    budget = 1.05 * max(fps)
    res = dwd.serve(reqs, hbm_budget_bytes=budget)
    assert all(r["status"] == 0 for r in res)
    for j, r in enumerate(res):  # resident footprint never exceeds the budget
        t = r["t_admit"]
        live = sum(f for f, o in zip(fps, res) if o["t_admit"] <= t < o["t_done"])
        assert live <= budget, (j, live, budget)
    big = dict(reqs[0])
    res = dwd.serve([big], hbm_budget_bytes=0.5 * fps[0])
    assert res[0]["status"] == -5  # DWD_E_BUSY: can never fit


def test_serve_steps_direct_problems_beside_smw_problems(dwd):
    # solver = AUTO: the paper's choice picks the direct (d+1)^2 factor for
    # d <= 5000 (dense FP32) and the SMW form otherwise; each result equals the
    # single solve with the same choice, alone and in the mix.
    specs = [(300, 2000, 1.0, 1.0), (54, 5000, 2.0, 0.5), (8000, 150, 1.0, 1.0),
             (2000, 900, 1.0, 3.0)]
    reqs = []
    for j, (d, n, q, C) in enumerate(specs):
        X, y = synth.random_two_class(d, n, seed=700 + j, mean=0.5, dtype="f32")
        reqs.append(dict(X=X, y=y, t_arrival=0.001 * j,
                         params=dict(C=C, q=q, tol=1e-5, storage="f32", solver=2,
                                     class_weights=j % 2)))
    mix = dwd.serve(reqs, iters_per_round=8)
    for j, (r, m) in enumerate(zip(reqs, mix)):
        p = r["params"]
        P = dwd.Problem(r["X"], r["y"], storage="f32", solver="auto")
        want_direct = specs[j][0] <= 5000
        assert P.inspect("solver")[0] == (1 if want_direct else 0)
        single = P.solve(p["C"], p["q"], tol=p["tol"], class_weights=p["class_weights"],
                         want_state=False)
        P.close()
        assert m["status"] == 0 and m["info"]["converged"] == 1, (j, m)
        assert m["info"]["iters"] == single["info"]["iters"], j
        assert np.array_equal(m["w"], single["w"]), j
        assert m["info"]["kkt_check"] < 1e-5, (j, m["info"])
        # and against the oracle's branch of the same kind at the same tolerance
        Xd = r["X"].astype(np.float64)
        o = O.solve(Xd, r["y"], p["C"], p["q"], tol=p["tol"], max_iter=2000,
                    solver="direct" if want_direct else "smw",
                    weights=bool(p["class_weights"]))
        assert abs(m["info"]["iters"] - o["iters"]) <= max(3, 0.1 * o["iters"]), j
        assert np.linalg.norm(m["w"] - o["w"]) <= 1e-4 * np.linalg.norm(o["w"]), j


def test_serve_stream_sample_matches_oracle_and_plain_solves(dwd):
    """A random sample of 50 requests of the seeded serving stream (the
    requests among its first 600 with d n <= 2e6, so that the oracle solves
    take seconds; dense FP32, dense BF16 and CSR as drawn), served together
    with every request queued at t = 0.  Each result equals the plain
    single solve bit for bit and agrees with the FP64 oracle run to the same
    tolerance: FP32 and CSR requests stop where the oracle stops (same
    iteration count within 10%, w within 1e-4), BF16 requests (whose first
    phase iterates on the BF16 image) reach the same objective within
    1e-5."""
    stream = synth.request_stream(600, rate=1.0)
    small = [r for r in stream if r.d * r.n <= 2e6]
    pick = sorted(np.random.default_rng(12).choice(len(small), size=50, replace=False))
    sample = [small[i] for i in pick]
    reqs, dense = [], []
    for r in sample:
        if r.layout == "csr":
            ip, ix, val, y = synth.request_csr_data(r)
            reqs.append(dict(csr=(ip, ix, val, r.d), y=y))
            dense.append(synth.csr_to_dense(ip, ix, val, r.d, np.float64))
        else:
            X, y = synth.request_dense_data(r)
            reqs.append(dict(X=X, y=y))
            dense.append(X.astype(np.float64))
        reqs[-1]["params"] = dict(C=r.C, q=r.q, tol=1e-5, storage=r.storage)
    out = dwd.serve(reqs, iters_per_round=8)
    kinds = {}
    for j, (r, rq, o, Xd) in enumerate(zip(sample, reqs, out, dense)):
        kind = "csr" if r.layout == "csr" else r.storage
        kinds[kind] = kinds.get(kind, 0) + 1
        assert o["status"] == 0 and o["info"]["converged"] == 1, (j, o["info"])
        assert o["info"]["kkt_check"] < 1e-5, (j, o["info"])
        p = rq["params"]
        if "csr" in rq:
            P = dwd.Problem(csr=rq["csr"], y=rq["y"], storage=p["storage"])
        else:
            P = dwd.Problem(rq["X"], rq["y"], storage=p["storage"])
        single = P.solve(p["C"], p["q"], tol=p["tol"], want_state=False)
        P.close()
        assert np.array_equal(single["w"], o["w"]), j
        same = O.solve(Xd, rq["y"], p["C"], p["q"], tol=1e-5, max_iter=2000)
        assert same["converged"], j
        f = _obj(Xd, rq["y"], o["w"], o["beta"], p["C"], p["q"])
        fo = _obj(Xd, rq["y"], same["w"], same["beta"], p["C"], p["q"])
        if kind == "bf16":
            assert abs(f - fo) <= 1e-5 * abs(fo), (j, f, fo)
        else:
            it, ito = o["info"]["iters"], same["iters"]
            assert abs(it - ito) <= max(3, 0.1 * ito), (j, it, ito)
            assert np.linalg.norm(o["w"] - same["w"]) <= 1e-4 * np.linalg.norm(same["w"]), j
    print("served sample:", kinds)
    assert len(kinds) == 3  # every kind of request is in the sample
