"""The allocation-free entry point dwd_suggest_C_noalloc against the
allocating dwd_suggest_C it mirrors: the same value, bit for bit, on two calls
in a row, the second on a smaller problem (the static work area keeps the
previous call's contents, which must not leak into the next)."""
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


def test_noalloc_suggest_C_matches_the_allocating_call(dwd):
    # larger problem first (odd pair count: one middle value), then a smaller
    # one (even count: two middle values), then the larger one again
    cases = [(3000, 1502, 0.3003, 91), (2000, 300, 0.5, 92), (3000, 1502, 0.3003, 91)]
    got = []
    for d, n, pf, seed in cases:
        X, y = synth.random_two_class(d, n, seed=seed, mean=0.5, pos_frac=pf, dtype="f32")
        P = dwd.Problem(X, y, storage="f32")
        for q in (1.0, 2.0, 0.5):
            a = P.suggest_C(q)
            b = P.suggest_C_noalloc(q)
            assert a == b, (d, n, q, a, b)
            got.append(b)
            # and the oracle's value (exact selection on both sides; the
            # distances differ only by rounding of the Gram matrix)
            c = O.suggest_C(X.astype(np.float64), y, q)
            assert abs(b - c) <= 1e-9 * c, (d, n, q, b, c)
        P.close()
    assert got[:3] == got[6:]


def test_noalloc_suggest_C_rejects_bad_arguments(dwd):
    X, y = synth.random_two_class(500, 40, seed=93, mean=0.5, dtype="f32")
    P = dwd.Problem(X, y, storage="f32")
    with pytest.raises(dwd.DwdError) as ei:
        P.suggest_C_noalloc(0.0)
    assert ei.value.status == -1
    P.close()
