"""Seeded synthetic inputs for the generalized-DWD solver and for its oracle.

This module is shared by the oracle tests and by the GPU path, so it holds no
arithmetic of the method itself: it only draws data matrices, labels and
problem parameters.  The paper's own benchmark (two-class UCI/LIBSVM sets,
Section 4) is not available, so these Gaussian two-class generators stand in
for it.  They follow the high-dimension, low-sample-size regime (d >> n) for
which the Sherman-Morrison-Woodbury branch of Section 3.3 is meant.

Layout convention: ``X`` is returned as a NumPy array of shape ``(n, d)``,
C-contiguous, so that row ``i`` is the sample ``x_i``.  Read as a d-by-n matrix
this is column-major with leading dimension d (each sample contiguous), which
is the layout the C ABI takes.  ``y`` is a float64 vector of +1/-1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Rows generated per chunk.  Fixed so that the stream of random numbers (and
# hence the data) does not depend on the problem size being generated.
_CHUNK_ROWS = 64


@dataclasses.dataclass(frozen=True)
class TwoClassSpec:
    """Recipe for one Gaussian two-class data set.

    x_i = diag(s) (mean * y_true_i * u + N(0, I_d)), with u a seeded random
    unit vector and s_j = 10**U(-log_scale, log_scale) (s = 1 if log_scale is
    0).  floor(pos_frac * n) samples have y_true = +1 (0.5: balanced classes).
    A fraction ``flip`` of the labels is then flipped (chosen without
    replacement), so the observed y differs from y_true.
    """

    d: int
    n: int
    seed: int
    mean: float
    flip: float = 0.0
    log_scale: float = 0.0
    dtype: str = "f64"  # storage type of record: "f64" or "f32"
    pos_frac: float = 0.5


def _draw_two_class(spec: TwoClassSpec):
    rng = np.random.default_rng(spec.seed)
    g = rng.standard_normal(spec.d)
    u = g / np.linalg.norm(g)
    n_pos = int(math.floor(spec.pos_frac * spec.n))
    y_true = np.concatenate([np.ones(n_pos), -np.ones(spec.n - n_pos)])
    y_true = y_true[rng.permutation(spec.n)]
    if spec.log_scale > 0:
        s = 10.0 ** rng.uniform(-spec.log_scale, spec.log_scale, spec.d)
    else:
        s = None
    n_flip = int(round(spec.flip * spec.n))
    flip_idx = rng.choice(spec.n, size=n_flip, replace=False) if n_flip else np.zeros(0, np.int64)
    out_dtype = np.float64 if spec.dtype == "f64" else np.float32
    X = np.empty((spec.n, spec.d), dtype=out_dtype)
    for r0 in range(0, spec.n, _CHUNK_ROWS):
        r1 = min(spec.n, r0 + _CHUNK_ROWS)
        block = rng.standard_normal((r1 - r0, spec.d))
        block += spec.mean * y_true[r0:r1, None] * u[None, :]
        if s is not None:
            block *= s[None, :]
        X[r0:r1] = block
    y = y_true.copy()
    y[flip_idx] = -y[flip_idx]
    return X, y, u


def two_class(spec: TwoClassSpec):
    """Return (X, y) for ``spec``; X has shape (n, d), y is +-1 float64."""
    X, y, _ = _draw_two_class(spec)
    return X, y


def two_class_with_direction(spec: TwoClassSpec):
    """Like :func:`two_class` but also return the class-mean direction u."""
    return _draw_two_class(spec)


# ---------------------------------------------------------------------------
# The five workloads.  Each names its data recipe and the (C, q, tol) of the
# problem; storage precision is a property of how the GPU stores Z, the data
# of record is X as generated.
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    data: TwoClassSpec
    C: float
    q: float
    tol: float
    storage: str  # "f64" | "f32" | "bf16"


SMALL_F64 = Workload(
    name="dwd_d200_n50_q1_C1_f64",
    data=TwoClassSpec(d=200, n=50, seed=1, mean=1.1, dtype="f64"),
    C=1.0, q=1.0, tol=1e-6, storage="f64")

HDLSS_F32 = Workload(
    name="dwd_d100000_n1000_q1_C10_f32",
    data=TwoClassSpec(d=100_000, n=1000, seed=2, mean=0.5, flip=0.1, dtype="f32"),
    C=10.0, q=1.0, tol=1e-5, storage="f32")

LARGE_BF16 = Workload(
    name="dwd_d1000000_n2000_q2_C1_bf16",
    data=TwoClassSpec(d=1_000_000, n=2000, seed=3, mean=0.5, flip=0.1,
                      log_scale=1.0, dtype="f32"),
    C=1.0, q=2.0, tol=1e-5, storage="bf16")

SWEEP_DATA = TwoClassSpec(d=200_000, n=1000, seed=4, mean=0.5, flip=0.1, dtype="f32")


def sweep_grid():
    """The 64 (C, q) pairs of the batched sweep: 16 C on a log grid in
    [1e-2, 1e2] times q in {0.5, 1, 2, 4}; problem j = a*4 + b."""
    out = []
    for a in range(16):
        C = 10.0 ** (-2.0 + 4.0 * a / 15.0)
        for q in (0.5, 1.0, 2.0, 4.0):
            out.append((C, q))
    return out


# ---------------------------------------------------------------------------
# Serving stream.
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Request:
    index: int
    t_arrival: float  # seconds from the start of the trace
    d: int
    n: int
    q: float
    C: float
    layout: str  # "dense" | "csr"
    storage: str  # "f32" | "bf16" (dense) ; "f32" (csr)
    seed: int  # seed of this request's data


def request_stream(count: int, rate: float, seed: int = 5) -> List[Request]:
    """Poisson arrivals at ``rate`` requests/s.  d is log-uniform in
    [1e3, 2e5], n uniform in {50..2000}, q in {1, 2}, C log-uniform in
    [1e-1, 1e1]; 20% of the requests are sparse (CSR at density 1e-3), the
    dense ones store Z in FP32 or BF16 with equal probability."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        d = int(round(10.0 ** rng.uniform(3.0, math.log10(2e5))))
        n = int(rng.integers(50, 2001))
        q = float(rng.choice([1.0, 2.0]))
        C = float(10.0 ** rng.uniform(-1.0, 1.0))
        sparse = rng.uniform() < 0.2
        storage = "f32" if sparse else ("f32" if rng.uniform() < 0.5 else "bf16")
        out.append(Request(i, t, d, n, q, C, "csr" if sparse else "dense", storage,
                           seed=int(1_000_000 + seed * 10_000 + i)))
    return out


def request_dense_data(req: Request):
    """Dense request data: the two-class generator with means +-0.5 u and
    10% label flips, in FP32."""
    return two_class(TwoClassSpec(d=req.d, n=req.n, seed=req.seed, mean=0.5,
                                  flip=0.1, dtype="f32"))


def request_dense_data_device(req: Request, torch, device):
    """The dense request recipe with the noise drawn on the device (for
    streams too large to draw on the host): u, the labels and the flips as
    in :func:`request_dense_data` from numpy with the request's seed, the
    N(0, I) noise from a torch generator seeded with it, in FP32.  The same
    distribution as :func:`request_dense_data`, other draws.  Returns
    (X, y): X a device tensor of shape (n, d), y a float64 numpy vector."""
    rng = np.random.default_rng(req.seed)
    g = rng.standard_normal(req.d)
    u = g / np.linalg.norm(g)
    n_pos = req.n // 2
    y_true = np.concatenate([np.ones(n_pos), -np.ones(req.n - n_pos)])[rng.permutation(req.n)]
    n_flip = int(round(0.1 * req.n))
    flip_idx = rng.choice(req.n, size=n_flip, replace=False)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(req.seed))
    X = torch.randn((req.n, req.d), generator=gen, device=device, dtype=torch.float32)
    X += (0.5 * torch.from_numpy(y_true.astype(np.float32)).to(device)[:, None]
          * torch.from_numpy(u.astype(np.float32)).to(device)[None, :])
    y = y_true.copy()
    y[flip_idx] = -y[flip_idx]
    return X, y


def request_csr_data(req: Request, density: float = 1e-3):
    """Sparse request data as CSR of X^T (one row per sample, like a LIBSVM
    file): each entry is nonzero with probability ``density``, nonzeros are
    N(0,1) in FP32, and a sample with no nonzero is drawn again.  Labels are
    balanced and randomly ordered.  Returns (indptr int64, indices int32,
    values float32, y)."""
    rng = np.random.default_rng(req.seed)
    indptr = [0]
    indices = []
    values = []
    for _ in range(req.n):
        while True:
            k = rng.binomial(req.d, density)
            if k > 0:
                break
        cols = np.sort(rng.choice(req.d, size=k, replace=False)).astype(np.int32)
        indices.append(cols)
        values.append(rng.standard_normal(k).astype(np.float32))
        indptr.append(indptr[-1] + k)
    n_pos = req.n // 2
    y = np.concatenate([np.ones(n_pos), -np.ones(req.n - n_pos)])[rng.permutation(req.n)]
    return (np.asarray(indptr, np.int64), np.concatenate(indices),
            np.concatenate(values), y)


def csr_to_dense(indptr, indices, values, d: int, dtype=np.float64):
    """Expand CSR of X^T into the (n, d) dense layout of this module."""
    n = len(indptr) - 1
    X = np.zeros((n, d), dtype=dtype)
    for i in range(n):
        X[i, indices[indptr[i]:indptr[i + 1]]] = values[indptr[i]:indptr[i + 1]]
    return X


# Unbalanced classes (about one positive in ten, Section 4.5 class weights):
# the high-dimension, low-sample-size shape of the main workload.
UNBALANCED_F32 = Workload(
    "unbalanced_f32", TwoClassSpec(d=100_000, n=1000, seed=6, mean=0.5, flip=0.05,
                                   pos_frac=0.1, dtype="f32"),
    C=10.0, q=1.0, tol=1e-5, storage="f32")


def penalty_vector(n: int, seed: int, low: float = 0.2):
    """Positive penalty weights e (eq-primal) drawn U(low, 1) and divided by
    their maximum, so that ||e||_inf = 1."""
    e = np.random.default_rng(seed).uniform(low, 1.0, n)
    return e / e.max()


def tiny_2d(seed: int = 11, n: int = 16):
    """Two-dimensional toy data for brute-force checks (d = 2)."""
    return two_class(TwoClassSpec(d=2, n=n, seed=seed, mean=1.0, flip=0.125, dtype="f64"))


def random_two_class(d: int, n: int, seed: int, mean: float = 0.8, flip: float = 0.1,
                     log_scale: float = 0.0, dtype: str = "f64", pos_frac: float = 0.5):
    """Convenience wrapper used by tests for ad-hoc shapes."""
    return two_class(TwoClassSpec(d=d, n=n, seed=seed, mean=mean, flip=flip,
                                  log_scale=log_scale, dtype=dtype, pos_frac=pos_frac))
