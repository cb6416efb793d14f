"""FP64 CPU oracle for generalized DWD solved by the inexact sGS-ADMM.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
GPU solver is checked against.  Only the test suite, the package smoke check
and the benchmark's CPU-baseline leg may import it; the solver library never
does, and this module imports nothing from the solver.

It follows the paper (arXiv 2305.12019) step by step, in its notation:

* problem: generalized DWD primal (Section 2, eq-primal), with a general
  positive penalty vector e (default 1) and, optionally, the class weights
  of Section 4.5 on the loss terms;
* reformulation with u = w and D (w - u) = 0 (Section 3, eq-gen);
* Algorithm 1 (Steps 1a, 1b, 1c, 2, 3) with the inexactness sequence
  eps_k = c / (k + 1)^1.5;
* Step 1a/1c linear system eq-linsys with T = 0, solved by the
  Sherman-Morrison-Woodbury form of Section 3.3.2 (eq-Anew, eq-Ainv, eq-H)
  with a Cholesky factor of I_n + Z^T D^-1 Z and the rank-one formula for
  H^-1, or (d much smaller than n) by a Cholesky factor of the whole
  (d+1) x (d+1) matrix (Section 3.3.1).  Every product with Z is an
  explicit product, as the paper counts them (three per SMW solve);
* Step 1b prox of theta_q by the Newton map of Section 3.2 (eq-varphi),
  warm-started at r^k;
* data scaling Z~ = Z / sqrt(||X||_F) (Section 4.2, eq-gen-scale);
* relative KKT residuals, duality gap and stopping rule (Section 4.3);
* sigma adaptation (Section 4.4).

Readings where the paper is silent or ambiguous (all are plain parameters
that a caller may change):

* mu: the (1,1) block of the eq-linsys matrix is Z Z^T + mu I, i.e. the
  scaling matrix of the constraint D (w - u) = 0 is D = sqrt(mu) I.  The
  default mu = 1 makes the three ways the paper writes this block agree.
* initial point (r, xi, w, beta, u) = (1, 1, 0, 0, 0), (alpha, rho) = (0, 0).
* eps_k constant c = 1 / ||Z~||_F by default; c = 0 means "always redo
  Step 1c" (the exact sGS-ADMM).
* Newton safeguard: a step that leaves (0, inf) restarts from the lower end
  of a bracket of the root (from there Newton increases monotonically to the
  root, because the derivative of the prox objective is increasing and
  concave); at most 50 steps; a step below 4 ulp also stops.
* the dual objective takes alpha^(q/(q+1)) on max(alpha, 0).
* the sigma rule runs after the stopping test of every second iteration
  (``sigma_every = 2``; the paper gives no cadence, 1 = every iteration);
  no update when eta_P or eta_D is below 1e-300.
* eta_D also carries eta_D3 = ||Z~ alpha + D rho|| / (1 + C), the dual
  feasibility of the multipliers: the infimum of the Lagrangian of eq-gen
  over w is finite only when Z~ alpha + D rho = 0.  The paper's eta_D1 and
  eta_D2 only measure the box 0 <= alpha <= C, which the iterates almost
  always satisfy, so with them alone eta_D is (nearly) zero, the sigma rule
  can only raise sigma, and the iteration stalls on many (C, q) pairs.
  ``rho_residual=False`` restores the literal two-term eta_D.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import scipy.linalg as sla

TAU_DEFAULT = 1.618          # Step 3 step length
THETA_SIGMA = 5.0            # sigma rule threshold (Section 4.4)
MAX_NEWTON = 50


# ---------------------------------------------------------------------------
# Section 2: loss, dual constant, reduced primal objective.
# ---------------------------------------------------------------------------

def theta(t, q):
    """theta_q(t) = t^-q for t > 0, +inf otherwise (Section 2, eq-primal)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.full(t.shape, np.inf)
    pos = t > 0
    out[pos] = t[pos] ** (-q)
    return out


def kappa(q):
    """kappa = (q+1)/q * q^(1/(q+1)): inf_r theta_q(r) + a r = kappa a^(q/(q+1))
    for a >= 0 (Section 2, the Lagrangian infima before eq-dual)."""
    return (q + 1.0) / q * q ** (1.0 / (q + 1.0))


def class_weights(y, q):
    """Section 4.5 class weights for unbalanced classes: the loss term of
    sample i becomes tau_i^q theta_q(r_i) with
    tau_i = tau_- / max(tau_+, tau_-) if y_i = +1, tau_+ / max(tau_+, tau_-)
    if y_i = -1, tau_+- = (n_+- / K)^(1/(1+q)), K = n / log(n).
    Returns w_i = tau_i^q (the factor on theta_q)."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    K = n / math.log(n)
    tp = (np.sum(y > 0) / K) ** (1.0 / (1.0 + q))
    tm = (np.sum(y < 0) / K) ** (1.0 / (1.0 + q))
    m = max(tp, tm)
    tau = np.where(y > 0, tm / m, tp / m)
    return tau ** q


def loss_weights(y, q, weights):
    """Loss weights for :func:`solve`: ones (False), the class weights of
    Section 4.5 (True), or a given array."""
    y = np.asarray(y, dtype=np.float64)
    if weights is True:
        return class_weights(y, q)
    if weights is False or weights is None:
        return np.ones(y.size)
    return np.asarray(weights, np.float64)


def suggest_C(X, y, q):
    """Section 4.1 choice of the penalty: with dist the median of the
    Euclidean distances between the samples of the two classes,
    C = 10^(q+1) max{1, 10^(q-1) log(n) max{1000, d}^(1/3) / dist^(q+1)}."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, d = X.shape
    P, N = X[y > 0], X[y < 0]
    D = np.sqrt(np.maximum(np.sum(P * P, 1)[:, None] + np.sum(N * N, 1)[None, :]
                           - 2.0 * P @ N.T, 0.0))
    dist = float(np.median(D))
    return 10.0 ** (q + 1) * max(1.0, 10.0 ** (q - 1) * math.log(n) * max(1000.0, d) ** (1.0 / 3.0)
                                 / dist ** (q + 1))


def scale_data(X, y):
    """Z = X diag(y) (eq-r), Z_scale = sqrt(||X||_F), Z~ = Z / Z_scale
    (Section 4.2).  ``X`` has shape (n, d) with row i = x_i; the returned
    Z~ is the d-by-n matrix of the paper as an ndarray of shape (d, n)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    Z = (X * y[:, None]).T
    zscale = math.sqrt(np.linalg.norm(X))
    return Z / zscale, zscale


def margins(X, y, w, beta):
    """m = Z^T w + beta y for the unscaled problem (eq-r without xi)."""
    X = np.asarray(X, dtype=np.float64)
    return y * (X @ w + beta)


def reduced_loss(m, C, q, wt=None, e=None):
    """min over xi >= 0 (with r = m + xi > 0) of wt theta_q(r) + C e xi
    (wt = e = 1 by default; in general the threshold t* below is
    (q wt / (C e))^(1/(q+1))).

    The minimiser is xi = max(0, t* - m) with t* = (q / C)^(1/(q+1)), where
    the derivative -q r^(-q-1) + C of the one-dimensional problem vanishes.
    This is the primal eq-primal with (r, xi) eliminated for fixed (w, beta).
    """
    m = np.asarray(m, dtype=np.float64)
    wt = np.ones_like(m) if wt is None else np.broadcast_to(np.asarray(wt, np.float64), m.shape)
    ce = C * (np.ones_like(m) if e is None else np.broadcast_to(np.asarray(e, np.float64), m.shape))
    ts = (q * wt / ce) ** (1.0 / (q + 1.0))
    out = np.empty_like(m)
    hi = m >= ts
    out[hi] = wt[hi] * m[hi] ** (-q)
    out[~hi] = wt[~hi] * ts[~hi] ** (-q) + ce[~hi] * (ts[~hi] - m[~hi])
    return out


def reduced_objective(X, y, w, beta, C, q, wt=None, e=None):
    """Primal objective of eq-primal at (w, beta) with the optimal (r, xi)
    for that (w, beta); requires ||w|| <= 1 to be feasible."""
    return float(np.sum(reduced_loss(margins(X, y, w, beta), C, q, wt, e)))


def primal_objective(r, xi, C, q):  # e = 1, no class weights
    """Phi(r, xi) = sum theta_q(r_i) + C <e, xi> (eq-primal, e = 1)."""
    return float(np.sum(theta(r, q)) + C * np.sum(xi))


def dual_objective_unscaled(X, y, alpha, q, wt=None):
    """-Psi(alpha) = kappa sum wt_i^(1/(q+1)) alpha_i^(q/(q+1)) - ||Z alpha||
    (eq-dual; wt = 1 without class weights: inf_r wt theta_q(r) + a r =
    kappa wt^(1/(q+1)) a^(q/(q+1)))."""
    Zalpha = np.asarray(X, dtype=np.float64).T @ (y * alpha)
    a = np.maximum(alpha, 0.0)
    wd = 1.0 if wt is None else np.asarray(wt, np.float64) ** (1.0 / (q + 1.0))
    return float(kappa(q) * np.sum(wd * a ** (q / (q + 1.0))) - np.linalg.norm(Zalpha))


def training_error(X, y, w, beta):
    """|{i : y_i sgn(beta + x_i^T w) <= 0}| / n (Section 4.5)."""
    return float(np.mean(y * np.sign(beta + np.asarray(X, np.float64) @ w) <= 0))


# ---------------------------------------------------------------------------
# Section 3.2: prox of theta_q by Newton (eq-varphi), and the q = 1 cubic.
# ---------------------------------------------------------------------------

def prox_grad(s, a, sigma, q):
    """phi'(s) for phi(s) = s^-q + sigma/2 (s - a)^2 (eq-varphi)."""
    return -q * s ** (-q - 1.0) + sigma * (s - a)


def prox_bracket(a, sigma, q):
    """Interval [lo, hi] that holds the minimiser of eq-varphi.

    With s0 = (q/sigma)^(1/(q+2)) (the root for a = 0): for a >= 0 the root
    lies in [max(a, s0), a + s0]; for a < 0 it lies in
    [(q / (sigma (s0 + |a|)))^(1/(q+1)), min(s0, (q / (sigma |a|))^(1/(q+1)))].
    Both follow from the optimality condition s - a = q sigma^-1 / s^(q+1)
    and the monotonicity of its two sides.
    """
    a = np.asarray(a, dtype=np.float64)
    sg = np.broadcast_to(np.asarray(sigma, np.float64), a.shape)  # per element allowed
    s0 = (q / sg) ** (1.0 / (q + 2.0))
    lo = np.empty_like(a)
    hi = np.empty_like(a)
    pos = a >= 0
    lo[pos] = np.maximum(a[pos], s0[pos])
    hi[pos] = a[pos] + s0[pos]
    na = -a[~pos]
    sn = sg[~pos]
    lo[~pos] = (q / (sn * (s0[~pos] + na))) ** (1.0 / (q + 1.0))
    hi[~pos] = np.minimum(s0[~pos], (q / (sn * na)) ** (1.0 / (q + 1.0)))
    return lo, hi


def prox_newton(a, sigma, q, s_init, tol, max_steps=MAX_NEWTON):
    """Newton's method of Section 3.2 for argmin_{s>0} s^-q + sigma/2 (s-a)^2,
    element by element, warm-started at ``s_init``.

    Iterates s <- s (q(q+2)/sigma + a s^(q+1)) / (q(q+1)/sigma + s^(q+2))
    until |phi'(s)| <= tol (the Step 1b accuracy test).  Safeguard: a
    non-positive or non-finite start or iterate is replaced by the lower end
    of :func:`prox_bracket`; a relative step below 4 ulp also ends the
    iteration.  Returns (s, steps) with steps the Newton steps per element.
    """
    a = np.asarray(a, dtype=np.float64)
    s = np.array(s_init, dtype=np.float64, copy=True)
    sg = np.broadcast_to(np.asarray(sigma, np.float64), a.shape)  # per element allowed
    tl = np.broadcast_to(np.asarray(tol, np.float64), a.shape)
    lo, _ = prox_bracket(a, sg, q)
    bad = ~(np.isfinite(s) & (s > 0))
    s[bad] = lo[bad]
    steps = np.zeros(a.shape, dtype=np.int64)
    done = np.abs(prox_grad(s, a, sg, q)) <= tl
    c1 = q * (q + 2.0) / sg
    c2 = q * (q + 1.0) / sg
    for _ in range(max_steps):
        act = ~done
        if not act.any():
            break
        sa = s[act]
        aa = a[act]
        s_new = sa * (c1[act] + aa * sa ** (q + 1.0)) / (c2[act] + sa ** (q + 2.0))
        out = ~(np.isfinite(s_new) & (s_new > 0))
        s_new[out] = lo[act][out]
        tiny = np.abs(s_new - sa) <= 4.0 * np.finfo(np.float64).eps * sa
        s[act] = s_new
        steps[act] += 1
        g_new = np.abs(prox_grad(s_new, aa, sg[act], q)) <= tl[act]
        done[act] = g_new | tiny
    return s, steps


def prox_weighted(a, sigma, q, wt, s_init, tol):
    """argmin_{s>0} wt s^-q + sigma/2 (s-a)^2 with the accuracy test
    |phi_wt'(s)| <= tol: dividing by wt gives the unweighted prox at
    sigma / wt with the test |phi'(s)| <= tol / wt."""
    wt = np.asarray(wt, np.float64)
    return prox_newton(a, sigma / wt, q, s_init, tol / wt)


def prox_cubic_q1(a, sigma):
    """Closed form of the q = 1 prox: the positive root of
    s^3 - a s^2 - 1/sigma = 0 (the optimality condition of eq-varphi times
    s^2).  For a >= 0 Cardano's formula has one real root and every term is
    non-negative.  For a < 0 the substitution s = 1/t gives
    t^3 + sigma a t - sigma = 0, whose positive root is the dominant one and
    comes from Cardano (one real root) or the trigonometric form (three)."""
    a = np.asarray(a, dtype=np.float64)
    out = np.empty_like(a)
    pos = a >= 0
    if pos.any():
        ap = a[pos]
        h = ap ** 3 / 27.0 + 0.5 / sigma            # -q'/2 of the depressed cubic
        disc = ap ** 3 / (27.0 * sigma) + 0.25 / sigma ** 2
        A = h + np.sqrt(disc)
        B = (ap ** 6 / 729.0) / A                    # h - sqrt(disc) without cancellation
        out[pos] = np.cbrt(A) + np.cbrt(B) + ap / 3.0
    if (~pos).any():
        an = a[~pos]
        p = sigma * an                                # < 0
        half = 0.5 * sigma                            # -q'/2 with q' = -sigma
        disc = half ** 2 + (p / 3.0) ** 3
        t = np.empty_like(an)
        one = disc >= 0
        if one.any():
            sd = np.sqrt(disc[one])
            A = half + sd
            B = (-(p[one] / 3.0) ** 3) / A
            t[one] = np.cbrt(A) + np.cbrt(B)
        three = ~one
        if three.any():
            pm = p[three]
            m = 2.0 * np.sqrt(-pm / 3.0)
            arg = (3.0 * (-sigma) / (2.0 * pm)) * np.sqrt(-3.0 / pm)
            arg = np.clip(arg, -1.0, 1.0)
            t[three] = m * np.cos(np.arccos(arg) / 3.0)
        out[~pos] = 1.0 / t
    return out


# ---------------------------------------------------------------------------
# Section 3.3.2: the Sherman-Morrison-Woodbury solve of eq-linsys (T = 0).
# ---------------------------------------------------------------------------

class SMWFactor:
    """Precomputation for eq-Ainv: the Cholesky factor of the first diagonal
    block of J, I_n + Z~^T D^-1 Z~ with D = mu I in the (1,1) block, and
    J^-1 ybar with ybar = [y/||y||; 1] (done once, Section 3.3.2)."""

    def __init__(self, Zt, y, mu=1.0):
        self.Zt = Zt
        self.y = np.asarray(y, dtype=np.float64)
        self.mu = float(mu)
        n = Zt.shape[1]
        self.ny = float(np.linalg.norm(self.y))
        Mmat = np.eye(n) + (Zt.T @ Zt) / self.mu
        self.cho = sla.cho_factor(Mmat, lower=True)
        # J = diag(M, -1), ybar = [y/||y||; 1]
        self.Jy_n = sla.cho_solve(self.cho, self.y / self.ny)
        self.Jy_l = -1.0
        self.denom = 1.0 + (self.y / self.ny) @ self.Jy_n + 1.0 * self.Jy_l

    def H_inv_apply(self, v_n, v_l):
        """H^-1 v = J^-1 v - (J^-1 ybar)(J^-1 ybar)^T v / (1 + ybar^T J^-1 ybar)."""
        Jv_n = sla.cho_solve(self.cho, v_n)
        Jv_l = -v_l
        coef = (self.Jy_n @ v_n + self.Jy_l * v_l) / self.denom
        return Jv_n - coef * self.Jy_n, Jv_l - coef * self.Jy_l

    def solve(self, hw, hb):
        """[w; beta] = A^-1 [hw; hb] via eq-Ainv:
        A^-1 = Dhat^-1 - Dhat^-1 U H^-1 U^T Dhat^-1, Dhat = diag(mu I, ||y||^2),
        U = [[Z~, 0], [y^T, ||y||]]."""
        n = self.y.shape[0]
        xw = hw / self.mu
        xb = hb / (self.ny ** 2)
        # U^T x
        v_n = self.Zt.T @ xw + self.y * xb
        v_l = self.ny * xb
        z_n, z_l = self.H_inv_apply(v_n, v_l)
        # x - Dhat^-1 U z
        w = xw - (self.Zt @ z_n) / self.mu
        beta = xb - (self.y @ z_n + self.ny * z_l) / (self.ny ** 2)
        del n
        return w, float(beta)


class DirectFactor:
    """Section 3.3.1 (d much smaller than n): T = 0 and a Cholesky factor of
    the whole eq-linsys matrix
        A = [[Z~ Z~^T + mu I, Z~ y], [(Z~ y)^T, y^T y]]   ((d+1) x (d+1)),
    formed once; each solve is two triangular solves."""

    def __init__(self, Zt, y, mu=1.0):
        y = np.asarray(y, dtype=np.float64)
        d = Zt.shape[0]
        Zy = Zt @ y
        A = np.empty((d + 1, d + 1))
        A[:d, :d] = Zt @ Zt.T + float(mu) * np.eye(d)
        A[:d, d] = Zy
        A[d, :d] = Zy
        A[d, d] = y @ y
        self.cho = sla.cho_factor(A, lower=True)

    def solve(self, hw, hb):
        x = sla.cho_solve(self.cho, np.concatenate([hw, [hb]]))
        return x[:-1], float(x[-1])


def psqmr(apply_A, b, x0, apply_Minv, tol, max_steps):
    """Preconditioned symmetric QMR (Freund and Nachtigal) for a symmetric
    A and a symmetric positive definite preconditioner M: the Lanczos
    recurrences of the preconditioned CG direction q_j, with the iterate
    formed by the quasi-minimal-residual smoothing (theta_j, c_j, tau_j) of
    the unpreconditioned residual norms.  Stops when the true residual
    ||b - A x|| is at most ``tol``.  Returns (x, steps, converged)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_A(x)
    if np.linalg.norm(r) <= tol:
        return x, 0, True
    tau = np.linalg.norm(r)
    q = apply_Minv(r)
    rho = float(r @ q)
    theta = 0.0
    dvec = np.zeros_like(x)
    for j in range(1, max_steps + 1):
        t = apply_A(q)
        sig = float(q @ t)
        if sig == 0.0 or rho == 0.0:
            break
        alpha = rho / sig
        r = r - alpha * t
        theta_prev = theta
        theta = np.linalg.norm(r) / tau
        c2 = 1.0 / (1.0 + theta * theta)
        tau = tau * theta * math.sqrt(c2)
        dvec = c2 * theta_prev * theta_prev * dvec + c2 * alpha * q
        x = x + dvec
        if np.linalg.norm(b - apply_A(x)) <= tol:
            return x, j, True
        u = apply_Minv(r)
        rho_new = float(r @ u)
        q = u + (rho_new / rho) * q
        rho = rho_new
    return x, max_steps, np.linalg.norm(b - apply_A(x)) <= tol


def lanczos_start(dim):
    """Deterministic Lanczos start vector: entry i is the fractional part of
    (i + 1) * 0.6180339887498949 (golden-ratio sequence) minus 0.5,
    normalised."""
    i = np.arange(1, dim + 1, dtype=np.float64)
    v = np.mod(i * 0.6180339887498949, 1.0) - 0.5
    return v / np.linalg.norm(v)


def top_eigenpairs(apply_S, dim, ell, steps=None, v0=None):
    """The ``ell`` largest eigenpairs of a symmetric positive semidefinite
    operator by the Lanczos method with full reorthogonalisation (Section
    3.3.3 asks for them for eq-T): ``steps`` Lanczos vectors (default
    min(dim, 64)) from ``v0`` (default :func:`lanczos_start`), Ritz pairs
    from the tridiagonal matrix."""
    m = min(dim, steps if steps else 64)
    V = np.zeros((dim, m))
    a = np.zeros(m)
    b = np.zeros(m)
    v = lanczos_start(dim) if v0 is None else np.asarray(v0, np.float64) / np.linalg.norm(v0)
    k = m
    for j in range(m):
        V[:, j] = v
        w = apply_S(v)
        a[j] = v @ w
        w = w - V[:, :j + 1] @ (V[:, :j + 1].T @ w)
        w = w - V[:, :j + 1] @ (V[:, :j + 1].T @ w)
        if j + 1 < m:
            b[j] = np.linalg.norm(w)
            if b[j] <= 1e-14 * max(1.0, abs(a[j])):
                k = j + 1
                break
            v = w / b[j]
    Tm = np.diag(a[:k]) + np.diag(b[:k - 1], 1) + np.diag(b[:k - 1], -1)
    lam, S = np.linalg.eigh(Tm)
    order = np.argsort(lam)[::-1][:ell]
    return lam[order], V[:, :k] @ S[:, order]


class IterativeFactor:
    """Section 3.3.3 (n and d both large).  Step 1a and 1c first solve
    eq-linsys with T = 0 by PSQMR to the accuracy eq-linsys-tol (warm
    started at the current [w; beta]); once a solve needs more than
    ``psqmr_max`` steps, the proximal term T of eq-T is added for the rest
    of the solve, built from the ``ell`` largest eigenpairs of Z~ Z~^T:
        T = lam_ell I + sum_{i<ell} (lam_i - lam_ell) v_i v_i^T - Z~ Z~^T,
    so that Z~ Z~^T + mu I + T has the closed-form inverse
        (mu + lam_ell)^-1 I + sum_{i<ell} ((mu + lam_i)^-1 - (mu + lam_ell)^-1) v_i v_i^T
    and the system is solved through the Schur complement on beta (eq-schur).
    The PSQMR preconditioner is that T-modified matrix (its inverse is the
    closed form above with the Schur complement)."""

    def __init__(self, Zt, y, mu=1.0, ell=10, psqmr_max=50):
        self.Zt = Zt
        self.y = np.asarray(y, dtype=np.float64)
        self.mu = float(mu)
        d = Zt.shape[0]
        self.ell = min(ell, d)
        self.psqmr_max = psqmr_max
        lam, V = top_eigenpairs(lambda v: Zt @ (Zt.T @ v), d, self.ell)
        self.lam, self.V = lam, V
        self.Zy = Zt @ self.y
        self.yy = float(self.y @ self.y)
        self.g = self.Mw_inv(self.Zy)
        self.schur = self.yy - float(self.Zy @ self.g)
        self.use_T = psqmr_max <= 0
        self.steps = []

    def Mw_inv(self, x):
        """(Z~ Z~^T + mu I + T)^-1 x in closed form."""
        lam_l = self.lam[-1]
        out = x / (self.mu + lam_l)
        Vh = self.V[:, :-1]
        coef = 1.0 / (self.mu + self.lam[:-1]) - 1.0 / (self.mu + lam_l)
        return out + Vh @ (coef * (Vh.T @ x))

    def T_apply(self, w):
        lam_l = self.lam[-1]
        Vh = self.V[:, :-1]
        return (lam_l * w + Vh @ ((self.lam[:-1] - lam_l) * (Vh.T @ w))
                - self.Zt @ (self.Zt.T @ w))

    def solve_T(self, hw, hb):
        """[w; beta] of the T-modified system by eq-schur."""
        beta = (hb - float(self.g @ hw)) / self.schur
        return self.Mw_inv(hw) - beta * self.g, float(beta)

    def _A(self, x):
        top, bot = linsys_matrix_apply(self.Zt, self.y, self.mu, x[:-1], x[-1])
        return np.concatenate([top, [bot]])

    def _Minv(self, x):
        w, b = self.solve_T(x[:-1], x[-1])
        return np.concatenate([w, [b]])

    def solve_psqmr(self, hw, hb, w0, b0, tol):
        """T = 0: PSQMR from [w0; b0]; returns (w, beta, converged within
        psqmr_max steps)."""
        x, steps, ok = psqmr(self._A, np.concatenate([hw, [hb]]), np.concatenate([w0, [b0]]),
                             self._Minv, tol, self.psqmr_max)
        self.steps.append(steps)
        return x[:-1], float(x[-1]), ok


def select_solver(d, n):
    """The solver choice printed with the paper's pseudo-code: the SMW form
    when d > 5000, n < 0.2 d and n <= 2500; the iterative solver (PSQMR,
    Section 3.3.3) for the other cases with d > 5000; the direct Cholesky
    factor (Section 3.3.1) when d <= 5000."""
    if d > 5000 and n < 0.2 * d and n <= 2500:
        return "smw"
    if d > 5000:
        return "iterative"
    return "direct"


def linsys_matrix_apply(Zt, y, mu, w, beta):
    """A [w; beta] for the eq-linsys matrix with T = 0:
    A = [[Z~ Z~^T + mu I, Z~ y], [(Z~ y)^T, y^T y]]."""
    Zty = Zt @ y
    top = Zt @ (Zt.T @ w) + mu * w + Zty * beta
    bot = Zty @ w + (y @ y) * beta
    return top, float(bot)


def linsys_rhs(Zt, y, mu, sigma, r, xi, u, alpha, rho):
    """Right-hand side hbar of eq-linsys (T = 0, D = sqrt(mu) I):
    [-Z~(xi - r - alpha/sigma) + mu u + sqrt(mu) rho / sigma; -y^T(xi - r - alpha/sigma)]."""
    t = xi - r - alpha / sigma
    hw = -(Zt @ t) + mu * u + math.sqrt(mu) * rho / sigma
    hb = -float(y @ t)
    return hw, hb


# ---------------------------------------------------------------------------
# Section 4.3: KKT residuals, gap, stopping rule; Section 4.4: sigma rule.
# ---------------------------------------------------------------------------

def kkt_residuals(Zt, zscale, y, C, q, mu, r, w, beta, xi, u, alpha, rho=None,
                  Ztw=None, rho_residual=True, wt=None, e=None):
    """Relative residuals of Section 4.3 on the scaled problem eq-gen-scale.
    eta_C3 uses the squared norm as printed.  With ``rho`` given and
    ``rho_residual`` set, eta_D3 = ||Z~ alpha + D rho|| / (1 + C) joins
    eta_D.  Returns a dict with every eta, the maxima eta_P, eta_D, eta_C,
    the objectives and eta_gap.  ``wt``: loss weights (theta_q term of
    sample i times wt_i), ``e``: penalty vector; both default to 1."""
    if Ztw is None:
        Ztw = Zt.T @ w
    den = 1.0 + C
    ce = C * (np.ones(len(r)) if e is None else np.asarray(e, np.float64))
    eta = {}
    eta["P1"] = np.linalg.norm(Ztw + beta * y + xi - r) / den
    eta["P2"] = math.sqrt(mu) * np.linalg.norm(w - u) / den
    eta["P3"] = max(np.linalg.norm(w) - zscale, 0.0) / den
    eta["D1"] = np.linalg.norm(np.minimum(0.0, alpha)) / den
    eta["D2"] = np.linalg.norm(np.maximum(0.0, alpha - ce)) / den
    eta["C1"] = abs(float(y @ alpha)) / den
    eta["C2"] = abs(float(xi @ (ce - alpha))) / den
    wt = np.ones_like(r) if wt is None else np.asarray(wt, np.float64)
    s = q * wt / r ** (q + 1.0)
    eta["C3"] = float(np.sum((alpha - s) ** 2)) / den
    Zalpha = Zt @ alpha
    if rho is not None:
        eta["D3"] = np.linalg.norm(Zalpha + math.sqrt(mu) * rho) / den
    primobj = float(np.sum(wt * r ** (-q)) + np.sum(ce * xi))
    dualobj = float(kappa(q) * np.sum(wt ** (1.0 / (q + 1.0))
                                      * np.maximum(alpha, 0.0) ** (q / (q + 1.0)))
                    - zscale * np.linalg.norm(Zalpha))
    eta["primobj"] = primobj
    eta["dualobj"] = dualobj
    eta["gap"] = abs(primobj - dualobj) / (1.0 + abs(primobj) + abs(dualobj))
    eta["P"] = max(eta["P1"], eta["P2"], eta["P3"])
    eta["D"] = max(eta["D1"], eta["D2"], eta["D3"] if (rho_residual and "D3" in eta) else 0.0)
    eta["C"] = max(eta["C1"], eta["C2"], eta["C3"])
    return eta


def stop_test(e, tol):
    """max{eta_P, eta_D} < tol, min{eta_C, eta_gap} < sqrt(tol) and
    max{eta_C, eta_gap} < 0.05 (Section 4.3)."""
    return (max(e["P"], e["D"]) < tol and min(e["C"], e["gap"]) < math.sqrt(tol)
            and max(e["C"], e["gap"]) < 0.05)


def sigma_update(sigma, eta_p, eta_d):
    """Section 4.4: chi = eta_P/eta_D; sigma *= zeta if chi > 5, sigma /= zeta
    if 1/chi > 5; zeta = 2.2 if max(chi, 1/chi) > 500, 1.65 if > 50, else 1.1."""
    if eta_p < 1e-300 or eta_d < 1e-300:
        return sigma
    chi = eta_p / eta_d
    m = max(chi, 1.0 / chi)
    zeta = 2.2 if m > 500.0 else (1.65 if m > 50.0 else 1.1)
    if chi > THETA_SIGMA:
        return sigma * zeta
    if 1.0 / chi > THETA_SIGMA:
        return sigma / zeta
    return sigma


def step2(w, beta, r, alpha, rho, Ztw, y, C, sigma, mu, radius, e=1.0):
    """Step 2 of Algorithm 1: u = projection of g = w - sigma^-1 D^-1 rho onto
    the ball of radius ``radius``; xi = projection onto R^n_+ of
    r - Z~^T w - y beta + sigma^-1 alpha - sigma^-1 C e."""
    g = w - rho / (sigma * math.sqrt(mu))
    ng = np.linalg.norm(g)
    u = g if ng <= radius else g * (radius / ng)
    xi = np.maximum(0.0, r - Ztw - y * beta + (alpha - C * e) / sigma)
    return u, xi


def step3(alpha, rho, Ztw, y, beta, xi, r, w, u, sigma, mu, tau):
    """Step 3 of Algorithm 1: alpha -= tau sigma (Z~^T w + y beta + xi - r),
    rho -= tau sigma D (w - u)."""
    alpha = alpha - tau * sigma * (Ztw + y * beta + xi - r)
    rho = rho - tau * sigma * math.sqrt(mu) * (w - u)
    return alpha, rho


def default_sigma0(C, q, n):
    """sigma_0 = min{10 C, n}^q (Section 4.4)."""
    return min(10.0 * C, float(n)) ** q


# ---------------------------------------------------------------------------
# Algorithm 1.
# ---------------------------------------------------------------------------

def solve(X, y, C, q, tol=1e-5, max_iter=2000, mu=1.0, tau=TAU_DEFAULT,
          sigma0: Optional[float] = None, eps_c: Optional[float] = None,
          record: bool = False, start: Optional[Dict] = None,
          scale: bool = True, rho_residual: bool = True, sigma_every: int = 2,
          weights=False, e=None, solver: str = "smw", ell: int = 10,
          psqmr_max: int = 50) -> Dict:
    """Run Algorithm 1 on eq-gen-scale and return the unscaled solution.

    ``X`` has shape (n, d) (row i = sample x_i), ``y`` is +-1.  Returns a dict
    with w, u (unscaled), beta, r, xi, alpha, the scaled w~/u~/rho, the
    iteration count ``iters`` (number of completed iterations), ``n_double``
    (iterations in which Step 1c solved again), ``newton_max``, the final
    residuals ``eta`` and ``converged``.  ``start`` may hold a previous
    result's scaled state to resume from.  ``scale=False`` skips the data
    scaling of Section 4.2 (Z_scale = 1), for the check that scaling does
    not change the solution.  ``sigma_every``: the sigma rule of Section 4.4
    is applied after iterations whose count is a multiple of it (the paper
    gives no cadence; the default reading is every second iteration, 1 =
    every iteration).  ``weights``: True for the class weights of
    Section 4.5 (:func:`class_weights`) on the loss terms, or an array of n
    positive loss weights; ``e``: the positive penalty vector of eq-primal
    (n values; default 1).  ``solver``: "smw" (Section 3.3.2) or "direct"
    (Section 3.3.1) for the eq-linsys solves (both give the same iterates in
    exact arithmetic), or "iterative" (Section 3.3.3: PSQMR to the accuracy
    eq-linsys-tol, and the proximal T of eq-T from the ``ell`` largest
    eigenpairs once a solve needs more than ``psqmr_max`` steps; 0 = T from
    the start).
    """
    y = np.asarray(y, dtype=np.float64)
    if scale:
        Zt, zscale = scale_data(X, y)
    else:
        Zt, zscale = (np.asarray(X, np.float64) * y[:, None]).T.copy(), 1.0
    d, n = Zt.shape
    if solver == "smw":
        F = SMWFactor(Zt, y, mu)
    elif solver == "direct":
        F = DirectFactor(Zt, y, mu)
    elif solver == "iterative":
        F = IterativeFactor(Zt, y, mu, ell=ell, psqmr_max=psqmr_max)
    else:
        raise ValueError(f"unknown solver {solver}")
    it_mode = solver == "iterative"
    R = zscale
    wt = loss_weights(y, q, weights)
    ev = np.ones(n) if e is None else np.asarray(e, np.float64)
    if start is None:
        r = np.ones(n)
        xi = np.ones(n)
        w = np.zeros(d)
        beta = 0.0
        u = np.zeros(d)
        alpha = np.zeros(n)
        rho = np.zeros(d)
        sigma = default_sigma0(C, q, n) if sigma0 is None or sigma0 <= 0 else float(sigma0)
        k0 = 0
    else:
        r, xi, w, beta, u, alpha, rho = (start["r"].copy(), start["xi"].copy(),
                                         start["w_scaled"].copy(), start["beta"],
                                         start["u_scaled"].copy(), start["alpha"].copy(),
                                         start["rho"].copy())
        sigma = start["sigma"]
        k0 = start["iters"]
    c_eps = (1.0 / np.linalg.norm(Zt)) if (eps_c is None or eps_c < 0) else float(eps_c)
    n_double = 0
    newton_max = 0
    hist = []
    e = None
    converged = False
    it = k0
    for k in range(k0, k0 + max_iter):
        eps_k = c_eps / (k + 1.0) ** 1.5
        # Step 1a
        hw, hb = linsys_rhs(Zt, y, mu, sigma, r, xi, u, alpha, rho)
        Tw = None
        if not it_mode:
            wbar, bbar = F.solve(hw, hb)
        else:
            if not F.use_T:
                wbar, bbar, ok = F.solve_psqmr(hw, hb, w, beta, eps_k)
                if not ok:
                    F.use_T = True
            if F.use_T:
                Tw = F.T_apply(w)          # the proximal term adds T w^k
                wbar, bbar = F.solve_T(hw + Tw, hb)
        # Step 1b
        c = Zt.T @ wbar + y * bbar + xi - alpha / sigma
        r_new, steps = prox_weighted(c, sigma, q, wt, r, eps_k / math.sqrt(n))
        newton_max = max(newton_max, int(steps.max()))
        # Step 1c
        hw1, hb1 = linsys_rhs(Zt, y, mu, sigma, r_new, xi, u, alpha, rho)
        Aw, Ab = linsys_matrix_apply(Zt, y, mu, wbar, bbar)
        if Tw is not None:
            # with T: A_T [w; beta] = A [w; beta] + [T w; 0], rhs + [T w^k; 0]
            Aw = Aw + F.T_apply(wbar) - Tw
        res = math.sqrt(float(np.sum((hw1 - Aw) ** 2)) + (hb1 - Ab) ** 2)
        if res > 5.0 * eps_k:
            if not it_mode:
                w, beta = F.solve(hw1, hb1)
            elif Tw is not None:
                w, beta = F.solve_T(hw1 + Tw, hb1)
            else:
                w1, b1, ok = F.solve_psqmr(hw1, hb1, wbar, bbar, 5.0 * eps_k)
                if ok:
                    w, beta = w1, b1
                else:
                    F.use_T = True
                    Tw = F.T_apply(w)
                    w, beta = F.solve_T(hw1 + Tw, hb1)
            n_double += 1
        else:
            w, beta = wbar, bbar
        r = r_new
        # Step 2
        Ztw = Zt.T @ w
        u, xi = step2(w, beta, r, alpha, rho, Ztw, y, C, sigma, mu, R, ev)
        # Step 3
        alpha, rho = step3(alpha, rho, Ztw, y, beta, xi, r, w, u, sigma, mu, tau)
        # Section 4.3
        e = kkt_residuals(Zt, zscale, y, C, q, mu, r, w, beta, xi, u, alpha, rho=rho,
                          Ztw=Ztw, rho_residual=rho_residual, wt=wt, e=ev)
        it = k + 1
        if record:
            hist.append(dict(k=k, sigma=sigma, P=e["P"], D=e["D"], C=e["C"], gap=e["gap"],
                             doubled=res > 5.0 * eps_k))
        if stop_test(e, tol):
            converged = True
            break
        # Section 4.4
        if (k + 1) % sigma_every == 0:
            sigma = sigma_update(sigma, e["P"], e["D"])
    return dict(w=w / zscale, u=u / zscale, beta=float(beta), r=r, xi=xi, alpha=alpha,
                w_scaled=w, u_scaled=u, rho=rho, sigma=sigma, zscale=zscale,
                iters=it, n_double=n_double, newton_max=newton_max, eta=e,
                psqmr_steps=list(F.steps) if it_mode else None,
                used_T=bool(F.use_T) if it_mode else None,
                converged=converged, history=hist)


def kkt_of_solution(X, y, C, q, sol, mu=1.0, rho_residual=True, weights=False, e=None):
    """Recompute every residual of Section 4.3 in FP64 from a returned state
    (w and u unscaled, rho of the scaled problem, as :func:`solve` and the
    GPU solver return them)."""
    y = np.asarray(y, dtype=np.float64)
    Zt, zscale = scale_data(X, y)
    rho = sol.get("rho")
    return kkt_residuals(Zt, zscale, y, C, q, mu, np.asarray(sol["r"], np.float64),
                         np.asarray(sol["w"], np.float64) * zscale, float(sol["beta"]),
                         np.asarray(sol["xi"], np.float64),
                         np.asarray(sol["u"], np.float64) * zscale,
                         np.asarray(sol["alpha"], np.float64),
                         rho=None if rho is None else np.asarray(rho, np.float64),
                         rho_residual=rho_residual,
                         wt=loss_weights(y, q, weights), e=e)
