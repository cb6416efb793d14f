// Preconditioned symmetric QMR (Freund and Nachtigal) for eq-linsys with
// T = 0 (Section 3.3.3): the first solver of the iterative branch, before
// the proximal term of eq-T is switched on.
//
// The system is A [w; beta] = [h; h_beta] with
//     A = [[Z~ Z~^T + mu I, Z~ y], [(Z~ y)^T, y^T y]]   ((d+1) x (d+1)),
// and the preconditioner is the T-modified matrix, whose inverse is the
// closed form of eq-T with the Schur complement on beta (eq-schur), as in
// kernels_iterative.hip.  A vector of length d+1 is a d-vector (length ld,
// padding zero) plus its beta component, kept in the scalar array PqPtrs::s.
//
// One step: t = A q (two passes over X: Z~^T q_w, then Z~ (Z~^T q_w + y q_b)),
// sigma = q^T t, alpha = rho / sigma, r <- r - alpha t, theta = ||r|| / tau,
// c = 1 / (1 + theta^2), tau <- tau theta sqrt(c),
// d <- c theta_prev^2 d + c alpha q, x <- x + d; the true residual
// b - A x is carried by the same recurrence (A d <- c theta_prev^2 A d +
// c alpha t, rt <- rt - A d), so the stopping test ||b - A x|| <= tol costs
// no extra pass; then u = M^-1 r, rho' = r^T u, q <- u + (rho'/rho) q.
// Global sums are block partials summed in a fixed order by every block
// that needs them, so repeated solves are bit-identical; every kernel of a
// step returns at once when the solve has stopped (flag PqPtrs::flag->done).
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "dwd_device.h"
#include "dwd_internal.h"
#include "dwd_iterative.h"
#include "dwd_solver.h"

namespace dwd {

namespace {

constexpr int DSTRIDE = kItMaxLanczos + 2;
constexpr int PQ_EPB = 2048;  // d-space entries per block (8 per thread)

// Fixed-order sum of `slot` over the nb block partials (stride 8), valid in
// every thread of the block.
__device__ __forceinline__ double pq_sum(const double* __restrict__ part, int nb, int slot) {
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) v += part[(size_t)b * 8 + slot];
  return block_sum<256>(v);
}

// u = M^-1 r for the (d+1)-vector r (r_w, r_b) with the dots
// dx[j] = v_j^T r_w (j < ell - 1), dx[ell - 1] = g^T r_w (eq-T, eq-schur).
__device__ __forceinline__ double pq_precond_w(const Consts& c, const ItPtrs& p, const double* dx,
                                               double rw, int64_t f, double ub) {
  const int L = p.ell;
  const double lamL = p.lam[L - 1];
  const double cl = 1.0 / (c.mu + lamL);
  double v = rw * cl;
  for (int j = 0; j < L - 1; ++j)
    v = fma((1.0 / (c.mu + p.lam[j]) - cl) * dx[j], p.Wm[(size_t)j * c.ld + f], v);
  return v - ub * p.Wm[(size_t)(L - 1) * c.ld + f];
}

}  // namespace

// ---------------------------------------------------------------------------
// Start of a solve.  mode 0 (Step 1a): x0 = [w; beta] (the current iterate),
// r0 = [h; h_beta] - A x0 with A x0 = [Z~ Z~^T w + beta Z~ y + mu w;
// y^T Z~^T w + n beta] (Z~ Z~^T w and Z~^T w are kept by the iteration);
// mode 1 (Step 1c re-solve): x0 = [wbar; betabar], r0 = the Step 1c
// residual [Z~ dr + rt_w; y^T dr + rt_b] already in q.r.  r, rt = r0,
// d = A d = 0; block partials of ||r_w||^2 and (mode 0) of y^T Z~^T w.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_pq_start(Consts c, ItPtrs p, PqPtrs q, int mode) {
  if (p.sc->done) return;
  const double beta = p.sc->beta;
  double acc[2] = {0.0, 0.0};
  const int64_t base = (int64_t)blockIdx.x * PQ_EPB;
  for (int e = 0; e < PQ_EPB / 256; ++e) {
    const int64_t f = base + e * 256 + threadIdx.x;
    if (f < c.ld) {
      double r;
      if (mode == 0) {
        const double w = p.w[f];
        r = p.h[f] - (p.zz[3 * c.ld + f] + beta * q.zy[f] + c.mu * w);
        q.x[f] = w;
      } else {
        r = q.r[f];
        q.x[f] = p.wbar[f];
      }
      q.r[f] = r;
      q.rt[f] = r;
      q.d[f] = 0.0;
      q.ad[f] = 0.0;
      acc[0] = fma(r, r, acc[0]);
    }
    if (mode == 0 && f < c.n) acc[1] = fma(p.y[f], p.z[f], acc[1]);
  }
  block_sum_k<256, 2>(acc);
  if (threadIdx.x < 2) q.part[(size_t)blockIdx.x * 8 + threadIdx.x] = acc[threadIdx.x];
}

// One block: tau = ||r0||, the tolerance, the beta components, the stop
// test before any step.
__global__ void __launch_bounds__(256) k_pq_norm(Consts c, ItPtrs p, PqPtrs q, int mode, int nb) {
  if (p.sc->done) return;
  const double rw2 = pq_sum(q.part, nb, 0);
  const double ytz = mode == 0 ? pq_sum(q.part, nb, 1) : 0.0;
  if (threadIdx.x != 0) return;
  double* s = q.s;
  double rb;
  if (mode == 0) {
    const double beta = p.sc->beta;
    rb = p.sca[IS_HB] - (ytz + (double)c.n * beta);
    s[PQ_XB] = beta;
  } else {
    rb = s[PQ_RB];
    s[PQ_XB] = p.sca[IS_BETABAR];
  }
  s[PQ_RB] = rb;
  s[PQ_RTB] = rb;
  s[PQ_DB] = 0.0;
  s[PQ_ADB] = 0.0;
  s[PQ_THETA] = 0.0;
  const double tau = sqrt(rw2 + rb * rb);
  s[PQ_TAU] = tau;
  const double tol = (mode == 0 ? 1.0 : 5.0) * eps_k(c, p.sc->k);
  s[PQ_TOL] = tol;
  s[PQ_STEPS] = 0.0;
  s[PQ_RES] = tau;
  const bool ok = tau <= tol;
  s[PQ_OK] = ok ? 1.0 : 0.0;
  q.flag->done = ok ? 1 : 0;
}

// u = M^-1 r (dots of r_w with the rows of Wm in dots[ID_PQ]) and block
// partials of r^T u.  init = 1: q = u (start of the solve); else u goes
// into t (t is not needed again in this step).
__global__ void __launch_bounds__(256) k_pq_precond(Consts c, ItPtrs p, PqPtrs q, int init) {
  if (p.sc->done || q.flag->done) return;
  const int L = p.ell;
  const double* dx = p.dots + (size_t)ID_PQ * DSTRIDE;
  const double rb = q.s[PQ_RB];
  const double ub = (rb - dx[L - 1]) / p.sca[IS_SCHUR];
  double acc = 0.0;
  double* out = init ? q.q : q.t;
  const int64_t base = (int64_t)blockIdx.x * PQ_EPB;
  for (int e = 0; e < PQ_EPB / 256; ++e) {
    const int64_t f = base + e * 256 + threadIdx.x;
    if (f < c.ld) {
      const double rw = q.r[f];
      const double u = pq_precond_w(c, p, dx, rw, f, ub);
      out[f] = u;
      acc = fma(rw, u, acc);
    }
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) {
    q.part[(size_t)blockIdx.x * 8 + 2] = acc;
    if (blockIdx.x == 0) q.s[init ? PQ_QB : PQ_UB] = ub;
  }
}

// One block: rho = r^T u of the start.
__global__ void __launch_bounds__(256) k_pq_rho(ItPtrs p, PqPtrs q, int nb) {
  if (p.sc->done || q.flag->done) return;
  const double ru = pq_sum(q.part, nb, 2);
  if (threadIdx.x == 0) q.s[PQ_RHO] = ru + q.s[PQ_RB] * q.s[PQ_QB];
}

// ---------------------------------------------------------------------------
// t = A q, first half: a_i = (Z~^T q_w)_i + y_i q_b from the k_gemvT
// partials, and block partials of y^T Z~^T q_w (for t_b).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_pq_at(Consts c, ItPtrs p, PqPtrs q) {
  if (p.sc->done || q.flag->done) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double qb = q.s[PQ_QB];
  double acc = 0.0;
  if (i < c.n) {
    double raw = 0.0;
    for (int ch = 0; ch < p.nchunks; ++ch) raw += p.partT[((size_t)ch * 2) * c.n + i];
    const double yi = p.y[i];
    const double z = yi * raw * c.inv_zs;
    q.a[i] = z + yi * qb;
    acc = yi * z;
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) q.part_n[blockIdx.x] = acc;
}

// t_w = Z~ a + mu q_w, block partials of q_w^T t_w.
__global__ void __launch_bounds__(256) k_pq_t(Consts c, ItPtrs p, PqPtrs q) {
  if (p.sc->done || q.flag->done) return;
  double acc = 0.0;
  const int64_t base = (int64_t)blockIdx.x * PQ_EPB;
  for (int e = 0; e < PQ_EPB / 256; ++e) {
    const int64_t f = base + e * 256 + threadIdx.x;
    if (f < c.ld) {
      const double qw = q.q[f];
      const double t = q.t[f] + c.mu * qw;
      q.t[f] = t;
      acc = fma(qw, t, acc);
    }
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) q.part[(size_t)blockIdx.x * 8 + 3] = acc;
}

// sigma = q^T t, alpha = rho / sigma, r <- r - alpha t; block partials of
// ||r_w||^2.  (sigma = 0 or rho = 0 ends the solve, as a breakdown.)
__global__ void __launch_bounds__(256) k_pq_r(Consts c, ItPtrs p, PqPtrs q, int nb) {
  if (p.sc->done || q.flag->done) return;
  double ytz = 0.0;
  for (int b = threadIdx.x; b < p.nbn; b += 256) ytz += q.part_n[b];
  ytz = block_sum<256>(ytz);
  const double qtw = pq_sum(q.part, nb, 3);
  const double qb = q.s[PQ_QB];
  const double tb = ytz + (double)c.n * qb;  // (Z~ y)^T q_w + y^T y q_b
  const double sigma = qtw + qb * tb;
  const double rho = q.s[PQ_RHO];
  const bool brk = sigma == 0.0 || rho == 0.0;
  const double alpha = brk ? 0.0 : rho / sigma;
  double acc = 0.0;
  const int64_t base = (int64_t)blockIdx.x * PQ_EPB;
  for (int e = 0; e < PQ_EPB / 256; ++e) {
    const int64_t f = base + e * 256 + threadIdx.x;
    if (f < c.ld) {
      const double r = brk ? q.r[f] : q.r[f] - alpha * q.t[f];
      q.r[f] = r;
      acc = fma(r, r, acc);
    }
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) {
    q.part[(size_t)blockIdx.x * 8 + 4] = acc;
    if (blockIdx.x == 0) {
      q.s[PQ_TB] = tb;
      q.s[PQ_ALPHA] = alpha;
      q.s[PQ_BRK] = brk ? 1.0 : 0.0;
      if (!brk) q.s[PQ_RB] -= alpha * tb;
    }
  }
}

// theta = ||r|| / tau, c = 1/(1 + theta^2), tau <- tau theta sqrt(c);
// d <- c theta_prev^2 d + c alpha q, A d <- c theta_prev^2 A d + c alpha t,
// x <- x + d, rt <- rt - A d; block partials of ||rt_w||^2.
__global__ void __launch_bounds__(256) k_pq_x(Consts c, ItPtrs p, PqPtrs q, int nb) {
  if (p.sc->done || q.flag->done) return;
  const double rw2 = pq_sum(q.part, nb, 4);
  const double* s = q.s;
  const bool brk = s[PQ_BRK] != 0.0;
  const double rb = s[PQ_RB];
  const double theta_prev = s[PQ_THETA];
  const double theta = sqrt(rw2 + rb * rb) / s[PQ_TAU];
  const double c2 = 1.0 / (1.0 + theta * theta);
  const double ca = brk ? 1.0 : c2 * theta_prev * theta_prev;
  const double cb = brk ? 0.0 : c2 * s[PQ_ALPHA];
  double acc = 0.0;
  const int64_t base = (int64_t)blockIdx.x * PQ_EPB;
  for (int e = 0; e < PQ_EPB / 256; ++e) {
    const int64_t f = base + e * 256 + threadIdx.x;
    if (f < c.ld) {
      double dv = q.d[f], av = q.ad[f], rt = q.rt[f];
      if (!brk) {
        dv = ca * dv + cb * q.q[f];
        av = ca * av + cb * q.t[f];
        q.d[f] = dv;
        q.ad[f] = av;
        q.x[f] += dv;
        rt -= av;
        q.rt[f] = rt;
      }
      acc = fma(rt, rt, acc);
    }
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) {
    q.part[(size_t)blockIdx.x * 8 + 5] = acc;
    if (blockIdx.x == 0 && !brk) {
      double* sw = q.s;
      const double db = ca * sw[PQ_DB] + cb * sw[PQ_QB];
      const double adb = ca * sw[PQ_ADB] + cb * sw[PQ_TB];
      sw[PQ_DB] = db;
      sw[PQ_ADB] = adb;
      sw[PQ_XB] += db;
      sw[PQ_RTB] -= adb;
      // (theta and tau are read by every block of this kernel: the new
      // values wait in their own slots until k_pq_test moves them)
      sw[PQ_THETA_N] = theta;
      sw[PQ_TAU_N] = s[PQ_TAU] * theta * sqrt(c2);
    }
  }
}

// One block: the stop test ||b - A x|| <= tol after step j (or the end of
// the step budget, or a breakdown); sets the flag that ends the solve.
__global__ void __launch_bounds__(256) k_pq_test(ItPtrs p, PqPtrs q, int nb, int j, int max_steps) {
  if (p.sc->done || q.flag->done) return;
  const double rt2 = pq_sum(q.part, nb, 5);
  if (threadIdx.x != 0) return;
  double* s = q.s;
  if (s[PQ_BRK] == 0.0) {
    s[PQ_THETA] = s[PQ_THETA_N];
    s[PQ_TAU] = s[PQ_TAU_N];
  }
  const double rtb = s[PQ_RTB];
  const double res = sqrt(rt2 + rtb * rtb);
  s[PQ_RES] = res;
  const bool ok = res <= s[PQ_TOL];
  const bool brk = s[PQ_BRK] != 0.0;
  if (ok || brk || j >= max_steps) {
    s[PQ_OK] = ok ? 1.0 : 0.0;
    s[PQ_STEPS] = (double)((ok && !brk) ? j : max_steps);
    q.flag->done = 1;
  } else {
    s[PQ_STEPS] = (double)j;
  }
}

// rho' = r^T u, q <- u + (rho'/rho) q (u is in t).  Every block reads rho
// and q_b, so their new values are written by the one-block k_pq_qfin.
__global__ void __launch_bounds__(256) k_pq_q(Consts c, ItPtrs p, PqPtrs q, int nb) {
  if (p.sc->done || q.flag->done) return;
  const double ru = pq_sum(q.part, nb, 2);
  const double rho_new = ru + q.s[PQ_RB] * q.s[PQ_UB];
  const double ratio = rho_new / q.s[PQ_RHO];
  const int64_t base = (int64_t)blockIdx.x * PQ_EPB;
  for (int e = 0; e < PQ_EPB / 256; ++e) {
    const int64_t f = base + e * 256 + threadIdx.x;
    if (f < c.ld) q.q[f] = q.t[f] + ratio * q.q[f];
  }
}

__global__ void __launch_bounds__(256) k_pq_qfin(ItPtrs p, PqPtrs q, int nb) {
  if (p.sc->done || q.flag->done) return;
  const double ru = pq_sum(q.part, nb, 2);  // (the same fixed-order sum)
  if (threadIdx.x != 0) return;
  const double rho_new = ru + q.s[PQ_RB] * q.s[PQ_UB];
  const double ratio = rho_new / q.s[PQ_RHO];
  q.s[PQ_QB] = q.s[PQ_UB] + ratio * q.s[PQ_QB];
  q.s[PQ_RHO] = rho_new;
}

// ---------------------------------------------------------------------------
// Step 1c with T = 0: the residual ||h(r^{k+1}) - A [wbar; betabar]|| =
// ||[Z~ dr + rt_w; y^T dr + rt_b]|| (rt: the true residual the Step 1a solve
// ended with); the vector goes into q.r, the start residual of a re-solve.
// Block partials of ||.||^2; k_pq_decide takes the decision.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_pq_res1c(Consts c, ItPtrs p, PqPtrs q) {
  if (p.sc->done) return;
  double acc = 0.0;
  const int64_t base = (int64_t)blockIdx.x * PQ_EPB;
  for (int e = 0; e < PQ_EPB / 256; ++e) {
    const int64_t f = base + e * 256 + threadIdx.x;
    if (f < c.ld) {
      const double r = p.zz[f] + q.rt[f];
      q.r[f] = r;
      acc = fma(r, r, acc);
    }
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) q.part[(size_t)blockIdx.x * 8 + 6] = acc;
}

__global__ void __launch_bounds__(256) k_pq_decide(Consts c, ItPtrs p, PqPtrs q, int nb) {
  if (p.sc->done) return;
  const double rw2 = pq_sum(q.part, nb, 6);
  double ydr = 0.0;
  for (int b = threadIdx.x; b < p.nbn; b += 256) ydr += p.part_n[(size_t)b * kItNpn + 0];
  ydr = block_sum<256>(ydr);
  if (threadIdx.x != 0) return;
  const double rb = ydr + q.s[PQ_RTB];
  q.s[PQ_RB] = rb;
  const double res = sqrt(rw2 + rb * rb);
  q.s[PQ_RES1C] = res;
  q.s[PQ_REDO] = res > 5.0 * eps_k(c, p.sc->k) ? 1.0 : 0.0;
  p.sca[IS_YDR] = ydr;
}

// Commit Step 1a/1c with T = 0: keep = 1: [w; beta] = [wbar; betabar];
// keep = 0: [w; beta] = the re-solve's x.  Step 1a (to1a = 1): [wbar;
// betabar] = the Step 1a solve's x.  The doubled flag, n_double and the
// flag that skips the fresh Z~^T w pass follow Step 1c's outcome.
__global__ void __launch_bounds__(256) k_pq_commit(Consts c, ItPtrs p, PqPtrs q, int what) {
  if (p.sc->done) return;
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f < c.ld) {
    if (what == 0)
      p.wbar[f] = q.x[f];
    else if (what == 1)
      p.w[f] = p.wbar[f];
    else
      p.w[f] = q.x[f];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Scal* sc = p.sc;
    if (what == 0) {
      p.sca[IS_BETABAR] = q.s[PQ_XB];
    } else {
      const int redo = what == 2 ? 1 : 0;
      sc->beta = redo ? q.s[PQ_XB] : p.sca[IS_BETABAR];
      sc->doubled = redo;
      sc->n_double += redo;
      p.sc[1].done = redo ? 0 : 1;  // skip the fresh Z~^T w pass when wbar is kept
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
int pq_dblocks(int64_t ld) { return (int)((ld + PQ_EPB - 1) / PQ_EPB); }

hipError_t launch_pq_start(const Consts& c, const ItPtrs& p, const PqPtrs& q, int mode,
                           hipStream_t st) {
  const int64_t m = std::max<int64_t>(c.ld, c.n);
  const int nb = (int)((m + PQ_EPB - 1) / PQ_EPB);
  if (nb > q.npart) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pq_start, dim3((unsigned)nb), dim3(256), 0, st, c, p, q, mode);
  hipLaunchKernelGGL(k_pq_norm, dim3(1), dim3(256), 0, st, c, p, q, mode, nb);
  return hipGetLastError();
}

hipError_t launch_pq_precond(const Consts& c, const ItPtrs& p, const PqPtrs& q, int init,
                             hipStream_t st) {
  const int nb = pq_dblocks(c.ld);
  hipError_t e = launch_it_dots(c, p, q.r, p.Wm, p.ell, ID_PQ, 0, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pq_precond, dim3((unsigned)nb), dim3(256), 0, st, c, p, q, init);
  if (init) hipLaunchKernelGGL(k_pq_rho, dim3(1), dim3(256), 0, st, p, q, nb);
  return hipGetLastError();
}

hipError_t launch_pq_step(const void* X, int storage, const Consts& c, const ItPtrs& p,
                          const PqPtrs& q, int j, int max_steps, hipStream_t st) {
  const int nb = pq_dblocks(c.ld);
  hipError_t e;
  // t = A q
  if ((e = launch_gemvT(X, storage, c.ld, c.n, q.q, q.q, p.partT, q.flag, st)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_pq_at, dim3((unsigned)p.nbn), dim3(256), 0, st, c, p, q);
  if ((e = launch_it_zpass(X, storage, c, p, q.a, q.a, q.a, q.t, p.scratch, p.scratch + c.ld,
                           q.flag, st)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_pq_t, dim3((unsigned)nb), dim3(256), 0, st, c, p, q);
  hipLaunchKernelGGL(k_pq_r, dim3((unsigned)nb), dim3(256), 0, st, c, p, q, nb);
  hipLaunchKernelGGL(k_pq_x, dim3((unsigned)nb), dim3(256), 0, st, c, p, q, nb);
  hipLaunchKernelGGL(k_pq_test, dim3(1), dim3(256), 0, st, p, q, nb, j, max_steps);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // u = M^-1 r (into t), then q
  if ((e = launch_it_dots(c, p, q.r, p.Wm, p.ell, ID_PQ, 0, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pq_precond, dim3((unsigned)nb), dim3(256), 0, st, c, p, q, 0);
  hipLaunchKernelGGL(k_pq_q, dim3((unsigned)nb), dim3(256), 0, st, c, p, q, nb);
  hipLaunchKernelGGL(k_pq_qfin, dim3(1), dim3(256), 0, st, p, q, nb);
  return hipGetLastError();
}

hipError_t launch_pq_res1c(const Consts& c, const ItPtrs& p, const PqPtrs& q, hipStream_t st) {
  const int nb = pq_dblocks(c.ld);
  hipLaunchKernelGGL(k_pq_res1c, dim3((unsigned)nb), dim3(256), 0, st, c, p, q);
  hipLaunchKernelGGL(k_pq_decide, dim3(1), dim3(256), 0, st, c, p, q, nb);
  return hipGetLastError();
}

hipError_t launch_pq_commit(const Consts& c, const ItPtrs& p, const PqPtrs& q, int what,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_pq_commit, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, st, c, p, q,
                     what);
  return hipGetLastError();
}

}  // namespace dwd
