// Iterative branch (Section 3.3.3): set-up (Lanczos eigenpairs of Z~ Z~^T,
// the closed-form inverse of eq-T, eq-schur constants) and the solve loop.
// The kernels are in kernels_iterative.hip.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dwd_solver.h"

namespace dwd {

#define HIP_TRY_I(expr)                                  \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
  } while (0)

// Lanczos steps: min(d, 64) (enough for the ell <= 32 largest pairs of the
// spectra met here to converge to rounding; the same count as the oracle's)
static int lanczos_steps(int64_t d, int ell) {
  (void)ell;
  return (int)std::min<int64_t>(d, (int64_t)kItMaxLanczos);
}

int64_t iterative_footprint(int64_t d, int n, int storage, int ell) {
  const int64_t ld = padded_ld(d);
  const int64_t el = storage == DWD_FP64 ? 8 : 4;
  const int m = lanczos_steps(d, ell);
  int64_t b = ld * n * el;                                   // X
  b += (int64_t)n * 8 * 12;                                  // y, e, ten n-vectors
  b += ld * 8 * (11 + ell + m);                              // d-vectors, Wm, Lanczos basis
  b += (ld / kLdAlign) * 2 * (int64_t)n * 8;                 // Z~^T partials
  b += ((ld + kItDotsBlock - 1) / kItDotsBlock) * (kItMaxLanczos + 2) * 8;
  b += ((n + 255) / 256) * kItNpn * 16 + (ld / 256 + 1) * 64;
  b += (int64_t)it_zpass_splits(ld, n) * 3 * ld * 8;        // sample-split pass partials
  b += ld * 8 * 8 + (int64_t)n * 8 + ((std::max<int64_t>(ld, n) + 2047) / 2048) * 64 +
       ((n + 255) / 256) * 8 + PQ_COUNT * 8;                 // PSQMR state
  return b;
}

dwd_status setup_iterative(Problem* P, const dwd_params* p, hipStream_t st) {
  const int n = P->n;
  const int64_t d = P->d, ld = P->ld;
  const int ell = std::max(2, std::min<int>(p->ell > 0 ? p->ell : 10, (int)std::min<int64_t>(d, kItMaxEll)));
  const int m = lanczos_steps(d, ell);
  if (m < ell) return fail(DWD_E_INVALID, "the iterative solver needs d >= ell");
  ItPtrs& q = P->ipt;
  auto alloc = [&](double** dst, size_t count) -> hipError_t {
    return P->alloc((void**)dst, std::max<size_t>(count, 1) * 8);
  };
  double* nv = nullptr;
  HIP_TRY_I(alloc(&nv, (size_t)n * 10));
  double** nvs[] = {&q.r, &q.xi, &q.alpha, &q.zb, &q.z, &q.rn, &q.dr, &q.a0, &q.a1, &q.a2};
  for (int j = 0; j < 10; ++j) *nvs[j] = nv + (size_t)j * n;
  double* dv = nullptr;
  HIP_TRY_I(alloc(&dv, (size_t)ld * 11));
  q.w = dv;
  q.wbar = dv + ld;
  q.u = dv + 2 * ld;
  q.rho = dv + 3 * ld;
  q.h = dv + 4 * ld;
  q.zz = dv + 5 * ld;        // 4 ld
  q.scratch = dv + 9 * ld;   // 2 ld
  HIP_TRY_I(hipMemsetAsync(dv, 0, (size_t)ld * 11 * 8, st));
  HIP_TRY_I(alloc(&q.Wm, (size_t)ell * ld));
  HIP_TRY_I(hipMemsetAsync(q.Wm, 0, (size_t)ell * ld * 8, st));
  HIP_TRY_I(alloc(&q.lam, kItMaxEll));
  HIP_TRY_I(alloc(&q.dots, ID_COUNT * (kItMaxLanczos + 2)));
  HIP_TRY_I(hipMemsetAsync(q.dots, 0, ID_COUNT * (kItMaxLanczos + 2) * 8, st));
  HIP_TRY_I(alloc(&q.sca, 16));
  HIP_TRY_I(hipMemsetAsync(q.sca, 0, 16 * 8, st));
  q.nchunks = (int)(ld / kLdAlign);
  q.nbd = (int)((ld + kItDotsBlock - 1) / kItDotsBlock);
  q.nbn = (n + 255) / 256;
  q.nbd2 = (int)((ld + 255) / 256);
  HIP_TRY_I(alloc(&q.partT, (size_t)q.nchunks * 2 * n));
  HIP_TRY_I(alloc(&q.part_dd, (size_t)q.nbd * (kItMaxLanczos + 2)));
  HIP_TRY_I(alloc(&q.part_n, (size_t)q.nbn * kItNpn));
  HIP_TRY_I(alloc(&q.part_n2, (size_t)q.nbn * kItNpn));
  HIP_TRY_I(alloc(&q.part_d, (size_t)q.nbd2 * 8));
  q.zsplits = it_zpass_splits(ld, n);
  HIP_TRY_I(alloc(&q.part3, (size_t)q.zsplits * 3 * ld));
  // [problem, skip flag, PSQMR stop flag]
  HIP_TRY_I(P->alloc((void**)&q.sc, 3 * sizeof(Scal)));
  HIP_TRY_I(hipMemsetAsync(q.sc, 0, 3 * sizeof(Scal), st));
  {  // PSQMR state (kernels_psqmr.hip)
    PqPtrs& z = P->pq;
    double* pv = nullptr;
    HIP_TRY_I(alloc(&pv, (size_t)ld * 8));
    HIP_TRY_I(hipMemsetAsync(pv, 0, (size_t)ld * 8 * 8, st));
    double** pvs[] = {&z.x, &z.r, &z.rt, &z.q, &z.t, &z.d, &z.ad};
    for (int j = 0; j < 7; ++j) *pvs[j] = pv + (size_t)j * ld;
    z.zy = pv + 7 * (size_t)ld;
    HIP_TRY_I(alloc(&z.a, (size_t)n));
    z.npart = (int)((std::max<int64_t>(ld, n) + 2047) / 2048);
    HIP_TRY_I(alloc(&z.part, (size_t)z.npart * 8));
    HIP_TRY_I(alloc(&z.part_n, (size_t)((n + 255) / 256)));
    HIP_TRY_I(alloc(&z.s, PQ_COUNT));
    HIP_TRY_I(hipMemsetAsync(z.s, 0, PQ_COUNT * 8, st));
    z.flag = q.sc + 2;
  }
  q.y = P->y;
  q.e = P->e;
  q.ell = ell;

  Consts c{};
  c.d = d;
  c.ld = ld;
  c.n = n;
  c.mu = P->mu;
  c.inv_zs = 1.0 / P->zscale;
  // Lanczos on Z~ Z~^T (m steps, full reorthogonalisation twice per step)
  double *V = nullptr, *lan = nullptr;
  HIP_TRY_I(hipMalloc((void**)&V, (size_t)m * ld * 8));
  const size_t lan_count = 2 * (size_t)m + (size_t)m * ell + ell;
  hipError_t e = hipMalloc((void**)&lan, lan_count * 8);
  double* la = lan;          // alpha_j
  double* lb = lan + m;      // beta_j^2
  double* S = lan + 2 * m;   // m x ell eigenvector components, ell index slots
  double* W = q.h;           // work d-vector
  double* aux = q.dots + 3 * (kItMaxLanczos + 2);
  if (e == hipSuccess) e = hipMemsetAsync(lan, 0, lan_count * 8, st);
  if (e == hipSuccess) e = launch_it_lanczos_start(c, V, nullptr, 0, st);
  if (e == hipSuccess) e = launch_it_dots(c, q, V, nullptr, 0, ID_AUX, 1, st);
  if (e == hipSuccess) e = launch_it_scale(c, V, V, aux, st);
  for (int j = 0; j < m && e == hipSuccess; ++j) {
    double* vj = V + (size_t)j * ld;
    e = launch_gemvT(P->X_rec, P->st_rec, ld, n, vj, vj, q.partT, nullptr, st);
    if (e == hipSuccess) e = launch_it_reduceT(c, q, 3, st);
    if (e == hipSuccess)
      e = launch_it_zpass(P->X_rec, P->st_rec, c, q, q.a0, q.a0, q.a0, W, q.scratch,
                          q.scratch + ld, nullptr, st);
    if (e == hipSuccess) e = launch_it_dots(c, q, W, V, j + 1, ID_AUX, 0, st);
    if (e == hipSuccess) e = launch_it_copy(la + j, aux + j, 1, st);
    if (e == hipSuccess) e = launch_it_orth(c, W, V, j + 1, aux, st);
    if (e == hipSuccess) e = launch_it_dots(c, q, W, V, j + 1, ID_AUX, 0, st);
    if (e == hipSuccess) e = launch_it_orth(c, W, V, j + 1, aux, st);
    if (j + 1 < m) {
      if (e == hipSuccess) e = launch_it_dots(c, q, W, nullptr, 0, ID_AUX, 1, st);
      if (e == hipSuccess) e = launch_it_copy(lb + j, aux, 1, st);
      if (e == hipSuccess) e = launch_it_scale(c, V + (size_t)(j + 1) * ld, W, aux, st);
    }
  }
  if (e == hipSuccess) e = launch_it_eig(la, lb, m, ell, q.lam, S, st);
  if (e == hipSuccess) e = launch_it_ritz(c, V, m, S, ell, q.Wm, st);
  // Z~ y, g = (closed-form inverse) Z~ y, schur = y^T y - (Z~ y)^T g
  double* Zy = q.scratch;
  if (e == hipSuccess)
    e = launch_it_zpass(P->X_rec, P->st_rec, c, q, P->y, P->y, P->y, Zy, q.h, q.wbar, nullptr, st);
  if (e == hipSuccess) e = launch_it_dots(c, q, Zy, q.Wm, ell - 1, ID_AUX, 0, st);
  if (e == hipSuccess) e = launch_it_gvec(c, q, Zy, st);
  // (Z~ y is kept for the PSQMR start residual A [w; beta])
  if (e == hipSuccess) e = launch_it_copy((double*)P->pq.zy, Zy, ld, st);
  if (e == hipSuccess) e = hipMemsetAsync(dv, 0, (size_t)ld * 11 * 8, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(V);
  (void)hipFree(lan);
  if (e != hipSuccess) return hip_fail(e, "iterative set-up");
  double hs[2] = {0.0, 0.0};
  HIP_TRY_I(hipMemcpy(hs, q.sca + IS_SCHUR, 8, hipMemcpyDeviceToHost));
  double lam_h[kItMaxEll];
  HIP_TRY_I(hipMemcpy(lam_h, q.lam, ell * 8, hipMemcpyDeviceToHost));
  if (!(hs[0] > 0.0) || !std::isfinite(hs[0]) || !(lam_h[ell - 1] >= 0.0))
    return fail(DWD_E_NUMERIC, "eigenpairs or Schur complement of the proximal system failed");
  return DWD_OK;
}

// Pieces of one iteration, queued on st.
// Step 1a with the proximal term: h with T w^k, then the closed-form solve.
static hipError_t queue_step1a_T(Problem* P, const Consts& c, hipStream_t st) {
  const ItPtrs& q = P->ipt;
  const int L = q.ell;
  hipError_t e;
  if ((e = launch_it_dots(c, q, q.w, q.Wm, L - 1, ID_W, 0, st)) != hipSuccess) return e;
  if ((e = launch_it_rhs(c, q, st, 1)) != hipSuccess) return e;
  if ((e = launch_it_dots(c, q, q.h, q.Wm, L, ID_H, 0, st)) != hipSuccess) return e;
  return launch_it_solve(c, q, 0, st);
}

// Step 1b (Z~^T wbar, the prox) and the Z~ dr pass of Step 1c.
static hipError_t queue_step1b(Problem* P, const Consts& c, hipStream_t st) {
  const ItPtrs& q = P->ipt;
  const int64_t ld = P->ld;
  hipError_t e;
  if ((e = launch_gemvT(P->X_rec, P->st_rec, ld, c.n, q.wbar, q.wbar, q.partT, q.sc, st)) !=
      hipSuccess)
    return e;
  if ((e = launch_it_reduceT(c, q, 1, st)) != hipSuccess) return e;
  return launch_it_zpass(P->X_rec, P->st_rec, c, q, q.a0, q.a0, q.a0, q.zz, q.scratch,
                         q.scratch + ld, q.sc, st);
}

// Step 1c with the proximal term (mode 1: the residual test decides;
// mode 2: the re-solve is taken).
static hipError_t queue_step1c_T(Problem* P, const Consts& c, int mode, hipStream_t st) {
  const ItPtrs& q = P->ipt;
  hipError_t e;
  if ((e = launch_it_dots(c, q, q.zz, q.Wm, q.ell, ID_DR, 1, st)) != hipSuccess) return e;
  return launch_it_solve(c, q, mode, st);
}

// Steps 2-3: a fresh Z~^T w (skipped when Step 1c kept wbar), the n-space
// part, Z~ [xi - r, alpha, Z~^T w], the d-space part, residuals, stopping
// and sigma rules.
static hipError_t queue_steps23(Problem* P, const Consts& c, hipStream_t st) {
  const ItPtrs& q = P->ipt;
  const int64_t ld = P->ld;
  hipError_t e;
  if ((e = launch_gemvT(P->X_rec, P->st_rec, ld, c.n, q.w, q.w, q.partT, q.sc + 1, st)) !=
      hipSuccess)
    return e;
  if ((e = launch_it_reduceT(c, q, 2, st)) != hipSuccess) return e;
  if ((e = launch_it_zpass(P->X_rec, P->st_rec, c, q, q.a0, q.a1, q.a2, q.zz + ld,
                           q.zz + 2 * ld, q.zz + 3 * ld, q.sc, st)) != hipSuccess)
    return e;
  if ((e = launch_it_dspace(c, q, 0, st)) != hipSuccess) return e;
  if ((e = launch_it_dspace(c, q, 1, st)) != hipSuccess) return e;
  return launch_it_tail(c, q, st);
}

// One iteration with the proximal term (three passes over X, four when
// Step 1c solves again).
hipError_t queue_iterative_iteration(Problem* P, const Consts& c, hipStream_t st) {
  hipError_t e;
  if ((e = queue_step1a_T(P, c, st)) != hipSuccess) return e;
  if ((e = queue_step1b(P, c, st)) != hipSuccess) return e;
  if ((e = queue_step1c_T(P, c, 1, st)) != hipSuccess) return e;
  return queue_steps23(P, c, st);
}

// One PSQMR solve whose start (launch_pq_start, mode) is to be queued:
// steps in groups of four, the host reading the stop flag after each group.
// Returns the step count and whether ||b - A x|| reached the tolerance.
static hipError_t run_psqmr(Problem* P, const Consts& c, int mode, int max_steps, int* steps,
                            bool* ok) {
  const ItPtrs& q = P->ipt;
  const PqPtrs& z = P->pq;
  const hipStream_t st = P->stream;
  volatile int32_t* hf = (volatile int32_t*)P->h_flags + 64;
  double* hs = (double*)P->h_flags + 64;  // PQ_COUNT doubles (512..)
  hipError_t e;
  if ((e = launch_pq_start(c, q, z, mode, st)) != hipSuccess) return e;
  if ((e = launch_pq_precond(c, q, z, 1, st)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync((void*)hf, &z.flag->done, 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  constexpr int kGroup = 4;
  for (int j = 1; !*hf && j <= max_steps; j += kGroup) {
    for (int jj = j; jj < j + kGroup && jj <= max_steps; ++jj)
      if ((e = launch_pq_step(P->X_rec, P->st_rec, c, q, z, jj, max_steps, st)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync((void*)hf, &z.flag->done, 4, hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(hs, z.s, PQ_COUNT * 8, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  *steps = (int)hs[PQ_STEPS];
  *ok = hs[PQ_OK] != 0.0;
  return hipSuccess;
}

// One iteration in which Steps 1a and 1c solve eq-linsys with T = 0 by
// PSQMR (to eps_k and 5 eps_k).  A solve that needs more than max_steps
// steps switches the proximal term on (*switched) for the rest of the
// solve: Step 1a then solves with T w^k from its own right-hand side, and a
// Step 1c re-solve becomes [w; beta] = closed-form solve of h(r^{k+1}) +
// T w^k.
static hipError_t run_psqmr_iteration(Problem* P, const Consts& c, int max_steps,
                                      bool* switched) {
  const ItPtrs& q = P->ipt;
  const PqPtrs& z = P->pq;
  const hipStream_t st = P->stream;
  double* hs = (double*)P->h_flags + 64;
  hipError_t e;
  int steps = 0;
  bool ok = false;
  *switched = false;
  // Step 1a
  if ((e = launch_it_rhs(c, q, st, 0)) != hipSuccess) return e;
  if ((e = run_psqmr(P, c, 0, max_steps, &steps, &ok)) != hipSuccess) return e;
  P->psqmr_log.push_back(steps);
  if (ok) {
    if ((e = launch_pq_commit(c, q, z, 0, st)) != hipSuccess) return e;
  } else {
    *switched = true;
    if ((e = queue_step1a_T(P, c, st)) != hipSuccess) return e;
  }
  // Step 1b, Z~ dr
  if ((e = queue_step1b(P, c, st)) != hipSuccess) return e;
  // Step 1c
  if (*switched) {
    if ((e = queue_step1c_T(P, c, 1, st)) != hipSuccess) return e;
  } else {
    if ((e = launch_pq_res1c(c, q, z, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(hs, z.s, PQ_COUNT * 8, hipMemcpyDeviceToHost, st)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (hs[PQ_REDO] == 0.0) {
      if ((e = launch_pq_commit(c, q, z, 1, st)) != hipSuccess) return e;
    } else {
      if ((e = run_psqmr(P, c, 1, max_steps, &steps, &ok)) != hipSuccess) return e;
      P->psqmr_log.push_back(steps);
      if (ok) {
        if ((e = launch_pq_commit(c, q, z, 2, st)) != hipSuccess) return e;
      } else {
        *switched = true;
        // h(r^{k+1}) + T w^k = (h + T w^k) + [Z~ dr; y^T dr]: the closed-form
        // solve of the first part into [wbar; betabar], then the re-solve
        if ((e = queue_step1a_T(P, c, st)) != hipSuccess) return e;
        if ((e = queue_step1c_T(P, c, 2, st)) != hipSuccess) return e;
      }
    }
  }
  return queue_steps23(P, c, st);
}

dwd_status solve_iterative(Problem* P, const dwd_params* p, double* w, dwd_info* info,
                           double* alpha, double* r, double* xi, double* u, double* rho) {
  dwd_status s;
  if ((s = validate_params(p, true)) != DWD_OK) return s;
  if ((s = validate_penalty(p, P->n)) != DWD_OK) return s;
  if (p->representer == 1) return fail(DWD_E_INVALID, "the representer iteration needs the SMW set-up");
  HIP_TRY_I(hipSetDevice(P->device));
  const hipStream_t st = P->stream;
  HIP_TRY_I(hipStreamSynchronize(st));
  HIP_TRY_I(P->set_penalty(p->e));
  HIP_TRY_I(hipEventRecord(P->ev_a, st));
  const Consts c = make_consts(P, p);
  const ItPtrs& q = P->ipt;
  HIP_TRY_I(launch_it_init(c, q, default_sigma0(p, P->n), st));
  volatile int32_t* hf = (volatile int32_t*)P->h_flags;
  // PSQMR phase (Section 3.3.3): the host takes each iteration's decisions
  // (the solves' step counts, Step 1c), so it reads the device between the
  // pieces of an iteration; it ends when a solve needs more than psqmr_max
  // steps, or with the solve.
  P->psqmr_log.clear();
  P->psqmr_switch = p->psqmr_max > 0 ? -1 : 0;
  int k0 = 0;
  bool stopped = false;
  while (p->psqmr_max > 0 && P->psqmr_switch < 0 && k0 < c.max_iter) {
    bool sw = false;
    HIP_TRY_I(run_psqmr_iteration(P, c, p->psqmr_max, &sw));
    if (sw) P->psqmr_switch = k0;
    ++k0;
    HIP_TRY_I(hipMemcpyAsync((void*)(hf + 32), &q.sc->done, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY_I(hipStreamSynchronize(st));
    if (hf[32]) {
      stopped = true;
      break;
    }
  }
  // With the proximal term: chunks of check_every iterations, the stop flag
  // of a chunk read on the host while the next chunk runs.
  const int chunk = std::max(1, p->check_every > 0 ? p->check_every : 8);
  int queued = k0, pending = -1;
  for (int cidx = 0; !stopped && queued < c.max_iter; ++cidx) {
    for (int j = 0; j < chunk && queued < c.max_iter; ++j, ++queued)
      HIP_TRY_I(queue_iterative_iteration(P, c, st));
    const int slot = cidx & 1;
    HIP_TRY_I(hipMemcpyAsync((void*)(hf + slot * 16), &q.sc->done, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY_I(hipEventRecord(P->ev_chunk[slot], st));
    if (queued >= c.max_iter) break;
    if (pending >= 0) {
      HIP_TRY_I(hipEventSynchronize(P->ev_chunk[pending & 1]));
      if (hf[(pending & 1) * 16]) break;
    }
    pending = cidx;
  }
  HIP_TRY_I(hipEventRecord(P->ev_b, st));
  Scal hs;
  HIP_TRY_I(hipMemcpyAsync(&hs, q.sc, sizeof(Scal), hipMemcpyDeviceToHost, st));
  HIP_TRY_I(hipStreamSynchronize(st));
  const int64_t d = P->d;
  if (w) {
    HIP_TRY_I(hipMemcpy(w, q.w, d * 8, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < d; ++k) w[k] /= P->zscale;
  }
  if (u) {
    HIP_TRY_I(hipMemcpy(u, q.u, d * 8, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < d; ++k) u[k] /= P->zscale;
  }
  if (rho) HIP_TRY_I(hipMemcpy(rho, q.rho, d * 8, hipMemcpyDeviceToHost));
  if (alpha) HIP_TRY_I(hipMemcpy(alpha, q.alpha, (size_t)P->n * 8, hipMemcpyDeviceToHost));
  if (r) HIP_TRY_I(hipMemcpy(r, q.r, (size_t)P->n * 8, hipMemcpyDeviceToHost));
  if (xi) HIP_TRY_I(hipMemcpy(xi, q.xi, (size_t)P->n * 8, hipMemcpyDeviceToHost));
  // (the residuals of this branch come from explicit products, so the
  // check values are the in-loop ones; the rule is the same as elsewhere)
  const int conv =
      hs.converged && std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]) < p->tol ? 1 : 0;
  float ms = 0.0f;
  HIP_TRY_I(hipEventElapsedTime(&ms, P->ev_a, P->ev_b));
  if (info) {
    memset(info, 0, sizeof(*info));
    info->beta = hs.beta;
    info->primal_obj = hs.eta[E_PRIM];
    info->dual_obj = hs.eta[E_DUAL];
    info->eta_p = hs.eta[E_P];
    info->eta_d = hs.eta[E_D];
    info->eta_c = hs.eta[E_C];
    info->eta_gap = hs.eta[E_GAP];
    info->eta_p_check = hs.eta[E_PCHK];
    info->eta_d_check = hs.eta[E_DCHK];
    info->kkt_check = std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]);
    info->sigma = hs.sigma;
    info->iters = hs.k;
    info->n_double = hs.n_double;
    info->newton_max = hs.newton_max;
    info->converged = conv;
    info->setup_ms = P->setup_ms;
    info->solve_ms = ms;
    info->psqmr_solves = (int32_t)P->psqmr_log.size();
    for (int v : P->psqmr_log) info->psqmr_steps += v;
    info->psqmr_switch = P->psqmr_switch;
    info->status = conv ? DWD_OK : DWD_NOT_CONVERGED;
  }
  return conv ? DWD_OK : DWD_NOT_CONVERGED;
}

}  // namespace dwd
