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
  HIP_TRY_I(alloc(&q.dots, 4 * (kItMaxLanczos + 2)));
  HIP_TRY_I(hipMemsetAsync(q.dots, 0, 4 * (kItMaxLanczos + 2) * 8, st));
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
  HIP_TRY_I(P->alloc((void**)&q.sc, 2 * sizeof(Scal)));  // [problem, skip flag]
  HIP_TRY_I(hipMemsetAsync(q.sc, 0, 2 * sizeof(Scal), st));
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

hipError_t queue_iterative_iteration(Problem* P, const Consts& c, hipStream_t st) {
  const ItPtrs& q = P->ipt;
  const int L = q.ell;
  const int64_t ld = P->ld;
  hipError_t e;
  // Step 1a: h with T w^k, then the closed-form solve
  if ((e = launch_it_dots(c, q, q.w, q.Wm, L - 1, ID_W, 0, st)) != hipSuccess) return e;
  if ((e = launch_it_rhs(c, q, st)) != hipSuccess) return e;
  if ((e = launch_it_dots(c, q, q.h, q.Wm, L, ID_H, 0, st)) != hipSuccess) return e;
  if ((e = launch_it_solve(c, q, 0, st)) != hipSuccess) return e;
  // Step 1b: Z~^T wbar, the prox
  if ((e = launch_gemvT(P->X_rec, P->st_rec, ld, c.n, q.wbar, q.wbar, q.partT, q.sc, st)) !=
      hipSuccess)
    return e;
  if ((e = launch_it_reduceT(c, q, 1, st)) != hipSuccess) return e;
  // Step 1c: Z~ dr, the residual test and the re-solve
  if ((e = launch_it_zpass(P->X_rec, P->st_rec, c, q, q.a0, q.a0, q.a0, q.zz, q.scratch,
                           q.scratch + ld, q.sc, st)) != hipSuccess)
    return e;
  if ((e = launch_it_dots(c, q, q.zz, q.Wm, L, ID_DR, 1, st)) != hipSuccess) return e;
  if ((e = launch_it_solve(c, q, 1, st)) != hipSuccess) return e;
  // Steps 2-3 in n-space with a fresh Z~^T w (skipped when Step 1c kept wbar)
  if ((e = launch_gemvT(P->X_rec, P->st_rec, ld, c.n, q.w, q.w, q.partT, q.sc + 1, st)) !=
      hipSuccess)
    return e;
  if ((e = launch_it_reduceT(c, q, 2, st)) != hipSuccess) return e;
  // Z~ [xi - r, alpha, Z~^T w]
  if ((e = launch_it_zpass(P->X_rec, P->st_rec, c, q, q.a0, q.a1, q.a2, q.zz + ld,
                           q.zz + 2 * ld, q.zz + 3 * ld, q.sc, st)) != hipSuccess)
    return e;
  // Steps 2-3 in d-space, residuals, stopping and sigma rules
  if ((e = launch_it_dspace(c, q, 0, st)) != hipSuccess) return e;
  if ((e = launch_it_dspace(c, q, 1, st)) != hipSuccess) return e;
  return launch_it_tail(c, q, st);
}

dwd_status solve_iterative(Problem* P, const dwd_params* p, double* w, dwd_info* info,
                           double* alpha, double* r, double* xi, double* u, double* rho) {
  dwd_status s;
  if ((s = validate_params(p, true)) != DWD_OK) return s;
  if ((s = validate_penalty(p, P->n)) != DWD_OK) return s;
  if (p->representer) return fail(DWD_E_INVALID, "the representer iteration needs the SMW set-up");
  HIP_TRY_I(hipSetDevice(P->device));
  const hipStream_t st = P->stream;
  HIP_TRY_I(hipStreamSynchronize(st));
  HIP_TRY_I(P->set_penalty(p->e));
  HIP_TRY_I(hipEventRecord(P->ev_a, st));
  const Consts c = make_consts(P, p);
  const ItPtrs& q = P->ipt;
  HIP_TRY_I(launch_it_init(c, q, default_sigma0(p, P->n), st));
  const int chunk = std::max(1, p->check_every > 0 ? p->check_every : 8);
  volatile int32_t* hf = (volatile int32_t*)P->h_flags;
  int queued = 0, pending = -1;
  for (int cidx = 0;; ++cidx) {
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
    info->converged = hs.converged;
    info->setup_ms = P->setup_ms;
    info->solve_ms = ms;
    info->status = hs.converged ? DWD_OK : DWD_NOT_CONVERGED;
  }
  return hs.converged ? DWD_OK : DWD_NOT_CONVERGED;
}

}  // namespace dwd
