// Direct branch (Section 3.3.1): set-up of the (d+1) x (d+1) factor and the
// solve loop.  The kernels are in kernels_direct.hip.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dwd_solver.h"

namespace dwd {

#define HIP_TRY_D(expr)                                  \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
  } while (0)

int64_t direct_ld(int64_t d) { return (d + 15) / 16 * 16; }

// The solver choice printed with the paper's pseudo-code, with the direct
// factor only where this library builds it (dense X, FP32/FP64 storage).
int resolve_solver(const dwd_params* p, const dwd_matrix* X) {
  if (p->solver == DWD_SOLVER_DIRECT || p->solver == DWD_SOLVER_ITERATIVE) return p->solver;
  if (p->solver != DWD_SOLVER_AUTO) return DWD_SOLVER_SMW;
  // the choice printed with the paper's pseudo-code; sparse input and BF16
  // storage are taken by the SMW form only
  const bool dense = X->layout == DWD_DENSE && p->storage != DWD_BF16;
  if (!dense) return DWD_SOLVER_SMW;
  if (X->d <= 5000) return DWD_SOLVER_DIRECT;
  if ((double)X->n < 0.2 * (double)X->d && X->n <= 2500) return DWD_SOLVER_SMW;
  return DWD_SOLVER_ITERATIVE;
}

struct DirSizes {
  int64_t ld;
  int nblk, per_block, nred, splits;
  size_t factor_tmp;  // doubles of set-up scratch
};

static DirSizes dir_sizes(int64_t d, int n, int storage) {
  DirSizes z;
  z.ld = direct_ld(d);
  z.per_block = dir_sweep_samples_per_block(z.ld, n, storage);
  z.nblk = (n + z.per_block - 1) / z.per_block;
  z.nred = dir_reduce_blocks((int)d, 1);
  z.splits = fgram_splits((int)d, n);
  z.factor_tmp = std::max((size_t)z.splits * d * d, spd_inverse_work((int)d + 1));
  return z;
}

int64_t direct_footprint(int64_t d, int n, int storage) {
  const DirSizes z = dir_sizes(d, n, storage);
  const int64_t el = storage == DWD_FP64 ? 8 : 4;
  int64_t b = z.ld * n * el;                               // X
  b += (int64_t)n * 8 * 8;                                 // y, e, six n-vectors
  b += (d + 1) * (d + 1) * 8;                              // A^-1
  b += (z.ld * 8 + 2) * 8;                                 // d-vectors
  b += ((int64_t)z.nblk * (2 * z.ld + 2 * NPD) + z.nred) * 8;  // partials
  b += (int64_t)z.factor_tmp * 8;                          // set-up scratch
  return b;
}

dwd_status setup_direct(Problem* P, hipStream_t st) {
  const int n = P->n;
  const int64_t d = P->d, ld = P->ld;
  const DirSizes z = dir_sizes(d, n, P->st_rec);
  DirPtrs& dp = P->dp;
  auto alloc = [&](double** dst, size_t count) -> hipError_t {
    return P->alloc((void**)dst, std::max<size_t>(count, 1) * 8);
  };
  double* nv = nullptr;
  HIP_TRY_D(alloc(&nv, (size_t)n * 6));
  dp.r = nv;
  dp.xi = nv + n;
  dp.alpha = nv + 2 * (size_t)n;
  dp.zb = nv + 3 * (size_t)n;
  dp.rn = nv + 4 * (size_t)n;
  dp.dr = nv + 5 * (size_t)n;
  double* dv = nullptr;
  HIP_TRY_D(alloc(&dv, (size_t)ld * 8 + 2));
  dp.wbar = dv;                      // ld + 1
  dp.h = dv + ld + 1;                // ld + 1
  dp.w = dv + 2 * ld + 2;
  dp.u = dv + 3 * ld + 2;
  dp.rho = dv + 4 * ld + 2;
  dp.zz = dv + 5 * ld + 2;           // 3 ld
  HIP_TRY_D(hipMemsetAsync(dv, 0, ((size_t)ld * 8 + 2) * 8, st));
  HIP_TRY_D(alloc(&dp.part_d, (size_t)z.nblk * 2 * ld));
  HIP_TRY_D(alloc(&dp.part_n, (size_t)z.nblk * NPD));
  HIP_TRY_D(alloc(&dp.part_n2, (size_t)z.nblk * NPD));
  HIP_TRY_D(alloc(&dp.part_r, (size_t)z.nred));
  HIP_TRY_D(P->alloc((void**)&dp.sc, sizeof(Scal)));
  HIP_TRY_D(hipMemsetAsync(dp.sc, 0, sizeof(Scal), st));
  dp.nblk = z.nblk;
  dp.per_block = z.per_block;
  dp.nred = z.nred;
  dp.y = P->y;
  dp.e = P->e;
  double* A = nullptr;
  HIP_TRY_D(alloc(&A, (size_t)(d + 1) * (d + 1)));
  P->Ainv = A;
  dp.Ainv = A;

  // Z~ y = sum_i x_i / Z_scale (y_i^2 = 1), by the sweep kernel's plain mode
  Consts c{};
  c.d = d;
  c.ld = ld;
  c.n = n;
  c.inv_zs = 1.0 / P->zscale;
  HIP_TRY_D(launch_dir_sweep(P->X_rec, P->st_rec, c, dp, 0, st));
  HIP_TRY_D(launch_dir_reduce(c, dp, 0, 1, 1.0 / P->zscale, st));
  // A = [[Z~ Z~^T + mu I, Z~ y], [(Z~ y)^T, n]], then A^-1 in place
  double* tmp = nullptr;
  HIP_TRY_D(P->alloc_tmp((void**)&tmp, std::max<size_t>(z.factor_tmp, 1) * 8));
  hipError_t e = launch_fgram(P->X_rec, P->st_rec, ld, n, (int)d, tmp, z.splits, st);
  if (e == hipSuccess)
    e = launch_fgram_finish(tmp, z.splits, (int)d, n, dp.zz, 1.0 / (P->zscale * P->zscale),
                            P->mu, A, st);
  int* d_status = (int*)(P->d_scal + 8);
  if (e == hipSuccess) e = hipMemsetAsync(d_status, 0, 4, st);
  if (e == hipSuccess) e = spd_inverse_inplace(A, (int)d + 1, tmp, d_status, st);
  int hstat = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hstat, d_status, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) (void)hipStreamSynchronize(st);
  P->free_tmp(tmp);
  if (e != hipSuccess) return hip_fail(e, "direct factor");
  if (hstat != 0) return fail(DWD_E_NUMERIC, "factorisation of the (d+1)^2 matrix failed");
  return DWD_OK;
}

hipError_t queue_direct_iteration(Problem* P, const Consts& c, hipStream_t st) {
  const DirPtrs& dp = P->dp;
  const double inv_zs = 1.0 / P->zscale;
  hipError_t e;
  if ((e = launch_dir_gemv(c, dp, 0, st)) != hipSuccess) return e;
  if ((e = launch_dir_sweep(P->X_rec, P->st_rec, c, dp, 1, st)) != hipSuccess) return e;
  if ((e = launch_dir_reduce(c, dp, 0, 1, inv_zs, st)) != hipSuccess) return e;
  if ((e = launch_dir_gemv(c, dp, 1, st)) != hipSuccess) return e;
  if ((e = launch_dir_sweep(P->X_rec, P->st_rec, c, dp, 2, st)) != hipSuccess) return e;
  if ((e = launch_dir_reduce(c, dp, 1, 2, inv_zs, st)) != hipSuccess) return e;
  return launch_dir_tail(c, dp, st);
}

dwd_status solve_direct(Problem* P, const dwd_params* p, double* w, dwd_info* info,
                        double* alpha, double* r, double* xi, double* u, double* rho) {
  dwd_status s;
  if ((s = validate_params(p, true)) != DWD_OK) return s;
  if ((s = validate_penalty(p, P->n)) != DWD_OK) return s;
  if (p->representer == 1) return fail(DWD_E_INVALID, "the representer iteration needs the SMW set-up");
  HIP_TRY_D(hipSetDevice(P->device));
  const hipStream_t st = P->stream;
  HIP_TRY_D(hipStreamSynchronize(st));
  HIP_TRY_D(P->set_penalty(p->e));
  HIP_TRY_D(hipEventRecord(P->ev_a, st));
  const Consts c = make_consts(P, p);
  const DirPtrs& dp = P->dp;
  HIP_TRY_D(launch_dir_init(c, dp, default_sigma0(p, P->n), st));
  auto queue_iteration = [&]() -> hipError_t { return queue_direct_iteration(P, c, st); };
  // Chunks of check_every iterations; the stop flag of a chunk is read on
  // the host while the next chunk runs.
  const int chunk = std::max(1, p->check_every > 0 ? p->check_every : 8);
  volatile int32_t* hf = (volatile int32_t*)P->h_flags;
  int queued = 0, pending = -1;
  for (int cidx = 0;; ++cidx) {
    for (int j = 0; j < chunk && queued < c.max_iter; ++j, ++queued)
      HIP_TRY_D(queue_iteration());
    const int slot = cidx & 1;
    HIP_TRY_D(hipMemcpyAsync((void*)(hf + slot * 16), &dp.sc->done, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY_D(hipEventRecord(P->ev_chunk[slot], st));
    if (queued >= c.max_iter) break;
    if (pending >= 0) {
      HIP_TRY_D(hipEventSynchronize(P->ev_chunk[pending & 1]));
      if (hf[(pending & 1) * 16]) break;
    }
    pending = cidx;
  }
  HIP_TRY_D(hipEventRecord(P->ev_b, st));
  Scal hs;
  HIP_TRY_D(hipMemcpyAsync(&hs, dp.sc, sizeof(Scal), hipMemcpyDeviceToHost, st));
  HIP_TRY_D(hipStreamSynchronize(st));
  const int64_t d = P->d;
  if (w) {
    HIP_TRY_D(hipMemcpy(w, dp.w, d * 8, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < d; ++k) w[k] /= P->zscale;  // (as every other path unscales)
  }
  if (u) {
    HIP_TRY_D(hipMemcpy(u, dp.u, d * 8, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < d; ++k) u[k] /= P->zscale;
  }
  if (rho) HIP_TRY_D(hipMemcpy(rho, dp.rho, d * 8, hipMemcpyDeviceToHost));
  if (alpha) HIP_TRY_D(hipMemcpy(alpha, dp.alpha, (size_t)P->n * 8, hipMemcpyDeviceToHost));
  if (r) HIP_TRY_D(hipMemcpy(r, dp.r, (size_t)P->n * 8, hipMemcpyDeviceToHost));
  if (xi) HIP_TRY_D(hipMemcpy(xi, dp.xi, (size_t)P->n * 8, hipMemcpyDeviceToHost));
  // (the residuals of this branch come from explicit products, so the
  // check values are the in-loop ones; the rule is the same as elsewhere)
  const int conv =
      hs.converged && std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]) < p->tol ? 1 : 0;
  float ms = 0.0f;
  HIP_TRY_D(hipEventElapsedTime(&ms, P->ev_a, P->ev_b));
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
    info->status = conv ? DWD_OK : DWD_NOT_CONVERGED;
  }
  return conv ? DWD_OK : DWD_NOT_CONVERGED;
}

}  // namespace dwd
