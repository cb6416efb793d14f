// Iterative branch (Section 3.3.3): eq-linsys with the proximal term of eq-T
//     T = lam_ell I + sum_{j<ell} (lam_j - lam_ell) v_j v_j^T - Z~ Z~^T,
// so that the (1,1) block Z~ Z~^T + mu I + T = (mu + lam_ell) I +
// sum_{j<ell} (lam_j - lam_ell) v_j v_j^T has the closed-form inverse
//     (mu + lam_ell)^-1 I + sum_{j<ell} ((mu + lam_j)^-1 - (mu + lam_ell)^-1) v_j v_j^T,
// and [w; beta] follows from the Schur complement on beta (eq-schur) with
// g = (that inverse) Z~ y.  The eigenpairs come from Lanczos with full
// reorthogonalisation on Z~ Z~^T (set-up).
//
// Products with Z use the SMW layout: Z~^T v by the k_gemvT partials,
// reduced here; Z~ [a0, a1, a2] by a three-column pass split over samples as
// well as rows (k_it_zpass, below: n is large in this branch).  d-vectors are
// handled by grid-wide kernels over ld with block partials summed in a
// fixed order; every kernel of an iteration returns at once once the
// problem's stop flag is set.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "dwd_device.h"
#include "dwd_internal.h"
#include "dwd_iterative.h"

namespace dwd {

constexpr int DSTRIDE = kItMaxLanczos + 2;  // stride of the dot slots

// ---------------------------------------------------------------------------
// n-space: sum the Z~^T v partials over the 1024-row chunks (fixed order),
// z_i = y_i (X^T v)_i / Z_scale, then
//   mode 3 (Lanczos): a0 = z;
//   mode 1 (Step 1b): c = z + y betabar + xi - alpha/sigma, the prox, dr;
//                     a0 = dr (operand of Z~ dr);
//   mode 2 (Steps 2-3): z (fresh if Step 1c re-solved, else from mode 1),
//                     xi, alpha, the Section 4.3 terms; a0 = xi - r,
//                     a1 = alpha, a2 = z (operands of the next Z~ pass).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_it_reduceT(Consts c, ItPtrs p, int mode) {
  Scal* sc = p.sc;
  const int done = mode == 3 ? 0 : sc->done;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int n = c.n;
  const double sigma = mode == 3 ? 1.0 : sc->sigma;
  const int kk = mode == 3 ? 0 : sc->k;
  const int redo = mode == 2 ? sc->doubled : 1;
  const double beta = mode == 1 ? p.sca[IS_BETABAR] : (mode == 2 ? sc->beta : 0.0);
  if (done) return;
  double sums[10];
#pragma unroll
  for (int j = 0; j < 10; ++j) sums[j] = 0.0;
  if (i < n) {
    double z = 0.0;
    if (mode != 2 || redo) {
      double raw = 0.0;
      for (int ch = 0; ch < p.nchunks; ++ch) raw += p.partT[((size_t)ch * 2) * n + i];
      z = p.y[i] * raw * c.inv_zs;
    }
    if (mode == 3) {
      p.a0[i] = z;
    } else if (mode == 1) {
      const double yi = p.y[i], r0 = p.r[i];
      const double cc = z + yi * beta + p.xi[i] - p.alpha[i] / sigma;
      int steps = 0;
      const double tolN = eps_k(c, kk) / sqrt((double)n);
      const double rn = prox_weighted(cc, sigma, r0, tolN, loss_weight(c, yi), c, steps);
      const double dr = rn - r0;
      p.zb[i] = z;
      p.rn[i] = rn;
      p.dr[i] = dr;
      p.a0[i] = dr;
      sums[0] = yi * dr;
      sums[1] = (double)steps;
    } else {
      const double yi = p.y[i];
      const double zz = redo ? z : p.zb[i];
      const double rn = p.rn[i], al = p.alpha[i], ei = p.e[i];
      const double xin = fmax(0.0, rn - zz - yi * beta + (al - c.C * ei) / sigma);
      const double pres = zz + yi * beta + xin - rn;
      const double a1 = al - c.tau * sigma * pres;
      p.r[i] = rn;
      p.xi[i] = xin;
      p.alpha[i] = a1;
      p.z[i] = zz;
      p.a0[i] = xin - rn;
      p.a1[i] = a1;
      p.a2[i] = zz;
      double s9[9];
      nspace_sums(c, pow_q(rn, c), pow_qp1(rn, c), a1, xin, pres, yi, ei, s9);
#pragma unroll
      for (int j = 0; j < 9; ++j) sums[j] = s9[j];
      sums[9] = yi * (xin - rn);
    }
  }
  if (mode == 3) return;
  if (mode == 1) {
    // y^T dr summed; the Newton-step maximum
    double a[1] = {sums[0]};
    block_sum_k<256, 1>(a);
    double m = sums[1];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    __shared__ double smax[4];
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      p.part_n[(size_t)blockIdx.x * kItNpn + 0] = a[0];
      p.part_n[(size_t)blockIdx.x * kItNpn + 1] =
          fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
    }
    return;
  }
  block_sum_k<256, 10>(sums);
  if (threadIdx.x < 10) p.part_n2[(size_t)blockIdx.x * kItNpn + threadIdx.x] = sums[threadIdx.x];
}

hipError_t launch_it_reduceT(const Consts& c, const ItPtrs& p, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_it_reduceT, dim3((unsigned)p.nbn), dim3(256), 0, st, c, p, mode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dot products of x with `nrows` rows (stride ld) and, if `self`, with x
// itself (result index nrows), into dots[slot].  Blocks cover kItDotsBlock
// features each; wave j takes rows j, j+4, ...; a second one-block kernel
// sums the block partials in order.  For slot ID_DR it also sums y^T dr
// from the sweep-1 partials into index DSTRIDE - 1.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_it_dots(Consts c, ItPtrs p, const double* __restrict__ x,
                                                 const double* __restrict__ rows, int nrows,
                                                 int self, int check) {
  if (check && p.sc->done) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t f0 = (int64_t)blockIdx.x * kItDotsBlock;
  const int64_t f1 = min((int64_t)c.ld, f0 + kItDotsBlock);
  const int total = nrows + self;
  for (int r = wid; r < total; r += 4) {
    const double* v = r < nrows ? rows + (size_t)r * c.ld : x;
    double acc = 0.0;
    for (int64_t f = f0 + lane; f < f1; f += 64) acc = fma(v[f], x[f], acc);
    acc = wave_sum(acc);
    if (lane == 0) p.part_dd[(size_t)blockIdx.x * DSTRIDE + r] = acc;
  }
}

__global__ void __launch_bounds__(128) k_it_dots_reduce(ItPtrs p, int total, int slot,
                                                        int check) {
  if (check && p.sc->done) return;
  const int r = threadIdx.x;
  double* out = p.dots + (size_t)slot * DSTRIDE;
  if (r < total) {
    double s = 0.0;
    for (int b = 0; b < p.nbd; ++b) s += p.part_dd[(size_t)b * DSTRIDE + r];
    out[r] = s;
  }
  if (slot == ID_DR && r == 127) {
    double s = 0.0;
    for (int b = 0; b < p.nbn; ++b) s += p.part_n[(size_t)b * kItNpn + 0];
    out[DSTRIDE - 1] = s;
  }
}

hipError_t launch_it_dots(const Consts& c, const ItPtrs& p, const double* x, const double* rows,
                          int nrows, int slot, int self, hipStream_t st) {
  if (nrows + self > kItMaxLanczos + 1) return hipErrorInvalidValue;
  const int check = slot == ID_AUX ? 0 : 1;
  hipLaunchKernelGGL(k_it_dots, dim3((unsigned)p.nbd), dim3(256), 0, st, c, p, x, rows, nrows,
                     self, check);
  hipLaunchKernelGGL(k_it_dots_reduce, dim3(1), dim3(128), 0, st, p, nrows + self, slot, check);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Right-hand side of Step 1a with the proximal term:
//   h = -(Z~ (xi - r) - Z~ alpha / sigma) + mu u + sqrt(mu) rho / sigma + T w^k,
//   T w^k = lam_ell w + sum_{j<ell} (lam_j - lam_ell) (v_j^T w) v_j - Z~ Z~^T w.
// (h_beta = -y^T t is kept in sca[IS_HB] by the tail.)
// ---------------------------------------------------------------------------
// (with_T = 0: the right-hand side of eq-linsys itself, for the PSQMR solves)
__global__ void __launch_bounds__(256) k_it_rhs(Consts c, ItPtrs p, int with_T) {
  Scal* sc = p.sc;
  const int done = sc->done;
  const double sigma = sc->sigma;
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (done || f >= c.ld) return;
  const double* zxr = p.zz + c.ld;
  const double* za = p.zz + 2 * c.ld;
  double tw = 0.0;
  if (with_T) {
    const int L = p.ell;
    const double lamL = p.lam[L - 1];
    const double* dw = p.dots + (size_t)ID_W * DSTRIDE;
    const double* zzw = p.zz + 3 * c.ld;
    tw = lamL * p.w[f];
    for (int j = 0; j < L - 1; ++j)
      tw = fma((p.lam[j] - lamL) * dw[j], p.Wm[(size_t)j * c.ld + f], tw);
    tw -= zzw[f];
  }
  p.h[f] = -(zxr[f] - za[f] / sigma) + c.mu * p.u[f] + c.sqmu * p.rho[f] / sigma + tw;
}

hipError_t launch_it_rhs(const Consts& c, const ItPtrs& p, hipStream_t st, int with_T) {
  hipLaunchKernelGGL(k_it_rhs, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, st, c, p,
                     with_T);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Closed-form solves of the T-modified system (eq-schur):
//   beta = (x_beta - g^T x_w) / schur,
//   w = x_w / (mu + lam_ell) + sum_{j<ell} ((mu+lam_j)^-1 - (mu+lam_ell)^-1) (v_j^T x_w) v_j
//       - beta g.
//   mode 0 (Step 1a): x = [h; h_beta] -> [wbar; betabar].
//   mode 1 (Step 1c): x = [Z~ dr; y^T dr]; the residual ||x|| decides (5 eps_k)
//     whether [w; beta] = [wbar; betabar] + solve(x) or [wbar; betabar].
//     It also sets p.skip's flag so that the fresh Z~^T w pass is skipped
//     when Step 1c kept wbar.
//   mode 2: mode 1 with the re-solve taken (the switch from PSQMR to the
//     proximal term inside Step 1c, decided by the PSQMR residual).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_it_solve(Consts c, ItPtrs p, Scal* skip, int mode) {
  Scal* sc = p.sc;
  const int done = sc->done;
  const int k = sc->k;
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (done) return;
  const int L = p.ell;
  const double lamL = p.lam[L - 1];
  const double* dx = p.dots + (size_t)(mode == 0 ? ID_H : ID_DR) * DSTRIDE;
  const double xb = mode == 0 ? p.sca[IS_HB] : dx[DSTRIDE - 1];
  const double schur = p.sca[IS_SCHUR];
  const double bsol = (xb - dx[L - 1]) / schur;
  int redo = 1;
  if (mode == 1) {
    const double res = sqrt(fmax(dx[L] + xb * xb, 0.0));  // dx[L] = ||Z~ dr||^2
    redo = res > 5.0 * eps_k(c, k) ? 1 : 0;
  }
  if (mode == 2) mode = 1;
  const double bbar = p.sca[IS_BETABAR];
  if (f < c.ld) {
    const double* x = mode == 0 ? p.h : p.zz;
    const double* g = p.Wm + (size_t)(L - 1) * c.ld;
    double v = x[f] / (c.mu + lamL);
    const double cl = 1.0 / (c.mu + lamL);
    for (int j = 0; j < L - 1; ++j)
      v = fma((1.0 / (c.mu + p.lam[j]) - cl) * dx[j], p.Wm[(size_t)j * c.ld + f], v);
    v -= bsol * g[f];
    if (mode == 0) {
      p.wbar[f] = v;
    } else {
      p.w[f] = redo ? p.wbar[f] + v : p.wbar[f];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (mode == 0) {
      p.sca[IS_BETABAR] = bsol;
    } else {
      sc->beta = redo ? bbar + bsol : bbar;
      sc->doubled = redo;
      sc->n_double += redo;
      p.sca[IS_YDR] = xb;
      skip->done = redo ? 0 : 1;
    }
  }
}

hipError_t launch_it_solve(const Consts& c, const ItPtrs& p, int mode, hipStream_t st) {
  // the skip flag lives in the Scal right after the problem's own
  hipLaunchKernelGGL(k_it_solve, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, st, c, p,
                     p.sc + 1, mode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Steps 2-3 in d-space, two phases:
//   phase 0: g = w - rho/(sigma sqrt(mu)), block partials of ||g||^2;
//   phase 1: every block sums those partials (same order), gamma =
//     min(1, R/||g||), u = gamma g, rho <- rho - tau sigma sqrt(mu) (w - u),
//     block partials of ||w-u||^2, ||w||^2, ||Z~ alpha + sqrt(mu) rho||^2,
//     ||Z~ alpha||^2.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_it_dspace(Consts c, ItPtrs p, int phase) {
  Scal* sc = p.sc;
  const int done = sc->done;
  const double sigma = sc->sigma;
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (done) return;
  const bool in = f < c.ld;
  const double w = in ? p.w[f] : 0.0, rho = in ? p.rho[f] : 0.0;
  const double g = w - rho / (sigma * c.sqmu);
  if (phase == 0) {
    const double s = block_sum<256>(g * g);
    if (threadIdx.x == 0) p.part_d[(size_t)blockIdx.x * 8 + 0] = s;
    return;
  }
  double g2 = 0.0;
  for (int b = threadIdx.x; b < p.nbd2; b += 256) g2 += p.part_d[(size_t)b * 8 + 0];
  g2 = block_sum<256>(g2);
  const double ng = sqrt(g2);
  const double gamma = ng <= c.R ? 1.0 : c.R / ng;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (in) {
    const double u = gamma * g;
    const double rn = rho - c.tau * sigma * c.sqmu * (w - u);
    p.u[f] = u;
    p.rho[f] = rn;
    const double za = p.zz[2 * c.ld + f];
    const double dres = za + c.sqmu * rn;
    acc[0] = (w - u) * (w - u);
    acc[1] = w * w;
    acc[2] = dres * dres;
    acc[3] = za * za;
  }
  block_sum_k<256, 4>(acc);
  if (threadIdx.x < 4) p.part_d[(size_t)blockIdx.x * 8 + 1 + threadIdx.x] = acc[threadIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) p.sca[IS_G2] = g2;
}

hipError_t launch_it_dspace(const Consts& c, const ItPtrs& p, int phase, hipStream_t st) {
  hipLaunchKernelGGL(k_it_dspace, dim3((unsigned)p.nbd2), dim3(256), 0, st, c, p, phase);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// End of the iteration (one block): the residuals of Section 4.3 from this
// iteration's explicit sums, the stopping and sigma rules, and h_beta of the
// next right-hand side.
// ---------------------------------------------------------------------------
constexpr int NTI = 512;

__global__ void __launch_bounds__(NTI) k_it_tail(Consts c, ItPtrs p) {
  Scal* sc = p.sc;
  if (sc->done) return;
  const int k0 = sc->k;
  const double sigma = sc->sigma;
  const int nm = sc->newton_max;
  constexpr int K = 14;
  double acc[K];
#pragma unroll
  for (int j = 0; j < K; ++j) acc[j] = 0.0;
  double nmax = 0.0;
  for (int b = threadIdx.x; b < p.nbn; b += NTI) {
#pragma unroll
    for (int j = 0; j < 10; ++j) acc[j] += p.part_n2[(size_t)b * kItNpn + j];
    nmax = fmax(nmax, p.part_n[(size_t)b * kItNpn + 1]);
  }
  for (int b = threadIdx.x; b < p.nbd2; b += NTI)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[10 + j] += p.part_d[(size_t)b * 8 + 1 + j];
  block_sum_k<NTI, K>(acc);
  {
    __shared__ double smax[NTI / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nmax = fmax(nmax, __shfl_xor(nmax, off, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = nmax;
    __syncthreads();
    double m = smax[0];
    for (int w = 1; w < NTI / 64; ++w) m = fmax(m, smax[w]);
    nmax = m;
  }
  if (threadIdx.x != 0) return;
  double red[R_COUNT];
  for (int j = 0; j < 9; ++j) red[R_PRES2 + j] = acc[j];
  red[R_WU2] = acc[10];
  red[R_W2] = acc[11];
  red[R_DRES2] = acc[12];
  red[R_ZA2] = acc[13];
  red[R_G2] = p.sca[IS_G2];
  red[R_RHO2] = 0.0;
  double e[E_COUNT];
  finish_etas(c, red, e);
  e[E_PCHK] = e[E_P];
  e[E_DCHK] = e[E_D];
  for (int j = 0; j < R_COUNT; ++j) sc->red[j] = red[j];
  for (int j = 0; j < E_COUNT; ++j) sc->eta[j] = e[j];
  if ((int)nmax > nm) sc->newton_max = (int)nmax;
  const int k1 = k0 + 1;
  sc->k = k1;
  bool stop = false;
  const double sig = stop_and_sigma(c, e, sigma, k1, &stop);
  if (stop) {
    sc->converged = 1;
    sc->done = 1;
  } else if (k1 >= c.max_iter) {
    sc->done = 1;
  }
  sc->sigma = sig;
  // h_beta = -y^T t, t = xi - r - alpha / sigma'
  p.sca[IS_HB] = -(acc[9] - acc[3] / sig);
}

hipError_t launch_it_tail(const Consts& c, const ItPtrs& p, hipStream_t st) {
  hipLaunchKernelGGL(k_it_tail, dim3(1), dim3(NTI), 0, st, c, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Initial point (r, xi, w, beta, u) = (1, 1, 0, 0, 0), (alpha, rho) = (0, 0);
// Z~^T w = 0 and the first right-hand side is 0.
// ---------------------------------------------------------------------------
__global__ void k_it_init(Consts c, ItPtrs p, double sigma0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < c.n) {
    p.r[i] = 1.0;
    p.xi[i] = 1.0;
    p.alpha[i] = 0.0;
    p.z[i] = 0.0;
  }
  if (i < c.ld) {
    p.w[i] = 0.0;
    p.wbar[i] = 0.0;
    p.u[i] = 0.0;
    p.rho[i] = 0.0;
    p.h[i] = 0.0;
    for (int j = 0; j < 4; ++j) p.zz[(size_t)j * c.ld + i] = 0.0;
  }
  if (i == 0) {
    Scal* s = p.sc;
    s->sigma = sigma0;
    s->beta = 0.0;
    s->beta_bar = 0.0;
    s->gamma = 1.0;
    s->ytdr = 0.0;
    s->beta1 = 0.0;
    s->u2 = 0.0;
    s->k = 0;
    s->done = 0;
    s->converged = 0;
    s->n_double = 0;
    s->newton_max = 0;
    s->doubled = 0;
    s->status = 0;
    s->frozen_iter = 0;
    s->redo = 0;
    for (int j = 0; j < R_COUNT; ++j) s->red[j] = 0.0;
    for (int j = 0; j < E_COUNT; ++j) s->eta[j] = 0.0;
    p.sc[1].done = 0;  // skip flag
    p.sca[IS_HB] = 0.0;
    p.sca[IS_BETABAR] = 0.0;
  }
}

hipError_t launch_it_init(const Consts& c, const ItPtrs& p, double sigma0, hipStream_t st) {
  const int64_t m = std::max<int64_t>(c.n, c.ld);
  hipLaunchKernelGGL(k_it_init, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, c, p,
                     sigma0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Set-up.
// ---------------------------------------------------------------------------
// Lanczos start vector: entry f (0-based) = frac((f + 1) * 0.6180339887498949)
// - 0.5 for f < d, 0 in the padding (normalised by the caller).
__global__ void k_it_start(Consts c, double* __restrict__ v) {
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= c.ld) return;
  double x = 0.0;
  if (f < c.d) {
    const double t = (double)(f + 1) * 0.6180339887498949;
    x = (t - floor(t)) - 0.5;
  }
  v[f] = x;
}

hipError_t launch_it_lanczos_start(const Consts& c, double* v0, double*, int, hipStream_t st) {
  hipLaunchKernelGGL(k_it_start, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, st, c, v0);
  return hipGetLastError();
}

// w <- w - sum_{j<nrows} coef_j V_j (the sum formed first, then subtracted)
__global__ void k_it_orth(Consts c, double* __restrict__ w, const double* __restrict__ V,
                          int nrows, const double* __restrict__ coef) {
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= c.ld) return;
  double s = 0.0;
  for (int j = 0; j < nrows; ++j) s = fma(V[(size_t)j * c.ld + f], coef[j], s);
  w[f] -= s;
}

hipError_t launch_it_orth(const Consts& c, double* w, const double* V, int nrows,
                          const double* coef, hipStream_t st) {
  hipLaunchKernelGGL(k_it_orth, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, st, c, w, V,
                     nrows, coef);
  return hipGetLastError();
}

// out = in / sqrt(*nrm2) (0 if the norm vanishes)
__global__ void k_it_scale(Consts c, double* __restrict__ out, const double* __restrict__ in,
                           const double* __restrict__ nrm2) {
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= c.ld) return;
  const double nr = sqrt(fmax(*nrm2, 0.0));
  out[f] = nr > 1e-300 ? in[f] / nr : 0.0;
}

hipError_t launch_it_scale(const Consts& c, double* out, const double* in, const double* nrm2,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_it_scale, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, st, c, out,
                     in, nrm2);
  return hipGetLastError();
}

// Eigenpairs of the m x m Lanczos tridiagonal (diagonal alpha, off-diagonal
// sqrt(beta2)) by cyclic Jacobi rotations on one wave, the matrix and the
// rotations in LDS (m <= 64): lane k applies each rotation to row k of the
// columns p, q, then to column k of the rows p, q, then to row k of the
// accumulated rotations.  lam[0..ell) descending, S[j * ell + i] = component
// j of the eigenvector of lam[i]; S[m * ell + i] holds the chosen index.
__global__ void __launch_bounds__(64) k_it_eig(const double* __restrict__ alpha,
                                               const double* __restrict__ beta2, int m, int ell,
                                               double* __restrict__ lam, double* __restrict__ S) {
  __shared__ double A[kItMaxLanczos][kItMaxLanczos + 1];
  __shared__ double Q[kItMaxLanczos][kItMaxLanczos + 1];
  const int k = threadIdx.x;
  const bool on = k < m;
  for (int j = 0; j < kItMaxLanczos; ++j) {
    A[k][j] = 0.0;
    Q[k][j] = k == j ? 1.0 : 0.0;
  }
  if (on) {
    A[k][k] = alpha[k];
    if (k + 1 < m) A[k][k + 1] = sqrt(fmax(beta2[k], 0.0));
    if (k > 0) A[k][k - 1] = sqrt(fmax(beta2[k - 1], 0.0));
  }
  __syncthreads();
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, dia = 0.0;
    if (on) {
      dia = A[k][k] * A[k][k];
      for (int j = k + 1; j < m; ++j) off += A[k][j] * A[k][j];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      dia += __shfl_xor(dia, o, 64);
    }
    if (off <= 1e-32 * dia) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p][q];
        if (fabs(apq) <= 1e-300) continue;  // uniform: every lane reads the same value
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        __syncthreads();
        if (on) {  // columns p, q of row k
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = cs * akp - sn * akq;
          A[k][q] = sn * akp + cs * akq;
        }
        __syncthreads();
        if (on) {  // rows p, q of column k
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = cs * apk - sn * aqk;
          A[q][k] = sn * apk + cs * aqk;
          const double qkp = Q[k][p], qkq = Q[k][q];
          Q[k][p] = cs * qkp - sn * qkq;
          Q[k][q] = sn * qkp + cs * qkq;
        }
        __syncthreads();
      }
  }
  // the ell largest, descending (selection by repeated maxima)
  __shared__ int chosen[kItMaxEll];
  for (int i = 0; i < ell; ++i) {
    if (k == 0) {
      int best = -1;
      double bv = -DBL_MAX;
      for (int j = 0; j < m; ++j) {
        bool used = false;
        for (int t = 0; t < i; ++t) used = used || chosen[t] == j;
        if (!used && A[j][j] > bv) {
          bv = A[j][j];
          best = j;
        }
      }
      chosen[i] = best;
      S[(size_t)m * ell + i] = (double)best;
      lam[i] = bv;
    }
    __syncthreads();
    if (on) S[(size_t)k * ell + i] = Q[k][chosen[i]];
    __syncthreads();
  }
}

hipError_t launch_it_eig(const double* alpha, const double* beta, int m, int ell, double* lam,
                         double* S, hipStream_t st) {
  // S holds m * ell entries plus ell index slots
  if (m < 1 || m > kItMaxLanczos || ell < 1 || ell > kItMaxEll || ell > m)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_it_eig, dim3(1), dim3(64), 0, st, alpha, beta, m, ell, lam, S);
  return hipGetLastError();
}

// Ritz vectors: Wm[i] = sum_j V_j S[j][i] for i < ell - 1
__global__ void k_it_ritz(Consts c, const double* __restrict__ V, int m,
                          const double* __restrict__ S, int ell, double* __restrict__ Wm) {
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= c.ld) return;
  for (int i = 0; i < ell - 1; ++i) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s = fma(V[(size_t)j * c.ld + f], S[(size_t)j * ell + i], s);
    Wm[(size_t)i * c.ld + f] = s;
  }
}

hipError_t launch_it_ritz(const Consts& c, const double* V, int m, const double* S, int ell,
                          double* Wm, hipStream_t st) {
  hipLaunchKernelGGL(k_it_ritz, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, st, c, V, m,
                     S, ell, Wm);
  return hipGetLastError();
}

// g = (closed-form inverse) Z~ y into Wm row ell-1; dots[ID_AUX] must hold
// v_j^T Z~ y (j < ell - 1).
__global__ void k_it_gvec(Consts c, ItPtrs p, const double* __restrict__ Zy) {
  const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= c.ld) return;
  const int L = p.ell;
  const double lamL = p.lam[L - 1];
  const double cl = 1.0 / (c.mu + lamL);
  const double* dz = p.dots + (size_t)ID_AUX * DSTRIDE;
  double v = Zy[f] * cl;
  for (int j = 0; j < L - 1; ++j)
    v = fma((1.0 / (c.mu + p.lam[j]) - cl) * dz[j], p.Wm[(size_t)j * c.ld + f], v);
  p.Wm[(size_t)(L - 1) * c.ld + f] = v;
}

// schur = y^T y - (Z~ y)^T g with dots[ID_AUX][0] = (Z~ y)^T g
__global__ void k_it_schur(Consts c, ItPtrs p) {
  if (threadIdx.x == 0) p.sca[IS_SCHUR] = (double)c.n - p.dots[(size_t)ID_AUX * DSTRIDE];
}

hipError_t launch_it_gvec(const Consts& c, const ItPtrs& p, const double* Zy, hipStream_t st) {
  hipLaunchKernelGGL(k_it_gvec, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, st, c, p, Zy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_it_dots(c, p, Zy, p.Wm + (size_t)(p.ell - 1) * c.ld, 1, ID_AUX, 0, st)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_it_schur, dim3(1), dim3(64), 0, st, c, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Z~ [a0, a1, a2] split over samples as well as rows (n is large here, so
// row panels alone give too few blocks): block (panel, s) sums its share of
// the samples into part3[(s*3 + q)*ld + row]; the second kernel adds the
// shares in order.
// ---------------------------------------------------------------------------
constexpr int ZP_PANEL = 1024;

template <typename T>
__global__ void __launch_bounds__(256) k_it_zpass(const T* __restrict__ X, Consts c, ItPtrs p,
                                                  const double* __restrict__ a0,
                                                  const double* __restrict__ a1,
                                                  const double* __restrict__ a2,
                                                  const Scal* __restrict__ sc) {
  if (sc && sc->done) return;
  constexpr int V = Vec<T>::N;
  constexpr int ROWS = 64 * V;
  __shared__ double sv[3][ZP_PANEL];
  __shared__ double red[4][3][ROWS];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * ROWS;
  const T* xrow = X + rbase + lane * V;
  const int S = gridDim.y;
  const int per = (c.n + S - 1) / S;
  const int s0 = blockIdx.y * per, s1 = min(c.n, s0 + per);
  double acc[3][V];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int e = 0; e < V; ++e) acc[j][e] = 0.0;
  for (int pc = s0; pc < s1; pc += ZP_PANEL) {
    const int pn = min(ZP_PANEL, s1 - pc);
    for (int i = threadIdx.x; i < pn; i += 256) {
      const double yz = p.y[pc + i] * c.inv_zs;
      sv[0][i] = yz * a0[pc + i];
      sv[1][i] = yz * a1[pc + i];
      sv[2][i] = yz * a2[pc + i];
    }
    __syncthreads();
    const int pw = (pn + 3) / 4;
    const int j0 = wid * pw, j1 = min(pn, j0 + pw);
    int j = j0;
    // four columns in flight per lane, then their products in column order
    for (; j + 4 <= j1; j += 4) {
      typename Vec<T>::raw_t xr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xr[u] = Vec<T>::raw(xrow + (int64_t)(pc + j + u) * c.ld);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double x[V];
        Vec<T>::cvt(xr[u], x);
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int e = 0; e < V; ++e) acc[q][e] = fma(x[e], sv[q][j + u], acc[q][e]);
      }
    }
    for (; j < j1; ++j) {
      double x[V];
      Vec<T>::load(xrow + (int64_t)(pc + j) * c.ld, x);
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int e = 0; e < V; ++e) acc[q][e] = fma(x[e], sv[q][j], acc[q][e]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int e = 0; e < V; ++e) red[wid][q][lane * V + e] = acc[q][e];
  __syncthreads();
  for (int rr = threadIdx.x; rr < ROWS; rr += 256) {
    const int64_t k = rbase + rr;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      p.part3[((size_t)blockIdx.y * 3 + q) * c.ld + k] =
          (red[0][q][rr] + red[1][q][rr]) + (red[2][q][rr] + red[3][q][rr]);
  }
}

__global__ void __launch_bounds__(256) k_it_zreduce(Consts c, ItPtrs p, int S, double* o0,
                                                    double* o1, double* o2,
                                                    const Scal* __restrict__ sc) {
  if (sc && sc->done) return;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int q = blockIdx.y;
  if (k >= c.ld) return;
  double s = 0.0;
  for (int t = 0; t < S; ++t) s += p.part3[((size_t)t * 3 + q) * c.ld + k];
  (q == 0 ? o0 : (q == 1 ? o1 : o2))[k] = s;
}

int it_zpass_splits(int64_t ld, int n) {
  const int panels = (int)(ld / 256);
  int S = (2048 + panels - 1) / panels;
  S = std::min(S, std::max(1, (n + 255) / 256));
  return std::max(1, std::min(S, 256));
}

hipError_t launch_it_zpass(const void* X, int storage, const Consts& c, const ItPtrs& p,
                           const double* a0, const double* a1, const double* a2, double* o0,
                           double* o1, double* o2, const Scal* sc, hipStream_t st) {
  const int S = p.zsplits;
  const int rows = storage == DWD_FP64 ? 128 : 256;
  if (storage == DWD_FP64)
    hipLaunchKernelGGL(k_it_zpass<double>, dim3((unsigned)(c.ld / rows), S), dim3(256), 0, st,
                       (const double*)X, c, p, a0, a1, a2, sc);
  else if (storage == DWD_FP32)
    hipLaunchKernelGGL(k_it_zpass<float>, dim3((unsigned)(c.ld / rows), S), dim3(256), 0, st,
                       (const float*)X, c, p, a0, a1, a2, sc);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_it_zreduce, dim3((unsigned)((c.ld + 255) / 256), 3), dim3(256), 0, st, c,
                     p, S, o0, o1, o2, sc);
  return hipGetLastError();
}

__global__ void k_it_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) dst[i] = src[i];
}

hipError_t launch_it_copy(double* dst, const double* src, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_it_copy, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, dst, src,
                     count);
  return hipGetLastError();
}

}  // namespace dwd
