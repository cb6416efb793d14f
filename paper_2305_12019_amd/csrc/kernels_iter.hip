// Kernels of one iteration of Algorithm 1 (Steps 1a, 1b, 1c, 2, 3) on the
// scaled problem eq-gen-scale, with the linear system eq-linsys solved in
// n-space.  Writing v = Z~^T w + beta y and s = t + v with
// t = xi - r - alpha/sigma, the system A [w; beta] = hbar is equivalent to
//     w = (b - Z~ s) / mu,            b = mu u + sqrt(mu) rho / sigma,
//     s = M^-1 (t + Z~^T b / mu) + beta M^-1 y,   beta = -y^T f / y^T M^-1 y,
// with M = I + Z~^T Z~ / mu and f = M^-1 (t + Z~^T b / mu).  This is the
// Sherman-Morrison-Woodbury solve of Section 3.3.2 with the explicit M^-1
// (formed once) in place of two triangular solves per use; Z~^T w~bar + y
// beta~bar, needed by Step 1b, is v itself, so no extra pass over Z is
// needed, and the Step 1c residual ||h - A [wbar; betabar]|| equals
// sqrt(dr^T G~ dr + (y^T dr)^2) with dr = r^{k+1} - r^k.
//
// Every kernel returns at once when the problem's stop flag is set, so the
// host may queue iterations ahead of reading the flag.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "dwd_device.h"
#include "dwd_internal.h"

namespace dwd {


// ---------------------------------------------------------------------------
// Pass over Z, transposed: part[(chunk*2 + 0)*n + c] = sum_{k in chunk} X_kc v1_k
// and likewise for v2.  A chunk is 1024 consecutive rows; each lane keeps its
// slice of v1 and v2 in registers and a wave walks CPW columns.
// grid = (ceil(n / (4*CPW)), ld / 1024), block = 256.
// ---------------------------------------------------------------------------
template <typename T, int CPW>
__global__ void __launch_bounds__(256) k_gemvT(const T* __restrict__ X, int64_t ld, int n,
                                               const double* __restrict__ v1,
                                               const double* __restrict__ v2,
                                               double* __restrict__ part,
                                               const Scal* __restrict__ sc) {
  if (sc && sc->done) return;
  constexpr int V = Vec<T>::N;
  constexpr int U = kLdAlign / (64 * V);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t k0 = (int64_t)blockIdx.y * kLdAlign;
  double a1[U * V], a2[U * V];
#pragma unroll
  for (int uu = 0; uu < U; ++uu)
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int64_t kk = k0 + (int64_t)(uu * 64 + lane) * V + e;
      a1[uu * V + e] = v1[kk];
      a2[uu * V + e] = v2[kk];
    }
  const int cbase = (blockIdx.x * 4 + wid) * CPW;
  for (int j = 0; j < CPW; ++j) {
    const int c = cbase + j;
    if (c >= n) break;
    const T* col = X + (int64_t)c * ld + k0;
    double xv[U][V];
#pragma unroll
    for (int uu = 0; uu < U; ++uu) Vec<T>::load(col + (uu * 64 + lane) * V, xv[uu]);
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int uu = 0; uu < U; ++uu)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        s1 = fma(xv[uu][e], a1[uu * V + e], s1);
        s2 = fma(xv[uu][e], a2[uu * V + e], s2);
      }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      part[((int64_t)blockIdx.y * 2) * n + c] = s1;
      part[((int64_t)blockIdx.y * 2 + 1) * n + c] = s2;
    }
  }
}

constexpr int kCPW = 16;

template <typename T>
static hipError_t gemvT_t(const void* X, int64_t ld, int n, const double* v1, const double* v2,
                          double* part, const Scal* sc, hipStream_t st) {
  dim3 grid((n + 4 * kCPW - 1) / (4 * kCPW), (unsigned)(ld / kLdAlign));
  hipLaunchKernelGGL((k_gemvT<T, kCPW>), grid, dim3(256), 0, st, (const T*)X, ld, n, v1, v2, part,
                     sc);
  return hipGetLastError();
}

// Every pointer a kernel dereferences unconditionally must be non-NULL; the
// launchers refuse to launch otherwise.
bool iter_ptrs_ok(const IterPtrs& p) {
  const void* req[] = {p.y, p.my, p.Minv, p.G, p.r, p.xi, p.alpha, p.Pu, p.Prho, p.t, p.x,
                       p.f, p.s, p.v, p.dr, p.hG, p.rn, p.s1, p.v1, p.xi0, p.xi1, p.al0,
                       p.al1, p.au, p.arho, p.aw, p.au_n, p.arho_n, p.stg, p.u, p.rho, p.w,
                       p.part_g,
                       p.part_n1,
                       p.part_it, p.part_c, p.partT, p.sc};
  for (const void* q : req)
    if (!q) return false;
  return p.pg_ld >= 1;
}

hipError_t launch_gemvT(const void* X, int storage, int64_t ld, int n, const double* v1,
                        const double* v2, double* part, const Scal* sc, hipStream_t st) {
  if (!X || !v1 || !v2 || !part || ld % kLdAlign != 0) return hipErrorInvalidValue;
  if (storage == DWD_FP64) return gemvT_t<double>(X, ld, n, v1, v2, part, sc, st);
  if (storage == DWD_FP32) return gemvT_t<float>(X, ld, n, v1, v2, part, sc, st);
  return gemvT_t<uint16_t>(X, ld, n, v1, v2, part, sc, st);
}

// ---------------------------------------------------------------------------
// Initial point (r, xi, w, beta, u) = (1, 1, 0, 0, 0), (alpha, rho) = (0, 0).
// ---------------------------------------------------------------------------
__global__ void k_init(Consts c, IterPtrs p, double sigma0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < c.n) {
    p.r[i] = 1.0;
    p.xi[i] = 1.0;
    p.alpha[i] = 0.0;
    p.Pu[i] = 0.0;
    p.Prho[i] = 0.0;
    p.au[i] = 0.0;
    p.arho[i] = 0.0;
    p.aw[i] = 0.0;
  }
  if (i < c.ld) {
    p.u[i] = 0.0;
    p.rho[i] = 0.0;
    p.w[i] = 0.0;
  }
  if (i == 0) {
    Scal* s = p.sc;
    s->sigma = sigma0;
    s->beta = 0.0;
    s->beta_bar = 0.0;
    s->gamma = 1.0;
    s->ytdr = 0.0;
    s->k = 0;
    s->done = 0;
    s->converged = 0;
    s->n_double = 0;
    s->newton_max = 0;
    s->doubled = 0;
    s->status = 0;
    s->frozen_iter = 0;
    s->u2 = 0.0;
    for (int j = 0; j < R_COUNT; ++j) s->red[j] = 0.0;
    for (int j = 0; j < E_COUNT; ++j) s->eta[j] = 0.0;
  }
}

hipError_t launch_init(const Consts& c, const IterPtrs& p, double sigma0, hipStream_t st) {
  const int64_t m = c.ld > c.n ? c.ld : c.n;
  hipLaunchKernelGGL(k_init, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, c, p, sigma0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 1a, right-hand side in n-space.  If `fresh`, Z~^T u and Z~^T rho come
// from the pass partials (y_i / Z_scale folded in); otherwise from the
// recurrences kept by the tail kernel.  Then p = Z~^T b, t and x = t + p/mu.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rhs(Consts c, IterPtrs p, int nchunks, int fresh) {
  if (p.sc->done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  double Pu, Pr;
  if (fresh) {
    double su = 0.0, sr = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) {
      su += p.partT[((int64_t)ch * 2) * c.n + i];
      sr += p.partT[((int64_t)ch * 2 + 1) * c.n + i];
    }
    const double yi = p.y[i] * c.inv_zs;
    Pu = yi * su;
    Pr = yi * sr;
    p.Pu[i] = Pu;
    p.Prho[i] = Pr;
  } else {
    Pu = p.Pu[i];
    Pr = p.Prho[i];
  }
  const double sigma = p.sc->sigma;
  const double pb = c.mu * Pu + c.sqmu * Pr / sigma;
  const double t = p.xi[i] - p.r[i] - p.alpha[i] / sigma;
  p.t[i] = t;
  p.x[i] = t + pb / c.mu;
}

hipError_t launch_rhs(const Consts& c, const IterPtrs& p, int nchunks, int fresh, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs, dim3((c.n + 255) / 256), dim3(256), 0, st, c, p, nchunks, fresh);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// n x n FP64 products: o1 = A1 x1 and, if A2, o2 = A2 x2; one wave per row.
// part[block] = sum over the block's rows of wdot_i * o1_i.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_ngemv(int n, const double* __restrict__ A1,
                                               const double* __restrict__ x1,
                                               double* __restrict__ o1,
                                               const double* __restrict__ A2,
                                               const double* __restrict__ x2,
                                               double* __restrict__ o2,
                                               const double* __restrict__ wdot,
                                               double* __restrict__ part,
                                               const Scal* __restrict__ sc) {
  if (sc && sc->done) return;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wid;
  double contrib = 0.0;
  if (row < n) {
    const double* a = A1 + (size_t)row * n;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int j = lane;
    for (; j + 192 < n; j += 256) {
      s0 = fma(a[j], x1[j], s0);
      s1 = fma(a[j + 64], x1[j + 64], s1);
      s2 = fma(a[j + 128], x1[j + 128], s2);
      s3 = fma(a[j + 192], x1[j + 192], s3);
    }
    for (; j < n; j += 64) s0 = fma(a[j], x1[j], s0);
    double acc = wave_sum((s0 + s1) + (s2 + s3));
    if (lane == 0) o1[row] = acc;
    contrib = wdot ? wdot[row] * acc : 0.0;
    if (A2) {
      const double* b = A2 + (size_t)row * n;
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
      j = lane;
      for (; j + 192 < n; j += 256) {
        t0 = fma(b[j], x2[j], t0);
        t1 = fma(b[j + 64], x2[j + 64], t1);
        t2 = fma(b[j + 128], x2[j + 128], t2);
        t3 = fma(b[j + 192], x2[j + 192], t3);
      }
      for (; j < n; j += 64) t0 = fma(b[j], x2[j], t0);
      const double acc2 = wave_sum((t0 + t1) + (t2 + t3));
      if (lane == 0) o2[row] = acc2;
    }
  }
  __shared__ double wpart[4];
  if (lane == 0) wpart[wid] = contrib;
  __syncthreads();
  if (threadIdx.x == 0 && part) part[blockIdx.x] = (wpart[0] + wpart[1]) + (wpart[2] + wpart[3]);
}


hipError_t launch_ngemv(int n, const double* A1, const double* x1, double* o1, const double* A2,
                        const double* x2, double* o2, const double* wdot, double* part,
                        const Scal* sc, hipStream_t st) {
  if (!A1 || !x1 || !o1 || (A2 && (!x2 || !o2))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ngemv, dim3(ngemv_blocks(n)), dim3(256), 0, st, n, A1, x1, o1, A2, x2, o2,
                     wdot, part, sc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 1a (solve) fused with Step 1b (prox).  One wave per row i:
//   f_i = (M^-1 x)_i,  beta_bar = -y^T M^-1 x / y^T M^-1 y = -(M^-1 y)^T x / y^T M^-1 y
// (M^-1 is symmetric, so every wave forms beta_bar from x directly, with the
// loads of its row and in the same order), s_bar = f + beta_bar M^-1 y,
// v_bar = s_bar - t,
// c = v_bar + xi - alpha/sigma, r^{k+1}_i = prox(c_i), dr = r^{k+1} - r^k.
// Block partials: y^T dr and the most Newton steps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void step1ab_body(const Consts& c, const IterPtrs& p) {
  Scal* sc = p.sc;
  // (the stop flag, uniform over the launch, is tested once the first loads
  // are in flight; nothing is written before the test)
  const int done = sc->done;
  __shared__ double wy[4];
  __shared__ int ws[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wid;
  const bool mine = row < c.n && lane == 0;
  // per-row operands, loaded before the reductions
  double myr = 0.0, tr = 0.0, xir = 0.0, alr = 0.0, r0 = 1.0, yr = 0.0;
  if (mine) {
    myr = p.my[row];
    tr = p.t[row];
    xir = p.xi[row];
    alr = p.alpha[row];
    r0 = p.r[row];
    yr = p.y[row];
  }
  const double sigma = sc->sigma;
  const int kk = sc->k;
  if (done) return;
  double f = 0.0, mx = 0.0;
  if (row < c.n) wave_row_dot2(p.Minv + (size_t)row * c.n, p.my, p.x, c.n, lane, f, mx);
  const double beta_bar = -mx / c.ymy;
  double ydr = 0.0;
  int steps = 0;
  if (mine) {
    const double tolN = eps_k(c, kk) / sqrt((double)c.n);
    const double s = f + beta_bar * myr;
    const double v = s - tr;
    const double cc = v + xir - alr / sigma;
    const double rn = prox_weighted(cc, sigma, r0, tolN, loss_weight(c, yr), c, steps);
    const double dr = rn - r0;
    p.f[row] = f;
    p.s[row] = s;
    p.v[row] = v;
    p.rn[row] = rn;
    p.dr[row] = dr;
    ydr = yr * dr;
  }
  if (lane == 0) {
    wy[wid] = ydr;
    ws[wid] = steps;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    p.part_n1[blockIdx.x] = (wy[0] + wy[1]) + (wy[2] + wy[3]);
    p.part_it[blockIdx.x] = (double)max(max(ws[0], ws[1]), max(ws[2], ws[3]));
    if (blockIdx.x == 0) sc->beta_bar = beta_bar;
  }
}

__global__ void __launch_bounds__(256) k_step1ab(Consts c, IterPtrs p) { step1ab_body(c, p); }

hipError_t launch_step1ab(const Consts& c, const IterPtrs& p, hipStream_t st) {
  hipLaunchKernelGGL(k_step1ab, dim3(ngemv_blocks(c.n)), dim3(256), 0, st, c, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 1c, row-parallel.  One wave per row i forms (G~ dr)_i and (M^-1 dr)_i,
// and with the same round of loads (M^-1 y)^T dr.
// The test ||h - A [wbar; betabar]||^2 = dr^T G~ dr + (y^T dr)^2 <= (5 eps_k)^2
// needs a global sum, so each row prepares both outcomes:
//   0: keep Step 1a's solution:  s0 = s_bar = M^-1 (x + beta_bar y), v0 = v_bar;
//   1: solve again with r^{k+1}: s1 = M^-1 (x - dr + beta1 y) with
//      beta1 = beta_bar + (M^-1 y)^T dr / y^T M^-1 y,  v1 = s1 - (t - dr);
// and, for each, Step 2 (xi) and Step 3 (alpha) in n-space:
//   xi_o = max(0, r^{k+1} - v_o + (alpha - C)/sigma),
//   alpha_o = alpha - tau sigma (v_o + xi_o - r^{k+1}),
// the nine n-space sums of Section 4.3, and the two terms of
//   ||g||^2 = ||u||^2 - 2/mu (Z~^T u)^T s_o + s_o^T G~ s_o / mu^2
// (g = w - rho/(sigma sqrt(mu)) = u - Z~ s_o / mu), where
// G~ s_o = mu (x_o + beta_o y - s_o) because G~ M^-1 = mu (I - M^-1).
// The consumers take the decision from the same fixed-order sums.
// Slot 0 of part_c = block sum of dr_i (G~ dr)_i; slot 1 + o*NPO + j outcome o.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void step1c_body(const Consts& c, const IterPtrs& p) {
  Scal* sc = p.sc;
  const int done = sc->done;  // tested after the first loads (see k_step1ab)
  __shared__ double wsum[4][NPC];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wid;
  const bool mine = row < c.n && lane == 0;
  double dr = 0.0, rn = 1.0, a0 = 0.0, yi = 0.0, xr = 0.0, pu = 0.0, s0 = 0.0, v0 = 0.0;
  double f0 = 0.0, my0 = 0.0, t0 = 0.0, ei = 1.0;
  if (mine) {
    dr = p.dr[row];
    rn = p.rn[row];
    a0 = p.alpha[row];
    yi = p.y[row];
    xr = p.x[row];
    pu = p.Pu[row];
    s0 = p.s[row];
    v0 = p.v[row];
    f0 = p.f[row];
    my0 = p.my[row];
    t0 = p.t[row];
    ei = p.e[row];
  }
  const double sigma = sc->sigma;
  const double beta_bar = sc->beta_bar;
  if (done) return;
  double hg = 0.0, hm = 0.0, mdr = 0.0;
  if (row < c.n)
    wave_row_dot3(p.G + (size_t)row * c.n, p.Minv + (size_t)row * c.n, p.my, p.dr, c.n, lane, hg,
                  hm, mdr);
  const double beta1 = beta_bar + mdr / c.ymy;
  double out[NPC];
#pragma unroll
  for (int j = 0; j < NPC; ++j) out[j] = 0.0;
  if (mine) {
    const double rq1 = pow_qp1(rn, c);
    const double rq = pow_q(rn, c);
    double al0s = 0.0;  // alpha of outcome 0
    out[0] = dr * hg;
    {  // outcome 0
      const double s = s0;
      const double v = v0;
      const double xi = fmax(0.0, rn - v + (a0 - c.C * ei) / sigma);
      const double pres = v + xi - rn;
      const double a1 = a0 - c.tau * sigma * pres;
      p.xi0[row] = xi;
      p.al0[row] = a1;
      al0s = a1;
      nspace_sums(c, rq, rq1, a1, xi, pres, yi, ei, out + 1);
      out[1 + 9] = s * (c.mu * (xr + beta_bar * yi - s));
      out[1 + 10] = pu * s;
    }
    {  // outcome 1
      const double s = f0 - hm + beta1 * my0;
      const double v = s - (t0 - dr);
      const double xi = fmax(0.0, rn - v + (a0 - c.C * ei) / sigma);
      const double pres = v + xi - rn;
      const double a1 = a0 - c.tau * sigma * pres;
      p.s1[row] = s;
      p.v1[row] = v;
      p.xi1[row] = xi;
      p.al1[row] = a1;
      nspace_sums(c, rq, rq1, a1, xi, pres, yi, ei, out + 1 + NPO);
      out[1 + NPO + 9] = s * (c.mu * (xr - dr + beta1 * yi - s));
      out[1 + NPO + 10] = pu * s;
      // the pass's operands of both outcomes, scaled by the label sign and
      // 1/Z_scale
      const double yz = yi * c.inv_zs;
      double* st = p.stg + 4 * (size_t)row;
      st[0] = yz * s0;
      st[1] = yz * s;
      st[2] = yz * al0s;
      st[3] = yz * a1;
    }
    p.hG[row] = hg;
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NPC; ++j) wsum[wid][j] = out[j];
  }
  __syncthreads();
  if (threadIdx.x < NPC) {
    const int j = threadIdx.x;
    p.part_c[(size_t)j * ngemv_blocks(c.n) + blockIdx.x] =
        (wsum[0][j] + wsum[1][j]) + (wsum[2][j] + wsum[3][j]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->beta1 = beta1;
}

__global__ void __launch_bounds__(256) k_step1c_rows(Consts c, IterPtrs p) { step1c_body(c, p); }

hipError_t launch_step1c_rows(const Consts& c, const IterPtrs& p, hipStream_t st) {
  hipLaunchKernelGGL(k_step1c_rows, dim3(ngemv_blocks(c.n)), dim3(256), 0, st, c, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pass over Z: zs = Z~ s and za = Z~ alpha^{k+1} row by row (the label signs
// and 1/Z_scale come with s and alpha from Step 1c), fused with Steps 2 and 3
// in d-space:
//   w = (b - zs)/mu,  b = mu u + sqrt(mu) rho / sigma,  g = w - rho/(sigma sqrt(mu)),
//   u <- gamma g,  rho <- rho - tau sigma sqrt(mu) (w - u),
// and block partials of ||w-u||^2, ||w||^2, ||za + sqrt(mu) rho||^2,
// ||za||^2, ||rho||^2, ||u||^2.  Block = NW waves over the same 64*V rows,
// wave j walks its quarter of the columns; partial row sums meet in LDS.
// ---------------------------------------------------------------------------
constexpr int PANEL = 2048;  // columns staged at a time by the representer step

// The n-space prediction of ||g|| that sizes the ball projection is exact
// for the data the pass streams: the data of record with its factor, or the
// BF16 image with the factor of the BF16 image (BF16 phase).
//
// The scaled operands of both Step 1c outcomes, (y_j / Z_scale) [s, s1,
// alpha0, alpha1]_j, come from Step 1c as four consecutive FP64 values per
// column (p.stg); a wave reads them with scalar loads at addresses common to
// its lanes, so the column loop needs no staging and no barrier, and starts
// as soon as the first data columns arrive.  Both outcomes are accumulated;
// the plan that picks one (and sizes Step 2) is formed after the loop, from
// partials loaded at the start.
template <typename T, int NW>
__device__ __forceinline__ void pass2_body(const T* __restrict__ X, const Consts& c,
                                           const IterPtrs& p) {
  // The stop flag is tested after the first loads are issued (nothing is
  // written before the test), so its round trip overlaps theirs.
  const int done = p.sc->done;
  constexpr int NT = NW * 64;
  constexpr int V = Vec<T>::N;
  constexpr int ROWS = 64 * V;
  constexpr int RPT = (ROWS + NT - 1) / NT;  // epilogue rows per thread
  constexpr int RB = (512 + NT - 1) / NT;    // plan partial blocks per thread (n <= 2048)
  __shared__ double lds[2 * NW * ROWS];      // the per-wave row sums
  double(*red)[2][ROWS] = reinterpret_cast<double(*)[2][ROWS]>(lds);
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int64_t rbase = (int64_t)blockIdx.x * ROWS;
  const T* xrow = X + rbase + lane * V;
  // this wave's columns
  const int per = (c.n + NW - 1) / NW;
  const int j0 = min(c.n, wid * per), j1 = min(c.n, j0 + per);
  // First loads, all unconditional (clamped indexes, the surplus discarded,
  // which keeps the waits counted exactly): the first four data columns,
  // the rows' u and rho for the epilogue, and the plan partials.
  typename Vec<T>::raw_t pf[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) pf[u] = Vec<T>::raw(xrow + (int64_t)min(j0 + u, c.n - 1) * c.ld);
  double u_in[RPT], rho_in[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int rr = min((int)threadIdx.x + q * NT, ROWS - 1);
    u_in[q] = p.u[rbase + rr];
    rho_in[q] = p.rho[rbase + rr];
  }
  const int nb = ngemv_blocks(c.n);
  const bool few = nb <= RB * NT;
  double raw[RB][6];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int b = min((int)threadIdx.x + r * NT, nb - 1);
#pragma unroll
    for (int j = 0; j < 6; ++j) raw[r][j] = plan_part(p, j, b, nb);
  }
  const int k_it = p.sc->k;
  const double u2 = p.sc->u2;
  if (done) return;
  // a*: Z~ s of outcome 0 / 1, b*: Z~ alpha of outcome 0 / 1
  double a0[V], a1[V], b0[V], b1[V];
#pragma unroll
  for (int e = 0; e < V; ++e) a0[e] = a1[e] = b0[e] = b1[e] = 0.0;
  // (a global-memory pointer: the serving form takes p from a descriptor in
  // memory, and a generic pointer could not be read with scalar loads)
  typedef __attribute__((address_space(1))) const double gdouble;
  const gdouble* __restrict__ stg = (const gdouble*)p.stg;
  auto column = [&](const double (&x)[V], int j) {
    const double s0 = stg[4 * j], s1 = stg[4 * j + 1];
    const double t0 = stg[4 * j + 2], t1 = stg[4 * j + 3];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      a0[e] = fma(x[e], s0, a0[e]);
      a1[e] = fma(x[e], s1, a1[e]);
      b0[e] = fma(x[e], t0, b0[e]);
      b1[e] = fma(x[e], t1, b1[e]);
    }
  };
  auto group = [&](const typename Vec<T>::raw_t (&xr)[4], int j) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double x[V];
      Vec<T>::cvt(xr[u], x);
      column(x, j + u);
    }
  };
  int j = j0;
  if (j0 + 4 <= j1) {
    group(pf, j);
    j += 4;
  }
  for (; j + 4 <= j1; j += 4) {
    typename Vec<T>::raw_t x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = Vec<T>::raw(xrow + (int64_t)(j + u) * c.ld);
    group(x, j);
  }
  for (; j < j1; ++j) {
    double x0[V];
    Vec<T>::load(xrow + (int64_t)j * c.ld, x0);
    column(x0, j);
  }
  // the plan (every block forms the same one)
  double a[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) a[q] = 0.0;
  if (few) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < 6; ++q)
        if (threadIdx.x + r * NT < nb) a[q] += raw[r][q];
  } else {
    for (int b = threadIdx.x; b < nb; b += NT)
#pragma unroll
      for (int q = 0; q < 6; ++q) a[q] += plan_part(p, q, b, nb);
  }
  block_sum_k<NT, 6>(a);
  const Step2Plan pl = step2_plan_finish(c, a, k_it, u2);
  publish_plan(p, pl);
#pragma unroll
  for (int e = 0; e < V; ++e) {
    red[wid][0][lane * V + e] = pl.redo ? a1[e] : a0[e];
    red[wid][1][lane * V + e] = pl.redo ? b1[e] : b0[e];
  }
  __syncthreads();
  const double sigma = p.sc->sigma;
  const double gamma = pl.gamma;
  const double br = c.sqmu / sigma, gr = 1.0 / (sigma * c.sqmu);
  const double rs = c.tau * sigma * c.sqmu;
  double acc[NP2] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int rr = threadIdx.x + q * NT;
    if (rr >= ROWS) break;
    double zs = 0.0, za = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      zs += red[ww][0][rr];
      za += red[ww][1][rr];
    }
    const int64_t k = rbase + rr;
    const double rho = rho_in[q];
    const double b = c.mu * u_in[q] + br * rho;
    const double w = (b - zs) / c.mu;
    p.w[k] = w;
    const double u = gamma * (w - gr * rho);
    const double rn = rho - rs * (w - u);
    p.u[k] = u;
    p.rho[k] = rn;
    const double dres = za + c.sqmu * rn;
    acc[0] += (w - u) * (w - u);
    acc[1] += w * w;
    acc[2] += dres * dres;
    acc[3] += za * za;
    acc[4] += rn * rn;
    acc[5] += u * u;
  }
  block_sum_k<NW * 64, NP2>(acc);
  if (threadIdx.x < NP2) p.part_g[(size_t)threadIdx.x * p.pg_ld + blockIdx.x] = acc[threadIdx.x];
}

template <typename T, int NW>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW == 8 ? 4 : 2)))
k_pass2(const T* __restrict__ X, Consts c, IterPtrs p) {
  pass2_body<T, NW>(X, c, p);
}

// Blocks of the pass: 64 V rows each (V = 2, 4, 8 for FP64, FP32, BF16).
int pass2_blocks(int storage, int64_t ld) {
  const int rows = storage == DWD_FP64 ? 128 : (storage == DWD_FP32 ? 256 : 512);
  return (int)(ld / rows);
}

// Four waves per block for every storage type: with the column-major X each
// wave visits 1 KB per column, and eight waves per block (twice the open
// column streams) read about 5% slower at d=1e5, n=1e3.
hipError_t launch_pass2(const void* X, int storage, const Consts& c, const IterPtrs& p,
                        hipStream_t st) {
  if (!X || !iter_ptrs_ok(p) || c.ld % kLdAlign != 0) return hipErrorInvalidValue;
  const int nb = pass2_blocks(storage, c.ld);
  if (nb > p.pg_ld) return hipErrorInvalidValue;
  if (storage == DWD_FP64)
    hipLaunchKernelGGL((k_pass2<double, 4>), dim3(nb), dim3(256), 0, st, (const double*)X, c, p);
  else if (storage == DWD_FP32)
    hipLaunchKernelGGL((k_pass2<float, 4>), dim3(nb), dim3(256), 0, st, (const float*)X, c, p);
  else
    hipLaunchKernelGGL((k_pass2<uint16_t, 4>), dim3(nb), dim3(256), 0, st, (const uint16_t*)X,
                       c, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Representer iteration (params.representer): with a zero start and T = 0,
// every d-vector stays in range(Z~) (Steps 2-3 combine u, rho and
// w = (b - Z~ s)/mu linearly), so the pass is replaced by n-space algebra on
// the coefficients u~ = Z~ au, rho = Z~ arho, w~ = Z~ aw:
//   aw = au + arho/(sigma sqrt(mu)) - s/mu,   Z~^T w~ = v - beta y,
//   au' = gamma (aw - arho/(sigma sqrt(mu))),  arho' = arho - tau sigma sqrt(mu) (aw - au'),
// with Z~^T u' and Z~^T rho' from the recurrences the tail also applies, and
// every d-space norm as a dot product of a coefficient vector with its image
// under G~: ||Z~ a||^2 = a^T (G~ a).  The one n x n product per iteration is
// G~ alpha' (for ||Z~ alpha'|| and ||Z~ alpha' + D rho'||).  One wave per
// row; the block partials have the layout of the pass's (NP2).  Every block
// stages cv from the whole of au and arho, so the new coefficients go to
// au_n and arho_n (committed by the tail): a block that starts after another
// has finished still reads this iteration's au and arho.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rep_step_body(const Consts& c, const IterPtrs& p) {
  Scal* sc = p.sc;
  const int done = sc->done;  // tested after the plan's loads (see k_step1ab)
  const Step2Plan pl = step2_plan<256>(c, p);
  if (done) return;
  publish_plan(p, pl);
  const int o = pl.redo;
  const double* al = o ? p.al1 : p.al0;
  const double* so = o ? p.s1 : p.s;
  const double sigma = sc->sigma;
  const double gamma = pl.gamma;
  const double gr = 1.0 / (sigma * c.sqmu);
  const double rs = c.tau * sigma * c.sqmu;
  // Staged in LDS for the block's rows: alpha' and cv = alpha' + sqrt(mu) arho',
  // the coefficients of Z~ alpha' + D rho'.  ||Z~ alpha' + D rho'||^2 is then
  // the quadratic form cv^T G~ cv of one vector (no cancellation between
  // separately rounded terms near the solution, where the residual is tiny).
  __shared__ double s_al[PANEL], s_cv[PANEL];
  __shared__ double ws[4][NP2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wid;
  double h = 0.0, g = 0.0;
  for (int pc = 0; pc < c.n; pc += PANEL) {
    const int pn = min(PANEL, c.n - pc);
    __syncthreads();
    for (int j = threadIdx.x; j < pn; j += 256) {
      const int jj = pc + j;
      const double au = p.au[jj], ar = p.arho[jj], sj = so[jj];
      const double aw = au + gr * ar - sj / c.mu;
      const double au1 = gamma * (aw - gr * ar);
      const double ar1 = ar - rs * (aw - au1);
      s_al[j] = al[jj];
      s_cv[j] = al[jj] + c.sqmu * ar1;
    }
    __syncthreads();
    if (row < c.n) {
      const double* Ar = p.G + (size_t)row * c.n + pc;
      for (int j = lane; j < pn; j += 64) {
        const double m = Ar[j];
        h = fma(m, s_al[j], h);
        g = fma(m, s_cv[j], g);
      }
    }
  }
  h = wave_sum(h);
  g = wave_sum(g);
  double acc[NP2] = {0, 0, 0, 0, 0, 0};
  if (row < c.n && lane == 0) {
    const double beta = o ? sc->beta1 : sc->beta_bar;
    const double s = so[row];
    const double v = o ? p.v1[row] : p.v[row];
    const double au = p.au[row], ar = p.arho[row];
    const double pr = p.Prho[row];
    const double aw = au + gr * ar - s / c.mu;
    const double gaw = v - beta * p.y[row];
    const double au1 = gamma * (aw - gr * ar);
    const double pu1 = gamma * (gaw - gr * pr);
    const double ar1 = ar - rs * (aw - au1);
    const double pr1 = pr - rs * (gaw - pu1);
    p.aw[row] = aw;
    p.au_n[row] = au1;
    p.arho_n[row] = ar1;
    const double a = al[row];
    acc[0] = (aw - au1) * (gaw - pu1);           // ||w - u||^2
    acc[1] = aw * gaw;                           // ||w||^2
    acc[2] = (a + c.sqmu * ar1) * g;             // ||Z~ alpha + D rho||^2
    acc[3] = a * h;                              // ||Z~ alpha||^2
    acc[4] = ar1 * pr1;                          // ||rho||^2
    acc[5] = au1 * pu1;                          // ||u||^2
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NP2; ++j) ws[wid][j] = acc[j];
  }
  __syncthreads();
  if (threadIdx.x < NP2) {
    const int j = threadIdx.x;
    p.part_g[(size_t)j * p.pg_ld + blockIdx.x] = (ws[0][j] + ws[1][j]) + (ws[2][j] + ws[3][j]);
  }
}

__global__ void __launch_bounds__(256) k_rep_step(Consts c, IterPtrs p) { rep_step_body(c, p); }

hipError_t launch_rep_step(const Consts& c, const IterPtrs& p, hipStream_t st) {
  if (!iter_ptrs_ok(p) || ngemv_blocks(c.n) > p.pg_ld) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rep_step, dim3(ngemv_blocks(c.n)), dim3(256), 0, st, c, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Expansion of the representer coefficients: out_j = Z~ a_j (j < 3) row by
// row, the label signs and 1/Z_scale folded into the staged coefficients.
// 64 V rows per block of 4 waves; the waves split the columns.
// ---------------------------------------------------------------------------
constexpr int EX_PANEL = 1024;

template <typename T>
__global__ void __launch_bounds__(256) k_expand(const T* __restrict__ X, Consts c,
                                                const double* __restrict__ a0,
                                                const double* __restrict__ a1,
                                                const double* __restrict__ a2,
                                                const double* __restrict__ y,
                                                double* __restrict__ o0, double* __restrict__ o1,
                                                double* __restrict__ o2) {
  constexpr int V = Vec<T>::N;
  constexpr int ROWS = 64 * V;
  __shared__ double sv[3][EX_PANEL];
  __shared__ double red[4][3][ROWS];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * ROWS;
  const T* xrow = X + rbase + lane * V;
  double acc[3][V];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int e = 0; e < V; ++e) acc[j][e] = 0.0;
  for (int pc = 0; pc < c.n; pc += EX_PANEL) {
    const int pn = min(EX_PANEL, c.n - pc);
    for (int i = threadIdx.x; i < pn; i += 256) {
      const double yz = y[pc + i] * c.inv_zs;
      sv[0][i] = yz * a0[pc + i];
      sv[1][i] = yz * a1[pc + i];
      sv[2][i] = yz * a2[pc + i];
    }
    __syncthreads();
    const int per = (pn + 3) / 4;
    const int j0 = wid * per, j1 = min(pn, j0 + per);
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
    double* outs[3] = {o0, o1, o2};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double v = (red[0][q][rr] + red[1][q][rr]) + (red[2][q][rr] + red[3][q][rr]);
      outs[q][k] = v;
    }
  }
}

// out_j = Z~ a_j (j < 3) over dense storage.
hipError_t launch_expand3(const void* X, int storage, const Consts& c, const double* a0,
                          const double* a1, const double* a2, const double* y, double* o0,
                          double* o1, double* o2, hipStream_t st) {
  if (!X || !a0 || !a1 || !a2 || !y || !o0 || !o1 || !o2 || c.ld % kLdAlign != 0)
    return hipErrorInvalidValue;
  if (storage == DWD_FP64)
    hipLaunchKernelGGL(k_expand<double>, dim3((unsigned)(c.ld / 128)), dim3(256), 0, st,
                       (const double*)X, c, a0, a1, a2, y, o0, o1, o2);
  else if (storage == DWD_FP32)
    hipLaunchKernelGGL(k_expand<float>, dim3((unsigned)(c.ld / 256)), dim3(256), 0, st,
                       (const float*)X, c, a0, a1, a2, y, o0, o1, o2);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// w~ = Z~ aw, u~ = Z~ au, rho = Z~ arho over dense storage.
hipError_t launch_expand(const void* X, int storage, const Consts& c, const IterPtrs& p,
                         hipStream_t st) {
  if (!iter_ptrs_ok(p)) return hipErrorInvalidValue;
  return launch_expand3(X, storage, c, p.aw, p.au, p.arho, p.y, p.w, p.u, p.rho, st);
}

// ---------------------------------------------------------------------------
// Residuals of Section 4.3, stopping rule, sigma rule of Section 4.4; commit
// of the Step 1c outcome; recurrences Z~^T u^{k+1} = gamma (Z~^T w - Z~^T rho^k
// / (sigma sqrt(mu))) and Z~^T rho^{k+1} = Z~^T rho^k - tau sigma sqrt(mu)
// (Z~^T w - Z~^T u^{k+1}) with Z~^T w = v - beta y; and the next iteration's
// t = xi - r - alpha/sigma, x = t + Z~^T b / mu.  One block.
// ---------------------------------------------------------------------------
constexpr int NT1 = 512;

// Threads of the tail block, and rows per thread whose state it requests
// before its reductions.
constexpr int NTT = 1024;
constexpr int TAIL_PRE = 2;
// The tail's sums take one slot per group of TAIL_GROUP lanes: slots 0..8
// and 9..17 the nine n-space sums of outcome 0 and 1 (Step 1c partials),
// 18..23 the pass partials, 24 the most Newton steps (a maximum).  Lane g of
// a group adds blocks g, g + TAIL_GROUP, ... in order, TAIL_UNROLL loads in
// flight; the group then reduces over its lanes by a fixed tree.
constexpr int TAIL_GROUP = 32;
constexpr int TAIL_UNROLL = 16;
constexpr int TAIL_SLOTS = 2 * 9 + NP2 + 1;
static_assert(TAIL_SLOTS * TAIL_GROUP <= NTT, "every tail slot needs a lane group");

// Sum (or maximum, for the Newton steps) of src[b] over b = g,
// g + TAIL_GROUP, ... < nb, in that order.
template <bool MAX>
__device__ __forceinline__ double tail_lane_sum(const double* __restrict__ src, int nb, int g) {
  double v = 0.0;
  for (int b0 = g; b0 < nb; b0 += TAIL_GROUP * TAIL_UNROLL) {
    double t[TAIL_UNROLL];
#pragma unroll
    for (int u = 0; u < TAIL_UNROLL; ++u) {
      const int b = b0 + u * TAIL_GROUP;
      t[u] = b < nb ? src[b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < TAIL_UNROLL; ++u) v = MAX ? fmax(v, t[u]) : v + t[u];
  }
  return v;
}

// The outcome and gamma come from the kernel that sized Step 2 (sc->redo,
// sc->gamma).  Every load the tail needs before its scalar work is requested
// in one round: both outcomes' sums, the pass partials, and both outcomes of
// this thread's first TAIL_PRE rows; the outcome is picked afterwards.
__device__ __forceinline__ void tail_body(const Consts& c, const IterPtrs& p, int nblk_d) {
  Scal* sc = p.sc;
  // (the stop flag is tested once the loads below are in flight; nothing is
  // written before the test)
  const int done = sc->done;
  __shared__ double s_sigma;
  __shared__ double s_sum[TAIL_SLOTS];
  const int nb = ngemv_blocks(c.n);
  // every device scalar this kernel needs, loaded at once
  const int k0 = sc->k;
  const double sigma = sc->sigma;
  const double beta_bar = sc->beta_bar;
  const double beta_1 = sc->beta1;
  const int nd = sc->n_double;
  const int nm = sc->newton_max;
  const int o = sc->redo;
  const double gamma = sc->gamma;
  // state of the first rows: rn, xi0, xi1, al0, al1, v, v1, s1, y, Prho
  double pre[TAIL_PRE][10];
#pragma unroll
  for (int r = 0; r < TAIL_PRE; ++r) {
    const int i = threadIdx.x + r * NTT;
    const bool in = i < c.n;
    pre[r][0] = in ? p.rn[i] : 0.0;
    pre[r][1] = in ? p.xi0[i] : 0.0;
    pre[r][2] = in ? p.xi1[i] : 0.0;
    pre[r][3] = in ? p.al0[i] : 0.0;
    pre[r][4] = in ? p.al1[i] : 0.0;
    pre[r][5] = in ? p.v[i] : 0.0;
    pre[r][6] = in ? p.v1[i] : 0.0;
    pre[r][7] = in ? p.s1[i] : 0.0;
    pre[r][8] = in ? p.y[i] : 0.0;
    pre[r][9] = in ? p.Prho[i] : 0.0;
  }
  {
    const int slot = threadIdx.x / TAIL_GROUP, g = threadIdx.x % TAIL_GROUP;
    const bool is_max = slot == TAIL_SLOTS - 1;
    double v = 0.0;
    if (slot < 18)
      v = tail_lane_sum<false>(p.part_c + (size_t)(1 + (slot / 9) * NPO + slot % 9) * nb, nb, g);
    else if (slot < 18 + NP2)
      v = tail_lane_sum<false>(p.part_g + (size_t)(slot - 18) * p.pg_ld, nblk_d, g);
    else if (is_max)
      v = tail_lane_sum<true>(p.part_it, nb, g);
    if (done) return;
#pragma unroll
    for (int off = TAIL_GROUP / 2; off > 0; off >>= 1) {
      const double w = __shfl_xor(v, off, 64);
      v = is_max ? fmax(v, w) : v + w;
    }
    if (g == 0 && slot < TAIL_SLOTS) s_sum[slot] = v;
  }
  __syncthreads();
  const double beta = o ? beta_1 : beta_bar;
  if (threadIdx.x == 0) {
    const double m = s_sum[TAIL_SLOTS - 1];
    const double* so = s_sum + o * 9;
    const double* sd = s_sum + 18;
    double red[R_COUNT];
    for (int j = 0; j < 9; ++j) red[R_PRES2 + j] = so[j];
    red[R_WU2] = sd[0];
    red[R_W2] = sd[1];
    red[R_DRES2] = sd[2];
    red[R_ZA2] = sd[3];
    red[R_G2] = 0.0;
    red[R_RHO2] = sd[4];
    double e[E_COUNT];
    e[E_PCHK] = e[E_DCHK] = 0.0;
    finish_etas(c, red, e);
    for (int j = 0; j < R_COUNT; ++j) sc->red[j] = red[j];
    for (int j = 0; j < E_COUNT; ++j) sc->eta[j] = e[j];
    sc->u2 = sd[5];
    sc->gamma = gamma;
    sc->beta = beta;
    sc->doubled = o;
    sc->n_double = nd + o;
    if ((int)m > nm) sc->newton_max = (int)m;
    const int k1 = k0 + 1;
    sc->k = k1;
    bool stop = false;
    const double sig = stop_and_sigma(c, e, sigma, k1, &stop);
    if (stop) sc->converged = 1;
    if (stop || k1 >= c.max_iter) {
      sc->done = 1;
      // the host polls this word between chunks of queued iterations
      if (p.hdone) __hip_atomic_store(p.hdone, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    sc->sigma = sig;
    s_sigma = sig;
  }
  __syncthreads();
  const double sig1 = s_sigma;
  const double gr = 1.0 / (sigma * c.sqmu);
  const double rs = c.tau * sigma * c.sqmu;
  // representer iteration: the coefficients the step wrote aside
  if (c.representer)
    for (int i = threadIdx.x; i < c.n; i += NTT) {
      p.au[i] = p.au_n[i];
      p.arho[i] = p.arho_n[i];
    }
  // commit the outcome and form the next iteration's t and x
  auto commit = [&](int i, double rn, double xi, double al, double v, double s1, double yi,
                    double pr) {
    p.r[i] = rn;
    p.xi[i] = xi;
    p.alpha[i] = al;
    if (o) {
      p.s[i] = s1;
      p.v[i] = v;
    }
    const double ztw = v - beta * yi;
    const double pu = gamma * (ztw - gr * pr);
    const double prn = pr - rs * (ztw - pu);
    p.Pu[i] = pu;
    p.Prho[i] = prn;
    const double t = xi - rn - al / sig1;
    p.t[i] = t;
    p.x[i] = t + (c.mu * pu + c.sqmu * prn / sig1) / c.mu;
  };
#pragma unroll
  for (int r = 0; r < TAIL_PRE; ++r) {
    const int i = threadIdx.x + r * NTT;
    if (i < c.n)
      commit(i, pre[r][0], o ? pre[r][2] : pre[r][1], o ? pre[r][4] : pre[r][3],
             o ? pre[r][6] : pre[r][5], pre[r][7], pre[r][8], pre[r][9]);
  }
  const double* xs = o ? p.xi1 : p.xi0;
  const double* as = o ? p.al1 : p.al0;
  const double* vs = o ? p.v1 : p.v;
  for (int i = threadIdx.x + TAIL_PRE * NTT; i < c.n; i += NTT)
    commit(i, p.rn[i], xs[i], as[i], vs[i], p.s1[i], p.y[i], p.Prho[i]);
}

__global__ void __launch_bounds__(NTT) k_tail(Consts c, IterPtrs p, int nblk_d) {
  tail_body(c, p, nblk_d);
}

hipError_t launch_tail(const Consts& c, const IterPtrs& p, int nblk_d, hipStream_t st) {
  hipLaunchKernelGGL(k_tail, dim3(1), dim3(NTT), 0, st, c, p, nblk_d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final check in FP64 from the returned state: partT holds the pass over the
// data of record with v1 = w~, v2 = rho; hG holds G~ alpha.
//   eta_P1 check = ||Z~^T w + beta y + xi - r|| / (1+C) with an explicit pass,
//   eta_D3 check = sqrt(a^T G~ a + 2 sqrt(mu) a^T Z~^T rho + mu ||rho||^2) / (1+C).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT1) k_check(Consts c, IterPtrs p, int nchunks,
                                              const double* __restrict__ part_dres, int nblk) {
  Scal* sc = p.sc;
  double acc[2] = {0, 0};
  for (int i = threadIdx.x; i < c.n; i += NT1) {
    double sw = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) sw += p.partT[((int64_t)ch * 2) * c.n + i];
    const double yi = p.y[i];
    const double ztw = yi * sw * c.inv_zs;
    const double pres = ztw + sc->beta * yi + p.xi[i] - p.r[i];
    acc[0] += pres * pres;
  }
  for (int b = threadIdx.x; b < nblk; b += NT1) acc[1] += part_dres[b];
  block_sum_k<NT1, 2>(acc);
  if (threadIdx.x == 0) {
    const double den = c.opC;
    const double* e = sc->eta;
    const double p1 = sqrt(acc[0]) / den;
    const double d3 = sqrt(acc[1]) / den;
    sc->eta[E_PCHK] = fmax(p1, fmax(e[E_P2], e[E_P3]));
    sc->eta[E_DCHK] = fmax(e[E_D1], fmax(e[E_D2], c.rho_residual ? d3 : 0.0));
  }
}

hipError_t launch_check(const Consts& c, const IterPtrs& p, int nchunks, const double* part_dres,
                        int nblk, hipStream_t st) {
  if (!iter_ptrs_ok(p) || !part_dres) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_check, dim3(1), dim3(NT1), 0, st, c, p, nchunks, part_dres, nblk);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Explicit ||Z~ alpha + D rho||^2 for the final check: za = Z~ alpha row by row
// (label signs and 1/Z_scale folded into the staged alpha), then per-block
// partial sums of (za_k + sqrt(mu) rho_k)^2 in d-space.  64 V rows per block
// of 4 waves; the waves split the columns.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_dres(const T* __restrict__ X, Consts c,
                                              const double* __restrict__ alpha,
                                              const double* __restrict__ y,
                                              const double* __restrict__ rho,
                                              double* __restrict__ part) {
  constexpr int V = Vec<T>::N;
  constexpr int ROWS = 64 * V;
  __shared__ double sv[EX_PANEL];
  __shared__ double red[4][ROWS];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * ROWS;
  const T* xrow = X + rbase + lane * V;
  double acc[V];
#pragma unroll
  for (int e = 0; e < V; ++e) acc[e] = 0.0;
  for (int pc = 0; pc < c.n; pc += EX_PANEL) {
    const int pn = min(EX_PANEL, c.n - pc);
    for (int i = threadIdx.x; i < pn; i += 256) sv[i] = y[pc + i] * c.inv_zs * alpha[pc + i];
    __syncthreads();
    const int per = (pn + 3) / 4;
    const int j0 = wid * per, j1 = min(pn, j0 + per);
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      typename Vec<T>::raw_t xr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xr[u] = Vec<T>::raw(xrow + (int64_t)(pc + j + u) * c.ld);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double x[V];
        Vec<T>::cvt(xr[u], x);
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] = fma(x[e], sv[j + u], acc[e]);
      }
    }
    for (; j < j1; ++j) {
      double x[V];
      Vec<T>::load(xrow + (int64_t)(pc + j) * c.ld, x);
#pragma unroll
      for (int e = 0; e < V; ++e) acc[e] = fma(x[e], sv[j], acc[e]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < V; ++e) red[wid][lane * V + e] = acc[e];
  __syncthreads();
  double s2 = 0.0;
  for (int rr = threadIdx.x; rr < ROWS; rr += 256) {
    const double za = (red[0][rr] + red[1][rr]) + (red[2][rr] + red[3][rr]);
    const double dr = za + c.sqmu * rho[rbase + rr];
    s2 += dr * dr;
  }
  s2 = block_sum<256>(s2);
  if (threadIdx.x == 0) part[blockIdx.x] = s2;
}

int dres_blocks(int storage, int64_t ld) { return (int)(ld / (storage == DWD_FP64 ? 128 : 256)); }

hipError_t launch_dres(const void* X, int storage, const Consts& c, const double* alpha,
                       const double* y, const double* rho, double* part, hipStream_t st) {
  if (!X || !alpha || !y || !rho || !part || c.ld % kLdAlign != 0) return hipErrorInvalidValue;
  const int nb = dres_blocks(storage, c.ld);
  if (storage == DWD_FP64)
    hipLaunchKernelGGL(k_dres<double>, dim3(nb), dim3(256), 0, st, (const double*)X, c, alpha, y,
                       rho, part);
  else if (storage == DWD_FP32)
    hipLaunchKernelGGL(k_dres<float>, dim3(nb), dim3(256), 0, st, (const float*)X, c, alpha, y,
                       rho, part);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ||v||^2 over ld entries into out[0] (one block, fixed order).
__global__ void __launch_bounds__(1024) k_norm2(const double* __restrict__ v, int64_t m,
                                                double* __restrict__ out) {
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) acc += v[i] * v[i];
  acc = block_sum<1024>(acc);
  if (threadIdx.x == 0) out[0] = acc;
}

hipError_t launch_norm2(const double* v, int64_t m, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, st, v, m, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Multi-problem forms for serving: one launch steps every problem of a
// descriptor table (grid.y = table entries, grid.x = the largest problem's
// block count; blocks beyond a problem's own count return at once).  They
// run the same device code as the single-problem kernels.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_step1ab_m(const StepDesc* __restrict__ D) {
  const StepDesc* s = D + blockIdx.y;
  if ((int)blockIdx.x >= s->nrow) return;
  step1ab_body(s->c, s->p);
}

__global__ void __launch_bounds__(256) k_step1c_m(const StepDesc* __restrict__ D) {
  const StepDesc* s = D + blockIdx.y;
  if ((int)blockIdx.x >= s->nrow) return;
  step1c_body(s->c, s->p);
}

__global__ void __launch_bounds__(256) k_rep_step_m(const StepDesc* __restrict__ D) {
  const StepDesc* s = D + blockIdx.y;
  if ((int)blockIdx.x >= s->nrow) return;
  rep_step_body(s->c, s->p);
}

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_pass2_m(const StepDesc* __restrict__ D) {
  const StepDesc* s = D + blockIdx.y;
  if ((int)blockIdx.x >= s->npass) return;
  pass2_body<T, 4>((const T*)s->X, s->c, s->p);
}

__global__ void __launch_bounds__(NTT) k_tail_m(const StepDesc* __restrict__ D) {
  const StepDesc* s = D + blockIdx.y;
  tail_body(s->c, s->p, s->npass);
}

hipError_t launch_multi(int what, const StepDesc* D, int count, int gx, int storage,
                        hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (count > 65535 || gx < 1) return hipErrorInvalidValue;
  const dim3 g((unsigned)gx, (unsigned)count);
  switch (what) {
    case MULTI_STEP1AB: hipLaunchKernelGGL(k_step1ab_m, g, dim3(256), 0, st, D); break;
    case MULTI_STEP1C: hipLaunchKernelGGL(k_step1c_m, g, dim3(256), 0, st, D); break;
    case MULTI_REP: hipLaunchKernelGGL(k_rep_step_m, g, dim3(256), 0, st, D); break;
    case MULTI_TAIL:
      hipLaunchKernelGGL(k_tail_m, dim3(1, (unsigned)count), dim3(NTT), 0, st, D);
      break;
    case MULTI_PASS:
      if (storage == DWD_FP64)
        hipLaunchKernelGGL(k_pass2_m<double>, g, dim3(256), 0, st, D);
      else if (storage == DWD_FP32)
        hipLaunchKernelGGL(k_pass2_m<float>, g, dim3(256), 0, st, D);
      else
        hipLaunchKernelGGL(k_pass2_m<uint16_t>, g, dim3(256), 0, st, D);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dwd
