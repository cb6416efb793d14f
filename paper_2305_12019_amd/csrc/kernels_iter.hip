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

#include "dwd_internal.h"

namespace dwd {

// ---------------------------------------------------------------------------
// Vector loads of the stored data, converted to FP64.
// ---------------------------------------------------------------------------
template <typename T>
struct Vec;
template <>
struct Vec<double> {
  static constexpr int N = 2;
  __device__ static __forceinline__ void load(const double* p, double (&o)[2]) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct Vec<float> {
  static constexpr int N = 4;
  __device__ static __forceinline__ void load(const float* p, double (&o)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct Vec<uint16_t> {
  static constexpr int N = 8;
  __device__ static __forceinline__ void load(const uint16_t* p, double (&o)[8]) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = (double)__uint_as_float(w[i] << 16);
      o[2 * i + 1] = (double)__uint_as_float(w[i] & 0xFFFF0000u);
    }
  }
};

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
                       p.f, p.s, p.v, p.dr, p.hG, p.hM, p.sp, p.ap, p.u, p.rho, p.w, p.za,
                       p.part_g, p.part_d, p.part_n1, p.part_n2, p.partT, p.sc};
  for (const void* q : req)
    if (!q) return false;
  return true;
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
  }
  if (i < c.ld) {
    p.u[i] = 0.0;
    p.rho[i] = 0.0;
    p.w[i] = 0.0;
    p.za[i] = 0.0;
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
  __shared__ double lds[4];
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
  if (lane == 0) lds[wid] = contrib;
  __syncthreads();
  if (threadIdx.x == 0 && part) part[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

int ngemv_blocks(int n) { return (n + 3) / 4; }

hipError_t launch_ngemv(int n, const double* A1, const double* x1, double* o1, const double* A2,
                        const double* x2, double* o2, const double* wdot, double* part,
                        const Scal* sc, hipStream_t st) {
  if (!A1 || !x1 || !o1 || (A2 && (!x2 || !o2))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ngemv, dim3(ngemv_blocks(n)), dim3(256), 0, st, n, A1, x1, o1, A2, x2, o2,
                     wdot, part, sc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 1b: prox of theta_q by the Newton map of Section 3.2 (eq-varphi),
// warm-started at r^k, with the bracket safeguard.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow_qp1(double s, const Consts& c) {  // s^(q+1)
  switch (c.qkind) {
    case 1: return s * s;
    case 2: return s * s * s;
    case 4: {
      const double s2 = s * s;
      return s2 * s2 * s;
    }
    case 5: return s * sqrt(s);
    default: return pow(s, c.q + 1.0);
  }
}

__device__ __forceinline__ double pow_q(double s, const Consts& c) {  // s^q
  switch (c.qkind) {
    case 1: return s;
    case 2: return s * s;
    case 4: {
      const double s2 = s * s;
      return s2 * s2;
    }
    case 5: return sqrt(s);
    default: return pow(s, c.q);
  }
}

__device__ __forceinline__ double prox_lower(double a, double sigma, const Consts& c) {
  const double s0 = pow(c.q / sigma, 1.0 / (c.q + 2.0));
  if (a >= 0.0) return fmax(a, s0);
  return pow(c.q / (sigma * (s0 - a)), 1.0 / (c.q + 1.0));
}

__device__ double prox_newton(double a, double sigma, double s, double tol, const Consts& c,
                              int& steps) {
  steps = 0;
  if (!(s > 0.0) || !isfinite(s)) s = prox_lower(a, sigma, c);
  double sq1 = pow_qp1(s, c);
  double g = -c.q / sq1 + sigma * (s - a);
  if (fabs(g) <= tol) return s;
  const double c1 = c.c1 / sigma, c2 = c.c2 / sigma;
  for (int it = 0; it < 50; ++it) {
    double sn = s * (c1 + a * sq1) / (c2 + sq1 * s);
    if (!(sn > 0.0) || !isfinite(sn)) sn = prox_lower(a, sigma, c);
    const bool tiny = fabs(sn - s) <= 4.0 * DBL_EPSILON * s;
    s = sn;
    ++steps;
    sq1 = pow_qp1(s, c);
    g = -c.q / sq1 + sigma * (s - a);
    if (fabs(g) <= tol || tiny) break;
  }
  return s;
}

__device__ __forceinline__ double eps_k(const Consts& c, int k) {
  const double k1 = (double)k + 1.0;
  return c.eps_c / (k1 * sqrt(k1));
}

// ---------------------------------------------------------------------------
// Step 1a (finish) and Step 1b.  One block.
//   beta_bar = -y^T f / y^T M^-1 y, s_bar = f + beta_bar M^-1 y, v_bar = s_bar - t,
//   c = v_bar + xi - alpha/sigma, r^{k+1} = prox(c), dr = r^{k+1} - r^k.
// ---------------------------------------------------------------------------
constexpr int NT1 = 1024;

__global__ void __launch_bounds__(NT1) k_step1b(Consts c, IterPtrs p, int nblk_gemv) {
  Scal* sc = p.sc;
  if (sc->done) return;
  __shared__ double lds[(NT1 / 64) * 2];
  __shared__ int smax;
  if (threadIdx.x == 0) smax = 0;
  double yf = 0.0;
  for (int b = threadIdx.x; b < nblk_gemv; b += NT1) yf += p.part_n1[b];
  yf = block_sum<NT1>(yf, lds);
  const double beta_bar = -yf / c.ymy;
  const double sigma = sc->sigma;
  const double tolN = eps_k(c, sc->k) / sqrt((double)c.n);
  double ytdr = 0.0;
  int mx = 0;
  for (int i = threadIdx.x; i < c.n; i += NT1) {
    const double s = p.f[i] + beta_bar * p.my[i];
    const double v = s - p.t[i];
    const double cc = v + p.xi[i] - p.alpha[i] / sigma;
    const double r0 = p.r[i];
    int steps;
    const double rn = prox_newton(cc, sigma, r0, tolN, c, steps);
    mx = max(mx, steps);
    p.s[i] = s;
    p.v[i] = v;
    p.x[i] = rn;  // x is free after the M^-1 product; it now holds r^{k+1}
    const double dr = rn - r0;
    p.dr[i] = dr;
    ytdr += p.y[i] * dr;
  }
  atomicMax(&smax, mx);
  ytdr = block_sum<NT1>(ytdr, lds);
  if (threadIdx.x == 0) {
    sc->beta_bar = beta_bar;
    sc->ytdr = ytdr;
    if (smax > sc->newton_max) sc->newton_max = smax;
  }
}

hipError_t launch_step1b(const Consts& c, const IterPtrs& p, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_step1b, dim3(1), dim3(NT1), 0, st, c, p, nblk);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 1c test and solve, then the n-space parts of Steps 2 and 3 and the
// n-space residuals of Section 4.3.  One block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT1) k_step1c(Consts c, IterPtrs p, int nblk_gemv) {
  Scal* sc = p.sc;
  if (sc->done) return;
  __shared__ double lds[(NT1 / 64) * 9];
  double dGd = 0.0;
  for (int b = threadIdx.x; b < nblk_gemv; b += NT1) dGd += p.part_n2[b];
  dGd = block_sum<NT1>(dGd, lds);
  const double ek = eps_k(c, sc->k);
  const double res2 = dGd + sc->ytdr * sc->ytdr;
  const bool dbl = sqrt(fmax(res2, 0.0)) > 5.0 * ek;
  const double sigma = sc->sigma;
  double beta = sc->beta_bar;
  if (dbl) {
    double yf = 0.0;
    for (int i = threadIdx.x; i < c.n; i += NT1) {
      const double f = p.f[i] - p.hM[i];
      p.f[i] = f;
      yf += p.y[i] * f;
    }
    yf = block_sum<NT1>(yf, lds);
    beta = -yf / c.ymy;
  }
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < c.n; i += NT1) {
    const double rn = p.x[i];
    double s, v;
    if (dbl) {
      s = p.f[i] + beta * p.my[i];
      v = s - (p.t[i] - p.dr[i]);
      p.s[i] = s;
      p.v[i] = v;
    } else {
      s = p.s[i];
      v = p.v[i];
    }
    const double a0 = p.alpha[i];
    const double yi = p.y[i];
    // Step 2 (xi) and Step 3 (alpha)
    const double xi = fmax(0.0, rn - v + (a0 - c.C) / sigma);
    const double pres = v + xi - rn;
    const double a1 = a0 - c.tau * sigma * pres;
    p.xi[i] = xi;
    p.alpha[i] = a1;
    p.r[i] = rn;
    p.sp[i] = yi * s * c.inv_zs;
    p.ap[i] = yi * a1 * c.inv_zs;
    const double rq1 = pow_qp1(rn, c);
    const double comp = a1 - c.q / rq1;
    acc[0] += pres * pres;
    acc[1] += fmin(0.0, a1) * fmin(0.0, a1);
    acc[2] += fmax(0.0, a1 - c.C) * fmax(0.0, a1 - c.C);
    acc[3] += yi * a1;
    acc[4] += xi * (c.C - a1);
    acc[5] += comp * comp;
    acc[6] += 1.0 / pow_q(rn, c);
    acc[7] += xi;
    acc[8] += a1 > 0.0 ? pow(a1, c.qexp) : 0.0;
  }
  block_sum_k<NT1, 9>(acc, lds);
  if (threadIdx.x == 0) {
    sc->beta = beta;
    sc->doubled = dbl ? 1 : 0;
    if (dbl) sc->n_double += 1;
    for (int j = 0; j < 9; ++j) sc->red[R_PRES2 + j] = acc[j];
  }
}

hipError_t launch_step1c(const Consts& c, const IterPtrs& p, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_step1c, dim3(1), dim3(NT1), 0, st, c, p, nblk);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pass over Z: zs = Z~ s and za = Z~ alpha^{k+1} row by row (the label signs
// and 1/Z_scale are in sp, ap), fused with the Step 2 prologue:
//   w = (b - zs)/mu,  b = mu u + sqrt(mu) rho / sigma,  g = w - rho/(sigma sqrt(mu)),
// and a block partial of ||g||^2.  Block = NW waves over the same 64*V rows,
// wave j walks its share of the columns; partial row sums meet in LDS.
// ---------------------------------------------------------------------------
constexpr int PANEL = 2048;

template <typename T, int NW>
__global__ void __launch_bounds__(NW * 64) k_pass2(const T* __restrict__ X, Consts c, IterPtrs p) {
  if (p.sc->done) return;
  constexpr int V = Vec<T>::N;
  constexpr int ROWS = 64 * V;
  __shared__ double sv[2][PANEL];
  __shared__ double red[NW][2][ROWS];
  __shared__ double lds[NW];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * ROWS;
  const T* xrow = X + rbase + lane * V;
  double as[V], aa[V];
#pragma unroll
  for (int e = 0; e < V; ++e) as[e] = aa[e] = 0.0;
  for (int pc = 0; pc < c.n; pc += PANEL) {
    const int pn = min(PANEL, c.n - pc);
    for (int i = threadIdx.x; i < pn; i += NW * 64) {
      sv[0][i] = p.sp[pc + i];
      sv[1][i] = p.ap[pc + i];
    }
    __syncthreads();
    const int per = (pn + NW - 1) / NW;
    const int j0 = wid * per, j1 = min(pn, j0 + per);
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      double x0[V], x1[V], x2[V], x3[V];
      Vec<T>::load(xrow + (int64_t)(pc + j) * c.ld, x0);
      Vec<T>::load(xrow + (int64_t)(pc + j + 1) * c.ld, x1);
      Vec<T>::load(xrow + (int64_t)(pc + j + 2) * c.ld, x2);
      Vec<T>::load(xrow + (int64_t)(pc + j + 3) * c.ld, x3);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        as[e] = fma(x0[e], sv[0][j], as[e]);
        aa[e] = fma(x0[e], sv[1][j], aa[e]);
        as[e] = fma(x1[e], sv[0][j + 1], as[e]);
        aa[e] = fma(x1[e], sv[1][j + 1], aa[e]);
        as[e] = fma(x2[e], sv[0][j + 2], as[e]);
        aa[e] = fma(x2[e], sv[1][j + 2], aa[e]);
        as[e] = fma(x3[e], sv[0][j + 3], as[e]);
        aa[e] = fma(x3[e], sv[1][j + 3], aa[e]);
      }
    }
    for (; j < j1; ++j) {
      double x0[V];
      Vec<T>::load(xrow + (int64_t)(pc + j) * c.ld, x0);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        as[e] = fma(x0[e], sv[0][j], as[e]);
        aa[e] = fma(x0[e], sv[1][j], aa[e]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < V; ++e) {
    red[wid][0][lane * V + e] = as[e];
    red[wid][1][lane * V + e] = aa[e];
  }
  __syncthreads();
  const double sigma = p.sc->sigma;
  const double bu = c.mu, br = c.sqmu / sigma, gr = 1.0 / (sigma * c.sqmu);
  double g2 = 0.0;
  for (int rr = threadIdx.x; rr < ROWS; rr += NW * 64) {
    double zs = 0.0, za = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      zs += red[ww][0][rr];
      za += red[ww][1][rr];
    }
    const int64_t k = rbase + rr;
    const double rho = p.rho[k];
    const double b = bu * p.u[k] + br * rho;
    const double w = (b - zs) / c.mu;
    const double g = w - gr * rho;
    p.w[k] = w;
    p.za[k] = za;
    g2 += g * g;
  }
  g2 = block_sum<NW * 64>(g2, lds);
  if (threadIdx.x == 0) p.part_g[blockIdx.x] = g2;
}

template <typename T>
static constexpr int pass2_waves() {
  return sizeof(T) == 2 ? 4 : 8;
}

int pass2_blocks(int storage, int64_t ld) {
  const int rows = storage == DWD_FP64 ? 128 : (storage == DWD_FP32 ? 256 : 512);
  return (int)(ld / rows);
}

hipError_t launch_pass2(const void* X, int storage, const Consts& c, const IterPtrs& p,
                        hipStream_t st) {
  if (!X || !iter_ptrs_ok(p) || c.ld % kLdAlign != 0) return hipErrorInvalidValue;
  const int nb = pass2_blocks(storage, c.ld);
  if (storage == DWD_FP64)
    hipLaunchKernelGGL((k_pass2<double, 8>), dim3(nb), dim3(512), 0, st, (const double*)X, c, p);
  else if (storage == DWD_FP32)
    hipLaunchKernelGGL((k_pass2<float, 8>), dim3(nb), dim3(512), 0, st, (const float*)X, c, p);
  else
    hipLaunchKernelGGL((k_pass2<uint16_t, 4>), dim3(nb), dim3(256), 0, st, (const uint16_t*)X, c,
                       p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 2 (u: projection onto the ball of radius Z_scale) and Step 3 (rho),
// with the d-space partial sums ||w-u||^2, ||w||^2, ||Z~a + sqrt(mu) rho||^2,
// ||Z~a||^2, ||rho||^2 (5 per block).
// ---------------------------------------------------------------------------
constexpr int ND = 5;

__global__ void __launch_bounds__(256) k_dspace(Consts c, IterPtrs p, int nblk_p2) {
  Scal* sc = p.sc;
  if (sc->done) return;
  __shared__ double lds[4 * ND];
  double g2 = 0.0;
  for (int b = threadIdx.x; b < nblk_p2; b += 256) g2 += p.part_g[b];
  g2 = block_sum<256>(g2, lds);
  const double ng = sqrt(g2);
  const double gamma = (ng <= c.R) ? 1.0 : c.R / ng;
  const double sigma = sc->sigma;
  const double gr = 1.0 / (sigma * c.sqmu);
  const double rs = c.tau * sigma * c.sqmu;
  double acc[ND] = {0, 0, 0, 0, 0};
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < c.ld;
       k += (int64_t)gridDim.x * 256) {
    const double w = p.w[k];
    const double rho = p.rho[k];
    const double u = gamma * (w - gr * rho);
    const double rn = rho - rs * (w - u);
    p.u[k] = u;
    p.rho[k] = rn;
    const double za = p.za[k];
    const double dres = za + c.sqmu * rn;
    acc[0] += (w - u) * (w - u);
    acc[1] += w * w;
    acc[2] += dres * dres;
    acc[3] += za * za;
    acc[4] += rn * rn;
  }
  block_sum_k<256, ND>(acc, lds);
  if (threadIdx.x == 0) {
    for (int j = 0; j < ND; ++j) p.part_d[blockIdx.x * ND + j] = acc[j];
    if (blockIdx.x == 0) {
      sc->gamma = gamma;
      sc->red[R_G2] = g2;
    }
  }
}

int dspace_blocks(int64_t ld) {
  int64_t b = (ld + 255) / 256;
  return (int)(b > 1024 ? 1024 : b);
}

hipError_t launch_dspace(const Consts& c, const IterPtrs& p, int nblk_p2, hipStream_t st) {
  hipLaunchKernelGGL(k_dspace, dim3(dspace_blocks(c.ld)), dim3(256), 0, st, c, p, nblk_p2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residuals of Section 4.3, stopping rule, sigma rule of Section 4.4, and the
// recurrences Z~^T u^{k+1} = gamma (Z~^T w - Z~^T rho^k / (sigma sqrt(mu))),
// Z~^T rho^{k+1} = Z~^T rho^k - tau sigma sqrt(mu) (Z~^T w - Z~^T u^{k+1}),
// with Z~^T w = v - beta y.  One block.
// ---------------------------------------------------------------------------
__device__ void finish_etas(const Consts& c, Scal* sc) {
  const double den = c.opC;
  double* e = sc->eta;
  const double* r = sc->red;
  e[E_P1] = sqrt(r[R_PRES2]) / den;
  e[E_P2] = c.sqmu * sqrt(r[R_WU2]) / den;
  e[E_P3] = fmax(sqrt(r[R_W2]) - c.R, 0.0) / den;
  e[E_D1] = sqrt(r[R_AMIN2]) / den;
  e[E_D2] = sqrt(r[R_AMAX2]) / den;
  e[E_D3] = sqrt(r[R_DRES2]) / den;
  e[E_C1] = fabs(r[R_YA]) / den;
  e[E_C2] = fabs(r[R_XCA]) / den;
  e[E_C3] = r[R_COMP2] / den;
  const double prim = r[R_SUMRQ] + c.C * r[R_SUMXI];
  const double dual = c.kappa * r[R_SUMAQ] - c.R * sqrt(r[R_ZA2]);
  e[E_PRIM] = prim;
  e[E_DUAL] = dual;
  e[E_GAP] = fabs(prim - dual) / (1.0 + fabs(prim) + fabs(dual));
  e[E_P] = fmax(e[E_P1], fmax(e[E_P2], e[E_P3]));
  e[E_D] = fmax(e[E_D1], fmax(e[E_D2], c.rho_residual ? e[E_D3] : 0.0));
  e[E_C] = fmax(e[E_C1], fmax(e[E_C2], e[E_C3]));
}

__global__ void __launch_bounds__(NT1) k_tail(Consts c, IterPtrs p, int nblk_d) {
  Scal* sc = p.sc;
  if (sc->done) return;
  __shared__ double lds[(NT1 / 64) * ND];
  double acc[ND] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk_d; b += NT1)
#pragma unroll
    for (int j = 0; j < ND; ++j) acc[j] += p.part_d[b * ND + j];
  block_sum_k<NT1, ND>(acc, lds);
  const double sigma = sc->sigma;
  const double gamma = sc->gamma;
  const double beta = sc->beta;
  const double gr = 1.0 / (sigma * c.sqmu);
  const double rs = c.tau * sigma * c.sqmu;
  for (int i = threadIdx.x; i < c.n; i += NT1) {
    const double ztw = p.v[i] - beta * p.y[i];
    const double pr = p.Prho[i];
    const double pu = gamma * (ztw - gr * pr);
    p.Pu[i] = pu;
    p.Prho[i] = pr - rs * (ztw - pu);
  }
  if (threadIdx.x == 0) {
    sc->red[R_WU2] = acc[0];
    sc->red[R_W2] = acc[1];
    sc->red[R_DRES2] = acc[2];
    sc->red[R_ZA2] = acc[3];
    sc->red[R_RHO2] = acc[4];
    finish_etas(c, sc);
    const double* e = sc->eta;
    const int k1 = sc->k + 1;
    sc->k = k1;
    const double pd = fmax(e[E_P], e[E_D]);
    const double cg_min = fmin(e[E_C], e[E_GAP]), cg_max = fmax(e[E_C], e[E_GAP]);
    if (pd < c.tol && cg_min < sqrt(c.tol) && cg_max < 0.05) {
      sc->converged = 1;
      sc->done = 1;
    } else {
      if (k1 >= c.max_iter) sc->done = 1;
      const double ep = e[E_P], ed = e[E_D];
      if (ep >= 1e-300 && ed >= 1e-300) {
        const double chi = ep / ed;
        const double m = fmax(chi, 1.0 / chi);
        const double zeta = m > 500.0 ? 2.2 : (m > 50.0 ? 1.65 : 1.1);
        if (chi > 5.0) sc->sigma = sigma * zeta;
        else if (1.0 / chi > 5.0) sc->sigma = sigma / zeta;
      }
    }
  }
}

hipError_t launch_tail(const Consts& c, const IterPtrs& p, int nblk_d, hipStream_t st) {
  hipLaunchKernelGGL(k_tail, dim3(1), dim3(NT1), 0, st, c, p, nblk_d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final check in FP64 from the returned state: partT holds the pass over the
// data of record with v1 = w~, v2 = rho; hG holds G~ alpha.
//   eta_P1 check = ||Z~^T w + beta y + xi - r|| / (1+C) with an explicit pass,
//   eta_D3 check = sqrt(a^T G~ a + 2 sqrt(mu) a^T Z~^T rho + mu ||rho||^2) / (1+C).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NT1) k_check(Consts c, IterPtrs p, int nchunks) {
  Scal* sc = p.sc;
  __shared__ double lds[(NT1 / 64) * 3];
  double acc[3] = {0, 0, 0};
  for (int i = threadIdx.x; i < c.n; i += NT1) {
    double sw = 0.0, sr = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) {
      sw += p.partT[((int64_t)ch * 2) * c.n + i];
      sr += p.partT[((int64_t)ch * 2 + 1) * c.n + i];
    }
    const double yi = p.y[i];
    const double ztw = yi * sw * c.inv_zs;
    const double ztr = yi * sr * c.inv_zs;
    const double pres = ztw + sc->beta * yi + p.xi[i] - p.r[i];
    const double a = p.alpha[i];
    acc[0] += pres * pres;
    acc[1] += a * p.hG[i];
    acc[2] += a * ztr;
  }
  block_sum_k<NT1, 3>(acc, lds);
  if (threadIdx.x == 0) {
    const double den = c.opC;
    const double* e = sc->eta;
    const double p1 = sqrt(acc[0]) / den;
    const double rho2 = sc->red[R_RHO2];  // ||rho||^2 from the last d-space step
    const double dres2 = acc[1] + 2.0 * c.sqmu * acc[2] + c.mu * rho2;
    const double d3 = sqrt(fmax(dres2, 0.0)) / den;
    sc->eta[E_PCHK] = fmax(p1, fmax(e[E_P2], e[E_P3]));
    sc->eta[E_DCHK] = fmax(e[E_D1], fmax(e[E_D2], c.rho_residual ? d3 : 0.0));
  }
}

hipError_t launch_check(const Consts& c, const IterPtrs& p, int nchunks, hipStream_t st) {
  if (!iter_ptrs_ok(p)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_check, dim3(1), dim3(NT1), 0, st, c, p, nchunks);
  return hipGetLastError();
}

// ||v||^2 over ld entries into out[0] (one block, fixed order).
__global__ void __launch_bounds__(1024) k_norm2(const double* __restrict__ v, int64_t m,
                                                double* __restrict__ out) {
  __shared__ double lds[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) acc += v[i] * v[i];
  acc = block_sum<1024>(acc, lds);
  if (threadIdx.x == 0) out[0] = acc;
}

hipError_t launch_norm2(const double* v, int64_t m, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, st, v, m, out);
  return hipGetLastError();
}

}  // namespace dwd
