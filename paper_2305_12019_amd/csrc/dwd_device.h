// Device functions shared by the single-problem and the batched kernels.
#pragma once

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
// Loads of the streamed data are nontemporal: X is read once per pass and
// is far larger than the caches, so it should not evict the n x n matrices
// and the n-vectors that the other kernels of the iteration reuse.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));
// raw(): one nontemporal vector load, kept in its storage type until
// cvt() widens it to FP64 at the point of use (half the registers of loads
// in flight for FP32 data); load() = cvt(raw()).
template <>
struct Vec<double> {
  static constexpr int N = 2;
  typedef nt_d2 raw_t;
  __device__ static __forceinline__ raw_t raw(const double* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  }
  __device__ static __forceinline__ void cvt(const raw_t& v, double (&o)[2]) {
    o[0] = v.x;
    o[1] = v.y;
  }
  __device__ static __forceinline__ void load(const double* p, double (&o)[2]) { cvt(raw(p), o); }
};
template <>
struct Vec<float> {
  static constexpr int N = 4;
  typedef nt_f4 raw_t;
  __device__ static __forceinline__ raw_t raw(const float* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  }
  __device__ static __forceinline__ void cvt(const raw_t& v, double (&o)[4]) {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
  __device__ static __forceinline__ void load(const float* p, double (&o)[4]) { cvt(raw(p), o); }
};
template <>
struct Vec<uint16_t> {
  static constexpr int N = 8;
  typedef nt_u4 raw_t;
  __device__ static __forceinline__ raw_t raw(const uint16_t* p) {
    return __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p));
  }
  __device__ static __forceinline__ void cvt(const raw_t& v, double (&o)[8]) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = (double)__uint_as_float(w[i] << 16);
      o[2 * i + 1] = (double)__uint_as_float(w[i] & 0xFFFF0000u);
    }
  }
  __device__ static __forceinline__ void load(const uint16_t* p, double (&o)[8]) {
    cvt(raw(p), o);
  }
};


// ---------------------------------------------------------------------------
// Step 1b: prox of theta_q by the Newton map of Section 3.2 (eq-varphi),
// warm-started at r^k, with the bracket safeguard.
// ---------------------------------------------------------------------------
// General-q powers and the rarely taken bracket restart out of line: the
// integer and q = 0.5 cases do not need them, and inlined they cost the fused
// kernels many registers.
__device__ __noinline__ double pow_general(double a, double b) { return pow(a, b); }

__device__ __forceinline__ double pow_qp1(double s, const Consts& c) {  // s^(q+1)
  switch (c.qkind) {
    case 1: return s * s;
    case 2: return s * s * s;
    case 4: {
      const double s2 = s * s;
      return s2 * s2 * s;
    }
    case 5: return s * sqrt(s);
    default: return pow_general(s, c.q + 1.0);
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
    default: return pow_general(s, c.q);
  }
}

__device__ __noinline__ double prox_lower(double a, double sigma, const Consts& c) {
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

// Step 1b with a loss weight v on theta_q: v s^-q + sigma/2 (s - a)^2 has
// the minimiser of the unweighted problem at sigma / v, and its derivative
// is v times the unweighted one at sigma / v, so the accuracy test scales
// by 1 / v (v = 1: the unweighted prox, bit for bit).
__device__ __forceinline__ double loss_weight(const Consts& c, double yi) {
  return yi > 0.0 ? c.wpos : c.wneg;
}

__device__ __forceinline__ double prox_weighted(double a, double sigma, double s, double tol,
                                                double v, const Consts& c, int& steps) {
  return prox_newton(a, sigma / v, s, tol / v, c, steps);
}

__device__ __forceinline__ double eps_k(const Consts& c, int k) {
  const double k1 = (double)k + 1.0;
  return c.eps_c / (k1 * sqrt(k1));
}

// Sum one double over a block of NT threads; every thread gets the result.
template <int NT>
__device__ __forceinline__ double bsum(double v) {
  return block_sum<NT>(v);
}

// Dot products of one row of an n x n FP64 matrix with x by one wave, with
// CH loads per lane in flight before the reduction.
constexpr int CH = 16;

__device__ __forceinline__ double wave_row_dot(const double* __restrict__ a,
                                               const double* __restrict__ x, int n, int lane) {
  double acc = 0.0;
  for (int base = 0; base < n; base += 64 * CH) {
    double av[CH], xv[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int j = base + q * 64 + lane;
      av[q] = j < n ? a[j] : 0.0;
      xv[q] = j < n ? x[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) acc = fma(av[q], xv[q], acc);
  }
  return wave_sum(acc);
}

__device__ __forceinline__ void wave_row_dot2(const double* __restrict__ a,
                                              const double* __restrict__ b,
                                              const double* __restrict__ x, int n, int lane,
                                              double& ra, double& rb) {
  double sa = 0.0, sb = 0.0;
  for (int base = 0; base < n; base += 64 * CH) {
    double av[CH], bv[CH], xv[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int j = base + q * 64 + lane;
      av[q] = j < n ? a[j] : 0.0;
      bv[q] = j < n ? b[j] : 0.0;
      xv[q] = j < n ? x[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      sa = fma(av[q], xv[q], sa);
      sb = fma(bv[q], xv[q], sb);
    }
  }
  ra = wave_sum(sa);
  rb = wave_sum(sb);
}

// Three dot products with x by one wave (two matrix rows and one n-vector),
// every load of the three issued in one round.  With the same vector as c
// in every wave, each wave forms c^T x in the same fixed order, so a value
// that every row needs comes without a block reduction.
__device__ __forceinline__ void wave_row_dot3(const double* __restrict__ a,
                                              const double* __restrict__ b,
                                              const double* __restrict__ cv,
                                              const double* __restrict__ x, int n, int lane,
                                              double& ra, double& rb, double& rc) {
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int base = 0; base < n; base += 64 * CH) {
    double av[CH], bv[CH], cw[CH], xv[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int j = base + q * 64 + lane;
      av[q] = j < n ? a[j] : 0.0;
      bv[q] = j < n ? b[j] : 0.0;
      cw[q] = j < n ? cv[j] : 0.0;
      xv[q] = j < n ? x[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      sa = fma(av[q], xv[q], sa);
      sb = fma(bv[q], xv[q], sb);
      sc = fma(cw[q], xv[q], sc);
    }
  }
  ra = wave_sum(sa);
  rb = wave_sum(sb);
  rc = wave_sum(sc);
}


// a^(q/(q+1)) for a > 0: sqrt for q = 1, cube roots for q = 2 and 0.5
__device__ __forceinline__ double pow_qexp(double a, const Consts& c) {
  switch (c.qkind) {
    case 1: return sqrt(a);
    case 2: return cbrt(a * a);
    case 5: return cbrt(a);
    default: return pow_general(a, c.qexp);
  }
}

// Per-row terms of the Section 4.3 residuals and objectives, with the loss
// weight v_i of the row's class and the penalty weight e_i: alpha - q v / r^(q+1)
// (eta_C3), max(0, alpha - C e) (eta_D2), xi (C e - alpha) (eta_C2),
// v r^-q and e xi (primal), v^(1/(q+1)) alpha^(q/(q+1)) (dual).
__device__ __forceinline__ void nspace_sums(const Consts& c, double rq, double rq1, double a1,
                                            double xi, double pres, double yi, double ei,
                                            double* acc) {
  const bool pos = yi > 0.0;
  const double v = pos ? c.wpos : c.wneg, vd = pos ? c.wdpos : c.wdneg;
  const double ce = c.C * ei;
  const double comp = a1 - c.q * v / rq1;
  acc[0] = pres * pres;
  acc[1] = fmin(0.0, a1) * fmin(0.0, a1);
  acc[2] = fmax(0.0, a1 - ce) * fmax(0.0, a1 - ce);
  acc[3] = yi * a1;
  acc[4] = xi * (ce - a1);
  acc[5] = comp * comp;
  acc[6] = v / rq;
  acc[7] = ei * xi;
  acc[8] = a1 > 0.0 ? vd * pow_qexp(a1, c) : 0.0;
}


// The Step 1c decision and the Step 2 ball scaling gamma = min(1, R/||g||),
// from the block partials of both row kernels summed in a fixed order
// (identical in every caller).
struct Step2Plan {
  int redo;
  double gamma;
};

// a[0..5] are the summed plan partials (see plan_part); k and u2 the
// iteration index and ||u||^2.
__device__ __forceinline__ Step2Plan step2_plan_finish(const Consts& c, const double* a, int k,
                                                       double u2) {
  Step2Plan pl;
  const double res2 = a[0] + a[1] * a[1];
  pl.redo = sqrt(fmax(res2, 0.0)) > 5.0 * eps_k(c, k) ? 1 : 0;
  const double sGs = pl.redo ? a[4] : a[2];
  const double pus = pl.redo ? a[5] : a[3];
  const double g2 = fmax(u2 - 2.0 / c.mu * pus + sGs / (c.mu * c.mu), 0.0);
  const double ng = sqrt(g2);
  pl.gamma = (ng <= c.R) ? 1.0 : c.R / ng;
  return pl;
}


// The plan's outcome and gamma for the tail kernel, written once per launch
// by the kernel that sizes Step 2 (every block of it computes the same plan).
__device__ __forceinline__ void publish_plan(const IterPtrs& p, const Step2Plan& pl) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    p.sc->redo = pl.redo;
    p.sc->gamma = pl.gamma;
  }
}

// Residuals of Section 4.3 from the reduced sums r[], computed in registers.
__device__ __forceinline__ void finish_etas(const Consts& c, const double* r, double* e) {
  const double den = c.opC;
  // (squared norms that are quadratic forms in n-space can round below 0)
  e[E_P1] = sqrt(r[R_PRES2]) / den;
  e[E_P2] = c.sqmu * sqrt(fmax(r[R_WU2], 0.0)) / den;
  e[E_P3] = fmax(sqrt(fmax(r[R_W2], 0.0)) - c.R, 0.0) / den;
  e[E_D1] = sqrt(r[R_AMIN2]) / den;
  e[E_D2] = sqrt(r[R_AMAX2]) / den;
  e[E_D3] = sqrt(fmax(r[R_DRES2], 0.0)) / den;
  e[E_C1] = fabs(r[R_YA]) / den;
  e[E_C2] = fabs(r[R_XCA]) / den;
  e[E_C3] = r[R_COMP2] / den;
  const double prim = r[R_SUMRQ] + c.C * r[R_SUMXI];  // sums carry v and e
  const double dual = c.kappa * r[R_SUMAQ] - c.R * sqrt(fmax(r[R_ZA2], 0.0));
  e[E_PRIM] = prim;
  e[E_DUAL] = dual;
  e[E_GAP] = fabs(prim - dual) / (1.0 + fabs(prim) + fabs(dual));
  e[E_P] = fmax(e[E_P1], fmax(e[E_P2], e[E_P3]));
  e[E_D] = fmax(e[E_D1], fmax(e[E_D2], c.rho_residual ? e[E_D3] : 0.0));
  e[E_C] = fmax(e[E_C1], fmax(e[E_C2], e[E_C3]));
}


// Stopping rule of Section 4.3 and sigma rule of Section 4.4 on the residuals
// e[] after iteration count k1; returns the new sigma and sets *stop.
__device__ __forceinline__ double stop_and_sigma(const Consts& c, const double* e, double sigma,
                                                 int k1, bool* stop) {
  const double pd = fmax(e[E_P], e[E_D]);
  const double cg_min = fmin(e[E_C], e[E_GAP]), cg_max = fmax(e[E_C], e[E_GAP]);
  *stop = pd < c.tol && cg_min < sqrt(c.tol) && cg_max < 0.05;
  if (*stop || k1 % c.sigma_every != 0) return sigma;
  const double ep = e[E_P], ed = e[E_D];
  if (ep >= 1e-300 && ed >= 1e-300) {
    const double chi = ep / ed;
    const double mm = fmax(chi, 1.0 / chi);
    const double zeta = mm > 500.0 ? 2.2 : (mm > 50.0 ? 1.65 : 1.1);
    if (chi > 5.0) return sigma * zeta;
    if (1.0 / chi > 5.0) return sigma / zeta;
  }
  return sigma;
}

// Block partials that decide Step 1c and size the Step 2 ball scaling:
// 0: dr^T G~ dr, 1: y^T dr, 2/3: s^T G~ s and (Z~^T u)^T s of outcome 0,
// 4/5: the same for outcome 1.
__device__ __forceinline__ double plan_part(const IterPtrs& p, int q, int b, int nb) {
  const double* r = p.part_c + b;
  switch (q) {
    case 0: return r[0];
    case 1: return p.part_n1[b];
    case 2: return r[(size_t)(1 + 9) * nb];
    case 3: return r[(size_t)(1 + 10) * nb];
    case 4: return r[(size_t)(1 + NPO + 9) * nb];
    default: return r[(size_t)(1 + NPO + 10) * nb];
  }
}

// Every thread loads its share of the partials first (one round trip), then
// one block reduction.
template <int NT>
__device__ __forceinline__ void plan_sums(const IterPtrs& p, int nb, double (&a)[6]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) a[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) {
#pragma unroll
    for (int j = 0; j < 6; ++j) a[j] += plan_part(p, j, b, nb);
  }
  block_sum_k<NT, 6>(a);
}

template <int NT>
__device__ __forceinline__ Step2Plan step2_plan(const Consts& c, const IterPtrs& p) {
  const int k = p.sc->k;
  const double u2 = p.sc->u2;
  double a[6];
  plan_sums<NT>(p, ngemv_blocks(c.n), a);
  return step2_plan_finish(c, a, k, u2);
}

}  // namespace dwd
