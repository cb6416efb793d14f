// Sparse data (CSR).  X is kept twice on the device: CSR of X^T (one row per
// sample i, for Z~^T v) and CSR of X (one row per feature k, for Z~ s); the
// column indices of every row are sorted.  The label signs and 1/Z_scale are
// folded into the n-vectors exactly as for dense storage, so the n-space
// kernels are shared with the dense path.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dwd_device.h"
#include "dwd_internal.h"

namespace dwd {

// ||X||_F^2 partials over the nonzeros.
template <typename T>
__global__ void __launch_bounds__(256) k_csr_frob(const T* __restrict__ val, int64_t nnz,
                                                  double* __restrict__ part) {
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
    const double v = (double)val[e];
    acc += v * v;
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

hipError_t launch_csr_frob(const void* val, int dtype, int64_t nnz, double* part, int nblk,
                           hipStream_t st) {
  if (dtype == DWD_FP64)
    hipLaunchKernelGGL(k_csr_frob<double>, dim3(nblk), dim3(256), 0, st, (const double*)val, nnz,
                       part);
  else
    hipLaunchKernelGGL(k_csr_frob<float>, dim3(nblk), dim3(256), 0, st, (const float*)val, nnz,
                       part);
  return hipGetLastError();
}

// Gram X^T X from CSR(X^T): G_ij = sparse dot of sample rows i and j by a
// merge of their sorted index lists (one thread per (i, j), j >= i; fixed
// order, so deterministic).  Writes the upper triangle into Gpart (split 0),
// in the layout k_gram_finish reads (mirrored there).
template <typename T>
__global__ void __launch_bounds__(256) k_csr_gram(const int64_t* __restrict__ ip,
                                                  const int32_t* __restrict__ ix,
                                                  const T* __restrict__ val, int n,
                                                  double* __restrict__ G) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n || j < i) return;
  int64_t a = ip[i], ae = ip[i + 1], b = ip[j], be = ip[j + 1];
  double acc = 0.0;
  while (a < ae && b < be) {
    const int ca = ix[a], cb = ix[b];
    if (ca == cb) {
      acc = fma((double)val[a], (double)val[b], acc);
      ++a;
      ++b;
    } else if (ca < cb) {
      ++a;
    } else {
      ++b;
    }
  }
  G[(size_t)i * n + j] = acc;
  G[(size_t)j * n + i] = acc;
}

hipError_t launch_csr_gram(const int64_t* ip, const int32_t* ix, const void* val, int dtype, int n,
                           double* G, hipStream_t st) {
  dim3 grid((n + 255) / 256, n);
  if (dtype == DWD_FP64)
    hipLaunchKernelGGL(k_csr_gram<double>, grid, dim3(256), 0, st, ip, ix, (const double*)val, n,
                       G);
  else
    hipLaunchKernelGGL(k_csr_gram<float>, grid, dim3(256), 0, st, ip, ix, (const float*)val, n,
                       G);
  return hipGetLastError();
}

// Z~^T [v1, v2] per sample: one wave per row of CSR(X^T); results go to
// partT chunk 0 ([0*n + i] and [1*n + i]) as the dense pass would write them.
template <typename T>
__global__ void __launch_bounds__(256) k_csr_gemvT(const int64_t* __restrict__ ip,
                                                   const int32_t* __restrict__ ix,
                                                   const T* __restrict__ val, int n,
                                                   const double* __restrict__ v1,
                                                   const double* __restrict__ v2,
                                                   double* __restrict__ part,
                                                   const Scal* __restrict__ sc) {
  if (sc && sc->done) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t e = ip[i] + lane; e < ip[i + 1]; e += 64) {
    const double x = (double)val[e];
    const int k = ix[e];
    s1 = fma(x, v1[k], s1);
    s2 = fma(x, v2[k], s2);
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    part[i] = s1;
    part[(size_t)n + i] = s2;
  }
}

hipError_t launch_csr_gemvT(const int64_t* ip, const int32_t* ix, const void* val, int dtype,
                            int n, const double* v1, const double* v2, double* part,
                            const Scal* sc, hipStream_t st) {
  if (!ip || !ix || !val || !v1 || !v2 || !part) return hipErrorInvalidValue;
  if (dtype == DWD_FP64)
    hipLaunchKernelGGL(k_csr_gemvT<double>, dim3((n + 3) / 4), dim3(256), 0, st, ip, ix,
                       (const double*)val, n, v1, v2, part, sc);
  else
    hipLaunchKernelGGL(k_csr_gemvT<float>, dim3((n + 3) / 4), dim3(256), 0, st, ip, ix,
                       (const float*)val, n, v1, v2, part, sc);
  return hipGetLastError();
}

// The pass Z~ [s, alpha] over CSR(X) (one thread per feature row k < ld;
// rows k >= d are empty), fused with Steps 2-3 exactly as the dense pass
// (k_pass2 with FUSED = true), writing the same NP2 block partials.
constexpr int CSR_T = 256;

template <typename T>
__global__ void __launch_bounds__(CSR_T) k_csr_pass(const int64_t* __restrict__ ip,
                                                    const int32_t* __restrict__ ix,
                                                    const T* __restrict__ val, int64_t d,
                                                    Consts c, IterPtrs p) {
  if (p.sc->done) return;
  const Step2Plan pl = step2_plan<CSR_T>(c, p);
  publish_plan(p, pl);
  const double* ss = pl.redo ? p.s1 : p.s;
  const double* sa = pl.redo ? p.al1 : p.al0;
  const double sigma = p.sc->sigma;
  const double gamma = pl.gamma;
  const double br = c.sqmu / sigma, gr = 1.0 / (sigma * c.sqmu);
  const double rs = c.tau * sigma * c.sqmu;
  double acc[NP2] = {0, 0, 0, 0, 0, 0};
  const int64_t k = (int64_t)blockIdx.x * CSR_T + threadIdx.x;
  if (k < c.ld) {
    double zs = 0.0, za = 0.0;
    if (k < d) {
      for (int64_t e = ip[k]; e < ip[k + 1]; ++e) {
        const int i = ix[e];
        const double x = (double)val[e] * p.y[i] * c.inv_zs;
        zs = fma(x, ss[i], zs);
        za = fma(x, sa[i], za);
      }
    }
    const double rho = p.rho[k];
    const double b = c.mu * p.u[k] + br * rho;
    const double w = (b - zs) / c.mu;
    const double u = gamma * (w - gr * rho);
    const double rn = rho - rs * (w - u);
    p.w[k] = w;
    p.u[k] = u;
    p.rho[k] = rn;
    const double dres = za + c.sqmu * rn;
    acc[0] = (w - u) * (w - u);
    acc[1] = w * w;
    acc[2] = dres * dres;
    acc[3] = za * za;
    acc[4] = rn * rn;
    acc[5] = u * u;
  }
  block_sum_k<CSR_T, NP2>(acc);
  if (threadIdx.x < NP2) p.part_g[(size_t)threadIdx.x * p.pg_ld + blockIdx.x] = acc[threadIdx.x];
}

// Expansion of the representer coefficients over CSR(X): w~ = Z~ aw,
// u~ = Z~ au, rho = Z~ arho, one thread per feature row k < ld.
template <typename T>
__global__ void __launch_bounds__(CSR_T) k_csr_expand(const int64_t* __restrict__ ip,
                                                      const int32_t* __restrict__ ix,
                                                      const T* __restrict__ val, int64_t d,
                                                      Consts c, IterPtrs p) {
  const int64_t k = (int64_t)blockIdx.x * CSR_T + threadIdx.x;
  if (k >= c.ld) return;
  double w = 0.0, u = 0.0, r = 0.0;
  if (k < d) {
    for (int64_t e = ip[k]; e < ip[k + 1]; ++e) {
      const int i = ix[e];
      const double x = (double)val[e] * p.y[i] * c.inv_zs;
      w = fma(x, p.aw[i], w);
      u = fma(x, p.au[i], u);
      r = fma(x, p.arho[i], r);
    }
  }
  p.w[k] = w;
  p.u[k] = u;
  p.rho[k] = r;
}

hipError_t launch_csr_expand(const int64_t* ip, const int32_t* ix, const void* val, int dtype,
                             int64_t d, const Consts& c, const IterPtrs& p, hipStream_t st) {
  if (!ip || !ix || !val) return hipErrorInvalidValue;
  const int nb = (int)((c.ld + CSR_T - 1) / CSR_T);
  if (dtype == DWD_FP64)
    hipLaunchKernelGGL(k_csr_expand<double>, dim3(nb), dim3(CSR_T), 0, st, ip, ix,
                       (const double*)val, d, c, p);
  else
    hipLaunchKernelGGL(k_csr_expand<float>, dim3(nb), dim3(CSR_T), 0, st, ip, ix,
                       (const float*)val, d, c, p);
  return hipGetLastError();
}

// Explicit ||Z~ alpha + D rho||^2 for the final check over CSR(X): one thread
// per feature row, per-block partials.
template <typename T>
__global__ void __launch_bounds__(CSR_T) k_csr_dres(const int64_t* __restrict__ ip,
                                                    const int32_t* __restrict__ ix,
                                                    const T* __restrict__ val, int64_t d,
                                                    Consts c, const double* __restrict__ alpha,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ rho,
                                                    double* __restrict__ part) {
  const int64_t k = (int64_t)blockIdx.x * CSR_T + threadIdx.x;
  double s2 = 0.0;
  if (k < c.ld) {
    double za = 0.0;
    if (k < d)
      for (int64_t e = ip[k]; e < ip[k + 1]; ++e) {
        const int i = ix[e];
        za = fma((double)val[e] * y[i] * c.inv_zs, alpha[i], za);
      }
    const double dr = za + c.sqmu * rho[k];
    s2 = dr * dr;
  }
  s2 = block_sum<CSR_T>(s2);
  if (threadIdx.x == 0) part[blockIdx.x] = s2;
}

hipError_t launch_csr_dres(const int64_t* ip, const int32_t* ix, const void* val, int dtype,
                           int64_t d, const Consts& c, const double* alpha, const double* y,
                           const double* rho, double* part, hipStream_t st) {
  if (!ip || !ix || !val || !alpha || !y || !rho || !part) return hipErrorInvalidValue;
  const int nb = (int)((c.ld + CSR_T - 1) / CSR_T);
  if (dtype == DWD_FP64)
    hipLaunchKernelGGL(k_csr_dres<double>, dim3(nb), dim3(CSR_T), 0, st, ip, ix,
                       (const double*)val, d, c, alpha, y, rho, part);
  else
    hipLaunchKernelGGL(k_csr_dres<float>, dim3(nb), dim3(CSR_T), 0, st, ip, ix,
                       (const float*)val, d, c, alpha, y, rho, part);
  return hipGetLastError();
}

int csr_pass_blocks(int64_t ld) { return (int)((ld + CSR_T - 1) / CSR_T); }

hipError_t launch_csr_pass(const int64_t* ip, const int32_t* ix, const void* val, int dtype,
                           int64_t d, const Consts& c, const IterPtrs& p, hipStream_t st) {
  if (!ip || !ix || !val) return hipErrorInvalidValue;
  const int nb = csr_pass_blocks(c.ld);
  if (nb > p.pg_ld) return hipErrorInvalidValue;
  if (dtype == DWD_FP64)
    hipLaunchKernelGGL(k_csr_pass<double>, dim3(nb), dim3(CSR_T), 0, st, ip, ix,
                       (const double*)val, d, c, p);
  else
    hipLaunchKernelGGL(k_csr_pass<float>, dim3(nb), dim3(CSR_T), 0, st, ip, ix,
                       (const float*)val, d, c, p);
  return hipGetLastError();
}

}  // namespace dwd
