// Setup kernels: data scaling (Section 4.2), the Gram matrix Z~^T Z~ and
// the inverse of M = I_n + Z~^T D^-1 Z~ (the first diagonal block of J in
// eq-H, Section 3.3.2).  All of this runs once per problem.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "dwd_internal.h"

namespace dwd {

// ---------------------------------------------------------------------------
// a0: copy X (d x n, column-major, ld_in = d) into padded device storage and
// accumulate ||X||_F^2 in FP64.  For BF16 storage both an FP32 image (data
// of record) and a BF16 image are written.
// grid = (n, chunks); part[chunk * n + col] receives the block's sum.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  uint32_t lsb = (b >> 16) & 1u;
  b += 0x7FFFu + lsb;
  return (uint16_t)(b >> 16);
}

template <typename Tin>
__global__ void __launch_bounds__(256) k_frob_copy(const Tin* __restrict__ X, int64_t d, int n,
                                                   void* __restrict__ Xs, int storage, int64_t ld,
                                                   uint16_t* __restrict__ X16,
                                                   double* __restrict__ part) {
  const int col = blockIdx.x;
  const int64_t per = (ld + gridDim.y - 1) / gridDim.y;
  const int64_t r0 = (int64_t)blockIdx.y * per;
  const int64_t r1 = min(ld, r0 + per);
  double acc = 0.0;
  for (int64_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) {
    double v = 0.0;
    if (k < d) v = (double)X[(int64_t)col * d + k];
    acc += v * v;
    const int64_t o = (int64_t)col * ld + k;
    if (storage == DWD_FP64) {
      ((double*)Xs)[o] = v;
    } else {
      float f = (float)v;
      ((float*)Xs)[o] = f;
      if (X16) X16[o] = f32_to_bf16_rne(f);
    }
  }
  acc = block_sum<256>(acc);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * n + col] = acc;
}

hipError_t launch_frob_copy(const void* X, int in_dtype, int64_t d, int n, void* Xs, int storage,
                            int64_t ld, double* part, int nparts_y, hipStream_t st) {
  // storage == DWD_BF16: Xs is the FP32 image and the BF16 image follows it
  // at (char*)Xs + ld*n*4 (allocated contiguously by the caller).
  uint16_t* X16 = nullptr;
  int st_eff = storage;
  if (storage == DWD_BF16) {
    X16 = (uint16_t*)((char*)Xs + (size_t)ld * n * sizeof(float));
    st_eff = DWD_FP32;
  }
  dim3 grid(n, nparts_y);
  if (in_dtype == DWD_FP64)
    hipLaunchKernelGGL(k_frob_copy<double>, grid, dim3(256), 0, st, (const double*)X, d, n, Xs,
                       st_eff, ld, X16, part);
  else
    hipLaunchKernelGGL(k_frob_copy<float>, grid, dim3(256), 0, st, (const float*)X, d, n, Xs,
                       st_eff, ld, X16, part);
  return hipGetLastError();
}

// Deterministic sum of `count` doubles by one block.
__global__ void __launch_bounds__(1024) k_sum(const double* __restrict__ part, int count,
                                              double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += part[i];
  acc = block_sum<1024>(acc);
  if (threadIdx.x == 0) *out = acc;
}

hipError_t launch_sum(const double* part, int count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, part, count, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a1: Gram matrix X^T X (n x n) in FP64, upper-triangular 64x64 tiles,
// split over the d dimension into `splits` partial tiles (summed in a fixed
// order by k_gram_finish).  FP64 MFMA 16x16x4: each of the 4 waves of a
// block owns a 32x32 quarter of the 64x64 tile (2x2 MFMA blocks).
// ---------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int GT = 64;   // tile edge
constexpr int GK = 32;   // k-depth per LDS stage (divides the padded ld)

// Stage GK x 64 of the columns c0.. of the stored data into LDS as FP64,
// with 16-byte loads along k (the contiguous direction).
template <typename T>
__device__ __forceinline__ void gram_stage(const void* Xs, int64_t ld, int n, int c0, int64_t kb,
                                           double (*S)[GT + 1]) {
  constexpr int V = 16 / sizeof(T);             // elements per 16-byte load
  constexpr int PER_COL = GK / V;
  for (int e = threadIdx.x; e < GT * PER_COL; e += 256) {
    const int c = e / PER_COL, kq = (e % PER_COL) * V;
    const int gc = c0 + c;
    if (gc < n) {
      if constexpr (sizeof(T) == 8) {
        const double2 v = *reinterpret_cast<const double2*>((const double*)Xs + (int64_t)gc * ld +
                                                           kb + kq);
        S[kq][c] = v.x;
        S[kq + 1][c] = v.y;
      } else if constexpr (sizeof(T) == 2) {
        // BF16: the upper 16 bits of an FP32 value
        const uint4 v = *reinterpret_cast<const uint4*>((const uint16_t*)Xs + (int64_t)gc * ld +
                                                        kb + kq);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          S[kq + 2 * q][c] = (double)__uint_as_float(w[q] << 16);
          S[kq + 2 * q + 1][c] = (double)__uint_as_float(w[q] & 0xFFFF0000u);
        }
      } else {
        const float4 v = *reinterpret_cast<const float4*>((const float*)Xs + (int64_t)gc * ld +
                                                         kb + kq);
        S[kq][c] = v.x;
        S[kq + 1][c] = v.y;
        S[kq + 2][c] = v.z;
        S[kq + 3][c] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < V; ++q) S[kq + q][c] = 0.0;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gram_mfma(const void* __restrict__ Xs, int64_t ld, int n,
                                                   int ntile, int splits,
                                                   double* __restrict__ Gpart) {
  // tile index -> (ti, tj), tj >= ti
  int t = blockIdx.x;
  int ti = 0;
  while (t >= ntile - ti) { t -= ntile - ti; ++ti; }
  const int tj = ti + t;
  const int split = blockIdx.y;
  const int64_t per = ((ld / GK + splits - 1) / splits) * GK;
  const int64_t k0 = (int64_t)split * per;
  const int64_t k1 = min(ld, k0 + per);

  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;           // 0..3
  const int wr = (wid >> 1) * 32;     // wave's row offset in tile
  const int wc = (wid & 1) * 32;      // wave's col offset
  const int i0 = ti * GT, j0 = tj * GT;

  d4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (d4v){0.0, 0.0, 0.0, 0.0};

  for (int64_t kb = k0; kb < k1; kb += GK) {
    gram_stage<T>(Xs, ld, n, i0, kb, As);
    gram_stage<T>(Xs, ld, n, j0, kb, Bs);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      // A operand: element (row i = lane%16, k = lane/16) of a 16x4 block
      // B operand: element (k = lane/16, col j = lane%16) of a 4x16 block
      const int li = lane & 15, lk = lane >> 4;
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[ks + lk][wr + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[ks + lk][wc + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of the FP64 16x16 block: column j = lane%16; lane group
  // g = lane/16 holds rows g, g+4, g+8, g+12 in registers 0..3.
  double* out = Gpart + (size_t)split * n * n;
  const int lj = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = i0 + wr + a * 16 + v * 4 + lg;
        const int gj = j0 + wc + b * 16 + lj;
        if (gi < n && gj < n) out[(size_t)gi * n + gj] = acc[a][b][v];
      }
}

int gram_splits(int64_t ld, int n) {
  const int nt = (n + GT - 1) / GT;
  const int tiles = nt * (nt + 1) / 2;
  int s = (2048 + tiles - 1) / tiles;           // aim for >= 2048 blocks
  const int64_t kmax = ld / GK;
  if (s > kmax) s = (int)kmax;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return s;
}

hipError_t launch_gram(const void* Xs, int storage, int64_t ld, int n, double* Gpart, int splits,
                       hipStream_t st) {
  const int nt = (n + GT - 1) / GT;
  dim3 grid(nt * (nt + 1) / 2, splits);
  if (storage == DWD_FP64)
    hipLaunchKernelGGL(k_gram_mfma<double>, grid, dim3(256), 0, st, Xs, ld, n, nt, splits, Gpart);
  else if (storage == DWD_BF16)
    hipLaunchKernelGGL(k_gram_mfma<uint16_t>, grid, dim3(256), 0, st, Xs, ld, n, nt, splits,
                       Gpart);
  else
    hipLaunchKernelGGL(k_gram_mfma<float>, grid, dim3(256), 0, st, Xs, ld, n, nt, splits, Gpart);
  return hipGetLastError();
}

// G~_ij = y_i y_j (sum_s Gpart[s]_ij) / Z_scale^2 for the upper-tile entry,
// mirrored; M = I + G~/mu.
__global__ void __launch_bounds__(256) k_gram_finish(const double* __restrict__ Gpart, int splits,
                                                     int n, const double* __restrict__ y,
                                                     double inv_zs2, double mu,
                                                     double* __restrict__ G,
                                                     double* __restrict__ M) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  // entry stored in the upper tile triangle: tile(i) <= tile(j)
  int a = i, b = j;
  if (i / GT > j / GT) { a = j; b = i; }
  double s = 0.0;
  for (int p = 0; p < splits; ++p) s += Gpart[(size_t)p * n * n + (size_t)a * n + b];
  const double g = y[i] * y[j] * s * inv_zs2;
  G[idx] = g;
  M[idx] = (i == j ? 1.0 : 0.0) + g / mu;
}

hipError_t launch_gram_finish(const double* Gpart, int splits, int n, const double* y,
                              double inv_zs2, double mu, double* G, double* M, hipStream_t st) {
  const int64_t tot = (int64_t)n * n;
  hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Gpart,
                     splits, n, y, inv_zs2, mu, G, M);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a2: inverse of the SPD matrix M by Schur-complement recursion:
//   M = [A B; B^T C],  A^-1 by recursion, T = A^-1 B, S = C - B^T T,
//   S^-1 by recursion, M^-1 = [A^-1 + T S^-1 T^T, -T S^-1; (.)^T, S^-1].
// This is block LDL^T elimination (no pivoting is needed for SPD M, whose
// eigenvalues are >= 1 here).  Leaves of size <= 64 are inverted in LDS by
// Gauss-Jordan elimination with the diagonal pivots (positive for SPD).
// ---------------------------------------------------------------------------
constexpr int LEAF = 64;

__global__ void __launch_bounds__(256) k_spd_leaf_inv(double* __restrict__ M, int ldm, int m,
                                                      int* __restrict__ status) {
  // Thread t holds row i = t/4, columns [16*(t%4), 16*(t%4) + 16) in
  // registers; the block beyond m x m is the identity, which the
  // elimination leaves unchanged.
  __shared__ double prow[LEAF];
  __shared__ double pcol[LEAF];
  const int tid = threadIdx.x;
  const int i = tid >> 2;
  const int j0 = (tid & 3) * 16;
  double a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = j0 + q;
    a[q] = (i < m && j < m) ? M[(size_t)i * ldm + j] : (i == j ? 1.0 : 0.0);
  }
  for (int p = 0; p < m; ++p) {
    if (i == p) {
#pragma unroll
      for (int q = 0; q < 16; ++q) prow[j0 + q] = a[q];
    }
    if (p >= j0 && p < j0 + 16) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (j0 + q == p) pcol[i] = a[q];
    }
    __syncthreads();
    const double piv = prow[p];
    if (!(piv > 0.0)) {  // not positive definite (or NaN): same branch in every thread
      if (tid == 0) atomicExch(status, 1);
      return;
    }
    const double ip = 1.0 / piv;
    if (i == p) {
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = (j0 + q == p) ? ip : a[q] * ip;
    } else {
      const double f = pcol[i];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int j = j0 + q;
        a[q] = (j == p) ? -f * ip : fma(-f * ip, prow[j], a[q]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int j = j0 + q;
    if (i < m && j < m) M[(size_t)i * ldm + j] = a[q];
  }
}

// C(mxn) = alpha * op(A) op(B) + beta * C, row-major, FP64, 64x64 tiles.
// op(A) is m x k: transA=0 -> A[i*lda + l], 1 -> A[l*lda + i].
// op(B) is k x n: transB=0 -> B[l*ldb + j], 1 -> B[j*ldb + l].
__global__ void __launch_bounds__(256) k_gemm_f64(int m, int n, int k, double alpha,
                                                  const double* __restrict__ A, int lda, int ta,
                                                  const double* __restrict__ B, int ldb, int tb,
                                                  double beta, double* __restrict__ C, int ldc) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  double acc[4][4] = {};
  for (int l0 = 0; l0 < k; l0 += 16) {
    // consecutive threads read consecutive addresses of the stored layout
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      int ll, c;
      if (ta) { ll = e >> 6; c = e & 63; } else { c = e >> 4; ll = e & 15; }
      const int gi = i0 + c, gl = l0 + ll;
      double va = 0.0;
      if (gi < m && gl < k) va = ta ? A[(size_t)gl * lda + gi] : A[(size_t)gi * lda + gl];
      As[ll][c] = va;
    }
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      int ll, c;
      if (tb) { c = e >> 4; ll = e & 15; } else { ll = e >> 6; c = e & 63; }
      const int gj = j0 + c, gl = l0 + ll;
      double vb = 0.0;
      if (gj < n && gl < k) vb = tb ? B[(size_t)gj * ldb + gl] : B[(size_t)gl * ldb + gj];
      Bs[ll][c] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int ll = 0; ll < 16; ++ll) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = As[ll][ty * 4 + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[ll][tx * 4 + q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gi = i0 + ty * 4 + p, gj = j0 + tx * 4 + q;
      if (gi < m && gj < n) {
        const size_t o = (size_t)gi * ldc + gj;
        C[o] = alpha * acc[p][q] + (beta == 0.0 ? 0.0 : beta * C[o]);
      }
    }
}

// Dst(n2 x n1) = Src(n1 x n2)^T
__global__ void k_transpose(const double* __restrict__ S, int lds_, double* __restrict__ D,
                            int ldd, int r, int c) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)r * c) return;
  const int i = (int)(idx / c), j = (int)(idx % c);
  D[(size_t)j * ldd + i] = S[(size_t)i * lds_ + j];
}

static hipError_t gemm(int m, int n, int k, double alpha, const double* A, int lda, int ta,
                       const double* B, int ldb, int tb, double beta, double* C, int ldc,
                       hipStream_t st) {
  dim3 grid((n + 63) / 64, (m + 63) / 64);
  hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, st, m, n, k, alpha, A, lda, ta, B, ldb, tb,
                     beta, C, ldc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inverse of the SPD matrix M (n x n, row-major) in place by block sweeps
// (Gauss-Jordan elimination in the symmetric sign convention) over block
// columns K of width GJB.  Sweep K, with P = A[K,K]^-1 and R = P A[K,:]:
//   A[K,K] <- -P,  A[K,J] <- R[:,J],  A[I,K] <- A[I,K] P = R[:,I]^T,
//   A[I,J] <- A[I,J] - A[I,K] R[:,J]      (I, J != K).
// Each sweep keeps A symmetric, so one saved row panel serves as the column
// panel too; sweeping every block leaves -M^-1, negated at the end.  No
// pivoting: the pivot blocks are Schur complements of the SPD I + G~/mu.
// ---------------------------------------------------------------------------
constexpr int GJB = 32;  // pivot block width
constexpr int GJT = 64;  // output tile edge of the panel and update kernels

// One lane's double, read by the whole wave (lane p uniform).
__device__ __forceinline__ double lane_value(double v, int p) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, p);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), p);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// P = A[K,K]^-1 by Gauss-Jordan in one wave: lane i < GJB holds row i of the
// block in registers (rows beyond m are the identity; lanes >= GJB carry
// identity rows that no result uses); the pivot row is read lane by lane
// into scalar registers.  Writes P into Pbuf (GJB x GJB, row-major) and -P
// into A[K,K].
__global__ void __launch_bounds__(64) k_gj_pivot(double* __restrict__ M, int ld, int k0, int m,
                                                 double* __restrict__ Pbuf,
                                                 int* __restrict__ status) {
  const int i = threadIdx.x;
  double a[GJB];
#pragma unroll
  for (int j = 0; j < GJB; ++j)
    a[j] = (i < m && j < m) ? M[(size_t)(k0 + i) * ld + k0 + j] : (i == j ? 1.0 : 0.0);
  bool ok = true;
#pragma unroll
  for (int p = 0; p < GJB; ++p) {
    double rowp[GJB];
#pragma unroll
    for (int j = 0; j < GJB; ++j) rowp[j] = lane_value(a[j], p);
    const double piv = rowp[p];
    ok = ok && (piv > 0.0);
    const double ip = 1.0 / piv;
    if (i == p) {
#pragma unroll
      for (int j = 0; j < GJB; ++j) a[j] = (j == p) ? ip : a[j] * ip;
    } else {
      const double g = -a[p] * ip;
#pragma unroll
      for (int j = 0; j < GJB; ++j) a[j] = (j == p) ? g : fma(g, rowp[j], a[j]);
    }
  }
  if (i < GJB) {
    if (!ok && i == 0) atomicExch(status, 1);
#pragma unroll
    for (int j = 0; j < GJB; ++j) {
      Pbuf[i * GJB + j] = a[j];
      if (i < m && j < m) M[(size_t)(k0 + i) * ld + k0 + j] = -a[j];
    }
  }
}

// Row panel: for every column gj outside K, R[:, gj] = P A[K, gj]; keeps the
// old values in Rk and writes R into A[K, gj] and Rbuf.  Block = 64 columns.
__global__ void __launch_bounds__(256) k_gj_panel(double* __restrict__ M, int ld, int n, int k0,
                                                  int m, const double* __restrict__ Pbuf,
                                                  double* __restrict__ Rbuf,
                                                  double* __restrict__ Rk) {
  const int j0 = blockIdx.x * GJT;
  __shared__ double Ps[GJB][GJB + 1];
  __shared__ double As[GJB][GJT + 1];
  for (int e = threadIdx.x; e < GJB * GJB; e += 256) Ps[e / GJB][e % GJB] = Pbuf[e];
  for (int e = threadIdx.x; e < GJB * GJT; e += 256) {
    const int r = e / GJT, cc = e % GJT, gj = j0 + cc;
    As[r][cc] = (r < m && gj < n) ? M[(size_t)(k0 + r) * ld + gj] : 0.0;
  }
  __syncthreads();
  // thread: row r = t / 8 of R (GJB = 32 rows), columns 8 (t % 8) .. +7
  const int r = threadIdx.x >> 3, c0 = (threadIdx.x & 7) * 8;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 4
  for (int l = 0; l < GJB; ++l) {
    const double pv = Ps[r][l];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = fma(pv, As[l][c0 + q], acc[q]);
  }
  if (r < m) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int gj = j0 + c0 + q;
      if (gj < n && (gj < k0 || gj >= k0 + m)) {
        Rbuf[(size_t)r * n + gj] = acc[q];
        Rk[(size_t)r * n + gj] = As[r][c0 + q];
        M[(size_t)(k0 + r) * ld + gj] = acc[q];
      }
    }
  }
}

// For every element (gi, gj) with gi outside K:
//   gj in K:   A[gi, gj] = R[gj - k0, gi]        (= (A[gi, K] P)_gj by symmetry)
//   otherwise: A[gi, gj] -= sum_l Rk[l, gi] R[l, gj]   (A[gi, K] = Rk[:, gi]^T)
// Block = 64 x 64 output tile, thread = 4 x 4 outputs.
__global__ void __launch_bounds__(256) k_gj_update(double* __restrict__ M, int ld, int n, int k0,
                                                   int m, const double* __restrict__ Rbuf,
                                                   const double* __restrict__ Rk) {
  const int i0 = blockIdx.y * GJT, j0 = blockIdx.x * GJT;
  if (i0 >= k0 && i0 + GJT <= k0 + m) return;  // tile rows all inside K (not for GJB < GJT)
  __shared__ double Cs[GJB][GJT + 1];  // Cs[l][r] = Rk[l][i0 + r]
  __shared__ double Bs[GJB][GJT + 1];  // Bs[l][c] = R[l][j0 + c]
  for (int e = threadIdx.x; e < GJB * GJT; e += 256) {
    const int l = e / GJT, cc = e % GJT;
    const int gi = i0 + cc, gj = j0 + cc;
    const bool gi_out = gi < n && (gi < k0 || gi >= k0 + m);
    const bool gj_out = gj < n && (gj < k0 || gj >= k0 + m);
    Cs[l][cc] = (l < m && gi_out) ? Rk[(size_t)l * n + gi] : 0.0;
    Bs[l][cc] = (l < m && gj_out) ? Rbuf[(size_t)l * n + gj] : 0.0;
  }
  __syncthreads();
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  double acc[4][4] = {};
#pragma unroll 4
  for (int l = 0; l < GJB; ++l) {
    double ca[4], bb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ca[q] = Cs[l][tr * 4 + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) bb[q] = Bs[l][tc * 4 + q];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int yq = 0; yq < 4; ++yq) acc[x][yq] = fma(ca[x], bb[yq], acc[x][yq]);
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int yq = 0; yq < 4; ++yq) {
      const int gi = i0 + tr * 4 + x, gj = j0 + tc * 4 + yq;
      if (gi >= n || gj >= n || (gi >= k0 && gi < k0 + m)) continue;
      if (gj >= k0 && gj < k0 + m)
        M[(size_t)gi * ld + gj] = Rbuf[(size_t)(gj - k0) * n + gi];
      else
        M[(size_t)gi * ld + gj] -= acc[x][yq];
    }
}

__global__ void k_negate(double* __restrict__ v, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) v[i] = -v[i];
}

size_t spd_inverse_work(int n) { return (size_t)GJB * GJB + 2 * (size_t)GJB * n; }

// work holds >= spd_inverse_work(n) doubles.
hipError_t spd_inverse_inplace(double* M, int n, double* work, int* d_status, hipStream_t st) {
  double* Pbuf = work;
  double* Rbuf = work + GJB * GJB;
  double* Rk = Rbuf + (size_t)GJB * n;
  const int nt = (n + GJB - 1) / GJB;
  const int nto = (n + GJT - 1) / GJT;
  for (int kb = 0; kb < nt; ++kb) {
    const int k0 = kb * GJB, m = std::min(GJB, n - k0);
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(64), 0, st, M, n, k0, m, Pbuf, d_status);
    if (nt > 1) {
      hipLaunchKernelGGL(k_gj_panel, dim3(nto), dim3(256), 0, st, M, n, n, k0, m, Pbuf, Rbuf, Rk);
      hipLaunchKernelGGL(k_gj_update, dim3(nto, nto), dim3(256), 0, st, M, n, n, k0, m, Rbuf, Rk);
    }
  }
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(k_negate, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, M, nn);
  return hipGetLastError();
}

// out = A x, A n x n row-major FP64; one wave per row.
__global__ void __launch_bounds__(256) k_gemv_rows(const double* __restrict__ A, int n,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ out) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double acc = 0.0;
  for (int j = lane; j < n; j += 64) acc += A[(size_t)row * n + j] * x[j];
  acc = wave_sum(acc);
  if (lane == 0) out[row] = acc;
}

hipError_t launch_gemv_rows(const double* A, int n, const double* x, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_rows, dim3((n + 3) / 4), dim3(256), 0, st, A, n, x, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(1024) k_dot(const double* __restrict__ a,
                                              const double* __restrict__ b, int n,
                                              double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += a[i] * b[i];
  acc = block_sum<1024>(acc);
  if (threadIdx.x == 0) *out = acc;
}

hipError_t launch_dot(const double* a, const double* b, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dot, dim3(1), dim3(1024), 0, st, a, b, n, out);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Section 4.1 choice of C: one histogram step of an exact radix selection over
// the squared between-class distances, scaled by 1/Z_scale^2,
//     ||x_i - x_j||^2 / Z_scale^2 = G~_ii + G~_jj + 2 G~_ij   (y_i = +1, y_j = -1),
// keyed by their IEEE-754 bit patterns, which order non-negative doubles as
// unsigned integers.  Pairs whose key equals `prefix` in the bits above
// shift + 8 are counted into hist[256] by the digit (key >> shift) & 255.
// Nothing is stored per pair; each step re-evaluates them from G~.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_pair_hist(const double* __restrict__ G, int n,
                                                   const int* __restrict__ ipos, int npos,
                                                   const int* __restrict__ ineg, int nneg,
                                                   unsigned long long prefix, int shift,
                                                   unsigned int* __restrict__ hist) {
  __shared__ unsigned int h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t total = (int64_t)npos * nneg;
  const int hi = shift + 8;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int a = (int)(t / nneg);
    const int b = (int)(t - (int64_t)a * nneg);
    const size_t i = (size_t)ipos[a], j = (size_t)ineg[b];
    const double s = G[i * n + i] + G[j * n + j] + 2.0 * G[i * n + j];
    const double v = s > 0.0 ? s : 0.0;  // (+0 for rounding below zero and for -0)
    const unsigned long long key = (unsigned long long)__double_as_longlong(v);
    if (hi < 64 && (key >> hi) != (prefix >> hi)) continue;
    atomicAdd(&h[(key >> shift) & 255ull], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

hipError_t launch_pair_hist(const double* G, int n, const int* ipos, int npos, const int* ineg,
                            int nneg, unsigned long long prefix, int shift, unsigned int* hist,
                            hipStream_t st) {
  const int64_t total = (int64_t)npos * nneg;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (total + 255) / 256));
  hipLaunchKernelGGL(k_pair_hist, dim3(blocks), dim3(256), 0, st, G, n, ipos, npos, ineg, nneg,
                     prefix, shift, hist);
  return hipGetLastError();
}

}  // namespace dwd
