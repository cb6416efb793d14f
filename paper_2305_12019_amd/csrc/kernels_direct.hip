// Direct branch of eq-linsys (Section 3.3.1, d much smaller than n): T = 0
// and the whole (d+1) x (d+1) matrix
//     A = [[Z~ Z~^T + mu I, Z~ y], [(Z~ y)^T, y^T y]]
// formed once and inverted explicitly (one (d+1)^2 GEMV per solve in place
// of two triangular solves).  One iteration of Algorithm 1 reads Z twice,
// each time in one fused sweep over the samples:
//
//   sweep 1: z_i = (Z~^T wbar)_i, Step 1b prox c_i -> r_i^+, dr_i, and the
//            partial sums of Z~ dr (Step 1c residual and re-solve);
//   sweep 2: z_i = (Z~^T w)_i (reused from sweep 1 when Step 1c kept wbar),
//            Step 2 xi_i, Step 3 alpha_i, the n-space terms of Section 4.3,
//            and the partial sums of Z~ (xi - r) and Z~ alpha (the next
//            right-hand side and eta_D3).
//
// A sample's data is read once per sweep and used both for its dot product
// and for its share of the d-vector sums.  Samples are split over blocks;
// inside a block, groups of TPS threads each take one sample at a time, a
// thread holding NF feature quads (4 consecutive features) of it.  The
// block partials of the d-vector sums are reduced by a separate kernel in a
// fixed order (results do not depend on timing).
//
// Data layout: X is d x n, sample-contiguous, leading dimension ld = d
// rounded up to 16 (padding rows 0), FP32 or FP64.  Every kernel returns at
// once when the problem's stop flag is set.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "dwd_device.h"
#include "dwd_internal.h"

namespace dwd {

// ---------------------------------------------------------------------------
// Feature Gram X X^T (d x d) in FP64 on FP64 MFMA 16x16x4: upper 64x64 tiles
// over features, the sum over samples split into `splits` partial tiles.
// ---------------------------------------------------------------------------
typedef double d4v_t __attribute__((ext_vector_type(4)));
constexpr int FT = 64;  // tile edge (features)
constexpr int FK = 32;  // samples per LDS stage

template <typename T>
__device__ __forceinline__ void fgram_stage(const T* __restrict__ X, int64_t ld, int n, int f0,
                                            int s0, int s1, double (*S)[FT + 1]) {
  constexpr int V = 16 / sizeof(T);  // elements per 16-byte load
  constexpr int PER = FT / V;        // loads per sample row of the tile
  for (int e = threadIdx.x; e < FK * PER; e += 256) {
    const int k = e / PER, c = (e % PER) * V;
    const int s = s0 + k;
    const int64_t f = (int64_t)f0 + c;
    if (s < s1 && f < ld) {
      if constexpr (sizeof(T) == 8) {
        const double2 v = *reinterpret_cast<const double2*>(X + (int64_t)s * ld + f);
        S[k][c] = v.x;
        S[k][c + 1] = v.y;
      } else {
        const float4 v = *reinterpret_cast<const float4*>(X + (int64_t)s * ld + f);
        S[k][c] = v.x;
        S[k][c + 1] = v.y;
        S[k][c + 2] = v.z;
        S[k][c + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < V; ++q) S[k][c + q] = 0.0;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fgram_mfma(const T* __restrict__ X, int64_t ld, int n,
                                                    int d, int ntile, int splits,
                                                    double* __restrict__ Kpart) {
  int t = blockIdx.x;
  int ti = 0;
  while (t >= ntile - ti) { t -= ntile - ti; ++ti; }
  const int tj = ti + t;
  const int per = ((n + FK - 1) / FK + splits - 1) / splits * FK;
  const int s_lo = blockIdx.y * per;
  const int s_hi = min(n, s_lo + per);
  __shared__ double As[FK][FT + 1];
  __shared__ double Bs[FK][FT + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int wr = (wid >> 1) * 32, wc = (wid & 1) * 32;
  const int f0 = ti * FT, g0 = tj * FT;
  d4v_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (d4v_t){0.0, 0.0, 0.0, 0.0};
  for (int s0 = s_lo; s0 < s_hi; s0 += FK) {
    fgram_stage<T>(X, ld, n, f0, s0, s_hi, As);
    fgram_stage<T>(X, ld, n, g0, s0, s_hi, Bs);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < FK; ks += 4) {
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
  double* out = Kpart + (size_t)blockIdx.y * d * d;
  const int lj = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = f0 + wr + a * 16 + v * 4 + lg;
        const int gj = g0 + wc + b * 16 + lj;
        if (gi < d && gj < d) out[(size_t)gi * d + gj] = acc[a][b][v];
      }
}

int fgram_splits(int d, int n) {
  const int nt = (d + FT - 1) / FT;
  const int tiles = nt * (nt + 1) / 2;
  int s = (2048 + tiles - 1) / tiles;
  const int kmax = (n + FK - 1) / FK;
  s = std::min(s, kmax);
  s = std::min(s, 256);
  return std::max(s, 1);
}

hipError_t launch_fgram(const void* X, int storage, int64_t ld, int n, int d, double* Kpart,
                        int splits, hipStream_t st) {
  const int nt = (d + FT - 1) / FT;
  dim3 grid(nt * (nt + 1) / 2, splits);
  if (storage == DWD_FP64)
    hipLaunchKernelGGL(k_fgram_mfma<double>, grid, dim3(256), 0, st, (const double*)X, ld, n, d,
                       nt, splits, Kpart);
  else
    hipLaunchKernelGGL(k_fgram_mfma<float>, grid, dim3(256), 0, st, (const float*)X, ld, n, d,
                       nt, splits, Kpart);
  return hipGetLastError();
}

// A ((d+1) x (d+1), row-major): the split partials summed in order, scaled
// by 1/Z_scale^2 (y_i^2 = 1), mu on the diagonal, Z~ y in the last row and
// column, y^T y = n in the corner.
__global__ void __launch_bounds__(256) k_fgram_finish(const double* __restrict__ Kpart,
                                                      int splits, int d, int n,
                                                      const double* __restrict__ zy,
                                                      double inv_zs2, double mu,
                                                      double* __restrict__ A) {
  const int64_t m = (int64_t)(d + 1) * (d + 1);
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < m;
       t += (int64_t)gridDim.x * 256) {
    const int a = (int)(t / (d + 1)), b = (int)(t % (d + 1));
    double v;
    if (a < d && b < d) {
      const int lo = min(a, b), hi = max(a, b);
      double s = 0.0;
      for (int k = 0; k < splits; ++k) s += Kpart[(size_t)k * d * d + (size_t)lo * d + hi];
      v = s * inv_zs2 + (a == b ? mu : 0.0);
    } else if (a < d) {
      v = zy[a];
    } else if (b < d) {
      v = zy[b];
    } else {
      v = (double)n;
    }
    A[t] = v;
  }
}

hipError_t launch_fgram_finish(const double* Kpart, int splits, int d, int n, const double* zy,
                               double inv_zs2, double mu, double* A, hipStream_t st) {
  const int64_t m = (int64_t)(d + 1) * (d + 1);
  const int blocks = (int)std::min<int64_t>(4096, (m + 255) / 256);
  hipLaunchKernelGGL(k_fgram_finish, dim3(blocks), dim3(256), 0, st, Kpart, splits, d, n, zy,
                     inv_zs2, mu, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Initial point (r, xi, w, beta, u) = (1, 1, 0, 0, 0), (alpha, rho) = (0, 0);
// the first right-hand side is then 0.
// ---------------------------------------------------------------------------
__global__ void k_dir_init(Consts c, DirPtrs p, double sigma0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < c.n) {
    p.r[i] = 1.0;
    p.xi[i] = 1.0;
    p.alpha[i] = 0.0;
  }
  if (i <= c.ld) {
    p.h[i] = 0.0;
    p.wbar[i] = 0.0;
  }
  if (i < c.ld) {
    p.w[i] = 0.0;
    p.u[i] = 0.0;
    p.rho[i] = 0.0;
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
  }
}

hipError_t launch_dir_init(const Consts& c, const DirPtrs& p, double sigma0, hipStream_t st) {
  const int64_t m = std::max<int64_t>(c.n, c.ld + 1);
  hipLaunchKernelGGL(k_dir_init, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, c, p,
                     sigma0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Solves with A^-1 ((d+1)^2 row-major), one wave per row.
//   mode 0 (Step 1a): wbar = A^-1 h   (h = [h_w; h_beta], written by the tail).
//   mode 1 (Step 1c): the residual ||[Z~ dr; y^T dr]|| (the right-hand side
//     grows by exactly that vector when r moves by dr, and A [wbar; betabar]
//     = h) is summed by every wave in the same order; above 5 eps_k,
//     [w; beta] = [wbar; betabar] + A^-1 [Z~ dr; y^T dr], else [wbar; betabar].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_dir_gemv(Consts c, DirPtrs p, int mode) {
  Scal* sc = p.sc;
  const int done = sc->done;
  const int k = sc->k;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int d = (int)c.d;
  const int m = d + 1;
  if (done) return;
  int redo = 1;
  double ydr = 0.0;
  if (mode == 1) {
    double s2 = 0.0, sy = 0.0;
    for (int b = lane; b < p.nred; b += 64) s2 += p.part_r[b];
    for (int b = lane; b < p.nblk; b += 64) sy += p.part_n[b];  // slot 0
    s2 = wave_sum(s2);
    ydr = wave_sum(sy);
    const double res = sqrt(fmax(s2 + ydr * ydr, 0.0));
    redo = res > 5.0 * eps_k(c, k) ? 1 : 0;
  }
  if (row >= m) return;
  double acc = 0.0;
  if (redo) {
    const double* Ar = p.Ainv + (size_t)row * m;
    const double* rhs = mode == 0 ? p.h : p.zz;  // zz[0..d) = Z~ dr
    for (int j = lane; j < m; j += 64) {
      const double v = (mode == 1 && j == d) ? ydr : rhs[j];
      acc = fma(Ar[j], v, acc);
    }
    acc = wave_sum(acc);
  }
  if (lane != 0) return;
  if (mode == 0) {
    p.wbar[row] = acc;
  } else {
    const double x = p.wbar[row] + acc;
    if (row < d) {
      p.w[row] = x;
    } else {
      sc->beta = x;
      sc->doubled = redo;
      sc->n_double += redo;
    }
  }
}

hipError_t launch_dir_gemv(const Consts& c, const DirPtrs& p, int mode, hipStream_t st) {
  const int m = (int)c.d + 1;
  hipLaunchKernelGGL(k_dir_gemv, dim3((m + 3) / 4), dim3(256), 0, st, c, p, mode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The fused sweeps.
//   MODE 0: sum_i x_i                                (set-up: Z~ y = that / Z_scale)
//   MODE 1: sweep 1 of the iteration (see the file comment)
//   MODE 2: sweep 2
// Partials: part_d[(v*ld + f) * nblk + b] (v = 0, 1; feature-major, so that
// the reduction reads each feature's partials contiguously), part_n[j * nblk + b]
// for slots j < NPD (slot-major, read contiguously by the consumers).
// ---------------------------------------------------------------------------
// (ordinary cached loads: in the regime of this branch X is often small
// enough to stay in the last-level cache between the two sweeps; values are
// kept in their storage type and widened at use)
template <typename T>
struct Quad;
template <>
struct Quad<float> {
  __device__ static void load(const float* p, float (&o)[4]) {
    const nt_f4 v = *reinterpret_cast<const nt_f4*>(p);
    o[0] = v[0];
    o[1] = v[1];
    o[2] = v[2];
    o[3] = v[3];
  }
};
template <>
struct Quad<double> {
  __device__ static void load(const double* p, double (&o)[4]) {
    const nt_d2 a = *reinterpret_cast<const nt_d2*>(p);
    const nt_d2 b = *(reinterpret_cast<const nt_d2*>(p) + 1);
    o[0] = a[0];
    o[1] = a[1];
    o[2] = b[0];
    o[3] = b[1];
  }
};

template <int TPS>
__device__ __forceinline__ double group_sum(double v, double* lds) {
  if constexpr (TPS <= 64) {
#pragma unroll
    for (int off = TPS / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
  } else {
    // the whole block is one group
    return block_sum<256>(v);
  }
}

template <typename T, int TPS, int NF, int MODE>
__global__ void __launch_bounds__(256) k_dir_sweep(const T* __restrict__ X, Consts c, DirPtrs p) {
  constexpr int G = 256 / TPS;
  constexpr int NV = MODE == 2 ? 2 : 1;
  Scal* sc = p.sc;
  const int done = MODE == 0 ? 0 : sc->done;
  const int lg = threadIdx.x % TPS, g = threadIdx.x / TPS;
  const int64_t ld = c.ld;
  const int n = c.n;
  const int i0 = blockIdx.x * p.per_block;
  const int i1 = min(n, i0 + p.per_block);
  // the d-vector this sweep multiplies, in registers
  double wv[NF][4];
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    const int64_t f = 4 * (int64_t)(lg + j * TPS);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = 0.0;
      if (MODE != 0 && f < ld) v = (MODE == 1 ? p.wbar : p.w)[f + q];
      wv[j][q] = v;
    }
  }
  const double sigma = MODE == 0 ? 1.0 : sc->sigma;
  const double beta = MODE == 1 ? p.wbar[c.d] : (MODE == 2 ? sc->beta : 0.0);
  const int redo = MODE == 2 ? sc->doubled : 1;
  const int kk = MODE == 0 ? 0 : sc->k;
  if (done) return;
  const double tolN = eps_k(c, kk) / sqrt((double)n);
  double acc[NV][NF][4];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[v][j][q] = 0.0;
  constexpr int KS = MODE == 2 ? 10 : 2;
  double ssum[KS];
#pragma unroll
  for (int j = 0; j < KS; ++j) ssum[j] = 0.0;
  __shared__ double lds_red[4];
  // the group's next sample (its row of X and its n-vector entries) is
  // loaded while the current one is processed (its dot product, the Step
  // 1b-3 scalar work and the accumulation)
  constexpr int NS = MODE == 1 ? 4 : (MODE == 2 ? 5 : 0);
  auto load_sample = [&](int i, T (&xv)[NF][4], double (&sv)[NS > 0 ? NS : 1]) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int64_t f = 4 * (int64_t)(lg + j * TPS);
      if (i < i1 && f < ld) {
        Quad<T>::load(X + (int64_t)i * ld + f, xv[j]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) xv[j][q] = (T)0;
      }
    }
    if constexpr (NS > 0) {
      const bool in = i < i1;
      sv[0] = in ? p.y[i] : 0.0;
      sv[1] = in ? p.alpha[i] : 0.0;
      if constexpr (MODE == 1) {
        sv[2] = in ? p.r[i] : 0.0;
        sv[3] = in ? p.xi[i] : 0.0;
      } else {
        sv[2] = in ? p.zb[i] : 0.0;
        sv[3] = in ? p.rn[i] : 0.0;
        sv[4] = in ? p.e[i] : 0.0;
      }
    }
  };
  T xnext[NF][4];
  double snext[NS > 0 ? NS : 1];
  load_sample(i0 + g, xnext, snext);
  for (int ib = i0; ib < i1; ib += G) {
    const int i = ib + g;
    const bool live = i < i1;
    T xv[NF][4];
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) xv[j][q] = xnext[j][q];
    double sv[NS > 0 ? NS : 1];
#pragma unroll
    for (int j = 0; j < (NS > 0 ? NS : 1); ++j) sv[j] = snext[j];
    load_sample(i + G, xnext, snext);
    double cf0 = 1.0, cf1 = 0.0;
    if constexpr (MODE != 0) {
      double dot = 0.0;
      if (MODE == 1 || redo) {
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) dot = fma((double)xv[j][q], wv[j][q], dot);
        dot = group_sum<TPS>(dot, lds_red);
      }
      const double yi = sv[0], al = sv[1];
      // A group that spans several waves (TPS = 256): every wave has read
      // alpha_i (a step ago) before the group leader overwrites it in sweep 2.
      if constexpr (MODE == 2 && TPS > 64) __syncthreads();
      if (live) {
        if constexpr (MODE == 1) {
          const double z = yi * dot * c.inv_zs;
          const double r0 = sv[2];
          const double cc = z + yi * beta + sv[3] - al / sigma;
          int steps = 0;
          const double rn = prox_weighted(cc, sigma, r0, tolN, loss_weight(c, yi), c, steps);
          const double dr = rn - r0;
          cf0 = yi * dr;
          if (lg == 0) {
            p.zb[i] = z;
            p.rn[i] = rn;
            p.dr[i] = dr;
            ssum[0] += yi * dr;
            ssum[1] = fmax(ssum[1], (double)steps);
          }
        } else {
          const double z = redo ? yi * dot * c.inv_zs : sv[2];
          const double rn = sv[3];
          const double ei = sv[4];
          const double xin = fmax(0.0, rn - z - yi * beta + (al - c.C * ei) / sigma);
          const double pres = z + yi * beta + xin - rn;
          const double a1 = al - c.tau * sigma * pres;
          cf0 = yi * (xin - rn);
          cf1 = yi * a1;
          if (lg == 0) {
            p.r[i] = rn;
            p.xi[i] = xin;
            p.alpha[i] = a1;
            double s9[9];
            nspace_sums(c, pow_q(rn, c), pow_qp1(rn, c), a1, xin, pres, yi, ei, s9);
#pragma unroll
            for (int j = 0; j < 9; ++j) ssum[j] += s9[j];
            ssum[9] += yi * (xin - rn);
          }
        }
      } else {
        cf0 = 0.0;
        cf1 = 0.0;
      }
    } else {
      if (!live) cf0 = 0.0;
    }
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[0][j][q] = fma(cf0, (double)xv[j][q], acc[0][j][q]);
        if constexpr (NV == 2) acc[1][j][q] = fma(cf1, (double)xv[j][q], acc[1][j][q]);
      }
  }
  // d-vector partials: the groups of the block summed in order
  double* out = p.part_d + blockIdx.x;
  const size_t nb = (size_t)p.nblk;
  if constexpr (G == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        const int64_t f = 4 * (int64_t)(lg + j * TPS);
        if (f < ld) {
#pragma unroll
          for (int q = 0; q < 4; ++q) out[(v * ld + f + q) * nb] = acc[v][j][q];
        }
      }
  } else {
    // the groups of a wave hold the same features at lane offsets that are
    // multiples of TPS: a butterfly over those offsets, then the four waves
    // added in order through LDS
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double a = acc[v][j][q];
#pragma unroll
          for (int off = TPS; off < 64; off <<= 1) a += __shfl_xor(a, off, 64);
          acc[v][j][q] = a;
        }
    __shared__ double buf[NV][TPS * NF * 4];
    const int wid = threadIdx.x >> 6, lw = threadIdx.x & 63;
    for (int ww = 0; ww < 4; ++ww) {
      if (wid == ww && lw < TPS) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int o = 4 * (lg + j * TPS) + q;
              buf[v][o] = ww == 0 ? acc[v][j][q] : buf[v][o] + acc[v][j][q];
            }
      }
      __syncthreads();
    }
    for (int v = 0; v < NV; ++v)
      for (int o = threadIdx.x; o < TPS * NF * 4 && o < ld; o += 256)
        out[(v * ld + o) * nb] = buf[v][o];
  }
  // scalar partials: the group leaders summed in order
  if constexpr (MODE != 0) {
    __shared__ double sbuf[G][KS];
    if (lg == 0) {
#pragma unroll
      for (int j = 0; j < KS; ++j) sbuf[g][j] = ssum[j];
    }
    __syncthreads();
    if (threadIdx.x < KS) {
      const int j = threadIdx.x;
      double s = sbuf[0][j];
      for (int gg = 1; gg < G; ++gg)
        s = (MODE == 1 && j == 1) ? fmax(s, sbuf[gg][j]) : s + sbuf[gg][j];
      (MODE == 1 ? p.part_n : p.part_n2)[(size_t)j * p.nblk + blockIdx.x] = s;
    }
  }
}

// Threads per sample and feature quads per thread for a leading dimension:
// the fewest threads per sample (more samples per wave, so fewer passes of
// the scalar Step 1b-3 work) with at most four quads each, five at 64
// threads; above 320 quads the whole block takes one sample.
static void sweep_shape(int64_t ld, int* tps, int* nf) {
  const int64_t quads = ld / 4;
  for (int t = 4; t <= 64; t *= 2) {
    if (quads <= 4 * t) {
      *tps = t;
      *nf = quads <= 2 * t ? 2 : 4;
      return;
    }
  }
  if (quads <= 320) {
    *tps = 64;
    *nf = 5;
    return;
  }
  *tps = 256;
  *nf = (int)((quads + 255) / 256);
}

// ---------------------------------------------------------------------------
// Sweeps 1 and 2 through LDS, for leading dimensions up to 512.  A block
// takes its samples in chunks of S (64, 32 or 16) consecutive ones.  A
// chunk's rows, contiguous in X, are read with 16-byte loads into registers
// while the chunk before is processed, then written to LDS with an odd row
// stride rs (in 4-byte words, for FP32: lanes reading the same column of
// different rows hit different banks).  Dot products: the features split
// into NP = 256 / S equal ranges; lane l of wave v takes sample l mod S and
// range M v + l / S (M = 64 / S ranges per wave), so that each wave reads
// only M entries of the d-vector (staged in LDS) at a time.  The NP partial sums of a sample are added in range order by
// thread t = sample, which then does the sample's Step 1b-3 scalar work
// (a full lane per sample) and stages its coefficients.  Accumulation:
// lanes over features, each thread over its slice of the chunk's samples
// in order.  Every sum has a fixed order, so the results do not depend on
// timing.  The partials have the layout of k_dir_sweep.
// ---------------------------------------------------------------------------
constexpr int DL_NQ = 10;            // 16-byte row loads per thread and chunk
constexpr int DL_ROWS = 48 * 1024;   // LDS bytes of a chunk's rows (padded) at most
typedef unsigned int dl_u2 __attribute__((ext_vector_type(2)));
typedef double dl_d2 __attribute__((ext_vector_type(2)));

// 16 bytes to LDS at an address aligned to AL bytes
template <int AL>
__device__ __forceinline__ void lds_put16(void* dst, const nt_u4& v) {
  if constexpr (AL == 16) {
    *reinterpret_cast<nt_u4*>(dst) = v;
  } else if constexpr (AL == 8) {
    dl_u2* d = reinterpret_cast<dl_u2*>(dst);
    d[0] = dl_u2{v.x, v.y};
    d[1] = dl_u2{v.z, v.w};
  } else {
    unsigned* d = reinterpret_cast<unsigned*>(dst);
    d[0] = v.x;
    d[1] = v.y;
    d[2] = v.z;
    d[3] = v.w;
  }
}

template <typename T, int S, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_dir_sweepl(const T* __restrict__ X,
                                                    const double* __restrict__ wg, Consts c,
                                                    DirPtrs p, int rs, int rb) {
  static_assert(MODE == 1 || MODE == 2, "sweeps 1 and 2");
  static_assert(S == 16 || S == 32 || S == 64, "a whole number of samples per wave");
  constexpr int M = 64 / S, NP = 4 * M;
  constexpr int NV = MODE == 2 ? 2 : 1;
  constexpr int KS = MODE == 2 ? 10 : 2;
  constexpr int NS = MODE == 1 ? 4 : 5;
  constexpr int EQ = 16 / (int)sizeof(T);  // elements per 16-byte load
  extern __shared__ __align__(16) unsigned char dl_lds[];
  T* rows = reinterpret_cast<T*>(dl_lds);                    // [S][rs]
  double* dpart = reinterpret_cast<double*>(dl_lds + rb);    // [NP][S]
  double* cfs = dpart + NP * S;                              // [NV][S]
  double* wl = cfs + 2 * 64;                                 // [ld] the d-vector
  const int ldi = (int)c.ld;
  for (int f = threadIdx.x; f < ldi; f += 256) wl[f] = wg[f];
  Scal* sc = p.sc;
  const int done = sc->done;
  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int i0 = blockIdx.x * p.per_block;
  const int i1 = min(c.n, i0 + p.per_block);
  const double sigma = sc->sigma;
  const double beta = MODE == 1 ? p.wbar[c.d] : sc->beta;
  const int redo = MODE == 2 ? sc->doubled : 1;
  const int kk = sc->k;
  if (done) return;
  const double tolN = eps_k(c, kk) / sqrt((double)c.n);
  // dot products: sample s_me, feature range pm of the wave's M
  const int s_me = lane % S, pm = lane / S;
  const int lf = ldi / NP;                 // features per range (ld is a multiple of 16)
  const int fb = wv * M * lf;              // the wave's first feature (uniform)
  // accumulation: feature fa (and fa + 256), sample slice r
  int ldp = 16;
  while (ldp < ldi) ldp <<= 1;
  const int fw = min(ldp, 256), nsl = 256 / fw;
  const int fa = t % fw, r = t / fw;
  const int s_lo = r * (S / nsl), s_hi = s_lo + S / nsl;
  double acc[NV][2];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v][0] = acc[v][1] = 0.0;
  double ssum[KS];
#pragma unroll
  for (int j = 0; j < KS; ++j) ssum[j] = 0.0;
  nt_u4 pre[DL_NQ];
  double psv[NS];
  auto load_chunk = [&](int cb) {
    const int cnt = min(S, i1 - cb) * (ldi / EQ);
    const nt_u4* src = reinterpret_cast<const nt_u4*>(X + (int64_t)cb * ldi);
#pragma unroll
    for (int q = 0; q < DL_NQ; ++q) {
      const int u = t + 256 * q;
      pre[q] = u < cnt ? src[u] : nt_u4{0u, 0u, 0u, 0u};
    }
    // thread t < S: sample t's n-vector entries
    const int i = cb + t;
    const bool in = t < S && i < i1;
    psv[0] = in ? p.y[i] : 0.0;
    psv[1] = in ? p.alpha[i] : 0.0;
    if constexpr (MODE == 1) {
      psv[2] = in ? p.r[i] : 0.0;
      psv[3] = in ? p.xi[i] : 0.0;
    } else {
      psv[2] = in ? p.zb[i] : 0.0;
      psv[3] = in ? p.rn[i] : 0.0;
      psv[4] = in ? p.e[i] : 0.0;
    }
  };
  if (i0 < i1) load_chunk(i0);
  for (int cb = i0; cb < i1; cb += S) {
    const int ns = min(S, i1 - cb);
    {
      const int cnt = ns * (ldi / EQ);
#pragma unroll
      for (int q = 0; q < DL_NQ; ++q) {
        const int u = t + 256 * q;
        if (u < cnt) {
          const int e = u * EQ, s = e / ldi, col = e - s * ldi;
          lds_put16<(int)sizeof(T)>(rows + s * rs + col, pre[q]);
        }
      }
    }
    double sv[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) sv[j] = psv[j];
    if (cb + S < i1) load_chunk(cb + S);  // the next chunk in flight meanwhile
    __syncthreads();
    if (MODE == 1 || redo) {
      const T* rw = rows + s_me * rs + fb + pm * lf;  // range wv M + pm
      double dd[4] = {0.0, 0.0, 0.0, 0.0};
      int k = 0;

      const double* ww = wl + fb + pm * lf;  // (M addresses per wave: broadcast reads)
      for (; k + 4 <= lf; k += 4) {
        T xr[4];
        double wr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xr[u] = rw[k + u];
          wr[u] = ww[k + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) dd[u] = fma((double)xr[u], wr[u], dd[u]);
      }
      for (; k < lf; ++k) dd[k & 3] = fma((double)rw[k], ww[k], dd[k & 3]);
      dpart[(wv * M + pm) * S + s_me] = (dd[0] + dd[1]) + (dd[2] + dd[3]);
    }
    __syncthreads();
    if (t < S) {
      const int i = cb + t;
      double cf0 = 0.0, cf1 = 0.0;
      if (i < i1) {
        double dot = 0.0;
        if (MODE == 1 || redo) {
#pragma unroll
          for (int q = 0; q < NP; ++q) dot += dpart[q * S + t];
        }
        const double yi = sv[0], al = sv[1];
        if constexpr (MODE == 1) {
          const double z = yi * dot * c.inv_zs;
          const double r0 = sv[2];
          const double cc = z + yi * beta + sv[3] - al / sigma;
          int steps = 0;
          const double rn = prox_weighted(cc, sigma, r0, tolN, loss_weight(c, yi), c, steps);
          const double dr = rn - r0;
          cf0 = yi * dr;
          p.zb[i] = z;
          p.rn[i] = rn;
          p.dr[i] = dr;
          ssum[0] += yi * dr;
          ssum[1] = fmax(ssum[1], (double)steps);
        } else {
          const double z = redo ? yi * dot * c.inv_zs : sv[2];
          const double rn = sv[3];
          const double ei = sv[4];
          const double xin = fmax(0.0, rn - z - yi * beta + (al - c.C * ei) / sigma);
          const double pres = z + yi * beta + xin - rn;
          const double a1 = al - c.tau * sigma * pres;
          cf0 = yi * (xin - rn);
          cf1 = yi * a1;
          p.r[i] = rn;
          p.xi[i] = xin;
          p.alpha[i] = a1;
          double s9[9];
          nspace_sums(c, pow_q(rn, c), pow_qp1(rn, c), a1, xin, pres, yi, ei, s9);
#pragma unroll
          for (int j = 0; j < 9; ++j) ssum[j] += s9[j];
          ssum[9] += yi * (xin - rn);
        }
      }
      cfs[t] = cf0;
      if constexpr (NV == 2) cfs[S + t] = cf1;
    }
    __syncthreads();
    // (samples in order; eight rows and coefficients read before they are added)
    const int se = min(s_hi, ns);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int f = fa + 256 * m;
      if (f < ldi) {
        int s = s_lo;
        for (; s + 8 <= se; s += 8) {
          T xr[8];
          double c0[8], c1[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) xr[u] = rows[(s + u) * rs + f];
#pragma unroll
          for (int u = 0; u < 8; u += 2) {
            const dl_d2 a0 = *reinterpret_cast<const dl_d2*>(cfs + s + u);
            c0[u] = a0.x;
            c0[u + 1] = a0.y;
            if constexpr (NV == 2) {
              const dl_d2 a1 = *reinterpret_cast<const dl_d2*>(cfs + S + s + u);
              c1[u] = a1.x;
              c1[u + 1] = a1.y;
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            acc[0][m] = fma(c0[u], (double)xr[u], acc[0][m]);
            if constexpr (NV == 2) acc[1][m] = fma(c1[u], (double)xr[u], acc[1][m]);
          }
        }
        for (; s < se; ++s) {
          const double x = (double)rows[s * rs + f];
          acc[0][m] = fma(cfs[s], x, acc[0][m]);
          if constexpr (NV == 2) acc[1][m] = fma(cfs[S + s], x, acc[1][m]);
        }
      }
    }
    __syncthreads();  // the rows and coefficients are rewritten next
  }
  // d-vector partials: the slices of each feature added in slice order
  double* red = reinterpret_cast<double*>(dl_lds);
  if (nsl > 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) red[(r * NV + v) * fw + fa] = acc[v][0];
    __syncthreads();
    if (r == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double s = red[v * fw + fa];
        for (int rr = 1; rr < nsl; ++rr) s += red[(rr * NV + v) * fw + fa];
        acc[v][0] = s;
      }
    }
  }
  if (r == 0) {
    double* out = p.part_d + blockIdx.x;
    const size_t nb = (size_t)p.nblk;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int f = fa + 256 * m;
        if (f < ldi) out[((size_t)v * ldi + f) * nb] = acc[v][m];
      }
  }
  // scalar partials (Newton steps by maximum)
  double* part = (MODE == 1 ? p.part_n : p.part_n2) + blockIdx.x;  // slot j at j nblk
  if constexpr (MODE == 1) {
    double mx = ssum[1];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    __shared__ double wmax[4];
    if ((t & 63) == 0) wmax[t >> 6] = mx;
    double a[1] = {ssum[0]};
    block_sum_k<256, 1>(a);  // (its barriers also order the wmax writes)
    if (t == 0) {
      part[0] = a[0];
      part[p.nblk] = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    }
  } else {
    block_sum_k<256, KS>(ssum);
    if (t < KS) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < KS; ++j)
        if (t == j) v = ssum[j];
      part[(size_t)t * p.nblk] = v;
    }
  }
}

// Samples per chunk, LDS row stride and rows-area bytes of the LDS sweeps:
// the largest chunk whose padded rows fit in DL_ROWS and whose data fits
// the loads in registers; false above 512 features or when none fits.
static bool sweepl_shape(int64_t ld, int elem, int* sn, int* rs, int* rb) {
  if (ld > 512 || ld % 16 != 0) return false;
  const int r = (int)ld + 1;  // odd
  for (int s = 64; s >= 16; s /= 2) {
    const size_t bytes = (size_t)s * r * elem;
    const size_t loaded = (size_t)s * ld * elem;
    if (bytes <= (size_t)DL_ROWS && loaded <= (size_t)DL_NQ * 256 * 16) {
      *sn = s;
      *rs = r;
      // the rows area also takes the slice sums at the end
      *rb = (int)((std::max(bytes, (size_t)(2 * 256 * 8)) + 15) / 16 * 16);
      return true;
    }
  }
  return false;
}

int dir_sweep_samples_per_block(int64_t ld, int n, int storage) {
  int S, rs, rb;
  if (sweepl_shape(ld, storage == DWD_FP64 ? 8 : 4, &S, &rs, &rb)) {
    // whole chunks, one round of blocks (three per compute unit)
    int per = std::max(S, (n + 767) / 768);
    return (per + S - 1) / S * S;
  }
  int tps, nf;
  sweep_shape(ld, &tps, &nf);
  const int G = 256 / tps;
  // about 8 samples per group, at most 1024 blocks
  int per = std::max(G * 8, (n + 1023) / 1024);
  per = (per + G - 1) / G * G;
  return per;
}

template <typename T, int MODE>
static hipError_t sweep_t(const T* X, const Consts& c, const DirPtrs& p, hipStream_t st) {
  int tps, nf;
  const dim3 grid((unsigned)p.nblk), blk(256);
  int sn, rs, rb;
  if (MODE != 0 && sweepl_shape(c.ld, (int)sizeof(T), &sn, &rs, &rb)) {
    // (the samples per block are whole chunks of this shape)
    if (p.per_block % sn != 0) return hipErrorInvalidValue;
    constexpr int M = MODE == 0 ? 1 : MODE;
    const double* wg = M == 1 ? p.wbar : p.w;
    const size_t shm = (size_t)rb + 8 * (size_t)(256 + 2 * 64) + 8 * (size_t)c.ld;
    if (sn == 64)
      hipLaunchKernelGGL((k_dir_sweepl<T, 64, M>), grid, blk, shm, st, X, wg, c, p, rs, rb);
    else if (sn == 32)
      hipLaunchKernelGGL((k_dir_sweepl<T, 32, M>), grid, blk, shm, st, X, wg, c, p, rs, rb);
    else
      hipLaunchKernelGGL((k_dir_sweepl<T, 16, M>), grid, blk, shm, st, X, wg, c, p, rs, rb);
    return hipGetLastError();
  }
  sweep_shape(c.ld, &tps, &nf);
#define DWD_SWEEP(TP, NFV)                                                                 \
  if (tps == TP && nf == NFV) {                                                            \
    hipLaunchKernelGGL((k_dir_sweep<T, TP, NFV, MODE>), grid, blk, 0, st, X, c, p);        \
    return hipGetLastError();                                                              \
  }
  DWD_SWEEP(4, 2) DWD_SWEEP(4, 4) DWD_SWEEP(8, 2) DWD_SWEEP(8, 4)
  DWD_SWEEP(16, 2) DWD_SWEEP(16, 4) DWD_SWEEP(32, 2) DWD_SWEEP(32, 4)
  DWD_SWEEP(64, 2) DWD_SWEEP(64, 4) DWD_SWEEP(64, 5)
  DWD_SWEEP(256, 2) DWD_SWEEP(256, 3) DWD_SWEEP(256, 4) DWD_SWEEP(256, 5)
#undef DWD_SWEEP
  return hipErrorInvalidValue;
}

hipError_t launch_dir_sweep(const void* X, int storage, const Consts& c, const DirPtrs& p,
                            int mode, hipStream_t st) {
  if (storage == DWD_FP64) {
    const double* Xd = (const double*)X;
    if (mode == 0) return sweep_t<double, 0>(Xd, c, p, st);
    if (mode == 1) return sweep_t<double, 1>(Xd, c, p, st);
    return sweep_t<double, 2>(Xd, c, p, st);
  }
  const float* Xf = (const float*)X;
  if (mode == 0) return sweep_t<float, 0>(Xf, c, p, st);
  if (mode == 1) return sweep_t<float, 1>(Xf, c, p, st);
  return sweep_t<float, 2>(Xf, c, p, st);
}

// ---------------------------------------------------------------------------
// Sum the sweep partials over blocks into zz[v0 + v] (v < nvec), times
// `scale`: one wave per feature, lanes striding over the blocks, then a
// butterfly (a fixed order).  With nvec = 1 also the block partials of the
// squared norm (the Step 1c residual).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_dir_reduce(Consts c, DirPtrs p, int v0, int nvec,
                                                    double scale) {
  const int done = p.sc->done;
  const int64_t ld = c.ld;
  const int d = (int)c.d;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int t = blockIdx.x * 4 + wid;
  const int v = t / d, f = t % d;
  if (done) return;
  double s = 0.0;
  if (v < nvec) {
    const double* src = p.part_d + ((size_t)v * ld + f) * p.nblk;
    for (int b = lane; b < p.nblk; b += 64) s += src[b];
    s = wave_sum(s) * scale;
    if (lane == 0) p.zz[(size_t)(v0 + v) * ld + f] = s;
  }
  if (nvec == 1) {
    __shared__ double sq[4];
    if (lane == 0) sq[wid] = v < nvec ? s * s : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) p.part_r[blockIdx.x] = (sq[0] + sq[1]) + (sq[2] + sq[3]);
  }
}

int dir_reduce_blocks(int d, int nvec) { return (nvec * d + 3) / 4; }

hipError_t launch_dir_reduce(const Consts& c, const DirPtrs& p, int v0, int nvec, double scale,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_dir_reduce, dim3(dir_reduce_blocks((int)c.d, nvec)), dim3(256), 0, st, c,
                     p, v0, nvec, scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// End of the iteration (one block): Step 2 u, Step 3 rho, the d-space terms
// of Section 4.3, the residuals, the stopping and sigma rules, and the next
// right-hand side h = -Z~ t + mu u + sqrt(mu) rho / sigma, h_beta = -y^T t
// with t = xi - r - alpha / sigma (sigma the updated one).
// ---------------------------------------------------------------------------
constexpr int NTD = 1024;
constexpr int MAXF = 8;  // d <= NTD * MAXF

__global__ void __launch_bounds__(NTD) k_dir_tail(Consts c, DirPtrs p) {
  Scal* sc = p.sc;
  if (sc->done) return;
  const int d = (int)c.d;
  const int64_t ld = c.ld;
  const int k0 = sc->k;
  const double sigma = sc->sigma;
  const int nm = sc->newton_max;
  __shared__ double s_sig;
  // n-space sums of sweep 2, the Newton-step maximum of sweep 1
  constexpr int K = 10;
  double ns[K];
#pragma unroll
  for (int j = 0; j < K; ++j) ns[j] = 0.0;
  double nmax = 0.0;
  for (int b = threadIdx.x; b < p.nblk; b += NTD) {
#pragma unroll
    for (int j = 0; j < K; ++j) ns[j] += p.part_n2[(size_t)j * p.nblk + b];
    nmax = fmax(nmax, p.part_n[(size_t)p.nblk + b]);
  }
  block_sum_k<NTD, K>(ns);
  {
    __shared__ double smax[NTD / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nmax = fmax(nmax, __shfl_xor(nmax, off, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = nmax;
    __syncthreads();
    double m = smax[0];
    for (int w = 1; w < NTD / 64; ++w) m = fmax(m, smax[w]);
    nmax = m;
  }
  // Step 2: g = w - rho / (sigma sqrt(mu)), u = g min(1, R / ||g||)
  double wv[MAXF], rv[MAXF], gv[MAXF];
  double g2 = 0.0;
#pragma unroll
  for (int j = 0; j < MAXF; ++j) {
    const int f = threadIdx.x + j * NTD;
    wv[j] = f < d ? p.w[f] : 0.0;
    rv[j] = f < d ? p.rho[f] : 0.0;
    gv[j] = wv[j] - rv[j] / (sigma * c.sqmu);
    g2 = fma(gv[j], gv[j], g2);
  }
  g2 = block_sum<NTD>(g2);
  const double ng = sqrt(g2);
  const double gamma = ng <= c.R ? 1.0 : c.R / ng;
  // Step 3: rho' = rho - tau sigma sqrt(mu) (w - u); d-space sums
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // ||w-u||^2, ||w||^2, ||Z~a + D rho'||^2, ||Z~a||^2
  const double* za = p.zz + 2 * ld;
#pragma unroll
  for (int j = 0; j < MAXF; ++j) {
    const int f = threadIdx.x + j * NTD;
    const double u = gamma * gv[j];
    const double rn = rv[j] - c.tau * sigma * c.sqmu * (wv[j] - u);
    gv[j] = u;
    rv[j] = rn;
    if (f < d) {
      const double zf = za[f];
      const double dres = zf + c.sqmu * rn;
      acc[0] = fma(wv[j] - u, wv[j] - u, acc[0]);
      acc[1] = fma(wv[j], wv[j], acc[1]);
      acc[2] = fma(dres, dres, acc[2]);
      acc[3] = fma(zf, zf, acc[3]);
    }
  }
  block_sum_k<NTD, 4>(acc);
  if (threadIdx.x == 0) {
    double red[R_COUNT];
    for (int j = 0; j < 9; ++j) red[R_PRES2 + j] = ns[j];
    red[R_WU2] = acc[0];
    red[R_W2] = acc[1];
    red[R_DRES2] = acc[2];
    red[R_ZA2] = acc[3];
    red[R_G2] = g2;
    red[R_RHO2] = 0.0;
    double e[E_COUNT];
    finish_etas(c, red, e);
    // every residual here comes from explicit passes of this iteration
    e[E_PCHK] = e[E_P];
    e[E_DCHK] = e[E_D];
    for (int j = 0; j < R_COUNT; ++j) sc->red[j] = red[j];
    for (int j = 0; j < E_COUNT; ++j) sc->eta[j] = e[j];
    sc->gamma = gamma;
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
    s_sig = sig;
  }
  __syncthreads();
  const double sig1 = s_sig;
  const double* zxr = p.zz + ld;
#pragma unroll
  for (int j = 0; j < MAXF; ++j) {
    const int f = threadIdx.x + j * NTD;
    if (f < d) {
      p.u[f] = gv[j];
      p.rho[f] = rv[j];
      p.h[f] = -(zxr[f] - za[f] / sig1) + c.mu * gv[j] + c.sqmu * rv[j] / sig1;
    }
  }
  if (threadIdx.x == 0) {
    // h_beta = -y^T t = -(y^T (xi - r) - y^T alpha / sigma')
    p.h[d] = -(ns[9] - ns[3] / sig1);
  }
}

hipError_t launch_dir_tail(const Consts& c, const DirPtrs& p, hipStream_t st) {
  hipLaunchKernelGGL(k_dir_tail, dim3(1), dim3(NTD), 0, st, c, p);
  return hipGetLastError();
}

}  // namespace dwd
