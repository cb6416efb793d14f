// Kernels that step B problems over one shared X together (many (C, q)
// values of one data set).  The eq-linsys matrix A depends only on X, y and
// mu (Section 3.3.2), so G~, M^-1 and M^-1 y are shared; each problem keeps
// its own (C, q, sigma, ...) and iterates exactly as a single solve would.
// The pass over Z becomes one matrix product Z~ [s_1 .. s_B] on MFMA with
// the Step 2-3 epilogue, and the n x n products M^-1 [x_1 .. x_B],
// [G~; M^-1] [dr_1 .. dr_B] and G~ [alpha_1 .. alpha_B] become FP64 MFMA
// products in 16 x 16 tiles with the Step 1a-1c element work fused into
// their epilogues; blocks that read the same rows of M^-1 / G~ are placed on
// one XCD so that they share its L2.
#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include "dwd_device.h"
#include "dwd_internal.h"

namespace dwd {

// ---------------------------------------------------------------------------
// Initial point of every problem (as k_init) and t = x = 0 for the first
// Step 1a (with u = rho = 0, Z~^T b = 0 and t = xi - r - alpha/sigma = 0).
// ---------------------------------------------------------------------------
__global__ void k_init_b(BatchPtrs P, int B) {
  const int p = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t on = (size_t)p * P.n;
  if (i < P.n) {
    P.R[on + i] = 1.0;
    P.XI[on + i] = 1.0;
    P.AL[on + i] = 0.0;
    P.PU[on + i] = 0.0;
    P.PR[on + i] = 0.0;
    P.T[on + i] = 0.0;
    P.XX[on + i] = 0.0;
    if (P.rep) {
      P.AU[on + i] = 0.0;
      P.ARHO[on + i] = 0.0;
      P.AW[on + i] = 0.0;
    }
  }
  if (i < P.ld) {
    const size_t od = (size_t)p * P.ld;
    P.U[od + i] = 0.0;
    P.RHO[od + i] = 0.0;
    P.W[od + i] = 0.0;
  }
  if (i == 0) {
    Scal* s = P.sc + p;
    s->sigma = P.cs[p].sigma0;
    s->beta = s->beta_bar = s->beta1 = 0.0;
    s->gamma = 1.0;
    s->ytdr = 0.0;
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
  (void)B;
}

hipError_t launch_init_b(const BatchPtrs& P, int B, hipStream_t st) {
  const int64_t m = P.ld > P.n ? P.ld : P.n;
  hipLaunchKernelGGL(k_init_b, dim3((unsigned)((m + 255) / 256), B), dim3(256), 0, st, P, B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// n x n by n x B products on FP64 MFMA.  A block computes one 16 x 16 tile
// (16 rows of the n x n matrices, 16 active slots); its 8 waves split the
// inner dimension and their partial tiles are summed in a fixed order.
// Lane l = i + 16 q supplies A[row i][k] and B[k][slot i] for the k = q mod 4
// of each group of four, from four consecutive k that it loads itself (step t
// of a group multiplies the k = 4q + t terms).  A dot product of every slot's
// column with one fixed n-vector (m_y) rides along on the same loads.
// ---------------------------------------------------------------------------
constexpr int NM_W = 8, NM_T = NM_W * 64;

typedef double nm_acc_t __attribute__((ext_vector_type(4)));

// Block id -> (row tile, slot tile): the blocks of one row tile share an XCD.
__device__ __forceinline__ bool nm_tile(int nbx, int nby, int& bx, int& by) {
  const int b = blockIdx.x, xcd = b & 7, m = b >> 3;
  bx = xcd + 8 * (m / nby);
  by = m % nby;
  return bx < nbx;
}

int nm_grid(int n, int bact) {
  const int nbx = (n + 15) / 16, nby = (bact + 15) / 16;
  return 8 * ((nbx + 7) / 8) * nby;
}

template <int NA, bool DOT>
struct NmRegs {
  double a[NA][4], b[4], m[DOT ? 4 : 1];
};

template <int NA, bool DOT>
__device__ __forceinline__ void nm_load(const double* const (&A)[NA], const double* col,
                                        const double* dv, int n, int row, int k0, int kend,
                                        NmRegs<NA, DOT>& R) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = k0 + t;
    const bool ok = k < kend;
#pragma unroll
    for (int a = 0; a < NA; ++a) R.a[a][t] = (ok && row < n) ? A[a][(size_t)row * n + k] : 0.0;
    R.b[t] = (ok && col) ? col[k] : 0.0;
    if constexpr (DOT) R.m[t] = ok ? dv[k] : 0.0;
  }
}

// Products of this block's tile, left in red[a][i * 16 + j] (row i, slot j)
// of every output a, and the slot dot products in dot[j]; ends with a block
// barrier.  col: the B column of the lane's slot (null: zeros).
template <int NA, bool DOT>
__device__ __forceinline__ void nm_products(const double* const (&A)[NA], const double* col,
                                            const double* dv, int n, int r0,
                                            double (*red)[NM_W][256], double (*dsum)[16],
                                            double* out_red, double* dot) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int kper = (((n + NM_W - 1) / NM_W) + 15) & ~15;
  const int kw0 = wid * kper, kw1 = min(n, kw0 + kper);
  nm_acc_t acc[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) acc[a] = nm_acc_t{0.0, 0.0, 0.0, 0.0};
  double dacc = 0.0;
  const int row = r0 + i;
  NmRegs<NA, DOT> cur, nxt;
  if (kw0 < kw1) nm_load<NA, DOT>(A, col, dv, n, row, kw0 + 4 * q, kw1, cur);
  for (int kb = kw0; kb < kw1; kb += 16) {
    if (kb + 16 < kw1) nm_load<NA, DOT>(A, col, dv, n, row, kb + 16 + 4 * q, kw1, nxt);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int a = 0; a < NA; ++a)
        acc[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur.a[a][t], cur.b[t], acc[a], 0, 0, 0);
      if constexpr (DOT) dacc = fma(cur.m[t], cur.b[t], dacc);
    }
    cur = nxt;
  }
  // D[i'][j'] of a 16 x 16 f64 MFMA sits in register i'/4 of lane j' + 16 (i' % 4)
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[a][wid][(4 * v + q) * 16 + i] = acc[a][v];
  if constexpr (DOT) {
    dacc += __shfl_xor(dacc, 16, 64);
    dacc += __shfl_xor(dacc, 32, 64);
    if (q == 0) dsum[wid][i] = dacc;
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    const int e = threadIdx.x;
    const int ti = e & 15, tj = e >> 4;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < NM_W; ++w) v += red[a][w][ti * 16 + tj];
      out_red[a] = v;
    }
    if constexpr (DOT) {
      double d = 0.0;
#pragma unroll
      for (int w = 0; w < NM_W; ++w) d += dsum[w][tj];
      *dot = d;
    }
  }
}

// Sum (or max) over the 16 consecutive lanes that hold one slot's 16 rows.
__device__ __forceinline__ double sum16(double v) {
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double max16(double v) {
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// The lane's B column (slot c0 + lane % 16), or null if the slot is empty or
// its problem has stopped.
__device__ __forceinline__ const double* nm_col(const BatchPtrs& P, const int* idx, int bact,
                                                int c0, const double* base, int which) {
  const int slot = c0 + (threadIdx.x & 15);
  if (slot >= bact) return nullptr;
  const int pr = idx[slot];
  const Scal* sc = P.sc + pr;
  if (sc->done) return nullptr;
  if (which == 1) base = sc->redo ? P.AL1 : P.AL0;  // alpha of the chosen outcome
  return base + (size_t)pr * P.n;
}

// ---------------------------------------------------------------------------
// Steps 1a + 1b for every (row, problem) of the tile: f = M^-1 x, then
// beta_bar = -m_y^T x / (y^T m_y), s, v and the prox (see k_step1ab).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NM_T) k_s1ab_mm(BatchPtrs P, const int* __restrict__ idx,
                                                  int bact) {
  int bx, by;
  if (!nm_tile((P.n + 15) / 16, (bact + 15) / 16, bx, by)) return;
  __shared__ double red[1][NM_W][256];
  __shared__ double dsum[NM_W][16];
  const int r0 = bx * 16, c0 = by * 16;
  const double* A[1] = {P.Minv};
  double f, mx;
  nm_products<1, true>(A, nm_col(P, idx, bact, c0, P.XX, 0), P.my, P.n, r0, red, dsum, &f, &mx);
  if (threadIdx.x >= 256) return;
  const int e = threadIdx.x, row = r0 + (e & 15), slot = c0 + (e >> 4);
  double ydr = 0.0, steps_d = 0.0;
  int pr = -1;
  bool live = false;
  if (slot < bact) {
    pr = idx[slot];
    live = !P.sc[pr].done;
  }
  double beta_bar = 0.0;
  if (live) {
    Scal* sc = P.sc + pr;
    const Consts c = P.cs[pr];
    beta_bar = -mx / c.ymy;
    if (row < c.n) {
      const size_t on = (size_t)pr * P.n;
      const double sigma = sc->sigma;
      const double tolN = eps_k(c, sc->k) / sqrt((double)c.n);
      const double s = f + beta_bar * P.my[row];
      const double v = s - P.T[on + row];
      const double cc = v + P.XI[on + row] - P.AL[on + row] / sigma;
      const double r0v = P.R[on + row];
      int steps = 0;
      const double rn = prox_weighted(cc, sigma, r0v, tolN, loss_weight(c, P.y[row]), c, steps);
      const double dr = rn - r0v;
      P.F[on + row] = f;
      P.S[on + row] = s;
      P.V[on + row] = v;
      P.RN[on + row] = rn;
      P.DR[on + row] = dr;
      ydr = P.y[row] * dr;
      steps_d = (double)steps;
    }
  }
  ydr = sum16(ydr);
  steps_d = max16(steps_d);
  if (live && (e & 15) == 0) {
    const size_t o = (size_t)pr * P.nb + bx;
    P.part_n1[o] = ydr;
    P.part_it[o] = steps_d;
    if (bx == 0) P.sc[pr].beta_bar = beta_bar;
  }
}

// ---------------------------------------------------------------------------
// Step 1c for every (row, problem) of the tile: G~ dr and M^-1 dr, both
// outcomes and their NPC partials (see k_step1c_rows).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NM_T) k_s1c_mm(BatchPtrs P, const int* __restrict__ idx,
                                                 int bact) {
  int bx, by;
  if (!nm_tile((P.n + 15) / 16, (bact + 15) / 16, bx, by)) return;
  __shared__ double red[2][NM_W][256];
  __shared__ double dsum[NM_W][16];
  const int r0 = bx * 16, c0 = by * 16;
  const double* A[2] = {P.G, P.Minv};
  double hv[2], mdr;
  nm_products<2, true>(A, nm_col(P, idx, bact, c0, P.DR, 0), P.my, P.n, r0, red, dsum, hv, &mdr);
  if (threadIdx.x >= 256) return;
  const int e = threadIdx.x, row = r0 + (e & 15), slot = c0 + (e >> 4);
  int pr = -1;
  bool live = false;
  if (slot < bact) {
    pr = idx[slot];
    live = !P.sc[pr].done;
  }
  double out[NPC];
#pragma unroll
  for (int j = 0; j < NPC; ++j) out[j] = 0.0;
  double beta1 = 0.0;
  if (live) {
    Scal* sc = P.sc + pr;
    const Consts c = P.cs[pr];
    const double beta_bar = sc->beta_bar;
    beta1 = beta_bar + mdr / c.ymy;
    if (row < c.n) {
      const size_t on = (size_t)pr * P.n;
      const double sigma = sc->sigma;
      const double hg = hv[0], hm = hv[1];
      const double dr = P.DR[on + row], rn = P.RN[on + row], a0 = P.AL[on + row];
      const double yi = P.y[row], xr = P.XX[on + row], pu = P.PU[on + row];
      const double s0 = P.S[on + row], v0 = P.V[on + row], f0 = P.F[on + row];
      const double my0 = P.my[row], t0 = P.T[on + row], ei = P.E[on + row];
      const double rq1 = pow_qp1(rn, c);
      const double rq = pow_q(rn, c);
      out[0] = dr * hg;
      {
        const double xi = fmax(0.0, rn - v0 + (a0 - c.C * ei) / sigma);
        const double pres = v0 + xi - rn;
        const double a1 = a0 - c.tau * sigma * pres;
        P.XI0[on + row] = xi;
        P.AL0[on + row] = a1;
        nspace_sums(c, rq, rq1, a1, xi, pres, yi, ei, out + 1);
        out[1 + 9] = s0 * (c.mu * (xr + beta_bar * yi - s0));
        out[1 + 10] = pu * s0;
      }
      {
        const double s = f0 - hm + beta1 * my0;
        const double v = s - (t0 - dr);
        const double xi = fmax(0.0, rn - v + (a0 - c.C * ei) / sigma);
        const double pres = v + xi - rn;
        const double a1 = a0 - c.tau * sigma * pres;
        P.S1[on + row] = s;
        P.V1[on + row] = v;
        P.XI1[on + row] = xi;
        P.AL1[on + row] = a1;
        nspace_sums(c, rq, rq1, a1, xi, pres, yi, ei, out + 1 + NPO);
        out[1 + NPO + 9] = s * (c.mu * (xr - dr + beta1 * yi - s));
        out[1 + NPO + 10] = pu * s;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NPC; ++j) out[j] = sum16(out[j]);
  if (live && (e & 15) == 0) {
    double* dst = P.part_c + ((size_t)pr * P.nb + bx) * NPC;
#pragma unroll
    for (int j = 0; j < NPC; ++j) dst[j] = out[j];
    if (bx == 0) P.sc[pr].beta1 = beta1;
  }
}

// ---------------------------------------------------------------------------
// Per problem: the Step 1c decision and gamma = min(1, R/||g||) from the
// block partials (fixed order), as step2_plan does for one problem.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_plan_b(BatchPtrs P, const int* __restrict__ idx,
                                                int f32) {
  const int pr = idx[blockIdx.x];
  Scal* sc = P.sc + pr;
  if (sc->done) return;
  const Consts c = P.cs[pr];
  const int k = sc->k;
  const double u2 = sc->u2;
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < P.nb; b += 256) {
    const double* r = P.part_c + ((size_t)pr * P.nb + b) * NPC;
    a[0] += r[0];
    a[1] += P.part_n1[(size_t)pr * P.nb + b];
    a[2] += r[1 + 9];
    a[3] += r[1 + 10];
    a[4] += r[1 + NPO + 9];
    a[5] += r[1 + NPO + 10];
  }
  block_sum_k<256, 6>(a);
  const Step2Plan pl = step2_plan_finish(c, a, k, u2);
  if (threadIdx.x == 0) {
    sc->redo = pl.redo;
    sc->gamma = pl.gamma;
  }
  if (P.rep) return;  // no pass in the representer iteration
  // the pass's right-hand operand for this slot, dense and pre-scaled:
  // column blockIdx.x of the k-major S, in the pass's product type
  const double* src = (pl.redo ? P.S1 : P.S) + (size_t)pr * P.n;
  const size_t sl = P.sbld;
  if (f32) {
    float* dst = P.SBf + blockIdx.x;
    for (int i = threadIdx.x; i < P.n; i += 256) dst[i * sl] = (float)(P.y[i] * c.inv_zs * src[i]);
  } else {
    double* dst = P.SB + blockIdx.x;
    for (int i = threadIdx.x; i < P.n; i += 256) dst[i * sl] = P.y[i] * c.inv_zs * src[i];
  }
}

// ---------------------------------------------------------------------------
// The pass over Z for all active problems: W = (Bm - Z~ S) / mu with the
// dense, pre-scaled operand S (row k = sample k, column slot = y .* s / Z_scale
// of the slot's chosen Step 1c outcome), on MFMA 16x16x4 (f32 or f64), fused
// with Steps 2-3:  g = w - rho/(sigma sqrt(mu)), u = gamma g,
// rho -= tau sigma sqrt(mu)(w - u), and per-problem block partials (NP2
// layout of the single pass; the two Z~ alpha entries are 0 here: the batched
// tail gets them in n-space).
//
// Block tile: 64 rows x 16 NB slots, 4 waves, wave w owns rows 16w..16w+15
// and all 16 NB slots, so one block reads its rows of X once for all the
// slots of the tile (with NB = 4, once for 64 problems).  64-row tiles keep
// the work per CU within one tile of even at d = 1e5 (1568 tiles on 256
// CUs); the A operand comes straight from global memory into the MFMA
// registers (lane l: row l % 16, sample l / 16 of each 4-sample step), the
// B tile (BK samples x 16 NB slots, shared by the four waves) goes through
// LDS, double-buffered with one barrier per K tile, and both are loaded one
// K tile ahead.  Column i of product b is slot NB i + b, so each lane reads
// its NB B values of a step as one contiguous LDS vector.  Every output
// element is the same sequence of MFMA steps over k whatever NB is, so the
// tile width (chosen by the host's tuner) does not change any result.
// FP32 products are summed in FP32 over 128 samples (four K tiles) and
// those sums added in FP64; FP64 products accumulate in the MFMA registers
// throughout.
// ---------------------------------------------------------------------------
constexpr int BT_M = 64, BT_T = 256;
static_assert(BT_M == 16 * (BT_T / 64), "each wave owns 16 rows of the tile");
constexpr int BT_SUM = 128;  // samples per FP32 partial sum of the FP32 products

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v_b __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaB;
template <>
struct MfmaB<float> {
  typedef f4v acc_t;
  __device__ static __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of register v of lane l in a 16x16 output block (column = l % 16)
  __device__ static __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <>
struct MfmaB<double> {
  typedef d4v_b acc_t;
  __device__ static __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int l, int v) { return 4 * v + (l >> 4); }
};

// K tile depth (samples).
template <typename T>
constexpr int pass_b_bk() {
  return 32;
}
// Rows of the pre-scaled operand S (n padded with zero rows to whole K tiles
// of either depth).
int batch_sb_rows(int n) { return (n + 63) / 64 * 64; }

// LDS row of the B tile: the tile's 16 NB slots plus 16 bytes, so that the
// four sample rows a half-wave reads start in different banks.
template <typename T, int NB>
constexpr int pass_b_bstride() {
  return 16 * NB + 16 / (int)sizeof(T);
}
// LDS row of the epilogue's (slot, row) staging: 64 rows plus one double (the
// lanes of a write differ in slot).
constexpr int BT_ZS = BT_M + 1;

// The NB consecutive B values of a lane's step as one LDS vector read.
template <typename T, int NB>
__device__ __forceinline__ void b_frag(const T* s, T (&b)[NB]) {
  if constexpr (NB == 1) {
    b[0] = s[0];
  } else if constexpr (sizeof(T) == 4 && NB == 2) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = *reinterpret_cast<const v2*>(s);
    b[0] = v.x;
    b[1] = v.y;
  } else if constexpr (sizeof(T) == 4 && NB == 4) {
    const f4v v = *reinterpret_cast<const f4v*>(s);
    b[0] = v.x;
    b[1] = v.y;
    b[2] = v.z;
    b[3] = v.w;
  } else {
#pragma unroll
    for (int h = 0; h < NB; h += 2) {
      const nt_d2 v = *reinterpret_cast<const nt_d2*>(s + h);
      b[h] = v.x;
      b[h + 1] = v.y;
    }
  }
}

// 16-byte chunk of the B tile (4 floats or 2 doubles).
template <typename T>
struct BChunk;
template <>
struct BChunk<float> {
  typedef f4v v_t;
};
template <>
struct BChunk<double> {
  typedef nt_d2 v_t;
};

// Raw buffer resource over [p, p + bytes) (gfx9 descriptor, no swizzle);
// loads past the end return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// (streamed once: non-temporal)
template <typename TD>
__device__ __forceinline__ TD buf_load_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(TD) == 4)
    return __builtin_bit_cast(TD, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 2));
  else
    return __builtin_bit_cast(TD, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 2));
}

template <typename TD, typename T, int NB>
__global__ void __launch_bounds__(BT_T) __attribute__((amdgpu_waves_per_eu(sizeof(TD) == 8 && NB == 4 ? 3 : 4)))
k_pass_b(const TD* __restrict__ X, BatchPtrs P, const T* __restrict__ SBk,
         const int* __restrict__ idx, int bact, int ny) {
  typedef typename MfmaB<T>::acc_t acc_t;
  typedef typename BChunk<T>::v_t chunk_t;
  constexpr int BN = 16 * NB;
  constexpr int BK = pass_b_bk<T>();
  constexpr int BK_STEPS = BK / 4;
  constexpr int BS = pass_b_bstride<T, NB>();
  constexpr bool F64 = sizeof(T) == 8;
  constexpr int VW = 16 / (int)sizeof(T);            // elements per 16-byte chunk
  constexpr int CPR = BN / VW;                       // chunks per B tile row
  constexpr int BCH = (BK * CPR + BT_T - 1) / BT_T;  // chunks per thread per tile
  constexpr size_t BBYTES = sizeof(T) * 2 * BK * BS;
  constexpr size_t ZBYTES = sizeof(double) * BN * BT_ZS;
  __shared__ __align__(16) unsigned char smem[BBYTES > ZBYTES ? BBYTES : ZBYTES];
  T(*Bs)[BK][BS] = reinterpret_cast<T(*)[BK][BS]>(smem);
  double(*Tz)[BT_ZS] = reinterpret_cast<double(*)[BT_ZS]>(smem);
  __shared__ int s_p[BN];
  __shared__ int s_live[BN];
  __shared__ double s_sig[BN], s_gam[BN], s_tau[BN];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // blocks of one XCD (linear id mod 8) take consecutive (row tile, slot
  // tile) pairs, so the slot tiles of a row tile read its X rows from the
  // same L2 at about the same time
  const int L = blockIdx.x;
  const int gi = L >> 3;
  const int rt = (gi / ny) * 8 + (L & 7);
  const int yt = gi % ny;
  const int64_t m0 = (int64_t)rt * BT_M;
  const int slot0 = yt * BN;
  const int bact_tile = min(BN, bact - slot0);
  const int n = P.n;
  const int64_t ld = P.ld;
  if (tid < BN) {
    const int slot = slot0 + tid;
    int p = -1, live = 0;
    if (tid < bact_tile) {
      p = idx[slot];
      live = P.sc[p].done ? 0 : 1;
    }
    s_p[tid] = p;
    s_live[tid] = live;
    if (live) {
      const Scal* sc = P.sc + p;
      s_sig[tid] = sc->sigma;
      s_gam[tid] = sc->gamma;
      s_tau[tid] = P.cs[p].tau;
    }
  }
  // A and B through buffer loads: a block-uniform base (per K tile) in the
  // resource and the lane's 32-bit offset in a VGPR.  Lane (li, lk) reads
  // row li of the wave's 16 in sample k0 + 4 s + lk of step s.  The A
  // resource ends at the end of X, so in the last K tile the samples past n
  // read as 0 (the hardware's range check; the S rows past n are 0 too).
  const uint32_t aoff = ((uint32_t)(wid * 16 + li) + (uint32_t)lk * (uint32_t)ld) * sizeof(TD);
  const uint32_t astep = 4u * (uint32_t)ld * sizeof(TD);
  auto load_a = [&](int k0, TD (&a)[BK_STEPS]) {
    const int64_t left = ((int64_t)(n - k0) * ld - m0) * (int64_t)sizeof(TD);
    const uint32_t nrec = left > (int64_t)0xffffffffLL ? 0xffffffffu : (uint32_t)left;
    const __amdgpu_buffer_rsrc_t r = buf_rsrc(X + m0 + (int64_t)k0 * ld, nrec);
#pragma unroll
    for (int s = 0; s < BK_STEPS; ++s) a[s] = buf_load_nt<TD>(r, aoff + s * astep, 0);
  };
  // B tile chunk c = tid + BT_T h: sample row c / CPR, slots VW (c % CPR) ..
  const uint32_t sbld = (uint32_t)P.sbld;
  const __amdgpu_buffer_rsrc_t rb = buf_rsrc(SBk + slot0, 0xffffffffu);
  uint32_t boff[BCH];
#pragma unroll
  for (int h = 0; h < BCH; ++h) {
    const uint32_t c = tid + h * BT_T;
    boff[h] = ((c / CPR) * sbld + VW * (c % CPR)) * sizeof(T);
  }
  auto load_b = [&](int k0, chunk_t (&b)[BCH]) {
    const uint32_t so = (uint32_t)k0 * sbld * sizeof(T);
#pragma unroll
    for (int h = 0; h < BCH; ++h)
      if (BK * CPR % BT_T == 0 || tid + h * BT_T < BK * CPR)
        b[h] = __builtin_bit_cast(chunk_t, __builtin_amdgcn_raw_buffer_load_b128(rb, boff[h], so, 0));
  };
  auto store_b = [&](int buf, const chunk_t (&b)[BCH]) {
#pragma unroll
    for (int h = 0; h < BCH; ++h) {
      const int c = tid + h * BT_T;
      if (BK * CPR % BT_T == 0 || c < BK * CPR)
        *reinterpret_cast<chunk_t*>(&Bs[buf][c / CPR][VW * (c % CPR)]) = b[h];
    }
  };
  acc_t acc[NB];
  double acc64[F64 ? 1 : NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[b][v] = (T)0;
  if constexpr (!F64) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[b][v] = 0.0;
  }
  // A is loaded two K tiles ahead into a ring of three register tiles
  // (the loop is unrolled by three so the ring rotates without copies), B
  // one tile ahead through the double-buffered LDS tile.  The loads are
  // unconditional (past the last tile they repeat it), so every step has the
  // same loads in flight, and each step issues B before A: B's wait at the
  // end of the step then leaves the two A tiles ahead in flight.
  // (The prologue leaves the loads in flight as every step does: the A
  // tile of the step after next, nothing else.)
  TD a0[BK_STEPS], a1[BK_STEPS], a2[BK_STEPS];
  chunk_t bnext[BCH];
  const int ntile = (n + BK - 1) / BK;
  load_a(0, a0);
  load_b(0, bnext);
  store_b(0, bnext);
  load_a(min(1, ntile - 1) * BK, a1);
  __syncthreads();
  auto step = [&](int t, const TD (&a)[BK_STEPS], TD (&fill)[BK_STEPS]) {
    const int buf = t & 1;
    load_b(min(t + 1, ntile - 1) * BK, bnext);
    load_a(min(t + 2, ntile - 1) * BK, fill);
#pragma unroll
    for (int s = 0; s < BK_STEPS; ++s) {
      T bv[NB];
      b_frag<T, NB>(&Bs[buf][4 * s + lk][NB * li], bv);
      const T av = (T)a[s];
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = MfmaB<T>::op(av, bv[b], acc[b]);
    }
    if constexpr (!F64) {
      if ((t + 1) % (BT_SUM / BK) == 0 || t + 1 == ntile) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            acc64[b][v] += (double)acc[b][v];
            acc[b][v] = 0.0f;
          }
      }
    }
    // (after the last tile this rewrites the other buffer, which nobody
    // reads any more)
    store_b(buf ^ 1, bnext);
    // the next tile's B is visible, and nobody reads this tile's buffer
    // after it is rewritten two tiles on
    __syncthreads();
  };
  int t = 0;
  for (; t + 3 <= ntile; t += 3) {
    step(t, a0, a2);
    step(t + 1, a1, a0);
    step(t + 2, a2, a1);
  }
  if (t < ntile) step(t, a0, a2);
  if (t + 1 < ntile) step(t + 1, a1, a0);
  const double mu = P.cs[s_p[0] >= 0 ? s_p[0] : 0].mu;
  const double sqmu = sqrt(mu);
  // Epilogue: the tile's 64 x 16 NB results are staged in LDS by (slot, row)
  // (over the B buffers, free after the last barrier); then 16 consecutive
  // threads take one slot's 64 rows in pairs (16-byte FP64 loads and stores
  // of the d-vectors) and sum its partials in a fixed tree.
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double zs;
      if constexpr (F64)
        zs = acc[b][v];
      else
        zs = acc64[b][v];
      Tz[NB * li + b][wid * 16 + MfmaB<T>::row(lane, v)] = zs;
    }
  __syncthreads();
  // Groups of 16 slots, 16 threads per slot and two row pairs per thread,
  // whatever NB is (so each slot's partials are summed in the same order for
  // every tile width); the d-vector loads of all groups are issued first.
  constexpr int EP = 2;                // row pairs per thread
  const int eg = tid / 16, q = tid % 16;
  nt_d2 rho2[NB][EP], u2[NB][EP];
#pragma unroll
  for (int g = 0; g < NB; ++g) {
    const int jj = g * 16 + eg;
    if (s_live[jj]) {
      const size_t od = (size_t)s_p[jj] * P.ld + m0;
#pragma unroll
      for (int i = 0; i < EP; ++i) {
        const int r = 2 * (q + 16 * i);
        rho2[g][i] = *reinterpret_cast<const nt_d2*>(P.RHO + od + r);
        u2[g][i] = *reinterpret_cast<const nt_d2*>(P.U + od + r);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < NB; ++g) {
    const int jj = g * 16 + eg;
    const int p = s_p[jj];
    const bool live = s_live[jj] != 0;
    double pw[NP2] = {0, 0, 0, 0, 0, 0};
    if (live) {
      const double sigma = s_sig[jj], gamma = s_gam[jj];
      const double br = sqmu / sigma, gr = 1.0 / (sigma * sqmu);
      const double rs = s_tau[jj] * sigma * sqmu;
      const size_t od = (size_t)p * P.ld + m0;
#pragma unroll
      for (int i = 0; i < EP; ++i) {
        const int r = 2 * (q + 16 * i);
        nt_d2 w2, un2, rn2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double zs = Tz[jj][r + h];
          const double rho = rho2[g][i][h];
          const double bb = mu * u2[g][i][h] + br * rho;
          const double w = (bb - zs) / mu;
          const double u = gamma * (w - gr * rho);
          const double rn = rho - rs * (w - u);
          w2[h] = w;
          un2[h] = u;
          rn2[h] = rn;
          pw[0] += (w - u) * (w - u);
          pw[1] += w * w;
          pw[4] += rn * rn;
          pw[5] += u * u;
        }
        *reinterpret_cast<nt_d2*>(P.W + od + r) = w2;
        *reinterpret_cast<nt_d2*>(P.U + od + r) = un2;
        *reinterpret_cast<nt_d2*>(P.RHO + od + r) = rn2;
      }
    }
#pragma unroll
    for (int qq = 0; qq < NP2; ++qq)
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) pw[qq] += __shfl_xor(pw[qq], o, 64);
    if (live && q == 0) {
#pragma unroll
      for (int qq = 0; qq < NP2; ++qq)
        P.part_g[((size_t)p * P.npb + rt) * NP2 + qq] = pw[qq];
    }
  }
}

// ---------------------------------------------------------------------------
// G~ alpha^{k+1} for every (row, problem) of the tile, with the partials of
// alpha^T G~ alpha for ||Z~ alpha||^2 (dual objective) and
// ||Z~ alpha + D rho||^2 (eta_D3).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NM_T) k_ga_mm(BatchPtrs P, const int* __restrict__ idx,
                                                int bact, int mode) {
  // mode 0: G~ alpha' (HA, part_ga); mode 1: G~ CV (part_gc, representer)
  int bx, by;
  if (!nm_tile((P.n + 15) / 16, (bact + 15) / 16, bx, by)) return;
  __shared__ double red[1][NM_W][256];
  const int r0 = bx * 16, c0 = by * 16;
  const double* A[1] = {P.G};
  double h;
  nm_products<1, false>(A, nm_col(P, idx, bact, c0, mode ? P.CV : nullptr, mode ? 0 : 1),
                        nullptr, P.n, r0, red, nullptr, &h, nullptr);
  if (threadIdx.x >= 256) return;
  const int e = threadIdx.x, row = r0 + (e & 15), slot = c0 + (e >> 4);
  int pr = -1;
  bool live = false;
  if (slot < bact) {
    pr = idx[slot];
    live = !P.sc[pr].done;
  }
  double contrib = 0.0;
  if (live && row < P.n) {
    const size_t on = (size_t)pr * P.n;
    if (mode) {
      contrib = P.CV[on + row] * h;
    } else {
      const double* al = (P.sc[pr].redo ? P.AL1 : P.AL0) + on;
      P.HA[on + row] = h;
      contrib = al[row] * h;
    }
  }
  contrib = sum16(contrib);
  if (live && (e & 15) == 0) (mode ? P.part_gc : P.part_ga)[(size_t)pr * P.nb + bx] = contrib;
}

// ---------------------------------------------------------------------------
// Representer iteration, element part (in place of the pass): per (row,
// problem) the coefficient updates of Steps 2-3 (see k_rep_step), CV and the
// NP2 partials of the d-space norms as n-space dot products; slots 2 and 3
// (||Z~ a + D rho||^2, ||Z~ a||^2) come from the two G~ products.
// Block = 256 rows of one active problem.
// ---------------------------------------------------------------------------
constexpr int RB_T = 256;

__global__ void __launch_bounds__(RB_T) k_rep_b(BatchPtrs P, const int* __restrict__ idx) {
  const int pr = idx[blockIdx.y];
  const Scal* sc = P.sc + pr;
  if (sc->done) return;
  const Consts c = P.cs[pr];
  const int o = sc->redo;
  const double sigma = sc->sigma, gamma = sc->gamma;
  const double beta = o ? sc->beta1 : sc->beta_bar;
  const double gr = 1.0 / (sigma * c.sqmu);
  const double rs = c.tau * sigma * c.sqmu;
  const size_t on = (size_t)pr * P.n;
  const int i = blockIdx.x * RB_T + threadIdx.x;
  double acc[NP2] = {0, 0, 0, 0, 0, 0};
  if (i < P.n) {
    const double s = (o ? P.S1 : P.S)[on + i];
    const double v = (o ? P.V1 : P.V)[on + i];
    const double al = (o ? P.AL1 : P.AL0)[on + i];
    const double au = P.AU[on + i], ar = P.ARHO[on + i], prv = P.PR[on + i];
    const double aw = au + gr * ar - s / c.mu;
    const double gaw = v - beta * P.y[i];
    const double au1 = gamma * (aw - gr * ar);
    const double pu1 = gamma * (gaw - gr * prv);
    const double ar1 = ar - rs * (aw - au1);
    const double pr1 = prv - rs * (gaw - pu1);
    P.AW[on + i] = aw;
    P.AU[on + i] = au1;
    P.ARHO[on + i] = ar1;
    P.CV[on + i] = al + c.sqmu * ar1;
    acc[0] = (aw - au1) * (gaw - pu1);
    acc[1] = aw * gaw;
    acc[4] = ar1 * pr1;
    acc[5] = au1 * pu1;
  }
  block_sum_k<RB_T, NP2>(acc);
  if (threadIdx.x < NP2)
    P.part_g[((size_t)pr * P.npg + blockIdx.x) * NP2 + threadIdx.x] = acc[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Per problem: commit of the Step 1c outcome, recurrences of Z~^T u and
// Z~^T rho, residuals, stopping and sigma rules, next t and x (k_tail),
// with ||Z~ alpha + D rho||^2 = a^T G~ a + 2 sqrt(mu) a^T Z~^T rho + mu ||rho||^2.
// ---------------------------------------------------------------------------
constexpr int NTB = 512;

__global__ void __launch_bounds__(NTB) k_tail_b(BatchPtrs P, const int* __restrict__ idx) {
  const int pr = idx[blockIdx.x];
  Scal* sc = P.sc + pr;
  if (sc->done) return;
  const Consts c = P.cs[pr];
  __shared__ double s_sigma;
  __shared__ double smax[NTB / 64];
  const size_t on = (size_t)pr * P.n;
  const int k0 = sc->k;
  const double sigma = sc->sigma;
  const double gamma = sc->gamma;
  const int o = sc->redo;
  const double beta = o ? sc->beta1 : sc->beta_bar;
  const int nd = sc->n_double;
  const int nm = sc->newton_max;
  constexpr int K = 9 + NP2 + 1;
  double acc[K];
#pragma unroll
  for (int j = 0; j < K; ++j) acc[j] = 0.0;
  double nmax = 0.0;
  for (int b = threadIdx.x; b < P.nb; b += NTB) {
    const double* r = P.part_c + ((size_t)pr * P.nb + b) * NPC + 1 + o * NPO;
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[j] += r[j];
    acc[9 + NP2] += P.part_ga[(size_t)pr * P.nb + b];
    nmax = fmax(nmax, P.part_it[(size_t)pr * P.nb + b]);
  }
  double cgc = 0.0;  // representer: CV^T G~ CV = ||Z~ alpha' + D rho'||^2
  for (int b = threadIdx.x; b < P.npg; b += NTB)
#pragma unroll
    for (int j = 0; j < NP2; ++j) acc[9 + j] += P.part_g[((size_t)pr * P.npg + b) * NP2 + j];
  if (P.rep)
    for (int b = threadIdx.x; b < P.nb; b += NTB) cgc += P.part_gc[(size_t)pr * P.nb + b];
  // commit and recurrences (old sigma), with a^T Z~^T rho^{k+1}
  const double gr = 1.0 / (sigma * c.sqmu);
  const double rs = c.tau * sigma * c.sqmu;
  const double* xs = (o ? P.XI1 : P.XI0) + on;
  const double* as = (o ? P.AL1 : P.AL0) + on;
  const double* ss = (o ? P.S1 : P.S) + on;
  const double* vs = (o ? P.V1 : P.V) + on;
  double apr = 0.0;
  for (int i = threadIdx.x; i < c.n; i += NTB) {
    const double v = vs[i];
    const double al = as[i];
    P.R[on + i] = P.RN[on + i];
    P.XI[on + i] = xs[i];
    P.AL[on + i] = al;
    if (o) {
      P.S[on + i] = ss[i];
      P.V[on + i] = v;
    }
    const double ztw = v - beta * P.y[i];
    const double prv = P.PR[on + i];
    const double pu = gamma * (ztw - gr * prv);
    const double prn = prv - rs * (ztw - pu);
    P.PU[on + i] = pu;
    P.PR[on + i] = prn;
    apr += al * prn;
  }
  double all[K + 2];
#pragma unroll
  for (int j = 0; j < K; ++j) all[j] = acc[j];
  all[K] = apr;
  all[K + 1] = cgc;
  block_sum_k<NTB, K + 2>(all);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) nmax = fmax(nmax, __shfl_xor(nmax, off, 64));
  if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = nmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = smax[0];
    for (int w = 1; w < NTB / 64; ++w) m = fmax(m, smax[w]);
    const double aGa = all[9 + NP2];
    const double rho2 = all[9 + 4];
    double red[R_COUNT];
    for (int j = 0; j < 9; ++j) red[R_PRES2 + j] = all[j];
    red[R_WU2] = all[9 + 0];
    red[R_W2] = all[9 + 1];
    red[R_DRES2] = P.rep ? fmax(all[K + 1], 0.0)
                         : fmax(aGa + 2.0 * c.sqmu * all[K] + c.mu * rho2, 0.0);
    red[R_ZA2] = aGa;
    red[R_G2] = 0.0;
    red[R_RHO2] = rho2;
    double e[E_COUNT];
    e[E_PCHK] = e[E_DCHK] = 0.0;
    finish_etas(c, red, e);
    for (int j = 0; j < R_COUNT; ++j) sc->red[j] = red[j];
    for (int j = 0; j < E_COUNT; ++j) sc->eta[j] = e[j];
    sc->u2 = all[9 + 5];
    sc->beta = beta;
    sc->doubled = o;
    sc->n_double = nd + o;
    if ((int)m > nm) sc->newton_max = (int)m;
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
    if (sc->done) sc->frozen_iter = k1;
    sc->sigma = sig;
    s_sigma = sig;
  }
  __syncthreads();
  const double sig1 = s_sigma;
  for (int i = threadIdx.x; i < c.n; i += NTB) {
    const double t = P.XI[on + i] - P.R[on + i] - P.AL[on + i] / sig1;
    P.T[on + i] = t;
    P.XX[on + i] = t + (c.mu * P.PU[on + i] + c.sqmu * P.PR[on + i] / sig1) / c.mu;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
bool batch_ptrs_ok(const BatchPtrs& P) {
  const void* req[] = {P.y, P.my, P.Minv, P.G, P.R, P.XI, P.AL, P.PU, P.PR, P.T, P.XX, P.F,
                       P.S, P.V, P.DR, P.RN, P.S1, P.V1, P.XI0, P.XI1, P.AL0, P.AL1, P.HA,
                       P.U, P.RHO, P.W, P.SB, P.SBf, P.part_n1, P.part_it, P.part_c, P.part_g,
                       P.part_ga, P.sc, P.cs};
  for (const void* q : req)
    if (!q) return false;
  // (K tile offsets into X and offsets into S are 32-bit)
  return P.ld % kLdAlign == 0 && (P.ld / BT_M) % 8 == 0 && P.ld <= ((int64_t)1 << 23) &&
         P.sbld % 64 == 0 && (int64_t)batch_sb_rows(P.n) * P.sbld * 8 < ((int64_t)1 << 32);
}

// The pass with a tile of 16 * tile slots per block (tile = 1, 2 or 4).
// One-dimensional grid of (row tile, slot tile) pairs, grouped by XCD in
// the kernel (the row tile count ld / 64 is a multiple of 8).
template <int NB>
static void pass_b_nb(const void* X, int storage, int fp64_mfma, const BatchPtrs& P,
                      const int* idx, int bact, hipStream_t st) {
  const int ny = (bact + 16 * NB - 1) / (16 * NB);
  const dim3 gp((unsigned)(P.ld / BT_M * ny));
  if (storage == DWD_FP32 && !fp64_mfma)
    hipLaunchKernelGGL((k_pass_b<float, float, NB>), gp, dim3(BT_T), 0, st, (const float*)X, P,
                       (const float*)P.SBf, idx, bact, ny);
  else if (storage == DWD_FP32)
    hipLaunchKernelGGL((k_pass_b<float, double, NB>), gp, dim3(BT_T), 0, st, (const float*)X, P,
                       (const double*)P.SB, idx, bact, ny);
  else
    hipLaunchKernelGGL((k_pass_b<double, double, NB>), gp, dim3(BT_T), 0, st, (const double*)X,
                       P, (const double*)P.SB, idx, bact, ny);
}

hipError_t launch_pass_b(const void* X, int storage, int fp64_mfma, const BatchPtrs& P,
                         const int* idx, int bact, int tile, hipStream_t st) {
  switch (tile) {
    case 1: pass_b_nb<1>(X, storage, fp64_mfma, P, idx, bact, st); break;
    case 2: pass_b_nb<2>(X, storage, fp64_mfma, P, idx, bact, st); break;
    case 4: pass_b_nb<4>(X, storage, fp64_mfma, P, idx, bact, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_iteration(const void* X, int storage, int fp64_mfma, const BatchPtrs& P,
                                  const int* idx, int bact, int tile, hipStream_t st,
                                  hipEvent_t ev0, hipEvent_t ev1) {
  if (!X || !idx || bact < 1 || !batch_ptrs_ok(P)) return hipErrorInvalidValue;
  if (storage != DWD_FP32 && storage != DWD_FP64) return hipErrorInvalidValue;
  if (P.nb != (P.n + 15) / 16) return hipErrorInvalidValue;
  const dim3 gnm(nm_grid(P.n, bact));
  hipLaunchKernelGGL(k_s1ab_mm, gnm, dim3(NM_T), 0, st, P, idx, bact);
  hipLaunchKernelGGL(k_s1c_mm, gnm, dim3(NM_T), 0, st, P, idx, bact);
  if (bact > P.sbld) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_plan_b, dim3(bact), dim3(256), 0, st, P, idx,
                     storage == DWD_FP32 && !fp64_mfma ? 1 : 0);
  if (P.rep) {
    if (!P.AU || !P.ARHO || !P.AW || !P.CV || !P.part_gc || P.npg < (P.n + RB_T - 1) / RB_T)
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rep_b, dim3((P.n + RB_T - 1) / RB_T, bact), dim3(RB_T), 0, st, P, idx);
    hipLaunchKernelGGL(k_ga_mm, gnm, dim3(NM_T), 0, st, P, idx, bact, 1);
  } else {
    if (P.npg != P.npb) return hipErrorInvalidValue;
    if (ev0) (void)hipEventRecord(ev0, st);
    hipError_t e = launch_pass_b(X, storage, fp64_mfma, P, idx, bact, tile, st);
    if (e != hipSuccess) return e;
    if (ev1) (void)hipEventRecord(ev1, st);
  }
  hipLaunchKernelGGL(k_ga_mm, gnm, dim3(NM_T), 0, st, P, idx, bact, 0);
  hipLaunchKernelGGL(k_tail_b, dim3(bact), dim3(NTB), 0, st, P, idx);
  return hipGetLastError();
}

int batch_pass_row_blocks(int64_t ld) { return (int)(ld / BT_M); }

}  // namespace dwd

namespace dwd {

// Final FP64 check of problem p (as k_check): partT holds the pass over the
// data of record with v1 = w~_p; part_dres the explicit ||Z~ alpha_p +
// D rho_p||^2 partials (nblk of them).
__global__ void __launch_bounds__(512) k_check_b(BatchPtrs P, int p, const double* partT,
                                                 int nchunks, const double* part_dres,
                                                 int nblk) {
  Scal* sc = P.sc + p;
  const Consts c = P.cs[p];
  const size_t on = (size_t)p * P.n;
  double acc[2] = {0, 0};
  const double beta = sc->beta;
  for (int i = threadIdx.x; i < c.n; i += 512) {
    double sw = 0.0;
    for (int ch = 0; ch < nchunks; ++ch) sw += partT[((int64_t)ch * 2) * c.n + i];
    const double yi = P.y[i];
    const double pres = yi * sw * c.inv_zs + beta * yi + P.XI[on + i] - P.R[on + i];
    acc[0] += pres * pres;
  }
  for (int b = threadIdx.x; b < nblk; b += 512) acc[1] += part_dres[b];
  block_sum_k<512, 2>(acc);
  if (threadIdx.x == 0) {
    const double den = c.opC;
    const double* e = sc->eta;
    const double p1 = sqrt(acc[0]) / den;
    const double d3 = sqrt(acc[1]) / den;
    sc->eta[E_PCHK] = fmax(p1, fmax(e[E_P2], e[E_P3]));
    sc->eta[E_DCHK] = fmax(e[E_D1], fmax(e[E_D2], c.rho_residual ? d3 : 0.0));
  }
}

__global__ void k_resume_b(BatchPtrs P, const int* __restrict__ idx, int cnt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < cnt) {
    Scal* sc = P.sc + idx[j];
    sc->done = 0;
    sc->converged = 0;
  }
}

// Re-anchor problem p: Z~^T u and Z~^T rho from a pass (partT, with y and
// 1/Z_scale folded in), then t and x of the next Step 1a.
__global__ void __launch_bounds__(256) k_anchor_b(BatchPtrs P, int p, const double* partT,
                                                  int nchunks) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  const Consts c = P.cs[p];
  const size_t on = (size_t)p * P.n;
  double su = 0.0, sr = 0.0;
  for (int ch = 0; ch < nchunks; ++ch) {
    su += partT[((int64_t)ch * 2) * P.n + i];
    sr += partT[((int64_t)ch * 2 + 1) * P.n + i];
  }
  const double yz = P.y[i] * c.inv_zs;
  const double pu = yz * su, pr = yz * sr;
  const double sigma = P.sc[p].sigma;
  P.PU[on + i] = pu;
  P.PR[on + i] = pr;
  const double t = P.XI[on + i] - P.R[on + i] - P.AL[on + i] / sigma;
  P.T[on + i] = t;
  P.XX[on + i] = t + (c.mu * pu + c.sqmu * pr / sigma) / c.mu;
}

hipError_t launch_anchor_b(const BatchPtrs& P, int p, const double* partT, int nchunks,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_anchor_b, dim3((P.n + 255) / 256), dim3(256), 0, st, P, p, partT, nchunks);
  return hipGetLastError();
}

hipError_t launch_resume_b(const BatchPtrs& P, const int* idx, int cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_resume_b, dim3((cnt + 63) / 64), dim3(64), 0, st, P, idx, cnt);
  return hipGetLastError();
}

hipError_t launch_check_b(const BatchPtrs& P, int p, const double* partT, int nchunks,
                          const double* part_dres, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_check_b, dim3(1), dim3(512), 0, st, P, p, partT, nchunks, part_dres, nblk);
  return hipGetLastError();
}

}  // namespace dwd
