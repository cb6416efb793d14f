// Internal declarations shared by the HIP sources of libdwd.
//
// Data layout in HBM (per problem):
//   Xs   : d x n, column-major, sample-contiguous, leading dimension ld
//          (ld = d rounded up to a multiple of kLdAlign; padding rows are 0).
//          Holds X itself (not X diag(y)/Z_scale): the label signs and the
//          1/Z_scale of Section 4.2 are folded into the n-vectors that
//          multiply it, so the stored values are exactly the data of record
//          (FP64/FP32) or its round-to-nearest-even BF16 image.
//   G    : n x n FP64, G~ = Z~^T Z~ (Z~ = X diag(y) / Z_scale).
//   Minv : n x n FP64, inverse of M = I + G~/mu.
//   n-vectors FP64 (r, xi, alpha, ...), d-vectors FP64 of length ld.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dwd.h"

namespace dwd {

constexpr int kLdAlign = 1024;   // elements; every Z-streaming tile divides it
constexpr int kWave = 64;        // CDNA wavefront size
constexpr int kMaxEta = 24;
constexpr int NPO = 11;          // Step 1c partials per outcome: 9 sums + s^T G s + Pu^T s
constexpr int NPC = 1 + 2 * NPO; // Step 1c partials per block
constexpr int NP2 = 6;           // pass partials per block

// Blocks of the one-wave-per-row n x n kernels (4 rows per block).
__host__ __device__ inline int ngemv_blocks(int n) { return (n + 3) / 4; }

// Indices into Scal::red / Scal::eta.
enum RedIdx {
  R_PRES2 = 0,     // ||Z~^T w + beta y + xi - r||^2
  R_AMIN2,         // ||min(0, alpha)||^2
  R_AMAX2,         // ||max(0, alpha - C e)||^2
  R_YA,            // y^T alpha
  R_XCA,           // xi^T (C e - alpha)
  R_COMP2,         // ||alpha - q v / r^(q+1)||^2
  R_SUMRQ,         // sum v r^-q (v: loss weight)
  R_SUMXI,         // sum e xi
  R_SUMAQ,         // sum v^(1/(q+1)) max(alpha,0)^(q/(q+1))
  R_WU2,           // ||w - u||^2
  R_W2,            // ||w||^2
  R_DRES2,         // ||Z~ alpha + sqrt(mu) rho||^2
  R_ZA2,           // ||Z~ alpha||^2
  R_G2,            // ||g||^2
  R_RHO2,          // ||rho||^2
  R_COUNT
};

enum EtaIdx {
  E_P1 = 0, E_P2, E_P3, E_D1, E_D2, E_D3, E_C1, E_C2, E_C3, E_GAP,
  E_PRIM, E_DUAL, E_P, E_D, E_C, E_PCHK, E_DCHK, E_COUNT
};

// Device-resident scalar state of one problem.
struct Scal {
  double sigma;
  double beta;
  double beta_bar;
  double gamma;        // Step 2 ball scaling min(1, R/||g||) of this iteration
  double ytdr;         // y^T (r^{k+1} - r^k)
  double beta1;        // beta of the Step 1c re-solve
  double u2;           // ||u||^2 of the current u
  int32_t k;           // iterations completed
  int32_t done;        // stop flag read by every kernel
  int32_t converged;
  int32_t n_double;
  int32_t newton_max;
  int32_t doubled;     // this iteration redid Step 1c
  int32_t status;      // 0 ok, else a dwd_status error code
  int32_t frozen_iter; // batch: iteration at which the problem stopped
  int32_t redo;        // Step 1c outcome of this iteration (from the kernel that sizes Step 2)
  int32_t pad_;
  double red[R_COUNT];
  double eta[E_COUNT];
};

// Per-solve constants, passed to kernels by value.
struct Consts {
  int64_t d, ld;
  int32_t n, max_iter;
  double C, q, tau, mu, sqmu, R, inv_zs, tol, eps_c, ymy, kappa, opC;
  double c1, c2;       // q(q+2), q(q+1) (divided by sigma inside)
  double qexp;         // q/(q+1)
  int32_t rho_residual;
  int32_t qkind;       // 1,2,4: integer q; 5: q = 0.5; 0: general
  int32_t sigma_every; // the sigma rule runs after iterations k with k % sigma_every == 0
  int32_t representer; // 1: d-vectors carried as n-vector coefficients (w~ = Z~ a_w, ...)
  double sigma0;       // initial sigma (used by the batched initialiser)
  // loss weights of the theta_q terms by class (1 without class weights) and
  // their (q+1)-th roots, which enter the dual objective
  double wpos, wneg, wdpos, wdneg;
};

// Pointers of one problem's iteration state (all device).
struct IterPtrs {
  const double* y;
  const double* my;     // M^-1 y
  const double* Minv;
  const double* G;
  const double* e;      // penalty weights of eq-primal (ones by default)
  double *r, *xi, *alpha, *Pu, *Prho, *t, *x, *f, *s, *v, *dr, *hG, *rn;
  double *s1, *v1, *xi0, *xi1, *al0, *al1;  // the two outcomes of Step 1c
  double *au, *arho, *aw;  // representer coefficients: u~ = Z~ au, rho = Z~ arho, w~ = Z~ aw
  double *au_n, *arho_n;   // the representer step's new au, arho (the tail commits them)
  double *stg;             // 4 per column j: (y_j / Z_scale) [s, s1, alpha0, alpha1]_j
  double *u, *rho, *w;  // d-space, length ld
  // Block partials are stored slot-major, so that a reader summing one slot
  // over the blocks reads contiguous memory.
  double *part_g;       // pass partials: slot j of block b at part_g[j * pg_ld + b]
  double *part_n1;      // Step 1b block partials of y^T dr
  double *part_it;      // Step 1b block maxima of Newton steps
  double *part_c;       // Step 1c partials: slot j of block b at part_c[j * ngemv_blocks(n) + b]
  double *partT;        // GEMV-T partials: [chunks][2][n]
  Scal* sc;
  int32_t* hdone;       // pinned host word set to 1 with the stop flag (nullptr: none)
  int pg_ld;            // blocks per slot of part_g (the most blocks any pass launches)
};

// Pointers of a batch of B problems over one shared X.  n-space arrays are
// n x B and d-space arrays ld x B, column p = problem p (contiguous); block
// partials are indexed [problem][block][...].  idx maps active slots to
// problems.
struct BatchPtrs {
  const double* y;
  const double* my;
  const double* Minv;
  const double* G;
  const double* E;     // n x B penalty weights (column = problem)
  double *R, *XI, *AL, *PU, *PR, *T, *XX, *F, *S, *V, *DR, *RN, *S1, *V1, *XI0, *XI1, *AL0,
      *AL1, *HA;
  double *U, *RHO, *W;
  // the pass's operand S, k-major (row k = sample k, row length sbld >= B,
  // zero rows up to n rounded to 64): column slot = y .* s / Z_scale of the
  // slot's chosen outcome, in FP64 (SB) or FP32 (SBf) for the product type
  double* SB;
  float* SBf;
  int sbld;
  double *part_n1, *part_it, *part_c, *part_g, *part_ga;
  // representer mode: coefficients (u~ = Z~ AU, rho = Z~ ARHO, w~ = Z~ AW),
  // CV = alpha' + sqrt(mu) ARHO' (coefficients of Z~ alpha' + D rho') and the
  // block partials of CV^T G~ CV
  double *AU, *ARHO, *AW, *CV, *part_gc;
  Scal* sc;
  const Consts* cs;
  int n, nb, npb;      // nb: row blocks of the n x n kernels; npb: row blocks of the pass
  int npg;             // blocks of part_g per problem read by the tail (pass or element kernel)
  int rep;             // 1: representer iteration
  int64_t ld;
};

// Serving: one problem's entry in the table that the multi-problem
// kernels index by blockIdx.y (blockIdx.x stays the block index inside the
// problem, so each problem runs exactly the blocks of its own launch).
struct StepDesc {
  Consts c;
  IterPtrs p;
  const void* X;   // data the pass streams (dense)
  int npass;       // blocks of this problem's pass (or element step); the tail's nblk_d
  int nrow;        // ngemv_blocks(n)
};

enum MultiKernel { MULTI_STEP1AB = 0, MULTI_STEP1C, MULTI_REP, MULTI_PASS, MULTI_TAIL };

// Direct branch (Section 3.3.1): pointers of one problem's iteration state.
// d-vectors have length ld (ld + 1 for wbar and h, whose last entry is the
// beta component); zz holds [Z~ dr | Z~ (xi - r) | Z~ alpha], each ld long.
constexpr int NPD = 12;  // scalar partials per sweep block
struct DirPtrs {
  const double* y;
  const double* e;
  const double* Ainv;   // (d+1) x (d+1) row-major
  double *r, *xi, *alpha, *zb, *rn, *dr;   // n
  double *wbar, *w, *u, *rho, *h, *zz;     // d-space
  double* part_d;       // nblk x 2 ld: sweep partials of the d-vector sums
  double* part_n;       // NPD x nblk (slot-major): sweep 1 scalar partials (y^T dr, Newton steps)
  double* part_n2;      // NPD x nblk (slot-major): sweep 2 scalar partials (Section 4.3 terms)
  double* part_r;       // reduce-kernel partials of ||Z~ dr||^2
  Scal* sc;
  int nblk, per_block, nred;
};

// ---------------------------------------------------------------------------
// Reductions (fixed order, hence deterministic).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum K values over a block of NT threads; the result is valid in every
// thread.  Two levels (wave shuffles, then K threads over the waves), fixed
// order; the staging buffer is a block-level LDS array of this instantiation.
template <int NT, int K>
__device__ __forceinline__ void block_sum_k(double (&v)[K]) {
  constexpr int NW = NT / kWave;
  __shared__ double buf[NW * K + K];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = wave_sum(v[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) buf[wid * K + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int ww = 0; ww < NW; ++ww) s += buf[ww * K + threadIdx.x];
    buf[NW * K + threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = buf[NW * K + j];
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ double block_sum(double v) {
  double a[1] = {v};
  block_sum_k<NT, 1>(a);
  return a[0];
}

// bf16 (stored as uint16) -> float
__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) {
  return __uint_as_float(bits16 << 16);
}

// ---------------------------------------------------------------------------
// Host-side launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
struct Problem;

hipError_t launch_frob_copy(const void* X, int in_dtype, int64_t d, int n, void* Xs,
                            int storage, int64_t ld, double* part, int nparts, hipStream_t st);
hipError_t launch_sum(const double* part, int count, double* out, hipStream_t st);
hipError_t launch_gram(const void* Xs, int storage, int64_t ld, int n, double* Gpart,
                       int splits, hipStream_t st);
hipError_t launch_gram_finish(const double* Gpart, int splits, int n, const double* y,
                              double inv_zs2, double mu, double* G, double* M, hipStream_t st);
hipError_t spd_inverse_inplace(double* M, int n, double* work, int* d_status, hipStream_t st);
size_t spd_inverse_work(int n);  // doubles of work space spd_inverse_inplace needs
hipError_t launch_gemv_rows(const double* A, int n, const double* x, double* out,
                            hipStream_t st);
hipError_t launch_dot(const double* a, const double* b, int n, double* out, hipStream_t st);
// Histogram step of the radix selection over between-class squared distances
// (hist[256] must be zero on entry; see k_pair_hist).
hipError_t launch_pair_hist(const double* G, int n, const int* ipos, int npos, const int* ineg,
                            int nneg, unsigned long long prefix, int shift, unsigned int* hist,
                            hipStream_t st);
int gram_splits(int64_t ld, int n);
// Direct branch (kernels_direct.hip).
int fgram_splits(int d, int n);
hipError_t launch_fgram(const void* X, int storage, int64_t ld, int n, int d, double* Kpart,
                        int splits, hipStream_t st);
hipError_t launch_fgram_finish(const double* Kpart, int splits, int d, int n, const double* zy,
                               double inv_zs2, double mu, double* A, hipStream_t st);
int dir_sweep_samples_per_block(int64_t ld, int n, int storage);
int dir_reduce_blocks(int d, int nvec);

}  // namespace dwd
