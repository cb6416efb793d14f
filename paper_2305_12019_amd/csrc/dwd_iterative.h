// Iterative branch (Section 3.3.3, n and d both large): the proximal term
// of eq-T from the ell largest eigenpairs of Z~ Z~^T, which makes eq-linsys
// solvable in closed form through eq-schur.  Declarations shared by
// kernels_iterative.hip and dwd_iterative.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "dwd_internal.h"

namespace dwd {

constexpr int kItMaxEll = 32;      // largest ell
constexpr int kItMaxLanczos = 64;  // largest number of Lanczos steps
constexpr int kItDotsBlock = 4096; // features per block of the d-space dot kernel
constexpr int kItNpn = 12;         // scalar partials per n-space block

// Pointers of one problem's iterative-branch state (all device).  d-vectors
// have length ld (the SMW layout, padding entries zero).
struct ItPtrs {
  const double* y;
  const double* e;
  double *r, *xi, *alpha, *zb, *z, *rn, *dr;  // n
  double *a0, *a1, *a2;                       // n: operands of the 3-column Z~ pass
  double *w, *wbar, *u, *rho, *h;             // ld
  double *zz;          // 4 ld: [Z~ dr | Z~ (xi - r) | Z~ alpha | Z~ Z~^T w]
  double *scratch;     // 2 ld: unused outputs of the 3-column pass
  double *Wm;          // ell x ld: rows 0..ell-2 = v_1..v_{ell-1}, row ell-1 = g
  double *lam;         // ell eigenvalues, descending
  double *dots;        // ID_COUNT x (kItMaxLanczos + 2) dot results
  double *sca;         // iterative-branch scalars (see kernels_iterative.hip)
  double *partT;       // Z~^T pass partials, nchunks x 2 x n
  double *part_dd;     // d-space dot partials, nbd x (kItMaxLanczos + 2)
  double *part_n;      // n-space partials, nbn x kItNpn (sweep 1)
  double *part_n2;     // n-space partials, nbn x kItNpn (sweep 2)
  double *part_d;      // d-space partials, nbd2 x 8
  double *part3;       // Z~ [a0, a1, a2] sample-split partials, zsplits x 3 x ld
  Scal* sc;
  int ell, nchunks, nbd, nbn, nbd2, zsplits;
};

// Slots of ItPtrs::sca.
enum ItScal {
  IS_HB = 0,      // h_beta of the current right-hand side
  IS_BETABAR,     // betabar of Step 1a
  IS_SCHUR,       // y^T y - (Z~ y)^T g
  IS_YDR,         // y^T dr
  IS_G2,          // ||g||^2 of Step 2
  IS_COUNT
};

// Slots of ItPtrs::dots (each kItMaxLanczos + 2 long).
enum ItDots { ID_W = 0, ID_H = 1, ID_DR = 2, ID_AUX = 3, ID_PQ = 4, ID_COUNT = 5 };

// PSQMR (kernels_psqmr.hip): state of one solve of eq-linsys with T = 0.
// d-vectors have length ld; the beta components and the recurrence
// scalars are in s (slots below).
struct PqPtrs {
  double *x, *r, *rt, *q, *t, *d, *ad;  // ld each: iterate, residual, true
                                        // residual, direction, A q (then
                                        // M^-1 r), QMR update, A (update)
  const double* zy;    // ld: Z~ y
  double* a;           // n: Z~^T q_w + y q_b
  double* part;        // npart x 8 block partials
  double* part_n;      // nbn block partials of y^T Z~^T q_w
  double* s;           // scalars
  Scal* flag;          // done = 1 ends the solve (kernels return at once)
  int npart;
};

enum PqScal {
  PQ_XB = 0, PQ_RB, PQ_RTB, PQ_QB, PQ_TB, PQ_DB, PQ_ADB, PQ_UB,
  PQ_RHO, PQ_TAU, PQ_THETA, PQ_ALPHA, PQ_TAU_N, PQ_THETA_N, PQ_BRK,
  PQ_TOL, PQ_STEPS, PQ_OK, PQ_RES, PQ_RES1C, PQ_REDO, PQ_COUNT
};

hipError_t launch_it_reduceT(const Consts& c, const ItPtrs& p, int mode, hipStream_t st);
hipError_t launch_it_dots(const Consts& c, const ItPtrs& p, const double* x, const double* rows,
                          int nrows, int slot, int self, hipStream_t st);
hipError_t launch_it_rhs(const Consts& c, const ItPtrs& p, hipStream_t st, int with_T = 1);
hipError_t launch_it_solve(const Consts& c, const ItPtrs& p, int mode, hipStream_t st);
hipError_t launch_it_dspace(const Consts& c, const ItPtrs& p, int phase, hipStream_t st);
hipError_t launch_it_tail(const Consts& c, const ItPtrs& p, hipStream_t st);
hipError_t launch_it_init(const Consts& c, const ItPtrs& p, double sigma0, hipStream_t st);
// set-up: Lanczos steps and the small eigenproblem
hipError_t launch_it_lanczos_start(const Consts& c, double* v0, double* part, int nbd,
                                   hipStream_t st);
hipError_t launch_it_orth(const Consts& c, double* w, const double* V, int nrows,
                          const double* coef, hipStream_t st);
hipError_t launch_it_scale(const Consts& c, double* out, const double* in, const double* nrm2,
                           hipStream_t st);
hipError_t launch_it_eig(const double* alpha, const double* beta, int m, int ell, double* lam,
                         double* S, hipStream_t st);
hipError_t launch_it_ritz(const Consts& c, const double* V, int m, const double* S, int ell,
                          double* Wm, hipStream_t st);
hipError_t launch_it_gvec(const Consts& c, const ItPtrs& p, const double* Zy, hipStream_t st);
hipError_t launch_it_copy(double* dst, const double* src, int64_t count, hipStream_t st);
int it_zpass_splits(int64_t ld, int n);
// PSQMR launchers (kernels_psqmr.hip).  mode 0: Step 1a from [w; beta];
// mode 1: Step 1c re-solve from [wbar; betabar] with the residual in q.r.
int pq_dblocks(int64_t ld);
hipError_t launch_pq_start(const Consts& c, const ItPtrs& p, const PqPtrs& q, int mode,
                           hipStream_t st);
hipError_t launch_pq_precond(const Consts& c, const ItPtrs& p, const PqPtrs& q, int init,
                             hipStream_t st);
hipError_t launch_pq_step(const void* X, int storage, const Consts& c, const ItPtrs& p,
                          const PqPtrs& q, int j, int max_steps, hipStream_t st);
hipError_t launch_pq_res1c(const Consts& c, const ItPtrs& p, const PqPtrs& q, hipStream_t st);
// what 0: [wbar; betabar] = x; 1: [w; beta] = [wbar; betabar]; 2: [w; beta] = x
hipError_t launch_pq_commit(const Consts& c, const ItPtrs& p, const PqPtrs& q, int what,
                            hipStream_t st);
hipError_t launch_it_zpass(const void* X, int storage, const Consts& c, const ItPtrs& p,
                           const double* a0, const double* a1, const double* a2, double* o0,
                           double* o1, double* o2, const Scal* sc, hipStream_t st);

}  // namespace dwd
