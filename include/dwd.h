/*
 * dwd.h -- C ABI of an MI355X (gfx950) solver for generalized distance
 * weighted discrimination (DWD) by the inexact symmetric Gauss-Seidel ADMM
 * (arXiv 2305.12019), Sherman-Morrison-Woodbury branch.
 *
 * Problem (Section 2, eq-primal):
 *     min  sum_i v_i theta_q(r_i) + C <e, xi>
 *     s.t. Z^T w + beta y + xi - r = 0,  ||w|| <= 1,  xi >= 0,
 * with Z = X diag(y), theta_q(t) = t^-q for t > 0 (+inf otherwise), q > 0,
 * C > 0, a positive penalty vector e (default 1) and loss weights v_i
 * (default 1; the class weights of Section 4.5 on request).  X is d x n
 * (column i is the sample x_i), y in {-1,+1}^n.
 *
 * The solver scales the data as in Section 4.2 (Z~ = Z / sqrt(||X||_F)),
 * runs Algorithm 1 of Section 3 (Steps 1a, 1b, 1c, 2, 3) with the linear
 * system eq-linsys (T = 0) solved through eq-Ainv / eq-H, the Newton prox
 * of Section 3.2 and the residuals, stopping rule and sigma rule of
 * Sections 4.3-4.4, and returns the unscaled solution.
 *
 * Conventions for every call:
 *   - Inputs are borrowed for the duration of the call only.
 *   - Output arrays are caller-allocated HOST buffers of the stated length;
 *     a NULL output pointer means "not wanted".
 *   - No exception or longjmp crosses the ABI; every call returns a
 *     dwd_status.  Outputs are written only when the status is >= 0.
 *   - dwd_last_error() returns a message for the last failing call on the
 *     calling thread.
 *   - A dwd_problem handle is not thread-safe; distinct handles may be used
 *     from distinct threads on distinct streams.
 */
#ifndef DWD_H
#define DWD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DWD_OK = 0,             /* converged to the requested tolerance              */
  DWD_NOT_CONVERGED = 1,  /* iteration cap reached; outputs are valid          */
  DWD_E_INVALID = -1,     /* bad argument (message in dwd_last_error)          */
  DWD_E_NOMEM = -2,       /* device or host allocation failed / over budget    */
  DWD_E_DEVICE = -3,      /* HIP runtime error                                 */
  DWD_E_NUMERIC = -4,     /* non-positive pivot in the n x n factorisation     */
  DWD_E_BUSY = -5         /* serving: no slot could ever admit the request     */
} dwd_status;

typedef enum { DWD_FP64 = 0, DWD_FP32 = 1, DWD_BF16 = 2 } dwd_dtype;
typedef enum { DWD_DENSE = 0, DWD_CSR = 1 } dwd_layout;

/* How eq-linsys is solved (chosen at dwd_setup):
 *   DWD_SOLVER_SMW    Sherman-Morrison-Woodbury form (Section 3.3.2) with the
 *                     n x n factor; n <= 65536; every mode and input format.
 *   DWD_SOLVER_DIRECT the whole (d+1) x (d+1) matrix of eq-linsys, formed
 *                     and inverted once (Section 3.3.1); d <= 5120, dense X,
 *                     FP32 or FP64 storage, n limited only by memory;
 *                     dwd_solve and dwd_serve (not dwd_solve_batch or the
 *                     representer iteration).
 *   DWD_SOLVER_ITERATIVE  n and d both large (Section 3.3.3): eq-linsys is
 *                     first solved with T = 0 by PSQMR (two passes over X per
 *                     step), and once a solve needs more than
 *                     dwd_params.psqmr_max steps, with the proximal term T of
 *                     eq-T, built from the ell largest eigenpairs of Z~ Z~^T
 *                     (Lanczos at set-up), solved in closed form through
 *                     eq-schur (three passes over X per iteration, four when
 *                     Step 1c solves again).  Any n and d.  Dense X, FP32 or
 *                     FP64 storage, dwd_solve only.
 *   DWD_SOLVER_AUTO   the choice printed with the paper's solver pseudo-code
 *                     (Section 6.1): direct when d <= 5000; when d > 5000,
 *                     the SMW form if n < 0.2 d and n <= 2500, else the
 *                     iterative branch.  CSR input and BF16 storage, which
 *                     only the SMW form takes, resolve to SMW.               */
typedef enum {
  DWD_SOLVER_SMW = 0,
  DWD_SOLVER_DIRECT = 1,
  DWD_SOLVER_AUTO = 2,
  DWD_SOLVER_ITERATIVE = 3
} dwd_solver;

/* The data matrix X (d x n), Section 2 "X Matrix".
 * DWD_DENSE: values is d x n column-major with leading dimension d, i.e.
 *            sample i occupies values[i*d .. i*d+d-1]; dtype FP64 or FP32.
 * DWD_CSR:   X^T in compressed sparse rows: row i (sample i) holds the
 *            entries indices[indptr[i] .. indptr[i+1]-1] (feature ids in
 *            [0, d)) with values of type dtype (FP64 or FP32); nnz entries.
 * on_device: 1 if values/indptr/indices are device pointers on the current
 *            HIP device, 0 if host pointers.                                   */
typedef struct {
  int64_t d, n;
  int32_t dtype;
  int32_t layout;
  const void* values;
  const int64_t* indptr;
  const int32_t* indices;
  int64_t nnz;
  int32_t on_device;
  int32_t reserved;
} dwd_matrix;

/* Solver parameters.  dwd_default_params() fills the defaults below. */
typedef struct {
  double C;          /* penalty on xi, > 0 (Section 2)                          */
  double q;          /* exponent of theta_q, > 0 (Section 2)                    */
  double tol;        /* relative KKT tolerance in (0, 1) (Section 4.3); 1e-5    */
  int32_t max_iter;  /* iteration cap; 2000 (Section 4.3)                       */
  int32_t storage;   /* dwd_dtype of the device copy of X: FP64, FP32 or BF16;
                        BF16 requires an FP32 or FP64 X                         */
  double tau;        /* Step 3 step length; 1.618                               */
  double mu;         /* (1,1) shift of eq-linsys, D = sqrt(mu) I; 1             */
  double sigma0;     /* <= 0: min(10 C, n)^q (Section 4.4)                      */
  double eps_c;      /* constant of eps_k = c/(k+1)^1.5; < 0: 1/||Z~||_F,
                        0: always redo Step 1c                                  */
  int32_t rho_residual; /* 1: eta_D includes ||Z~ alpha + D rho||/(1+C)         */
  int32_t resync;    /* recompute Z~^T u and Z~^T rho by a pass over Z every
                        `resync` iterations (1 = two passes per iteration);
                        default 0: only at the start, otherwise carried by exact
                        n-space recurrences and verified by the final check   */
  int32_t check_every; /* iterations queued between host reads of the stop flag */
  int32_t refine;    /* BF16 storage: continue on FP32 data until tol is met;
                        0: stop after the BF16 phase (the final FP64 check then
                        only reports the residual against the data of record) */
  double lowp_tol;   /* BF16 storage: tolerance of the BF16 phase; <= 0: 30*tol */
  int32_t profile;   /* 1: time the Z-streaming kernels with HIP events
                        (dwd_solve_batch reads it from p[0])                    */
  int32_t batch_fp32; /* dwd_solve_batch: 1 (default) = FP32 MFMA products when
                        every tol >= 1e-5 (FP64 sums across K tiles, relative
                        error ~1e-7 per pass; each problem is then checked in
                        FP64 and, if the check misses tol, resumed from
                        re-anchored n-space state with FP64 products);
                        0 = FP64 MFMA products throughout                     */
  int32_t batch_tile; /* dwd_solve_batch: slots per block of the Z~ [s_1..s_B]
                        product, in units of 16: 1, 2 or 4; 0 (default) = chosen
                        per active-slot count by timing the candidates on the
                        first iterations (cached per device and shape).  Every
                        choice gives bit-identical results.                    */
  int32_t graph;     /* dwd_solve_batch: 1 (default) = replay each chunk of
                        check_every iterations as a captured hipGraph once the
                        tile is fixed (not with profile = 1); 0 = launch each
                        kernel.  Results are identical either way.             */
  int32_t sigma_every; /* apply the sigma rule of Section 4.4 after every
                        sigma_every-th iteration (the paper gives no cadence);
                        default 2 (1 = every iteration)                        */
  int32_t representer; /* dwd_solve / dwd_serve: 1 = representer iteration:
                        w, u, rho stay in range(Z~) (zero start, T = 0), so
                        they are carried as n-vectors (w~ = Z~ a_w, ...) and
                        every d-space norm of Steps 2-3 and Section 4.3 is an
                        n-space quadratic form with G~; an iteration reads
                        only the n x n matrices, and Z is streamed once at the
                        end (w = Z~ a_w) and by the final FP64 check.  Same
                        iterates as 0 in exact arithmetic.  0 (default) = one
                        pass over Z per iteration.  BF16 storage is not used
                        by the iteration in this mode.  2 = choose per
                        problem: the representer iteration when one more read
                        of the n x n G~ (8 n^2 bytes) costs less than the pass
                        it replaces (Z once in its storage type plus five
                        FP64 d-vectors), else the pass; the SMW set-up only
                        (the direct and iterative set-ups take 2 as 0).
                        dwd_info.representer reports the choice.              */
  int32_t class_weights; /* 1: weight the loss term of sample i by tau_i^q, the
                        class weights of Section 4.5 (tau_i = tau_-/max(tau_+,
                        tau_-) for y_i = +1, tau_+/max(tau_+, tau_-) for
                        y_i = -1, tau_+- = (n_+- log(n) / n)^(1/(1+q))); the
                        prox of Step 1b, eta_C3 (alpha_i - q v_i / r_i^(q+1))
                        and the objectives (sum v_i r_i^-q; kappa sum
                        v_i^(1/(q+1)) alpha_i^(q/(q+1))) carry the weight.
                        0 (default) = all weights 1.                         */
  int32_t solver;    /* dwd_solver, used by dwd_setup; default DWD_SOLVER_SMW  */
  int32_t ell;       /* DWD_SOLVER_ITERATIVE: eigenpairs in eq-T, 2..32; 0 = 10
                        (used by dwd_setup)                                    */
  const double* e;   /* host array of n positive finite penalty weights e_i of
                        eq-primal (the paper normalises ||e||_inf = 1), read
                        during the call; NULL (default) = e = 1.  C e replaces
                        C in Step 2, eta_D2, eta_C2 and the primal objective.
                        dwd_solve_batch takes each problem's own e.           */
  int32_t psqmr_max; /* DWD_SOLVER_ITERATIVE: Steps 1a and 1c first solve
                        eq-linsys with T = 0 by preconditioned symmetric QMR
                        to the accuracy of eq-linsys-tol (eps_k, 5 eps_k),
                        warm started, with the eq-T system as preconditioner;
                        once a solve needs more than psqmr_max steps, the
                        proximal term of eq-T is used for the rest of the
                        solve (Section 3.3.3).  Default 50; 0 = the proximal
                        term from the first iteration.                        */
  int32_t reserved;
} dwd_params;

/* Per-solve report.  Residuals are those of Section 4.3 on the scaled
 * problem (eq-gen-scale); *_check are recomputed after the loop with an
 * explicit pass Z~^T w over the data of record, in FP64.                       */
typedef struct {
  double beta;
  double primal_obj, dual_obj;
  double eta_p, eta_d, eta_c, eta_gap;
  double eta_p_check, eta_d_check, kkt_check;  /* kkt_check = max of the two   */
  double sigma;                                 /* final sigma                  */
  int32_t iters;        /* iterations performed                                */
  int32_t n_double;     /* iterations where Step 1c solved again               */
  int32_t newton_max;   /* most Newton steps of any prox in the solve          */
  int32_t converged;    /* 1 if the stopping rule of Section 4.3 was met       */
  int32_t iters_lowp;   /* iterations run on BF16 storage                      */
  int32_t status;       /* dwd_status of this problem                          */
  double setup_ms, solve_ms;
  double stream_ms;     /* profile=1: summed duration of the Z~ [s, alpha] passes
                           (dwd_solve_batch: of all Z~ [s_1..s_B] launches of the
                           batch, the same value in every report)              */
  int32_t stream_launches; /* profile=1: number of such launches               */
  int32_t resumed;      /* times the loop resumed because the final check failed */
  double streamT_ms;    /* profile=1: summed duration of the Z~^T [u, rho] passes */
  int32_t streamT_launches;
  int32_t graph_launches; /* dwd_solve_batch: chunks replayed as a captured graph */
  int32_t psqmr_steps;  /* DWD_SOLVER_ITERATIVE: PSQMR steps over the solve     */
  int32_t psqmr_solves; /* DWD_SOLVER_ITERATIVE: PSQMR solves (Steps 1a and 1c) */
  int32_t psqmr_switch; /* DWD_SOLVER_ITERATIVE: iteration from which the
                           proximal term of eq-T was used (0 with psqmr_max = 0);
                           -1 if PSQMR solved every system                     */
  int32_t representer;  /* the iteration form that ran: 1 representer, 0 pass   */
} dwd_info;

typedef struct dwd_problem_s* dwd_problem;

/* Fill *p with the defaults listed in dwd_params. */
void dwd_default_params(dwd_params* p);

/* Set up a problem on the current HIP device: validate X and y, copy X into
 * device storage of type p->storage (column-major, sample-contiguous, padded
 * leading dimension), compute Z_scale = sqrt(||X||_F) (Section 4.2), the
 * Gram matrix G~ = Z~^T Z~ and the inverse of I_n + G~/mu (the first
 * diagonal block of J in eq-H, Section 3.3.2), and J^-1 ybar.
 *   X:       data matrix (see dwd_matrix).
 *   y:       host array of n labels, each exactly +1 or -1, both present.
 *   p:       parameters (storage and mu are used here; C, q, tol are not).
 *   stream:  hipStream_t to run on (NULL: the default stream).
 *   out:     receives the handle; free it with dwd_free.
 * Errors: DWD_E_INVALID (sizes < 1, labels not +-1 or one class empty,
 * non-finite or all-zero X, CSR indices out of range), DWD_E_NOMEM,
 * DWD_E_NUMERIC (factorisation failed), DWD_E_DEVICE.                          */
dwd_status dwd_setup(const dwd_matrix* X, const double* y, const dwd_params* p,
                     void* stream, dwd_problem* out);

/* Run Algorithm 1 on the problem set up in P with the (C, q, tol, ...) of p,
 * from the initial point (r, xi, w, beta, u) = (1, 1, 0, 0, 0),
 * (alpha, rho) = (0, 0).  May be called repeatedly on one handle with
 * different parameters (the eq-linsys matrix depends only on X, y and mu).
 *   w:     d doubles, the unscaled normal vector (w~ / Z_scale).
 *   info:  report (may be NULL).
 *   alpha, r, xi: n doubles each (nullable).
 *   u:     d doubles, unscaled (nullable).   rho: d doubles, scaled (nullable).
 * Returns DWD_OK, DWD_NOT_CONVERGED (outputs valid), or an error.               */
dwd_status dwd_solve(dwd_problem P, const dwd_params* p, double* w, dwd_info* info,
                     double* alpha, double* r, double* xi, double* u, double* rho);

/* Solve B problems that share P's X and y but have their own (C, q, tol,
 * sigma0, ...) in p[0..B-1], stepping all of them together: the products
 * with Z become d x n by n x B and n x d by d x B matrix products.  This
 * rests on the matrix of eq-linsys depending on X, y and the (1,1) shift
 * only, not on sigma, C or q (Section 3.3.2, eq-Anew): one factor serves
 * every problem of the batch (a sweep over C and q, or the folds of a
 * cross-validation over one X).
 *   W:    d x B column-major host array (column j = w of problem j).
 *   info: B reports (nullable).
 * Each problem follows exactly the iteration it would follow alone; a
 * converged problem is frozen.  Needs a dense FP32 or FP64 set-up with the
 * SMW solver and d <= 8388608 (the product addresses a K tile of X with
 * 32-bit offsets), else DWD_E_INVALID.  Returns DWD_OK if all converged,
 * else DWD_NOT_CONVERGED, or an error.                                          */
dwd_status dwd_solve_batch(dwd_problem P, int32_t B, const dwd_params* p, double* W,
                           dwd_info* info);

/* Release every device and host resource of P (NULL is allowed). */
void dwd_free(dwd_problem P);

/* ---------------------------------------------------------------------
 * Serving: a trace of solve requests with arrival times is replayed in
 * real time.  Each request is a whole problem of Section 2 (its own X, y, C,
 * q, tolerance) solved by Algorithm 1 as dwd_solve would solve it; serving is
 * not in the paper, it is how such solves are run side by side on one GPU.
 * Requests are admitted while their device footprint fits the HBM budget and
 * a slot is free; their set-up runs beside the stepping; admitted problems of
 * the SMW form are stepped together, one iteration of each per round, by
 * launches that each cover all of them (direct-branch problems and sparse
 * passes per problem), so requests that arrive while others run join them.
 * Device memory comes from one allocation made when the replay starts.
 * ------------------------------------------------------------------- */
typedef struct {
  dwd_matrix X;        /* data (host or device)                               */
  const double* y;     /* n labels, host                                      */
  dwd_params params;   /* per-request parameters (storage, C, q, tol, ...)    */
  double t_arrival;    /* seconds after the start of the replay               */
} dwd_request;

typedef struct {
  double hbm_budget_bytes;  /* admission budget; <= 0: 80% of free device memory */
  int32_t max_slots;        /* problems stepped together; <= 0: 64               */
  int32_t iters_per_round;  /* iterations per admitted problem per round; >= 1   */
} dwd_serve_opts;

typedef struct {
  double* w;           /* caller-allocated, d doubles (nullable)              */
  dwd_info info;       /* filled by dwd_serve                                  */
  double t_admit, t_done;  /* seconds after the start of the replay            */
  int32_t status;      /* dwd_status of this request                          */
  int32_t reserved;
} dwd_response;

/* Replay nreq requests (sorted by t_arrival).  Returns DWD_OK when every
 * request was served (each response carries its own status), or an error
 * that stopped the replay.  A request whose footprint exceeds the whole
 * budget gets status DWD_E_BUSY and is skipped.                                */
dwd_status dwd_serve(const dwd_request* reqs, int32_t nreq, const dwd_serve_opts* opts,
                     dwd_response* out);

/* The penalty parameter of Section 4.1 for exponent q on P's data:
 *     C = 10^(q+1) max{1, 10^(q-1) log(n) max{1000, d}^(1/3) / dist^(q+1)},
 * dist = the median of the n_+ n_- Euclidean distances ||x_i - x_j|| between
 * a sample of each class (the mean of the two middle values for an even
 * count).  The distances come from the FP64 Gram matrix of dwd_setup
 * (||x_i - x_j||^2 = Z_scale^2 (G~_ii + G~_jj + 2 G~_ij) for y_i = -y_j) and
 * the median is an exact selection on the device (radix select on the
 * IEEE bit patterns of the squared distances), without storing the pairs.
 *   q: exponent (> 0).   C: receives the value.
 * Errors: DWD_E_INVALID (NULL handle or output, q <= 0), DWD_E_NOMEM,
 * DWD_E_DEVICE.                                                                */
dwd_status dwd_suggest_C(dwd_problem P, double q, double* C);

/* Allocation-free form of dwd_suggest_C, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, errors and value (bit for bit) as
 * dwd_suggest_C; the class split and the histogram of the radix selection
 * live in a fixed static device work area of 263,424 bytes that each GPU the
 * library runs on holds until the process ends, and the call performs no
 * device or host allocation (only small reads into stack variables; the
 * call synchronises P's stream).
 *   Limit: n <= 65536 samples; a larger n returns DWD_E_INVALID.
 *   Every call on one GPU shares that GPU's work area: calls that overlap in
 *   time on one GPU (several threads, or several streams) race, and the
 *   caller must serialise them.                                                */
dwd_status dwd_suggest_C_noalloc(dwd_problem P, double q, double* C);

/* Diagnostics: copy a set-up quantity of P to the host array out (count
 * doubles, must equal the quantity's size).  what is one of
 *   "zscale" (1): Z_scale = sqrt(||X||_F) of Section 4.2;
 *   "ymy"    (1): y^T M^-1 y with M = I + Z~^T Z~ / mu;
 *   "G"    (n*n): G~ = Z~^T Z~, row-major;
 *   "Minv" (n*n): M^-1, row-major;
 *   "my"     (n): M^-1 y;
 *   "psqmr_count" (1): PSQMR solves of the last dwd_solve (iterative branch);
 *   "psqmr_steps" (psqmr_count): the steps of each of those solves, in order.
 * Returns DWD_E_INVALID for an unknown name or a wrong count.                  */
dwd_status dwd_inspect(dwd_problem P, const char* what, double* out, int64_t count);

/* Device bytes dwd_setup would allocate for X with parameters p (used for
 * admission); 0 on invalid input.                                              */
int64_t dwd_footprint(const dwd_matrix* X, const dwd_params* p);

const char* dwd_status_str(dwd_status s);
const char* dwd_last_error(void);
const char* dwd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DWD_H */
