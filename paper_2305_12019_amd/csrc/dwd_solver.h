// Host-side problem object and the launchers used by the drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "dwd_internal.h"
#include "dwd_iterative.h"

namespace dwd {

// launchers (kernels_iter.hip)
hipError_t launch_gemvT(const void* X, int storage, int64_t ld, int n, const double* v1,
                        const double* v2, double* part, const Scal* sc, hipStream_t st);
hipError_t launch_init(const Consts& c, const IterPtrs& p, double sigma0, hipStream_t st);
hipError_t launch_rhs(const Consts& c, const IterPtrs& p, int nchunks, int fresh, hipStream_t st);
hipError_t launch_ngemv(int n, const double* A1, const double* x1, double* o1, const double* A2,
                        const double* x2, double* o2, const double* wdot, double* part,
                        const Scal* sc, hipStream_t st);
hipError_t launch_step1ab(const Consts& c, const IterPtrs& p, hipStream_t st);
// Multi-problem launches over a device table of count StepDesc entries;
// gx = the largest block count among them (the pass: per storage type).
hipError_t launch_multi(int what, const StepDesc* D, int count, int gx, int storage,
                        hipStream_t st);
hipError_t launch_step1c_rows(const Consts& c, const IterPtrs& p, hipStream_t st);
hipError_t launch_pass2(const void* X, int storage, const Consts& c, const IterPtrs& p,
                        hipStream_t st);
int pass2_blocks(int storage, int64_t ld);
hipError_t launch_tail(const Consts& c, const IterPtrs& p, int nblk_d, hipStream_t st);
hipError_t launch_check(const Consts& c, const IterPtrs& p, int nchunks, const double* part_dres,
                        int nblk, hipStream_t st);
hipError_t launch_dres(const void* X, int storage, const Consts& c, const double* alpha,
                       const double* y, const double* rho, double* part, hipStream_t st);
int dres_blocks(int storage, int64_t ld);
hipError_t launch_csr_dres(const int64_t* ip, const int32_t* ix, const void* val, int dtype,
                           int64_t d, const Consts& c, const double* alpha, const double* y,
                           const double* rho, double* part, hipStream_t st);
bool iter_ptrs_ok(const IterPtrs& p);
// launchers of the direct branch (kernels_direct.hip)
hipError_t launch_dir_init(const Consts& c, const DirPtrs& p, double sigma0, hipStream_t st);
hipError_t launch_dir_gemv(const Consts& c, const DirPtrs& p, int mode, hipStream_t st);
hipError_t launch_dir_sweep(const void* X, int storage, const Consts& c, const DirPtrs& p,
                            int mode, hipStream_t st);
hipError_t launch_dir_reduce(const Consts& c, const DirPtrs& p, int v0, int nvec, double scale,
                             hipStream_t st);
hipError_t launch_dir_tail(const Consts& c, const DirPtrs& p, hipStream_t st);
hipError_t launch_csr_frob(const void* val, int dtype, int64_t nnz, double* part, int nblk,
                           hipStream_t st);
hipError_t launch_csr_gram(const int64_t* ip, const int32_t* ix, const void* val, int dtype, int n,
                           double* G, hipStream_t st);
hipError_t launch_csr_gemvT(const int64_t* ip, const int32_t* ix, const void* val, int dtype,
                            int n, const double* v1, const double* v2, double* part,
                            const Scal* sc, hipStream_t st);
hipError_t launch_csr_pass(const int64_t* ip, const int32_t* ix, const void* val, int dtype,
                           int64_t d, const Consts& c, const IterPtrs& p, hipStream_t st);
int csr_pass_blocks(int64_t ld);
hipError_t launch_norm2(const double* v, int64_t m, double* out, hipStream_t st);
hipError_t launch_rep_step(const Consts& c, const IterPtrs& p, hipStream_t st);
hipError_t launch_expand(const void* X, int storage, const Consts& c, const IterPtrs& p,
                         hipStream_t st);
hipError_t launch_expand3(const void* X, int storage, const Consts& c, const double* a0,
                          const double* a1, const double* a2, const double* y, double* o0,
                          double* o1, double* o2, hipStream_t st);
hipError_t launch_csr_expand(const int64_t* ip, const int32_t* ix, const void* val, int dtype,
                             int64_t d, const Consts& c, const IterPtrs& p, hipStream_t st);

// A device memory pool that a problem's buffers are taken from instead of
// hipMalloc (serving: one allocation up front, so that admitting and
// finishing requests neither allocates nor frees device memory, which would
// synchronise the device).  take() returns nullptr when no block fits.
struct DeviceArena {
  virtual void* take(size_t bytes) = 0;
  virtual void give(void* ptr) = 0;
  virtual ~DeviceArena() {}
};

// Word of Problem::h_flags that the n-space solver's tail kernel sets when it
// stops.  Words 0 and 16 take the direct and iterative solvers' copies of
// their flags, words 64 on the iterative solver's scalars.
constexpr int kHostDoneWord = 48;

struct Problem {
  int device = 0;
  DeviceArena* arena = nullptr;  // buffers from this pool (serving), else hipMalloc
  hipStream_t stream = nullptr;
  int64_t d = 0, ld = 0;
  int n = 0;
  int storage = DWD_FP32;
  int layout = DWD_DENSE;
  int64_t nnz = 0;
  double mu = 1.0, zscale = 1.0, ymy = 1.0;
  double setup_ms = 0.0;
  void* Xs = nullptr;          // storage image(s)
  const void* X_rec = nullptr; // data of record (FP64 or FP32 image)
  int st_rec = DWD_FP32;
  const void* X_lowp = nullptr;  // BF16 image (storage == BF16)
  int solver = DWD_SOLVER_SMW;  // factor built at set-up (SMW or direct)
  double* Ainv = nullptr;      // direct: inverse of the (d+1)^2 eq-linsys matrix
  DirPtrs dp{};                // direct: iteration state
  ItPtrs ipt{};                // iterative: iteration state
  PqPtrs pq{};                 // iterative: PSQMR state
  std::vector<int> psqmr_log;  // iterative: steps of each PSQMR solve of the last solve
  int psqmr_switch = -1;       // iterative: iteration at which eq-T was switched on
  double* y = nullptr;
  double* e = nullptr;         // penalty weights of eq-primal (n)
  bool e_ones = true;          // e currently holds all ones
  int64_t npos = 0, nneg = 0;  // class sizes (Section 4.5 weights)
  double* G = nullptr;
  double* Minv = nullptr;
  double* my = nullptr;
  double* d_scal = nullptr;
  // BF16 storage: the FP64 factor of the BF16 image (G~, M^-1, M^-1 y,
  // y^T M^-1 y of the problem the BF16 phase solves), and the iteration
  // pointers that use it.
  double* G_lp = nullptr;
  double* Minv_lp = nullptr;
  double* my_lp = nullptr;
  double ymy_lp = 1.0;
  IterPtrs ip{};
  IterPtrs ip_lp{};
  int nchunks = 0;
  void* h_flags = nullptr;     // pinned host words for stop flags (see kHostDoneWord)
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  hipEvent_t ev_chunk[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;    // 0: Z~ [s, alpha] pass, 1: Z~^T [u, rho] pass
  std::vector<int> ev_iter;    // iteration index of the timed launch
  std::vector<char> ev_live;   // 0 if the launch came after the stop flag was set
  int ev_used = 0;
  std::vector<void*> allocs;
  // CSR storage (layout == DWD_CSR): X^T by samples and X by features,
  // values FP64 (storage FP64) or FP32.
  const int64_t* ipT = nullptr;
  const int32_t* ixT = nullptr;
  const void* valT = nullptr;
  const int64_t* ipX = nullptr;
  const int32_t* ixX = nullptr;
  const void* valX = nullptr;
  int csr_dtype = DWD_FP32;

  hipError_t alloc(void** ptr, size_t bytes);
  // set-up scratch released before set-up returns (from the arena if any)
  hipError_t alloc_tmp(void** ptr, size_t bytes);
  void free_tmp(void* ptr);
  std::vector<void*> tmp_from_arena;
  hipError_t host_objects();
  hipError_t alloc_iter_buffers();
  // Load the penalty weights e of eq-primal for the next solve (host array
  // of n values, validated by the caller; NULL = all ones).
  hipError_t set_penalty(const double* eh);
  hipError_t queue_iteration(const Consts& c, const void* Xit, int st_it, bool fresh,
                             bool profile, int k);
  hipError_t run_loop(const Consts& c, const void* Xit, int st_it, int resync, int check_every,
                      bool profile, int k_start);
  // Z~^T [v1, v2] over the data of record into ip.partT (dense or CSR).
  hipError_t pass_T(const double* v1, const double* v2, const Scal* sc);
  // Representer mode: w, u, rho in d-space from their coefficients.
  hipError_t expand();
  // Explicit ||Z~ alpha + D rho||^2 partials of (alpha, rho) over the data of
  // record into part; returns the number of partials in *nblk.
  hipError_t dres(const Consts& c, const double* alpha, const double* rho, double* part,
                  int* nblk);
  // The final FP64 check of the single solve (expansion in representer
  // mode, Z~^T w pass, explicit dual residual, k_check), queued on stream.
  hipError_t queue_check(const Consts& c);
  hipEvent_t next_event(int kind, int k);
};

dwd_status fail(dwd_status s, const std::string& msg);
dwd_status hip_fail(hipError_t e, const char* where);
dwd_status validate_params(const dwd_params* p, bool for_solve);
// p->e, when given, must hold n positive finite values.
dwd_status validate_penalty(const dwd_params* p, int64_t n);
Consts make_consts(const Problem* P, const dwd_params* p);
// iteration form for dwd_params.representer (0, 1, or 2 = by bytes moved)
int choose_representer(const Problem* P, int req);
// Constants of the BF16 phase: its own y^T M^-1 y and the looser tolerance.
Consts lowp_consts(const Problem* P, const dwd_params* p);
double default_sigma0(const dwd_params* p, int n);
// The final FP64 check (Section 4.3 eta_P and eta_D recomputed over the data
// of record) decides convergence.  When the loop stopped on its in-loop
// residuals but the check reads chk >= tol, the loop resumes with its
// primal-dual target shrunk by the factor the check missed by (with margin);
// at most kMaxResume times.
constexpr int kMaxResume = 3;
inline double resume_tol(double cur, double tol, double chk) {
  const double f = 0.7 * tol / chk;
  return cur * (f < 0.05 ? 0.05 : (f > 0.5 ? 0.5 : f));
}
int64_t padded_ld(int64_t d);
int64_t problem_footprint(int64_t d, int n, int storage, int layout, int64_t nnz);
// With an arena (serving) every device buffer comes from it, and the
// host-side completion flags and timing events of dwd_solve are not made.
dwd_status setup_problem(const dwd_matrix* X, const double* y, const dwd_params* p,
                         hipStream_t st, Problem** out, DeviceArena* arena = nullptr);
// Release every resource of P (buffers back to its arena or hipFree) and delete it.
void destroy_problem(Problem* P);
dwd_status suggest_C(Problem* P, double q, double* C);
// The Section 4.1 formula from the bit patterns of the two middle squared
// distances (equal for an odd count).
dwd_status C_from_median_keys(const Problem* P, double q, unsigned long long k1,
                              unsigned long long k2, double* C);
// suggest_C without any allocation: its work area is a static device array
// (dwd_static.hip); n <= kStaticMaxN.
constexpr int kStaticMaxN = 65536;
dwd_status suggest_C_static(Problem* P, double q, double* C);
// Direct branch (dwd_direct.hip): the factor and buffers after the data are
// staged (Z_scale known), and the solve loop.
constexpr int64_t kDirectMaxD = 5120;
int64_t direct_ld(int64_t d);
dwd_status setup_direct(Problem* P, hipStream_t st);
dwd_status solve_direct(Problem* P, const dwd_params* p, double* w, dwd_info* info,
                        double* alpha, double* r, double* xi, double* u, double* rho);
int64_t direct_footprint(int64_t d, int n, int storage);
// One iteration of the direct branch queued on st (seven launches).
hipError_t queue_direct_iteration(Problem* P, const Consts& c, hipStream_t st);
// Iterative branch (dwd_iterative.hip).
dwd_status setup_iterative(Problem* P, const dwd_params* p, hipStream_t st);
dwd_status solve_iterative(Problem* P, const dwd_params* p, double* w, dwd_info* info,
                           double* alpha, double* r, double* xi, double* u, double* rho);
hipError_t queue_iterative_iteration(Problem* P, const Consts& c, hipStream_t st);
int64_t iterative_footprint(int64_t d, int n, int storage, int ell);
// The factor a set-up request resolves to (DWD_SOLVER_SMW or DWD_SOLVER_DIRECT).
int resolve_solver(const dwd_params* p, const dwd_matrix* X);
dwd_status solve_problem(Problem* P, const dwd_params* p, double* w, dwd_info* info,
                         double* alpha, double* r, double* xi, double* u, double* rho);
dwd_status solve_batch(Problem* P, int B, const dwd_params* p, double* W, dwd_info* info);

}  // namespace dwd
