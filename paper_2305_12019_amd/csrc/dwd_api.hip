// C ABI of libdwd: argument validation, problem set-up and the host driver
// of the iteration (Algorithm 1).  Device work is queued on the caller's
// stream; the host reads the device stop flag only every `check_every`
// iterations, one chunk behind the queue, so the GPU never waits for it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "dwd_internal.h"
#include "dwd_solver.h"

namespace dwd {

thread_local std::string g_err;

dwd_status fail(dwd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

dwd_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? DWD_E_NOMEM : DWD_E_DEVICE;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
  } while (0)

int64_t padded_ld(int64_t d) { return ((d + kLdAlign - 1) / kLdAlign) * kLdAlign; }

static size_t storage_bytes(int storage, int64_t ld, int n) {
  const size_t cnt = (size_t)ld * n;
  if (storage == DWD_FP64) return cnt * 8;
  if (storage == DWD_FP32) return cnt * 4;
  return cnt * 6;  // FP32 image of record + BF16 image
}

// Device bytes held by a set-up problem plus the set-up peak.
int64_t problem_footprint(int64_t d, int n, int storage, int layout, int64_t nnz) {
  const int64_t ld = padded_ld(d);
  int64_t b = (int64_t)storage_bytes(storage, ld, n);
  if (layout == DWD_CSR) b = 2 * nnz * (4 + (storage == DWD_FP64 ? 8 : 4)) + (n + d + 2) * 8;
  const int64_t nn = (int64_t)n * n * 8;
  b += 2 * nn;                                          // G~, M^-1
  if (storage == DWD_BF16 && layout != DWD_CSR) b += 2 * nn + (int64_t)n * 8;  // BF16 factor
  b += (int64_t)n * 8 * 33 + ld * 8 * 3;                // vectors (incl. y, e)
  b += (ld / kLdAlign) * 2 * (int64_t)n * 8;            // pass partials
  const int splits = gram_splits(ld, n);
  b += std::max<int64_t>({(int64_t)splits * nn, nn, (int64_t)spd_inverse_work(n) * 8});  // set-up scratch
  return b;
}

dwd_status validate_params(const dwd_params* p, bool for_solve) {
  if (!p) return fail(DWD_E_INVALID, "params is NULL");
  if (!(p->mu > 0.0) || !std::isfinite(p->mu)) return fail(DWD_E_INVALID, "mu must be > 0");
  if (p->storage != DWD_FP64 && p->storage != DWD_FP32 && p->storage != DWD_BF16)
    return fail(DWD_E_INVALID, "storage must be DWD_FP64, DWD_FP32 or DWD_BF16");
  if (!for_solve) return DWD_OK;
  if (!(p->C > 0.0) || !std::isfinite(p->C)) return fail(DWD_E_INVALID, "C must be > 0");
  if (!(p->q > 0.0) || !std::isfinite(p->q) || p->q > 64.0)
    return fail(DWD_E_INVALID, "q must be in (0, 64]");
  if (!(p->tol > 0.0 && p->tol < 1.0)) return fail(DWD_E_INVALID, "tol must be in (0, 1)");
  if (p->max_iter < 1) return fail(DWD_E_INVALID, "max_iter must be >= 1");
  if (!(p->tau > 0.0 && p->tau < 0.5 * (1.0 + sqrt(5.0))))
    return fail(DWD_E_INVALID, "tau must be in (0, (1+sqrt 5)/2)");
  if (!std::isfinite(p->sigma0) || !std::isfinite(p->eps_c))
    return fail(DWD_E_INVALID, "sigma0 and eps_c must be finite");
  if (p->batch_tile != 0 && p->batch_tile != 1 && p->batch_tile != 2 && p->batch_tile != 4)
    return fail(DWD_E_INVALID, "batch_tile must be 0, 1, 2 or 4");
  if (p->sigma_every < 1) return fail(DWD_E_INVALID, "sigma_every must be >= 1");
  if (p->representer < 0 || p->representer > 2)
    return fail(DWD_E_INVALID, "representer must be 0, 1 or 2");
  if (p->psqmr_max < 0 || p->psqmr_max > 100000)
    return fail(DWD_E_INVALID, "psqmr_max must be in [0, 100000]");
  if (p->class_weights != 0 && p->class_weights != 1)
    return fail(DWD_E_INVALID, "class_weights must be 0 or 1");
  if (p->solver < DWD_SOLVER_SMW || p->solver > DWD_SOLVER_ITERATIVE)
    return fail(DWD_E_INVALID, "solver must be DWD_SOLVER_SMW, _DIRECT, _AUTO or _ITERATIVE");
  if (p->ell < 0 || p->ell == 1 || p->ell > kItMaxEll)
    return fail(DWD_E_INVALID, "ell must be 0 (default) or 2..32");
  return DWD_OK;
}

dwd_status validate_penalty(const dwd_params* p, int64_t n) {
  if (!p->e) return DWD_OK;
  for (int64_t i = 0; i < n; ++i)
    if (!(p->e[i] > 0.0) || !std::isfinite(p->e[i]))
      return fail(DWD_E_INVALID, "penalty weights e must be positive and finite");
  return DWD_OK;
}

static dwd_status validate_matrix(const dwd_matrix* X) {
  if (!X) return fail(DWD_E_INVALID, "X is NULL");
  if (X->d < 1 || X->n < 1) return fail(DWD_E_INVALID, "d and n must be >= 1");
  if (X->n > 2147483647LL) return fail(DWD_E_INVALID, "n must fit in 32 bits");
  if (X->d > ((int64_t)1 << 40)) return fail(DWD_E_INVALID, "d too large");
  if (X->dtype != DWD_FP64 && X->dtype != DWD_FP32)
    return fail(DWD_E_INVALID, "X dtype must be DWD_FP64 or DWD_FP32");
  if (X->layout != DWD_DENSE && X->layout != DWD_CSR)
    return fail(DWD_E_INVALID, "X layout must be DWD_DENSE or DWD_CSR");
  if (!X->values) return fail(DWD_E_INVALID, "X values is NULL");
  if (X->layout == DWD_CSR) {
    if (!X->indptr || !X->indices) return fail(DWD_E_INVALID, "CSR indptr/indices is NULL");
    if (X->nnz < 0) return fail(DWD_E_INVALID, "nnz < 0");
  }
  return DWD_OK;
}

static dwd_status validate_labels(const double* y, int64_t n) {
  if (!y) return fail(DWD_E_INVALID, "y is NULL");
  int64_t npos = 0, nneg = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (y[i] == 1.0) ++npos;
    else if (y[i] == -1.0) ++nneg;
    else return fail(DWD_E_INVALID, "labels must be exactly +1 or -1");
  }
  if (npos == 0 || nneg == 0) return fail(DWD_E_INVALID, "both classes must be present");
  return DWD_OK;
}

// ---------------------------------------------------------------------------
// Problem set-up.
// ---------------------------------------------------------------------------
static void release(Problem* P) {
  if (!P) return;
  for (void* ptr : P->allocs) {
    if (P->arena)
      P->arena->give(ptr);
    else
      (void)hipFree(ptr);
  }
  P->allocs.clear();
  if (P->h_flags) (void)hipHostFree(P->h_flags);
  P->h_flags = nullptr;
  for (auto& e : P->ev_pool) (void)hipEventDestroy(e);
  P->ev_pool.clear();
  if (P->ev_a) (void)hipEventDestroy(P->ev_a);
  if (P->ev_b) (void)hipEventDestroy(P->ev_b);
  for (auto& e : P->ev_chunk) if (e) (void)hipEventDestroy(e);
  P->ev_a = P->ev_b = nullptr;
}

// Pinned completion flags and events of dwd_solve.
hipError_t Problem::host_objects() {
  hipError_t e;
  if ((e = hipHostMalloc((void**)&h_flags, 4096, 0)) != hipSuccess) return e;
  // the tail kernel of the n-space solver sets this word when it stops
  void* dflags = nullptr;
  if ((e = hipHostGetDevicePointer(&dflags, h_flags, 0)) != hipSuccess) return e;
  ip.hdone = ip_lp.hdone = (int32_t*)dflags + kHostDoneWord;
  if ((e = hipEventCreate(&ev_a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&ev_b)) != hipSuccess) return e;
  for (auto& ev : ev_chunk)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
  return hipSuccess;
}

void destroy_problem(Problem* P) {
  release(P);
  delete P;
}

hipError_t Problem::alloc(void** ptr, size_t bytes) {
  if (arena) {
    *ptr = arena->take(bytes ? bytes : 8);
    if (!*ptr) return hipErrorOutOfMemory;
    allocs.push_back(*ptr);
    return hipSuccess;
  }
  hipError_t e = hipMalloc(ptr, bytes ? bytes : 8);
  if (e == hipSuccess) allocs.push_back(*ptr);
  return e;
}

// (a fragmented arena falls back to hipMalloc for set-up scratch)
hipError_t Problem::alloc_tmp(void** ptr, size_t bytes) {
  if (arena && (*ptr = arena->take(bytes ? bytes : 8)) != nullptr) {
    tmp_from_arena.push_back(*ptr);
    return hipSuccess;
  }
  return hipMalloc(ptr, bytes ? bytes : 8);
}

void Problem::free_tmp(void* ptr) {
  if (!ptr) return;
  for (void* a : tmp_from_arena)
    if (a == ptr) {
      arena->give(ptr);
      tmp_from_arena.erase(std::find(tmp_from_arena.begin(), tmp_from_arena.end(), ptr));
      return;
    }
  (void)hipFree(ptr);
}

dwd_status setup_problem(const dwd_matrix* X, const double* y, const dwd_params* p,
                         hipStream_t st, Problem** out, DeviceArena* arena) {
  dwd_status s;
  if ((s = validate_matrix(X)) != DWD_OK) return s;
  if ((s = validate_params(p, false)) != DWD_OK) return s;
  if (p->solver < DWD_SOLVER_SMW || p->solver > DWD_SOLVER_ITERATIVE)
    return fail(DWD_E_INVALID, "solver must be DWD_SOLVER_SMW, _DIRECT, _AUTO or _ITERATIVE");
  if (p->ell < 0 || p->ell == 1 || p->ell > kItMaxEll)
    return fail(DWD_E_INVALID, "ell must be 0 (default) or 2..32");
  const int solver = resolve_solver(p, X);
  if (solver == DWD_SOLVER_ITERATIVE) {
    if (X->layout != DWD_DENSE) return fail(DWD_E_INVALID, "the iterative solver needs dense X");
    if (p->storage == DWD_BF16)
      return fail(DWD_E_INVALID, "the iterative solver needs FP32 or FP64 storage");
  } else if (solver == DWD_SOLVER_DIRECT) {
    if (X->layout != DWD_DENSE) return fail(DWD_E_INVALID, "the direct solver needs dense X");
    if (p->storage == DWD_BF16)
      return fail(DWD_E_INVALID, "the direct solver needs FP32 or FP64 storage");
    if (X->d > kDirectMaxD) return fail(DWD_E_INVALID, "the direct solver needs d <= 5120");
  } else if (X->n > 65536) {
    return fail(DWD_E_INVALID, "n > 65536 is not supported by the n x n factor");
  }
  if ((s = validate_labels(y, X->n)) != DWD_OK) return s;
  auto t0 = std::chrono::steady_clock::now();
  Problem* P = new Problem();
  P->arena = arena;
  P->stream = st;
  P->d = X->d;
  P->n = (int)X->n;
  P->solver = solver;
  P->ld = solver == DWD_SOLVER_DIRECT ? direct_ld(X->d) : padded_ld(X->d);
  const int ell_req = p->ell;
  P->storage = p->storage;
  P->mu = p->mu;
  P->layout = X->layout;
  HIP_TRY(hipGetDevice(&P->device));
  const int n = P->n;
  const int64_t d = P->d, ld = P->ld;

  // Stage the input as a dense d x n device array in its own dtype.
  const void* Xdev = X->values;
  void* Xtmp = nullptr;
  const size_t in_el = X->dtype == DWD_FP64 ? 8 : 4;
  std::vector<int64_t> ipT_h, ipX_h;
  std::vector<int32_t> ixT_h, ixX_h;
  std::vector<double> valT_h, valX_h;
  if (X->layout == DWD_CSR) {
    // Validate on the host; sort each sample row by feature index; build
    // the by-feature transpose (rows stay sorted by sample index).
    ipT_h.resize(n + 1);
    if (X->on_device) {
      HIP_TRY(hipMemcpy(ipT_h.data(), X->indptr, (n + 1) * 8, hipMemcpyDeviceToHost));
    } else {
      memcpy(ipT_h.data(), X->indptr, (n + 1) * 8);
    }
    if (ipT_h[0] != 0 || ipT_h[n] != X->nnz) {
      delete P;
      return fail(DWD_E_INVALID, "CSR indptr must start at 0 and end at nnz");
    }
    for (int i = 0; i < n; ++i)
      if (ipT_h[i + 1] < ipT_h[i]) {
        delete P;
        return fail(DWD_E_INVALID, "CSR indptr must be non-decreasing");
      }
    const int64_t nnz = X->nnz;
    ixT_h.resize(nnz);
    valT_h.resize(nnz);
    std::vector<char> raw(nnz * in_el);
    if (X->on_device) {
      HIP_TRY(hipMemcpy(ixT_h.data(), X->indices, nnz * 4, hipMemcpyDeviceToHost));
      HIP_TRY(hipMemcpy(raw.data(), X->values, nnz * in_el, hipMemcpyDeviceToHost));
    } else {
      memcpy(ixT_h.data(), X->indices, nnz * 4);
      memcpy(raw.data(), X->values, nnz * in_el);
    }
    for (int64_t e = 0; e < nnz; ++e)
      valT_h[e] = X->dtype == DWD_FP64 ? ((const double*)raw.data())[e]
                                        : (double)((const float*)raw.data())[e];
    std::vector<int64_t> ord;
    for (int i = 0; i < n; ++i) {
      const int64_t a = ipT_h[i], b = ipT_h[i + 1];
      ord.resize(b - a);
      for (int64_t e = a; e < b; ++e) ord[e - a] = e;
      std::sort(ord.begin(), ord.end(), [&](int64_t u, int64_t v) { return ixT_h[u] < ixT_h[v]; });
      std::vector<int32_t> ci(b - a);
      std::vector<double> cv(b - a);
      for (int64_t e = a; e < b; ++e) {
        ci[e - a] = ixT_h[ord[e - a]];
        cv[e - a] = valT_h[ord[e - a]];
      }
      for (int64_t e = a; e < b; ++e) {
        ixT_h[e] = ci[e - a];
        valT_h[e] = cv[e - a];
        if (ixT_h[e] < 0 || ixT_h[e] >= d) {
          delete P;
          return fail(DWD_E_INVALID, "CSR column index out of range");
        }
        if (e > a && ixT_h[e] == ixT_h[e - 1]) {
          delete P;
          return fail(DWD_E_INVALID, "duplicate column index in a CSR row");
        }
        if (!std::isfinite(valT_h[e])) {
          delete P;
          return fail(DWD_E_INVALID, "X has non-finite entries");
        }
      }
    }
    ipX_h.assign(d + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) ipX_h[ixT_h[e] + 1] += 1;
    for (int64_t k = 0; k < d; ++k) ipX_h[k + 1] += ipX_h[k];
    ixX_h.resize(nnz);
    valX_h.resize(nnz);
    std::vector<int64_t> fill(ipX_h.begin(), ipX_h.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int64_t e = ipT_h[i]; e < ipT_h[i + 1]; ++e) {
        const int64_t o = fill[ixT_h[e]]++;
        ixX_h[o] = i;
        valX_h[o] = valT_h[e];
      }
    P->nnz = nnz;
  } else if (!X->on_device) {
    size_t bytes = (size_t)d * n * in_el;
    hipError_t e = P->alloc_tmp(&Xtmp, bytes);
    if (e != hipSuccess) { delete P; return hip_fail(e, "hipMalloc(X staging)"); }
    e = hipMemcpyAsync(Xtmp, X->values, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(st);
      P->free_tmp(Xtmp);
      delete P;
      return hip_fail(e, "H2D X");
    }
    Xdev = Xtmp;
  }

  auto cleanup = [&](dwd_status st_) {
    (void)hipStreamSynchronize(st);
    if (Xtmp) P->free_tmp(Xtmp);
    release(P);
    delete P;
    return st_;
  };

  hipError_t e;
  const bool csr = X->layout == DWD_CSR;
  if (csr) {
    // CSR storage: values FP64 for FP64 storage, else FP32 (no BF16 phase).
    if (P->storage == DWD_BF16) P->storage = DWD_FP32;
    P->csr_dtype = P->storage == DWD_FP64 ? DWD_FP64 : DWD_FP32;
    const size_t vb = P->csr_dtype == DWD_FP64 ? 8 : 4;
    const int64_t nnz = P->nnz;
    void *ipT, *ixT, *vT, *ipX, *ixX, *vX;
    if ((e = P->alloc(&ipT, (n + 1) * 8)) != hipSuccess ||
        (e = P->alloc(&ixT, nnz * 4)) != hipSuccess || (e = P->alloc(&vT, nnz * vb)) != hipSuccess ||
        (e = P->alloc(&ipX, (d + 1) * 8)) != hipSuccess ||
        (e = P->alloc(&ixX, nnz * 4)) != hipSuccess || (e = P->alloc(&vX, nnz * vb)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMalloc(CSR)"));
    std::vector<float> f32;
    auto up = [&](void* dst, const std::vector<double>& src) -> hipError_t {
      if (vb == 8) return hipMemcpy(dst, src.data(), nnz * 8, hipMemcpyHostToDevice);
      f32.resize(nnz);
      for (int64_t q = 0; q < nnz; ++q) f32[q] = (float)src[q];
      return hipMemcpy(dst, f32.data(), nnz * 4, hipMemcpyHostToDevice);
    };
    if ((e = hipMemcpy(ipT, ipT_h.data(), (n + 1) * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(ixT, ixT_h.data(), nnz * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = up(vT, valT_h)) != hipSuccess ||
        (e = hipMemcpy(ipX, ipX_h.data(), (d + 1) * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(ixX, ixX_h.data(), nnz * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = up(vX, valX_h)) != hipSuccess)
      return cleanup(hip_fail(e, "H2D CSR"));
    P->ipT = (const int64_t*)ipT;
    P->ixT = (const int32_t*)ixT;
    P->valT = vT;
    P->ipX = (const int64_t*)ipX;
    P->ixX = (const int32_t*)ixX;
    P->valX = vX;
    P->st_rec = P->csr_dtype;
  } else {
    // Storage of Z (X itself; signs and 1/Z_scale are applied in n-space).
    if ((e = P->alloc(&P->Xs, storage_bytes(P->storage, ld, n))) != hipSuccess)
      return cleanup(hip_fail(e, "hipMalloc(Z storage)"));
    P->X_rec = P->Xs;
    P->st_rec = P->storage == DWD_FP64 ? DWD_FP64 : DWD_FP32;
    if (P->storage == DWD_BF16) {
      P->X_lowp = (char*)P->Xs + (size_t)ld * n * 4;
    }
  }
  // scalars + y
  double* dscal = nullptr;
  if ((e = P->alloc((void**)&dscal, 64 * 8)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  P->d_scal = dscal;
  if ((e = P->alloc((void**)&P->y, (size_t)n * 8)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = hipMemcpyAsync(P->y, y, (size_t)n * 8, hipMemcpyHostToDevice, st)) != hipSuccess)
    return cleanup(hip_fail(e, "H2D y"));
  for (int i = 0; i < n; ++i) (y[i] > 0.0 ? P->npos : P->nneg) += 1;
  if ((e = P->alloc((void**)&P->e, (size_t)n * 8)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  P->e_ones = false;
  if ((e = P->set_penalty(nullptr)) != hipSuccess) return cleanup(hip_fail(e, "H2D e"));

  // a0: copy + ||X||_F^2
  const int ychunks = (int)std::max<int64_t>(1, std::min<int64_t>(64, ld / 8192));
  const int nfb = 256;  // blocks of the CSR norm
  double* part = nullptr;
  if ((e = P->alloc_tmp((void**)&part, (size_t)std::max(n * ychunks, nfb) * 8)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMalloc(part)"));
  if (csr) {
    e = launch_csr_frob(P->valT, P->csr_dtype, P->nnz, part, nfb, st);
    if (e == hipSuccess) e = launch_sum(part, nfb, dscal, st);
  } else {
    e = launch_frob_copy(Xdev, X->dtype, d, n, P->Xs, P->storage, ld, part, ychunks, st);
    if (e == hipSuccess) e = launch_sum(part, n * ychunks, dscal, st);
  }
  double frob2 = 0.0;
  if (e == hipSuccess) e = hipMemcpyAsync(&frob2, dscal, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  P->free_tmp(part);
  if (Xtmp) {
    P->free_tmp(Xtmp);
    Xtmp = nullptr;
  }
  if (e != hipSuccess) return cleanup(hip_fail(e, "frob/copy"));
  if (!std::isfinite(frob2)) return cleanup(fail(DWD_E_INVALID, "X has non-finite entries"));
  if (!(frob2 > 0.0)) return cleanup(fail(DWD_E_INVALID, "X is all zero"));
  P->zscale = sqrt(sqrt(frob2));  // Z_scale = sqrt(||X||_F)
  if (P->solver == DWD_SOLVER_DIRECT || P->solver == DWD_SOLVER_ITERATIVE) {
    dwd_params pe = *p;
    pe.ell = ell_req;
    if ((s = P->solver == DWD_SOLVER_DIRECT ? setup_direct(P, st) : setup_iterative(P, &pe, st)) !=
        DWD_OK)
      return cleanup(s);
    if (!arena && (e = P->host_objects()) != hipSuccess) return cleanup(hip_fail(e, "host objects"));
    P->setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = P;
    return DWD_OK;
  }

  // a1-a2: Gram G~ = Z~^T Z~ of the streamed image, M = I + G~/mu, M^-1 in
  // place, M^-1 y and y^T M^-1 y.  BF16 storage factors the BF16 image too:
  // the BF16 phase then solves the BF16 problem exactly (its n-space
  // recurrences and ||g|| prediction match the data it streams).
  const size_t nn = (size_t)n * n;
  auto factor = [&](const void* Xsrc, int st_src, double** G, double** Minv, double** my,
                    double* ymy) -> dwd_status {
    hipError_t e2;
    if ((e2 = P->alloc((void**)G, nn * 8)) != hipSuccess) return hip_fail(e2, "hipMalloc(G)");
    if ((e2 = P->alloc((void**)Minv, nn * 8)) != hipSuccess)
      return hip_fail(e2, "hipMalloc(Minv)");
    const int splits = csr ? 1 : gram_splits(ld, n);
    double* Gpart = nullptr;
    if ((e2 = P->alloc_tmp((void**)&Gpart, std::max({nn * splits, nn, spd_inverse_work(n)}) * 8)) !=
        hipSuccess)
      return hip_fail(e2, "hipMalloc(Gram partials)");
    if (csr)
      e2 = launch_csr_gram(P->ipT, P->ixT, P->valT, P->csr_dtype, n, Gpart, st);
    else
      e2 = launch_gram(Xsrc, st_src, ld, n, Gpart, splits, st);
    if (e2 == hipSuccess)
      e2 = launch_gram_finish(Gpart, splits, n, P->y, 1.0 / (P->zscale * P->zscale), P->mu, *G,
                              *Minv, st);
    int* d_status = (int*)(dscal + 8);
    int zero = 0;
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(d_status, &zero, 4, hipMemcpyHostToDevice, st);
    if (e2 == hipSuccess) e2 = spd_inverse_inplace(*Minv, n, Gpart, d_status, st);
    if (e2 == hipSuccess) e2 = P->alloc((void**)my, (size_t)n * 8);
    if (e2 == hipSuccess) e2 = launch_gemv_rows(*Minv, n, P->y, *my, st);
    if (e2 == hipSuccess) e2 = launch_dot(P->y, *my, n, dscal + 1, st);
    double hv[2] = {0, 0};
    int hstat = 0;
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(hv, dscal, 16, hipMemcpyDeviceToHost, st);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(&hstat, d_status, 4, hipMemcpyDeviceToHost, st);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
    if (e2 != hipSuccess) (void)hipStreamSynchronize(st);
    P->free_tmp(Gpart);
    if (e2 != hipSuccess) return hip_fail(e2, "Gram/inverse");
    if (hstat != 0 || !(hv[1] > 0.0) || !std::isfinite(hv[1]))
      return fail(DWD_E_NUMERIC, "factorisation of I + Z~^T Z~/mu failed");
    *ymy = hv[1];
    return DWD_OK;
  };
  if ((s = factor(P->X_rec, P->st_rec, &P->G, &P->Minv, &P->my, &P->ymy)) != DWD_OK)
    return cleanup(s);
  if (P->storage == DWD_BF16 &&
      (s = factor(P->X_lowp, DWD_BF16, &P->G_lp, &P->Minv_lp, &P->my_lp, &P->ymy_lp)) != DWD_OK)
    return cleanup(s);

  // Iteration buffers.
  if ((e = P->alloc_iter_buffers()) != hipSuccess) return cleanup(hip_fail(e, "iteration buffers"));
  if (csr) P->nchunks = 1;  // the sparse Z~^T pass writes one chunk
  if (!arena && (e = P->host_objects()) != hipSuccess) return cleanup(hip_fail(e, "host objects"));
  auto t1 = std::chrono::steady_clock::now();
  P->setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  *out = P;
  return DWD_OK;
}

hipError_t Problem::alloc_iter_buffers() {
  const int n_ = n;
  hipError_t e;
  // 31 n-vectors: 24 named, and the pass operands (4 per column)
  double* nb = nullptr;
  if ((e = alloc((void**)&nb, (size_t)n_ * 8 * 31)) != hipSuccess) return e;
  double* q = nb;
  auto take = [&](double*& dst) {
    dst = q;
    q += n_;
  };
  take(ip.r); take(ip.xi); take(ip.alpha); take(ip.Pu); take(ip.Prho); take(ip.t); take(ip.x);
  take(ip.f); take(ip.s); take(ip.v); take(ip.dr); take(ip.hG); take(ip.rn); take(ip.s1);
  take(ip.v1); take(ip.xi0); take(ip.xi1); take(ip.al0); take(ip.al1);
  take(ip.au); take(ip.arho); take(ip.aw); take(ip.au_n); take(ip.arho_n);
  ip.stg = q;  // 4 n
  q += 4 * (size_t)n_;
  double* db = nullptr;
  if ((e = alloc((void**)&db, (size_t)ld * 8 * 3)) != hipSuccess) return e;
  ip.u = db;
  ip.rho = db + ld;
  ip.w = db + 2 * ld;
  nchunks = (int)(ld / kLdAlign);
  if ((e = alloc((void**)&ip.partT, (size_t)nchunks * 2 * n_ * 8)) != hipSuccess) return e;
  // partials of the pass (FP64 has the most blocks) or of the representer step
  const int npb = std::max({pass2_blocks(DWD_FP64, ld), csr_pass_blocks(ld), ngemv_blocks(n_), 1});
  if ((e = alloc((void**)&ip.part_g, (size_t)npb * NP2 * 8)) != hipSuccess) return e;
  ip.pg_ld = npb;
  if ((e = alloc((void**)&ip.part_n1, (size_t)ngemv_blocks(n_) * 8)) != hipSuccess) return e;
  if ((e = alloc((void**)&ip.part_it, (size_t)ngemv_blocks(n_) * 8)) != hipSuccess) return e;
  if ((e = alloc((void**)&ip.part_c, (size_t)ngemv_blocks(n_) * NPC * 8)) != hipSuccess) return e;
  if ((e = alloc((void**)&ip.sc, sizeof(Scal))) != hipSuccess) return e;
  ip.y = y;
  ip.e = this->e;
  ip.my = my;
  ip.Minv = Minv;
  ip.G = G;
  ip_lp = ip;
  if (G_lp) {
    ip_lp.G = G_lp;
    ip_lp.Minv = Minv_lp;
    ip_lp.my = my_lp;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Solve.
// ---------------------------------------------------------------------------
static int qkind_of(double q) {
  if (q == 1.0) return 1;
  if (q == 2.0) return 2;
  if (q == 4.0) return 4;
  if (q == 0.5) return 5;
  return 0;
}

hipError_t Problem::set_penalty(const double* eh) {
  if (!eh && e_ones) return hipSuccess;
  std::vector<double> ones;
  if (!eh) {
    ones.assign(n, 1.0);
    eh = ones.data();
  }
  // synchronous: eh is borrowed for the duration of the call only
  const hipError_t r = hipMemcpy(e, eh, (size_t)n * 8, hipMemcpyHostToDevice);
  if (r == hipSuccess) e_ones = !ones.empty();
  return r;
}

// The iteration form (dwd_params.representer; 2 = by the bytes an iteration
// moves): the representer iteration reads G~ once more (8 n^2 bytes) instead
// of streaming Z (in the storage type of its main phase) and the five FP64
// d-vectors of Steps 2-3.  Only the SMW set-up has the representer form.
int choose_representer(const Problem* P, int req) {
  if (P->solver != DWD_SOLVER_SMW) return 0;
  if (req != 2) return req ? 1 : 0;
  const double n = (double)P->n, ld = (double)P->ld;
  double zbytes;
  if (P->layout == DWD_CSR)
    zbytes = (double)P->nnz * (4.0 + (P->csr_dtype == DWD_FP64 ? 8.0 : 4.0));
  else
    zbytes = ld * n * (P->storage == DWD_FP64 ? 8.0 : (P->storage == DWD_BF16 ? 2.0 : 4.0));
  return 8.0 * n * n < zbytes + 5.0 * 8.0 * ld ? 1 : 0;
}

Consts make_consts(const Problem* P, const dwd_params* p) {
  Consts c;
  c.d = P->d;
  c.ld = P->ld;
  c.n = P->n;
  c.max_iter = p->max_iter;
  c.C = p->C;
  c.q = p->q;
  c.tau = p->tau;
  c.mu = P->mu;
  c.sqmu = sqrt(P->mu);
  c.R = P->zscale;
  c.inv_zs = 1.0 / P->zscale;
  c.tol = p->tol;
  // ||Z~||_F = ||X||_F / Z_scale = Z_scale
  c.eps_c = p->eps_c < 0.0 ? 1.0 / P->zscale : p->eps_c;
  c.ymy = P->ymy;
  c.kappa = (p->q + 1.0) / p->q * pow(p->q, 1.0 / (p->q + 1.0));
  c.opC = 1.0 + p->C;
  c.c1 = p->q * (p->q + 2.0);
  c.c2 = p->q * (p->q + 1.0);
  c.qexp = p->q / (p->q + 1.0);
  c.rho_residual = p->rho_residual ? 1 : 0;
  c.qkind = qkind_of(p->q);
  c.sigma_every = p->sigma_every;
  c.representer = choose_representer(P, p->representer);
  // Section 4.5: tau_+- = (n_+- / K)^(1/(1+q)), K = n / log(n); the loss term
  // of class +1 carries tau_-/max(tau_+, tau_-), of class -1
  // tau_+/max(tau_+, tau_-), raised to q.
  c.wpos = c.wneg = 1.0;
  if (p->class_weights) {
    const double K = (double)P->n / log((double)P->n);
    const double tp = pow((double)P->npos / K, 1.0 / (1.0 + p->q));
    const double tm = pow((double)P->nneg / K, 1.0 / (1.0 + p->q));
    const double m = std::max(tp, tm);
    c.wpos = pow(tm / m, p->q);
    c.wneg = pow(tp / m, p->q);
  }
  c.wdpos = pow(c.wpos, 1.0 / (p->q + 1.0));
  c.wdneg = pow(c.wneg, 1.0 / (p->q + 1.0));
  return c;
}

Consts lowp_consts(const Problem* P, const dwd_params* p) {
  Consts c = make_consts(P, p);
  c.ymy = P->ymy_lp;
  c.tol = p->lowp_tol > 0.0 ? p->lowp_tol : std::min(0.5, 30.0 * p->tol);
  return c;
}

double default_sigma0(const dwd_params* p, int n) {
  return p->sigma0 > 0.0 ? p->sigma0 : pow(std::min(10.0 * p->C, (double)n), p->q);
}

// Queue one iteration of Algorithm 1 for problem P on its stream.
hipError_t Problem::queue_iteration(const Consts& c, const void* Xit, int st_it, bool fresh,
                                    bool profile, int k) {
  hipError_t e;
  const hipStream_t s = stream;
  // The BF16 phase iterates on the BF16 image with that image's own factor.
  const IterPtrs& I = st_it == DWD_BF16 ? ip_lp : ip;
  if (c.representer) {
    // Representer iteration: no pass over Z.  A fresh start anchors
    // Z~^T u = G~ au and Z~^T rho = G~ arho exactly.
    // (Otherwise t and x were formed by the previous tail kernel.)
    if (fresh) {
      if ((e = launch_ngemv(n, I.G, I.au, I.Pu, I.G, I.arho, I.Prho, nullptr, nullptr, I.sc, s)) !=
          hipSuccess)
        return e;
      if ((e = launch_rhs(c, I, nchunks, 0, s)) != hipSuccess) return e;
    }
    if ((e = launch_step1ab(c, I, s)) != hipSuccess) return e;
    if ((e = launch_step1c_rows(c, I, s)) != hipSuccess) return e;
    if ((e = launch_rep_step(c, I, s)) != hipSuccess) return e;
    return launch_tail(c, I, ngemv_blocks(n), s);
  }
  if (fresh) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile) {
      e0 = next_event(1, k);
      e1 = next_event(1, k);
      (void)hipEventRecord(e0, s);
    }
    if (layout == DWD_CSR)
      e = launch_csr_gemvT(ipT, ixT, valT, csr_dtype, n, I.u, I.rho, I.partT, I.sc, s);
    else
      e = launch_gemvT(Xit, st_it, ld, n, I.u, I.rho, I.partT, I.sc, s);
    if (e != hipSuccess) return e;
    if (profile) (void)hipEventRecord(e1, s);
  }
  // Without a fresh pass, t and x were formed by the previous tail kernel.
  if (fresh && (e = launch_rhs(c, I, nchunks, 1, s)) != hipSuccess) return e;
  if ((e = launch_step1ab(c, I, s)) != hipSuccess) return e;
  if ((e = launch_step1c_rows(c, I, s)) != hipSuccess) return e;
  {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile) {
      e0 = next_event(0, k);
      e1 = next_event(0, k);
      (void)hipEventRecord(e0, s);
    }
    if (layout == DWD_CSR)
      e = launch_csr_pass(ipX, ixX, valX, csr_dtype, d, c, I, s);
    else
      e = launch_pass2(Xit, st_it, c, I, s);
    if (e != hipSuccess) return e;
    if (profile) (void)hipEventRecord(e1, s);
  }
  const int nblk = layout == DWD_CSR ? csr_pass_blocks(ld) : pass2_blocks(st_it, ld);
  return launch_tail(c, I, nblk, s);
}

hipError_t Problem::expand() {
  Consts c{};
  c.d = d;
  c.ld = ld;
  c.n = n;
  c.inv_zs = 1.0 / zscale;
  if (layout == DWD_CSR) return launch_csr_expand(ipX, ixX, valX, csr_dtype, d, c, ip, stream);
  return launch_expand(X_rec, st_rec, c, ip, stream);
}

hipError_t Problem::dres(const Consts& c, const double* alpha, const double* rho, double* part,
                        int* nblk) {
  if (layout == DWD_CSR) {
    *nblk = csr_pass_blocks(ld);
    return launch_csr_dres(ipX, ixX, valX, csr_dtype, d, c, alpha, y, rho, part, stream);
  }
  *nblk = dres_blocks(st_rec, ld);
  return launch_dres(X_rec, st_rec, c, alpha, y, rho, part, stream);
}

hipError_t Problem::queue_check(const Consts& c) {
  hipError_t e;
  if (c.representer && (e = expand()) != hipSuccess) return e;
  if ((e = pass_T(ip.w, ip.rho, nullptr)) != hipSuccess) return e;
  int nblk = 0;
  if ((e = dres(c, ip.alpha, ip.rho, ip.part_g, &nblk)) != hipSuccess) return e;
  return launch_check(c, ip, nchunks, ip.part_g, nblk, stream);
}

hipError_t Problem::pass_T(const double* v1, const double* v2, const Scal* sc) {
  if (layout == DWD_CSR)
    return launch_csr_gemvT(ipT, ixT, valT, csr_dtype, n, v1, v2, ip.partT, sc, stream);
  return launch_gemvT(X_rec, st_rec, ld, n, v1, v2, ip.partT, sc, stream);
}

hipEvent_t Problem::next_event(int kind, int k) {
  if (ev_used >= (int)ev_pool.size()) {
    // timing-only events: no system-scope fence (cache writeback and
    // invalidate) at record, which would both inflate the timed interval and
    // flush what the following kernels reuse
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    ev_pool.push_back(ev);
    ev_kind.push_back(kind);
    ev_iter.push_back(k);
    ev_live.push_back(1);
  }
  ev_kind[ev_used] = kind;
  ev_iter[ev_used] = k;
  ev_live[ev_used] = 1;
  return ev_pool[ev_used++];
}

// Run iterations until the device stop flag is set.  Returns the number of
// iterations queued.
hipError_t Problem::run_loop(const Consts& c, const void* Xit, int st_it, int resync,
                             int check_every, bool profile, int k_start) {
  const int chunk = std::max(1, check_every);
  const int ev_first = ev_used;
  int queued = 0;
  int pending = -1;  // index of the chunk last queued before this one
  // The tail kernel sets the pinned word when it sets the stop flag; every
  // earlier launch on the stream is done (and its writes visible) once a
  // chunk's event has completed.  Nothing writes the word while the host
  // clears it: the stream is idle between solve phases.
  volatile int32_t* hd = (volatile int32_t*)h_flags + kHostDoneWord;
  *hd = 0;
  hipError_t e;
  for (int cidx = 0;; ++cidx) {
    for (int j = 0; j < chunk && k_start + queued < c.max_iter; ++j, ++queued) {
      const int k = k_start + queued;
      const bool fresh = (queued == 0) || (resync > 0 && (k % resync) == 0);
      if ((e = queue_iteration(c, Xit, st_it, fresh, profile, k)) != hipSuccess) return e;
    }
    const int slot = cidx & 1;
    if ((e = hipEventRecord(ev_chunk[slot], stream)) != hipSuccess) return e;
    if (k_start + queued >= c.max_iter) break;
    if (pending >= 0) {
      if ((e = hipEventSynchronize(ev_chunk[pending & 1])) != hipSuccess) return e;
      if (*hd) break;
    }
    pending = cidx;
  }
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  if (profile) {
    // launches queued past the iteration that set the stop flag returned at once
    int32_t kdone = 0;
    if ((e = hipMemcpy(&kdone, &ip.sc->k, 4, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    for (int j = ev_first; j < ev_used; ++j)
      if (ev_iter[j] >= kdone) ev_live[j] = 0;
  }
  return hipSuccess;
}

__global__ void k_reset_done(Scal* sc) {
  sc->done = 0;
  sc->converged = 0;
}

dwd_status solve_problem(Problem* P, const dwd_params* p, double* w, dwd_info* info,
                         double* alpha, double* r, double* xi, double* u, double* rho) {
  dwd_status s;
  if (!P) return fail(DWD_E_INVALID, "problem is NULL");
  if (P->solver == DWD_SOLVER_DIRECT) return solve_direct(P, p, w, info, alpha, r, xi, u, rho);
  if (P->solver == DWD_SOLVER_ITERATIVE)
    return solve_iterative(P, p, w, info, alpha, r, xi, u, rho);
  if ((s = validate_params(p, true)) != DWD_OK) return s;
  if ((s = validate_penalty(p, P->n)) != DWD_OK) return s;
  HIP_TRY(hipSetDevice(P->device));
  const hipStream_t st = P->stream;
  HIP_TRY(hipStreamSynchronize(st));  // (e may still be read by a previous solve)
  HIP_TRY(P->set_penalty(p->e));
  HIP_TRY(hipEventRecord(P->ev_a, st));
  Consts c = make_consts(P, p);
  if (!iter_ptrs_ok(P->ip)) return fail(DWD_E_DEVICE, "iteration buffers are not allocated");
  const double sigma0 = default_sigma0(p, P->n);
  HIP_TRY(launch_init(c, P->ip, sigma0, st));
  P->ev_used = 0;
  const bool profile = p->profile != 0;
  const int check_every = p->check_every > 0 ? p->check_every : 8;
  int iters_lowp = 0;
  if (P->storage == DWD_BF16 && !c.representer) {
    // Phase 1 on the BF16 image, to the looser tolerance.
    const Consts c1 = lowp_consts(P, p);
    HIP_TRY(P->run_loop(c1, P->X_lowp, DWD_BF16, p->resync, check_every, profile, 0));
    Scal hs;
    HIP_TRY(hipMemcpy(&hs, P->ip.sc, sizeof(Scal), hipMemcpyDeviceToHost));
    iters_lowp = hs.k;
    if (p->refine && hs.k < p->max_iter) {
      hipLaunchKernelGGL(k_reset_done, dim3(1), dim3(1), 0, st, P->ip.sc);
      HIP_TRY(hipGetLastError());
      HIP_TRY(P->run_loop(c, P->X_rec, P->st_rec, p->resync, check_every, profile, hs.k));
    }
  } else {
    HIP_TRY(P->run_loop(c, P->X_rec, P->st_rec, p->resync, check_every, profile, 0));
  }
  // Final check over the data of record.  If the loop stopped on its
  // in-loop residuals but the explicit FP64 check misses the tolerance
  // (rounding drift of the n-space recurrences), resume with a fresh pass
  // every iteration and a tighter in-loop target.  The solve counts as
  // converged only when the check itself meets the tolerance.
  Scal hs;
  int resumed = 0;
  double chk = 0.0;
  for (;;) {
    HIP_TRY(P->queue_check(c));
    HIP_TRY(hipMemcpyAsync(&hs, P->ip.sc, sizeof(Scal), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    chk = std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]);
    // (BF16 storage without refinement: the check only reports the residual
    // of the BF16 solution against the data of record.)
    const bool no_refine = P->storage == DWD_BF16 && !p->refine && !c.representer;
    if (!hs.converged || chk < p->tol || resumed >= kMaxResume || hs.k >= p->max_iter ||
        no_refine)
      break;
    ++resumed;
    c.tol = resume_tol(c.tol, p->tol, chk);
    hipLaunchKernelGGL(k_reset_done, dim3(1), dim3(1), 0, st, P->ip.sc);
    HIP_TRY(hipGetLastError());
    HIP_TRY(P->run_loop(c, P->X_rec, P->st_rec, 1, check_every, profile, hs.k));
  }
  const int conv = hs.converged && chk < p->tol ? 1 : 0;
  HIP_TRY(hipEventRecord(P->ev_b, st));
  std::vector<double> hw;
  const bool want_w = w || u || rho;
  if (want_w) hw.resize(P->ld);
  if (w) HIP_TRY(hipMemcpyAsync(hw.data(), P->ip.w, P->d * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (w)
    for (int64_t k = 0; k < P->d; ++k) w[k] = hw[k] / P->zscale;
  if (u) {
    HIP_TRY(hipMemcpy(u, P->ip.u, P->d * 8, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < P->d; ++k) u[k] /= P->zscale;
  }
  if (rho) HIP_TRY(hipMemcpy(rho, P->ip.rho, P->d * 8, hipMemcpyDeviceToHost));
  if (alpha) HIP_TRY(hipMemcpy(alpha, P->ip.alpha, P->n * 8, hipMemcpyDeviceToHost));
  if (r) HIP_TRY(hipMemcpy(r, P->ip.r, P->n * 8, hipMemcpyDeviceToHost));
  if (xi) HIP_TRY(hipMemcpy(xi, P->ip.xi, P->n * 8, hipMemcpyDeviceToHost));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, P->ev_a, P->ev_b));
  double stream_ms[2] = {0.0, 0.0};
  int launches[2] = {0, 0};
  if (profile) {
    for (int j = 0; j + 1 < P->ev_used; j += 2) {
      float t = 0.0f;
      if (!P->ev_live[j]) continue;
      if (hipEventElapsedTime(&t, P->ev_pool[j], P->ev_pool[j + 1]) == hipSuccess) {
        const int kd = P->ev_kind[j] ? 1 : 0;
        stream_ms[kd] += t;
        ++launches[kd];
      }
    }
  }
  if (info) {
    memset(info, 0, sizeof(*info));
    info->beta = hs.beta;
    info->primal_obj = hs.eta[E_PRIM];
    info->dual_obj = hs.eta[E_DUAL];
    info->eta_p = hs.eta[E_P];
    info->eta_d = hs.eta[E_D];
    info->eta_c = hs.eta[E_C];
    info->eta_gap = hs.eta[E_GAP];
    info->eta_p_check = hs.eta[E_PCHK];
    info->eta_d_check = hs.eta[E_DCHK];
    info->kkt_check = std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]);
    info->sigma = hs.sigma;
    info->iters = hs.k;
    info->n_double = hs.n_double;
    info->newton_max = hs.newton_max;
    info->converged = conv;
    info->iters_lowp = iters_lowp;
    info->setup_ms = P->setup_ms;
    info->solve_ms = ms;
    info->stream_ms = stream_ms[0];
    info->stream_launches = launches[0];
    info->streamT_ms = stream_ms[1];
    info->streamT_launches = launches[1];
    info->resumed = resumed;
    info->representer = c.representer;
    info->status = conv ? DWD_OK : DWD_NOT_CONVERGED;
  }
  return conv ? DWD_OK : DWD_NOT_CONVERGED;
}

// Section 4.1: C = 10^(q+1) max{1, 10^(q-1) log(n) max{1000, d}^(1/3) / dist^(q+1)}
// with dist the median between-class Euclidean distance, selected exactly on
// the device from G~ (eight radix steps of 8 bits per order statistic).
dwd_status suggest_C(Problem* P, double q, double* C) {
  if (!(q > 0.0) || !std::isfinite(q)) return fail(DWD_E_INVALID, "q must be > 0");
  if (P->solver != DWD_SOLVER_SMW)
    return fail(DWD_E_INVALID, "dwd_suggest_C needs the n x n Gram matrix of the SMW set-up");
  HIP_TRY(hipSetDevice(P->device));
  const hipStream_t st = P->stream;
  const int n = P->n;
  std::vector<double> hy(n);
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(hy.data(), P->y, (size_t)n * 8, hipMemcpyDeviceToHost));
  std::vector<int> idx;
  idx.reserve(n);
  for (int i = 0; i < n; ++i)
    if (hy[i] > 0.0) idx.push_back(i);
  const int npos = (int)idx.size();
  for (int i = 0; i < n; ++i)
    if (!(hy[i] > 0.0)) idx.push_back(i);
  const int nneg = n - npos;
  int* didx = nullptr;
  unsigned int* hist = nullptr;
  HIP_TRY(hipMalloc((void**)&didx, (size_t)n * 4));
  hipError_t e = hipMalloc((void**)&hist, 256 * 4);
  if (e == hipSuccess) e = hipMemcpy(didx, idx.data(), (size_t)n * 4, hipMemcpyHostToDevice);
  const int64_t total = (int64_t)npos * nneg;
  // k-th smallest key (0-based) by radix selection from the top digit down
  auto select = [&](int64_t k, unsigned long long* key) -> hipError_t {
    unsigned long long prefix = 0;
    unsigned int hh[256];
    for (int shift = 56; shift >= 0; shift -= 8) {
      hipError_t r;
      if ((r = hipMemsetAsync(hist, 0, 256 * 4, st)) != hipSuccess) return r;
      if ((r = launch_pair_hist(P->G, n, didx, npos, didx + npos, nneg, prefix, shift, hist,
                                st)) != hipSuccess)
        return r;
      if ((r = hipMemcpyAsync(hh, hist, 256 * 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return r;
      if ((r = hipStreamSynchronize(st)) != hipSuccess) return r;
      int64_t cum = 0;
      int b = 0;
      for (; b < 255 && k >= cum + (int64_t)hh[b]; ++b) cum += hh[b];
      k -= cum;
      prefix |= (unsigned long long)b << shift;
    }
    *key = prefix;
    return hipSuccess;
  };
  unsigned long long k1 = 0, k2 = 0;
  if (e == hipSuccess) e = select((total - 1) / 2, &k1);
  if (e == hipSuccess) e = (total % 2) ? (k2 = k1, hipSuccess) : select(total / 2, &k2);
  (void)hipFree(didx);
  (void)hipFree(hist);
  if (e != hipSuccess) return hip_fail(e, "suggest_C");
  return C_from_median_keys(P, q, k1, k2, C);
}

dwd_status C_from_median_keys(const Problem* P, double q, unsigned long long k1,
                              unsigned long long k2, double* C) {
  double v1, v2;
  memcpy(&v1, &k1, 8);
  memcpy(&v2, &k2, 8);
  const double dist = 0.5 * (P->zscale * sqrt(v1) + P->zscale * sqrt(v2));
  if (!(dist > 0.0)) return fail(DWD_E_INVALID, "the median between-class distance is zero");
  const double t = pow(10.0, q - 1.0) * log((double)P->n) *
                   cbrt(std::max(1000.0, (double)P->d)) / pow(dist, q + 1.0);
  *C = pow(10.0, q + 1.0) * std::max(1.0, t);
  return DWD_OK;
}

}  // namespace dwd

// ---------------------------------------------------------------------------
// extern "C"
// ---------------------------------------------------------------------------
using namespace dwd;

struct dwd_problem_s {
  Problem* P;
};

extern "C" {

void dwd_default_params(dwd_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->C = 1.0;
  p->q = 1.0;
  p->tol = 1e-5;
  p->max_iter = 2000;
  p->storage = DWD_FP32;
  p->tau = 1.618;
  p->mu = 1.0;
  p->sigma0 = 0.0;
  p->eps_c = -1.0;
  p->rho_residual = 1;
  p->resync = 0;
  p->check_every = 8;
  p->refine = 1;
  p->lowp_tol = 0.0;
  p->profile = 0;
  p->batch_fp32 = 1;
  p->batch_tile = 0;
  p->graph = 1;
  p->sigma_every = 2;
  p->psqmr_max = 50;
}

dwd_status dwd_setup(const dwd_matrix* X, const double* y, const dwd_params* p, void* stream,
                     dwd_problem* out) {
  if (!out) return fail(DWD_E_INVALID, "out is NULL");
  *out = nullptr;
  try {
    Problem* P = nullptr;
    dwd_status s = setup_problem(X, y, p, (hipStream_t)stream, &P);
    if (s != DWD_OK) return s;
    *out = new dwd_problem_s{P};
    return DWD_OK;
  } catch (const std::bad_alloc&) {
    return fail(DWD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(DWD_E_DEVICE, "unexpected exception in dwd_setup");
  }
}

dwd_status dwd_solve(dwd_problem H, const dwd_params* p, double* w, dwd_info* info,
                     double* alpha, double* r, double* xi, double* u, double* rho) {
  if (!H) return fail(DWD_E_INVALID, "problem is NULL");
  try {
    return solve_problem(H->P, p, w, info, alpha, r, xi, u, rho);
  } catch (const std::bad_alloc&) {
    return fail(DWD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(DWD_E_DEVICE, "unexpected exception in dwd_solve");
  }
}

dwd_status dwd_solve_batch(dwd_problem H, int32_t B, const dwd_params* p, double* W,
                           dwd_info* info) {
  if (!H) return fail(DWD_E_INVALID, "problem is NULL");
  if (B < 1 || !p) return fail(DWD_E_INVALID, "B must be >= 1 and p non-NULL");
  try {
    return solve_batch(H->P, B, p, W, info);
  } catch (const std::bad_alloc&) {
    return fail(DWD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(DWD_E_DEVICE, "unexpected exception in dwd_solve_batch");
  }
}

void dwd_free(dwd_problem H) {
  if (!H) return;
  if (H->P) {
    (void)hipSetDevice(H->P->device);
    (void)hipStreamSynchronize(H->P->stream);
    release(H->P);
    delete H->P;
  }
  delete H;
}

dwd_status dwd_suggest_C(dwd_problem H, double q, double* C) {
  if (!H || !H->P || !C) return fail(DWD_E_INVALID, "NULL argument");
  try {
    return suggest_C(H->P, q, C);
  } catch (const std::bad_alloc&) {
    return fail(DWD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(DWD_E_DEVICE, "unexpected exception in dwd_suggest_C");
  }
}

dwd_status dwd_suggest_C_noalloc(dwd_problem H, double q, double* C) {
  if (!H || !H->P || !C) return fail(DWD_E_INVALID, "NULL argument");
  try {
    return suggest_C_static(H->P, q, C);
  } catch (...) {
    return fail(DWD_E_DEVICE, "unexpected exception in dwd_suggest_C_noalloc");
  }
}

dwd_status dwd_inspect(dwd_problem H, const char* what, double* out, int64_t count) {
  if (!H || !H->P || !what || !out) return fail(DWD_E_INVALID, "NULL argument");
  Problem* P = H->P;
  const std::string w(what);
  const int64_t nn = (int64_t)P->n * P->n;
  if (w == "psqmr_count") {
    if (count != 1) return fail(DWD_E_INVALID, "count must be 1");
    out[0] = (double)P->psqmr_log.size();
    return DWD_OK;
  }
  if (w == "psqmr_steps") {
    if (count != (int64_t)P->psqmr_log.size()) return fail(DWD_E_INVALID, "wrong count");
    for (int64_t j = 0; j < count; ++j) out[j] = (double)P->psqmr_log[j];
    return DWD_OK;
  }
  if (w == "zscale" || w == "ymy" || w == "solver" || w == "ell") {
    if (count != 1) return fail(DWD_E_INVALID, "count must be 1");
    out[0] = w == "zscale" ? P->zscale
                           : (w == "ymy" ? P->ymy
                                         : (w == "solver" ? (double)P->solver : (double)P->ipt.ell));
    return DWD_OK;
  }
  const double* src = nullptr;
  int64_t m = 0;
  const bool direct = P->solver == DWD_SOLVER_DIRECT;
  if (w == "G" && !direct) { src = P->G; m = nn; }
  else if (w == "Minv" && !direct) { src = P->Minv; m = nn; }
  else if (w == "my" && !direct) { src = P->my; m = P->n; }
  else if (w == "Ainv" && direct) { src = P->Ainv; m = (P->d + 1) * (P->d + 1); }
  else if (w == "lam" && P->solver == DWD_SOLVER_ITERATIVE) { src = P->ipt.lam; m = P->ipt.ell; }
  else return fail(DWD_E_INVALID, "unknown quantity for this problem's solver");
  if (count != m) return fail(DWD_E_INVALID, "wrong count");
  hipError_t e = hipSetDevice(P->device);
  if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
  if (e == hipSuccess) e = hipMemcpy(out, src, (size_t)m * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "dwd_inspect");
  return DWD_OK;
}

int64_t dwd_footprint(const dwd_matrix* X, const dwd_params* p) {
  if (!X || !p || X->d < 1 || X->n < 1) return 0;
  const int sv = resolve_solver(p, X);
  if (sv == DWD_SOLVER_DIRECT) return direct_footprint(X->d, (int)X->n, p->storage);
  if (sv == DWD_SOLVER_ITERATIVE)
    return iterative_footprint(X->d, (int)X->n, p->storage, p->ell > 0 ? p->ell : 10);
  return problem_footprint(X->d, (int)X->n, p->storage, X->layout, X->nnz);
}

const char* dwd_status_str(dwd_status s) {
  switch (s) {
    case DWD_OK: return "DWD_OK";
    case DWD_NOT_CONVERGED: return "DWD_NOT_CONVERGED";
    case DWD_E_INVALID: return "DWD_E_INVALID";
    case DWD_E_NOMEM: return "DWD_E_NOMEM";
    case DWD_E_DEVICE: return "DWD_E_DEVICE";
    case DWD_E_NUMERIC: return "DWD_E_NUMERIC";
    case DWD_E_BUSY: return "DWD_E_BUSY";
  }
  return "unknown dwd_status";
}

const char* dwd_last_error(void) { return g_err.c_str(); }

const char* dwd_version(void) { return "libdwd 0.1 (gfx950)"; }

}  // extern "C"
