// dwd_serve: replay a trace of solve requests in real time with continuous
// batching.  A request is admitted, first come first served, as soon as a
// slot is free and its device footprint fits what is left of the HBM budget;
// it is set up on a stream of its own and then stepped in chunks of
// iterations, interleaved by the host with every other admitted problem, so
// that requests which arrive while others run share the GPU with them.  Each
// problem runs exactly the kernel sequence of dwd_solve (the chunking only
// decides when the host looks at its stop flag), so its result does not
// depend on the mix.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <vector>

#include "dwd_solver.h"

namespace dwd {

__global__ void k_serve_reset(Scal* sc) {
  sc->done = 0;
  sc->converged = 0;
}

namespace {

enum Phase { MAIN = 0, REFINE = 1, CHECK = 2, RESUME = 3, DONE = 4 };

struct Slot {
  int req = -1;
  Problem* P = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  Scal* hs = nullptr;        // pinned copy of the device scalars
  Consts c{}, c_lowp{};
  dwd_params prm{};
  Phase phase = MAIN;
  int queued = 0;            // iterations queued in the current phase
  int k_base = 0;            // device iteration count when the phase started
  bool in_flight = false;
  int resumed = 0;
  int iters_lowp = 0;
  int64_t footprint = 0;
  double t_admit = 0.0;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void destroy_slot(Slot& s) {
  if (s.P) {
    (void)hipStreamSynchronize(s.stream);
    for (void* q : s.P->allocs) (void)hipFree(q);
    if (s.P->h_flags) (void)hipHostFree(s.P->h_flags);
    for (auto& e : s.P->ev_pool) (void)hipEventDestroy(e);
    if (s.P->ev_a) (void)hipEventDestroy(s.P->ev_a);
    if (s.P->ev_b) (void)hipEventDestroy(s.P->ev_b);
    for (auto& e : s.P->ev_chunk)
      if (e) (void)hipEventDestroy(e);
    delete s.P;
    s.P = nullptr;
  }
  if (s.ev) (void)hipEventDestroy(s.ev);
  if (s.hs) (void)hipHostFree(s.hs);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s.ev = nullptr;
  s.hs = nullptr;
  s.stream = nullptr;
}

// Queue up to `chunk` iterations of the current phase and the flag copy.
hipError_t queue_chunk(Slot& s, int chunk) {
  Problem* P = s.P;
  if (P->solver == DWD_SOLVER_DIRECT) {
    // direct branch: one phase; its residuals come from explicit passes
    hipError_t e;
    for (int j = 0; j < chunk && s.k_base + s.queued < s.prm.max_iter; ++j, ++s.queued)
      if ((e = queue_direct_iteration(P, s.c, s.stream)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(s.hs, P->dp.sc, sizeof(Scal), hipMemcpyDeviceToHost, s.stream)) !=
        hipSuccess)
      return e;
    if ((e = hipEventRecord(s.ev, s.stream)) != hipSuccess) return e;
    s.in_flight = true;
    return hipSuccess;
  }
  const bool lowp = (s.phase == MAIN && P->storage == DWD_BF16 && !s.c.representer);
  const Consts& c = lowp ? s.c_lowp : s.c;
  const void* X = lowp ? P->X_lowp : P->X_rec;
  const int st_it = lowp ? DWD_BF16 : P->st_rec;
  const int resync = s.phase == RESUME ? 1 : s.prm.resync;
  hipError_t e;
  for (int j = 0; j < chunk && s.k_base + s.queued < s.prm.max_iter; ++j, ++s.queued) {
    const int k = s.k_base + s.queued;
    const bool fresh = (s.queued == 0) || (resync > 0 && (k % resync) == 0);
    if ((e = P->queue_iteration(c, X, st_it, fresh, false, k)) != hipSuccess) return e;
  }
  if ((e = hipMemcpyAsync(s.hs, P->ip.sc, sizeof(Scal), hipMemcpyDeviceToHost, s.stream)) !=
      hipSuccess)
    return e;
  if ((e = hipEventRecord(s.ev, s.stream)) != hipSuccess) return e;
  s.in_flight = true;
  return hipSuccess;
}

hipError_t queue_check(Slot& s) {
  Problem* P = s.P;
  hipError_t e;
  if ((e = P->queue_check(s.c)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(s.hs, P->ip.sc, sizeof(Scal), hipMemcpyDeviceToHost, s.stream)) !=
      hipSuccess)
    return e;
  if ((e = hipEventRecord(s.ev, s.stream)) != hipSuccess) return e;
  s.in_flight = true;
  return hipSuccess;
}

hipError_t start_phase(Slot& s, Phase ph) {
  s.phase = ph;
  s.queued = 0;
  s.k_base = s.hs->k;
  hipLaunchKernelGGL(k_serve_reset, dim3(1), dim3(1), 0, s.stream, s.P->ip.sc);
  return hipGetLastError();
}

// Advance a slot whose last queued work has completed.  Returns DONE when the
// request is finished (outputs are then written).
hipError_t advance(Slot& s, int chunk) {
  const Scal& hs = *s.hs;
  switch (s.phase) {
    case MAIN:
      if (s.queued > 0 && (hs.done || s.k_base + s.queued >= s.prm.max_iter)) {
        if (s.P->solver == DWD_SOLVER_DIRECT) {
          s.phase = DONE;
          return hipSuccess;
        }
        const bool bf16 = s.P->storage == DWD_BF16 && !s.c.representer;
        if (bf16) s.iters_lowp = hs.k;
        if (bf16 && s.prm.refine && hs.k < s.prm.max_iter) {
          hipError_t e = start_phase(s, REFINE);
          if (e != hipSuccess) return e;
          return queue_chunk(s, chunk);
        }
        s.phase = CHECK;
        return queue_check(s);
      }
      return queue_chunk(s, chunk);
    case REFINE:
    case RESUME:
      if (s.queued > 0 && (hs.done || s.k_base + s.queued >= s.prm.max_iter)) {
        s.phase = CHECK;
        return queue_check(s);
      }
      return queue_chunk(s, chunk);
    case CHECK: {
      const double chk = std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]);
      const bool no_refine = s.P->storage == DWD_BF16 && !s.prm.refine && !s.c.representer;
      if (hs.converged && chk >= s.prm.tol && s.resumed < 2 && hs.k < s.prm.max_iter &&
          !no_refine) {
        ++s.resumed;
        hipError_t e = start_phase(s, RESUME);
        if (e != hipSuccess) return e;
        return queue_chunk(s, chunk);
      }
      s.phase = DONE;
      return hipSuccess;
    }
    default:
      return hipSuccess;
  }
}

void fill_info(const Slot& s, dwd_info* info) {
  const Scal& hs = *s.hs;
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
  info->converged = hs.converged;
  info->iters_lowp = s.iters_lowp;
  info->resumed = s.resumed;
  info->setup_ms = s.P->setup_ms;
  info->status = hs.converged ? DWD_OK : DWD_NOT_CONVERGED;
}

}  // namespace

dwd_status serve(const dwd_request* reqs, int nreq, const dwd_serve_opts* opts,
                 dwd_response* out) {
  if (nreq < 0 || (nreq > 0 && (!reqs || !out))) return fail(DWD_E_INVALID, "bad request array");
  for (int i = 1; i < nreq; ++i)
    if (reqs[i].t_arrival < reqs[i - 1].t_arrival)
      return fail(DWD_E_INVALID, "requests must be sorted by t_arrival");
  for (int i = 0; i < nreq; ++i) {
    dwd_status s = validate_params(&reqs[i].params, true);
    if (s == DWD_OK) s = validate_penalty(&reqs[i].params, reqs[i].X.n);
    if (s == DWD_OK && reqs[i].params.representer &&
        resolve_solver(&reqs[i].params, &reqs[i].X) == DWD_SOLVER_DIRECT)
      s = fail(DWD_E_INVALID, "the representer iteration needs the SMW set-up");
    if (s == DWD_OK && resolve_solver(&reqs[i].params, &reqs[i].X) == DWD_SOLVER_ITERATIVE)
      s = fail(DWD_E_INVALID, "dwd_serve does not run the iterative solver");
    if (s != DWD_OK) return s;
    memset(&out[i].info, 0, sizeof(dwd_info));
    out[i].status = DWD_E_BUSY;
    out[i].t_admit = out[i].t_done = -1.0;
  }
  size_t freeb = 0, totb = 0;
  hipError_t he = hipMemGetInfo(&freeb, &totb);
  if (he != hipSuccess) return hip_fail(he, "hipMemGetInfo");
  const double budget = (opts && opts->hbm_budget_bytes > 0) ? opts->hbm_budget_bytes
                                                             : 0.8 * (double)freeb;
  const int max_slots = (opts && opts->max_slots > 0) ? opts->max_slots : 64;
  const int chunk = (opts && opts->iters_per_round > 0) ? opts->iters_per_round : 16;

  const auto t0 = std::chrono::steady_clock::now();
  std::deque<int> waiting;
  std::vector<Slot> slots;
  int next = 0, finished = 0;
  double used = 0.0;
  dwd_status fatal = DWD_OK;

  auto finish = [&](Slot& s, int status) {
    dwd_response& r = out[s.req];
    if (s.hs && s.P) {
      fill_info(s, &r.info);
      r.info.solve_ms = (now_s(t0) - s.t_admit) * 1e3 - s.P->setup_ms;
      if (r.w) {
        std::vector<double> hw(s.P->d);
        const double* wsrc = s.P->solver == DWD_SOLVER_DIRECT ? s.P->dp.w : s.P->ip.w;
        if (hipMemcpy(hw.data(), wsrc, s.P->d * 8, hipMemcpyDeviceToHost) == hipSuccess)
          for (int64_t k = 0; k < s.P->d; ++k) r.w[k] = hw[k] / s.P->zscale;
        else
          status = DWD_E_DEVICE;
      }
    }
    r.status = status < 0 ? status : r.info.status;
    r.t_done = now_s(t0);
    used -= (double)s.footprint;
    destroy_slot(s);
    s.req = -1;
    ++finished;
  };

  while (finished < nreq && fatal == DWD_OK) {
    const double t = now_s(t0);
    while (next < nreq && reqs[next].t_arrival <= t) waiting.push_back(next++);
    // admission, first come first served
    while (!waiting.empty()) {
      int active = 0;
      for (const Slot& s : slots) active += s.req >= 0;
      if (active >= max_slots) break;
      const int r = waiting.front();
      const dwd_request& q = reqs[r];
      const bool direct = resolve_solver(&q.params, &q.X) == DWD_SOLVER_DIRECT;
      const int64_t fp = direct ? direct_footprint(q.X.d, (int)q.X.n, q.params.storage)
                                : problem_footprint(q.X.d, (int)q.X.n, q.params.storage,
                                                    q.X.layout, q.X.nnz);
      if ((double)fp > budget) {  // can never fit
        out[r].status = DWD_E_BUSY;
        out[r].t_done = now_s(t0);
        ++finished;
        waiting.pop_front();
        continue;
      }
      if (used + (double)fp > budget) break;
      waiting.pop_front();
      Slot s;
      s.req = r;
      s.footprint = fp;
      s.prm = q.params;
      s.t_admit = now_s(t0);
      out[r].t_admit = s.t_admit;
      dwd_status st = DWD_OK;
      if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess ||
          hipHostMalloc((void**)&s.hs, sizeof(Scal), 0) != hipSuccess) {
        st = DWD_E_DEVICE;
      } else {
        st = setup_problem(&q.X, q.y, &q.params, s.stream, &s.P);
      }
      if (st != DWD_OK) {
        out[r].status = st;
        out[r].t_done = now_s(t0);
        destroy_slot(s);
        ++finished;
        if (st == DWD_E_DEVICE) fatal = st;
        continue;
      }
      used += (double)fp;
      s.c = make_consts(s.P, &s.prm);
      s.c_lowp = s.P->storage == DWD_BF16 ? lowp_consts(s.P, &s.prm) : s.c;
      memset(s.hs, 0, sizeof(Scal));
      const double sigma0 = default_sigma0(&s.prm, s.P->n);
      if (s.P->set_penalty(s.prm.e) != hipSuccess ||
          (s.P->solver == DWD_SOLVER_DIRECT
               ? launch_dir_init(s.c, s.P->dp, sigma0, s.stream)
               : launch_init(s.c, s.P->ip, sigma0, s.stream)) != hipSuccess ||
          queue_chunk(s, chunk) != hipSuccess) {
        out[r].status = DWD_E_DEVICE;
        fatal = DWD_E_DEVICE;
      }
      bool placed = false;
      for (Slot& o : slots)
        if (o.req < 0) {
          o = s;
          placed = true;
          break;
        }
      if (!placed) slots.push_back(s);
    }
    // stepping: advance every slot whose queued work has completed
    bool progressed = false;
    for (Slot& s : slots) {
      if (s.req < 0) continue;
      if (s.in_flight) {
        const hipError_t q = hipEventQuery(s.ev);
        if (q == hipErrorNotReady) continue;
        s.in_flight = false;
        if (q != hipSuccess) {
          finish(s, hip_fail(q, "serve"));
          fatal = DWD_E_DEVICE;
          continue;
        }
      }
      progressed = true;
      const hipError_t e = advance(s, chunk);
      if (e != hipSuccess) {
        finish(s, hip_fail(e, "serve"));
        fatal = DWD_E_DEVICE;
        continue;
      }
      if (s.phase == DONE) finish(s, DWD_OK);
    }
    if (!progressed) {
      int active = 0;
      for (const Slot& s : slots) active += s.req >= 0;
      if (active == 0 && waiting.empty() && next < nreq) {
        const double wait = reqs[next].t_arrival - now_s(t0);
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.01)));
      } else {
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
    }
  }
  for (Slot& s : slots)
    if (s.req >= 0) destroy_slot(s);
  return fatal;
}

}  // namespace dwd

extern "C" dwd_status dwd_serve(const dwd_request* reqs, int32_t nreq, const dwd_serve_opts* opts,
                                dwd_response* out) {
  try {
    return dwd::serve(reqs, nreq, opts, out);
  } catch (const std::bad_alloc&) {
    return dwd::fail(DWD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return dwd::fail(DWD_E_DEVICE, "unexpected exception in dwd_serve");
  }
}
