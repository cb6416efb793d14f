// dwd_serve: replay a trace of solve requests in real time with continuous
// batching on the device.
//
//  * Admission: first come first served, as soon as a slot is free and the
//    request's device footprint fits what is left of the HBM budget.
//  * Memory: one device allocation (the arena) up front; every admitted
//    problem takes its buffers from it and gives them back when it is done,
//    so the stepping loop never calls hipMalloc or hipFree (both would
//    synchronise the device).
//  * Set-up (staging, scaling, Gram matrix, inverse) runs on a worker
//    thread with a stream of its own, overlapping the stepping of the
//    problems already admitted.
//  * Stepping: every admitted problem of the SMW form advances by one
//    iteration per round, and a round is a handful of launches that each
//    cover all of them: the Step 1a/1b kernel, the Step 1c kernel, the pass
//    over Z (one launch per storage type), the representer step and the
//    tail (residuals, stopping and sigma rules) take a device table of
//    problem descriptors and index it by blockIdx.y.  Only what is
//    particular to one problem is launched per problem: the pass that
//    anchors Z~^T u and Z~^T rho at the start of a phase, sparse passes,
//    direct-branch iterations, the final FP64 check.
//  * The host queues rounds in chunks and, one chunk behind, reads every
//    live problem's device scalars (gathered into one copy), and moves
//    problems between phases (BF16 phase, FP32 refinement, final check,
//    resume) and out of the table.
// Each problem runs the device code of dwd_solve on its own state, so its
// result does not depend on the mix.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "dwd_solver.h"

namespace dwd {

__global__ void k_serve_reset(Scal* sc) {
  sc->done = 0;
  sc->converged = 0;
}

// Copy every listed problem's scalars into one array (one device-to-host
// copy per chunk).
__global__ void k_serve_gather(const Scal* const* __restrict__ src, Scal* __restrict__ dst,
                               int count) {
  const int j = blockIdx.x;
  if (j >= count) return;
  const unsigned int* s = reinterpret_cast<const unsigned int*>(src[j]);
  unsigned int* d = reinterpret_cast<unsigned int*>(dst + j);
  for (int w = threadIdx.x; w < (int)(sizeof(Scal) / 4); w += blockDim.x) d[w] = s[w];
}

namespace {

// ---------------------------------------------------------------------------
// Device arena: one hipMalloc, first-fit blocks of 256-byte granules with
// coalescing on release.  Thread-safe (set-up runs on a worker thread).
// ---------------------------------------------------------------------------
class Arena : public DeviceArena {
 public:
  ~Arena() override {
    if (base_) (void)hipFree(base_);
  }
  hipError_t init(size_t bytes) {
    size_ = (bytes + 255) & ~(size_t)255;
    hipError_t e = hipMalloc((void**)&base_, size_);
    if (e == hipSuccess) free_[0] = size_;
    return e;
  }
  void* take(size_t bytes) override {
    const size_t need = (bytes + 255) & ~(size_t)255;
    std::lock_guard<std::mutex> g(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_[off] = need;
      return base_ + off;
    }
    return nullptr;
  }
  void give(void* ptr) override {
    std::lock_guard<std::mutex> g(mu_);
    const size_t off = (size_t)((char*)ptr - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, len = u->second;
    used_.erase(u);
    auto nx = free_.lower_bound(start);
    if (nx != free_.end() && nx->first == start + len) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        start = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = len;
  }

 private:
  char* base_ = nullptr;
  size_t size_ = 0;
  std::mutex mu_;
  std::map<size_t, size_t> free_, used_;
};

// ---------------------------------------------------------------------------
// Set-up worker: one thread, requests in order of admission.
// ---------------------------------------------------------------------------
struct SetupJob {
  int req = -1;
  Problem* P = nullptr;
  dwd_status status = DWD_OK;
};

class SetupWorker {
 public:
  SetupWorker(const dwd_request* reqs, Arena* arena, int device)
      : reqs_(reqs), arena_(arena), device_(device) {}
  ~SetupWorker() { stop(); }
  hipError_t start() {
    hipError_t e = hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    th_ = std::thread([this] { run(); });
    return hipSuccess;
  }
  void stop() {
    {
      std::lock_guard<std::mutex> g(mu_);
      quit_ = true;
    }
    cv_.notify_all();
    if (th_.joinable()) th_.join();
    if (stream_) (void)hipStreamDestroy(stream_);
    stream_ = nullptr;
  }
  void submit(int req) {
    {
      std::lock_guard<std::mutex> g(mu_);
      todo_.push_back(req);
    }
    cv_.notify_all();
  }
  bool poll(SetupJob* out) {
    std::lock_guard<std::mutex> g(mu_);
    if (done_.empty()) return false;
    *out = done_.front();
    done_.pop_front();
    return true;
  }

 private:
  void run() {
    (void)hipSetDevice(device_);
    for (;;) {
      int r;
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [this] { return quit_ || !todo_.empty(); });
        if (quit_) return;
        r = todo_.front();
        todo_.pop_front();
      }
      SetupJob j;
      j.req = r;
      const dwd_request& q = reqs_[r];
      j.status = setup_problem(&q.X, q.y, &q.params, stream_, &j.P, arena_);
      std::lock_guard<std::mutex> g(mu_);
      done_.push_back(j);
    }
  }
  const dwd_request* reqs_;
  Arena* arena_;
  int device_;
  hipStream_t stream_ = nullptr;
  std::thread th_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<int> todo_;
  std::deque<SetupJob> done_;
  bool quit_ = false;
};

enum Phase { MAIN = 0, REFINE = 1, CHECK = 2, RESUME = 3, FINISH = 4 };

struct Live {
  int req = -1;
  Problem* P = nullptr;
  Consts c{}, c_lowp{};
  dwd_params prm{};
  Phase phase = MAIN;
  bool fresh = true;        // the next iteration starts a phase (anchoring pass)
  int resync = 0;           // fresh pass every `resync` iterations (RESUME: 1)
  int k_next = 0;           // iterations queued so far (for the resync cadence)
  long phase_chunk = 0;     // first chunk queued in the current phase: the
                            // scalars of earlier chunks (queued before the
                            // phase's reset) say nothing about it
  long check_chunk = -1;    // CHECK: first chunk whose scalar copy follows the check
  long finish_chunk = -1;   // FINISH: first chunk whose event follows the copy of w
  int resumed = 0, iters_lowp = 0;
  int64_t footprint = 0;
  double t_admit = 0.0;
  Scal hs{};                // last scalars read
  double* hw = nullptr;     // pinned staging of w (FINISH)
  int wslot = -1;
  bool direct = false;
  bool lowp() const { return phase == MAIN && P->storage == DWD_BF16 && !c.representer; }
  const Consts& cur_c() const { return lowp() ? c_lowp : c; }
  const IterPtrs& cur_ip() const { return lowp() ? P->ip_lp : P->ip; }
  const void* cur_X() const { return lowp() ? P->X_lowp : P->X_rec; }
  int cur_st() const { return lowp() ? DWD_BF16 : P->st_rec; }
  bool stepping() const { return phase == MAIN || phase == REFINE || phase == RESUME; }
  Scal* scal() const { return direct ? P->dp.sc : P->ip.sc; }
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void fill_info(const Live& s, dwd_info* info) {
  const Scal& hs = s.hs;
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
  // converged only when the final FP64 check meets the tolerance
  const int conv = hs.converged && info->kkt_check < s.prm.tol ? 1 : 0;
  info->converged = conv;
  info->iters_lowp = s.iters_lowp;
  info->resumed = s.resumed;
  info->representer = s.c.representer;
  info->setup_ms = s.P->setup_ms;
  info->status = conv ? DWD_OK : DWD_NOT_CONVERGED;
}

}  // namespace

dwd_status serve(const dwd_request* reqs, int nreq, const dwd_serve_opts* opts,
                 dwd_response* out) {
  if (nreq < 0 || (nreq > 0 && (!reqs || !out))) return fail(DWD_E_INVALID, "bad request array");
  for (int i = 1; i < nreq; ++i)
    if (reqs[i].t_arrival < reqs[i - 1].t_arrival)
      return fail(DWD_E_INVALID, "requests must be sorted by t_arrival");
  int64_t max_d = 1;
  for (int i = 0; i < nreq; ++i) {
    dwd_status s = validate_params(&reqs[i].params, true);
    if (s == DWD_OK) s = validate_penalty(&reqs[i].params, reqs[i].X.n);
    if (s == DWD_OK && reqs[i].params.representer == 1 &&
        resolve_solver(&reqs[i].params, &reqs[i].X) == DWD_SOLVER_DIRECT)
      s = fail(DWD_E_INVALID, "the representer iteration needs the SMW set-up");
    if (s == DWD_OK && resolve_solver(&reqs[i].params, &reqs[i].X) == DWD_SOLVER_ITERATIVE)
      s = fail(DWD_E_INVALID, "dwd_serve does not run the iterative solver");
    if (s != DWD_OK) return s;
    memset(&out[i].info, 0, sizeof(dwd_info));
    out[i].status = DWD_E_BUSY;
    out[i].t_admit = out[i].t_done = -1.0;
    max_d = std::max<int64_t>(max_d, reqs[i].X.d);
  }
  if (nreq == 0) return DWD_OK;
  int device = 0;
  hipError_t he = hipGetDevice(&device);
  if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
  size_t freeb = 0, totb = 0;
  if ((he = hipMemGetInfo(&freeb, &totb)) != hipSuccess) return hip_fail(he, "hipMemGetInfo");
  const double budget = (opts && opts->hbm_budget_bytes > 0) ? opts->hbm_budget_bytes
                                                             : 0.8 * (double)freeb;
  const int max_slots = (opts && opts->max_slots > 0) ? std::min(opts->max_slots, 4096) : 64;
  const int chunk = (opts && opts->iters_per_round > 0) ? opts->iters_per_round : 16;

  // Footprints, and the set-up scratch the arena must also hold (one set-up
  // at a time): staging of host data, Gram partials or the inverse's work.
  std::vector<int64_t> fps(nreq, 0);
  size_t scratch = 0;
  double fp_max = 1.0;
  for (int r = 0; r < nreq; ++r) {
    const dwd_request& q = reqs[r];
    const bool direct = resolve_solver(&q.params, &q.X) == DWD_SOLVER_DIRECT;
    fps[r] = direct ? direct_footprint(q.X.d, (int)q.X.n, q.params.storage)
                    : problem_footprint(q.X.d, (int)q.X.n, q.params.storage, q.X.layout, q.X.nnz);
    if ((double)fps[r] <= budget) fp_max = std::max(fp_max, (double)fps[r]);
    const size_t n = (size_t)q.X.n, ld = (size_t)padded_ld(q.X.d);
    size_t t = 0;
    if (q.X.layout == DWD_DENSE && !q.X.on_device)
      t += (size_t)q.X.d * n * (q.X.dtype == DWD_FP64 ? 8 : 4);
    if (direct) {
      const size_t dd = (size_t)q.X.d + 1;
      t += dd * dd * 8 * 4;
    } else {
      t += std::max({n * n * (size_t)gram_splits((int64_t)ld, (int)n), n * n,
                     spd_inverse_work((int)n)}) * 8 + n * 64 * 8;
    }
    scratch = std::max(scratch, t);
  }
  // (granule rounding and fragmentation: an eighth more, and 64 MiB)
  const double resident = std::min(budget, fp_max * max_slots) * 1.125;
  const size_t arena_bytes = std::min((size_t)resident + 2 * scratch + ((size_t)64 << 20),
                                      (size_t)(0.95 * (double)freeb));
  Arena arena;
  if ((he = arena.init(arena_bytes)) != hipSuccess) return hip_fail(he, "hipMalloc(serving arena)");

  // Pinned host staging: gathered scalars and descriptor tables (one set per
  // chunk in flight), w of finishing problems; their device twins.
  struct Res {
    std::vector<void*> host, dev;
    std::vector<hipEvent_t> evs;
    hipStream_t s = nullptr;
    ~Res() {
      if (s) (void)hipStreamSynchronize(s);
      for (void* p : host) (void)hipHostFree(p);
      for (void* p : dev) (void)hipFree(p);
      for (hipEvent_t e : evs) (void)hipEventDestroy(e);
      if (s) (void)hipStreamDestroy(s);
    }
  } res;
  if ((he = hipStreamCreateWithFlags(&res.s, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(he, "hipStreamCreate");
  const hipStream_t S = res.s;
  const int cap = max_slots;
  auto hmal = [&](void** p, size_t b) -> hipError_t {
    hipError_t e = hipHostMalloc(p, b, 0);
    if (e == hipSuccess) res.host.push_back(*p);
    return e;
  };
  auto dmal = [&](void** p, size_t b) -> hipError_t {
    hipError_t e = hipMalloc(p, b);
    if (e == hipSuccess) res.dev.push_back(*p);
    return e;
  };
  Scal *h_sc = nullptr, *d_sc = nullptr;
  StepDesc *h_tab = nullptr, *d_tab = nullptr;
  const Scal **h_src = nullptr, **d_src = nullptr;
  double* h_w = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if ((he = hmal((void**)&h_sc, 2 * (size_t)cap * sizeof(Scal))) != hipSuccess ||
      (he = hmal((void**)&h_tab, 2 * (size_t)cap * sizeof(StepDesc))) != hipSuccess ||
      (he = hmal((void**)&h_src, 2 * (size_t)cap * sizeof(Scal*))) != hipSuccess ||
      (he = hmal((void**)&h_w, (size_t)cap * max_d * 8)) != hipSuccess ||
      (he = dmal((void**)&d_sc, (size_t)cap * sizeof(Scal))) != hipSuccess ||
      (he = dmal((void**)&d_tab, 2 * (size_t)cap * sizeof(StepDesc))) != hipSuccess ||
      (he = dmal((void**)&d_src, (size_t)cap * sizeof(Scal*))) != hipSuccess)
    return hip_fail(he, "serving buffers");
  for (auto& e : ev) {
    if ((he = hipEventCreateWithFlags(&e, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(he, "hipEventCreate");
    res.evs.push_back(e);
  }
  std::vector<char> w_used(cap, 0);

  SetupWorker worker(reqs, &arena, device);
  if ((he = worker.start()) != hipSuccess) return hip_fail(he, "set-up worker");

  const auto t0 = std::chrono::steady_clock::now();
  std::deque<int> waiting;
  std::vector<Live> live;     // admitted and set up (slots reused once free)
  int pending_setup = 0;      // admitted, set-up not yet returned
  int next = 0, finished = 0;
  double used = 0.0;
  dwd_status fatal = DWD_OK;
  long chunk_idx = 0;         // chunks queued so far
  long seen = -1;             // last chunk whose scalars were read
  std::vector<std::pair<int, int>> gathered[2];  // (live slot, request) of each copy

  auto release = [&](Live& s) {
    if (s.P) destroy_problem(s.P);
    s.P = nullptr;
    if (s.wslot >= 0) w_used[s.wslot] = 0;
    s.wslot = -1;
    s.hw = nullptr;
    used -= (double)s.footprint;
    s.req = -1;
    ++finished;
  };

  // Phase changes from chunk ci's scalars (its event has completed).
  auto read_chunk = [&](long ci) -> dwd_status {
    const int slot = (int)(ci & 1);
    const std::vector<std::pair<int, int>>& gl = gathered[slot];
    seen = ci;
    for (size_t i = 0; i < gl.size(); ++i) {
      Live& s = live[gl[i].first];
      if (s.req != gl[i].second) continue;
      s.hs = h_sc[(size_t)slot * cap + i];
      const Scal& hs = s.hs;
      hipError_t e = hipSuccess;
      if (s.stepping() && hs.done && ci >= s.phase_chunk) {
        if (s.direct) {
          s.phase = FINISH;
        } else if (s.lowp() && s.prm.refine && hs.k < s.prm.max_iter) {
          s.iters_lowp = hs.k;
          s.phase = REFINE;
          s.phase_chunk = chunk_idx;
          s.fresh = true;
          s.k_next = hs.k;
          hipLaunchKernelGGL(k_serve_reset, dim3(1), dim3(1), 0, S, s.P->ip.sc);
          e = hipGetLastError();
        } else {
          if (s.lowp()) s.iters_lowp = hs.k;
          s.phase = CHECK;
          e = s.P->queue_check(s.c);
          s.check_chunk = chunk_idx;  // the next chunk's copy follows the check
        }
      } else if (s.phase == CHECK && ci >= s.check_chunk) {
        const double chk = std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]);
        const bool no_refine = s.P->storage == DWD_BF16 && !s.prm.refine && !s.c.representer;
        if (hs.converged && chk >= s.prm.tol && s.resumed < kMaxResume &&
            hs.k < s.prm.max_iter && !no_refine) {
          ++s.resumed;
          s.c.tol = resume_tol(s.c.tol, s.prm.tol, chk);
          s.phase = RESUME;
          s.phase_chunk = chunk_idx;
          s.fresh = true;
          s.resync = 1;
          s.k_next = hs.k;
          hipLaunchKernelGGL(k_serve_reset, dim3(1), dim3(1), 0, S, s.P->ip.sc);
          e = hipGetLastError();
        } else {
          s.phase = FINISH;
        }
      }
      if (e == hipSuccess && s.phase == FINISH && !s.hw) {
        // w to pinned staging; the problem's memory goes back once the copy
        // (and so every kernel that used it) has completed
        int ws = 0;
        while (ws < cap && w_used[ws]) ++ws;
        if (ws >= cap) return fail(DWD_E_DEVICE, "serve: no staging slot");
        w_used[ws] = 1;
        s.wslot = ws;
        s.hw = h_w + (size_t)ws * max_d;
        const double* wsrc = s.direct ? s.P->dp.w : s.P->ip.w;
        e = hipMemcpyAsync(s.hw, wsrc, s.P->d * 8, hipMemcpyDeviceToHost, S);
        s.finish_chunk = chunk_idx;
      }
      if (e != hipSuccess) return hip_fail(e, "serve (phase)");
    }
    for (Live& s : live) {
      if (s.req < 0 || s.phase != FINISH || !s.hw || ci < s.finish_chunk) continue;
      dwd_response& r = out[s.req];
      fill_info(s, &r.info);
      r.info.solve_ms = (now_s(t0) - s.t_admit) * 1e3 - s.P->setup_ms;
      if (r.w)
        for (int64_t k = 0; k < s.P->d; ++k) r.w[k] = s.hw[k] / s.P->zscale;
      r.status = r.info.status;
      r.t_done = now_s(t0);
      release(s);
    }
    return DWD_OK;
  };

  while (finished < nreq && fatal == DWD_OK) {
    const double t = now_s(t0);
    while (next < nreq && reqs[next].t_arrival <= t) waiting.push_back(next++);
    // admission, first come first served
    while (!waiting.empty()) {
      int active = pending_setup;
      for (const Live& s : live) active += s.req >= 0;
      if (active >= max_slots) break;
      const int r = waiting.front();
      if ((double)fps[r] > budget) {  // can never fit
        out[r].status = DWD_E_BUSY;
        out[r].t_done = now_s(t0);
        ++finished;
        waiting.pop_front();
        continue;
      }
      if (used + (double)fps[r] > budget) break;
      waiting.pop_front();
      used += (double)fps[r];
      out[r].t_admit = now_s(t0);
      ++pending_setup;
      worker.submit(r);
    }
    // problems whose set-up has returned join at the next round
    SetupJob job;
    while (worker.poll(&job)) {
      --pending_setup;
      const int r = job.req;
      if (job.status != DWD_OK) {
        out[r].status = job.status;
        out[r].t_done = now_s(t0);
        used -= (double)fps[r];
        ++finished;
        if (job.status == DWD_E_DEVICE) fatal = job.status;
        continue;
      }
      Live s;
      s.req = r;
      s.P = job.P;
      s.P->stream = S;
      s.prm = reqs[r].params;
      s.footprint = fps[r];
      s.t_admit = out[r].t_admit;
      s.direct = s.P->solver == DWD_SOLVER_DIRECT;
      s.c = make_consts(s.P, &s.prm);
      s.c_lowp = s.P->storage == DWD_BF16 ? lowp_consts(s.P, &s.prm) : s.c;
      s.resync = s.prm.resync;
      s.phase_chunk = chunk_idx;
      const double sigma0 = default_sigma0(&s.prm, s.P->n);
      if (s.P->set_penalty(s.prm.e) != hipSuccess ||
          (s.direct ? launch_dir_init(s.c, s.P->dp, sigma0, S)
                    : launch_init(s.c, s.P->ip, sigma0, S)) != hipSuccess) {
        fatal = fail(DWD_E_DEVICE, "serve: problem initialisation failed");
        destroy_problem(s.P);
        break;
      }
      bool placed = false;
      for (Live& o : live)
        if (o.req < 0) {
          o = s;
          placed = true;
          break;
        }
      if (!placed) live.push_back(s);
    }
    if (fatal != DWD_OK) break;

    std::vector<int> stepping;
    bool any_live = false;
    for (int j = 0; j < (int)live.size(); ++j) {
      if (live[j].req < 0) continue;
      any_live = true;
      if (live[j].stepping()) stepping.push_back(j);
    }
    if (any_live) {
      // Queue chunk K = chunk_idx; chunk K - 2 (the same staging) is read.
      const int slot = (int)(chunk_idx & 1);
      // descriptor table of the SMW problems in stepping phases, grouped as
      // [dense FP64 | dense FP32 | dense BF16 | sparse | representer]
      std::vector<int> grp[5];
      for (int j : stepping) {
        const Live& s = live[j];
        if (s.direct) continue;
        int g;
        if (s.c.representer)
          g = 4;
        else if (s.P->layout == DWD_CSR)
          g = 3;
        else
          g = s.cur_st() == DWD_FP64 ? 0 : (s.cur_st() == DWD_FP32 ? 1 : 2);
        grp[g].push_back(j);
      }
      std::vector<int> order;
      int goff[6];
      for (int g = 0; g < 5; ++g) {
        goff[g] = (int)order.size();
        order.insert(order.end(), grp[g].begin(), grp[g].end());
      }
      goff[5] = (int)order.size();
      const int m = (int)order.size();
      StepDesc* tab = h_tab + (size_t)slot * cap;
      StepDesc* dtab = d_tab + (size_t)slot * cap;
      int gx_row = 1, gx_pass[5] = {1, 1, 1, 1, 1};
      for (int g = 0; g < 5; ++g)
        for (int i = goff[g]; i < goff[g + 1]; ++i) {
          const Live& s = live[order[i]];
          StepDesc& D = tab[i];
          D.c = s.cur_c();
          D.p = s.cur_ip();
          D.X = s.cur_X();
          D.nrow = ngemv_blocks(s.P->n);
          D.npass = g == 4 ? D.nrow
                           : (g == 3 ? csr_pass_blocks(s.P->ld) : pass2_blocks(s.cur_st(), s.P->ld));
          gx_row = std::max(gx_row, D.nrow);
          gx_pass[g] = std::max(gx_pass[g], D.npass);
        }
      hipError_t e = hipSuccess;
      if (m > 0) e = hipMemcpyAsync(dtab, tab, m * sizeof(StepDesc), hipMemcpyHostToDevice, S);
      for (int round = 0; round < chunk && e == hipSuccess; ++round) {
        // per-problem work at the start of a phase (and every `resync`)
        for (int i = 0; i < m && e == hipSuccess; ++i) {
          Live& s = live[order[i]];
          const bool fresh = s.fresh || (s.resync > 0 && s.k_next % s.resync == 0);
          if (!fresh) continue;
          const Consts& c = s.cur_c();
          const IterPtrs& I = s.cur_ip();
          Problem* P = s.P;
          if (c.representer) {
            e = launch_ngemv(P->n, I.G, I.au, I.Pu, I.G, I.arho, I.Prho, nullptr, nullptr, I.sc,
                             S);
            if (e == hipSuccess) e = launch_rhs(c, I, P->nchunks, 0, S);
          } else {
            if (P->layout == DWD_CSR)
              e = launch_csr_gemvT(P->ipT, P->ixT, P->valT, P->csr_dtype, P->n, I.u, I.rho,
                                   I.partT, I.sc, S);
            else
              e = launch_gemvT(s.cur_X(), s.cur_st(), P->ld, P->n, I.u, I.rho, I.partT, I.sc, S);
            if (e == hipSuccess) e = launch_rhs(c, I, P->nchunks, 1, S);
          }
          s.fresh = false;
        }
        if (m > 0 && e == hipSuccess) e = launch_multi(MULTI_STEP1AB, dtab, m, gx_row, 0, S);
        if (m > 0 && e == hipSuccess) e = launch_multi(MULTI_STEP1C, dtab, m, gx_row, 0, S);
        for (int g = 0; g < 3 && e == hipSuccess; ++g)
          if (goff[g + 1] > goff[g])
            e = launch_multi(MULTI_PASS, dtab + goff[g], goff[g + 1] - goff[g], gx_pass[g],
                             g == 0 ? DWD_FP64 : (g == 1 ? DWD_FP32 : DWD_BF16), S);
        for (int j : grp[3]) {
          if (e != hipSuccess) break;
          const Live& s = live[j];
          const Problem* P = s.P;
          e = launch_csr_pass(P->ipX, P->ixX, P->valX, P->csr_dtype, P->d, s.cur_c(), s.cur_ip(),
                              S);
        }
        if (goff[5] > goff[4] && e == hipSuccess)
          e = launch_multi(MULTI_REP, dtab + goff[4], goff[5] - goff[4], gx_row, 0, S);
        if (m > 0 && e == hipSuccess) e = launch_multi(MULTI_TAIL, dtab, m, 1, 0, S);
        for (int j : stepping)
          if (live[j].direct && e == hipSuccess) e = queue_direct_iteration(live[j].P, live[j].c, S);
        for (int j : stepping) live[j].k_next += 1;
      }
      // the scalars of every live problem still read, in one copy
      std::vector<std::pair<int, int>>& gl = gathered[slot];
      gl.clear();
      const Scal** src = h_src + (size_t)slot * cap;
      for (int j = 0; j < (int)live.size(); ++j)
        if (live[j].req >= 0 && live[j].phase != FINISH) {
          src[gl.size()] = live[j].scal();
          gl.emplace_back(j, live[j].req);
        }
      const int ng = (int)gl.size();
      if (ng > 0) {
        if (e == hipSuccess)
          e = hipMemcpyAsync(d_src, src, ng * sizeof(Scal*), hipMemcpyHostToDevice, S);
        if (e == hipSuccess) {
          hipLaunchKernelGGL(k_serve_gather, dim3(ng), dim3(64), 0, S, d_src, d_sc, ng);
          e = hipGetLastError();
        }
        if (e == hipSuccess)
          e = hipMemcpyAsync(h_sc + (size_t)slot * cap, d_sc, ng * sizeof(Scal),
                             hipMemcpyDeviceToHost, S);
      }
      if (e == hipSuccess) e = hipEventRecord(ev[slot], S);
      if (e != hipSuccess) {
        fatal = hip_fail(e, "serve (queue)");
        break;
      }
      ++chunk_idx;
    }
    // Read one chunk behind: with two unread chunks, wait for the older (its
    // staging and event are the next chunk's); with one, read it if done.
    const long unread = chunk_idx - 1 - seen;
    if (unread >= 2 || (unread == 1 && hipEventQuery(ev[(seen + 1) & 1]) != hipErrorNotReady)) {
      if ((he = hipEventSynchronize(ev[(seen + 1) & 1])) != hipSuccess) {
        fatal = hip_fail(he, "serve");
        break;
      }
      fatal = read_chunk(seen + 1);
    } else if (!any_live) {
      if (pending_setup == 0 && waiting.empty() && next < nreq) {
        const double wait = reqs[next].t_arrival - now_s(t0);
        if (wait > 0)
          std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.01)));
      } else {
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
    }
  }
  worker.stop();
  (void)hipStreamSynchronize(S);
  for (Live& s : live)
    if (s.req >= 0 && s.P) destroy_problem(s.P);
  SetupJob job;  // a set-up that returned after the loop ended
  while (worker.poll(&job))
    if (job.P) destroy_problem(job.P);
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
