// dwd_solve_batch: B problems over one shared X stepped together.  The host
// queues iterations in chunks and, one chunk behind, reads every problem's
// stop flag; converged problems leave the active-slot list (double-buffered
// on the device, so the chunk in flight keeps its own list).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "dwd_solver.h"

namespace dwd {

hipError_t launch_init_b(const BatchPtrs& P, int B, hipStream_t st);
hipError_t launch_batch_iteration(const void* X, int storage, int fp64_mfma, const BatchPtrs& P,
                                  const int* idx, int bact, int tile, hipStream_t st,
                                  hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_check_b(const BatchPtrs& P, int p, const double* partT, int nchunks,
                          const double* part_dres, int nblk, hipStream_t st);
hipError_t launch_resume_b(const BatchPtrs& P, const int* idx, int cnt, hipStream_t st);
hipError_t launch_anchor_b(const BatchPtrs& P, int p, const double* partT, int nchunks,
                           hipStream_t st);
int batch_pass_row_blocks(int64_t ld);
int batch_sb_rows(int n);

namespace {

// Tile tuner for the batched pass.  The tile width (16, 32 or 64 slots per
// block) that runs fastest depends on the number of active slots, on the
// shape and on the device; every width gives bit-identical results, so the
// tuner simply times the candidates on real iterations of the solve (a
// rotation over the candidates until each has two completed timings) and
// caches the winner per (device, storage, product precision, ld, n, slot
// bucket) for the rest of the process.
constexpr int kTiles[3] = {1, 2, 4};
constexpr int kTrialsPerTile = 2;

struct TuneKey {
  int device, storage, fp64, n, bucket;
  int64_t ld;
  bool operator<(const TuneKey& o) const {
    return std::tie(device, storage, fp64, n, bucket, ld) <
           std::tie(o.device, o.storage, o.fp64, o.n, o.bucket, o.ld);
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;  // key -> tile

int slot_bucket(int bact) { return std::min(4, (bact + 15) / 16); }

struct Tuner {
  TuneKey base;
  int forced = 0;
  struct Trial {
    int bucket, ti, chunk;
    hipEvent_t a, b;
  };
  std::vector<Trial> trials;
  std::map<int, int> rot;                       // bucket -> trial launches issued
  std::map<int, std::array<double, 3>> sum;     // bucket -> summed ms per candidate
  std::map<int, std::array<int, 3>> cnt;
  std::vector<hipEvent_t> pool;
  ~Tuner() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  int cached(int bucket) {
    if (forced) return forced;
    TuneKey k = base;
    k.bucket = bucket;
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(k);
    return it == g_tuned.end() ? 0 : it->second;
  }
  // Tile for the next launch at `bact` active slots.  While the bucket is
  // untuned the launch is a timed trial: it uses the events in *ea/*eb if
  // the caller brings a pair (profiling), else a pair from the pool.
  hipError_t pick(int bact, int chunk, int* tile, hipEvent_t* ea, hipEvent_t* eb) {
    const int bucket = slot_bucket(bact);
    const int t = cached(bucket);
    if (t) {
      *tile = t;
      return hipSuccess;
    }
    const int ti = rot[bucket]++ % 3;
    *tile = kTiles[ti];
    if (!*ea) {
      hipError_t e;
      if ((e = hipEventCreateWithFlags(ea, hipEventDisableSystemFence)) != hipSuccess) return e;
      pool.push_back(*ea);
      if ((e = hipEventCreateWithFlags(eb, hipEventDisableSystemFence)) != hipSuccess) return e;
      pool.push_back(*eb);
    }
    trials.push_back({bucket, ti, chunk, *ea, *eb});
    return hipSuccess;
  }
  // Fold in the trials of chunks <= done_chunk (their work has completed).
  void collect(int done_chunk) {
    std::vector<Trial> left;
    for (const Trial& t : trials) {
      if (t.chunk > done_chunk) {
        left.push_back(t);
        continue;
      }
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) continue;
      auto& s = sum[t.bucket];  // value-initialised (zeros) on first use
      auto& c = cnt[t.bucket];
      s[t.ti] += ms;
      c[t.ti] += 1;
      if (c[0] >= kTrialsPerTile && c[1] >= kTrialsPerTile && c[2] >= kTrialsPerTile) {
        int best = 0;
        for (int i = 1; i < 3; ++i)
          if (s[i] / c[i] < s[best] / c[best]) best = i;
        TuneKey k = base;
        k.bucket = t.bucket;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned.emplace(k, kTiles[best]);
      }
    }
    trials.swap(left);
  }
};

struct BatchBuffers {
  std::vector<void*> dev;
  std::vector<void*> host;
  ~BatchBuffers() {
    for (void* q : dev) (void)hipFree(q);
    for (void* q : host) (void)hipHostFree(q);
  }
  hipError_t dalloc(void** q, size_t bytes) {
    hipError_t e = hipMalloc(q, bytes ? bytes : 8);
    if (e == hipSuccess) dev.push_back(*q);
    return e;
  }
  hipError_t halloc(void** q, size_t bytes) {
    hipError_t e = hipHostMalloc(q, bytes ? bytes : 8, 0);
    if (e == hipSuccess) host.push_back(*q);
    return e;
  }
};

}  // namespace

#define HIP_TRY_B(expr)                                  \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);    \
  } while (0)

dwd_status solve_batch(Problem* P, int B, const dwd_params* p, double* W, dwd_info* info) {
  for (int j = 0; j < B; ++j) {
    dwd_status s = validate_params(&p[j], true);
    if (s == DWD_OK) s = validate_penalty(&p[j], P->n);
    if (s != DWD_OK) return s;
  }
  if (P->layout != DWD_DENSE) return fail(DWD_E_INVALID, "dwd_solve_batch needs dense X");
  if (P->solver != DWD_SOLVER_SMW)
    return fail(DWD_E_INVALID, "dwd_solve_batch needs the SMW set-up");
  if (P->ld > (int64_t)1 << 23) return fail(DWD_E_INVALID, "dwd_solve_batch needs d <= 8388608");
  HIP_TRY_B(hipSetDevice(P->device));
  const hipStream_t st = P->stream;
  const int n = P->n;
  const int64_t ld = P->ld;
  BatchBuffers bb;
  BatchPtrs bp{};
  bp.y = P->y;
  bp.my = P->my;
  bp.Minv = P->Minv;
  bp.G = P->G;
  bp.n = n;
  bp.ld = ld;
  bp.nb = (n + 15) / 16;  // 16-row tiles of the n x n products
  bp.npb = batch_pass_row_blocks(ld);
  // Representer iteration (params[0].representer): no pass; the element
  // kernel writes the d-norm partials in blocks of 256 rows.
  bp.rep = choose_representer(P, p[0].representer);
  bp.npg = bp.rep ? (n + 255) / 256 : bp.npb;
  const size_t nB = (size_t)n * B;
  double* nv = nullptr;
  HIP_TRY_B(bb.dalloc((void**)&nv, nB * 19 * 8));
  double* q = nv;
  for (double** dst : {&bp.R, &bp.XI, &bp.AL, &bp.PU, &bp.PR, &bp.T, &bp.XX, &bp.F, &bp.S, &bp.V,
                       &bp.DR, &bp.RN, &bp.S1, &bp.V1, &bp.XI0, &bp.XI1, &bp.AL0, &bp.AL1,
                       &bp.HA}) {
    *dst = q;
    q += nB;
  }
  double* dv = nullptr;
  HIP_TRY_B(bb.dalloc((void**)&dv, (size_t)ld * B * 3 * 8));
  bp.U = dv;
  bp.RHO = dv + (size_t)ld * B;
  bp.W = dv + 2 * (size_t)ld * B;
  bp.sbld = (B + 63) / 64 * 64;
  {
    const size_t sbn = (size_t)batch_sb_rows(n) * bp.sbld;
    HIP_TRY_B(bb.dalloc((void**)&bp.SB, sbn * 8));
    HIP_TRY_B(bb.dalloc((void**)&bp.SBf, sbn * 4));
    // the zero rows past n stay zero; columns past the active slots are
    // read by the product but their results are never used
    HIP_TRY_B(hipMemsetAsync(bp.SB, 0, sbn * 8, st));
    HIP_TRY_B(hipMemsetAsync(bp.SBf, 0, sbn * 4, st));
  }
  {  // penalty weights of each problem (column j = p[j].e or ones)
    double* E = nullptr;
    HIP_TRY_B(bb.dalloc((void**)&E, nB * 8));
    std::vector<double> he(nB, 1.0);
    for (int j = 0; j < B; ++j)
      if (p[j].e) std::copy(p[j].e, p[j].e + n, he.begin() + (size_t)j * n);
    HIP_TRY_B(hipMemcpy(E, he.data(), nB * 8, hipMemcpyHostToDevice));
    bp.E = E;
  }
  HIP_TRY_B(bb.dalloc((void**)&bp.part_n1, (size_t)B * bp.nb * 8));
  HIP_TRY_B(bb.dalloc((void**)&bp.part_it, (size_t)B * bp.nb * 8));
  HIP_TRY_B(bb.dalloc((void**)&bp.part_ga, (size_t)B * bp.nb * 8));
  HIP_TRY_B(bb.dalloc((void**)&bp.part_c, (size_t)B * bp.nb * NPC * 8));
  HIP_TRY_B(bb.dalloc((void**)&bp.part_g, (size_t)B * std::max(bp.npb, bp.npg) * NP2 * 8));
  if (bp.rep) {
    double* rv = nullptr;
    HIP_TRY_B(bb.dalloc((void**)&rv, nB * 4 * 8));
    bp.AU = rv;
    bp.ARHO = rv + nB;
    bp.AW = rv + 2 * nB;
    bp.CV = rv + 3 * nB;
    HIP_TRY_B(bb.dalloc((void**)&bp.part_gc, (size_t)B * bp.nb * 8));
  }
  HIP_TRY_B(bb.dalloc((void**)&bp.sc, (size_t)B * sizeof(Scal)));
  Consts* dcs = nullptr;
  HIP_TRY_B(bb.dalloc((void**)&dcs, (size_t)B * sizeof(Consts)));
  bp.cs = dcs;
  int* didx[2];
  HIP_TRY_B(bb.dalloc((void**)&didx[0], (size_t)B * 4));
  HIP_TRY_B(bb.dalloc((void**)&didx[1], (size_t)B * 4));
  int* hidx[2];
  HIP_TRY_B(bb.halloc((void**)&hidx[0], (size_t)B * 4));
  HIP_TRY_B(bb.halloc((void**)&hidx[1], (size_t)B * 4));
  Scal* hsc[2];
  HIP_TRY_B(bb.halloc((void**)&hsc[0], (size_t)B * sizeof(Scal)));
  HIP_TRY_B(bb.halloc((void**)&hsc[1], (size_t)B * sizeof(Scal)));
  Consts* hcs = nullptr;
  HIP_TRY_B(bb.halloc((void**)&hcs, (size_t)B * sizeof(Consts)));
  // FP32 MFMA products (FP64 sums across K tiles) when every problem asks
  // for tol >= 1e-5 and none opts out; they carry a relative error of about
  // 1e-7 per pass, which the n-space recurrences of Z~^T u and Z~^T rho
  // accumulate; the final FP64 check and the re-anchored FP64 resume below
  // repair that.  Otherwise FP64 MFMA products.
  int max_iter = 1;
  int fp64_mfma = 0;
  for (int j = 0; j < B; ++j) {
    if (!p[j].batch_fp32 || p[j].tol < 1e-5) fp64_mfma = 1;
    hcs[j] = make_consts(P, &p[j]);
    hcs[j].sigma0 = default_sigma0(&p[j], n);
    max_iter = std::max(max_iter, p[j].max_iter);
    hidx[0][j] = j;
  }
  hipEvent_t e0, e1, ev[2];
  HIP_TRY_B(hipEventCreate(&e0));
  HIP_TRY_B(hipEventCreate(&e1));
  HIP_TRY_B(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HIP_TRY_B(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* a;
    int k;
    ~EvGuard() {
      for (int i = 0; i < k; ++i) (void)hipEventDestroy(a[i]);
    }
  };
  hipEvent_t all_ev[4] = {e0, e1, ev[0], ev[1]};
  EvGuard guard{all_ev, 4};
  // Optional timing of every pass launch (params[0].profile): event pairs
  // around the Z~ [s_1..s_B] product, summed after the solve.
  const bool profile = p[0].profile != 0 && !bp.rep;  // (no pass to time)
  std::vector<hipEvent_t> pev;
  struct PoolGuard {
    std::vector<hipEvent_t>& v;
    ~PoolGuard() {
      for (hipEvent_t e : v) (void)hipEventDestroy(e);
    }
  } pguard{pev};
  auto pass_events = [&](hipEvent_t* a, hipEvent_t* b) -> hipError_t {
    *a = *b = nullptr;
    if (!profile) return hipSuccess;
    hipEvent_t x, y;
    hipError_t e;
    if ((e = hipEventCreateWithFlags(&x, hipEventDisableSystemFence)) != hipSuccess) return e;
    pev.push_back(x);
    if ((e = hipEventCreateWithFlags(&y, hipEventDisableSystemFence)) != hipSuccess) return e;
    pev.push_back(y);
    *a = x;
    *b = y;
    return hipSuccess;
  };
  HIP_TRY_B(hipEventRecord(e0, st));
  HIP_TRY_B(hipMemcpyAsync(dcs, hcs, (size_t)B * sizeof(Consts), hipMemcpyHostToDevice, st));
  HIP_TRY_B(hipMemcpyAsync(didx[0], hidx[0], (size_t)B * 4, hipMemcpyHostToDevice, st));
  HIP_TRY_B(launch_init_b(bp, B, st));

  const int chunk = std::max(1, p[0].check_every > 0 ? p[0].check_every : 8);
  Tuner tuner;
  tuner.base = TuneKey{P->device, P->st_rec, fp64_mfma, n, 0, ld};
  tuner.forced = p[0].batch_tile;
  // Chunks of iterations replayed as a captured graph once the tile of the
  // current slot count is fixed; re-captured when the active list, the tile
  // or the product precision changes.  Capture needs a stream other than the
  // legacy default one, so it is done on a stream of its own; the graph is
  // launched on the solve's stream.
  const bool use_graph = p[0].graph != 0 && !profile;
  struct GraphCache {
    hipStream_t cap = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    int bact = -1, cur = -1, tile = 0, fp64 = -1;
    void drop() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (g) (void)hipGraphDestroy(g);
      exec = nullptr;
      g = nullptr;
    }
    ~GraphCache() {
      drop();
      if (cap) (void)hipStreamDestroy(cap);
    }
  } gc;
  int graph_launches = 0, graph_captures = 0;
  int cur = 0;
  auto queue_chunk = [&](int bact, int len, int fp64, int cidx) -> dwd_status {
    const int fixed = bp.rep ? 1 : tuner.cached(slot_bucket(bact));
    if (use_graph && fixed && len == chunk) {
      if (!(gc.exec && gc.bact == bact && gc.cur == cur && gc.tile == fixed && gc.fp64 == fp64)) {
        gc.drop();
        if (!gc.cap) HIP_TRY_B(hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking));
        HIP_TRY_B(hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipSuccess;
        for (int j = 0; j < len && ce == hipSuccess; ++j)
          ce = launch_batch_iteration(P->X_rec, P->st_rec, fp64, bp, didx[cur], bact, fixed,
                                      gc.cap, nullptr, nullptr);
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(gc.cap, &g);
        if (ce != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return hip_fail(ce, "batched iteration (capture)");
        }
        HIP_TRY_B(ee);
        gc.g = g;
        HIP_TRY_B(hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0));
        gc.bact = bact;
        gc.cur = cur;
        gc.tile = fixed;
        gc.fp64 = fp64;
        ++graph_captures;
      }
      HIP_TRY_B(hipGraphLaunch(gc.exec, st));
      ++graph_launches;
      return DWD_OK;
    }
    for (int j = 0; j < len; ++j) {
      hipEvent_t pa, pb;
      HIP_TRY_B(pass_events(&pa, &pb));
      int tile = 1;
      if (!bp.rep) HIP_TRY_B(tuner.pick(bact, cidx, &tile, &pa, &pb));
      HIP_TRY_B(launch_batch_iteration(P->X_rec, P->st_rec, fp64, bp, didx[cur], bact, tile, st,
                                       pa, pb));
    }
    return DWD_OK;
  };
  // Run the stepping loop over the active list in didx[cur] (bact entries)
  // until every listed problem has stopped or `budget` iterations are queued.
  auto run = [&](int bact, int budget, int fp64) -> dwd_status {
    int queued = 0, pending = -1;
    for (int cidx = 0;; ++cidx) {
      const int len = std::min(chunk, budget - queued);
      dwd_status qs = queue_chunk(bact, len, fp64, cidx);
      if (qs != DWD_OK) return qs;
      queued += len;
      const int slot = cidx & 1;
      HIP_TRY_B(hipMemcpyAsync(hsc[slot], bp.sc, (size_t)B * sizeof(Scal),
                               hipMemcpyDeviceToHost, st));
      HIP_TRY_B(hipEventRecord(ev[slot], st));
      if (queued >= budget) break;
      if (pending >= 0) {
        HIP_TRY_B(hipEventSynchronize(ev[pending & 1]));
        tuner.collect(pending);
        const Scal* hs = hsc[pending & 1];
        int nact = 0;
        int* nidx = hidx[1 - cur];
        for (int j = 0; j < B; ++j)
          if (!hs[j].done) nidx[nact++] = j;
        if (nact == 0) break;
        if (nact < bact) {
          HIP_TRY_B(hipMemcpyAsync(didx[1 - cur], nidx, (size_t)nact * 4,
                                   hipMemcpyHostToDevice, st));
          cur = 1 - cur;
          bact = nact;
        }
      }
      pending = cidx;
    }
    HIP_TRY_B(hipStreamSynchronize(st));
    tuner.collect(1 << 30);
    return DWD_OK;
  };
  // Final FP64 check of every listed problem over the data of record.
  auto check = [&](const int* list, int cnt) -> dwd_status {
    for (int i = 0; i < cnt; ++i) {
      const int j = list[i];
      if (bp.rep)
        HIP_TRY_B(launch_expand3(P->X_rec, P->st_rec, hcs[j], bp.AW + (size_t)j * n,
                                 bp.AU + (size_t)j * n, bp.ARHO + (size_t)j * n, bp.y,
                                 bp.W + (size_t)j * ld, bp.U + (size_t)j * ld,
                                 bp.RHO + (size_t)j * ld, st));
      HIP_TRY_B(launch_gemvT(P->X_rec, P->st_rec, ld, n, bp.W + (size_t)j * ld,
                             bp.RHO + (size_t)j * ld, P->ip.partT, nullptr, st));
      int nblk = 0;
      HIP_TRY_B(P->dres(hcs[j], bp.AL + (size_t)j * n, bp.RHO + (size_t)j * ld, P->ip.part_g,
                        &nblk));
      HIP_TRY_B(launch_check_b(bp, j, P->ip.partT, P->nchunks, P->ip.part_g, nblk, st));
    }
    HIP_TRY_B(hipMemcpyAsync(hsc[0], bp.sc, (size_t)B * sizeof(Scal), hipMemcpyDeviceToHost, st));
    HIP_TRY_B(hipStreamSynchronize(st));
    return DWD_OK;
  };
  dwd_status rs;
  if ((rs = run(B, max_iter, fp64_mfma)) != DWD_OK) return rs;
  std::vector<int> all(B);
  for (int j = 0; j < B; ++j) all[j] = j;
  if ((rs = check(all.data(), B)) != DWD_OK) return rs;
  // Problems that stopped on their in-loop residuals but miss the tolerance
  // in the FP64 check continue with FP64 products and a tighter in-loop
  // target; a problem counts as converged only when its check meets tol.
  std::vector<int> resumed(B, 0);
  for (int round = 0; round < kMaxResume; ++round) {
    std::vector<int> again;
    int left = 0;
    for (int j = 0; j < B; ++j) {
      const Scal& hs = hsc[0][j];
      const double chk = std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]);
      if (hs.converged && chk >= p[j].tol && hs.k < p[j].max_iter) {
        again.push_back(j);
        left = std::max(left, p[j].max_iter - hs.k);
        hcs[j].tol = resume_tol(hcs[j].tol, p[j].tol, chk);
      }
    }
    if (again.empty()) break;
    HIP_TRY_B(hipMemcpyAsync(dcs, hcs, (size_t)B * sizeof(Consts), hipMemcpyHostToDevice, st));
    for (size_t i = 0; i < again.size(); ++i) {
      hidx[1 - cur][i] = again[i];
      resumed[again[i]] += 1;
    }
    HIP_TRY_B(hipMemcpyAsync(didx[1 - cur], hidx[1 - cur], again.size() * 4,
                             hipMemcpyHostToDevice, st));
    cur = 1 - cur;
    HIP_TRY_B(launch_resume_b(bp, didx[cur], (int)again.size(), st));
    for (int j : again) {
      HIP_TRY_B(launch_gemvT(P->X_rec, P->st_rec, ld, n, bp.U + (size_t)j * ld,
                             bp.RHO + (size_t)j * ld, P->ip.partT, nullptr, st));
      HIP_TRY_B(launch_anchor_b(bp, j, P->ip.partT, P->nchunks, st));
    }
    if ((rs = run((int)again.size(), left, 1)) != DWD_OK) return rs;
    if ((rs = check(again.data(), (int)again.size())) != DWD_OK) return rs;
  }
  HIP_TRY_B(hipEventRecord(e1, st));
  HIP_TRY_B(hipStreamSynchronize(st));
  float ms = 0.0f;
  HIP_TRY_B(hipEventElapsedTime(&ms, e0, e1));
  double pass_ms = 0.0;
  for (size_t j = 0; j + 1 < pev.size(); j += 2) {
    float t = 0.0f;
    HIP_TRY_B(hipEventElapsedTime(&t, pev[j], pev[j + 1]));
    pass_ms += t;
  }
  if (W) {
    std::vector<double> hw((size_t)P->d);
    for (int j = 0; j < B; ++j) {
      HIP_TRY_B(hipMemcpy(hw.data(), bp.W + (size_t)j * ld, P->d * 8, hipMemcpyDeviceToHost));
      for (int64_t k = 0; k < P->d; ++k) W[(size_t)j * P->d + k] = hw[k] / P->zscale;
    }
  }
  bool all_conv = true;
  for (int j = 0; j < B; ++j) {
    const Scal& hs = hsc[0][j];
    const int conv =
        hs.converged && std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]) < p[j].tol ? 1 : 0;
    all_conv = all_conv && conv;
    if (info) {
      dwd_info& in = info[j];
      memset(&in, 0, sizeof(in));
      in.beta = hs.beta;
      in.primal_obj = hs.eta[E_PRIM];
      in.dual_obj = hs.eta[E_DUAL];
      in.eta_p = hs.eta[E_P];
      in.eta_d = hs.eta[E_D];
      in.eta_c = hs.eta[E_C];
      in.eta_gap = hs.eta[E_GAP];
      in.eta_p_check = hs.eta[E_PCHK];
      in.eta_d_check = hs.eta[E_DCHK];
      in.kkt_check = std::max(hs.eta[E_PCHK], hs.eta[E_DCHK]);
      in.sigma = hs.sigma;
      in.iters = hs.k;
      in.n_double = hs.n_double;
      in.newton_max = hs.newton_max;
      in.converged = conv;
      in.setup_ms = P->setup_ms;
      in.solve_ms = ms;
      in.status = conv ? DWD_OK : DWD_NOT_CONVERGED;
      in.resumed = resumed[j];
      in.representer = bp.rep;
      in.stream_ms = pass_ms;  // all pass launches of the batch
      in.stream_launches = (int32_t)(pev.size() / 2);
      in.graph_launches = graph_launches;
    }
  }
  return all_conv ? DWD_OK : DWD_NOT_CONVERGED;
}

}  // namespace dwd
