// Allocation-free form of the Section 4.1 choice of C (dwd_suggest_C_noalloc).
//
// dwd_suggest_C allocates two small device buffers per call (the sample
// indices of each class and a 256-bin histogram).  This form keeps them in
// one static device array of fixed size, `scratch`, so a call performs no
// device (or host) allocation: the class split is done on the device, the
// histogram is cleared by a fill kernel, and only a few words are read back
// into stack variables.  The value is the same as dwd_suggest_C's, bit for
// bit: the radix selection counts the same multiset of squared distances,
// and the order of the indices inside each class does not enter the counts.
//
// The array lives once per GPU for the life of the process.  Its device
// address is taken with hipGetSymbolAddress once per device (the array's
// name is only a host-side stand-in) and kept per device; every call on a
// GPU shares that GPU's array, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "dwd_solver.h"

namespace dwd {

namespace {

// Layout of the work area:
//   [0, 4 kStaticMaxN)           sample indices, class +1 first (int32)
//   [kHistOff, kHistOff + 1024)  256 histogram counters (uint32)
//   [kCountOff, kCountOff + 4)   number of samples of class +1 (int32)
constexpr size_t kHistOff = 4 * (size_t)kStaticMaxN;
constexpr size_t kCountOff = kHistOff + 256 * 4;
constexpr size_t kScratchBytes = kCountOff + 256;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the work area (taken once).
hipError_t scratch_ptr(int device, unsigned char** out) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (unsigned char*)ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// Stable split of the samples by class on one block of 1024 threads:
// idx[0 .. npos) = samples with y > 0 in increasing order, then the others.
__global__ void __launch_bounds__(1024) k_class_split(const double* __restrict__ y, int n,
                                                      int* __restrict__ idx,
                                                      int* __restrict__ npos_out) {
  __shared__ int wcnt[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // count of class +1
  int c = 0;
  for (int i = threadIdx.x; i < n; i += 1024) c += y[i] > 0.0 ? 1 : 0;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if (lane == 0) wcnt[wid] = c;
  __syncthreads();
  int npos = 0;
  for (int w = 0; w < 16; ++w) npos += wcnt[w];
  __syncthreads();
  // scatter: a sample of class +1 goes after the positives before it, any
  // other after all positives and the negatives before it
  int run = 0;
  for (int b = 0; b < n; b += 1024) {
    const int i = b + threadIdx.x;
    const bool f = i < n && y[i] > 0.0;
    const unsigned long long m = __ballot(f);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wid] = __popcll(m);
    __syncthreads();
    int pre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      pre += w < wid ? wcnt[w] : 0;
      tot += wcnt[w];
    }
    if (i < n) {
      const int pb = run + pre + below;  // samples of class +1 before i
      if (f)
        idx[pb] = i;
      else
        idx[npos + (i - pb)] = i;
    }
    run += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *npos_out = npos;
}

__global__ void k_zero_u32(unsigned int* __restrict__ p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

}  // namespace

dwd_status suggest_C_static(Problem* P, double q, double* C) {
  if (!(q > 0.0) || !std::isfinite(q)) return fail(DWD_E_INVALID, "q must be > 0");
  if (P->solver != DWD_SOLVER_SMW)
    return fail(DWD_E_INVALID, "dwd_suggest_C_noalloc needs the n x n Gram matrix of the SMW set-up");
  if (P->n > kStaticMaxN)
    return fail(DWD_E_INVALID, "dwd_suggest_C_noalloc: n exceeds the 65536 samples of its static "
                               "work area");
  if (P->device < 0 || P->device >= kMaxDevices)
    return fail(DWD_E_INVALID, "dwd_suggest_C_noalloc: device index out of range");
  hipError_t e;
  if ((e = hipSetDevice(P->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  unsigned char* base = nullptr;
  if ((e = scratch_ptr(P->device, &base)) != hipSuccess)
    return hip_fail(e, "hipGetSymbolAddress(scratch)");
  int* idx = (int*)base;
  unsigned int* hist = (unsigned int*)(base + kHistOff);
  int* dnpos = (int*)(base + kCountOff);
  const hipStream_t st = P->stream;
  const int n = P->n;
  hipLaunchKernelGGL(k_class_split, dim3(1), dim3(1024), 0, st, P->y, n, idx, dnpos);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "k_class_split");
  int npos = 0;
  if ((e = hipMemcpyAsync(&npos, dnpos, 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(e, "class count");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "class split");
  const int nneg = n - npos;
  if (npos < 1 || nneg < 1) return fail(DWD_E_INVALID, "both classes must be present");
  const int64_t total = (int64_t)npos * nneg;
  // k-th smallest key (0-based) by radix selection from the top digit down
  auto select = [&](int64_t k, unsigned long long* key) -> hipError_t {
    unsigned long long prefix = 0;
    unsigned int hh[256];
    for (int shift = 56; shift >= 0; shift -= 8) {
      hipError_t r;
      hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, hist, 256);
      if ((r = hipGetLastError()) != hipSuccess) return r;
      if ((r = launch_pair_hist(P->G, n, idx, npos, idx + npos, nneg, prefix, shift, hist,
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
  if ((e = select((total - 1) / 2, &k1)) != hipSuccess) return hip_fail(e, "suggest_C (static)");
  if (total % 2)
    k2 = k1;
  else if ((e = select(total / 2, &k2)) != hipSuccess)
    return hip_fail(e, "suggest_C (static)");
  return C_from_median_keys(P, q, k1, k2, C);
}

}  // namespace dwd
