// Allocation-free active-set compaction (sdc_select_noalloc in sdc.h): the
// operation of sdc_select without a context, without host synchronisation
// and without any device allocation.  Its only scratch memory, the per-block
// counts and output offsets, is the file-scope device array below: one copy
// per device, held until the process ends, reached from host code through
// the address hipGetSymbolAddress returns on that device.
#include "sdc.h"

#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>

#include "device.hpp"

namespace {

constexpr int kNaBlock = 256;                                  // list entries per block
constexpr int kNaMaxBlocks = SDC_NOALLOC_MAX_IN / kNaBlock;    // 65536: 256 KiB of counts
constexpr int kNaScanThreads = 1024;
constexpr int kNaMaxDevices = 64;

static_assert(SDC_NOALLOC_MAX_IN % kNaBlock == 0, "whole blocks");

}  // namespace

// Per-block kept counts (INT_MIN: the block holds an entry outside amax),
// turned in place into per-block output offsets.
static __device__ __align__(256) int32_t scratch[kNaMaxBlocks];

namespace {

__device__ inline bool entry_in_range(int32_t i, int64_t n_amax) { return i >= 0 && i < n_amax; }

// Pass 1: kept entries of each block of kNaBlock list entries.
__global__ __launch_bounds__(kNaBlock) void k_na_count(const double* __restrict__ amax, int64_t n_amax,
                                                       const int32_t* __restrict__ idx, int64_t n, double theta,
                                                       int32_t* __restrict__ cnt) {
  __shared__ int wc[kNaBlock / 64], wb[kNaBlock / 64];
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kNaBlock + threadIdx.x;
  const int32_t i = q < n ? idx[q] : 0;
  const bool in = q < n && entry_in_range(i, n_amax);
  const bool keep = in && sdc::keep_row(amax[i], theta);
  const unsigned long long kept = __ballot(keep), bad = __ballot(q < n && !in);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    wc[wid] = __popcll(kept);
    wb[wid] = bad != 0ull;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0, b = 0;
    for (int w = 0; w < kNaBlock / 64; ++w) {
      c += wc[w];
      b |= wb[w];
    }
    cnt[blockIdx.x] = b ? INT_MIN : c;
  }
}

// Pass 2 (one block): exclusive scan of the nb counts in place; the total
// goes to n_out, or -1 when a block held an entry outside amax.
__global__ __launch_bounds__(kNaScanThreads) void k_na_scan(int32_t* __restrict__ cnt, int nb,
                                                            int64_t* __restrict__ n_out) {
  __shared__ int64_t sh[kNaScanThreads];
  __shared__ int any_bad;
  const int t = threadIdx.x;
  if (t == 0) any_bad = 0;
  __syncthreads();
  const int per = (nb + kNaScanThreads - 1) / kNaScanThreads;
  const int lo = min(nb, t * per), hi = min(nb, lo + per);
  int64_t s = 0;
  bool bad = false;
  for (int q = lo; q < hi; ++q) {
    bad = bad || cnt[q] < 0;
    s += cnt[q] < 0 ? 0 : cnt[q];
  }
  if (bad) any_bad = 1;
  sh[t] = s;
  __syncthreads();
  for (int off = 1; off < kNaScanThreads; off <<= 1) {   // inclusive scan of the thread sums
    const int64_t add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t run = sh[t] - s;
  for (int q = lo; q < hi; ++q) {
    const int64_t c = cnt[q] < 0 ? 0 : cnt[q];
    cnt[q] = static_cast<int32_t>(run);
    run += c;
  }
  if (t == kNaScanThreads - 1) n_out[0] = any_bad ? -1 : sh[t];
}

// Pass 3: the kept entries in order, at their block's offset plus their rank.
__global__ __launch_bounds__(kNaBlock) void k_na_write(const double* __restrict__ amax, int64_t n_amax,
                                                       const int32_t* __restrict__ idx, int64_t n, double theta,
                                                       const int32_t* __restrict__ off,
                                                       const int64_t* __restrict__ n_out,
                                                       int32_t* __restrict__ out) {
  __shared__ int wc[kNaBlock / 64];
  if (n_out[0] < 0) return;   // an entry outside amax: nothing is written
  const int64_t q = static_cast<int64_t>(blockIdx.x) * kNaBlock + threadIdx.x;
  const int32_t i = q < n ? idx[q] : 0;
  const bool keep = q < n && entry_in_range(i, n_amax) && sdc::keep_row(amax[i], theta);
  const unsigned long long kept = __ballot(keep);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) wc[wid] = __popcll(kept);
  __syncthreads();
  int base = off[blockIdx.x];
  for (int w = 0; w < wid; ++w) base += wc[w];
  if (keep) out[base + __popcll(kept & ((1ull << lane) - 1ull))] = i;
}

std::mutex g_mu;
int32_t* g_scratch[kNaMaxDevices] = {};   // per device: the device address of `scratch`

// The address of this device's copy of `scratch`, looked up once per device
// with the device current.
int scratch_of(int device, int32_t** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[device]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return SDC_ERR_HIP;
    if (cur != device && hipSetDevice(device) != hipSuccess) return SDC_ERR_HIP;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return SDC_ERR_HIP;
    g_scratch[device] = static_cast<int32_t*>(ptr);
  }
  *out = g_scratch[device];
  return SDC_OK;
}

}  // namespace

extern "C" int sdc_select_noalloc(int32_t device, void* stream, const double* amax, int64_t n_amax,
                                  const int32_t* idx_in, int64_t n_in, double theta, int32_t* idx_out,
                                  int64_t* n_out) {
  if (!n_out || n_in < 0 || n_in > SDC_NOALLOC_MAX_IN || n_amax < 0 ||
      (n_in > 0 && (!amax || !idx_in || !idx_out)))
    return SDC_ERR_ARG;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess) return SDC_ERR_HIP;
  if (device < 0 || device >= n_dev || device >= kNaMaxDevices) return SDC_ERR_ARG;
  int32_t* cnt = nullptr;
  const int rc = scratch_of(device, &cnt);
  if (rc != SDC_OK) return rc;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return SDC_ERR_HIP;
  if (cur != device && hipSetDevice(device) != hipSuccess) return SDC_ERR_HIP;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = static_cast<int>((n_in + kNaBlock - 1) / kNaBlock);
  if (nb > 0) k_na_count<<<nb, kNaBlock, 0, s>>>(amax, n_amax, idx_in, n_in, theta, cnt);
  k_na_scan<<<1, kNaScanThreads, 0, s>>>(cnt, nb, n_out);
  if (nb > 0) k_na_write<<<nb, kNaBlock, 0, s>>>(amax, n_amax, idx_in, n_in, theta, cnt, n_out, idx_out);
  const hipError_t e = hipGetLastError();
  if (cur != device) (void)hipSetDevice(cur);
  return e == hipSuccess ? SDC_OK : SDC_ERR_HIP;
}
