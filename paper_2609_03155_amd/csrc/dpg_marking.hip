// Dörfler marking of the adaptive refinement (paper §4.2, the Fichera case:
// cells ranked by their residual norms; the largest are marked for refinement
// until they carry 30% of the total, the smallest for coarsening while they
// stay within 5% of it).
//
// On the GPU: a stable radix sort of (value, cell) pairs in decreasing value
// (equal values keep increasing cell order), then the exclusive prefix sums
// of the sorted values in a fixed order (per-workgroup sums, one sequential
// pass over those, then each workgroup's own scan), and one flag per cell:
//   refine   when the sum ranked before it is below f_r T,
//   coarsen  when T minus that sum is at most f_c T (and not refined).
// Every step is deterministic: the same values give the same flags.
#include <hipcub/hipcub.hpp>

#include <mutex>
#include <unordered_map>

#include "dpg_kernels.h"

namespace dpg {

namespace {

constexpr int MT = 256;                 // threads per workgroup
constexpr int MPT = 4;                  // consecutive sorted values per thread
constexpr int64_t MCH = (int64_t)MT * MPT;

// keys = values with -0 made +0 (so that zeros tie), vals = cell ids
__global__ __launch_bounds__(MT) void k_mark_init(int64_t n, const double* __restrict__ v, double* __restrict__ keys,
                                                  int64_t* __restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x;
  if (i >= n) return;
  keys[i] = v[i] + 0.0;
  ids[i] = i;
}

// Sum of one thread's run and of the workgroup's chunk (fixed order).
__device__ __forceinline__ double run_sum(const double* __restrict__ s, int64_t n, int64_t i0) {
  double a = 0.0;
#pragma unroll
  for (int u = 0; u < MPT; ++u)
    if (i0 + u < n) a += s[i0 + u];
  return a;
}

__device__ __forceinline__ double chunk_excl_scan(double a, double* red) {
  // exclusive scan of the MT thread sums: thread 0 walks them in order
  red[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int t = 0; t < MT; ++t) {
      const double x = red[t];
      red[t] = run;
      run += x;
    }
    red[MT] = run;
  }
  __syncthreads();
  return red[threadIdx.x];
}

__global__ __launch_bounds__(MT) void k_mark_chunk_sums(int64_t n, const double* __restrict__ s,
                                                        double* __restrict__ csum) {
  __shared__ double red[MT + 1];
  const int64_t i0 = (int64_t)blockIdx.x * MCH + (int64_t)threadIdx.x * MPT;
  (void)chunk_excl_scan(run_sum(s, n, i0), red);
  if (threadIdx.x == 0) csum[blockIdx.x] = red[MT];
}

// One thread: exclusive prefix of the chunk sums in place, total at [nc].
__global__ void k_mark_chunk_scan(int64_t nc, double* __restrict__ csum) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double run = 0.0;
  for (int64_t c = 0; c < nc; ++c) {
    const double x = csum[c];
    csum[c] = run;
    run += x;
  }
  csum[nc] = run;
}

__global__ __launch_bounds__(MT) void k_mark_flags(int64_t n, const double* __restrict__ s,
                                                   const int64_t* __restrict__ ids, const double* __restrict__ csum,
                                                   int64_t nc, double fr, double fc, int8_t* __restrict__ flags) {
  __shared__ double red[MT + 1];
  const int64_t i0 = (int64_t)blockIdx.x * MCH + (int64_t)threadIdx.x * MPT;
  const double base = chunk_excl_scan(run_sum(s, n, i0), red);
  const double total = csum[nc];
  double before = csum[blockIdx.x] + base;
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int64_t i = i0 + u;
    if (i < n) {
      int8_t f = 0;
      if (before < fr * total) f = 1;
      else if (total - before <= fc * total) f = -1;
      flags[ids[i]] = f;
      before += s[i];
    }
  }
}

// Bytes of the marking's temporaries for n cells (keys and ids in and out,
// chunk sums, the sort's temporaries); *sort_bytes receives the last.
hipError_t mark_scratch_bytes(int64_t n, size_t* total, size_t* sort_bytes, hipStream_t st) {
  const int64_t nc = (n + MCH - 1) / MCH;
  *sort_bytes = 0;
  const hipError_t e = hipcub::DeviceRadixSort::SortPairsDescending(
      nullptr, *sort_bytes, (const double*)nullptr, (double*)nullptr, (const int64_t*)nullptr, (int64_t*)nullptr,
      (int)n, 0, 64, st);
  if (e != hipSuccess) return e;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  *total = 2 * up(sizeof(double) * n) + 2 * up(sizeof(int64_t) * n) + up(sizeof(double) * (nc + 1)) + up(*sort_bytes);
  return hipSuccess;
}

// The marking of n > 0 cells with its temporaries in ws (at least
// mark_scratch_bytes, 256-byte aligned).  Stream-ordered.
hipError_t dorfler_mark_ws(int64_t n, const double* values, double fr, double fc, int8_t* flags, char* ws,
                           size_t sort_bytes, hipStream_t st) {
  const int64_t nc = (n + MCH - 1) / MCH;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t kb = up(sizeof(double) * n), ib = up(sizeof(int64_t) * n), cb = up(sizeof(double) * (nc + 1));
  double* k_in = reinterpret_cast<double*>(ws);
  double* k_out = reinterpret_cast<double*>(ws + kb);
  int64_t* i_in = reinterpret_cast<int64_t*>(ws + 2 * kb);
  int64_t* i_out = reinterpret_cast<int64_t*>(ws + 2 * kb + ib);
  double* csum = reinterpret_cast<double*>(ws + 2 * kb + 2 * ib);
  void* tmp = ws + 2 * kb + 2 * ib + cb;
  hipLaunchKernelGGL(k_mark_init, dim3((unsigned)((n + MT - 1) / MT)), dim3(MT), 0, st, n, values, k_in, i_in);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairsDescending(tmp, sort_bytes, k_in, k_out, i_in, i_out, (int)n, 0, 64, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mark_chunk_sums, dim3((unsigned)nc), dim3(MT), 0, st, n, k_out, csum);
    hipLaunchKernelGGL(k_mark_chunk_scan, dim3(1), dim3(64), 0, st, nc, csum);
    hipLaunchKernelGGL(k_mark_flags, dim3((unsigned)nc), dim3(MT), 0, st, n, k_out, i_out, csum, nc, fr, fc, flags);
    e = hipGetLastError();
  }
  return e;
}

// Temporaries of the allocation-free marking: one copy of this array on
// every GPU the library runs on, held until the process ends.  Host code
// never uses its name as an address: the device address of each GPU's copy
// comes from hipGetSymbolAddress (mark_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[kMarkScratchBytes];

std::mutex g_scratch_mu;
std::unordered_map<int, char*> g_scratch_ptr;   // device -> address of its copy of `scratch`

}  // namespace

hipError_t dorfler_mark_workspace(int64_t n, size_t* bytes) {
  *bytes = 0;
  if (n <= 0) return hipSuccess;
  size_t sort_bytes = 0;
  return mark_scratch_bytes(n, bytes, &sort_bytes, nullptr);
}

hipError_t dorfler_mark(int64_t n, const double* values, double fr, double fc, int8_t* flags, void* workspace,
                        size_t workspace_bytes, hipStream_t st, bool* too_small) {
  *too_small = false;
  if (n <= 0) return hipSuccess;
  size_t total = 0, sort_bytes = 0;
  hipError_t e = mark_scratch_bytes(n, &total, &sort_bytes, st);
  if (e != hipSuccess) return e;
  if (workspace) {
    if (workspace_bytes < total || reinterpret_cast<uintptr_t>(workspace) % 256 != 0) {
      *too_small = true;
      return hipSuccess;
    }
    return dorfler_mark_ws(n, values, fr, fc, flags, static_cast<char*>(workspace), sort_bytes, st);
  }
  char* ws = nullptr;
  e = hipMalloc(reinterpret_cast<void**>(&ws), total);
  if (e != hipSuccess) return e;
  e = dorfler_mark_ws(n, values, fr, fc, flags, ws, sort_bytes, st);
  const hipError_t es = hipStreamSynchronize(st);
  const hipError_t ef = hipFree(ws);
  return e != hipSuccess ? e : (es != hipSuccess ? es : ef);
}

// Device address of this GPU's copy of `scratch`, looked up once per device
// (with that device current) and kept.
static hipError_t mark_scratch_ptr(char** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *ptr = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = static_cast<char*>(p);
  *ptr = static_cast<char*>(p);
  return hipSuccess;
}

hipError_t dorfler_mark_noalloc(int64_t n, const double* values, double fr, double fc, int8_t* flags,
                                hipStream_t st, bool* too_large) {
  *too_large = false;
  if (n <= 0) return hipSuccess;
  if (n > kMarkMaxCells) {
    *too_large = true;
    return hipSuccess;
  }
  size_t total = 0, sort_bytes = 0;
  hipError_t e = mark_scratch_bytes(n, &total, &sort_bytes, st);
  if (e != hipSuccess) return e;
  if (total > kMarkScratchBytes) {
    *too_large = true;
    return hipSuccess;
  }
  char* ws = nullptr;
  e = mark_scratch_ptr(&ws);
  if (e != hipSuccess) return e;
  return dorfler_mark_ws(n, values, fr, fc, flags, ws, sort_bytes, st);
}

}  // namespace dpg
