// Device helpers of the serving loop (server.cpp):
//   gather_copy    device-submitted candidate ids into the arena, one launch
//                  for a whole admission round (a copy call per request costs a
//                  launch each);
//   sort_accepted  an iteration's accepted pairs by arena position (rocPRIM
//                  radix sort), so that the host hands each request its
//                  contiguous range instead of locating every pair's request.
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>

#include "device_common.h"

namespace blsh {

namespace {
constexpr int kCopyBlock = 256;
constexpr int kCopyChunk = 16 * kCopyBlock;  // ids per block step: 16 per lane, all loads before the stores
struct CopyBatch {
  uint32_t *arena;
  int32_t n_jobs;
  int64_t chunk_end[kCopyJobs];              // running count of chunks
  CopyJob job[kCopyJobs];
};
}  // namespace

__global__ __launch_bounds__(kCopyBlock) void k_gather_copy(CopyBatch b) {
  const int64_t total = b.chunk_end[b.n_jobs - 1];
  int j = 0;
  for (int64_t c = blockIdx.x; c < total; c += gridDim.x) {
    while (c >= b.chunk_end[j]) ++j;         // c grows, so j only moves forward; stops below n_jobs
    const int64_t base = (c - (j ? b.chunk_end[j - 1] : 0)) * kCopyChunk;
    const int64_t len = min<int64_t>(kCopyChunk, b.job[j].n - base);
    const uint32_t *src = b.job[j].src + base;
    uint32_t *dst = b.arena + b.job[j].dst + base;
    uint32_t v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = u * kCopyBlock + int(threadIdx.x);
      if (i < len) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = u * kCopyBlock + int(threadIdx.x);
      if (i < len) dst[i] = v[u];
    }
  }
}

int gather_copy(const CopyJob *jobs, int n_jobs, uint32_t *arena, hipStream_t s) {
  if (n_jobs <= 0) return BLSH_OK;
  if (n_jobs > kCopyJobs) return fail(BLSH_EINVAL, "gather_copy: %d jobs > %d", n_jobs, kCopyJobs);
  CopyBatch b{};
  b.arena = arena;
  b.n_jobs = n_jobs;
  int64_t acc = 0;
  for (int j = 0; j < n_jobs; ++j) {
    if (jobs[j].n < 0) return fail(BLSH_EINVAL, "gather_copy: negative length");
    b.job[j] = jobs[j];
    acc += (jobs[j].n + kCopyChunk - 1) / kCopyChunk;
    b.chunk_end[j] = acc;
  }
  if (acc == 0) return BLSH_OK;
  const unsigned grid = unsigned(std::min<int64_t>(acc, 65536));
  hipLaunchKernelGGL(k_gather_copy, dim3(grid), dim3(kCopyBlock), 0, s, b);
  if (hipGetLastError() != hipSuccess) return fail(BLSH_EDEVICE, "gather_copy launch");
  return BLSH_OK;
}

int sort_accepted(const uint64_t *key_in, const float *val_in, uint64_t *key_out, float *val_out, int64_t n,
                  int key_bits, void *tmp, size_t *tmp_bytes, hipStream_t s) {
  if (n < 0 || key_bits < 1 || key_bits > 64) return fail(BLSH_EINVAL, "sort_accepted: bad size");
  const hipError_t e = rocprim::radix_sort_pairs(tmp, *tmp_bytes, key_in, key_out, val_in, val_out, size_t(n), 0,
                                                 unsigned(key_bits), s);
  if (e != hipSuccess) return fail(BLSH_EDEVICE, "sort_accepted: %s", hipGetErrorString(e));
  return BLSH_OK;
}

}  // namespace blsh
