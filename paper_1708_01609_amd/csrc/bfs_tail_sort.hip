// Device-side ordering of a job's tail records by (segment, template_id,
// lag), for fetches of many tails: the host then only copies the sorted
// records.  Keys are segment << 48 | template_id << 17 | lag, which every
// record of a plan fits (segments < 2^16, lags < 2^17, template ids < 2^31
// are checked by the caller); the sort is hipCUB's LSD radix sort of
// (key, index) pairs, and a gather writes the records in key order.  Keys are
// unique (one tail per segment, template and lag), so the order is total and
// the result does not depend on the order the kernels produced the records.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "bfs_tail_sort.h"

namespace bfs {

namespace {

template <typename R>
__global__ __launch_bounds__(256) void tail_keys_kernel(const R* __restrict__ t, uint64_t n,
                                                        uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const R r = t[i];
  keys[i] = (uint64_t(r.segment) << 48) | (uint64_t(r.template_id) << 17) | uint64_t(r.lag);
  idx[i] = uint32_t(i);
}

template <typename R>
__global__ __launch_bounds__(256) void tail_gather_kernel(const R* __restrict__ t, const uint32_t* __restrict__ idx,
                                                          uint64_t n, R* __restrict__ out) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = t[idx[i]];
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t cub_temp_bytes(uint64_t n) {
  size_t bytes = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, static_cast<const uint64_t*>(nullptr),
                                         static_cast<uint64_t*>(nullptr), static_cast<const uint32_t*>(nullptr),
                                         static_cast<uint32_t*>(nullptr), int(n), 0, 64) != hipSuccess)
    return 0;
  return bytes;
}

}  // namespace

size_t tail_sort_work_bytes(uint64_t n) {
  if (n == 0 || n > 0x7fffffffull) return 0;
  const size_t t = cub_temp_bytes(n);
  if (!t) return 0;
  return 2 * align256(n * sizeof(uint64_t)) + 2 * align256(n * sizeof(uint32_t)) + align256(t);
}

template <typename R>
hipError_t tail_sort_t(const R* tails, uint64_t n, uint32_t end_bit, void* work, size_t work_bytes, R* out,
                       hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (n > 0x7fffffffull || end_bit < 17 || end_bit > 64 || work_bytes < tail_sort_work_bytes(n))
    return hipErrorInvalidValue;
  char* w = static_cast<char*>(work);
  auto* k0 = reinterpret_cast<uint64_t*>(w);
  w += align256(n * sizeof(uint64_t));
  auto* k1 = reinterpret_cast<uint64_t*>(w);
  w += align256(n * sizeof(uint64_t));
  auto* i0 = reinterpret_cast<uint32_t*>(w);
  w += align256(n * sizeof(uint32_t));
  auto* i1 = reinterpret_cast<uint32_t*>(w);
  w += align256(n * sizeof(uint32_t));
  size_t temp = cub_temp_bytes(n);
  const dim3 grid(uint32_t((n + 255) / 256));
  hipLaunchKernelGGL(tail_keys_kernel<R>, grid, dim3(256), 0, st, tails, n, k0, i0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipcub::DeviceRadixSort::SortPairs(static_cast<void*>(w), temp, k0, k1, i0, i1, int(n), 0, int(end_bit), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(tail_gather_kernel<R>, grid, dim3(256), 0, st, tails, i1, n, out);
  return hipGetLastError();
}

hipError_t tail_sort(const void* tails, size_t rec_bytes, uint64_t n, uint32_t end_bit, void* work,
                     size_t work_bytes, void* out, hipStream_t st) {
  if (rec_bytes == sizeof(tail_rec))
    return tail_sort_t(static_cast<const tail_rec*>(tails), n, end_bit, work, work_bytes, static_cast<tail_rec*>(out),
                       st);
  if (rec_bytes == sizeof(tail_rec64))
    return tail_sort_t(static_cast<const tail_rec64*>(tails), n, end_bit, work, work_bytes,
                       static_cast<tail_rec64*>(out), st);
  return hipErrorInvalidValue;
}

}  // namespace bfs
