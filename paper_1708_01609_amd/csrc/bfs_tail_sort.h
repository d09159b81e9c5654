// Device-side ordering of tail records (bfs_tail_sort.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_records.h"

namespace bfs {

// Device bytes of the work area for sorting n records (0 if n is 0 or above 2^31 - 1).
size_t tail_sort_work_bytes(uint64_t n);

// Queue on st: out[0..n) = tails[0..n) in (segment, template_id, lag) order,
// for records of rec_bytes bytes (sizeof(tail_rec) or sizeof(tail_rec64)).
// end_bit: highest key bit + 1 that can be set (48 + the bits of the largest
// segment index; 64 always works).  work: tail_sort_work_bytes(n) device bytes.
hipError_t tail_sort(const void* tails, size_t rec_bytes, uint64_t n, uint32_t end_bit, void* work,
                     size_t work_bytes, void* out, hipStream_t st);

}  // namespace bfs
