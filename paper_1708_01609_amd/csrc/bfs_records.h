// Tail records as the correlation kernels write them, the device sort orders
// them and the ABI returns them (include/bfsearch.h): 16 bytes with an FP32
// rho for the FP32 path (bfs_tail), 24 bytes with an FP64 rho for the FP64
// path (bfs_tail64).  The first three fields sit at the same offsets in both.
#pragma once

#include <stdint.h>

namespace bfs {

struct tail_rec {
  uint32_t segment, template_id, lag;
  float rho;
};

struct tail_rec64 {
  uint32_t segment, template_id, lag, reserved;
  double rho;
};

// The record of a path computing in real type T.
template <typename T>
struct tail_rec_sel {
  using type = tail_rec;
};
template <>
struct tail_rec_sel<double> {
  using type = tail_rec64;
};
template <typename T>
using tail_rec_t = typename tail_rec_sel<T>::type;

}  // namespace bfs
