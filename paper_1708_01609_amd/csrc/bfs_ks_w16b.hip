// Kernel sets for FP32 transforms, template spectra stored as BF16.
#include "bfs_kernelset.h"

namespace bfs {

Candidates candidates_w16b(uint32_t m) { return candidates_t<float, bf16x2>(m); }

}  // namespace bfs
