// Kernel sets for FP32 transforms, template spectra stored as FP16.
#include "bfs_kernelset.h"

namespace bfs {

Candidates candidates_w16f(uint32_t m) { return candidates_t<float, __half2>(m); }

}  // namespace bfs
