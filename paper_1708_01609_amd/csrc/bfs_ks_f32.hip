// Kernel sets for FP32 samples and spectra.
#include "bfs_kernelset.h"

namespace bfs {

Candidates candidates_f32(uint32_t m) { return candidates_t<float, cx<float>>(m); }

}  // namespace bfs
