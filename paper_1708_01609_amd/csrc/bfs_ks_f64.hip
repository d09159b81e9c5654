// Kernel sets for FP64 samples and spectra.
#include "bfs_kernelset.h"

namespace bfs {

Candidates candidates_f64(uint32_t m) { return candidates_t<double, cx<double>>(m); }

}  // namespace bfs
