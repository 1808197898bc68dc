// D3Q27 instances of the fused step, precision 0 (0 FP64, 1 FP32, 2 FP16 storage).
#include "lbm_launch.hpp"

namespace lbm {
hipError_t launch_d3q27_p0(int ns, int kind, const StepArgs &a, int nblocks, hipStream_t st,
                            const double *Ph, const double *u, const double *scal) {
  return launch_ns<27, 0>(ns, kind, a, nblocks, st, Ph, u, scal);
}
}  // namespace lbm
