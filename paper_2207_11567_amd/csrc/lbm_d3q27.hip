// D3Q27 precision dispatch (instances live in one translation unit per precision).
#include "lbm_launch.hpp"

namespace lbm {
hipError_t launch_d3q27_p0(int, int, const StepArgs &, int, hipStream_t, const double *, const double *,
                           const double *);
hipError_t launch_d3q27_p1(int, int, const StepArgs &, int, hipStream_t, const double *, const double *,
                           const double *);
hipError_t launch_d3q27_p2(int, int, const StepArgs &, int, hipStream_t, const double *, const double *,
                           const double *);

hipError_t launch_d3q27(int prec, int ns, int kind, const StepArgs &a, int nblocks, hipStream_t st,
                        const double *Ph, const double *u, const double *scal) {
  switch (prec) {
    case 0: return launch_d3q27_p0(ns, kind, a, nblocks, st, Ph, u, scal);
    case 1: return launch_d3q27_p1(ns, kind, a, nblocks, st, Ph, u, scal);
    case 2: return launch_d3q27_p2(ns, kind, a, nblocks, st, Ph, u, scal);
  }
  return hipErrorInvalidValue;
}
}  // namespace lbm
