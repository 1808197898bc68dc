// Host-side launch entry points of the step kernels, one set per (lattice, precision,
// scalar count) instance; defined in the per-lattice translation units.
#pragma once

#include "lbm_step.hpp"

namespace lbm {

// LAUNCH_STEP: every cell in one instance (FULL with curved walls, observables or mixture
// transport); LAUNCH_STEP_INTERIOR / LAUNCH_STEP_LIST: the two halves of a split step
// (interior cells on the tile grid, FULL with mixture transport; then the listed boundary
// cells, FULL with curved walls or mixture transport).
enum LaunchKind { LAUNCH_STEP = 0, LAUNCH_EXTRACT = 1, LAUNCH_INIT = 2, LAUNCH_STEP_INTERIOR = 3, LAUNCH_STEP_LIST = 4 };

// Returns hipSuccess or the launch error.  nblocks covers N cells with 256 threads.
hipError_t launch_d2q9(int prec, int ns, int kind, const StepArgs &a, int nblocks, hipStream_t st,
                       const double *Ph, const double *u, const double *scal);
hipError_t launch_d3q27(int prec, int ns, int kind, const StepArgs &a, int nblocks, hipStream_t st,
                        const double *Ph, const double *u, const double *scal);
hipError_t launch_geometry(int Q, const uint8_t *solid, void *geom, int nx, int ny, int nz, long long N,
                           const int *face, hipStream_t st);
hipError_t launch_geometry_levelset(int Q, const double *phi, void *geom, int nx, int ny, int nz, long long N,
                                    const int *face, hipStream_t st);
// Adjoint launches (lbm_adjoint.hip).  kind 0: reverse step (p0 lamB, p1 lamT', p2 lamA out,
// p3 lamT out, p4 coefficient scratch); 1/2: objective sums / gradient (p2 lamA, p3 lamT);
// 3: reverse of the initialisation (p0 lamA, p1 lamT, u0, gu out, p3 grad T out).
hipError_t launch_adjoint(int prec, int ns, int kind, const StepArgs &sa, int nblocks, hipStream_t st, const void *p0,
                          const void *p1, void *p2, void *p3, void *p4, double mean_T, const double *u0, double *gu);
// Sums of the per-block records into out[NSUM]; with thermo (closed domain) also the
// thermodynamic pressure of the next level.
hipError_t launch_finalize(const double *partials, int nblocks, double *stage, double *out, hipStream_t st,
                           double *thermo = nullptr);
hipError_t launch_set_thermo(double *thermo, double pi, double q, double K, hipStream_t st);
// Closed domain: (pi, q, K) of the next level from the step's nrec block records.
hipError_t launch_thermo(const double *partials, int nrec, double *thermo, hipStream_t st);
// Observables: flame-surface block records (slot 0 of the partials) and mean / RMS fields.
hipError_t launch_surface(int Q, int prec, const StepArgs &a, int nblocks, hipStream_t st, double T_u, double T_b);
hipError_t launch_statistics(const double *acc, int D, long long N, long long k, double P0, double *mean, double *rms,
                             hipStream_t st);

// Collision instance for the parameters: BGK, or the cumulant operator with every order
// >= 3 at rate one (decided in the compute precision, as the kernel would), or general
// (other rates, or the parameterised higher orders, a runtime switch of that instance).
template <int Q, int PREC>
int collision_instance(const StepArgs &a) {
  using R = typename Prec<PREC>::R;
  if (a.collision != 0) return COLL_BGK;
  return (Q == 27 && ((R)a.wh != R(1) || a.p4)) ? COLL_CUM : COLL_CUM1;
}

template <int Q, int PREC, int NS, bool FULL, int MODE>
hipError_t launch_step(const StepArgs &a, int nblocks, hipStream_t st) {
  using R = typename Prec<PREC>::R;
  switch (collision_instance<Q, PREC>(a)) {
    case COLL_CUM1:
      // the plain production instances also come with cached pull loads (large grids)
      if constexpr (!FULL && MODE != MODE_LIST)
        if (a.pull_cached) {
          hipLaunchKernelGGL((step_kernel<Q, PREC, NS, false, false, COLL_CUM1, MODE, true>), dim3(nblocks), dim3(256),
                             0, st, to_kargs<R>(a));
          break;
        }
      hipLaunchKernelGGL((step_kernel<Q, PREC, NS, false, FULL, COLL_CUM1, MODE>), dim3(nblocks), dim3(256), 0, st,
                         to_kargs<R>(a));
      break;
    case COLL_CUM:
      if constexpr (Q == 27)
        hipLaunchKernelGGL((step_kernel<Q, PREC, NS, false, FULL, COLL_CUM, MODE>), dim3(nblocks), dim3(256), 0, st,
                           to_kargs<R>(a));
      else
        return hipErrorInvalidValue;
      break;
    default:
      hipLaunchKernelGGL((step_kernel<Q, PREC, NS, false, FULL, COLL_BGK, MODE>), dim3(nblocks), dim3(256), 0, st,
                         to_kargs<R>(a));
  }
  return hipGetLastError();
}

template <int Q, int PREC, int NS>
hipError_t launch_one(int kind, const StepArgs &a, int nblocks, hipStream_t st, const double *Ph,
                      const double *u, const double *scal) {
  using R = typename Prec<PREC>::R;
  const bool full = a.lvl || a.stats || a.probe_out || a.mix;
  switch (kind) {
    case LAUNCH_STEP:
      return full ? launch_step<Q, PREC, NS, true, MODE_ALL>(a, nblocks, st)
                  : launch_step<Q, PREC, NS, false, MODE_ALL>(a, nblocks, st);
    case LAUNCH_STEP_INTERIOR:   // on the 64x4 tile grid when it fits, else on linear tiles
      if (a.band_rows)
        return a.mix ? launch_step<Q, PREC, NS, true, MODE_INTERIOR>(a, nblocks, st)
                     : launch_step<Q, PREC, NS, false, MODE_INTERIOR>(a, nblocks, st);
      return a.mix ? launch_step<Q, PREC, NS, true, MODE_INTERIOR_LIN>(a, nblocks, st)
                   : launch_step<Q, PREC, NS, false, MODE_INTERIOR_LIN>(a, nblocks, st);
    case LAUNCH_STEP_LIST:
      return (a.lvl || a.mix) ? launch_step<Q, PREC, NS, true, MODE_LIST>(a, nblocks, st)
                   : launch_step<Q, PREC, NS, false, MODE_LIST>(a, nblocks, st);
    case LAUNCH_EXTRACT:   // no collision on the extract path
      if (full)
        hipLaunchKernelGGL((step_kernel<Q, PREC, NS, true, true, COLL_CUM1, MODE_ALL>), dim3(nblocks), dim3(256), 0,
                           st, to_kargs<R>(a));
      else
        hipLaunchKernelGGL((step_kernel<Q, PREC, NS, true, false, COLL_CUM1, MODE_ALL>), dim3(nblocks), dim3(256), 0,
                           st, to_kargs<R>(a));
      break;
    default:
      hipLaunchKernelGGL((init_kernel<Q, PREC, NS>), dim3(nblocks), dim3(256), 0, st, to_kargs<double>(a), Ph, u,
                         scal);
  }
  return hipGetLastError();
}

template <int Q, int PREC>
hipError_t launch_ns(int ns, int kind, const StepArgs &a, int nblocks, hipStream_t st, const double *Ph,
                     const double *u, const double *scal) {
  switch (ns) {
    case 0: return launch_one<Q, PREC, 0>(kind, a, nblocks, st, Ph, u, scal);
    case 1: return launch_one<Q, PREC, 1>(kind, a, nblocks, st, Ph, u, scal);
    case 2: return launch_one<Q, PREC, 2>(kind, a, nblocks, st, Ph, u, scal);
    case 6: return launch_one<Q, PREC, 6>(kind, a, nblocks, st, Ph, u, scal);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
