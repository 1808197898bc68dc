// D2Q9 instances of the fused step (all precisions and scalar counts).
#include "lbm_launch.hpp"

namespace lbm {
hipError_t launch_d2q9(int prec, int ns, int kind, const StepArgs &a, int nblocks, hipStream_t st,
                       const double *Ph, const double *u, const double *scal) {
  switch (prec) {
    case 0: return launch_ns<9, 0>(ns, kind, a, nblocks, st, Ph, u, scal);
    case 1: return launch_ns<9, 1>(ns, kind, a, nblocks, st, Ph, u, scal);
    case 2: return launch_ns<9, 2>(ns, kind, a, nblocks, st, Ph, u, scal);
  }
  return hipErrorInvalidValue;
}

template <class Src>
static hipError_t geometry(int Q, const Src *solid, void *geom, int nx, int ny, int nz, long long N, const int *f,
                           hipStream_t st) {
  const int nb = (int)((N + 255) / 256);
  if (Q == 9)
    hipLaunchKernelGGL((geometry_kernel<9, Src>), dim3(nb), dim3(256), 0, st, solid, geom, nx, ny, nz, N, f[0],
                       f[1], f[2], f[3], f[4], f[5]);
  else
    hipLaunchKernelGGL((geometry_kernel<27, Src>), dim3(nb), dim3(256), 0, st, solid, geom, nx, ny, nz, N, f[0],
                       f[1], f[2], f[3], f[4], f[5]);
  return hipGetLastError();
}

hipError_t launch_geometry(int Q, const uint8_t *solid, void *geom, int nx, int ny, int nz, long long N,
                           const int *f, hipStream_t st) {
  return geometry(Q, solid, geom, nx, ny, nz, N, f, st);
}

hipError_t launch_geometry_levelset(int Q, const double *phi, void *geom, int nx, int ny, int nz, long long N,
                                    const int *f, hipStream_t st) {
  return geometry(Q, phi, geom, nx, ny, nz, N, f, st);
}

hipError_t launch_finalize(const double *partials, int nblocks, double *stage, double *out, hipStream_t st,
                           double *thermo) {
  const int nb1 = nblocks < 256 ? nblocks : 256;
  const int chunk = (nblocks + nb1 - 1) / nb1;
  hipLaunchKernelGGL(finalize_stage, dim3(nb1), dim3(256), 0, st, partials, nblocks, chunk, stage, (double *)nullptr);
  hipLaunchKernelGGL(finalize_stage, dim3(1), dim3(256), 0, st, (const double *)stage, nb1, nb1, out, thermo);
  return hipGetLastError();
}

hipError_t launch_thermo(const double *partials, int nrec, double *thermo, hipStream_t st) {
  hipLaunchKernelGGL(thermo_kernel, dim3(1), dim3(1024), 0, st, partials, nrec, thermo);
  return hipGetLastError();
}

hipError_t launch_surface(int Q, int prec, const StepArgs &a, int nblocks, hipStream_t st, double T_u, double T_b) {
  const KArgs<double> k = to_kargs<double>(a);
  const double inv = 1.0 / (T_b - T_u);
  if (Q == 9) {
    if (prec == 0) hipLaunchKernelGGL((surface_kernel<9, 0>), dim3(nblocks), dim3(256), 0, st, k, inv);
    else hipLaunchKernelGGL((surface_kernel<9, 1>), dim3(nblocks), dim3(256), 0, st, k, inv);
  } else {
    if (prec == 0) hipLaunchKernelGGL((surface_kernel<27, 0>), dim3(nblocks), dim3(256), 0, st, k, inv);
    else hipLaunchKernelGGL((surface_kernel<27, 1>), dim3(nblocks), dim3(256), 0, st, k, inv);
  }
  return hipGetLastError();
}

hipError_t launch_statistics(const double *acc, int D, long long N, long long k, double P0, double *mean, double *rms,
                             hipStream_t st) {
  const int nb = (int)((N + 255) / 256);
  hipLaunchKernelGGL(statistics_kernel, dim3(nb), dim3(256), 0, st, acc, D, N, (double)k, P0, mean, rms);
  return hipGetLastError();
}

hipError_t launch_set_thermo(double *thermo, double pi, double q, double K, hipStream_t st) {
  hipLaunchKernelGGL(set_thermo_kernel, dim3(1), dim3(64), 0, st, thermo, pi, q, K);
  return hipGetLastError();
}
}  // namespace lbm
