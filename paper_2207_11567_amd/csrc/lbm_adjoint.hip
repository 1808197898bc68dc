// Adjoint kernels and their C entry points (include/lbm.h, differentiation section):
// one reverse step of the fused LB/FD step, the objective J = sum rho |u|^2 / 2 +
// sum (T - mean T)^2 with its gradient with respect to the state, and the reverse of the
// equilibrium initialisation.  Scope: D3Q27, periodic faces, no solids, isothermal or
// passive temperature, cumulant collision with every order >= 3 at rate one; FP64 or FP32.
#include <math.h>
#include <string.h>

#include <string>

#include "../../include/lbm.h"
#include "lbm_adjoint.hpp"

namespace lbm {

template <int PREC, int NS>
__global__ __launch_bounds__(256) void adjoint_kernel(KArgs<typename Prec<PREC>::R> a,
                                                      const typename Prec<PREC>::R *__restrict__ lamB,
                                                      const typename Prec<PREC>::R *__restrict__ lamT1,
                                                      typename Prec<PREC>::R *__restrict__ lamA,
                                                      typename Prec<PREC>::R *__restrict__ coef) {
  using P = Prec<PREC>;
  using St = typename P::St;
  using R = typename P::R;
  using Sc = typename P::Sc;
  constexpr R s = R(1.0 / 3.0);
  const int n = blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
  const int N = a.N;
  if (n >= N) return;
  const unsigned un = (unsigned)n;
  const St *__restrict__ pin = (const St *)a.pop_in;
  const Sc *__restrict__ sin_ = (const Sc *)a.scal_in;
  const int nxy = a.nx * a.ny;
  const int z = n / nxy, rem = n - z * nxy, y = rem / a.nx, x = rem - y * a.nx;
  int off[3][5];
  {
    const AxisNb ax = axis_nb(x, a.nx, -1, -1), ay = axis_nb(y, a.ny, -1, -1), az = axis_nb(z, a.nz, -1, -1);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      off[0][k] = ax.idx[k] - x;
      off[1][k] = (ay.idx[k] - y) * a.nx;
      off[2][k] = (az.idx[k] - z) * nxy;
    }
  }
  // pull (forward recompute)
  R g[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const unsigned m = un + (unsigned)(off[0][2 - cx(i)] + off[1][2 - cy(i)] + off[2][2 - cz(i)]);
    g[i] = decode<R>(ldg(pin + (size_t)i * N, m));
  }
  const R rho0 = a.th.rho_ref;
  const R mom = fdiv(a.P0, s * rho0);
  R mx = R(0), my = R(0), mz = R(0);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    if (cx(i)) mx += R(cx(i)) * g[i];
    if (cy(i)) my += R(cy(i)) * g[i];
    if (cz(i)) mz += R(cz(i)) * g[i];
  }
  const R u[3] = {mx * mom, my * mom, mz * mom};
  R lu[3] = {R(0), R(0), R(0)};
  if constexpr (NS == 1) {
    // T' = T + K lap T - sum_d |u_d| W_d: adjoint of the advection part, per axis
    const R T0 = (R)ldg(sin_, un);
    const R lT = lamT1[n];
    R self = R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const R vp1 = (R)ldg(sin_, un + (unsigned)off[d][3]), vm1 = (R)ldg(sin_, un + (unsigned)off[d][1]);
      const R vp2 = (R)ldg(sin_, un + (unsigned)off[d][4]), vm2 = (R)ldg(sin_, un + (unsigned)off[d][0]);
      const bool up = u[d] >= R(0);
      const R U2 = up ? vm2 : vp2, U1 = up ? vm1 : vp1, D1 = up ? vp1 : vm1;
      R dW[4];
      const R W = weno3_diff_grad(U2, U1, T0, D1, a.eps[0], dW);
      lu[d] += up ? -lT * W : lT * W;               // d(-|u| W)/du = -sign(u) W
      const R c = -lT * fabs(u[d]);
      // contributions to the positions -2, -1, +1, +2 along d (and to the cell itself)
      const R cU2 = c * dW[0], cU1 = c * dW[1], cD1 = c * dW[3];
      coef[(4 * d + 0) * N + n] = up ? cU2 : R(0);
      coef[(4 * d + 1) * N + n] = up ? cU1 : cD1;
      coef[(4 * d + 2) * N + n] = up ? cD1 : cU1;
      coef[(4 * d + 3) * N + n] = up ? R(0) : cU2;
      self += c * dW[2];
    }
    coef[12 * N + n] = self;
  }
  // collision reverse pass
  R lam[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) lam[i] = lamB[i * N + n];
  Rates<R> rt;
  rt.tau0 = viscosity(a.th, rho0) * R(3) + R(0.5);
  rt.smag18 = a.smag18;
  rt.wb = a.wb;
  rt.wh = a.wh;
  rt.gal = false;
  rt.p4 = false;
  collide_d3q27_vjp(g, mom, rt, lam, lu);
  // transposed streaming: the adjoint of g_i(r) = A_i(r - c_i) is pushed to r - c_i
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const unsigned m = un + (unsigned)(off[0][2 - cx(i)] + off[1][2 - cy(i)] + off[2][2 - cz(i)]);
    stg(lamA + (size_t)i * N, m, lam[i]);
  }
}

// lamT(s) = lamT'(s) + K lap(lamT')(s) + self(s) + gathered advection contributions.
template <int PREC>
__global__ __launch_bounds__(256) void adjoint_scalar_kernel(KArgs<typename Prec<PREC>::R> a,
                                                             const typename Prec<PREC>::R *__restrict__ lamT1,
                                                             const typename Prec<PREC>::R *__restrict__ coef,
                                                             typename Prec<PREC>::R *__restrict__ lamT) {
  using R = typename Prec<PREC>::R;
  const int n = blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
  const int N = a.N;
  if (n >= N) return;
  const int nxy = a.nx * a.ny;
  const int z = n / nxy, rem = n - z * nxy, y = rem / a.nx, x = rem - y * a.nx;
  const AxisNb ax = axis_nb(x, a.nx, -1, -1), ay = axis_nb(y, a.ny, -1, -1), az = axis_nb(z, a.nz, -1, -1);
  int off[3][5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    off[0][k] = ax.idx[k] - x;
    off[1][k] = (ay.idx[k] - y) * a.nx;
    off[2][k] = (az.idx[k] - z) * nxy;
  }
  const R rho0 = a.th.rho_ref;
  const R rhoD0 = rho0 * viscosity(a.th, rho0) * a.th.inv_Pr;
  const R K = fdiv(a.th.F, rho0) * rhoD0;
  const R l0 = lamT1[n];
  R lap = R(0), acc = coef[12 * N + n];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lap += lamT1[n + off[d][3]] + lamT1[n + off[d][1]] - R(2) * l0;
    acc += coef[(4 * d + 0) * N + n + off[d][4]];      // from the cell at +2 (its -2 slot)
    acc += coef[(4 * d + 1) * N + n + off[d][3]];      // from +1 (its -1 slot)
    acc += coef[(4 * d + 2) * N + n + off[d][1]];      // from -1 (its +1 slot)
    acc += coef[(4 * d + 3) * N + n + off[d][0]];      // from -2 (its +2 slot)
  }
  lamT[n] = l0 + K * lap + acc;
}

// Objective pieces at the state: block records of (rho|u|^2/2, T, T^2).
template <int PREC, int NS>
__global__ __launch_bounds__(256) void objective_kernel(KArgs<typename Prec<PREC>::R> a, double mean_T, int pass,
                                                        typename Prec<PREC>::R *__restrict__ lamA,
                                                        typename Prec<PREC>::R *__restrict__ lamT) {
  using P = Prec<PREC>;
  using St = typename P::St;
  using R = typename P::R;
  using Sc = typename P::Sc;
  constexpr R s = R(1.0 / 3.0);
  const int n = blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
  const int N = a.N;
  double red[NSUM];
#pragma unroll
  for (int k = 0; k < NSUM; ++k) red[k] = 0.0;
  if (n < N) {
    const unsigned un = (unsigned)n;
    const St *__restrict__ pin = (const St *)a.pop_in;
    const int nxy = a.nx * a.ny;
    const int z = n / nxy, rem = n - z * nxy, y = rem / a.nx, x = rem - y * a.nx;
    const AxisNb ax = axis_nb(x, a.nx, -1, -1), ay = axis_nb(y, a.ny, -1, -1), az = axis_nb(z, a.nz, -1, -1);
    R mx = R(0), my = R(0), mz = R(0);
    unsigned src[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      src[i] = un + (unsigned)((ax.idx[2 - cx(i)] - x) + (ay.idx[2 - cy(i)] - y) * a.nx + (az.idx[2 - cz(i)] - z) * nxy);
      const R gi = decode<R>(ldg(pin + (size_t)i * N, src[i]));
      if (cx(i)) mx += R(cx(i)) * gi;
      if (cy(i)) my += R(cy(i)) * gi;
      if (cz(i)) mz += R(cz(i)) * gi;
    }
    const R rho0 = a.th.rho_ref;
    const R mom = fdiv(a.P0, s * rho0);
    const R ux = mx * mom, uy = my * mom, uz = mz * mom;
    const R T = NS ? (R)((const Sc *)a.scal_in)[n] : R(0);
    if (pass == 0) {
      red[0] = 0.5 * (double)rho0 * ((double)ux * ux + (double)uy * uy + (double)uz * uz);
      red[1] = (double)T;
      red[2] = (double)T * (double)T;
    } else {
      // dJ/dA_i at the pull source of link i: rho mom (c_i . u)
#pragma unroll
      for (int i = 0; i < 27; ++i)
        stg(lamA + (size_t)i * N, src[i], rho0 * mom * (R(cx(i)) * ux + R(cy(i)) * uy + R(cz(i)) * uz));
      if (NS) lamT[n] = R(2) * (T - R(mean_T));
    }
  }
  if (pass == 0) block_sums(red, a.partials + (size_t)blockIdx.x * NSUM);
}

// Reverse of the equilibrium initialisation (Eq. 6) with respect to u0 (FP64 fields).
template <int PREC>
__global__ __launch_bounds__(256) void init_adjoint_kernel(KArgs<double> a, const typename Prec<PREC>::R *lamA,
                                                           const double *u0, double *gu) {
  const int n = blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
  const int N = a.N;
  if (n >= N) return;
  const double ux = u0[n], uy = u0[N + n], uz = u0[2 * N + n];
  const double kq = a.th.rho_ref * (1.0 / 3.0) / a.P0;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int i = 0; i < 27; ++i) {
    const double l = (double)lamA[(size_t)i * N + n] * wgt<27>(i) * kq;
    const double cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
    gx += l * (3.0 * cx(i) + 9.0 * cu * cx(i) - 3.0 * ux);
    gy += l * (3.0 * cy(i) + 9.0 * cu * cy(i) - 3.0 * uy);
    gz += l * (3.0 * cz(i) + 9.0 * cu * cz(i) - 3.0 * uz);
  }
  gu[n] = gx;
  gu[N + n] = gy;
  gu[2 * N + n] = gz;
}

template <class T> __global__ void convert_kernel(const T *in, double *out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

template <int PREC>
hipError_t launch_adjoint_p(int ns, int kind, const StepArgs &sa, int nblocks, hipStream_t st, const void *p0,
                            const void *p1, void *p2, void *p3, void *p4, double mean_T, const double *u0, double *gu) {
  using R = typename Prec<PREC>::R;
  KArgs<R> a = to_kargs<R>(sa);
  if (kind == 0) {   // adjoint step
    if (ns == 0)
      hipLaunchKernelGGL((adjoint_kernel<PREC, 0>), dim3(nblocks), dim3(256), 0, st, a, (const R *)p0, (const R *)p1,
                         (R *)p2, (R *)p4);
    else {
      hipLaunchKernelGGL((adjoint_kernel<PREC, 1>), dim3(nblocks), dim3(256), 0, st, a, (const R *)p0, (const R *)p1,
                         (R *)p2, (R *)p4);
      hipLaunchKernelGGL((adjoint_scalar_kernel<PREC>), dim3(nblocks), dim3(256), 0, st, a, (const R *)p1,
                         (const R *)p4, (R *)p3);
    }
  } else if (kind == 1 || kind == 2) {   // objective pass 0 (sums) / pass 1 (gradient)
    if (ns == 0)
      hipLaunchKernelGGL((objective_kernel<PREC, 0>), dim3(nblocks), dim3(256), 0, st, a, mean_T, kind - 1, (R *)p2,
                         (R *)p3);
    else
      hipLaunchKernelGGL((objective_kernel<PREC, 1>), dim3(nblocks), dim3(256), 0, st, a, mean_T, kind - 1, (R *)p2,
                         (R *)p3);
  } else {   // init adjoint
    hipLaunchKernelGGL((init_adjoint_kernel<PREC>), dim3(nblocks), dim3(256), 0, st, to_kargs<double>(sa),
                       (const R *)p0, u0, gu);
    if (ns && p3)
      hipLaunchKernelGGL((convert_kernel<R>), dim3((sa.N + 255) / 256), dim3(256), 0, st, (const R *)p1, (double *)p3,
                         (long long)sa.N);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(int prec, int ns, int kind, const StepArgs &sa, int nblocks, hipStream_t st, const void *p0,
                          const void *p1, void *p2, void *p3, void *p4, double mean_T, const double *u0,
                          double *gu) {
  if (prec == 0) return launch_adjoint_p<0>(ns, kind, sa, nblocks, st, p0, p1, p2, p3, p4, mean_T, u0, gu);
  return launch_adjoint_p<1>(ns, kind, sa, nblocks, st, p0, p1, p2, p3, p4, mean_T, u0, gu);
}

}  // namespace lbm
