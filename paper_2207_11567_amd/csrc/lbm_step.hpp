// Fused time-step kernel of the hybrid LB/FD scheme (one thread per cell) and the
// auxiliary kernels (geometry words, equilibrium initialisation, FP64 sum finalisation).
//
// Per fluid cell, in one pass:
//   scalars at the cell and its axis neighbours (ghost rules at walls, inlet, outlet)
//   -> rho (ideal gas), grad rho, diffusion + reaction right-hand sides, Lambda (Eq. 3)
//   -> pull-streaming of the Q populations with boundary substitutions (Eq. 1)
//   -> moments P_h, u (Eq. 7) -> WENO3 advection, explicit Euler scalar update (Sec. 2.3)
//   -> source Xi (Eq. 2) -> pre-conditioning (Eq. 13) -> cumulant collision (Eqs. 9-12)
//   -> post-collision populations (Eq. 8) stored as deviations from the lattice weights
//   -> FP64 block partial sums (wavefront shuffles + LDS), one record per block.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

struct StepArgs {
  const void *pop_in;
  void *pop_out;
  const void *scal_in;
  void *scal_out;
  const void *geom;    // per-cell geometry words or nullptr
  double *partials;    // [nblocks][8]
  int *flag;           // bit 0: non-finite value seen
  double *f_P, *f_rho, *f_u, *f_scal;   // field outputs (extract mode)
  int nx, ny, nz;
  long long N;
  int face[6];         // ST_* code of each face, -1 for periodic
  long long step;
  int collision;       // 0 cumulant, 1 BGK
  int remap;           // XCD-aware block order
  double P0;           // rho_ref cs2
  double wb, wh, smag18;
  double inlet_u[3], inlet_noise, outlet_P;
  double phi_in[8];    // inlet scalars
  double eps[8];       // WENO eps per scalar
  unsigned long long seed;
  Thermo th;
};

template <int Q> struct GeomWord { using T = uint64_t; };
template <> struct GeomWord<9> { using T = uint32_t; };
// bit i < Q: the source cell of link i is solid; bit Q: the cell itself is solid;
// bit Q+1+2d (+1): the cell at +2 e_d (-2 e_d) is solid.
template <int Q> __host__ __device__ constexpr int bit_self() { return Q; }
template <int Q> __host__ __device__ constexpr int bit_far(int d, int neg) { return Q + 1 + 2 * d + neg; }

// XCD-aware block order: hardware hands consecutive workgroups to the 8 XCDs in turn;
// remapping gives each XCD a contiguous slab of cells so that halo rows shared between
// neighbouring blocks stay in the same L2.
__device__ __forceinline__ int tile_of_block(int b, int nb, int remap) {
  if (!remap) return b;
  const int per = nb / 8;
  if (b >= per * 8) return b;
  return (b % 8) * per + b / 8;
}

__device__ __forceinline__ double splitmix_xi(unsigned long long seed, unsigned long long a,
                                              unsigned long long b, unsigned long long n) {
  unsigned long long z = seed + ((n << 40) | (b << 20) | a) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double U = (double)(z >> 11) * 0x1.0p-53;
  return 1.7320508075688772 * (2.0 * U - 1.0);
}

// Per-axis neighbour coordinates k = -2..2 with periodic wrap; out-of-domain positions
// through a non-periodic face get the face's status code.
struct AxisNb {
  int idx[5];
  int code[5];   // -1: inside (or wrapped), else ST_SOLID / ST_INLET / ST_OUTLET
};
__device__ __forceinline__ AxisNb axis_nb(int c, int n, int flo, int fhi) {
  AxisNb r;
#pragma unroll
  for (int k = -2; k <= 2; ++k) {
    int p = c + k;
    int code = -1;
    if (p < 0) {
      if (flo < 0) p += n; else code = flo;
    } else if (p >= n) {
      if (fhi < 0) p -= n; else code = fhi;
    }
    // very small periodic extents: wrap again
    if (code < 0) { p = ((p % n) + n) % n; }
    r.idx[k + 2] = code < 0 ? p : c;
    r.code[k + 2] = code;
  }
  return r;
}

template <class T> __device__ __forceinline__ double to_d(T v) { return (double)v; }

// Block reduction of 8 doubles into partials[tile*8 ..]: wavefront shuffles, then LDS.
__device__ __forceinline__ void block_sums(double (&v)[8], double *out) {
  __shared__ double sh[8][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sh[wv][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int nw = (blockDim.x + 63) >> 6;
    double acc = 0.0;
    for (int w = 0; w < nw; ++w) acc += sh[w][threadIdx.x];
    out[threadIdx.x] = acc;
  }
}

template <int Q, int PREC, int NS, bool EXTRACT>
__global__ __launch_bounds__(256) void step_kernel(StepArgs a) {
  using P = Prec<PREC>;
  using St = typename P::St;
  using R = typename P::R;
  using Sc = typename P::Sc;
  using GW = typename GeomWord<Q>::T;
  constexpr int D = Lat<Q>::D;
  constexpr int NSV = NS > 0 ? NS : 1;
  constexpr R s = R(1.0 / 3.0);

  const int tile = tile_of_block(blockIdx.x, gridDim.x, a.remap);
  const long long n = (long long)tile * blockDim.x + threadIdx.x;
  double red[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long N = a.N;
  const St *__restrict__ pin = (const St *)a.pop_in;
  St *__restrict__ pout = (St *)a.pop_out;
  const Sc *__restrict__ sin_ = (const Sc *)a.scal_in;
  Sc *__restrict__ sout = (Sc *)a.scal_out;

  if (n < N) {
    const int x = (int)(n % a.nx);
    const int y = (int)((n / a.nx) % a.ny);
    const int z = (int)(n / ((long long)a.nx * a.ny));
    const GW gw = a.geom ? ((const GW *)a.geom)[n] : GW(0);
    if (gw & (GW(1) << bit_self<Q>())) {
      if (!EXTRACT) {
#pragma unroll
        for (int i = 0; i < Q; ++i) pout[i * N + n] = pin[i * N + n];
#pragma unroll
        for (int k = 0; k < NS; ++k) sout[k * N + n] = sin_[k * N + n];
      } else {
        if (a.f_P) a.f_P[n] = 0.0;
        if (a.f_rho) a.f_rho[n] = 0.0;
        if (a.f_u)
#pragma unroll
          for (int d = 0; d < D; ++d) a.f_u[d * N + n] = 0.0;
        if (a.f_scal)
#pragma unroll
          for (int k = 0; k < NS; ++k) a.f_scal[k * N + n] = (double)sin_[k * N + n];
      }
    } else {
      const AxisNb ax = axis_nb(x, a.nx, a.face[0], a.face[1]);
      const AxisNb ay = axis_nb(y, a.ny, a.face[2], a.face[3]);
      const AxisNb az = D == 3 ? axis_nb(z, a.nz, a.face[4], a.face[5]) : AxisNb{{z, z, z, z, z}, {-1, -1, -1, -1, -1}};
      auto lin = [&](int X, int Y, int Z) -> long long {
        return (long long)X + (long long)a.nx * ((long long)Y + (long long)a.ny * Z);
      };
      // status of position k (= -2..2) along axis d
      auto status = [&](int d, int k) -> int {
        const AxisNb &A = d == 0 ? ax : d == 1 ? ay : az;
        const int c = A.code[k + 2];
        if (c >= 0) return c;
        if (k == 1) return (gw >> link_from_plus<Q>(d)) & 1 ? ST_SOLID : ST_FLUID;
        if (k == -1) return (gw >> link_from_minus<Q>(d)) & 1 ? ST_SOLID : ST_FLUID;
        if (k == 2) return (gw >> bit_far<Q>(d, 0)) & 1 ? ST_SOLID : ST_FLUID;
        return (gw >> bit_far<Q>(d, 1)) & 1 ? ST_SOLID : ST_FLUID;
      };
      auto nb_index = [&](int d, int k) -> long long {
        return d == 0 ? lin(ax.idx[k + 2], y, z) : d == 1 ? lin(x, ay.idx[k + 2], z) : lin(x, y, az.idx[k + 2]);
      };

      // ---------------------------------------------------------------- scalars at n
      R phi0[NSV];
      R rho0 = R(a.th.rho_ref);
      R R_s[NSV];
      R gradrho[3] = {R(0), R(0), R(0)};
      R Lam = R(0);
      R phin[NSV];
#pragma unroll
      for (int k = 0; k < NSV; ++k) { phi0[k] = R(0); R_s[k] = R(0); phin[k] = R(a.phi_in[k]); }
      if constexpr (NS > 0) {
#pragma unroll
        for (int k = 0; k < NS; ++k) phi0[k] = (R)sin_[k * N + n];
        rho0 = density<NS, R>(a.th, phi0);
        const R rhoD0 = rho0 * viscosity(a.th, rho0) * R(a.th.inv_Pr);
        const R rho_in = density<NS, R>(a.th, phin);
        const R rhoD_in = rho_in * viscosity(a.th, rho_in) * R(a.th.inv_Pr);
        R diff[NSV];
#pragma unroll
        for (int k = 0; k < NS; ++k) diff[k] = R(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          R rk[2];
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int k = side == 0 ? 1 : -1;
            const int st = status(d, k);
            R v[NSV];
            if (st == ST_FLUID) {
              const long long m = nb_index(d, k);
#pragma unroll
              for (int q = 0; q < NS; ++q) v[q] = (R)sin_[q * N + m];
            } else {
#pragma unroll
              for (int q = 0; q < NS; ++q) v[q] = st == ST_INLET ? phin[q] : phi0[q];
            }
            R rhok = rho0;
            if (st == ST_FLUID) rhok = density<NS, R>(a.th, v);
            else if (st == ST_INLET) rhok = rho_in;
            rk[side] = rhok;
            if (st == ST_FLUID || st == ST_INLET) {
              const R rDk = st == ST_INLET ? rhoD_in : rhok * viscosity(a.th, rhok) * R(a.th.inv_Pr);
              const R cf = R(0.5) * (rhoD0 + rDk);
#pragma unroll
              for (int q = 0; q < NS; ++q) diff[q] += cf * (v[q] - phi0[q]);
            }
          }
          gradrho[d] = R(0.5) * (rk[0] - rk[1]);
        }
        const R Fr = R(a.th.F) / rho0;
#pragma unroll
        for (int q = 0; q < NS; ++q) R_s[q] = Fr * diff[q];
        // chemistry (reaction over F) and Lambda
        const R invF = R(1.0 / a.th.F);
        if constexpr (NS == 2) {
          const double *ch = a.th.chem;
          const R r = R(ch[0]) * fmax(phi0[1], R(0)) * exp(-R(ch[1]) / phi0[0]);
          R_s[0] += R((ch[3] - ch[2]) / ch[4]) * r * invF;
          R_s[1] -= r * invF;
          Lam = R_s[0] / phi0[0];
        } else if constexpr (NS == 6) {
          const double *ch = a.th.chem;
          R conc[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) conc[q] = rho0 * fmax(phi0[1 + q], R(0)) * R(1.0 / ch[5 + q]);
          const R T = phi0[0];
          const R q1 = R(ch[0]) * exp(-R(ch[1]) / T) * conc[0] * conc[1];
          const R q2 = R(ch[2]) * exp(-R(ch[3]) / T) * conc[2] * sqrt(conc[1]);
          const R ir = R(1) / rho0;
          // molar rates per mass: nu_k1 q1 + nu_k2 q2 over rho
          const R m0 = -q1 * ir, m1 = (R(-1.5) * q1 - R(0.5) * q2) * ir, m2 = (q1 - q2) * ir,
                  m3 = q2 * ir, m4 = R(2) * q1 * ir;
          R_s[1] += R(ch[5]) * m0 * invF;
          R_s[2] += R(ch[6]) * m1 * invF;
          R_s[3] += R(ch[7]) * m2 * invF;
          R_s[4] += R(ch[8]) * m3 * invF;
          R_s[5] += R(ch[9]) * m4 * invF;
          const R heat = -(R(ch[11]) * m0 + R(ch[12]) * m1 + R(ch[13]) * m2 + R(ch[14]) * m3 +
                           R(ch[15]) * m4) * R(1.0 / ch[4]);
          R_s[0] += heat * invF;
          // Lambda = R_T/T + W sum_k R_k/W_k (N2 by closure: R_N2 = -sum R_k)
          R ysum = R(0), invW = R(0), acc = R(0), rsum = R(0);
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            ysum += phi0[1 + q];
            invW += phi0[1 + q] * R(1.0 / ch[5 + q]);
            acc += R_s[1 + q] * R(1.0 / ch[5 + q]);
            rsum += R_s[1 + q];
          }
          invW += (R(1) - ysum) * R(1.0 / ch[10]);
          acc -= rsum * R(1.0 / ch[10]);
          Lam = R_s[0] / T + acc / invW;
        }
      }

      // ---------------------------------------------------------------- pull (Eq. 1)
      R gh[Q];
      const bool border = ax.code[1] >= 0 || ax.code[3] >= 0 || ay.code[1] >= 0 || ay.code[3] >= 0 ||
                          (D == 3 && (az.code[1] >= 0 || az.code[3] >= 0));
      constexpr GW linkmask = (GW(1) << Q) - GW(1);
      if (!border && !(gw & linkmask)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const long long m = lin(ax.idx[2 - cx(i)], ay.idx[2 - cy(i)], D == 3 ? az.idx[2 - cz(i)] : z);
          gh[i] = decode<R>(pin[i * N + m]);
        }
      } else {
        // boundary cell: bounce-back, moving-wall inlet, anti-bounce-back outlet
        R uw_in[3] = {R(a.inlet_u[0]), R(a.inlet_u[1]), R(a.inlet_u[2])};
        if (a.inlet_noise != 0.0) {
          // in-face coordinates of the inlet face
          int fa = -1;
#pragma unroll
          for (int d = 0; d < D; ++d)
            if (a.face[2 * d] == ST_INLET || a.face[2 * d + 1] == ST_INLET) fa = d;
          if (fa >= 0) {
            const int c3[3] = {x, y, z};
            const int o0 = fa == 0 ? 1 : 0, o1 = fa == 2 ? 1 : 2;
            const double xi = splitmix_xi(a.seed, (unsigned long long)c3[o0],
                                          (unsigned long long)c3[o1], (unsigned long long)a.step);
            const R sc = R(1.0 + a.inlet_noise * xi);
            uw_in[0] *= sc; uw_in[1] *= sc; uw_in[2] *= sc;
          }
        }
        const R rho_in = NS > 0 ? density<NS, R>(a.th, phin) : R(a.th.rho_ref);
        // outlet: velocity of the cell's own post-collision populations, rho at n
        R uo[3] = {R(0), R(0), R(0)};
        bool has_out = false;
#pragma unroll
        for (int d = 0; d < D; ++d) has_out |= a.face[2 * d] == ST_OUTLET || a.face[2 * d + 1] == ST_OUTLET;
        if (has_out) {
#pragma unroll
          for (int j = 0; j < Q; ++j) {
            const R gj = decode<R>(pin[j * N + n]);
            uo[0] += R(cx(j)) * gj;
            uo[1] += R(cy(j)) * gj;
            if (D == 3) uo[2] += R(cz(j)) * gj;
          }
          const R f = R(a.P0) / (s * rho0);
          uo[0] *= f; uo[1] *= f; uo[2] *= f;
        }
        const R uo2 = uo[0] * uo[0] + uo[1] * uo[1] + uo[2] * uo[2];
        const R invP0 = R(1.0 / a.P0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int c[3] = {cx(i), cy(i), D == 3 ? cz(i) : 0};
          bool wall = false, inl = false, outl = false;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            if (c[d] == 0) continue;
            const AxisNb &A = d == 0 ? ax : d == 1 ? ay : az;
            const int code = A.code[2 - c[d]];
            wall |= code == ST_SOLID;
            inl |= code == ST_INLET;
            outl |= code == ST_OUTLET;
          }
          const bool solid_src = (gw >> i) & 1;
          const int io = Q - 1 - i;
          if (wall || (!inl && !outl && solid_src)) {
            gh[i] = decode<R>(pin[io * N + n]);
          } else if (inl) {
            const R cu = R(c[0]) * uw_in[0] + R(c[1]) * uw_in[1] + R(c[2]) * uw_in[2];
            gh[i] = decode<R>(pin[io * N + n]) + R(2.0 * wgt<Q>(i)) * rho_in * cu * invP0;
          } else if (outl) {
            const R cu = R(c[0]) * uo[0] + R(c[1]) * uo[1] + R(c[2]) * uo[2];
            gh[i] = -decode<R>(pin[io * N + n]) +
                    R(2.0 * wgt<Q>(i)) * ((R(a.outlet_P) + rho0 * (cu * cu * R(1.5) - uo2 * R(0.5))) * invP0 - R(1));
          } else {
            const long long m = lin(ax.idx[2 - c[0]], ay.idx[2 - c[1]], D == 3 ? az.idx[2 - c[2]] : z);
            gh[i] = decode<R>(pin[i * N + m]);
          }
        }
      }

      // ---------------------------------------------------------------- moments (Eq. 7)
      R sg = R(0), mx = R(0), my = R(0), mz = R(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        sg += gh[i];
        if (cx(i)) mx += R(cx(i)) * gh[i];
        if (cy(i)) my += R(cy(i)) * gh[i];
        if (D == 3 && cz(i)) mz += R(cz(i)) * gh[i];
      }
      const R P0 = R(a.P0);
      const R mom = P0 / (s * rho0);             // rho u = P0 sum c ghat / cs2
      R u[3] = {mx * mom, my * mom, D == 3 ? mz * mom : R(0)};
      const R Ph = P0 * (sg + R(1)) + R(0.5) * rho0 * s * Lam;

      if (EXTRACT) {
        if (a.f_P) a.f_P[n] = (double)Ph;
        if (a.f_rho) a.f_rho[n] = (double)rho0;
        if (a.f_u)
#pragma unroll
          for (int d = 0; d < D; ++d) a.f_u[d * N + n] = (double)u[d];
        if (a.f_scal)
#pragma unroll
          for (int k = 0; k < NS; ++k) a.f_scal[k * N + n] = (double)phi0[k];
      }

      // ---------------------------------------------------------------- scalar update
      bool bad = false;
      if constexpr (NS > 0) {
        if (!EXTRACT) {
#pragma unroll
          for (int q = 0; q < NS; ++q) {
            R adv = R(0);
            const R eps = R(a.eps[q]);
#pragma unroll
            for (int d = 0; d < D; ++d) {
              const int s1 = status(d, 1), sm1 = status(d, -1);
              const int s2 = status(d, 2), sm2 = status(d, -2);
              const R v0 = phi0[q];
              const R pin_q = phin[q];
              R vp1 = v0, vm1 = v0;
              if (s1 == ST_FLUID) vp1 = (R)sin_[q * N + nb_index(d, 1)];
              else if (s1 == ST_INLET) vp1 = pin_q;
              if (sm1 == ST_FLUID) vm1 = (R)sin_[q * N + nb_index(d, -1)];
              else if (sm1 == ST_INLET) vm1 = pin_q;
              R vp2, vm2;
              if (s1 == ST_FLUID) {
                if (s2 == ST_FLUID) vp2 = (R)sin_[q * N + nb_index(d, 2)];
                else vp2 = s2 == ST_INLET ? pin_q : vp1;
              } else {
                vp2 = s1 == ST_SOLID ? vm1 : s1 == ST_INLET ? pin_q : v0;
              }
              if (sm1 == ST_FLUID) {
                if (sm2 == ST_FLUID) vm2 = (R)sin_[q * N + nb_index(d, -2)];
                else vm2 = sm2 == ST_INLET ? pin_q : vm1;
              } else {
                vm2 = sm1 == ST_SOLID ? vp1 : sm1 == ST_INLET ? pin_q : v0;
              }
              R D_;
              if (u[d] >= R(0))
                D_ = weno3_face(vm1, v0, vp1, eps) - weno3_face(vm2, vm1, v0, eps);
              else
                D_ = weno3_face(vp2, vp1, v0, eps) - weno3_face(vp1, v0, vm1, eps);
              adv += u[d] * D_;
            }
            const R nv = phi0[q] + (R_s[q] - adv);
            bad |= !isfinite(nv);
            sout[q * N + n] = (Sc)nv;
          }
        }
      }

      // ---------------------------------------------------------------- collision
      if (!EXTRACT) {
        const R r = R(a.th.rho_ref) / rho0;             // P0/(rho cs2)
        R Xi[Q];
        R e[Q];
        R Es = R(0), Xs = R(0);
        const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const R ugr = u[0] * gradrho[0] + u[1] * gradrho[1] + u[2] * gradrho[2];
        const R half_rcs = R(0.5) / (rho0 * s);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          if constexpr (NS >= 2) {
            const R cu = R(cx(i)) * u[0] + R(cy(i)) * u[1] + (D == 3 ? R(cz(i)) * u[2] : R(0));
            const R cg = R(cx(i)) * gradrho[0] + R(cy(i)) * gradrho[1] + (D == 3 ? R(cz(i)) * gradrho[2] : R(0));
            const R wi = R(wgt<Q>(i));
            // Eq. 2: cs2 (f_eq/rho - w)(c - u).grad rho + w rho cs2 Lambda
            Xi[i] = s * wi * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu) * (cg - ugr) + wi * rho0 * s * Lam;
          } else {
            Xi[i] = R(0);
          }
          e[i] = r * gh[i] + Xi[i] * half_rcs;           // Eq. 13 minus the weights
          Es += e[i];
          Xs += Xi[i];
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) e[i] -= R(wgt<Q>(i)) * Es;   // d = f~ - w
        const R nu = viscosity(a.th, rho0);
        Rates<R> rt;
        rt.tau0 = nu / s + R(0.5);
        rt.smag18 = R(a.smag18);
        rt.wb = R(a.wb);
        rt.wh = R(a.wh);
        const R base = sg + Xs * R(0.5) / P0;             // (1/r) m0 - 1
        const R invr = rho0 / R(a.th.rho_ref);
        if (a.collision == 0) {
          if constexpr (Q == 9) collide_d2q9(e, u[0], u[1], rt);
          else collide_d3q27(e, u[0], u[1], u[2], rt);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const R gs = R(wgt<Q>(i)) * base + e[i] * invr + Xi[i] * R(0.5) / P0;   // Eq. 8
            pout[i * N + n] = encode<St>(gs);
          }
        } else {
          // BGK in the pre-conditioned frame (Eq. 5 with the half-source split)
          const R om = shear_rate(rt, pipi_of<Q, R>(e, u));
          const R ph1 = Ph / P0 - R(1);
          const R kq = rho0 * s / P0;
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const R cu = R(cx(i)) * u[0] + R(cy(i)) * u[1] + (D == 3 ? R(cz(i)) * u[2] : R(0));
            const R geq = R(wgt<Q>(i)) * (ph1 + kq * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
            const R xh = Xi[i] * R(0.5) / P0;
            const R gp = gh[i] + xh;
            pout[i * N + n] = encode<St>(gp - om * (gp - geq) + xh);
          }
        }
        bad |= !isfinite(Ph + u[0] + u[1] + u[2]);
        if (bad) atomicOr(a.flag, 1);
      }

      // ---------------------------------------------------------------- FP64 sums
      const double rd = (double)rho0;
      red[0] = rd;
      red[1] = (double)Ph;
      red[2] = rd * (double)u[0];
      red[3] = rd * (double)u[1];
      red[4] = rd * (double)u[2];
      red[5] = 0.5 * rd * ((double)u[0] * u[0] + (double)u[1] * u[1] + (double)u[2] * u[2]);
      if constexpr (NS <= 1) {
        red[6] = 1.0 / a.th.T_ref;
      } else if constexpr (NS == 2) {
        red[6] = 1.0 / (double)phi0[0];
      } else {
        double ys = 0.0, inv = 0.0;
#pragma unroll
        for (int q = 0; q < 5; ++q) { ys += (double)phi0[1 + q]; inv += (double)phi0[1 + q] / a.th.chem[5 + q]; }
        inv += (1.0 - ys) / a.th.chem[10];
        red[6] = 1.0 / (inv * (double)phi0[0]);
      }
      if constexpr (NS >= 2) red[7] = rd * (double)phi0[1];
    }
  }
  block_sums(red, a.partials + (long long)tile * 8);
}

// Deterministic second pass: one block sums the per-block records in a fixed order.
static __global__ __launch_bounds__(256) void finalize_sums(const double *partials, int nblocks, double *out) {
  __shared__ double sh[256];
  for (int k = 0; k < 8; ++k) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) acc += partials[(long long)b * 8 + k];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
    __syncthreads();
  }
}

// Geometry words from a solid mask (see GeomWord).
template <int Q>
__global__ __launch_bounds__(256) void geometry_kernel(const uint8_t *solid, void *geom, int nx, int ny,
                                                        int nz, long long N, int f0, int f1, int f2,
                                                        int f3, int f4, int f5) {
  using GW = typename GeomWord<Q>::T;
  constexpr int D = Lat<Q>::D;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((long long)nx * ny));
  const AxisNb ax = axis_nb(x, nx, f0, f1), ay = axis_nb(y, ny, f2, f3);
  const AxisNb az = D == 3 ? axis_nb(z, nz, f4, f5) : AxisNb{{z, z, z, z, z}, {-1, -1, -1, -1, -1}};
  auto lin = [&](int X, int Y, int Z) -> long long {
    return (long long)X + (long long)nx * ((long long)Y + (long long)ny * Z);
  };
  GW w = 0;
  if (solid[n]) w |= GW(1) << bit_self<Q>();
  for (int i = 0; i < Q; ++i) {
    const int c[3] = {cx(i), cy(i), D == 3 ? cz(i) : 0};
    bool out = ax.code[2 - c[0]] >= 0 || ay.code[2 - c[1]] >= 0 || (D == 3 && az.code[2 - c[2]] >= 0);
    if (out || i == (Q - 1) / 2) continue;
    const long long m = lin(ax.idx[2 - c[0]], ay.idx[2 - c[1]], D == 3 ? az.idx[2 - c[2]] : z);
    if (solid[m]) w |= GW(1) << i;
  }
  for (int d = 0; d < D; ++d) {
    const AxisNb &A = d == 0 ? ax : d == 1 ? ay : az;
    for (int neg = 0; neg < 2; ++neg) {
      const int k = neg ? 0 : 4;   // position -2 or +2
      if (A.code[k] >= 0) continue;
      const long long m = d == 0 ? lin(A.idx[k], y, z) : d == 1 ? lin(x, A.idx[k], z) : lin(x, y, A.idx[k]);
      if (solid[m]) w |= GW(1) << bit_far<Q>(d, neg);
    }
  }
  ((GW *)geom)[n] = w;
}

// Equilibrium initialisation (Eq. 6) from FP64 fields; populations stored as deviations.
template <int Q, int PREC, int NS>
__global__ __launch_bounds__(256) void init_kernel(StepArgs a, const double *Ph, const double *u,
                                                   const double *scal) {
  using P = Prec<PREC>;
  using St = typename P::St;
  using Sc = typename P::Sc;
  constexpr int D = Lat<Q>::D;
  constexpr int NSV = NS > 0 ? NS : 1;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long N = a.N;
  if (n >= N) return;
  double v[NSV];
  for (int k = 0; k < NSV; ++k) v[k] = 0.0;
  for (int k = 0; k < NS; ++k) {
    v[k] = scal[k * N + n];
    ((Sc *)a.scal_out)[k * N + n] = (Sc)v[k];
  }
  const double rho = density<NS, double>(a.th, v);
  const double ux = u[n], uy = u[N + n], uz = D == 3 ? u[2 * N + n] : 0.0;
  const double uu = ux * ux + uy * uy + uz * uz;
  const double ph1 = Ph[n] / a.P0 - 1.0;
  const double kq = rho * (1.0 / 3.0) / a.P0;
  for (int i = 0; i < Q; ++i) {
    const double cu = cx(i) * ux + cy(i) * uy + (D == 3 ? cz(i) * uz : 0.0);
    const double gh = wgt<Q>(i) * (ph1 + kq * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    ((St *)a.pop_out)[i * N + n] = (St)gh;
  }
}

}  // namespace lbm
