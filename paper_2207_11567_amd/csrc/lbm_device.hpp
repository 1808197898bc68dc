// Device-side building blocks of the hybrid LB/FD time step for gfx950 (CDNA4):
// velocity sets, storage codecs, the cumulant collision in the pre-conditioned frame,
// and the thermochemistry / finite-difference helpers.  Everything here runs in one
// thread per lattice cell; all loops over populations are unrolled at compile time so
// the Q populations and their moments live in registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ------------------------------------------------------------------------ velocity sets
// Population i has velocity (i%3-1, (i/3)%3-1, i/9-1); weights are the tensor product of
// the 1-D third-order Gauss-Hermite weights (1/6, 2/3, 1/6) (Sec. 2.1: D2Q9, D3Q27).
template <int Q> struct Lat;
template <> struct Lat<9> {
  static constexpr int D = 2;
  static constexpr int Q = 9;
};
template <> struct Lat<27> {
  static constexpr int D = 3;
  static constexpr int Q = 27;
};

__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i / 9 - 1; }
__host__ __device__ constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
template <int Q> __host__ __device__ constexpr double wgt(int i) {
  return Q == 9 ? w1(cx(i)) * w1(cy(i)) : w1(cx(i)) * w1(cy(i)) * w1(cz(i));
}
// index of the link whose velocity is -e_d (its source is the +e_d neighbour)
template <int Q> __host__ __device__ constexpr int link_from_plus(int d) {
  return (Q - 1) / 2 - (d == 0 ? 1 : d == 1 ? 3 : 9);
}
template <int Q> __host__ __device__ constexpr int link_from_minus(int d) {
  return (Q - 1) / 2 + (d == 0 ? 1 : d == 1 ? 3 : 9);
}

// ------------------------------------------------------------------------ precisions
// PREC 0: FP64 storage and math; 1: FP32 storage and math; 2: FP16 storage, FP32 math.
template <int PREC> struct Prec;
template <> struct Prec<0> { using St = double; using R = double; using Sc = double; };
template <> struct Prec<1> { using St = float; using R = float; using Sc = float; };
template <> struct Prec<2> { using St = _Float16; using R = float; using Sc = float; };

template <class R, class St> __device__ __forceinline__ R decode(St v) { return (R)v; }
template <class St, class R> __device__ __forceinline__ St encode(R v) { return (St)v; }

// status of a neighbour position for the stencils and the links
enum : int { ST_FLUID = 0, ST_SOLID = 1, ST_INLET = 2, ST_OUTLET = 3 };

// Division: IEEE in FP64; in FP32 the hardware reciprocal (1 ulp) times the numerator.
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Exponential, base-2 logarithm and square root: the library's in FP64; in FP32 the
// hardware's base-2 exponential, logarithm and square root (about 1 ulp for normal
// arguments) without the library's range reduction and denormal scaling, which cost about
// fifteen instructions each.  Their arguments here (temperature ratios, Arrhenius exponents
// above -90, non-negative rates and concentrations) are normal or zero, and results that
// would be denormal are physically zero.
__device__ __forceinline__ double hexp(double x) { return exp(x); }
__device__ __forceinline__ float hexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ double hexp2(double x) { return exp2(x); }
__device__ __forceinline__ float hexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double hlog2(double x) { return log2(x); }
__device__ __forceinline__ float hlog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double hsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ------------------------------------------------------------------------ 1-D chimera
// Central moments of orders 0,1,2 about u of a 3-point distribution on {-1,0,+1}
// (Geier et al. 2015, the 1-D factor of the D2Q9/D3Q27 moment transform), in place.
template <class R> __device__ __forceinline__ void fwd3(R &m, R &z, R &p, R u) {
  // k0 = m + z + p, k1 = (p - m) - u k0, k2 = (p + m) - 2u (p - m) + u^2 k0
  //                                      = (p + m) - u ((p - m) + k1)
  const R sp = p + m, d = p - m;
  const R k0 = sp + z;
  const R k1 = d - u * k0;
  const R k2 = sp - u * (d + k1);
  m = k0; z = k1; p = k2;
}
template <class R> __device__ __forceinline__ void inv3(R &k0, R &k1, R &k2, R u) {
  // raw moments m1 = k1 + u k0, m2 = k2 + 2u k1 + u^2 k0 = k2 + u (k1 + m1);
  // populations f0 = k0 - m2, f+ = (m2 + m1)/2, f- = (m2 - m1)/2
  const R m1 = k1 + u * k0;
  const R m2 = k2 + u * (k1 + m1);
  const R h1 = R(0.5) * m1;
  const R zero = k0 - m2;
  const R plus = R(0.5) * m2 + h1;
  const R minus = R(0.5) * m2 - h1;
  k0 = minus; k1 = zero; k2 = plus;
}

// ------------------------------------------------------------------------ collision
// Cumulant collision (Sec. 2.2) on the density-one distribution f~ = w + d of the
// pre-conditioned populations, centred on u.  d holds the deviations (sum d = 0) and is
// replaced by the post-collision deviations.  The central moments of f~ are split into
// the analytically known weight part kappa^w = prod_d K_{a_d}(u_d), K = (1, -u, cs2+u^2),
// and the transformed deviation part kappa^d; second-order diagonal moments are carried
// as A = kappa_aa - cs2 so that no O(1) quantity is ever subtracted from another.
// Returns the shear rate used (Smagorinsky closed form on tau).
//
// Galilean correction (Geier et al. 2015): on these velocity sets c^3 = c, so the
// equilibrium third diagonal moment misses u_a^3 and the Chapman-Enskog stress carries
// (1/omega - 1/2) 3 u_a^2 d_a u_a on each diagonal.  With d_a u_a estimated from the
// pre-collision non-equilibrium second cumulants (A, B, C: deviatoric part at the shear
// rate, trace at the bulk rate), the post-collision diagonal receives the cancelling
// source -3 (1 - omega/2) u_a^2 d_a u_a, omega being the shear rate for the deviatoric
// differences and the bulk rate for the trace.
template <class R> struct Rates {
  R tau0;      // nu/cs2 + 1/2 (Eq. 12 read as relaxation time)
  R smag18;    // 18 Cs^2 = 2 Cs^2 / cs2^2
  R wb, wh;    // bulk and higher-order rates
  bool gal;    // Galilean correction of the diagonal second-order cumulants
  bool p4;     // D3Q27: parameterised higher-order relaxation (fourth-order diffusion)
};

template <class R>
__device__ __forceinline__ R shear_rate(const Rates<R> &r, R PiPi) {
  // tau = (tau0 + sqrt(tau0^2 + 2 Cs^2 Qbar / cs2^2)) / 2, Qbar = sqrt(2 Pi:Pi)
  if (r.smag18 == R(0)) return fdiv(R(1), r.tau0);
  const R Qbar = hsqrt(R(2) * PiPi);
  const R tau = R(0.5) * (r.tau0 + hsqrt(r.tau0 * r.tau0 + r.smag18 * Qbar));
  return fdiv(R(1), tau);
}

template <class R>
__device__ __forceinline__ R collide_d2q9(R (&d)[9], R ux, R uy, const Rates<R> &rt) {
  constexpr R s = R(1.0 / 3.0);
  // forward: y sweep on lines x = 0,1,2 (stride 3), then x sweep (stride 1)
#pragma unroll
  for (int a = 0; a < 3; ++a) fwd3(d[a], d[a + 3], d[a + 6], uy);
#pragma unroll
  for (int b = 0; b < 3; ++b) fwd3(d[3 * b], d[3 * b + 1], d[3 * b + 2], ux);
  // kappa^d_ab at d[a + 3b]
  const R ux2 = ux * ux, uy2 = uy * uy;
  const R A = ux2 + d[2], B = uy2 + d[6];
  const R k11 = ux * uy + d[4];
  const R k21 = d[5] - (s + ux2) * uy;
  const R k12 = d[7] - ux * (s + uy2);
  const R c22 = d[8] - s * (d[2] + d[6]) + ux2 * uy2 - A * B - R(2) * k11 * k11;
  const R om = shear_rate(rt, A * A + B * B + R(2) * k11 * k11);
  // relax
  R Dxy = (R(1) - om) * (A - B);
  R Tr = (R(1) - rt.wb) * (A + B);
  if (rt.gal) {
    // d_x u, d_y v = -(3 om / 4) (A - B) -+ ... - (3 wb / 4) (A + B)
    const R dv = R(0.75) * om * (A - B), tv = R(0.75) * rt.wb * (A + B);
    const R Sx = R(-3) * ux2 * (-dv - tv), Sy = R(-3) * uy2 * (dv - tv);
    Dxy += (R(1) - R(0.5) * om) * (Sx - Sy);
    Tr += (R(1) - R(0.5) * rt.wb) * (Sx + Sy);
  }
  const R As = R(0.5) * (Tr + Dxy), Bs = R(0.5) * (Tr - Dxy);
  const R k11s = (R(1) - om) * k11;
  const R h = R(1) - rt.wh;
  const R c21s = h * k21, c12s = h * k12, c22s = h * c22;
  // back to deviation moments (orders 0 and 1 pass through)
  d[2] = As - ux2;
  d[6] = Bs - uy2;
  d[4] = k11s - ux * uy;
  d[5] = c21s + (s + ux2) * uy;
  d[7] = c12s + ux * (s + uy2);
  d[8] = c22s + s * (As - ux2 + Bs - uy2) + As * Bs - ux2 * uy2 + R(2) * k11s * k11s;
#pragma unroll
  for (int b = 0; b < 3; ++b) inv3(d[3 * b], d[3 * b + 1], d[3 * b + 2], ux);
#pragma unroll
  for (int a = 0; a < 3; ++a) inv3(d[a], d[a + 3], d[a + 6], uy);
  return om;
}

// HIGH1: every cumulant of order >= 3 relaxes with rate one, i.e. is set to its
// equilibrium 0; the pre-collision higher-order cumulants are then not needed.
template <class R, bool HIGH1>
__device__ __forceinline__ R collide_d3q27(R (&d)[27], R ux, R uy, R uz, const Rates<R> &rt) {
  constexpr R s = R(1.0 / 3.0);
  // forward sweeps z (stride 9), y (stride 3), x (stride 1); kappa^d_abc at d[a+3b+9c]
#pragma unroll
  for (int j = 0; j < 9; ++j) fwd3(d[j], d[j + 9], d[j + 18], uz);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) fwd3(d[a + 9 * c], d[a + 3 + 9 * c], d[a + 6 + 9 * c], uy);
#pragma unroll
  for (int j = 0; j < 9; ++j) fwd3(d[3 * j], d[3 * j + 1], d[3 * j + 2], ux);

#define KD(a, b, c) d[(a) + 3 * (b) + 9 * (c)]
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R Kx2 = s + ux2, Ky2 = s + uy2, Kz2 = s + uz2;
  // second order (diagonal shifted by cs2)
  const R A = ux2 + KD(2, 0, 0), B = uy2 + KD(0, 2, 0), C = uz2 + KD(0, 0, 2);
  const R k110 = ux * uy + KD(1, 1, 0), k101 = ux * uz + KD(1, 0, 1), k011 = uy * uz + KD(0, 1, 1);
  // third order: kappa = kappa^w + kappa^d (unused when they all relax to zero)
  R k210 = R(0), k201 = R(0), k120 = R(0), k021 = R(0), k102 = R(0), k012 = R(0), k111 = R(0);
  R c211 = R(0), c121 = R(0), c112 = R(0), c220 = R(0), c202 = R(0), c022 = R(0);
  R c221 = R(0), c212 = R(0), c122 = R(0), c222 = R(0);
  const R s2 = s * s;
  if constexpr (!HIGH1) {
  // third order: kappa = kappa^w + kappa^d
    k210 = KD(2, 1, 0) - Kx2 * uy;
    k201 = KD(2, 0, 1) - Kx2 * uz;
    k120 = KD(1, 2, 0) - ux * Ky2;
    k021 = KD(0, 2, 1) - Ky2 * uz;
    k102 = KD(1, 0, 2) - ux * Kz2;
    k012 = KD(0, 1, 2) - uy * Kz2;
    k111 = KD(1, 1, 1) - ux * uy * uz;
    // fourth order cumulants
    c211 = KD(2, 1, 1) - s * KD(0, 1, 1) + ux2 * uy * uz - A * k011 - R(2) * k110 * k101;
    c121 = KD(1, 2, 1) - s * KD(1, 0, 1) + uy2 * ux * uz - B * k101 - R(2) * k110 * k011;
    c112 = KD(1, 1, 2) - s * KD(1, 1, 0) + uz2 * ux * uy - C * k110 - R(2) * k101 * k011;
    c220 = KD(2, 2, 0) - s * (KD(2, 0, 0) + KD(0, 2, 0)) + ux2 * uy2 - A * B - R(2) * k110 * k110;
    c202 = KD(2, 0, 2) - s * (KD(2, 0, 0) + KD(0, 0, 2)) + ux2 * uz2 - A * C - R(2) * k101 * k101;
    c022 = KD(0, 2, 2) - s * (KD(0, 2, 0) + KD(0, 0, 2)) + uy2 * uz2 - B * C - R(2) * k011 * k011;
    // fifth order cumulants
    c221 = KD(2, 2, 1) + uz * (s2 - ux2 * uy2) - s * (KD(0, 2, 1) + KD(2, 0, 1)) - A * k021 -
                 B * k201 - R(4) * k110 * k111 - R(2) * (k101 * k120 + k011 * k210);
    c212 = KD(2, 1, 2) + uy * (s2 - ux2 * uz2) - s * (KD(0, 1, 2) + KD(2, 1, 0)) - A * k012 -
                 C * k210 - R(4) * k101 * k111 - R(2) * (k110 * k102 + k011 * k201);
    c122 = KD(1, 2, 2) + ux * (s2 - uy2 * uz2) - s * (KD(1, 0, 2) + KD(1, 2, 0)) - B * k102 -
                 C * k120 - R(4) * k011 * k111 - R(2) * (k110 * k012 + k101 * k021);
    // sixth order cumulant
    c222 = KD(2, 2, 2) - s2 * (KD(2, 0, 0) + KD(0, 2, 0) + KD(0, 0, 2)) +
                 s * (ux2 * uy2 + uy2 * uz2 + uz2 * ux2 - A * B - B * C - C * A) +
                 ux2 * uy2 * uz2 - A * B * C - (s + A) * c022 - (s + B) * c202 - (s + C) * c220 -
                 R(4) * (k110 * c112 + k101 * c121 + k011 * c211) - R(4) * k111 * k111 -
                 R(2) * (k210 * k012 + k201 * k021 + k120 * k102) -
                 R(2) * ((s + A) * k011 * k011 + (s + B) * k101 * k101 + (s + C) * k110 * k110) -
                 R(8) * k110 * k101 * k011;

  }
  const R om = shear_rate(rt, A * A + B * B + C * C + R(2) * (k110 * k110 + k101 * k101 + k011 * k011));
  // relaxation towards the cumulant equilibria
  const R o1 = R(1) - om, h = HIGH1 ? R(0) : R(1) - rt.wh;
  R Dxy = o1 * (A - B), Dxz = o1 * (A - C);
  R Tr = (R(1) - rt.wb) * (A + B + C);
  if (rt.gal) {
    // d_a u_a = -(om / 2) (3 A_a - tr) - (wb / 2) tr, tr = A + B + C
    const R tr = A + B + C, ho = R(0.5) * om, tb = R(0.5) * rt.wb * tr;
    const R Sx = R(-3) * ux2 * (-ho * (R(3) * A - tr) - tb);
    const R Sy = R(-3) * uy2 * (-ho * (R(3) * B - tr) - tb);
    const R Sz = R(-3) * uz2 * (-ho * (R(3) * C - tr) - tb);
    const R gs = R(1) - ho;
    Dxy += gs * (Sx - Sy);
    Dxz += gs * (Sx - Sz);
    Tr += (R(1) - R(0.5) * rt.wb) * (Sx + Sy + Sz);
  }
  const R As = (Tr + Dxy + Dxz) * R(1.0 / 3.0);
  const R Bs = As - Dxy, Cs = As - Dxz;
  const R q110 = o1 * k110, q101 = o1 * k101, q011 = o1 * k011;
  R q210 = h * k210, q201 = h * k201, q120 = h * k120, q021 = h * k021, q102 = h * k102,
    q012 = h * k012, q111 = h * k111;
  R q211 = h * c211, q121 = h * c121, q112 = h * c112, q220 = h * c220, q202 = h * c202,
    q022 = h * c022;
  R q221 = h * c221, q212 = h * c212, q122 = h * c122, q222 = h * c222;
  if constexpr (!HIGH1) {
    if (rt.p4) {
      // Parameterisation of Geier, Pasquali and Schoenherr (2017) for fourth-order accurate
      // diffusion: third-order rates from the shear rate om and the bulk rate wb (sums
      // C_120 + C_102 and permutations at w3, their differences at w4, C_111 at w5), the
      // fourth-order cumulants set to equilibria proportional to the velocity gradients
      // estimated from the pre-collision second cumulants, fifth and sixth order to zero.
      const R w1 = om, w2 = rt.wb;
      const R w3 = fdiv(R(8) * (w1 - R(2)) * (w2 * (R(3) * w1 - R(1)) - R(5) * w1),
                        R(8) * (R(5) - R(2) * w1) * w1 + w2 * (R(8) + w1 * (R(9) * w1 - R(26))));
      const R w4 = fdiv(R(8) * (w1 - R(2)) * (w1 + w2 * (R(3) * w1 - R(7))),
                        w2 * (R(56) - R(42) * w1 + R(9) * w1 * w1) - R(8) * w1);
      const R w5 = fdiv(R(24) * (w1 - R(2)) *
                            (R(4) * w1 * w1 + w1 * w2 * (R(18) - R(13) * w1) + w2 * w2 * (R(2) + w1 * (R(6) * w1 - R(11)))),
                        R(16) * w1 * w1 * (w1 - R(6)) - R(2) * w1 * w2 * (R(216) + R(5) * w1 * (R(9) * w1 - R(46))) +
                            w2 * w2 * (w1 * (R(3) * w1 - R(10)) * (R(15) * w1 - R(28)) - R(48)));
      const R iden = fdiv(R(1), (w1 - w2) * (w2 * (R(2) + R(3) * w1) - R(8) * w1));
      const R cA = (R(4) * w1 * w1 + R(2) * w1 * w2 * (w1 - R(6)) + w2 * w2 * (w1 * (R(10) - R(3) * w1) - R(4))) * iden;
      const R cB = (R(4) * w1 * w2 * (R(9) * w1 - R(16)) - R(4) * w1 * w1 -
                    R(2) * w2 * w2 * (R(2) + R(9) * w1 * (w1 - R(2)))) * iden * R(1.0 / 3.0);
      const R h3 = R(0.5) * (R(1) - w3), h4 = R(0.5) * (R(1) - w4);
      q120 = h3 * (k120 + k102) + h4 * (k120 - k102);
      q102 = h3 * (k120 + k102) - h4 * (k120 - k102);
      q210 = h3 * (k210 + k012) + h4 * (k210 - k012);
      q012 = h3 * (k210 + k012) - h4 * (k210 - k012);
      q201 = h3 * (k201 + k021) + h4 * (k201 - k021);
      q021 = h3 * (k201 + k021) - h4 * (k201 - k021);
      q111 = (R(1) - w5) * k111;
      // d_a u_a = -(om / 2) (3 A_a - tr) - (wb / 2) tr (tr of the cs2-shifted diagonal);
      // d_a u_b + d_b u_a = -3 om k_ab
      const R tr = A + B + C, ho = R(0.5) * om, tb = R(0.5) * w2 * tr;
      const R dx = -ho * (R(3) * A - tr) - tb, dy = -ho * (R(3) * B - tr) - tb, dz = -ho * (R(3) * C - tr) - tb;
      const R vis = fdiv(R(1), om) - R(0.5);
      const R fa = R(-2.0 / 3.0) * cA * vis, fb = cB * vis * om;   // -(1/3) B vis (-3 om k)
      q220 = fa * (dx + dy);
      q202 = fa * (dx + dz);
      q022 = fa * (dy + dz);
      q112 = fb * k110;
      q121 = fb * k101;
      q211 = fb * k011;
      q221 = q212 = q122 = q222 = R(0);
    }
  }

  // back to deviation central moments: kappa*^d = kappa* - kappa^w
  KD(2, 0, 0) = As - ux2;
  KD(0, 2, 0) = Bs - uy2;
  KD(0, 0, 2) = Cs - uz2;
  KD(1, 1, 0) = q110 - ux * uy;
  KD(1, 0, 1) = q101 - ux * uz;
  KD(0, 1, 1) = q011 - uy * uz;
  if constexpr (HIGH1) {
    // all post-collision cumulants of order >= 3 vanish
    KD(2, 1, 0) = Kx2 * uy;
    KD(2, 0, 1) = Kx2 * uz;
    KD(1, 2, 0) = ux * Ky2;
    KD(0, 2, 1) = Ky2 * uz;
    KD(1, 0, 2) = ux * Kz2;
    KD(0, 1, 2) = uy * Kz2;
    KD(1, 1, 1) = ux * uy * uz;
    KD(2, 1, 1) = s * (q011 - uy * uz) + As * q011 - ux2 * uy * uz + R(2) * q110 * q101;
    KD(1, 2, 1) = s * (q101 - ux * uz) + Bs * q101 - uy2 * ux * uz + R(2) * q110 * q011;
    KD(1, 1, 2) = s * (q110 - ux * uy) + Cs * q110 - uz2 * ux * uy + R(2) * q101 * q011;
    KD(2, 2, 0) = s * (As - ux2 + Bs - uy2) + As * Bs - ux2 * uy2 + R(2) * q110 * q110;
    KD(2, 0, 2) = s * (As - ux2 + Cs - uz2) + As * Cs - ux2 * uz2 + R(2) * q101 * q101;
    KD(0, 2, 2) = s * (Bs - uy2 + Cs - uz2) + Bs * Cs - uy2 * uz2 + R(2) * q011 * q011;
    KD(2, 2, 1) = uz * Kx2 * Ky2;
    KD(2, 1, 2) = uy * Kx2 * Kz2;
    KD(1, 2, 2) = ux * Ky2 * Kz2;
    KD(2, 2, 2) = s2 * (As - ux2 + Bs - uy2 + Cs - uz2) +
                  s * (As * Bs + Bs * Cs + Cs * As - ux2 * uy2 - uy2 * uz2 - uz2 * ux2) +
                  As * Bs * Cs - ux2 * uy2 * uz2 +
                  R(2) * ((s + As) * q011 * q011 + (s + Bs) * q101 * q101 + (s + Cs) * q110 * q110) +
                  R(8) * q110 * q101 * q011;
  } else {
    KD(2, 1, 0) = q210 + Kx2 * uy;
    KD(2, 0, 1) = q201 + Kx2 * uz;
    KD(1, 2, 0) = q120 + ux * Ky2;
    KD(0, 2, 1) = q021 + Ky2 * uz;
    KD(1, 0, 2) = q102 + ux * Kz2;
    KD(0, 1, 2) = q012 + uy * Kz2;
    KD(1, 1, 1) = q111 + ux * uy * uz;
    KD(2, 1, 1) = q211 + s * (q011 - uy * uz) + As * q011 - ux2 * uy * uz + R(2) * q110 * q101;
    KD(1, 2, 1) = q121 + s * (q101 - ux * uz) + Bs * q101 - uy2 * ux * uz + R(2) * q110 * q011;
    KD(1, 1, 2) = q112 + s * (q110 - ux * uy) + Cs * q110 - uz2 * ux * uy + R(2) * q101 * q011;
    KD(2, 2, 0) = q220 + s * (As - ux2 + Bs - uy2) + As * Bs - ux2 * uy2 + R(2) * q110 * q110;
    KD(2, 0, 2) = q202 + s * (As - ux2 + Cs - uz2) + As * Cs - ux2 * uz2 + R(2) * q101 * q101;
    KD(0, 2, 2) = q022 + s * (Bs - uy2 + Cs - uz2) + Bs * Cs - uy2 * uz2 + R(2) * q011 * q011;
    KD(2, 2, 1) = q221 + (s + As) * q021 + (s + Bs) * q201 + R(4) * q110 * q111 +
                  R(2) * (q101 * q120 + q011 * q210) + uz * Kx2 * Ky2;
    KD(2, 1, 2) = q212 + (s + As) * q012 + (s + Cs) * q210 + R(4) * q101 * q111 +
                  R(2) * (q110 * q102 + q011 * q201) + uy * Kx2 * Kz2;
    KD(1, 2, 2) = q122 + (s + Bs) * q102 + (s + Cs) * q120 + R(4) * q011 * q111 +
                  R(2) * (q110 * q012 + q101 * q021) + ux * Ky2 * Kz2;
    KD(2, 2, 2) = q222 + s2 * (As - ux2 + Bs - uy2 + Cs - uz2) +
                  s * (As * Bs + Bs * Cs + Cs * As - ux2 * uy2 - uy2 * uz2 - uz2 * ux2) +
                  As * Bs * Cs - ux2 * uy2 * uz2 + (s + As) * q022 + (s + Bs) * q202 + (s + Cs) * q220 +
                  R(4) * (q110 * q112 + q101 * q121 + q011 * q211) + R(4) * q111 * q111 +
                  R(2) * (q210 * q012 + q201 * q021 + q120 * q102) +
                  R(2) * ((s + As) * q011 * q011 + (s + Bs) * q101 * q101 + (s + Cs) * q110 * q110) +
                  R(8) * q110 * q101 * q011;
  }
#undef KD
  // inverse sweeps x, y, z
#pragma unroll
  for (int j = 0; j < 9; ++j) inv3(d[3 * j], d[3 * j + 1], d[3 * j + 2], ux);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) inv3(d[a + 9 * c], d[a + 3 + 9 * c], d[a + 6 + 9 * c], uy);
#pragma unroll
  for (int j = 0; j < 9; ++j) inv3(d[j], d[j + 9], d[j + 18], uz);
  return om;
}

// Second central moments of the deviation (for the BGK test mode's shear rate).
template <int Q, class R>
__device__ __forceinline__ R pipi_of(const R (&d)[Q], const R (&u)[3]) {
  constexpr int D = Lat<Q>::D;
  R P[3][3];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) P[a][b] = u[a] * u[b];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R c[3] = {R(cx(i)) - u[0], R(cy(i)) - u[1], R(Q == 27 ? cz(i) : 0) - u[2]};
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) P[a][b] += c[a] * c[b] * d[i];
  }
  R s = R(0);
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) s += P[a][b] * P[a][b];
  return s;
}

// ------------------------------------------------------------------------ scalars
// Physics selected by the number of transported scalars: 0 isothermal, 1 passive
// temperature, 2 (T, Y_fuel) one-step, 6 (T, CH4, O2, CO, CO2, H2O) two-step.
template <class R> struct ThermoT {
  R rho_ref, nu_ref, mu_ref, inv_Pr, F, invF;
  int const_mu;          // 1: nu = mu_ref / rho, 0: nu = nu_ref
  R rhoT;                // rho_ref T_ref (one-step: rho = rhoT / T)
  R rhoT_W;              // rho_ref T_ref / W_ref (two-step: rho = rhoT_W W / T)
  R B1, Ta1, B2, Ta2;    // Arrhenius factors and activation temperatures
  R heat1;               // one-step: (T_ad - T_u)/Y_u
  R inv_cp;
  R W[6], inv_W[6], h[6];
  R dinv_W[5];           // 1/W_k - 1/W_N2: 1/W = 1/W_N2 + sum_k Y_k (1/W_k - 1/W_N2)
};


// Mixture-averaged transport for the two-step scalars (species CH4, O2, CO, CO2, H2O, N2):
// binary coefficients D_kj = D0_kj (T/T_ref)^sD / pi, c_p,k = a_k + b_k T, mu ~ T^smu.
template <class R> struct MixT {
  int on;
  R invB[6][6];          // 1/D0_kj (diagonal 0)
  R cpa[6], cpb[6];
  R s_mu, s_D, inv_Tref;
  R hc[6];               // h_k(T) = hc_k + W_k T (a_k + b_k T / 2)
  R in_kap, in_coef[6], in_X[6], in_Y[6];   // the inlet state's transport point
};

// Transport point of a cell state: lambda = mu c_p / Pr, rho D_k W_k/W (Hirschfelder-
// Curtiss D_k = (1 - Y_k)/sum_{j != k} X_j/D_kj), mole and mass fractions; mu and c_p.
template <class R> struct MixPoint {
  R kap, coef[6], X[6], Y[6];
};
template <class R>
__device__ __forceinline__ void mix_point(const MixT<R> &m, const ThermoT<R> &th, const R (&v)[6], R rho, R pi,
                                          MixPoint<R> &o, R &mu, R &cp) {
  R ys = R(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    o.Y[k] = v[1 + k];
    ys += v[1 + k];
  }
  o.Y[5] = R(1) - ys;
  R invW = R(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) invW += o.Y[k] * th.inv_W[k];
  const R W = fdiv(R(1), invW);
#pragma unroll
  for (int k = 0; k < 6; ++k) o.X[k] = o.Y[k] * W * th.inv_W[k];
  const R T = v[0];
  const R lt = hlog2(T * m.inv_Tref);       // (T/T_ref)^s = 2^(s log2(T/T_ref))
  mu = th.mu_ref * hexp2(m.s_mu * lt);
  const R scale = fdiv(hexp2(m.s_D * lt), pi);
  cp = R(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) cp += o.Y[k] * (m.cpa[k] + m.cpb[k] * T);
  o.kap = mu * cp * th.inv_Pr;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    R sum = R(0);
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j != k) sum += o.X[j] * m.invB[k][j];
    o.coef[k] = rho * fdiv((R(1) - o.Y[k]) * scale, sum) * th.W[k] * invW;
  }
}

// Ideal-gas density at the thermodynamic pressure pi P_th(0) (pi = 1 in open domains).
template <int NS, class R>
__device__ __forceinline__ R density(const ThermoT<R> &t, const R (&v)[NS > 0 ? NS : 1], R pi = R(1)) {
  if constexpr (NS <= 1) {
    return t.rho_ref;
  } else if constexpr (NS == 2) {
    return fdiv(t.rhoT * pi, v[0]);
  } else {
    // rho = rho_ref (T_ref/T)(W/W_ref), 1/W = sum Y_k/W_k with N2 by closure
    R inv = t.inv_W[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) inv += v[1 + k] * t.dinv_W[k];
    return fdiv(t.rhoT_W * pi, v[0] * inv);
  }
}

template <class R> __device__ __forceinline__ R viscosity(const ThermoT<R> &t, R rho) {
  return t.const_mu ? fdiv(t.mu_ref, rho) : t.nu_ref;
}
// The same from 1/rho, for the cell whose reciprocal density is at hand.
template <class R> __device__ __forceinline__ R viscosity_irho(const ThermoT<R> &t, R irho) {
  return t.const_mu ? t.mu_ref * irho : t.nu_ref;
}

// Upwind WENO3 derivative across a cell (Jiang-Shu weights: candidates -a/2 + 3b/2 and
// (b + c)/2 of the upwind-biased triple (a, b, c), linear weights 1/3, 2/3, smoothness
// (b-a)^2 and (c-b)^2, alpha = d/(eps + beta)^2) from the upwind neighbours U2, U1, the
// cell value v0 and the downwind neighbour D1: face(U1, v0, D1) - face(U2, U1, v0), with
// the two faces sharing the difference v0 - U1.  Each face value is b + (1/2) q with
// q = (S1 d0 + 2 S0 d1)/(S1 + 2 S0), d0 = b - a, d1 = c - b, S = (eps + d^2)^2.  In FP64
// the two quotients share one division (the product of the denominators stays far inside
// the FP64 range); FP32 keeps two reciprocals, as that product can leave the FP32 range
// for small scalar scales.
template <class R> __device__ __forceinline__ R weno3_diff(R U2, R U1, R v0, R D1, R eps) {
  const R dA = U1 - U2, dB = v0 - U1, dC = D1 - v0;
  const R eA = eps + dA * dA, eB = eps + dB * dB, eC = eps + dC * dC;
  const R SA = eA * eA, SB = eB * eB, SC = eC * eC;
  const R n1 = SC * dB + R(2) * (SB * dC), d1 = SC + R(2) * SB;
  const R n2 = SB * dA + R(2) * (SA * dB), d2 = SB + R(2) * SA;
  if constexpr (sizeof(R) == 8) return dB + R(0.5) * fdiv(n1 * d2 - n2 * d1, d1 * d2);
  else return dB + R(0.5) * (fdiv(n1, d1) - fdiv(n2, d2));
}

}  // namespace lbm
