// Hand-written discrete adjoint of the fused step for periodic D3Q27 flows with an
// optional passive temperature (the differentiation workload): vector-Jacobian products of
// the cumulant collision (higher-order rates one, Smagorinsky shear rate), of the WENO3
// advection and the centred diffusion, and transposed (push) streaming.
//
// Forward map at one cell (iso/passive, rho = rho_ref):
//   E = sum g, m = sum c g, u = mom m,  d = g - w E,
//   kappa = chimera_fwd(d; u),  (A,B,C,k110,k101,k011) = 2nd-order cumulants,
//   omega = Smagorinsky(Pi:Pi),  relax -> (As,Bs,Cs,q110,q101,q011),
//   kappa* = back(As.., q.., u; pass-through orders 0,1),  d* = chimera_inv(kappa*; u),
//   out = w E + d*,
//   T' = T + K lap(T) - sum_d |u_d| W_d(T).
// The reverse pass below differentiates exactly these operations.
#pragma once

#include "lbm_step.hpp"

namespace lbm {

// VJP of one forward 1-D chimera triple (m, z, p; u) -> (k0, k1, k2); the inputs are the
// forward inputs, l* are the adjoints of the outputs on entry and of the inputs on exit.
template <class R>
__device__ __forceinline__ void fwd3_vjp(R m, R z, R p, R u, R &lm, R &lz, R &lp, R &lu) {
  const R sp = p + m, d = p - m;
  const R k0 = sp + z;
  const R k1 = d - u * k0;
  const R lk0 = lm, lk1 = lz, lk2 = lp;
  // k2 = sp - u (d + k1)
  R lsp = lk2, ld = -u * lk2, lk1t = lk1 - u * lk2;
  lu += -(d + k1) * lk2;
  // k1 = d - u k0
  ld += lk1t;
  const R lk0t = lk0 - u * lk1t;
  lu += -k0 * lk1t;
  // k0 = sp + z
  lsp += lk0t;
  lz = lk0t;
  lp = ld + lsp;
  lm = -ld + lsp;
}

// VJP of one inverse 1-D chimera triple (k0, k1, k2; u) -> (f-, f0, f+).
template <class R>
__device__ __forceinline__ void inv3_vjp(R k0, R k1, R /*k2: the outputs are linear in it*/, R u, R &l0, R &l1, R &l2, R &lu) {
  const R m1 = k1 + u * k0;
  const R lminus = l0, lzero = l1, lplus = l2;
  // f0 = k0 - m2, f+ = m2/2 + m1/2, f- = m2/2 - m1/2
  const R lm2 = -lzero + R(0.5) * (lplus + lminus);
  R lm1 = R(0.5) * (lplus - lminus);
  // m2 = k2 + u (k1 + m1)
  const R lk2 = lm2;
  R lk1 = u * lm2;
  lm1 += u * lm2;
  lu += (k1 + m1) * lm2;
  // m1 = k1 + u k0
  lk1 += lm1;
  const R lk0 = lzero + u * lm1;
  lu += k0 * lm1;
  l0 = lk0; l1 = lk1; l2 = lk2;
}

template <class R> __device__ __forceinline__ void sweep_fwd(R (&d)[27], int axis, R u) {
  if (axis == 2) {
#pragma unroll
    for (int j = 0; j < 9; ++j) fwd3(d[j], d[j + 9], d[j + 18], u);
  } else if (axis == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) fwd3(d[a + 9 * c], d[a + 3 + 9 * c], d[a + 6 + 9 * c], u);
  } else {
#pragma unroll
    for (int j = 0; j < 9; ++j) fwd3(d[3 * j], d[3 * j + 1], d[3 * j + 2], u);
  }
}
template <class R> __device__ __forceinline__ void sweep_inv(R (&d)[27], int axis, R u) {
  if (axis == 2) {
#pragma unroll
    for (int j = 0; j < 9; ++j) inv3(d[j], d[j + 9], d[j + 18], u);
  } else if (axis == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) inv3(d[a + 9 * c], d[a + 3 + 9 * c], d[a + 6 + 9 * c], u);
  } else {
#pragma unroll
    for (int j = 0; j < 9; ++j) inv3(d[3 * j], d[3 * j + 1], d[3 * j + 2], u);
  }
}
// adjoint of a sweep given the sweep's inputs x; l holds output adjoints -> input adjoints
template <class R>
__device__ __forceinline__ void sweep_fwd_vjp(const R (&x)[27], R (&l)[27], int axis, R u, R &lu) {
  if (axis == 2) {
#pragma unroll
    for (int j = 0; j < 9; ++j) fwd3_vjp(x[j], x[j + 9], x[j + 18], u, l[j], l[j + 9], l[j + 18], lu);
  } else if (axis == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int i0 = a + 9 * c;
        fwd3_vjp(x[i0], x[i0 + 3], x[i0 + 6], u, l[i0], l[i0 + 3], l[i0 + 6], lu);
      }
  } else {
#pragma unroll
    for (int j = 0; j < 9; ++j)
      fwd3_vjp(x[3 * j], x[3 * j + 1], x[3 * j + 2], u, l[3 * j], l[3 * j + 1], l[3 * j + 2], lu);
  }
}
template <class R>
__device__ __forceinline__ void sweep_inv_vjp(const R (&x)[27], R (&l)[27], int axis, R u, R &lu) {
  if (axis == 2) {
#pragma unroll
    for (int j = 0; j < 9; ++j) inv3_vjp(x[j], x[j + 9], x[j + 18], u, l[j], l[j + 9], l[j + 18], lu);
  } else if (axis == 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int i0 = a + 9 * c;
        inv3_vjp(x[i0], x[i0 + 3], x[i0 + 6], u, l[i0], l[i0 + 3], l[i0 + 6], lu);
      }
  } else {
#pragma unroll
    for (int j = 0; j < 9; ++j)
      inv3_vjp(x[3 * j], x[3 * j + 1], x[3 * j + 2], u, l[3 * j], l[3 * j + 1], l[3 * j + 2], lu);
  }
}

// Reverse pass of the D3Q27 cumulant collision with every order >= 3 at rate one.
// g: pre-collision deviations ghat (27), u = mom * sum c g; lam: on entry the adjoint of
// the post-collision ghat*, on exit the adjoint of ghat (through E, u and d).  lu_extra
// carries adjoints of u from elsewhere (the scalar advection) and is folded in.
template <class R>
__device__ void collide_d3q27_vjp(const R (&g)[27], R mom, const Rates<R> &rt, R (&lam)[27], const R (&lu_extra)[3]) {
  constexpr R s = R(1.0 / 3.0);
  const R s2 = s * s;
  // ---------------- forward recompute
  R E = R(0), mx = R(0), my = R(0), mz = R(0);
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    E += g[i];
    if (cx(i)) mx += R(cx(i)) * g[i];
    if (cy(i)) my += R(cy(i)) * g[i];
    if (cz(i)) mz += R(cz(i)) * g[i];
  }
  const R ux = mx * mom, uy = my * mom, uz = mz * mom;
  R dv[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) dv[i] = g[i] - R(wgt<27>(i)) * E;
  R k[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) k[i] = dv[i];
  sweep_fwd(k, 2, uz);
  sweep_fwd(k, 1, uy);
  sweep_fwd(k, 0, ux);
#define KI(a, b, c) ((a) + 3 * (b) + 9 * (c))
  const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const R Kx2 = s + ux2, Ky2 = s + uy2, Kz2 = s + uz2;
  const R A = ux2 + k[KI(2, 0, 0)], B = uy2 + k[KI(0, 2, 0)], C = uz2 + k[KI(0, 0, 2)];
  const R k110 = ux * uy + k[KI(1, 1, 0)], k101 = ux * uz + k[KI(1, 0, 1)], k011 = uy * uz + k[KI(0, 1, 1)];
  const R PiPi = A * A + B * B + C * C + R(2) * (k110 * k110 + k101 * k101 + k011 * k011);
  // shear rate and its derivative with respect to Pi:Pi
  R om, dom_dP = R(0);
  if (rt.smag18 == R(0)) {
    om = fdiv(R(1), rt.tau0);
  } else {
    const R Qb = sqrt(R(2) * PiPi);
    const R R2 = sqrt(rt.tau0 * rt.tau0 + rt.smag18 * Qb);
    const R tau = R(0.5) * (rt.tau0 + R2);
    om = fdiv(R(1), tau);
    // d omega/d PiPi = -1/tau^2 * smag18 / (4 R2) * 1/Qb  (zero where Pi vanishes)
    if (Qb > R(0)) dom_dP = -om * om * fdiv(rt.smag18, R(4) * R2 * Qb);
  }
  const R o1 = R(1) - om, ob = R(1) - rt.wb;
  const R Dxy = o1 * (A - B), Dxz = o1 * (A - C);
  const R Tr = ob * (A + B + C);
  const R As = (Tr + Dxy + Dxz) * R(1.0 / 3.0);
  const R Bs = As - Dxy, Cs = As - Dxz;
  const R q110 = o1 * k110, q101 = o1 * k101, q011 = o1 * k011;
  // post-collision central moments (deviation part) kappa*
  R ks[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) ks[i] = k[i];        // orders 0 and 1 pass through
  ks[KI(2, 0, 0)] = As - ux2;
  ks[KI(0, 2, 0)] = Bs - uy2;
  ks[KI(0, 0, 2)] = Cs - uz2;
  ks[KI(1, 1, 0)] = q110 - ux * uy;
  ks[KI(1, 0, 1)] = q101 - ux * uz;
  ks[KI(0, 1, 1)] = q011 - uy * uz;
  ks[KI(2, 1, 0)] = Kx2 * uy;
  ks[KI(2, 0, 1)] = Kx2 * uz;
  ks[KI(1, 2, 0)] = ux * Ky2;
  ks[KI(0, 2, 1)] = Ky2 * uz;
  ks[KI(1, 0, 2)] = ux * Kz2;
  ks[KI(0, 1, 2)] = uy * Kz2;
  ks[KI(1, 1, 1)] = ux * uy * uz;
  ks[KI(2, 1, 1)] = s * (q011 - uy * uz) + As * q011 - ux2 * uy * uz + R(2) * q110 * q101;
  ks[KI(1, 2, 1)] = s * (q101 - ux * uz) + Bs * q101 - uy2 * ux * uz + R(2) * q110 * q011;
  ks[KI(1, 1, 2)] = s * (q110 - ux * uy) + Cs * q110 - uz2 * ux * uy + R(2) * q101 * q011;
  ks[KI(2, 2, 0)] = s * (As - ux2 + Bs - uy2) + As * Bs - ux2 * uy2 + R(2) * q110 * q110;
  ks[KI(2, 0, 2)] = s * (As - ux2 + Cs - uz2) + As * Cs - ux2 * uz2 + R(2) * q101 * q101;
  ks[KI(0, 2, 2)] = s * (Bs - uy2 + Cs - uz2) + Bs * Cs - uy2 * uz2 + R(2) * q011 * q011;
  ks[KI(2, 2, 1)] = uz * Kx2 * Ky2;
  ks[KI(2, 1, 2)] = uy * Kx2 * Kz2;
  ks[KI(1, 2, 2)] = ux * Ky2 * Kz2;
  ks[KI(2, 2, 2)] = s2 * (As - ux2 + Bs - uy2 + Cs - uz2) +
                    s * (As * Bs + Bs * Cs + Cs * As - ux2 * uy2 - uy2 * uz2 - uz2 * ux2) +
                    As * Bs * Cs - ux2 * uy2 * uz2 +
                    R(2) * ((s + As) * q011 * q011 + (s + Bs) * q101 * q101 + (s + Cs) * q110 * q110) +
                    R(8) * q110 * q101 * q011;

  // ---------------- reverse
  R lE = R(0), lux = lu_extra[0], luy = lu_extra[1], luz = lu_extra[2];
  // out = w E + d*
#pragma unroll
  for (int i = 0; i < 27; ++i) lE += R(wgt<27>(i)) * lam[i];
  // d* = inv_z(inv_y(inv_x(kappa*))): reverse z, y, x with recomputed stage inputs
  {
    R t[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) t[i] = ks[i];
    sweep_inv(t, 0, ux);
    sweep_inv(t, 1, uy);                               // t = input of the z sweep
    sweep_inv_vjp(t, lam, 2, uz, luz);
#pragma unroll
    for (int i = 0; i < 27; ++i) t[i] = ks[i];
    sweep_inv(t, 0, ux);                               // t = input of the y sweep
    sweep_inv_vjp(t, lam, 1, uy, luy);
    sweep_inv_vjp(ks, lam, 0, ux, lux);                // lam = adjoint of kappa*
  }
  // kappa* as functions of (As, Bs, Cs, q110, q101, q011, u); orders 0, 1 pass through
  R lAs = R(0), lBs = R(0), lCs = R(0), lq110 = R(0), lq101 = R(0), lq011 = R(0);
  {
    R l;
    l = lam[KI(2, 0, 0)]; lAs += l; lux -= R(2) * ux * l;
    l = lam[KI(0, 2, 0)]; lBs += l; luy -= R(2) * uy * l;
    l = lam[KI(0, 0, 2)]; lCs += l; luz -= R(2) * uz * l;
    l = lam[KI(1, 1, 0)]; lq110 += l; lux -= uy * l; luy -= ux * l;
    l = lam[KI(1, 0, 1)]; lq101 += l; lux -= uz * l; luz -= ux * l;
    l = lam[KI(0, 1, 1)]; lq011 += l; luy -= uz * l; luz -= uy * l;
    l = lam[KI(2, 1, 0)]; lux += R(2) * ux * uy * l; luy += Kx2 * l;
    l = lam[KI(2, 0, 1)]; lux += R(2) * ux * uz * l; luz += Kx2 * l;
    l = lam[KI(1, 2, 0)]; luy += R(2) * uy * ux * l; lux += Ky2 * l;
    l = lam[KI(0, 2, 1)]; luy += R(2) * uy * uz * l; luz += Ky2 * l;
    l = lam[KI(1, 0, 2)]; luz += R(2) * uz * ux * l; lux += Kz2 * l;
    l = lam[KI(0, 1, 2)]; luz += R(2) * uz * uy * l; luy += Kz2 * l;
    l = lam[KI(1, 1, 1)]; lux += uy * uz * l; luy += ux * uz * l; luz += ux * uy * l;
    // 211: s(q011 - uy uz) + As q011 - ux2 uy uz + 2 q110 q101
    l = lam[KI(2, 1, 1)];
    lq011 += (s + As) * l; lAs += q011 * l; lq110 += R(2) * q101 * l; lq101 += R(2) * q110 * l;
    lux -= R(2) * ux * uy * uz * l; luy -= (s + ux2) * uz * l; luz -= (s + ux2) * uy * l;
    // 121: s(q101 - ux uz) + Bs q101 - uy2 ux uz + 2 q110 q011
    l = lam[KI(1, 2, 1)];
    lq101 += (s + Bs) * l; lBs += q101 * l; lq110 += R(2) * q011 * l; lq011 += R(2) * q110 * l;
    luy -= R(2) * uy * ux * uz * l; lux -= (s + uy2) * uz * l; luz -= (s + uy2) * ux * l;
    // 112: s(q110 - ux uy) + Cs q110 - uz2 ux uy + 2 q101 q011
    l = lam[KI(1, 1, 2)];
    lq110 += (s + Cs) * l; lCs += q110 * l; lq101 += R(2) * q011 * l; lq011 += R(2) * q101 * l;
    luz -= R(2) * uz * ux * uy * l; lux -= (s + uz2) * uy * l; luy -= (s + uz2) * ux * l;
    // 220: s(As - ux2 + Bs - uy2) + As Bs - ux2 uy2 + 2 q110^2
    l = lam[KI(2, 2, 0)];
    lAs += (s + Bs) * l; lBs += (s + As) * l; lq110 += R(4) * q110 * l;
    lux -= R(2) * ux * (s + uy2) * l; luy -= R(2) * uy * (s + ux2) * l;
    // 202
    l = lam[KI(2, 0, 2)];
    lAs += (s + Cs) * l; lCs += (s + As) * l; lq101 += R(4) * q101 * l;
    lux -= R(2) * ux * (s + uz2) * l; luz -= R(2) * uz * (s + ux2) * l;
    // 022
    l = lam[KI(0, 2, 2)];
    lBs += (s + Cs) * l; lCs += (s + Bs) * l; lq011 += R(4) * q011 * l;
    luy -= R(2) * uy * (s + uz2) * l; luz -= R(2) * uz * (s + uy2) * l;
    // 221: uz Kx2 Ky2 ; 212: uy Kx2 Kz2 ; 122: ux Ky2 Kz2
    l = lam[KI(2, 2, 1)];
    luz += Kx2 * Ky2 * l; lux += R(2) * ux * uz * Ky2 * l; luy += R(2) * uy * uz * Kx2 * l;
    l = lam[KI(2, 1, 2)];
    luy += Kx2 * Kz2 * l; lux += R(2) * ux * uy * Kz2 * l; luz += R(2) * uz * uy * Kx2 * l;
    l = lam[KI(1, 2, 2)];
    lux += Ky2 * Kz2 * l; luy += R(2) * uy * ux * Kz2 * l; luz += R(2) * uz * ux * Ky2 * l;
    // 222
    l = lam[KI(2, 2, 2)];
    lAs += (s2 + s * (Bs + Cs) + Bs * Cs + R(2) * q011 * q011) * l;
    lBs += (s2 + s * (As + Cs) + As * Cs + R(2) * q101 * q101) * l;
    lCs += (s2 + s * (As + Bs) + As * Bs + R(2) * q110 * q110) * l;
    lq011 += (R(4) * (s + As) * q011 + R(8) * q110 * q101) * l;
    lq101 += (R(4) * (s + Bs) * q101 + R(8) * q110 * q011) * l;
    lq110 += (R(4) * (s + Cs) * q110 + R(8) * q101 * q011) * l;
    lux -= R(2) * ux * (s2 + s * (uy2 + uz2) + uy2 * uz2) * l;
    luy -= R(2) * uy * (s2 + s * (ux2 + uz2) + ux2 * uz2) * l;
    luz -= R(2) * uz * (s2 + s * (ux2 + uy2) + ux2 * uy2) * l;
  }
  // relaxation: As = (Tr + Dxy + Dxz)/3, Bs = As - Dxy, Cs = As - Dxz, q = o1 k
  const R lAt = lAs + lBs + lCs;
  const R lDxy = lAt * R(1.0 / 3.0) - lBs, lDxz = lAt * R(1.0 / 3.0) - lCs, lTr = lAt * R(1.0 / 3.0);
  R lA = o1 * (lDxy + lDxz) + ob * lTr;
  R lB = -o1 * lDxy + ob * lTr;
  R lC = -o1 * lDxz + ob * lTr;
  R lk110 = o1 * lq110, lk101 = o1 * lq101, lk011 = o1 * lq011;
  const R lo1 = (A - B) * lDxy + (A - C) * lDxz + k110 * lq110 + k101 * lq101 + k011 * lq011;
  // o1 = 1 - omega(PiPi)
  const R lP = -lo1 * dom_dP;
  lA += R(2) * A * lP;
  lB += R(2) * B * lP;
  lC += R(2) * C * lP;
  lk110 += R(4) * k110 * lP;
  lk101 += R(4) * k101 * lP;
  lk011 += R(4) * k011 * lP;
  // second-order cumulants from kappa^d and u
  R lk[27];
#pragma unroll
  for (int i = 0; i < 27; ++i) lk[i] = R(0);
  lk[KI(0, 0, 0)] = lam[KI(0, 0, 0)];
  lk[KI(1, 0, 0)] = lam[KI(1, 0, 0)];
  lk[KI(0, 1, 0)] = lam[KI(0, 1, 0)];
  lk[KI(0, 0, 1)] = lam[KI(0, 0, 1)];
  lk[KI(2, 0, 0)] = lA; lux += R(2) * ux * lA;
  lk[KI(0, 2, 0)] = lB; luy += R(2) * uy * lB;
  lk[KI(0, 0, 2)] = lC; luz += R(2) * uz * lC;
  lk[KI(1, 1, 0)] = lk110; lux += uy * lk110; luy += ux * lk110;
  lk[KI(1, 0, 1)] = lk101; lux += uz * lk101; luz += ux * lk101;
  lk[KI(0, 1, 1)] = lk011; luy += uz * lk011; luz += uy * lk011;
#undef KI
  // kappa = fwd_x(fwd_y(fwd_z(d))): reverse x, y, z with recomputed stage inputs
  {
    R t[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) t[i] = dv[i];
    sweep_fwd(t, 2, uz);
    sweep_fwd(t, 1, uy);                               // input of the x sweep
    sweep_fwd_vjp(t, lk, 0, ux, lux);
#pragma unroll
    for (int i = 0; i < 27; ++i) t[i] = dv[i];
    sweep_fwd(t, 2, uz);                               // input of the y sweep
    sweep_fwd_vjp(t, lk, 1, uy, luy);
    sweep_fwd_vjp(dv, lk, 2, uz, luz);                 // lk = adjoint of d
  }
  // d = g - w E ; E = sum g ; u = mom sum c g
  R lsum = R(0);
#pragma unroll
  for (int i = 0; i < 27; ++i) lsum += R(wgt<27>(i)) * lk[i];
  lE -= lsum;
  const R mlx = mom * lux, mly = mom * luy, mlz = mom * luz;
#pragma unroll
  for (int i = 0; i < 27; ++i) lam[i] = lk[i] + lE + R(cx(i)) * mlx + R(cy(i)) * mly + R(cz(i)) * mlz;
}

// Forward value and partial derivatives of the WENO3 pair difference weno3_diff with
// respect to (U2, U1, v0, D1).
template <class R>
__device__ __forceinline__ R weno3_diff_grad(R U2, R U1, R v0, R D1, R eps, R (&dW)[4]) {
  const R dA = U1 - U2, dB = v0 - U1, dC = D1 - v0;
  const R eA = eps + dA * dA, eB = eps + dB * dB, eC = eps + dC * dC;
  const R SA = eA * eA, SB = eB * eB, SC = eC * eC;
  const R M1 = SC + R(2) * SB, M2 = SB + R(2) * SA;
  const R iM1 = fdiv(R(1), M1), iM2 = fdiv(R(1), M2);
  const R q1 = (SC * dB + R(2) * (SB * dC)) * iM1;
  const R q2 = (SB * dA + R(2) * (SA * dB)) * iM2;
  // q1(SC, SB, dB, dC), q2(SB, SA, dA, dB); dS/dd = 4 e d
  const R dq1_dSC = (dB - q1) * iM1, dq1_dSB = R(2) * (dC - q1) * iM1;
  const R dq2_dSB = (dA - q2) * iM2, dq2_dSA = R(2) * (dB - q2) * iM2;
  const R gA = -R(0.5) * (SB * iM2 + dq2_dSA * R(4) * eA * dA);
  const R gB = R(1) + R(0.5) * (SC * iM1 + dq1_dSB * R(4) * eB * dB) -
               R(0.5) * (R(2) * SA * iM2 + dq2_dSB * R(4) * eB * dB);
  const R gC = R(0.5) * (R(2) * SB * iM1 + dq1_dSC * R(4) * eC * dC);
  dW[0] = -gA;          // U2
  dW[1] = gA - gB;      // U1
  dW[2] = gB - gC;      // v0
  dW[3] = gC;           // D1
  return dB + R(0.5) * (q1 - q2);
}

}  // namespace lbm
