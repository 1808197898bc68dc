// Fused time-step kernel of the hybrid LB/FD scheme (one thread per cell) and the
// auxiliary kernels (geometry words, equilibrium initialisation, FP64 sum finalisation).
//
// Per fluid cell, in one pass:
//   scalars at the cell and its axis neighbours (ghost rules at walls, inlet, outlet)
//   -> rho (ideal gas), grad rho, diffusion + reaction right-hand sides, Lambda (Eq. 3)
//   -> pull-streaming of the Q populations with boundary substitutions (Eq. 1)
//   -> moments P_h, u (Eq. 7) -> WENO3 advection, explicit Euler scalar update (Sec. 2.3)
//   -> source Xi (Eq. 2) -> pre-conditioning (Eq. 13) -> cumulant collision (Eqs. 9-12,
//      optionally with Geier's Galilean correction)
//   -> post-collision populations (Eq. 8) stored as deviations from the lattice weights
//   -> FP64 block partial sums (wavefront shuffles + LDS), one record per block.
// In a closed domain the thermodynamic pressure P_th = pi P_th(0) scales the ideal-gas
// density, its rate q = dln(pi)/dt adds the pressure work kappa T q to the temperature
// right-hand side and shifts Lambda to the velocity divergence Lambda - q, and the
// finalisation of the sums sets pi for the next step from the mass the domain holds.
// With a signed wall distance bound (curved walls), links from solid cells use the
// linearly interpolated bounce-back and scalar stencil points in solid cells take the
// value at their mirror image about the wall (boundary cells only).
#pragma once

#include <type_traits>

#include "lbm_device.hpp"

namespace lbm {

// Per-block FP64 sums: rho, P_h, rho u (3), rho |u|^2/2, W/T, rho Y_1 at level n, and
// W/T of the updated scalars (level n+1; formed in closed domains only).
constexpr int NSUM = 9;
// collision operator compiled into a step instance
enum : int { COLL_CUM1 = 0, COLL_CUM = 1, COLL_BGK = 2 };
// cells a step instance updates: every cell (64x4 tile grid when it fits, else linear
// 256-cell tiles), the interior cells only (the code of boundaries, solids and curved walls
// is not compiled in; on the tile grid, where a wave's y and z are scalars, or on linear
// tiles for grids the tiles do not fit), or the cells of a list (one thread per listed
// cell: the cells the interior instance leaves)
enum : int { MODE_ALL = 0, MODE_INTERIOR = 1, MODE_LIST = 2, MODE_INTERIOR_LIN = 3 };

// Host-side description of one launch (double precision constants).
struct Thermo {
  double rho_ref, T_ref, nu_ref, inv_Pr, F, visc_const_mu;
  double chem[32];
};

struct StepArgs {
  const void *pop_in;
  void *pop_out;
  const void *scal_in;
  void *scal_out;
  const void *geom;    // per-cell geometry words or nullptr
  double *partials;    // [nblocks][NSUM]
  int *flag;           // bit 0: non-finite value seen
  const double *thermo;  // closed domain: device (pi, q, K); nullptr when P_th is constant
  double kappa;        // (gamma - 1)/gamma
  const double *lvl;   // signed wall distance per node (curved walls) or nullptr
  double *stats;       // running statistics [2(D+1)][N] (means, then sums of squared
                       // deviations) of u_d and P_h - P0, or nullptr when not sampled
  double inv_k;        // 1/k for the k-th sample
  double *probe_out;   // row of this level in the probe record ([nprobe][D+1]) or nullptr
  int nprobe;
  int probe[8];        // probe cells
  int mix;             // mixture-averaged transport (two-step scalars)
  double transport[32];  // binary D0 (15), c_p a_k (6), b_k (6), exponents of mu and D
  double mix_in[19];   // inlet transport point: lambda, rho D_k W_k/W (6), X_k (6), Y_k (6)
  double *f_P, *f_rho, *f_u, *f_scal;   // field outputs (extract mode)
  const int *cells;    // MODE_LIST: linear indices of the cells to update
  int ncells;
  int nx, ny, nz;
  long long N;
  int face[6];         // ST_* code of each face, -1 for periodic
  long long step;
  int collision;       // 0 cumulant, 1 BGK
  int gal;             // Galilean correction of the cumulant collision
  int p4;              // D3Q27 parameterised higher-order relaxation (fourth-order diffusion)
  int remap;           // XCD-aware block order
  int band_rows;       // 0: linear 256-cell tiles; else 64x4 tiles in bands of this many rows
  int pull_cached;     // production instance with cached pull loads (else streaming loads)
  double P0;           // rho_ref cs2
  double wb, wh, smag18;
  double inlet_u[3], inlet_noise, outlet_P;
  double phi_in[8];    // inlet scalars
  double eps[8];       // WENO eps per scalar
  unsigned long long seed;
  Thermo th;
};

// Kernel arguments with every floating constant already in the compute precision R, so
// that the kernel reads uniform values straight from the argument segment.
template <class R> struct KArgs {
  const void *pop_in;
  void *pop_out;
  const void *scal_in;
  void *scal_out;
  const void *geom;
  double *partials;
  int *flag;
  const double *thermo;
  const double *lvl;
  double *stats;
  double inv_k;
  double *probe_out;
  int nprobe;
  int probe[8];
  double *f_P, *f_rho, *f_u, *f_scal;
  const int *cells;
  int ncells;
  int nx, ny, nz, N;
  int face[6];
  long long step;
  int collision, remap, band_rows, gal, p4;
  int big;             // a population copy exceeds the 256 MB Infinity Cache
  R P0, invP0, wb, wh, smag18, kap;
  R inlet_u[3], outlet_P;
  double inlet_noise;
  R phi_in[8], eps[8];
  unsigned long long seed;
  double inv_T_ref_d, W_d[6];
  double P0d;          // P0 in FP64 (field outputs and sums of P_h)
  ThermoT<R> th;
  MixT<R> mx;
};

template <class R> KArgs<R> to_kargs(const StepArgs &a) {
  KArgs<R> k;
  k.pop_in = a.pop_in; k.pop_out = a.pop_out; k.scal_in = a.scal_in; k.scal_out = a.scal_out;
  k.geom = a.geom; k.partials = a.partials; k.flag = a.flag; k.thermo = a.thermo; k.lvl = a.lvl;
  k.stats = a.stats; k.inv_k = a.inv_k; k.probe_out = a.probe_out; k.nprobe = a.nprobe;
  for (int j = 0; j < 8; ++j) k.probe[j] = a.probe[j];
  k.kap = (R)a.kappa;
  k.f_P = a.f_P; k.f_rho = a.f_rho; k.f_u = a.f_u; k.f_scal = a.f_scal;
  k.cells = a.cells; k.ncells = a.ncells;
  k.nx = a.nx; k.ny = a.ny; k.nz = a.nz; k.N = (int)a.N;
  for (int f = 0; f < 6; ++f) k.face[f] = a.face[f];
  k.step = a.step; k.collision = a.collision; k.remap = a.remap; k.band_rows = a.band_rows;
  k.big = a.pull_cached;
  k.gal = a.gal;
  k.p4 = a.p4;
  k.P0 = (R)a.P0; k.invP0 = (R)(1.0 / a.P0); k.wb = (R)a.wb; k.wh = (R)a.wh; k.smag18 = (R)a.smag18;
  for (int d = 0; d < 3; ++d) k.inlet_u[d] = (R)a.inlet_u[d];
  k.outlet_P = (R)a.outlet_P; k.inlet_noise = a.inlet_noise;
  for (int q = 0; q < 8; ++q) { k.phi_in[q] = (R)a.phi_in[q]; k.eps[q] = (R)a.eps[q]; }
  k.seed = a.seed;
  const double *ch = a.th.chem;
  k.inv_T_ref_d = 1.0 / a.th.T_ref;
  k.P0d = a.P0;
  for (int q = 0; q < 6; ++q) k.W_d[q] = ch[5 + q] > 0.0 ? ch[5 + q] : 1.0;
  ThermoT<R> &t = k.th;
  t.rho_ref = (R)a.th.rho_ref; t.nu_ref = (R)a.th.nu_ref; t.mu_ref = (R)(a.th.nu_ref * a.th.rho_ref);
  t.inv_Pr = (R)a.th.inv_Pr; t.F = (R)a.th.F; t.invF = (R)(1.0 / a.th.F);
  t.const_mu = a.th.visc_const_mu != 0.0;
  t.rhoT = (R)(a.th.rho_ref * a.th.T_ref);
  t.rhoT_W = (R)(ch[17] > 0.0 ? a.th.rho_ref * a.th.T_ref / ch[17] : 0.0);
  t.B1 = (R)ch[0]; t.Ta1 = (R)ch[1]; t.B2 = (R)ch[2]; t.Ta2 = (R)ch[3];
  t.heat1 = (R)(ch[4] > 0.0 ? (ch[3] - ch[2]) / ch[4] : 0.0);
  t.inv_cp = (R)(ch[4] > 0.0 ? 1.0 / ch[4] : 0.0);
  for (int q = 0; q < 6; ++q) {
    t.W[q] = (R)ch[5 + q];
    t.inv_W[q] = (R)(ch[5 + q] > 0.0 ? 1.0 / ch[5 + q] : 0.0);
    t.h[q] = (R)ch[11 + q];
  }
  for (int q = 0; q < 5; ++q)
    t.dinv_W[q] = (R)(ch[5 + q] > 0.0 && ch[10] > 0.0 ? 1.0 / ch[5 + q] - 1.0 / ch[10] : 0.0);
  MixT<R> &m = k.mx;
  m.on = a.mix;
  const double *tr = a.transport;
  for (int i = 0, n = 0; i < 6; ++i) {
    m.invB[i][i] = R(0);
    for (int j = i + 1; j < 6; ++j, ++n) m.invB[i][j] = m.invB[j][i] = (R)(tr[n] > 0.0 ? 1.0 / tr[n] : 0.0);
  }
  const double T0 = 298.15;     // reference temperature of the formation enthalpies
  for (int q = 0; q < 6; ++q) {
    m.cpa[q] = (R)tr[15 + q];
    m.cpb[q] = (R)tr[21 + q];
    m.hc[q] = (R)(ch[11 + q] - ch[5 + q] * (tr[15 + q] * T0 + 0.5 * tr[21 + q] * T0 * T0));
  }
  m.s_mu = (R)tr[27];
  m.s_D = (R)tr[28];
  m.inv_Tref = (R)(1.0 / a.th.T_ref);
  m.in_kap = (R)a.mix_in[0];
  for (int q = 0; q < 6; ++q) {
    m.in_coef[q] = (R)a.mix_in[1 + q];
    m.in_X[q] = (R)a.mix_in[7 + q];
    m.in_Y[q] = (R)a.mix_in[13 + q];
  }
  return k;
}

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
    // extents of one cell: wrap a second time (|k| <= 2), no division
    if (code < 0) {
      if (p < 0) p += n;
      if (p >= n) p -= n;
    }
    r.idx[k + 2] = code < 0 ? p : c;
    r.code[k + 2] = code;
  }
  return r;
}

// Offsets (times the axis stride) and face codes of positions c-2..c+2 on one axis; cells at
// least two away from both ends take the plain offsets without any wrap logic.
__device__ __forceinline__ void axis_offsets(int c, int n, int flo, int fhi, int stride, int (&off)[5],
                                             int (&code)[5]) {
  if (c >= 2 && c < n - 2) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      off[k] = (k - 2) * stride;
      code[k] = -1;
    }
  } else if (flo < 0 && fhi < 0) {
    // periodic axis: the wrap alone, by selects (twice, for extents of one cell)
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      int p = c + k - 2;
      p += p < 0 ? n : 0;
      p -= p >= n ? n : 0;
      p += p < 0 ? n : 0;
      p -= p >= n ? n : 0;
      off[k] = (p - c) * stride;
      code[k] = -1;
    }
  } else {
    const AxisNb A = axis_nb(c, n, flo, fhi);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      off[k] = (A.idx[k] - c) * stride;
      code[k] = A.code[k];
    }
  }
}

// A cell needs the general (boundary) code when its geometry word is not zero (it is
// solid, or a solid lies within its links or its +-2 stencil) or a non-periodic face lies
// within two cells on some axis; every other cell is interior.  The host builds the list
// of general cells with the same rule (lbm_capi.hip), so the interior and list instances
// of a step cover every cell exactly once.
__device__ __forceinline__ bool near_face(int c, int n, int flo, int fhi) {
  return (flo >= 0 && c < 2) || (fhi >= 0 && c >= n - 2);
}

// Element access through a wave-uniform base pointer and a 32-bit byte offset, so that
// the compiler can address with the scalar base + vector offset form.
template <class T> __device__ __forceinline__ T ldg(const T *base, unsigned idx) {
  return *(const T *)((const char *)base + idx * (unsigned)sizeof(T));
}
template <class T> __device__ __forceinline__ void stg(T *base, unsigned idx, T v) {
  *(T *)((char *)base + idx * (unsigned)sizeof(T)) = v;
}

// Raw buffer access: one descriptor (SGPRs) per array slice (a population or a scalar
// field, under 4 GiB since Q N < 2^31 elements) and a 32-bit byte offset per lane, so the
// neighbours of a cell share offset registers and no load needs 64-bit address arithmetic.
// AUX 2 marks a streaming (non-temporal) access.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slice(const void *p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, -1, 0x00020000);
}
template <class T, int AUX = 0> __device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, unsigned idx) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8u, 0, AUX));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4u, 0, AUX));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, idx * 2u, 0, AUX));
}
template <class T, int AUX = 0> __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned idx, T v) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, idx * 8u, 0, AUX);
  else if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, idx * 4u, 0, AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, idx * 2u, 0, AUX);
}

// (1 - p) a + p b, exact at p = 0 and p = 1.
template <class R> __device__ __forceinline__ R lerp(R a, R b, R p) { return (R(1) - p) * a + p * b; }

// Interpolation weight toward the second node for a mirror image at distance p <= 1 from
// the first fluid node: p itself, or, for an image between the wall and that node
// (p < 0), the even quadratic through the two nodes (zero gradient at the wall).
template <class R> __device__ __forceinline__ R image_weight(R p) { return p >= R(0) ? p : fdiv(p, R(2) - p); }


// Block reduction of NSUM doubles into partials[tile*NSUM ..] in a fixed order: every
// thread parks its values in LDS, then thread t < 8 NSUM sums 32 cells of counter t/8, and
// the 8 threads of each counter (aligned groups inside one wave) combine by xor-shuffles.
// 256 threads per block.
__device__ __forceinline__ void block_sums(double (&v)[NSUM], double *out) {
  __shared__ double sh[NSUM][256];
  const int t = threadIdx.x;
  const int slot = (t & 31) * 8 + (t >> 5);          // part (t>>5) of 8, element t&31
#pragma unroll
  for (int k = 0; k < NSUM; ++k) sh[k][slot] = v[k];
  __syncthreads();
  if (t < 8 * NSUM) {
    const int k = t >> 3, part = t & 7;
    double acc = 0.0;
#pragma unroll 8
    for (int j = 0; j < 32; ++j) acc += sh[k][j * 8 + part];
    acc += __shfl_xor(acc, 4, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 1, 64);
    if (part == 0) out[k] = acc;
  }
}

// W/T of a cell up to a constant factor (the density per unit thermodynamic pressure):
// 1/T_ref without a temperature, 1/T for the one-step model's constant W.
template <int NS, class R>
__device__ __forceinline__ double w_over_T(const ThermoT<R> &t, const R (&v)[NS > 0 ? NS : 1], double inv_T_ref) {
  if constexpr (NS <= 1) {
    return inv_T_ref;
  } else if constexpr (NS == 2) {
    return (double)fdiv(R(1), v[0]);
  } else {
    R inv = t.inv_W[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) inv += v[1 + q] * t.dinv_W[q];
    return (double)fdiv(R(1), inv * v[0]);
  }
}

// FULL: the instance that also carries curved walls (a.lvl) and the observables
// (a.stats, a.probe_out), each switched on by its pointer; the plain instances carry none
// of that code, so their register allocation is that of the bare step.
// COLL: the collision compiled in: COLL_CUM1 cumulant with every order >= 3 relaxed at
// rate one (D3Q27; any rate on D2Q9), COLL_CUM general cumulant rates, COLL_BGK the BGK
// test mode.  Each instance holds one operator, so the registers of the unused ones do not
// count against the production path.
// The FP32-arithmetic two-step D3Q27 step (FP32 or FP16 storage) asks for four waves per
// SIMD (at most 128 VGPRs): its allocation otherwise lands a few registers above that, at
// three waves; the few spilled values cost less than the lost wave (measured 9 % faster on
// the reacting box in both storage precisions, 12 % for the interior half of the step
// with mixture-averaged transport).
template <int Q, int PREC, int NS, bool EXTRACT, bool FULL, int COLL, int MODE>
constexpr int step_waves_per_eu() {
  return (Q == 27 && PREC != 0 && NS == 6 && !EXTRACT && COLL == COLL_CUM1 && MODE != MODE_LIST &&
          (!FULL || MODE == MODE_INTERIOR || MODE == MODE_INTERIOR_LIN))
             ? 4
             : 1;
}
template <int Q, int PREC, int NS, bool EXTRACT, bool FULL, int COLL, int MODE, bool PULLC = false>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(step_waves_per_eu<Q, PREC, NS, EXTRACT, FULL, COLL, MODE>())))
void step_kernel(KArgs<typename Prec<PREC>::R> a) {
  using P = Prec<PREC>;
  using St = typename P::St;
  using R = typename P::R;
  using Sc = typename P::Sc;
  using GW = typename GeomWord<Q>::T;
  constexpr int D = Lat<Q>::D;
  constexpr int NSV = NS > 0 ? NS : 1;
  constexpr R s = R(1.0 / 3.0);
  constexpr bool INTER = MODE == MODE_INTERIOR || MODE == MODE_INTERIOR_LIN;   // interior cells only
  // the plain interior instance takes y and z as scalars (the FULL one keeps them per lane:
  // as scalars its register pressure spills more)
  constexpr bool UNIYZ = MODE == MODE_INTERIOR && !FULL;

  // Interior instance: the wave runs at a raised priority until its populations and cell
  // scalars are loaded and the velocity is formed, so that waves about to issue loads
  // are not starved by waves deep in their arithmetic (reacting box 0.869 -> 0.860 ms;
  // keeping it raised through the scalar stencils too was slower, 0.883 ms).
  if constexpr (INTER) __builtin_amdgcn_s_setprio(2);
  const int tile = tile_of_block(blockIdx.x, gridDim.x, a.remap);
  // Banded tile order: 64x4-cell tiles, visited band of rows by band, and inside a band
  // plane by plane, so the +-1 and +-2 planes of the scalar stencils were touched a few
  // dozen tiles earlier and are still in L2.
  int n, x, y, z;
  bool listed = true;
  if constexpr (MODE == MODE_LIST) {
    const int idx = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
    listed = idx < a.ncells;
    n = listed ? a.cells[idx] : 0;
    const int nxy = a.nx * a.ny;
    z = n / nxy;
    const int rem = n - z * nxy;
    y = rem / a.nx;
    x = rem - y * a.nx;
  } else if (MODE == MODE_INTERIOR || (MODE == MODE_ALL && a.band_rows)) {
    const int nxt = a.nx >> 6, bt = a.band_rows >> 2;
    const int per_plane = nxt * bt, per_band = per_plane * a.nz;
    const int band = tile / per_band, r = tile - band * per_band;
    const int zz = r / per_plane, r2 = r - zz * per_plane;
    const int xt = r2 / bt, ys = r2 - xt * bt;
    x = (xt << 6) + ((int)threadIdx.x & 63);
    y = band * a.band_rows + (ys << 2) + ((int)threadIdx.x >> 6);
    z = zz;
    if constexpr (UNIYZ) {
      // a wave is 64 cells of one row of one plane: y and z are the same in every lane,
      // so their offsets are scalar values
      y = __builtin_amdgcn_readfirstlane(y);
      z = __builtin_amdgcn_readfirstlane(z);
    }
    n = x + a.nx * (y + a.ny * z);
  } else {
    n = tile * (int)blockDim.x + (int)threadIdx.x;
    const int nxy = a.nx * a.ny;
    z = n / nxy;
    const int rem = n - z * nxy;
    y = rem / a.nx;
    x = rem - y * a.nx;
  }
  double red[NSUM] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int N = a.N;
  const unsigned un = (unsigned)n;
  const St *__restrict__ pin = (const St *)a.pop_in;
  St *__restrict__ pout = (St *)a.pop_out;
  const Sc *__restrict__ sin_ = (const Sc *)a.scal_in;
  Sc *__restrict__ sout = (Sc *)a.scal_out;

  bool active = listed && n < N;
  const GW gw = active && a.geom ? ((const GW *)a.geom)[n] : GW(0);
  if constexpr (INTER)
    active = active && gw == GW(0) && !near_face(x, a.nx, a.face[0], a.face[1]) &&
             !near_face(y, a.ny, a.face[2], a.face[3]) && !near_face(z, a.nz, a.face[4], a.face[5]);
  if (active) {
    const int nxy = a.nx * a.ny;
    if (!INTER && (gw & (GW(1) << bit_self<Q>()))) {
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
      // neighbour offsets (relative linear index) and face codes for k = -2..2 per axis
      int off[3][5], code[3][5];
      axis_offsets(x, a.nx, a.face[0], a.face[1], 1, off[0], code[0]);
      axis_offsets(y, a.ny, a.face[2], a.face[3], a.nx, off[1], code[1]);
      if (D == 3) {
        axis_offsets(z, a.nz, a.face[4], a.face[5], nxy, off[2], code[2]);
      } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          off[2][k] = 0;
          code[2][k] = -1;
        }
      }
      // status of the axis neighbours at -2, -1, +1, +2
      auto status = [&](int d, int k) -> int {
        const int c = code[d][k + 2];
        if (c >= 0) return c;
        const int b = k == 1 ? link_from_plus<Q>(d) : k == -1 ? link_from_minus<Q>(d) : bit_far<Q>(d, k < 0 ? 1 : 0);
        return (gw >> b) & 1 ? ST_SOLID : ST_FLUID;
      };

      // ---------------------------------------------------------------- cell scalars, rho
      // closed domain: density scaled by pi = P_th/P_th(0); q = dln(pi)/dt of this level
      R pim = R(1), qn = R(0);
      if (a.thermo) {
        pim = (R)a.thermo[0];
        qn = (R)a.thermo[1];
      }
      R phi0[NSV], phin[NSV];
#pragma unroll
      for (int k = 0; k < NSV; ++k) { phi0[k] = R(0); phin[k] = R(a.phi_in[k]); }
#pragma unroll
      for (int k = 0; k < NS; ++k) phi0[k] = (R)bld<Sc>(slice(sin_ + (size_t)k * N), un);
      const R rho0 = NS > 0 ? density<NS, R>(a.th, phi0, pim) : R(a.th.rho_ref);
      const R irho0 = fdiv(R(1), rho0);            // every later division by rho uses it
      const R rho_in = NS > 0 ? density<NS, R>(a.th, phin, pim) : R(a.th.rho_ref);

      // mixture-averaged diffusion (Hirschfelder-Curtiss fluxes with the correction flux,
      // lambda grad T), formed before the populations are pulled to keep registers free
      R R_s[NSV];
#pragma unroll
      for (int k = 0; k < NSV; ++k) R_s[k] = R(0);
      R mu_c = R(0), cp_c = R(1);
      if constexpr (FULL && NS == 6) {
        if (a.mx.on) {
          MixPoint<R> mc;
          mix_point<R>(a.mx, a.th, phi0, rho0, pim, mc, mu_c, cp_c);
          for (int d = 0; d < D; ++d) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
              const int sn = status(d, side == 0 ? 1 : -1);
              if (sn != ST_FLUID && sn != ST_INLET) continue;
              MixPoint<R> mn;
              R vn[NSV];
              if (sn == ST_FLUID) {
                const unsigned mq = un + (unsigned)off[d][side == 0 ? 3 : 1];
#pragma unroll
                for (int q = 0; q < NS; ++q) vn[q] = (R)bld<Sc>(slice(sin_ + (size_t)q * N), mq);
                R mu_n, cp_n;
                mix_point<R>(a.mx, a.th, vn, density<NS, R>(a.th, vn, pim), pim, mn, mu_n, cp_n);
              } else {
#pragma unroll
                for (int q = 0; q < NS; ++q) vn[q] = phin[q];
                mn.kap = a.mx.in_kap;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                  mn.coef[k] = a.mx.in_coef[k];
                  mn.X[k] = a.mx.in_X[k];
                  mn.Y[k] = a.mx.in_Y[k];
                }
              }
              R_s[0] += R(0.5) * (mc.kap + mn.kap) * (vn[0] - phi0[0]);
              R J[6], Js = R(0);
#pragma unroll
              for (int k = 0; k < 6; ++k) {
                J[k] = -R(0.5) * (mc.coef[k] + mn.coef[k]) * (mn.X[k] - mc.X[k]);
                Js += J[k];
              }
#pragma unroll
              for (int k = 0; k < 5; ++k) R_s[1 + k] -= J[k] - R(0.5) * (mc.Y[k] + mn.Y[k]) * Js;
            }
          }
        }
      }

      // ---------------------------------------------------------------- pull (Eq. 1)
      R gh[Q];
      const bool border = code[0][1] >= 0 || code[0][3] >= 0 || code[1][1] >= 0 || code[1][3] >= 0 ||
                          (D == 3 && (code[2][1] >= 0 || code[2][3] >= 0));
      constexpr GW linkmask = (GW(1) << Q) - GW(1);
      if (INTER || (!border && !(gw & linkmask))) {
        // PULLC (grids larger than the Infinity Cache): ordinary cached loads.  A wave's 64
        // shifted values of a population with c_x != 0 straddle a cache line that the
        // neighbouring tile in x reads too, and with streaming loads that line was often
        // gone again (256^3 FP32 step: 0.688 -> 0.656 ms, HBM reads 1.08 -> 1.00 of the
        // algorithmic ones).  Grids that fit keep streaming loads, which leave the cache
        // to the freshly written populations the next step reads (cached: 4-12 % slower).
        // Each pulled value is read once per step, so only the line that a shifted
        // population (c_x != 0) shares with the neighbouring tile benefits from the cache:
        // populations with c_x = 0 stream in every instance (reacting box 0.847 -> 0.842
        // ms, HIT 256^3 FP32 0.660 -> 0.656 ms).
        constexpr int PULL_AUX = PULLC ? 0 : 2;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          if constexpr (UNIYZ) {
            // the wave-uniform y/z part of the offset moves the slice's base (scalar
            // arithmetic); the lanes add only the x part (three distinct offsets)
            const long long yz = (long long)off[1][2 - cy(i)] + (D == 3 ? off[2][2 - cz(i)] : 0);
            const St *base = (const St *)((const char *)pin + ((long long)i * N + yz) * (long long)sizeof(St));
            if (cx(i) == 0) gh[i] = decode<R>(bld<St, 2>(slice(base), un));
            else gh[i] = decode<R>(bld<St, PULL_AUX>(slice(base), un + (unsigned)off[0][2 - cx(i)]));
          } else {
            const unsigned m = un + (unsigned)(off[0][2 - cx(i)] + off[1][2 - cy(i)] + (D == 3 ? off[2][2 - cz(i)] : 0));
            if (cx(i) == 0) gh[i] = decode<R>(bld<St, 2>(slice(pin + (size_t)i * N), m));
            else gh[i] = decode<R>(bld<St, PULL_AUX>(slice(pin + (size_t)i * N), m));
          }
        }
      } else if constexpr (!INTER) {
        // boundary cell: bounce-back, moving-wall inlet, anti-bounce-back outlet
        R uw_in[3] = {R(a.inlet_u[0]), R(a.inlet_u[1]), R(a.inlet_u[2])};
        if (a.inlet_noise != 0.0) {
          int fa = -1;
#pragma unroll
          for (int d = 0; d < D; ++d)
            if (a.face[2 * d] == ST_INLET || a.face[2 * d + 1] == ST_INLET) fa = d;
          if (fa >= 0) {
            const int c3[3] = {x, y, z};
            const int o0 = fa == 0 ? 1 : 0, o1 = fa == 2 ? 1 : 2;
            const double xi = splitmix_xi(a.seed, (unsigned long long)c3[o0], (unsigned long long)c3[o1],
                                          (unsigned long long)a.step);
            const R sc = R(1.0 + a.inlet_noise * xi);
            uw_in[0] *= sc; uw_in[1] *= sc; uw_in[2] *= sc;
          }
        }
        R uo[3] = {R(0), R(0), R(0)};
        bool has_out = false;
#pragma unroll
        for (int d = 0; d < D; ++d) has_out |= a.face[2 * d] == ST_OUTLET || a.face[2 * d + 1] == ST_OUTLET;
        if (has_out) {
#pragma unroll
          for (int j = 0; j < Q; ++j) {
            const R gj = decode<R>(bld<St>(slice(pin + (size_t)j * N), un));
            uo[0] += R(cx(j)) * gj;
            uo[1] += R(cy(j)) * gj;
            if (D == 3) uo[2] += R(cz(j)) * gj;
          }
          const R f = R(3) * R(a.P0) * irho0;
          uo[0] *= f; uo[1] *= f; uo[2] *= f;
        }
        const R uo2 = uo[0] * uo[0] + uo[1] * uo[1] + uo[2] * uo[2];
        const R invP0 = a.invP0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int c[3] = {cx(i), cy(i), D == 3 ? cz(i) : 0};
          bool wall = false, inl = false, outl = false;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            if (c[d] == 0) continue;
            const int cd = code[d][2 - c[d]];
            wall |= cd == ST_SOLID;
            inl |= cd == ST_INLET;
            outl |= cd == ST_OUTLET;
          }
          const bool solid_src = (gw >> i) & 1;
          const int io = Q - 1 - i;
          if (wall || (!inl && !outl && solid_src)) {
            const R gopp = decode<R>(bld<St>(slice(pin + (size_t)io * N), un));
            gh[i] = gopp;
            if (FULL && !wall && a.lvl) {
              // interpolated bounce-back, the wall at the fraction q of the link to r - c_i
              const unsigned ms = un + (unsigned)(off[0][2 - c[0]] + off[1][2 - c[1]] + (D == 3 ? off[2][2 - c[2]] : 0));
              const double l0 = a.lvl[n];
              const R qf = (R)(l0 / (l0 - a.lvl[ms]));
              if (qf < R(0.5)) {
                bool ahead_fluid = !((gw >> io) & 1);        // r + c_i is a fluid node
#pragma unroll
                for (int d = 0; d < D; ++d)
                  if (c[d] != 0 && code[d][2 + c[d]] >= 0) ahead_fluid = false;
                if (ahead_fluid) {
                  const unsigned ma = un + (unsigned)(off[0][2 + c[0]] + off[1][2 + c[1]] + (D == 3 ? off[2][2 + c[2]] : 0));
                  gh[i] = lerp(decode<R>(bld<St>(slice(pin + (size_t)io * N), ma)), gopp, R(2) * qf);
                }
              } else {
                const R h = fdiv(R(1), R(2) * qf);
                gh[i] = gopp * h + (R(1) - h) * decode<R>(bld<St>(slice(pin + (size_t)i * N), un));
              }
            }
          } else if (inl) {
            const R cu = R(c[0]) * uw_in[0] + R(c[1]) * uw_in[1] + R(c[2]) * uw_in[2];
            gh[i] = decode<R>(bld<St>(slice(pin + (size_t)io * N), un)) + R(2.0 * wgt<Q>(i)) * rho_in * cu * invP0;
          } else if (outl) {
            const R cu = R(c[0]) * uo[0] + R(c[1]) * uo[1] + R(c[2]) * uo[2];
            gh[i] = -decode<R>(bld<St>(slice(pin + (size_t)io * N), un)) +
                    R(2.0 * wgt<Q>(i)) * ((R(a.outlet_P) + rho0 * (cu * cu * R(1.5) - uo2 * R(0.5))) * invP0 - R(1));
          } else {
            const unsigned m = un + (unsigned)(off[0][2 - c[0]] + off[1][2 - c[1]] + (D == 3 ? off[2][2 - c[2]] : 0));
            gh[i] = decode<R>(bld<St, 2>(slice(pin + (size_t)i * N), m));
          }
        }
      }

      // ---------------------------------------------------------------- moments (Eq. 7b)
      R sg = R(0), mx = R(0), my = R(0), mz = R(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        sg += gh[i];
        if (cx(i)) mx += R(cx(i)) * gh[i];
        if (cy(i)) my += R(cy(i)) * gh[i];
        if (D == 3 && cz(i)) mz += R(cz(i)) * gh[i];
      }
      const R P0 = R(a.P0);
      const R mom = R(3) * P0 * irho0;           // rho u = P0 sum c ghat / cs2
      const R u[3] = {mx * mom, my * mom, D == 3 ? mz * mom : R(0)};
      if constexpr (INTER) __builtin_amdgcn_s_setprio(0);

      // ---------------------------------------------------------------- scalar stencils
      // One pass per axis: the five stencil values of every scalar (ghost rules at walls,
      // inlet, outlet), density at +-1 for grad rho and the diffusion coefficients, the
      // centred diffusion fluxes and the WENO3 advective derivative.
      R gradrho[3] = {R(0), R(0), R(0)};
      R Lam = R(0);
      R adv[NSV];
#pragma unroll
      for (int k = 0; k < NSV; ++k) adv[k] = R(0);
      if constexpr (NS > 0) {
        const R rhoD0 = rho0 * viscosity_irho(a.th, irho0) * a.th.inv_Pr;
        const R rhoD_in = rho_in * viscosity(a.th, rho_in) * a.th.inv_Pr;
        // cells whose +-2 stencil touches no face and no solid take the plain path
        bool interior = gw == GW(0);
#pragma unroll
        for (int d = 0; d < D; ++d)
          interior = interior && code[d][0] < 0 && code[d][1] < 0 && code[d][3] < 0 && code[d][4] < 0;
        auto stencils = [&](auto fast_tag) {
          constexpr bool FAST = decltype(fast_tag)::value;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const int sp1 = FAST ? ST_FLUID : status(d, 1), sm1 = FAST ? ST_FLUID : status(d, -1);
            const int sp2 = FAST ? ST_FLUID : status(d, 2), sm2 = FAST ? ST_FLUID : status(d, -2);
            const unsigned mp1 = un + (unsigned)off[d][3], mm1 = un + (unsigned)off[d][1];
            const unsigned mp2 = un + (unsigned)off[d][4], mm2 = un + (unsigned)off[d][0];
            const R ud = u[d];
            const bool up = ud >= R(0);
            // FAST: vp1 holds the downwind neighbour and vm1 the upwind one (addresses
            // chosen once per axis instead of values per scalar); diffusion and density are
            // symmetric in the two, grad rho takes the sign back
            const unsigned mdw = up ? mp1 : mm1, muw = up ? mm1 : mp1;
            R vp1[NSV], vm1[NSV];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
              const Sc *sq = sin_ + (size_t)q * N;
              if (FAST) {
                vp1[q] = (R)bld<Sc>(slice(sq), mdw);
                vm1[q] = (R)bld<Sc>(slice(sq), muw);
              } else {
                vp1[q] = sp1 == ST_FLUID ? (R)bld<Sc>(slice(sq), mp1) : sp1 == ST_INLET ? phin[q] : phi0[q];
                vm1[q] = sm1 == ST_FLUID ? (R)bld<Sc>(slice(sq), mm1) : sm1 == ST_INLET ? phin[q] : phi0[q];
              }
            }
            // curved walls: mirror images of solid cells at -1 / +1 (c1), of the stencil
            // points at -2 / +2 behind them (c2, image at p2 from the cell) and of a solid
            // cell at -2 / +2 behind a fluid neighbour (c3, weight w3 from that neighbour)
            bool c1m = false, c1p = false, c2m = false, c2p = false, c3m = false, c3p = false;
            R w1m = R(0), w1p = R(0), p2m = R(0), p2p = R(0), w3m = R(0), w3p = R(0);
            if (FULL && !FAST && a.lvl) {
              const double l0 = a.lvl[n];
              if (sm1 == ST_SOLID && code[d][1] < 0 && sp1 == ST_FLUID) {
                const R qw = (R)(l0 / (l0 - a.lvl[mm1]));
                c1m = true;
                w1m = image_weight(R(1) - R(2) * qw);
                p2m = R(2) - R(2) * qw;
                c2m = p2m <= R(1) || sp2 == ST_FLUID;
              } else if (sm1 == ST_FLUID && sm2 == ST_SOLID && code[d][0] < 0) {
                const double l1 = a.lvl[mm1];
                c3m = true;
                w3m = image_weight(R(1) - R(2) * (R)(l1 / (l1 - a.lvl[mm2])));
              }
              if (sp1 == ST_SOLID && code[d][3] < 0 && sm1 == ST_FLUID) {
                const R qw = (R)(l0 / (l0 - a.lvl[mp1]));
                c1p = true;
                w1p = image_weight(R(1) - R(2) * qw);
                p2p = R(2) - R(2) * qw;
                c2p = p2p <= R(1) || sm2 == ST_FLUID;
              } else if (sp1 == ST_FLUID && sp2 == ST_SOLID && code[d][4] < 0) {
                const double l1 = a.lvl[mp1];
                c3p = true;
                w3p = image_weight(R(1) - R(2) * (R)(l1 / (l1 - a.lvl[mp2])));
              }
#pragma unroll
              for (int q = 0; q < NS; ++q) {
                const R am = vm1[q], ap = vp1[q];
                if (c1m) vm1[q] = lerp(phi0[q], ap, w1m);
                if (c1p) vp1[q] = lerp(phi0[q], am, w1p);
              }
            }
            // density at +-1 and diffusion through the two faces
            R rp = rho0, rm = rho0;
            if (FAST || sp1 == ST_FLUID) rp = density<NS, R>(a.th, vp1, pim);
            else if (sp1 == ST_INLET) rp = rho_in;
            else if (c1p) rp = density<NS, R>(a.th, vp1, pim);
            if (FAST || sm1 == ST_FLUID) rm = density<NS, R>(a.th, vm1, pim);
            else if (sm1 == ST_INLET) rm = rho_in;
            else if (c1m) rm = density<NS, R>(a.th, vm1, pim);
            gradrho[d] = R(0.5) * (rp - rm);
            if (FAST && !up) gradrho[d] = -gradrho[d];
            // face coefficients: arithmetic mean of rho D (uniform when rho nu is constant)
            R cfp, cfm;
            if (FAST) {
              cfp = a.th.const_mu ? rhoD0 : R(0.5) * (rhoD0 + rp * viscosity(a.th, rp) * a.th.inv_Pr);
              cfm = a.th.const_mu ? rhoD0 : R(0.5) * (rhoD0 + rm * viscosity(a.th, rm) * a.th.inv_Pr);
            } else {
              const bool fp = sp1 == ST_FLUID || sp1 == ST_INLET, fm = sm1 == ST_FLUID || sm1 == ST_INLET;
              cfp = fp ? R(0.5) * (rhoD0 + (sp1 == ST_INLET ? rhoD_in : rp * viscosity(a.th, rp) * a.th.inv_Pr)) : R(0);
              cfm = fm ? R(0.5) * (rhoD0 + (sm1 == ST_INLET ? rhoD_in : rm * viscosity(a.th, rm) * a.th.inv_Pr)) : R(0);
            }
            const bool mixed = FULL && NS == 6 && a.mx.on;   // diffusion done before the pull
            if (!mixed) {
              // differences first: a sum of neighbours minus 2D phi0 would round with a
              // bias near binade boundaries (values near 1 and 4) in FP32
#pragma unroll
              for (int q = 0; q < NS; ++q) R_s[q] += cfp * (vp1[q] - phi0[q]) + cfm * (vm1[q] - phi0[q]);
            }
            if (!EXTRACT) {
              // WENO3 upwinded on the sign of u_d, written branch-free: with the upwind
              // neighbours U1, U2 and the downwind neighbour D1,
              // u_d dphi/dx_d = |u_d| (face(U1, 0, D1) - face(U2, U1, 0)).
              const R au = fabs(ud);
              const unsigned mfar = up ? mm2 : mp2;
#pragma unroll
              for (int q = 0; q < NS; ++q) {
                const Sc *sq = sin_ + (size_t)q * N;
                const R v0 = phi0[q];
                R vU2;
                if (FAST) {
                  vU2 = (R)bld<Sc>(slice(sq), mfar);
                } else {
                  R vm2, vp2;
                  if (sm1 == ST_FLUID) vm2 = sm2 == ST_FLUID ? (R)bld<Sc>(slice(sq), mm2) : sm2 == ST_INLET ? phin[q] : vm1[q];
                  else vm2 = sm1 == ST_SOLID ? vp1[q] : sm1 == ST_INLET ? phin[q] : v0;
                  if (sp1 == ST_FLUID) vp2 = sp2 == ST_FLUID ? (R)bld<Sc>(slice(sq), mp2) : sp2 == ST_INLET ? phin[q] : vp1[q];
                  else vp2 = sp1 == ST_SOLID ? vm1[q] : sp1 == ST_INLET ? phin[q] : v0;
                  if (c2m) vm2 = p2m <= R(1) ? lerp(v0, vp1[q], p2m) : lerp(vp1[q], (R)bld<Sc>(slice(sq), mp2), p2m - R(1));
                  else if (c3m) vm2 = lerp(vm1[q], v0, w3m);
                  if (c2p) vp2 = p2p <= R(1) ? lerp(v0, vm1[q], p2p) : lerp(vm1[q], (R)bld<Sc>(slice(sq), mm2), p2p - R(1));
                  else if (c3p) vp2 = lerp(vp1[q], v0, w3p);
                  vU2 = up ? vm2 : vp2;
                }
                const R vU1 = FAST || up ? vm1[q] : vp1[q];
                const R vD1 = FAST || up ? vp1[q] : vm1[q];
                adv[q] += au * weno3_diff(vU2, vU1, v0, vD1, a.eps[q]);
              }
            }
          }
        };
        if (INTER || interior) stencils(std::true_type{});
        else if constexpr (!INTER) stencils(std::false_type{});
        const R Fr = a.th.F * irho0;
#pragma unroll
        for (int q = 0; q < NS; ++q) R_s[q] *= Fr;
        if constexpr (FULL && NS == 6) {
          if (a.mx.on) R_s[0] = fdiv(R_s[0], cp_c);
        }
        // chemistry (reaction over F) and Lambda (Eq. 3)
        const R invF = a.th.invF;
        if constexpr (NS == 2) {
          const R r = a.th.B1 * fmax(phi0[1], R(0)) * hexp(-fdiv(a.th.Ta1, phi0[0]));
          R_s[0] += a.th.heat1 * r * invF;
          R_s[1] -= r * invF;
          if (a.thermo) R_s[0] += a.kap * qn * phi0[0];   // pressure work
          Lam = fdiv(R_s[0], phi0[0]);
          if (a.thermo) Lam -= qn;                        // div u = Lambda - dln(pi)/dt
        } else if constexpr (NS == 6) {
          R conc[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) conc[q] = rho0 * fmax(phi0[1 + q], R(0)) * a.th.inv_W[q];
          const R T = phi0[0];
          const R iT = fdiv(R(1), T);
          const R q1 = a.th.B1 * hexp(-a.th.Ta1 * iT) * conc[0] * conc[1];
          const R q2 = a.th.B2 * hexp(-a.th.Ta2 * iT) * conc[2] * hsqrt(conc[1]);
          const R ir = irho0;
          // molar rates per mass: sum over reactions of nu_k,r q_r, over rho
          const R m0 = -q1 * ir, m1 = (R(-1.5) * q1 - R(0.5) * q2) * ir, m2 = (q1 - q2) * ir,
                  m3 = q2 * ir, m4 = R(2) * q1 * ir;
          R_s[1] += a.th.W[0] * m0 * invF;
          R_s[2] += a.th.W[1] * m1 * invF;
          R_s[3] += a.th.W[2] * m2 * invF;
          R_s[4] += a.th.W[3] * m3 * invF;
          R_s[5] += a.th.W[4] * m4 * invF;
          R heat = -(a.th.h[0] * m0 + a.th.h[1] * m1 + a.th.h[2] * m2 + a.th.h[3] * m3 +
                     a.th.h[4] * m4) * a.th.inv_cp;
          if constexpr (FULL) {
            if (a.mx.on) {
              // full molar enthalpies h_k(T) and the mixture c_p
              R hT[5];
#pragma unroll
              for (int q = 0; q < 5; ++q)
                hT[q] = a.mx.hc[q] + a.th.W[q] * T * (a.mx.cpa[q] + R(0.5) * a.mx.cpb[q] * T);
              heat = -fdiv(hT[0] * m0 + hT[1] * m1 + hT[2] * m2 + hT[3] * m3 + hT[4] * m4, cp_c);
            }
          }
          R_s[0] += heat * invF;
          if (a.thermo) R_s[0] += a.kap * qn * T;         // pressure work
          // Lambda = R_T/T + W sum_k R_k/W_k (N2 by closure: R_N2 = -sum R_k)
          R invW = a.th.inv_W[5], acc = R(0);
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            invW += phi0[1 + q] * a.th.dinv_W[q];
            acc += R_s[1 + q] * a.th.dinv_W[q];
          }
          Lam = R_s[0] * iT + fdiv(acc, invW);
          if (a.thermo) Lam -= qn;                        // div u = Lambda - dln(pi)/dt
        }
      }
      // Eq. 7a: P_h = P0 (1 + sum ghat) + (dt/2) rho cs2 Lambda, formed in FP64 from the
      // deviation sum (1 + sum ghat in the compute precision would round away the pressure
      // fluctuation's last digits, and P0 in it is rounded too)
      const R hLam = R(0.5) * rho0 * s * Lam;
      const double Ph = a.P0d * (1.0 + (double)sg) + (double)hLam;

      if (EXTRACT) {
        if (a.f_P) a.f_P[n] = Ph;
        if (a.f_rho) a.f_rho[n] = (double)rho0;
        if (a.f_u)
#pragma unroll
          for (int d = 0; d < D; ++d) a.f_u[d * N + n] = (double)u[d];
        if (a.f_scal)
#pragma unroll
          for (int k = 0; k < NS; ++k) a.f_scal[k * N + n] = (double)phi0[k];
      } else {
        // ------------------------------------------------------------ observables
        // running mean and squared-deviation sums (Welford) of u and P_h - P0 at sampled
        // levels; probe rows (u, P_h) at the probe cells
        if (FULL && a.stats) {
          const double x[4] = {(double)u[0], (double)u[1], (double)u[2], Ph - a.P0d};
#pragma unroll
          for (int j = 0; j <= D; ++j) {
            const double xv = x[j == D ? 3 : j];
            double *mp = a.stats + (size_t)j * N + n, *sp = a.stats + (size_t)(D + 1 + j) * N + n;
            const double m0 = *mp;
            const double m1 = m0 + (xv - m0) * a.inv_k;
            *mp = m1;
            *sp += (xv - m0) * (xv - m1);
          }
        }
        if (FULL && a.probe_out) {
          for (int j = 0; j < a.nprobe; ++j)
            if (n == a.probe[j]) {
#pragma unroll
              for (int d = 0; d < D; ++d) a.probe_out[j * (D + 1) + d] = (double)u[d];
              a.probe_out[j * (D + 1) + D] = Ph;
            }
        }
        // ------------------------------------------------------------ scalar update
        // one finiteness test for the step's outputs: a NaN or an infinity in any of
        // them makes the sum non-finite (the finite values are far below overflow)
        R chk = R(0);
        R phi1[NSV];
        phi1[0] = R(0);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const R nv = phi0[q] + (R_s[q] - adv[q]);
          chk += nv;
          // streaming stores where the grid exceeds the Infinity Cache (reacting box
          // 0.857 -> 0.853 ms, with mixture transport 1.194 -> 1.186 ms); smaller grids
          // keep the scalars in the cache for the next step's stencils.  The plain
          // instances decide at compile time (the cached-pull ones are the large-grid
          // ones; a run-time test there cost the 2-D chamber 2 %), the FULL ones at run time
          if (PULLC || (FULL && a.big)) bst<Sc, 2>(slice(sout + (size_t)q * N), un, (Sc)nv);
          else bst<Sc>(slice(sout + (size_t)q * N), un, (Sc)nv);
          phi1[q] = (R)(Sc)nv;
        }
        if (a.thermo) red[8] = w_over_T<NS>(a.th, phi1, a.inv_T_ref_d);
        // ------------------------------------------------------------ collision
        const R r = a.th.rho_ref * irho0;               // P0/(rho cs2)
        const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const R ugr = u[0] * gradrho[0] + u[1] * gradrho[1] + u[2] * gradrho[2];
        const R rsL = rho0 * s * Lam;
        // Eq. 2: Xi_i = cs2 (f_eq/rho - w)(c - u).grad rho + w rho cs2 Lambda, formed once
        // per population and kept for the post-collision form (Eq. 8), here already over
        // 2 rho cs2 (the factor of Eq. 13) and less w_i Es (below).  Opposite velocities
        // share c.u and c.grad rho up to sign: with a = c.u, b = c.grad rho,
        // f_eq/rho - w = w (3a + 4.5a^2 - 1.5u.u), so each pair needs one square and the two
        // signs of the odd parts.
        R Xh[NS >= 2 ? Q : 1];
        R e[Q];
        // sum_i Xi_i = cs2 (rho Lambda + u . grad rho) (the moments of Eq. 2)
        const R Xs = NS >= 2 ? s * (rho0 * Lam + ugr) : R(0);
        // Es = sum_i of the pre-conditioned populations minus the weights (Eq. 13), from the
        // moments: r sum ghat + sum Xi / (2 rho cs2); d = f~ - w = e - w Es has zero sum
        const R Es = NS >= 2 ? r * sg + Xs * (R(1.5) * irho0) : sg;
        if constexpr (NS >= 2) {
          const R k1 = R(0.5) * irho0;                   // cs2 / (2 rho cs2)
          const R k0 = R(0.5) * Lam - Es;                // rho cs2 Lambda / (2 rho cs2) - Es
          const R e0 = R(-1.5) * uu;
#pragma unroll
          for (int i = 0; i < Q / 2; ++i) {
            const int o = Q - 1 - i;
            R a0 = R(0), b0 = R(0);
            if (cx(i)) { a0 += R(cx(i)) * u[0]; b0 += R(cx(i)) * gradrho[0]; }
            if (cy(i)) { a0 += R(cy(i)) * u[1]; b0 += R(cy(i)) * gradrho[1]; }
            if (D == 3 && cz(i)) { a0 += R(cz(i)) * u[2]; b0 += R(cz(i)) * gradrho[2]; }
            const R ev = R(4.5) * a0 * a0 + e0, od = R(3) * a0;
            const R wk1 = R(wgt<Q>(i)) * k1, wk0 = R(wgt<Q>(i)) * k0;
            Xh[i] = wk1 * ((ev + od) * (b0 - ugr)) + wk0;
            Xh[o] = wk1 * ((ev - od) * (-b0 - ugr)) + wk0;
          }
          constexpr int c0 = Q / 2;
          Xh[c0] = R(wgt<Q>(c0)) * (k1 * (e0 * -ugr) + k0);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          if constexpr (NS >= 2) e[i] = r * gh[i] + Xh[i];          // d = f~ - w (Eq. 13)
          else e[i] = gh[i] - R(wgt<Q>(i)) * Es;                     // rho = rho_ref, Xi = 0
        }
        R nu = viscosity_irho(a.th, irho0);
        if constexpr (FULL && NS == 6) {
          if (a.mx.on) nu = mu_c * irho0;
        }
        Rates<R> rt;
        rt.tau0 = nu * R(3) + R(0.5);                    // nu / cs2 + 1/2
        rt.smag18 = a.smag18;
        rt.wb = a.wb;
        rt.wh = a.wh;
        rt.gal = a.gal != 0;
        rt.p4 = a.p4 != 0;
        const R hP0 = R(0.5) * a.invP0;
        const R base = sg + Xs * hP0;                    // (1/r) m0 - 1
        const R invr = rho0 * a.invP0 * s;              // rho/rho_ref = rho cs2/P0
        const R baseE = NS >= 2 ? base + Es * invr : base;   // with the w_i Es taken from Xh
        if constexpr (COLL != COLL_BGK) {
          if constexpr (Q == 9) collide_d2q9(e, u[0], u[1], rt);
          else collide_d3q27<R, COLL == COLL_CUM1>(e, u[0], u[1], u[2], rt);
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            R gs;
            if constexpr (NS >= 2) gs = R(wgt<Q>(i)) * baseE + (e[i] + Xh[i]) * invr;   // Eq. 8
            else gs = R(wgt<Q>(i)) * base + e[i];
            bst<St, 2>(slice(pout + (size_t)i * N), un, encode<St>(gs));
          }
        } else {
          // BGK in the pre-conditioned frame (Eq. 5 with the half-source split)
          const R om = shear_rate(rt, pipi_of<Q, R>(e, u));
          const R ph1 = sg + hLam * a.invP0;
          const R kq = rho0 * s * a.invP0;
#pragma unroll
          for (int i = 0; i < Q; ++i) {
            const R cu = R(cx(i)) * u[0] + R(cy(i)) * u[1] + (D == 3 ? R(cz(i)) * u[2] : R(0));
            const R geq = R(wgt<Q>(i)) * (ph1 + kq * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu));
            R xh = R(0);
            if constexpr (NS >= 2) xh = (Xh[i] + R(wgt<Q>(i)) * Es) * invr;
            const R gp = gh[i] + xh;
            bst<St, 2>(slice(pout + (size_t)i * N), un, encode<St>(gp - om * (gp - geq) + xh));
          }
        }
        if (!isfinite(chk + sg + hLam + u[0] + u[1] + u[2])) atomicOr(a.flag, 1);
      }

      // ---------------------------------------------------------------- FP64 sums
      // (cell values in the compute precision, accumulated in FP64)
      red[0] = (double)rho0;
      red[1] = Ph;
      red[2] = (double)(rho0 * u[0]);
      red[3] = (double)(rho0 * u[1]);
      red[4] = (double)(rho0 * u[2]);
      red[5] = (double)(R(0.5) * rho0 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
      red[6] = w_over_T<NS>(a.th, phi0, a.inv_T_ref_d);
      if constexpr (NS >= 2) red[7] = (double)(rho0 * phi0[1]);
    }
  }
  block_sums(red, a.partials + (size_t)(MODE == MODE_LIST ? (int)blockIdx.x : tile) * NSUM);
}


// Deterministic reduction of the per-block records: stage 1 gives each of up to 256
// blocks a contiguous range of records, stage 2 sums the stage-1 records in one block.
// The order of every addition is fixed by the launch shape, so results are bitwise
// repeatable.  Given thermo (closed domain, stage 2 only), the final sums also advance
// (pi, q, K): K = pi sum W/T at the first step, pi' = K / sum W/T of the updated
// scalars (the total mass is held), q' = (pi' - pi)/pi.
static __global__ __launch_bounds__(256) void finalize_stage(const double *in, int nrec, int chunk, double *out,
                                                             double *thermo) {
  __shared__ double sh[NSUM][256];
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(nrec, b0 + chunk);
  double acc[NSUM];
#pragma unroll
  for (int k = 0; k < NSUM; ++k) acc[k] = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += 256)
#pragma unroll
    for (int k = 0; k < NSUM; ++k) acc[k] += in[(size_t)b * NSUM + k];
#pragma unroll
  for (int k = 0; k < NSUM; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
#pragma unroll
      for (int k = 0; k < NSUM; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < NSUM) out[(size_t)blockIdx.x * NSUM + threadIdx.x] = sh[threadIdx.x][0];
  if (thermo && threadIdx.x == 0) {
    const double pi = thermo[0];
    double K = thermo[2];
    if (!(K > 0.0)) K = pi * sh[6][0];
    const double pn = K / sh[8][0];
    thermo[0] = pn;
    thermo[1] = (pn - pi) / pi;
    thermo[2] = K;
  }
}

// Closed domain, after every step: (pi, q, K) advanced from the two sums it needs, sum W/T
// at level n and of the updated scalars (record entries 6 and 8), in one block of 1024
// threads: thread t adds records t, t + 1024, ..., then the lanes of each wave by a
// butterfly (lane 0's value kept) and the 16 waves in order.  A fixed order of additions,
// so the result is bitwise repeatable; one short kernel instead of the two stages of
// finalize_stage over all NSUM entries (chamber 2500x500: 9.4 us of dependent latency).
static __global__ __launch_bounds__(1024) void thermo_kernel(const double *rec, int nrec, double *thermo) {
  __shared__ double part[2][16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double s6 = 0.0, s8 = 0.0;
  for (int b = t; b < nrec; b += 1024) {
    s6 += rec[(size_t)b * NSUM + 6];
    s8 += rec[(size_t)b * NSUM + 8];
  }
  for (int o = 32; o > 0; o >>= 1) {
    s6 += __shfl_xor(s6, o, 64);
    s8 += __shfl_xor(s8, o, 64);
  }
  if (lane == 0) {
    part[0][w] = s6;
    part[1][w] = s8;
  }
  __syncthreads();
  if (t == 0) {
    double a6 = 0.0, a8 = 0.0;
    for (int j = 0; j < 16; ++j) {
      a6 += part[0][j];
      a8 += part[1][j];
    }
    const double pi = thermo[0];
    double K = thermo[2];
    if (!(K > 0.0)) K = pi * a6;
    const double pn = K / a8;
    thermo[0] = pn;
    thermo[1] = (pn - pi) / pi;
    thermo[2] = K;
  }
}

// (pi, q, K) set from the host's values (a kernel rather than a copy, so that the call
// needs no host buffer to outlive it).
static __global__ void set_thermo_kernel(double *thermo, double pi, double q, double K) {
  if (threadIdx.x == 0) {
    thermo[0] = pi;
    thermo[1] = q;
    thermo[2] = K;
  }
}

// Generalised flame surface: |grad c| summed over fluid cells, c = (T - T_u)/(T_b - T_u),
// central differences with the ghost rules of grad rho (own value across walls, solids
// and the outlet, the inlet temperature across the inlet); FP64 block records.
template <int Q, int PREC>
__global__ __launch_bounds__(256) void surface_kernel(KArgs<double> a, double inv_dT) {
  using Sc = typename Prec<PREC>::Sc;
  using GW = typename GeomWord<Q>::T;
  constexpr int D = Lat<Q>::D;
  const int n = blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
  double red[NSUM];
#pragma unroll
  for (int k = 0; k < NSUM; ++k) red[k] = 0.0;
  if (n < a.N) {
    const GW gw = a.geom ? ((const GW *)a.geom)[n] : GW(0);
    if (!(gw & (GW(1) << bit_self<Q>()))) {
      const Sc *T = (const Sc *)a.scal_in;
      const int nxy = a.nx * a.ny, z = n / nxy, rem = n - z * nxy, y = rem / a.nx, x = rem - y * a.nx;
      const int cc[3] = {x, y, z}, ext[3] = {a.nx, a.ny, a.nz};
      const double t0 = (double)T[n];
      double g2 = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const AxisNb ax = axis_nb(cc[d], ext[d], a.face[2 * d], a.face[2 * d + 1]);
        const int stride = d == 0 ? 1 : d == 1 ? a.nx : nxy;
        double v[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int k = s == 0 ? 3 : 1;                    // +1, -1
          const int code = ax.code[k];
          const int bit = s == 0 ? link_from_plus<Q>(d) : link_from_minus<Q>(d);
          if (code == ST_INLET) v[s] = a.phi_in[0];
          else if (code >= 0 || ((gw >> bit) & 1)) v[s] = t0;
          else v[s] = (double)T[n + (ax.idx[k] - cc[d]) * stride];
        }
        const double gd = 0.5 * (v[0] - v[1]) * inv_dT;
        g2 += gd * gd;
      }
      red[0] = sqrt(g2);
    }
  }
  block_sums(red, a.partials + (size_t)blockIdx.x * NSUM);
}

// Mean and RMS fields from the running statistics (k samples): mean [D+1][N] (u_d, then
// P_h with P0 added back), rms = sqrt(M2/k).
static __global__ __launch_bounds__(256) void statistics_kernel(const double *acc, int D, long long N, double k,
                                                                 double P0, double *mean, double *rms) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int j = 0; j <= D; ++j) {
    if (mean) mean[j * N + n] = acc[j * N + n] + (j == D ? P0 : 0.0);
    if (rms) rms[j * N + n] = sqrt(fmax(acc[(D + 1 + j) * N + n], 0.0) / k);
  }
}

__device__ __forceinline__ bool solid_at(const uint8_t *s, long long m) { return s[m] != 0; }
__device__ __forceinline__ bool solid_at(const double *phi, long long m) { return phi[m] < 0.0; }

// Geometry words from a solid mask, or from a signed wall distance (solid where < 0).
template <int Q, class Src>
__global__ __launch_bounds__(256) void geometry_kernel(const Src *solid, void *geom, int nx, int ny,
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
  if (solid_at(solid, n)) w |= GW(1) << bit_self<Q>();
  for (int i = 0; i < Q; ++i) {
    const int c[3] = {cx(i), cy(i), D == 3 ? cz(i) : 0};
    bool out = ax.code[2 - c[0]] >= 0 || ay.code[2 - c[1]] >= 0 || (D == 3 && az.code[2 - c[2]] >= 0);
    if (out || i == (Q - 1) / 2) continue;
    const long long m = lin(ax.idx[2 - c[0]], ay.idx[2 - c[1]], D == 3 ? az.idx[2 - c[2]] : z);
    if (solid_at(solid, m)) w |= GW(1) << i;
  }
  for (int d = 0; d < D; ++d) {
    const AxisNb &A = d == 0 ? ax : d == 1 ? ay : az;
    for (int neg = 0; neg < 2; ++neg) {
      const int k = neg ? 0 : 4;   // position -2 or +2
      if (A.code[k] >= 0) continue;
      const long long m = d == 0 ? lin(A.idx[k], y, z) : d == 1 ? lin(x, A.idx[k], z) : lin(x, y, A.idx[k]);
      if (solid_at(solid, m)) w |= GW(1) << bit_far<Q>(d, neg);
    }
  }
  ((GW *)geom)[n] = w;
}

// Equilibrium initialisation (Eq. 6) from FP64 fields; populations stored as deviations.
template <int Q, int PREC, int NS>
__global__ __launch_bounds__(256) void init_kernel(KArgs<double> a, const double *Ph, const double *u,
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
