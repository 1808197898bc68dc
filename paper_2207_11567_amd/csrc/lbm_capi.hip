// C ABI of the hybrid LB/FD time step (include/lbm.h): parameter validation, buffer
// binding, launch sequencing on the caller's stream, and the synchronising read-backs.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_launch.hpp"

using namespace lbm;

struct lbm_solver {
  lbm_params p;
  hipStream_t stream;
  void *pop[2];
  void *scal[2];
  unsigned char *work;
  int cur;
  long long step;
  bool initialized;
  bool has_geom;
  long long N;
  int Q, NS, D, prec, nblocks;
  int *flag;
  double *sums;
  double *partials;   // block records of lbm_step: [nblocks] interior, then [list blocks]
  double *aux;        // block records of field extraction, flame surface and objective
  int *cells;         // linear indices of the boundary cells (the step's list half)
  int ncells;         // their number
  int nrec;           // block records the last step wrote
  // the list half of a split step runs on a side stream (default priority), forked from
  // and joined back into the caller's stream around each step; created on first use
  hipStream_t side;
  hipEvent_t ev_fork, ev_join;
  bool side_ready;
  ~lbm_solver() {
    if (side_ready) {
      (void)hipStreamSynchronize(side);
      (void)hipEventDestroy(ev_fork);
      (void)hipEventDestroy(ev_join);
      (void)hipStreamDestroy(side);
    }
  }
  double *stage;
  double *thermo;     // (pi, q, K) of the closed-domain thermodynamic pressure
  bool closed;
  const double *lvl;  // bound signed wall distance (curved walls) or nullptr
  double *stats;      // running statistics buffer or nullptr
  int stats_every;
  long long stats_k;  // samples taken
  double *probe_rec;  // probe record or nullptr
  int nprobe;
  int probe[8];
  long long probe_cap, probe_rows;
  void *geom;
  double *scratch;     // this device's copy of the allocation-free scratch (or nullptr)
  std::string scratch_err;
  std::string err;
};

static thread_local std::string g_create_err;

static int n_scalars(int physics) {
  switch (physics) {
    case LBM_ISOTHERMAL: return 0;
    case LBM_PASSIVE: return 1;
    case LBM_ONE_STEP: return 2;
    case LBM_TWO_STEP: return 6;
  }
  return -1;
}

static size_t pop_elem(int prec) { return prec == LBM_FP64 ? 8 : prec == LBM_FP32 ? 4 : 2; }
static size_t scal_elem(int prec) { return prec == LBM_FP64 ? 8 : 4; }
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
  long long N;
  int Q, NS, D, nblocks;
  size_t pop_bytes, scal_bytes, off_flag, off_sums, off_thermo, off_stage, off_partials, off_geom, off_cells,
      work_bytes;
};

static lbm_status validate(const lbm_params *p, Layout *L, std::string &err, std::string *warn_out = nullptr) {
  std::string warn;
  char buf[256];
  auto fail = [&](const char *m) { err = m; return LBM_E_INVALID; };
  if (!p) return fail("params is NULL");
  if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q27) return fail("lattice must be LBM_D2Q9 or LBM_D3Q27");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail("grid sizes must be >= 1");
  if (p->lattice == LBM_D2Q9 && p->nz != 1) return fail("D2Q9 requires nz == 1");
  if (p->precision < 0 || p->precision > 2) return fail("precision must be LBM_FP64, LBM_FP32 or LBM_FP16S");
  if (p->collision != LBM_CUMULANT && p->collision != LBM_BGK) return fail("unknown collision operator");
  if (p->galilean != 0 && p->galilean != 1) return fail("galilean must be 0 or 1");
  if (p->galilean && p->collision != LBM_CUMULANT) return fail("the Galilean correction belongs to the cumulant collision");
  if (p->fourth_order != 0 && p->fourth_order != 1) return fail("fourth_order must be 0 or 1");
  if (p->fourth_order) {
    if (p->lattice != LBM_D3Q27 || p->collision != LBM_CUMULANT)
      return fail("the fourth-order parameterisation belongs to the D3Q27 cumulant collision");
    // rates at the molecular shear rate (Eq. 12 read as a relaxation time)
    const double w1 = 1.0 / (3.0 * p->nu_ref + 0.5), w2 = p->omega_bulk;
    const double w3 = (8 * (w1 - 2) * (w2 * (3 * w1 - 1) - 5 * w1)) / (8 * (5 - 2 * w1) * w1 + w2 * (8 + w1 * (9 * w1 - 26)));
    const double w4 = (8 * (w1 - 2) * (w1 + w2 * (3 * w1 - 7))) / (w2 * (56 - 42 * w1 + 9 * w1 * w1) - 8 * w1);
    const double w5 = (24 * (w1 - 2) * (4 * w1 * w1 + w1 * w2 * (18 - 13 * w1) + w2 * w2 * (2 + w1 * (6 * w1 - 11)))) /
                      (16 * w1 * w1 * (w1 - 6) - 2 * w1 * w2 * (216 + 5 * w1 * (9 * w1 - 46)) +
                       w2 * w2 * (w1 * (3 * w1 - 10) * (15 * w1 - 28) - 48));
    const double den = (w1 - w2) * (w2 * (2 + 3 * w1) - 8 * w1);
    const bool ok = w3 > 0 && w3 < 2 && w4 > 0 && w4 < 2 && w5 > 0 && w5 < 2 && fabs(den) > 1e-3;
    if (!ok) {
      char b2[200];
      snprintf(b2, sizeof b2,
               "fourth-order parameterisation outside its stable range at omega_1 = %g, omega_bulk = %g "
               "(omega_3..5 = %g, %g, %g)", w1, w2, w3, w4, w5);
      err = b2;
      return LBM_E_INVALID;
    }
  }
  const int NS = n_scalars(p->physics);
  if (NS < 0) return fail("unknown physics");
  if (p->visc_law != LBM_VISC_CONST_NU && p->visc_law != LBM_VISC_CONST_MU) return fail("unknown visc_law");
  if (!(p->nu_ref > 0.0) || !isfinite(p->nu_ref)) return fail("nu_ref must be > 0 (tau0 > 1/2)");
  if (!(p->omega_bulk >= 0.0 && p->omega_bulk <= 2.0)) return fail("omega_bulk must lie in [0, 2]");
  if (!(p->omega_high >= 0.0 && p->omega_high <= 2.0)) return fail("omega_high must lie in [0, 2]");
  if (!(p->cs_smag >= 0.0)) return fail("cs_smag must be >= 0");
  if (!(p->rho_ref > 0.0) || !(p->T_ref > 0.0)) return fail("rho_ref and T_ref must be > 0");
  if (NS > 0) {
    if (!(p->prandtl > 0.0)) return fail("prandtl must be > 0");
    if (!(p->thickening > 0.0)) return fail("thickening must be > 0");
    for (int k = 0; k < NS; ++k)
      if (!(p->weno_scale[k] > 0.0)) return fail("weno_scale must be > 0 for every scalar");
    const double D = p->lattice == LBM_D2Q9 ? 2.0 : 3.0;
    const double FD = p->thickening * p->nu_ref / p->prandtl;
    if (FD > 1.0 / (2.0 * D)) {
      snprintf(buf, sizeof buf, "explicit diffusion unstable: F nu/Pr = %g > 1/(2d) = %g", FD, 1.0 / (2.0 * D));
      err = buf;
      return LBM_E_INVALID;
    }
  }
  if (p->physics == LBM_ONE_STEP && !(p->chem[4] > 0.0)) return fail("one-step chemistry needs Y_u > 0");
  if (p->physics == LBM_TWO_STEP) {
    for (int k = 5; k < 11; ++k)
      if (!(p->chem[k] > 0.0)) return fail("two-step chemistry needs molar masses > 0");
    if (!(p->chem[4] > 0.0) || !(p->chem[17] > 0.0)) return fail("two-step chemistry needs c_p > 0, W_ref > 0");
  }
  // The same explicit-diffusion limit in the hottest gas the chemistry can make, where the
  // density is lowest: with rho nu constant the kinematic viscosity (and F D = F nu/Pr)
  // grows as rho_ref/rho; with mixture transport the binary coefficients grow as
  // (T/T_ref)^s_D and lambda/(rho c_p) as (T/T_ref)^s_mu rho_ref/rho.  Hottest gas: T_ad of
  // the one-step model, or the inlet mixture burnt completely to CO2 and H2O (two-step).
  if ((p->physics == LBM_ONE_STEP || p->physics == LBM_TWO_STEP) &&
      (p->visc_law == LBM_VISC_CONST_MU || p->transport_model == LBM_TRANSPORT_MIXTURE)) {
    const double Dm = p->lattice == LBM_D2Q9 ? 2.0 : 3.0;
    double T_hot = 0.0, rho_ratio = 1.0;        // rho_ref / rho at T_hot
    if (p->physics == LBM_ONE_STEP) {
      T_hot = fmax(p->chem[3], p->inlet_T);
      rho_ratio = T_hot / p->T_ref;
    } else {
      const double *ch = p->chem;
      double Y[6], ys = 0.0;
      for (int k = 0; k < 5; ++k) {
        Y[k] = fmax(p->inlet_Y[k], 0.0);
        ys += Y[k];
      }
      Y[5] = 1.0 - ys;
      // CH4 + 2 O2 -> CO2 + 2 H2O, limited by fuel or oxygen (mol per kg)
      const double xi = fmin(Y[0] / ch[5], 0.5 * Y[1] / ch[6]);
      const double q = xi * (ch[11] + 2.0 * ch[12] - ch[14] - 2.0 * ch[15]);   // J/kg
      T_hot = fmax(p->inlet_T, p->T_ref) + fmax(q, 0.0) / ch[4];
      double Yb[6];
      for (int k = 0; k < 6; ++k) Yb[k] = Y[k];
      Yb[0] -= xi * ch[5];
      Yb[1] -= 2.0 * xi * ch[6];
      Yb[3] += xi * ch[8];
      Yb[4] += 2.0 * xi * ch[9];
      double invW = 0.0;
      for (int k = 0; k < 6; ++k) invW += Yb[k] / ch[5 + k];
      rho_ratio = (T_hot / p->T_ref) * (invW * ch[17]);        // rho_ref/rho = (T/T_ref)(W_ref/W)
    }
    double FD_hot = 0.0;
    if (p->transport_model == LBM_TRANSPORT_MIXTURE) {
      const double th = T_hot / p->T_ref;
      double D0max = 0.0;
      for (int k = 0; k < 15; ++k) D0max = fmax(D0max, p->transport[k]);
      FD_hot = p->thickening * fmax(D0max * pow(th, p->transport[28]),
                                    p->nu_ref * pow(th, p->transport[27]) * rho_ratio / p->prandtl);
    } else {
      FD_hot = p->thickening * p->nu_ref * rho_ratio / p->prandtl;
    }
    if (FD_hot > 1.0 / (2.0 * Dm)) {
      // a warning, not an error: short runs and states that never get this hot are valid
      snprintf(buf, sizeof buf,
               "warning: explicit diffusion unstable in the hottest gas the chemistry can make (T = %g): "
               "F D = %g > 1/(2d) = %g", T_hot, FD_hot, 1.0 / (2.0 * Dm));
      warn = buf;
    }
  }
  const int Dm = p->lattice == LBM_D2Q9 ? 2 : 3;
  for (int f = 0; f < 6; ++f)
    if (p->face_bc[f] < LBM_PERIODIC || p->face_bc[f] > LBM_OUTLET) return fail("unknown face condition");
  if (p->pth_mode != LBM_PTH_OPEN && p->pth_mode != LBM_PTH_CLOSED) return fail("unknown pth_mode");
  if (p->transport_model != LBM_TRANSPORT_SIMPLE && p->transport_model != LBM_TRANSPORT_MIXTURE)
    return fail("unknown transport_model");
  if (p->transport_model == LBM_TRANSPORT_MIXTURE) {
    if (p->physics != LBM_TWO_STEP) return fail("mixture-averaged transport needs the two-step scalars");
    for (int k = 0; k < 15; ++k)
      if (!(p->transport[k] > 0.0) || !isfinite(p->transport[k])) return fail("mixture transport: D0_kj must be > 0");
    for (int k = 0; k < 6; ++k)
      if (!(p->transport[15 + k] > 0.0)) return fail("mixture transport: c_p coefficients a_k must be > 0");
  }
  if (p->pth_mode == LBM_PTH_CLOSED) {
    if (!(p->gamma > 1.0) || !isfinite(p->gamma)) return fail("closed domain needs gamma > 1");
    for (int f = 0; f < 2 * Dm; ++f)
      if (p->face_bc[f] == LBM_INLET || p->face_bc[f] == LBM_OUTLET)
        return fail("a closed domain has no inlet or outlet face");
  }
  for (int d = 0; d < Dm; ++d)
    if ((p->face_bc[2 * d] == LBM_PERIODIC) != (p->face_bc[2 * d + 1] == LBM_PERIODIC))
      return fail("periodic faces must come in pairs");
  for (int d = 0; d < Dm; ++d)
    for (int side = 0; side < 2; ++side)
      if ((p->face_bc[2 * d + side] == LBM_INLET || p->face_bc[2 * d + side] == LBM_OUTLET) &&
          (d == 0 ? p->nx : d == 1 ? p->ny : p->nz) < 3)
        return fail("inlet/outlet axis needs at least 3 cells");
  const long long N = (long long)p->nx * p->ny * p->nz;
  const int Q = p->lattice;
  if ((long long)Q * N > (1ll << 31) - 1) return fail("grid too large: Q*N must stay below 2^31");
  L->N = N;
  L->Q = Q;
  L->NS = NS;
  L->D = Dm;
  L->nblocks = (int)((N + 255) / 256);
  // step records (interior tiles, then list blocks, each at most nblocks), then those of
  // the other reductions
  const int nrec = 3 * L->nblocks;
  L->pop_bytes = (size_t)Q * N * pop_elem(p->precision);
  L->scal_bytes = (size_t)NS * N * scal_elem(p->precision);
  L->off_flag = 0;
  L->off_sums = 64;                       // NSUM doubles
  L->off_thermo = 192;                    // 3 doubles
  L->off_stage = 256;
  L->off_partials = L->off_stage + 256 * NSUM * sizeof(double);
  L->off_geom = align256(L->off_partials + (size_t)nrec * NSUM * sizeof(double));
  L->off_cells = align256(L->off_geom + (size_t)N * (Q == 9 ? 4 : 8));
  L->work_bytes = align256(L->off_cells + (size_t)N * sizeof(int));
  if (warn_out) *warn_out = warn;
  return LBM_OK;
}

static lbm_status hip_fail(lbm_solver *s, hipError_t e, const char *what) {
  s->err = std::string(what) + ": " + hipGetErrorString(e);
  return LBM_E_HIP;
}

// The inlet state's mixture transport point (FP64, same formulas as the kernel's).
static void mix_inlet_point(const lbm_params &p, double *out) {
  const double *ch = p.chem, *tr = p.transport;
  double Y[6], ys = 0.0;
  for (int k = 0; k < 5; ++k) {
    Y[k] = p.inlet_Y[k];
    ys += Y[k];
  }
  Y[5] = 1.0 - ys;
  double invW = 0.0;
  for (int k = 0; k < 6; ++k) invW += Y[k] / ch[5 + k];
  const double T = p.inlet_T, rho = p.rho_ref * (p.T_ref / T) / (invW * ch[17]);
  const double lt = log(T / p.T_ref), mu = p.nu_ref * p.rho_ref * exp(tr[27] * lt), scale = exp(tr[28] * lt);
  double cp = 0.0, X[6];
  for (int k = 0; k < 6; ++k) {
    cp += Y[k] * (tr[15 + k] + tr[21 + k] * T);
    X[k] = Y[k] / (invW * ch[5 + k]);
  }
  out[0] = mu * cp / p.prandtl;
  double B[6][6];
  for (int i = 0, n = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j, ++n) B[i][j] = B[j][i] = tr[n];
  for (int k = 0; k < 6; ++k) {
    double sum = 0.0;
    for (int j = 0; j < 6; ++j)
      if (j != k) sum += X[j] / B[k][j];
    out[1 + k] = rho * (1.0 - Y[k]) * scale / sum * ch[5 + k] * invW;
    out[7 + k] = X[k];
    out[13 + k] = Y[k];
  }
}

static StepArgs make_args(const lbm_solver *s) {
  const lbm_params &p = s->p;
  StepArgs a;
  memset(&a, 0, sizeof a);
  a.geom = s->has_geom ? s->geom : nullptr;
  a.partials = s->partials;
  a.flag = s->flag;
  a.thermo = s->closed ? s->thermo : nullptr;
  a.lvl = s->has_geom ? s->lvl : nullptr;
  a.kappa = s->closed ? (p.gamma - 1.0) / p.gamma : 0.0;
  a.nx = p.nx;
  a.ny = p.ny;
  a.nz = p.nz;
  a.N = s->N;
  for (int f = 0; f < 6; ++f) {
    const int c = p.face_bc[f];
    a.face[f] = c == LBM_PERIODIC ? -1 : c == LBM_WALL ? ST_SOLID : c == LBM_INLET ? ST_INLET : ST_OUTLET;
  }
  if (s->D == 2) a.face[4] = a.face[5] = -1;
  a.step = s->step;
  a.collision = p.collision;
  a.gal = p.galilean;
  a.p4 = p.fourth_order;
  a.remap = 1;
  // population copies larger than the 256 MB Infinity Cache: cached pull loads
  a.pull_cached = (size_t)s->Q * (size_t)s->N * pop_elem(s->prec) > ((size_t)256 << 20);
  a.band_rows = 0;
  if (p.nx % 64 == 0 && p.ny % 4 == 0)
    for (int b : {32, 16, 8, 4})
      if (p.ny % b == 0) {
        a.band_rows = b;
        break;
      }
  a.P0 = p.rho_ref / 3.0;
  a.wb = p.omega_bulk;
  a.wh = p.omega_high;
  a.smag18 = 18.0 * p.cs_smag * p.cs_smag;
  for (int d = 0; d < 3; ++d) a.inlet_u[d] = p.inlet_u[d];
  a.inlet_noise = p.inlet_noise;
  a.outlet_P = p.outlet_P;
  a.phi_in[0] = p.inlet_T;
  for (int k = 1; k < 8; ++k) a.phi_in[k] = p.inlet_Y[k - 1];
  for (int k = 0; k < 8; ++k) a.eps[k] = 1e-6 * p.weno_scale[k] * p.weno_scale[k];
  a.seed = p.seed;
  a.th.rho_ref = p.rho_ref;
  a.th.T_ref = p.T_ref;
  a.th.nu_ref = p.nu_ref;
  a.th.inv_Pr = s->NS > 0 ? 1.0 / p.prandtl : 0.0;
  a.th.F = s->NS > 0 ? p.thickening : 1.0;
  a.th.visc_const_mu = p.visc_law == LBM_VISC_CONST_MU ? 1.0 : 0.0;
  for (int k = 0; k < 32; ++k) a.th.chem[k] = p.chem[k];
  a.mix = p.transport_model == LBM_TRANSPORT_MIXTURE ? 1 : 0;
  for (int k = 0; k < 32; ++k) a.transport[k] = p.transport[k];
  if (a.mix) mix_inlet_point(p, a.mix_in);
  return a;
}

static hipError_t launch(const lbm_solver *s, int kind, const StepArgs &a, const double *Ph = nullptr,
                         const double *u = nullptr, const double *scal = nullptr) {
  if (s->Q == 9) return launch_d2q9(s->prec, s->NS, kind, a, s->nblocks, s->stream, Ph, u, scal);
  return launch_d3q27(s->prec, s->NS, kind, a, s->nblocks, s->stream, Ph, u, scal);
}

static lbm_status check_flag(lbm_solver *s) {
  int f = 0;
  hipError_t e = hipMemcpyAsync(&f, s->flag, sizeof(int), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "reading the divergence flag");
  if (f & 1) {
    s->err = "a non-finite value appeared during a time step";
    return LBM_E_DIVERGED;
  }
  return LBM_OK;
}

// The boundary cells of the split step, in increasing linear index: a non-zero geometry
// word or a non-periodic face within two cells on some axis (the rule of near_face and the
// interior instance).  Built on the host from the geometry words; synchronises.
static bool host_near_face(int c, int n, int flo, int fhi) { return (flo >= 0 && c < 2) || (fhi >= 0 && c >= n - 2); }

static hipError_t build_cell_list(lbm_solver *s) {
  const lbm_params &p = s->p;
  StepArgs a = make_args(s);
  const long long N = s->N;
  const size_t gsz = s->Q == 9 ? 4 : 8;
  std::vector<unsigned char> gw;
  hipError_t e = hipSuccess;
  if (s->has_geom) {
    gw.resize((size_t)N * gsz);
    e = hipMemcpyAsync(gw.data(), s->geom, gw.size(), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return e;
  }
  std::vector<int> list;
  for (int z = 0; z < p.nz; ++z)
    for (int y = 0; y < p.ny; ++y) {
      const bool row = host_near_face(y, p.ny, a.face[2], a.face[3]) || host_near_face(z, p.nz, a.face[4], a.face[5]);
      for (int x = 0; x < p.nx; ++x) {
        const long long n = x + (long long)p.nx * (y + (long long)p.ny * z);
        bool g = row || host_near_face(x, p.nx, a.face[0], a.face[1]);
        if (!g && s->has_geom) {
          const unsigned char *w = gw.data() + (size_t)n * gsz;
          for (size_t b = 0; b < gsz; ++b) g = g || w[b] != 0;
        }
        if (g) list.push_back((int)n);
      }
    }
  s->ncells = (int)list.size();
  if (!list.empty()) {
    e = hipMemcpyAsync(s->cells, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  }
  return e;
}

// One step from a.pop_in / a.scal_in, either as one instance over every cell or split into
// the interior instance over the tile grid and the list instance over the boundary cells.
// The split pays where the all-cell instance carries boundary code that costs the interior
// cells: curved walls (the FULL instance; its list half is FULL) and, on large grids, the
// steps with transported scalars (their stencil ghost rules are most of that code); with
// mixture transport both halves are FULL instances; with observables (statistics, probes)
// the step stays one FULL instance.  The isothermal and
// passive steps measured slower as interior instances, and on small grids the second
// kernel adds a pass of latency.  The interior half writes block records [0, nblocks), the
// list half the records after them.
static hipError_t launch_step_pass(lbm_solver *s, const StepArgs &a0) {
  StepArgs a = a0;
  a.partials = s->partials;
  const bool split = !(a.stats || a.probe_out) && (a.lvl || (s->NS >= 2 && s->nblocks >= 4096));
  if (!split) {
    s->nrec = s->nblocks;
    return launch(s, LAUNCH_STEP, a);
  }
  hipError_t e = hipSuccess;
  s->nrec = s->nblocks;
  if (s->ncells == 0) return launch(s, LAUNCH_STEP_INTERIOR, a);
  if (!s->side_ready) {
    e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    s->side_ready = true;
  }
  // fork: the list half waits for everything before this step on the caller's stream,
  // then runs beside the interior half (the two write disjoint cells and records)
  StepArgs b = a;
  b.cells = s->cells;
  b.ncells = s->ncells;
  b.partials = s->partials + (size_t)s->nblocks * NSUM;
  const int nlb = (s->ncells + 255) / 256;
  e = hipEventRecord(s->ev_fork, s->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s->side, s->ev_fork, 0);
  if (e != hipSuccess) return e;
  if (s->Q == 9) e = launch_d2q9(s->prec, s->NS, LAUNCH_STEP_LIST, b, nlb, s->side, nullptr, nullptr, nullptr);
  else e = launch_d3q27(s->prec, s->NS, LAUNCH_STEP_LIST, b, nlb, s->side, nullptr, nullptr, nullptr);
  if (e == hipSuccess) e = hipEventRecord(s->ev_join, s->side);
  if (e == hipSuccess) e = launch(s, LAUNCH_STEP_INTERIOR, a);
  // join: later work on the caller's stream sees both halves
  if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->ev_join, 0);
  s->nrec = s->nblocks + nlb;
  return e;
}

// ------------------------------------------------------------------ allocation-free surface
// Device scratch of lbm_flame_surface_noalloc, held by the library on every device it runs
// on until the process ends: the surface kernel's block records [NOALLOC_MAX_BLOCKS][NSUM],
// then the 256 stage records of the two-stage sum, then the NSUM final sums.  Every record
// a call reads was written earlier in the same call, so nothing needs clearing.  In host
// code the name `scratch` only stands in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_ptr.
constexpr int NOALLOC_MAX_BLOCKS = 131072;                        // 33.5 M cells, 256 per block
constexpr size_t NOALLOC_STAGE = (size_t)NOALLOC_MAX_BLOCKS * NSUM;
constexpr size_t NOALLOC_OUT = NOALLOC_STAGE + (size_t)256 * NSUM;
static __device__ __align__(256) double scratch[NOALLOC_OUT + NSUM];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static bool g_scratch_looked_up[NOALLOC_MAX_DEVICES];
static double *g_scratch_ptr[NOALLOC_MAX_DEVICES];
static hipError_t g_scratch_status[NOALLOC_MAX_DEVICES];

// The scratch address on the current device (looked up once per device); nullptr with the
// reason in why when the lookup failed.
static double *scratch_on_current_device(std::string &why) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    why = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return nullptr;
  }
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    why = "device index beyond the scratch table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_looked_up[dev]) {
    void *ptr = nullptr;
    g_scratch_status[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_status[dev] == hipSuccess ? (double *)ptr : nullptr;
    g_scratch_looked_up[dev] = true;
  }
  if (!g_scratch_ptr[dev]) why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(g_scratch_status[dev]);
  return g_scratch_ptr[dev];
}

static __global__ void copy_first_kernel(const double *src, double *dst) {
  if (threadIdx.x == 0) dst[0] = src[0];
}

// Device copy through the step's own memory forms: 4-byte raw buffer loads (streaming when
// bit 0 of MODE is set, else cached) and 4-byte raw buffer stores (streaming when bit 1 is
// set), one element per lane and 64 consecutive ones per wave, eight loads in flight per
// lane.  n < 2^29 elements, so every byte offset fits the 32-bit buffer offset.
template <int MODE>
__global__ __launch_bounds__(256) void copy_probe_kernel(const float *src, float *dst, unsigned n) {
  constexpr int LA = (MODE & 1) ? 2 : 0, SA = (MODE & 2) ? 2 : 0;
  const auto rs = slice(src);
  const auto rd = slice(dst);
  const unsigned stride = gridDim.x * 256u;
  unsigned i = blockIdx.x * 256u + threadIdx.x;
  for (; i + 7u * stride < n; i += 8u * stride) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = bld<float, LA>(rs, i + (unsigned)j * stride);
#pragma unroll
    for (int j = 0; j < 8; ++j) bst<float, SA>(rd, i + (unsigned)j * stride, v[j]);
  }
  for (; i < n; i += stride) bst<float, SA>(rd, i, bld<float, LA>(rs, i));
}

extern "C" {

lbm_status lbm_query_sizes(const lbm_params *p, size_t *pop_bytes, size_t *scal_bytes, size_t *work_bytes) {
  Layout L;
  std::string warn;
  lbm_status st = validate(p, &L, g_create_err, &warn);
  if (st != LBM_OK) return st;
  g_create_err = warn;
  if (pop_bytes) *pop_bytes = L.pop_bytes;
  if (scal_bytes) *scal_bytes = L.scal_bytes;
  if (work_bytes) *work_bytes = L.work_bytes;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_params *p, void *stream, void *pop_a, void *pop_b, void *scal_a, void *scal_b,
                      void *work, lbm_solver **out) {
  if (!out) return LBM_E_INVALID;
  *out = nullptr;
  Layout L;
  std::string warn;
  lbm_status st = validate(p, &L, g_create_err, &warn);
  if (st != LBM_OK) return st;
  if (!pop_a || !pop_b || !work || pop_a == pop_b) {
    g_create_err = "pop_a, pop_b (distinct) and work are required";
    return LBM_E_INVALID;
  }
  if (L.NS > 0 && (!scal_a || !scal_b || scal_a == scal_b)) {
    g_create_err = "scal_a and scal_b (distinct) are required when scalars are transported";
    return LBM_E_INVALID;
  }
  lbm_solver *s = new lbm_solver();
  s->p = *p;
  s->stream = (hipStream_t)stream;
  s->pop[0] = pop_a;
  s->pop[1] = pop_b;
  s->scal[0] = scal_a;
  s->scal[1] = scal_b;
  s->work = (unsigned char *)work;
  s->cur = 0;
  s->step = 0;
  s->initialized = false;
  s->has_geom = false;
  s->N = L.N;
  s->Q = L.Q;
  s->NS = L.NS;
  s->D = L.D;
  s->prec = p->precision;
  s->nblocks = L.nblocks;
  s->flag = (int *)(s->work + L.off_flag);
  s->sums = (double *)(s->work + L.off_sums);
  s->partials = (double *)(s->work + L.off_partials);
  s->aux = s->partials + (size_t)2 * L.nblocks * NSUM;
  s->cells = (int *)(s->work + L.off_cells);
  s->ncells = 0;
  s->nrec = L.nblocks;
  s->side_ready = false;
  s->stage = (double *)(s->work + L.off_stage);
  s->thermo = (double *)(s->work + L.off_thermo);
  s->closed = p->pth_mode == LBM_PTH_CLOSED;
  s->lvl = nullptr;
  s->stats = nullptr;
  s->stats_every = 1;
  s->stats_k = 0;
  s->probe_rec = nullptr;
  s->nprobe = 0;
  s->probe_cap = s->probe_rows = 0;
  s->geom = s->work + L.off_geom;
  s->scratch = scratch_on_current_device(s->scratch_err);   // the solver's device is the current one
  hipError_t e = hipMemsetAsync(s->work, 0, 256, s->stream);
  if (e == hipSuccess) e = launch_set_thermo(s->thermo, 1.0, 0.0, 0.0, s->stream);
  if (e == hipSuccess) e = build_cell_list(s);
  if (e != hipSuccess) {
    g_create_err = std::string("setting up the work buffer: ") + hipGetErrorString(e);
    delete s;
    return LBM_E_HIP;
  }
  s->err = warn;                  // empty, or the warning of the parameter check
  *out = s;
  return LBM_OK;
}

lbm_status lbm_set_geometry(lbm_solver *s, const uint8_t *solid_dev) {
  if (!s) return LBM_E_INVALID;
  s->lvl = nullptr;
  if (!solid_dev) {
    s->has_geom = false;
    hipError_t e = build_cell_list(s);
    return e == hipSuccess ? LBM_OK : hip_fail(s, e, "boundary cell list");
  }
  StepArgs a = make_args(s);
  hipError_t e = launch_geometry(s->Q, solid_dev, s->geom, s->p.nx, s->p.ny, s->p.nz, s->N, a.face, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "geometry kernel");
  s->has_geom = true;
  e = build_cell_list(s);
  if (e != hipSuccess) return hip_fail(s, e, "boundary cell list");
  return LBM_OK;
}

lbm_status lbm_set_wall_distance(lbm_solver *s, const double *phi_dev) {
  if (!s) return LBM_E_INVALID;
  s->lvl = nullptr;
  if (!phi_dev) {
    s->has_geom = false;
    hipError_t e = build_cell_list(s);
    return e == hipSuccess ? LBM_OK : hip_fail(s, e, "boundary cell list");
  }
  StepArgs a = make_args(s);
  hipError_t e = launch_geometry_levelset(s->Q, phi_dev, s->geom, s->p.nx, s->p.ny, s->p.nz, s->N, a.face,
                                          s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "geometry kernel");
  s->has_geom = true;
  s->lvl = phi_dev;
  e = build_cell_list(s);
  if (e != hipSuccess) return hip_fail(s, e, "boundary cell list");
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_solver *s, const double *P_h, const double *u, const double *scal) {
  if (!s) return LBM_E_INVALID;
  if (!P_h || !u || (s->NS > 0 && !scal)) {
    s->err = "P_h, u (and scal when scalars are transported) are required";
    return LBM_E_INVALID;
  }
  s->step = 0;
  StepArgs a = make_args(s);
  a.pop_out = s->pop[s->cur];
  a.scal_out = s->scal[s->cur];
  hipError_t e = launch(s, LAUNCH_INIT, a, P_h, u, scal);
  if (e != hipSuccess) return hip_fail(s, e, "init kernel");
  e = launch_set_thermo(s->thermo, 1.0, 0.0, 0.0, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "resetting the thermodynamic pressure");
  e = hipMemsetAsync(s->flag, 0, sizeof(int), s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "clearing the divergence flag");
  s->initialized = true;
  return LBM_OK;
}

lbm_status lbm_step(lbm_solver *s, int32_t nsteps) {
  if (!s) return LBM_E_INVALID;
  if (!s->initialized) {
    s->err = "lbm_step before lbm_init_fields or lbm_set_state";
    return LBM_E_STATE;
  }
  if (nsteps < 0) {
    s->err = "nsteps must be >= 0";
    return LBM_E_INVALID;
  }
  StepArgs a = make_args(s);
  for (int k = 0; k < nsteps; ++k) {
    a.pop_in = s->pop[s->cur];
    a.pop_out = s->pop[1 - s->cur];
    a.scal_in = s->scal[s->cur];
    a.scal_out = s->scal[1 - s->cur];
    a.step = s->step;
    a.stats = nullptr;
    if (s->stats && s->step % s->stats_every == 0) {
      s->stats_k += 1;
      a.stats = s->stats;
      a.inv_k = 1.0 / (double)s->stats_k;
    }
    a.probe_out = nullptr;
    if (s->probe_rec && s->probe_rows < s->probe_cap) {
      a.probe_out = s->probe_rec + (size_t)s->probe_rows * s->nprobe * (s->D + 1);
      a.nprobe = s->nprobe;
      for (int j = 0; j < 8; ++j) a.probe[j] = s->probe[j];
      s->probe_rows += 1;
    }
    hipError_t e = launch_step_pass(s, a);
    if (e != hipSuccess) return hip_fail(s, e, "step kernel");
    if (s->closed) {
      e = launch_thermo(s->partials, s->nrec, s->thermo, s->stream);
      if (e != hipSuccess) return hip_fail(s, e, "thermodynamic pressure update");
    }
    s->cur ^= 1;
    s->step += 1;
  }
  return LBM_OK;
}

lbm_status lbm_step_from(lbm_solver *s, const void *pops_in, const void *scal_in, void *pops_out, void *scal_out,
                         int64_t step) {
  if (!s) return LBM_E_INVALID;
  if (!pops_in || !pops_out || pops_in == pops_out || step < 0 ||
      (s->NS > 0 && (!scal_in || !scal_out || scal_in == scal_out))) {
    s->err = "lbm_step_from: distinct input and output buffers are required";
    return LBM_E_INVALID;
  }
  if (s->closed) {
    s->err = "lbm_step_from: a closed domain carries its thermodynamic pressure in the solver";
    return LBM_E_UNSUPPORTED;
  }
  StepArgs a = make_args(s);
  a.pop_in = pops_in;
  a.pop_out = pops_out;
  a.scal_in = scal_in;
  a.scal_out = scal_out;
  a.step = step;
  hipError_t e = launch_step_pass(s, a);
  if (e != hipSuccess) return hip_fail(s, e, "step kernel");
  return LBM_OK;
}

lbm_status lbm_step_sums(lbm_solver *s, double *sums_host) {
  if (!s) return LBM_E_INVALID;
  hipError_t e = launch_finalize(s->partials, s->nrec, s->stage, s->sums, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "finalize kernel");
  if (sums_host) {
    e = hipMemcpyAsync(sums_host, s->sums, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "copying sums");
  }
  return check_flag(s);
}

lbm_status lbm_fields(lbm_solver *s, double *P_h, double *rho, double *u, double *scal, double *sums_host) {
  if (!s) return LBM_E_INVALID;
  if (!s->initialized) {
    s->err = "lbm_fields before initialisation";
    return LBM_E_STATE;
  }
  StepArgs a = make_args(s);
  a.pop_in = s->pop[s->cur];
  a.scal_in = s->scal[s->cur];
  a.f_P = P_h;
  a.f_rho = rho;
  a.f_u = u;
  a.f_scal = scal;
  a.partials = s->aux;                  // the step's own records stay for lbm_step_sums
  hipError_t e = launch(s, LAUNCH_EXTRACT, a);
  if (e != hipSuccess) return hip_fail(s, e, "field extraction kernel");
  e = launch_finalize(s->aux, s->nblocks, s->stage, s->sums, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "finalize kernel");
  if (sums_host) {
    e = hipMemcpyAsync(sums_host, s->sums, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "copying sums");
  }
  return check_flag(s);
}

lbm_status lbm_get_state(lbm_solver *s, void *pops_dst, void *scal_dst, int64_t *step) {
  if (!s) return LBM_E_INVALID;
  const size_t pb = (size_t)s->Q * s->N * pop_elem(s->prec), sb = (size_t)s->NS * s->N * scal_elem(s->prec);
  hipError_t e = hipSuccess;
  if (pops_dst) e = hipMemcpyAsync(pops_dst, s->pop[s->cur], pb, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess && scal_dst && sb)
    e = hipMemcpyAsync(scal_dst, s->scal[s->cur], sb, hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "copying the state out");
  if (step) *step = s->step;
  return check_flag(s);
}

lbm_status lbm_set_state(lbm_solver *s, const void *pops_src, const void *scal_src, int64_t step) {
  if (!s) return LBM_E_INVALID;
  if (!pops_src || (s->NS > 0 && !scal_src) || step < 0) {
    s->err = "pops_src (and scal_src when scalars are transported) required, step >= 0";
    return LBM_E_INVALID;
  }
  const size_t pb = (size_t)s->Q * s->N * pop_elem(s->prec), sb = (size_t)s->NS * s->N * scal_elem(s->prec);
  hipError_t e = hipMemcpyAsync(s->pop[s->cur], pops_src, pb, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess && sb) e = hipMemcpyAsync(s->scal[s->cur], scal_src, sb, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->flag, 0, sizeof(int), s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "copying the state in");
  s->step = step;
  s->initialized = true;
  return LBM_OK;
}

lbm_status lbm_set_statistics(lbm_solver *s, double *acc_dev, int32_t every) {
  if (!s) return LBM_E_INVALID;
  if (acc_dev && every < 1) {
    s->err = "statistics: every must be >= 1";
    return LBM_E_INVALID;
  }
  s->stats = acc_dev;
  s->stats_every = acc_dev ? every : 1;
  s->stats_k = 0;
  if (acc_dev) {
    hipError_t e = hipMemsetAsync(acc_dev, 0, (size_t)2 * (s->D + 1) * s->N * sizeof(double), s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "clearing the statistics");
  }
  return LBM_OK;
}

lbm_status lbm_statistics(lbm_solver *s, double *mean_dev, double *rms_dev, int64_t *samples) {
  if (!s) return LBM_E_INVALID;
  if (!s->stats || s->stats_k == 0) {
    s->err = "statistics: no samples (bind a buffer with lbm_set_statistics, then step)";
    return LBM_E_STATE;
  }
  hipError_t e = launch_statistics(s->stats, s->D, s->N, s->stats_k, s->p.rho_ref / 3.0, mean_dev, rms_dev, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "statistics kernel");
  if (samples) *samples = s->stats_k;
  return check_flag(s);
}

lbm_status lbm_set_probes(lbm_solver *s, const int64_t *cells_host, int32_t nprobe, double *record_dev,
                          int64_t capacity) {
  if (!s) return LBM_E_INVALID;
  if (!record_dev || nprobe == 0) {
    s->probe_rec = nullptr;
    s->nprobe = 0;
    s->probe_cap = s->probe_rows = 0;
    return LBM_OK;
  }
  if (nprobe < 0 || nprobe > 8 || !cells_host || capacity < 1) {
    s->err = "probes: 1..8 cells, a record buffer and capacity >= 1 required";
    return LBM_E_INVALID;
  }
  for (int j = 0; j < nprobe; ++j)
    if (cells_host[j] < 0 || cells_host[j] >= s->N) {
      s->err = "probes: cell index out of range";
      return LBM_E_INVALID;
    }
  for (int j = 0; j < 8; ++j) s->probe[j] = j < nprobe ? (int)cells_host[j] : -1;
  s->nprobe = nprobe;
  s->probe_rec = record_dev;
  s->probe_cap = capacity;
  s->probe_rows = 0;
  return LBM_OK;
}

lbm_status lbm_probe_rows(lbm_solver *s, int64_t *rows) {
  if (!s || !rows) return LBM_E_INVALID;
  *rows = s->probe_rows;
  return LBM_OK;
}

lbm_status lbm_flame_surface(lbm_solver *s, double T_u, double T_b, double *surface_host) {
  if (!s || !surface_host) return LBM_E_INVALID;
  if (s->NS < 1 || !(T_b != T_u)) {
    s->err = "flame surface: needs a temperature and T_b != T_u";
    return LBM_E_INVALID;
  }
  if (!s->initialized) {
    s->err = "flame surface before initialisation";
    return LBM_E_STATE;
  }
  StepArgs a = make_args(s);
  a.scal_in = s->scal[s->cur];
  a.partials = s->aux;
  hipError_t e = launch_surface(s->Q, s->prec, a, s->nblocks, s->stream, T_u, T_b);
  if (e == hipSuccess) e = launch_finalize(s->aux, s->nblocks, s->stage, s->sums, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(surface_host, s->sums, sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "flame surface");
  return LBM_OK;
}

lbm_status lbm_flame_surface_noalloc(lbm_solver *s, double T_u, double T_b, double *surface_dev) {
  if (!s || !surface_dev) return LBM_E_INVALID;
  if (s->nblocks > NOALLOC_MAX_BLOCKS) {
    char buf[160];
    snprintf(buf, sizeof buf, "flame surface (no allocation): %lld cells exceed the scratch maximum of %lld",
             s->N, (long long)NOALLOC_MAX_BLOCKS * 256);
    s->err = buf;
    return LBM_E_INVALID;
  }
  if (s->NS < 1 || !(T_b != T_u)) {
    s->err = "flame surface: needs a temperature and T_b != T_u";
    return LBM_E_INVALID;
  }
  if (!s->initialized) {
    s->err = "flame surface before initialisation";
    return LBM_E_STATE;
  }
  if (!s->scratch) {
    s->err = "flame surface (no allocation): " + s->scratch_err;
    return LBM_E_HIP;
  }
  StepArgs a = make_args(s);
  a.scal_in = s->scal[s->cur];
  a.partials = s->scratch;
  hipError_t e = launch_surface(s->Q, s->prec, a, s->nblocks, s->stream, T_u, T_b);
  if (e == hipSuccess)
    e = launch_finalize(s->scratch, s->nblocks, s->scratch + NOALLOC_STAGE, s->scratch + NOALLOC_OUT, s->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(copy_first_kernel, dim3(1), dim3(64), 0, s->stream, (const double *)(s->scratch + NOALLOC_OUT),
                       surface_dev);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(s, e, "flame surface (no allocation)");
  return LBM_OK;
}

lbm_status lbm_copy_probe(const void *src, void *dst, size_t bytes, int32_t mode, void *stream) {
  if (!src || !dst || bytes == 0 || bytes % 4 != 0 || bytes > ((size_t)1 << 31) || mode < 0 || mode > 3) {
    g_create_err = "lbm_copy_probe: device pointers, 0 < bytes <= 2^31 and a multiple of 4, mode 0..3 are required";
    return LBM_E_INVALID;
  }
  const char *a = (const char *)src, *b = (const char *)dst;
  if (a < b + bytes && b < a + bytes) {
    g_create_err = "lbm_copy_probe: source and destination overlap";
    return LBM_E_INVALID;
  }
  const unsigned n = (unsigned)(bytes / 4);
  const unsigned blocks = std::min<unsigned>((n + 255u) / 256u, 8192u);
  hipStream_t st = (hipStream_t)stream;
  const float *fs = (const float *)src;
  float *fd = (float *)dst;
  switch (mode) {
    case 0: hipLaunchKernelGGL(copy_probe_kernel<0>, dim3(blocks), dim3(256), 0, st, fs, fd, n); break;
    case 1: hipLaunchKernelGGL(copy_probe_kernel<1>, dim3(blocks), dim3(256), 0, st, fs, fd, n); break;
    case 2: hipLaunchKernelGGL(copy_probe_kernel<2>, dim3(blocks), dim3(256), 0, st, fs, fd, n); break;
    default: hipLaunchKernelGGL(copy_probe_kernel<3>, dim3(blocks), dim3(256), 0, st, fs, fd, n); break;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_create_err = std::string("lbm_copy_probe: ") + hipGetErrorString(e);
    return LBM_E_HIP;
  }
  g_create_err.clear();
  return LBM_OK;
}

lbm_status lbm_get_thermo_pressure(lbm_solver *s, double *pqk_host) {
  if (!s || !pqk_host) return LBM_E_INVALID;
  hipError_t e = hipMemcpyAsync(pqk_host, s->thermo, 3 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "reading the thermodynamic pressure");
  return LBM_OK;
}

lbm_status lbm_set_thermo_pressure(lbm_solver *s, const double *pqk_host) {
  if (!s || !pqk_host) return LBM_E_INVALID;
  if (!(pqk_host[0] > 0.0) || !isfinite(pqk_host[0]) || !isfinite(pqk_host[1]) || !(pqk_host[2] >= 0.0) ||
      !isfinite(pqk_host[2])) {
    s->err = "thermodynamic pressure: pi > 0, finite q, K >= 0 required";
    return LBM_E_INVALID;
  }
  hipError_t e = launch_set_thermo(s->thermo, pqk_host[0], pqk_host[1], pqk_host[2], s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "setting the thermodynamic pressure");
  return LBM_OK;
}

const char *lbm_last_error(const lbm_solver *s) { return s ? s->err.c_str() : g_create_err.c_str(); }

void lbm_destroy(lbm_solver *s) { delete s; }

}  // extern "C"

// ------------------------------------------------------------------ differentiation
static lbm_status adjoint_supported(lbm_solver *s) {
  const lbm_params &p = s->p;
  const char *why = nullptr;
  if (p.lattice != LBM_D3Q27) why = "the adjoint is built for D3Q27";
  else if (p.physics != LBM_ISOTHERMAL && p.physics != LBM_PASSIVE) why = "the adjoint covers isothermal and passive-temperature flows";
  else if (p.collision != LBM_CUMULANT) why = "the adjoint covers the cumulant collision";
  else if (p.omega_high != 1.0) why = "the adjoint needs omega_high == 1";
  else if (p.galilean) why = "the adjoint covers the collision without the Galilean correction";
  else if (p.fourth_order) why = "the adjoint covers the collision without the fourth-order parameterisation";
  else if (p.precision == LBM_FP16S) why = "the adjoint runs in FP64 or FP32";
  else if (s->has_geom) why = "the adjoint covers domains without solid cells";
  else if (s->closed) why = "the adjoint covers a constant thermodynamic pressure";
  else
    for (int f = 0; f < 6; ++f)
      if (p.face_bc[f] != LBM_PERIODIC) why = "the adjoint covers periodic domains";
  if (why) {
    s->err = why;
    return LBM_E_UNSUPPORTED;
  }
  return LBM_OK;
}

extern "C" {

lbm_status lbm_adjoint_sizes(lbm_solver *s, size_t *adj_pop_bytes, size_t *adj_scal_bytes, size_t *adj_work_bytes) {
  if (!s) return LBM_E_INVALID;
  lbm_status st = adjoint_supported(s);
  if (st != LBM_OK) return st;
  const size_t r = s->prec == LBM_FP64 ? 8 : 4;
  if (adj_pop_bytes) *adj_pop_bytes = (size_t)s->Q * s->N * r;
  if (adj_scal_bytes) *adj_scal_bytes = (size_t)s->NS * s->N * r;
  if (adj_work_bytes) *adj_work_bytes = (size_t)(s->NS ? 13 : 1) * s->N * r;
  return LBM_OK;
}

lbm_status lbm_adjoint_step(lbm_solver *s, const void *state_pops, const void *state_scal, const void *adj_pop_in,
                            const void *adj_scal_in, void *adj_pop_out, void *adj_scal_out, void *adj_work) {
  if (!s) return LBM_E_INVALID;
  lbm_status st = adjoint_supported(s);
  if (st != LBM_OK) return st;
  if (!state_pops || !adj_pop_in || !adj_pop_out || adj_pop_in == adj_pop_out ||
      (s->NS && (!state_scal || !adj_scal_in || !adj_scal_out || !adj_work || adj_scal_in == adj_scal_out))) {
    s->err = "adjoint step: state, distinct in/out adjoint buffers and the work buffer are required";
    return LBM_E_INVALID;
  }
  StepArgs a = make_args(s);
  a.pop_in = state_pops;
  a.scal_in = state_scal;
  hipError_t e = launch_adjoint(s->prec, s->NS, 0, a, s->nblocks, s->stream, adj_pop_in, adj_scal_in, adj_pop_out,
                                adj_scal_out, adj_work, 0.0, nullptr, nullptr);
  if (e != hipSuccess) return hip_fail(s, e, "adjoint kernels");
  return LBM_OK;
}

lbm_status lbm_objective(lbm_solver *s, const void *state_pops, const void *state_scal, double *J_host,
                         void *adj_pop_out, void *adj_scal_out) {
  if (!s) return LBM_E_INVALID;
  lbm_status st = adjoint_supported(s);
  if (st != LBM_OK) return st;
  if (!state_pops || (s->NS && !state_scal)) {
    s->err = "objective: state buffers are required";
    return LBM_E_INVALID;
  }
  StepArgs a = make_args(s);
  a.pop_in = state_pops;
  a.scal_in = state_scal;
  a.partials = s->aux;
  hipError_t e = launch_adjoint(s->prec, s->NS, 1, a, s->nblocks, s->stream, nullptr, nullptr, nullptr, nullptr,
                                nullptr, 0.0, nullptr, nullptr);
  if (e != hipSuccess) return hip_fail(s, e, "objective sums");
  double sums[8];
  e = launch_finalize(s->aux, s->nblocks, s->stage, s->sums, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(sums, s->sums, sizeof sums, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "objective sums");
  const double mean_T = sums[1] / (double)s->N;
  if (J_host) *J_host = sums[0] + (s->NS ? sums[2] - sums[1] * mean_T : 0.0);
  if (adj_pop_out) {
    e = launch_adjoint(s->prec, s->NS, 2, a, s->nblocks, s->stream, nullptr, nullptr, adj_pop_out, adj_scal_out,
                       nullptr, mean_T, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(s, e, "objective gradient");
  }
  return LBM_OK;
}

lbm_status lbm_init_adjoint(lbm_solver *s, const void *adj_pop, const void *adj_scal, const double *u0,
                            double *grad_u, double *grad_scal) {
  if (!s) return LBM_E_INVALID;
  lbm_status st = adjoint_supported(s);
  if (st != LBM_OK) return st;
  if (!adj_pop || !u0 || !grad_u || (s->NS && grad_scal && !adj_scal)) {
    s->err = "init adjoint: adjoint populations, u0 and grad_u are required";
    return LBM_E_INVALID;
  }
  StepArgs a = make_args(s);
  hipError_t e = launch_adjoint(s->prec, s->NS, 3, a, s->nblocks, s->stream, adj_pop, adj_scal, nullptr, grad_scal,
                                nullptr, 0.0, u0, grad_u);
  if (e != hipSuccess) return hip_fail(s, e, "init adjoint");
  return LBM_OK;
}

}  // extern "C"
