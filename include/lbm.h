/*
 * lbm.h - C ABI of the MI355X (gfx950) hybrid low-Mach lattice-Boltzmann /
 * finite-difference time step of Hosseini, Darabiha, Thevenin, "Low Mach number lattice
 * Boltzmann model for turbulent combustion: flow in confined geometries"
 * (arXiv 2207.11567).
 *
 * One time step (Sec. 2, Eq. 1): pull-streaming of the pressure/momentum populations g_i
 * (D2Q9 or D3Q27, Sec. 2.1), the source term Xi_i of Eq. 2 with Lambda of Eq. 3, the
 * moments of Eq. 7, pre-conditioning (Eq. 13), the cumulant collision in the
 * pre-conditioned frame (Eqs. 9-12, Sec. 2.2) with a Smagorinsky shear rate, the
 * post-collision form of Eq. 8, and the explicit-Euler finite-difference update of
 * temperature and species (third-order WENO advection, centred diffusion, Sec. 2.3) with
 * Arrhenius chemistry, thickened-flame scaling and ideal-gas density; bounce-back walls,
 * a velocity inlet and a pressure outlet.  Global FP64 sums (mass, pressure, momentum,
 * kinetic energy, thermodynamic-pressure integral) are formed every step.
 *
 * Closed domains (pth_mode = LBM_PTH_CLOSED; the confined deflagration of Sec. 3.1, whose
 * pressure climbs as the flame accelerates): Eq. 3 holds at a constant thermodynamic
 * pressure P_th and the paper gives no closed-domain form, so the library takes the usual
 * low-Mach one.  pi = P_th/P_th(0) scales the ideal-gas density; q = dln(pi)/dt adds the
 * pressure work kappa T q (kappa = (gamma-1)/gamma) to the temperature right-hand side and
 * the velocity divergence that enters Xi (Eq. 2) and P_h (Eq. 7a) is Lambda - q; after
 * each step pi is set so that the total mass sum rho over fluid cells is that of level 0
 * (pi' = K / sum W/T of the updated scalars, K = pi sum W/T at level 0) and q is the
 * backward difference (pi' - pi)/pi, used by the next step.
 *
 * Conventions
 *  - Lattice units: dr = dt = 1, cs^2 = 1/3.  P0 = rho_ref cs^2.
 *  - Cells are ordered x fastest: n = x + nx (y + ny z); nz = 1 for D2Q9.
 *  - Population i has velocity (cx, cy, cz) with i = (cx+1) + 3 (cy+1) + 9 (cz+1); its
 *    opposite is Q-1-i.  Populations are stored structure-of-arrays, [Q][nz][ny][nx],
 *    as the deviation ghat_i = g_i/P0 - w_i in the storage precision (FP64, FP32, or FP16
 *    for LBM_FP16S).
 *  - Scalars are stored [S][nz][ny][nx] in FP64 (LBM_FP64) or FP32 (otherwise), with
 *    S = 0 (isothermal), 1 (passive T), 2 (T, Y_fuel), 6 (T, Y_CH4, Y_O2, Y_CO, Y_CO2,
 *    Y_H2O; Y_N2 = 1 - sum).
 *  - Field arrays exchanged with lbm_init_fields / lbm_fields are FP64: P_h and rho
 *    [nz][ny][nx], u [D][nz][ny][nx], scalars [S][nz][ny][nx].
 *  - The state at level n is (post-collision populations of level n-1, scalars at n, n).
 *
 * Ownership: every device buffer is allocated by the caller and passed as a device
 * pointer; the library keeps the pointers for the solver's lifetime, never frees them and
 * allocates no device memory of its own.  All work is ordered on the caller's HIP stream:
 * where a step runs split (boundary cells in a second kernel), that kernel runs on a side
 * stream the solver creates on first use, forked from the caller's stream by an event
 * before the step and joined back into it after, so later work on the caller's stream sees
 * the whole step.  lbm_step does not synchronise, lbm_fields and the state copies do;
 * lbm_destroy waits for the side stream.
 * Errors: every call returns an lbm_status; lbm_last_error gives a message.  A
 * non-finite value produced by a step raises a device flag reported as LBM_E_DIVERGED by
 * the next synchronising call.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_solver lbm_solver;

typedef enum {
  LBM_OK = 0,
  LBM_E_INVALID = -1,     /* bad parameter, size or null pointer */
  LBM_E_UNSUPPORTED = -2, /* valid but not built (e.g. BGK with an adjoint) */
  LBM_E_HIP = -3,         /* a HIP runtime call failed */
  LBM_E_DIVERGED = -4,    /* a non-finite value appeared in a step */
  LBM_E_STATE = -5        /* call out of order (e.g. step before init) */
} lbm_status;

enum { LBM_D2Q9 = 9, LBM_D3Q27 = 27 };
enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16S = 2 };
enum { LBM_CUMULANT = 0, LBM_BGK = 1 };
enum { LBM_ISOTHERMAL = 0, LBM_PASSIVE = 1, LBM_ONE_STEP = 2, LBM_TWO_STEP = 3 };
enum { LBM_VISC_CONST_NU = 0, LBM_VISC_CONST_MU = 1 };
enum { LBM_PERIODIC = 0, LBM_WALL = 1, LBM_INLET = 2, LBM_OUTLET = 3 };
enum { LBM_PTH_OPEN = 0, LBM_PTH_CLOSED = 1 };
enum { LBM_TRANSPORT_SIMPLE = 0, LBM_TRANSPORT_MIXTURE = 1 };

/* Problem statement (Sec. 2 and 3 of the paper), lattice units. */
typedef struct {
  int32_t lattice;    /* LBM_D2Q9 | LBM_D3Q27 */
  int32_t nx, ny, nz; /* grid; nz == 1 for D2Q9 */
  int32_t precision;  /* LBM_FP64 | LBM_FP32 | LBM_FP16S (FP16 storage, FP32 math) */
  int32_t collision;  /* LBM_CUMULANT (Sec. 2.2) | LBM_BGK (Eq. 5, test mode) */
  int32_t physics;    /* LBM_ISOTHERMAL | LBM_PASSIVE | LBM_ONE_STEP | LBM_TWO_STEP */
  int32_t visc_law;   /* LBM_VISC_CONST_NU | LBM_VISC_CONST_MU (nu = nu_ref rho_ref/rho) */
  double nu_ref;      /* kinematic viscosity at rho_ref: tau0 = nu/cs2 + 1/2 (Eq. 12) */
  double omega_bulk;  /* rate of the second-order cumulant trace */
  double omega_high;  /* rate of every cumulant of order >= 3 */
  double cs_smag;     /* Smagorinsky constant (0 = off) */
  double prandtl;     /* D = nu/Pr, unity Lewis number */
  double thickening;  /* thickened-flame factor F: D -> F D, reaction -> reaction/F */
  double rho_ref, T_ref;
  int32_t face_bc[6]; /* -x,+x,-y,+y,-z,+z: LBM_PERIODIC|LBM_WALL|LBM_INLET|LBM_OUTLET */
  double inlet_u[3];  /* inlet velocity */
  double inlet_noise; /* relative amplitude a of u_w = u_in (1 + a xi), xi unit variance */
  double outlet_P;    /* hydrodynamic pressure imposed at the outlet */
  double inlet_T;     /* inlet temperature (Dirichlet) */
  double inlet_Y[8];  /* inlet mass fractions of the transported species */
  double weno_scale[8]; /* range R of each scalar: WENO eps = 1e-6 R^2 */
  double chem[32];    /* LBM_ONE_STEP: B, Ta, T_u, T_ad, Y_u.
                         LBM_TWO_STEP: B1, Ta1, B2, Ta2, c_p, W_k[6], h_k[6], W_ref. */
  uint64_t seed;      /* counter-based inlet noise (SplitMix64) */
  int32_t pth_mode;   /* LBM_PTH_OPEN (constant P_th, Eq. 3) | LBM_PTH_CLOSED (mass held) */
  double gamma;       /* ratio of specific heats (closed domains; must exceed 1) */
  int32_t transport_model; /* LBM_TRANSPORT_SIMPLE (unity Lewis, constant c_p) |
                              LBM_TRANSPORT_MIXTURE (LBM_TWO_STEP only, see below) */
  double transport[32];    /* mixture data: binary D0_kj at T_ref for pairs k < j of
                              (CH4, O2, CO, CO2, H2O, N2) in the order (0,1) (0,2) .. (4,5)
                              [0..14], c_p,k = a_k + b_k T: a [15..20], b [21..26] (J/kg/K),
                              exponents s_mu [27], s_D [28] */
  int32_t galilean;        /* 0 | 1: Galilean correction of the cumulant collision (Geier
                              et al. 2015, whose operator Sec. 2.2 applies), see below;
                              requires LBM_CUMULANT */
  int32_t fourth_order;    /* 0 | 1: D3Q27 only, requires LBM_CUMULANT: the higher-order
                              cumulant relaxation of Geier, Pasquali and Schoenherr (2017)
                              for fourth-order accurate diffusion, see below (omega_high is
                              then unused) */
} lbm_params;

/* Fourth-order parameterisation (Geier, Pasquali, Schoenherr 2017, J. Comput. Phys. 348,
 * "Parametrization of the cumulant lattice Boltzmann method for fourth order accurate
 * diffusion, part I"; the paper's operator, Sec. 2.2, has one rate per cumulant, W = diag(
 * omega_0 .. omega_xxyyzz)): with omega_1 the shear rate of the cell and omega_2 = omega_bulk,
 * the third-order sums C_120 + C_102, C_210 + C_012, C_201 + C_021 relax to zero at
 * omega_3(omega_1, omega_2), their differences at omega_4, C_111 at omega_5; the fourth-order
 * cumulants are set to C_220 = -(2/3) A (1/omega_1 - 1/2)(d_x u_x + d_y u_y) and
 * C_112 = -(1/3) B (1/omega_1 - 1/2)(d_x u_y + d_y u_x) (and permutations), the velocity
 * gradients estimated from the pre-collision second cumulants; fifth and sixth order relax to
 * zero.  The rates are rational functions of omega_1 and omega_2 that leave (0, 2) around
 * omega_1 = 1.55 (for omega_2 = 1) and A, B are singular at omega_1 = omega_2: lbm_create
 * rejects molecular shear rates for which omega_3..5 leave (0, 2) or A, B are not finite;
 * the sub-grid model lowers the cell's rate below the molecular one, and no limiter is
 * applied.  Not covered by the adjoint. */

/* Galilean correction: on D2Q9 and D3Q27 c^3 = c, so the equilibrium third diagonal moment
 * lacks u_a^3 and the viscous stress picks up (1/omega - 1/2) 3 u_a^2 d_a u_a on each
 * diagonal.  With galilean = 1 the collision estimates d_a u_a from the pre-collision
 * second cumulants (deviatoric part at the shear rate, trace at omega_bulk) and adds
 * -3 (1 - omega/2) u_a^2 d_a u_a to the post-collision diagonal (shear rate on the
 * deviatoric differences, omega_bulk on the trace).  Not covered by the adjoint. */

/* Mixture-averaged transport (the paper evaluates its thermodynamic and transport
 * properties with mixture-averaged approximations, Sec. 2.3; the module and data are
 * not given, read as follows): mu = nu_ref rho_ref (T/T_ref)^s_mu, c_p = sum Y_k c_p,k(T),
 * lambda = mu c_p / Pr; D_kj = D0_kj (T/T_ref)^s_D / pi; D_k = (1 - Y_k)/sum_{j!=k} X_j/D_kj;
 * face fluxes J*_k = -(rho D_k W_k/W)_f (X_k,nb - X_k), J_k = J*_k - (Y_k)_f sum_j J*_j
 * (face values: means of the two cells); R_T = F/(rho c_p) div(lambda grad T) plus the
 * heat release -sum_k h_k(T) omega_k/(F rho c_p) with h_k(T) = h0_k + W_k int_{298.15}^T
 * c_p,k; R_k = -(F/rho) div J_k + omega_k/(F rho); the LB viscosity is mu(T)/rho. */

/* Sizes (bytes) of the caller-provided device buffers for these parameters: one
 * population array (two are needed, A and B), one scalar array (two needed), and the
 * work buffer (geometry words, the boundary-cell list, per-block FP64 partial sums,
 * flags).
 * Returns LBM_E_INVALID for invalid parameters. */
lbm_status lbm_query_sizes(const lbm_params *p, size_t *pop_bytes, size_t *scal_bytes,
                           size_t *work_bytes);

/* Validates parameters (tau0 > 1/2, F D <= 1/(2 d) Fourier limit of the explicit
 * diffusion at rho_ref, nz == 1 for D2Q9, sizes > 0, 0 <= omegas <= 2; a closed domain has
 * no inlet or outlet face and gamma > 1) and binds the buffers.  With rho nu constant or
 * mixture transport the same limit is also estimated in the hottest gas the chemistry can
 * make (T_ad of the one-step model; the inlet mixture burnt completely to CO2 and H2O for
 * the two-step one); beyond it lbm_create (and lbm_query_sizes) still succeed but leave a
 * message starting "warning:" in lbm_last_error (of the solver; of NULL for
 * lbm_query_sizes), since runs that never get that hot are valid.  stream is a
 * hipStream_t (NULL = default stream).  scal_a/scal_b may be NULL when S == 0.
 * Builds the list of boundary cells (cells within two of a non-periodic face) for a
 * split step; synchronises the stream. */
lbm_status lbm_create(const lbm_params *p, void *stream, void *pop_a, void *pop_b,
                      void *scal_a, void *scal_b, void *work, lbm_solver **out);

/* Solid cells (device uint8 [nz][ny][nx], nonzero = solid) for bounce-back walls and
 * zero-flux scalars; NULL clears the geometry.  The mask is read once here; the list of
 * boundary cells (solid, or a solid within their links or +-2 stencil, or near a
 * non-periodic face) is rebuilt on the host.  Synchronises the stream. */
lbm_status lbm_set_geometry(lbm_solver *s, const uint8_t *solid_dev);

/* Curved walls (the paper's treatment of curved boundaries for both solvers, Sec. 1 and
 * Sec. 3; methods not given, read as below).  phi_dev: device FP64 [nz][ny][nx], the
 * signed wall distance at the nodes (>= 0 fluid, < 0 solid, in cells); the solid cells are
 * phi < 0 and, along a link or grid line from a fluid node r to a solid node s, the wall
 * lies at the fraction q = phi(r)/(phi(r) - phi(s)) of the way.  Populations arriving from
 * a solid node take the linearly interpolated bounce-back of Bouzidi, Firdaouss and
 * Lallemand (2001): q < 1/2: g_i(r) = 2q g*_ib(r) + (1-2q) g*_ib(r+c_i) (halfway if
 * r + c_i is not fluid); q >= 1/2: g_i(r) = g*_ib(r)/(2q) + (1 - 1/(2q)) g*_i(r).  Scalar
 * stencil points in solid cells take the value at their mirror image about the wall on
 * the grid line (linear interpolation between fluid nodes; an image between the wall and
 * the first node takes the even quadratic through the two nearest nodes), the density
 * there is the ideal gas of those values, and diffusion fluxes through solid faces stay
 * zero.  Domain faces keep the halfway rules.  The library keeps phi_dev (the caller keeps
 * it alive until the next geometry call); NULL clears the geometry.  The boundary-cell
 * list is rebuilt as for lbm_set_geometry; steps then run split, the boundary cells in
 * the curved-wall kernel and the others in the interior kernel.  Synchronises. */
lbm_status lbm_set_wall_distance(lbm_solver *s, const double *phi_dev);

/* Equilibrium initialisation (Eq. 6): post-collision populations of level -1 are set to
 * g_eq(P_h, rho(T, Y), u); scalars copied; step counter 0; thermodynamic pressure
 * (pi, q, K) = (1, 0, 0).  Device FP64 inputs; scal may be NULL when S == 0. */
lbm_status lbm_init_fields(lbm_solver *s, const double *P_h, const double *u,
                           const double *scal);

/* Advances nsteps time steps (Eq. 1 + Sec. 2.3) asynchronously on the stream.  A closed
 * domain adds two small reduction launches per step (the pressure update). */
lbm_status lbm_step(lbm_solver *s, int32_t nsteps);

/* Fields at the current level n (P_h of Eq. 7a, rho, u of Eq. 7b, scalars), each pointer
 * may be NULL; sums_host (may be NULL) receives 8 FP64 sums over fluid cells:
 * rho, P_h, rho u_x, rho u_y, rho u_z, rho |u|^2 / 2, W/T, rho Y_1.  Synchronises. */
lbm_status lbm_fields(lbm_solver *s, double *P_h, double *rho, double *u, double *scal,
                      double *sums_host);

/* One time step from an explicit state (populations and scalars in the storage format,
 * at level `step`) into explicit output buffers, leaving the solver's own state alone;
 * used to refill a checkpoint segment before its adjoint steps.  Asynchronous.
 * LBM_E_UNSUPPORTED in a closed domain (its pressure is solver state). */
lbm_status lbm_step_from(lbm_solver *s, const void *pops_in, const void *scal_in,
                         void *pops_out, void *scal_out, int64_t step);

/* The 8 sums formed by the last lbm_step or lbm_step_from (at the level of its last step);
 * lbm_fields, lbm_flame_surface and lbm_objective keep their block records apart and
 * leave them untouched.  Synchronises. */
lbm_status lbm_step_sums(lbm_solver *s, double *sums_host);

/* Raw state copies (device-to-device, storage format): pops [Q][N], scal [S][N].
 * Synchronise.  The thermodynamic pressure is copied separately (below). */
lbm_status lbm_get_state(lbm_solver *s, void *pops_dst, void *scal_dst, int64_t *step);
lbm_status lbm_set_state(lbm_solver *s, const void *pops_src, const void *scal_src,
                         int64_t step);

/* ------------------------------------------------------------------ observables (Sec. 3)
 * Running statistics (Sec. 3.2: time-averaged velocity components, their RMS and the RMS of
 * the pressure fluctuations).  acc_dev: caller buffer of 2 (D+1) N FP64 values, zeroed
 * here; every lbm_step level n with n % every == 0 (the state before that step) is sampled
 * into running means and sums of squared deviations (Welford) of u_d and P_h.  NULL stops
 * sampling.  every < 1 with a buffer: LBM_E_INVALID. */
lbm_status lbm_set_statistics(lbm_solver *s, double *acc_dev, int32_t every);

/* Mean [D+1][N] (u_x, u_y, [u_z,] P_h) and RMS (population standard deviation) fields of
 * the samples so far, FP64 device outputs (either may be NULL), and the sample count.
 * LBM_E_STATE without samples.  Synchronises. */
lbm_status lbm_statistics(lbm_solver *s, double *mean_dev, double *rms_dev, int64_t *samples);

/* Probes (Sec. 3.2: velocity and pressure recorded at every step at points of the burner
 * axis, for their spectra): up to 8 cell indices (host array); record_dev receives one row
 * [nprobe][D+1] = (u..., P_h) per stepped level, until `capacity` rows.  NULL record or
 * nprobe 0 stops recording.  Out-of-range cells, nprobe > 8: LBM_E_INVALID. */
lbm_status lbm_set_probes(lbm_solver *s, const int64_t *cells_host, int32_t nprobe, double *record_dev,
                          int64_t capacity);
lbm_status lbm_probe_rows(lbm_solver *s, int64_t *rows);

/* Generalised flame surface (Sec. 3.1: flame-surface evolution in the chamber): the sum over
 * fluid cells of |grad c|, c = (T - T_u)/(T_b - T_u), central differences with the ghost
 * rules of grad rho, in lattice units (area in 3-D, length in 2-D), at the current level.
 * Needs a temperature (S >= 1).  Synchronises. */
lbm_status lbm_flame_surface(lbm_solver *s, double T_u, double T_b, double *surface_host);

/* The flame surface of lbm_flame_surface, for callers that cannot allocate or synchronise
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * allocates nothing and does not synchronise.  Its partial sums live in a device scratch
 * array of the library (about 9.5 MB per device, held until the process ends), not in the
 * solver's work buffer; grids up to 131072 blocks of 256 cells (33,554,432 cells) are
 * accepted, larger ones return LBM_E_INVALID.  The sum (FP64, bit for bit the value
 * lbm_flame_surface returns) is written to surface_dev, a device double, in stream order.
 * All calls on one device share that device's scratch: calls that overlap in time on one
 * device (different streams, threads or solvers) race and must be ordered by the caller.
 * Errors: LBM_E_INVALID (NULL pointers, no temperature, T_b == T_u, too many cells),
 * LBM_E_STATE (before initialisation), LBM_E_HIP (launch failure, or the scratch address
 * could not be resolved on the solver's device). */
lbm_status lbm_flame_surface_noalloc(lbm_solver *s, double T_u, double T_b, double *surface_dev);

/* Thermodynamic pressure state of the current level, three FP64 values on the host:
 * pi = P_th/P_th(0), q = dln(pi)/dt of this level (per time step), K = the held
 * mass constant (0 until the first step of a closed domain fixes it).  Open domains keep
 * (1, 0, 0).  get synchronises; set (pi > 0, finite q, K >= 0, else LBM_E_INVALID) is
 * queued on the stream, for restarts together with lbm_set_state. */
lbm_status lbm_get_thermo_pressure(lbm_solver *s, double *pqk_host);
lbm_status lbm_set_thermo_pressure(lbm_solver *s, const double *pqk_host);

/* ------------------------------------------------------------------ differentiation
 * Discrete adjoint of one time step (reverse-mode vector-Jacobian product of the exact
 * discrete step: collision, Smagorinsky shear rate, WENO3 advection with its nonlinear
 * weights, centred diffusion, streaming).  Scope: D3Q27, periodic faces, no solid cells,
 * LBM_ISOTHERMAL or LBM_PASSIVE, LBM_CUMULANT with omega_high == 1, LBM_FP64 or LBM_FP32,
 * LBM_PTH_OPEN; anything else returns LBM_E_UNSUPPORTED.  Adjoint arrays are in the compute precision
 * (FP64 or FP32), laid out like the state: populations [27][N], scalars [S][N].
 * At the upwind switch u_d = 0 the derivative of |u_d| is taken as +1. */

/* Byte sizes of one adjoint population array, one adjoint scalar array, and the scratch
 * buffer lbm_adjoint_step needs. */
lbm_status lbm_adjoint_sizes(lbm_solver *s, size_t *adj_pop_bytes, size_t *adj_scal_bytes,
                             size_t *adj_work_bytes);

/* One reverse step: given the state at level n (populations and scalars in the storage
 * format, as lbm_get_state returns them) and the adjoint of the state at level n+1,
 * writes the adjoint of the state at level n.  In and out buffers must be distinct.
 * Asynchronous on the stream. */
lbm_status lbm_adjoint_step(lbm_solver *s, const void *state_pops, const void *state_scal,
                            const void *adj_pop_in, const void *adj_scal_in, void *adj_pop_out,
                            void *adj_scal_out, void *adj_work);

/* Objective J = sum rho |u|^2 / 2 + sum (T - mean T)^2 at the given state (the second
 * term only with a passive temperature), returned on the host in FP64, and, when
 * adj_pop_out is not NULL, dJ/dstate written to adj_pop_out / adj_scal_out.
 * Synchronises. */
lbm_status lbm_objective(lbm_solver *s, const void *state_pops, const void *state_scal,
                         double *J_host, void *adj_pop_out, void *adj_scal_out);

/* Reverse of lbm_init_fields with respect to the initial velocity (and temperature):
 * from the adjoint of the level-0 state, writes grad_u [3][N] and, if grad_scal is not
 * NULL, grad_scal [S][N], both FP64.  u0 is the velocity given to lbm_init_fields. */
lbm_status lbm_init_adjoint(lbm_solver *s, const void *adj_pop, const void *adj_scal,
                            const double *u0, double *grad_u, double *grad_scal);

/* Measurement support, not part of the method: copies `bytes` (0 < bytes <= 2^31, a
 * multiple of 4) from src to dst (device pointers of the current device, not overlapping)
 * with the 4-byte raw buffer loads and stores that the step kernel uses, one element per
 * lane and 64 consecutive ones per wave.  mode bit 0: streaming (non-temporal) loads, else
 * cached ones (the step's scalar loads and its pull loads on large grids); bit 1: streaming
 * stores (the step's population stores), else cached ones (its scalar stores).  For
 * calibrating the memory counters (FETCH_SIZE, WRITE_SIZE) of exactly these forms against a
 * known byte count, and for the bandwidth they reach.  Asynchronous on `stream` (a
 * hipStream_t, NULL for the default stream); the caller keeps both buffers alive until the
 * stream has passed the copy.  LBM_E_INVALID for a bad size, mode or pointer (message in
 * lbm_last_error(NULL)), LBM_E_HIP if the launch fails. */
lbm_status lbm_copy_probe(const void *src, void *dst, size_t bytes, int32_t mode, void *stream);

/* Human-readable message of the last failure on this solver. */
const char *lbm_last_error(const lbm_solver *s);

void lbm_destroy(lbm_solver *s);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
