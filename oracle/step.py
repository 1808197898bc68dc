"""One time step of the hybrid scheme (Eq. 1 with Eqs. 2-14 and the scalar update of
Sec. 2.3), the equilibrium initialisation, field extraction and the FP64 global sums.

State at level n: post-collision populations g*(n-1) (before streaming; Q x grid), the
scalars (T, Y_1..) at level n, and the step counter n.  One step, for every cell r:
 1. pull g_i(r, n) = g*_i(r - c_i, n-1) with boundary substitutions (below);
 2. rho^n from the ideal gas; non-advective RHS R and Lambda (Eq. 3);
 3. P_h, u from Eq. 7;  4. grad(rho) by central differences;  5. Xi (Eq. 2);
 6. f' (Eq. 13);  7. collision (cumulant, Eq. 9 as read, optionally with the Galilean
    correction of the cumulant module; or BGK in the same frame);
 8. g* (Eq. 8);  9. explicit Euler update of the scalars with u^n (Sec. 2.3);
10. FP64 sums over fluid cells at level n;
11. closed domains only: the thermodynamic pressure of level n+1 from mass conservation
    (module pressure), whose rate also enters steps 2 and 9.
Solid cells keep their populations and scalars unchanged.

Boundary readings (the paper names no-slip/zero-flux/adiabatic walls, an inlet and an
exhaust without giving the methods): a link whose source r - c_i is a solid cell or
lies beyond a wall face is bounced back halfway, g_i(r) = g*_opp(i)(r); beyond an inlet
face it is a moving wall, g_i(r) = g*_opp(i)(r) + 2 w_i rho_in (c_i . u_w) with
u_w = u_in (1 + a xi) and xi the counter-based noise; beyond an outlet face it is an
anti-bounce-back pressure condition, g_i(r) = -g*_opp(i)(r) + 2 w_i [P_out +
rho ((c_i . u_w)^2/(2 cs2) - u_w^2/2)] with rho = rho^n(r) and u_w the momentum of the
cell's own post-collision populations.  A link leaving through several faces takes the
first of wall, inlet, outlet.  Periodic faces wrap.  With a signed wall distance phi
(curved walls, module curved) links from solid cells use the interpolated bounce-back.
"""
import torch

from . import cumulant, curved, equations, noise, pressure, scalars
from .grid import INLET, OUTLET, SOLID, Grid
from .lattice import CS2, get as get_lattice


def _w(lat, i):
    return float(lat.w[i])


def inlet_velocity(params, grid, n):
    """u_w on every cell (only read at links that cross the inlet face)."""
    D = grid.D
    u_in = torch.tensor([float(v) for v in params["inlet_u"][:D]], dtype=torch.float64)
    amp = float(params["inlet_noise"])
    face_axis = None
    for d in range(D):
        if "inlet" in (params["face_bc"][2 * d], params["face_bc"][2 * d + 1]):
            face_axis = d
    scale = torch.ones(grid.shape, dtype=torch.float64)
    if face_axis is not None and amp != 0.0:
        others = [a for a in range(3) if a != face_axis]
        # coordinates in the full domain (a sub-window declares its origin)
        origin = params.get("noise_origin", (0, 0, 0))
        coords = [grid.coord[d] + int(origin[d]) for d in range(3)]
        a_c = coords[others[0]].numpy()
        b_c = coords[others[1]].numpy()
        xi = noise.xi(params["seed"], a_c, b_c, n)
        scale = 1.0 + amp * torch.from_numpy(xi)
    return u_in.reshape(D, 1, 1, 1) * scale


def pull(params, lat, grid, A, rho, n):
    D = grid.D
    g = torch.empty_like(A)
    rho_in = scalars.density(params, scalars.inlet_scalars(params).reshape(-1, 1, 1, 1),
                             (1, 1, 1)).reshape(())
    u_in = inlet_velocity(params, grid, n)
    u_out = torch.einsum("qd,q...->d...", lat.c, A) / (CS2 * rho)
    uu_out = (u_out * u_out).sum(0)
    P_out = float(params["outlet_P"])
    for i in range(lat.Q):
        c = [int(v) for v in lat.ci[i]]
        offs = [-c[d] for d in range(D)] + [0] * (3 - D)
        src = grid.shift_vec(A[i], offs)
        solid_src = grid.shift_vec(grid.solid, offs)
        wall = torch.zeros(grid.shape, dtype=torch.bool)
        inl = torch.zeros_like(wall)
        outl = torch.zeros_like(wall)
        for d in range(D):
            if c[d] == 0:
                continue
            outside, code = grid.face_of(d, -c[d])
            wall |= outside & (code == SOLID)
            inl |= outside & (code == INLET)
            outl |= outside & (code == OUTLET)
        opp = A[int(lat.opp[i])]
        val_solid = opp
        if grid.phi is not None:
            phi_src = grid.shift_vec(grid.phi, offs)
            q = curved.fraction(grid.phi, torch.where(solid_src, phi_src, grid.phi - 1.0))
            ahead = [c[d] for d in range(D)] + [0] * (3 - D)            # r + c_i
            nxt_fluid = ~grid.shift_vec(grid.solid, ahead)
            for d in range(D):
                if c[d]:
                    nxt_fluid &= ~grid.face_of(d, c[d])[0]
            val_solid = curved.bounce_back(q, opp, grid.shift_vec(opp, ahead), A[i], nxt_fluid)
        cu_in = sum(c[d] * u_in[d] for d in range(D))
        cu_out = sum(c[d] * u_out[d] for d in range(D))
        val_bb = opp
        val_in = opp + 2.0 * _w(lat, i) * rho_in * cu_in
        val_out = -opp + 2.0 * _w(lat, i) * (P_out + rho * (cu_out * cu_out / (2 * CS2) - uu_out / 2))
        g[i] = torch.where(wall, val_bb,
                           torch.where(inl, val_in,
                                       torch.where(outl, val_out,
                                                   torch.where(solid_src, val_solid, src))))
    return g


def _grid_of(params, solid, phi=None):
    return Grid(params, solid, phi)


def init_state(params, P_h, u, scal, solid=None, phi=None):
    """Populations at the equilibrium of Eq. 6 for the given fields (no non-equilibrium
    part): g*(-1) := g_eq(P_h, rho(T, Y), u).  Fields are (nz, ny, nx) / (D, nz, ny, nx).
    phi (optional): signed wall distance at the nodes for curved walls; the solid cells are
    then phi < 0."""
    lat = get_lattice(params["lattice"])
    if phi is not None:
        phi = phi.to(torch.float64)
        solid = phi < 0
    grid = _grid_of(params, solid, phi)
    scal = scal.to(torch.float64) if scal is not None else torch.zeros((0,) + grid.shape,
                                                                       dtype=torch.float64)
    rho = scalars.density(params, scal, grid.shape)
    A = equations.g_eq(lat, P_h.to(torch.float64), rho, u.to(torch.float64))
    return {"pops": A, "scal": scal.clone(), "step": 0, "solid": grid.solid,
            "thermo": pressure.initial(), "phi": phi}


def _thermo(state):
    return state.get("thermo", pressure.initial())


def _level_n(params, state):
    """Everything the step computes at level n before collision."""
    lat = get_lattice(params["lattice"])
    grid = _grid_of(params, state["solid"], state.get("phi"))
    scal = state["scal"]
    thermo = _thermo(state)
    rho = scalars.density(params, scal, grid.shape, thermo[0])
    g = pull(params, lat, grid, state["pops"], rho, state["step"])
    R, Lam = scalars.nonadvective_rhs(params, grid, scal, rho, thermo[0])
    R, Lam = pressure.apply(params, R, Lam, scal[0] if scal.shape[0] else None, thermo)
    P_h, u = equations.moments(lat, g, rho, Lam)
    if params["physics"] in ("one_step", "two_step"):
        rho_in = scalars.density(params, scalars.inlet_scalars(params).reshape(-1, 1, 1, 1),
                                 (1, 1, 1)).reshape(())
        grad_rho = scalars.density_gradient(params, grid, scal, rho, float(rho_in), thermo[0])
    else:
        grad_rho = torch.zeros((grid.D,) + grid.shape, dtype=torch.float64)
    return lat, grid, rho, g, R, Lam, P_h, u, grad_rho


def _w_over_T_sum(params, grid, scal):
    f = grid.fluid
    if params["physics"] in ("isothermal", "passive"):
        return float(f.sum()) / float(params["T_ref"])
    return float(scalars.w_over_T(params, scal, grid.shape)[f].sum())


def reductions(params, grid, rho, P_h, u, scal):
    f = grid.fluid
    out = torch.zeros(8, dtype=torch.float64)
    out[0] = rho[f].sum()
    out[1] = P_h[f].sum()
    for d in range(grid.D):
        out[2 + d] = (rho * u[d])[f].sum()
    out[5] = 0.5 * (rho * (u * u).sum(0))[f].sum()
    out[6] = _w_over_T_sum(params, grid, scal)
    if scal.shape[0] >= 2:
        out[7] = (rho * scal[1])[f].sum()
    return out


def step(params, state):
    """Advance the state by one time step; returns (new_state, sums at level n)."""
    lat, grid, rho, g, R, Lam, P_h, u, grad_rho = _level_n(params, state)
    Xi = equations.source_Xi(lat, rho, u, grad_rho, Lam)
    fp = equations.precondition(g, Xi, rho)
    nu = scalars.viscosity(params, rho, state["scal"][0] if state["scal"].shape[0] else None)
    if params["collision"] == "cumulant":
        fps, _ = cumulant.cumulant_collide(lat, fp, u, nu, params["cs_smag"],
                                           params["omega_bulk"], params["omega_high"],
                                           galilean=bool(params.get("galilean", 0)),
                                           fourth_order=bool(params.get("fourth_order", 0)))
    else:
        w = lat.w.reshape((-1,) + (1,) * 3)
        f_t = fp - w * (fp.sum(0) - 1.0)
        kappa = cumulant.central_moments(lat, f_t, u)
        om = cumulant.smagorinsky_omega(lat, kappa, nu, params["cs_smag"])
        fps = equations.bgk_preconditioned(lat, fp, P_h, rho, u, om)
    gs = equations.post_collision(fps, Xi, rho)
    new_scal = scalars.advance(params, grid, state["scal"], u, R)
    solid = grid.solid
    gs = torch.where(solid, state["pops"], gs)
    if new_scal.shape[0]:
        new_scal = torch.where(solid, state["scal"], new_scal)
    sums = reductions(params, grid, rho, P_h, u, state["scal"])
    thermo = _thermo(state)
    if pressure.closed(params):
        thermo = pressure.update(thermo, float(sums[6]), _w_over_T_sum(params, grid, new_scal))
    return ({"pops": gs, "scal": new_scal, "step": state["step"] + 1,
             "solid": state["solid"], "thermo": thermo, "phi": state.get("phi")}, sums)


def fields(params, state):
    """(P_h, rho, u, scalars, sums) at the state's level n."""
    lat, grid, rho, g, R, Lam, P_h, u, grad_rho = _level_n(params, state)
    return P_h, rho, u, state["scal"], reductions(params, grid, rho, P_h, u, state["scal"])


def run(params, state, nsteps):
    sums = None
    for _ in range(nsteps):
        state, sums = step(params, state)
    return state, sums


# ------------------------------------------------------------------ storage-format bridge
def from_storage(params, ghat, P0=None):
    """Populations from the library's storage format ghat_i = g_i/P0 - w_i (P0 = rho_ref cs2)."""
    lat = get_lattice(params["lattice"])
    P0 = params["rho_ref"] * CS2 if P0 is None else P0
    return P0 * (ghat.to(torch.float64) + lat.w.reshape((-1, 1, 1, 1)))


def to_storage(params, g):
    lat = get_lattice(params["lattice"])
    P0 = params["rho_ref"] * CS2
    return g / P0 - lat.w.reshape((-1, 1, 1, 1))
