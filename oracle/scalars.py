"""Energy and species balance of Sec. 2.3 (finite differences, explicit Euler, third-order
WENO advection, centred second-order diffusion), the low-Mach ideal-gas density that
enters Eq. 3, the thickened-flame scaling and the chemistry.

Readings (the paper defers the coupling details to earlier work):
* Non-conservative balances with constant c_p and unity Lewis number:
  DT/Dt = (1/rho) div(rho F D grad T) + omega_T/(F rho c_p),
  DY_k/Dt = (1/rho) div(rho F D grad Y_k) + omega_k/(F rho),
  D = nu/Pr; F the uniform thickening factor (diffusion times F, reaction over F).
* Diffusion: flux across face i+1/2 is (rho D)_{i+1/2} (phi_{i+1} - phi_i) with the
  arithmetic mean of rho D; no flux through walls, solid faces and the outlet; the inlet
  ghost holds the inlet value.
* Lambda of Eq. 3 uses the non-advective right-hand sides R (diffusion + reaction) at the
  current level: Lambda = R_T/T + sum_k (W/W_k) R_k, the same numbers that drive the
  update, so that D/Dt is consistent between the flow and the scalar solver.
* WENO3 (Jiang-Shu): face values from stencils {i-1, i} and {i, i+1}, linear weights 1/3
  and 2/3, smoothness (difference)^2, alpha = d/(eps + beta)^2, eps = 1e-6 R^2 with R the
  scalar's range, upwinded per axis on the sign of u_d at the cell (u_d >= 0 left-biased).
* Ghost values for stencils at walls/solids are mirror images about the wall face; at the
  inlet the inlet value; at the outlet the nearest interior value.
* Ideal gas: rho = rho_ref (T_ref/T)(W/W_ref) pi, pi = P_th/P_th(0) the thermodynamic
  pressure relative to the one at which rho_ref is given (pi = 1 in an open domain).
"""
import torch

from . import curved, transport
from .grid import FLUID, INLET, OUTLET, SOLID


# ----------------------------------------------------------------------------- thermo
def mixture_W(params, Y):
    """W = 1 / sum_k Y_k/W_k over the transported species and N2 by closure."""
    ch = params["chem"]
    Wk = ch[5:11]
    yn2 = 1.0 - Y.sum(0)
    inv = yn2 / Wk[5]
    for k in range(5):
        inv = inv + Y[k] / Wk[k]
    return 1.0 / inv


def density(params, scal, shape, pth=1.0):
    phys = params["physics"]
    if phys in ("isothermal", "passive"):
        return torch.full(shape, float(params["rho_ref"]), dtype=torch.float64)
    T = scal[0]
    if phys == "one_step":
        return params["rho_ref"] * params["T_ref"] / T * pth
    W = mixture_W(params, scal[1:])
    return params["rho_ref"] * (params["T_ref"] / T) * (W / params["chem"][17]) * pth


def w_over_T(params, scal, shape):
    """W/T per cell: the density per unit thermodynamic pressure up to a constant
    (1/T for the one-step model's constant W, 1/T_ref without a temperature)."""
    phys = params["physics"]
    if phys in ("isothermal", "passive"):
        return torch.full(shape, 1.0 / float(params["T_ref"]), dtype=torch.float64)
    if phys == "one_step":
        return 1.0 / scal[0]
    return mixture_W(params, scal[1:]) / scal[0]


def viscosity(params, rho, T=None):
    """Molecular kinematic viscosity: constant nu, constant dynamic viscosity, or (with
    mixture-averaged transport) the power law of module transport."""
    if transport.enabled(params):
        return transport.viscosity(params, T) / rho
    if params["visc_law"] == "const_nu":
        return params["nu_ref"] + torch.zeros_like(rho)
    return params["nu_ref"] * params["rho_ref"] / rho


def inlet_scalars(params):
    S = n_scalars(params)
    vals = [float(params["inlet_T"])] + [float(y) for y in params["inlet_Y"][:S - 1]]
    return torch.tensor(vals[:S], dtype=torch.float64)


def n_scalars(params):
    return {"isothermal": 0, "passive": 1, "one_step": 2, "two_step": 6}[params["physics"]]


# ----------------------------------------------------------------------------- stencils
def stencil(grid, phi, d, phi_in):
    """Values v[-2..2] along axis d around every cell, with the ghost rules."""
    st = {k: grid.status(d, k) for k in (-2, -1, 1, 2)}
    raw = {k: grid.shift(phi, d, k) for k in (-2, -1, 1, 2)}
    pin = torch.full_like(phi, float(phi_in))
    v0 = phi

    def first(k):
        s = st[k]
        return torch.where(s == FLUID, raw[k], torch.where(s == INLET, pin, v0))

    v = {0: v0, 1: first(1), -1: first(-1)}
    for k in (1, -1):
        s1, s2 = st[k], st[2 * k]
        beyond = torch.where(s2 == FLUID, raw[2 * k], torch.where(s2 == INLET, pin, v[k]))
        ghost = torch.where(s1 == SOLID, v[-k], torch.where(s1 == INLET, pin, v0))
        v[2 * k] = torch.where(s1 == FLUID, beyond, ghost)
    if grid.phi is not None:
        v = _curved_ghosts(grid, d, v, raw, st)
    return v


def _curved_ghosts(grid, d, v, raw, st):
    """Mirror-image ghosts about curved walls (module curved) for stencil points that are
    solid cells; faces and cells without a fluid line behind them keep the plain rule."""
    out = dict(v)
    phi = grid.phi
    for k in (1, -1):
        cell1, cell2 = grid.solid_cell(d, k), grid.solid_cell(d, 2 * k)
        back1 = st[-k] == FLUID
        back2 = st[-2 * k] == FLUID
        # wall between node 0 and node k
        q1 = curved.fraction(phi, torch.where(cell1, grid.shift(phi, d, k), phi - 1.0))
        g1 = curved.mirror_value(1.0 - 2.0 * q1, v[0], raw[-k], raw[-2 * k])
        p2 = 2.0 - 2.0 * q1
        g2 = curved.mirror_value(p2, v[0], raw[-k], raw[-2 * k])
        ok1 = cell1 & back1
        out[k] = torch.where(ok1, g1, out[k])
        out[2 * k] = torch.where(ok1 & ((p2 <= 1.0) | back2), g2, out[2 * k])
        # wall between node k (fluid) and node 2k
        pk = grid.shift(phi, d, k)
        q2 = curved.fraction(pk, torch.where(cell2, grid.shift(phi, d, 2 * k), pk - 1.0))
        g3 = curved.mirror_value(1.0 - 2.0 * q2, raw[k], v[0], v[0])
        out[2 * k] = torch.where((st[k] == FLUID) & cell2, g3, out[2 * k])
    return out


def weno3_face(a, b, c, eps):
    """Face value between b and c reconstructed from the upwind-biased triple (a, b, c)."""
    beta0 = (b - a) ** 2
    beta1 = (c - b) ** 2
    alpha0 = (1.0 / 3.0) / (eps + beta0) ** 2
    alpha1 = (2.0 / 3.0) / (eps + beta1) ** 2
    return (alpha0 * (-0.5 * a + 1.5 * b) + alpha1 * (0.5 * b + 0.5 * c)) / (alpha0 + alpha1)


def weno3_derivative(v, u_d, eps):
    """d(phi)/dx_d at the cell from WENO3 face values, upwinded on the sign of u_d."""
    pos = (weno3_face(v[-1], v[0], v[1], eps) - weno3_face(v[-2], v[-1], v[0], eps))
    neg = (weno3_face(v[2], v[1], v[0], eps) - weno3_face(v[1], v[0], v[-1], eps))
    return torch.where(u_d >= 0, pos, neg)


def diffusion(grid, phi, rhoD, d, phi_in, rhoD_in):
    """Centred second-order div(rho D grad phi) contribution of axis d."""
    out = torch.zeros_like(phi)
    for k in (1, -1):
        s = grid.status(d, k)
        phi_n = grid.shift(phi, d, k)
        rd_n = grid.shift(rhoD, d, k)
        flux_f = 0.5 * (rhoD + rd_n) * (phi_n - phi)
        flux_i = 0.5 * (rhoD + rhoD_in) * (phi_in - phi)
        out = out + torch.where(s == FLUID, flux_f, torch.where(s == INLET, flux_i, 0.0))
    return out


def density_gradient(params, grid, scal, rho, rho_in, pth=1.0):
    """Central differences of the density; with curved walls the ghost of a solid cell
    is the ideal-gas density of the ghost scalars (module curved), else as gradient()."""
    if grid.phi is None:
        return gradient(grid, rho, rho_in)
    S = n_scalars(params)
    phin = inlet_scalars(params)
    out = []
    for d in range(grid.D):
        st = [stencil(grid, scal[s], d, phin[s]) for s in range(S)]
        vals = []
        for k in (1, -1):
            s = grid.status(d, k)
            ghost_scal = torch.stack([st[q][k] for q in range(S)])
            rho_ghost = density(params, ghost_scal, grid.shape, pth)
            plain = torch.where(s == FLUID, grid.shift(rho, d, k),
                                torch.where(s == INLET, torch.full_like(rho, rho_in), rho))
            vals.append(torch.where(grid.solid_cell(d, k), rho_ghost, plain))
        out.append(0.5 * (vals[0] - vals[1]))
    return torch.stack(out)


def gradient(grid, f, f_in):
    """Central differences of f along each axis with the first-neighbour ghost rule
    (mirror at solids/walls, inlet value at the inlet, nearest value at the outlet)."""
    out = []
    for d in range(grid.D):
        vals = []
        for k in (1, -1):
            s = grid.status(d, k)
            vals.append(torch.where(s == FLUID, grid.shift(f, d, k),
                                    torch.where(s == INLET, torch.full_like(f, f_in), f)))
        out.append(0.5 * (vals[0] - vals[1]))
    return torch.stack(out)


# ----------------------------------------------------------------------------- chemistry
def reaction_rates(params, rho, scal):
    """Reaction source terms omega_k/rho (per species) and omega_T/(rho c_p) before the
    1/F thickening scaling.  Returns (rT, [rY_k])."""
    ch = params["chem"]
    T = scal[0]
    if params["physics"] == "one_step":
        B, Ta, Tu, Tad, Yu = ch[0], ch[1], ch[2], ch[3], ch[4]
        r = B * torch.clamp(scal[1], min=0.0) * torch.exp(-Ta / T)
        return (Tad - Tu) / Yu * r, [-r]
    # two-step: CH4 + 1.5 O2 -> CO + 2 H2O ; CO + 0.5 O2 -> CO2
    B1, Ta1, B2, Ta2, cp = ch[0], ch[1], ch[2], ch[3], ch[4]
    Wk, hk = ch[5:11], ch[11:17]
    Y = scal[1:]
    conc = [rho * torch.clamp(Y[k], min=0.0) / Wk[k] for k in range(5)]
    q1 = B1 * torch.exp(-Ta1 / T) * conc[0] * conc[1]
    q2 = B2 * torch.exp(-Ta2 / T) * conc[2] * torch.sqrt(conc[1])
    nu1 = [-1.0, -1.5, 1.0, 0.0, 2.0, 0.0]
    nu2 = [0.0, -0.5, -1.0, 1.0, 0.0, 0.0]
    molar = [(nu1[k] * q1 + nu2[k] * q2) / rho for k in range(6)]   # mol/mass/time
    rY = [Wk[k] * molar[k] for k in range(5)]
    rT = -sum(hk[k] * molar[k] for k in range(6)) / cp
    return rT, rY


def nonadvective_rhs(params, grid, scal, rho, pth=1.0):
    """R_phi = (1/rho) sum_d div_d(rho F D grad phi) + reaction/F, and Lambda (Eq. 3);
    with mixture-averaged transport the diffusive parts come from module transport."""
    S = n_scalars(params)
    F = params["thickening"]
    if transport.enabled(params):
        phin = inlet_scalars(params)
        rho_in = density(params, phin.reshape(S, 1, 1, 1), (1, 1, 1), pth).reshape(())
        RT, RY, cp = transport.rhs(params, grid, scal, rho, phin, rho_in, pth)
        _, rY = reaction_rates(params, rho, scal)
        Wk = params["chem"][5:11]
        rT = -sum(transport.enthalpy(params, scal[0], k) * rY[k] / Wk[k] for k in range(5)) / cp
        R = [RT + rT / F] + [RY[k] + rY[k] / F for k in range(5)]
        R = torch.stack(R)
        Wk = params["chem"][5:11]
        W = mixture_W(params, scal[1:])
        R_n2 = -R[1:].sum(0)
        Lam = R[0] / scal[0] + W * (sum(R[1 + k] / Wk[k] for k in range(5)) + R_n2 / Wk[5])
        return R, Lam
    nu = viscosity(params, rho)
    rhoD = rho * nu / params["prandtl"]
    phin = inlet_scalars(params)
    rho_in = density(params, phin.reshape(S, 1, 1, 1), (1, 1, 1)).reshape(())
    rhoD_in = rho_in * viscosity(params, rho_in) / params["prandtl"]
    R = []
    for s in range(S):
        acc = torch.zeros_like(rho)
        for d in range(grid.D):
            acc = acc + diffusion(grid, scal[s], rhoD, d, phin[s], rhoD_in)
        R.append(F * acc / rho)
    phys = params["physics"]
    if phys in ("one_step", "two_step"):
        rT, rY = reaction_rates(params, rho, scal)
        R[0] = R[0] + rT / F
        for k, r in enumerate(rY):
            R[1 + k] = R[1 + k] + r / F
    R = torch.stack(R) if S else torch.zeros((0,) + rho.shape, dtype=torch.float64)
    if phys == "one_step":
        Lam = R[0] / scal[0]                       # constant molar mass: species sum is 0
    elif phys == "two_step":
        Wk = params["chem"][5:11]
        W = mixture_W(params, scal[1:])
        R_n2 = -R[1:].sum(0)
        Lam = R[0] / scal[0] + W * (sum(R[1 + k] / Wk[k] for k in range(5)) + R_n2 / Wk[5])
    else:
        Lam = torch.zeros_like(rho)
    return R, Lam


def advance(params, grid, scal, u, R):
    """Explicit Euler: phi^{n+1} = phi^n + dt (-sum_d u_d dphi/dx_d + R_phi)."""
    S = n_scalars(params)
    phin = inlet_scalars(params)
    out = []
    for s in range(S):
        eps = 1e-6 * float(params["weno_scale"][s]) ** 2
        adv = torch.zeros_like(scal[s])
        for d in range(grid.D):
            v = stencil(grid, scal[s], d, phin[s])
            adv = adv + u[d] * weno3_derivative(v, u[d], eps)
        out.append(scal[s] + (-adv + R[s]))
    return torch.stack(out) if S else scal
