"""Mixture-averaged transport and variable heat capacity for the two-step CH4/air scalars
(the paper evaluates every thermodynamic and transport property by mixture-averaged
approximations in its REGATH module, Sec. 2.3; the module and its data are not
available, so this is a reading with declared placeholder data, parity unpinned against
the paper, pinned in the tests against binary Fick diffusion, the trace limit, exact
species-mass conservation, the unity-Lewis special case and the adiabatic flame
temperature of a variable-c_p reactor).

Test infrastructure: see the package header.

Species k = CH4, O2, CO, CO2, H2O, N2 (N2 by closure); data in params["transport"]:
  [0..14]  binary diffusion coefficients D0_kj at T_ref (lattice units), pairs k < j in
           the order (0,1), (0,2), ..., (0,5), (1,2), ..., (4,5);
  [15..20] a_k, [21..26] b_k: c_p,k(T) = a_k + b_k T (J/kg/K);
  [27]     viscosity exponent s_mu: mu = mu_ref (T/T_ref)^s_mu, mu_ref = nu_ref rho_ref;
  [28]     diffusion exponent s_D:  D_kj = D0_kj (T/T_ref)^s_D / pi (pi = P_th/P_th(0)).
Readings:
* mixture heat capacity c_p = sum_k Y_k c_p,k(T); conductivity lambda = mu c_p / Pr;
* mixture-averaged diffusion (Hirschfelder and Curtiss): D_k = (1 - Y_k) / sum_{j != k}
  X_j / D_kj, mole fractions X_k = Y_k W / W_k, fluxes driven by mole-fraction gradients,
  J*_k = -rho D_k (W_k / W) grad X_k;
* correction flux so that the six fluxes sum to zero at every face:
  J_k = J*_k - Y_k sum_j J*_j;
* face values (rho D_k W_k/W, mu c_p, Y_k) are arithmetic means of the two cells; no flux
  through walls, solid faces and the outlet; the inlet ghost holds the inlet state;
* T:   R_T = (F / (rho c_p)) div(lambda grad T) + omega_T / (F rho c_p), with the heat
  release omega_T = -sum_k h_k(T) omega_k from the full molar enthalpies
  h_k(T) = h0_k + W_k int_{T0}^{T} c_p,k (T0 = 298.15 K, h0_k the formation enthalpies),
  so that a uniform reactor keeps sum_k Y_k h_k(T)/W_k;
  Y_k: R_k = -(F / rho) div J_k + omega_k / (F rho)
  (the species-enthalpy diffusion term sum_k c_p,k J_k . grad T is neglected);
* Lambda (Eq. 3) and everything else as in the unity-Lewis model.
"""
import torch

from .grid import FLUID, INLET

PAIRS = [(k, j) for k in range(6) for j in range(k + 1, 6)]


def enabled(params):
    return params.get("transport_model", "simple") == "mixture"


def binary_matrix(params):
    """Symmetric 6x6 D0_kj (diagonal unused, set to 1)."""
    tr = params["transport"]
    M = torch.ones((6, 6), dtype=torch.float64)
    for n, (k, j) in enumerate(PAIRS):
        M[k, j] = M[j, k] = float(tr[n])
    return M


def full_Y(Y5):
    """(6, ...) mass fractions with N2 by closure."""
    return torch.cat([Y5, (1.0 - Y5.sum(0))[None]])


def heat_capacity(params, T, Y6):
    tr = params["transport"]
    return sum(Y6[k] * (float(tr[15 + k]) + float(tr[21 + k]) * T) for k in range(6))


T0_FORMATION = 298.15


def enthalpy(params, T, k):
    """Molar enthalpy h_k(T) (J/mol) of species k."""
    tr, ch = params["transport"], params["chem"]
    a, b = float(tr[15 + k]), float(tr[21 + k])
    return ch[11 + k] + ch[5 + k] * (a * (T - T0_FORMATION) + 0.5 * b * (T * T - T0_FORMATION ** 2))


def viscosity(params, T):
    tr = params["transport"]
    mu_ref = params["nu_ref"] * params["rho_ref"]
    return mu_ref * (T / params["T_ref"]) ** float(tr[27])


def mixture_diffusion(params, T, Y6, pth=1.0):
    """D_k (6, ...) from the binary coefficients at T and the thermodynamic pressure."""
    tr = params["transport"]
    Wk = params["chem"][5:11]
    W = 1.0 / sum(Y6[k] / Wk[k] for k in range(6))
    X = [Y6[k] * W / Wk[k] for k in range(6)]
    scale = (T / params["T_ref"]) ** float(tr[28]) / pth
    B = binary_matrix(params)
    out = []
    for k in range(6):
        s = sum(X[j] / (float(B[k, j]) * scale) for j in range(6) if j != k)
        out.append((1.0 - Y6[k]) / s)
    return torch.stack(out), torch.stack(X), W


def _neighbour(grid, f, d, k, f_in):
    s = grid.status(d, k)
    return torch.where(s == FLUID, grid.shift(f, d, k), torch.where(s == INLET, f_in, f)), \
        (s == FLUID) | (s == INLET)


def rhs(params, grid, scal, rho, scal_in, rho_in, pth=1.0):
    """Diffusive parts of R_T and of R_k for all six species (N2 last), and c_p."""
    F = params["thickening"]
    Wk = params["chem"][5:11]
    T = scal[0]
    Y6 = full_Y(scal[1:])
    cp = heat_capacity(params, T, Y6)
    Dk, X, W = mixture_diffusion(params, T, Y6, pth)
    coef = torch.stack([rho * Dk[k] * Wk[k] / W for k in range(6)])           # rho D_k W_k/W
    kap = viscosity(params, T) * cp / params["prandtl"]                       # lambda
    # inlet state
    Yin = full_Y(torch.as_tensor(scal_in[1:], dtype=torch.float64).reshape(5, *([1] * T.dim())))
    Tin = torch.as_tensor(scal_in[0], dtype=torch.float64).reshape([1] * T.dim())
    cp_in = heat_capacity(params, Tin, Yin)
    D_in, X_in, W_in = mixture_diffusion(params, Tin, Yin, pth)
    coef_in = torch.stack([rho_in * D_in[k] * Wk[k] / W_in for k in range(6)])
    kap_in = viscosity(params, Tin) * cp_in / params["prandtl"]
    RT = torch.zeros_like(T)
    RY = torch.zeros((6,) + T.shape, dtype=torch.float64)
    for d in range(grid.D):
        for k in (1, -1):
            Tn, open_ = _neighbour(grid, T, d, k, Tin)
            kn, _ = _neighbour(grid, kap, d, k, kap_in)
            RT = RT + torch.where(open_, 0.5 * (kap + kn) * (Tn - T), 0.0)
            Jstar, Yf = [], []
            for q in range(6):
                Xn, _ = _neighbour(grid, X[q], d, k, X_in[q])
                cn, _ = _neighbour(grid, coef[q], d, k, coef_in[q])
                Yn, _ = _neighbour(grid, Y6[q], d, k, Yin[q])
                # flux from the cell toward the neighbour: -coef_f (X_n - X)
                Jstar.append(-0.5 * (coef[q] + cn) * (Xn - X[q]))
                Yf.append(0.5 * (Y6[q] + Yn))
            Jsum = sum(Jstar)
            for q in range(6):
                J = Jstar[q] - Yf[q] * Jsum
                RY[q] = RY[q] + torch.where(open_, -J, 0.0)
    RT = F * RT / (rho * cp)
    RY = F * RY / rho
    return RT, RY, cp
