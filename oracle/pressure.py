"""Thermodynamic pressure of a closed domain (the low-Mach limit behind Eq. 3).

Test infrastructure: see the package header.

Eq. 3 is the divergence constraint at a constant thermodynamic pressure P_th, which is
the open-domain case.  In a closed vessel (the deflagration chamber of Sec. 3.1, where the
pressure climbs as the flame accelerates through the obstacles) P_th varies in time and is
fixed by the mass the vessel holds.  The paper writes none of this down; the reading here
(parity unpinned against the paper itself, pinned against constant-volume thermodynamics
and the continuity constraint in the tests) is:

* ideal gas: rho = pi rho_hat(T, Y), pi = P_th/P_th(0), rho_hat the open-domain density;
* energy: the pressure work (dP_th/dt)/(rho c_p) = kappa T dln(pi)/dt, kappa = (gamma-1)/gamma
  for a constant ratio of specific heats gamma, joins the temperature right-hand side
  (and with it the temperature term of Lambda);
* continuity of the low-Mach system: div u = Lambda - dln(pi)/dt, which replaces Lambda in
  the source Xi (Eq. 2) and in P_h (Eq. 7a);
* mass: after the explicit update of the scalars, pi^{n+1} is the factor that keeps the
  total mass sum_fluid rho at its initial value, pi^{n+1} = K / sum_fluid (W/T)^{n+1}, with
  K = pi^0 sum_fluid (W/T)^0 (W/T per cell, up to a constant factor, is rho_hat);
* dln(pi)/dt at level n is the backward difference q^n = (pi^n - pi^{n-1})/pi^{n-1} (time
  step 1), q^0 = 0: explicit, lagging by one step like the rest of the first-order march.

The state carries (pi, q, K); K = 0 means "not yet fixed" and is set from the first step's
level-0 sum.
"""


def closed(params):
    return params.get("pth_mode", "open") == "closed"


def initial():
    """(pi, q, K) right after initialisation."""
    return (1.0, 0.0, 0.0)


def kappa(params):
    g = float(params.get("gamma", 1.4))
    return (g - 1.0) / g


def apply(params, R, Lam, T, thermo):
    """Pressure-work term on the temperature right-hand side and the continuity shift of
    Lambda.  R: stacked non-advective right-hand sides (R[0] is temperature), Lam: Lambda
    of Eq. 3 at constant P_th.  Returns (R, Lambda entering Xi and P_h)."""
    if not closed(params) or R.shape[0] == 0:
        return R, Lam
    q = float(thermo[1])
    R = R.clone()
    R[0] = R[0] + kappa(params) * T * q
    Lam = Lam + kappa(params) * q          # temperature term of Eq. 3 with the new R_T
    return R, Lam - q


def update(thermo, S_n, S_next):
    """(pi, q, K) of level n+1 from the fluid sums of W/T at levels n and n+1."""
    pi, _, K = thermo
    if not K > 0.0:
        K = pi * S_n
    pi_next = K / S_next
    return (pi_next, (pi_next - pi) / pi, K)
