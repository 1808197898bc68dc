"""Cumulant collision of Sec. 2.2 (Eqs. 8-14) in the pre-conditioned frame, with the
Smagorinsky closure for the shear rate.

The paper applies the cumulant operator of Geier et al. (2015) to the pre-conditioned
populations f' of Eq. 13 and defers the transforms to a supplement that is not available.
Readings taken here (they are the specification of this operator):

* Eq. 9 as printed, M^-1 (I - W) K' + M^-1 W K', collapses to K'; it is read as
  f'* = M^-1 [(I - W) K' + W K'_eq]: every cumulant relaxes towards its equilibrium with
  its own rate.
* Eq. 12 gives nu/(cs2 dt) + 1/2, which is the relaxation *time* tau_s; the shear rate is
  omega_s = 1/tau_s.
* Pre-conditioning normalises the populations by density, so that f^eq/rho has zeroth
  moment 1 and first moment u.  The remaining isotropic pressure content of f' (its zeroth
  moment m0 = sum f' differs from 1 by the hydrodynamic-pressure excess) is carried by
  the rest-weight shape: the cumulant operator acts on the density-one distribution
  f~_i = f'_i - w_i (m0 - 1), centred on the velocity u of Eq. 7b, and the shift is added
  back after collision.  m0 and the first moment are not relaxed.
* Equilibria: off-diagonal and deviatoric second-order cumulants 0, their trace D cs2;
  every cumulant of order >= 3 is 0.  Rates: omega_s for shear/deviatoric, omega_bulk for
  the trace, omega_high for every order >= 3 (Geier's fourth-order parameterisation is
  not used).
* Optional Galilean correction (Geier et al. 2015, switched on by
  params["galilean"]): on the velocity sets used here c^3 = c, so the equilibrium third
  diagonal moment of f~ is u_a instead of u_a + u_a^3 and the Chapman-Enskog stress
  carries an error (1/omega - 1/2) d_a(u_a^3) ~ (1/omega - 1/2) 3 u_a^2 d_a u_a on each
  diagonal (f~ has density one).  A post-collision source S_aa = -3 (1 - omega/2) u_a^2
  d_a u_a cancels it to that order: the deviatoric differences take it with omega_s, the
  trace with omega_bulk.  The diagonal velocity derivatives come from the pre-collision
  non-equilibrium second cumulants through the same balance:
  d_a u_a = -(omega_s / (2 cs2)) (C_aa - tr/D) - (omega_bulk / (2 cs2 D)) (tr - D cs2).
* Sub-grid model (Smagorinsky, Hou et al. closed form): with the non-equilibrium second
  moment Pi = kappa_2(f~) - cs2 I of the pre-collision state and Qbar = sqrt(2 Pi:Pi),
  tau = (tau0 + sqrt(tau0^2 + 2 Cs^2 Qbar / cs2^2)) / 2, filter width dr = 1.

The central moments are taken from their definition, the cumulants from the
multivariate moment-cumulant relation over set partitions (blocks of size one vanish
because the distribution is centred), and the back transform goes through raw moments
and the inverse of the dense moment matrix M.
"""
import itertools
import math
from functools import lru_cache

import torch

from .lattice import CS2


def set_partitions(items):
    """All partitions of the list `items` into non-empty blocks."""
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in set_partitions(rest):
        # put `first` in a block of its own, or into each existing block
        yield [[first]] + part
        for k in range(len(part)):
            yield part[:k] + [[first] + part[k]] + part[k + 1:]


def _exps_of_block(block, labels, D):
    e = [0] * D
    for p in block:
        e[labels[p]] += 1
    return tuple(e)


@lru_cache(maxsize=None)
def partition_terms(e):
    """For the multi-index e, the partitions of its multiset of axis labels that have no
    block of size one, as a list of (moment->cumulant coefficient, block multi-indices)."""
    D = len(e)
    labels = [d for d in range(D) for _ in range(e[d])]
    terms = {}
    for part in set_partitions(list(range(len(labels)))):
        if any(len(b) == 1 for b in part):
            continue
        blocks = tuple(sorted(_exps_of_block(b, labels, D) for b in part))
        k = len(part)
        coef = (-1) ** (k - 1) * math.factorial(k - 1)
        c, n = terms.get(blocks, (coef, 0))
        terms[blocks] = (c, n + 1)
    return [(coef, n, blocks) for blocks, (coef, n) in terms.items()]


def central_moments(lat, f, u):
    """kappa_e = sum_i prod_d (c_{i,d} - u_d)^{e_d} f_i for every e in the basis."""
    nd = f.ndim - 1
    out = {}
    for e in lat.exps:
        wgt = torch.ones_like(f)
        for d in range(lat.D):
            if e[d]:
                diff = lat.c[:, d].reshape((-1,) + (1,) * nd) - u[d]
                wgt = wgt * diff ** e[d]
        out[e] = (wgt * f).sum(0)
    return out


def moments_to_cumulants(kappa):
    """c_e = sum over partitions pi of (-1)^{|pi|-1} (|pi|-1)! prod_{B in pi} kappa_B."""
    C = {}
    for e, k in kappa.items():
        if sum(e) < 2:
            continue
        acc = torch.zeros_like(k)
        for coef, n, blocks in partition_terms(e):
            prod = torch.ones_like(k)
            for b in blocks:
                prod = prod * kappa[b]
            acc = acc + coef * n * prod
        C[e] = acc
    return C


def cumulants_to_moments(C, like):
    """kappa_e = sum over partitions pi of prod_{B in pi} c_B (centred: no singletons)."""
    kappa = {}
    for e in C:
        acc = torch.zeros_like(like)
        for _coef, n, blocks in partition_terms(e):
            prod = torch.ones_like(like)
            for b in blocks:
                prod = prod * C[b]
            acc = acc + n * prod
        kappa[e] = acc
    return kappa


def _unit(D, *axes):
    e = [0] * D
    for a in axes:
        e[a] += 1
    return tuple(e)


def smagorinsky_omega(lat, kappa, nu, cs_smag):
    """Shear rate from Eq. 12 (tau0 = nu/cs2 + 1/2) with the Smagorinsky eddy viscosity
    in closed form; Pi from the pre-collision second central moments."""
    D = lat.D
    tau0 = nu / CS2 + 0.5
    if cs_smag == 0.0:
        return 1.0 / tau0 + torch.zeros_like(kappa[_unit(D)])
    PiPi = torch.zeros_like(kappa[_unit(D)])
    for a in range(D):
        for b in range(D):
            Pi_ab = kappa[_unit(D, a, b)] - (CS2 if a == b else 0.0)
            PiPi = PiPi + Pi_ab * Pi_ab
    Qbar = torch.sqrt(2.0 * PiPi)
    tau = 0.5 * (tau0 + torch.sqrt(tau0 * tau0 + 2.0 * cs_smag ** 2 * Qbar / (CS2 * CS2)))
    return 1.0 / tau


def diagonal_strain(lat, C, omega_s, omega_bulk):
    """d_a u_a (a = 0..D-1) from the pre-collision second cumulants of the density-one
    distribution: C_aa - tr/D = -(2 cs2/omega_s) (d_a u_a - div u / D) and
    tr - D cs2 = -(2 cs2/omega_bulk) div u (first-order Chapman-Enskog balance)."""
    D = lat.D
    diag = [C[_unit(D, a, a)] for a in range(D)]
    trace = sum(diag)
    div = -omega_bulk / (2.0 * CS2) * (trace - D * CS2)
    return [-omega_s / (2.0 * CS2) * (diag[a] - trace / D) + div / D for a in range(D)]


def relax(lat, C, omega_s, omega_bulk, omega_high, u=None):
    """Relaxation (Eq. 9 as read): K* = (I - W) K + W K_eq, cumulant by cumulant; with
    the velocity u given, the diagonal second cumulants also take Geier's Galilean
    correction source S_aa = -3 (1 - omega/2) u_a^2 d_a u_a (omega_s on the deviatoric
    differences, omega_bulk on the trace)."""
    D = lat.D
    Cs = {}
    diag = [_unit(D, a, a) for a in range(D)]
    trace = sum(C[e] for e in diag)
    trace_s = trace + omega_bulk * (D * CS2 - trace)
    devs = [(1.0 - omega_s) * (C[diag[0]] - C[diag[a]]) for a in range(1, D)]
    if u is not None:
        dd = diagonal_strain(lat, C, omega_s, omega_bulk)
        S = [-3.0 * u[a] * u[a] * dd[a] for a in range(D)]
        trace_s = trace_s + (1.0 - 0.5 * omega_bulk) * sum(S)
        devs = [devs[a - 1] + (1.0 - 0.5 * omega_s) * (S[0] - S[a]) for a in range(1, D)]
    # c_aa* from trace* and the deviators (c_xx - c_aa)*
    cxx = (trace_s + sum(devs)) / D
    Cs[diag[0]] = cxx
    for a in range(1, D):
        Cs[diag[a]] = cxx - devs[a - 1]
    for e, v in C.items():
        if sum(e) == 2 and e not in diag:
            Cs[e] = (1.0 - omega_s) * v
        elif sum(e) >= 3:
            Cs[e] = (1.0 - omega_high) * v
    return Cs


def parameterised_rates(omega_1, omega_2):
    """Rates of the third-order cumulants and coefficients of the fourth-order equilibria
    of the parameterisation of Geier, Pasquali and Schoenherr (2017, J. Comput. Phys. 348,
    "Parametrization of the cumulant lattice Boltzmann method for fourth order accurate
    diffusion, part I"), functions of the shear rate omega_1 and the bulk rate omega_2:
    omega_3 for the sums C_120 + C_102 (and their permutations), omega_4 for the
    differences, omega_5 for C_111, A and B for the equilibria of the fourth-order
    diagonal and mixed cumulants.  Singular where omega_1 = omega_2."""
    w1, w2 = omega_1, omega_2
    w3 = (8 * (w1 - 2) * (w2 * (3 * w1 - 1) - 5 * w1)) / (8 * (5 - 2 * w1) * w1 + w2 * (8 + w1 * (9 * w1 - 26)))
    w4 = (8 * (w1 - 2) * (w1 + w2 * (3 * w1 - 7))) / (w2 * (56 - 42 * w1 + 9 * w1 * w1) - 8 * w1)
    w5 = (24 * (w1 - 2) * (4 * w1 * w1 + w1 * w2 * (18 - 13 * w1) + w2 * w2 * (2 + w1 * (6 * w1 - 11)))) / (
        16 * w1 * w1 * (w1 - 6) - 2 * w1 * w2 * (216 + 5 * w1 * (9 * w1 - 46))
        + w2 * w2 * (w1 * (3 * w1 - 10) * (15 * w1 - 28) - 48))
    den = (w1 - w2) * (w2 * (2 + 3 * w1) - 8 * w1)
    A = (4 * w1 * w1 + 2 * w1 * w2 * (w1 - 6) + w2 * w2 * (w1 * (10 - 3 * w1) - 4)) / den
    B = (4 * w1 * w2 * (9 * w1 - 16) - 4 * w1 * w1 - 2 * w2 * w2 * (2 + 9 * w1 * (w1 - 2))) / (3 * den)
    return w3, w4, w5, A, B


def relax_parameterised(lat, C, omega_s, omega_bulk, u=None):
    """The relaxation of Geier et al. (2017) for D3Q27 (fourth-order accurate diffusion):
    second order as in relax() (with the Galilean correction when u is given); the
    third-order sums C_120 + C_102, C_210 + C_012, C_201 + C_021 relax to zero at
    omega_3, their differences at omega_4, C_111 at omega_5; the fourth-order cumulants
    are set to equilibria proportional to the velocity gradients (rate one),
    C_220 = -(2/3) A (1/omega_s - 1/2)(d_x u_x + d_y u_y) (and permutations),
    C_112 = -(1/3) B (1/omega_s - 1/2)(d_x u_y + d_y u_x) (and permutations), the
    gradients estimated from the pre-collision second cumulants (diagonal as in
    diagonal_strain, mixed d_a u_b + d_b u_a = -(omega_s/cs2) C_ab); fifth and sixth
    order relax to zero."""
    assert lat.D == 3, "the fourth-order parameterisation is defined for D3Q27"
    Cs = relax(lat, {e: v for e, v in C.items() if sum(e) == 2}, omega_s, omega_bulk, 1.0, u)
    w3, w4, w5, A, B = parameterised_rates(omega_s, omega_bulk)
    # third order: (x y y, x z z) pairs and the like, by the axis that appears once
    for a in range(3):
        b, c = [d for d in range(3) if d != a]
        e_b = _unit(3, a, b, b)          # e.g. C_120 for a = x: x y y
        e_c = _unit(3, a, c, c)          #      C_102:          x z z
        S = C[e_b] + C[e_c]
        Dif = C[e_b] - C[e_c]
        Cs[e_b] = 0.5 * ((1.0 - w3) * S + (1.0 - w4) * Dif)
        Cs[e_c] = 0.5 * ((1.0 - w3) * S - (1.0 - w4) * Dif)
    Cs[(1, 1, 1)] = (1.0 - w5) * C[(1, 1, 1)]
    # fourth order
    dd = diagonal_strain(lat, C, omega_s, omega_bulk)
    visc = 1.0 / omega_s - 0.5
    for a in range(3):
        for b in range(a + 1, 3):
            Cs[_unit(3, a, a, b, b)] = -(2.0 / 3.0) * A * visc * (dd[a] + dd[b])
            c = 3 - a - b
            mixed = -omega_s / CS2 * C[_unit(3, a, b)]          # d_a u_b + d_b u_a
            Cs[_unit(3, a, b, c, c)] = -(1.0 / 3.0) * B * visc * mixed
    for e, v in C.items():
        if sum(e) >= 5:
            Cs[e] = torch.zeros_like(v)
    return Cs


def central_to_raw(lat, kappa, u):
    """m_e = sum_{k <= e} prod_d binom(e_d, k_d) u_d^{e_d - k_d} kappa_k
    (expansion of c = (c - u) + u in the moment definition)."""
    m = {}
    for e in lat.exps:
        acc = torch.zeros_like(kappa[e])
        ranges = [range(e[d] + 1) for d in range(lat.D)]
        for k in itertools.product(*ranges):
            coef = torch.ones_like(acc)
            for d in range(lat.D):
                coef = coef * math.comb(e[d], k[d]) * u[d] ** (e[d] - k[d])
            acc = acc + coef * kappa[k]
        m[e] = acc
    return m


def cumulant_collide(lat, f_prime, u, nu, cs_smag, omega_bulk, omega_high, omega_s=None, galilean=False,
                     fourth_order=False):
    """Post-collision pre-conditioned populations f'* (Eq. 9 as read).

    f_prime: (Q, *grid); u: (D, *grid) the velocity of Eq. 7b; nu: molecular kinematic
    viscosity (scalar or *grid); omega_s, if given, replaces the shear rate of Eq. 12 and
    the sub-grid model; galilean adds the Galilean correction; fourth_order selects the
    parameterised relaxation of Geier et al. (2017) (D3Q27; omega_high is then unused).
    Returns (f'*, omega_s)."""
    nd = f_prime.ndim - 1
    w = lat.w.reshape((-1,) + (1,) * nd)
    m0 = f_prime.sum(0)
    f_t = f_prime - w * (m0 - 1.0)
    kappa = central_moments(lat, f_t, u)
    if omega_s is None:
        omega_s = smagorinsky_omega(lat, kappa, nu, cs_smag)
    C = moments_to_cumulants(kappa)
    if fourth_order:
        Cs = relax_parameterised(lat, C, omega_s, omega_bulk, u if galilean else None)
    else:
        Cs = relax(lat, C, omega_s, omega_bulk, omega_high, u if galilean else None)
    kappa_s = cumulants_to_moments(Cs, m0)
    for e in lat.exps:           # orders 0 and 1 pass through unrelaxed
        if sum(e) < 2:
            kappa_s[e] = kappa[e]
    m_s = central_to_raw(lat, kappa_s, u)
    m_vec = torch.stack([m_s[e] for e in lat.exps])
    f_t_s = torch.einsum("ij,j...->i...", lat.Minv, m_vec)
    return f_t_s + w * (m0 - 1.0), omega_s
