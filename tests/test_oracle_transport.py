"""Pins of the oracle's mixture-averaged transport (variable c_p, mu(T), Hirschfelder-
Curtiss species diffusion with a correction flux):

* CO2 in N2 only: the mixture-averaged model must reduce to binary Fick diffusion in
  mole fractions, J = -rho (W_CO2 W_N2 / W^2) D_CO2,N2 grad X (textbook binary law), with
  no flux of the absent species;
* a trace species in N2 diffuses with its binary coefficient;
* the six face fluxes sum to zero (N2's own flux closes the set) and every species' mass
  sum rho Y_k is conserved exactly on a periodic box;
* equal molar masses, equal binary coefficients D ~ T, constant c_p and mu reduce the model
  to the unity-Lewis one (independently pinned elsewhere), boundaries included;
* a uniform two-step reactor keeps its total enthalpy sum_k Y_k h_k(T)/W_k up to a
  first-order time-step error and burns to the adiabatic temperature of that balance
  (closed-form root of the quadratic enthalpy of the burnt mixture)."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import scalars as SC
from oracle import step as S
from oracle import transport as TR
from oracle.grid import Grid
from oracle.lattice import CS2


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


def _params(nx, ny, nz=1, lattice="D2Q9", **kw):
    chem = L.two_step_chem(B1=0.0, B2=0.0)
    p = L.base_params(lattice, nx, ny, nz, physics="two_step", visc_law="const_mu", nu_ref=0.02,
                      T_ref=320.0, thickening=2.0, chem=chem, transport_model="mixture",
                      transport=L.mixture_transport(0.02), weno_scale=[1630.0, 0.05, 0.22, 0.05, 0.13, 0.11])
    p.update(kw)
    return p


def test_binary_mixture_is_binary_fick():
    nx = 32
    p = _params(nx, 1)
    x = np.arange(nx)
    Y = 0.1 + 0.08 * np.sin(2 * np.pi * x / nx) + 0.03 * np.cos(6 * np.pi * x / nx)
    T = np.full(nx, 600.0)
    scal = np.zeros((6, 1, 1, nx))
    scal[0, 0, 0] = T
    scal[4, 0, 0] = Y                                         # CO2; N2 by closure
    grid = Grid(p)
    rho = SC.density(p, t(scal), grid.shape)
    R, _ = SC.nonadvective_rhs(p, grid, t(scal), rho)
    W = L.W_SPECIES
    Wmix = 1.0 / (Y / W[3] + (1 - Y) / W[5])
    X = Y * Wmix / W[3]
    D = L.mixture_transport(0.02)[9 + 4] * (600.0 / 320.0) ** 1.75        # pair (3, 5)
    r = rho.numpy()[0, 0]
    c = r * W[3] * W[5] / Wmix ** 2 * D
    cf_p = 0.5 * (c + np.roll(c, -1))
    cf_m = 0.5 * (c + np.roll(c, 1))
    exp = 2.0 / r * (cf_p * (np.roll(X, -1) - X) + cf_m * (np.roll(X, 1) - X))
    assert np.abs(R[4, 0, 0].numpy() - exp).max() < 1e-12 * np.abs(exp).max()
    for k in (1, 2, 3, 5):
        assert float(R[k].abs().max()) == 0.0


def test_trace_species_has_its_binary_coefficient():
    p = _params(2, 1)
    Y6 = torch.zeros((6, 1), dtype=torch.float64)
    Y6[0] = 1e-9
    Y6[5] = 1.0 - 1e-9
    D, _, _ = TR.mixture_diffusion(p, torch.tensor([320.0], dtype=torch.float64), Y6)
    assert abs(float(D[0, 0]) / L.mixture_transport(0.02)[4] - 1) < 1e-8     # pair (0, 5)


def test_fluxes_close_and_species_mass_is_conserved():
    shape = (6, 7, 8)
    p = _params(8, 7, 6, lattice="D3Q27")
    scal = L.random_scalars("two_step", shape, 5)
    grid = Grid(p)
    rho = SC.density(p, t(scal), grid.shape)
    phin = SC.inlet_scalars(p)
    RT, RY, cp = TR.rhs(p, grid, t(scal), rho, phin, rho)
    assert float(RY.sum(0).abs().max()) < 1e-13 * float(RY.abs().max())
    for k in range(6):
        tot = float((rho * RY[k]).sum())
        assert abs(tot) < 1e-13 * float((rho * RY[k]).abs().sum())


def test_equal_molar_masses_reduce_to_unity_lewis():
    shape = (1, 11, 30)
    nu, Pr, cp = 0.02, 0.7, 1400.0
    chem = L.two_step_chem(B1=0.0, B2=0.0, cp=cp)
    chem = chem[:5] + [chem[17]] * 6 + chem[11:17] + [chem[17]]        # every W_k = W_ref
    tr = [nu / Pr] * 15 + [cp] * 6 + [0.0] * 6 + [0.0, 1.0, 0.0, 0.0, 0.0]
    faces = ["inlet", "outlet", "wall", "wall", "periodic", "periodic"]
    common = dict(chem=chem, face_bc=faces, inlet_T=320.0, inlet_Y=[0.05, 0.22, 0.0, 0.0, 0.0, 0, 0, 0])
    pm = _params(30, 11, transport=tr, **common)
    ps = _params(30, 11, transport_model="simple", **common)
    scal = L.random_scalars("two_step", shape, 7)
    solid = torch.zeros(shape, dtype=torch.bool)
    solid[0, 4:6, 12:15] = True
    grid = Grid(pm, solid)
    rho = SC.density(pm, t(scal), grid.shape)
    Rm, Lm = SC.nonadvective_rhs(pm, grid, t(scal), rho)
    Rs, Ls = SC.nonadvective_rhs(ps, grid, t(scal), rho)
    f = grid.fluid
    for k in range(6):
        assert torch.allclose(Rm[k][f], Rs[k][f], rtol=1e-11, atol=1e-11 * float(Rs[k].abs().max()))
    assert torch.allclose(Lm[f], Ls[f], rtol=1e-11, atol=1e-14)


def _reactor(B1, B2, steps, T0=1100.0):
    p = _params(2, 2, chem=L.two_step_chem(B1=B1, B2=B2), nu_ref=0.01, transport=L.mixture_transport(0.01))
    yf, yo, _ = L.fresh_ch4_air(0.83)
    scal = np.stack([np.full((1, 2, 2), T0)] + [np.full((1, 2, 2), y) for y in [yf, yo, 0, 0, 0]])
    st = S.init_state(p, t(np.full((1, 2, 2), CS2)), t(np.zeros((2, 1, 2, 2))), t(scal))

    def H(sc):
        Y6 = TR.full_Y(sc[1:])
        return float(sum(Y6[k] * TR.enthalpy(p, sc[0], k) / p["chem"][5 + k] for k in range(6)).mean())

    H0 = H(st["scal"])
    for _ in range(steps):
        st, _ = S.step(p, st)
    return p, H0, H(st["scal"]) - H0, float(st["scal"][0].mean()), st["scal"]


def test_variable_cp_reactor_enthalpy_and_adiabatic_temperature():
    p, H0, dH1, T1, sc1 = _reactor(300.0, 10.0, 400)
    _, _, dH2, T2, _ = _reactor(150.0, 5.0, 800)
    assert float(sc1[1].max()) < 1e-6 and float(sc1[3].max()) < 1e-6      # CH4 and CO burnt
    assert 1.8 < dH1 / dH2 < 2.2                                            # first order in dt
    # burnt composition and the quadratic enthalpy balance sum_k Y_k h_k(T)/W_k = H0
    Yb = [float(sc1[k].mean()) for k in range(1, 6)]
    Yb.append(1.0 - sum(Yb))
    tr, ch, T0f = p["transport"], p["chem"], TR.T0_FORMATION
    A = sum(Yb[k] * 0.5 * tr[21 + k] for k in range(6))
    B = sum(Yb[k] * tr[15 + k] for k in range(6))
    C = sum(Yb[k] * (ch[11 + k] / ch[5 + k] - tr[15 + k] * T0f - 0.5 * tr[21 + k] * T0f ** 2)
            for k in range(6)) - H0
    T_ad = (-B + math.sqrt(B * B - 4 * A * C)) / (2 * A)
    assert abs(T2 - T_ad) < 2e-3 * T_ad
    assert abs(T1 - T_ad) > abs(T2 - T_ad)
