"""Pins of the oracle's closed-domain thermodynamic pressure (the low-Mach form of Eq. 3
with a time-dependent P_th, for the confined deflagration of Sec. 3.1).

A uniform reacting mixture in a periodic box is a closed adiabatic constant-volume
reactor: nothing moves, the density cannot change, the ideal gas then ties P_th to T, the
first law at constant volume makes the temperature rise gamma times the constant-pressure
rise, the continuity constraint (div u = 0) keeps the hydrodynamic pressure still, and the
trajectory converges at first order in the time step to the constant-volume ODE
integrated by scipy.  A closed box with walls and a flame conserves its mass exactly.
"""
import math

import numpy as np
import pytest
import torch
from scipy.integrate import solve_ivp

import lbm_inputs as L
from oracle import scalars
from oracle import step as S
from oracle.lattice import CS2

GAMMA = 1.4
T0, DT_P = 1000.0, 1700.0          # initial T; constant-pressure rise of the fuel (T_ad - T_u)


def t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def _reactor(B, steps, mode="closed", n=2):
    p = L.base_params("D2Q9", n, n, physics="one_step", chem=[B, 3000.0, 300.0, 2000.0, 1.0] + [0.0] * 27,
                      pth_mode=mode, gamma=GAMMA, weno_scale=[DT_P, 1.0] + [1.0] * 6, nu_ref=0.05)
    shape = (1, n, n)
    scal = np.stack([np.full(shape, T0), np.ones(shape)])
    st = S.init_state(p, t(np.full(shape, CS2)), t(np.zeros((2,) + shape)), t(scal))
    P0, rho0, _, _, _ = S.fields(p, st)
    hist = {"T": [T0], "pi": [1.0], "rho_err": 0.0, "u": 0.0, "Ph_drift": 0.0}
    for k in range(steps):
        st, _ = S.step(p, st)
        hist["T"].append(float(st["scal"][0].mean()))
        hist["pi"].append(st["thermo"][0])
        if k % 25 == 24 or k == steps - 1:
            P, rho, u, _, _ = S.fields(p, st)
            hist["rho_err"] = max(hist["rho_err"], float((rho / rho0 - 1).abs().max()))
            hist["u"] = max(hist["u"], float(u.abs().max()))
            hist["Ph_drift"] = max(hist["Ph_drift"], float((P - P0).abs().max()))
    hist["Y_end"] = float(st["scal"][1].max())
    hist["T_spread"] = float(st["scal"][0].max() - st["scal"][0].min())
    return hist


@pytest.fixture(scope="module")
def coarse():
    return _reactor(0.3, 400)


def test_constant_volume_reactor_thermodynamics(coarse):
    h = coarse
    assert h["Y_end"] < 1e-8 and h["T_spread"] == 0.0
    assert h["rho_err"] < 1e-13                        # constant volume: density fixed
    assert h["u"] < 1e-13                              # nothing moves
    ratio = np.array(h["pi"]) / (np.array(h["T"]) / T0)
    assert np.abs(ratio - 1).max() < 1e-12             # ideal gas at fixed density: P ~ T
    # first law at constant volume: c_v dT = q, so the rise is gamma times c_p's rise
    T_v, T_p = T0 + GAMMA * DT_P, T0 + DT_P
    assert abs(h["T"][-1] - T_v) < 0.015 * (T_v - T0)
    assert abs(h["T"][-1] - T_p) > 0.2 * (T_v - T0)
    # continuity (div u = 0) keeps P_h still up to the one-step lag of dP_th/dt; leaving
    # out the -dln(pi)/dt shift of Lambda would move it by about rho cs2 ln(T_end/T0)
    rho = 1.0 * 300.0 / T0
    assert h["Ph_drift"] < 0.1 * rho * CS2 * math.log(h["T"][-1] / T0)


def test_reactor_converges_to_constant_volume_ode(coarse):
    """Halving the step (rate B halved, twice the steps) halves the distance to the
    constant-volume ODE dT/dt = gamma (T_ad - T_u)/Y_u r, dY/dt = -r (first order)."""
    def rhs(_, y):
        r = 0.3 * max(y[1], 0.0) * math.exp(-3000.0 / y[0])
        return [GAMMA * DT_P * r, -r]

    sol = solve_ivp(rhs, (0.0, 400.0), [T0, 1.0], method="Radau", rtol=1e-11, atol=1e-12,
                    dense_output=True)
    fine = _reactor(0.15, 800)
    e_c = np.abs(np.array(coarse["T"]) - sol.sol(np.arange(401.0))[0]).max()
    e_f = np.abs(np.array(fine["T"][::2]) - sol.sol(np.arange(401.0))[0]).max()
    assert e_f < 0.03 * GAMMA * DT_P
    assert 1.6 < e_c / e_f < 2.4


def test_two_step_reactor_keeps_density():
    """Mixture molar mass changes with the moles of the two-step scheme; the density of a
    uniform closed reactor must still not move (mass and volume fixed)."""
    chem = L.two_step_chem(B1=50.0, B2=5.0)
    p = L.base_params("D2Q9", 2, 2, 1, physics="two_step", visc_law="const_mu", nu_ref=0.01,
                      T_ref=320.0, chem=chem, pth_mode="closed", gamma=GAMMA)
    yf, yo, _ = L.fresh_ch4_air(0.83)
    scal = np.stack([np.full((1, 2, 2), 1500.0)] + [np.full((1, 2, 2), y) for y in [yf, yo, 0, 0, 0]])
    st = S.init_state(p, t(np.full((1, 2, 2), CS2)), t(np.zeros((2, 1, 2, 2))), t(scal))
    _, rho0, _, _, _ = S.fields(p, st)
    for _ in range(30):
        st, _ = S.step(p, st)
    _, rho, _, sc, _ = S.fields(p, st)
    assert float(sc[1].max()) < 0.9 * yf                  # fuel burnt
    assert st["thermo"][0] > 1.05                          # pressure rose
    assert float((rho / rho0 - 1).abs().max()) < 1e-13


def _flame_box(mode, nx=32, ny=20):
    p = L.base_params("D2Q9", nx, ny, physics="one_step", chem=list(L.ONE_STEP_CHEM) + [0.0] * 27,
                      pth_mode=mode, gamma=GAMMA, weno_scale=[DT_P, 1.0] + [1.0] * 6, nu_ref=0.02,
                      thickening=2.0, face_bc=["wall"] * 4 + ["periodic"] * 2, visc_law="const_mu")
    shape = (1, ny, nx)
    y, x = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    c = 0.5 * (1 - np.tanh((np.hypot(x, y - ny / 2) - 6.0) / 2.0))
    scal = np.stack([(300.0 + 1700.0 * c).reshape(shape), (1 - c).reshape(shape)])
    solid = torch.zeros(shape, dtype=torch.bool)
    solid[0, 8:12, 20:23] = True
    return p, S.init_state(p, t(np.full(shape, CS2)), t(np.zeros((2,) + shape)), t(scal), solid)


def test_closed_box_conserves_mass():
    """Walls all round: the total mass sum rho is fixed to rounding in the closed mode
    (the open mode, with P_th held, visibly loses mass through the non-conservative scalar
    update), and the pressure rises as the kernel burns."""
    drift = {}
    for mode in ("closed", "open"):
        p, st = _flame_box(mode)
        m0 = None
        worst = 0.0
        for _ in range(25):
            st, sums = S.step(p, st)
            m0 = float(sums[0]) if m0 is None else m0
            worst = max(worst, abs(float(sums[0]) / m0 - 1))
        drift[mode] = worst
        if mode == "closed":
            assert st["thermo"][0] > 1.0
    assert drift["closed"] < 1e-13
    assert drift["open"] > 1e-4


def test_closed_mode_without_heat_release_equals_open_mode():
    """No temperature change: P_th stays exactly at its initial value and the closed step
    is the open step, bit for bit (isothermal shear flow and a passive scalar)."""
    for phys, S_n in (("isothermal", 0), ("passive", 1)):
        res = {}
        for mode in ("closed", "open"):
            p = L.base_params("D2Q9", 12, 10, physics=phys, pth_mode=mode, nu_ref=0.03,
                              face_bc=["periodic", "periodic", "wall", "wall", "periodic", "periodic"],
                              weno_scale=[1.0] * 8)
            yy = np.arange(10, dtype=float)[None, :, None] * np.ones((1, 10, 12))
            u = np.stack([0.04 * np.sin(2 * np.pi * yy / 10), np.zeros((1, 10, 12))])
            scal = (0.5 + 0.1 * np.cos(2 * np.pi * yy / 10))[None] if S_n else None
            st = S.init_state(p, t(np.full((1, 10, 12), CS2)), t(u), None if scal is None else t(scal))
            for _ in range(5):
                st, _ = S.step(p, st)
            res[mode] = st
        assert res["closed"]["thermo"][:2] == (1.0, 0.0)
        assert torch.equal(res["closed"]["pops"], res["open"]["pops"])
        assert torch.equal(res["closed"]["scal"], res["open"]["scal"])


def test_density_scales_with_thermodynamic_pressure():
    chem = L.two_step_chem()
    p = L.base_params("D2Q9", 2, 1, 1, physics="two_step", T_ref=320.0, rho_ref=1.3, chem=chem)
    yf, yo, _ = L.fresh_ch4_air(0.83)
    sc = t(np.array([700.0, yf, yo, 0, 0, 0]).reshape(6, 1, 1, 1))
    r1 = float(scalars.density(p, sc, (1, 1, 1)))
    r2 = float(scalars.density(p, sc, (1, 1, 1), 2.5))
    assert abs(r2 / r1 - 2.5) < 1e-15
    w = float(scalars.w_over_T(p, sc, (1, 1, 1)))
    assert abs(r1 - 1.3 * 320.0 / chem[17] * w) < 1e-12 * r1
