"""Pins of the oracle's inlet and outlet under through-flow (Sec. 3.1-3.2: walls, a
mass-flow inlet and an exhaust; the methods are read as a moving-wall bounce-back inlet
and an anti-bounce-back pressure outlet):

* plug flow: uniform velocity u_in (oblique to the faces as well) at the outlet pressure
  is an exact fixed point of inlet + interior + outlet in the single-relaxation mode,
  whose equilibrium (Eq. 6) is exactly the state; every term of the outlet's even
  equilibrium, P_out + rho ((c.u)^2/(2 cs2) - u^2/2), must be right for that, so a dropped,
  flipped or mis-scaled velocity term, or a wrong density, moves the populations;
* Poiseuille channel fed by the inlet and drained by the outlet between halfway
  bounce-back walls: the steady mass flux equals the inlet's injection at every cross
  section, the developed profile is the parabola of the mean velocity and the pressure
  gradient is -12 rho nu u_mean / H^2, both converging at second order in the cell size."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import step as S
from oracle.lattice import CS2


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


@pytest.mark.parametrize("name,shape", [("D2Q9", (1, 3, 12)), ("D3Q27", (3, 2, 8))])
def test_plug_flow_is_a_fixed_point_of_inlet_and_outlet(name, shape):
    nz, ny, nx = shape
    D = 2 if name == "D2Q9" else 3
    u_in = [0.05, 0.02, -0.01][:D] + [0.0] * (3 - D)
    P_out = CS2 * 1.01
    p = L.base_params(name, nx, ny, nz, nu_ref=0.02, collision="bgk", rho_ref=1.3,
                      face_bc=["inlet", "outlet"] + ["periodic"] * 4, inlet_u=u_in,
                      outlet_P=P_out)
    u = np.zeros((D,) + shape)
    for d in range(D):
        u[d] = u_in[d]
    st = S.init_state(p, t(np.full(shape, P_out)), t(u), None)
    g0 = st["pops"].clone()
    for _ in range(5):
        st, _ = S.step(p, st)
    assert float((st["pops"] - g0).abs().max()) < 1e-15
    P, _, uu, _, _ = S.fields(p, st)
    assert float((P - P_out).abs().max()) < 1e-15
    for d in range(D):
        assert float((uu[d] - u_in[d]).abs().max()) < 1e-14


def _channel(H, nu=0.25, u_in=0.02):
    """Channel of height H and length 3H, inlet at -x, outlet at +x, walls at -y/+y,
    started from the parabola and linear pressure it should keep; run for H^2/nu steps
    (about ten decay times of its slowest shear mode)."""
    nx = 3 * H
    p = L.base_params("D2Q9", nx, H, 1, nu_ref=nu,
                      face_bc=["inlet", "outlet", "wall", "wall", "periodic", "periodic"],
                      inlet_u=[u_in, 0.0, 0.0], outlet_P=CS2)
    shape = (1, H, nx)
    # the two corner links of the inlet column cross a wall too and bounce back without
    # injection: the inlet feeds u_in (H - 1/3) per step (unit density)
    ub = u_in * (H - 1.0 / 3.0) / H
    y = np.arange(H)[:, None] + 0.5
    x = np.arange(nx)[None, :]
    u = np.zeros((2,) + shape)
    u[0, 0] = 6 * ub * y * (H - y) / H ** 2 + 0 * x
    P = CS2 + 12 * nu * ub * (nx - 0.5 - x) / H ** 2 + 0 * y
    st = S.init_state(p, t(P[None]), t(u), None)
    st, _ = S.run(p, st, int(H * H / nu))
    P, _, uu, _, _ = S.fields(p, st)
    ux = uu[0, 0].numpy()
    Pm = P[0].numpy().mean(0)
    flux = ux.sum(0) / (u_in * (H - 1.0 / 3.0))
    xm = nx // 2
    um = ux[:, xm].mean()
    yc = np.arange(H) + 0.5
    prof_err = np.abs(ux[:, xm] - 6 * um * yc * (H - yc) / H ** 2).max() / um
    xs = np.arange(nx // 4, nx - 4)
    dPdx = np.polyfit(xs, Pm[xs], 1)[0]
    grad_err = abs(dPdx / (-12 * nu * um / H ** 2) - 1)
    return np.abs(flux - 1).max(), prof_err, grad_err


def test_poiseuille_channel_through_inlet_and_outlet():
    f8, p8, g8 = _channel(8)
    f16, p16, g16 = _channel(16)
    # mass flux through every cross section equals the injection (steady within 1e-4)
    assert f16 < 1e-4 and f8 < 1e-3
    # profile: parabola of the measured mean, second-order convergence
    assert p16 < 8e-3
    assert 3.0 < p8 / p16 < 5.0
    # pressure gradient -12 rho nu u_mean / H^2, converging
    assert g16 < 1.5e-2
    assert g8 / g16 > 2.5
