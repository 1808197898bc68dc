"""Pins of the oracle's flow solver: closed-form viscous decays (Taylor-Green vortex,
shear waves between halfway bounce-back walls and in periodic 3-D boxes), exact
conservation on periodic and walled boxes, exact inlet mass injection, and the outlet's
rest state."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import step as S
from oracle.lattice import CS2, get


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


def test_taylor_green_decay_128():
    """128^2 TGV, nu = 0.01, Ma 0.05, 1000 steps: amplitude falls as exp(-2 nu k^2 t)
    (0.952951 after 1000 steps) and kinetic energy as exp(-4 nu k^2 t), within the
    scheme's O(k^2, Ma^2) error."""
    p, P, u = L.tgv(128)
    st = S.init_state(p, t(P), t(u), None)
    u0 = t(u[0])
    ks, amps, kes = [], [], []
    for k in range(1001):
        if k % 100 == 0:
            _, rho, uu, _, sums = S.fields(p, st)
            ks.append(k)
            amps.append(float((uu[0] * u0).sum() / (u0 ** 2).sum()))
            kes.append(float(sums[5]))
        if k < 1000:
            st, _ = S.step(p, st)
    kk = 2 * math.pi / 128
    fit = -np.polyfit(ks[1:], np.log(amps[1:]), 1)[0]
    assert abs(fit / (2 * 0.01 * kk * kk) - 1) < 2e-3
    assert abs(amps[-1] / amps[0] - math.exp(-2 * 0.01 * kk * kk * 1000)) < 2e-4
    assert abs(kes[-1] / kes[0] - math.exp(-4 * 0.01 * kk * kk * 1000)) < 4e-4


def test_shear_wave_between_walls():
    """u_x = U sin(pi (y + 1/2)/H) between halfway bounce-back walls at y = -1/2 and
    H - 1/2 decays as exp(-nu (pi/H)^2 t)."""
    H, nu = 32, 0.05
    p = L.base_params("D2Q9", 4, H, 1, nu_ref=nu,
                      face_bc=["periodic", "periodic", "wall", "wall", "periodic", "periodic"])
    y = np.arange(H)[None, :, None] + 0.5
    u = np.zeros((2, 1, H, 4))
    u[0] = 0.01 * np.sin(math.pi * y / H) * np.ones((1, H, 4))
    st = S.init_state(p, t(np.full((1, H, 4), CS2)), t(u), None)
    prof = t(u[0])
    amps = []
    for k in range(801):
        if k in (200, 800):
            _, _, uu, _, _ = S.fields(p, st)
            amps.append(float((uu[0] * prof).sum() / (prof ** 2).sum()))
        st, _ = S.step(p, st)
    rate = math.log(amps[0] / amps[1]) / 600
    assert abs(rate / (nu * (math.pi / H) ** 2) - 1) < 1e-2


def test_shear_wave_3d_periodic():
    n, nu = 32, 0.02
    p = L.base_params("D3Q27", 4, 4, n, nu_ref=nu)
    z = np.arange(n)[:, None, None]
    u = np.zeros((3, n, 4, 4))
    u[0] = 0.01 * np.sin(2 * math.pi * z / n) * np.ones((n, 4, 4))
    st = S.init_state(p, t(np.full((n, 4, 4), CS2)), t(u), None)
    prof = t(u[0])
    amps = []
    for k in range(401):
        if k in (100, 400):
            _, _, uu, _, _ = S.fields(p, st)
            amps.append(float((uu[0] * prof).sum() / (prof ** 2).sum()))
        st, _ = S.step(p, st)
    rate = math.log(amps[0] / amps[1]) / 300
    assert abs(rate / (nu * (2 * math.pi / n) ** 2) - 1) < 1e-2


@pytest.mark.parametrize("name,shape", [("D2Q9", (1, 12, 10)), ("D3Q27", (6, 5, 7))])
def test_periodic_conservation(name, shape):
    """Isothermal periodic box from a random non-equilibrium state: sum g and sum c g are
    constant to round-off every step (collision keeps m0, m1; streaming permutes)."""
    lat = get(name)
    p = L.base_params(name, shape[2], shape[1], shape[0], cs_smag=0.17, nu_ref=0.005)
    ghat = L.random_deviation(lat.Q, shape, 3)
    st = {"pops": S.from_storage(p, t(ghat)), "scal": torch.zeros((0,) + shape,
                                                                  dtype=torch.float64),
          "step": 0, "solid": torch.zeros(shape, dtype=torch.bool)}
    m0 = float(st["pops"].sum())
    m1 = torch.einsum("qd,q...->d", lat.c, st["pops"])
    for _ in range(10):
        st, _ = S.step(p, st)
        assert abs(float(st["pops"].sum()) - m0) < 1e-12
        assert torch.allclose(torch.einsum("qd,q...->d", lat.c, st["pops"]), m1, atol=1e-13)


def test_closed_box_mass_and_rest():
    n = 16
    p = L.base_params("D2Q9", n, n, 1, nu_ref=0.02, cs_smag=0.17,
                      face_bc=["wall"] * 4 + ["periodic"] * 2)
    solid = torch.zeros(1, n, n, dtype=torch.bool)
    solid[0, 5:9, 6:8] = True
    rng = np.random.default_rng(1)
    u = 0.02 * rng.standard_normal((2, 1, n, n))
    st = S.init_state(p, t(np.full((1, n, n), CS2)), t(u), None, solid)
    fl = ~solid
    m0 = float(st["pops"][:, fl].sum())
    for _ in range(20):
        st, _ = S.step(p, st)
        assert abs(float(st["pops"][:, fl].sum()) - m0) < 1e-12
    rest = S.init_state(p, t(np.full((1, n, n), CS2)), t(np.zeros((2, 1, n, n))), None, solid)
    g0 = rest["pops"].clone()
    for _ in range(5):
        rest, _ = S.step(p, rest)
    assert torch.allclose(rest["pops"], g0, atol=1e-16, rtol=0)


def test_inlet_injects_exact_mass():
    """Inlet at -x (moving-wall bounce-back), wall at +x, periodic y, isothermal: per step
    sum g grows by exactly n_y cs2 rho_in u_in (sum of w_i over the incoming links = 1/6)."""
    nx, ny, uin = 12, 6, 0.03
    for name, nz in (("D2Q9", 1), ("D3Q27", 3)):
        faces = ["inlet", "wall", "periodic", "periodic", "periodic", "periodic"]
        p = L.base_params(name, nx, ny, nz, nu_ref=0.02, face_bc=faces,
                          inlet_u=[uin, 0.0, 0.0])
        D = 2 if nz == 1 else 3
        st = S.init_state(p, t(np.full((nz, ny, nx), CS2)), t(np.zeros((D, nz, ny, nx))), None)
        for _ in range(5):
            m = float(st["pops"].sum())
            st, _ = S.step(p, st)
            assert abs(float(st["pops"].sum()) - m - ny * nz * CS2 * 1.0 * uin) < 1e-13


def test_outlet_rest_state_fixed_point():
    """At rest with P_h = P_out everywhere the anti-bounce-back outlet returns the
    populations unchanged."""
    p = L.base_params("D3Q27", 6, 4, 5, face_bc=["wall", "outlet", "periodic", "periodic",
                                                  "wall", "wall"], outlet_P=CS2 * 1.02)
    shape = (5, 4, 6)
    st = S.init_state(p, t(np.full(shape, CS2 * 1.02)), t(np.zeros((3,) + shape)), None)
    g0 = st["pops"].clone()
    for _ in range(4):
        st, _ = S.step(p, st)
    assert torch.allclose(st["pops"], g0, atol=1e-16, rtol=0)
