"""Pins of the oracle's curved walls (interpolated bounce-back for the populations,
mirror-image ghosts for the scalar stencils; the wall is the zero level of a signed
distance at the nodes).

* A level set with |phi| the same at every node puts every wall halfway: the curved path
  must then be the staircase path bit for bit.
* Viscous decay of a shear wave between flat walls off the lattice, in both branches of
  the interpolation (q = 0.9 and q = 0.2): the rate nu (pi/H)^2 with H the true wall
  distance, where the staircase walls are off by several percent.
* The slowest swirling mode of a circular cavity of radius R (curved wall):
  u_theta ~ J1(j11 r/R) decays at nu (j11/R)^2 (Bessel functions from scipy).
* Ghost values of a field even about an off-lattice flat wall: exact where the image
  falls between the wall and the first node, within the linear-interpolation bound
  elsewhere."""
import math

import numpy as np
import pytest
import torch
from scipy.special import jn_zeros, jv

import lbm_inputs as L
from oracle import scalars
from oracle import step as S
from oracle.grid import Grid
from oracle.lattice import CS2


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 12, 20)), ("D3Q27", (6, 7, 8))])
def test_halfway_level_set_is_the_staircase(lat, shape):
    nz, ny, nx = shape
    p = L.base_params(lat, nx, ny, nz, physics="one_step", visc_law="const_mu", nu_ref=0.02,
                      chem=[3.0, 15000.0, 300.0, 2000.0, 1.0], weno_scale=[1700.0, 1.0],
                      thickening=2.0, cs_smag=0.17,
                      face_bc=["wall", "wall", "periodic", "periodic", "periodic", "periodic"])
    Q = 9 if lat == "D2Q9" else 27
    rng = np.random.default_rng(4)
    solid = rng.uniform(size=shape) < 0.15
    ghat = L.random_deviation(Q, shape, 9, 0.01)
    scal = L.random_scalars("one_step", shape, 10)
    phi = np.where(solid, -0.7, 0.7)
    runs = []
    for kw in ({"solid": t(solid).bool()}, {"phi": t(phi)}):
        st = S.init_state(p, t(np.full(shape, CS2)), t(np.zeros((3 if nz > 1 else 2,) + shape)), t(scal), **kw)
        st["pops"] = S.from_storage(p, t(ghat))
        for _ in range(2):
            st, sums = S.step(p, st)
        runs.append((st, sums))
    assert torch.equal(runs[0][0]["pops"], runs[1][0]["pops"])
    assert torch.equal(runs[0][0]["scal"], runs[1][0]["scal"])
    assert torch.equal(runs[0][1], runs[1][1])


def _shear_wave(y_lo, y_hi, curved, ny=34, nu=0.05, steps=(100, 400)):
    p = L.base_params("D2Q9", 4, ny, 1, nu_ref=nu)
    y = np.arange(ny, dtype=float)[None, :, None] * np.ones((1, ny, 4))
    phi = np.minimum(y - y_lo, y_hi - y)
    H = y_hi - y_lo
    prof = np.where(phi >= 0, np.sin(math.pi * (y - y_lo) / H), 0.0)
    u = np.zeros((2, 1, ny, 4))
    u[0] = 0.01 * prof
    geo = {"phi": t(phi)} if curved else {"solid": t(phi < 0).bool()}
    st = S.init_state(p, t(np.full((1, ny, 4), CS2)), t(u), None, **geo)
    amps = []
    for k in range(steps[1] + 1):
        if k in steps:
            _, _, uu, _, _ = S.fields(p, st)
            amps.append(float((uu[0] * t(prof)).sum() / (t(prof) ** 2).sum()))
        st, _ = S.step(p, st)
    rate = math.log(amps[0] / amps[1]) / (steps[1] - steps[0])
    return rate / (nu * (math.pi / H) ** 2) - 1


@pytest.mark.parametrize("y_lo,y_hi", [(1.1, 31.9), (1.8, 31.2)])     # q = 0.9 and q = 0.2
def test_shear_wave_between_off_lattice_walls(y_lo, y_hi):
    assert abs(_shear_wave(y_lo, y_hi, True)) < 3e-3
    assert abs(_shear_wave(y_lo, y_hi, False)) > 3e-2


def _cavity(curved, R=15.3, n=36, cx=17.3, cy=17.6, nu=0.05, steps=(100, 400)):
    p = L.base_params("D2Q9", n, n, 1, nu_ref=nu)
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    dx, dy = x - cx, y - cy
    r = np.hypot(dx, dy)
    j11 = jn_zeros(1, 1)[0]
    ut = 0.01 * jv(1, j11 * r / R) * (r < R)
    u = np.zeros((2, 1, n, n))
    u[0, 0] = -ut * dy / np.maximum(r, 1e-12)
    u[1, 0] = ut * dx / np.maximum(r, 1e-12)
    phi = (R - r)[None]
    geo = {"phi": t(phi)} if curved else {"solid": t(phi < 0).bool()}
    st = S.init_state(p, t(np.full((1, n, n), CS2)), t(u), None, **geo)
    amps = []
    for k in range(steps[1] + 1):
        if k in steps:
            _, _, uu, _, _ = S.fields(p, st)
            amps.append(float((uu * t(u)).sum() / (t(u) ** 2).sum()))
        st, _ = S.step(p, st)
    rate = math.log(amps[0] / amps[1]) / (steps[1] - steps[0])
    return rate / (nu * (j11 / R) ** 2) - 1


def test_circular_cavity_bessel_mode_decay():
    assert abs(_cavity(True)) < 3e-3
    assert abs(_cavity(False)) > 1.5e-2


@pytest.mark.parametrize("y_w", [2.3, 2.6, 2.95])
def test_ghosts_of_a_field_even_about_the_wall(y_w):
    """f = 1 + (y - y_w)^2 has zero normal gradient at the wall; the ghosts below the
    wall should reproduce its even extension f(image) = f(2 y_w - y)."""
    ny = 12
    p = L.base_params("D2Q9", 3, ny, 1, face_bc=["periodic"] * 6)
    y = np.arange(ny, dtype=float)[None, :, None] * np.ones((1, ny, 3))
    phi = np.minimum(y - y_w, 10.5 - y)
    grid = Grid(p, t(phi < 0).bool(), t(phi))
    f = 1.0 + (y - y_w) ** 2
    v = scalars.stencil(grid, t(f), 1, 0.0)
    j = 3                                           # first fluid row above the wall
    q = (j - y_w)
    for k in (-1, -2):
        got = float(v[k][0, j, 0])
        exact = 1.0 + (2 * y_w - (j + k) - y_w) ** 2
        p_img = j - (2 * y_w - (j + k))            # image position below node j (< 0: above)
        pos = -p_img                                # distance of the image from node j, into the fluid
        if pos < 0:
            assert abs(got - exact) < 1e-13
        else:
            frac = pos - math.floor(pos)
            assert abs(got - exact) <= frac * (1 - frac) + 1e-13
    # the plain mirror rule ignores the wall position
    if abs(q - 0.5) > 0.2:
        plain = Grid(p, t(phi < 0).bool())
        vp = scalars.stencil(plain, t(f), 1, 0.0)
        exact = 1.0 + (2 * y_w - (j - 1) - y_w) ** 2
        assert abs(float(vp[-1][0, j, 0]) - exact) > 0.2
