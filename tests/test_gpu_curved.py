"""GPU tests of curved walls (signed wall distance bound with lbm_set_wall_distance)
against the FP64 oracle.

Parity: random non-equilibrium states around circular / spherical obstacles given by
their signed distance, D2Q9 and D3Q27, isothermal, one- and two-step physics, cumulant
and BGK, linear and banded tile orders; FP64 bounds as the other one-step parity tests
(1e-12 in ghat, 1e-12 of the scalar ranges), FP32 as the reduced-precision ones.
A level set of constant magnitude puts every wall halfway and must reproduce the solid
mask path.  At scale: the swirling Bessel mode of a circular cavity of radius 120.3 on a
256^2 grid decays at nu (j11/R)^2 within 0.1 %."""
import math

import numpy as np
import pytest
import torch
from scipy.special import jn_zeros, jv

import lbm_inputs as L
from oracle import step as OS
from tests.gpu_helpers import fetch, gpu_state, make_solver, oracle_ghat, random_state

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


def _levelset(shape, D):
    """Signed distance to two solid discs (2-D) or balls (3-D): positive in the fluid."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                          np.arange(nx, dtype=float), indexing="ij")
    out = np.full(shape, np.inf)
    for cx, cy, cz, r in ((0.31 * nx, 0.43 * ny, 0.47 * nz, 0.23 * min(ny, nx, nz if D == 3 else ny)),
                          (0.72 * nx, 0.58 * ny, 0.52 * nz, 0.17 * min(ny, nx, nz if D == 3 else ny))):
        dist = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + ((z - cz) ** 2 if D == 3 else 0.0)) - r
        out = np.minimum(out, dist)
    return out


def _params(lat, shape, phys, coll, prec="fp64"):
    nz, ny, nx = shape
    chem = {"one_step": [3.0, 15000.0, 300.0, 2000.0, 1.0],
            "two_step": L.two_step_chem(B1=50.0, B2=5.0)}.get(phys, [0.0] * 32)
    ws = {"one_step": [1700.0, 1.0], "two_step": [1630.0, 0.05, 0.22, 0.05, 0.13, 0.11]}.get(phys, [1.0])
    return L.base_params(lat, nx, ny, nz, physics=phys, collision=coll, nu_ref=0.02, cs_smag=0.17,
                         omega_bulk=1.2, omega_high=0.9, thickening=2.0, chem=chem,
                         visc_law="const_mu" if phys in ("one_step", "two_step") else "const_nu",
                         T_ref=300.0 if phys != "two_step" else 320.0, precision=prec,
                         weno_scale=ws + [1.0] * (8 - len(ws)),
                         face_bc=["wall", "wall", "periodic", "periodic", "periodic", "periodic"])


def _run(p, ghat, scal, phi, steps, solid_mask=None):
    s = make_solver(p)
    if solid_mask is None:
        s.set_wall_distance(torch.from_numpy(phi))
    else:
        s.set_geometry(torch.from_numpy(solid_mask.astype(np.uint8)))
    gpu_state(s, ghat, scal)
    s.step(steps)
    pops, sc, _ = fetch(s)
    sums = s.step_sums()
    s.close()
    return pops, sc, sums


def _oracle(p, ghat, scal, phi, steps):
    st = {"pops": OS.from_storage(p, torch.from_numpy(ghat)), "scal": torch.from_numpy(scal), "step": 0,
          "solid": torch.from_numpy(phi < 0), "phi": torch.from_numpy(phi)}
    sums = None
    for _ in range(steps):
        st, sums = OS.step(p, st)
    return oracle_ghat(p, st), st["scal"].numpy(), sums.numpy()


CASES = [("D2Q9", (1, 13, 70), "isothermal", "cumulant"), ("D2Q9", (1, 13, 70), "one_step", "cumulant"),
         ("D2Q9", (1, 16, 128), "one_step", "bgk"), ("D2Q9", (1, 12, 40), "two_step", "cumulant"),
         ("D3Q27", (7, 6, 9), "isothermal", "cumulant"), ("D3Q27", (9, 10, 11), "one_step", "cumulant"),
         ("D3Q27", (8, 8, 64), "two_step", "cumulant"), ("D3Q27", (7, 6, 9), "two_step", "bgk")]


@pytest.mark.parametrize("lat,shape,phys,coll", CASES)
def test_curved_parity_fp64(lat, shape, phys, coll):
    print(f"curved parity {lat} {shape} {phys} {coll}", flush=True)
    p = _params(lat, shape, phys, coll)
    phi = _levelset(shape, 2 if lat == "D2Q9" else 3)
    assert (phi < 0).any()
    ghat, scal = random_state(p, 31)
    g_pops, g_scal, g_sums = _run(p, ghat, scal, phi, 3)
    o_pops, o_scal, o_sums = _oracle(p, ghat, scal, phi, 3)
    fl = phi >= 0
    assert np.abs(g_pops - o_pops)[:, fl].max() < 1e-12
    if scal.shape[0]:
        scale = np.array(p["weno_scale"][:scal.shape[0]]).reshape(-1, 1)
        assert (np.abs(g_scal - o_scal)[:, fl] / scale).max() < 1e-12
    assert np.allclose(g_sums, o_sums, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("lat,shape,phys", [("D2Q9", (1, 13, 70), "one_step"), ("D3Q27", (7, 6, 9), "two_step")])
def test_curved_parity_fp32(lat, shape, phys):
    print(f"curved parity fp32 {lat} {shape} {phys}", flush=True)
    p = _params(lat, shape, phys, "cumulant", prec="fp32")
    phi = _levelset(shape, 2 if lat == "D2Q9" else 3)
    ghat, scal = random_state(p, 33)
    g_pops, g_scal, _ = _run(p, ghat, scal, phi, 1)
    o_pops, o_scal, _ = _oracle(p, ghat, scal, phi, 1)
    fl = phi >= 0
    assert np.abs(g_pops - o_pops)[:, fl].max() < 2e-7
    scale = np.maximum(np.array(p["weno_scale"][:scal.shape[0]]).reshape(-1, 1), np.abs(o_scal[:, fl]))
    assert (np.abs(g_scal - o_scal)[:, fl] / scale).max() < 2e-6


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 13, 70)), ("D3Q27", (7, 6, 9))])
def test_halfway_level_set_matches_mask(lat, shape):
    p = _params(lat, shape, "one_step", "cumulant")
    rng = np.random.default_rng(8)
    solid = rng.uniform(size=shape) < 0.12
    phi = np.where(solid, -0.6, 0.6)
    ghat, scal = random_state(p, 35)
    a = _run(p, ghat, scal, phi, 3)
    b = _run(p, ghat, scal, phi, 3, solid_mask=solid)
    fl = ~solid
    assert np.abs(a[0] - b[0])[:, fl].max() < 1e-14
    assert np.abs(a[1] - b[1])[:, fl].max() < 1e-12


def test_circular_cavity_at_scale():
    n, R, nu = 256, 120.3, 0.1
    cx, cy = 127.6, 128.3
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
    rates = {}
    for curved in (True, False):
        s = make_solver(p)
        if curved:
            s.set_wall_distance(torch.from_numpy(phi))
        else:
            s.set_geometry(torch.from_numpy((phi < 0).astype(np.uint8)))
        s.init_fields(torch.from_numpy(np.full((1, n, n), CS2)), torch.from_numpy(u))
        amps = []
        prof = torch.from_numpy(u).cuda()
        for k in (1000, 3000):
            s.step(k - (1000 if amps else 0))
            amps.append(float((s.fields()["u"] * prof).sum() / (prof ** 2).sum()))
        s.close()
        rates[curved] = math.log(amps[0] / amps[1]) / 2000 / (nu * (j11 / R) ** 2) - 1
    print("cavity rate errors", rates, flush=True)
    assert abs(rates[True]) < 1e-3
    assert abs(rates[False]) > 2 * abs(rates[True])


@pytest.mark.parametrize("lat,shape,phys", [("D2Q9", (1, 13, 70), "one_step"), ("D3Q27", (8, 8, 64), "two_step")])
def test_curved_closed_domain_parity(lat, shape, phys):
    """Curved walls in a closed domain: the step runs split (interior and boundary-list
    instances), and the thermodynamic pressure comes from the block records of both."""
    p = _params(lat, shape, phys, "cumulant")
    p["pth_mode"] = "closed"
    phi = _levelset(shape, 2 if lat == "D2Q9" else 3)
    ghat, scal = random_state(p, 35)
    s = make_solver(p)
    s.set_wall_distance(torch.from_numpy(phi))
    gpu_state(s, ghat, scal)
    s.step(4)
    g_pops, g_scal, _ = fetch(s)
    th = s.thermo_pressure()
    s.close()
    st = {"pops": OS.from_storage(p, torch.from_numpy(ghat)), "scal": torch.from_numpy(scal), "step": 0,
          "solid": torch.from_numpy(phi < 0), "phi": torch.from_numpy(phi)}
    for _ in range(4):
        st, _ = OS.step(p, st)
    fl = phi >= 0
    assert np.abs(g_pops - oracle_ghat(p, st))[:, fl].max() < 1e-11
    scale = np.array(p["weno_scale"][:scal.shape[0]]).reshape(-1, 1)
    assert (np.abs(g_scal - st["scal"].numpy())[:, fl] / scale).max() < 1e-11
    assert abs(th[0] / float(st["thermo"][0]) - 1) < 1e-13 and float(st["thermo"][0]) != 1.0
