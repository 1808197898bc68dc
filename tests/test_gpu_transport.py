"""GPU parity of mixture-averaged transport (two-step scalars, FULL kernel instances)
against the FP64 oracle: random non-equilibrium states with walls, inlet, outlet and
solids, one step (FP64: 1e-12 in ghat and of the scalar ranges; FP32: the reduced-
precision bounds; random temperature fields violate the explicit diffusion limit with the
hot binary coefficients, so they are not advanced further), a flame kernel over 10 steps, and the closed-domain
combination (pi to 1e-13)."""
import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import step as OS
from tests.gpu_helpers import fetch, gpu_state, make_solver, oracle_ghat, oracle_state, random_state

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


def _params(lat, shape, prec="fp64", faces=None, **kw):
    nz, ny, nx = shape
    yf, yo, _ = L.fresh_ch4_air(0.83)
    p = L.base_params(lat, nx, ny, nz, physics="two_step", visc_law="const_mu", nu_ref=0.01, cs_smag=0.17,
                      thickening=2.0, chem=L.two_step_chem(B1=50.0, B2=5.0), T_ref=320.0, precision=prec,
                      weno_scale=[1630.0, 0.05, 0.22, 0.05, 0.13, 0.11], transport_model="mixture",
                      transport=L.mixture_transport(0.01), inlet_T=320.0,
                      inlet_Y=[yf, yo, 0.0, 0.0, 0.0, 0, 0, 0], inlet_u=[0.03, 0.01, 0.0],
                      face_bc=faces or ["inlet", "outlet", "wall", "wall", "periodic", "periodic"])
    p.update(kw)
    return p


@pytest.mark.parametrize("lat,shape,faces", [
    ("D2Q9", (1, 13, 70), None),
    ("D3Q27", (7, 6, 9), ["inlet", "outlet", "periodic", "periodic", "wall", "wall"]),
    ("D3Q27", (6, 8, 64), ["periodic", "periodic", "wall", "wall", "inlet", "outlet"]),
])
def test_mixture_parity_fp64(lat, shape, faces):
    print(f"mixture parity {lat} {shape}", flush=True)
    p = _params(lat, shape, faces=faces)
    ghat, scal = random_state(p, 41)
    solid = np.random.default_rng(2).uniform(size=shape) < 0.06
    s = make_solver(p)
    s.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
    gpu_state(s, ghat, scal)
    s.step(1)
    g_pops, g_scal, _ = fetch(s)
    s.close()
    st, _ = OS.step(p, oracle_state(p, ghat, scal, solid))
    fl = ~solid
    assert np.abs(g_pops - oracle_ghat(p, st))[:, fl].max() < 1e-12
    scale = np.array(p["weno_scale"][:6]).reshape(-1, 1)
    assert (np.abs(g_scal - st["scal"].numpy())[:, fl] / scale).max() < 1e-12


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
@pytest.mark.parametrize("lat,shape,faces,solids", [
    ("D2Q9", (1, 13, 70), None, False),
    ("D3Q27", (7, 6, 9), None, False),
    # on the 64x4 tile grid: neighbour points across the x/y tile edges, wrapped (periodic
    # x, y) or stopped at walls and solids
    ("D3Q27", (6, 8, 64), ["periodic", "periodic", "wall", "wall", "inlet", "outlet"], True),
    ("D3Q27", (4, 8, 128), ["periodic", "periodic", "periodic", "periodic", "wall", "wall"], False),
])
def test_mixture_parity_fp32(lat, shape, faces, solids, prec):
    """FP32 arithmetic with FP32 or FP16 population storage against the FP64 oracle on
    inputs rounded to the storage precision; the FP16-storage bound adds half an FP16 ulp of
    the value (the output is rounded to half precision)."""
    print(f"mixture parity {prec} {lat} {shape}", flush=True)
    p = _params(lat, shape, prec=prec, faces=faces)
    ghat, scal = random_state(p, 43)
    solid = np.random.default_rng(3).uniform(size=shape) < 0.06 if solids else np.zeros(shape, bool)
    s = make_solver(p)
    if solids:
        s.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
    gpu_state(s, ghat, scal)
    s.step(1)
    g_pops, g_scal, _ = fetch(s)
    s.close()
    st, _ = OS.step(p, oracle_state(p, ghat, scal, solid if solids else None))
    fl = ~solid
    g_pops, g_scal = g_pops[:, fl], g_scal[:, fl]
    o_pops = oracle_ghat(p, st)[:, fl]
    tol = 2e-7 + (np.abs(o_pops) * 2.0 ** -11 if prec == "fp16s" else 0.0)
    assert (np.abs(g_pops - o_pops) <= tol).all(), np.abs(g_pops - o_pops).max()
    o = st["scal"].numpy()[:, fl]
    scale = np.maximum(np.array(p["weno_scale"][:6]).reshape(-1, 1), np.abs(o))
    assert (np.abs(g_scal - o) / scale).max() < 2e-6


def _flame(lat, shape, **kw):
    nz, ny, nx = shape
    p = _params(lat, shape, faces=["wall", "outlet", "periodic", "periodic", "periodic", "periodic"] if lat == "D2Q9"
                else ["wall", "outlet", "periodic", "periodic", "wall", "wall"], **kw)
    yf, yo, _ = L.fresh_ch4_air(0.83)
    b = L.burnt_ch4_air(0.83)
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    c = 0.5 * (1 - np.tanh((x - nx / 3) / 2.0))[None]
    scal = np.concatenate([320.0 + 1630.0 * c, yf * (1 - c), yo * (1 - c) + b["O2"] * c, 0.0 * c,
                           b["CO2"] * c, b["H2O"] * c])
    D = 2 if lat == "D2Q9" else 3
    return p, np.full(shape, CS2), np.zeros((D,) + shape), scal


@pytest.mark.parametrize("pth", ["open", "closed"])
def test_mixture_flame_ten_steps(pth):
    kw = {"pth_mode": pth}
    if pth == "closed":
        kw["face_bc"] = ["wall", "wall", "periodic", "periodic", "periodic", "periodic"]
    p, P, u, scal = _flame("D2Q9", (1, 16, 64), **kw)
    s = make_solver(p)
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    s.step(10)
    g_pops, g_scal, _ = fetch(s)
    th = s.thermo_pressure()
    s.close()
    st = OS.init_state(p, torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    for _ in range(10):
        st, _ = OS.step(p, st)
    assert np.abs(g_pops - oracle_ghat(p, st)).max() < 1e-11
    scale = np.array(p["weno_scale"][:6]).reshape(-1, 1, 1, 1)
    assert (np.abs(g_scal - st["scal"].numpy()) / scale).max() < 1e-11
    if pth == "closed":
        assert abs(th[0] / st["thermo"][0] - 1) < 1e-13 and st["thermo"][0] != 1.0
