"""GPU parity on the through-flow and low-Mach configurations that pin the oracle: the
plug flow through inlet and outlet (exact fixed point of the single-relaxation mode), the
Poiseuille channel fed by the inlet, and the expanding slab of non-uniform density
(div u = Lambda).  FP64 against the oracle over tens of steps (1e-12 per step in ghat),
FP32 over the same horizon (2e-7 per step)."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import step as OS
from oracle.lattice import CS2

pytestmark = pytest.mark.gpu


def _both(params, P, u, scal, steps):
    from paper_2207_11567_amd import Solver
    s = Solver(params)
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u),
                  None if scal is None else torch.from_numpy(scal))
    s.step(steps)
    pops, sc, k = s.get_state()
    f = s.fields()
    s.close()
    st = OS.init_state(params, torch.from_numpy(P), torch.from_numpy(u),
                       None if scal is None else torch.from_numpy(scal))
    st, _ = OS.run(params, st, steps)
    og = OS.to_storage(params, st["pops"]).numpy()
    dpop = float(np.abs(pops.double().cpu().numpy() - og).max())
    dsc = 0.0
    if scal is not None:
        dsc = float((np.abs(sc.double().cpu().numpy() - st["scal"].numpy()) /
                     np.array(params["weno_scale"][:scal.shape[0]]).reshape(-1, 1, 1, 1)).max())
    return dpop, dsc, f, st


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,shape", [("D2Q9", (1, 3, 12)), ("D3Q27", (3, 2, 8))])
def test_plug_flow_through_inlet_and_outlet(name, shape, prec):
    nz, ny, nx = shape
    D = 2 if name == "D2Q9" else 3
    u_in = [0.05, 0.02, -0.01][:D] + [0.0] * (3 - D)
    P_out = CS2 * 1.01
    for coll in ("bgk", "cumulant"):
        p = L.base_params(name, nx, ny, nz, nu_ref=0.02, collision=coll, rho_ref=1.3,
                          face_bc=["inlet", "outlet"] + ["periodic"] * 4, inlet_u=u_in,
                          outlet_P=P_out, precision=prec)
        u = np.zeros((D,) + shape)
        for d in range(D):
            u[d] = u_in[d]
        dpop, _, _, _ = _both(p, np.full(shape, P_out), u, None, 20)
        assert dpop <= (1e-12 if prec == "fp64" else 2e-7) * 20, (coll, dpop)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_poiseuille_channel(prec):
    H, nu, u_in = 16, 0.25, 0.02
    nx = 3 * H
    p = L.base_params("D2Q9", nx, H, 1, nu_ref=nu, precision=prec,
                      face_bc=["inlet", "outlet", "wall", "wall", "periodic", "periodic"],
                      inlet_u=[u_in, 0.0, 0.0], outlet_P=CS2)
    shape = (1, H, nx)
    P = np.full(shape, CS2)
    u = np.zeros((2,) + shape)
    steps = 200
    dpop, _, f, _ = _both(p, P, u, None, steps)
    assert dpop <= (1e-12 if prec == "fp64" else 2e-7) * steps, dpop


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_expanding_slab(prec):
    nx, ny = 32, 2
    xc = (np.arange(nx) + 0.5) / nx
    T = (1000.0 + 600.0 * xc)[None, None, :] * np.ones((1, ny, 1))
    scal = np.stack([T, np.full((1, ny, nx), 0.5)])
    p = L.base_params("D2Q9", nx, ny, 1, physics="one_step", visc_law="const_mu",
                      nu_ref=0.05, prandtl=1e9, thickening=4.0, T_ref=300.0, precision=prec,
                      face_bc=["wall", "outlet", "periodic", "periodic", "periodic", "periodic"],
                      outlet_P=CS2, inlet_T=300.0, weno_scale=[1700.0, 1.0],
                      chem=[20.0, 15000.0, 300.0, 2000.0, 1.0])
    if prec == "fp32":
        scal = scal.astype(np.float32).astype(np.float64)
    u = np.zeros((2, 1, ny, nx))
    u[0] = 0.001 * (np.arange(nx) + 0.5) / nx
    steps = 50
    dpop, dsc, _, _ = _both(p, np.full((1, ny, nx), CS2), u, scal, steps)
    tol_p, tol_s = (1e-12, 1e-12) if prec == "fp64" else (2e-7, 2e-6)
    assert dpop <= tol_p * steps, dpop
    assert dsc <= tol_s * steps, dsc
