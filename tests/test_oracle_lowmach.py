"""Pin of the low-Mach coupling of Sec. 2.1 on a non-uniform density field: the source
term Xi of Eq. 2 (its grad(rho) part and the rho cs2 Lambda part), the half source of the
pre-conditioning (Eq. 13) and of the post-collision form (Eq. 8) must together make the
simulated velocity satisfy the continuity constraint div u = Lambda of Eq. 3.

Set-up: a quasi-1-D slab closed by a wall at x = -1/2 and open to a pressure outlet at
x = nx - 1/2, filled with a lean mixture whose temperature rises linearly along x (so the
ideal-gas density varies by a factor 1.6) and which burns slowly, without diffusion.
Every cell is then a small reactor expanding at its own rate Lambda(x), and in 1-D the
low-Mach velocity is fixed by kinematics alone: u(x) = int_{-1/2}^{x} Lambda.  The flow
starts from that velocity at a uniform pressure; the acoustic waves of the missing
pressure field are averaged out over one period of the slab's quarter-wave mode
(4 nx / cs steps).  The averaged velocity must follow the averaged integral within
1 % of the outflow velocity (the remainder is the lag of the weakly compressible scheme
behind the changing Lambda, O(Ma^2)).  Dropping the grad(rho) part of Xi, the density
factor of its Lambda part, or doubling either half source moves it by 6-400 %.

The half-source term of P_h (Eq. 7a) does not reach the cumulant operator (the zeroth
moment of f' passes through it); in the single-relaxation mode the equilibrium is built
from P_h, and mass is conserved by that collision only if P_h carries exactly
rho cs2 Lambda / 2: a uniform reactor at rest then gains exactly rho cs2 Lambda per step
in sum g (the test below runs it in both modes)."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import scalars as SC
from oracle import step as S
from oracle.grid import Grid
from oracle.lattice import CS2


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


def _lambda(p, scal, solid):
    grid = Grid(p, solid, None)
    rho = SC.density(p, scal, grid.shape)
    return SC.nonadvective_rhs(p, grid, scal, rho)[1]


def _from_wall(Lam):
    """int_{-1/2}^{x} Lambda at the cell centres (midpoint rule)."""
    return torch.cumsum(Lam, -1) - Lam / 2


def test_expanding_slab_velocity_is_the_integral_of_lambda():
    nx, ny = 32, 2
    xc = (np.arange(nx) + 0.5) / nx
    T = (1000.0 + 600.0 * xc)[None, None, :] * np.ones((1, ny, 1))
    scal = t(np.stack([T, np.full((1, ny, nx), 0.5)]))
    p = L.base_params("D2Q9", nx, ny, 1, physics="one_step", visc_law="const_mu",
                      nu_ref=0.05, prandtl=1e9, thickening=4.0, T_ref=300.0,
                      face_bc=["wall", "outlet", "periodic", "periodic", "periodic", "periodic"],
                      outlet_P=CS2, inlet_T=300.0, weno_scale=[1700.0, 1.0],
                      chem=[20.0, 15000.0, 300.0, 2000.0, 1.0])
    solid = torch.zeros((1, ny, nx), dtype=torch.bool)
    u0 = torch.zeros((2, 1, ny, nx), dtype=torch.float64)
    u0[0] = _from_wall(_lambda(p, scal, solid))
    st = S.init_state(p, torch.full((1, ny, nx), CS2, dtype=torch.float64), u0, scal)
    period = int(round(4 * nx / math.sqrt(CS2)))
    u_acc = torch.zeros(nx, dtype=torch.float64)
    ref_acc = torch.zeros(nx, dtype=torch.float64)
    for k in range(2 * period):
        if k >= period:
            _, rho, u, _, _ = S.fields(p, st)
            assert float((u[0, 0, 0] - u[0, 0, 1]).abs().max()) < 1e-15  # stays 1-D
            u_acc += u[0, 0, 0]
            ref_acc += _from_wall(_lambda(p, st["scal"], solid))[0, 0]
        st, _ = S.step(p, st)
    rho = SC.density(p, st["scal"], (1, ny, nx))
    assert float(rho.max() / rho.min()) > 1.5                         # non-uniform density
    assert float(ref_acc[-1]) / period > 1e-3                         # a real expansion
    err = float((u_acc - ref_acc).abs().max() / ref_acc[-1])
    assert err < 1e-2, err
