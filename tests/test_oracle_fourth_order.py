"""Pins of the oracle's fourth-order cumulant parameterisation (Geier, Pasquali and
Schoenherr 2017, applied to the operator the paper takes from Geier et al. 2015, Sec. 2.2):

* the property the parameterisation is derived for: the viscosity of shear waves is
  fourth-order accurate in the wavenumber.  Measured on three linear shear waves in
  periodic D3Q27 boxes (along an axis, u_x(y); along a face diagonal in plane, u_x = -u_y
  of x + y; and out of plane, u_z(x + y), which drives C_111): the relative error of the
  decay rate against nu k^2 falls by more than 9x when the wavelength doubles from 16 to
  32 cells (fourth order: 16x; measured 11x, 16x and 11x), and the unparameterised
  operator's error (second order, pinned elsewhere) is at least 20x larger at 32 cells
  (2x on the face diagonal, where the unparameterised error is already small).  A flipped sign of either
  fourth-order equilibrium, swapped third-order rates (sums against differences), the
  C_111 rate replaced by another one, or a dropped 1/2 in (1/omega - 1/2) each fail;
* the relaxation itself, on one collision with brute-force cumulants (the power-series
  route of test_oracle_cumulant): second order as in the unparameterised operator, each
  third-order pair relaxed in its sum and difference at omega_3 and omega_4, C_111 at
  omega_5, the fourth-order cumulants at their gradient equilibria, orders five and six
  at zero; conservation of the zeroth and first moments;
* the published rate functions with the bulk rate one reduce to the forms with that
  substitution made (two different algebraic forms of the same functions agree)."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import cumulant as C
from oracle import step as S
from oracle.lattice import CS2, get
from tests.lattice_ref import velocities
from tests.test_oracle_cumulant import _random_fprime, _velocity, mgf_cumulants


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


def _decay_error(Lc, nu, kind, **kw):
    """Relative error of the decay rate of a linear shear wave against nu k^2."""
    if kind == "axis":
        shape = (1, Lc, 1)
    else:
        shape = (1, Lc, Lc)
    p = L.base_params("D3Q27", shape[2], shape[1], shape[0], nu_ref=nu, **kw)
    z, y, x = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), np.arange(shape[2]), indexing="ij")
    u = np.zeros((3,) + shape)
    U = 1e-5
    if kind == "axis":
        comp, k2 = 0, (2 * math.pi / Lc) ** 2
        u[0] = U * np.sin(2 * math.pi * y / Lc)
    elif kind == "diagonal":
        comp, k2 = 0, 2 * (2 * math.pi / Lc) ** 2
        ph = 2 * math.pi * (x + y) / Lc
        u[0], u[1] = U * np.sin(ph), -U * np.sin(ph)
    else:
        comp, k2 = 2, 2 * (2 * math.pi / Lc) ** 2
        u[2] = U * np.sin(2 * math.pi * (x + y) / Lc)
    st = S.init_state(p, t(np.full(shape, CS2)), t(u), None)
    prof = t(u[comp])
    # after the transient of the equilibrium start (the slowest third-order rate is 0.08
    # at the shear rate used below), over a fifth of the decay time
    n1 = 300
    n2 = n1 + int(0.2 / (nu * k2))
    amps = []
    for k in range(n2 + 1):
        if k in (n1, n2):
            _, _, uu, _, _ = S.fields(p, st)
            amps.append(float((uu[comp] * prof).sum() / (prof ** 2).sum()))
        if k < n2:
            st, _ = S.step(p, st)
    return math.log(amps[0] / amps[1]) / (n2 - n1) / (nu * k2) - 1


@pytest.mark.parametrize("kind", ["axis", "diagonal", "out_of_plane"])
def test_shear_wave_viscosity_is_fourth_order(kind):
    nu = 0.01                                    # shear rate 1.887, bulk rate 1
    e16 = _decay_error(16, nu, kind, fourth_order=1)
    e32 = _decay_error(32, nu, kind, fourth_order=1)
    p32 = _decay_error(32, nu, kind)
    print(kind, e16, e32, p32)
    assert abs(e16 / e32) > 9.0, (e16, e32)                     # parameterised: fourth order
    assert abs(e32) * (20 if kind != "diagonal" else 2) < abs(p32), (e32, p32)


def test_parameterised_relaxation_cumulant_by_cumulant():
    lat = get("D3Q27")
    c = velocities(lat.Q)
    n = 6
    fp = _random_fprime(lat, n, 13, amp=0.03)
    u = _velocity(lat, fp)
    ws, wb = 1.9, 0.8
    w3, w4, w5, A, B = C.parameterised_rates(ws, wb)
    out, _ = C.cumulant_collide(lat, fp, u, 0.01, 0.0, wb, 0.5, fourth_order=True,
                                omega_s=torch.full((n,), ws, dtype=torch.float64))
    assert torch.allclose(out.sum(0), fp.sum(0), atol=1e-14, rtol=0)
    assert torch.allclose(torch.einsum("qd,qn->dn", lat.c, out), torch.einsum("qd,qn->dn", lat.c, fp),
                          atol=1e-15, rtol=0)
    m0 = fp.sum(0)
    vis = 1.0 / ws - 0.5
    for j in range(n):
        ci = mgf_cumulants((fp[:, j] - lat.w * (m0[j] - 1)).numpy(), c)
        co = mgf_cumulants((out[:, j] - lat.w * (m0[j] - 1)).numpy(), c)
        tr = ci[(2, 0, 0)] + ci[(0, 2, 0)] + ci[(0, 0, 2)]
        tro = co[(2, 0, 0)] + co[(0, 2, 0)] + co[(0, 0, 2)]
        assert abs((tro - 3 * CS2) - (1 - wb) * (tr - 3 * CS2)) < 1e-15
        for e in ((1, 1, 0), (1, 0, 1), (0, 1, 1)):
            assert abs(co[e] - (1 - ws) * ci[e]) < 1e-15
        for a, b in (((1, 2, 0), (1, 0, 2)), ((2, 1, 0), (0, 1, 2)), ((2, 0, 1), (0, 2, 1))):
            assert abs((co[a] + co[b]) - (1 - w3) * (ci[a] + ci[b])) < 1e-14
            assert abs((co[a] - co[b]) - (1 - w4) * (ci[a] - ci[b])) < 1e-14
        assert abs(co[(1, 1, 1)] - (1 - w5) * ci[(1, 1, 1)]) < 1e-14
        # velocity gradients from the pre-collision second cumulants
        dd = [-ws / (2 * CS2) * (ci[e] - tr / 3) - wb / (6 * CS2) * (tr - 3 * CS2)
              for e in ((2, 0, 0), (0, 2, 0), (0, 0, 2))]
        for (a, b), e4 in (((0, 1), (2, 2, 0)), ((0, 2), (2, 0, 2)), ((1, 2), (0, 2, 2))):
            assert abs(co[e4] + (2 / 3) * A * vis * (dd[a] + dd[b])) < 1e-14
        for e2, e4 in (((1, 1, 0), (1, 1, 2)), ((1, 0, 1), (1, 2, 1)), ((0, 1, 1), (2, 1, 1))):
            assert abs(co[e4] - (1 / 3) * B * vis * ws / CS2 * ci[e2]) < 1e-14
        for e in ((2, 2, 1), (2, 1, 2), (1, 2, 2), (2, 2, 2)):
            assert abs(co[e]) < 1e-14


def test_rate_functions_at_unit_bulk_rate():
    for w in (0.7, 1.3, 1.8, 1.95):
        w3, w4, w5, A, B = C.parameterised_rates(w, 1.0)
        assert math.isclose(w3, 8 * (w - 2) * (1 + 2 * w) / (-8 - 14 * w + 7 * w * w), rel_tol=1e-12)
        assert math.isclose(w4, 8 * (w - 2) * (-7 + 4 * w) / (56 - 50 * w + 9 * w * w), rel_tol=1e-12)
        assert math.isclose(w5, 24 * (w - 2) * (-2 - 7 * w + 3 * w * w) / (48 + 152 * w - 130 * w * w + 29 * w ** 3),
                            rel_tol=1e-12)
        assert math.isclose(A, (4 + 2 * w - 3 * w * w) / (2 - 7 * w + 5 * w * w), rel_tol=1e-12)
        assert math.isclose(B, (4 + 28 * w - 14 * w * w) / (6 - 21 * w + 15 * w * w), rel_tol=1e-12)
