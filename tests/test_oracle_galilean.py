"""Pins of the oracle's optional Galilean correction of the cumulant collision (Geier et al.
2015; the paper applies that operator after pre-conditioning, Sec. 2.2):

* the diagonal strain estimated from the pre-collision second cumulants is the velocity
  gradient of the flow (spectral derivative of the simulated field) to first order, for
  a compressional and shear wave with the bulk rate above and below one, so both its
  deviatoric and its trace coefficient are fixed;
* Navier-Stokes is Galilean invariant: a small-amplitude vortex field decays at the same
  rate in a frame moving at Ma ~ 0.25; without the correction the lattice's c^3 = c
  aliasing changes the rate by several per cent, with it the rate agrees to a few 1e-3
  (2-D Taylor-Green cell advected diagonally; 3-D superposed cells in the three planes,
  advected obliquely);
* a uniform flow at equilibrium has no strain, so the correction leaves it unchanged."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import cumulant as CU
from oracle import equations
from oracle import step as S
from oracle.lattice import CS2


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


@pytest.mark.parametrize("wb", [0.8, 1.6])
def test_strain_estimate_matches_velocity_gradient(wb):
    n, ny, nu = 32, 4, 0.02
    p = L.base_params("D2Q9", n, ny, 1, nu_ref=nu, omega_bulk=wb)
    x = np.arange(n)[None, None, :] * np.ones((1, ny, n))
    k = 2 * math.pi / n
    P = CS2 + 1e-3 * CS2 * np.cos(k * x)               # standing sound wave: div u != 0
    u = np.zeros((2, 1, ny, n))
    u[1] = 1e-3 * np.sin(k * x)                         # and a shear wave
    st = S.init_state(p, t(P), t(u), None)
    for _ in range(37):
        st, _ = S.step(p, st)
    lat, _, rho, g, _, Lam, _, uu, grad_rho = S._level_n(p, st)
    fp = equations.precondition(g, equations.source_Xi(lat, rho, uu, grad_rho, Lam), rho)
    f_t = fp - lat.w.reshape((-1, 1, 1, 1)) * (fp.sum(0) - 1.0)
    C = CU.moments_to_cumulants(CU.central_moments(lat, f_t, uu))
    dd = CU.diagonal_strain(lat, C, 1.0 / (nu / CS2 + 0.5), wb)
    ux = uu[0, 0, 0].numpy()
    dux = np.real(np.fft.ifft(1j * 2 * np.pi * np.fft.fftfreq(n) * np.fft.fft(ux)))
    scale = np.abs(dux).max()
    assert scale > 5e-5
    assert np.abs(dd[0][0, 0].numpy() - dux).max() < 0.03 * scale
    assert np.abs(dd[1][0, 0].numpy()).max() < 0.03 * scale          # d_y v = 0


def _decay_rate(p, P, u, steps, every):
    st = S.init_state(p, t(P), t(u), None)
    ks, es = [], []
    for s in range(steps + 1):
        if s % every == 0:
            _, _, uu, _, _ = S.fields(p, st)
            f = uu - uu.mean(dim=tuple(range(1, uu.dim())), keepdim=True)
            ks.append(s)
            es.append(float((f ** 2).sum()))
        if s < steps:
            st, _ = S.step(p, st)
    return -np.polyfit(ks[1:], np.log(es[1:]), 1)[0]


def test_advected_taylor_green_decay_2d():
    n, nu = 32, 0.02
    rates = {}
    for Ua, gal in (((0.0, 0.0), 0), ((0.1, 0.1), 0), ((0.1, 0.1), 1)):
        p, P, u = L.tgv(n, U0=0.02, nu=nu)
        p["galilean"] = gal
        u = u + np.array(Ua).reshape(2, 1, 1, 1)
        rates[(Ua, gal)] = _decay_rate(p, P, u, 300, 20)
    r0 = rates[((0.0, 0.0), 0)]
    kk = 2 * math.pi / n
    assert abs(r0 / (4 * nu * kk * kk) - 1) < 2e-3
    assert abs(rates[((0.1, 0.1), 0)] / r0 - 1) > 3e-2               # the aliasing error
    assert abs(rates[((0.1, 0.1), 1)] / r0 - 1) < 3e-3               # removed


def test_advected_vortex_decay_3d():
    n, nu, A = 12, 0.02, 0.01
    k = 2 * math.pi / n
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    u = np.zeros((3, n, n, n))
    for a, b, c in ((0, 1, (x, y)), (1, 2, (y, z)), (2, 0, (z, x))):
        u[a] += A * np.sin(k * c[0]) * np.cos(k * c[1])
        u[b] -= A * np.cos(k * c[0]) * np.sin(k * c[1])
    P = np.full((n, n, n), CS2)
    rates = {}
    for Ua, gal in (((0.0, 0.0, 0.0), 0), ((0.1, 0.07, -0.08), 0), ((0.1, 0.07, -0.08), 1)):
        p = L.base_params("D3Q27", n, n, n, nu_ref=nu, galilean=gal)
        rates[(Ua, gal)] = _decay_rate(p, P, u + np.array(Ua).reshape(3, 1, 1, 1), 100, 10)
    r0 = rates[((0.0, 0.0, 0.0), 0)]
    assert abs(rates[((0.1, 0.07, -0.08), 0)] / r0 - 1) > 2e-2
    assert abs(rates[((0.1, 0.07, -0.08), 1)] / r0 - 1) < 6e-3


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 5, 6)), ("D3Q27", (4, 5, 3))])
def test_uniform_flow_is_untouched(lat, shape):
    nz, ny, nx = shape
    D = 2 if lat == "D2Q9" else 3
    u = np.zeros((D,) + shape) + np.array([0.12, -0.07, 0.05][:D]).reshape(D, 1, 1, 1)
    P = np.full(shape, CS2)
    out = []
    for gal in (0, 1):
        p = L.base_params(lat, nx, ny, nz, nu_ref=0.03, omega_bulk=1.3, galilean=gal)
        st, _ = S.step(p, S.init_state(p, t(P), t(u), None))
        out.append(st["pops"])
    assert float((out[0] - out[1]).abs().max()) < 1e-15
