"""Pins of the oracle's scalar solver (Sec. 2.3), Lambda (Eq. 3), chemistry, ideal gas and
the noise generator: exact discrete identities, invariants and recurrences."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import noise, scalars
from oracle.grid import Grid
from oracle import step as S
from oracle.lattice import CS2


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


# ------------------------------------------------------------------------------ WENO3
def test_weno3_linear_limit_and_invariances():
    rng = np.random.default_rng(0)
    a, b, c = (t(rng.standard_normal(100)) for _ in range(3))
    # eps -> infinity: the optimal (linear) weights give the third-order upwind face value
    big = scalars.weno3_face(a, b, c, 1e30)
    assert torch.allclose(big, -a / 6 + 5 * b / 6 + c / 3, atol=1e-14, rtol=0)
    # constant data reconstructs the constant
    k = torch.full((5,), 3.7, dtype=torch.float64)
    assert torch.allclose(scalars.weno3_face(k, k, k, 1e-6), k, atol=1e-15, rtol=0)
    # affine equivariance with eps scaled by the square of the factor
    s, off, eps = -2.5, 7.0, 1e-3
    lhs = scalars.weno3_face(s * a + off, s * b + off, s * c + off, eps * s * s)
    assert torch.allclose(lhs, s * scalars.weno3_face(a, b, c, eps) + off, atol=1e-12, rtol=0)


def test_weno3_convergence_order():
    """Mean-norm error of the WENO3 derivative on smooth periodic data falls at least as
    h^2 (the Jiang-Shu third-order scheme degrades near critical points)."""
    errs = []
    for n in (64, 128, 256):
        x = torch.arange(n, dtype=torch.float64) * 2 * math.pi / n
        phi = torch.sin(x) + 0.5 * torch.cos(2 * x)
        v = {k: torch.roll(phi, -k) for k in (-2, -1, 0, 1, 2)}
        for sign in (1.0, -1.0):
            d = scalars.weno3_derivative(v, torch.full_like(phi, sign), 1e-6) * n / (2 * math.pi)
            exact = torch.cos(x) - torch.sin(2 * x)
            errs.append(float((d - exact).abs().mean()))
    e = np.array(errs).reshape(3, 2)
    order = np.log2(e[:-1] / e[1:])
    assert (order > 1.9).all(), order


# ------------------------------------------------------------------------------ diffusion
@pytest.mark.parametrize("lattice,n,nz", [("D2Q9", 48, 1), ("D3Q27", 32, 32)])
def test_gaussian_variance_grows_2FD_per_step(lattice, n, nz):
    """Fluid at rest, passive scalar: second moment about a fixed centre grows by exactly
    2 F D dt per step and axis (three-point Laplacian identity); mass is conserved."""
    F, nu, Pr = 2.0, 0.02, 0.8
    p = L.base_params(lattice, n, n, nz, physics="passive", nu_ref=nu, prandtl=Pr,
                      thickening=F)
    D = 2 if lattice == "D2Q9" else 3
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(n), np.arange(n), indexing="ij")
    c = (n - 1) / 2.0
    r2 = (xx - c) ** 2 + (yy - c) ** 2 + ((zz - (nz - 1) / 2.0) ** 2 if D == 3 else 0)
    T = np.exp(-r2 / (2 * 2.0 ** 2))
    st = S.init_state(p, t(np.full((nz, n, n), CS2)), t(np.zeros((D, nz, n, n))), t(T[None]))
    coords = [t(xx - c), t(yy - c), t(zz - (nz - 1) / 2.0)]
    FD = F * nu / Pr
    m0 = float(st["scal"][0].sum())
    prev = [float((coords[d] ** 2 * st["scal"][0]).sum()) for d in range(D)]
    for _ in range(5):
        st, _ = S.step(p, st)
        assert abs(float(st["scal"][0].sum()) - m0) < 1e-12 * m0
        cur = [float((coords[d] ** 2 * st["scal"][0]).sum()) for d in range(D)]
        for d in range(D):
            assert abs(cur[d] - prev[d] - 2 * FD * m0) < 1e-11 * m0
        prev = cur


def test_zero_flux_walls_conserve_scalar():
    n = 24
    p = L.base_params("D2Q9", n, n, 1, physics="passive", nu_ref=0.05,
                      face_bc=["wall"] * 4 + ["periodic"] * 2)
    solid = torch.zeros(1, n, n, dtype=torch.bool)
    solid[0, 8:14, 10:12] = True
    T = L.random_scalars("passive", (1, n, n), 3)
    st = S.init_state(p, t(np.full((1, n, n), CS2)), t(np.zeros((2, 1, n, n))), t(T), solid)
    fl = ~solid
    m0 = float(st["scal"][0][fl].sum())
    for _ in range(10):
        st, _ = S.step(p, st)
    assert abs(float(st["scal"][0][fl].sum()) - m0) < 1e-12


# ------------------------------------------------------------------------------ coupling
def test_unity_lewis_progress_invariant():
    """theta + y = 1 initially stays 1 (same operators, affine-invariant WENO weights)."""
    n = 32
    p = L.base_params("D2Q9", n, n, 1, physics="one_step", visc_law="const_mu", nu_ref=0.01,
                      thickening=3.0, cs_smag=0.17, T_ref=300.0,
                      weno_scale=[1700.0, 1.0], chem=[0.5, 15000.0, 300.0, 2000.0, 1.0])
    rng = np.random.default_rng(4)
    x = np.arange(n)[None, None, :]
    th = 0.5 * (1 + np.tanh((x - n / 2) / 3.0)) * np.ones((1, n, n))
    th = np.clip(th + 0.02 * rng.standard_normal((1, n, n)), 0, 1)
    scal = np.stack([300 + 1700 * th, 1 - th])
    u = 0.02 * rng.standard_normal((2, 1, n, n))
    st = S.init_state(p, t(np.full((1, n, n), CS2)), t(u), t(scal))
    for _ in range(5):
        st, _ = S.step(p, st)
        T, Y = st["scal"]
        assert torch.allclose((T - 300) / 1700 + Y, torch.ones_like(Y), atol=1e-13, rtol=0)


@pytest.mark.parametrize("collision", ["cumulant", "bgk"])
def test_zero_d_reactor_one_step(collision):
    """Uniform mixture at rest (periodic): u stays 0, T and Y follow the explicit-Euler
    Arrhenius recurrence, and sum_i g grows per step by rho cs2 Lambda = rho cs2 R_T/T.
    In the single-relaxation mode the equilibrium is built from P_h of Eq. 7a, so the
    growth is exact only if P_h carries the half source rho cs2 Lambda / 2."""
    B, Ta, Tu, Tad, F = 2.0, 15000.0, 300.0, 2000.0, 4.0
    p = L.base_params("D2Q9", 4, 4, 1, physics="one_step", visc_law="const_mu", nu_ref=0.01,
                      thickening=F, T_ref=Tu, chem=[B, Ta, Tu, Tad, 1.0], collision=collision)
    T0, Y0 = 1200.0, 0.6
    scal = np.stack([np.full((1, 4, 4), T0), np.full((1, 4, 4), Y0)])
    st = S.init_state(p, t(np.full((1, 4, 4), 0.35)), t(np.zeros((2, 1, 4, 4))), t(scal))
    T, Y = T0, Y0
    for _ in range(6):
        gsum = float(st["pops"].sum(0)[0, 0, 0])
        rho = Tu / T
        r = B * Y * math.exp(-Ta / T) / F
        Lam = (Tad - Tu) * r / T
        st, _ = S.step(p, st)
        T, Y = T + (Tad - Tu) * r, Y - r
        assert abs(float(st["scal"][0, 0, 0, 0]) - T) < 1e-10
        assert abs(float(st["scal"][1, 0, 0, 0]) - Y) < 1e-14
        assert abs(float(st["pops"].sum(0)[0, 0, 0]) - gsum - rho * CS2 * Lam) < 1e-15
        _, _, u, _, _ = S.fields(p, st)
        assert float(u.abs().max()) < 1e-16


def test_zero_d_reactor_two_step_conserves_elements_and_enthalpy():
    chem = L.two_step_chem(B1=5.0e4, B2=5.0e3)
    W, h, cp = chem[5:11], chem[11:17], chem[4]
    p = L.base_params("D2Q9", 4, 4, 1, physics="two_step", visc_law="const_mu", nu_ref=0.01,
                      thickening=2.0, T_ref=320.0, chem=chem)
    yf, yo, yn = L.fresh_ch4_air(0.83)
    Y = [yf, yo, 0.0, 0.0, 0.0]
    scal = np.stack([np.full((1, 4, 4), 1500.0)] + [np.full((1, 4, 4), y) for y in Y])
    st = S.init_state(p, t(np.full((1, 4, 4), CS2)), t(np.zeros((2, 1, 4, 4))), t(scal))

    def invariants(s):
        Yk = [float(s[1 + k, 0, 0, 0]) for k in range(5)]
        Yk.append(1 - sum(Yk))
        Tt = float(s[0, 0, 0, 0])
        C = Yk[0] / W[0] + Yk[2] / W[2] + Yk[3] / W[3]
        H = 4 * Yk[0] / W[0] + 2 * Yk[4] / W[4]
        O = 2 * Yk[1] / W[1] + Yk[2] / W[2] + 2 * Yk[3] / W[3] + Yk[4] / W[4]
        N = Yk[5] / W[5]
        E = cp * Tt + sum(h[k] * Yk[k] / W[k] for k in range(6))
        return np.array([C, H, O, N, E])

    ref = invariants(st["scal"])
    for _ in range(20):
        st, _ = S.step(p, st)
    cur = invariants(st["scal"])
    assert np.allclose(cur, ref, rtol=1e-12, atol=1e-12)
    assert float(st["scal"][1, 0, 0, 0]) < yf            # fuel was consumed
    assert float(st["scal"][0, 0, 0, 0]) > 1500.0        # heat was released


def test_ideal_gas_density():
    chem = L.two_step_chem()
    p = L.base_params("D2Q9", 2, 1, 1, physics="two_step", T_ref=320.0, rho_ref=1.3, chem=chem)
    yf, yo, yn = L.fresh_ch4_air(0.83)
    b = L.burnt_ch4_air(0.83)
    for T, Y in [(320.0, [yf, yo, 0, 0, 0]), (1900.0, [0, b["O2"], 0, b["CO2"], b["H2O"]])]:
        scal = t(np.array([T] + Y).reshape(6, 1, 1, 1))
        rho = float(scalars.density(p, scal, (1, 1, 1)))
        Yfull = Y + [1 - sum(Y)]
        Wm = 1 / sum(y / w for y, w in zip(Yfull, L.W_SPECIES))
        assert abs(rho * T / Wm - 1.3 * 320.0 / chem[17]) < 1e-9
    p1 = L.base_params("D2Q9", 2, 1, 1, physics="one_step", T_ref=300.0, rho_ref=1.0)
    assert abs(float(scalars.density(p1, t(np.array([2000.0, 0]).reshape(2, 1, 1, 1)),
                                     (1, 1, 1))) - 0.15) < 1e-15


# ------------------------------------------------------------------------------ noise
def test_splitmix_published_vector_and_moments():
    """SplitMix64 from state 0 yields 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
    0x06C45D188009454F (published reference outputs); xi has zero mean, unit variance."""
    assert noise.raw(0, 1) == 0xE220A8397B1DCDAF
    assert noise.raw(0, 2) == 0x6E789E6AA1B965F4
    assert noise.raw(0, 3) == 0x06C45D188009454F
    a, b = np.meshgrid(np.arange(256), np.arange(256))
    x = noise.xi(2207, a, b, 5)
    assert abs(x.mean()) < 0.02 and abs(x.var() - 1) < 0.02
    assert np.abs(x).max() <= math.sqrt(3)


def test_reacting_box_chemistry_is_in_the_explicit_stable_range():
    """Workload recipe: with the default 2-step constants the explicit CO update of the
    reacting box is contractive (lambda_CO < 1 per step): over 60 steps of an axial column
    of the box CO stays non-negative up to WENO/diffusion round-off and T does not
    overshoot the burnt temperature."""
    p, P, u, sc = L.reacting_box(4, 4, 384)
    st = S.init_state(p, t(P), t(u), t(sc))
    for _ in range(60):
        st, _ = S.step(p, st)
    s = st["scal"].numpy()
    ch, F = p["chem"], p["thickening"]
    rho = scalars.density(p, st["scal"], Grid(p).shape).numpy()
    lam = ch[2] / F * np.exp(-ch[3] / s[0]) * np.sqrt(rho * np.maximum(s[2], 0) / L.W_SPECIES[1])
    assert lam.max() < 0.5
    assert s[3].min() > -1e-5
    assert s[0].max() < 1970.0
