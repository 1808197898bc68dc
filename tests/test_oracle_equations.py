"""Pins of the oracle's pointwise relations (Sec. 2.1-2.2, Eqs. 2, 4, 6, 7, 8, 13) against
closed-form moment identities that follow from the equations, with velocities rebuilt
from the documented population ordering (not from the oracle's tables)."""
import numpy as np
import pytest
import torch

from oracle import equations as E
from oracle.lattice import CS2, get
from tests.lattice_ref import velocities

LATS = ["D2Q9", "D3Q27"]


def _rand_fields(D, n, seed):
    g = torch.Generator().manual_seed(seed)
    rho = 0.5 + torch.rand(n, generator=g, dtype=torch.float64)
    u = 0.1 * (torch.rand(D, n, generator=g, dtype=torch.float64) - 0.5)
    P = CS2 * (0.8 + 0.4 * torch.rand(n, generator=g, dtype=torch.float64))
    grad = 0.05 * (torch.rand(D, n, generator=g, dtype=torch.float64) - 0.5)
    Lam = 0.01 * (torch.rand(n, generator=g, dtype=torch.float64) - 0.5)
    return rho, u, P, grad, Lam


@pytest.mark.parametrize("name", LATS)
def test_quadrature_weights(name):
    """Third-order quadrature: sum w = 1, sum w c_a c_b = cs2 delta, sum w c_a^2 c_b^2 =
    cs2^2 (a != b), sum w c_a^4 = 3 cs2^2, odd moments vanish."""
    lat = get(name)
    c = velocities(lat.Q)
    w = lat.w.numpy()
    D = c.shape[1]
    assert np.allclose(lat.c.numpy(), c)
    assert abs(w.sum() - 1) < 1e-15
    for a in range(D):
        assert abs((w * c[:, a]).sum()) < 1e-16
        assert abs((w * c[:, a] ** 4).sum() - 3 * CS2 ** 2) < 1e-15
        for b in range(D):
            assert abs((w * c[:, a] * c[:, b]).sum() - CS2 * (a == b)) < 1e-15
            if a != b:
                assert abs((w * c[:, a] ** 2 * c[:, b] ** 2).sum() - CS2 ** 2) < 1e-15
                assert abs((w * c[:, a] ** 3 * c[:, b]).sum()) < 1e-16
    assert [int(x) for x in lat.opp] == list(range(lat.Q - 1, -1, -1))


@pytest.mark.parametrize("name", LATS)
def test_equilibrium_moments(name):
    """sum g_eq = P_h, sum c g_eq = cs2 rho u, sum c c g_eq = cs2 (P_h I + rho u u)."""
    lat = get(name)
    c = torch.from_numpy(velocities(lat.Q))
    rho, u, P, _, _ = _rand_fields(lat.D, 50, 1)
    geq = E.g_eq(lat, P, rho, u)
    assert torch.allclose(geq.sum(0), P, atol=1e-15, rtol=0)
    m1 = torch.einsum("qd,qn->dn", c, geq)
    assert torch.allclose(m1, CS2 * rho * u, atol=1e-15, rtol=0)
    for a in range(lat.D):
        for b in range(lat.D):
            m2 = (c[:, a, None] * c[:, b, None] * geq).sum(0)
            ref = CS2 * (P * (a == b) + rho * u[a] * u[b])
            assert torch.allclose(m2, ref, atol=1e-15, rtol=0)
    feq = E.f_eq(lat, rho, u)
    assert torch.allclose(feq.sum(0), rho, atol=1e-14, rtol=0)
    assert torch.allclose(torch.einsum("qd,qn->dn", c, feq), rho * u, atol=1e-15, rtol=0)


@pytest.mark.parametrize("name", LATS)
def test_source_moments(name):
    """sum Xi = cs2 (rho Lambda + u.grad rho);  sum c Xi = 0."""
    lat = get(name)
    c = torch.from_numpy(velocities(lat.Q))
    rho, u, P, grad, Lam = _rand_fields(lat.D, 50, 2)
    Xi = E.source_Xi(lat, rho, u, grad, Lam)
    assert torch.allclose(Xi.sum(0), CS2 * (rho * Lam + (u * grad).sum(0)), atol=1e-16, rtol=0)
    assert torch.allclose(torch.einsum("qd,qn->dn", c, Xi), torch.zeros(lat.D, 50, dtype=torch.float64),
                          atol=1e-17, rtol=0)


@pytest.mark.parametrize("name", LATS)
def test_moments_and_half_source(name):
    """Eq. 7 on an equilibrium returns its pressure plus the half-Lambda term and u;
    Eq. 8 undoes Eq. 13 up to the full source (no collision: g* = g + Xi, Eq. 1)."""
    lat = get(name)
    rho, u, P, grad, Lam = _rand_fields(lat.D, 40, 3)
    geq = E.g_eq(lat, P, rho, u)
    Ph, uu = E.moments(lat, geq, rho, Lam)
    assert torch.allclose(Ph, P + 0.5 * rho * CS2 * Lam, atol=1e-15, rtol=0)
    assert torch.allclose(uu, u, atol=1e-15, rtol=0)
    Xi = E.source_Xi(lat, rho, u, grad, Lam)
    fp = E.precondition(geq, Xi, rho)
    assert torch.allclose(E.post_collision(fp, Xi, rho), geq + Xi, atol=1e-15, rtol=0)


@pytest.mark.parametrize("name", LATS)
def test_rest_state_preconditioned_is_weights(name):
    """At rest with P_h = rho cs2 and no source, f'_i = w_i exactly (any rho)."""
    lat = get(name)
    rho = torch.tensor([0.3, 1.0, 2.5], dtype=torch.float64)
    u = torch.zeros(lat.D, 3, dtype=torch.float64)
    geq = E.g_eq(lat, rho * CS2, rho, u)
    fp = E.precondition(geq, torch.zeros_like(geq), rho)
    assert torch.allclose(fp, lat.w[:, None].expand_as(fp), atol=1e-16, rtol=0)


@pytest.mark.parametrize("name", LATS)
def test_bgk_relaxes_to_equilibrium(name):
    """BGK with omega = 1 returns the pre-conditioned equilibrium; omega = 0 is identity."""
    lat = get(name)
    rho, u, P, _, _ = _rand_fields(lat.D, 30, 4)
    g = E.g_eq(lat, P, rho, u) * (1 + 0.01 * torch.randn(lat.Q, 30, dtype=torch.float64,
                                                         generator=torch.Generator().manual_seed(9)))
    fp = g / (rho * CS2)
    out1 = E.bgk_preconditioned(lat, fp, P, rho, u, 1.0)
    assert torch.allclose(out1, E.g_eq(lat, P, rho, u) / (rho * CS2), atol=1e-15, rtol=0)
    assert torch.equal(E.bgk_preconditioned(lat, fp, P, rho, u, 0.0), fp)
