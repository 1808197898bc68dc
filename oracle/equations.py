"""Pointwise relations of Sec. 2.1-2.2 of the paper, each written as printed.

Tensor conventions: populations (Q, *grid); vectors (D, *grid); scalars (*grid); all
float64.  Lattice units dr = dt = 1, c_s^2 = 1/3.
"""
import torch

from .lattice import CS2


def _bc(t, ndim):
    """Broadcast a (Q,) table against (Q, *grid)."""
    return t.reshape(t.shape + (1,) * ndim)


def c_dot(lat, v):
    """c_i . v for v of shape (D, *grid) -> (Q, *grid)."""
    return torch.einsum("qd,d...->q...", lat.c, v)


def f_eq(lat, rho, u):
    """Eq. 4: density equilibrium w_i rho (1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u^2/(2 cs2))."""
    cu = c_dot(lat, u)
    uu = (u * u).sum(0)
    return _bc(lat.w, rho.ndim) * rho * (1.0 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2))


def g_eq(lat, P_h, rho, u):
    """Eq. 6: pressure-based equilibrium w_i (P_h - rho cs2) + cs2 f_eq_i."""
    return _bc(lat.w, rho.ndim) * (P_h - rho * CS2) + CS2 * f_eq(lat, rho, u)


def source_Xi(lat, rho, u, grad_rho, Lam):
    """Eq. 2: Xi_i = cs2 (f_eq_i/rho - w_i) (c_i - u).grad(rho) + w_i rho cs2 Lambda."""
    w = _bc(lat.w, rho.ndim)
    c_minus_u_dot_grad = c_dot(lat, grad_rho) - (u * grad_rho).sum(0)
    return CS2 * (f_eq(lat, rho, u) / rho - w) * c_minus_u_dot_grad + w * rho * CS2 * Lam


def moments(lat, g, rho, Lam):
    """Eq. 7a/7b: P_h = sum g + (dt/2) rho cs2 Lambda;  rho u = sum c g / cs2.
    Returns (P_h, u)."""
    P_h = g.sum(0) + 0.5 * rho * CS2 * Lam
    rho_u = torch.einsum("qd,q...->d...", lat.c, g) / CS2
    return P_h, rho_u / rho


def precondition(g, Xi, rho):
    """Eq. 13: f'_i = g_i/(rho cs2) + dt Xi_i/(2 rho cs2)."""
    return g / (rho * CS2) + Xi / (2.0 * rho * CS2)


def post_collision(f_prime_star, Xi, rho):
    """Eq. 8: g*_i = rho cs2 f'*_i + (dt/2) Xi_i."""
    return rho * CS2 * f_prime_star + 0.5 * Xi


def bgk_preconditioned(lat, f_prime, P_h, rho, u, omega):
    """Single-relaxation-time operator of Eq. 5 applied in the pre-conditioned frame:
    f'* = f' - omega (f' - g_eq/(rho cs2)), with g_eq of Eq. 6.  Test/ablation mode; the
    paper's production operator is the cumulant one."""
    feq_p = g_eq(lat, P_h, rho, u) / (rho * CS2)
    return f_prime - omega * (f_prime - feq_p)
