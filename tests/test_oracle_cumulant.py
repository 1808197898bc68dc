"""Pins of the oracle's cumulant collision (Sec. 2.2, Eqs. 9-14 as read):
* set-partition enumeration against Bell numbers and the no-singleton counts;
* cumulants against an independent brute force: the Taylor coefficients of the log of
  the moment generating function, by truncated power-series arithmetic;
* collision invariants (zeroth/first moments), identity at zero rates, the product-form
  equilibrium as fixed point and as the exact output at unit rates, rest state;
* Smagorinsky closed form (root of the quadratic in tau) and Cs = 0."""
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import cumulant as C
from oracle.lattice import CS2, get
from tests.lattice_ref import velocities

LATS = ["D2Q9", "D3Q27"]


def test_set_partitions_counts():
    bell = [1, 1, 2, 5, 15, 52, 203]
    no_single = [1, 0, 1, 1, 4, 11, 41]
    for n in range(7):
        parts = list(C.set_partitions(list(range(n))))
        assert len(parts) == bell[n]
        assert sum(1 for p in parts if all(len(b) > 1 for b in p)) == no_single[n]


def _series_mul(a, b):
    D = a.ndim
    out = np.zeros_like(a)
    for ea in itertools.product(range(3), repeat=D):
        if a[ea] == 0:
            continue
        for eb in itertools.product(range(3), repeat=D):
            e = tuple(x + y for x, y in zip(ea, eb))
            if max(e) <= 2:
                out[e] += a[ea] * b[eb]
    return out


def mgf_cumulants(p, c):
    """Cumulants c_e (exponents <= 2 per axis) of the discrete distribution p on velocities
    c, from ln M(lambda), M = sum_i p_i exp(lambda . c_i), by power series."""
    Q, D = c.shape
    X = np.zeros((3,) * D)
    for e in itertools.product(range(3), repeat=D):
        if sum(e) == 0:
            continue
        X[e] = sum(p[i] * np.prod([c[i, d] ** e[d] / math.factorial(e[d]) for d in range(D)])
                   for i in range(Q))
    logM = np.zeros_like(X)
    Xk = np.zeros_like(X)
    Xk[(0,) * D] = 1.0
    for k in range(1, 2 * D + 1):
        Xk = _series_mul(Xk, X)
        logM += (-1) ** (k + 1) * Xk / k
    return {e: logM[e] * np.prod([math.factorial(x) for x in e])
            for e in itertools.product(range(3), repeat=D)}


@pytest.mark.parametrize("name", LATS)
def test_cumulants_brute_force(name):
    lat = get(name)
    c = velocities(lat.Q)
    rng = np.random.default_rng(7)
    for trial in range(3):
        p = lat.w.numpy() * (1 + 0.3 * rng.uniform(-1, 1, lat.Q))
        p /= p.sum()
        mean = torch.from_numpy(p @ c)
        kappa = C.central_moments(lat, torch.from_numpy(p), mean)
        cum = C.moments_to_cumulants(kappa)
        ref = mgf_cumulants(p, c)
        for e, v in cum.items():
            assert abs(float(v) - ref[e]) < 1e-14, (e, float(v), ref[e])
        back = C.cumulants_to_moments(cum, kappa[(0,) * lat.D])
        for e in back:
            assert abs(float(back[e] - kappa[e])) < 1e-15


def _random_fprime(lat, n, seed, amp=0.02):
    g = torch.Generator().manual_seed(seed)
    fp = lat.w[:, None] * (1.05 + amp * torch.randn(lat.Q, n, dtype=torch.float64, generator=g))
    fp = fp + 0.02 * lat.w[:, None] * lat.c[:, 0, None]          # some x-momentum
    return fp


def _velocity(lat, fp):
    m0 = fp.sum(0)
    f_t = fp - lat.w[:, None] * (m0 - 1)
    return torch.einsum("qd,qn->dn", lat.c, f_t)


@pytest.mark.parametrize("name", LATS)
def test_collision_conserves_and_identity(name):
    lat = get(name)
    fp = _random_fprime(lat, 64, 1)
    u = _velocity(lat, fp)
    out, _ = C.cumulant_collide(lat, fp, u, 0.01, 0.0, 1.3, 0.8, omega_s=torch.full((64,), 1.7,
                                                                                     dtype=torch.float64))
    assert torch.allclose(out.sum(0), fp.sum(0), atol=1e-14, rtol=0)
    assert torch.allclose(torch.einsum("qd,qn->dn", lat.c, out),
                          torch.einsum("qd,qn->dn", lat.c, fp), atol=1e-15, rtol=0)
    zero = torch.zeros(64, dtype=torch.float64)
    same, _ = C.cumulant_collide(lat, fp, u, 0.01, 0.0, 0.0, 0.0, omega_s=zero)
    assert torch.allclose(same, fp, atol=1e-14, rtol=0)


def _product_form(lat, u, m0):
    """prod_d phi(c_d; u_d) with the 1-D law of mean u and variance cs2, plus the
    rest-weight pressure shift w (m0 - 1)."""
    out = torch.ones(lat.Q, u.shape[1], dtype=torch.float64)
    for d in range(lat.D):
        cd = lat.c[:, d, None]
        ud = u[d][None]
        phi = torch.where(cd == 0, 1 - CS2 - ud ** 2,
                          torch.where(cd > 0, (CS2 + ud ** 2 + ud) / 2, (CS2 + ud ** 2 - ud) / 2))
        out = out * phi
    return out + lat.w[:, None] * (m0 - 1)


@pytest.mark.parametrize("name", LATS)
def test_product_form_is_equilibrium(name):
    lat = get(name)
    fp = _random_fprime(lat, 32, 2)
    u = _velocity(lat, fp)
    m0 = fp.sum(0)
    one = torch.ones(32, dtype=torch.float64)
    out, _ = C.cumulant_collide(lat, fp, u, 0.0, 0.0, 1.0, 1.0, omega_s=one)
    assert torch.allclose(out, _product_form(lat, u, m0), atol=1e-15, rtol=0)
    eq = _product_form(lat, u, m0)
    again, _ = C.cumulant_collide(lat, eq, u, 0.0, 0.0, 0.6, 1.4, omega_s=1.9 * one)
    assert torch.allclose(again, eq, atol=1e-15, rtol=0)


@pytest.mark.parametrize("name", LATS)
def test_rest_state_fixed_point(name):
    lat = get(name)
    fp = lat.w[:, None].repeat(1, 4)
    out, om = C.cumulant_collide(lat, fp, torch.zeros(lat.D, 4, dtype=torch.float64),
                                 0.02, 0.17, 1.2, 0.7)
    assert torch.allclose(out, fp, atol=1e-15, rtol=0)
    assert torch.allclose(om, torch.full((4,), 1.0 / (0.02 / CS2 + 0.5), dtype=torch.float64))


@pytest.mark.parametrize("name", LATS)
def test_smagorinsky_closed_form(name):
    """tau solves tau^2 - tau0 tau - Cs^2 Qbar/(2 cs2^2) = 0 with Qbar = sqrt(2 Pi:Pi), Pi
    computed here directly from the distribution; the shear cumulant relaxes by 1 - 1/tau."""
    lat = get(name)
    c = torch.from_numpy(velocities(lat.Q))
    fp = _random_fprime(lat, 16, 3, amp=0.05)
    u = _velocity(lat, fp)
    nu, cs = 0.004, 0.17
    m0 = fp.sum(0)
    f_t = fp - lat.w[:, None] * (m0 - 1)
    PiPi = torch.zeros(16, dtype=torch.float64)
    for a in range(lat.D):
        for b in range(lat.D):
            Pab = ((c[:, a, None] - u[a]) * (c[:, b, None] - u[b]) * f_t).sum(0) - CS2 * (a == b)
            PiPi += Pab ** 2
    Qbar = torch.sqrt(2 * PiPi)
    out, om = C.cumulant_collide(lat, fp, u, nu, cs, 1.0, 1.0)
    tau, tau0 = 1 / om, nu / CS2 + 0.5
    assert torch.allclose(tau * tau - tau0 * tau - cs * cs * Qbar / (2 * CS2 ** 2),
                          torch.zeros(16, dtype=torch.float64), atol=1e-15, rtol=0)
    _, om0 = C.cumulant_collide(lat, fp, u, nu, 0.0, 1.0, 1.0)
    assert torch.allclose(om0, torch.full((16,), 1 / tau0, dtype=torch.float64))
    fo = out - lat.w[:, None] * (m0 - 1)
    k_in = ((c[:, 0, None] - u[0]) * (c[:, 1, None] - u[1]) * f_t).sum(0)
    k_out = ((c[:, 0, None] - u[0]) * (c[:, 1, None] - u[1]) * fo).sum(0)
    assert torch.allclose(k_out, (1 - om) * k_in, atol=1e-16, rtol=0)


@pytest.mark.parametrize("name", LATS)
def test_relaxation_at_intermediate_rates(name):
    """One collision at rates strictly between 0 and 1 (shear 0.3, bulk 0.45, order >= 3
    0.6), cumulants of input and output from the independent brute force above: every
    cumulant of order >= 3 comes out scaled by exactly 1 - omega_high, the off-diagonal and
    deviatoric second-order ones by 1 - omega_s, the trace's distance from D cs2 by
    1 - omega_bulk, and the mean is untouched (rates 0 and 1 alone cannot tell 1 - w from,
    say, (1 - w)^2)."""
    lat = get(name)
    c = velocities(lat.Q)
    n = 8
    fp = _random_fprime(lat, n, 11, amp=0.05)
    u = _velocity(lat, fp)
    ws, wb, wh = 0.3, 0.45, 0.6
    out, _ = C.cumulant_collide(lat, fp, u, 0.01, 0.0, wb, wh,
                                omega_s=torch.full((n,), ws, dtype=torch.float64))
    m0 = fp.sum(0)
    D = lat.D
    diag = [tuple(2 if k == d else 0 for k in range(D)) for d in range(D)]
    for j in range(n):
        f_in = (fp[:, j] - lat.w * (m0[j] - 1)).numpy()
        f_out = (out[:, j] - lat.w * (m0[j] - 1)).numpy()
        assert abs(f_in.sum() - 1) < 1e-14 and abs(f_out.sum() - 1) < 1e-14
        ci, co = mgf_cumulants(f_in, c), mgf_cumulants(f_out, c)
        checked = 0
        for e in ci:
            order = sum(e)
            if order == 1:
                assert abs(co[e] - ci[e]) < 1e-15
            elif order >= 3:
                assert abs(co[e] - (1 - wh) * ci[e]) < 1e-14, (e, co[e], ci[e])
                checked += abs(ci[e]) > 1e-9              # the input really has them
            elif order == 2 and e not in diag:
                assert abs(co[e] - (1 - ws) * ci[e]) < 1e-15
        tr_in = sum(ci[e] for e in diag)
        tr_out = sum(co[e] for e in diag)
        assert abs((tr_out - D * CS2) - (1 - wb) * (tr_in - D * CS2)) < 1e-15
        for e in diag:
            assert abs((co[e] - tr_out / D) - (1 - ws) * (ci[e] - tr_in / D)) < 1e-15
        assert checked == (3 if D == 2 else 17)
