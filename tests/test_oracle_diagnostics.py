"""Pins of the oracle's observables: the generalised flame surface of a planar front is
the front's extent exactly (the central differences telescope), that of a circular
front of radius R is its circumference 2 pi R within the profile's discretisation error,
and that of a spherical front its mean iso-surface area 4 pi (R^2 + pi^2 w^2/12) (tanh
profile of width w: r - R = w artanh(1 - 2c), whose square averages to pi^2 w^2/12 over
c in (0, 1)); mean / RMS of a sampled sinusoid are its mean and
amplitude / sqrt(2)."""
import math

import numpy as np
import torch

import lbm_inputs as L
from oracle import diagnostics as DG
from oracle.grid import Grid


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)


def test_planar_front_surface_telescopes():
    nx, ny = 64, 24
    p = L.base_params("D2Q9", nx, ny, 1, face_bc=["wall", "wall", "periodic", "periodic", "periodic", "periodic"])
    x = np.arange(nx, dtype=float)[None, None, :] * np.ones((1, ny, nx))
    c = 0.5 * (1 + np.tanh((x - 30.3) / 2.5))
    T = 300.0 + 1700.0 * c
    A = DG.flame_surface(p, Grid(p), t(T), 300.0, 2000.0)
    # per row: sum_x (c(x+1) - c(x-1))/2 with mirror ghosts = (c_last + c_last - c_0 - c_0)/2
    exact = ny * (c[0, 0, -1] - c[0, 0, 0])
    assert abs(A - exact) < 1e-12 * ny
    assert abs(A - ny) < 1e-4 * ny


def test_circular_front_surface_is_circumference():
    n, R = 128, 30.0
    p = L.base_params("D2Q9", n, n, 1)
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    r = np.hypot(x - 63.7, y - 64.2)
    c = 0.5 * (1 - np.tanh((r - R) / 2.0))
    A = DG.flame_surface(p, Grid(p), t((300.0 + 1700.0 * c)[None]), 300.0, 2000.0)
    assert abs(A / (2 * math.pi * R) - 1) < 5e-3


def test_spherical_front_surface_is_area():
    n, R = 48, 15.0
    p = L.base_params("D3Q27", n, n, n)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    r = np.sqrt((x - 23.6) ** 2 + (y - 24.1) ** 2 + (z - 23.8) ** 2)
    c = 0.5 * (1 - np.tanh((r - R) / 2.0))
    A = DG.flame_surface(p, Grid(p), t(300.0 + 1700.0 * c), 300.0, 2000.0)
    assert abs(A / (4 * math.pi * (R ** 2 + math.pi ** 2 * 2.0 ** 2 / 12)) - 1) < 2e-3


def test_mean_and_rms_of_a_sinusoid():
    k = np.arange(400)
    samples = [t(np.full((2, 3), 0.3 + 0.02 * math.sin(2 * math.pi * i / 40))) for i in k]
    m, r = DG.mean_and_rms(samples)
    assert torch.allclose(m, torch.full((2, 3), 0.3, dtype=torch.float64), atol=1e-15)
    assert torch.allclose(r, torch.full((2, 3), 0.02 / math.sqrt(2), dtype=torch.float64), atol=1e-15)
