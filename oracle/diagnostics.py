"""Observables of Sec. 3: the flame surface of the deflagration chamber (its evolution is
compared with DNS and LES in Sec. 3.1), time-averaged velocities with their RMS and the
RMS of the pressure fluctuations (Sec. 3.2), and velocity / pressure recorded every step
at probe points for spectra (Sec. 3.2, precessing vortex core).

Test infrastructure: see the package header.

Readings (the paper names the quantities, not their discretisation):
* flame surface = the generalised surface: the integral over the fluid of |grad c| with
  c = (T - T_u)/(T_b - T_u) the progress variable (by the coarea formula the mean over
  iso-levels of the iso-surface area), grad c by the central differences and ghost rules
  of the density gradient (R6: mirror at walls and solids, inlet value, own value at the
  outlet); lattice units (cells of area 1, or length 1 in 2-D);
* statistics over the sampled levels: mean of u_d and of P_h, RMS = the population standard
  deviation sqrt(mean((x - mean)^2)), here by the two-pass definition;
* probes: u and P_h of Eq. 7 at the probe cells, at every level n (before the step).
"""
import torch

from . import scalars


def progress(T, T_u, T_b):
    return (T - T_u) / (T_b - T_u)


def flame_surface(params, grid, T, T_u, T_b):
    """sum over fluid cells of |grad c| (central differences, ghost rules of grad rho)."""
    c = progress(T, T_u, T_b)
    c_in = (float(params["inlet_T"]) - T_u) / (T_b - T_u)
    g = scalars.gradient(grid, c, c_in)
    mag = torch.sqrt((g * g).sum(0))
    return float(mag[grid.fluid].sum())


def mean_and_rms(samples):
    """samples: list of tensors of one shape; returns (mean, rms) by two passes."""
    x = torch.stack(samples)
    mean = x.mean(0)
    rms = torch.sqrt(((x - mean) ** 2).mean(0))
    return mean, rms
