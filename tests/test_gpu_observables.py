"""GPU tests of the observables of Sec. 3 against the FP64 oracle: running mean / RMS of
u and P_h over sampled levels (GPU: Welford inside the step kernel; oracle: two-pass
definition over the same levels), probe records at every level, the generalised flame
surface; and that switching the observables on leaves the time step itself unchanged.

Bounds (FP64): means and RMS to 1e-12 absolute (values <= 0.34, Welford and two-pass
differ by rounding only), probes to 1e-12, the flame surface to 1e-12 relative.  FP32
state over 20 steps: means and RMS to 2e-6 absolute (the FP32 run drifts from the FP64
oracle by ~1e-6 in 20 steps; the accumulation itself is FP64).  At full
size the chamber's initial flame surface is the half circle pi R of its burnt kernel
within 1 %."""
import math

import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import diagnostics as DG
from oracle import step as OS
from tests.gpu_helpers import fetch, gpu_state, make_solver, random_state

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


def _flame_box(prec="fp64", lat="D2Q9", shape=(1, 24, 40)):
    nz, ny, nx = shape
    p = L.base_params(lat, nx, ny, nz, physics="one_step", visc_law="const_mu", nu_ref=0.02, cs_smag=0.17,
                      thickening=2.0, chem=[4.0, 15000.0, 300.0, 2000.0, 1.0], weno_scale=[1700.0, 1.0],
                      face_bc=["wall", "outlet", "wall", "wall", "periodic", "periodic"], precision=prec)
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    c = 0.5 * (1 - np.tanh((np.sqrt(x ** 2 + (y - ny / 2) ** 2) - 8.0) / 2.0))
    scal = np.stack([300.0 + 1700.0 * c, 1.0 - c])
    if prec != "fp64":
        scal = scal.astype(np.float32).astype(np.float64)
    solid = np.zeros(shape, dtype=bool)
    solid[:, 5:8, 25:28] = True
    D = 2 if lat == "D2Q9" else 3
    return p, np.full(shape, CS2), np.zeros((D,) + shape), scal, solid


def _oracle_levels(p, P, u, scal, solid, steps):
    st = OS.init_state(p, torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal), torch.from_numpy(solid))
    levels = []
    for _ in range(steps):
        P_h, rho, uu, sc, _ = OS.fields(p, st)
        levels.append((uu.clone(), P_h.clone(), sc.clone()))
        st, _ = OS.step(p, st)
    return levels, st


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_statistics_match_two_pass_oracle(prec):
    print(f"statistics {prec}", flush=True)
    p, P, u, scal, solid = _flame_box(prec)
    steps, every = 20, 3
    s = make_solver(p)
    s.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    s.set_statistics(every)
    s.step(steps)
    mean, rms, k = s.statistics()
    s.close()
    levels, _ = _oracle_levels(p, P, u, scal, solid, steps)
    sampled = [lv for n, lv in enumerate(levels) if n % every == 0]
    assert k == len(sampled)
    fields = [torch.cat([uu, P_h[None]]) for uu, P_h, _ in sampled]
    om, orr = DG.mean_and_rms(fields)
    fl = torch.from_numpy(~solid)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert (mean.cpu() - om)[:, fl].abs().max() < tol
    assert (rms.cpu() - orr)[:, fl].abs().max() < tol
    assert float(orr[:, fl].max()) > 1e-5                    # the fields did fluctuate


def test_probes_record_every_level():
    p, P, u, scal, solid = _flame_box("fp64", "D3Q27", (6, 10, 20))
    cells = [0 + 20 * (5 + 10 * 3), 7 + 20 * (2 + 10 * 1), 19 + 20 * (9 + 10 * 5)]
    s = make_solver(p)
    s.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    s.set_probes(cells, capacity=8)
    s.step(10)                                   # records stop at the capacity
    rec = s.probes().cpu()
    s.close()
    assert rec.shape == (8, 3, 4)
    levels, _ = _oracle_levels(p, P, u, scal, solid, 8)
    for n, (uu, P_h, _) in enumerate(levels):
        for j, c in enumerate(cells):
            exp = torch.cat([uu.reshape(3, -1)[:, c], P_h.reshape(-1)[c:c + 1]])
            assert (rec[n, j] - exp).abs().max() < 1e-12


def test_observables_leave_the_step_unchanged():
    p, P, u, scal, solid = _flame_box("fp64")
    out = []
    for on in (False, True):
        s = make_solver(p)
        s.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
        s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
        if on:
            s.set_statistics(1)
            s.set_probes([5, 17], capacity=100)
        s.step(15)
        out.append(fetch(s))
        s.close()
    assert np.abs(out[0][0] - out[1][0]).max() < 1e-15
    assert np.abs(out[0][1] - out[1][1]).max() < 1e-12


def test_flame_surface_matches_oracle():
    p, P, u, scal, solid = _flame_box("fp64")
    s = make_solver(p)
    s.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    got = [s.flame_surface(300.0, 2000.0)]
    s.step(10)
    got.append(s.flame_surface(300.0, 2000.0))
    s.close()
    _, st = _oracle_levels(p, P, u, scal, solid, 10)
    st0 = OS.init_state(p, torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal), torch.from_numpy(solid))
    for g, state in zip(got, (st0, st)):
        grid = OS._grid_of(p, state["solid"])
        exp = DG.flame_surface(p, grid, state["scal"][0], 300.0, 2000.0)
        assert abs(g / exp - 1) < 1e-12


def test_chamber_initial_flame_surface_full_size():
    p, P, u, scal, mask = L.chamber2d()
    s = make_solver(p)
    s.set_geometry(torch.from_numpy(mask.astype(np.uint8)))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    A = s.flame_surface(300.0, 2000.0)
    s.close()
    grid = OS._grid_of(p, torch.from_numpy(mask))
    exp = DG.flame_surface(p, grid, torch.from_numpy(scal[0]), 300.0, 2000.0)
    assert abs(A / exp - 1) < 1e-12
    assert abs(A / (math.pi * 100.0) - 1) < 1e-2


def test_step_sums_survive_other_reductions():
    """The sums of the last step are not overwritten by the flame-surface, field-extraction
    or other block reductions that run in between."""
    p, P, u, scal, solid = _flame_box("fp64")
    s = make_solver(p)
    s.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    s.step(4)
    before = s.step_sums()
    s.flame_surface(300.0, 2000.0)
    f = s.fields()
    after = s.step_sums()
    s.close()
    assert before == after
    assert f["sums"] != before                    # the extraction sums the next level
