"""Parity at the workloads' full sizes, in the launch configuration bench.py times: the
GPU initialises the full grid from the workload's seeded fields and advances it a few
steps; the oracle initialises sampled windows from the same fields (window + halo cut
from the workload's input arrays, never from the GPU) and advances them as many steps.
Faces that a window does not share with the domain are fake; every output of a cell
depends on inputs at most 2 cells away per step, so a halo of 3 cells per step is
excluded from the comparison.  Bounds per step as the one-step parity tests (FP64 1e-12;
FP32 2e-7 in ghat and 2e-6 of the scalar ranges), times the number of steps; FP16 storage
is compared after one step (its output rounding is half an FP16 ulp)."""
import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import step as OS
from tests.gpu_helpers import SCAL_NP, STORE_NP

pytestmark = pytest.mark.gpu


def _gpu_run(params, P, u, scal, mask, steps):
    from paper_2207_11567_amd import Solver
    s = Solver(params)
    if mask is not None and mask.dtype == np.float64:
        s.set_wall_distance(torch.from_numpy(mask))         # signed wall distance
    elif mask is not None:
        s.set_geometry(torch.from_numpy(mask))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u),
                  torch.from_numpy(scal) if scal is not None else None)
    s.step(steps)
    p1, s1, _ = s.get_state()
    out = [t.double().cpu().numpy() for t in (p1, s1)]
    s.close()
    return out + [P, u, scal, steps]


def _window(params, full, mask, origin, size, state=None):
    """Oracle run of a window from the workload's fields (or, with state = (ghat, scal), from
    that stored host state); returns the largest GPU-vs-oracle differences."""
    p1, s1, P, u, scal, steps = full
    HALO = 3 * steps
    dims = [params["nx"], params["ny"], params["nz"]]
    faces = params["face_bc"]
    D = 2 if params["lattice"] == "D2Q9" else 3
    idx, wf, keep = [], [], []
    for d in range(3):
        if d >= D:
            idx.append(np.arange(1)); wf += ["periodic", "periodic"]; keep.append(np.ones(1, bool))
            continue
        lo, hi, n = origin[d], origin[d] + size[d], dims[d]
        real_lo = lo == 0 and faces[2 * d] != "periodic"
        real_hi = hi == n and faces[2 * d + 1] != "periodic"
        a = lo if real_lo else lo - HALO
        b = hi if real_hi else hi + HALO
        ix = np.arange(a, b)
        if faces[2 * d] == "periodic":
            ix = ix % n
        assert ix.min() >= 0 and ix.max() < n
        idx.append(ix)
        if b - a == n and faces[2 * d] == "periodic":
            wf += ["periodic", "periodic"]
            k = np.ones(b - a, bool)
        else:
            flo = faces[2 * d] if real_lo else ("outlet" if faces[2 * d] == "periodic" else "wall")
            fhi = faces[2 * d + 1] if real_hi else ("outlet" if faces[2 * d] == "periodic" else "wall")
            wf += [flo, fhi]
            k = np.ones(b - a, bool)
            if not real_lo:
                k[:HALO] = False
            if not real_hi:
                k[-HALO:] = False
        keep.append(k)
    sel = np.ix_(idx[2], idx[1], idx[0])
    wp = dict(params, nx=len(idx[0]), ny=len(idx[1]), nz=len(idx[2]), face_bc=wf,
              noise_origin=(int(idx[0][0]), int(idx[1][0]), int(idx[2][0])))
    phi = None
    if mask is not None and mask.dtype == np.float64:
        phi = torch.from_numpy(np.ascontiguousarray(mask[sel]))
        mask = mask < 0
    solid = None if mask is None else torch.from_numpy(mask[sel].astype(bool))
    # the window's inputs: equilibrium from the FP64 fields, then stored (scalars and
    # populations rounded to the storage precision as the GPU stores them)
    sc_w = None if scal is None else np.ascontiguousarray(scal[(slice(None),) + sel])
    if state is not None:
        gh, sc = state
        shape = (len(idx[2]), len(idx[1]), len(idx[0]))
        st = {"pops": OS.from_storage(wp, torch.from_numpy(np.ascontiguousarray(gh[(slice(None),) + sel]).astype(np.float64))),
              "scal": (torch.zeros((0,) + shape, dtype=torch.float64) if sc is None else
                       torch.from_numpy(np.ascontiguousarray(sc[(slice(None),) + sel]).astype(np.float64))),
              "step": 0, "solid": torch.zeros(shape, dtype=torch.bool) if solid is None else solid}
    else:
        st = OS.init_state(wp, torch.from_numpy(np.ascontiguousarray(P[sel])),
                           torch.from_numpy(np.ascontiguousarray(u[(slice(None),) + sel])),
                           None if sc_w is None else torch.from_numpy(sc_w), solid, phi)
    if sc_w is not None and state is None:
        st["scal"] = torch.from_numpy(sc_w.astype(SCAL_NP[params["precision"]]).astype(np.float64))
    if params["precision"] != "fp64" and state is None:
        # populations enter storage once at initialisation, rounded once (numpy converts
        # FP64 to FP16 in one rounding, as the device does; a detour through FP32 would not)
        gh = OS.to_storage(wp, st["pops"]).numpy().astype(STORE_NP[params["precision"]])
        st["pops"] = OS.from_storage(wp, torch.from_numpy(gh.astype(np.float64)))
    out = st
    for _ in range(steps):
        out, _ = OS.step(wp, out)
    kk = np.ix_(keep[2], keep[1], keep[0])
    fl = np.ones(out["solid"].shape, bool) if solid is None else ~solid.numpy()
    fl = fl[kk]
    og = OS.to_storage(wp, out["pops"]).numpy()[(slice(None),) + kk]
    gg = p1[(slice(None),) + sel][(slice(None),) + kk]
    dpop = np.abs(og - gg)[:, fl]
    beyond = dpop - 2.0 ** -11 * np.abs(og[:, fl]) - 2.0 ** -25
    w = np.unravel_index(int(np.argmax(beyond)), beyond.shape)
    res = {"pop_abs": float(dpop.max()), "pop_beyond_half_fp16_ulp": float(beyond.max()),
           "cells": int(fl.sum()),
           "worst": {"i": int(w[0]), "oracle": float(og[:, fl][w]), "gpu": float(gg[:, fl][w])}}
    if s1.shape[0]:
        os_ = out["scal"].numpy()[(slice(None),) + kk]
        gs = s1[(slice(None),) + sel][(slice(None),) + kk]
        scale = np.maximum(np.array(params["weno_scale"][:s1.shape[0]]).reshape(-1, 1), np.abs(os_[:, fl]))
        res["scal_rel"] = float((np.abs(gs - os_)[:, fl] / scale).max())
    return res


def _developed(params, P, u, scal, seed, amp=2e-3):
    """A developed, non-equilibrium stored state built on the host from the workload's
    fields: the oracle's equilibrium (Eq. 6) plus a seeded random deviation, populations
    rounded to the storage precision, scalars to theirs."""
    st = OS.init_state(params, torch.from_numpy(P), torch.from_numpy(u),
                       None if scal is None else torch.from_numpy(scal))
    gh = OS.to_storage(params, st["pops"]).numpy()
    del st
    Q = gh.shape[0]
    for i in range(Q):        # one population at a time keeps the host memory bounded
        gh[i] += L.random_deviation(1, gh.shape[1:], seed + i, amp)[0]
    gh = gh.astype(STORE_NP[params["precision"]])
    sc = None if scal is None else scal.astype(SCAL_NP[params["precision"]])
    return gh, sc


def _gpu_run_from(params, state, steps):
    from paper_2207_11567_amd import Solver
    gh, sc = state
    s = Solver(params)
    s.set_state(torch.from_numpy(gh), None if sc is None else torch.from_numpy(sc), 0)
    s.step(steps)
    p1, s1, k = s.get_state()
    assert k == steps
    out = [t.double().cpu().numpy() for t in (p1, s1)]
    s.close()
    return out + [None, None, None, steps]


def _check(res, prec, steps):
    if prec == "fp64":
        assert res["pop_abs"] <= 1e-12 * steps, res
        assert res.get("scal_rel", 0.0) <= 1e-12 * steps, res
    else:
        assert res.get("scal_rel", 0.0) <= 2e-6 * steps, res
        if prec == "fp32":
            assert res["pop_abs"] <= 2e-7 * steps, res


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flame2d_full_size_windows(prec):
    params, P, u, scal, mask = L.flame2d()
    params["precision"] = prec
    full = _gpu_run(params, P, u, scal, mask, 2)
    for origin, size in (((0, 108, 0), (40, 40, 1)),        # ignition at the closed end
                         ((150, 0, 0), (120, 64, 1)),       # first obstacle, bottom wall
                         ((960, 200, 0), (64, 56, 1))):     # outlet and top wall corner
        _check(_window(params, full, mask, origin, size), prec, 2)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_hit_256_windows(prec):
    params, P, u = L.hit(256)
    params["precision"] = prec
    full = _gpu_run(params, P, u, None, None, 1)
    for origin in ((0, 0, 0), (120, 37, 250), (249, 128, 64)):
        res = _window(params, full, None, origin, (10, 10, 10))
        if prec == "fp16s":
            # output rounded to half precision: half an FP16 ulp (subnormal floor 2^-25)
            # plus the FP32 rounding bound
            assert res["pop_beyond_half_fp16_ulp"] <= 2e-7, res
        else:
            _check(res, prec, 1)


def test_reacting_box_full_size_windows():
    params, P, u, scal = L.reacting_box()
    full = _gpu_run(params, P, u, scal, None, 2)
    for origin, size in (((50, 60, 0), (12, 12, 10)),         # inlet face
                         ((90, 100, 184), (12, 12, 16)),      # flame front
                         ((180, 3, 374), (12, 12, 10))):      # outlet face
        res = _window(params, full, None, origin, size)
        _check(res, "fp32", 2)


def test_chamber_open_full_size_windows():
    """The 2500x500 chamber geometry with constant thermodynamic pressure (its step runs
    split: interior instance and the listed wall and baffle cells)."""
    params, P, u, scal, mask = L.chamber2d(closed=False)
    full = _gpu_run(params, P, u, scal, mask.astype(np.uint8), 2)
    for origin, size in (((0, 220, 0), (40, 60, 1)),         # burnt kernel at the left wall
                         ((180, 190, 0), (60, 120, 1)),     # first baffle row
                         ((2440, 440, 0), (60, 60, 1))):    # right wall, top corner
        _check(_window(params, full, mask.astype(np.uint8), origin, size), "fp64", 2)


def test_reacting_box_fp16_storage_full_size_windows():
    """The reacting box with FP16 population storage (split step: the interior instance at
    four waves per SIMD and the boundary list), one step: half an FP16 ulp of each output
    plus the FP32 bounds."""
    params, P, u, scal = L.reacting_box()
    params["precision"] = "fp16s"
    full = _gpu_run(params, P, u, scal, None, 1)
    for origin, size in (((50, 60, 0), (12, 12, 10)), ((90, 100, 184), (12, 12, 16)),
                         ((180, 3, 374), (12, 12, 10))):
        res = _window(params, full, None, origin, size)
        assert res["pop_beyond_half_fp16_ulp"] <= 2e-7, res
        assert res["scal_rel"] <= 2e-6, res


def test_reacting_box_fp64_full_size_windows():
    """The reacting box in FP64: on this size the step runs split into the interior
    instance and the list instance over the inlet and outlet planes."""
    params, P, u, scal = L.reacting_box()
    params["precision"] = "fp64"
    full = _gpu_run(params, P, u, scal, None, 2)
    for origin, size in (((50, 60, 0), (12, 12, 10)), ((90, 100, 184), (12, 12, 16)),
                         ((180, 3, 374), (12, 12, 10))):
        _check(_window(params, full, None, origin, size), "fp64", 2)


def test_reacting_box_mixture_transport_full_size_windows():
    """The reacting box with mixture-averaged transport (FULL kernel instance)."""
    params, P, u, scal = L.reacting_box()
    params.update(transport_model="mixture", transport=L.mixture_transport(params["nu_ref"]))
    full = _gpu_run(params, P, u, scal, None, 2)
    for origin, size in (((50, 60, 0), (12, 12, 10)), ((90, 100, 184), (12, 12, 16))):
        _check(_window(params, full, None, origin, size), "fp32", 2)


def test_reacting_box_cone_curved_walls_full_size_windows():
    """The reacting box with a conical bluff body given by its signed distance (curved
    walls, FULL kernel instance): windows at the cone's base edge and its apex."""
    params, P, u, scal = L.reacting_box()
    phi = L.cone_levelset(params["nx"], params["ny"], params["nz"])
    full = _gpu_run(params, P, u, scal, phi, 2)
    for origin, size in (((52, 90, 12), (14, 12, 10)),        # base rim
                         ((90, 90, 70), (12, 12, 12))):       # apex
        _check(_window(params, full, phi, origin, size), "fp32", 2)


@pytest.mark.parametrize("phys,prec,n,reps", [
    ("isothermal", "fp64", (96, 96, 96), (2, 2, 2)),
    ("isothermal", "fp32", (96, 96, 96), (2, 2, 2)),
    ("isothermal", "fp16s", (96, 96, 96), (2, 2, 2)),
    ("two_step", "fp32", (128, 128, 128), (1, 2, 2))])
def test_large_grid_instances_match_a_tiled_small_grid(phys, prec, n, reps):
    """A periodic box tiled along its axes evolves exactly as the box itself: every output
    of a cell depends only on its neighbours, which hold the same values in both grids.
    The tiled grid's population copy exceeds 256 MB, so it runs the cached-pull instance,
    the box the streaming one, each with its own tile order; both run the same kernel
    otherwise (with two-step scalars both grids are large enough for the split step's
    interior instance), so after three steps they must agree bit for bit."""
    from tests.gpu_helpers import fetch, gpu_state, make_solver, random_state
    from tests.test_gpu_parity import _params
    steps = 3
    small = _params("D3Q27", n, phys, "cumulant", precision=prec, omega_high=1.0)
    big = dict(small, nz=reps[0] * n[0], ny=reps[1] * n[1], nx=reps[2] * n[2])
    ghat, scal = random_state(small, 23)
    out = []
    for params, r in ((small, (1, 1, 1, 1)), (big, (1,) + reps)):
        print(f"tiled-box case: {phys} {prec} {params['nz']}x{params['ny']}x{params['nx']}", flush=True)
        s = make_solver(params)
        gpu_state(s, np.tile(ghat, r), np.tile(scal, r))
        s.step(steps)
        out.append(fetch(s))
        s.close()
    (p0, s0, k0), (p1, s1, k1) = out
    assert k0 == k1 == steps
    assert np.array_equal(np.tile(p0, (1,) + reps), p1)
    assert np.array_equal(np.tile(s0, (1,) + reps), s1)


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_hit_256_developed_state_windows(prec):
    """One step of the full 256^3 HIT grid (cached-pull instance) from a developed state
    (equilibrium of the workload's field plus a seeded non-equilibrium part), against the
    oracle on windows of that same stored state."""
    params, P, u = L.hit(256)
    params["precision"] = prec
    state = _developed(params, P, u, None, 9100)
    print(f"developed HIT 256^3 {prec}: state built", flush=True)
    full = _gpu_run_from(params, state, 1)
    for origin in ((0, 0, 0), (120, 37, 250), (249, 128, 64)):
        res = _window(params, full, None, origin, (10, 10, 10), state=state)
        print(prec, origin, res, flush=True)
        if prec == "fp16s":
            assert res["pop_beyond_half_fp16_ulp"] <= 2e-7, res
        else:
            _check(res, prec, 1)


def test_reacting_box_fp16_storage_developed_state_windows():
    """The reacting box in FP16 storage (split step) from a developed stored state."""
    params, P, u, scal = L.reacting_box()
    params["precision"] = "fp16s"
    state = _developed(params, P, u, scal, 9200)
    print("developed reacting box fp16s: state built", flush=True)
    full = _gpu_run_from(params, state, 1)
    for origin, size in (((50, 60, 0), (12, 12, 10)), ((90, 100, 184), (12, 12, 16)),
                         ((180, 3, 374), (12, 12, 10))):
        res = _window(params, full, None, origin, size, state=state)
        print("reacting fp16s", origin, res, flush=True)
        assert res["pop_beyond_half_fp16_ulp"] <= 2e-7, res
        assert res["scal_rel"] <= 2e-6, res
