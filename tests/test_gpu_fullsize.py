"""Parity at the workloads' full sizes, in the launch configuration bench.py times: the
GPU advances the full grid one step from a developed state; the oracle recomputes sampled
windows of that step (window + 3-cell halo cut from the same input state, faces that the
window does not share with the domain treated as fake and excluded with their 3-cell
neighbourhood: every output of a cell depends on inputs at most 2 cells away)."""
import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import step as OS
from tests.gpu_helpers import SCAL_NP, STORE_NP

pytestmark = pytest.mark.gpu
HALO = 3


def _gpu_step(params, P, u, scal, mask, warm):
    from paper_2207_11567_amd import Solver
    s = Solver(params)
    if mask is not None:
        s.set_geometry(torch.from_numpy(mask))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u),
                  torch.from_numpy(scal) if scal is not None else None)
    s.step(warm)
    p0, s0, n0 = s.get_state()
    s.step(1)
    p1, s1, _ = s.get_state()
    out = [t.double().cpu().numpy() for t in (p0, s0, p1, s1)]
    s.close()
    return out + [n0]


def _window(params, full, mask, origin, size):
    """Oracle one-step on a window; returns (gpu-vs-oracle max errors)."""
    p0, s0, p1, s1, n0 = full
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
    solid = None if mask is None else torch.from_numpy(mask[sel].astype(bool))
    st = {"pops": OS.from_storage(wp, torch.from_numpy(p0[(slice(None),) + sel])),
          "scal": torch.from_numpy(s0[(slice(None),) + sel]), "step": n0,
          "solid": solid if solid is not None else torch.zeros((len(idx[2]), len(idx[1]), len(idx[0])), dtype=torch.bool)}
    out, _ = OS.step(wp, st)
    kk = np.ix_(keep[2], keep[1], keep[0])
    fl = np.ones(st["solid"].shape, bool) if solid is None else ~solid.numpy()
    fl = fl[kk]
    og = OS.to_storage(wp, out["pops"]).numpy()[(slice(None),) + kk]
    gg = p1[(slice(None),) + sel][(slice(None),) + kk]
    dpop = np.abs(og - gg)[:, fl]
    res = {"pop_abs": float(dpop.max()),
           "pop_beyond_half_fp16_ulp": float((dpop - 2.0 ** -11 * np.abs(og[:, fl]) - 2.0 ** -25).max()),
           "cells": int(fl.sum())}
    if s0.shape[0]:
        os_ = out["scal"].numpy()[(slice(None),) + kk]
        gs = s1[(slice(None),) + sel][(slice(None),) + kk]
        scale = np.maximum(np.array(params["weno_scale"][:s0.shape[0]]).reshape(-1, 1), np.abs(os_[:, fl]))
        res["scal_rel"] = float((np.abs(gs - os_)[:, fl] / scale).max())
    return res


def _check(res, prec):
    if prec == "fp64":
        assert res["pop_abs"] <= 1e-12, res
        assert res.get("scal_rel", 0.0) <= 1e-12, res
    else:
        assert res.get("scal_rel", 0.0) <= 2e-6, res
        if prec == "fp32":
            assert res["pop_abs"] <= 2e-7, res


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_flame2d_full_size_windows(prec):
    params, P, u, scal, mask = L.flame2d()
    params["precision"] = prec
    full = _gpu_step(params, P, u, scal, mask, warm=20)
    for origin, size in (((0, 108, 0), (40, 40, 1)),        # ignition at the closed end
                         ((150, 0, 0), (120, 64, 1)),       # first obstacle, bottom wall
                         ((960, 200, 0), (64, 56, 1))):     # outlet and top wall corner
        _check(_window(params, full, mask, origin, size), prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_hit_256_windows(prec):
    params, P, u = L.hit(256)
    params["precision"] = prec
    full = _gpu_step(params, P, u, None, None, warm=5)
    for origin in ((0, 0, 0), (120, 37, 250), (249, 128, 64)):
        res = _window(params, full, None, origin, (10, 10, 10))
        if prec == "fp16s":
            # output rounded to half precision: half an FP16 ulp (subnormal floor 2^-25)
            # plus the FP32 rounding bound
            assert res["pop_beyond_half_fp16_ulp"] <= 2e-7, res
        else:
            _check(res, prec)


def test_reacting_box_full_size_windows():
    params, P, u, scal = L.reacting_box()
    full = _gpu_step(params, P, u, scal, None, warm=10)
    for origin, size in (((50, 60, 0), (12, 12, 10)),         # inlet face
                         ((90, 100, 184), (12, 12, 16)),      # flame front
                         ((180, 3, 374), (12, 12, 10))):      # outlet face
        res = _window(params, full, None, origin, size)
        _check(res, "fp32")
