"""Shared helpers for the GPU parity tests: build the same seeded state on both sides,
advance the HIP library and the oracle, and compare."""
import numpy as np
import torch

import lbm_inputs as L
from oracle import step as OS

STORE_NP = {"fp64": np.float64, "fp32": np.float32, "fp16s": np.float16}
SCAL_NP = {"fp64": np.float64, "fp32": np.float32, "fp16s": np.float32}


def make_solver(params):
    from paper_2207_11567_amd import Solver
    return Solver(params)


def random_state(params, seed, amp=0.01, solid=None):
    """(ghat, scal) rounded to the storage precisions, as float64 numpy arrays."""
    Q = 9 if params["lattice"] == "D2Q9" else 27
    shape = (params["nz"], params["ny"], params["nx"])
    ghat = L.random_deviation(Q, shape, seed, amp).astype(STORE_NP[params["precision"]])
    kind = params["physics"]
    if kind == "isothermal":
        scal = np.zeros((0,) + shape)
    else:
        scal = L.random_scalars(kind, shape, seed + 1)
    scal = scal.astype(SCAL_NP[params["precision"]])
    return ghat.astype(np.float64), scal.astype(np.float64)


def oracle_state(params, ghat, scal, solid=None, step=0):
    shape = (params["nz"], params["ny"], params["nx"])
    sol = torch.zeros(shape, dtype=torch.bool) if solid is None else torch.as_tensor(solid).bool()
    return {"pops": OS.from_storage(params, torch.from_numpy(ghat)),
            "scal": torch.from_numpy(scal), "step": step, "solid": sol}


def gpu_state(solver, ghat, scal, step=0):
    solver.set_state(torch.from_numpy(ghat), torch.from_numpy(scal) if scal.shape[0] else None, step)


def fetch(solver):
    pops, scal, step = solver.get_state()
    return pops.double().cpu().numpy(), scal.double().cpu().numpy(), step


def oracle_ghat(params, st):
    return OS.to_storage(params, st["pops"]).numpy()
