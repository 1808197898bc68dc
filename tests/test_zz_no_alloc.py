"""The allocation-free flame surface (lbm_flame_surface_noalloc) against the existing
entry point lbm_flame_surface, through the C ABI: bit for bit the same sum, on two calls
in a row (the second on a smaller grid, so that records of the first call are left in the
shared scratch), and sizes beyond the scratch maximum rejected with LBM_E_INVALID."""
import ctypes

import numpy as np
import pytest
import torch

import lbm_inputs as L

pytestmark = pytest.mark.gpu


def _solver(nx, ny, steps):
    from paper_2207_11567_amd import Solver
    params, P, u, scal, mask = L.flame2d(nx=nx, ny=ny)
    s = Solver(params, device="cuda:0")
    s.set_geometry(torch.from_numpy(mask))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    s.step(steps)
    return s, params


def _both(s, params):
    from paper_2207_11567_amd import _capi as C
    T_u, T_b = params["chem"][2], params["chem"][3]
    ref = ctypes.c_double()
    C.check(C.lib().lbm_flame_surface(s._h, T_u, T_b, ctypes.byref(ref)), s._h)
    out = torch.full((1,), float("nan"), dtype=torch.float64, device=s.device)
    C.check(C.lib().lbm_flame_surface_noalloc(s._h, T_u, T_b, ctypes.c_void_p(out.data_ptr())), s._h)
    torch.cuda.synchronize()
    return ref.value, float(out.item())


def test_noalloc_flame_surface_matches_the_existing_entry_point():
    first, p1 = _solver(512, 128, 20)            # 256 blocks of records
    second, p2 = _solver(96, 32, 5)              # 12 blocks: fewer than the first call left
    a_ref, a = _both(first, p1)
    b_ref, b = _both(second, p2)
    print(f"no-alloc flame surface: {a!r} vs {a_ref!r}; {b!r} vs {b_ref!r}", flush=True)
    assert a > 0 and b > 0 and a != b
    assert a == a_ref and b == b_ref
    # the first solver again, after the second one's call
    a2_ref, a2 = _both(first, p1)
    assert a2 == a_ref and a2_ref == a_ref
    first.close()
    second.close()


def test_noalloc_flame_surface_rejects_grids_beyond_the_scratch():
    from paper_2207_11567_amd import Solver
    from paper_2207_11567_amd import _capi as C
    params = L.base_params("D2Q9", 8192, 4097, 1, physics="one_step", precision="fp16s",
                           chem=list(L.ONE_STEP_CHEM), weno_scale=[1700.0, 1.0])
    s = Solver(params, device="cuda:0")            # 33,562,624 cells: 131,104 blocks
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    st = C.lib().lbm_flame_surface_noalloc(s._h, 300.0, 2000.0, ctypes.c_void_p(out.data_ptr()))
    assert st == C.LBM_E_INVALID
    assert "scratch maximum" in C.lib().lbm_last_error(s._h).decode()
    s.close()
    del s
    torch.cuda.empty_cache()
