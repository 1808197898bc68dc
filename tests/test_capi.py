"""CPU tests of the C ABI: the library loads, exports every entry point that
include/lbm.h declares, and rejects invalid parameters in its host-side validation
(no GPU needed: no call here reaches the device)."""
import ctypes
import os
import re

import pytest

import lbm_inputs as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2207_11567_amd import _capi as C
    if not os.path.exists(C.LIB_PATH):
        from paper_2207_11567_amd import build
        build.build(verbose=False)
    return C, C.lib()


def test_exports_every_declared_symbol():
    C, lib = _lib()
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    names = set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src))
    assert len(names) >= 15
    for name in sorted(names):
        assert hasattr(lib, name), name


@pytest.mark.parametrize("change,needle", [
    ({"nu_ref": 0.0}, "nu_ref"),
    ({"nz": 4}, "D2Q9"),
    ({"omega_bulk": 2.5}, "omega_bulk"),
    ({"face_bc": ["periodic", "wall", "periodic", "periodic", "periodic", "periodic"]}, "pairs"),
    ({"physics": "passive", "nu_ref": 0.4}, "unstable"),
    ({"pth_mode": "closed", "face_bc": ["inlet", "outlet", "wall", "wall", "periodic", "periodic"]},
     "closed domain"),
    ({"pth_mode": "closed", "gamma": 1.0}, "gamma"),
    ({"galilean": 2}, "galilean"),
    ({"lattice": "D3Q27", "nx": 1024, "ny": 1024, "nz": 100}, "too large"),
    ({"nx": 0}, ">= 1"),
    ({"galilean": 1, "collision": "bgk"}, "cumulant"),
    ({"fourth_order": 1}, "D3Q27"),
    ({"fourth_order": 1, "lattice": "D3Q27", "nz": 4, "nu_ref": 1.0 / 18.0}, "stable range"),
    ({"fourth_order": 1, "lattice": "D3Q27", "nz": 4, "nu_ref": 1.0 / 6.0, "omega_bulk": 1.0}, "stable range"),
])
def test_validation_rejects(change, needle):
    C, lib = _lib()
    p = L.base_params("D2Q9", 16, 8, 1)
    p.update(change)
    sz = C.c_size_t()
    st = lib.lbm_query_sizes(ctypes.byref(C.make_params(p)), ctypes.byref(sz), None, None)
    assert st == C.LBM_E_INVALID
    assert needle in lib.lbm_last_error(None).decode()


def test_sizes_of_valid_parameters():
    C, lib = _lib()
    p, _, _, _ = L.reacting_box(16, 16, 32)
    pb, sb, wb = C.c_size_t(), C.c_size_t(), C.c_size_t()
    assert lib.lbm_query_sizes(ctypes.byref(C.make_params(p)), ctypes.byref(pb), ctypes.byref(sb),
                               ctypes.byref(wb)) == C.LBM_OK
    N = 16 * 16 * 32
    assert pb.value == 27 * N * 4 and sb.value == 6 * N * 4
    assert wb.value >= N * 8 + (N // 256) * 72


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback: without the built HIP library the binding raises instead of running
    anything else."""
    from paper_2207_11567_amd import _capi as C
    monkeypatch.setattr(C, "LIB_PATH", os.path.join(ROOT, "_no_such_dir", "liblbm.so"))
    with pytest.raises(RuntimeError, match="not built"):
        C._load()


def test_hot_gas_diffusion_limit_warns():
    """rho nu constant: the kinematic viscosity grows as rho_ref/rho, so F nu/Pr is checked
    at the one-step model's adiabatic temperature too; beyond the limit the call succeeds
    and leaves a warning."""
    C, lib = _lib()
    p = L.base_params("D2Q9", 16, 8, 1, physics="one_step", visc_law="const_mu", nu_ref=0.02,
                      thickening=4.0, chem=[4.0, 15000.0, 300.0, 2000.0, 1.0], T_ref=300.0)
    assert lib.lbm_query_sizes(ctypes.byref(C.make_params(p)), None, None, None) == C.LBM_OK
    assert lib.lbm_last_error(None).decode().startswith("warning: explicit diffusion unstable in the hottest gas")
    p["nu_ref"] = 0.002
    assert lib.lbm_query_sizes(ctypes.byref(C.make_params(p)), None, None, None) == C.LBM_OK
    assert lib.lbm_last_error(None).decode() == ""


def test_copy_probe_rejects_bad_arguments():
    """Host-side checks of lbm_copy_probe (no copy is launched): size, mode, null and
    overlapping pointers."""
    C, lib = _lib()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
    for src, dst, nbytes, mode in [(a, b, 6, 0), (a, b, 0, 0), (a, b, (1 << 31) + 4, 0), (a, b, 64, 4),
                                   (a, b, 64, -1), (None, b, 64, 0), (a, None, 64, 0),
                                   (a, ctypes.c_void_p((1 << 20) + 32), 64, 0)]:
        assert lib.lbm_copy_probe(src, dst, nbytes, mode, None) == C.LBM_E_INVALID
        assert lib.lbm_last_error(None).decode().startswith("lbm_copy_probe:")
