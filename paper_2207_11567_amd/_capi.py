"""ctypes binding of include/lbm.h: the same entry-point names, argument marshalling only.

Loads liblbm.so built in-tree next to this file.  There is no fallback: if the library is
missing, importing the binding raises."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

c_int32, c_double, c_uint64, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                                    ctypes.c_void_p, ctypes.c_size_t)

LBM_OK, LBM_E_INVALID, LBM_E_UNSUPPORTED, LBM_E_HIP, LBM_E_DIVERGED, LBM_E_STATE = 0, -1, -2, -3, -4, -5
LATTICE = {"D2Q9": 9, "D3Q27": 27}
PRECISION = {"fp64": 0, "fp32": 1, "fp16s": 2}
COLLISION = {"cumulant": 0, "bgk": 1}
PHYSICS = {"isothermal": 0, "passive": 1, "one_step": 2, "two_step": 3}
VISC = {"const_nu": 0, "const_mu": 1}
FACE = {"periodic": 0, "wall": 1, "inlet": 2, "outlet": 3}
PTH = {"open": 0, "closed": 1}
TRANSPORT = {"simple": 0, "mixture": 1}
N_SCALARS = {"isothermal": 0, "passive": 1, "one_step": 2, "two_step": 6}


class LbmParams(ctypes.Structure):
    _fields_ = [("lattice", c_int32), ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("precision", c_int32), ("collision", c_int32), ("physics", c_int32),
                ("visc_law", c_int32),
                ("nu_ref", c_double), ("omega_bulk", c_double), ("omega_high", c_double),
                ("cs_smag", c_double), ("prandtl", c_double), ("thickening", c_double),
                ("rho_ref", c_double), ("T_ref", c_double),
                ("face_bc", c_int32 * 6), ("inlet_u", c_double * 3), ("inlet_noise", c_double),
                ("outlet_P", c_double), ("inlet_T", c_double), ("inlet_Y", c_double * 8),
                ("weno_scale", c_double * 8), ("chem", c_double * 32), ("seed", c_uint64),
                ("pth_mode", c_int32), ("gamma", c_double),
                ("transport_model", c_int32), ("transport", c_double * 32),
                ("galilean", c_int32), ("fourth_order", c_int32)]


def make_params(d):
    """lbm_params from a plain dict (the workload description used throughout tests)."""
    p = LbmParams()
    p.lattice = LATTICE[d["lattice"]]
    p.nx, p.ny, p.nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
    p.precision = PRECISION[d["precision"]]
    p.collision = COLLISION[d["collision"]]
    p.physics = PHYSICS[d["physics"]]
    p.visc_law = VISC[d["visc_law"]]
    for k in ("nu_ref", "omega_bulk", "omega_high", "cs_smag", "prandtl", "thickening",
              "rho_ref", "T_ref", "inlet_noise", "outlet_P", "inlet_T"):
        setattr(p, k, float(d[k]))
    for i, f in enumerate(d["face_bc"]):
        p.face_bc[i] = FACE[f]
    for i, v in enumerate(d["inlet_u"][:3]):
        p.inlet_u[i] = float(v)
    for i, v in enumerate(list(d["inlet_Y"])[:8]):
        p.inlet_Y[i] = float(v)
    for i, v in enumerate(list(d["weno_scale"])[:8]):
        p.weno_scale[i] = float(v)
    for i, v in enumerate(list(d["chem"])[:32]):
        p.chem[i] = float(v)
    p.seed = int(d["seed"]) & 0xFFFFFFFFFFFFFFFF
    p.pth_mode = PTH[d.get("pth_mode", "open")]
    p.gamma = float(d.get("gamma", 1.4))
    p.transport_model = TRANSPORT[d.get("transport_model", "simple")]
    for i, v in enumerate(list(d.get("transport", [0.0] * 32))[:32]):
        p.transport[i] = float(v)
    p.galilean = int(d.get("galilean", 0))
    p.fourth_order = int(d.get("fourth_order", 0))
    return p


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                           "(python -m paper_2207_11567_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "lbm_query_sizes": [P(LbmParams), P(c_size_t), P(c_size_t), P(c_size_t)],
        "lbm_create": [P(LbmParams), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                       P(c_void_p)],
        "lbm_set_geometry": [c_void_p, c_void_p],
        "lbm_set_wall_distance": [c_void_p, c_void_p],
        "lbm_init_fields": [c_void_p, c_void_p, c_void_p, c_void_p],
        "lbm_step": [c_void_p, c_int32],
        "lbm_fields": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, P(c_double)],
        "lbm_step_sums": [c_void_p, P(c_double)],
        "lbm_step_from": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_int64],
        "lbm_get_state": [c_void_p, c_void_p, c_void_p, P(ctypes.c_int64)],
        "lbm_set_state": [c_void_p, c_void_p, c_void_p, ctypes.c_int64],
        "lbm_adjoint_sizes": [c_void_p, P(c_size_t), P(c_size_t), P(c_size_t)],
        "lbm_adjoint_step": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p],
        "lbm_objective": [c_void_p, c_void_p, c_void_p, P(c_double), c_void_p, c_void_p],
        "lbm_init_adjoint": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
        "lbm_get_thermo_pressure": [c_void_p, P(c_double)],
        "lbm_set_statistics": [c_void_p, c_void_p, c_int32],
        "lbm_statistics": [c_void_p, c_void_p, c_void_p, P(ctypes.c_int64)],
        "lbm_set_probes": [c_void_p, P(ctypes.c_int64), c_int32, c_void_p, ctypes.c_int64],
        "lbm_probe_rows": [c_void_p, P(ctypes.c_int64)],
        "lbm_flame_surface": [c_void_p, c_double, c_double, P(c_double)],
        "lbm_flame_surface_noalloc": [c_void_p, c_double, c_double, c_void_p],
        "lbm_set_thermo_pressure": [c_void_p, P(c_double)],
        "lbm_copy_probe": [c_void_p, c_void_p, ctypes.c_size_t, c_int32, c_void_p],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c_int32
    lib.lbm_last_error.argtypes = [c_void_p]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_destroy.argtypes = [c_void_p]
    lib.lbm_destroy.restype = None
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


def check(status, handle=None):
    if status != LBM_OK:
        msg = lib().lbm_last_error(handle)
        raise LbmError(status, msg.decode() if msg else "")
