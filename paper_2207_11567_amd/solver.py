"""Python face of the HIP library: torch supplies device memory and the stream; every
step of the time-step path runs in the library's kernels (include/lbm.h)."""
import ctypes

import torch

from . import _capi as C

STORAGE_DTYPE = {"fp64": torch.float64, "fp32": torch.float32, "fp16s": torch.float16}
SCALAR_DTYPE = {"fp64": torch.float64, "fp32": torch.float32, "fp16s": torch.float32}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def copy_probe(src, dst, mode, stream=None):
    """lbm_copy_probe: copy the bytes of contiguous device tensor src into dst with the step
    kernel's raw buffer loads (mode bit 0: streaming) and stores (bit 1: streaming), on
    `stream` (torch's current stream by default); measurement support."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("copy_probe: contiguous device tensors are required")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy_probe: source and destination sizes differ")
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    lib = C.lib()
    status = lib.lbm_copy_probe(_ptr(src), _ptr(dst), nbytes, int(mode), ctypes.c_void_p(st.cuda_stream))
    if status != 0:
        raise C.LbmError(status, lib.lbm_last_error(None).decode())


class Solver:
    """One lattice (D2Q9 or D3Q27) with its A/B population and scalar buffers on a GPU."""

    def __init__(self, params, device="cuda", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU; none is visible")
        self.params = dict(params)
        self.device = torch.device(device)
        self._p = C.make_params(self.params)
        lib = C.lib()
        pb, sb, wb = C.c_size_t(), C.c_size_t(), C.c_size_t()
        C.check(lib.lbm_query_sizes(ctypes.byref(self._p), ctypes.byref(pb), ctypes.byref(sb),
                                    ctypes.byref(wb)))
        self.Q = C.LATTICE[self.params["lattice"]]
        self.D = 2 if self.Q == 9 else 3
        self.NS = C.N_SCALARS[self.params["physics"]]
        self.shape = (self.params["nz"], self.params["ny"], self.params["nx"])
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        prec = self.params["precision"]
        self.pop_dtype = STORAGE_DTYPE[prec]
        self.scal_dtype = SCALAR_DTYPE[prec]
        dev = self.device
        with torch.cuda.device(dev):
            self.pop = [torch.empty(pb.value, dtype=torch.uint8, device=dev) for _ in range(2)]
            self.scal = [torch.empty(max(sb.value, 1), dtype=torch.uint8, device=dev) for _ in range(2)]
            self.work = torch.zeros(wb.value, dtype=torch.uint8, device=dev)
            self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        C.check(lib.lbm_create(ctypes.byref(self._p), ctypes.c_void_p(self.stream.cuda_stream),
                               _ptr(self.pop[0]), _ptr(self.pop[1]),
                               _ptr(self.scal[0]) if self.NS else None,
                               _ptr(self.scal[1]) if self.NS else None,
                               _ptr(self.work), ctypes.byref(h)))
        self._h = h
        self._mask = None
        msg = lib.lbm_last_error(h)
        if msg and msg.startswith(b"warning:"):
            import warnings
            warnings.warn(msg.decode(), RuntimeWarning, stacklevel=2)

    # ---------------------------------------------------------------- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            C.lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, status):
        C.check(status, self._h)

    def _dev(self, a, dtype=torch.float64):
        t = torch.as_tensor(a, dtype=dtype)
        return t.to(self.device).contiguous()

    # ---------------------------------------------------------------- API
    def set_geometry(self, solid):
        if solid is None:
            self._chk(C.lib().lbm_set_geometry(self._h, None))
            return
        self._mask = self._dev(solid, torch.uint8).reshape(self.shape)
        self._chk(C.lib().lbm_set_geometry(self._h, _ptr(self._mask)))

    def set_wall_distance(self, phi):
        """Curved walls from the signed wall distance at the nodes (solid where < 0); the
        device copy is kept alive by the solver while bound."""
        if phi is None:
            self._phi = None
            self._chk(C.lib().lbm_set_wall_distance(self._h, None))
            return
        self._phi = self._dev(phi, torch.float64).reshape(self.shape).contiguous()
        self._chk(C.lib().lbm_set_wall_distance(self._h, _ptr(self._phi)))

    def init_fields(self, P_h, u, scal=None):
        P = self._dev(P_h).reshape(self.shape)
        U = self._dev(u).reshape((self.D,) + self.shape)
        S = self._dev(scal).reshape((self.NS,) + self.shape) if self.NS else None
        self._chk(C.lib().lbm_init_fields(self._h, _ptr(P), _ptr(U), _ptr(S)))
        torch.cuda.synchronize(self.device)

    def step(self, n=1):
        self._chk(C.lib().lbm_step(self._h, int(n)))

    def fields(self):
        dev = self.device
        P = torch.empty(self.shape, dtype=torch.float64, device=dev)
        rho = torch.empty_like(P)
        u = torch.empty((self.D,) + self.shape, dtype=torch.float64, device=dev)
        S = torch.empty((max(self.NS, 1),) + self.shape, dtype=torch.float64, device=dev)
        sums = (ctypes.c_double * 8)()
        self._chk(C.lib().lbm_fields(self._h, _ptr(P), _ptr(rho), _ptr(u),
                                     _ptr(S) if self.NS else None, sums))
        return {"P_h": P, "rho": rho, "u": u, "scal": S[:self.NS], "sums": list(sums)}

    def step_from(self, state, out, step):
        """One step from state = (pops, scal) into out = (pops, scal)."""
        self._chk(C.lib().lbm_step_from(self._h, _ptr(state[0]), _ptr(state[1]) if self.NS else None,
                                        _ptr(out[0]), _ptr(out[1]) if self.NS else None, int(step)))

    def step_sums(self):
        sums = (ctypes.c_double * 8)()
        self._chk(C.lib().lbm_step_sums(self._h, sums))
        return list(sums)

    def thermo_pressure(self):
        """(pi, q, K): P_th/P_th(0), its logarithmic rate per step, the held mass constant."""
        v = (ctypes.c_double * 3)()
        self._chk(C.lib().lbm_get_thermo_pressure(self._h, v))
        return tuple(v)

    def set_thermo_pressure(self, pqk):
        v = (ctypes.c_double * 3)(*[float(x) for x in pqk])
        self._chk(C.lib().lbm_set_thermo_pressure(self._h, v))

    # ---------------------------------------------------------------- observables
    def set_statistics(self, every=1):
        """Start sampling running statistics every `every` levels (None: stop)."""
        if every is None:
            self._stats = None
            self._chk(C.lib().lbm_set_statistics(self._h, None, 1))
            return
        self._stats = torch.empty(2 * (self.D + 1) * self.N, dtype=torch.float64, device=self.device)
        self._chk(C.lib().lbm_set_statistics(self._h, _ptr(self._stats), int(every)))

    def statistics(self):
        """(mean, rms, samples): mean/rms [D+1, *shape] of (u..., P_h)."""
        mean = torch.empty((self.D + 1,) + self.shape, dtype=torch.float64, device=self.device)
        rms = torch.empty_like(mean)
        k = ctypes.c_int64()
        self._chk(C.lib().lbm_statistics(self._h, _ptr(mean), _ptr(rms), ctypes.byref(k)))
        return mean, rms, k.value

    def set_probes(self, cells, capacity):
        """Record (u..., P_h) at up to 8 cells (linear indices) for `capacity` steps."""
        cells = [int(c) for c in cells]
        self._probe = torch.zeros((capacity, len(cells), self.D + 1), dtype=torch.float64, device=self.device)
        arr = (ctypes.c_int64 * max(len(cells), 1))(*cells)
        self._chk(C.lib().lbm_set_probes(self._h, arr, len(cells), _ptr(self._probe), int(capacity)))

    def probes(self):
        rows = ctypes.c_int64()
        self._chk(C.lib().lbm_probe_rows(self._h, ctypes.byref(rows)))
        torch.cuda.synchronize(self.device)
        return self._probe[:rows.value]

    def flame_surface(self, T_u, T_b):
        v = ctypes.c_double()
        self._chk(C.lib().lbm_flame_surface(self._h, float(T_u), float(T_b), ctypes.byref(v)))
        return v.value

    def flame_surface_noalloc(self, T_u, T_b, out):
        """The flame surface written to `out` (a float64 device tensor of one element) in
        stream order, without allocation or synchronisation."""
        if out.dtype != torch.float64 or out.device != self.device or out.numel() < 1:
            raise ValueError("out must be a float64 tensor on the solver's device")
        self._chk(C.lib().lbm_flame_surface_noalloc(self._h, float(T_u), float(T_b), _ptr(out)))
        return out

    def get_state(self):
        pops = torch.empty((self.Q,) + self.shape, dtype=self.pop_dtype, device=self.device)
        scal = torch.empty((self.NS,) + self.shape, dtype=self.scal_dtype, device=self.device)
        step = ctypes.c_int64()
        self._chk(C.lib().lbm_get_state(self._h, _ptr(pops), _ptr(scal) if self.NS else None,
                                        ctypes.byref(step)))
        return pops, scal, step.value

    # ---------------------------------------------------------------- differentiation
    def adjoint_buffers(self):
        """(adjoint populations, adjoint scalars, scratch) allocated for lbm_adjoint_step."""
        pb, sb, wb = C.c_size_t(), C.c_size_t(), C.c_size_t()
        self._chk(C.lib().lbm_adjoint_sizes(self._h, ctypes.byref(pb), ctypes.byref(sb),
                                            ctypes.byref(wb)))
        rdt = torch.float64 if self.params["precision"] == "fp64" else torch.float32
        dev = self.device
        return (torch.zeros((self.Q,) + self.shape, dtype=rdt, device=dev),
                torch.zeros((self.NS,) + self.shape, dtype=rdt, device=dev),
                torch.empty(max(wb.value, 4), dtype=torch.uint8, device=dev))

    def adjoint_step(self, state, lam_pop, lam_scal, work, out_pop=None, out_scal=None):
        """Adjoint of the state at level n from the adjoint at n+1; state = (pops, scal)."""
        pops, scal = state[0], state[1]
        out_pop = torch.empty_like(lam_pop) if out_pop is None else out_pop
        out_scal = torch.empty_like(lam_scal) if out_scal is None else out_scal
        self._chk(C.lib().lbm_adjoint_step(self._h, _ptr(pops), _ptr(scal) if self.NS else None,
                                           _ptr(lam_pop), _ptr(lam_scal) if self.NS else None,
                                           _ptr(out_pop), _ptr(out_scal) if self.NS else None,
                                           _ptr(work)))
        return out_pop, out_scal

    def objective(self, state, with_grad=True):
        """J = sum rho|u|^2/2 + sum (T - mean T)^2 at the state, and dJ/dstate."""
        pops, scal = state[0], state[1]
        J = ctypes.c_double()
        lp = ls = None
        if with_grad:
            lp, ls, _ = self.adjoint_buffers()
        self._chk(C.lib().lbm_objective(self._h, _ptr(pops), _ptr(scal) if self.NS else None,
                                        ctypes.byref(J), _ptr(lp) if with_grad else None,
                                        _ptr(ls) if (with_grad and self.NS) else None))
        return J.value, lp, ls

    def init_adjoint(self, lam_pop, lam_scal, u0):
        U = self._dev(u0).reshape((self.D,) + self.shape)
        gu = torch.empty_like(U)
        gs = torch.empty((self.NS,) + self.shape, dtype=torch.float64, device=self.device)
        self._chk(C.lib().lbm_init_adjoint(self._h, _ptr(lam_pop), _ptr(lam_scal) if self.NS else None,
                                           _ptr(U), _ptr(gu), _ptr(gs) if self.NS else None))
        torch.cuda.synchronize(self.device)
        return gu, gs

    def set_state(self, pops, scal=None, step=0):
        P = self._dev(pops, self.pop_dtype).reshape((self.Q,) + self.shape)
        S = self._dev(scal, self.scal_dtype).reshape((self.NS,) + self.shape) if self.NS else None
        self._chk(C.lib().lbm_set_state(self._h, _ptr(P), _ptr(S), int(step)))
