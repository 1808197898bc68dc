"""Throughput of the hybrid low-Mach LB/FD time step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--repeats R] [--workload reacting_box]
                [--no-cpu] [--no-extra] [--kernel-only]

Prints one JSON line.  A step is one pass of the whole hot path over the grid: pull
streaming with boundary conditions, scalar stencils and chemistry, moments, source,
cumulant collision, the finite-difference scalar update and the FP64 block sums.
value = lattice updates per second (MLUPS) with every buffer resident in HBM; timed with
HIP events on the stream the kernels run on, R regions of K steps (default 3), the step
time being the median of the regions' means.  The roofline figure uses the algorithmic
bytes of one launch (2 Q s_pop + 2 S s_scal + geometry word + block partials, per cell)
over the average launch duration.  The CPU baseline times the FP64 oracle on a bounded
sample of the same workload on the host cores.
"""
import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import lbm_inputs as L  # noqa: E402

HBM_PEAK_GBS = 8000.0
VALU_ISSUE_PEAK = 256 * 2.4e9          # wave instructions per second (one per CU per cycle)
CS2 = 1.0 / 3.0


def source_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2207_11567_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ------------------------------------------------------------------------ workloads
def workload(name, precision=None):
    """(params, P_h, u, scal or None, solid mask or None, description)."""
    if name == "reacting_box":
        p, P, u, s = L.reacting_box()
        desc = "reacting box 192x192x384 D3Q27 FP32, 2-step CH4/air (6 scalars), F=5, inlet/outlet z"
        solid = None
    elif name == "flame2d":
        p, P, u, s, solid = L.flame2d()
        desc = "2-D flame 1024x256 D2Q9, 1-step Arrhenius, F=4, 3 obstacles, walls + outlet"
    elif name == "hit":
        p, P, u = L.hit(256)
        s, solid = None, None
        desc = "decaying isotropic turbulence 256^3 D3Q27, Smagorinsky 0.17"
    elif name in ("chamber2d", "chamber2d_open"):
        closed = name == "chamber2d"
        p, P, u, s, solid = L.chamber2d(closed=closed)
        desc = ("deflagration chamber 2500x500 D2Q9 (Sec. 3.1 geometry), 1-step Arrhenius, F=4, "
                + ("closed: thermodynamic pressure from the held mass" if closed else
                   "walls, constant thermodynamic pressure"))
    elif name == "tgv":
        p, P, u = L.tgv(128)
        s, solid = None, None
        desc = "Taylor-Green vortex 128^2 D2Q9"
    elif name == "reacting_box_mixture":
        p, P, u, s = L.reacting_box()
        p.update(transport_model="mixture", transport=L.mixture_transport(p["nu_ref"]))
        desc = "reacting box 192x192x384 D3Q27 FP32 with mixture-averaged transport and c_p(T)"
        solid = None
    elif name == "reacting_box_cone":
        p, P, u, s = L.reacting_box()
        solid = L.cone_levelset(p["nx"], p["ny"], p["nz"])
        desc = "reacting box 192x192x384 D3Q27 FP32 with a conical bluff body (curved walls)"
    elif name == "passive_box":
        p, P, u = L.hit(128, seed=11567)
        s = L.passive_field(128)[None]
        p.update(physics="passive", prandtl=0.7, weno_scale=[1.0] * 8, precision="fp32")
        solid = None
        desc = "HIT 128^3 D3Q27 FP32 with a passive temperature"
    else:
        raise ValueError(name)
    if precision is not None:
        p["precision"] = precision
    return p, P, u, s, solid, desc


def bytes_per_cell(p):
    Q = 9 if p["lattice"] == "D2Q9" else 27
    NS = {"isothermal": 0, "passive": 1, "one_step": 2, "two_step": 6}[p["physics"]]
    sp = {"fp64": 8, "fp32": 4, "fp16s": 2}[p["precision"]]
    ss = 8 if p["precision"] == "fp64" else 4
    return 2 * Q * sp + 2 * NS * ss + 64.0 / 256.0


def run_gpu(name, steps, warmup, precision=None, observables=False, repeats=3):
    import torch

    from paper_2207_11567_amd import Solver
    p, P, u, s, solid, desc = workload(name, precision)
    solver = Solver(p, device="cuda:0")
    if solid is not None and solid.dtype == np.float64:
        solver.set_wall_distance(torch.from_numpy(solid))          # signed wall distance
        solid = solid < 0
    elif solid is not None:
        solver.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
    solver.init_fields(torch.from_numpy(P), torch.from_numpy(u),
                       torch.from_numpy(s) if s is not None else None)
    del P, u, s
    N = p["nx"] * p["ny"] * p["nz"]
    n_fluid = N - (int(np.count_nonzero(solid)) if solid is not None else 0)
    extra = {}
    if observables:
        # running statistics at every level and 8 probes along the mid-line
        solver.set_statistics(1)
        cells = [int(p["nx"] * (k + 1) / 9) + p["nx"] * (p["ny"] // 2) for k in range(8)]
        solver.set_probes(cells, capacity=warmup + steps * max(1, repeats))
    solver.step(warmup)
    torch.cuda.synchronize()
    # `repeats` timed regions of `steps` steps each, every one bracketed by device
    # synchronisation; the step time is the median of the regions' means
    rep_ms = []
    for _ in range(max(1, repeats)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(solver.stream)
        solver.step(steps)
        e1.record(solver.stream)
        torch.cuda.synchronize()
        rep_ms.append(e0.elapsed_time(e1) / steps)
    ms = float(np.median(rep_ms)) * steps
    sums = solver.step_sums()            # raises on a non-finite value
    if p["physics"] in ("one_step", "two_step"):
        T_u, T_b = (p["chem"][2], p["chem"][3]) if p["physics"] == "one_step" else (p["inlet_T"], 1950.0)
        solver.flame_surface(T_u, T_b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            extra["flame_surface"] = solver.flame_surface(T_u, T_b)
        extra["flame_surface_ms"] = (time.perf_counter() - t0) / 20 * 1e3
    if p.get("pth_mode") == "closed":
        extra["pth_ratio"] = solver.thermo_pressure()[0]
    bpc = bytes_per_cell(p) + (4 if (solid is not None and p["lattice"] == "D2Q9") else 0) \
        + (8 if (solid is not None and p["lattice"] == "D3Q27") else 0)
    t_launch = ms / 1e3 / steps
    achieved = bpc * N / t_launch / 1e9
    solver.close()
    del solver
    torch.cuda.empty_cache()
    return {"workload": name, "desc": desc, "params": p, "cells": N, "steps": steps,
            "ms_per_step": ms / steps, "mlups": N * steps / (ms / 1e3) / 1e6,
            "fluid_mlups": n_fluid * steps / (ms / 1e3) / 1e6,
            "bytes_per_cell": bpc, "achieved_gbs": achieved, "sums": sums, "observables": extra,
            "repeat_ms_per_step": [round(v, 5) for v in rep_ms]}


def cpu_baseline(name, budget_s=15.0):
    """The FP64 oracle as it stands, on a bounded sample of the workload."""
    import torch

    from oracle import step as OS
    if name == "reacting_box":
        p, P, u, s = L.reacting_box(32, 32, 64)
        solid = None
        sample = "reacting box 32x32x64 copy (same physics), oracle steps until the time budget"
    elif name == "flame2d":
        p, P, u, s, solid = L.flame2d(256, 64)
        sample = "2-D flame 256x64 copy"
    elif name == "hit":
        p, P, u = L.hit(48)
        s, solid = None, None
        sample = "HIT 48^3 copy"
    else:
        p, P, u = L.tgv(128)
        s, solid = None, None
        sample = "TGV 128^2"
    st = OS.init_state(p, torch.from_numpy(P), torch.from_numpy(u),
                       torch.from_numpy(s) if s is not None else None,
                       torch.from_numpy(solid).bool() if solid is not None else None)
    N = p["nx"] * p["ny"] * p["nz"]
    OS.step(p, st)

    def timed(budget):
        nonlocal st
        t0 = time.time()
        n = 0
        while n < 2 or time.time() - t0 < budget:
            st, _ = OS.step(p, st)
            n += 1
            if n >= 200:
                break
        return n, time.time() - t0

    n, dt = timed(budget_s)
    threads = torch.get_num_threads()
    torch.set_num_threads(1)                   # the same oracle on one host thread
    n1, dt1 = timed(budget_s / 3)
    torch.set_num_threads(threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": N * n / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "sample": f"{sample}: {N} cells x {n} steps in {dt:.1f} s (FP64)",
            "single_thread_value": N * n1 / dt1 / 1e6, "host_cpu": model}


def traffic_for(name, p, bpc, N):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on
    the current kernel sources."""
    f = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def copy_bandwidth(nbytes=2 << 30, reps=10):
    """Read + write bandwidth of plain device-to-device copies of nbytes, timed with HIP
    events: torch's copy, and the library's copy probe with streaming loads and stores (the
    step kernel's own memory forms); the practical HBM ceilings beside the 8 TB/s
    specification."""
    import torch
    from paper_2207_11567_amd.solver import copy_probe
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("torch", lambda: b.copy_(a)), ("probe", lambda: copy_probe(a, b, 3))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def valu_for(name):
    """VALU issue figures of the step kernel from the committed SQ-counter run, if it was
    taken on the current kernel sources."""
    f = os.path.join(ROOT, "profiles", f"valu_{name}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    return {"valu_per_wave": round(rec["valu_per_wave"], 1), "valu_insts_per_launch": rec["valu_insts"],
            "issue_frac_profiled": round(rec["valu_issue_frac"], 4),
            "issue_limit": "one wave instruction per CU per cycle: 256 CUs x 2.4 GHz = 614 G/s"}


def precision_errors(steps=2000, n=256, rsteps=200):
    """FP32 and FP16-storage runs against the FP64 run of the same seeded input: the HIT
    field at the workload's size (256^3, 2000 steps; velocity and P_h errors, shell-averaged
    energy spectrum) and the reacting box (192x192x384, 200 steps; velocity, P_h, T and the
    five transported species).  Field errors are relative L2 norms of the difference over
    the norm of the FP64 field's deviation from its mean; the FP64 path itself matches the
    oracle to 1e-11.  Also the step time of each precision (HIP events) and its speedup over
    FP64."""
    import torch

    from paper_2207_11567_amd import Solver

    def spectrum(v):
        e = np.zeros(n // 2 - 1)
        k = np.fft.fftfreq(n) * n
        K = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
        shells = np.rint(K).astype(np.int64).ravel()
        for c in range(3):
            vk = np.fft.fftn(v[c])
            e += np.bincount(shells, (0.5 * np.abs(vk) ** 2).ravel(), minlength=n)[1:n // 2]
        return e

    def rel(a, ref):
        dev = ref - ref.mean(axis=tuple(range(1, ref.ndim)), keepdims=True)
        return float(np.sqrt(((a - ref) ** 2).sum() / (dev ** 2).sum()))

    def run(p, P, u, sc, k):
        s = Solver(p, device="cuda:0")
        s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(sc) if sc is not None else None)
        s.step(10)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(k - 10)
        e1.record(s.stream)
        f = s.fields()
        ms = e0.elapsed_time(e1) / (k - 10)
        out = {"u": f["u"].cpu().numpy(), "P_h": f["P_h"].cpu().numpy()[None], "scal": f["scal"].cpu().numpy()}
        s.close()
        torch.cuda.empty_cache()
        return out, ms

    res = {"hit": {}, "reacting_box": {}}
    speed = {"hit": {}, "reacting_box": {}}
    p0, P, u = L.hit(n)
    ref = None
    spectra = {}
    for prec in ("fp64", "fp32", "fp16s"):
        f, ms = run(dict(p0, precision=prec), P, u, None, steps)
        speed["hit"][prec] = ms
        spectra[prec] = spectrum(f["u"])
        if prec == "fp64":
            ref = f
            continue
        r = {"u_rel_l2": rel(f["u"], ref["u"]), "P_h_rel_l2": rel(f["P_h"], ref["P_h"])}
        sp = np.abs(spectra[prec] - spectra["fp64"]) / spectra["fp64"]
        r["spectrum_max_rel_err"] = float(sp.max())
        r["spectrum_rel_err_k_le_16"] = float(sp[:16].max())
        r["case"] = f"HIT {n}^3 D3Q27, {steps} steps, Smagorinsky 0.17"
        res["hit"][prec] = r
    del ref, spectra
    p0, P, u, sc = L.reacting_box()
    names = ["T", "CH4", "O2", "CO", "CO2", "H2O"]
    ref = None
    for prec in ("fp64", "fp32", "fp16s"):
        f, ms = run(dict(p0, precision=prec), P, u, sc, rsteps)
        speed["reacting_box"][prec] = ms
        if prec == "fp64":
            ref = f
            continue
        r = {"u_rel_l2": rel(f["u"], ref["u"]), "P_h_rel_l2": rel(f["P_h"], ref["P_h"])}
        for k, nm in enumerate(names):
            r[f"{nm}_rel_l2"] = rel(f["scal"][k:k + 1], ref["scal"][k:k + 1])
        r["case"] = f"reacting box 192x192x384 D3Q27 two-step, {rsteps} steps"
        res["reacting_box"][prec] = r
    sp = {w: {"ms_per_step": {k: round(v, 4) for k, v in t.items()},
              "speedup_over_fp64": {k: round(t["fp64"] / v, 3) for k, v in t.items() if k != "fp64"}}
          for w, t in speed.items()}
    return res, sp


def differentiation(nsteps=2000, seg=100, n=128):
    """Cost of the hand-written adjoint on the differentiation workload: 128^3 D3Q27 FP32
    with a passive temperature, J = sum rho|u|^2/2 + sum (T - mean T)^2 after nsteps,
    checkpoints every seg steps."""
    import torch

    from paper_2207_11567_amd import Solver
    from paper_2207_11567_amd.adjoint import rollout_objective
    p, P, u = L.hit(n, seed=11567)
    T = L.passive_field(n)
    p.update(physics="passive", prandtl=0.7, weno_scale=[1.0] * 8, precision="fp32")
    s = Solver(p, device="cuda:0")
    Pd = torch.from_numpy(P).cuda()
    u0 = torch.from_numpy(u).cuda().requires_grad_(True)
    T0 = torch.from_numpy(T).cuda().requires_grad_(True)
    rollout_objective(s, u0.detach(), T0.detach(), Pd, 50, 25)        # warm-up
    torch.cuda.synchronize()
    t0 = time.time()
    J = rollout_objective(s, u0, T0, Pd, nsteps, seg)
    torch.cuda.synchronize()
    t1 = time.time()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.time()
    # per-step kernel costs on a fixed state
    state = s.get_state()
    lp, ls, work = s.adjoint_buffers()
    lp.normal_()
    ls.normal_()
    out = (torch.empty_like(state[0]), torch.empty_like(state[1]))
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    reps = 50
    e[0].record()
    for _ in range(reps):
        s.step_from(state[:2], out, 0)
    e[1].record()
    for _ in range(reps):
        s.adjoint_step(state[:2], lp, ls, work)
    e[2].record()
    torch.cuda.synchronize()
    fwd_ms = e[0].elapsed_time(e[1]) / reps
    adj_ms = e[1].elapsed_time(e[2]) / reps
    s.close()
    return {"case": f"{n}^3 D3Q27 FP32 passive T, {nsteps} steps, checkpoints every {seg}",
            "J": float(J.detach()), "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
            "backward_over_forward": round((t2 - t1) / (t1 - t0), 3),
            "step_ms": round(fwd_ms, 4), "adjoint_step_ms": round(adj_ms, 4),
            "adjoint_step_over_step": round(adj_ms / fwd_ms, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed regions of --steps steps each; ms_per_step is their median")
    ap.add_argument("--workload", default="reacting_box",
                    choices=["reacting_box", "flame2d", "hit", "tgv", "passive_box", "chamber2d",
                             "chamber2d_open", "reacting_box_mixture", "reacting_box_cone"])
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "fp32", "fp16s"])
    ap.add_argument("--observables", action="store_true",
                    help="sample running statistics and 8 probes at every step of the main workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--kernel-only", action="store_true",
                    help="time the main workload only (for profiler runs)")
    ap.add_argument("--diff-only", action="store_true",
                    help="run a 200-step differentiation of the 128^3 workload (for profiler runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain 1 GiB device copy 3 times (counter calibration) and exit")
    args = ap.parse_args()
    if args.diff_only:
        print(json.dumps(differentiation(nsteps=200, seg=100)))
        return
    if args.copy_calib:
        import torch
        from paper_2207_11567_amd.solver import copy_probe
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        # the same bytes through the step kernel's own load and store forms (library copy
        # probe, modes 0-3: cached / streaming loads x cached / streaming stores), timed
        gbs = {}
        for mode in range(4):
            copy_probe(a, b, mode)                        # first launch of this form: untimed
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                copy_probe(a, b, mode)
            e1.record()
            torch.cuda.synchronize()
            gbs[mode] = round(3 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)
        if not torch.equal(a, b):
            raise RuntimeError("copy probe: destination differs from source")
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4,
                          "launches": 3, "probe_gbs_by_mode": gbs}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library steps one grid on one GPU: the time step is measured on one "
                                   "MI355X; sharding across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    main_res = run_gpu(args.workload, args.steps, args.warmup, args.precision, args.observables,
                       repeats=args.repeats)
    p = main_res["params"]
    N = main_res["cells"]
    print(f"# {args.workload}: {main_res['mlups']:.1f} MLUPS, {main_res['ms_per_step']:.3f} ms/step",
          file=sys.stderr, flush=True)
    if args.kernel_only:
        return
    traffic = traffic_for(args.workload, p, main_res["bytes_per_cell"], N)
    achieved = main_res["achieved_gbs"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": main_res["bytes_per_cell"] * N}
    copy_gbs = copy_bandwidth()
    extra = {}
    valu = valu_for(args.workload)
    if valu is not None:
        # the step's other limit: VALU issue (counted instructions over the live launch time)
        valu["issue_frac"] = round(valu["valu_insts_per_launch"] / (main_res["ms_per_step"] * 1e-3) / VALU_ISSUE_PEAK, 4)
        extra["step_kernel_valu"] = valu
        roofline["valu_issue_frac"] = valu["issue_frac"]
    extra["hbm_copy_gbs"] = round(copy_gbs["torch"], 1)
    extra["hbm_probe_copy_gbs"] = round(copy_gbs["probe"], 1)
    extra["frac_of_copy"] = round(achieved / max(copy_gbs.values()), 4)
    if not args.no_extra:
        for name, prec, k in (("tgv", "fp64", 1000), ("flame2d", "fp64", 400),
                              ("flame2d", "fp32", 400), ("hit", "fp64", 40), ("hit", "fp32", 60),
                              ("hit", "fp16s", 60), ("passive_box", "fp32", 100),
                              ("chamber2d", "fp64", 400), ("chamber2d_open", "fp64", 400),
                              ("chamber2d+observables", "fp64", 400), ("reacting_box_mixture", "fp32", 40),
                              ("reacting_box_cone", "fp32", 40)):
            obs = name.endswith("+observables")
            r = run_gpu(name.split("+")[0], k, 10, prec, observables=obs)
            extra[f"{name}_{prec}"] = {"mlups": round(r["mlups"], 1), "fluid_mlups": round(r["fluid_mlups"], 1),
                                       "ms_per_step": round(r["ms_per_step"], 4),
                                       "achieved_gbs": round(r["achieved_gbs"], 1),
                                       "hbm_frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                                       "cells": r["cells"], "desc": r["desc"]}
            if r["observables"]:
                extra[f"{name}_{prec}"]["observables"] = {k2: round(v, 6) for k2, v in r["observables"].items()}
            print(f"# {name} {prec}: {r['mlups']:.1f} MLUPS", file=sys.stderr, flush=True)
        extra["precision_error_vs_fp64"], extra["precision_speed"] = precision_errors()
        print(f"# precision: {extra['precision_speed']}", file=sys.stderr, flush=True)
        extra["differentiation"] = differentiation()
        print(f"# differentiation: {extra['differentiation']}", file=sys.stderr, flush=True)
    cpu = None if args.no_cpu else cpu_baseline(args.workload)
    line = {
        "metric": "MLUPS of full hybrid step, % HBM roofline; FP16/32 vs FP64 error; adjoint/fwd",
        "value": round(main_res["mlups"], 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64", "fp32": "f32",
                                                          "fp16s": "f16-storage/f32"}[p["precision"]],
        "data": "synthetic (seeded)",
        "config": {"workload": main_res["desc"], "nx": p["nx"], "ny": p["ny"], "nz": p["nz"],
                   "lattice": p["lattice"], "precision": p["precision"], "physics": p["physics"],
                   "parallelism": "single GPU"},
        "timing": {"repeats": len(main_res["repeat_ms_per_step"]),
                   "ms_per_step_each": main_res["repeat_ms_per_step"],
                   "ms_per_step_min": min(main_res["repeat_ms_per_step"]),
                   "ms_per_step_max": max(main_res["repeat_ms_per_step"]),
                   "ms_per_step_is": "median over the repeats"},
        "roofline": roofline, "cpu_baseline": cpu,
        "paper_context": {"value": 0.4, "unit": "MLUPS", "hardware": "SuperMUC-NG CPU cluster",
                          "note": "LB + FD + thermochemistry on PRECCINSTA (about 30 Mi points); "
                                  "not a target"},
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
