"""GPU tests of the closed-domain thermodynamic pressure against the FP64 oracle.

Parity: flame kernels in walled boxes with solid blocks, D2Q9 and D3Q27, one- and
two-step chemistry, linear and banded tile orders; populations, scalars and (pi, q, K)
after tens of steps.  FP64 bounds as the open-domain horizon tests (1e-11 in ghat, 1e-11
of each scalar's range); pi to 1e-13 relative and q to 1e-13 absolute (both come from FP64
sums of ~1e3 terms).  FP32: 1e-6 in ghat and 1e-5 of the scalar ranges after 10 steps,
pi to 1e-7 relative (the sums are FP64 over FP32 cell values).

Full size (the 2500 x 500 chamber of Sec. 3.1): the total mass is held to 1e-12 over
2000 steps and the unburnt gas far from the flame follows the isentropic compression
T/T_u = pi^((gamma-1)/gamma) of a closed vessel."""
import numpy as np
import pytest
import torch

import lbm_inputs as L
from oracle import step as OS
from tests.gpu_helpers import fetch, make_solver, oracle_ghat

pytestmark = pytest.mark.gpu

CS2 = 1.0 / 3.0


def _box(lat, shape, phys, prec, closed=True):
    nz, ny, nx = shape
    D = 2 if lat == "D2Q9" else 3
    faces = ["wall"] * 4 + (["periodic"] * 2 if D == 2 else ["wall"] * 2)
    if D == 3:
        faces[2] = faces[3] = "periodic"
    if phys == "one_step":
        chem = [4.0, 15000.0, 300.0, 2000.0, 1.0]
        ws = [1700.0, 1.0]
    else:
        chem = L.two_step_chem(B1=50.0, B2=5.0)
        ws = [1630.0, 0.05, 0.22, 0.05, 0.13, 0.11]
    p = L.base_params(lat, nx, ny, nz, physics=phys, visc_law="const_mu", nu_ref=0.02,
                      cs_smag=0.17, prandtl=0.7, thickening=2.0, face_bc=faces, chem=chem,
                      T_ref=300.0 if phys == "one_step" else 320.0, weno_scale=ws + [1.0] * (8 - len(ws)),
                      pth_mode="closed" if closed else "open", gamma=1.4, precision=prec)
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    r = np.sqrt(x ** 2 + (y - ny / 2) ** 2 + ((z - nz / 2) ** 2 if D == 3 else 0.0))
    c = 0.5 * (1 - np.tanh((r - min(nx, ny) / 3.0) / 2.0))[None]
    if phys == "one_step":
        scal = np.concatenate([300.0 + 1700.0 * c, 1.0 - c])
    else:
        yf, yo, _ = L.fresh_ch4_air(0.83)
        b = L.burnt_ch4_air(0.83)
        scal = np.concatenate([320.0 + 1630.0 * c, yf * (1 - c), yo * (1 - c) + b["O2"] * c, 0.0 * c,
                               b["CO2"] * c, b["H2O"] * c])
    solid = np.zeros(shape, dtype=bool)
    solid[:, ny // 4: ny // 4 + 3, nx // 2: nx // 2 + 3] = True
    P = np.full(shape, CS2)
    u = np.zeros((D,) + shape)
    return p, P, u, scal, solid


def _gpu(p, P, u, scal, solid, steps):
    s = make_solver(p)
    s.set_geometry(torch.from_numpy(solid.astype(np.uint8)))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    s.step(steps)
    pops, sc, _ = fetch(s)
    th = s.thermo_pressure()
    sums = s.step_sums()
    s.close()
    return pops, sc, th, sums


def _oracle(p, P, u, scal, solid, steps):
    st = OS.init_state(p, torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal),
                       torch.from_numpy(solid))
    sums = None
    for _ in range(steps):
        st, sums = OS.step(p, st)
    return oracle_ghat(p, st), st["scal"].numpy(), st["thermo"], sums.numpy()


@pytest.mark.parametrize("lat,shape,phys,steps", [
    ("D2Q9", (1, 13, 70), "one_step", 20),      # linear tiles, ragged last block
    ("D2Q9", (1, 16, 128), "one_step", 20),     # banded 64x4 tiles
    ("D2Q9", (1, 12, 40), "two_step", 15),
    ("D3Q27", (7, 6, 9), "two_step", 10),
    ("D3Q27", (6, 8, 64), "one_step", 10),      # banded tiles in 3-D
])
def test_closed_parity_fp64(lat, shape, phys, steps):
    print(f"closed parity {lat} {shape} {phys}", flush=True)
    args = _box(lat, shape, phys, "fp64")
    g_pops, g_scal, g_th, g_sums = _gpu(*args, steps)
    o_pops, o_scal, o_th, o_sums = _oracle(*args, steps)
    p, solid = args[0], args[4]
    fl = ~solid
    assert np.abs(g_pops - o_pops)[:, fl].max() < 1e-11
    scale = np.array(p["weno_scale"][:o_scal.shape[0]]).reshape(-1, 1)
    assert (np.abs(g_scal - o_scal)[:, fl] / scale).max() < 1e-11
    assert abs(g_th[0] / o_th[0] - 1) < 1e-13 and abs(g_th[1] - o_th[1]) < 1e-13
    assert abs(g_th[2] / o_th[2] - 1) < 1e-13
    assert o_th[0] != 1.0 and abs(o_th[1]) > 0.0          # the pressure did move
    assert np.allclose(g_sums[:8], o_sums, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("lat,shape,phys", [("D2Q9", (1, 16, 128), "one_step"),
                                            ("D3Q27", (7, 6, 9), "two_step")])
def test_closed_parity_fp32(lat, shape, phys):
    print(f"closed parity fp32 {lat} {shape} {phys}", flush=True)
    args = list(_box(lat, shape, phys, "fp32"))
    args[3] = args[3].astype(np.float32).astype(np.float64)       # inputs as stored
    g_pops, g_scal, g_th, _ = _gpu(*args, 10)
    o_pops, o_scal, o_th, _ = _oracle(*args, 10)
    p, solid = args[0], args[4]
    fl = ~solid
    assert np.abs(g_pops - o_pops)[:, fl].max() < 1e-6
    scale = np.array(p["weno_scale"][:o_scal.shape[0]]).reshape(-1, 1)
    assert (np.abs(g_scal - o_scal)[:, fl] / scale).max() < 1e-5
    assert abs(g_th[0] / o_th[0] - 1) < 1e-7


def test_closed_without_heat_release_is_open():
    """Isothermal flow in a walled box: P_th stays exactly at 1 and the closed run equals
    the open run bit for bit."""
    res = {}
    for closed in (True, False):
        p = L.base_params("D3Q27", 64, 8, 6, nu_ref=0.02, pth_mode="closed" if closed else "open",
                          face_bc=["wall", "wall", "periodic", "periodic", "wall", "wall"])
        z = np.arange(6)[:, None, None] + 0.5
        u = np.zeros((3, 6, 8, 64))
        u[1] = 0.03 * np.sin(np.pi * z / 6) * np.ones((6, 8, 64))
        s = make_solver(p)
        s.init_fields(torch.from_numpy(np.full((6, 8, 64), CS2)), torch.from_numpy(u))
        s.step(50)
        res[closed] = (fetch(s)[0], s.thermo_pressure())
        s.close()
    assert res[True][1][:2] == (1.0, 0.0)
    assert np.array_equal(res[True][0], res[False][0])


def test_chamber_full_size_mass_and_isentropic_compression():
    """2500 x 500 closed chamber, FP64, 2000 steps: sum rho held to 1e-12 (sampled every
    250 steps), pi rises, and the unburnt gas at the far end (uniform, so neither diffused
    nor advected) is compressed isentropically, T/T_u = pi^kappa to 1e-4."""
    p, P, u, scal, mask = L.chamber2d()
    print("chamber 2500x500 closed fp64", flush=True)
    s = make_solver(p)
    s.set_geometry(torch.from_numpy(mask.astype(np.uint8)))
    s.init_fields(torch.from_numpy(P), torch.from_numpy(u), torch.from_numpy(scal))
    m0 = s.fields()["sums"][0]
    worst = 0.0
    for _ in range(8):
        s.step(250)
        worst = max(worst, abs(s.step_sums()[0] / m0 - 1))
    f = s.fields()
    pi, q, K = s.thermo_pressure()
    T_far = float(f["scal"][0, 0, 250, 2400])
    s.close()
    assert worst < 1e-12
    assert pi > 1.0 + 1e-4
    kappa = 0.4 / 1.4
    assert abs(T_far / 300.0 / pi ** kappa - 1) < 1e-4


def test_closed_split_step_on_the_tile_grid_matches_the_small_box():
    """A closed box periodic in x and y with walls in z, and the same box tiled 4 x 4 in x
    and y: the tiled one (about a million cells) runs the split step on the 64x4 tile grid
    (interior instance with a wave's y and z as scalars, list instance at the z walls, the
    pi update over both halves' records), the small one the single all-cell instance.
    Every cell sees the same neighbours and the sums scale by 16 exactly, so after 10 steps
    the two agree to the rounding of the differently ordered sums: ghat to 1e-12, each
    scalar to 1e-12 of its range, pi to 1e-13 and a pi that moved."""
    from tests.gpu_helpers import fetch as _fetch
    nz, ny, nx = 16, 64, 64
    yf, yo, _ = L.fresh_ch4_air(0.83)
    b = L.burnt_ch4_air(0.83)
    base = L.base_params("D3Q27", nx, ny, nz, physics="two_step", visc_law="const_mu", nu_ref=0.02,
                         cs_smag=0.17, prandtl=0.7, thickening=2.0, chem=L.two_step_chem(B1=50.0, B2=5.0),
                         T_ref=320.0, weno_scale=[1630.0, 0.05, 0.22, 0.05, 0.13, 0.11, 1.0, 1.0],
                         face_bc=["periodic"] * 4 + ["wall", "wall"], pth_mode="closed", gamma=1.4,
                         precision="fp64")
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    c = 0.5 * (1 - np.tanh((z - nz / 2 + 2.0 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny)) / 2.0))[None]
    scal = np.concatenate([320.0 + 1630.0 * c, yf * (1 - c), yo * (1 - c) + b["O2"] * c, 0.0 * c,
                           b["CO2"] * c, b["H2O"] * c])
    P = np.full((nz, ny, nx), CS2)
    u = np.zeros((3, nz, ny, nx))
    out = []
    for r in (1, 4):
        p = dict(base, ny=r * ny, nx=r * nx)
        print(f"closed tiled box {nz}x{p['ny']}x{p['nx']}", flush=True)
        s = make_solver(p)
        s.init_fields(torch.from_numpy(np.tile(P, (1, r, r))), torch.from_numpy(np.tile(u, (1, 1, r, r))),
                      torch.from_numpy(np.tile(scal, (1, 1, r, r))))
        s.step(10)
        pops, sc, _ = _fetch(s)
        out.append((pops, sc, s.thermo_pressure()))
        s.close()
    (p0, s0, t0), (p1, s1, t1) = out
    assert np.abs(np.tile(p0, (1, 1, 4, 4)) - p1).max() < 1e-12
    scale = np.array(base["weno_scale"][:6]).reshape(-1, 1, 1, 1)
    assert (np.abs(np.tile(s0, (1, 1, 4, 4)) - s1) / scale).max() < 1e-12
    assert abs(t1[0] / t0[0] - 1) < 1e-13 and t0[0] != 1.0
