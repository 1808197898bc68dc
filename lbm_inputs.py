"""Seeded synthetic inputs for the hybrid LB/FD time step: the only module shared by the
oracle-side tests and the GPU path's tests and benchmark.  It builds workloads (fields,
geometry masks, parameter sets, random population deviations) and holds none of the
scheme's arithmetic: no equilibria, moments, collision, stencils or chemistry.

Every workload is in lattice units (dr = dt = 1).  Field layout: scalars (nz, ny, nx),
vectors (D, nz, ny, nx), x fastest; all numpy float64.
"""
import math

import numpy as np

CS2 = 1.0 / 3.0
FACES = ("periodic",) * 6


# ----------------------------------------------------------------------------- params
def base_params(lattice, nx, ny, nz=1, **kw):
    p = dict(lattice=lattice, nx=nx, ny=ny, nz=nz, precision="fp64", collision="cumulant",
             physics="isothermal", visc_law="const_nu", nu_ref=0.01, omega_bulk=1.0,
             omega_high=1.0, cs_smag=0.0, prandtl=0.7, thickening=1.0, rho_ref=1.0,
             T_ref=300.0, face_bc=list(FACES), inlet_u=[0.0, 0.0, 0.0], inlet_noise=0.0,
             outlet_P=1.0 * CS2, inlet_T=300.0, inlet_Y=[0.0] * 8, weno_scale=[1.0] * 8,
             chem=[0.0] * 32, seed=2207, pth_mode="open", gamma=1.4,
             transport_model="simple", transport=[0.0] * 32, galilean=0, fourth_order=0)
    p.update(kw)
    return p


# 1-step chemistry constants (Arrhenius fuel consumption, lattice units):
# [B (1/step), Ta (K), T_u (K), T_ad (K), Y_u]
ONE_STEP_CHEM = [4.0, 15000.0, 300.0, 2000.0, 1.0]

# 2-step CH4/air placeholder constants (structure CH4 + 1.5 O2 -> CO + 2 H2O,
# CO + 0.5 O2 -> CO2; calibrated constants of the paper's scheme are not available):
# [B1, Ta1, B2, Ta2, c_p (J/kg/K), W_k (kg/mol) x6 (CH4, O2, CO, CO2, H2O, N2),
#  h_k (J/mol) x6, W_ref (kg/mol)]
_AC, _AH, _AO, _AN = 12.011e-3, 1.008e-3, 15.999e-3, 14.007e-3      # kg/mol
W_SPECIES = [_AC + 4 * _AH, 2 * _AO, _AC + _AO, _AC + 2 * _AO, 2 * _AH + _AO, 2 * _AN]
H_SPECIES = [-74.87e3, 0.0, -110.53e3, -393.52e3, -241.83e3, 0.0]


def fresh_ch4_air(phi):
    """Mass fractions of a CH4/air mixture at equivalence ratio phi (air = O2 + 3.76 N2);
    textbook atom balance.  Returns (Y_CH4, Y_O2, Y_N2)."""
    n_ch4, n_o2, n_n2 = phi, 2.0, 2.0 * 3.76
    m = [n_ch4 * W_SPECIES[0], n_o2 * W_SPECIES[1], n_n2 * W_SPECIES[5]]
    tot = sum(m)
    return m[0] / tot, m[1] / tot, m[2] / tot


def burnt_ch4_air(phi):
    """Complete-combustion products of a lean CH4/air mixture (CO2, H2O, O2 left, N2)."""
    n_ch4, n_o2, n_n2 = phi, 2.0, 2.0 * 3.76
    prod = {"CO2": n_ch4, "H2O": 2.0 * n_ch4, "O2": n_o2 - 2.0 * n_ch4, "N2": n_n2}
    m = {"CO2": prod["CO2"] * W_SPECIES[3], "H2O": prod["H2O"] * W_SPECIES[4],
         "O2": prod["O2"] * W_SPECIES[1], "N2": prod["N2"] * W_SPECIES[5]}
    tot = sum(m.values())
    return {k: v / tot for k, v in m.items()}


def mean_W(Y):
    """Mean molar mass 1/sum(Y_k/W_k) of a composition given as a 6-list (N2 last)."""
    return 1.0 / sum(y / w for y, w in zip(Y, W_SPECIES))


def two_step_chem(B1=2.0e4, Ta1=15000.0, B2=1.0e2, Ta2=6000.0, cp=1400.0, phi=0.83):
    """Placeholder 2-step CH4/air constants (lattice units; the paper's calibrated set is not
    available).  The scalars advance by explicit Euler, so the CO oxidation rate per step,
    lambda_CO = (B2/F) exp(-Ta2/T) (rho Y_O2/W_O2)^(1/2), must stay below one for a monotone
    update: B2 = 100 gives about 0.4 in the burnt gas of the reacting box (F = 5); B2 = 2000
    gave about 8, an unstable update whose CO swung negative and turned the burnt region
    chaotic."""
    yf, yo, yn = fresh_ch4_air(phi)
    W_ref = mean_W([yf, yo, 0.0, 0.0, 0.0, yn])
    return [B1, Ta1, B2, Ta2, cp] + W_SPECIES + H_SPECIES + [W_ref]


def mixture_transport(nu_ref, prandtl=0.7, s_mu=0.7, s_D=1.75):
    """Placeholder mixture-averaged transport data for CH4, O2, CO, CO2, H2O, N2 (the
    paper's REGATH data are not available): binary diffusion coefficients in the ratios
    of typical values at room conditions (relative to O2-N2), scaled so that O2-N2 has
    the thermal diffusivity nu_ref/Pr at T_ref; linear c_p,k(T) = a_k + b_k T fits
    (J/kg/K); power-law exponents of mu(T) and D(T).  Layout as the transport array of
    the parameter set."""
    rel = {(0, 1): 0.22, (0, 2): 0.22, (0, 3): 0.17, (0, 4): 0.29, (0, 5): 0.22,
           (1, 2): 0.21, (1, 3): 0.16, (1, 4): 0.26, (1, 5): 0.21,
           (2, 3): 0.16, (2, 4): 0.26, (2, 5): 0.21,
           (3, 4): 0.20, (3, 5): 0.16, (4, 5): 0.26}
    alpha = nu_ref / prandtl
    D0 = [alpha * rel[(k, j)] / 0.21 for k in range(6) for j in range(k + 1, 6)]
    a = [1650.0, 878.0, 990.0, 733.0, 1672.0, 990.0]
    b = [1.9, 0.14, 0.17, 0.39, 0.625, 0.17]
    return D0 + a + b + [s_mu, s_D, 0.0, 0.0, 0.0]


# ----------------------------------------------------------------------------- workloads
def tgv(n=128, U0=0.05 * math.sqrt(CS2), nu=0.01, rho=1.0):
    """2-D Taylor-Green vortex u = U0 sin(kx) cos(ky), v = -U0 cos(kx) sin(ky),
    P_h = rho cs2 - rho U0^2/4 (cos 2kx + cos 2ky), k = 2 pi / n."""
    k = 2 * math.pi / n
    x = np.arange(n)[None, None, :].astype(np.float64)
    y = np.arange(n)[None, :, None].astype(np.float64)
    u = np.zeros((2, 1, n, n))
    u[0] = U0 * np.sin(k * x) * np.cos(k * y)
    u[1] = -U0 * np.cos(k * x) * np.sin(k * y)
    P = rho * CS2 - rho * U0 ** 2 / 4.0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    P = np.broadcast_to(P, (1, n, n)).copy()
    params = base_params("D2Q9", n, n, 1, nu_ref=nu, rho_ref=rho)
    return params, P, u


def hit(n=256, k0=4.0, urms=0.05 * math.sqrt(CS2), seed=11567, nu=1e-3, cs_smag=0.17):
    """Seeded solenoidal random velocity with E(k) ~ k^4 exp(-2 (k/k0)^2), rescaled to the
    given per-component rms; uniform P_h = rho cs2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kx = np.fft.fftfreq(n) * n
    KX, KY, KZ = np.meshgrid(kx, kx, np.fft.rfftfreq(n) * n, indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    K = np.sqrt(K2)
    K2s = np.where(K2 == 0, 1.0, K2)
    amp = np.sqrt(K ** 4 * np.exp(-2.0 * (K / k0) ** 2) / (4 * np.pi * np.maximum(K, 1.0) ** 2))
    comps = []
    for _ in range(3):
        comps.append((rng.standard_normal(K.shape) + 1j * rng.standard_normal(K.shape)) * amp)
    kdotu = (KX * comps[0] + KY * comps[1] + KZ * comps[2]) / K2s
    comps = [comps[0] - KX * kdotu, comps[1] - KY * kdotu, comps[2] - KZ * kdotu]
    u = np.stack([np.fft.irfftn(c, s=(n, n, n), axes=(0, 1, 2)) for c in comps])   # (x, y, z)
    u = u.transpose(0, 3, 2, 1).copy()                               # -> (D, z, y, x)
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    u *= urms / np.sqrt((u ** 2).mean())
    P = np.full((n, n, n), CS2)
    params = base_params("D3Q27", n, n, n, nu_ref=nu, cs_smag=cs_smag)
    return params, P, u


def obstacles(nx=1024, ny=256, seed=2207):
    """Three rectangular solid blocks from a SplitMix64 stream (seed): block k spans
    x0 = 160 + 224k + floor(64 r), width 12 + floor(20 r), height 48 + floor(96 r),
    y0 = 16 + floor((224 - h) r), scaled to the grid size."""
    state = [seed & 0xFFFFFFFFFFFFFFFF]

    def rnd():
        state[0] = (state[0] + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
        z = state[0]
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
        z ^= z >> 31
        return (z >> 11) * 2.0 ** -53

    sx, sy = nx / 1024.0, ny / 256.0
    mask = np.zeros((1, ny, nx), dtype=np.uint8)
    for k in range(3):
        x0 = 160 + 224 * k + math.floor(64 * rnd())
        w = 12 + math.floor(20 * rnd())
        h = 48 + math.floor(96 * rnd())
        y0 = 16 + math.floor((224 - h) * rnd())
        mask[0, int(y0 * sy):int((y0 + h) * sy), int(x0 * sx):max(int((x0 + w) * sx), int(x0 * sx) + 1)] = 1
    return mask


def flame2d(nx=1024, ny=256, radius=20.0, width=2.0, Tu=300.0, Tb=2000.0, F=4.0,
            FD=0.03, cs_smag=0.17, seed=2207):
    """2-D premixed flame in a channel: walls left/top/bottom, outlet right, three solid
    blocks, ignition as a burnt half-disc of the given radius at the middle of the closed
    left end (tanh profile of the given width).  Constant rho D with F D = FD at T_u."""
    mask = obstacles(nx, ny, seed)
    x = np.arange(nx)[None, None, :] + 0.5
    y = np.arange(ny)[None, :, None] + 0.5
    r = np.sqrt(x ** 2 + (y - ny / 2.0) ** 2)
    theta = 0.5 * (1.0 - np.tanh((r - radius) / width))     # 1 burnt, 0 fresh
    T = Tu + (Tb - Tu) * theta
    Y = 1.0 - theta
    scal = np.stack([T, Y]).reshape(2, 1, ny, nx)
    P = np.full((1, ny, nx), CS2)
    u = np.zeros((2, 1, ny, nx))
    D_u = FD / F
    params = base_params("D2Q9", nx, ny, 1, physics="one_step", visc_law="const_mu",
                         nu_ref=0.7 * D_u, prandtl=0.7, thickening=F, cs_smag=cs_smag,
                         T_ref=Tu, face_bc=["wall", "outlet", "wall", "wall",
                                            "periodic", "periodic"],
                         outlet_P=CS2, inlet_T=Tu, weno_scale=[Tb - Tu, 1.0],
                         chem=list(ONE_STEP_CHEM[:2]) + [Tu, Tb, 1.0])
    return params, P, u, scal, mask


def chamber_mask(nx=2500, ny=500):
    """Solid mask of the deflagration chamber of Sec. 3.1 (250 mm x 50 mm) on an nx x ny
    grid (nx/250 cells per mm): three rows of five 3 mm x 4 mm baffles whose row centres
    sit 20, 50 and 80 mm from the left wall, 9 mm apart vertically (centre to centre,
    centred on the mid-height), and a 12 mm square obstacle whose upstream face is 94 mm
    from the left wall, centred vertically."""
    s = nx / 250.0
    mask = np.zeros((1, ny, nx), dtype=bool)

    def block(x0, x1, y0, y1):
        mask[0, int(round(y0 * s)):int(round(y1 * s)), int(round(x0 * s)):int(round(x1 * s))] = True

    for xc in (20.0, 50.0, 80.0):
        for k in range(-2, 3):
            yc = 25.0 + 9.0 * k
            block(xc - 1.5, xc + 1.5, yc - 2.0, yc + 2.0)
    block(94.0, 106.0, 19.0, 31.0)
    return mask


def chamber2d(nx=2500, ny=500, Tu=300.0, Tb=2000.0, F=4.0, FD=0.03, cs_smag=0.17, closed=True,
              gamma=1.4, precision="fp64"):
    """Closed 2-D deflagration chamber of Sec. 3.1 on the paper's 2500 x 500 grid
    (0.1 mm cells): walls on all four sides, the obstacles of chamber_mask, burnt gas in a
    half-disc of radius 10 mm at the middle of the left wall (tanh edge of 2 cells), the
    one-step chemistry and thickened-flame settings of flame2d, and (closed=True) the
    thermodynamic pressure held by the mass the chamber contains."""
    mask = chamber_mask(nx, ny)
    radius = 10.0 * nx / 250.0
    x = np.arange(nx)[None, None, :] + 0.5
    y = np.arange(ny)[None, :, None] + 0.5
    r = np.sqrt(x ** 2 + (y - ny / 2.0) ** 2)
    theta = 0.5 * (1.0 - np.tanh((r - radius) / 2.0))
    T = Tu + (Tb - Tu) * theta
    Y = 1.0 - theta
    scal = np.stack([T, Y]).reshape(2, 1, ny, nx)
    P = np.full((1, ny, nx), CS2)
    u = np.zeros((2, 1, ny, nx))
    D_u = FD / F
    params = base_params("D2Q9", nx, ny, 1, physics="one_step", visc_law="const_mu",
                         nu_ref=0.7 * D_u, prandtl=0.7, thickening=F, cs_smag=cs_smag,
                         T_ref=Tu, face_bc=["wall", "wall", "wall", "wall", "periodic", "periodic"],
                         inlet_T=Tu, weno_scale=[Tb - Tu, 1.0],
                         chem=list(ONE_STEP_CHEM[:2]) + [Tu, Tb, 1.0],
                         pth_mode="closed" if closed else "open", gamma=gamma, precision=precision)
    return params, P, u, scal, mask


def cone_levelset(nx, ny, nz, base=0.2, height=0.16, z0=0.04):
    """Signed distance (cells, positive in the fluid) to a solid cone on the axis of an
    nx x ny x nz box, pointing downstream (+z): base radius base*min(nx, ny) at z0*nz,
    apex height*nz further on; a stand-in for the burner's conical bluff body.  Inside
    the cone the distance is the negative distance to its mantle or base."""
    R = base * min(nx, ny)
    H = height * nz
    zb = z0 * nz
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    r = np.hypot(x - nx / 2.0, y - ny / 2.0)
    h = z - zb                                     # height above the base plane
    L = math.hypot(R, H)
    # distance to the (infinite) mantle line in the (r, h) half-plane, signed
    d_mantle = (r * H + h * R - R * H) / L         # > 0 outside, < 0 inside
    inside = (h >= 0) & (h <= H) & (d_mantle < 0)
    d_base = -h                                    # > 0 below the base plane
    outside = np.maximum(d_mantle, d_base)         # convex solid: max of the half-spaces
    return np.where(inside, np.maximum(d_mantle, np.maximum(d_base, h - H)), outside)


def reacting_box(nx=192, ny=192, nz=384, u_in=0.1, noise=0.05, phi=0.83, T_in=320.0,
                 T_b=1950.0, F=5.0, nu=5e-4, cs_smag=0.17, seed=2207, chem=None):
    """3-D box, periodic in x and y, inlet at z = 0 and outlet at z = nz-1, fresh CH4/air
    at phi flowing in at u_in (+ relative noise), burnt products beyond a tanh front of
    width 2F cells at mid-length."""
    chem = two_step_chem(phi=phi) if chem is None else chem
    yf, yo, yn = fresh_ch4_air(phi)
    b = burnt_ch4_air(phi)
    z = np.arange(nz)[:, None, None] + 0.5
    theta = 0.5 * (1.0 + np.tanh((z - nz / 2.0) / (2.0 * F)))
    shape = (nz, ny, nx)
    T = np.broadcast_to(T_in + (T_b - T_in) * theta, shape)
    Y_ch4 = np.broadcast_to(yf * (1 - theta), shape)
    Y_o2 = np.broadcast_to(yo * (1 - theta) + b["O2"] * theta, shape)
    Y_co = np.zeros(shape)
    Y_co2 = np.broadcast_to(b["CO2"] * theta, shape)
    Y_h2o = np.broadcast_to(b["H2O"] * theta, shape)
    scal = np.stack([T, Y_ch4, Y_o2, Y_co, Y_co2, Y_h2o]).astype(np.float64)
    u = np.zeros((3,) + shape)
    u[2] = u_in
    P = np.full(shape, CS2)
    params = base_params("D3Q27", nx, ny, nz, physics="two_step", visc_law="const_mu",
                         nu_ref=nu, prandtl=0.7, thickening=F, cs_smag=cs_smag, T_ref=T_in,
                         face_bc=["periodic", "periodic", "periodic", "periodic",
                                  "inlet", "outlet"],
                         inlet_u=[0.0, 0.0, u_in], inlet_noise=noise, outlet_P=CS2,
                         inlet_T=T_in, inlet_Y=[yf, yo, 0.0, 0.0, 0.0, 0, 0, 0],
                         weno_scale=[T_b - T_in, yf, yo, 0.05, b["CO2"], b["H2O"]],
                         chem=chem, seed=seed, precision="fp32")
    return params, P, u, scal


def passive_field(n, seed=5, kmax=4):
    """Smooth seeded random scalar with unit variance (low-wavenumber Fourier modes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.arange(n) * 2 * np.pi / n
    X = x[None, None, :]
    Yc = x[None, :, None]
    Z = x[:, None, None]
    T = np.zeros((n, n, n))
    for _ in range(12):
        k = rng.integers(-kmax, kmax + 1, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        T += rng.standard_normal() * np.cos(k[0] * X + k[1] * Yc + k[2] * Z + ph)
    T -= T.mean()
    return T / max(T.std(), 1e-12)


def random_deviation(Q, shape, seed, amp=0.01):
    """Random population deviations ghat_i (storage format g_i/P0 - w_i): smooth part +
    white noise, for one-step parity tests away from equilibrium."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return amp * rng.standard_normal((Q,) + tuple(shape))


def random_scalars(kind, shape, seed):
    """Smooth positive scalar fields for parity tests of the scalar solver."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nz, ny, nx = shape
    z = np.arange(nz)[:, None, None] / max(nz, 1)
    y = np.arange(ny)[None, :, None] / ny
    x = np.arange(nx)[None, None, :] / nx
    def smooth():
        a = rng.uniform(0, 2 * np.pi, 3)
        return (np.sin(2 * np.pi * x + a[0]) * np.cos(2 * np.pi * y + a[1])
                * np.cos(2 * np.pi * z + a[2]))
    noise = lambda s: s * rng.standard_normal(shape)
    if kind == "passive":
        return np.stack([smooth() + noise(0.05)])
    if kind == "one_step":
        th = np.clip(0.5 + 0.45 * smooth() + noise(0.02), 0.0, 1.0)
        return np.stack([300.0 + 1700.0 * th, np.clip(1 - th + noise(0.01), 0, 1)])
    if kind == "two_step":
        yf, yo, yn = fresh_ch4_air(0.83)
        th = np.clip(0.5 + 0.45 * smooth() + noise(0.02), 0.0, 1.0)
        b = burnt_ch4_air(0.83)
        T = 320.0 + 1630.0 * th
        return np.stack([T, yf * (1 - th), yo * (1 - th) + b["O2"] * th,
                         0.01 * th * (1 - th) * 4, b["CO2"] * th * 0.9, b["H2O"] * th])
    raise ValueError(kind)
