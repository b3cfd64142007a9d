"""The workloads, as seeded synthetic ``Case`` objects.

The dimensionless groups are Re = U L / nu, Pe = U L / D, Da = k_r / U and
PeDa = k_r L / D (paper, definitions of the dimensionless numbers), with
D = c_s^2 (tau_AD - 1/2) and the rest fraction J0 chosen so that c_s^2 gives the
wanted D at fixed tau_AD (paper, rest fraction method; generalised to D2Q9 and
D3Q19 as c_s^2 = (1/3)(1 - J0)/(1 - w0_std)).
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from .case import Case, MECH_PRE, SCHEME_SNEW
from . import geometry


def j0_for_cs2(q: int, cs2: float) -> float:
    """Rest fraction giving squared sound speed cs2 on the generalised lattice."""
    w0 = 4.0 / 9.0 if q == 9 else 1.0 / 3.0
    return 1.0 - cs2 * 3.0 * (1.0 - w0)


def j0_reduced_for_cs2(dim: int, cs2: float) -> float:
    """Rest fraction giving cs2 on D2Q5 / D3Q7 (c_s^2 = (1 - J0)/dim)."""
    return 1.0 - dim * cs2


def with_reduced_solute(case):
    """The same workload with the solute on D2Q5 / D3Q7 at the same c_s^2
    (so the same diffusivity at the same tau_AD)."""
    w0 = 4.0 / 9.0 if case.q == 9 else 1.0 / 3.0
    cs2 = 1.0 / 3.0 if case.j0 < 0 else (1.0 - case.j0) / (3.0 * (1.0 - w0))
    return case.replace(qs=5 if case.q == 9 else 7, j0=j0_reduced_for_cs2(case.dim, cs2),
                        name=case.name + ("_d2q5" if case.q == 9 else "_d3q7"))


# --------------------------------------------------------------------------
# workload 0: 64 x 32 reactive channel, pure diffusion, FP64
# --------------------------------------------------------------------------
def robin_channel(nx=64, ny=32, tau_ad=0.8, k_r=1e-3, c_eq=1.0, steps=2000,
                  mechanics=MECH_PRE, scheme=SCHEME_SNEW) -> Case:
    solid, normals = geometry.plane_channel(nx, ny, (0, ny - 1))
    return Case(name=f"robin_channel_{nx}x{ny}", dim=2, nx=nx, ny=ny, nz=1, q=9,
                solid=solid, normals=normals, tau_ns=1.0, tau_ad=tau_ad, j0=-1.0,
                c_eq=c_eq, k_r=k_r, v_m=1.0, periodic=(1, 1, 1), c0=0.0, c_ref=0.0,
                mechanics=mechanics, scheme=scheme, steps=steps)


def robin_1d(ny_fluid=24, nx=3, tau_ad=0.8, k_r=2e-2, c_eq=1.0, c_in=0.25,
             mechanics=MECH_PRE, scheme=SCHEME_SNEW) -> Case:
    """Column with a fixed-concentration inlet plane below row 0 and a reactive
    solid row on top; periodic in x.  Used for the exact linear steady state."""
    ny = ny_fluid + 1
    solid = np.zeros((1, ny, nx), np.uint8)
    solid[0, ny - 1, :] = 1
    normals = np.zeros((1, ny, nx, 3))
    normals[0, ny - 1, :, 1] = -1.0
    return Case(name="robin_1d", dim=2, nx=nx, ny=ny, nz=1, q=9, solid=solid,
                normals=normals, tau_ns=1.0, tau_ad=tau_ad, c_eq=c_eq, k_r=k_r,
                v_m=0.0, periodic=(1, 0, 1), inlet_axis=1, c_in=c_in, c0=c_in,
                mechanics=mechanics, scheme=scheme)


# --------------------------------------------------------------------------
# the paper's 2D reaction-diffusion verification, configuration A
# --------------------------------------------------------------------------
def reaction_diffusion_2d(peda=1.0, scheme=SCHEME_SNEW, a=100, b=80, pe=1.0, U=1e-3, c0=1.0,
                          c_eq=0.0, j0=-1.0, qs=5, collision=0, mechanics=MECH_PRE,
                          c_init=None) -> Case:
    """Configuration A of the paper's analytic reaction-diffusion case (its
    default parameter table): pure diffusion in an a x b box aligned with the
    grid; fixed concentration C0 on the left (the solute inlet plane at x = 0),
    zero gradient on the right (the outlet plane at x = a - 1) and at the
    bottom (a solid row with k_r = 0, i.e. bounce-back), the first-order
    reaction with C_eq on the top (a solid row with k_r).  D = U b / Pe, the
    solute on D2Q5 by default; tau_AD from D and c_s^2 = (1 - J0)/2 (J0 = 1/3
    when j0 < 0), k_r = PeDa D / b.  Fluid rows y = 1..b; solid rows 0 and
    b + 1."""
    D = U * b / pe
    if qs == 5:
        cs2 = (1.0 - (1.0 / 3.0 if j0 < 0 else j0)) / 2.0
    else:   # the solute on D2Q9
        cs2 = 1.0 / 3.0 if j0 < 0 else 3.0 * (1.0 - j0) / 5.0
    tau_ad = 0.5 + D / cs2
    k_r = peda * D / b
    ny = b + 2
    solid, normals = geometry.plane_channel(a, ny, (0, ny - 1))
    kr = np.zeros((1, ny, a))
    kr[0, ny - 1, :] = k_r
    return Case(name=f"rd2d_A_peda{peda:g}_s{scheme}", dim=2, nx=a, ny=ny, nz=1, q=9,
                qs=qs if qs != 9 else 0, solid=solid, normals=normals, tau_ns=1.0, tau_ad=tau_ad,
                j0=j0, c_eq=c_eq, k_r=0.0, k_r_field=kr.reshape(-1), v_m=0.0,
                periodic=(1, 0, 1), inlet_axis=0, c_in=c0, c0=c0, c_init=c_init,
                mechanics=mechanics, scheme=scheme, collision=collision,
                info=dict(D=D, k_r=k_r, cs2=cs2, a=a, b=b, peda=peda))


# --------------------------------------------------------------------------
# the paper's reactive object in a channel flow (Molins et al.'s benchmark)
# --------------------------------------------------------------------------
MOLINS_CASES = {1: (600.0, 178.0), 2: (600.0, 17800.0), 3: (6.0, 178.0), 4: (6.0, 0.178)}


def reactive_cylinder(case=4, scheme=SCHEME_SNEW, scale=4, re=0.6, collision=1, c_in=0.0,
                      c_eq=1.0) -> Case:
    """The paper's channel-flow case: a 600 x 1200 channel (H = 0.05 cm,
    W = 0.1 cm) with a reactive cylinder of diameter 240 (0.02 cm) in its
    middle, plug inflow and fixed outlet density, Re = 0.6, Pe and Da of the
    paper's four cases with the channel height as the length (Re = U H / nu,
    Pe = U H / D, Da = k_r / U: with H = 0.05 cm and u_in = 0.12 cm/s these
    give water's viscosity and D = 1e-5 cm^2/s at Pe = 600), J0 = 0.99 at
    Pe = 600 and 1/3 at Pe = 6 on a D2Q5 solute, TRT.  Lengths
    are divided by ``scale`` and the lattice velocity 0.001 multiplied by it,
    which keeps both relaxation times.  Walls: solid rows below and above the
    H fluid rows (k_r = 0); the cylinder's solid nodes carry k_r."""
    pe, da = MOLINS_CASES[case]
    H, W, d = 600 // scale, 1200 // scale, 240.0 / scale
    U = 0.001 * scale
    nu = U * H / re
    Dm = U * H / pe
    j0 = 0.99 if pe > 100 else 1.0 / 3.0
    cs2 = (1.0 - j0) / 2.0
    ny = H + 2
    y, x = np.mgrid[0:ny, 0:W].astype(np.float64)
    cx, cy = W / 2.0 - 0.5, ny / 2.0 - 0.5
    r = np.hypot(x - cx, y - cy)
    cyl = r <= d / 2.0
    solid = np.zeros((1, ny, W), np.uint8)
    solid[0, 0, :] = solid[0, ny - 1, :] = 1
    solid[0][cyl] = 1
    normals = np.zeros((1, ny, W, 3))
    normals[0, 0, :, 1], normals[0, ny - 1, :, 1] = 1.0, -1.0
    rr = np.maximum(r, 1e-12)
    normals[0, :, :, 0] = np.where(cyl, (x - cx) / rr, normals[0, :, :, 0])
    normals[0, :, :, 1] = np.where(cyl, (y - cy) / rr, normals[0, :, :, 1])
    kr = np.where(cyl, da * U, 0.0)[None]
    return Case(name=f"molins_case{case}_s{scheme}_1over{scale}", dim=2, nx=W, ny=ny, nz=1, q=9,
                qs=5, solid=solid, normals=normals, tau_ns=0.5 + 3.0 * nu, tau_ad=0.5 + Dm / cs2,
                j0=j0, c_eq=c_eq, k_r=0.0, k_r_field=kr.reshape(-1), v_m=0.0, periodic=(0, 1, 1),
                inlet_axis=0, c_in=c_in, c0=c_in, scheme=scheme, collision=collision,
                fluid_open=1, u_in=U, rho_out=1.0,
                info=dict(pe=pe, da=da, H=H, W=W, d=d, U=U, case=case))


def reactive_cylinder_rate(case, c, ux):
    """R_avg of the paper's channel case in lattice units: (outlet flux of C
    minus inlet flux) / (pi d), from the concentration and velocity fields of
    the fluid rows [ny, nx] (the outlet column is the last one)."""
    inf = case.info
    return ((c[1:-1, -1] * ux[1:-1, -1]).sum() - case.c_in * inf["U"] * inf["H"]) / (math.pi * inf["d"])


# --------------------------------------------------------------------------
# the paper's pattern formation during precipitation
# --------------------------------------------------------------------------
def grain_growth(rot_deg=0.0, scheme=SCHEME_SNEW, n=300, v_m=0.2, k_r=0.0014, c0=1.0) -> Case:
    """The paper's precipitation case: a circular domain of diameter n whose
    rim holds C = 1 (solid nodes outside the circle reacting toward C_eq = 1
    with a rate so large that the rim is anti-bounce-back), and a seed in the
    centre with the boundary r(theta) = n (0.1 + 0.02 cos 4 theta), turned
    clockwise by rot_deg, reacting toward C_eq = 0 with k_r = 0.0014; pure
    diffusion on D2Q5 (tau_AD = 1), precipitation with phase change, wall
    normals from the isotropic lattice gradient (none given).  The solute
    starts at c0.  V_m (not given by the paper) sets the growth speed."""
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    c = (n - 1) / 2.0
    r = np.hypot(x - c, y - c)
    th = np.arctan2(y - c, x - c) + math.radians(rot_deg)
    seed = r <= n * (0.1 + 0.02 * np.cos(4.0 * th))
    rim = r > n / 2.0 - 1.0
    solid = (seed | rim).astype(np.uint8)[None]
    kr = np.where(rim, 1e3, k_r)
    ceq = np.where(rim, 1.0, 0.0)
    return Case(name=f"grain_s{scheme}_{rot_deg:g}deg", dim=2, nx=n, ny=n, nz=1, q=9, qs=5,
                solid=solid, tau_ns=1.0, tau_ad=1.0, c_eq=0.0, k_r=0.0, k_r_field=kr.reshape(-1),
                c_eq_field=ceq.reshape(-1), v_m=v_m, periodic=(1, 1, 1), c0=c0, phase_change=1,
                scheme=scheme, info=dict(seed=seed, rim=rim, rot=rot_deg))


# --------------------------------------------------------------------------
# workload 1: 512 x 512 tilted channel, Poiseuille flow + solute, Pe x Da sweep
# --------------------------------------------------------------------------
def channel_flow_params(pe: float, da: float, L: float, tau_ns: float, q: int = 9,
                        tau_ad: float = 1.0):
    nu = (tau_ns - 0.5) / 3.0
    U = min(0.01, pe * 0.3 / L)
    D = U * L / pe
    cs2 = D / (tau_ad - 0.5)
    return dict(U=U, D=D, nu=nu, F=12.0 * nu * U / (L * L), k_r=da * U,
                j0=j0_for_cs2(q, cs2), cs2=cs2, tau_ad=tau_ad)


def tilted_channel(pe=10.0, da=1.0, n=512, shift=296, width=256, aligned=False,
                   tau_ns=0.6, steps=20000, c_ref=0.5) -> Case:
    if aligned:
        L = math.hypot(n, shift)
        ny = int(round(n * n / L))
        solid, normals, info = geometry.tilted_band(n, ny, 0, width)
        nx = n
    else:
        solid, normals, info = geometry.tilted_band(n, n, shift, width)
        nx, ny = n, n
    p = channel_flow_params(pe, da, width, tau_ns)
    t = info["t"]
    d = info["d"][0]
    fluid = solid[0] == 0
    prof = np.where(fluid, p["F"] / (2 * p["nu"]) * d * (width - d), 0.0)
    u = np.zeros((1, ny, nx, 3))
    u[0, :, :, 0] = prof * t[0]
    u[0, :, :, 1] = prof * t[1]
    F = (p["F"] * t[0], p["F"] * t[1], 0.0)
    info.update(p)
    return Case(name=f"tilted_{'0' if aligned else '30'}deg_pe{pe:g}_da{da:g}", dim=2,
                nx=nx, ny=ny, nz=1, q=9, solid=solid, normals=normals, tau_ns=tau_ns,
                tau_ad=p["tau_ad"], j0=p["j0"], force=F, c_eq=1.0, k_r=p["k_r"],
                v_m=1.0, periodic=(1, 1, 1), xwrap_shift_y=0 if aligned else shift,
                u_init=u, c0=0.0, c_ref=c_ref, steps=steps, info=info)


def tilted_sweep(aligned=False, n=512, shift=296, width=256, steps=20000) -> List[Case]:
    return [tilted_channel(pe, da, n, shift, width, aligned, steps=steps)
            for pe in (1.0, 10.0, 100.0) for da in (0.1, 1.0, 10.0)]


# --------------------------------------------------------------------------
# workload 2: 256^3 sphere packing, pressure-driven flow, precipitation
# --------------------------------------------------------------------------
def sphere_precipitation(n=256, seed=3, porosity=0.40, r_min=8.0, r_max=16.0,
                         steps=10000, phase_change=1) -> Case:
    solid, normals, info = geometry.sphere_packing(n, r_min, r_max, porosity, seed)
    nu = 1.0 / 6.0
    D = nu / 1000.0
    cs2 = D / 0.5
    return Case(name=f"spheres_{n}^3_precip", dim=3, nx=n, ny=n, nz=n, q=19,
                solid=solid, normals=normals, tau_ns=1.0, tau_ad=1.0,
                j0=j0_for_cs2(19, cs2), force=(0.0, 0.0, 1e-5), c_eq=1.0, k_r=1e-2,
                v_m=0.1, periodic=(1, 1, 1), inlet_axis=2, c_in=2.0, c0=1.0,
                c_ref=1.0, phase_change=phase_change, steps=steps, info=info)


# --------------------------------------------------------------------------
# workload 3: 1024 uneven 2D flow + solute domains (batched sweep)
# --------------------------------------------------------------------------
def batch_domains(count=1024, seed=4, steps=5000, w_range=(32, 256), h_range=(32, 128),
                  tau_ns=0.8) -> List[Case]:
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(count):
        W = int(rng.integers(w_range[0], w_range[1] + 1))
        H = int(rng.integers(h_range[0], h_range[1] + 1))
        por = float(rng.uniform(0.5, 0.8))
        pe = 10.0 ** rng.uniform(-1.0, 2.0)
        da = 10.0 ** rng.uniform(-2.0, 2.0)
        gseed = int(rng.integers(0, 2 ** 31 - 1))
        solid, normals, info = geometry.disk_medium(W, H, por, 3.0, 12.0, gseed)
        p = channel_flow_params(pe, da, H, tau_ns)
        info.update(p, pe=pe, da=da)
        cases.append(Case(name=f"batch_{k}", dim=2, nx=W, ny=H, nz=1, q=9, solid=solid,
                          normals=normals, tau_ns=tau_ns, tau_ad=p["tau_ad"], j0=p["j0"],
                          force=(p["F"], 0.0, 0.0), c_eq=1.0, k_r=p["k_r"], v_m=1.0,
                          periodic=(1, 1, 1), c0=0.0, c_ref=0.5, steps=steps, info=info))
    return cases


# --------------------------------------------------------------------------
# workload 4: rate-field recovery by the adjoint (128^3 sphere packing)
# --------------------------------------------------------------------------
def lognormal_rate_field(solid: np.ndarray, seed: int, mu=math.log(1e-3), sigma=0.5):
    rng = np.random.default_rng(seed)
    return np.exp(rng.normal(mu, sigma, size=solid.size)) * solid.reshape(-1)


def rate_recovery(n=128, seed=5, porosity=0.45, r_min=8.0, r_max=16.0, steps=2000,
                  k_seed=51) -> Case:
    solid, normals, info = geometry.sphere_packing(n, r_min, r_max, porosity, seed)
    k = lognormal_rate_field(solid, k_seed)
    return Case(name=f"rate_recovery_{n}^3", dim=3, nx=n, ny=n, nz=n, q=19, solid=solid,
                normals=normals, tau_ns=1.0, tau_ad=0.8, j0=-1.0, c_eq=1.0, k_r=1e-3,
                k_r_field=k, v_m=0.0, periodic=(1, 1, 1), c0=0.0, c_ref=0.0,
                steps=steps, info=info)
