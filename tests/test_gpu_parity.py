"""Parity of the HIP library (called through the C ABI) with the FP64 oracle.

Tolerances: FP64 populations and fields agree to 1e-12 of their scale (the
oracle and the kernels round differently, e.g. fused multiply-adds).  An FP64
velocity is a difference of populations of size ~w_i rho, so after T steps its
rounding error is ~T Q eps max f (about 1e-13 here) whatever |u| is: it is
compared against the lattice sound speed c_s = 1/sqrt(3) as its scale.  FP32
deviation storage agrees to 1e-5 of the field scale (max over fluid nodes of
|gpu - oracle| / max |oracle|; u scaled by max |u|, C by max(|C|, C_eq)), and
the solid fraction's change phi - phi0 to 1e-5 of its largest value.  Node
classes (solid / fluid) and the set of reactive links must match exactly.
"""
import math

import numpy as np
import pytest

from lbm_inputs import (Case, configs, geometry, MECH_PRE, MECH_POST, SCHEME_SNEW, SCHEME_SV,
                        SCHEME_SPJ, SCHEME_ABB)

from parity import log, rel_errors, run_pair

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}
CS = 3 ** -0.5   # lattice sound speed: the FP64 velocity scale


def _assert_parity(case, precision, steps, name=None, tol=None):
    res = run_pair(case, precision, steps, name)
    err = rel_errors(res, case, u_floor=CS if precision == FP64 else 0.0)
    log(f"[parity] errors {err}")
    t = tol if tol is not None else TOL[precision]
    assert err["type"] == 0
    assert err["link_set"] == 0
    for k in ("rho", "u", "c", "f", "g", "q", "phi"):
        assert err[k] <= t, (k, err[k])
    return res


def _tilted(n=100, shift=58, width=40.0, pe=10.0, da=1.0, aligned=False):
    return configs.tilted_channel(pe=pe, da=da, n=n, shift=shift, width=width,
                                  aligned=aligned, steps=0)


def _spheres(nx=30, ny=28, nz=26, seed=7, porosity=0.6, inlet=True):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, [nx, ny, nz], size=(10, 3))
    radii = rng.uniform(2.5, 5.0, size=10)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = np.zeros((nz, ny, nx), np.uint8)
    normals = np.zeros((nz, ny, nx, 3))
    depth = np.full((nz, ny, nx), np.inf)
    for c, r in zip(centres, radii):
        d = np.stack([x - c[0], y - c[1], z - c[2]], -1)
        for a, n in enumerate((nx, ny, nz)):
            d[..., a] -= n * np.round(d[..., a] / n)
        dist = np.sqrt((d ** 2).sum(-1))
        inside = (dist <= r) & (r - dist < depth)
        solid[inside] = 1
        depth[inside] = (r - dist)[inside]
        normals[inside] = d[inside] / np.maximum(dist[inside], 1e-12)[:, None]
    return Case(name="spheres", dim=3, nx=nx, ny=ny, nz=nz, q=19, solid=solid, normals=normals,
                tau_ns=0.9, tau_ad=0.8, j0=0.6, force=(0.0, 0.0, 2e-5), c_eq=1.0, k_r=2e-2,
                v_m=0.1, inlet_axis=2 if inlet else -1, c_in=2.0, c0=1.0, c_ref=1.0)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mech,scheme", [(MECH_PRE, SCHEME_SNEW), (MECH_POST, SCHEME_SV)])
def test_reactive_channel_fp64(mech, scheme):
    """64 x 32 reactive channel (pure diffusion), FP64."""
    _assert_parity(configs.robin_channel(mechanics=mech, scheme=scheme), FP64, 600)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_tilted_channel_flow(precision):
    """Tilted band (30 deg, shifted-periodic x wrap) with Poiseuille flow,
    rest-fraction solute and dissolution from the walls; N = 10000 (ragged
    last tile)."""
    _assert_parity(_tilted(), precision, 300)


@pytest.mark.parametrize("dim", [2, 3])
def test_fp32_long_run_steady_channel(dim):
    """FP32 deviation storage over a run long enough for a force-driven
    channel with reactive walls (H = 62 fluid rows) to approach its steady
    profile (12,000 steps, about half the viscous time H^2/nu).  A relative
    bias b in the momentum or mass that each collision returns (lattice
    weights rounded to FP32 and used as they are, for instance) acts at every
    step; near steady state it shifts the velocity by about omega b H^2/(8 nu),
    several 1e-5 for b = 3e-8.  Short runs cannot tell a biased FP32 collision
    from an unbiased one; this one can."""
    h = 62
    nx, ny, nz, q = (4, h + 2, 1, 9) if dim == 2 else (4, h + 2, 4, 19)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, -1, :] = 1
    nu = (1.0 - 0.5) / 3.0
    force = 0.04 * 8.0 * nu / h ** 2   # centre-line velocity 0.04
    case = Case(name=f"long channel {dim}D", dim=dim, nx=nx, ny=ny, nz=nz, q=q, solid=solid,
                tau_ns=1.0, tau_ad=0.9, j0=0.3 if dim == 2 else -1.0, force=(force, 0.0, 0.0),
                c_eq=1.0, k_r=2e-3, v_m=0.05, c0=0.2, c_ref=0.5)
    _assert_parity(case, FP32, 12000)


@pytest.mark.parametrize("dim,collision,qs", [(2, 1, 5), (3, 1, 0), (3, 0, 7)])
def test_fp32_long_run_steady_channel_variants(dim, collision, qs):
    """The same 12,000-step bias check for the TRT collision and the reduced
    solute sets (D2Q5 / D3Q7), each a separate kernel instantiation with its
    own arithmetic."""
    h = 62
    nx, ny, nz, q = (4, h + 2, 1, 9) if dim == 2 else (4, h + 2, 4, 19)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, -1, :] = 1
    nu = (1.0 - 0.5) / 3.0
    force = 0.04 * 8.0 * nu / h ** 2
    case = Case(name=f"long channel {dim}D collision {collision} qs {qs}", dim=dim, nx=nx, ny=ny,
                nz=nz, q=q, qs=qs, solid=solid, tau_ns=1.0, tau_ad=0.9, j0=0.3,
                force=(force, 0.0, 0.0), c_eq=1.0, k_r=2e-3, v_m=0.05, c0=0.2, c_ref=0.5,
                collision=collision)
    _assert_parity(case, FP32, 12000)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_spheres_3d_inlet_outlet(precision):
    """3D D3Q19 sphere pack with an inlet and a zero-gradient outlet on z,
    ragged 30 x 28 x 26 box."""
    _assert_parity(_spheres(), precision, 120)


@pytest.mark.parametrize("scheme", [SCHEME_SV, SCHEME_SPJ, SCHEME_ABB])
@pytest.mark.parametrize("mech", [MECH_PRE, MECH_POST])
def test_schemes_disk_medium(scheme, mech):
    solid, normals, _ = geometry.disk_medium(70, 44, 0.6, 3.0, 8.0, seed=21)
    rng = np.random.default_rng(5)
    case = Case(name="disks", dim=2, nx=70, ny=44, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=0.8, tau_ad=0.9, j0=0.2, force=(1e-5, 0, 0), c_eq=1.0,
                k_r_field=rng.uniform(0, 0.05, solid.size), v_m=0.5, mechanics=mech,
                scheme=scheme, c_init=rng.uniform(0.0, 2.0, solid.size))
    _assert_parity(case, FP64, 150)


def test_random_solid_gaps_and_fd_normals():
    """30% random solid sites: one-node gaps (pre-collision fallback), corners,
    isolated fluid nodes; normals from the lattice gradient of the indicator."""
    rng = np.random.default_rng(9)
    solid = (rng.uniform(size=(1, 37, 53)) < 0.3).astype(np.uint8)
    case = Case(name="noise", dim=2, nx=53, ny=37, nz=1, q=9, solid=solid, normals=None,
                tau_ns=0.9, tau_ad=0.7, j0=-1.0, c_eq=1.0, k_r=0.03, v_m=1.0,
                c_init=rng.uniform(0.0, 1.0, solid.size))
    _assert_parity(case, FP64, 100)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_isolated_solid_voxels_many_links(precision):
    """Single solid voxels on every third site, each with 18 reactive links:
    the solid-side kernel gathers more than its 512-link round per wavefront
    of 64 solid nodes (1,152 links: three rounds), and every node's sum
    straddles a round boundary somewhere; dissolution lowers each voxel's
    phi every step."""
    n = 24
    solid = np.zeros((n, n, n), np.uint8)
    solid[1::3, 1::3, 1::3] = 1
    rng = np.random.default_rng(14)
    case = Case(name="voxels", dim=3, nx=n, ny=n, nz=n, q=19, solid=solid, normals=None,
                tau_ns=0.9, tau_ad=0.7, j0=0.5, c_eq=1.0, k_r=0.05, v_m=1.0,
                c_init=rng.uniform(0.0, 0.5, solid.size))
    log(f"[parity] isolated voxels precision={precision} solid={int(solid.sum())}")
    _assert_parity(case, precision, 60)


def test_open_box_walls_fp64():
    """Non-periodic box faces act as plain bounce-back walls for both lattices."""
    rng = np.random.default_rng(10)
    solid = np.zeros((9, 11, 13), np.uint8)
    solid[3:6, 4:7, 5:9] = 1
    normals = np.zeros((9, 11, 13, 3))
    normals[..., 0] = 1.0
    case = Case(name="box", dim=3, nx=13, ny=11, nz=9, q=19, solid=solid, normals=normals,
                tau_ns=0.8, tau_ad=0.75, force=(1e-4, 0, 0), c_eq=0.5, k_r=0.05, v_m=1.0,
                periodic=(0, 0, 0), c_init=rng.uniform(0, 1, solid.size))
    _assert_parity(case, FP64, 80)


def test_all_fluid_periodic_and_column():
    """No reactive link at all, and a one-node-wide periodic column."""
    rng = np.random.default_rng(11)
    solid = np.zeros((1, 17, 19), np.uint8)
    case = Case(name="free", dim=2, nx=19, ny=17, nz=1, q=9, solid=solid, tau_ns=0.7,
                tau_ad=1.1, j0=0.5, force=(1e-5, -2e-5, 0), c_init=rng.uniform(0, 1, solid.size))
    _assert_parity(case, FP64, 60)
    col = Case(name="column", dim=2, nx=1, ny=12, nz=1, q=9, solid=np.zeros((1, 12, 1), np.uint8),
               tau_ad=0.8, c_init=rng.uniform(0, 1, 12))
    _assert_parity(col, FP64, 40)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_all_solid_lattice_and_zero_steps(precision):
    """The degenerate lattices: no fluid node at all (no task, link or solid
    interface node; every field as the oracle's), and a step count of zero
    (the populations unchanged bit for bit)."""
    import torch
    from oracle import Oracle
    from paper_2306_10794_amd import Simulation
    solid = np.ones((1, 10, 12), np.uint8)
    rock = Case(name="rock", dim=2, nx=12, ny=10, nz=1, q=9, solid=solid, tau_ad=0.8,
                k_r=0.01, c_eq=1.0, v_m=0.1)
    log(f"[parity] all-solid 12x10 precision={precision}")
    sim = Simulation(rock, precision=precision)
    sim.step(5)
    torch.cuda.synchronize()
    d = sim.diag()
    assert d["status"] == 0 and d["n_links"] == 0
    fg = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    qg = sim.exchange().cpu().numpy()
    sim.close()
    ora = Oracle(rock)
    ora.step(5)
    fo = ora.fields()
    for k in ("phi", "type"):   # the fields a solid node carries
        assert np.array_equal(np.asarray(fg[k], np.float64).reshape(fo[k].shape), fo[k]), k
    for k in ("rho", "u", "c"):
        assert np.isfinite(fg[k]).all(), k
    assert not qg.any()
    rng = np.random.default_rng(12)
    solid2 = np.zeros((1, 16, 20), np.uint8)
    solid2[0, 5:9, 6:11] = 1
    case = Case(name="zero steps", dim=2, nx=20, ny=16, nz=1, q=9, solid=solid2, tau_ad=0.9,
                k_r=0.02, c_eq=1.0, c_init=rng.uniform(0, 1, solid2.size))
    sim = Simulation(case, precision=precision)
    sim.step(3)
    f0, g0 = (t.cpu().numpy().copy() for t in sim.pops())
    sim.step(0)
    f1, g1 = (t.cpu().numpy() for t in sim.pops())
    torch.cuda.synchronize()
    assert np.array_equal(f0, f1) and np.array_equal(g0, g1)
    assert sim.diag()["status"] == 0
    sim.close()


def test_linear_robin_steady_on_gpu():
    """The exact linear steady state (inlet + reactive wall) reproduced by the
    library itself in FP64."""
    import torch
    from paper_2306_10794_amd import Simulation
    from analytic import linear_robin_steady
    case = configs.robin_1d(ny_fluid=20, tau_ad=0.8, k_r=2e-2)
    sim = Simulation(case, precision=FP64)
    sim.step(40000)
    c = sim.fields()["c"].cpu().numpy().reshape(case.ny, case.nx)[:-1]
    exact = linear_robin_steady(case.ny - 1, 0.8, 1 / 3, 2e-2, case.c_in, case.c_eq, 0.0)
    assert np.abs(c - exact[:, None]).max() < 1e-11


def test_mass_invariant_and_diag_fp64():
    """sum C + sum phi / V_m is invariant and the device reductions agree with
    the oracle's."""
    solid, normals, _ = geometry.disk_medium(64, 48, 0.65, 3.0, 7.0, seed=12)
    rng = np.random.default_rng(6)
    case = Case(name="mass", dim=2, nx=64, ny=48, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=0.8, tau_ad=0.75, j0=0.2, force=(2e-5, 0, 0), c_eq=1.0, k_r=0.03,
                v_m=0.3, c_init=rng.uniform(0.0, 2.0, solid.size))
    res = _assert_parity(case, FP64, 200)
    d, do = res["gpu"]["diag"], res["ora"]["diag"]
    assert d["status"] == 0
    assert d["mass_c"] == pytest.approx(do["mass_c"], rel=1e-12)
    assert d["phi_sum"] == pytest.approx(do["phi_sum"], rel=1e-12)
    assert d["wall_exchange"] == pytest.approx(do["wall_exchange"], rel=1e-10, abs=1e-13)


def _plane_case(axis):
    """A 2D disk medium with an inlet and an outlet along x (axis 0: every
    task mixes plane and interior nodes) or y (axis 1: tasks span rows, some
    on the planes), or the 3D sphere pack along z (whole tasks on a plane)."""
    if axis == 2:
        return _spheres()
    solid, normals, _ = geometry.disk_medium(45, 38, 0.7, 2.5, 5.0, seed=31 + axis)
    if axis == 1:
        # the channel turned by 90 degrees: walls at x = 0 and x = nx - 1
        solid = np.ascontiguousarray(solid[0].T[None])
        nt = np.zeros((1, 45, 38, 3))
        nt[0, :, :, 0] = normals[0, :, :, 1].T
        nt[0, :, :, 1] = normals[0, :, :, 0].T
        normals = nt
    nx, ny = (45, 38) if axis == 0 else (38, 45)
    rng = np.random.default_rng(40 + axis)
    force = (1e-5, 0, 0) if axis == 0 else (0, 1e-5, 0)
    per = (0, 1, 1) if axis == 0 else (1, 0, 1)
    return Case(name=f"planes{axis}", dim=2, nx=nx, ny=ny, nz=1, q=9, solid=solid,
                normals=normals, tau_ns=0.8, tau_ad=0.7, j0=0.3, force=force, periodic=per,
                c_eq=1.0, k_r=0.02, v_m=0.2, inlet_axis=axis, c_in=1.7,
                c_init=rng.uniform(0.5, 1.5, solid.size))


@pytest.mark.parametrize("axis,precision", [(0, FP64), (1, FP64), (2, FP64), (2, FP32), (0, FP32)])
def test_inlet_outlet_exchange_matches_oracle(axis, precision):
    """lbm_get_diag's cumulative inlet and outlet exchange against the
    oracle's, and the mass budget they close (Sec. 2.4, eq.
    solidFractionUpdate): sum C + sum phi / V_m changes by exactly the
    inlet plus the outlet exchange."""
    case = _plane_case(axis)
    res = _assert_parity(case, precision, 150, name=f"planes axis {axis}")
    d, do = res["gpu"]["diag"], res["ora"]["diag"]
    from oracle import Oracle
    d0 = Oracle(case).diag()
    log(f"[parity] inlet {d['inlet_exchange']:.15e} / {do['inlet_exchange']:.15e}, outlet "
        f"{d['outlet_exchange']:.15e} / {do['outlet_exchange']:.15e}")
    # scale: the mass that entered (the outlet's net is a small difference of
    # the populations crossing it, whose FP32 rounding the inlet's size sets)
    tol = 1e-12 if precision == FP64 else 1e-5
    scale = abs(do["inlet_exchange"])
    for k in ("inlet_exchange", "outlet_exchange"):
        assert abs(do[k]) > 1e-3
        assert abs(d[k] - do[k]) <= tol * scale, k
    tot = lambda x: x["mass_c"] + x["phi_sum"] / case.v_m
    budget = d["inlet_exchange"] + d["outlet_exchange"]
    assert tot(d) - tot(d0) == pytest.approx(budget, rel=1e-12 if precision == FP64 else 1e-5)


def test_fp32_phi_accumulation_is_fp64():
    """In FP32 storage the solid fraction is still accumulated in FP64: the
    device phi equals a host FP64 re-accumulation of the exported per-link
    exchange of one step, node by node, in link order."""
    import torch
    from paper_2306_10794_amd import Simulation
    case = _tilted(n=64, shift=37, width=24.0)
    sim = Simulation(case, precision=FP32)
    sim.step(50)
    phi_a = sim.fields()["phi"].cpu().numpy()
    sim.step(1)
    q = sim.exchange().cpu().numpy()
    phi_b = sim.fields()["phi"].cpu().numpy()
    torch.cuda.synchronize()
    # rebuild the step's update on the host
    solid = case.solid_flat() == 1
    expect = phi_a.copy()
    neg = np.where(q < 0, -q, 0.0)
    for n in np.nonzero(~solid & (np.abs(q).sum(1) > 0))[0]:
        s = 0.0
        for i in range(1, 9):
            s += neg[n, i]
        expect[n] += case.v_m * s
    changed = ~solid
    assert np.abs(phi_b[changed] - expect[changed]).max() <= 1e-15


def test_save_load_resume_bitwise():
    import torch
    from paper_2306_10794_amd import Simulation
    case = _tilted(n=64, shift=37, width=24.0)
    sim = Simulation(case, precision=FP32)
    sim.step(40)
    buf = sim.save_state()
    sim.step(40)
    fa, ga = (t.cpu().numpy() for t in sim.pops())
    pa = sim.fields()["phi"].cpu().numpy()
    sim.load_state(buf)
    sim.step(40)
    fb, gb = (t.cpu().numpy() for t in sim.pops())
    pb = sim.fields()["phi"].cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb) and np.array_equal(pa, pb)


def test_nonfinite_state_reported():
    """An unstable parameter set yields LBM_ENUMERIC from lbm_get_diag."""
    from paper_2306_10794_amd import Simulation
    solid = np.zeros((1, 16, 16), np.uint8)
    u = np.zeros((256, 3))
    u[:, 0] = 0.4
    case = Case(name="unstable", dim=2, nx=16, ny=16, nz=1, q=9, solid=solid, tau_ns=0.5001,
                tau_ad=0.5001, j0=0.99, u_init=u, c_init=np.linspace(0, 1, 256))
    sim = Simulation(case, precision=FP32)
    sim.step(3000)
    d = sim.diag()
    assert d["status"] == -5 and d["nan_flag"] == 1


def test_capacity_error():
    from paper_2306_10794_amd import Simulation, LbmError
    solid = np.zeros((1, 128, 128), np.uint8)
    solid[:, ::2, :] = 1
    case = Case(name="cap", dim=2, nx=128, ny=128, nz=1, q=9, solid=solid)
    with pytest.raises(LbmError) as ei:
        Simulation(case, precision=FP64, max_links=4096)
    assert ei.value.status == -6


def test_invalid_pointer_rejected():
    """A host pointer where the ABI wants device memory is an argument error.
    (Pinned host memory is used so that even a wrong acceptance could not
    fault the device.)"""
    import torch
    from paper_2306_10794_amd import Simulation, LbmError, _lib
    case = configs.robin_channel()
    sim = Simulation(case, precision=FP64)
    host = torch.zeros(case.n, dtype=torch.float64, pin_memory=True)
    with pytest.raises(LbmError) as ei:
        _lib.lbm_get_fields(sim.ctx, host.data_ptr())
    assert ei.value.status == -1


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_wide_rows_3d(precision):
    """Rows of 10 words (600 wide): tasks hold a window of row words instead of
    whole rows; random spheres, an inlet and periodic x wrap."""
    rng = np.random.default_rng(21)
    nx, ny, nz = 600, 10, 12
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = np.zeros((nz, ny, nx), np.uint8)
    normals = np.zeros((nz, ny, nx, 3))
    for c, r in zip(rng.uniform(0, [nx, ny, nz], size=(60, 3)), rng.uniform(2.0, 4.5, size=60)):
        d = np.stack([x - c[0], y - c[1], z - c[2]], -1)
        for a, n in enumerate((nx, ny, nz)):
            d[..., a] -= n * np.round(d[..., a] / n)
        dist = np.sqrt((d ** 2).sum(-1))
        inside = dist <= r
        solid[inside] = 1
        normals[inside] = d[inside] / np.maximum(dist[inside], 1e-12)[:, None]
    case = Case(name="wide3d", dim=3, nx=nx, ny=ny, nz=nz, q=19, solid=solid, normals=normals,
                tau_ns=0.9, tau_ad=0.8, j0=0.5, force=(2e-5, 0.0, 0.0), c_eq=1.0, k_r=2e-2,
                v_m=0.1, inlet_axis=2, c_in=2.0, c0=1.0, c_ref=1.0)
    _assert_parity(case, precision, 80)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_wide_rows_2d_tilted(precision):
    """A 1500-wide tilted band (24 words per row, shifted x wrap, Poiseuille
    flow, dissolution from the walls)."""
    case = configs.tilted_channel(pe=10.0, da=1.0, n=1500, shift=866, width=60.0, steps=0)
    _assert_parity(case, precision, 60)
