"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them compares the oracle with a
second copy of its own formulas: each uses a closed form, an invariant, a
limit stated in the paper, a value printed in the paper, or a different
computation (a Fourier matrix power) of the same linear dynamics.
"""
import math
import os

import numpy as np
import pytest

from lbm_inputs import (Case, configs, geometry, MECH_PRE, MECH_POST, SCHEME_SNEW, SCHEME_SV,
                        SCHEME_SPJ, SCHEME_ABB)
from oracle import Oracle

from analytic import linear_robin_steady, paper_2d_verification, plane_wall_robin

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small_case(**kw):
    solid, normals = geometry.plane_channel(8, 6, (0, 5))
    base = dict(name="t", dim=2, nx=8, ny=6, nz=1, q=9, solid=solid, normals=normals)
    base.update(kw)
    return Case(**base)


# --------------------------------------------------------------------------
# lattices
# --------------------------------------------------------------------------
def test_d2q9_matches_paper_table():
    """Velocity set and weights equal the paper's appendix table (golden file)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "d2q9_velocity_set.txt"))
    lat = Oracle(_small_case()).lattice()
    assert np.array_equal(lat["e"][:, :2], rows[:, 1:3].astype(int))
    assert np.allclose(lat["wf"], rows[:, 3] / rows[:, 4], rtol=0, atol=1e-16)
    assert lat["cs2f"] == pytest.approx(1 / 3, abs=1e-16)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("j0", [-1.0, 0.0, 0.2, 0.6, 0.99933])
def test_lattice_moments_and_rest_fraction(q, j0):
    """Isotropy that fixes the weights: sum w = 1, sum w e = 0,
    sum w e e = c_s^2 I on both lattices, the fourth moment of the fluid
    lattice is c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc), and w_0 = J0 on the
    rest-fraction solute lattice (paper, eq. RestFraction)."""
    dim = 2 if q == 9 else 3
    if q == 9:
        case = _small_case(j0=j0)
    else:
        solid = np.zeros((3, 3, 3), np.uint8)
        case = Case(name="t", dim=3, nx=3, ny=3, nz=3, q=19, solid=solid, j0=j0)
    lat = Oracle(case).lattice()
    e = lat["e"][:, :dim].astype(float)
    I = np.eye(dim)
    for w, cs2 in ((lat["wf"], lat["cs2f"]), (lat["ws"], lat["cs2s"])):
        assert w.sum() == pytest.approx(1.0, abs=1e-15)
        assert np.abs(w @ e).max() < 1e-16
        assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), cs2 * I, atol=1e-15)
        assert (w >= 0).all()
    w4 = np.einsum("i,ia,ib,ic,id->abcd", lat["wf"], e, e, e, e)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I) +
           np.einsum("ad,bc->abcd", I, I)) / 9.0
    assert np.allclose(w4, iso, atol=1e-15)
    if j0 >= 0:
        assert lat["ws"][0] == j0


@pytest.mark.parametrize("q", [9, 19])
def test_rest_fraction_at_standard_weight_is_standard_lattice(q):
    """J0 equal to the standard rest weight reproduces the standard lattice
    (paper, rest fraction section: J0 = 1/3 on D2Q5 gives the usual values)."""
    w0 = 4 / 9 if q == 9 else 1 / 3
    if q == 9:
        a, b = _small_case(j0=-1.0), _small_case(j0=w0)
    else:
        solid = np.zeros((3, 3, 3), np.uint8)
        a = Case(name="t", dim=3, nx=3, ny=3, nz=3, q=19, solid=solid, j0=-1.0)
        b = a.replace(j0=w0)
    la, lb = Oracle(a).lattice(), Oracle(b).lattice()
    assert np.allclose(la["ws"], lb["ws"], rtol=0, atol=1e-16)
    assert lb["cs2s"] == pytest.approx(la["cs2s"], abs=1e-16)


# --------------------------------------------------------------------------
# bulk dynamics
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q,j0,tau,u", [
    (9, -1.0, 0.8, (0.0, 0.0, 0.0)),
    (9, 0.3, 1.3, (0.02, -0.01, 0.0)),
    (19, 0.6, 0.7, (0.01, 0.015, -0.02)),
])
def test_fourier_mode_matches_matrix_power(q, j0, tau, u):
    """One periodic Fourier mode of C under uniform flow evolves by the power of
    the Q x Q step matrix M(k) = (I - (I - E)/tau) diag(exp(-i k.e_i)) with
    E_ij = w_i (1 + e_i.u/c_s^2) (von Neumann analysis of the solute
    eqs. solute_BGK and solute_equilibrium_function).  The fluid stays exactly
    uniform, so u is the same at every node."""
    dim = 2 if q == 9 else 3
    n = (16, 12, 1) if dim == 2 else (8, 6, 10)
    solid = np.zeros((n[2], n[1], n[0]), np.uint8)
    N = solid.size
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    kv = np.array([2 * np.pi * 2 / n[0], 2 * np.pi * 1 / n[1], (2 * np.pi / n[2]) if dim == 3 else 0.0])
    phase = (kv[0] * x + kv[1] * y + kv[2] * z).reshape(-1)
    A, C0 = 0.3, 1.1
    c = C0 + A * np.cos(phase + 0.4)
    uu = np.tile(np.array(u, float), (N, 1))
    case = Case(name="f", dim=dim, nx=n[0], ny=n[1], nz=n[2], q=q, solid=solid, tau_ns=0.9,
                tau_ad=tau, j0=j0, c_init=c, u_init=uu)
    o = Oracle(case)
    lat = o.lattice()
    e, ws, cs2 = lat["e"].astype(float), lat["ws"], lat["cs2s"]
    steps = 25
    o.step(steps)
    _, g = o.pops()
    E = np.outer(ws * (1 + e @ np.array(u) / cs2), np.ones(q))
    S = np.diag(np.exp(-1j * (e @ kv)))
    M = (np.eye(q) - (np.eye(q) - E) / tau) @ S
    v0 = A * np.exp(0.4j) * ws * (1 + e @ np.array(u) / cs2)
    vn = np.linalg.matrix_power(M, steps) @ v0
    pred = C0 * ws[:, None] * (1 + e @ np.array(u) / cs2)[:, None] + \
        np.real(vn[:, None] * np.exp(1j * phase)[None, :])
    assert np.abs(g - pred).max() < 1e-12


@pytest.mark.parametrize("j0", [-1.0, 0.1, 0.7])
def test_diffusion_coefficient_from_mode_decay(j0):
    """A long-wavelength mode decays as exp(-D k^2 t) with
    D = c_s^2 (tau_AD - 1/2) (paper, eq. solute_BGK and the rest fraction
    relation D = (1 - J0)/dim (tau - 1/2), generalised to D2Q9 as
    c_s^2 = 3 (1 - J0)/5).  Accuracy O(k^2)."""
    nx, tau = 128, 0.9
    solid = np.zeros((1, 1, nx), np.uint8)
    x = np.arange(nx)
    k = 2 * np.pi / nx
    case = Case(name="d", dim=2, nx=nx, ny=1, nz=1, q=9, solid=solid, tau_ad=tau, j0=j0,
                c_init=1.0 + 0.1 * np.cos(k * x))
    o = Oracle(case)
    steps = 400
    o.step(steps)
    c = o.fields()["c"]
    amp = 2 * np.abs(np.fft.rfft(c - c.mean())[1]) / nx
    cs2 = 1 / 3 if j0 < 0 else 3 * (1 - j0) / 5
    D = cs2 * (tau - 0.5)
    assert amp / 0.1 == pytest.approx(math.exp(-D * k * k * steps), rel=2e-3)


@pytest.mark.parametrize("tau", [0.6, 0.5 + math.sqrt(3 / 16), 1.0])
def test_poiseuille_body_force(tau):
    """Force-driven channel flow between bounce-back walls: the bulk profile is
    exactly parabolic with curvature -F/nu, nu = c_s^2 (tau - 1/2)
    (eq. fluid_BGK_visc).  At (tau - 1/2)^2 = 3/16 the walls lie exactly
    halfway (the paper's statement on the magic parameter for BGK = TRT with
    equal rates), so the whole profile equals the parabola."""
    ny, nx, F = 18, 2, 1e-5
    solid, normals = geometry.plane_channel(nx, ny, (0, ny - 1))
    case = Case(name="p", dim=2, nx=nx, ny=ny, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=tau, force=(F, 0, 0))
    o = Oracle(case)
    o.step(30000)
    u = o.fields()["u"].reshape(ny, nx, 3)[1:-1, 0, 0]
    nu = (tau - 0.5) / 3
    d2 = u[2:] - 2 * u[1:-1] + u[:-2]
    assert np.allclose(d2, -F / nu, rtol=1e-9)
    if abs((tau - 0.5) ** 2 - 3 / 16) < 1e-12:
        y = np.arange(1, ny - 1)
        exact = F / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
        assert np.abs(u - exact).max() < 1e-10 * exact.max()


# --------------------------------------------------------------------------
# TRT collision
# --------------------------------------------------------------------------
COLL_BGK, COLL_TRT = 0, 1


@pytest.mark.parametrize("tau", [0.6, 1.7, 3.0])
def test_trt_poiseuille_walls_halfway_at_any_tau(tau):
    """TRT with the magic parameter 3/16 (eq. fluid_TRT_visc) places the
    bounce-back walls exactly halfway whatever tau+ is: the whole steady
    profile of a force-driven channel equals the parabola with walls at
    y = 1/2 and ny - 3/2.  BGK at the same tau does not (checked at 1.7)."""
    ny, nx, F = 18, 2, 1e-5
    solid, normals = geometry.plane_channel(nx, ny, (0, ny - 1))
    nu = (tau - 0.5) / 3
    y = np.arange(1, ny - 1)
    exact = F / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    steps = int(40 * ny * ny / nu) + 2000
    errs = {}
    for coll in (COLL_TRT, COLL_BGK) if tau == 1.7 else (COLL_TRT,):
        case = Case(name="p", dim=2, nx=nx, ny=ny, nz=1, q=9, solid=solid, normals=normals,
                    tau_ns=tau, force=(F, 0, 0), collision=coll)
        o = Oracle(case)
        o.step(steps)
        u = o.fields()["u"].reshape(ny, nx, 3)[1:-1, 0, 0]
        errs[coll] = np.abs(u - exact).max() / exact.max()
    assert errs[COLL_TRT] < 1e-9
    if COLL_BGK in errs:
        assert errs[COLL_BGK] > 1e-3


def test_trt_equals_bgk_when_the_rates_coincide():
    """At (tau - 1/2)^2 = 3/16 the TRT rates tau+ and tau- coincide and the
    operator is BGK (eqs. fluid_TRT and solute_TRT with equal rates): the same
    run agrees with the BGK run, flow, solute, reactive walls and force."""
    tau = 0.5 + math.sqrt(3 / 16)
    solid, normals, _ = geometry.disk_medium(40, 30, 0.65, 3.0, 6.0, seed=3)
    rng = np.random.default_rng(2)
    base = dict(name="trt", dim=2, nx=40, ny=30, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=tau, tau_ad=tau, j0=0.3, force=(2e-5, 1e-5, 0), c_eq=1.0, k_r=0.03,
                v_m=0.2, c_init=rng.uniform(0.0, 2.0, solid.size))
    a, b = Oracle(Case(**base, collision=COLL_TRT)), Oracle(Case(**base, collision=COLL_BGK))
    a.step(150)
    b.step(150)
    fa, ga = a.pops()
    fb, gb = b.pops()
    assert np.abs(fa - fb).max() < 1e-13
    assert np.abs(ga - gb).max() < 1e-13


@pytest.mark.parametrize("tau", [0.7, 1.2, 2.5])
def test_trt_diffusion_from_the_odd_rate(tau):
    """Solute TRT (eqs. solute_TRT, solute_TRT_visc): the odd parts relax with
    1/tau+ and D = c_s^2 (tau+ - 1/2), so a long-wavelength mode decays as
    exp(-D k^2 t) with D from tau_AD = tau+, not from tau- (which differs from
    tau+ at these tau)."""
    nx = 128
    solid = np.zeros((1, 1, nx), np.uint8)
    x = np.arange(nx)
    k = 2 * np.pi / nx
    case = Case(name="d", dim=2, nx=nx, ny=1, nz=1, q=9, solid=solid, tau_ad=tau,
                c_init=1.0 + 0.1 * np.cos(k * x), collision=COLL_TRT)
    o = Oracle(case)
    steps = 400
    o.step(steps)
    c = o.fields()["c"]
    amp = 2 * np.abs(np.fft.rfft(c - c.mean())[1]) / nx
    D = (tau - 0.5) / 3
    assert amp / 0.1 == pytest.approx(math.exp(-D * k * k * steps), rel=2e-3)


# --------------------------------------------------------------------------
# reduced solute lattices D2Q5 / D3Q7 (the paper's solute lattices)
# --------------------------------------------------------------------------
def _box3(n=(3, 3, 3), **kw):
    solid = np.zeros((n[2], n[1], n[0]), np.uint8)
    base = dict(name="t", dim=3, nx=n[0], ny=n[1], nz=n[2], q=19, solid=solid)
    base.update(kw)
    return Case(**base)


def test_d2q5_matches_paper_table():
    """The solute set of a D2Q5 run is the paper's D2Q5 (appendix, velocity
    sets; golden file) in the paper's order, with its weights 1/3, 1/6 and
    c_s^2 = 1/3 when no rest fraction is set."""
    rows = np.loadtxt(os.path.join(GOLDEN, "d2q5_velocity_set.txt"))
    o = Oracle(_small_case(qs=5))
    lat = o.lattice()
    sd = lat["sd"]
    assert o.QS == 5
    assert np.array_equal(lat["e"][sd, :2], rows[:, 1:3].astype(int))
    assert np.allclose(lat["ws"][sd], rows[:, 3] / rows[:, 4], rtol=0, atol=1e-16)
    assert lat["cs2s"] == pytest.approx(1 / 3, abs=1e-16)
    outside = np.setdiff1d(np.arange(9), sd)
    assert (lat["ws"][outside] == 0).all()


@pytest.mark.parametrize("q,qs", [(9, 5), (19, 7)])
@pytest.mark.parametrize("j0", [-1.0, 0.0, 0.25, 0.6, 0.99])
def test_reduced_lattice_moments_and_rest_fraction(q, qs, j0):
    """D2Q5 / D3Q7: the solute set is the rest vector plus the 2 dim unit
    vectors; sum w = 1, sum w e = 0, sum w e e = c_s^2 I; with a rest fraction
    w_0 = J0 and c_s^2 = (1 - J0)/dim (eqs. RestFraction, RestFractionCs2),
    without one the common lattice (J0 = 1/3 in 2D, 1/4 in 3D)."""
    dim = 2 if q == 9 else 3
    case = _small_case(j0=j0, qs=qs) if q == 9 else _box3(j0=j0, qs=qs)
    o = Oracle(case)
    lat = o.lattice()
    sd = lat["sd"]
    e = lat["e"][sd, :dim].astype(float)
    w = lat["ws"][sd]
    assert len(sd) == qs == 1 + 2 * dim
    assert sorted(map(tuple, e.astype(int))) == sorted(
        [tuple([0] * dim)] + [tuple(s * np.eye(dim, dtype=int)[a]) for a in range(dim) for s in (1, -1)])
    jj = j0 if j0 >= 0 else (1 / 3 if dim == 2 else 1 / 4)
    cs2 = (1 - jj) / dim
    assert lat["cs2s"] == pytest.approx(cs2, abs=1e-16)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.abs(w @ e).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), cs2 * np.eye(dim), atol=1e-15)
    assert w[0] == pytest.approx(jj, abs=1e-16)


@pytest.mark.parametrize("q,qs,j0,tau,u", [
    (9, 5, -1.0, 0.8, (0.0, 0.0, 0.0)),
    (9, 5, 0.6, 1.3, (0.02, -0.01, 0.0)),
    (19, 7, 0.1, 0.7, (0.01, 0.015, -0.02)),
])
def test_reduced_fourier_mode_matches_matrix_power(q, qs, j0, tau, u):
    """As for the full lattices: one periodic Fourier mode of C on D2Q5 / D3Q7
    evolves by the power of the QS x QS von Neumann step matrix."""
    dim = 2 if q == 9 else 3
    n = (16, 12, 1) if dim == 2 else (8, 6, 10)
    solid = np.zeros((n[2], n[1], n[0]), np.uint8)
    N = solid.size
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    kv = np.array([2 * np.pi * 2 / n[0], 2 * np.pi * 1 / n[1], (2 * np.pi / n[2]) if dim == 3 else 0.0])
    phase = (kv[0] * x + kv[1] * y + kv[2] * z).reshape(-1)
    A, C0 = 0.3, 1.1
    c = C0 + A * np.cos(phase + 0.4)
    uu = np.tile(np.array(u, float), (N, 1))
    case = Case(name="f", dim=dim, nx=n[0], ny=n[1], nz=n[2], q=q, qs=qs, solid=solid,
                tau_ns=0.9, tau_ad=tau, j0=j0, c_init=c, u_init=uu)
    o = Oracle(case)
    lat = o.lattice()
    sd = lat["sd"]
    e, ws, cs2 = lat["e"][sd].astype(float), lat["ws"][sd], lat["cs2s"]
    steps = 25
    o.step(steps)
    _, g = o.pops()
    assert g.shape == (qs, N)
    E = np.outer(ws * (1 + e @ np.array(u) / cs2), np.ones(qs))
    S = np.diag(np.exp(-1j * (e @ kv)))
    M = (np.eye(qs) - (np.eye(qs) - E) / tau) @ S
    v0 = A * np.exp(0.4j) * ws * (1 + e @ np.array(u) / cs2)
    vn = np.linalg.matrix_power(M, steps) @ v0
    pred = C0 * ws[:, None] * (1 + e @ np.array(u) / cs2)[:, None] + \
        np.real(vn[:, None] * np.exp(1j * phase)[None, :])
    assert np.abs(g - pred).max() < 1e-12


@pytest.mark.parametrize("q,qs,j0", [(9, 5, -1.0), (9, 5, 0.8), (19, 7, -1.0), (19, 7, 0.9)])
def test_reduced_diffusion_coefficient_from_mode_decay(q, qs, j0):
    """A long-wavelength mode decays as exp(-D k^2 t) with the paper's
    D = (1 - J0)/dim (tau_AD - 1/2) (rest fraction section)."""
    nx, tau = 128, 0.9
    dim = 2 if q == 9 else 3
    solid = np.zeros((1, 1, nx), np.uint8)
    x = np.arange(nx)
    k = 2 * np.pi / nx
    case = Case(name="d", dim=dim, nx=nx, ny=1, nz=1, q=q, qs=qs, solid=solid, tau_ad=tau,
                j0=j0, c_init=1.0 + 0.1 * np.cos(k * x))
    o = Oracle(case)
    steps = 400
    o.step(steps)
    c = o.fields()["c"]
    amp = 2 * np.abs(np.fft.rfft(c - c.mean())[1]) / nx
    jj = j0 if j0 >= 0 else (1 / 3 if dim == 2 else 1 / 4)
    D = (1 - jj) / dim * (tau - 0.5)
    assert amp / 0.1 == pytest.approx(math.exp(-D * k * k * steps), rel=2e-3)


@pytest.mark.parametrize("mech,scheme,offset,factor", [
    (MECH_PRE, SCHEME_SNEW, 0.0, "1"),
    (MECH_POST, SCHEME_SV, 0.5, "1"),
    (MECH_PRE, SCHEME_SV, 0.0, "1/gamma"),
])
@pytest.mark.parametrize("j0", [-1.0, 0.6])
def test_reduced_linear_steady_robin(mech, scheme, offset, factor, j0):
    """The exact linear steady state between an equilibrium inlet and a
    reactive wall holds on D2Q5 with c_s^2 = (1 - J0)/2, the wall on the node
    (pre-collision source) or halfway (post-collision source)."""
    tau, k_r = 0.8, 2e-2
    case = configs.robin_1d(ny_fluid=20, tau_ad=tau, k_r=k_r, mechanics=mech, scheme=scheme)
    case = case.replace(qs=5, j0=j0)
    o = Oracle(case)
    o.step(40000)
    c = o.fields()["c"].reshape(case.ny, case.nx)[:-1]
    gamma = tau / (tau - 0.5)
    keff = {"1": k_r, "gamma": gamma * k_r, "1/gamma": k_r / gamma}[factor]
    cs2 = (1 - (j0 if j0 >= 0 else 1 / 3)) / 2
    exact = linear_robin_steady(case.ny - 1, tau, cs2, keff, case.c_in, case.c_eq, offset)
    for col in range(case.nx):
        assert np.abs(c[:, col] - exact).max() < 1e-11


@pytest.mark.parametrize("coll", [COLL_BGK, COLL_TRT])
def test_reduced_equals_full_lattice_on_a_plane_channel(coll):
    """Fields that vary only across a flat reactive channel reduce both solute
    lattices to the same three-velocity lattice: the populations of D2Q9 with
    e_y = +1 sum to D2Q5's (0, 1) (weights 1/36 + 1/9 + 1/36 = 1/6), and all of
    them see the same k_i (e_i.n = 1).  With flow along the channel and a
    force, the concentration and the total wall exchange of D2Q5 (J0 = 1/3)
    and D2Q9 runs agree to rounding; likewise D3Q7 with J0 = 0 (c_s^2 = 1/3)
    and D3Q19."""
    rng = np.random.default_rng(5)
    for dim in (2, 3):
        if dim == 2:
            nx, ny, nz = 4, 14, 1
            solid, normals = geometry.plane_channel(nx, ny, (0, ny - 1))
            prof = rng.uniform(0.0, 2.0, ny)
            c0 = np.broadcast_to(prof[None, :, None], (1, ny, nx)).copy()
            full = dict(q=9, j0=-1.0)
            red = dict(q=9, qs=5, j0=-1.0)
            F = (1e-5, 0.0, 0.0)
        else:
            nx, ny, nz = 3, 3, 12
            solid = np.zeros((nz, ny, nx), np.uint8)
            solid[0], solid[-1] = 1, 1
            normals = np.zeros((nz, ny, nx, 3))
            normals[0, ..., 2], normals[-1, ..., 2] = 1.0, -1.0
            prof = rng.uniform(0.0, 2.0, nz)
            c0 = np.broadcast_to(prof[:, None, None], (nz, ny, nx)).copy()
            full = dict(q=19, j0=-1.0)
            red = dict(q=19, qs=7, j0=0.0)
            F = (1e-5, 0.0, 0.0)
        runs = []
        for lat in (full, red):
            case = Case(name="eq", dim=dim, nx=nx, ny=ny, nz=nz, solid=solid, normals=normals,
                        tau_ns=0.8, tau_ad=1.1, force=F, c_eq=1.0, k_r=0.02, v_m=0.1,
                        c_init=c0, collision=coll, **lat)
            o = Oracle(case)
            o.step(300)
            runs.append((o.fields()["c"], o.diag()["wall_exchange"]))
        assert np.abs(runs[0][0] - runs[1][0]).max() < 1e-13
        assert runs[0][1] == pytest.approx(runs[1][1], rel=1e-12)
        assert abs(runs[0][1]) > 1e-3


@pytest.mark.parametrize("q,qs", [(9, 5), (19, 7)])
def test_reduced_solute_plus_solid_mass_invariant(q, qs):
    """Closed periodic domain on D2Q5 / D3Q7: sum C + sum phi / V_m is
    invariant and the solute mass changes by the wall exchange."""
    rng = np.random.default_rng(6)
    if q == 9:
        solid, normals, _ = geometry.disk_medium(40, 32, 0.65, 3.0, 6.0, seed=12)
        dims = dict(dim=2, nx=40, ny=32, nz=1)
    else:
        solid, normals, _ = geometry.sphere_packing(16, 2.0, 4.0, 0.7, seed=5)
        dims = dict(dim=3, nx=16, ny=16, nz=16)
    case = Case(name="m", q=q, qs=qs, solid=solid, normals=normals, tau_ns=0.8, tau_ad=0.75,
                j0=0.4, force=(2e-5, 0, 0), c_eq=1.0, k_r_field=rng.uniform(0, 0.05, solid.size),
                v_m=0.3, mechanics=MECH_POST, scheme=SCHEME_SV,
                c_init=rng.uniform(0.0, 2.0, solid.size), **dims)
    o = Oracle(case)
    d0 = o.diag()
    tot0 = d0["mass_c"] + d0["phi_sum"] / case.v_m
    o.step(200)
    d = o.diag()
    assert d["mass_c"] + d["phi_sum"] / case.v_m == pytest.approx(tot0, rel=1e-12)
    assert d["mass_c"] - d0["mass_c"] == pytest.approx(d["wall_exchange"], rel=1e-9, abs=1e-12)
    q_, kind = o.exchange()
    lat = o.lattice()
    outside = np.setdiff1d(np.arange(q), lat["sd"])
    assert (kind[:, outside] == 0).all() and (q_[:, outside] == 0).all()
    assert (kind[:, lat["sd"]] == 1).any()


def test_reduced_refusals():
    """The oracle takes D2Q5 only with D2Q9 and D3Q7 only with D3Q19."""
    with pytest.raises(ValueError):
        Oracle(_small_case(qs=7))
    with pytest.raises(ValueError):
        Oracle(_box3(qs=5))


# --------------------------------------------------------------------------
# reactive boundary condition
# --------------------------------------------------------------------------
READINGS = [  # (mechanics, scheme, wall offset, factor on k_r that is realised)
    (MECH_PRE, SCHEME_SNEW, 0.0, "1"),
    (MECH_POST, SCHEME_SV, 0.5, "1"),
    (MECH_PRE, SCHEME_SV, 0.0, "1/gamma"),
    (MECH_POST, SCHEME_SNEW, 0.5, "gamma"),
]


@pytest.mark.parametrize("mech,scheme,offset,factor", READINGS)
@pytest.mark.parametrize("tau,k_r", [(0.8, 2e-2), (1.4, 5e-3)])
def test_linear_steady_robin(mech, scheme, offset, factor, tau, k_r):
    """1D steady diffusion between an equilibrium inlet and a reactive wall:
    the exact discrete solution is linear (see ``analytic.linear_robin_steady``).
    With the pre-collision source the new scheme (gamma included, eq.
    k_i_S_New) realises k_r exactly with the wall on the boundary node, and the
    scheme without gamma (eq. k_i_S_Ve) realises k_r/gamma -- the shift of the
    effective PeDa by 1/gamma that the paper reports for Verhaeghe's scheme.
    With the post-collision source the roles swap (wall halfway)."""
    case = configs.robin_1d(ny_fluid=20, tau_ad=tau, k_r=k_r, mechanics=mech, scheme=scheme)
    o = Oracle(case)
    o.step(40000)
    c = o.fields()["c"].reshape(case.ny, case.nx)[:-1]
    gamma = tau / (tau - 0.5)
    keff = {"1": k_r, "gamma": gamma * k_r, "1/gamma": k_r / gamma}[factor]
    exact = linear_robin_steady(case.ny - 1, tau, 1 / 3, keff, case.c_in, case.c_eq, offset)
    for col in range(case.nx):
        assert np.abs(c[:, col] - exact).max() < 1e-11


@pytest.mark.parametrize("mech,scheme,H", [(MECH_PRE, SCHEME_SNEW, 29.0),
                                           (MECH_POST, SCHEME_SV, 30.0)])
def test_reactive_channel_against_series(mech, scheme, H):
    """The 64x32 reactive channel (C = 0 at t = 0, C_eq = 1, tau = 0.8,
    k_r = 1e-3) at t = 2000 against the plane-wall Robin eigen-series (the
    classical solution family the paper cites for its analytic case).  Walls
    on rows 1 and 30 (pre-collision source) or halfway (post-collision)."""
    case = configs.robin_channel(mechanics=mech, scheme=scheme)
    o = Oracle(case)
    o.step(2000)
    c = o.fields()["c"].reshape(32, 64)
    D = (case.tau_ad - 0.5) / 3
    L = H / 2
    y = np.arange(1, 31)
    exact = plane_wall_robin((y - 15.5) / L, 2000, D, L, case.k_r, 1.0)
    assert np.abs(c[1:31] - exact[:, None]).max() < 1e-4
    # x-invariance of a periodic channel
    assert np.abs(c - c[:, :1]).max() < 1e-13


def test_zero_rate_is_bounce_back():
    """k_r = 0 reduces the scheme to bounce-back (paper, RBC limits): with the
    post-collision source a channel with solid rows is bitwise the channel
    with non-periodic box walls, and the solute mass is conserved."""
    ny, nx = 12, 10
    rng = np.random.default_rng(0)
    c0 = rng.uniform(0.2, 1.0, size=(1, ny, nx))
    u0 = np.zeros((1, ny, nx, 3))
    u0[..., 0] = rng.uniform(-0.02, 0.02, size=(1, ny, nx))
    solid, normals = geometry.plane_channel(nx, ny, (0, ny - 1))
    a = Case(name="a", dim=2, nx=nx, ny=ny, nz=1, q=9, solid=solid, normals=normals,
             tau_ns=0.8, tau_ad=0.9, j0=0.3, k_r=0.0, c_eq=1.0, mechanics=MECH_POST,
             c_init=c0, u_init=u0, force=(1e-5, 0, 0))
    b = Case(name="b", dim=2, nx=nx, ny=ny - 2, nz=1, q=9, solid=solid[:, 1:-1].copy(),
             tau_ns=0.8, tau_ad=0.9, j0=0.3, c_eq=1.0, periodic=(1, 0, 1), mechanics=MECH_POST,
             c_init=c0[:, 1:-1].copy(), u_init=u0[:, 1:-1].copy(), force=(1e-5, 0, 0))
    oa, ob = Oracle(a), Oracle(b)
    m0 = oa.diag()["mass_c"]
    oa.step(300)
    ob.step(300)
    fa, ga = oa.pops()
    fb, gb = ob.pops()
    sl = fa.reshape(9, ny, nx)[:, 1:-1].reshape(9, -1)
    assert np.array_equal(sl, fb)
    assert np.array_equal(ga.reshape(9, ny, nx)[:, 1:-1].reshape(9, -1), gb)
    assert abs(oa.diag()["mass_c"] - m0) < 1e-12 * m0


def test_zero_rate_pre_collision_wall_flux_vanishes():
    """k_r = 0 with the pre-collision source: alpha = 0 and beta = 1, so the
    wall carries no net flux once the profile is steady."""
    case = configs.robin_channel(k_r=0.0)
    rng = np.random.default_rng(1)
    case = case.replace(c_init=rng.uniform(0.0, 1.0, size=case.n))
    o = Oracle(case)
    o.step(20000)
    q, kind = o.exchange()
    assert np.abs(q[kind == 1]).max() < 1e-12


def test_infinite_rate_is_anti_bounce_back():
    """k_r -> infinity gives anti-bounce-back with C_eq (paper, RBC limits and
    SI on the PeDa -> infinity limit): k_r = 1e15 matches the ABB scheme."""
    case = configs.robin_channel(k_r=1e15, steps=500)
    a = Oracle(case)
    b = Oracle(case.replace(scheme=SCHEME_ABB))
    a.step(500)
    b.step(500)
    assert np.abs(a.pops()[1] - b.pops()[1]).max() < 1e-12


def test_anti_bounce_back_spares_non_reactive_walls():
    """Anti-bounce-back is the k -> infinity limit of the rate condition (paper,
    extended PeDa range): at a solid node with k_r = 0 it leaves plain
    bounce-back, so a channel whose walls both have k_r = 0 runs bit for bit
    as under the new scheme with k_r = 0."""
    case = configs.robin_channel(k_r=0.0, steps=300)
    rng = np.random.default_rng(8)
    case = case.replace(c_init=rng.uniform(0.0, 1.0, size=case.n))
    a = Oracle(case.replace(scheme=SCHEME_ABB))
    b = Oracle(case)
    a.step(300)
    b.step(300)
    assert np.array_equal(a.pops()[1], b.pops()[1])


def _config_a_small(scheme, peda, kfac=1.0):
    """The paper's configuration A (2D reaction-diffusion, D2Q5, tau_AD =
    0.74) scaled to a = 25, b = 20 at the same D = 0.08, started from the
    analytic field (with the rate k_r kfac) and run to its steady state."""
    a, b, U = 25, 20, 0.004
    D = U * b
    kr = peda * D / b
    an = _config_a_analytic(a, b, D, kr * kfac, 0.74)
    init = np.ones((b + 2, a))
    init[1:b + 1] = an
    case = configs.reaction_diffusion_2d(peda, scheme, a=a, b=b, U=U, c_init=init.reshape(-1))
    assert abs(case.tau_ad - 0.74) < 1e-12
    o = Oracle(case)
    o.step(16000)
    return o.fields()["c"].reshape(b + 2, a)[1:b + 1], (a, b, D, kr)


def _config_a_analytic(a, b, D, kr, tau):
    """The paper's analytic field (eq. analytical2Dverification) on the fluid
    nodes x = 0..a-1, rows 1..b, with each boundary plane where the lattice
    puts it for a linear profile: the equilibrium inlet fixes C at x = -tau
    (see analytic.linear_robin_steady), the zero-gradient outlet copy mirrors
    about x = a - 1/2, bounce-back at the bottom is halfway to the solid row,
    and the pre-collision source with the new scheme puts the reactive wall on
    the top fluid row (test_linear_steady_robin)."""
    x = np.arange(a) + tau
    y = np.arange(1, b + 1) - 0.5
    X, Y = np.meshgrid(x, y)
    return paper_2d_verification(X, Y, a - 0.5 + tau, b - 0.5, D, kr, 1.0, 0.0)


def test_configuration_a_scheme_trends():
    """Configuration A against the paper's analytic solution (Sec. 3.1): on
    grid-aligned walls S.P.J. and the new scheme coincide exactly (e.n = 1 on
    every D2Q5 link); the new scheme matches the analytic field; S.V. is far
    off at PeDa = 1 and matches once its rate is divided by gamma (the PeDa
    shift the paper reports)."""
    C_new, (a, b, D, kr) = _config_a_small(SCHEME_SNEW, 1.0)
    C_spj, _ = _config_a_small(SCHEME_SPJ, 1.0)
    gamma = 0.74 / 0.24
    C_sv, _ = _config_a_small(SCHEME_SV, 1.0, kfac=1 / gamma)
    assert np.array_equal(C_new, C_spj)
    an = _config_a_analytic(a, b, D, kr, 0.74)
    mae_new = np.abs(C_new - an).mean()
    mae_sv = np.abs(C_sv - an).mean()
    mae_sv_shift = np.abs(C_sv - _config_a_analytic(a, b, D, kr / gamma, 0.74)).mean()
    assert mae_new < 1e-2
    assert mae_sv > 10 * mae_new
    assert mae_sv_shift < 2 * mae_new


def _open_channel(coll, tau, u_in=0.01, nx=60, ny=14, steps=30000):
    solid, normals = geometry.plane_channel(nx, ny, (0, ny - 1))
    case = Case(name="open", dim=2, nx=nx, ny=ny, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=tau, tau_ad=0.8, periodic=(0, 1, 1), inlet_axis=0, c_in=1.0, c0=1.0,
                fluid_open=1, u_in=u_in, rho_out=1.0, collision=coll)
    o = Oracle(case)
    o.step(steps)
    f = o.fields()
    rho = f["rho"].reshape(ny, nx)[1:-1]
    ux = f["u"].reshape(ny, nx, 3)[1:-1, :, 0]
    return rho, ux


@pytest.mark.parametrize("coll,tau", [(COLL_BGK, 0.8), (COLL_TRT, 0.8), (COLL_TRT, 1.7)])
def test_open_channel_carries_the_inlet_flux(coll, tau):
    """Open channel (plug inflow, fixed outlet density; Sec. 3.3's channel
    boundary conditions): each inlet link adds exactly 2 w_i rho_out
    (e_i.u_in)/c_s^2, i.e. rho_out u_in per inlet node, so at steady state
    every cross-section carries rho_out u_in H.  The developed flow is
    Poiseuille's: the pressure gradient is 12 nu rho u_in / H^2 (within 1 %),
    and with TRT (walls exactly halfway) the profile across the walls at
    y = 0 and H is a parabola; the density extrapolated to the outlet plane is
    rho_out up to the dropped O(u^2) terms."""
    H, u_in = 12, 0.01
    rho, ux = _open_channel(coll, tau)
    flux = (rho * ux).sum(0)
    assert np.abs(flux / (u_in * H) - 1).max() < 1e-10
    nu = (tau - 0.5) / 3
    rc = rho.mean(0)
    grad = np.polyfit(np.arange(20, 40), rc[20:40], 1)[0] / 3.0
    assert grad / (-12 * nu * u_in / H ** 2) == pytest.approx(1.0, abs=0.01)
    assert abs(rc[-1] + 0.5 * (rc[-1] - rc[-2]) - 1.0) < 1e-3
    if coll == COLL_TRT:
        prof = (rho * ux)[:, 30]
        y = np.arange(H) + 0.5
        par = 1 - (2 * (y - H / 2) / H) ** 2
        par *= u_in * H / par.sum()        # the exact discrete flux fixes the amplitude
        assert np.abs(prof - par).max() < 1e-4 * par.max()


@pytest.mark.parametrize("qs", [0, 5])
def test_per_node_equilibrium_concentration(qs):
    """A per-node C_eq (eq. general_RBC with C_eq taken at each link's solid
    node): a field equal to c_eq everywhere runs bit for bit as the uniform
    value; with C_eq = a on the bottom wall and b on the top wall of a
    pure-diffusion channel the steady profile is the exact linear one, each
    wall on its boundary node with flux k (C_eq - C_wall) (pre-collision
    source, new scheme; see test_linear_steady_robin):
    slope = (b - a) / (n - 1 + 2 D / k)."""
    nx, ny, tau, k_r = 3, 22, 0.8, 0.02
    solid, normals = geometry.plane_channel(nx, ny, (0, ny - 1))
    a, b = 0.3, 1.7
    base = dict(name="ceq", dim=2, nx=nx, ny=ny, nz=1, q=9, qs=qs, solid=solid, normals=normals,
                tau_ad=tau, k_r=k_r, c_eq=a, c0=1.0)
    u1 = Oracle(Case(**base))
    u2 = Oracle(Case(**base, c_eq_field=np.full(nx * ny, a)))
    u1.step(200)
    u2.step(200)
    assert np.array_equal(u1.pops()[1], u2.pops()[1])
    field = np.full((ny, nx), a)
    field[ny - 1, :] = b
    o = Oracle(Case(**base, c_eq_field=field.reshape(-1)))
    o.step(60000)
    c = o.fields()["c"].reshape(ny, nx)[1:ny - 1, 0]
    D = (tau - 0.5) / 3.0          # c_s^2 = 1/3 on D2Q9 and on the standard D2Q5
    n = ny - 2
    slope = (b - a) / (n - 1 + 2 * D / k_r)
    exact = a + D * slope / k_r + slope * np.arange(n)
    assert np.abs(c - exact).max() < 1e-11


def test_gradient_normals_of_straight_walls():
    """Without given normals the oracle uses the isotropic lattice gradient of
    the solid indicator.  On a straight wall that gradient is exactly normal to
    the wall: +y for the bottom row of a channel, (1, 1)/sqrt(2) on the
    interface of a 45 degree half-plane away from its ends."""
    solid, _ = geometry.plane_channel(12, 10, (0, 9))
    o = Oracle(Case(name="n", dim=2, nx=12, ny=10, nz=1, q=9, solid=solid), init=False)
    n = o.normals().reshape(10, 12, 3)
    assert np.allclose(n[0, :, :], [0, 1, 0], atol=1e-15)
    assert np.allclose(n[9, :, :], [0, -1, 0], atol=1e-15)
    N = 24
    y, x = np.mgrid[0:N, 0:N]
    solid = ((x + y) < N).astype(np.uint8)[None]
    o = Oracle(Case(name="d", dim=2, nx=N, ny=N, nz=1, q=9, solid=solid, periodic=(0, 0, 1)),
               init=False)
    n = o.normals().reshape(N, N, 3)
    iface = (x + y == N - 1) & (x > 2) & (y > 2)
    assert np.allclose(n[iface][:, :2], np.sqrt(0.5), atol=1e-15)


@pytest.mark.parametrize("nx,shift", [(512, 0), (512, 256), (512, 296), (512, 512), (300, 97)])
def test_orientation_identity(nx, shift):
    """Sum over the reactive links of w_i max(0, e_i.n), per unit wall length,
    is c_s^2/2 for any wall angle on D2Q9 (half the second moment of the
    weights; lattice links of direction e_i cross a straight wall with density
    |e_i.n|).  The new scheme's k_i (eq. k_i_S_New) is proportional to that
    projection, so the wall flux is orientation-invariant (paper, config. B).
    Patel/Ju's k_i (eq. k_i_S2) divides instead, and its sum depends on the
    angle -- the grid dependence the paper reports."""
    ny = nx
    solid, normals, info = geometry.tilted_band(nx, ny, shift, width=nx * 0.3)
    tau, k_r = 0.8, 1e-3
    gamma = tau / (tau - 0.5)
    case = Case(name="o", dim=2, nx=nx, ny=ny, nz=1, q=9, solid=solid, normals=normals,
                tau_ad=tau, k_r=k_r, xwrap_shift_y=shift)
    o = Oracle(case, init=False)
    k = o.link_k()
    w = np.array([4 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9, 1 / 36, 1 / 9])
    wall_length = 2 * math.hypot(nx, shift)
    proj = np.where(k >= 0, k, 0.0) / (3 * gamma * k_r)       # c_s^-2 = 3
    total = (proj * w[None, :]).sum() / wall_length
    assert total == pytest.approx(1 / 6, abs=1e-12)
    spj = Oracle(case.replace(scheme=SCHEME_SPJ), init=False).link_k()
    inv = np.where(spj > 0, 3 * gamma * k_r / np.where(spj > 0, spj, 1.0), 0.0)
    assert np.allclose(inv[spj > 0], proj[spj > 0], rtol=1e-12)


def test_orientation_simulated_flux():
    """Pure diffusion from reactive walls: the total wall exchange per unit
    wall length of a 30.03 deg band equals that of the 0 deg twin to O(dx/W)
    (the orientation invariance the paper demonstrates with config. B)."""
    out = []
    for aligned in (False, True):
        n, shift, width = 128, 74, 40.0
        if aligned:
            L = math.hypot(n, shift)
            ny = int(round(n * n / L))
            solid, normals, info = geometry.tilted_band(n, ny, 0, width)
            nx, sh = n, 0
        else:
            solid, normals, info = geometry.tilted_band(n, n, shift, width)
            nx, ny, sh = n, n, shift
        case = Case(name="fl", dim=2, nx=nx, ny=ny, nz=1, q=9, solid=solid, normals=normals,
                    tau_ad=0.8, k_r=5e-3, c_eq=1.0, v_m=1.0, xwrap_shift_y=sh)
        o = Oracle(case)
        o.step(1500)
        out.append(o.diag()["wall_exchange"] / (2 * math.hypot(nx, sh)))
    assert out[0] == pytest.approx(out[1], rel=0.02)


# --------------------------------------------------------------------------
# mass accounting with the solid fraction
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mech", [MECH_PRE, MECH_POST])
@pytest.mark.parametrize("scheme", [SCHEME_SNEW, SCHEME_SPJ, SCHEME_ABB])
def test_solute_plus_solid_mass_invariant(mech, scheme):
    """Closed periodic domain: every change of solute mass crosses a reactive
    link, and eq. solidFractionUpdate books the same amount into phi, so
    sum C + sum phi / V_m is invariant."""
    solid, normals, _ = geometry.disk_medium(48, 40, 0.65, 3.0, 7.0, seed=11)
    rng = np.random.default_rng(2)
    case = Case(name="m", dim=2, nx=48, ny=40, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=0.8, tau_ad=0.75, j0=0.2, force=(2e-5, 0, 0), c_eq=1.0,
                k_r_field=rng.uniform(0, 0.05, solid.size), v_m=0.3, mechanics=mech,
                scheme=scheme, c_init=rng.uniform(0.0, 2.0, solid.size))
    o = Oracle(case)
    d0 = o.diag()
    tot0 = d0["mass_c"] + d0["phi_sum"] / case.v_m
    o.step(400)
    d = o.diag()
    assert d["mass_c"] + d["phi_sum"] / case.v_m == pytest.approx(tot0, rel=1e-12)
    assert d["mass_c"] - d0["mass_c"] == pytest.approx(d["wall_exchange"], rel=1e-9, abs=1e-12)


def test_mass_budget_with_inlet_and_outlet():
    """With an inlet and an outlet plane the change of sum C + sum phi / V_m is
    the exchange through the two planes."""
    rng = np.random.default_rng(3)
    n = 12
    solid = np.zeros((n, n, n), np.uint8)
    solid[3:7, 4:9, 5:8] = 1
    normals = np.zeros((n, n, n, 3))
    normals[..., 2] = 1.0
    case = Case(name="b", dim=3, nx=n, ny=n, nz=n, q=19, solid=solid, normals=normals,
                tau_ns=0.9, tau_ad=0.8, j0=0.5, force=(0, 0, 1e-4), c_eq=1.0, k_r=0.02,
                v_m=0.2, inlet_axis=2, c_in=2.0, c_init=rng.uniform(0.5, 1.5, solid.size))
    o = Oracle(case)
    d0 = o.diag()
    o.step(200)
    d = o.diag()
    tot0 = d0["mass_c"] + d0["phi_sum"] / case.v_m
    tot = d["mass_c"] + d["phi_sum"] / case.v_m
    assert tot - tot0 == pytest.approx(d["inlet_exchange"] + d["outlet_exchange"], rel=1e-10)
    assert abs(d["inlet_exchange"]) > 1e-3


def test_phase_change_conserves_mass():
    """Dissolution and precipitation events (thresholds phi = 0 and 1, paper
    Sec. 2.4) move mass between the two phases without creating any."""
    solid, normals = geometry.plane_channel(24, 16, (0, 15))
    solid[0, 1:4, 10:13] = 1
    normals[0, 1:4, 10:13, 1] = 1.0
    rng = np.random.default_rng(4)
    phi0 = np.where(solid.reshape(-1) == 1, 0.02, 0.0)
    case = Case(name="e", dim=2, nx=24, ny=16, nz=1, q=9, solid=solid, normals=normals,
                tau_ad=0.8, c_eq=0.0, k_r=0.05, v_m=1.0, phase_change=1, phi0=phi0,
                c_init=rng.uniform(0.5, 1.5, solid.size))
    o = Oracle(case)
    d0 = o.diag()
    o.step(300)
    d = o.diag()
    assert d["n_events"] > 0
    assert d["mass_c"] + d["phi_sum"] == pytest.approx(d0["mass_c"] + d0["phi_sum"], rel=1e-12)
