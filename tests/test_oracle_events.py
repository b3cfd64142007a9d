"""Pins of the oracle's phase-change rules and of its one-node-gap rate rule.

The expected values here come from the paper's wording, applied by the test
itself to the state just before the event: the state after one step with the
thresholds off (the step is the same with them on; events come after it).

- Dissolution (Sec. 2.4, threshold phi = 0): the new fluid cell starts at the
  mean concentration of its fluid neighbours (equilibrium populations at rest,
  the density likewise the neighbours' mean), and the solid fraction that
  concentration stands for, V_m C - phi, is removed from the surrounding solid
  cells, split by their rate constants.
- Precipitation (threshold phi = 1): the local concentration is turned into
  phi, phi - 1 goes to the surrounding fluid cells in equal shares, phi = 1.
- Wall normals of solid nodes within two sites of a change are recomputed
  from the solid indicator; all other normals stay as given.
- A one-node gap under the pre-collision reading (both ends of a link solid,
  Sec. 2.3, eq. general_RBC with eqs. k_i_S_New and gammaAppendix): with no
  pre-collision population to reflect, the source is the node's own
  post-collision population with k divided by gamma, which is exactly the
  Verhaeghe scheme with the post-collision source (whose linear steady
  profile is pinned exactly in test_oracle_pins.py).

Each check takes an optional oracle library so that test_oracle_mutations.py
can run it against copies of the oracle with a rule deliberately broken.
"""
import numpy as np
import pytest

from lbm_inputs import Case, MECH_POST, MECH_PRE, SCHEME_SNEW, SCHEME_SV
from oracle import Oracle

NX, NY = 12, 10
V_M = 0.5
TILT = np.array([0.6, 0.8, 0.0])   # a given normal no lattice gradient produces


def _block_case(phi_override, lib_seed=0):
    """12 x 10 periodic D2Q9 lattice with an 8 x 4 solid block (x 2..9, y 2..5),
    random C, rho and rate constants; every given normal is TILT."""
    solid = np.zeros((1, NY, NX), np.uint8)
    solid[0, 2:6, 2:10] = 1
    normals = np.zeros((1, NY, NX, 3))
    normals[solid == 1] = TILT
    rng = np.random.default_rng(40 + lib_seed)
    n = NX * NY
    flat = solid.reshape(-1)
    kr = np.where(flat == 1, rng.uniform(0.01, 0.1, n), 0.0)
    phi0 = np.where(flat == 1, 1.0, 0.0)
    for node, v in phi_override.items():
        phi0[node] = v
    return Case(name="ev", dim=2, nx=NX, ny=NY, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=0.9, tau_ad=0.8, c_eq=1.0, k_r_field=kr, v_m=V_M, phi0=phi0,
                c_init=rng.uniform(0.5, 1.5, n), rho_init=rng.uniform(0.98, 1.02, n))


def _neighbours(node):
    """The eight D2Q9 neighbours of a node (periodic lattice)."""
    x, y = node % NX, node // NX
    out = []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx or dy:
                out.append((x + dx) % NX + NX * ((y + dy) % NY))
    return out


def _before_and_after(case, lib):
    """(fields, pops) after one step with the thresholds off and on."""
    a = Oracle(case.replace(phase_change=0), lib=lib)
    b = Oracle(case.replace(phase_change=1), lib=lib)
    a.step(1)
    b.step(1)
    return a, b


S_NODE = 5 + NX * 5     # top face of the block; 3 fluid and 5 solid neighbours
P_NODE = 5 + NX * 6     # fluid node just above it; 5 fluid and 3 solid neighbours


def check_dissolution(lib=None):
    a, b = _before_and_after(_block_case({S_NODE: -0.2}), lib)
    A, B = a.fields(), b.fields()
    assert b.diag()["n_events"] == 1
    s = S_NODE
    nb = _neighbours(s)
    fl = [y for y in nb if A["type"][y] == 0]
    so = [y for y in nb if A["type"][y] == 1]
    assert len(fl) == 3 and len(so) == 5
    c_s = sum(A["c"][y] for y in fl) / len(fl)
    rho_s = sum(A["rho"][y] for y in fl) / len(fl)
    # the new fluid cell: mean C and rho of its fluid neighbours, at rest
    assert B["type"][s] == 0
    assert B["c"][s] == pytest.approx(c_s, rel=1e-14)
    assert B["rho"][s] == pytest.approx(rho_s, rel=1e-14)
    assert np.abs(B["u"][s]).max() < 1e-15
    lat = b.lattice()
    f, g = b.pops()
    assert np.allclose(f[:, s], lat["wf"] * rho_s, rtol=1e-14, atol=0)
    assert np.allclose(g[:, s], lat["ws"][lat["sd"]] * c_s, rtol=1e-14, atol=0)
    assert B["phi"][s] == 0.0
    # V_m C_s - phi_s removed from the solid neighbours by their rate constants
    kr = a.case.k_r_field
    need = V_M * c_s - A["phi"][s]
    ksum = sum(kr[y] for y in so)
    for y in so:
        assert B["phi"][y] == pytest.approx(A["phi"][y] - need * kr[y] / ksum, abs=1e-14)
    # nothing else moves
    rest = np.setdiff1d(np.arange(NX * NY), so + [s])
    assert np.array_equal(B["phi"][rest], A["phi"][rest])
    assert np.array_equal(B["type"][rest], A["type"][rest])
    assert np.array_equal(B["c"][rest], A["c"][rest])
    return a, b


def check_precipitation(lib=None):
    a, b = _before_and_after(_block_case({P_NODE: 1.1}), lib)
    A, B = a.fields(), b.fields()
    assert b.diag()["n_events"] == 1
    x = P_NODE
    nb = _neighbours(x)
    fl = [y for y in nb if A["type"][y] == 0]
    assert len(fl) == 5
    assert A["phi"][x] >= 1.0
    # the local concentration turned into phi, the excess in equal shares
    excess = A["phi"][x] + V_M * A["c"][x] - 1.0
    assert B["type"][x] == 1
    assert B["phi"][x] == 1.0
    assert B["c"][x] == 0.0
    f, g = b.pops()
    assert not f[:, x].any() and not g[:, x].any()
    for y in fl:
        assert B["phi"][y] == pytest.approx(A["phi"][y] + excess / len(fl), abs=1e-14)
    rest = np.setdiff1d(np.arange(NX * NY), fl + [x])
    assert np.array_equal(B["phi"][rest], A["phi"][rest])
    assert np.array_equal(B["c"][rest], A["c"][rest])
    # solute plus solid mass is kept
    tot = lambda F: F["c"].sum() + F["phi"].sum() / V_M
    assert tot(B) == pytest.approx(tot(A), rel=1e-14)


def check_normal_refresh(lib=None):
    a, b = _before_and_after(_block_case({S_NODE: -0.2}), lib)
    B = b.fields()
    # the lattice-gradient normals of the new geometry (pinned on straight walls)
    fresh = Oracle(a.case.replace(solid=B["type"].reshape(1, NY, NX).copy(), normals=None),
                   init=False, lib=lib).normals()
    got = b.normals()
    sx, sy = S_NODE % NX, S_NODE // NX
    for n in np.flatnonzero(B["type"] == 1):
        x, y = n % NX, n // NX
        dx = min((x - sx) % NX, (sx - x) % NX)
        dy = min((y - sy) % NY, (sy - y) % NY)
        if max(dx, dy) <= 2:
            assert np.allclose(got[n], fresh[n], atol=1e-15), (n, got[n], fresh[n])
            assert not np.allclose(got[n], TILT)
        else:
            assert np.array_equal(got[n], TILT)


def _slit_case(q, qs, mech, scheme):
    """A fluid layer one node thick between two solid layers (periodic), with
    flow along x: every reactive link has solid at both ends."""
    rng = np.random.default_rng(7)
    if q == 9:
        shape, axis, dim = (1, 3, 16), 1, 2
        force = (1e-5, 0, 0)
    else:
        shape, axis, dim = (3, 6, 8), 0, 3
        force = (1e-5, 0, 0)
    solid = np.ones(shape, np.uint8)
    normals = np.zeros(shape + (3,))
    sl = [slice(None)] * 3
    sl[axis] = 1
    solid[tuple(sl)] = 0
    nax = 2 - axis      # solid layer 0 faces +axis, layer 2 faces -axis
    sl[axis] = 0
    normals[tuple(sl) + (nax,)] = 1.0
    sl[axis] = 2
    normals[tuple(sl) + (nax,)] = -1.0
    n = solid.size
    return Case(name="slit", dim=dim, nx=shape[2], ny=shape[1], nz=shape[0], q=q, qs=qs,
                solid=solid, normals=normals, tau_ns=0.8, tau_ad=0.8, j0=0.3, force=force,
                c_eq=1.0, k_r_field=rng.uniform(0.005, 0.05, n), v_m=0.3, mechanics=mech,
                scheme=scheme, c_init=rng.uniform(0.2, 1.8, n))


SLITS = [(9, 0), (9, 5), (19, 0), (19, 7)]


def check_gap(q, qs, lib=None, steps=60):
    runs = []
    for mech, scheme in ((MECH_PRE, SCHEME_SNEW), (MECH_POST, SCHEME_SV), (MECH_PRE, SCHEME_SV)):
        o = Oracle(_slit_case(q, qs, mech, scheme), lib=lib)
        o.step(steps)
        F = o.fields()
        runs.append((F["c"], F["phi"], o.pops()[1], o.diag()["wall_exchange"]))
    (c1, p1, g1, w1), (c2, p2, g2, w2), (c3, _, _, _) = runs
    assert abs(w1) > 1e-3                      # the walls do react
    assert np.abs(c1 - c2).max() <= 1e-13 * np.abs(c2).max()
    assert np.abs(g1 - g2).max() <= 1e-13 * np.abs(g2).max()
    assert np.abs(p1 - p2).max() <= 1e-13
    assert w1 == pytest.approx(w2, rel=1e-12)
    # and the pairing matters: the Verhaeghe rate with the same fallback is
    # divided by gamma once more
    assert np.abs(c3 - c2).max() > 1e-6


def test_dissolution_event_rule():
    check_dissolution()


def test_precipitation_event_rule():
    check_precipitation()


def test_event_refreshes_normals_within_two_sites():
    check_normal_refresh()


@pytest.mark.parametrize("q,qs", SLITS)
def test_one_node_gap_is_verhaeghe_post_collision(q, qs):
    check_gap(q, qs)
