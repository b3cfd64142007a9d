"""Pins of the oracle's adjoint: the gradient of a loss on the final
concentrations with respect to the rate constants of the solid nodes, and the
adjoint populations at the start.

* Transposition: for a fixed velocity history the solute step is affine in
  the populations, so <w, C_T(g0 + v) - C_T(g0)> = <lambda_0, v> for the
  adjoint lambda_0 of dL/dC_T = w, to rounding (a dropped term, a wrong sign
  or a mis-routed source in the transposed step fails it).
* Rate gradient: central finite differences of the oracle's own forward run
  (truncation O(h^2)), on single nodes and along a random direction.
* Anti-bounce-back has no rate: its gradient is exactly zero.
"""
import math

import numpy as np
import pytest

from lbm_inputs import (Case, configs, geometry, MECH_PRE, MECH_POST, SCHEME_SNEW, SCHEME_SV,
                        SCHEME_SPJ, SCHEME_ABB)
from oracle import Oracle
from test_oracle_events import _slit_case


def _disk_case(mech, scheme, flow=True, seed=3):
    solid, normals, _ = geometry.disk_medium(36, 28, 0.65, 2.5, 6.0, seed)
    k = configs.lognormal_rate_field(solid, seed + 100, mu=math.log(2e-2), sigma=0.5)
    return Case(name="adj_disks", dim=2, nx=36, ny=28, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=0.8, tau_ad=0.7, j0=0.4, force=(2e-5 if flow else 0.0, 0.0, 0.0),
                c_eq=1.0, k_r=2e-2, k_r_field=k, v_m=0.0, periodic=(1, 1, 1), c0=0.2,
                mechanics=mech, scheme=scheme)


def _sphere_case(inlet=True, walls=False, seed=9):
    nx, ny, nz = 14, 12, 16
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = np.zeros((nz, ny, nx), np.uint8)
    normals = np.zeros((nz, ny, nx, 3))
    for c, r in zip(rng.uniform(0, [nx, ny, nz], size=(5, 3)), rng.uniform(2.0, 3.5, size=5)):
        d = np.stack([x - c[0], y - c[1], z - c[2]], -1)
        for a, n in enumerate((nx, ny, nz)):
            d[..., a] -= n * np.round(d[..., a] / n)
        dist = np.sqrt((d ** 2).sum(-1))
        inside = dist <= r
        solid[inside] = 1
        normals[inside] = d[inside] / np.maximum(dist[inside], 1e-12)[:, None]
    k = configs.lognormal_rate_field(solid, seed + 7, mu=math.log(3e-2), sigma=0.5)
    return Case(name="adj_spheres", dim=3, nx=nx, ny=ny, nz=nz, q=19, solid=solid,
                normals=normals, tau_ns=0.9, tau_ad=0.8, j0=0.5, force=(0.0, 0.0, 2e-5),
                c_eq=1.0, k_r=3e-2, k_r_field=k, v_m=0.0,
                periodic=(1, 0, 1) if walls else (1, 1, 1), inlet_axis=2 if inlet else -1,
                c_in=2.0, c0=0.5)


def _loss(case, steps, target, lib=None):
    o = Oracle(case, lib=lib)
    o.step(steps)
    c = o.fields()["c"]
    fl = case.solid_flat() == 0
    return float(((c - target)[fl] ** 2).sum()), c


def _grad(case, steps, target, lib=None):
    o = Oracle(case, lib=lib)
    fl = case.solid_flat() == 0
    o2 = Oracle(case, lib=lib)
    o2.step(steps)
    c = o2.fields()["c"]
    dLdC = np.where(fl, 2.0 * (c - target), 0.0)
    grad, _ = o.adjoint(steps, dLdC)
    return grad


CASES = [
    ("disks R1 S.New flow", lambda: _disk_case(MECH_PRE, SCHEME_SNEW)),
    ("disks R2 S.V. flow", lambda: _disk_case(MECH_POST, SCHEME_SV)),
    ("disks R1 S.P.J.", lambda: _disk_case(MECH_PRE, SCHEME_SPJ, flow=False)),
    ("disks R2 anti-BB", lambda: _disk_case(MECH_POST, SCHEME_ABB)),
    ("spheres inlet/outlet", lambda: _sphere_case(inlet=True)),
    ("spheres walls", lambda: _sphere_case(inlet=False, walls=True)),
    ("disks D2Q5 R1 S.New flow", lambda: _disk_case(MECH_PRE, SCHEME_SNEW).replace(qs=5)),
    ("disks D2Q5 R2 S.P.J.", lambda: _disk_case(MECH_POST, SCHEME_SPJ, flow=False).replace(qs=5)),
    ("spheres D3Q7 inlet/outlet", lambda: _sphere_case(inlet=True).replace(qs=7)),
    ("disks TRT R1 S.New flow", lambda: _disk_case(MECH_PRE, SCHEME_SNEW).replace(collision=1, tau_ad=1.3)),
    ("disks TRT D2Q5 R2 S.V.", lambda: _disk_case(MECH_POST, SCHEME_SV).replace(collision=1, qs=5)),
    ("spheres TRT inlet/outlet", lambda: _sphere_case(inlet=True).replace(collision=1)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_adjoint_is_the_transpose_of_the_step(name, make):
    case = make()
    steps = 40
    rng = np.random.default_rng(1)
    fl = case.solid_flat() == 0
    w = np.where(fl, rng.normal(size=case.n), 0.0)
    base = Oracle(case)
    qs = base.QS
    v = np.where(fl[None, :], rng.normal(size=(qs, case.n)), 0.0) * 1e-2
    _, lam0 = base.adjoint(steps, w, want_lam0=True)
    # lambda_0 by fluid direction; the solute set's rows carry the populations
    assert np.all(np.delete(lam0, base.sdirs, axis=0) == 0.0)
    lam0 = lam0[base.sdirs]
    c_base = base.fields()["c"]
    pert = Oracle(case)
    f0, g0 = pert.pops()
    pert.set_pops(g=g0 + v)
    pert.step(steps)
    lhs = float(w @ (pert.fields()["c"] - c_base))
    rhs = float((lam0 * v).sum())
    scale = np.linalg.norm(lam0) * np.linalg.norm(v)
    assert abs(lhs - rhs) <= 1e-11 * scale, (lhs, rhs, scale)
    assert abs(rhs) > 1e-5 * scale   # not vacuous (random vectors: ~ scale / sqrt(dim))


@pytest.mark.parametrize("name,make", [c for c in CASES if "anti" not in c[0]],
                         ids=[c[0] for c in CASES if "anti" not in c[0]])
def test_rate_gradient_matches_central_differences(name, make):
    case = make()
    steps = 60
    rng = np.random.default_rng(2)
    fl = case.solid_flat() == 0
    target = np.where(fl, rng.uniform(0.0, 1.5, case.n), 0.0)
    grad = _grad(case, steps, target)
    k0 = case.k_r_field.copy()
    nz = np.flatnonzero(np.abs(grad) > 1e-6 * np.abs(grad).max())
    assert nz.size > 5
    # single nodes
    for s in rng.choice(nz, size=4, replace=False):
        h = 1e-4 * k0[s]
        kp, km = k0.copy(), k0.copy()
        kp[s] += h
        km[s] -= h
        fd = (_loss(case.replace(k_r_field=kp), steps, target)[0] -
              _loss(case.replace(k_r_field=km), steps, target)[0]) / (2 * h)
        assert abs(fd - grad[s]) <= 1e-6 * abs(grad).max(), (s, fd, grad[s])
    # a random direction over every solid node
    d = np.where(case.solid_flat() == 1, rng.normal(size=case.n), 0.0) * k0
    h = 1e-4
    fd = (_loss(case.replace(k_r_field=k0 + h * d), steps, target)[0] -
          _loss(case.replace(k_r_field=k0 - h * d), steps, target)[0]) / (2 * h)
    ad = float(grad @ d)
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_anti_bounce_back_has_no_rate_gradient():
    case = _disk_case(MECH_POST, SCHEME_ABB)
    fl = case.solid_flat() == 0
    grad = _grad(case, 30, np.where(fl, 0.7, 0.0))
    assert np.all(grad == 0.0)


def test_zero_loss_gradient_is_zero():
    case = _disk_case(MECH_PRE, SCHEME_SNEW)
    o = Oracle(case)
    grad, lam0 = o.adjoint(20, np.zeros(case.n), want_lam0=True)
    assert np.all(grad == 0.0) and np.all(lam0 == 0.0)


def check_gap_adjoint(lib=None, steps=50):
    """A layer one node thick (every reactive link has solid at both ends):
    the pre-collision reading falls back to the post-collision source with
    k / gamma, and its rate gradient must carry the same 1/gamma (central
    differences of the forward run)."""
    case = _slit_case(9, 0, MECH_PRE, SCHEME_SNEW)
    rng = np.random.default_rng(5)
    fl = case.solid_flat() == 0
    target = np.where(fl, rng.uniform(0.0, 1.5, case.n), 0.0)
    grad = _grad(case, steps, target, lib)
    k0 = case.k_r_field.copy()
    d = np.where(case.solid_flat() == 1, rng.normal(size=case.n), 0.0) * k0
    h = 1e-4
    fd = (_loss(case.replace(k_r_field=k0 + h * d), steps, target, lib)[0] -
          _loss(case.replace(k_r_field=k0 - h * d), steps, target, lib)[0]) / (2 * h)
    ad = float(grad @ d)
    assert abs(ad) > 0
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_rate_gradient_across_a_one_node_gap():
    check_gap_adjoint()
