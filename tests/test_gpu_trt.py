"""The TRT collision (Sec. 2.1, eqs. fluid_TRT, solute_TRT; magic parameter
3/16) on the GPU against the FP64 oracle, FP64 to 1e-12 and FP32 deviation
storage to 1e-5 of the field scales, and its limit: a batch that mixes
collision operators is refused (the adjoint of TRT is tested with the
others, test_gpu_adjoint)."""
import numpy as np
import pytest

from lbm_inputs import Case, geometry, MECH_PRE, MECH_POST, SCHEME_SNEW, SCHEME_SV

from parity import log, rel_errors, run_pair

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TRT = 1
TOL = {FP64: 1e-12, FP32: 1e-5}
CS = 3 ** -0.5


def _check(case, precision, steps):
    res = run_pair(case, precision, steps, case.name)
    err = rel_errors(res, case, u_floor=CS if precision == FP64 else 0.0)
    log(f"[trt] {case.name} precision={precision} errors {err}")
    assert err["type"] == 0 and err["link_set"] == 0
    for k in ("rho", "u", "c", "f", "g", "q", "phi"):
        assert err[k] <= TOL[precision], (k, err[k])


def _disks(mech=MECH_PRE, scheme=SCHEME_SNEW, tau_ns=1.7, tau_ad=1.3):
    solid, normals, _ = geometry.disk_medium(70, 44, 0.6, 3.0, 8.0, seed=21)
    rng = np.random.default_rng(5)
    return Case(name="trt disks", dim=2, nx=70, ny=44, nz=1, q=9, solid=solid, normals=normals,
                tau_ns=tau_ns, tau_ad=tau_ad, j0=0.2, force=(1e-5, 0, 0), c_eq=1.0,
                k_r_field=rng.uniform(0, 0.05, solid.size), v_m=0.5, mechanics=mech,
                scheme=scheme, c_init=rng.uniform(0.0, 2.0, solid.size), collision=TRT)


def _spheres():
    nx, ny, nz = 30, 28, 26
    rng = np.random.default_rng(7)
    centres = rng.uniform(0, [nx, ny, nz], size=(10, 3))
    radii = rng.uniform(2.5, 5.0, size=10)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = np.zeros((nz, ny, nx), np.uint8)
    for c, r in zip(centres, radii):
        d = np.stack([x - c[0], y - c[1], z - c[2]], -1)
        for a, n in enumerate((nx, ny, nz)):
            d[..., a] -= n * np.round(d[..., a] / n)
        solid[np.sqrt((d ** 2).sum(-1)) <= r] = 1
    return Case(name="trt spheres", dim=3, nx=nx, ny=ny, nz=nz, q=19, solid=solid,
                tau_ns=2.0, tau_ad=0.7, j0=0.6, force=(0.0, 0.0, 2e-5), c_eq=1.0, k_r=2e-2,
                v_m=0.1, inlet_axis=2, c_in=2.0, c0=1.0, c_ref=1.0, collision=TRT)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_trt_disk_medium(precision):
    _check(_disks(), precision, 200)


def test_trt_post_collision_sv():
    _check(_disks(MECH_POST, SCHEME_SV, tau_ns=0.6, tau_ad=2.5), FP64, 150)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_trt_spheres_inlet_outlet(precision):
    _check(_spheres(), precision, 120)


def test_trt_limits():
    import torch
    from paper_2306_10794_amd import (Simulation, BatchSimulation, LbmError, LBM_EINVAL)
    case = _disks().replace(force=(0.0, 0.0, 0.0))
    with pytest.raises(LbmError) as ei:
        BatchSimulation([case, case.replace(collision=0)], precision=FP32)
    assert ei.value.status == LBM_EINVAL
    torch.cuda.synchronize()
