"""The solute on the paper's reduced velocity sets D2Q5 / D3Q7 (appendix,
velocity sets; Sec. 2.2, eqs. RestFraction, RestFractionCs2) on the GPU
against the FP64 oracle: FP64 to 1e-12 and FP32 deviation storage to 1e-5 of
the field scales, with BGK and TRT, inlet/outlet planes, phase change, a batch
and a save/load round trip; and the limits (mixed batches).  The adjoint on
these sets is tested with the others (test_gpu_adjoint)."""
import numpy as np
import pytest

from lbm_inputs import Case, configs, geometry, MECH_PRE, MECH_POST, SCHEME_SNEW, SCHEME_SV, SCHEME_SPJ

from parity import log, rel_errors, run_pair

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}
CS = 3 ** -0.5


def _check(case, precision, steps, keys=("rho", "u", "c", "f", "g", "q", "phi")):
    res = run_pair(case, precision, steps, case.name)
    err = rel_errors(res, case, u_floor=CS if precision == FP64 else 0.0)
    log(f"[reduced] {case.name} qs={case.qs} precision={precision} errors {err}")
    assert res["gpu"]["g"].shape[0] == case.qs
    assert err["type"] == 0 and err["link_set"] == 0
    for k in keys:
        assert err[k] <= TOL[precision], (k, err[k])
    return res


def _disks(mech=MECH_PRE, scheme=SCHEME_SNEW, collision=0, tau_ns=0.8, tau_ad=0.9):
    solid, normals, _ = geometry.disk_medium(70, 44, 0.6, 3.0, 8.0, seed=23)
    rng = np.random.default_rng(9)
    return Case(name="d2q5 disks", dim=2, nx=70, ny=44, nz=1, q=9, qs=5, solid=solid,
                normals=normals, tau_ns=tau_ns, tau_ad=tau_ad, j0=0.4, force=(1e-5, 0, 0),
                c_eq=1.0, k_r_field=rng.uniform(0, 0.05, solid.size), v_m=0.5, mechanics=mech,
                scheme=scheme, c_init=rng.uniform(0.0, 2.0, solid.size), collision=collision)


def _spheres(collision=0):
    nx, ny, nz = 30, 28, 26
    rng = np.random.default_rng(17)
    centres = rng.uniform(0, [nx, ny, nz], size=(10, 3))
    radii = rng.uniform(2.5, 5.0, size=10)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = np.zeros((nz, ny, nx), np.uint8)
    for c, r in zip(centres, radii):
        d = np.stack([x - c[0], y - c[1], z - c[2]], -1)
        for a, n in enumerate((nx, ny, nz)):
            d[..., a] -= n * np.round(d[..., a] / n)
        solid[np.sqrt((d ** 2).sum(-1)) <= r] = 1
    return Case(name="d3q7 spheres", dim=3, nx=nx, ny=ny, nz=nz, q=19, qs=7, solid=solid,
                tau_ns=0.9, tau_ad=0.7, j0=0.7, force=(0.0, 0.0, 2e-5), c_eq=1.0, k_r=2e-2,
                v_m=0.1, inlet_axis=2, c_in=2.0, c0=1.0, c_ref=1.0, collision=collision)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_d2q5_disk_medium(precision):
    _check(_disks(), precision, 250)


@pytest.mark.parametrize("scheme", [SCHEME_SV, SCHEME_SPJ])
def test_d2q5_post_collision_trt(scheme):
    _check(_disks(MECH_POST, scheme, collision=1, tau_ns=1.6, tau_ad=2.2), FP64, 150)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_d3q7_spheres_inlet_outlet(precision):
    _check(_spheres(), precision, 150)


def test_d3q7_trt():
    _check(_spheres(collision=1), FP64, 100)


def test_d2q5_phase_change():
    """Dissolution events on D2Q5: the same events and node classes as the
    oracle; the exchange of an event step belongs to the rebuilt link list."""
    solid, normals = geometry.plane_channel(40, 20, (0, 19))
    solid[0, 1:5, 10:14] = 1
    normals[0, 1:5, 10:14, 1] = 1.0
    solid[0, 12:19, 25:29] = 1
    normals[0, 12:19, 25:29, 1] = -1.0
    rng = np.random.default_rng(14)
    phi0 = np.where(solid.reshape(-1) == 1, rng.uniform(0.005, 0.05, solid.size), 0.0)
    case = Case(name="d2q5 dissolving", dim=2, nx=40, ny=20, nz=1, q=9, qs=5, solid=solid,
                normals=normals, tau_ns=0.8, tau_ad=0.8, force=(1e-5, 0.0, 0.0), c_eq=0.0,
                k_r=0.05, v_m=1.0, phase_change=1, phi0=phi0,
                c_init=rng.uniform(0.5, 1.5, solid.size))
    res = _check(case, FP64, 300, keys=("rho", "u", "c", "f", "g", "phi"))
    assert res["ora"]["diag"]["n_events"] > 0
    assert res["gpu"]["diag"]["n_events"] == res["ora"]["diag"]["n_events"]


def test_d2q5_batch_matches_oracle_per_domain():
    import torch
    from oracle import Oracle
    from paper_2306_10794_amd import BatchSimulation
    cases = [c.replace(qs=5, c_ref=0.25 * (i % 2), mechanics=(MECH_PRE, MECH_POST)[i % 2])
             for i, c in enumerate(configs.batch_domains(count=4, seed=31, steps=0,
                                                         w_range=(20, 90), h_range=(16, 50)))]
    steps = 200
    log(f"[reduced] batch {[(c.nx, c.ny) for c in cases]}")
    bs = BatchSimulation(cases, precision=FP32)
    bs.step(steps)
    torch.cuda.synchronize()
    fields = bs.fields()
    f, g = bs.pops()
    q = bs.exchange()
    assert g.shape[0] == 5
    for d, case in enumerate(cases):
        gd = dict(fields={k: bs.split(fields[k])[d].cpu().numpy() for k in fields},
                  f=bs.split(f, 1)[d].cpu().numpy(), g=bs.split(g, 1)[d].cpu().numpy(),
                  q=bs.split(q)[d].cpu().numpy())
        ora = Oracle(case)
        ora.step(steps)
        qo, kind = ora.exchange()
        fo, go = ora.pops()
        err = rel_errors(dict(gpu=gd, ora=dict(fields=ora.fields(), f=fo, g=go, q=qo, kind=kind)),
                         case)
        log(f"[reduced] batch domain {d} errors {err}")
        assert err["type"] == 0 and err["link_set"] == 0
        for k in ("rho", "u", "c", "f", "g", "q", "phi"):
            assert err[k] <= TOL[FP32], (d, k, err[k])
    bs.close()


def test_d3q7_save_load_resume_bitwise():
    import torch
    from paper_2306_10794_amd import Simulation
    sim = Simulation(_spheres(), precision=FP32)
    sim.step(20)
    buf = sim.save_state()
    sim.step(20)
    fa, ga = (t.cpu().numpy() for t in sim.pops())
    sim.load_state(buf)
    sim.step(20)
    fb, gb = (t.cpu().numpy() for t in sim.pops())
    torch.cuda.synchronize()
    assert ga.shape[0] == 7
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)
    sim.close()


def test_reduced_limits():
    import torch
    from paper_2306_10794_amd import Simulation, BatchSimulation, LbmError, LBM_EINVAL
    case = _disks().replace(force=(0.0, 0.0, 0.0))
    with pytest.raises(LbmError) as ei:
        BatchSimulation([case, case.replace(qs=0)], precision=FP32)
    assert ei.value.status == LBM_EINVAL
    torch.cuda.synchronize()
