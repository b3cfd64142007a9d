"""Per-node equilibrium concentration (ceq_field = 1, lbm_set_ceq) on the GPU
against the oracle: a porous medium whose solid nodes react toward different
C_eq, FP64 and FP32 deviation storage, the full and the D2Q5 solute, BGK and
TRT, with phase change; and the limits."""
import numpy as np
import pytest

from lbm_inputs import Case, geometry, MECH_PRE, MECH_POST, SCHEME_SNEW, SCHEME_SV

from parity import log, rel_errors, run_pair

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TOL = {FP64: 1e-12, FP32: 1e-5}
CS = 3 ** -0.5


def _disks(qs=0, collision=0, mech=MECH_PRE, scheme=SCHEME_SNEW, phase_change=0, v_m=0.3):
    solid, normals, _ = geometry.disk_medium(64, 40, 0.6, 3.0, 8.0, seed=27)
    rng = np.random.default_rng(13)
    return Case(name=f"ceq disks qs{qs}", dim=2, nx=64, ny=40, nz=1, q=9, qs=qs, solid=solid,
                normals=normals, tau_ns=0.8, tau_ad=0.9, j0=0.3, force=(1e-5, 0, 0), c_eq=1.0,
                k_r_field=rng.uniform(0.01, 0.08, solid.size), v_m=v_m, mechanics=mech, scheme=scheme,
                c_init=rng.uniform(0.2, 1.2, solid.size), c_eq_field=rng.uniform(0.0, 1.5, solid.size),
                collision=collision, phase_change=phase_change)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_ceq_field_disk_medium(precision):
    case = _disks()
    res = run_pair(case, precision, 200, case.name)
    err = rel_errors(res, case, u_floor=CS if precision == FP64 else 0.0)
    log(f"[ceq] {case.name} precision={precision} errors {err}")
    assert err["type"] == 0 and err["link_set"] == 0
    for k in ("rho", "u", "c", "f", "g", "q", "phi"):
        assert err[k] <= TOL[precision], (k, err[k])


def test_ceq_field_d2q5_trt_phase_change():
    case = _disks(qs=5, collision=1, mech=MECH_POST, scheme=SCHEME_SV, phase_change=1, v_m=4.0)
    res = run_pair(case, FP64, 150, case.name)
    err = rel_errors(res, case, u_floor=CS)
    log(f"[ceq] {case.name} events gpu {res['gpu']['diag']['n_events']} oracle "
        f"{res['ora']['diag']['n_events']} errors {err}")
    assert res["gpu"]["diag"]["n_events"] == res["ora"]["diag"]["n_events"] > 0
    assert err["type"] == 0
    for k in ("rho", "u", "c", "f", "g", "phi"):
        assert err[k] <= TOL[FP64], (k, err[k])


def test_ceq_field_limits():
    import torch
    from paper_2306_10794_amd import Simulation, LbmError, LBM_EINVAL
    from paper_2306_10794_amd import _lib as L
    case = _disks().replace(force=(0.0, 0.0, 0.0))
    sim = Simulation(case, precision=FP32)
    with pytest.raises(LbmError) as ei:
        sim.record(4, 2)                      # the adjoint takes a uniform C_eq
    assert ei.value.status == LBM_EINVAL
    sim.close()
    plain = Simulation(case.replace(c_eq_field=None), precision=FP32)
    field = torch.zeros(case.n, dtype=torch.float64, device="cuda")
    with pytest.raises(LbmError) as ei:
        L.lbm_set_ceq(plain.ctx, field)       # the context has no per-node C_eq
    assert ei.value.status == LBM_EINVAL
    plain.close()
    torch.cuda.synchronize()
