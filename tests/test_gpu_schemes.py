"""The rate-scheme family on the GPU against the paper's own verification
cases (Sec. 3.1):

* configuration A (2D reaction-diffusion on D2Q5, walls aligned with the
  grid) over PeDa = 0.1 .. 1e5 for the new scheme, S.V., S.P.J. and
  anti-bounce-back, at steady state, against the analytic field of
  eq. analytical2Dverification;
* the rest-fraction table of the appendix (the same case at J0 = 0.1, 1/3,
  0.5, 0.9 with BGK and TRT);
* the orientation artefact of S.P.J. (configuration B and the
  pattern-formation discussion: its k_i divides by e.n, so diagonal walls
  react faster): the wall flux of a 45 degree band against its 0 degree twin.

Each question is one batched launch sequence in FP64 (graph replay), and the
batch is first checked against the oracle."""
import math

import numpy as np
import pytest

from lbm_inputs import Case, configs, geometry, SCHEME_SNEW, SCHEME_SV, SCHEME_SPJ, SCHEME_ABB

from analytic import paper_2d_verification
from parity import log, rel_errors, run_pair

pytestmark = pytest.mark.gpu

FP64 = 0
A, B, D = 100, 80, 0.08
STEADY = 600000
SCHEMES = (SCHEME_SNEW, SCHEME_SV, SCHEME_SPJ, SCHEME_ABB)
PEDAS = (0.1, 1.0, 10.0, 100.0, 1e3, 1e4, 1e5)


def _analytic(kr, tau=0.74, inlet=None, top=B - 0.5):
    """Analytic field on the fluid nodes (x = 0..A-1, rows 1..B), each
    boundary plane where the lattice puts it for a linear profile: C fixed at
    x = -tau by the equilibrium inlet, the zero-gradient mirror at x = A - 1/2,
    the bottom zero-flux plane halfway to the solid row, the reactive plane
    on the top fluid row (pre-collision source, new scheme).  inlet: the
    distance of the fixed-C plane before the first node column in place of
    tau (0: the plane on that column); top: the height of the reactive plane
    above the zero-flux plane (B - 1/2: on the top fluid row)."""
    x0 = tau if inlet is None else inlet
    x = np.arange(A) + x0
    y = np.arange(1, B + 1) - 0.5
    X, Y = np.meshgrid(x, y)
    return paper_2d_verification(X, Y, A - 0.5 + x0, top, D, kr, 1.0, 0.0)


def _steady(cases, steps=STEADY):
    """Runs a batch to its steady state; returns each domain's C on the fluid
    rows and the largest change over the last 50k steps."""
    import torch
    from paper_2306_10794_amd import BatchSimulation
    from paper_2306_10794_amd import _lib as L
    bs = BatchSimulation(cases, precision=FP64)
    L.lbm_set_launch_config(bs.ctx, 4, 1, 64, 0)
    bs.step(steps - 50000)
    torch.cuda.synchronize()
    c0 = bs.fields()["c"].cpu().numpy()
    bs.step(50000)
    torch.cuda.synchronize()
    c1 = bs.fields()["c"].cpu().numpy()
    d = bs.diag()
    bs.close()
    assert d["status"] == 0
    out = []
    for k, c in enumerate(cases):
        sl = slice(bs.offsets[k], bs.offsets[k + 1])
        out.append(c1[sl].reshape(c.ny, c.nx)[1:B + 1])
    return out, float(np.abs(c1 - c0).max())


def test_configuration_a_batch_matches_oracle():
    """The cases of the sweep (all four schemes, BGK and TRT) against the
    oracle for 300 steps from the uniform start."""
    for s in SCHEMES:
        case = configs.reaction_diffusion_2d(1.0, s)
        res = run_pair(case, FP64, 300, case.name)
        err = rel_errors(res, case)
        log(f"[schemes] {case.name} errors {err}")
        assert err["type"] == 0 and err["link_set"] == 0
        for k in ("c", "g", "q"):
            assert err[k] <= 1e-12, (s, k, err[k])
    case = configs.reaction_diffusion_2d(10.0, SCHEME_SNEW, j0=0.9, collision=1)
    err = rel_errors(run_pair(case, FP64, 300, case.name), case)
    log(f"[schemes] {case.name} TRT errors {err}")
    assert err["c"] <= 1e-12 and err["g"] <= 1e-12


def test_configuration_a_peda_sweep():
    """The paper's configuration-A findings: S.P.J. and the new scheme agree
    exactly on grid-aligned walls; the new scheme stays close to the analytic
    field at every PeDa; S.V. is far off for 0.1 <= PeDa <= 100 and matches
    once PeDa is divided by gamma; every scheme approaches anti-bounce-back
    as PeDa grows."""
    cases = [configs.reaction_diffusion_2d(p, s) for p in PEDAS for s in SCHEMES]
    fields, change = _steady(cases)
    log(f"[schemes] config A sweep: last-50k change {change:.2e}")
    assert change < 1e-5
    C = {(c.info["peda"], c.scheme): f for c, f in zip(cases, fields)}
    gamma = cases[0].tau_ad / (cases[0].tau_ad - 0.5)
    mae = {}
    for p in PEDAS:
        kr = p * D / B
        an = _analytic(kr)
        for s in SCHEMES:
            mae[(p, s)] = float(np.abs(C[(p, s)] - an).mean())
        mae[(p, "sv/gamma")] = float(np.abs(C[(p, SCHEME_SV)] - _analytic(kr / gamma)).mean())
        dabb = {s: float(np.abs(C[(p, s)] - C[(p, SCHEME_ABB)]).mean()) for s in SCHEMES[:3]}
        mae[(p, "dabb")] = dabb
        log(f"[schemes] PeDa {p:g}: MAE new {mae[(p, SCHEME_SNEW)]:.3e} S.V. {mae[(p, SCHEME_SV)]:.3e} "
            f"S.P.J. {mae[(p, SCHEME_SPJ)]:.3e} anti-BB {mae[(p, SCHEME_ABB)]:.3e} "
            f"S.V.(k/gamma) {mae[(p, 'sv/gamma')]:.3e} |C - C_antiBB| {dabb}")
    for p in PEDAS:
        assert np.array_equal(C[(p, SCHEME_SPJ)], C[(p, SCHEME_SNEW)])
        assert mae[(p, SCHEME_SNEW)] < 1.5e-3
        assert mae[(p, "sv/gamma")] < 1.5 * mae[(p, SCHEME_SNEW)] + 1e-4
    for p in (0.1, 1.0, 10.0, 100.0):
        assert mae[(p, SCHEME_SV)] > 5 * mae[(p, SCHEME_SNEW)]
    for s in SCHEMES[:3]:
        assert mae[(1e5, "dabb")][s] < 0.02 * mae[(1.0, "dabb")][s]


def test_rest_fraction_table():
    """The appendix's rest-fraction table: configuration A at PeDa = 1 with
    J0 = 0.1, 1/3, 0.5 (BGK and TRT) and 0.9 (TRT, tau_AD = 2.1).  The
    paper's point: neither the rest fraction nor TRT adds significant error
    (MAE 1.200 .. 1.219 e-3 throughout).  Here TRT matches BGK to 3 % at each
    J0 and every J0 <= 0.5 stays below 1.5e-3.  Our MAE is lower than the
    paper's and varies more with J0, and at J0 = 0.9 it is 3.5e-3: the
    equilibrium inlet fixes C at x = -tau, exact only for a linear profile,
    and tau reaches 2.1 there (the paper does not say which Dirichlet
    condition its code uses).  The same fields against the analytic field
    with the fixed-C plane half a site before the first column, or on it, lie
    further off at every J0 (that plane is where the inlet puts C), and none
    of the three placements gives the paper's J0-independent value.  Values
    are logged beside the paper's."""
    gold = np.loadtxt(__file__.replace("test_gpu_schemes.py", "golden/restfraction_mae.txt"))
    kr = 1.0 * D / B
    m = {}
    for coll, j0s in ((0, gold[:3, 0]), (1, gold[:, 0])):
        cases = [configs.reaction_diffusion_2d(1.0, SCHEME_SNEW, j0=float(j), collision=coll) for j in j0s]
        for c, row in zip(cases, gold):
            assert abs(c.tau_ad - row[2]) < 1e-9
        fields, change = _steady(cases)
        assert change < 1e-5
        m[coll] = np.array([np.abs(f - _analytic(kr, c.tau_ad)).mean() for c, f in zip(cases, fields)])
        paper = gold[:len(j0s), 3 + coll] * 1e-3
        log(f"[schemes] rest fraction, collision {coll}: J0 {list(j0s)} MAE {list(m[coll])} "
            f"paper {list(paper)}")
        # the same fields against the analytic field with the fixed-C plane
        # placed elsewhere: on the first node column, half a site before it
        for x0 in (0.5, 0.0):
            alt = np.array([np.abs(f - _analytic(kr, c.tau_ad, inlet=x0)).mean() for c, f in zip(cases, fields)])
            log(f"[schemes] rest fraction, collision {coll}, inlet plane at x = -{x0}: MAE {list(alt)}")
            assert np.all(alt > m[coll])
        # and with the reactive plane half a site higher (halfway to the
        # solid row), for each inlet placement
        for x0 in (None, 0.5, 0.0):
            alt = [np.abs(f - _analytic(kr, c.tau_ad, inlet=x0, top=B)).mean() for c, f in zip(cases, fields)]
            log(f"[schemes] rest fraction, collision {coll}, inlet plane at x = "
                f"{'-tau' if x0 is None else -x0}, reactive plane at y = B: MAE {alt}")
    assert np.all(np.abs(m[1][:3] / m[0] - 1) < 0.03)
    assert m[0].max() < 1.5e-3 and m[1][:3].max() < 1.5e-3
    assert np.isfinite(m[1][3]) and m[1][3] < 5e-3


def test_spj_orientation_artefact():
    """Wall flux per unit length of a 45 degree band against its 0 degree
    twin, early in a dissolution run (C = 0, C_eq = 1, pure diffusion; the
    diffusion length stays well inside the band).  The new scheme and S.V.
    have k_i proportional to e.n and keep the flux (configuration B); S.P.J.
    divides by e.n and reacts faster on diagonal walls, most in the
    reaction-limited regime."""
    import torch
    from paper_2306_10794_amd import BatchSimulation
    n, W, steps = 128, 40.0, 400
    solid45, nrm45, info45 = geometry.diagonal_band(n, W)
    ny0 = int(round(info45["period"]))
    solid0, nrm0, _ = geometry.tilted_band(n, ny0, 0, W)
    cases, lengths = [], []
    for p in (0.1, 10.0, 1000.0):
        for s in (SCHEME_SNEW, SCHEME_SV, SCHEME_SPJ):
            for tag, sol, nrm, ny, length in (("0", solid0, nrm0, ny0, 2.0 * n),
                                              ("45", solid45, nrm45, n, info45["wall_length"])):
                cases.append(Case(name=f"band{tag}_p{p:g}_s{s}", dim=2, nx=n, ny=ny, nz=1, q=9, qs=5,
                                  solid=sol, normals=nrm, tau_ns=1.0, tau_ad=0.74, c_eq=1.0,
                                  k_r=p * D / W, v_m=0.0, c0=0.0, scheme=s,
                                  info=dict(peda=p, tag=tag)))
                lengths.append(length)
    bs = BatchSimulation(cases, precision=FP64)
    bs.step(steps)
    torch.cuda.synchronize()
    c = bs.fields()["c"].cpu().numpy()
    bs.close()
    flux = {}
    for k, (case, length) in enumerate(zip(cases, lengths)):
        mass = c[bs.offsets[k]:bs.offsets[k + 1]].sum()
        flux[(case.info["peda"], case.scheme, case.info["tag"])] = mass / length
    ratio = {(p, s): flux[(p, s, "45")] / flux[(p, s, "0")]
             for p in (0.1, 10.0, 1000.0) for s in (SCHEME_SNEW, SCHEME_SV, SCHEME_SPJ)}
    log(f"[schemes] wall flux 45 / 0 degrees: {ratio}")
    for p in (0.1, 10.0, 1000.0):
        assert abs(ratio[(p, SCHEME_SNEW)] - 1) < 0.05
        assert abs(ratio[(p, SCHEME_SV)] - 1) < 0.05
    assert ratio[(0.1, SCHEME_SPJ)] > 1.5
    assert ratio[(1000.0, SCHEME_SPJ)] < ratio[(0.1, SCHEME_SPJ)]
