"""Launch configurations, graph replay and the autotuner change nothing but
speed: populations and solid fractions stay bit-identical to plain launches."""
import numpy as np
import pytest

from lbm_inputs import configs

from parity import log

pytestmark = pytest.mark.gpu

FP32 = 1


def _case():
    return configs.tilted_channel(pe=10.0, da=1.0, n=100, shift=58, width=40.0, steps=0)


def _state(sim):
    import torch
    torch.cuda.synchronize()
    f, g = (t.cpu().numpy() for t in sim.pops())
    return f, g, sim.fields()["phi"].cpu().numpy(), sim.diag()["step"]


def _run(cfg, pre=0, steps=300):
    from paper_2306_10794_amd import Simulation, lbm_set_launch_config
    sim = Simulation(_case(), precision=FP32)
    if pre:
        sim.step(pre)          # leaves the state in buffer 1 before a graph run
    if cfg:
        lbm_set_launch_config(sim.ctx, **cfg)
    sim.step(steps - pre)
    out = _state(sim)
    sim.close()
    return out


@pytest.mark.parametrize("cfg,pre", [
    (dict(wg_waves=1, xcd_remap=0, graph_steps=0), 0),
    (dict(wg_waves=2, xcd_remap=1, graph_steps=16), 1),
    (dict(wg_waves=8, xcd_remap=0, graph_steps=64, overlap=1), 3),
    (dict(wg_waves=4, xcd_remap=1, graph_steps=0, overlap=1), 1),
    (dict(wg_waves=4, xcd_remap=1, graph_steps=7), 0),
])
def test_launch_config_is_bitwise_neutral(cfg, pre):
    log(f"[launch] cfg={cfg} pre={pre}")
    ref = _run(None)
    got = _run(cfg, pre)
    assert got[3] == ref[3] == 300
    for a, b in zip(got[:3], ref[:3]):
        assert np.array_equal(a, b)


def test_autotune_runs_real_steps_and_keeps_results():
    from paper_2306_10794_amd import Simulation, lbm_autotune, lbm_get_launch_config
    ref = _run(None)
    sim = Simulation(_case(), precision=FP32)
    cfg, ms, n = lbm_autotune(sim.ctx, 8)
    log(f"[launch] autotune -> {cfg}, {ms:.4f} ms/step, {n} steps")
    assert cfg == lbm_get_launch_config(sim.ctx)
    assert cfg["wg_waves"] in (1, 2, 4, 8) and cfg["xcd_remap"] in (0, 1)
    assert ms > 0 and 0 < n < 300
    sim.step(300 - n)
    got = _state(sim)
    sim.close()
    assert got[3] == 300
    for a, b in zip(got[:3], ref[:3]):
        assert np.array_equal(a, b)


def test_graph_on_a_batch_matches_plain_launches():
    from paper_2306_10794_amd import BatchSimulation, lbm_set_launch_config
    cases = configs.batch_domains(count=6, seed=21, steps=0, w_range=(20, 70), h_range=(16, 40))
    out = []
    for cfg in (None, dict(wg_waves=4, xcd_remap=1, graph_steps=32)):
        bs = BatchSimulation(cases, precision=FP32)
        if cfg:
            lbm_set_launch_config(bs.ctx, **cfg)
        bs.step(100)
        out.append(_state(bs))
        bs.close()
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)


def test_bad_launch_config_rejected():
    from paper_2306_10794_amd import Simulation, lbm_set_launch_config, LbmError, LBM_EINVAL
    sim = Simulation(_case(), precision=FP32)
    for bad in (dict(wg_waves=3), dict(xcd_remap=2), dict(graph_steps=-1), dict(overlap=2)):
        with pytest.raises(LbmError) as ei:
            lbm_set_launch_config(sim.ctx, **bad)
        assert ei.value.status == LBM_EINVAL
    sim.close()


@pytest.mark.parametrize("phase_change", [0, 1])
def test_timed_steps_equal_plain_steps(phase_change):
    """lbm_step_timed (an event pair around every kernel, one step at a time)
    gives the state of lbm_step bit for bit, with the phase-change thresholds
    off and on (in the second case with events during the run, which lbm_step
    takes in batches of steps and lbm_step_timed one step at a time)."""
    import torch
    from paper_2306_10794_amd import Simulation, lbm_step, lbm_step_timed
    case = configs.sphere_precipitation(n=24, seed=3, phase_change=phase_change, r_min=2.0, r_max=4.0)
    if phase_change:
        zi = np.arange(case.n) // (case.nx * case.ny)
        case = case.replace(phi0=np.where(case.solid_flat() == 1, 1.0, np.where(zi < 2, 0.9999, 0.0)))
    out = []
    for timed in (False, True):
        sim = Simulation(case, precision=FP32)
        if timed:
            ms = lbm_step_timed(sim.ctx, 80)
            assert ms[0] > 0.0 and ms[1] > 0.0
        else:
            lbm_step(sim.ctx, 80)
        torch.cuda.synchronize()
        st = _state(sim)
        out.append((st, sim.diag()["n_events"]))
        sim.close()
    (a, ea), (b, eb) = out
    log(f"[launch] timed vs plain, phase change {phase_change}: events {ea} / {eb}")
    assert a[3] == b[3] == 80 and ea == eb
    if phase_change:
        assert ea > 0
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
