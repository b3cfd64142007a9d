#!/usr/bin/env python3
"""Throughput of the fused reactive-LBM step on one MI355X.

One step = one launch of the fused stream-collide-RBC kernel over every node
of both lattices plus the solid-fraction kernel of the interface nodes.  The
default workload is the 256^3 D3Q19 sphere packing (porosity 0.40, pressure-
driven flow via an equivalent body force, D3Q19 solute with rest fraction,
supersaturated inlet) in FP32 deviation storage.  Prints one JSON line.

MLUPS counts fluid nodes updated per second (each update advances both
lattices).  ``roofline.achieved`` is the algorithmic bytes of one launch of the
fused kernel divided by its average duration, measured with HIP events on the
stream the kernel runs on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM peak (fused step); adjoint/forward time ratio; batched vs plain"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2306_10794_amd", "csrc")
# sources that determine the step kernel's code
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("lbm_step.hip", "lbm_device.hpp", "lbm_internal.hpp")]
STEP_KERNEL = "lbm::k_step<lbm::D3Q19, float, 4, false, false, false, false>"
PHI_KERNEL = "lbm::k_phi_solid<lbm::D3Q19, float, false>"
# the same workload with the solute on D3Q7
RED_STEP_KERNEL = "lbm::k_step<lbm::D3Q19, float, 4, false, true, false, false>"
RED_PHI_KERNEL = "lbm::k_phi_solid<lbm::D3Q19, float, true>"
COPY_KERNEL = "neg_kernel"   # torch elementwise negation: one read, one write per element
# the rocprofv3 runs whose summaries are committed (run from the repository
# root after `cd /tmp && export TMPDIR=/tmp && cd -`)
PROFILE_ARGS = ("--steps 50 --warmup 5 --no-cpu-baseline --no-batch --no-adjoint --no-phase-change "
                "--reduced-steps 50 --calib-copy-mib 1024")
PMC_ARGS = ("--steps 5 --warmup 1 --no-cpu-baseline --no-batch --no-adjoint --no-phase-change "
            "--reduced-steps 5 --calib-copy-mib 1024")
PROFILE_CMDS = {
    "trace": f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof/trace -o run -- "
             f"python3 bench.py {PROFILE_ARGS}",
    "fetch": f"rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof/fetch -o run -- python3 bench.py {PMC_ARGS}",
    "write": f"rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof/write -o run -- python3 bench.py {PMC_ARGS}",
    "summary": "python3 bench.py --summarize-profiles gpurun_out/prof",
    # every leg of the default run, for the per-kernel durations of the batch,
    # adjoint, phase-change and reduced-solute legs
    "legs": "rocprofv3 --kernel-trace --stats -d gpurun_out/prof/legs -o run -- "
            "python3 bench.py --steps 50 --warmup 5 --no-cpu-baseline --batch-steps 200 "
            "--adjoint-steps 400 --phase-change-steps 100 --reduced-steps 50",
}
# instruction-level counters of the step and adjoint kernels, one pass per group
# (at most 8 SQ counters per pass); the adjoint leg runs 20 steps
SQ_GROUPS = {
    "sq1": "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR "
           "SQ_INSTS_SMEM SQ_INSTS_BRANCH",
    "sq2": "SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_MUL_F64 "
           "SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_CVT SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32",
    "sq3": "SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_SCA SQ_ACTIVE_INST_LDS "
           "SQ_ACTIVE_INST_VMEM SQ_WAIT_INST_ANY SQ_WAIT_ANY",
    "sq4": "SQ_INST_CYCLES_VMEM_RD SQ_INST_CYCLES_VMEM_WR SQ_INST_CYCLES_SALU SQ_THREAD_CYCLES_VALU "
           "SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_VALU_FMA_F32 SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_LDS",
}
SQ_ARGS = ("--steps 5 --warmup 1 --no-cpu-baseline --no-batch --no-phase-change --no-reduced "
           "--adjoint-steps 20 --adjoint-ckpt 10")
for _g, _c in SQ_GROUPS.items():
    PROFILE_CMDS[_g] = f"rocprofv3 --pmc {_c} -d gpurun_out/prof/{_g} -o run -- python3 bench.py {SQ_ARGS}"
# HBM bytes of every kernel of the step and adjoint legs
for _c, _d in (("FETCH_SIZE", "fetch_all"), ("WRITE_SIZE", "write_all")):
    PROFILE_CMDS[_d] = (f"rocprofv3 --pmc {_c} -d gpurun_out/prof/{_d} -o run -- python3 bench.py {SQ_ARGS} "
                        f"--calib-copy-mib 1024 --dump-bytes gpurun_out/prof/{_d}/algo_bytes.json")
PROFILE_CMDS["traffic_summary"] = "python3 bench.py --summarize-traffic gpurun_out/prof"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(q, ts, n_fluid, n_links, n_fluid_iface, qs=None, n_tasks=0, n_row_words=0):
    """Algorithmic HBM bytes of one launch of the fused step kernel.

    Per fluid node: the fluid lattice reads and writes Q populations and the
    solute lattice QS (= Q unless the solute runs on D2Q5 / D3Q7) of ts bytes
    each (a reactive link reads the node's own population toward the wall in
    place of a pulled one), and 8 bytes of node metadata (its dense index and
    the base of its links).  Per reactive link: the link coefficient read and
    the exchange written (2 x ts).  Per fluid interface node: its FP64 solid
    fraction read and written (16 B).  Per launch: each 32-byte task record
    and each 16-byte row word once.
    """
    qs = q if qs is None else qs
    return (n_fluid * ((q + qs) * ts * 2 + 8) + n_links * 2 * ts + n_fluid_iface * 16 +
            n_tasks * 32 + n_row_words * 16)


def adjoint_kernel_bytes(q, ts, n_fluid, n_links, qs=None, seg=100):
    """Algorithmic HBM bytes of one launch of each of the adjoint's kernels.

    Recomputation (one solute-only step at rest): per fluid node QS values
    read and QS written; per reactive link its coefficient read and the
    source value of its rate condition written.  Transposed step: per fluid
    node QS adjoint values read and QS written; per reactive link its
    coefficient and that source value read and the step's dL/dbeta term
    written over the source value (ts each).  Fold (once per segment of seg
    steps): per reactive link the segment's seg terms read (ts each) and its
    FP64 dL/dbeta read and written (16 B)."""
    qs = q if qs is None else qs
    return (n_fluid * qs * ts * 2 + n_links * 2 * ts,
            n_fluid * qs * ts * 2 + n_links * 3 * ts,
            n_links * (seg * ts + 16))


def phi_kernel_bytes(ts, n_links, n_solid_iface):
    """Algorithmic HBM bytes of one launch of the solid-side kernel: per solid
    interface node its link offset (4 B) and its FP64 solid fraction read and
    written (16 B); per reactive link its index in the node's list (4 B) and
    its exchange (ts)."""
    return n_solid_iface * 20 + n_links * (4 + ts)


# kernel names as the profiler reports them, for the per-kernel byte counts
SOL_KERNEL = "lbm::k_sol_step<lbm::D3Q19, float, false, false>"
ADJ_KERNEL = "lbm::k_adj_step<lbm::D3Q19, float, false, false>"
FOLD_KERNEL = "lbm::k_adj_fold<float>"
ALGO_BYTES = {}   # kernel -> algorithmic bytes per launch, filled by the legs that run


def kernel_sha256():
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def traffic_from_profile(workload, key="bytes_per_launch"):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source (key: bytes_per_launch for the
    step kernel, reduced_bytes_per_launch for its D3Q7-solute variant)."""
    path = os.path.join(ROOT, "profiles", f"k_step_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("kernel_sha256") != kernel_sha256():
            return None
        return rec.get(key)
    except Exception:
        return None


def make_case(workload):
    from lbm_inputs import configs
    if workload == "spheres256":
        # the event thresholds are not part of the timed step (a separate leg times them)
        return configs.sphere_precipitation(n=256, seed=3, phase_change=0)
    if workload == "spheres128":
        return configs.sphere_precipitation(n=128, seed=3, phase_change=0)
    raise SystemExit(f"unknown workload {workload}")


def batch_vs_plain(batch_steps, plain_steps, tune_steps):
    """The 1024-domain 2D sweep (D2Q9 flow + solute, FP32 deviation storage):
    one batched context stepped by graph replay under the autotuned launch
    configuration, against one context per domain with its own launches, on
    one stream and on eight streams."""
    import torch
    from lbm_inputs import configs
    from paper_2306_10794_amd import (BatchSimulation, Simulation, LBM_FP32_DEV, lbm_step,
                                      lbm_autotune, lbm_set_launch_config, lbm_step_timed)
    t0 = time.perf_counter()
    cases = configs.batch_domains(count=1024, seed=4)
    nf = sum(c.n_fluid for c in cases)
    log(f"[batch] 1024 domains built in {time.perf_counter() - t0:.1f} s; "
        f"nodes {sum(c.n for c in cases)}, fluid {nf}")
    bs = BatchSimulation(cases, precision=LBM_FP32_DEV, device="cuda:0")
    cfg, tune_ms, tune_n = lbm_autotune(bs.ctx, tune_steps)
    log(f"[batch] autotuned {cfg} at {tune_ms:.4f} ms/step ({tune_n} trial steps)")

    def timed(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        lbm_step(bs.ctx, steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    # the same launch configuration with plain launches and with graph replay
    # of 64 and of 256 steps per graph launch (persistent-launch candidates)
    modes = {}
    for gs in (0, 64, 256):
        lbm_set_launch_config(bs.ctx, cfg["wg_waves"], cfg["xcd_remap"], gs, cfg["overlap"])
        n = max(batch_steps // max(gs, 1) * max(gs, 1), max(gs, 1))
        timed(2 * max(gs, 8))
        modes[gs] = timed(n) / n * 1e3
        log(f"[batch] graph_steps {gs}: {modes[gs]:.4f} ms/step over {n} steps")
    # the two kernels' own durations (HIP events around each launch)
    k_ms, phi_ms = lbm_step_timed(bs.ctx, 200)
    kern = (k_ms + phi_ms) / 200
    lbm_set_launch_config(bs.ctx, **cfg)
    lbm_step(bs.ctx, 2 * max(cfg["graph_steps"], 8))
    tb = timed(batch_steps)
    d = bs.diag()
    bs.close()
    del bs
    torch.cuda.empty_cache()
    log(f"[batch] batched: {batch_steps} steps in {tb:.3f} s; status {d['status']}")

    def plain(nstreams):
        streams = [torch.cuda.Stream(device="cuda:0") for _ in range(nstreams)]
        sims = [Simulation(c, precision=LBM_FP32_DEV, device="cuda:0",
                           stream=streams[i % nstreams]) for i, c in enumerate(cases)]
        for s in sims:
            lbm_step(s.ctx, 2)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for s in sims:
            lbm_step(s.ctx, plain_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        for s in sims:
            s.close()
        del sims
        torch.cuda.empty_cache()
        log(f"[batch] plain, {nstreams} stream(s): {plain_steps} steps in {dt:.3f} s")
        return nf * plain_steps / dt / 1e6

    mb = nf * batch_steps / tb / 1e6
    p1 = plain(1)
    p8 = plain(8)
    return {
        "workload": "1024 uneven 2D domains, sizes U{32..256}x U{32..128}, disk obstacles, "
                    "porosity U[0.5,0.8], log-uniform Pe in [0.1,100] and Da in [0.01,100]; "
                    "D2Q9 fluid + D2Q9 solute, FP32 deviation storage",
        "fluid_nodes": int(nf), "unit": "MLUPS",
        "batched": round(mb, 1), "batched_steps": batch_steps, "launch_config": cfg,
        "ms_per_step_plain_launches": round(modes[0], 4),
        "ms_per_step_graph_64": round(modes[64], 4), "ms_per_step_graph_256": round(modes[256], 4),
        "kernels_ms_per_step": round(kern, 4),
        "launch_gap_ms_per_step": round(modes[0] - kern, 4),
        "plain_1_stream": round(p1, 1), "plain_8_streams": round(p8, 1), "plain_steps": plain_steps,
        "speedup_vs_1_stream": round(mb / p1, 2), "speedup_vs_8_streams": round(mb / p8, 2),
    }


def adjoint_ratio(steps, ckpt):
    """Rate-field recovery workload (128^3 sphere packing, porosity 0.45, D3Q19
    solute, fluid at rest, log-normal k_r): time of the forward run recorded
    for the adjoint, and of the adjoint pass (segment recomputation plus the
    transposed steps), per step, FP32 deviation storage."""
    import torch
    from lbm_inputs import configs
    from paper_2306_10794_amd import Simulation, LBM_FP32_DEV, lbm_step, lbm_adjoint_timed
    case = configs.rate_recovery(n=128, seed=5)
    sim = Simulation(case, precision=LBM_FP32_DEV, device="cuda:0")
    d0 = sim.diag()
    nf, nl = d0["n_fluid"], d0["n_links"]
    lbm_step(sim.ctx, 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbm_step(sim.ctx, steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    sim.init_fields(None, None, case.c_flat())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.record(steps, ckpt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    rng = np.random.default_rng(55)
    dl = torch.as_tensor(rng.normal(size=case.n) * (case.solid_flat() == 0), device="cuda:0")
    sim.adjoint(dl)
    torch.cuda.synchronize()
    sim.init_fields(None, None, case.c_flat())
    sim.record(steps, ckpt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = sim.adjoint(dl)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    ok = bool(torch.isfinite(g).all())
    # the backward pass's kernels timed one by one (same gradient)
    grad_t = torch.empty_like(g)
    sol_ms, adj_ms, fold_ms = lbm_adjoint_timed(sim.ctx, dl, grad_t)
    torch.cuda.synchronize()
    same = bool(torch.equal(grad_t, g))
    sim.close()
    nseg = (steps + ckpt - 1) // ckpt
    # one recomputation launch per step (the last of a segment records the
    # source values only), one transposed step per step, one fold per segment
    sol_us = sol_ms / steps * 1e3
    adj_us = adj_ms / steps * 1e3
    fold_us = fold_ms / nseg * 1e3
    sol_b, adj_b, fold_b = adjoint_kernel_bytes(case.q, 4, nf, nl, seg=ckpt)
    ALGO_BYTES[SOL_KERNEL] = sol_b
    ALGO_BYTES[ADJ_KERNEL] = adj_b
    ALGO_BYTES[FOLD_KERNEL] = fold_b
    del sim
    torch.cuda.empty_cache()
    return {
        "workload": f"rate recovery, {case.nx}^3 sphere packing (porosity "
                    f"{1 - float(case.solid.mean()):.3f}), D3Q19 solute, fluid at rest, "
                    f"log-normal k_r, FP32 deviation storage",
        "fluid_nodes": int(nf), "steps": steps, "checkpoint_every": ckpt,
        "forward_ms_per_step": round(t_fwd / steps * 1e3, 4),
        "plain_step_ms": round(t_plain / steps * 1e3, 4),
        "adjoint_ms_per_step": round(t_adj / steps * 1e3, 4),
        "ratio": round(t_adj / t_fwd, 3), "finite": ok,
        # the backward pass against the solute-only step it transposes (the
        # recomputation kernel is that step): a fairer measure than the
        # recorded fused step, which also streams the idle fluid lattice
        "ratio_vs_solute_step": round(t_adj / steps * 1e6 / sol_us, 3),
        "reactive_links": int(nl),
        "recompute_kernel": {"kernel": "k_sol_step", "avg_us": round(sol_us, 2), "bytes_per_launch": int(sol_b),
                             "achieved_gbs": round(sol_b / sol_us / 1e3, 1),
                             "frac": round(sol_b / sol_us / 1e3 / HBM_PEAK_GBS, 4)},
        "transposed_kernel": {"kernel": "k_adj_step", "avg_us": round(adj_us, 2), "bytes_per_launch": int(adj_b),
                              "achieved_gbs": round(adj_b / adj_us / 1e3, 1),
                              "frac": round(adj_b / adj_us / 1e3 / HBM_PEAK_GBS, 4)},
        "fold_kernel": {"kernel": "k_adj_fold", "launches": nseg, "avg_us": round(fold_us, 2),
                        "bytes_per_launch": int(fold_b), "achieved_gbs": round(fold_b / fold_us / 1e3, 1),
                        "frac": round(fold_b / fold_us / 1e3 / HBM_PEAK_GBS, 4)},
        "timed_gradient_identical": same,
    }


def phase_change_run(case, steps, planes, phi_near):
    """The same workload with the phase-change thresholds on.  The fluid nodes
    of the first `planes` planes at the inlet start at solid fraction
    phi_near, just below the precipitation threshold, so that a burst of
    events (each with relinking and re-layout) happens within a short run;
    all other nodes start as in the workload.  Time per step including the
    per-step candidate scan and the event passes, and the events applied."""
    import torch
    from paper_2306_10794_amd import Simulation, LBM_FP32_DEV, lbm_step
    zi = np.arange(case.n) // (case.nx * case.ny)
    phi0 = np.where(case.solid_flat() == 1, 1.0, np.where(zi < planes, phi_near, 0.0))
    sim = Simulation(case.replace(phase_change=1, phi0=phi0), precision=LBM_FP32_DEV, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbm_step(sim.ctx, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d = sim.diag()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"steps": steps, "near_threshold_planes": planes, "initial_phi": phi_near,
            "ms_per_step": round(dt / steps * 1e3, 4), "events": int(d["n_events"]),
            "fluid_nodes_after": int(d["n_fluid"]), "status": int(d["status"])}


def phase_change_quiet(case, steps, warmup):
    """The workload as specified, with the phase-change thresholds on and no
    node started near a threshold: each step checks for crossed thresholds
    and waits for that answer on the host before the next step."""
    import torch
    from paper_2306_10794_amd import Simulation, LBM_FP32_DEV, lbm_step
    sim = Simulation(case.replace(phase_change=1), precision=LBM_FP32_DEV, device="cuda:0")
    lbm_step(sim.ctx, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbm_step(sim.ctx, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    d = sim.diag()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"steps": steps, "ms_per_step": round(dt / steps * 1e3, 4),
            "mlups": round(d["n_fluid"] * steps / dt / 1e6, 1), "events": int(d["n_events"]),
            "status": int(d["status"])}


def reduced_run(case, steps, warmup):
    """The same workload with the solute on D3Q7 (the paper's 3D solute set)
    at the same diffusivity: fewer solute populations and links per node."""
    import torch
    from lbm_inputs import configs
    from paper_2306_10794_amd import Simulation, LBM_FP32_DEV, lbm_step, lbm_step_timed
    rc = configs.with_reduced_solute(case)
    sim = Simulation(rc, precision=LBM_FP32_DEV, device="cuda:0")
    lbm_step(sim.ctx, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbm_step(sim.ctx, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms, phi_ms = lbm_step_timed(sim.ctx, steps)
    d = sim.diag()
    sim.close()
    kb = kernel_bytes(rc.q, 4, d["n_fluid"], d["n_links"], d["n_fluid_iface"], qs=rc.qs,
                      n_tasks=d["n_tasks"], n_row_words=d["n_row_words"])
    k_s = k_ms / steps / 1e3
    return {"lattices": f"D3Q19 fluid + D3Q{rc.qs} solute", "j0": round(rc.j0, 6),
            "mlups": round(d["n_fluid"] * steps / wall / 1e6, 1), "ms_per_step": round(wall / steps * 1e3, 4),
            "steps": steps, "reactive_links": int(d["n_links"]), "bytes_per_launch": int(kb),
            "avg_kernel_us": round(k_s * 1e6, 2), "phi_kernel_us": round(phi_ms / steps * 1e3, 2),
            "achieved_gbs": round(kb / k_s / 1e9, 1), "frac": round(kb / k_s / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile("spheres256", "reduced_bytes_per_launch"),
            "status": d["status"]}


def _oracle_rate(case, steps, threads=None):
    import oracle
    n_all = oracle.threads() if threads is None else None
    if threads is not None:
        oracle.set_threads(threads)
    try:
        o = oracle.Oracle(case)
        o.step(1)
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
    finally:
        if threads is not None:
            oracle.set_threads(_ORACLE_ALL_THREADS)
    return case.n_fluid * steps / dt / 1e6, dt, (threads or n_all)


_ORACLE_ALL_THREADS = 0


def cpu_baseline(case, steps):
    """The oracle timed on this host: all cores on the full workload (the
    reported value), one core on the same recipe at 128^3, and all / one core
    on the 512^2 tilted channel."""
    global _ORACLE_ALL_THREADS
    import oracle
    from lbm_inputs import configs
    _ORACLE_ALL_THREADS = oracle.threads()
    v, dt, cores = _oracle_rate(case, steps)
    out = dict(value=v, unit="MLUPS", cores=cores, kind="oracle",
               sample=f"full {case.nx}x{case.ny}x{case.nz} workload, FP64, {steps} steps after "
                      f"1 warm-up step ({dt:.1f} s)")
    small = configs.sphere_precipitation(n=128, seed=3, phase_change=0)
    v1, dt1, _ = _oracle_rate(small, 1, threads=1)
    out["single_thread"] = dict(value=v1, unit="MLUPS", cores=1,
                                sample=f"the same recipe at 128^3, 1 step after 1 warm-up step ({dt1:.1f} s)")
    tc = configs.tilted_channel(pe=10.0, da=1.0, steps=0)
    v2, dt2, c2 = _oracle_rate(tc, 20)
    v3, dt3, _ = _oracle_rate(tc, 5, threads=1)
    out["tilted_512"] = dict(all_cores=v2, cores=c2, single_thread=v3, unit="MLUPS",
                             sample=f"512^2 tilted channel D2Q9 + D2Q9, 20 steps ({dt2:.1f} s) and "
                                    f"5 steps on one core ({dt3:.1f} s)")
    out["batch_1024"] = _oracle_batch_rate(_ORACLE_ALL_THREADS)
    return out


def _oracle_batch_rate(cores, every=16, steps=50, steps1=10):
    """The oracle on the 1024-domain sweep: every 16th domain (64 domains, the
    size mix of the whole set), domains stepped in parallel on a pool of host
    threads, one oracle instance each (the library call releases the GIL; a
    domain this small runs its own step on one thread), and the same domains
    one after another on one core."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from lbm_inputs import configs
    cases = configs.batch_domains(count=1024, seed=4)[::every]
    nf = sum(c.n_fluid for c in cases)
    oracle.set_threads(1)
    try:
        oras = [oracle.Oracle(c) for c in cases]
        for o in oras:
            o.step(1)
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=cores) as ex:
            list(ex.map(lambda o: o.step(steps), oras))
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        for o in oras:
            o.step(steps1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(_ORACLE_ALL_THREADS)
    return dict(all_cores=nf * steps / dt / 1e6, cores=cores, single_thread=nf * steps1 / dt1 / 1e6,
                unit="MLUPS", sample=f"{len(cases)} of the 1024 domains (every {every}th, "
                                     f"{nf} fluid nodes), {steps} steps in parallel over domains "
                                     f"({dt:.1f} s) and {steps1} steps on one core ({dt1:.1f} s)")


def _db(d):
    import glob
    import sqlite3
    files = sorted(glob.glob(os.path.join(d, "**", "*results.db"), recursive=True))
    if not files:
        raise SystemExit(f"no rocprofv3 database under {d}")
    return sqlite3.connect(files[-1])


def _medians(db, by_grid=False):
    """Median dispatch duration (ns) per kernel name (and grid size)."""
    vals = {}
    q = ("select name, grid_x * grid_y * grid_z, end - start from kernels" if by_grid
         else "select name, 0, end - start from kernels")
    for name, grid, d in db.execute(q):
        vals.setdefault((name, grid) if by_grid else name, []).append(d)
    return {k: float(np.median(v)) for k, v in vals.items()}


def summarize_profiles(prof_dir, workload="spheres256", calib_mib=1024):
    """Per-kernel durations from the kernel-trace run and HBM bytes from the
    FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch), scaled by what the same
    counters read for a device-to-device copy of calib_mib MiB (which reads
    and writes exactly that many bytes).  Writes <prof_dir>/summary/."""
    out_dir = os.path.join(prof_dir, "summary")
    os.makedirs(out_dir, exist_ok=True)
    tr = _db(os.path.join(prof_dir, "trace"))
    rows = tr.execute("select name, count(*), avg(end - start), min(end - start), max(end - start), "
                      "sum(end - start) from kernels group by name order by sum(end - start) desc"
                      ).fetchall()
    total = sum(r[5] for r in rows) or 1
    lines = [f"# Kernel durations, {workload} (rocprofv3 --kernel-trace --stats)", "",
             "Command (repository root):", "", "    cd /tmp && export TMPDIR=/tmp && cd -",
             f"    {PROFILE_CMDS['trace']}", "",
             "| kernel | calls | avg us | median us | min us | max us | % of GPU time |",
             "|---|---|---|---|---|---|---|"]
    med = _medians(tr)
    step_avg = None
    for name, n, avg, mn, mx, tot in rows[:14]:
        short = name.split("(")[0].replace("void ", "")
        if short == STEP_KERNEL:
            step_avg = avg
        lines.append(f"| `{short}` | {n} | {avg / 1e3:.1f} | {med[name] / 1e3:.1f} | {mn / 1e3:.1f} | "
                     f"{mx / 1e3:.1f} | {100.0 * tot / total:.1f} |")
    if step_avg is None:
        for name, n, avg, *_ in rows:
            if name.split("(")[0].replace("void ", "") == STEP_KERNEL:
                step_avg = avg
    open(os.path.join(out_dir, f"k_step_{workload}_trace.md"), "w").write("\n".join(lines) + "\n")

    def counter(d, cname):
        db = _db(os.path.join(prof_dir, d))
        res = {}
        for name, val in db.execute("select kernel_name, value from counters_collection "
                                    "where counter_name = ?", (cname,)):
            res.setdefault(name.split("(")[0].replace("void ", ""), []).append(float(val))
        return res

    fetch, write = counter("fetch", "FETCH_SIZE"), counter("write", "WRITE_SIZE")
    calib = calib_mib * 2 ** 20

    def copy_kib(res):
        vals = [v for k, vs in res.items() if COPY_KERNEL in k for v in vs]
        if not vals:
            raise SystemExit("no calibration dispatches in the counter runs")
        return sum(vals) / len(vals)

    f_fetch = calib / (copy_kib(fetch) * 1024.0)
    f_write = calib / (copy_kib(write) * 1024.0)
    rec = {"workload": workload, "kernel": STEP_KERNEL, "kernel_sha256": kernel_sha256(),
           "calibration_copy_bytes": calib, "fetch_scale": f_fetch, "write_scale": f_write,
           "commands": [PROFILE_CMDS["fetch"], PROFILE_CMDS["write"]],
           "avg_duration_ns": step_avg}
    lines = [f"# HBM traffic per dispatch, {workload} (rocprofv3 --pmc)", "",
             "Commands (repository root):", "", "    cd /tmp && export TMPDIR=/tmp && cd -",
             f"    {PROFILE_CMDS['fetch']}", f"    {PROFILE_CMDS['write']}", "",
             f"Calibration: an elementwise negation of {calib_mib} MiB (float32) reads and writes "
             f"{calib} B; "
             f"FETCH_SIZE reads {copy_kib(fetch):.0f} KiB for it (scale {f_fetch:.3f}) and "
             f"WRITE_SIZE {copy_kib(write):.0f} KiB (scale {f_write:.3f}).", "",
             "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled read B | scaled write B | "
             "scaled total B |", "|---|---|---|---|---|---|---|"]
    for k in (STEP_KERNEL, PHI_KERNEL, RED_STEP_KERNEL, RED_PHI_KERNEL):
        if k in fetch and k in write:
            fk = sum(fetch[k]) / len(fetch[k])
            wk = sum(write[k]) / len(write[k])
            rb, wb = fk * 1024 * f_fetch, wk * 1024 * f_write
            lines.append(f"| `{k}` | {len(fetch[k])} | {fk:.0f} | {wk:.0f} | {rb:.4g} | {wb:.4g} | "
                         f"{rb + wb:.4g} |")
            if k == STEP_KERNEL:
                rec.update(read_bytes=rb, write_bytes=wb, bytes_per_launch=rb + wb)
            if k == RED_STEP_KERNEL:
                rec.update(reduced_bytes_per_launch=rb + wb)
    open(os.path.join(out_dir, f"k_step_{workload}_pmc.md"), "w").write("\n".join(lines) + "\n")
    json.dump(rec, open(os.path.join(out_dir, f"k_step_{workload}_pmc.json"), "w"), indent=1)
    print(json.dumps(rec), flush=True)


def summarize_legs(prof_dir):
    """Per-kernel durations of the run PROFILE_CMDS['legs'] (its trace under
    prof_dir/legs), written to prof_dir/summary/kernels_all_legs_trace.md."""
    out_dir = os.path.join(prof_dir, "summary")
    os.makedirs(out_dir, exist_ok=True)
    tr = _db(os.path.join(prof_dir, "legs"))
    # one row per kernel and grid size (the legs launch some kernels on
    # lattices of different sizes)
    rows = tr.execute("select name, grid_x * grid_y * grid_z, count(*), avg(end - start), min(end - start), "
                      "max(end - start), sum(end - start) from kernels group by name, grid_x * grid_y * grid_z "
                      "order by sum(end - start) desc").fetchall()
    total = sum(r[6] for r in rows) or 1
    lines = ["# Kernel durations, every leg of bench.py (rocprofv3 --kernel-trace --stats)", "",
             "Legs: the 256^3 sphere packing (D3Q19 and D3Q7 solute), the 1024-domain batch, the",
             "phase-change burst and the 128^3 adjoint (record + adjoint).  One row per kernel and",
             "grid size.", "",
             "Command (repository root):", "", "    cd /tmp && export TMPDIR=/tmp && cd -",
             f"    {PROFILE_CMDS['legs']}", "",
             "| kernel | grid (work-items) | calls | avg us | median us | min us | max us | % of GPU time |",
             "|---|---|---|---|---|---|---|---|"]
    med = _medians(tr, by_grid=True)
    for name, grid, n, avg, mn, mx, tot in rows[:36]:
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"| `{short}` | {grid} | {n} | {avg / 1e3:.1f} | {med[(name, grid)] / 1e3:.1f} | "
                     f"{mn / 1e3:.1f} | {mx / 1e3:.1f} | {100.0 * tot / total:.1f} |")
    path = os.path.join(out_dir, "kernels_all_legs_trace.md")
    open(path, "w").write("\n".join(lines) + "\n")
    print(path, flush=True)


def summarize_counters(prof_dir, runs):
    """Average per-dispatch value of every counter of the rocprofv3 --pmc runs
    prof_dir/<run> (one directory per pass), per kernel; written to
    prof_dir/summary/kernels_step_adjoint_sq_counters.md with the commands of PROFILE_CMDS."""
    out_dir = os.path.join(prof_dir, "summary")
    os.makedirs(out_dir, exist_ok=True)
    table = {}
    for r in runs:
        db = _db(os.path.join(prof_dir, r))
        for name, grid, cname, val in db.execute("select kernel_name, grid_size, counter_name, value from "
                                                 "counters_collection"):
            k = (name.split("(")[0].replace("void ", ""), int(grid))
            table.setdefault(k, {}).setdefault(cname, []).append(float(val))
    # the kernels the bench legs time
    timed = (STEP_KERNEL, PHI_KERNEL, RED_STEP_KERNEL, RED_PHI_KERNEL, SOL_KERNEL, ADJ_KERNEL, FOLD_KERNEL)
    keep = [k for k in table if k[0] in timed]
    cnames = sorted({c for k in keep for c in table[k]})
    lines = ["# SQ counters per dispatch (rocprofv3 --pmc, one pass per counter group)", "",
             "Commands (repository root):", "", "    cd /tmp && export TMPDIR=/tmp && cd -"]
    lines += [f"    {PROFILE_CMDS[r]}" for r in runs if r in PROFILE_CMDS]
    lines += ["", "One row per kernel and grid size: the step leg runs the 256^3 sphere packing, the "
              "adjoint leg the 128^3 rate-recovery packing (whose recorded forward run launches the "
              "step kernels too).", "",
              "| kernel | grid (work-items) | dispatches | " + " | ".join(cnames) + " |",
              "|---|---|---|" + "---|" * len(cnames)]
    for k in sorted(keep, key=lambda k: (k[0], -k[1])):
        vals = table[k]
        n = max(len(v) for v in vals.values())
        cells = [f"{sum(vals[c]) / len(vals[c]):.4g}" if c in vals else "" for c in cnames]
        lines.append(f"| `{k[0]}` | {k[1]} | {n} | " + " | ".join(cells) + " |")
    path = os.path.join(out_dir, "kernels_step_adjoint_sq_counters.md")
    open(path, "w").write("\n".join(lines) + "\n")
    print(path, flush=True)


def summarize_traffic(prof_dir, calib_mib=1024):
    """HBM bytes per dispatch of every kernel of the runs PROFILE_CMDS
    ['fetch_all'] and ['write_all'] (FETCH_SIZE and WRITE_SIZE in KiB, scaled
    by what they read for a copy of calib_mib MiB that reads and writes exactly
    that many bytes), beside the algorithmic bytes the same run wrote with
    --dump-bytes; written to prof_dir/summary/kernels_step_adjoint_traffic_pmc.md."""
    out_dir = os.path.join(prof_dir, "summary")
    os.makedirs(out_dir, exist_ok=True)

    def counter(d, cname):
        # per (kernel, grid size): the dispatches' values and the first dispatch
        db = _db(os.path.join(prof_dir, d))
        res = {}
        for name, grid, disp, val in db.execute(
                "select kernel_name, grid_size, dispatch_id, value from counters_collection "
                "where counter_name = ?", (cname,)):
            key = (name.split("(")[0].replace("void ", ""), int(grid))
            e = res.setdefault(key, [[], disp])
            e[0].append(float(val))
            e[1] = min(e[1], disp)
        return res

    fetch, write = counter("fetch_all", "FETCH_SIZE"), counter("write_all", "WRITE_SIZE")
    algo = {}
    for d in ("fetch_all", "write_all"):
        path = os.path.join(prof_dir, d, "algo_bytes.json")
        if os.path.exists(path):
            algo.update(json.load(open(path)))
    calib = calib_mib * 2 ** 20

    def copy_kib(res):
        vals = [v for (k, _), (vs, _) in res.items() if COPY_KERNEL in k for v in vs]
        if not vals:
            raise SystemExit("no calibration dispatches in the counter runs")
        return sum(vals) / len(vals)

    f_fetch = calib / (copy_kib(fetch) * 1024.0)
    f_write = calib / (copy_kib(write) * 1024.0)
    lines = ["# HBM traffic per dispatch of every kernel of the step and adjoint legs (rocprofv3 --pmc)",
             "", "Commands (repository root):", "", "    cd /tmp && export TMPDIR=/tmp && cd -",
             f"    {PROFILE_CMDS['fetch_all']}", f"    {PROFILE_CMDS['write_all']}",
             f"    {PROFILE_CMDS['traffic_summary']}", "",
             f"Calibration: an elementwise negation of {calib_mib} MiB (float32) reads and writes "
             f"{calib} B; FETCH_SIZE reads {copy_kib(fetch):.0f} KiB for it (scale {f_fetch:.3f}) and "
             f"WRITE_SIZE {copy_kib(write):.0f} KiB (scale {f_write:.3f}).  The step leg (the 256^3 "
             "sphere packing, D3Q19 + D3Q19, FP32 storage) runs first, then the adjoint leg (the "
             "128^3 rate-recovery packing, whose recorded forward run also launches the step "
             "kernels): a kernel appears once per grid size, and the algorithmic bytes belong to "
             "its first grid (the leg that timed it).", "",
             "| kernel | grid (work-items) | dispatches | scaled read B | scaled write B | scaled total B | "
             "algorithmic B | total / algorithmic |", "|---|---|---|---|---|---|---|---|"]
    keys = [k for k in fetch if k[0].startswith("lbm::") and k in write]
    first = {}
    for k in sorted(keys, key=lambda k: fetch[k][1]):
        first.setdefault(k[0], k)
    keys.sort(key=lambda k: -sum(fetch[k][0]) / len(fetch[k][0]))
    for k in keys:
        fv, wv = fetch[k][0], write[k][0]
        rb = sum(fv) / len(fv) * 1024 * f_fetch
        wb = sum(wv) / len(wv) * 1024 * f_write
        ab = algo.get(k[0]) if first[k[0]] == k else None
        lines.append(f"| `{k[0]}` | {k[1]} | {len(fv)} | {rb:.4g} | {wb:.4g} | {rb + wb:.4g} | "
                     f"{'' if ab is None else f'{ab:.4g}'} | "
                     f"{'' if ab is None else f'{(rb + wb) / ab:.3f}'} |")
    path = os.path.join(out_dir, "kernels_step_adjoint_traffic_pmc.md")
    open(path, "w").write("\n".join(lines) + "\n")
    print(path, flush=True)


def calibration_copies(mib):
    """Three copy-like passes of a known size (counter calibration): an
    elementwise negation reads and writes every element once."""
    import torch
    x = torch.ones(mib * 2 ** 20 // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="spheres256")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain sweep")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratio")
    ap.add_argument("--no-phase-change", action="store_true",
                    help="skip the run with the phase-change thresholds on")
    ap.add_argument("--no-reduced", action="store_true",
                    help="skip the run with the solute on D3Q7")
    ap.add_argument("--reduced-steps", type=int, default=200)
    ap.add_argument("--phase-change-steps", type=int, default=300)
    ap.add_argument("--phase-change-planes", type=int, default=2,
                    help="inlet planes whose fluid nodes start near the precipitation threshold")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--adjoint-ckpt", type=int, default=100)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--plain-steps", type=int, default=20)
    ap.add_argument("--tune-steps", type=int, default=32)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the measurement, copy this many MiB three times (counter calibration)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="summarise rocprofv3 runs under DIR/{trace,fetch,write} and exit")
    ap.add_argument("--summarize-legs", metavar="DIR",
                    help="summarise the all-legs kernel trace under DIR/legs and exit")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="summarise the counter passes DIR/<run> named by --runs and exit")
    ap.add_argument("--dump-bytes", metavar="PATH",
                    help="write the algorithmic bytes per launch of the kernels the run timed")
    ap.add_argument("--summarize-traffic", metavar="DIR",
                    help="summarise the FETCH_SIZE / WRITE_SIZE passes DIR/fetch_all, DIR/write_all")
    ap.add_argument("--runs", default="sq1,sq2,sq3,sq4",
                    help="comma-separated pass directories for --summarize-counters")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.workload)
        return
    if args.summarize_legs:
        summarize_legs(args.summarize_legs)
        return
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.runs.split(","))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "runs on more than one GPU are not part of this benchmark.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2306_10794_amd import Simulation, LBM_FP32_DEV, lbm_step, lbm_step_timed

    t0 = time.perf_counter()
    case = make_case(args.workload)
    log(f"[bench] workload {case.name} built in {time.perf_counter() - t0:.1f} s; "
        f"N={case.n} fluid={case.n_fluid}")
    torch.cuda.set_device(0)
    sim = Simulation(case, precision=LBM_FP32_DEV, device="cuda:0")
    d = sim.diag()
    log(f"[bench] geometry: links={d['n_links']} fluid={d['n_fluid']} "
        f"fluid_iface={d['n_fluid_iface']} solid_iface={d['n_solid_iface']}")
    lbm_step(sim.ctx, args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps done")
    t0 = time.perf_counter()
    lbm_step(sim.ctx, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps in {wall:.3f} s")
    k_ms, phi_ms = lbm_step_timed(sim.ctx, args.steps)
    d = sim.diag()
    log(f"[bench] per-kernel: k_step {k_ms / args.steps * 1e3:.1f} us, "
        f"k_phi_solid {phi_ms / args.steps * 1e3:.1f} us; status {d['status']}")

    n_fluid = d["n_fluid"]
    mlups = n_fluid * args.steps / wall / 1e6
    kb = kernel_bytes(case.q, 4, n_fluid, d["n_links"], d["n_fluid_iface"], n_tasks=d["n_tasks"],
                      n_row_words=d["n_row_words"])
    k_avg_s = k_ms / args.steps / 1e3
    achieved = kb / k_avg_s / 1e9
    pb = phi_kernel_bytes(4, d["n_links"], d["n_solid_iface"])
    phi_avg_s = phi_ms / args.steps / 1e3
    ALGO_BYTES[STEP_KERNEL] = kb
    ALGO_BYTES[PHI_KERNEL] = pb
    line = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # populations stored as FP32 deviations, computed in FP64 registers
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{case.name}: D3Q19 fluid + D3Q19 solute, FP32 deviation storage, "
                        f"FP64 arithmetic and solid fraction",
            "storage": "f32 deviations", "arithmetic": "f64",
            "nodes": case.n, "fluid_nodes": int(n_fluid), "reactive_links": int(d["n_links"]),
            "porosity": round(1 - float(case.solid.mean()), 4),
            "phase_change_in_step": False,
            "total_node_mlups": round(case.n * args.steps / wall / 1e6, 1),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile(args.workload),
            "kernel": "k_step", "bytes_per_launch": int(kb),
            "avg_kernel_us": round(k_avg_s * 1e6, 2),
            "phi_kernel_us": round(phi_ms / args.steps * 1e3, 2),
            "phi_kernel": {"kernel": "k_phi_solid", "bytes_per_launch": int(pb),
                           "achieved_gbs": round(pb / phi_avg_s / 1e9, 1),
                           "frac": round(pb / phi_avg_s / 1e9 / HBM_PEAK_GBS, 4)},
        },
        "cpu_baseline": None,
        "batch": None,
        "adjoint": None,
        "phase_change": None,
        "phase_change_quiet": None,
        "reduced_solute": None,
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if args.calib_copy_mib > 0:
        calibration_copies(args.calib_copy_mib)
    if not args.no_reduced:
        line["reduced_solute"] = reduced_run(case, args.reduced_steps, max(5, args.warmup // 2))
        log(f"[bench] reduced solute {line['reduced_solute']}")
    if not args.no_batch:
        line["batch"] = batch_vs_plain(args.batch_steps, args.plain_steps, args.tune_steps)
        log(f"[bench] batch {line['batch']}")
    if not args.no_phase_change:
        line["phase_change"] = phase_change_run(case, args.phase_change_steps,
                                                args.phase_change_planes, 0.9999)
        log(f"[bench] phase change {line['phase_change']}")
        line["phase_change_quiet"] = phase_change_quiet(case, args.phase_change_steps,
                                                        max(5, args.warmup // 2))
        log(f"[bench] phase change on, no burst {line['phase_change_quiet']}")
    if not args.no_adjoint:
        line["adjoint"] = adjoint_ratio(args.adjoint_steps, args.adjoint_ckpt)
        log(f"[bench] adjoint {line['adjoint']}")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
        log(f"[bench] cpu baseline {line['cpu_baseline']}")
    if args.dump_bytes:
        os.makedirs(os.path.dirname(os.path.abspath(args.dump_bytes)), exist_ok=True)
        json.dump(ALGO_BYTES, open(args.dump_bytes, "w"), indent=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
