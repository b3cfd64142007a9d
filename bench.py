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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM peak (fused step); adjoint/forward time ratio; batched vs plain"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2306_10794_amd", "csrc", "lbm_step.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(q, ts, n_fluid, n_links, n_fluid_iface):
    """Algorithmic HBM bytes of one launch of the fused step kernel.

    Per fluid node: both lattices read and write Q populations of ts bytes
    (a reactive link reads the node's own population toward the wall in place
    of a pulled one), plus 4 bytes of node metadata.  Per reactive link: the
    link coefficient read and the exchange written (2 x ts).  Per fluid
    interface node: its FP64 solid fraction read and written (16 B).
    """
    return n_fluid * (2 * q * ts * 2 + 4) + n_links * 2 * ts + n_fluid_iface * 16


def traffic_from_profile(workload):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_step_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if rec.get("kernel_sha256") != sha:
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def make_case(workload):
    from lbm_inputs import configs
    if workload == "spheres256":
        # the event thresholds are not part of this build's timed step
        return configs.sphere_precipitation(n=256, seed=3, phase_change=0)
    if workload == "spheres128":
        return configs.sphere_precipitation(n=128, seed=3, phase_change=0)
    raise SystemExit(f"unknown workload {workload}")


def cpu_baseline(case, steps):
    import oracle
    o = oracle.Oracle(case)
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return dict(value=case.n_fluid * steps / dt / 1e6, unit="MLUPS", cores=oracle.threads(),
                kind="oracle",
                sample=f"full {case.nx}x{case.ny}x{case.nz} workload, FP64, {steps} steps after "
                       f"1 warm-up step ({dt:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="spheres256")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU layout is described in DESIGN.md and not run.", file=sys.stderr)
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
    kb = kernel_bytes(case.q, 4, n_fluid, d["n_links"], d["n_fluid_iface"])
    k_avg_s = k_ms / args.steps / 1e3
    achieved = kb / k_avg_s / 1e9
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{case.name}: D3Q19 fluid + D3Q19 solute, FP32 deviation storage, "
                        f"FP64 solid fraction",
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
        },
        "cpu_baseline": None,
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
        log(f"[bench] cpu baseline {line['cpu_baseline']}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
