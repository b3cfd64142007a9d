"""Helpers for comparing the HIP library with the FP64 oracle (test-side)."""
from __future__ import annotations

import sys

import numpy as np


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def run_pair(case, precision, steps, log_name=None):
    """Run the oracle and the GPU library side by side; return numpy results."""
    import torch
    from oracle import Oracle
    from paper_2306_10794_amd import Simulation

    log(f"[parity] {log_name or case.name} precision={precision} steps={steps} "
        f"shape=({case.nx},{case.ny},{case.nz}) q={case.q}")
    ora = Oracle(case)
    ora.step(steps)
    sim = Simulation(case, precision=precision)
    sim.step(steps)
    torch.cuda.synchronize()
    gf = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    f, g = (t.cpu().numpy() for t in sim.pops())
    q = sim.exchange().cpu().numpy()
    d = sim.diag()
    of = ora.fields()
    fo, go = ora.pops()
    qo, kind = ora.exchange()
    sim.close()
    return dict(gpu=dict(fields=gf, f=f, g=g, q=q, diag=d),
                ora=dict(fields=of, f=fo, g=go, q=qo, kind=kind, diag=ora.diag()))


def rel_errors(res, case, u_floor=0.0):
    """Max errors per field, each divided by its scale (solid nodes excluded).

    u is scaled by max(max |u|, u_floor); the FP64 tests pass the lattice sound
    speed as the floor, since the rounding error of a velocity is set by the
    populations it is summed from, not by |u|."""
    fl = res["ora"]["fields"]["type"] == 0
    g, o = res["gpu"], res["ora"]
    out = {}
    umax = np.abs(o["fields"]["u"][fl]).max() if fl.any() else 0.0
    cscale = max(np.abs(o["fields"]["c"][fl]).max(), abs(case.c_eq), 1e-300)
    out["rho"] = np.abs(g["fields"]["rho"][fl] - o["fields"]["rho"][fl]).max() / 1.0
    us = max(umax, u_floor)
    out["u"] = (np.abs(g["fields"]["u"][fl] - o["fields"]["u"][fl]).max() / us) if us > 1e-12 else 0.0
    out["c"] = np.abs(g["fields"]["c"][fl] - o["fields"]["c"][fl]).max() / cscale
    out["f"] = np.abs(g["f"][:, fl] - o["f"][:, fl]).max() / np.abs(o["f"][:, fl]).max()
    out["g"] = np.abs(g["g"][:, fl] - o["g"][:, fl]).max() / max(np.abs(o["g"][:, fl]).max(), 1e-300)
    # the exchange is a difference of two populations, so its rounding error is
    # relative to the populations, not to the (often much smaller) exchange
    link = o["kind"] == 1
    qs = max(np.abs(o["q"][link]).max(), np.abs(o["g"][:, fl]).max()) if link.any() else 0.0
    out["q"] = (np.abs(g["q"][link] - o["q"][link]).max() / qs) if qs > 0 else 0.0
    dphi = o["fields"]["phi"] - (case.solid_flat() == 1).astype(float) if case.phi0 is None \
        else o["fields"]["phi"] - case.phi0
    ps = np.abs(dphi).max()
    out["phi"] = (np.abs(g["fields"]["phi"] - o["fields"]["phi"]).max() / ps) if ps > 0 else \
        np.abs(g["fields"]["phi"] - o["fields"]["phi"]).max()
    out["type"] = int((g["fields"]["type"] != o["fields"]["type"]).sum())
    # no link may exist on one side only
    out["link_set"] = int(((np.abs(g["q"]) > 0) & ~link).sum())
    return out
