"""Writes spheres32_10k.npz: the FP64 oracle's state after the full 10,000
steps of the sphere-packing precipitation workload scaled to 32^3 (radii 2-4,
porosity 0.40, seed 3, no phase change), sampled at 256 seeded fluid nodes,
with the oracle's FP64 sums.  It calls only the oracle and the input
generators; the GPU test compares its own run at the same nodes.

    python tests/golden/make_spheres32_10k.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from lbm_inputs import configs  # noqa: E402
from oracle import Oracle  # noqa: E402


def case():
    return configs.sphere_precipitation(n=32, seed=3, r_min=2.0, r_max=4.0, phase_change=0)


def main():
    c = case()
    o = Oracle(c)
    t0 = time.time()
    o.step(c.steps)
    f = o.fields()
    d = o.diag()
    fluid = np.nonzero(c.solid_flat() == 0)[0]
    idx = np.sort(np.random.default_rng(77).choice(fluid, 256, replace=False))
    iface = np.nonzero((c.solid_flat() == 1) & (np.abs(f["phi"] - 1.0) > 0))[0]
    sidx = np.sort(np.random.default_rng(78).choice(iface, min(64, iface.size), replace=False))
    np.savez(os.path.join(HERE, "spheres32_10k.npz"), steps=c.steps, idx=idx, rho=f["rho"][idx],
             u=f["u"][idx], c=f["c"][idx], phi=f["phi"][idx], sidx=sidx, sphi=f["phi"][sidx],
             mass_c=d["mass_c"], phi_sum=d["phi_sum"], wall_exchange=d["wall_exchange"])
    print(f"{c.steps} steps in {time.time() - t0:.0f} s; mass_c {d['mass_c']:.12e}")


if __name__ == "__main__":
    main()
