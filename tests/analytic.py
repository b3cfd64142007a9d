"""Closed forms used to pin the FP64 oracle (test-side only)."""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


def robin_eigenvalues(Bi: float, nterms: int = 200) -> np.ndarray:
    """Roots of lam tan(lam) = Bi, one per branch (n pi, n pi + pi/2)."""
    out = []
    for n in range(nterms):
        lo, hi = n * np.pi + 1e-12, n * np.pi + np.pi / 2 - 1e-12
        out.append(brentq(lambda l: l * np.tan(l) - Bi, lo, hi))
    return np.array(out)


def plane_wall_robin(yhat, t, D, L, k_r, c_eq, nterms=200):
    """Slab |yhat| <= 1 (half width L), C = 0 at t = 0, both faces with the
    first-order surface reaction D dC/dn = k_r (C_eq - C).  Classical
    eigen-series (Carslaw and Jaeger family; the paper's reference for its 2D
    analytic case)."""
    Bi = k_r * L / D
    lam = robin_eigenvalues(Bi, nterms)
    A = 4 * np.sin(lam) / (2 * lam + np.sin(2 * lam))
    yhat = np.asarray(yhat, float)
    s = (A[None, :] * np.cos(lam[None, :] * yhat[:, None]) *
         np.exp(-lam ** 2 * D * t / L ** 2)[None, :]).sum(1)
    return c_eq * (1.0 - s)


def paper_2d_verification(x, y, a, b, D, k_r, c0, c_eq, nterms=100):
    """The paper's analytic 2D reaction-diffusion solution (eq.
    analytical2Dverification with N_n^2 and the transcendental equation
    Analytical_PeDa), n = 1..nterms."""
    PeDa = k_r * b / D
    beta_b = robin_eigenvalues(PeDa, nterms)
    beta = beta_b / b
    N2 = b / 2 * (1 + np.sin(2 * beta * b) / (2 * beta * b))
    x = np.asarray(x, float)[..., None]
    y = np.asarray(y, float)[..., None]
    term = (np.sin(beta * b) / (N2 * beta) * np.cosh(beta * (x - a)) / np.cosh(beta * a) *
            np.cos(beta * y))
    return (c0 - c_eq) * term.sum(-1) + c_eq


def linear_robin_steady(ny_fluid, tau, cs2, k_eff, c_in, c_eq, wall_offset):
    """Exact discrete steady state of the BGK advection-diffusion lattice with
    u = 0 between an equilibrium inlet plane below row 0 and a reactive wall
    ``wall_offset`` above the top fluid row (0 when the wall sits on the node,
    1/2 when it lies halfway to the solid node).

    A linear profile C = a + b y has pre-collision populations
    w_i (C - tau e_iy b) in the bulk; the equilibrium inlet then fixes
    a - tau b = c_in, and the wall carries the diffusive flux D b = k (C_eq - C_w)
    with D = cs2 (tau - 1/2).
    """
    D = cs2 * (tau - 0.5)
    yt = ny_fluid - 1
    b = k_eff * (c_eq - c_in) / (D + k_eff * (yt + wall_offset + tau))
    a = c_in + tau * b
    y = np.arange(ny_fluid)
    return a + b * y
