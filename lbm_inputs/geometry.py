"""Seeded synthetic geometries: solid masks plus analytic unit wall normals.

Every generator is deterministic for a given seed (``numpy.random.default_rng``,
PCG64).  Normals point from the solid into the fluid and are stored for every
node (zero where no wall is defined); only solid nodes adjacent to fluid use
them.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np


def plane_channel(nx: int, ny: int, wall_rows=(0, -1)) -> Tuple[np.ndarray, np.ndarray]:
    """2D channel periodic in x with solid rows; bottom wall normal +y, top -y."""
    solid = np.zeros((1, ny, nx), np.uint8)
    normals = np.zeros((1, ny, nx, 3), np.float64)
    for r in wall_rows:
        rr = r % ny
        solid[0, rr, :] = 1
        normals[0, rr, :, 1] = 1.0 if rr < ny // 2 else -1.0
    return solid, normals


def tilted_band(nx: int, ny: int, shift: int, width: float, s0: float = 0.37):
    """Fluid band of perpendicular width ``width`` on the torus whose sites
    (x + nx, y) and (x, y + shift) coincide, and (x, y + ny) and (x, y).

    The trivial translations are (nx, -shift) and (0, ny).  The band runs along
    t = (nx, -shift)/|(nx, shift)|; its unit normal is m = (shift, nx)/|(nx, shift)|.
    The perpendicular coordinate s = m.(x, y) is invariant under the first
    translation and increases by the period P = nx*ny/|(nx, shift)| under the
    second, so ``(s - s0) mod P`` is well defined on the torus.  Nodes with that value in [0, width) are fluid.
    ``shift = 0`` gives the axis-aligned twin with the same width and period.
    Returns (solid, normals, info) where info carries t, m, P and per-node d.
    """
    L = math.hypot(nx, shift)
    t = np.array([nx / L, -shift / L, 0.0])
    m = np.array([shift / L, nx / L, 0.0])
    P = nx * ny / L
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    s = m[0] * x + m[1] * y
    d = np.mod(s - s0, P)
    fluid = d < width
    solid = (~fluid).astype(np.uint8)[None]
    normals = np.zeros((1, ny, nx, 3), np.float64)
    # solid node: nearer to the band's upper surface (d = width) -> normal -m,
    # nearer to the next band's lower surface (d = P) -> normal +m
    upper = (d - width) < (P - d)
    sol = ~fluid
    for k in range(2):
        normals[0, :, :, k] = np.where(sol & upper, -m[k], np.where(sol, m[k], 0.0))
    info = dict(t=t, m=m, period=P, d=d[None], angle_deg=math.degrees(math.atan2(-shift, nx)))
    return solid, normals, info


def diagonal_band(n: int, width: float, s0: float = 0.37):
    """Fluid band at 45 degrees on the plain n x n torus: s = (x + y)/sqrt(2)
    grows by the period P = n/sqrt(2) under either translation, so
    ``(s - s0) mod P`` is well defined; nodes with that value in [0, width)
    are fluid.  Normals of solid nodes are -+m, m = (1, 1)/sqrt(2), toward the
    nearer band surface.  Returns (solid, normals, info) like tilted_band."""
    r = 1.0 / math.sqrt(2.0)
    m = np.array([r, r, 0.0])
    P = n * r
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    d = np.mod(m[0] * x + m[1] * y - s0, P)
    fluid = d < width
    solid = (~fluid).astype(np.uint8)[None]
    normals = np.zeros((1, n, n, 3), np.float64)
    upper = (d - width) < (P - d)
    sol = ~fluid
    for k in range(2):
        normals[0, :, :, k] = np.where(sol & upper, -m[k], np.where(sol, m[k], 0.0))
    info = dict(t=np.array([r, -r, 0.0]), m=m, period=P, d=d[None], angle_deg=-45.0,
                wall_length=2.0 * n * math.sqrt(2.0))
    return solid, normals, info


def _wrap_delta(d, n):
    return d - n * np.round(d / n)


def pack_spheres(n: int, r_min: float, r_max: float, porosity: float, seed: int,
                 max_iter: int = 4000, tol: float = 0.02):
    """Periodic polydisperse sphere packing densified by overlap relaxation.

    Radii are drawn uniform in [r_min, r_max] until their total volume reaches
    the target solid fraction; centres start uniform in the box and overlapping
    pairs are pushed apart (minimum image) until the largest overlap is below
    ``tol`` lattice units.  Returns (centres [K,3], radii [K]).
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    target = (1.0 - porosity) * float(n) ** 3
    radii = []
    vol = 0.0
    while vol < target:
        r = rng.uniform(r_min, r_max)
        radii.append(r)
        vol += 4.0 / 3.0 * math.pi * r ** 3
    radii = np.array(radii)
    centres = rng.uniform(0.0, n, size=(len(radii), 3))
    # grow radii from 85% while relaxing, which avoids locking in early jams
    for it in range(max_iter):
        scale = min(1.0, 0.85 + 0.15 * it / 600.0)
        r = radii * scale
        tree = cKDTree(np.mod(centres, n), boxsize=n)
        pairs = tree.query_pairs(2.0 * r_max * scale, output_type="ndarray")
        if len(pairs) == 0:
            if scale >= 1.0:
                break
            continue
        i, j = pairs[:, 0], pairs[:, 1]
        dv = _wrap_delta(centres[j] - centres[i], n)
        dist = np.sqrt((dv * dv).sum(1))
        ov = r[i] + r[j] - dist
        mask = ov > 0
        if scale >= 1.0 and (not mask.any() or ov[mask].max() < tol):
            break
        i, j, dv, dist, ov = i[mask], j[mask], dv[mask], dist[mask], ov[mask]
        dist = np.maximum(dist, 1e-9)
        u = dv / dist[:, None]
        push = 0.5 * 1.02 * ov[:, None] * u
        disp = np.zeros_like(centres)
        np.add.at(disp, i, -push)
        np.add.at(disp, j, push)
        centres = np.mod(centres + disp, n)
    return centres, radii


def voxelize_spheres(n: int, centres: np.ndarray, radii: np.ndarray):
    """Solid mask and analytic normals of a periodic sphere set on an n^3 lattice.

    A node is solid when its centre lies inside a sphere.  Its normal is the
    outward radial direction of the containing sphere whose surface is nearest.
    """
    solid = np.zeros((n, n, n), np.uint8)
    depth = np.full((n, n, n), np.inf)
    normals = np.zeros((n, n, n, 3), np.float64)
    for c, r in zip(centres, radii):
        lo = np.floor(c - r).astype(int)
        hi = np.ceil(c + r).astype(int)
        xs = np.arange(lo[0], hi[0] + 1)
        ys = np.arange(lo[1], hi[1] + 1)
        zs = np.arange(lo[2], hi[2] + 1)
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        dx, dy, dz = X - c[0], Y - c[1], Z - c[2]
        dist = np.sqrt(dx * dx + dy * dy + dz * dz)
        inside = dist <= r
        if not inside.any():
            continue
        zi, yi, xi = np.mod(Z[inside], n), np.mod(Y[inside], n), np.mod(X[inside], n)
        dep = r - dist[inside]
        better = dep < depth[zi, yi, xi]
        zi, yi, xi, dep = zi[better], yi[better], xi[better], dep[better]
        dd = np.maximum(dist[inside][better], 1e-12)
        solid[zi, yi, xi] = 1
        depth[zi, yi, xi] = dep
        normals[zi, yi, xi, 0] = dx[inside][better] / dd
        normals[zi, yi, xi, 1] = dy[inside][better] / dd
        normals[zi, yi, xi, 2] = dz[inside][better] / dd
    return solid, normals


def sphere_packing(n: int, r_min: float, r_max: float, porosity: float, seed: int):
    centres, radii = pack_spheres(n, r_min, r_max, porosity, seed)
    solid, normals = voxelize_spheres(n, centres, radii)
    info = dict(centres=centres, radii=radii, porosity=1.0 - solid.mean())
    return solid, normals, info


def disk_medium(W: int, H: int, porosity: float, r_min: float, r_max: float, seed: int):
    """2D channel (solid rows y=0 and y=H-1, periodic x) with random disks.

    Disks (overlap allowed) are added until the fluid fraction of the whole
    W x H box drops to ``porosity``; a disk that would break x-percolation of
    the fluid is rejected.  Normals: walls +-y, disks radial (nearest surface).
    """
    from scipy import ndimage

    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    solid = np.zeros((H, W), bool)
    solid[0, :] = True
    solid[H - 1, :] = True
    depth = np.full((H, W), np.inf)
    nrm = np.zeros((H, W, 2))
    nrm[0, :, 1] = 1.0
    nrm[H - 1, :, 1] = -1.0
    depth[0, :] = -1.0
    depth[H - 1, :] = -1.0

    def percolates(s):
        fl = np.concatenate([~s, ~s], axis=1)
        lab, _ = ndimage.label(fl)
        left = set(np.unique(lab[:, 0])) - {0}
        right = set(np.unique(lab[:, -1])) - {0}
        return bool(left & right)

    tries = 0
    while (1.0 - solid.mean()) > porosity and tries < 20000:
        tries += 1
        r = rng.uniform(r_min, r_max)
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        dx = _wrap_delta(x - cx, W)
        dy = y - cy
        dist = np.sqrt(dx * dx + dy * dy)
        inside = dist <= r
        trial = solid | inside
        if not percolates(trial):
            continue
        dep = r - dist
        better = inside & (dep < depth)
        dd = np.maximum(dist, 1e-12)
        nrm[..., 0] = np.where(better, dx / dd, nrm[..., 0])
        nrm[..., 1] = np.where(better, dy / dd, nrm[..., 1])
        depth = np.where(better, dep, depth)
        solid = trial
    normals = np.zeros((1, H, W, 3))
    normals[0, :, :, :2] = nrm
    return solid.astype(np.uint8)[None], normals, dict(porosity=1.0 - solid.mean())
