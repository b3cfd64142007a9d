"""Problem description shared, as plain data, by every consumer of a workload.

A ``Case`` carries the lattice dimensions, the physical and lattice parameters
and the seeded geometry arrays.  It holds no part of the lattice Boltzmann
arithmetic: the FP64 reference and the GPU library each read the same bytes
and do their own computation.

Node ordering everywhere is x fastest, then y, then z (C order over
``[nz][ny][nx]``); node index ``n = x + nx * (y + ny * z)``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

# Selector values (mirrored by name in the C header and the reference).
MECH_PRE = 0    # RBC source: pre-collision population at the fluid boundary node
MECH_POST = 1   # RBC source: own post-collision population streamed to the wall
SCHEME_SNEW = 0
SCHEME_SV = 1
SCHEME_SPJ = 2
SCHEME_ABB = 3


@dataclasses.dataclass
class Case:
    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    q: int                      # fluid lattice: 9 (D2Q9) or 19 (D3Q19)
    solid: np.ndarray           # uint8 [nz, ny, nx], 1 = solid
    tau_ns: float = 1.0
    tau_ad: float = 1.0
    j0: float = -1.0            # rest fraction; < 0 selects the standard lattice weights
    force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    c_eq: float = 1.0
    k_r: float = 0.0            # uniform rate constant (used where k_r_field is None)
    v_m: float = 0.0
    a_m: float = 1.0
    periodic: Tuple[int, int, int] = (1, 1, 1)
    xwrap_shift_y: int = 0
    inlet_axis: int = -1
    c_in: float = 0.0
    mechanics: int = MECH_PRE
    scheme: int = SCHEME_SNEW
    rho0: float = 1.0           # deviation reference for the fluid populations
    c_ref: float = 0.0          # deviation reference for the solute populations
    phase_change: int = 0
    collision: int = 0          # 0 BGK, 1 TRT (magic parameter 3/16 for both lattices)
    qs: int = 0                 # solute lattice: 0 (the fluid's), 5 (D2Q5) or 7 (D3Q7)
    fluid_open: int = 0         # 1: plug inflow u_in at the inlet face, density rho_out
    u_in: float = 0.0           #    at the outlet face (inlet axis not periodic)
    rho_out: float = 1.0
    c_eq_field: Optional[np.ndarray] = None  # float64 [N]: per-node C_eq at solid nodes
    normals: Optional[np.ndarray] = None   # float64 [N, 3], unit normal solid -> fluid
    k_r_field: Optional[np.ndarray] = None  # float64 [N]
    phi0: Optional[np.ndarray] = None       # float64 [N]
    rho_init: Optional[np.ndarray] = None   # float64 [N]
    u_init: Optional[np.ndarray] = None     # float64 [N, 3]
    c_init: Optional[np.ndarray] = None     # float64 [N]
    c0: float = 0.0             # uniform initial concentration where c_init is None
    steps: int = 0              # step count of the workload as specified
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_fluid(self) -> int:
        return int(self.n - int(self.solid.sum()))

    def solid_flat(self) -> np.ndarray:
        return np.ascontiguousarray(self.solid.reshape(-1), dtype=np.uint8)

    def normals_flat(self) -> Optional[np.ndarray]:
        if self.normals is None:
            return None
        return np.ascontiguousarray(self.normals.reshape(self.n, 3), dtype=np.float64)

    def rho_flat(self) -> np.ndarray:
        if self.rho_init is None:
            return np.ones(self.n, dtype=np.float64)
        return np.ascontiguousarray(self.rho_init.reshape(-1), dtype=np.float64)

    def u_flat(self) -> np.ndarray:
        if self.u_init is None:
            return np.zeros((self.n, 3), dtype=np.float64)
        return np.ascontiguousarray(self.u_init.reshape(self.n, 3), dtype=np.float64)

    def c_flat(self) -> np.ndarray:
        if self.c_init is None:
            return np.full(self.n, self.c0, dtype=np.float64)
        return np.ascontiguousarray(self.c_init.reshape(-1), dtype=np.float64)

    def replace(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)
