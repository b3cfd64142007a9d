"""A small convenience wrapper around the C ABI for one lattice on one GPU.

torch provides the device memory (the workspace, input and output arrays) and
the stream; the library does all the work.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import _lib as L


def params_from_case(case, precision: int = L.LBM_FP32_DEV, max_links: int = 0) -> L.lbm_params:
    """lbm_params of an ``lbm_inputs.Case`` (plain field copy)."""
    p = L.lbm_params()
    p.dim, p.nx, p.ny, p.nz = case.dim, case.nx, case.ny, case.nz
    p.fluid_q = case.q
    p.solute_q = getattr(case, "qs", 0) or case.q
    p.precision = precision
    p.rbc_mechanics, p.rbc_scheme = case.mechanics, case.scheme
    p.tau_ns, p.tau_ad, p.j0 = case.tau_ns, case.tau_ad, case.j0
    p.force[:] = list(case.force)
    p.rho0, p.c_ref = case.rho0, case.c_ref
    p.c_eq, p.k_r, p.v_m, p.a_m = case.c_eq, case.k_r, case.v_m, case.a_m
    p.periodic[:] = list(case.periodic)
    p.xwrap_shift_y, p.inlet_axis, p.c_in = case.xwrap_shift_y, case.inlet_axis, case.c_in
    p.phase_change = case.phase_change
    p.collision = getattr(case, "collision", 0)
    p.max_links = max_links
    p.fluid_open = getattr(case, "fluid_open", 0)
    p.u_in, p.rho_out = getattr(case, "u_in", 0.0), getattr(case, "rho_out", 1.0)
    p.ceq_field = 0 if getattr(case, "c_eq_field", None) is None else 1
    return p


def _dev(a, dtype, device):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)


class Simulation:
    """One reactive-LBM context: workspace + geometry + state on ``device``."""

    def __init__(self, case, precision: int = L.LBM_FP32_DEV, device="cuda", stream=None,
                 max_links: int = 0, init: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("the reactive LBM library needs a GPU (none is visible)")
        self.case = case
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = params_from_case(case, precision, max_links)
        self.nbytes = L.lbm_workspace_bytes(self.params)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = L.lbm_create(self.params, self.workspace, self.nbytes, self.stream)
        self.N, self.Q = case.n, case.q
        self.QS = self.params.solute_q
        self._geom = dict(
            solid=_dev(case.solid_flat(), torch.uint8, self.device),
            normals=_dev(case.normals_flat(), torch.float64, self.device),
            k_r=_dev(case.k_r_field, torch.float64, self.device),
            phi0=_dev(case.phi0, torch.float64, self.device))
        if getattr(case, "c_eq_field", None) is not None:
            self._ceq = _dev(np.asarray(case.c_eq_field).reshape(-1), torch.float64, self.device)
            L.lbm_set_ceq(self.ctx, self._ceq)
        L.lbm_set_geometry(self.ctx, **self._geom)
        if init:
            self.init_fields(case.rho_flat(), case.u_flat(), case.c_flat())

    def init_fields(self, rho=None, u=None, c=None):
        self._init = [_dev(rho, torch.float64, self.device), _dev(u, torch.float64, self.device),
                      _dev(c, torch.float64, self.device)]
        L.lbm_init_fields(self.ctx, *self._init)

    def step(self, n: int = 1):
        L.lbm_step(self.ctx, n)

    def fields(self) -> dict:
        kw = dict(rho=torch.empty(self.N, dtype=torch.float64, device=self.device),
                  u=torch.empty((self.N, 3), dtype=torch.float64, device=self.device),
                  c=torch.empty(self.N, dtype=torch.float64, device=self.device),
                  phi=torch.empty(self.N, dtype=torch.float64, device=self.device),
                  type=torch.empty(self.N, dtype=torch.uint8, device=self.device))
        L.lbm_get_fields(self.ctx, **kw)
        return kw

    def pops(self):
        f = torch.empty((self.Q, self.N), dtype=torch.float64, device=self.device)
        g = torch.empty((self.QS, self.N), dtype=torch.float64, device=self.device)
        L.lbm_get_pops(self.ctx, f, g)
        return f, g

    def exchange(self):
        q = torch.empty((self.N, self.Q), dtype=torch.float64, device=self.device)
        L.lbm_get_exchange(self.ctx, q)
        return q

    def diag(self) -> dict:
        return L.lbm_get_diag(self.ctx)

    def set_rates(self, k_r):
        """New per-node rate constants (geometry prep again; the state must be
        initialised afterwards)."""
        self._geom["k_r"] = _dev(k_r, torch.float64, self.device)
        L.lbm_set_geometry(self.ctx, **self._geom)
        self.records = getattr(self, "records", 0) + 1

    def record(self, nsteps: int, ckpt_every: int):
        """Run nsteps steps keeping the checkpoints the adjoint needs."""
        n = L.lbm_adjoint_workspace_bytes(self.ctx, nsteps, ckpt_every)
        if getattr(self, "_adj_ws", None) is None or self._adj_ws.numel() < n:
            self._adj_ws = None
            self._adj_ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        L.lbm_record(self.ctx, nsteps, ckpt_every, self._adj_ws, self._adj_ws.numel())
        # a recorded run is identified by this counter: a later record (or a
        # new geometry) makes the gradients of earlier ones unavailable
        self.records = getattr(self, "records", 0) + 1

    def adjoint(self, dL_dC) -> torch.Tensor:
        """dL/dk_r [N] of the recorded run for dL/dC_T = dL_dC [N]."""
        dl = _dev(dL_dC, torch.float64, self.device)
        grad = torch.empty(self.N, dtype=torch.float64, device=self.device)
        L.lbm_adjoint(self.ctx, dl, grad)
        return grad

    def save_state(self) -> torch.Tensor:
        n = L.lbm_state_bytes(self.ctx)
        buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        L.lbm_save_state(self.ctx, buf, n)
        return buf

    def load_state(self, buf: torch.Tensor):
        L.lbm_load_state(self.ctx, buf, buf.numel())

    def close(self):
        if getattr(self, "ctx", None):
            L.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RateToConcentration(torch.autograd.Function):
    """C_T = final concentrations [N] of an nsteps run from the initial
    concentration c0, as a function of the per-node rate constants k_r [N];
    the backward pass is the library's hand-written adjoint (checkpoints every
    ckpt_every steps)."""

    @staticmethod
    def forward(ctx, k_r, sim, nsteps, ckpt_every, c0):
        sim.set_rates(k_r.detach())
        sim.init_fields(None, None, c0)
        sim.record(int(nsteps), int(ckpt_every))
        ctx.sim = sim
        ctx.record = sim.records
        return sim.fields()["c"]

    @staticmethod
    def backward(ctx, grad_c):
        if ctx.sim.records != ctx.record:
            raise RuntimeError("the simulation has recorded another run since this forward "
                               "call; its gradient is no longer available (use one Simulation "
                               "per live forward call)")
        return ctx.sim.adjoint(grad_c.contiguous()), None, None, None, None


def final_concentration(k_r, sim, nsteps: int, ckpt_every: int, c0=None):
    """Differentiable C_T(k_r) (see RateToConcentration)."""
    return RateToConcentration.apply(k_r, sim, nsteps, ckpt_every, c0)


class BatchSimulation:
    """Many independent domains stepped by the same launches (one context).

    Per-node arrays are the domains' arrays concatenated in domain order;
    ``offsets`` gives the first node of every domain.
    """

    def __init__(self, cases, precision: int = L.LBM_FP32_DEV, device="cuda", stream=None,
                 max_links: int = 0, init: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("the reactive LBM library needs a GPU (none is visible)")
        self.cases = list(cases)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = [params_from_case(c, precision, max_links) for c in self.cases]
        self.nbytes = L.lbm_batch_workspace_bytes(self.params)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = L.lbm_create_batch(self.params, self.workspace, self.nbytes, self.stream)
        self.offsets = L.lbm_batch_offsets(self.ctx, len(self.cases))
        self.N, self.Q = self.offsets[-1], self.cases[0].q
        self.QS = getattr(self.cases[0], "qs", 0) or self.Q

        def cat(get, dtype, width=None):
            parts = [get(c) for c in self.cases]
            if all(p is None for p in parts):
                return None
            full = []
            for c, p in zip(self.cases, parts):
                if p is None:
                    raise ValueError("an optional per-node array must be given for all domains "
                                     "of a batch or for none")
                full.append(np.asarray(p).reshape(c.n, -1) if width else np.asarray(p).reshape(-1))
            return _dev(np.concatenate(full), dtype, self.device)

        self._geom = dict(solid=cat(lambda c: c.solid_flat(), torch.uint8),
                          normals=cat(lambda c: c.normals_flat(), torch.float64, 3),
                          k_r=cat(lambda c: c.k_r_field, torch.float64),
                          phi0=cat(lambda c: c.phi0, torch.float64))
        self._ceq = cat(lambda c: getattr(c, "c_eq_field", None), torch.float64)
        if self._ceq is not None:
            L.lbm_set_ceq(self.ctx, self._ceq)
        L.lbm_set_geometry(self.ctx, **self._geom)
        if init:
            self._init = [cat(lambda c: c.rho_flat(), torch.float64),
                          cat(lambda c: c.u_flat(), torch.float64, 3),
                          cat(lambda c: c.c_flat(), torch.float64)]
            L.lbm_init_fields(self.ctx, *self._init)

    def step(self, n: int = 1):
        L.lbm_step(self.ctx, n)

    def split(self, t: torch.Tensor, axis: int = 0):
        """Per-domain views of a concatenated per-node tensor."""
        o = self.offsets
        return [t.narrow(axis, o[d], o[d + 1] - o[d]) for d in range(len(self.cases))]

    def fields(self) -> dict:
        kw = dict(rho=torch.empty(self.N, dtype=torch.float64, device=self.device),
                  u=torch.empty((self.N, 3), dtype=torch.float64, device=self.device),
                  c=torch.empty(self.N, dtype=torch.float64, device=self.device),
                  phi=torch.empty(self.N, dtype=torch.float64, device=self.device),
                  type=torch.empty(self.N, dtype=torch.uint8, device=self.device))
        L.lbm_get_fields(self.ctx, **kw)
        return kw

    def pops(self):
        f = torch.empty((self.Q, self.N), dtype=torch.float64, device=self.device)
        g = torch.empty((self.QS, self.N), dtype=torch.float64, device=self.device)
        L.lbm_get_pops(self.ctx, f, g)
        return f, g

    def exchange(self):
        q = torch.empty((self.N, self.Q), dtype=torch.float64, device=self.device)
        L.lbm_get_exchange(self.ctx, q)
        return q

    def diag(self) -> dict:
        return L.lbm_get_diag(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            L.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
