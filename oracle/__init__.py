"""FP64 CPU oracle of the reactive lattice Boltzmann step (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package.  The product library never imports it, and
it imports nothing from the product.  The C source is ``lbm_oracle.c``; see its
header for the paper passages each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(force: bool = False, src: str = SRC, lib: str = LIB) -> str:
    """Compile the oracle with gcc (plain -O3, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, lib)
    return lib


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("q", C.c_int), ("mechanics", C.c_int), ("scheme", C.c_int),
                ("tau_ns", C.c_double), ("tau_ad", C.c_double), ("j0", C.c_double),
                ("force", C.c_double * 3), ("c_eq", C.c_double), ("k_r", C.c_double),
                ("v_m", C.c_double), ("a_m", C.c_double), ("periodic", C.c_int * 3),
                ("xwrap_shift_y", C.c_int), ("inlet_axis", C.c_int), ("c_in", C.c_double),
                ("phase_change", C.c_int), ("collision", C.c_int), ("qs", C.c_int),
                ("fluid_open", C.c_int), ("u_in", C.c_double), ("rho_out", C.c_double)]


_lib = None


def _bind(lib):
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [C.POINTER(_Params), P, P, P, P]
    lib.orc_destroy.argtypes = [P]
    lib.orc_init.argtypes = [P, P, P, P]
    lib.orc_step.argtypes = [P, C.c_int]
    lib.orc_get_fields.argtypes = [P, P, P, P, P, P]
    lib.orc_get_pops.argtypes = [P, P, P]
    lib.orc_set_pops.argtypes = [P, P, P]
    lib.orc_get_exchange.argtypes = [P, P, P]
    lib.orc_get_link_k.argtypes = [P, P]
    lib.orc_get_lattice.argtypes = [P, P, P, P, P]
    lib.orc_get_normals.argtypes = [P, P]
    lib.orc_diag.argtypes = [P, dp]
    lib.orc_adjoint.restype = C.c_int
    lib.orc_adjoint.argtypes = [P, C.c_int, P, P, P]
    lib.orc_threads.restype = C.c_int
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_ceq.argtypes = [P, P]
    lib.orc_get_solute_set.restype = C.c_int
    lib.orc_get_solute_set.argtypes = [P, P]
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = _bind(C.CDLL(build()))
    return _lib


def load_variant(source: str, directory: str):
    """Compile ``source`` (a modified copy of lbm_oracle.c) into ``directory``
    and return the loaded library, for ``Oracle(case, lib=...)``.  The test
    suite uses this to check that its pins reject planted mistakes."""
    src = os.path.join(directory, "lbm_oracle_variant.c")
    with open(src, "w") as fh:
        fh.write(source)
    return _bind(C.CDLL(build(force=True, src=src,
                              lib=os.path.join(directory, "liblbm_oracle_variant.so"))))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def threads() -> int:
    return int(_load().orc_threads())


def set_threads(n: int):
    """Threads of the oracle's node loop from now on (CPU-baseline timing)."""
    _load().orc_set_threads(int(n))


class Oracle:
    """Stateful FP64 reference run of one ``lbm_inputs.Case``."""

    def __init__(self, case, init: bool = True, lib=None):
        lib = _load() if lib is None else lib
        self._lib = lib
        self.case = case
        p = _Params()
        p.dim, p.nx, p.ny, p.nz, p.q = case.dim, case.nx, case.ny, case.nz, case.q
        p.mechanics, p.scheme = case.mechanics, case.scheme
        p.tau_ns, p.tau_ad, p.j0 = case.tau_ns, case.tau_ad, case.j0
        p.force[:] = list(case.force)
        p.c_eq, p.k_r, p.v_m, p.a_m = case.c_eq, case.k_r, case.v_m, case.a_m
        p.periodic[:] = list(case.periodic)
        p.xwrap_shift_y, p.inlet_axis, p.c_in = case.xwrap_shift_y, case.inlet_axis, case.c_in
        p.phase_change = case.phase_change
        p.collision = getattr(case, "collision", 0)
        p.qs = getattr(case, "qs", 0)
        p.fluid_open = getattr(case, "fluid_open", 0)
        p.u_in, p.rho_out = getattr(case, "u_in", 0.0), getattr(case, "rho_out", 1.0)
        self._solid = case.solid_flat()
        self._normals = case.normals_flat()
        self._kr = None if case.k_r_field is None else np.ascontiguousarray(case.k_r_field, np.float64)
        self._phi0 = None if case.phi0 is None else np.ascontiguousarray(case.phi0, np.float64)
        self._h = lib.orc_create(C.byref(p), _ptr(self._solid), _ptr(self._normals),
                                 _ptr(self._kr), _ptr(self._phi0))
        if not self._h:
            raise ValueError(f"oracle refuses solute lattice qs={p.qs} with q={p.q}")
        self.N, self.Q = case.n, case.q
        sd = np.empty(19, np.int32)
        self.QS = int(lib.orc_get_solute_set(self._h, _ptr(sd)))
        self.sdirs = sd[:self.QS].copy()
        ceq = getattr(case, "c_eq_field", None)
        if ceq is not None:
            self._ceq = np.ascontiguousarray(ceq, np.float64).reshape(-1)
            lib.orc_set_ceq(self._h, _ptr(self._ceq))
        if init:
            self.init(case.rho_flat(), case.u_flat(), case.c_flat())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def init(self, rho=None, u=None, c=None):
        rho = None if rho is None else np.ascontiguousarray(rho, np.float64)
        u = None if u is None else np.ascontiguousarray(u, np.float64)
        c = None if c is None else np.ascontiguousarray(c, np.float64)
        self._lib.orc_init(self._h, _ptr(rho), _ptr(u), _ptr(c))

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, int(n))

    def fields(self) -> dict:
        N = self.N
        rho, u, c, phi = (np.empty(N), np.empty((N, 3)), np.empty(N), np.empty(N))
        typ = np.empty(N, np.uint8)
        self._lib.orc_get_fields(self._h, _ptr(rho), _ptr(u), _ptr(c), _ptr(phi), _ptr(typ))
        return dict(rho=rho, u=u, c=c, phi=phi, type=typ)

    def pops(self):
        """(f [Q, N], g [QS, N]); g in the solute set's order."""
        f = np.empty((self.Q, self.N))
        g = np.empty((self.QS, self.N))
        self._lib.orc_get_pops(self._h, _ptr(f), _ptr(g))
        return f, g

    def set_pops(self, f=None, g=None):
        f = None if f is None else np.ascontiguousarray(f, np.float64)
        g = None if g is None else np.ascontiguousarray(g, np.float64)
        self._lib.orc_set_pops(self._h, _ptr(f), _ptr(g))

    def exchange(self):
        """(q [N,Q], kind [N,Q]) of the last step; kind 1 marks reactive links."""
        q = np.empty((self.N, self.Q))
        kind = np.empty((self.N, self.Q), np.uint8)
        self._lib.orc_get_exchange(self._h, _ptr(q), _ptr(kind))
        return q, kind

    def link_k(self):
        k = np.empty((self.N, self.Q))
        self._lib.orc_get_link_k(self._h, _ptr(k))
        return k

    def normals(self):
        n = np.empty((self.N, 3))
        self._lib.orc_get_normals(self._h, _ptr(n))
        return n

    def lattice(self):
        e = np.empty((self.Q, 3), np.int32)
        wf, ws, cs2 = np.empty(self.Q), np.empty(self.Q), np.empty(2)
        self._lib.orc_get_lattice(self._h, _ptr(e), _ptr(wf), _ptr(ws), _ptr(cs2))
        # ws by fluid direction (0 outside the solute set); sd: the fluid
        # direction of each solute direction
        return dict(e=e, wf=wf, ws=ws, cs2f=cs2[0], cs2s=cs2[1], sd=self.sdirs.copy())

    def adjoint(self, nsteps: int, dLdC, want_lam0: bool = False):
        """Runs nsteps forward, then the adjoint of a loss with gradient dLdC [N]
        with respect to the final concentrations.  Returns (dL/dk_r [N],
        dL/dg*(0) as [Q, N] or None)."""
        dLdC = np.ascontiguousarray(dLdC, np.float64)
        grad = np.zeros(self.N)
        lam0 = np.zeros((self.N, self.Q)) if want_lam0 else None
        rc = self._lib.orc_adjoint(self._h, int(nsteps), _ptr(dLdC), _ptr(grad), _ptr(lam0))
        if rc != 0:
            raise RuntimeError(f"orc_adjoint failed ({rc})")
        return grad, (None if lam0 is None else np.ascontiguousarray(lam0.T))

    def diag(self) -> dict:
        d = (C.c_double * 7)()
        self._lib.orc_diag(self._h, d)
        return dict(mass_c=d[0], phi_sum=d[1], wall_exchange=d[2], inlet_exchange=d[3],
                    outlet_exchange=d[4], step=int(d[5]), n_events=int(d[6]))
