"""ctypes binding of ``liblbmrbc.so`` (the C ABI in ``include/lbmrbc.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of the shared library.  Device arrays are passed as torch tensors (their
``data_ptr()``); streams as torch streams.  There is no fallback: if the
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmrbc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbmrbc.h")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE, LBM_ENUMERIC, LBM_ECAPACITY = \
    0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
                -4: "LBM_ESTATE", -5: "LBM_ENUMERIC", -6: "LBM_ECAPACITY"}
LBM_FP64, LBM_FP32_DEV = 0, 1
LBM_PRECOLL, LBM_POSTCOLL = 0, 1
LBM_SNEW, LBM_SV, LBM_SPJ, LBM_ABB = 0, 1, 2, 3
LBM_BGK, LBM_TRT = 0, 1


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


class lbm_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("fluid_q", C.c_int32), ("solute_q", C.c_int32), ("precision", C.c_int32),
                ("rbc_mechanics", C.c_int32), ("rbc_scheme", C.c_int32),
                ("tau_ns", C.c_double), ("tau_ad", C.c_double), ("j0", C.c_double),
                ("force", C.c_double * 3), ("rho0", C.c_double), ("c_ref", C.c_double),
                ("c_eq", C.c_double), ("k_r", C.c_double), ("v_m", C.c_double),
                ("a_m", C.c_double), ("periodic", C.c_int32 * 3), ("xwrap_shift_y", C.c_int32),
                ("inlet_axis", C.c_int32), ("c_in", C.c_double), ("phase_change", C.c_int32),
                ("collision", C.c_int32), ("max_links", C.c_int64),
                ("fluid_open", C.c_int32), ("ceq_field", C.c_int32), ("u_in", C.c_double),
                ("rho_out", C.c_double)]


class lbm_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_events", C.c_int64), ("n_links", C.c_int64),
                ("n_solid_iface", C.c_int64), ("n_fluid", C.c_int64),
                ("n_fluid_iface", C.c_int64), ("mass_c", C.c_double), ("phi_sum", C.c_double),
                ("wall_exchange", C.c_double), ("nan_flag", C.c_int32), ("reserved0", C.c_int32),
                ("inlet_exchange", C.c_double), ("outlet_exchange", C.c_double),
                ("n_tasks", C.c_int64), ("n_row_words", C.c_int64)]


class lbm_launch_config(C.Structure):
    _fields_ = [("wg_waves", C.c_int32), ("xcd_remap", C.c_int32), ("graph_steps", C.c_int32),
                ("overlap", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "or python paper_2306_10794_amd/build.py")

# torch carries its own copy of the HIP runtime (same soname).  Loading torch
# first makes this library bind to that copy, so that both share one runtime
# and torch's device pointers are valid here; loaded the other way round, the
# process would hold two runtimes that do not know each other's allocations.
try:
    import torch  # noqa: F401
except ImportError:  # the ABI can still be inspected without torch
    pass

lib = C.CDLL(LIB_PATH)
_P = C.c_void_p
_SIGS = {
    "lbm_workspace_bytes": [C.POINTER(lbm_params), C.POINTER(C.c_size_t)],
    "lbm_create": [C.POINTER(lbm_params), _P, C.c_size_t, _P, C.POINTER(_P)],
    "lbm_batch_workspace_bytes": [C.POINTER(lbm_params), C.c_int32, C.POINTER(C.c_size_t)],
    "lbm_create_batch": [C.POINTER(lbm_params), C.c_int32, _P, C.c_size_t, _P, C.POINTER(_P)],
    "lbm_batch_offsets": [_P, C.POINTER(C.c_int64)],
    "lbm_set_geometry": [_P, _P, _P, _P, _P],
    "lbm_set_ceq": [_P, _P],
    "lbm_init_fields": [_P, _P, _P, _P],
    "lbm_step": [_P, C.c_int32],
    "lbm_step_timed": [_P, C.c_int32, C.POINTER(C.c_double)],
    "lbm_set_launch_config": [_P, C.POINTER(lbm_launch_config)],
    "lbm_get_launch_config": [_P, C.POINTER(lbm_launch_config)],
    "lbm_autotune": [_P, C.c_int32, C.POINTER(lbm_launch_config), C.POINTER(C.c_double),
                     C.POINTER(C.c_int64)],
    "lbm_adjoint_workspace_bytes": [_P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
    "lbm_record": [_P, C.c_int32, C.c_int32, _P, C.c_size_t],
    "lbm_adjoint": [_P, _P, _P],
    "lbm_record_static": [_P, C.c_int32, C.c_int32],
    "lbm_adjoint_timed": [_P, _P, _P, C.POINTER(C.c_double)],
    "lbm_get_fields": [_P, _P, _P, _P, _P, _P],
    "lbm_get_pops": [_P, _P, _P],
    "lbm_get_exchange": [_P, _P],
    "lbm_get_diag": [_P, C.POINTER(lbm_diag)],
    "lbm_state_bytes": [_P, C.POINTER(C.c_size_t)],
    "lbm_save_state": [_P, _P, C.c_size_t],
    "lbm_load_state": [_P, _P, C.c_size_t],
}
for _name, _args in _SIGS.items():
    fn = getattr(lib, _name)
    fn.argtypes = _args
    fn.restype = C.c_int
lib.lbm_last_error.argtypes = [_P]
lib.lbm_last_error.restype = C.c_char_p
lib.lbm_destroy.argtypes = [_P]
lib.lbm_destroy.restype = None


def header_symbols() -> list:
    """Function names declared in include/lbmrbc.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _check(status: int, where: str, ctx=None):
    if status != LBM_OK:
        msg = lib.lbm_last_error(ctx)
        raise LbmError(status, where, (msg or b"").decode())


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return getattr(stream, "cuda_stream", stream)


# ---- the C ABI, one Python function per entry point -------------------------
def lbm_last_error(ctx=None) -> str:
    return (lib.lbm_last_error(ctx) or b"").decode()


def lbm_workspace_bytes(params: lbm_params) -> int:
    n = C.c_size_t(0)
    _check(lib.lbm_workspace_bytes(C.byref(params), C.byref(n)), "lbm_workspace_bytes")
    return n.value


def lbm_create(params: lbm_params, workspace, nbytes: int, stream=None):
    h = C.c_void_p()
    _check(lib.lbm_create(C.byref(params), _ptr(workspace), nbytes, _stream_handle(stream),
                          C.byref(h)), "lbm_create")
    return h.value


def lbm_batch_workspace_bytes(params_list) -> int:
    arr = (lbm_params * len(params_list))(*params_list)
    n = C.c_size_t(0)
    _check(lib.lbm_batch_workspace_bytes(arr, len(params_list), C.byref(n)),
           "lbm_batch_workspace_bytes")
    return n.value


def lbm_create_batch(params_list, workspace, nbytes: int, stream=None):
    arr = (lbm_params * len(params_list))(*params_list)
    h = C.c_void_p()
    _check(lib.lbm_create_batch(arr, len(params_list), _ptr(workspace), nbytes,
                                _stream_handle(stream), C.byref(h)), "lbm_create_batch")
    return h.value


def lbm_batch_offsets(ctx, n: int) -> list:
    off = (C.c_int64 * (n + 1))()
    _check(lib.lbm_batch_offsets(ctx, off), "lbm_batch_offsets", ctx)
    return list(off)


def lbm_set_geometry(ctx, solid, normals=None, k_r=None, phi0=None):
    _check(lib.lbm_set_geometry(ctx, _ptr(solid), _ptr(normals), _ptr(k_r), _ptr(phi0)),
           "lbm_set_geometry", ctx)


def lbm_set_ceq(ctx, c_eq):
    _check(lib.lbm_set_ceq(ctx, _ptr(c_eq)), "lbm_set_ceq", ctx)


def lbm_init_fields(ctx, rho=None, u=None, c=None):
    _check(lib.lbm_init_fields(ctx, _ptr(rho), _ptr(u), _ptr(c)), "lbm_init_fields", ctx)


def lbm_step(ctx, nsteps: int):
    _check(lib.lbm_step(ctx, int(nsteps)), "lbm_step", ctx)


def lbm_step_timed(ctx, nsteps: int):
    """Returns (ms fused-step kernel, ms solid-fraction kernel), summed."""
    ms = (C.c_double * 2)()
    _check(lib.lbm_step_timed(ctx, int(nsteps), ms), "lbm_step_timed", ctx)
    return ms[0], ms[1]


def lbm_set_launch_config(ctx, wg_waves: int = 4, xcd_remap: int = 1, graph_steps: int = 0,
                          overlap: int = 0):
    cfg = lbm_launch_config(int(wg_waves), int(xcd_remap), int(graph_steps), int(overlap))
    _check(lib.lbm_set_launch_config(ctx, C.byref(cfg)), "lbm_set_launch_config", ctx)


def lbm_get_launch_config(ctx) -> dict:
    cfg = lbm_launch_config()
    _check(lib.lbm_get_launch_config(ctx, C.byref(cfg)), "lbm_get_launch_config", ctx)
    return dict(wg_waves=cfg.wg_waves, xcd_remap=cfg.xcd_remap, graph_steps=cfg.graph_steps,
                overlap=cfg.overlap)


def lbm_autotune(ctx, trial_steps: int):
    """Returns (chosen launch config as a dict, ms per step, steps run)."""
    cfg = lbm_launch_config()
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    _check(lib.lbm_autotune(ctx, int(trial_steps), C.byref(cfg), C.byref(ms), C.byref(n)),
           "lbm_autotune", ctx)
    return (dict(wg_waves=cfg.wg_waves, xcd_remap=cfg.xcd_remap, graph_steps=cfg.graph_steps,
                 overlap=cfg.overlap), ms.value, n.value)


def lbm_adjoint_workspace_bytes(ctx, nsteps: int, ckpt_every: int) -> int:
    n = C.c_size_t(0)
    _check(lib.lbm_adjoint_workspace_bytes(ctx, int(nsteps), int(ckpt_every), C.byref(n)),
           "lbm_adjoint_workspace_bytes", ctx)
    return n.value


def lbm_record(ctx, nsteps: int, ckpt_every: int, workspace, nbytes: int):
    _check(lib.lbm_record(ctx, int(nsteps), int(ckpt_every), _ptr(workspace), int(nbytes)),
           "lbm_record", ctx)


def lbm_record_static(ctx, nsteps: int, ckpt_every: int):
    _check(lib.lbm_record_static(ctx, int(nsteps), int(ckpt_every)), "lbm_record_static", ctx)


def lbm_adjoint(ctx, dL_dC, grad_k):
    _check(lib.lbm_adjoint(ctx, _ptr(dL_dC), _ptr(grad_k)), "lbm_adjoint", ctx)


def lbm_adjoint_timed(ctx, dL_dC, grad_k):
    """lbm_adjoint; returns (ms of the recomputation kernels, ms of the
    transposed-step kernels, ms of the per-segment dL/dbeta folds), summed
    over the backward pass."""
    ms = (C.c_double * 3)()
    _check(lib.lbm_adjoint_timed(ctx, _ptr(dL_dC), _ptr(grad_k), ms), "lbm_adjoint_timed", ctx)
    return ms[0], ms[1], ms[2]


def lbm_get_fields(ctx, rho=None, u=None, c=None, phi=None, type=None):
    _check(lib.lbm_get_fields(ctx, _ptr(rho), _ptr(u), _ptr(c), _ptr(phi), _ptr(type)),
           "lbm_get_fields", ctx)


def lbm_get_pops(ctx, f=None, g=None):
    _check(lib.lbm_get_pops(ctx, _ptr(f), _ptr(g)), "lbm_get_pops", ctx)


def lbm_get_exchange(ctx, q):
    _check(lib.lbm_get_exchange(ctx, _ptr(q)), "lbm_get_exchange", ctx)


def lbm_get_diag(ctx) -> dict:
    d = lbm_diag()
    st = lib.lbm_get_diag(ctx, C.byref(d))
    out = {name: getattr(d, name) for name, _ in lbm_diag._fields_ if not name.startswith("reserved")}
    if st not in (LBM_OK, LBM_ENUMERIC):
        _check(st, "lbm_get_diag", ctx)
    out["status"] = st
    return out


def lbm_state_bytes(ctx) -> int:
    n = C.c_size_t(0)
    _check(lib.lbm_state_bytes(ctx, C.byref(n)), "lbm_state_bytes", ctx)
    return n.value


def lbm_save_state(ctx, buf, nbytes: int):
    _check(lib.lbm_save_state(ctx, _ptr(buf), nbytes), "lbm_save_state", ctx)


def lbm_load_state(ctx, buf, nbytes: int):
    _check(lib.lbm_load_state(ctx, _ptr(buf), nbytes), "lbm_load_state", ctx)


def lbm_destroy(ctx):
    if ctx:
        lib.lbm_destroy(ctx)
