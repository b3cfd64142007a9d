"""MI355X-native reactive lattice Boltzmann hot path (Weinmiller et al., 2023).

The compute lives in ``liblbmrbc.so`` (hand-written HIP for gfx950) behind the C
ABI of ``include/lbmrbc.h``; this package is its thin Python binding.
"""
from . import _lib
from ._lib import (LbmError, lbm_params, lbm_workspace_bytes, lbm_create, lbm_set_geometry, lbm_set_ceq,
                   lbm_batch_workspace_bytes, lbm_create_batch, lbm_batch_offsets,
                   lbm_init_fields, lbm_step, lbm_step_timed, lbm_set_launch_config,
                   lbm_get_launch_config, lbm_autotune, lbm_adjoint_workspace_bytes,
                   lbm_record, lbm_record_static, lbm_adjoint, lbm_adjoint_timed, lbm_get_fields, lbm_get_pops,
                   lbm_get_exchange,
                   lbm_get_diag, lbm_state_bytes, lbm_save_state, lbm_load_state,
                   lbm_last_error, lbm_destroy, LBM_FP64, LBM_FP32_DEV, LBM_PRECOLL,
                   LBM_POSTCOLL, LBM_SNEW, LBM_SV, LBM_SPJ, LBM_ABB, LBM_BGK, LBM_TRT, LBM_OK,
                   LBM_EINVAL,
                   LBM_ENOMEM, LBM_EDEVICE, LBM_ESTATE, LBM_ENUMERIC, LBM_ECAPACITY)

__all__ = [n for n in dir() if n.startswith("lbm_") or n.startswith("LBM_")] + [
    "LbmError", "Simulation", "BatchSimulation", "params_from_case", "RateToConcentration",
    "final_concentration"]


def __getattr__(name):
    # torch-based helpers are imported lazily so that the C ABI can be loaded
    # and inspected without initialising torch
    if name in ("Simulation", "BatchSimulation", "params_from_case", "RateToConcentration",
                "final_concentration"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
