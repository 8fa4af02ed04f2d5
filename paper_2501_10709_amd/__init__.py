"""MI355X (gfx950) massively parallel trading-environment rollout.

The library (libfinrl_mi.so, C ABI in include/finrl_mi.h) runs the simulation phase of the
paper's producer-consumer training loop: N vectorised stock-trading environments stepped by a
K-actor ensemble, with hand-written HIP kernels.  This package is its thin Python binding.
"""
from . import binding
from .binding import (FM_BF16, FM_F32, FM_PATH_FUSED, FM_PATH_PLAIN, FmError, ensemble_act,
                      ensemble_create, ensemble_destroy, ensemble_workspace_bytes, env_create, env_day,
                      env_destroy, env_read_state, env_reset, env_rollout, env_step, env_workspace_bytes,
                      env_write_state, fm_last_error, fm_noise, fm_version)

__all__ = [
    "binding", "FM_BF16", "FM_F32", "FM_PATH_FUSED", "FM_PATH_PLAIN", "FmError", "ensemble_act",
    "ensemble_create", "ensemble_destroy", "ensemble_workspace_bytes", "env_create", "env_day",
    "env_destroy", "env_read_state", "env_reset", "env_rollout", "env_step", "env_workspace_bytes",
    "env_write_state", "fm_last_error", "fm_noise", "fm_version",
]
