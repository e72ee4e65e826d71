"""Batched JAGP wave function on MI355X (gfx950): HIP kernels behind a C ABI.

The compute lives in libqmc_jagp.so (see include/qmc.h); `binding` marshals
torch device tensors into its calls.
"""
from .binding import (JAGPSystem, Walkers, QMCError, JAGPFunction, MultiSystem, philox_draws, QMC_FP64,  # noqa: F401
                      QMC_W_FP32, QMC_MIXED, QMC_MIXED_BF16, QMC_W_BF16, QMC_W_FP8, QMC_REFINED, WALKERS_ADJOINT, load,
                      STATE_R, STATE_LOGABS, STATE_SIGN, STATE_W, STATE_AINV, STATE_PHI, STATE_RESIDUAL, STATE_KEPT, LR_TERMS,
                      swct, reweight, sr_step, workspace_size)
