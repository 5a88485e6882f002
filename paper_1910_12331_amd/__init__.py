"""MI355X-native Gauss-Newton (preconditioned implicit CG) and ALS for dense CP decomposition.

The compute path is libcpgn.so (HIP kernels for gfx950 behind the C ABI in include/cpgn.h);
this package is its Python binding.
"""
from . import _lib
from .api import (CpError, SplitBF16Tensor, Workspace, als_sweep, armijo_stats_buffer,
                  BegunStep, GNBatchProgram, damping_advance, device_clock_hz, device_timestamp, gn_cg_batch, gn_step_begin, gn_step_end, factor_dtype, gn_gradient, gn_step, gn_step_armijo,
                  gn_step_devlam, gn_step_noalloc, jtj_matvec, objective_gradient, mttkrp, mttkrp_all, read_armijo_stats, read_stats,
                  residual, stats_buffer, to_bf16, Tiles, set_tiles, get_tiles, tiles)
from .autograd import CPObjective, cp_objective
from .optim import (ALS, Acceptance, Armijo, BatchedGaussNewton, BatchedTuning, ConstantDamping,
                    DampingSchedule, GaussNewton, GNConfig, StepDecay, autotune_batched, batch_key,
                    gn_ladder_to_target, gn_mixed_to_target, gn_to_target)

__all__ = ["CpError", "SplitBF16Tensor", "factor_dtype", "to_bf16", "Workspace", "als_sweep", "gn_gradient", "gn_step", "gn_step_devlam", "gn_step_noalloc", "gn_step_armijo", "armijo_stats_buffer", "read_armijo_stats", "BegunStep", "GNBatchProgram", "gn_step_begin", "gn_cg_batch", "gn_step_end", "damping_advance", "device_clock_hz", "device_timestamp", "jtj_matvec", "objective_gradient", "mttkrp", "mttkrp_all",
           "read_stats", "residual", "stats_buffer", "Tiles", "set_tiles", "get_tiles", "tiles", "ALS", "Acceptance", "Armijo", "ConstantDamping", "StepDecay", "BatchedTuning", "autotune_batched", "batch_key", "DampingSchedule", "GaussNewton",
           "GNConfig", "BatchedGaussNewton", "gn_to_target", "gn_mixed_to_target", "gn_ladder_to_target", "CPObjective", "cp_objective"]
