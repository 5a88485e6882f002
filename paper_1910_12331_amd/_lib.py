"""ctypes declarations of the libcpgn.so C ABI (include/cpgn.h). Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpgn.so")

MAX_ORDER = 8
CP_F64, CP_F32, CP_BF16, CP_BF16X3 = 0, 1, 2, 3
CP_OK, CP_EINVAL, CP_EUNSUPPORTED, CP_EWORKSPACE, CP_EHIP = 0, -1, -2, -3, -4
CP_ENOTSPD, CP_EBREAKDOWN, CP_ENONFINITE, CP_ESCRATCH = -5, -6, -7, -8
NOALLOC_SCRATCH_BYTES = 64 << 20
OP_MTTKRP, OP_GN_GRADIENT, OP_GN_JTJ_MATVEC, OP_GN_STEP, OP_ALS_SWEEP, OP_RESIDUAL, OP_MTTKRP_ALL = range(7)
GN_DIAG_DAMPING = 1
GN_CHOL_PRECOND = 2
LS_F0_GIVEN = 1
RESIDUAL_DIRECT, RESIDUAL_EXPANSION = 0, 1

EXPORTS = ["cp_workspace_bytes", "cp_mttkrp", "cp_mttkrp_marked", "cp_mttkrp_all", "cp_gn_gradient", "cp_objective_gradient", "cp_gn_jtj_matvec", "cp_gn_step",
           "cp_gn_step_devlam", "cp_gn_step_noalloc", "cp_gn_step_armijo", "cp_damping_advance", "cp_gn_step_begin", "cp_gn_cg_batch", "cp_gn_step_end", "cp_gn_batch_create", "cp_gn_batch_step", "cp_gn_batch_destroy", "cp_device_timestamp", "cp_device_clock_hz", "cp_als_sweep", "cp_residual",
           "cp_tensor_to_bf16", "cp_set_tuning", "cp_get_tuning", "cp_status_string", "cp_abi_version"]


class CpProblem(C.Structure):
    _fields_ = [("order", C.c_int32), ("rank", C.c_int32), ("dims", C.c_int64 * MAX_ORDER),
                ("x_dtype", C.c_int32), ("f_dtype", C.c_int32)]


class CpGnParams(C.Structure):
    _fields_ = [("lam", C.c_double), ("cg_tol", C.c_double), ("cg_maxiter", C.c_int32),
                ("flags", C.c_uint32)]


class CpGnStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("cg_iters", C.c_int32), ("grad_norm_sum", C.c_double),
                ("cg_res_norm_sum", C.c_double), ("alpha_last", C.c_double),
                ("beta_last", C.c_double), ("update_norm", C.c_double)]


class CpArmijoParams(C.Structure):
    _fields_ = [("c", C.c_double), ("shrink", C.c_double), ("max_trials", C.c_int32),
                ("flags", C.c_uint32)]


class CpArmijoStats(C.Structure):
    _fields_ = [("alpha", C.c_double), ("f0", C.c_double), ("f", C.c_double), ("gv", C.c_double),
                ("x_norm", C.c_double), ("trials", C.c_int32), ("accepted", C.c_int32)]


class CpTuning(C.Structure):
    _fields_ = [("mttkrp_min_items", C.c_int32), ("mttkrp_wg_per_cu", C.c_int32),
                ("mttkrp_row_block", C.c_int32), ("reserved", C.c_int32)]


PTRS = C.c_void_p * MAX_ORDER
MAX_CG_BATCH = 128
_lib = None


def load(path: str = LIB_PATH):
    """Load libcpgn.so and declare its signatures. Raises if the library was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1910_12331_amd.build`")
    lib = C.CDLL(path)
    vp, sz, i32 = C.c_void_p, C.c_size_t, C.c_int
    P = C.POINTER
    lib.cp_abi_version.restype = i32
    lib.cp_abi_version.argtypes = []
    lib.cp_status_string.restype = C.c_char_p
    lib.cp_status_string.argtypes = [i32]
    lib.cp_workspace_bytes.restype = i32
    lib.cp_workspace_bytes.argtypes = [P(CpProblem), i32, P(sz)]
    lib.cp_mttkrp.restype = i32
    lib.cp_mttkrp.argtypes = [P(CpProblem), vp, PTRS, i32, vp, vp, sz, vp]
    lib.cp_mttkrp_marked.restype = i32
    lib.cp_mttkrp_marked.argtypes = [P(CpProblem), vp, PTRS, i32, vp, vp, sz, vp, vp, vp]
    lib.cp_mttkrp_all.restype = i32
    lib.cp_mttkrp_all.argtypes = [P(CpProblem), vp, PTRS, PTRS, vp, sz, vp]
    lib.cp_gn_gradient.restype = i32
    lib.cp_gn_gradient.argtypes = [P(CpProblem), vp, PTRS, PTRS, vp, vp, sz, vp]
    lib.cp_objective_gradient.restype = i32
    lib.cp_objective_gradient.argtypes = [P(CpProblem), vp, PTRS, PTRS, vp, vp, sz, vp]
    lib.cp_gn_jtj_matvec.restype = i32
    lib.cp_gn_jtj_matvec.argtypes = [P(CpProblem), PTRS, PTRS, C.c_double, PTRS, vp, sz, vp]
    lib.cp_gn_step.restype = i32
    lib.cp_gn_step.argtypes = [P(CpProblem), vp, PTRS, P(CpGnParams), vp, vp, sz, vp]
    lib.cp_gn_step_devlam.restype = i32
    lib.cp_gn_step_devlam.argtypes = [P(CpProblem), vp, PTRS, P(CpGnParams), vp, vp, vp, sz, vp]
    lib.cp_gn_step_noalloc.restype = i32
    lib.cp_gn_step_noalloc.argtypes = [P(CpProblem), vp, PTRS, P(CpGnParams), vp, vp]
    lib.cp_gn_step_armijo.restype = i32
    lib.cp_gn_step_armijo.argtypes = [P(CpProblem), vp, PTRS, P(CpGnParams), P(CpArmijoParams),
                                      vp, vp, vp, sz, vp]
    lib.cp_damping_advance.restype = i32
    lib.cp_damping_advance.argtypes = [vp, vp]
    lib.cp_gn_step_begin.restype = i32
    lib.cp_gn_step_begin.argtypes = [P(CpProblem), vp, PTRS, P(CpGnParams), vp, vp, sz, vp]
    lib.cp_gn_cg_batch.restype = i32
    lib.cp_gn_cg_batch.argtypes = [i32, P(CpProblem), P(vp), P(sz), i32, vp]
    lib.cp_gn_step_end.restype = i32
    lib.cp_gn_step_end.argtypes = [P(CpProblem), PTRS, vp, vp, sz, vp]
    lib.cp_gn_batch_create.restype = i32
    lib.cp_gn_batch_create.argtypes = [i32, P(CpProblem), P(vp), P(vp), P(CpGnParams), P(vp),
                                       P(vp), P(vp), P(vp), P(sz), vp, sz, P(sz), P(vp)]
    lib.cp_gn_batch_step.restype = i32
    lib.cp_gn_batch_step.argtypes = [vp, vp]
    lib.cp_gn_batch_destroy.restype = i32
    lib.cp_gn_batch_destroy.argtypes = [vp]
    lib.cp_device_timestamp.restype = i32
    lib.cp_device_timestamp.argtypes = [vp, vp]
    lib.cp_device_clock_hz.restype = i32
    lib.cp_device_clock_hz.argtypes = [P(C.c_int64)]
    lib.cp_als_sweep.restype = i32
    lib.cp_als_sweep.argtypes = [P(CpProblem), vp, PTRS, C.c_double, vp, vp, sz, vp]
    lib.cp_residual.restype = i32
    lib.cp_residual.argtypes = [P(CpProblem), vp, PTRS, i32, vp, vp, sz, vp]
    lib.cp_tensor_to_bf16.restype = i32
    lib.cp_tensor_to_bf16.argtypes = [vp, C.c_int64, i32, vp, vp]
    lib.cp_set_tuning.restype = i32
    lib.cp_set_tuning.argtypes = [P(CpTuning)]
    lib.cp_get_tuning.restype = i32
    lib.cp_get_tuning.argtypes = [P(CpTuning)]
    if lib.cp_abi_version() != 1:
        raise RuntimeError("libcpgn.so ABI version mismatch")
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().cp_status_string(int(code)).decode()
