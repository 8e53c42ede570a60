"""ctypes declarations of the C-ABI in include/qfmi.h (argument marshalling only).

Loading fails loudly when libqfmi.so has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QFMI_LIB") or os.path.join(HERE, "libqfmi.so")  # QFMI_LIB: another build

QF_OK, QF_ERR_ARG, QF_ERR_PLAN, QF_ERR_WORKSPACE, QF_ERR_HIP, QF_ERR_UNSUPPORTED, QF_ERR_INJECTED = 0, -1, -2, -3, -4, -5, -6
QF_FP32, QF_BF16X3, QF_FP16 = 0, 1, 2
QF_OP_1Q, QF_OP_2Q_DIAG = 1, 2
QF_PLAN_NO_HOIST = 1
QF_PLAN_BACKWARD = 2
QF_PLAN_GRAPH = 4
QF_PLAN_NO_RENORM = 8
GEMM_VARIANTS = ("auto", "tiled4x4", "tiled2x2", "tiled1x2", "large", "skinny", "splitk", "simt", "tall")

STATUS_NAMES = {0: "QF_OK", -1: "QF_ERR_ARG", -2: "QF_ERR_PLAN", -3: "QF_ERR_WORKSPACE", -4: "QF_ERR_HIP",
                -5: "QF_ERR_UNSUPPORTED", -6: "QF_ERR_INJECTED"}


class qf_op(C.Structure):
    _fields_ = [("cycle", C.c_int32), ("kind", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("values", C.c_float * 8)]


class qf_cut(C.Structure):
    _fields_ = [("q0", C.c_int32), ("q1", C.c_int32), ("bit_lo", C.c_int32), ("nbits", C.c_int32)]


class qf_plan_desc(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("steps", C.POINTER(C.c_int32)), ("n_cuts", C.c_int32),
                ("cuts", C.POINTER(qf_cut)), ("n_open", C.c_int32), ("open", C.POINTER(C.c_int32)),
                ("precision", C.c_int32), ("flags", C.c_int32), ("batch", C.c_int32)]


class qf_plan_info(C.Structure):
    _fields_ = [("n_slices", C.c_int64), ("n_open", C.c_int32), ("n_steps", C.c_int32), ("peak_bits", C.c_int32),
                ("n_qubits", C.c_int32), ("flops_per_slice", C.c_double), ("flops_hoisted", C.c_double),
                ("flops_first_slice", C.c_double), ("flops_next_slice", C.c_double),
                ("permute_bytes", C.c_double), ("workspace_bytes", C.c_size_t),
                ("mfma_flops_per_slice", C.c_double)]


class qf_step_info(C.Structure):
    _fields_ = [("lhs", C.c_int32), ("rhs", C.c_int32), ("a_node", C.c_int32), ("b_node", C.c_int32),
                ("m_bits", C.c_int32), ("n_bits", C.c_int32), ("k_bits", C.c_int32),
                ("a_permuted", C.c_int32), ("b_permuted", C.c_int32), ("a_reordered", C.c_int32),
                ("b_reordered", C.c_int32), ("presplit", C.c_int32), ("persistent", C.c_int32),
                ("out_q", C.c_int32), ("out_nh", C.c_int32), ("out_split", C.c_int32),
                ("flops", C.c_double)]


EXPORTS = {
    "qf_ctx_create": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    "qf_ctx_set_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "qf_ctx_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "qf_ctx_destroy": (None, [C.c_void_p]),
    "qf_last_error": (C.c_char_p, [C.c_void_p]),
    "qf_circuit_create": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.POINTER(qf_op),
                                    C.POINTER(C.c_void_p)]),
    "qf_circuit_set_values": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "qf_circuit_destroy": (None, [C.c_void_p]),
    "qf_plan_step_info": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(qf_step_info)]),
    "qf_amplitudes_static": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]),
    "qf_static_scratch_bytes": (C.c_int, [C.POINTER(C.c_size_t)]),
    "qf_plan_graph_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "qf_plan_create": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(qf_plan_desc), C.POINTER(C.c_void_p)]),
    "qf_plan_info_get": (C.c_int, [C.c_void_p, C.POINTER(qf_plan_info)]),
    "qf_plan_destroy": (None, [C.c_void_p]),
    "qf_plan_flops": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_double)]),
    "qf_amplitudes": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]),
    "qf_backward": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]),
    "qf_permute": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.c_int64,
                             C.c_float]),
    "qf_cgemm": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int64]),
    "qf_cgemm_variant": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int64]),
    "qf_split_bf16": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "qf_split_f16": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int]),
    "qf_cgemm_presplit": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_int64, C.c_int64]),
    "qf_time_cgemm_presplit": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int,
                                         C.POINTER(C.c_float)]),
    "qf_time_cgemm": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_int, C.POINTER(C.c_float)]),
    "qf_time_permute": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.c_int,
                                  C.POINTER(C.c_float)]),
    "qf_time_ceiling": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int64, C.c_int, C.POINTER(C.c_float),
                                  C.POINTER(C.c_double)]),
    "qf_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "qf_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_char_p]),
    "qf_tuned_variant": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                   C.POINTER(C.c_int)]),
    "qf_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.c_int]),
}

_lib = None


def load() -> C.CDLL:
    """Load libqfmi.so (raises if it is missing: build it with python -m paper_1905_00444_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run: python -m paper_1905_00444_amd.build)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class QfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, ctx=None) -> None:
    if status != QF_OK:
        msg = load().qf_last_error(ctx).decode() if ctx else ""
        raise QfError(status, msg)
