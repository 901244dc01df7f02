"""ctypes binding of libmitnc.so: the C ABI of include/mitnc.h, same names.

Argument marshalling only.  Loading fails loudly when the library has not
been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmitnc.so")

MITNC_OK = 0
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "PATH_INVALID", -3: "WORKSPACE_TOO_SMALL",
                -4: "HIP_ERROR", -5: "UNSUPPORTED", -6: "NUMERIC"}
MITNC_C64, MITNC_CF16, MITNC_CBF16 = 0, 1, 2
K_SMALL, K_STEM, K_TILE, K_TALL, K_SPLITK = 0, 1, 2, 3, 4
KERNEL_NAMES = {0: "small", 1: "stem", 2: "tile", 3: "tall", 4: "splitk", 5: "stream", 6: "section"}


class MitncError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class mitnc_gate(C.Structure):
    _fields_ = [("arity", C.c_int32), ("q0", C.c_int32), ("q1", C.c_int32),
                ("mat", C.POINTER(C.c_double))]


class mitnc_search_opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("trials", C.c_int32), ("max_log2_elems", C.c_int32),
                ("min_sliced", C.c_int32), ("max_sliced", C.c_int32), ("keep_slicing", C.c_int32),
                ("method", C.c_int32), ("window_bits", C.c_int32), ("merge_bits", C.c_int32),
                ("branch_exchange", C.c_int32), ("launch_cost_flops", C.c_double)]


class mitnc_plan_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("reuse", C.c_int32),
                ("cache_budget_bytes", C.c_uint64), ("force_kernel", C.c_int32),
                ("differentiable", C.c_int32), ("fuse_sections", C.c_int32), ("no_rerun", C.c_int32),
                ("splitk_max_mn_bits", C.c_int32), ("splitk_target_bits", C.c_int32),
                ("merge_bits", C.c_int32), ("no_hoist", C.c_int32), ("prologue_bits", C.c_int32),
                ("reverse_defer", C.c_int32)]


class mitnc_plan_stats(C.Structure):
    _fields_ = [("workspace_bytes", C.c_uint64), ("result_elems", C.c_uint64),
                ("n_sliced", C.c_int32), ("n_steps", C.c_int32), ("max_log2_elems", C.c_int32),
                ("n_kernel_classes", C.c_int32),
                ("flops_full_slice", C.c_double), ("flops_reused_slice", C.c_double),
                ("bytes_full_slice", C.c_double), ("bytes_reused_slice", C.c_double),
                ("steps_by_class", C.c_int32 * 8), ("flops_by_class", C.c_double * 8),
                ("n_grad_gates", C.c_int32), ("n_reverse_ops", C.c_int32),
                ("flops_reverse_slice", C.c_double), ("n_merged", C.c_int32),
                ("merge_align_bits", C.c_int32), ("merged_mask", C.c_uint64), ("n_reverse_groups", C.c_int32),
                ("n_batched_small", C.c_int32), ("n_batched_launches", C.c_int32)]


class mitnc_step_info(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("out", C.c_int32), ("root", C.c_int32),
                ("kernel_class", C.c_int32), ("section", C.c_int32), ("section_pos", C.c_int32),
                ("section_len", C.c_int32), ("mb", C.c_int32), ("nb", C.c_int32), ("kb", C.c_int32),
                ("bb", C.c_int32)] + [(f, C.c_uint8 * 32) for f in ("am", "ak", "ab", "bk", "bn", "bbt",
                                                                     "cm", "cn", "cb")] + [
        ("tm", C.c_int32), ("tn", C.c_int32), ("tk", C.c_int32), ("a_tile", C.c_uint8 * 16),
        ("b_tile", C.c_uint8 * 16), ("lds_a_swz", C.c_uint8 * 8), ("lds_b_swz", C.c_uint8 * 8),
        ("lds_a_row", C.c_uint16 * 8), ("lds_b_row", C.c_uint16 * 8), ("lds_k_col", C.c_uint8 * 8),
        ("vec_a", C.c_int32), ("vec_b", C.c_int32)]


class mitnc_node_info(C.Structure):
    _fields_ = [("is_leaf", C.c_int32), ("rank", C.c_int32), ("full_rank", C.c_int32), ("level", C.c_int32),
                ("hoisted", C.c_int32), ("n_slice_bits", C.c_int32), ("slice_bit", C.c_int32 * 64),
                ("slice_pos", C.c_int32 * 64), ("ws_offset", C.c_uint64), ("elig_mask", C.c_uint64),
                ("recompute_mask", C.c_uint64), ("merge_mask", C.c_uint64), ("merge_tmp_offset", C.c_uint64)]


_VP = C.c_void_p
_I32 = C.c_int32
_SIGS = {
    "mitnc_network_from_circuit": [_I32, _I32, C.POINTER(mitnc_gate), C.POINTER(_VP)],
    "mitnc_network_set_output": [_VP, C.POINTER(C.c_int8), _I32, C.POINTER(C.c_uint8)],
    "mitnc_network_info": [_VP, C.POINTER(_I32), C.POINTER(_I32)],
    "mitnc_path_search": [_VP, C.POINTER(mitnc_search_opts)],
    "mitnc_get_path": [_VP, C.POINTER(_I32)],
    "mitnc_set_path": [_VP, _I32, C.POINTER(_I32)],
    "mitnc_get_slicing": [_VP, C.POINTER(_I32), C.POINTER(C.c_int64)],
    "mitnc_set_slicing": [_VP, _I32, C.POINTER(C.c_int64)],
    "mitnc_slice_greedy": [_VP, _I32, _I32, _I32, C.POINTER(_I32), C.POINTER(C.c_int64)],
    "mitnc_index_overhead": [_VP, C.c_int64, C.POINTER(C.c_double)],
    "mitnc_branch_exchange": [_VP, _I32, _I32, _I32, _I32, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)],
    "mitnc_plan_create": [_VP, C.POINTER(mitnc_plan_opts), C.POINTER(_VP)],
    "mitnc_plan_query": [_VP, C.POINTER(mitnc_plan_stats)],
    "mitnc_plan_steps": [_VP, C.POINTER(C.c_double)],
    "mitnc_plan_step_info": [_VP, _I32, C.POINTER(mitnc_step_info)],
    "mitnc_plan_reverse_info": [_VP, _I32, C.POINTER(mitnc_step_info), C.POINTER(_I32)],
    "mitnc_plan_node_info": [_VP, _I32, C.POINTER(mitnc_node_info)],
    "mitnc_plan_schedule": [_VP, C.c_uint64, C.c_uint64, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "mitnc_plan_leaf_data": [_VP, _I32, C.POINTER(C.c_float), C.c_uint64, C.POINTER(C.c_uint64)],
    "mitnc_plan_upload": [_VP, _VP, C.c_size_t, _VP],
    "mitnc_execute": [_VP, _VP, C.c_size_t, C.c_uint64, C.c_uint64, _VP, _VP],
    "mitnc_plan_timing": [_VP, _I32],
    "mitnc_plan_timing_read": [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)],
    "mitnc_calibrate": [_VP, _VP, C.c_size_t, C.c_uint64, C.c_uint64, _VP],
    "mitnc_step_maxima": [_VP, _VP, C.c_size_t, C.POINTER(C.c_float), _I32, _VP],
    "mitnc_plan_exponents": [_VP, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32)],
    "mitnc_backward": [_VP, _VP, C.c_size_t, C.c_uint64, C.c_uint64, _VP, _VP, _VP],
    "mitnc_plan_set_gates": [_VP, _VP, C.c_size_t, C.POINTER(C.c_double), _VP],
    "mitnc_contract": [_VP, _I32, C.POINTER(C.c_int64), _VP, _I32, C.POINTER(C.c_int64), _VP, _I32,
                       C.POINTER(C.c_int64), _I32, C.c_float, _I32, _VP, C.c_size_t, C.POINTER(C.c_size_t),
                       _VP],
    "mitnc_contract_noalloc": [_VP, _I32, C.POINTER(C.c_int64), _VP, _I32, C.POINTER(C.c_int64), _VP, _I32,
                               C.POINTER(C.c_int64), _I32, C.c_float, _I32, _VP],
}
_VOID = {"mitnc_plan_destroy": [_VP], "mitnc_network_destroy": [_VP]}

# Every symbol include/mitnc.h declares (checked by the CPU tests).
EXPORTED = sorted(list(_SIGS) + list(_VOID) + ["mitnc_last_error"])

_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2504_09186_amd.build")
    # torch brings its own HIP runtime; loading it first makes the library
    # bind to that same runtime (with two runtimes in one process the second
    # one finds no device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = _I32
    for name, args in _VOID.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = None
    lib.mitnc_last_error.argtypes = []
    lib.mitnc_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != MITNC_OK:
        msg = load().mitnc_last_error().decode(errors="replace")
        raise MitncError(code, msg)


def call(name: str, *args) -> None:
    """Calls a status-returning entry point and raises MitncError on failure."""
    check(getattr(load(), name)(*args))
