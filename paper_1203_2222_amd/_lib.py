"""ctypes declarations of libsymtensor.so (the C-ABI in include/symtensor.h).

Argument marshalling only: every step of the contraction path runs in the
library's HIP kernels.  Importing this module loads the library; a missing
library raises at once, so no caller can silently fall back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsymtensor.so")

SYM_OK = 0
STATUS_NAMES = {0: "SYM_OK", 1: "SYM_E_ARG", 2: "SYM_E_SPECTRUM", 3: "SYM_E_ARROW", 4: "SYM_E_CHARGE",
                5: "SYM_E_DTYPE", 6: "SYM_E_NOMEM", 7: "SYM_E_HIP", 8: "SYM_E_UNSUPPORTED", 9: "SYM_E_MISMATCH"}
SYM_U1, SYM_SU2, SYM_Z2, SYM_U1U1, SYM_Z2F = 0, 1, 2, 3, 4
SYM_F32, SYM_BF16 = 0, 1
SYM_IN, SYM_OUT = 0, 1
SYM_TREE_NONE, SYM_TREE_OPERATOR, SYM_TREE_LEFT, SYM_TREE_RIGHT, SYM_TREE_CHAIN = 0, 1, 2, 3, 4
MAX_RANK = 8


class SymLeg(ctypes.Structure):
    _fields_ = [("n", c_int32), ("label", POINTER(c_int32)), ("deg", POINTER(c_int64)), ("arrow", c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)

P = c_void_p
PP = POINTER(c_void_p)
I32P = POINTER(c_int32)
I64P = POINTER(c_int64)

# name -> (restype, argtypes)
SIGNATURES = {
    "sym_ctx_create": (c_int32, [ALLOC_FN, FREE_FN, c_void_p, PP]),
    "sym_ctx_destroy": (None, [P]),
    "sym_ctx_clear": (c_int32, [P]),
    "sym_hold_begin": (c_int32, [P, PP]),
    "sym_hold_end": (c_int32, [P]),
    "sym_hold_count": (c_int32, [P, I64P]),
    "sym_hold_destroy": (None, [P]),
    "sym_tensor_create": (c_int32, [P, c_int32, c_int32, POINTER(SymLeg), c_int32, c_int32, c_int32, c_int32, P, PP]),
    "sym_tensor_destroy": (None, [P]),
    "sym_tensor_set_data": (c_int32, [P, P]),
    "sym_tensor_numel": (c_int32, [P, I64P]),
    "sym_tensor_num_blocks": (c_int32, [P, I64P]),
    "sym_tensor_num_sectors": (c_int32, [P, I64P]),
    "sym_tensor_block_info": (c_int32, [P, c_int64, I32P, I32P, I64P, I64P, I64P]),
    "sym_tensor_sector_info": (c_int32, [P, c_int64, I32P, I64P, I64P, I64P]),
    "sym_tensor_block_inner": (c_int32, [P, c_int64, I32P, I32P]),
    "sym_permute_fuse_output": (c_int32, [P, P, I32P, c_int32, c_int32, P, PP]),
    "sym_permute_fuse": (c_int32, [P, P, I32P, c_int32, P, P]),
    "sym_permute_tree_output": (c_int32, [P, P, I32P, c_int32, c_int32, P, PP]),
    "sym_permute_tree": (c_int32, [P, P, I32P, c_int32, c_int32, P, P]),
    "sym_su2_permute_output": (c_int32, [P, P, I32P, I32P, c_int32, P, PP]),
    "sym_su2_permute": (c_int32, [P, P, I32P, I32P, c_int32, P, P]),
    "sym_tensor_leg": (c_int32, [P, c_int32, c_int32, I32P, I32P, I64P, I32P]),
    "sym_su2_fuse_output": (c_int32, [P, P, c_int32, c_int32, P, PP]),
    "sym_contract_operand_output": (c_int32, [P, P, P, c_int32, I32P, I32P, c_int32, c_int32, P, PP]),
    "sym_su2_fuse": (c_int32, [P, P, c_int32, c_int32, P, P]),
    "sym_su2_split_output": (c_int32, [P, P, c_int32, POINTER(SymLeg), c_int32, P, PP]),
    "sym_su2_split": (c_int32, [P, P, c_int32, P, P]),
    "sym_su2_gamma": (c_int32, [c_int32, I32P, c_int32, I32P, c_int32, I32P, I32P, I32P, POINTER(c_double)]),
    "sym_su2_chain_gamma": (c_int32, [c_int32, I32P, I32P, I32P, I32P, c_int32, I32P, I32P, I32P, I32P, I32P,
                                      POINTER(c_double)]),
    "sym_contract_output": (c_int32, [P, P, P, c_int32, I32P, I32P, P, PP]),
    "sym_contract": (c_int32, [P, P, P, c_int32, I32P, I32P, c_int32, P, P]),
    "sym_contract_noalloc": (c_int32, [P, P, P, c_int32, I32P, I32P, c_int32, P, P]),
    "sym_noalloc_capacity": (c_int32, [I64P]),
    "sym_contract_backward": (c_int32, [P, P, P, P, c_int32, I32P, I32P, c_int32, P, P, P]),
    "sym_contract_batched": (c_int32, [P, c_int32, PP, PP, c_int32, I32P, I32P, c_int32, PP, P]),
    "sym_contract_flops": (c_int32, [P, P, P, c_int32, I32P, I32P, I64P]),
    "sym_graph_create_batched": (c_int32, [P, c_int32, PP, PP, c_int32, I32P, I32P, c_int32, PP, P, PP]),
    "sym_graph_launch": (c_int32, [P, P]),
    "sym_graph_destroy": (None, [P]),
    "sym_ctx_set_timing": (c_int32, [P, c_int32]),
    "sym_ctx_phase_ms": (c_int32, [P, c_int32, POINTER(c_float)]),
    "sym_tune_batched": (c_int32, [P, c_int32, PP, PP, c_int32, I32P, I32P, c_int32, PP, P, I32P]),
    "sym_ctx_set_variant": (c_int32, [P, c_int32, c_int32]),
    "sym_num_variants": (c_int32, [c_int32, I32P]),
    "sym_variant_name": (c_int32, [c_int32, c_int32, POINTER(c_char_p)]),
    "sym_variant_kernel": (c_int32, [c_int32, c_int32, POINTER(c_char_p)]),
    "sym_svd_sizes": (c_int32, [P, I64P, I64P, I64P]),
    "sym_svd": (c_int32, [P, P, P, P, P, I32P, c_int32, P]),
    "sym_svd_truncate": (c_int32, [P, P, c_int64, c_double, I32P, POINTER(c_double)]),
    "sym_eigh_sizes": (c_int32, [P, I64P, I64P]),
    "sym_eigh": (c_int32, [P, P, P, P, I32P, c_int32, P]),
    "sym_polar_sizes": (c_int32, [P, I64P, I64P]),
    "sym_polar": (c_int32, [P, P, P, P, I32P, c_int32, P]),
    "sym_default_variant": (c_int32, [c_int32, I32P]),
    "sym_fmove_coeff": (c_double, [c_int32] * 6),
    "sym_last_error": (c_char_p, []),
    "sym_version": (c_char_p, []),
}


class SymError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1203_2222_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int) -> None:
    if status != SYM_OK:
        raise SymError(status, lib().sym_last_error().decode())


def i32_array(values):
    values = list(values)
    return (c_int32 * max(1, len(values)))(*values)


def ptr_array(values):
    values = list(values)
    return (c_void_p * max(1, len(values)))(*values)
