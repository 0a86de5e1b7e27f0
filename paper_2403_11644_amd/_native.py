"""ctypes loader for libptd.so (the C ABI declared in include/ptd.h).

The library is built in-tree by ``python -m paper_2403_11644_amd.build``.
Nothing here falls back to another implementation: if the library is
missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptd.so")

_lib = None
_lock = threading.Lock()

P = ctypes.c_void_p
I = ctypes.c_int
U = ctypes.c_uint
I64 = ctypes.c_int64
SZ = ctypes.c_size_t
D = ctypes.c_double

# name -> (restype, argtypes); mirrors include/ptd.h
SIGNATURES = {
    "ptd_workspace_bytes": (SZ, [I, I, U, I]),
    "ptd_reconstruct_workspace_bytes": (SZ, [I, I, U]),
    "ptd_num_nonempty_x": (I, [I, U, I]),
    "ptd_nonempty_x": (I, [I, U, I, P]),
    "pauli_decompose": (I, [I, I, U, I, P, I64, P, P, SZ, P]),
    "pauli_reconstruct": (I, [I, I, U, P, P, I64, P, SZ, P]),
    "ptd_workspace_status": (I, [P, SZ, P]),
    "pauli_decompose_noalloc": (I, [I, I, U, I, P, I64, P, P]),
    "ptd_reduce_workspace_bytes": (SZ, []),
    "ptd_parseval_residual": (I, [I, I, U, P, I64, P, P, P, SZ, P]),
    "ptd_batched_workspace_bytes": (SZ, [I, I, P]),
    "pauli_decompose_batched": (I, [I, I, U, P, P, P, P, P, P, SZ, P]),
    "pauli_reconstruct_batched": (I, [I, I, U, P, P, P, P, P, P, SZ, P]),
    "ptd_batch_plan_create": (I, [I, I, U, P, P, P, P, P, P]),
    "ptd_batch_plan_launch": (I, [P, P]),
    "ptd_batch_plan_destroy": (None, [P]),
    "ptd_block_diagonal": (I, [I, I, I, U, P, P, P]),
    "ptd_direct_sum": (I, [I, I, U, P, P, P, P]),
    "ptd_hermitian_augment": (I, [I, I, U, P, P, P]),
    "ptd_linear_combination": (I, [I, I, D, D, P, P, P, P]),
    "ptd_lcu_amplitudes": (I, [I, I, U, P, P, P, P, SZ, P]),
    "ptd_sparse_workspace_bytes": (SZ, [I]),
    "ptd_sparse_nonempty_x": (I, [I, I64, P, P, P, P, P, SZ, P]),
    "pauli_decompose_sparse": (I, [I, I, U, I64, P, P, P, P, I, P, P, SZ, P]),
    "ptd_csr_nonempty_x": (I, [I, I64, P, P, P, P, P, SZ, P]),
    "pauli_decompose_csr": (I, [I, I, U, I64, P, P, P, P, I, P, P, SZ, P]),
    "ptd_host_tree_decompose": (I, [I, U, P, I64, P, I, I64, I64, I, P]),
    "ptd_autotune": (I, [I, I, U, I, P, P, P, P, P, P]),
    "ptd_describe_tuning": (I, [I, I, U, I, P, P, P]),
    "ptd_set_tuning": (I, [I, I, U, I, I]),
    "ptd_get_tuning": (I, [I, I, U, P, P]),
    "ptd_clear_tuning": (None, []),
    "ptd_autotune_report": (I, [I, I, U, P, P, P, P]),
    "ptd_zero_pad": (I, [I, P, I64, I64, I64, P, I, P]),
    "ptd_status_str": (ctypes.c_char_p, [I]),
    "ptd_last_hip_error": (I, []),
    "ptd_build_arch": (ctypes.c_char_p, []),
    # testing hooks (not part of ptd.h)
    "ptd_debug_decompose_path": (I, [I, I, U, P, I64, P, I, P]),
    "ptd_debug_reconstruct_path": (I, [I, I, U, P, P, I64, I, P]),
    "ptd_debug_decompose_stage": (I, [I, I, U, P, I64, P, I, P]),
    "ptd_debug_decompose_fused": (I, [I, I, U, P, I64, P, P, SZ, I, I, P]),
    "ptd_debug_copy": (I, [P, P, SZ, P]),
    "ptd_debug_bandwidth": (I, [I, P, P, SZ, P]),
    "ptd_debug_wait_test_mode": (None, [I]),
    "ptd_debug_xcc_ids": (I, [P, P]),
}


class PtdError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = lib().ptd_status_str(status).decode()
        if status == -4:
            msg += " (hip error %d)" % lib().ptd_last_hip_error()
        super().__init__("%s: %s" % (what, msg))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "libptd.so is not built (%s); run `python -m paper_2403_11644_amd.build`" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name, None)
                if fn is None:
                    continue
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def check(status: int, what: str) -> None:
    if status != 0:
        raise PtdError(status, what)
