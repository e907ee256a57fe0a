"""ctypes loader for ``libpylom.so`` (the gfx950 HIP library).

There is no fallback: if the shared library is missing or does not export
every entry point declared in ``include/pylom.h``, importing the binding
raises.  Build it with ``python -m paper_2405_15529_amd.build`` (or
``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpylom.so")

I64 = ctypes.c_int64
VP = ctypes.c_void_p
DP = ctypes.POINTER(ctypes.c_double)
I64P = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes); mirrors include/pylom.h
SIGNATURES = {
    "pylom_create": (ctypes.c_int, [ctypes.POINTER(VP), ctypes.c_int]),
    "pylom_destroy": (ctypes.c_int, [VP]),
    "pylom_set_stream": (ctypes.c_int, [VP, VP]),
    "pylom_set_option": (ctypes.c_int, [VP, ctypes.c_char_p, I64]),
    "pylom_get_option": (ctypes.c_int, [VP, ctypes.c_char_p, I64P]),
    "pylom_workspace_query": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, I64, I64,
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "pylom_reserve": (ctypes.c_int, [VP, ctypes.c_size_t]),
    "pylom_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pylom_last_error": (ctypes.c_char_p, [VP]),
    "pylom_pod": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, I64, I64, VP, I64, ctypes.c_int,
                                 ctypes.c_double, VP, VP, I64, VP, VP, I64, VP]),
    "pylom_pod_host": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, I64, I64, VP, I64,
                                      ctypes.c_int, ctypes.c_double, VP, VP, I64, VP, VP, I64,
                                      VP]),
    "pylom_ooc_workspace_query": (ctypes.c_int, [VP, ctypes.c_int, I64, I64,
                                                 ctypes.POINTER(ctypes.c_size_t), I64P, I64P]),
    "pylom_tsvd": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, I64, I64, VP, I64,
                                  ctypes.c_double, VP, I64, VP, VP, I64, VP]),
    "pylom_tsqr": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, I64, I64, VP, I64, VP, I64, VP,
                                  I64]),
    "pylom_matmul": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, I64, I64, I64,
                                    VP, I64, VP, I64, VP, I64]),
    "pylom_matmul_noalloc": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, I64, I64,
                                            I64, VP, I64, VP, I64, VP, I64]),
    "pylom_tree_plan": (I64, [I64, I64P, I64]),
    "pylom_plan_query": (ctypes.c_int, [VP, I64, I64, I64P, I64P, I64P, I64P]),
    "pylom_check": (ctypes.c_int, [VP, I64P]),
    "pylom_phase_times": (ctypes.c_int, [VP, DP, ctypes.c_int]),
    "pylom_kernel_times": (ctypes.c_int, [VP, DP, I64P, ctypes.c_int]),
    "pylom_spod": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, I64, I64, VP, I64, ctypes.c_double,
                                  I64, I64, ctypes.c_int, ctypes.c_int, VP, VP, VP, VP]),
    "pylom_spod_query": (ctypes.c_int, [VP, ctypes.c_int, I64, I64, I64, I64, I64P, I64P,
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "pylom_pod_batched": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, I64, VP, ctypes.c_int]),
    "pylom_tune_block_rows": (I64, [VP, I64, I64]),
    "pylom_autotune": (ctypes.c_int, [VP, ctypes.c_int, ctypes.c_int, I64, I64, VP, I64,
                                      ctypes.c_int, ctypes.c_int, I64P, DP]),
    "pylom_tune_save": (ctypes.c_int, [VP, ctypes.c_char_p]),
    "pylom_tune_load": (ctypes.c_int, [VP, ctypes.c_char_p]),
    "pylom_dmd": (ctypes.c_int, [VP, ctypes.c_int, I64, I64, VP, I64, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, VP, I64, VP, VP, VP, VP, VP]),
    "pylom_dmd_workspace_query": (ctypes.c_int, [VP, ctypes.c_int, I64, I64, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
}


class Problem(ctypes.Structure):
    """Mirror of pylom_problem (include/pylom.h)."""
    _fields_ = [("m", I64), ("n", I64), ("D", VP), ("ldd", I64), ("remove_mean", ctypes.c_int),
                ("residual", ctypes.c_double), ("mean", VP), ("U", VP), ("ldu", I64),
                ("S", VP), ("VT", VP), ("ldvt", I64), ("n_r", VP)]

_lib = None


def load():
    """Load libpylom.so and bind every declared entry point (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -m paper_2405_15529_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)  # AttributeError if the symbol is not exported
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
