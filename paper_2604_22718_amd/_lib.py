"""ctypes loader for librtt.so (the HIP library built in-tree).

There is no fallback: if the library is missing or cannot be loaded the
import fails with an error that says how to build it.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtt.so")

_lib = None

# name -> (restype, argtypes); every entry point declared in include/rtt.h
P = C.c_void_p
SIGNATURES = {
    "rtt_last_error": (C.c_char_p, []),
    "rtt_abi_version": (C.c_int32, []),
    "rtt_create": (C.c_int, [C.c_int32, C.c_int32, P, P, P, C.c_int32, C.POINTER(P)]),
    "rtt_lincomb": (C.c_int, [C.c_int32, P, P, C.POINTER(P)]),
    "rtt_destroy": (C.c_int, [P]),
    "rtt_info": (C.c_int, [P, P]),
    "rtt_get_cores": (C.c_int, [P, C.c_int32, P]),
    "rtt_tfim_create": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, C.POINTER(P)]),
    "rtt_tfim_destroy": (C.c_int, [P]),
    "rtt_evaluate": (C.c_int, [P, P, C.c_int32, P, P, P, P, P, P, P, P]),
    "rtt_evaluate_noalloc": (C.c_int, [P, P, C.c_int32, P, P, P, P, P, P, P, P]),
    "rtt_amplitudes": (C.c_int, [P, C.c_int32, P, P, P, P]),
    "rtt_flip_ratios": (C.c_int, [P, C.c_int32, P, P, P, P]),
    "rtt_local_energy": (C.c_int, [P, P, C.c_int32, P, P, P]),
    "rtt_mcmc_sweep": (C.c_int, [P, C.c_int32, P, P, P, C.c_uint64, C.c_uint64, C.c_uint64,
                                 C.c_int32, P, P, P]),
    "rtt_energy_reduce": (C.c_int, [C.c_int32, P, P, P]),
    "rtt_pair_sums": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P, P, P, P]),
    "rtt_mixed_estimators": (C.c_int, [C.c_int32, P, P, C.c_int32, P, P, P, P, P, P, P]),
    "rtt_tt_round": (C.c_int, [C.c_int32, P, P, C.c_int32, C.c_double, P, P, C.c_int64, C.POINTER(C.c_int64)]),
    "rtt_pauli_apply": (C.c_int, [C.c_int32, P, P, C.c_int32, P, P, C.c_double, C.c_double, C.c_int32,
                                  C.c_int32, C.c_double, P, P, C.c_int64, C.POINTER(C.c_int64)]),
    "rtt_tt_combine": (C.c_int, [C.c_int32, C.c_int32, P, P, P, C.c_int32, C.c_double, P, P, C.c_int64,
                                 C.POINTER(C.c_int64)]),
    "rtt_tfim_power_step": (C.c_int, [C.c_int32, C.c_int32, P, P, P, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_double, C.c_double, C.c_double, C.c_int32, C.c_double, P, P,
                                      C.c_int64, C.POINTER(C.c_int64)]),
    "rtt_batch_create": (C.c_int, [C.c_int32, P, P, P, P, P, C.c_uint64, C.POINTER(P)]),
    "rtt_batch_step": (C.c_int, [P, C.c_int32, P, P]),
    "rtt_batch_autotune": (C.c_int, [P, C.c_int32, C.c_int32, C.c_char_p, P, P]),
    "rtt_batch_destroy": (C.c_int, [P]),
    "rtt_net_create": (C.c_int, [C.c_int32, C.c_int32, P, C.POINTER(P)]),
    "rtt_net_destroy": (C.c_int, [P]),
    "rtt_net_get_params": (C.c_int, [P, C.c_int32, P]),
    "rtt_net_forward": (C.c_int, [P, C.c_int32, P, P, P]),
    "rtt_mh_learned_step": (C.c_int, [P, P, C.c_int32, P, P, P, C.c_uint64, C.c_uint64, C.c_uint64,
                                      P, P, P, P, P, P]),
    "rtt_net_grad": (C.c_int, [P, C.c_int32, P, P, P, P, P]),
    "rtt_net_train": (C.c_int, [P, C.c_int32, P, P, P, C.c_float, C.c_float, C.c_float, C.c_float, P]),
}


class RTTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rtt status {status}: {msg}")
        self.status = status


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2604_22718_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != 0:
        raise RTTError(status, lib().rtt_last_error().decode())
