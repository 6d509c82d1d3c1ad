"""ctypes binding of libmmf.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; this module
only turns torch device tensors and numpy host arrays into the pointers and
sizes of the C ABI declared in include/mmf.h.  There is no fallback: if the
library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmmf.so")

MMF_C128, MMF_C64_REFINED, MMF_C64_RAW = 0, 1, 2
MMF_OK, MMF_ERR_HIP, MMF_ERR_WORKSPACE, MMF_ERR_NOT_IMPLEMENTED = 0, 1, 2, 3
MMF_ERR_NO_CONVERGENCE, MMF_ERR_SELECTION, MMF_ERR_TOO_LARGE, MMF_ERR_DEGENERATE = 4, 5, 6, 7


class MMFProblem(C.Structure):
    _fields_ = [
        ("D", C.c_int32), ("F", C.c_int32), ("K", C.c_int32),
        ("omega", C.c_void_p), ("N", C.c_void_p), ("axis", C.c_void_p), ("harm", C.c_void_p),
        ("E", C.c_void_p), ("V", C.c_void_p),
    ]


class MMFEighOpts(C.Structure):
    _fields_ = [("refine_max_iters", C.c_int32), ("secular_max_iters", C.c_int32),
                ("leaf_max_iters", C.c_int32)]


class MMFBatchOpts(C.Structure):
    _fields_ = [("small_threads", C.c_int32 * 8)]


class MMFError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


_lib = None

_SIGS = {
    "mmf_strerror": (C.c_char_p, [C.c_int]),
    "mmf_floquet_dim": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mmf_build_floquet_workspace": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mmf_build_floquet": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mmf_build_floquet_dev": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "mmf_batched_workspace": (C.c_int, [C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
    "mmf_build_floquet_batched": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_size_t, C.c_void_p]),
    "mmf_observables_batched": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                          C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_size_t, C.c_void_p]),
    "mmf_eigh_workspace": (C.c_int, [C.c_int64, C.c_int, C.c_void_p]),
    "mmf_eigh": (C.c_int, [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p,
                           C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_eigh_ex": (C.c_int, [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                              C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_eigh_batched_workspace": (C.c_int, [C.c_int64, C.c_void_p, C.c_int, C.c_void_p]),
    "mmf_eigh_batched": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                   C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_eigh_batched_ex": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                      C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_eigh_window_workspace": (C.c_int, [C.c_int64, C.c_int64, C.c_void_p]),
    "mmf_eigh_band_workspace": (C.c_int, [C.c_int64, C.c_int64, C.c_void_p]),
    "mmf_eigh_band": (C.c_int, [C.c_int64, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_eigh_band_window_workspace": (C.c_int, [C.c_int64, C.c_int64, C.c_int64, C.c_void_p]),
    "mmf_eigh_band_window": (C.c_int, [C.c_int64, C.c_void_p, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                       C.c_int64, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_eigh_window": (C.c_int, [C.c_int64, C.c_void_p, C.c_int64, C.c_double, C.c_double, C.c_int64,
                                  C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_size_t,
                                  C.c_void_p, C.c_void_p]),
    "mmf_eigvalsh_batched_workspace": (C.c_int, [C.c_int64, C.c_void_p, C.c_int, C.c_void_p]),
    "mmf_eigvalsh_batched": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                       C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_hetrd": (C.c_int, [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_size_t, C.c_void_p]),
    "mmf_stedc": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                            C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_unmtr": (C.c_int, [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                            C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mmf_evolve_workspace": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "mmf_evolve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_double, C.c_int32,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "mmf_micromotion": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_size_t, C.c_void_p, C.c_void_p]),
    "mmf_dressed_evolution": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p]),
    "mmf_avg_prob_workspace": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mmf_avg_prob": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_size_t, C.c_void_p]),
    "mmf_avg_prob_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "mmf_eigh_two_stage_min": (C.c_int64, []),
    "mmf_ktimer_arm": (C.c_int, [C.c_char_p]),
    "mmf_ktimer_read": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mmf_profile_sync_every": (C.c_int, [C.c_int64]),
}

EXPORTED = tuple(_SIGS.keys())


def lib():
    """Load libmmf.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it first (python -m paper_2005_03426_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(fn: str, code: int):
    if code != 0:
        msg = lib().mmf_strerror(code).decode()
        raise MMFError(fn, code, msg)
    return code


def call(fn: str, *args):
    return check(fn, getattr(lib(), fn)(*args))
