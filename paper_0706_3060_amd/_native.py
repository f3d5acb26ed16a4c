"""ctypes view of libnbody.so (the C ABI declared in include/nbody.h).

Loading rules:
* ``torch`` is imported first, so that the HIP runtime libnbody.so links
  against (soname libamdhip64.so.7) resolves to the one torch already loaded:
  one HIP runtime per process, and torch's streams are valid handles for it.
* There is no fallback: if the library is missing or does not load, every
  entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the library load, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbody.so")

NBODY_OK = 0
NBODY_EINVAL = -1
NBODY_ENOTSUP = -2
NBODY_EWORKSPACE = -3
NBODY_EHIP = -4

API_FORCES, API_BATCHED, API_BACKWARD, API_LEAPFROG, API_JERK, API_HERMITE = 0, 1, 2, 3, 4, 5
API_BACKWARD_BATCHED = 6

EXPORTED = (
    "nbody_forces", "nbody_forces_subset", "nbody_forces_batched", "nbody_forces_backward",
    "leapfrog_step", "nbody_workspace_bytes", "nbody_last_error", "nbody_set_config",
    "nbody_get_config", "nbody_autotune", "nbody_tune_save", "nbody_tune_load",
    "nbody_timing_enable", "nbody_timing_read", "nbody_flops_per_pair", "nbody_version",
    "nbody_forces_jerk", "hermite_step", "hermite_block_init", "hermite_block_steps",
    "nbody_autotune_jerk", "nbody_forces_excl", "nbody_forces_batched_excl",
    "nbody_forces_backward_excl", "nbody_forces_backward_batched",
    "nbody_probe_workspace_bytes", "nbody_probe_issue_rates", "nbody_forces_noalloc",
    "nbody_forces_share",
)


class NBodyLaw(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("precision", ctypes.c_int32), ("G", ctypes.c_double),
                ("softening", ctypes.c_double), ("coulomb_k", ctypes.c_double),
                ("dielectric", ctypes.c_double), ("zeta", ctypes.c_double * 4)]


class NBodyConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("i_per_lane", ctypes.c_int32),
                ("j_tile", ctypes.c_int32), ("j_split", ctypes.c_int32),
                ("j_stage", ctypes.c_int32)]


class NBodyExclusions(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("index", ctypes.c_void_p), ("count", ctypes.c_int64)]


class NBodyError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("nbody error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libnbody.so is not built (%s); run __graft_entry__.build() or "
                              "python -m paper_0706_3060_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, D, SZ = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                              ctypes.c_size_t)
        LAW = ctypes.POINTER(NBodyLaw)
        EXC = ctypes.POINTER(NBodyExclusions)
        CFG = ctypes.POINTER(NBodyConfig)
        sig = {
            "nbody_forces": ([P, P, I64, LAW, P, P, P, SZ, P], ctypes.c_int),
            "nbody_forces_noalloc": ([P, P, I64, LAW, P, P, P], ctypes.c_int),
            "nbody_forces_subset": ([P, P, I64, P, I64, LAW, P, P, P, SZ, P], ctypes.c_int),
            "nbody_forces_share": ([P, P, I64, LAW, I32, I32, P, P, P, SZ, P], ctypes.c_int),
            "nbody_forces_batched": ([P, I64, P, P, LAW, P, P, P, SZ, P], ctypes.c_int),
            "nbody_forces_backward": ([P, P, I64, LAW, P, P, P, P, I32, P, P, SZ, P], ctypes.c_int),
            "leapfrog_step": ([P, P, P, P, P, I64, LAW, D, I32, P, P, SZ, P], ctypes.c_int),
            "nbody_workspace_bytes": ([I32, I64, I64, LAW], SZ),
            "nbody_last_error": ([], ctypes.c_char_p),
            "nbody_set_config": ([I32, CFG], ctypes.c_int),
            "nbody_get_config": ([I32, I64, I64, LAW, CFG], ctypes.c_int),
            "nbody_autotune": ([I32, P, I64, P, P, I64, LAW, P, P, P, SZ, P, CFG,
                                ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "nbody_tune_save": ([ctypes.c_char_p], ctypes.c_int),
            "nbody_tune_load": ([ctypes.c_char_p], ctypes.c_int),
            "nbody_timing_enable": ([I32], ctypes.c_int),
            "nbody_timing_read": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64), I32],
                                  ctypes.c_int),
            "nbody_flops_per_pair": ([I32, I32, I32], I32),
            "nbody_version": ([], ctypes.c_char_p),
            "nbody_probe_workspace_bytes": ([], SZ),
            "nbody_probe_issue_rates": ([ctypes.POINTER(ctypes.c_double), I32, P, SZ, P], ctypes.c_int),
            "nbody_forces_jerk": ([P, P, P, I64, P, I64, LAW, P, P, P, P, SZ, P], ctypes.c_int),
            "hermite_step": ([P, P, P, P, P, I64, LAW, D, I32, P, SZ, P], ctypes.c_int),
            "hermite_block_init": ([P, P, I64, D, D, P, P, P], ctypes.c_int),
            "hermite_block_steps": ([P, P, P, P, P, P, P, I64, LAW, D, D, D, I32, P, P, P, SZ, P],
                                    ctypes.c_int),
            "nbody_autotune_jerk": ([P, P, P, I64, LAW, P, P, P, P, SZ, P, CFG,
                                     ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "nbody_forces_excl": ([P, P, I64, EXC, LAW, P, P, P, SZ, P], ctypes.c_int),
            "nbody_forces_batched_excl": ([P, I64, P, P, EXC, LAW, P, P, P, SZ, P], ctypes.c_int),
            "nbody_forces_backward_excl": ([P, P, I64, EXC, LAW, P, P, P, P, I32, P, P, SZ, P],
                                           ctypes.c_int),
            "nbody_forces_backward_batched": ([P, I64, P, P, EXC, LAW, P, P, P, P, I32, P, P, SZ, P],
                                              ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(rc: int):
    if rc != NBODY_OK:
        raise NBodyError(rc, lib().nbody_last_error().decode())
    return rc


def runtime_path() -> str:
    """Path of the HIP runtime the library resolved to (one per process)."""
    lib()
    for line in open("/proc/self/maps"):
        if "libamdhip64" in line:
            return line.split()[-1]
    return ""
