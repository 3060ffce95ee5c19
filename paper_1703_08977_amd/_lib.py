"""ctypes loader and structure layouts for libhefk.so (the C ABI of include/he_fk.h).

torch is imported first so that the HIP runtime torch ships is the one the
library binds to (both carry the soname libamdhip64.so.7).  The library must
have been built in-tree (``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime before libhefk)

_HERE = os.path.dirname(os.path.abspath(__file__))
# HEFK_LIBRARY may point at another in-tree build of the same sources (e.g. other launch bounds)
LIB_PATH = os.environ.get("HEFK_LIBRARY") or os.path.join(_HERE, "libhefk.so")

HE_FK_OK = 0
HE_FK_EINVAL = -1
HE_FK_EDEVICE = -2
HE_FK_ENONFINITE = -3
HE_FK_EALLDEAD = -4
HE_FK_ESCRATCH = -5

TRIAL = {"expo": 0, "pade": 1, "triplet": 2, "pz": 3, "triplet_r0": 4, "pz_sum": 5}
PRECISION = {"fp64": 0, "mixed": 1}
NOISE = {"gauss": 0, "pm1": 1}
QUAD = {"trapezoid": 0, "right": 1}
E_METHOD = {"fd": 0, "window": 1, "fit": 2, "mixed": 3}
GRAD_SCORE = 1
GRAD_MOMENT2 = 2  # gL carries a second block of weights, on L2_s = ln <w^2>_s
FLAG_PLAIN = 1   # plain Feynman-Kac walk: no drift, integrand V - e_ref
FLAG_BRIDGE = 2  # node-touch (Brownian bridge) survival weight per step (node trials)

EXPORTS = ["he_fk_init", "he_fk_propagate_workspace_bytes", "he_fk_propagate", "he_fk_propagate_noalloc",
           "he_fk_energy", "he_fk_energy_blocks", "he_fk_grad_scratch_bytes", "he_fk_grad", "he_fk_strerror"]
NOALLOC_SCRATCH_BYTES = 16 << 20  # HE_FK_NOALLOC_SCRATCH_BYTES


class HeFkParams(ctypes.Structure):
    _fields_ = [
        ("trial", ctypes.c_int32), ("sym", ctypes.c_int32), ("ee", ctypes.c_int32),
        ("noise", ctypes.c_int32), ("quad", ctypes.c_int32), ("contract", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("n_metropolis", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("Z", ctypes.c_double), ("theta", ctypes.c_double * 6), ("dt", ctypes.c_double),
        ("e_ref", ctypes.c_double), ("metropolis_sigma", ctypes.c_double), ("init_sigma", ctypes.c_double),
        ("drift_limit", ctypes.c_double), ("seed", ctypes.c_uint64), ("walker_offset", ctypes.c_uint64), ("n_walkers", ctypes.c_int64),
    ]


class HeFkWalkers(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("lnw", ctypes.c_void_p), ("el", ctypes.c_void_p)]


class HeFkError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, strerror(code), code))


_lib = None


def lib():
    """The loaded library; raises if it was not built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhefk.so is not built: run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950) before using paper_1703_08977_amd")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        pp, wp, dp, vp = P(HeFkParams), P(HeFkWalkers), P(ctypes.c_double), ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.he_fk_init.argtypes = [pp, wp, vp]
        L.he_fk_init.restype = ctypes.c_int
        L.he_fk_propagate_workspace_bytes.argtypes = [pp, i64, i32]
        L.he_fk_propagate_workspace_bytes.restype = ctypes.c_size_t
        L.he_fk_propagate.argtypes = [pp, wp, i64, i64, i32, vp, vp, i32, vp, ctypes.c_size_t, vp]
        L.he_fk_propagate.restype = ctypes.c_int
        L.he_fk_propagate_noalloc.argtypes = [pp, wp, i64, i64, i32, vp, vp, i32, vp]
        L.he_fk_propagate_noalloc.restype = ctypes.c_int
        L.he_fk_energy.argtypes = [dp, i64, ctypes.c_double, ctypes.c_double, i32, dp, dp, dp]
        L.he_fk_energy.restype = ctypes.c_int
        L.he_fk_energy_blocks.argtypes = [dp, i64, i64, i32, ctypes.c_double, ctypes.c_double, i32, dp, dp]
        L.he_fk_energy_blocks.restype = ctypes.c_int
        L.he_fk_grad_scratch_bytes.argtypes = [pp, i64, i32, i32]
        L.he_fk_grad_scratch_bytes.restype = ctypes.c_size_t
        L.he_fk_grad.argtypes = [pp, vp, vp, dp, i64, i32, i32, i32, vp, ctypes.c_size_t, vp, vp]
        L.he_fk_grad.restype = ctypes.c_int
        L.he_fk_strerror.argtypes = [ctypes.c_int]
        L.he_fk_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().he_fk_strerror(int(code)).decode()


def check(code: int, where: str) -> int:
    if code != HE_FK_OK:
        raise HeFkError(code, where)
    return code
