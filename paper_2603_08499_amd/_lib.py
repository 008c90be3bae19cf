"""ctypes declarations of the C ABI in include/vbgs.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvbgs.so")

VBGS_ABI_VERSION = 1
STATUS = {0: "VBGS_OK", -1: "VBGS_ERR_ARG", -2: "VBGS_ERR_SHAPE", -3: "VBGS_ERR_HIP", -4: "VBGS_ERR_NOT_PD",
          -5: "VBGS_ERR_NONFINITE", -6: "VBGS_ERR_STATE", -7: "VBGS_ERR_UNSUPPORTED"}
NPHASE = 10
PHASES = ["prep", "coeffs", "pass1", "pass2", "fold", "update", "elbo", "proposal", "sort", "lse"]
H = 128
SCRATCH_BYTES = 64 << 20  # VBGS_SCRATCH_BYTES
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "auto": 4, "fp8": 5, "fp64_culled": 6}


class Params(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("D", ctypes.c_int32), ("K", ctypes.c_int64),
                ("n_max", ctypes.c_int64), ("kappa0", ctypes.c_double), ("nu0", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("score_prec", ctypes.c_int32), ("exact", ctypes.c_int32),
                ("screen_margin", ctypes.c_double), ("n_split", ctypes.c_int32), ("proposal", ctypes.c_int32),
                ("C", ctypes.c_int32), ("train_batch", ctypes.c_int32), ("cull", ctypes.c_int32),
                ("modal_split", ctypes.c_int32), ("cull_dims", ctypes.c_int32),
                ("proposal_prec", ctypes.c_int32), ("reserved", ctypes.c_int64 * 3)]


_lib = None
vp = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64


def load():
    """Load the in-tree HIP library; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libvbgs.so is missing at %s: build it with `python -c 'import __graft_entry__ as g; "
                          "g.build()'` (hipcc, gfx950)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    sig = {
        "vbgs_default_params": (i32, [P, i32, i64, i64]),
        "vbgs_query_sizes": (i32, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "vbgs_init": (i32, [ctypes.POINTER(vp), P, vp, vp, vp, vp, vp]),
        "vbgs_attach": (i32, [ctypes.POINTER(vp), P, vp, vp]),
        "vbgs_estep_stats": (i32, [vp, vp, i64, vp, vp, vp]),
        "vbgs_estep_stats_scratch": (i32, [vp, vp, i64, vp, vp, vp]),
        "vbgs_update": (i32, [vp, i32, vp]),
        "vbgs_elbo": (i32, [vp, vp, i64, vp, vp]),
        "vbgs_get_params": (i32, [vp, i32, vp, vp, vp, vp, vp, vp]),
        "vbgs_set_params": (i32, [vp, i32, vp, vp, vp, vp, vp, vp]),
        "vbgs_sync_status": (i32, [vp, vp]),
        "vbgs_clear_flags": (i32, [vp, vp]),
        "vbgs_counters": (i32, [vp, ctypes.POINTER(i64), vp]),
        "vbgs_reassign": (i32, [vp, vp, i64, vp, vp, i64, vp, vp, vp]),
        "vbgs_render": (i32, [vp, vp, vp, i64, vp, vp, vp, vp]),
        "vbgs_psnr": (i32, [vp, vp, i64, vp, vp]),
        "vbgs_proposal_set": (i32, [vp] + [vp] * 8 + [vp]),
        "vbgs_proposal_get": (i32, [vp] + [vp] * 6 + [vp]),
        "vbgs_estep_stats_pruned": (i32, [vp, vp, i64, vp, i64, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp]),
        "vbgs_export_targets": (i32, [vp, vp, i64, vp, vp, vp]),
        "vbgs_proposal_candidates": (i32, [vp, vp, i64, vp, vp]),
        "vbgs_proposal_train_step": (i32, [vp, vp, vp, vp, vp, i32, ctypes.c_float, i32, vp, vp, vp]),
        "vbgs_timing": (i32, [vp, i32]),
        "vbgs_timing_phases": (i32, [vp, ctypes.c_uint32]),
        "vbgs_timing_read": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), vp]),
        "vbgs_last_error": (ctypes.c_char_p, [vp]),
        "vbgs_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L
