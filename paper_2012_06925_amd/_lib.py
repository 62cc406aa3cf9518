"""ctypes declarations of the C ABI in include/bldtt.h.

torch is imported before the library is loaded so the process holds one HIP
runtime (torch's), which the library then shares: torch allocates the device
memory and owns the streams, the library only receives pointers.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbldtt.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EUNSUPPORTED"}

KERNELS = {"coulomb": 0, "yukawa": 1, "oscillatory": 2, "regcoulomb": 3, "poly": 100}
DEFAULT_PARAM = {"coulomb": 0.0, "yukawa": 0.5, "oscillatory": 0.0, "regcoulomb": 0.005, "poly": 0.0}
FP32_EVAL, LEARNED_DEGREE, SYNC, PROFILE, PP_CC_ONLY, AUTOTUNE, VALU_PASSES, MFMA_LEAF, ONE_SIDED_PP = (
    1, 2, 4, 8, 16, 32, 64, 128, 256)
BLTC, CP_BLTC, DEVICE_TRAVERSAL, DEVICE_TREE = 512, 1024, 2048, 4096
PHASES = ("up", "cp_cc", "down_transfer", "pp_pc", "down_leaf", "pp_pc_sep", "pp_sym", "pp_self")
TYPES = ("PP", "PC", "CP", "CC")

_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)


class Particles(C.Structure):
    _fields_ = [("M", C.c_int64), ("tx", C.c_void_p), ("ty", C.c_void_p), ("tz", C.c_void_p),
                ("N", C.c_int64), ("sx", C.c_void_p), ("sy", C.c_void_p), ("sz", C.c_void_p), ("q", C.c_void_p)]


class TreeView(C.Structure):
    _fields_ = [("n_clusters", C.c_int64), ("n_particles", C.c_int64), ("depth", C.c_int32),
                ("lo", _D), ("hi", _D), ("center", _D), ("radius", _D),
                ("begin", _I64), ("count", _I64), ("parent", _I64), ("child", _I64), ("perm", _I64),
                ("level", _I32), ("nchild", _I32)]


class Stats(C.Structure):
    _fields_ = [("n_entries", C.c_int64 * 4), ("interactions", C.c_double * 4),
                ("n_target_clusters", C.c_int64), ("n_source_clusters", C.c_int64),
                ("target_depth", C.c_int32), ("source_depth", C.c_int32),
                ("setup_ms", C.c_double), ("traverse_ms", C.c_double), ("compute_host_ms", C.c_double),
                ("phase_ms", C.c_double * 8), ("profiled_computes", C.c_int64),
                ("down_degree", C.c_int32), ("degree_mask", C.c_uint32), ("sep_pairs", C.c_int64),
                ("sep_fallback", C.c_int64), ("sep_direct", C.c_int64), ("pairs_per_degree", C.c_int64 * 13),
                ("pass_interactions", C.c_double * 5), ("host_marks_ms", C.c_double * 4),
                ("fp64_close_pairs", C.c_double)]


class BatchStats(C.Structure):
    _fields_ = [("n_problems", C.c_int32), ("n_targets", C.c_int64), ("n_sources", C.c_int64),
                ("n_target_clusters", C.c_int64), ("n_source_clusters", C.c_int64),
                ("n_entries", C.c_int64 * 4), ("interactions", C.c_double * 4), ("n_tasks", C.c_int64),
                ("tpt", C.c_int32), ("groups_per_cu", C.c_int32), ("grid", C.c_int32), ("tuned", C.c_int32),
                ("setup_ms", C.c_double), ("tree_ms", C.c_double), ("traverse_ms", C.c_double),
                ("tune_ms", C.c_double), ("tune_best_ms", C.c_double)]


# Every symbol the header declares, with its signature.
SIGNATURES = {
    "bldtt_setup": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Particles), C.c_int32, C.c_double, C.c_double,
                              C.c_int32, C.c_int64, C.c_uint32, C.c_void_p]),
    "bldtt_setup_host": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(Particles), C.c_int32, C.c_double,
                                   C.c_double, C.c_int32, C.c_int64, C.c_uint32]),
    "bldtt_traverse_host": (C.c_int, [C.c_void_p]),
    "bldtt_compute": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "bldtt_destroy": (C.c_int, [C.c_void_p]),
    "bldtt_last_error": (C.c_char_p, []),
    "bldtt_get_tree": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(TreeView)]),
    "bldtt_get_lists": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(C.c_int64)]),
    "bldtt_get_list_degrees": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.POINTER(C.c_int8)), C.POINTER(C.c_int64)]),
    "bldtt_get_qhat": (C.c_int, [C.c_void_p, _D]),
    "bldtt_get_phihat": (C.c_int, [C.c_void_p, _D]),
    "bldtt_get_stats": (C.c_int, [C.c_void_p, C.POINTER(Stats)]),
    "bldtt_direct_sum": (C.c_int, [C.c_int32, C.c_double, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "bldtt_version": (C.c_char_p, []),
    "bldtt_set_allocator": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "bldtt_mlp_model_size": (C.c_int, []),
    "bldtt_set_degree_model": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_double]),
    "bldtt_set_degree_test_rule": (C.c_int, [C.c_void_p]),
    "bldtt_pair_errors": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.POINTER(C.c_float)),
                                    C.POINTER(C.POINTER(C.c_float)), C.POINTER(_I64)]),
    "bldtt_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "bldtt_mlp_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "bldtt_mlp_loss_grad_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                              C.c_void_p, C.c_void_p]),
    "bldtt_set_tune_cache": (C.c_int, [C.c_char_p]),
    "bldtt_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "bldtt_batch_setup": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(Particles), C.c_int32, C.c_double,
                                    C.c_double, C.c_int32, C.c_int64, C.c_uint32, C.c_void_p]),
    "bldtt_batch_setup_host": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(Particles), C.c_int32,
                                         C.c_double, C.c_double, C.c_int32, C.c_int64, C.c_uint32, C.c_int32]),
    "bldtt_batch_get_tree": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(TreeView)]),
    "bldtt_batch_get_lists": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(C.c_int64)]),
    "bldtt_batch_compute": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p]),
    "bldtt_batch_check": (C.c_int, [C.c_void_p, C.c_void_p]),
    "bldtt_batch_tune": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "bldtt_batch_set_tile": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "bldtt_batch_set_spin_limit": (C.c_int, [C.c_void_p, C.c_int32]),
    "bldtt_batch_get_stats": (C.c_int, [C.c_void_p, C.POINTER(BatchStats)]),
    "bldtt_batch_destroy": (C.c_int, [C.c_void_p]),
    "bldtt_mlp_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_uint64,
                                  C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None

# Callback types of bldtt_set_allocator.
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class BldttError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def lib():
    """The loaded library; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2012_06925_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != OK:
        raise BldttError(code, lib().bldtt_last_error().decode())
