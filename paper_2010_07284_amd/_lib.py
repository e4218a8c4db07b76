"""ctypes loader for libvlg.so.  Fails loudly when the library is missing and
cannot be built: there is no fallback implementation."""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvlg.so")

# every symbol declared in include/vlg.h
EXPORTS = [
    "vlg_create", "vlg_destroy", "vlg_sync", "vlg_set_loop_cap", "vlg_set_mode", "vlg_load_image", "vlg_image_free",
    "vlg_image_shape", "vlg_compile_formula", "vlg_formula_info", "vlg_formula_output_name", "vlg_formula_plan",
    "vlg_formula_free", "vlg_check", "vlg_check_all", "vlg_check_batch", "vlg_ccl_labels", "vlg_ccl_labels_noalloc", "vlg_ccl_labels_pj",
    "vlg_load_volume", "vlg_image_shape3", "vlg_ccl_labels3", "vlg_profile_step", "vlg_stream_copy",
    "vlg_ccl_read_counters", "vlg_profile", "vlg_profile_batch", "vlg_set_tunable", "vlg_get_tunable", "vlg_autotune", "vlg_autotune_batch",
    "vlg_tune_save", "vlg_tune_load", "vlg_server_create", "vlg_server_submit", "vlg_server_wait",
    "vlg_server_read_stats", "vlg_server_destroy", "vlg_evaluation_bytes", "vlg_last_error",
]

ERRORS = {-1: "VLG_EINVAL", -2: "VLG_EPARSE", -3: "VLG_ESHAPE", -4: "VLG_ENOMEM", -5: "VLG_EHIP",
          -6: "VLG_ENOCONV"}


class VlgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class FormulaStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("parsed_nodes", "nodes", "reach_nodes", "atoms", "outputs", "steps_perop", "steps_fused",
                 "peak_masks", "launches_fused", "labellings", "labelling_reuse", "segments")]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("which", ctypes.c_int), ("best", ctypes.c_int), ("n", ctypes.c_int),
                ("candidates", ctypes.c_int * 8), ("ms", ctypes.c_double * 8)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "rejected", "max_inflight", "max_queued",
                                              "peak_reserved_bytes", "budget_bytes")]


class CclCounters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("merge_unions", "merge_retries", "launches_per_ccl", "pj_labellings",
                                              "pj_main_iterations", "pj_rounds", "pj_launches")]


class PjStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("main_iterations", "rounds", "launches")]


_lib = None


def loaded():
    return _lib is not None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        sig = {
            "vlg_create": ([P, I, P], I),
            "vlg_destroy": ([P], None),
            "vlg_sync": ([P], I),
            "vlg_set_loop_cap": ([P, I], I),
            "vlg_set_mode": ([P, I], I),
            "vlg_load_image": ([P, P, I, I, I, I, I64, I, P], I),
            "vlg_image_free": ([P], I),
            "vlg_image_shape": ([P, P, P, P], I),
            "vlg_compile_formula": ([P, ctypes.c_char_p, P], I),
            "vlg_formula_info": ([P, P], I),
            "vlg_formula_output_name": ([P, I], ctypes.c_char_p),
            "vlg_formula_plan": ([P, I, I, P, I64, P], I),
            "vlg_formula_free": ([P], I),
            "vlg_check": ([P, P, P, I, P, I, I], I),
            "vlg_check_all": ([P, P, P, P, I, I], I),
            "vlg_check_batch": ([P, P, P, I, P, I, I], I),
            "vlg_ccl_labels": ([P, P, I, I, P], I),
            "vlg_ccl_labels_noalloc": ([P, P, I, I, P], I),
            "vlg_ccl_labels_pj": ([P, P, I, I, I, P, P], I),
            "vlg_load_volume": ([P, P, I, I, I, I, I, I, P], I),
            "vlg_image_shape3": ([P, P, P, P, P], I),
            "vlg_ccl_labels3": ([P, P, I, I, I, P], I),
            "vlg_profile_step": ([P, P, P, ctypes.c_char_p, I, P, P], I),
            "vlg_stream_copy": ([P, P, P, I64, I, I, P], I),
            "vlg_ccl_read_counters": ([P, P], I),
            "vlg_profile": ([P, P, P, I, P, I, P], I),
            "vlg_profile_batch": ([P, P, P, I, I, P, I, P], I),
            "vlg_set_tunable": ([P, I, I], I),
            "vlg_get_tunable": ([P, I, I, I, P], I),
            "vlg_autotune": ([P, P, P, I, P, I, P], I),
            "vlg_autotune_batch": ([P, P, P, I, I, P, I, P], I),
            "vlg_tune_save": ([P, ctypes.c_char_p], I),
            "vlg_tune_load": ([P, ctypes.c_char_p], I),
            "vlg_server_create": ([P, I, I, I64], I),
            "vlg_server_submit": ([P, P, P, P, P], I),
            "vlg_server_wait": ([P, I64, P, P], I),
            "vlg_server_read_stats": ([P, P], I),
            "vlg_server_destroy": ([P], I),
            "vlg_evaluation_bytes": ([P, P, P], I),
            "vlg_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def call(name, *args):
    L = lib()
    rc = getattr(L, name)(*args)
    if rc != 0:
        raise VlgError(rc, (L.vlg_last_error() or b"").decode())
    return rc
