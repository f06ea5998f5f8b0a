"""ctypes loader for libct.so: the C-ABI entry points of include/ct.h, same names.

The library is built in-tree by `python -m paper_2606_28372_amd.build`.  There
is no fallback: if the shared library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libct.so")

CT_OK, CT_EINVAL, CT_ENOMEM, CT_EOVERFLOW, CT_EEMPTY, CT_EDEVICE, CT_ESYNTAX = 0, -1, -2, -3, -4, -5, -6
STATUS = {CT_EINVAL: "CT_EINVAL", CT_ENOMEM: "CT_ENOMEM", CT_EOVERFLOW: "CT_EOVERFLOW", CT_EEMPTY: "CT_EEMPTY",
          CT_EDEVICE: "CT_EDEVICE", CT_ESYNTAX: "CT_ESYNTAX"}
CT_HAMMING, CT_INDEX_L1, CT_TIER_EUCLID, CT_TIER_RANDOM, CT_HAM1_RANDOM = 0, 1, 2, 3, 4
CT_DE, CT_PSO, CT_GA, CT_FIREFLY = 0, 1, 2, 3
CT_STEP_PLAIN, CT_STEP_BATCHED, CT_STEP_GRAPH = 0, 1, 2
CT_SCAN_SERIAL, CT_SCAN_STREAMS, CT_SCAN_FUSED = 0, 1, 2


class CtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class ct_pop_params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_uint32), ("pop_size", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("F_q16", ctypes.c_uint32), ("de_method", ctypes.c_uint32), ("CR_q32", ctypes.c_uint64),
                ("w_q16", ctypes.c_uint32), ("c1_q16", ctypes.c_uint32), ("c2_q16", ctypes.c_uint32),
                ("mutation_chance", ctypes.c_uint32), ("beta_b", ctypes.c_uint32),
                ("ff_B0_q16", ctypes.c_uint32), ("ff_gamma_q16", ctypes.c_uint32), ("ff_alpha_q16", ctypes.c_uint32),
                ("de_crossover", ctypes.c_uint32), ("ga_crossover", ctypes.c_uint32),
                ("unaware", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 4)]


_vp, _u32, _u64, _i32, _sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
_P = ctypes.POINTER

ct_objective_fn = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.POINTER(ctypes.c_float))


class ct_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_active", ctypes.c_uint32),
                ("max_admit_per_step", ctypes.c_uint32), ("keep_snapshots", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("objective", ct_objective_fn), ("objective_ctx", ctypes.c_void_p)]


class ct_run_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("generations", ctypes.c_uint32),
                ("n_valid", ctypes.c_uint64), ("footprint", ctypes.c_uint64), ("best_pos", ctypes.c_uint32),
                ("best_f", ctypes.c_float), ("reinits", ctypes.c_uint32), ("pop_size", ctypes.c_uint32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ct_server_counters(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("steps", "run_generations", "submitted", "admitted", "rejected",
                                               "completed", "queued", "active", "used_bytes", "peak_bytes")]

# name -> (restype, argtypes), exactly the declarations of include/ct.h
SIGNATURES = {
    "ct_last_error": (ctypes.c_char_p, []),
    "ct_version": (_i32, []),
    "ct_compile": (_i32, [_P(ctypes.c_char_p), _u32, _vp, _vp, _P(ctypes.c_char_p), _u32, _vp, _u32, _vp, _P(_u32)]),
    "ct_space_build": (_i32, [_vp, _vp, _u32, _vp, _vp, _u32, _vp, _P(_vp)]),
    "ct_space_count": (_i32, [_vp, _P(_u64), _P(_u64)]),
    "ct_space_info": (_i32, [_vp, _P(_u32), _P(_u32)]),
    "ct_space_valid_list": (_i32, [_vp, _P(_vp), _P(_vp)]),
    "ct_space_bitmask": (_i32, [_vp, _P(_vp), _P(_u64)]),
    "ct_space_copy_list": (_i32, [_vp, _vp, _vp, _vp]),
    "ct_space_copy_bitmask": (_i32, [_vp, _vp, _vp]),
    "ct_space_free": (None, [_vp]),
    "ct_valid_mask": (_i32, [_vp, _vp, _u64, _vp, _vp]),
    "ct_rank": (_i32, [_vp, _vp, _u64, _vp, _vp]),
    "ct_repair": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _vp, _vp, _vp, _vp]),
    "ct_repair_noalloc": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _vp, _vp, _vp, _vp]),
    "ct_repair_enum": (_i32, [_vp, _vp, _u64, _u32, _u64, _u32, _vp, _vp, _u64, _vp, _vp, _vp, _vp]),
    "ct_pop_create": (_i32, [_vp, _P(ct_pop_params), _vp, _vp, _P(_vp)]),
    "ct_step": (_i32, [_P(_vp), _u32, _u32, _u32, _vp]),
    "ct_pop_read": (_i32, [_vp, _vp, _vp, _P(_u32), _P(ctypes.c_float), _P(_u32), _P(_u32)]),
    "ct_pop_counters": (_i32, [_vp, _P(_u64), _P(_u64)]),
    "ct_pop_evaluated": (_i32, [_vp, _vp]),
    "ct_batch_create": (_i32, [_P(_vp), _u32, _P(_vp)]),
    "ct_batch_create_lanes": (_i32, [_P(_vp), _u32, _u32, _P(_vp)]),
    "ct_prof_sample": (_i32, [_u32]),
    "ct_prof_seen": (_i32, [ctypes.c_char_p, _P(_u64)]),
    "ct_batch_step": (_i32, [_vp, _u32, _u32, _vp]),
    "ct_batch_free": (None, [_vp]),
    "ct_batch_autotune": (_i32, [_vp, _u32, _u32, _u32, _vp]),
    "ct_batch_set_tuning": (_i32, [_vp, _u32, _u32, _u32, _u32]),
    "ct_batch_tuning": (_i32, [_vp, _P(_u32), _P(_u32), _P(_u32), _P(_u32), _P(_u32)]),
    "ct_pop_snapshot": (_i32, [_vp, _vp, _P(_sz)]),
    "ct_pop_restore": (_i32, [_vp, _vp, _sz]),
    "ct_pop_free": (None, [_vp]),
    "ct_space_footprint": (_i32, [_vp, _P(_u64)]),
    "ct_pop_footprint": (_i32, [_vp, _P(_u64)]),
    "ct_server_create": (_i32, [_P(ct_server_config), _P(_vp)]),
    "ct_server_submit": (_i32, [_vp, _vp, _vp, _u32, _vp, _vp, _u32, _P(ct_pop_params), _u32, ctypes.c_double,
                                _P(_u64)]),
    "ct_server_step": (_i32, [_vp, _P(_u32)]),
    "ct_server_now": (ctypes.c_double, [_vp]),
    "ct_server_poll": (_i32, [_vp, _P(ct_run_result), _u32, _P(_u32)]),
    "ct_server_snapshot": (_i32, [_vp, _u64, _vp, _P(_sz)]),
    "ct_server_release": (_i32, [_vp, _u64]),
    "ct_server_stats": (_i32, [_vp, _P(ct_server_counters)]),
    "ct_server_step_times": (_i32, [_vp, _vp, _vp, _u64, _P(_u64)]),
    "ct_server_free": (None, [_vp]),
    "ct_prof_enable": (_i32, [_i32]),
    "ct_prof_read": (_i32, [ctypes.c_char_p, _P(ctypes.c_double), _P(_u64)]),
    "ct_prof_select": (_i32, [ctypes.c_char_p]),
    "ct_prof_count_boxes": (_i32, [_i32]),
    "ct_prof_boxes": (_i32, [_vp]),
}

_lock = threading.Lock()
_lib = None


def load() -> ctypes.CDLL:
    """The loaded libct.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_28372_amd.build`")
            # torch carries its own HIP runtime under the same soname as the system one; loading torch
            # first makes libct bind to that runtime, so there is one runtime per process and torch's
            # streams and allocations are the library's too
            import torch  # noqa: F401
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(rc: int) -> None:
    if rc != CT_OK:
        raise CtError(rc, load().ct_last_error().decode())
