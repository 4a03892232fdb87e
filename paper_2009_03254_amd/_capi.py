"""ctypes declarations of the C ABI in include/bcmc.h.

Loads the in-tree libbcmc.so and raises if it is missing: there is no other
implementation to fall back to."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbcmc.so")

OK, E_INVALID, E_NOMEM, E_CACHE_CAP, E_CAPACITY, E_HIP, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
_NAMES = {E_INVALID: "BCMC_E_INVALID", E_NOMEM: "BCMC_E_NOMEM", E_CACHE_CAP: "BCMC_E_CACHE_CAP",
          E_CAPACITY: "BCMC_E_CAPACITY", E_HIP: "BCMC_E_HIP", E_NONFINITE: "BCMC_E_NONFINITE"}


class BcmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Stats(C.Structure):
    _fields_ = [("n_blocks", C.c_uint64), ("n_active", C.c_uint64), ("n_new", C.c_uint64),
                ("n_evicted", C.c_uint64), ("n_occupied", C.c_uint64),
                ("n_candidates", C.c_uint64), ("n_slots", C.c_uint64),
                ("n_triangles", C.c_uint64), ("calls", C.c_uint64), ("n_general", C.c_uint64),
                ("hit_rate", C.c_double),
                ("alg_bytes", C.c_double), ("stage_ms", C.c_double * 8)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "stage_ms"}
        d["stage_ms"] = list(self.stage_ms)
        return d


class BatchInfo(C.Structure):
    _fields_ = [("n_volumes", C.c_uint64), ("n_jobs", C.c_uint64), ("n_blocks", C.c_uint64),
                ("n_job_blocks", C.c_uint64), ("n_resident", C.c_uint64), ("n_new", C.c_uint64),
                ("n_pairs", C.c_uint64), ("n_vertices", C.c_uint64),
                ("stage_blocks", C.c_uint32), ("grid", C.c_uint32),
                ("workgroups_per_cu", C.c_uint32), ("front_grid", C.c_uint32),
                ("scan_schedule", C.c_uint32),
                ("decode_grid", C.c_uint32), ("ran_front_grid", C.c_uint32),
                ("ran_decode_grid", C.c_uint32), ("ran_grid", C.c_uint32),
                ("graph", C.c_int32),
                ("graph_unsupported", C.c_int32), ("last_ms", C.c_float),
                ("phase_ms", C.c_float * 8)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["phase_ms"] = [float(x) for x in self.phase_ms]
        return d


_P, _u32, _u64, _i32, _f32, _int = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_float, C.c_int

SIGNATURES = {
    "bcmc_load_compressed": (_int, [_P, _u64, _int, _u32, _u32, _u32, _int, _u32, _P, _P]),
    "bcmc_volume_from_blocks": (_int, [_P, _u32, _u32, _u32, _P, _P]),
    "bcmc_set_cache_budget": (_int, [_P, _u64, _u64]),
    "bcmc_rebind_blocks": (_int, [_P, _P, _P]),
    "bcmc_reset_cache": (_int, [_P, _P]),
    "bcmc_extract": (_int, [_P, _f32, _P, _u64, _P, _P]),
    "bcmc_backward": (_int, [_P, _f32, _P, _u64, _P, _P, _P]),
    "bcmc_get_stats": (_int, [_P, _P]),
    "bcmc_set_profiling": (_int, [_P, _int]),
    "bcmc_set_profiling_stages": (_int, [_P, _u32]),
    "bcmc_set_vertex_format": (_int, [_P, _int]),
    "bcmc_free": (None, [_P]),
    "bcmc_last_error": (C.c_char_p, []),
    "bcmc_num_blocks": (_u64, [_u32, _u32, _u32]),
    "bcmc_encode": (_int, [_P, _int, _u32, _u32, _u32, _u32, _P, _P]),
    "bcmc_decode_all": (_int, [_P, _P, _P]),
    "bcmc_mc_table": (_int, [_P]),
    "bcmc_copy_calibration": (_int, [_P, _P, _u64, _P]),
    "bcmc_batch_create": (_int, [_P, _u32, _P, _P, _u32, _P, _P]),
    "bcmc_batch_set_isos": (_int, [_P, _P, _P]),
    "bcmc_batch_reset": (_int, [_P, _P]),
    "bcmc_batch_set_graph": (_int, [_P, _int]),
    "bcmc_batch_run": (_int, [_P, _P, _u64, _P, _P]),
    "bcmc_batch_set_schedule": (_int, [_P, _int, _int, _int, _int]),
    "bcmc_batch_tune": (_int, [_P, C.c_char_p, _P]),
    "bcmc_batch_get_info": (_int, [_P, _P]),
    "bcmc_batch_free": (None, [_P]),
    "bcmc_dense_create": (_int, [_u32, _u32, _u32, _P]),
    "bcmc_dense_extract": (_int, [_P, _P, _f32, _P, _u64, _P, _P]),
    "bcmc_dense_active_cells": (_int, [_P, _P]),
    "bcmc_dense_free": (None, [_P]),
    "bcmc_extract_blocks_noalloc": (_int, [_P, _u32, _u32, _u32, _f32, _P, _u64, _P, _P]),
    "bcmc_debug_ranges": (_int, [_P, _P]),
    "bcmc_debug_active": (_int, [_P, _P, _P, _P]),
    "bcmc_debug_new": (_int, [_P, _P, _P]),
    "bcmc_debug_cache_state": (_int, [_P, _P, _P, _P, _P]),
    "bcmc_debug_slot_data": (_int, [_P, _P]),
    "bcmc_vertices_to_q10": (_int, [_P, _u64, _P, _P]),
    "bcmc_debug_age_cache": (_int, [_P, _u32, _P]),
    "bcmc_debug_block_counts": (_int, [_P, _P, _P, _u64]),
    "bcmc_debug_cases": (_int, [_P, _f32, _P, _P]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run python -m paper_2009_03254_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != OK:
        raise BcmcError(rc, lib().bcmc_last_error().decode(errors="replace"))
    return rc
