"""ctypes binding of libcc.so (the HIP two-way collision-handling step).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library. Arrays are torch tensors on the GPU; the binding passes their data
pointers and torch's current stream. There is no fallback: without the built
library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcc.so")

CC_EDGE_LEN = 1
CC_TIME_KERNELS = 2
CC_TRACE = 4
CC_MIXED = 8
CC_VALIDATE_INPUT = 16
CC_CCD_ALL = 32
CC_TIME_ONE = 64
CC_UNGUARDED = 128
CC_CCD_STEP = 256
CC_NO_AUTOTUNE = 512
CC_GAUSS_SEIDEL = 0
CC_JACOBI = 1
K_NAMES = ["search", "pair", "color", "gs", "forward", "cert"]

ERRORS = {0: "ok", -1: "invalid argument", -2: "device allocation failed",
          -3: "pair capacity exceeded", -4: "HIP runtime error",
          -5: "colour palette exhausted", -6: "call out of order",
          -7: "over the HBM budget", -8: "step still running",
          -9: "x_prev is not in the free space"}
CC_EAGAIN = -7
CC_EBUSY = -8
CC_ENOTFREE = -9


class CCError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [("delta", C.c_double), ("d_min", C.c_double), ("d_max", C.c_double),
                ("sigma", C.c_double), ("gamma", C.c_double), ("eps", C.c_double),
                ("kappa", C.c_double), ("max_iters", C.c_int32), ("gs_sweeps", C.c_int32),
                ("max_colors", C.c_int32), ("flags", C.c_uint32), ("seed", C.c_uint64),
                ("omega", C.c_double), ("backward", C.c_int32), ("time_kind", C.c_int32)]


class IterInfo(C.Structure):
    _fields_ = [("searched", C.c_int32), ("n_colors", C.c_int32), ("n_p", C.c_int64),
                ("n_pf", C.c_int64), ("n_a", C.c_int64), ("ccd_fail", C.c_int64),
                ("ccd_hits", C.c_int64), ("n_back", C.c_int64), ("n_scaled", C.c_int64),
                ("d_before", C.c_double),
                ("d_after", C.c_double), ("move_max", C.c_double),
                ("r_inf", C.c_double), ("fp_pf", C.c_uint64), ("fp_a", C.c_uint64),
                ("fp_col", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SceneDesc(C.Structure):
    _fields_ = [("x_prev", C.c_void_p), ("x_tilde", C.c_void_p), ("inv_mass", C.c_void_p),
                ("n_verts", C.c_int32), ("tris", C.c_void_p), ("n_tris", C.c_int32),
                ("edges", C.c_void_p), ("n_edges", C.c_int32), ("x_next", C.c_void_p)]


class TuneEntry(C.Structure):
    _fields_ = [("device", C.c_int32), ("kernel", C.c_int32), ("size_class", C.c_int32),
                ("choice", C.c_int32), ("ms", C.c_float * 8)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("searches", C.c_int32), ("status", C.c_int32),
                ("max_colors_used", C.c_int32), ("pair_updates", C.c_int64),
                ("row_updates", C.c_int64), ("ccd_fail", C.c_int64), ("ccd_hits", C.c_int64),
                ("n_back", C.c_int64), ("n_scaled", C.c_int64), ("r_inf", C.c_double),
                ("kernel_ms", C.c_double * 6), ("kernel_launches", C.c_int64 * 6),
                ("kernel_bytes", C.c_double * 6)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_[:11]}
        d["kernels"] = {K_NAMES[i]: dict(ms=self.kernel_ms[i], launches=self.kernel_launches[i],
                                         bytes=self.kernel_bytes[i]) for i in range(6)}
        return d


_lib = None


def load():
    """Load libcc.so; raises if it is missing (build with build.py first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2211_04045_amd/build.py "
                          "(the HIP library has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, d, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
    P = C.POINTER
    sigs = {
        "cc_default_params": (None, [P(Params)]),
        "cc_strerror": (C.c_char_p, [C.c_int]),
        "cc_context_create": (C.c_int, [C.c_int, P(vp)]),
        "cc_context_destroy": (None, [vp]),
        "cc_collide_step": (C.c_int, [vp, vp, vp, vp, i32, vp, i32, vp, i32, P(Params), vp,
                                      P(Stats), vp]),
        "cc_collide_step_batched": (C.c_int, [vp, P(SceneDesc), i32, P(Params), P(Stats), vp]),
        "cc_solver_create": (C.c_int, [vp, i32, vp, vp, i32, vp, i32, P(Params), P(vp), vp]),
        "cc_solver_destroy": (None, [vp]),
        "cc_solver_begin": (C.c_int, [vp, vp, vp, vp]),
        "cc_solver_iterate": (C.c_int, [vp, P(i32), P(IterInfo), vp]),
        "cc_solver_run": (C.c_int, [vp, vp, P(Stats), vp]),
        "cc_solver_get_state": (C.c_int, [vp, vp, vp, vp, P(d), vp]),
        "cc_solver_set_state": (C.c_int, [vp, vp, vp, vp, d, vp, i64, vp]),
        "cc_solver_get_P": (C.c_int, [vp, vp, i64, P(i64), vp]),
        "cc_solver_get_A": (C.c_int, [vp, vp, vp, i64, P(i64), vp]),
        "cc_solver_get_Di": (C.c_int, [vp, vp, vp]),
        "cc_solver_search": (C.c_int, [vp, vp, d, vp, i64, P(i64), vp]),
        "cc_solver_stats": (C.c_int, [vp, P(Stats)]),
        "cc_context_set_budget": (C.c_int, [vp, C.c_size_t]),
        "cc_scene_bytes": (C.c_size_t, [i32, i32, i32]),
        "cc_scene_admit": (C.c_int, [vp, P(SceneDesc), P(Params), P(i32)]),
        "cc_scene_submit": (C.c_int, [vp, i32, vp]),
        "cc_scene_poll": (C.c_int, [vp, i32, vp, P(Stats)]),
        "cc_scene_release": (C.c_int, [vp, i32]),
        "cc_edges_from_tris_host": (C.c_int, [vp, i32, vp, i32, P(i32)]),
        "cc_normal_flow_target": (C.c_int, [vp, vp, i32, vp, i32, d, d, i32, vp, vp]),
        "cc_normal_flow_target_noalloc": (C.c_int, [vp, vp, i32, vp, i32, d, d, i32, vp, vp]),
        "cc_autotune_entries": (C.c_int, [P(TuneEntry), i32, P(i32)]),
        "cc_autotune_reset": (None, []),
        "cc_autotune_force": (C.c_int, [i32, i32]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


EXPORTED = ["cc_default_params", "cc_strerror", "cc_context_create", "cc_context_destroy",
            "cc_collide_step", "cc_collide_step_batched", "cc_solver_create", "cc_solver_destroy", "cc_solver_begin",
            "cc_solver_iterate", "cc_solver_run", "cc_solver_get_state",
            "cc_solver_set_state", "cc_solver_get_P", "cc_solver_get_A", "cc_solver_get_Di",
            "cc_solver_search", "cc_solver_stats", "cc_context_set_budget", "cc_scene_bytes",
            "cc_scene_admit", "cc_scene_submit", "cc_scene_poll", "cc_scene_release",
            "cc_edges_from_tris_host", "cc_normal_flow_target", "cc_normal_flow_target_noalloc",
            "cc_autotune_entries", "cc_autotune_reset", "cc_autotune_force"]
