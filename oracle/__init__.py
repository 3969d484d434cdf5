"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark import
this package. It never touches the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborcc.so")
_lib = None

KEY_EE = 1 << 63
KEY_VV = 1 << 62

# Table 2 defaults (L depends on the time step; the scene may override)
DEFAULTS = dict(delta=1e-3, d_min=2e-3, d_max=4e-3, sigma=1.1, gamma=0.9, eps=1e-4,
                kappa=1e-3, max_iters=512, gs_sweeps=1, max_colors=1024, edge_len=1,
                seed=0x2211_04045, omega=0.5, backward=0, ccd_all=0, unguarded=0, ccd_step=0)


class Params(C.Structure):
    _fields_ = [("delta", C.c_double), ("d_min", C.c_double), ("d_max", C.c_double),
                ("sigma", C.c_double), ("gamma", C.c_double), ("eps", C.c_double),
                ("kappa", C.c_double), ("max_iters", C.c_int32),
                ("gs_sweeps", C.c_int32), ("max_colors", C.c_int32),
                ("edge_len", C.c_int32), ("seed", C.c_uint64), ("omega", C.c_double),
                ("backward", C.c_int32), ("ccd_all", C.c_int32),
                ("unguarded", C.c_int32), ("ccd_step", C.c_int32)]


class Iter(C.Structure):
    _fields_ = [("searched", C.c_int32), ("n_colors", C.c_int32), ("n_p", C.c_int64),
                ("n_pf", C.c_int64), ("n_a", C.c_int64), ("ccd_fail", C.c_int64),
                ("ccd_hits", C.c_int64), ("n_back", C.c_int64), ("n_scaled", C.c_int64),
                ("d_before", C.c_double), ("d_after", C.c_double),
                ("move_max", C.c_double), ("r_inf", C.c_double),
                ("fp_pf", C.c_uint64), ("fp_a", C.c_uint64), ("fp_col", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    d, i32, i64, u64, vp = C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [i32, vp, vp, i32, vp, i32, P(Params)]
    lib.orc_destroy.argtypes = [vp]
    lib.orc_begin.argtypes = [vp, vp, vp]
    lib.orc_begin.restype = C.c_int
    lib.orc_iterate.argtypes = [vp, P(Iter)]
    lib.orc_iterate.restype = C.c_int
    lib.orc_run.argtypes = [vp, vp, P(Iter), i32]
    lib.orc_run.restype = C.c_int
    lib.orc_get_state.argtypes = [vp, vp, vp, vp, P(d)]
    lib.orc_set_state.argtypes = [vp, vp, vp, vp, d, vp, i64]
    lib.orc_set_state.restype = C.c_int
    lib.orc_get_P.argtypes = [vp, vp, i64]
    lib.orc_get_P.restype = i64
    lib.orc_get_A.argtypes = [vp, vp, vp, i64]
    lib.orc_get_A.restype = i64
    lib.orc_get_Di.argtypes = [vp, vp]
    lib.orc_pt_tri_d2.argtypes = [vp, vp, vp, vp, vp]
    lib.orc_pt_tri_d2.restype = d
    lib.orc_seg_seg_d2.argtypes = [vp, vp, vp, vp, vp]
    lib.orc_seg_seg_d2.restype = d
    lib.orc_contact_row.argtypes = [vp, vp, u64, vp, P(d), vp, P(d)]
    lib.orc_contact_row.restype = C.c_int
    lib.orc_search.argtypes = [vp, vp, d, C.c_int, vp, i64]
    lib.orc_search.restype = i64
    lib.orc_color_rows.argtypes = [vp, i64, vp, vp, vp]
    lib.orc_color_rows.restype = i32
    lib.orc_color_rows_greedy.argtypes = [vp, i64, vp, vp, vp]
    lib.orc_color_rows_greedy.restype = i32
    lib.orc_greedy_prio.argtypes = [C.c_uint64, C.c_uint64]
    lib.orc_greedy_prio.restype = C.c_uint64
    lib.orc_mix64.argtypes = [u64]
    lib.orc_mix64.restype = u64
    lib.orc_ccd_hit.argtypes = [vp, vp, C.c_int, d, P(d)]
    lib.orc_ccd_hit.restype = C.c_int
    lib.orc_seg_tri_meet.argtypes = [vp, vp, vp, vp, vp, d]
    lib.orc_seg_tri_meet.restype = C.c_int
    lib.orc_validate.argtypes = [vp, vp, d]
    lib.orc_validate.restype = C.c_int
    lib.orc_particles.argtypes = [vp, vp]
    lib.orc_particles.restype = i32
    lib.orc_normal_flow.argtypes = [i32, vp, vp, i32, d, d, i32, vp]
    lib.orc_normal_flow.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None and a.size else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(**over) -> Params:
    v = dict(DEFAULTS)
    v.update(over)
    if v.get("backward") == "jacobi":
        v["backward"] = 1
    elif v.get("backward") == "gs":
        v["backward"] = 0
    return Params(**v)


def mix64(z: int) -> int:
    return int(_load().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def pt_tri_d2(p, a, b, c):
    bary = np.zeros(3)
    d2 = _load().orc_pt_tri_d2(_ptr(_f64(p)), _ptr(_f64(a)), _ptr(_f64(b)),
                               _ptr(_f64(c)), _ptr(bary))
    return d2, bary


def seg_seg_d2(a, b, c, e):
    st = np.zeros(2)
    d2 = _load().orc_seg_seg_d2(_ptr(_f64(a)), _ptr(_f64(b)), _ptr(_f64(c)),
                                _ptr(_f64(e)), _ptr(st))
    return d2, st


def ccd_hit(q, dq, ee, eta: float = 1e-12):
    """Continuous test of points q moving by dq over t in [0,1]: ee False/0 vertex-
    triangle (4,3), True/1 edge-edge (4,3), 2 vertex-vertex (2,3)."""
    t = C.c_double(-1.0)
    qq = np.zeros(12)
    dd = np.zeros(12)
    qf, df = _f64(q).reshape(-1), _f64(dq).reshape(-1)
    qq[:len(qf)] = qf
    dd[:len(df)] = df
    hit = _load().orc_ccd_hit(_ptr(qq), _ptr(dd), int(ee), eta, C.byref(t))
    return bool(hit), t.value


def seg_tri_meet(p, q, a, b, c, tol: float = 1e-9) -> bool:
    return bool(_load().orc_seg_tri_meet(*(_ptr(_f64(v)) for v in (p, q, a, b, c)), float(tol)))


def normal_flow(x, tris, beta: float, alpha: float, iters: int = 3):
    """y^[k+1] of the globally injective normal flow (orc_normal_flow)."""
    x = _f64(x)
    tris = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    y = np.zeros_like(x)
    rc = _load().orc_normal_flow(len(x), _ptr(x), _ptr(tris), len(tris), float(beta),
                                 float(alpha), int(iters), _ptr(y))
    if rc != 0:
        raise ValueError("orc_normal_flow: bad argument")
    return y


def vt_key(a: int, f: int) -> int:
    return (a << 32) | f


def ee_key(e: int, g: int) -> int:
    return KEY_EE | (e << 32) | g


def vv_key(a: int, b: int) -> int:
    return KEY_VV | (min(a, b) << 32) | max(a, b)


class Scene:
    """One collision-handling problem held by the oracle."""

    def __init__(self, w, tris, edges, **over):
        self.lib = _load()
        self.w = _f64(w)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
        self.edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        self.n = len(self.w)
        self.p = params(**over)
        self.h = self.lib.orc_create(self.n, _ptr(self.w), _ptr(self.tris), len(self.tris),
                                     _ptr(self.edges), len(self.edges), C.byref(self.p))

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_destroy(self.h)
            self.h = None

    def particles(self):
        """Vertices in no triangle and no edge (the vertex-vertex pair universe)."""
        n = self.lib.orc_particles(self.h, None)
        out = np.zeros(n, np.int32)
        self.lib.orc_particles(self.h, _ptr(out))
        return out

    def begin(self, x, xt):
        rc = self.lib.orc_begin(self.h, _ptr(_f64(x)), _ptr(_f64(xt)))
        if rc != 0:
            raise RuntimeError(f"orc_begin failed: {rc}")

    def iterate(self):
        it = Iter()
        rc = self.lib.orc_iterate(self.h, C.byref(it))
        if rc < 0:
            raise RuntimeError(f"orc_iterate failed: {rc}")
        return rc == 1, it.as_dict()

    def run(self, x, xt, trace_cap: int = 0):
        self.begin(x, xt)
        out = np.zeros((self.n, 3))
        tr = (Iter * max(trace_cap, 1))()
        n = self.lib.orc_run(self.h, _ptr(out), tr if trace_cap else None, trace_cap)
        if n < 0:
            raise RuntimeError(f"orc_run failed: {n}")
        return out, n, [tr[i].as_dict() for i in range(min(n, trace_cap))]

    def state(self):
        x = np.zeros((self.n, 3))
        y = np.zeros((self.n, 3))
        r = np.zeros(self.n)
        D = C.c_double()
        self.lib.orc_get_state(self.h, _ptr(x), _ptr(y), _ptr(r), C.byref(D))
        return x, y, r, D.value

    def set_state(self, x, y, r, D, P):
        P = np.ascontiguousarray(P, dtype=np.uint64)
        self.lib.orc_set_state(self.h, _ptr(_f64(x)), _ptr(_f64(y)), _ptr(_f64(r)),
                               float(D), _ptr(P), len(P))

    def P(self):
        n = self.lib.orc_get_P(self.h, None, 0)
        out = np.zeros(n, np.uint64)
        self.lib.orc_get_P(self.h, _ptr(out), n)
        return out

    def A(self):
        n = self.lib.orc_get_A(self.h, None, None, 0)
        k = np.zeros(n, np.uint64)
        c = np.zeros(n, np.int32)
        self.lib.orc_get_A(self.h, _ptr(k), _ptr(c), n)
        return k, c

    def Di(self):
        out = np.zeros(self.n)
        self.lib.orc_get_Di(self.h, _ptr(out))
        return out

    def validate(self, x, tol=1e-9):
        """1 when x is not in the free space (see orc_validate), else 0."""
        return int(self.lib.orc_validate(self.h, _ptr(_f64(x)), float(tol)))

    def search(self, x, dmax, brute=False):
        x = _f64(x)
        n = self.lib.orc_search(self.h, _ptr(x), dmax, int(brute), None, 0)
        out = np.zeros(n, np.uint64)
        self.lib.orc_search(self.h, _ptr(x), dmax, int(brute), _ptr(out), n)
        return out

    def contact_row(self, x, key):
        v = np.zeros(4, np.int32)
        J = np.zeros(12)
        c0 = C.c_double()
        inv = C.c_double()
        kind = self.lib.orc_contact_row(self.h, _ptr(_f64(x)), int(key), _ptr(v),
                                        C.byref(c0), _ptr(J), C.byref(inv))
        return dict(kind=kind, v=v, c0=c0.value, J=J.reshape(4, 3), inv_a=inv.value)

    def color(self, rows, keys):
        rows = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, 4)
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        col = np.zeros(len(rows), np.int32)
        nc = self.lib.orc_color_rows(self.h, len(rows), _ptr(rows), _ptr(keys), _ptr(col))
        if nc < 0:
            raise RuntimeError("palette exhausted")
        return col, nc

    def color_greedy(self, rows, keys):
        """The edge-length rows' colouring: greedy in decreasing greedy_prio order."""
        rows = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, 4)
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        col = np.zeros(len(rows), np.int32)
        nc = self.lib.orc_color_rows_greedy(self.h, len(rows), _ptr(rows), _ptr(keys), _ptr(col))
        if nc < 0:
            raise RuntimeError("palette exhausted")
        return col, nc

    def greedy_prio(self, key, seed):
        return int(self.lib.orc_greedy_prio(int(key), int(seed)))


def collide_step(scene: dict, **over):
    """Run one full step of the oracle on a scene dict from `scenes`."""
    p = dict(scene.get("params", {}))
    p.update(over)
    s = Scene(scene["w"], scene["tris"], scene["edges"], **p)
    out, n, trace = s.run(scene["x"], scene["xt"], trace_cap=p.get("max_iters", 512))
    return out, n, trace
