"""MI355X two-way continuous collision handling (HIP, gfx950).

The Python surface mirrors the C ABI of include/cc.h: a Context per device, a
resident Solver per scene (begin / iterate / run / state access), and
collide_step for one complete step. Arrays are torch tensors on the GPU:
positions float64 (N,3), inverse masses float64 (N,), triangles int32 (F,3),
edges int32 (E,2). All work runs in the HIP library on torch's current stream.
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import (CC_CCD_ALL, CC_EDGE_LEN, CC_MIXED, CC_TIME_KERNELS, CC_TIME_ONE, CC_TRACE,
                   CC_CCD_STEP, CC_UNGUARDED, CC_VALIDATE_INPUT, CCError, IterInfo, Params,
                   SceneDesc, Stats)

__all__ = ["Context", "Solver", "Server", "collide_step", "collide_step_batched", "params",
           "edges_from_tris", "normal_flow_target", "CC_EDGE_LEN", "CC_TIME_KERNELS",
           "CC_TIME_ONE", "CC_TRACE", "CC_MIXED", "CC_VALIDATE_INPUT", "CC_CCD_ALL",
           "CC_UNGUARDED", "CC_CCD_STEP", "CCError"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc, where):
    if rc != 0:
        raise CCError(rc, where)


def _dev(t, dtype, shape_last=None, name="array"):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    if t.device.type != "cuda":
        t = t.to("cuda")
    t = t.to(dtype).contiguous()
    if shape_last is not None and t.numel() and t.shape[-1] != shape_last:
        raise ValueError(f"{name}: last dimension must be {shape_last}")
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def params(**over) -> Params:
    """Defaults of Table 2 (cc_default_params) with keyword overrides; the flags
    are set with edge_len=, time_kernels=, trace=, mixed=, validate=, ccd_all=,
    unguarded= and ccd_step= (booleans) and time_one= (a family name of K_NAMES: that family alone
    is timed);
    backward= takes "gs" (default) or "jacobi"."""
    p = Params()
    _lib.load().cc_default_params(C.byref(p))
    for k, v in over.items():
        if k == "edge_len":
            p.flags = (p.flags | CC_EDGE_LEN) if v else (p.flags & ~CC_EDGE_LEN)
        elif k == "time_kernels":
            p.flags = (p.flags | CC_TIME_KERNELS) if v else (p.flags & ~CC_TIME_KERNELS)
        elif k == "time_one":
            if v is None:
                p.flags &= ~CC_TIME_ONE
            else:
                p.flags |= CC_TIME_ONE
                p.time_kind = _lib.K_NAMES.index(v) if isinstance(v, str) else int(v)
        elif k == "trace":
            p.flags = (p.flags | CC_TRACE) if v else (p.flags & ~CC_TRACE)
        elif k == "mixed":
            p.flags = (p.flags | CC_MIXED) if v else (p.flags & ~CC_MIXED)
        elif k == "ccd_all":
            p.flags = (p.flags | CC_CCD_ALL) if v else (p.flags & ~CC_CCD_ALL)
        elif k == "autotune":
            p.flags = (p.flags & ~_lib.CC_NO_AUTOTUNE) if v else (p.flags | _lib.CC_NO_AUTOTUNE)
        elif k == "ccd_step":
            p.flags = (p.flags | CC_CCD_STEP) if v else (p.flags & ~CC_CCD_STEP)
        elif k == "unguarded":
            p.flags = (p.flags | CC_UNGUARDED) if v else (p.flags & ~CC_UNGUARDED)
        elif k == "validate":
            p.flags = (p.flags | CC_VALIDATE_INPUT) if v else (p.flags & ~CC_VALIDATE_INPUT)
        elif k == "backward":
            p.backward = {"gs": 0, "jacobi": 1}.get(v, v)
        else:
            setattr(p, k, v)
    return p


def normal_flow_target(ctx: "Context", x, tris, beta: float, alpha: float, iters: int = 3):
    """Target y^[k+1] of the globally injective normal flow at x (cc_normal_flow_target):
    offset beta along the vertex normals, then `iters` cotangent-Laplacian Jacobi
    steps of intensity alpha. Returns a new (N, 3) float64 tensor."""
    torch = _torch()
    x = _dev(x, torch.float64, 3, "x").reshape(-1, 3)
    tris = _dev(tris, torch.int32, 3, "tris").reshape(-1, 3)
    y = torch.empty_like(x)
    _check(ctx.lib.cc_normal_flow_target(ctx.h, _ptr(x), x.shape[0], _ptr(tris), tris.shape[0],
                                         float(beta), float(alpha), int(iters), _ptr(y),
                                         _stream()), "cc_normal_flow_target")
    return y


def autotune_table():
    """The process-wide autotuner table: one dict per tuned (device, kernel, size
    class) with the choice and the measured time of each variant (ms)."""
    lib = _lib.load()
    n = C.c_int32()
    _check(lib.cc_autotune_entries(None, 0, C.byref(n)), "cc_autotune_entries")
    rows = (_lib.TuneEntry * max(n.value, 1))()
    _check(lib.cc_autotune_entries(rows, n.value, C.byref(n)), "cc_autotune_entries")
    names = {0: "traverse"}
    return [dict(device=r.device, kernel=names.get(r.kernel, r.kernel), size_class=r.size_class,
                 choice=r.choice, ms=[round(float(v), 4) for v in r.ms[:6]])
            for r in rows[:n.value]]


def edges_from_tris(tris):
    """Every side of every triangle once, as sorted (min, max) int32 pairs (host;
    cc_edges_from_tris_host)."""
    import numpy as np
    lib = _lib.load()
    t = np.ascontiguousarray(np.asarray(tris, dtype=np.int32).reshape(-1, 3))
    n = C.c_int32()
    tp = t.ctypes.data_as(C.c_void_p) if len(t) else None
    _check(lib.cc_edges_from_tris_host(tp, len(t), None, 0, C.byref(n)), "cc_edges_from_tris_host")
    out = np.zeros((n.value, 2), np.int32)
    if n.value:
        _check(lib.cc_edges_from_tris_host(tp, len(t), out.ctypes.data_as(C.c_void_p), n.value,
                                           C.byref(n)), "cc_edges_from_tris_host")
    return out


class Context:
    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        h = C.c_void_p()
        _check(self.lib.cc_context_create(device, C.byref(h)), "cc_context_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.cc_context_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Solver:
    """A resident scene: topology, state (x, y, r, D, P) and workspace on the GPU."""

    def __init__(self, ctx: Context, w, tris, edges, **over):
        torch = _torch()
        self.ctx = ctx
        self.lib = ctx.lib
        self.w = _dev(w, torch.float64, name="w").reshape(-1)
        self.tris = _dev(tris, torch.int32, 3, "tris").reshape(-1, 3)
        self.edges = _dev(edges, torch.int32, 2, "edges").reshape(-1, 2)
        self.n = self.w.numel()
        self.p = params(**over)
        h = C.c_void_p()
        _check(self.lib.cc_solver_create(ctx.h, self.n, _ptr(self.w), _ptr(self.tris),
                                         self.tris.shape[0], _ptr(self.edges),
                                         self.edges.shape[0], C.byref(self.p), C.byref(h),
                                         _stream()), "cc_solver_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.cc_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def begin(self, x, xt):
        torch = _torch()
        self._x0 = _dev(x, torch.float64, 3, "x").reshape(-1, 3)
        self._xt = _dev(xt, torch.float64, 3, "x_tilde").reshape(-1, 3)
        _check(self.lib.cc_solver_begin(self.h, _ptr(self._x0), _ptr(self._xt), _stream()),
               "cc_solver_begin")

    def iterate(self):
        stop = C.c_int32()
        info = IterInfo()
        _check(self.lib.cc_solver_iterate(self.h, C.byref(stop), C.byref(info), _stream()),
               "cc_solver_iterate")
        return bool(stop.value), info.as_dict()

    def run(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        st = Stats()
        _check(self.lib.cc_solver_run(self.h, _ptr(out), C.byref(st), _stream()), "cc_solver_run")
        return out, st.as_dict()

    def stats(self):
        st = Stats()
        _check(self.lib.cc_solver_stats(self.h, C.byref(st)), "cc_solver_stats")
        return st.as_dict()

    def state(self):
        torch = _torch()
        x = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        r = torch.empty(self.n, dtype=torch.float64, device="cuda")
        D = C.c_double()
        _check(self.lib.cc_solver_get_state(self.h, _ptr(x), _ptr(y), _ptr(r), C.byref(D),
                                            _stream()), "cc_solver_get_state")
        return x, y, r, D.value

    def set_state(self, x, y, r, D, P):
        torch = _torch()
        x = _dev(x, torch.float64, 3, "x")
        y = _dev(y, torch.float64, 3, "y")
        r = _dev(r, torch.float64, name="r")
        P = _dev(torch.as_tensor(P).view(torch.int64) if not isinstance(P, torch.Tensor) else P,
                 torch.int64, name="P")
        _check(self.lib.cc_solver_set_state(self.h, _ptr(x), _ptr(y), _ptr(r), float(D), _ptr(P),
                                            P.numel(), _stream()), "cc_solver_set_state")

    def P(self):
        torch = _torch()
        n = C.c_int64()
        _check(self.lib.cc_solver_get_P(self.h, None, 0, C.byref(n), _stream()), "get_P")
        out = torch.empty(n.value, dtype=torch.int64, device="cuda")
        _check(self.lib.cc_solver_get_P(self.h, _ptr(out), n.value, C.byref(n), _stream()),
               "get_P")
        return out

    def A(self):
        torch = _torch()
        n = C.c_int64()
        _check(self.lib.cc_solver_get_A(self.h, None, None, 0, C.byref(n), _stream()), "get_A")
        k = torch.empty(n.value, dtype=torch.int64, device="cuda")
        c = torch.empty(n.value, dtype=torch.int32, device="cuda")
        _check(self.lib.cc_solver_get_A(self.h, _ptr(k), _ptr(c), n.value, C.byref(n),
                                        _stream()), "get_A")
        return k, c

    def Di(self):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(self.lib.cc_solver_get_Di(self.h, _ptr(out), _stream()), "get_Di")
        return out

    def search(self, x, dmax):
        torch = _torch()
        x = _dev(x, torch.float64, 3, "x")
        n = C.c_int64()
        _check(self.lib.cc_solver_search(self.h, _ptr(x), float(dmax), None, 0, C.byref(n),
                                         _stream()), "search")
        out = torch.empty(n.value, dtype=torch.int64, device="cuda")
        _check(self.lib.cc_solver_search(self.h, _ptr(x), float(dmax), _ptr(out), n.value,
                                         C.byref(n), _stream()), "search")
        return out


def collide_step(ctx: Context, x, xt, w, tris, edges, **over):
    """One complete two-way step; returns (x_next, stats)."""
    torch = _torch()
    x = _dev(x, torch.float64, 3, "x").reshape(-1, 3)
    xt = _dev(xt, torch.float64, 3, "x_tilde").reshape(-1, 3)
    w = _dev(w, torch.float64, name="w").reshape(-1)
    tris = _dev(tris, torch.int32, 3, "tris").reshape(-1, 3)
    edges = _dev(edges, torch.int32, 2, "edges").reshape(-1, 2)
    p = params(**over)
    out = torch.empty_like(x)
    st = Stats()
    _check(ctx.lib.cc_collide_step(ctx.h, _ptr(x), _ptr(xt), _ptr(w), x.shape[0], _ptr(tris),
                                   tris.shape[0], _ptr(edges), edges.shape[0], C.byref(p),
                                   _ptr(out), C.byref(st), _stream()), "cc_collide_step")
    return out, st.as_dict()


def collide_step_batched(ctx: Context, scenes, **over):
    """One step for each scene (dicts with x, xt, w, tris, edges); the scenes run
    concurrently on the GPU. Returns a list of (x_next, stats)."""
    torch = _torch()
    keep, descs = [], (SceneDesc * max(len(scenes), 1))()
    outs = []
    for i, sc in enumerate(scenes):
        x = _dev(sc["x"], torch.float64, 3, "x").reshape(-1, 3)
        xt = _dev(sc["xt"], torch.float64, 3, "x_tilde").reshape(-1, 3)
        w = _dev(sc["w"], torch.float64, name="w").reshape(-1)
        tris = _dev(sc["tris"], torch.int32, 3, "tris").reshape(-1, 3)
        edges = _dev(sc["edges"], torch.int32, 2, "edges").reshape(-1, 2)
        out = torch.empty_like(x)
        keep += [x, xt, w, tris, edges]
        outs.append(out)
        descs[i] = SceneDesc(_ptr(x), _ptr(xt), _ptr(w), x.shape[0], _ptr(tris), tris.shape[0],
                             _ptr(edges), edges.shape[0], _ptr(out))
    p = params(**over)
    st = (Stats * max(len(scenes), 1))()
    _check(ctx.lib.cc_collide_step_batched(ctx.h, descs, len(scenes), C.byref(p), st, _stream()),
           "cc_collide_step_batched")
    return [(outs[i], st[i].as_dict()) for i in range(len(scenes))]


class Server:
    """Resident scenes admitted against an HBM budget (cc_scene_* of the C ABI).

    admit() returns a handle or None when the budget is full; submit() starts one
    step towards x~ from the scene's resident state; poll() returns None while the
    step runs, else (x_next, stats); release() frees the scene."""

    def __init__(self, ctx: Context, budget_bytes: int = 0):
        self.ctx = ctx
        self.lib = ctx.lib
        _check(self.lib.cc_context_set_budget(ctx.h, int(budget_bytes)), "cc_context_set_budget")
        self._keep = {}

    def scene_bytes(self, n, nt, ne):
        return int(self.lib.cc_scene_bytes(n, nt, ne))

    def admit(self, x, w, tris, edges, **over):
        torch = _torch()
        x = _dev(x, torch.float64, 3, "x").reshape(-1, 3)
        w = _dev(w, torch.float64, name="w").reshape(-1)
        tris = _dev(tris, torch.int32, 3, "tris").reshape(-1, 3)
        edges = _dev(edges, torch.int32, 2, "edges").reshape(-1, 2)
        d = SceneDesc(_ptr(x), None, _ptr(w), x.shape[0], _ptr(tris), tris.shape[0],
                      _ptr(edges), edges.shape[0], None)
        p = params(**over)
        h = C.c_int32()
        rc = self.lib.cc_scene_admit(self.ctx.h, C.byref(d), C.byref(p), C.byref(h))
        if rc == _lib.CC_EAGAIN:
            return None
        _check(rc, "cc_scene_admit")
        self._keep[h.value] = [x.shape[0], None]
        return h.value

    def submit(self, h, xt):
        torch = _torch()
        xt = _dev(xt, torch.float64, 3, "x_tilde").reshape(-1, 3)
        # the step reads x~ on the library's stream: finish torch's work first
        torch.cuda.current_stream().synchronize()
        self._keep[h][1] = xt
        _check(self.lib.cc_scene_submit(self.ctx.h, h, _ptr(xt)), "cc_scene_submit")

    def poll(self, h, out=None):
        torch = _torch()
        n = self._keep[h][0]
        if out is None:
            out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        torch.cuda.current_stream().synchronize()  # out may reuse memory torch still writes
        st = Stats()
        rc = self.lib.cc_scene_poll(self.ctx.h, h, _ptr(out), C.byref(st))
        if rc == _lib.CC_EBUSY:
            return None
        _check(rc, "cc_scene_poll")
        return out, st.as_dict()

    def release(self, h):
        _check(self.lib.cc_scene_release(self.ctx.h, h), "cc_scene_release")
        self._keep.pop(h, None)
