"""Continuous serving of collision-handling steps over resident scenes.

A request is one scene that needs `steps` consecutive time steps. Requests arrive
over time; each is admitted into the library's resident-scene server as soon as
the HBM budget (and the cap on concurrently resident scenes) allows, in arrival
order. The scene's state, pair set and tree then stay on the device between its
steps. When a step completes, the next target is formed from the result by the
caller's time integration (x~_{n+1} = 2 x_{n+1} - x_n + h^2 g for free vertices,
the velocity being the step's own displacement over h), and the next step is
submitted at once. The library's scheduler runs the steps of all running scenes
together, in the same kernel launches; a new step joins at the next iteration
boundary.

Latency of a step: from the moment it could start (the request's arrival for its
first step, the previous step's completion for the others) to the moment its
result is back.

A step that fails (the library returns an error for it, e.g. a colour palette too
small for its contact set) ends its request: the scene is released, the error is
recorded with the request and step, and the other requests go on.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np

GRAVITY = (0.0, 0.0, -9.81)


def next_target(x_prev, x_new, w, h):
    """x~ = x + h v + h^2 g with v = (x_new - x_prev)/h; vertices with w = 0 stay."""
    import torch
    g = torch.tensor(GRAVITY, dtype=x_new.dtype, device=x_new.device)
    xt = x_new + (x_new - x_prev) + (h * h) * g
    static = (w == 0).unsqueeze(1)
    return torch.where(static, x_new, xt)


class _Live:
    __slots__ = ("req", "handle", "step", "t_ready", "x_prev", "x_cur", "w", "out", "iters",
                 "pairs")


def run_stream(ctx, requests, arrivals, steps: int = 10, budget_bytes: int = 0,
               max_resident: int = 64, keep_results: bool = False, poll_sleep: float = 2e-4,
               progress=None, **over):
    """Serve `requests` (scene dicts with x, xt, w, tris, edges, h) arriving at
    `arrivals` (seconds from the start; all zero = a closed batch). Returns a dict
    with per-step latencies (s), the wall time, completed steps, and per-request
    results when keep_results is set."""
    import torch

    from . import Server
    srv = Server(ctx, budget_bytes)
    order = np.argsort(np.asarray(arrivals), kind="stable")
    pending = deque(int(i) for i in order)
    live: dict[int, _Live] = {}
    from . import CCError
    lat, iters, pairs, failed = [], [], [], []
    peak_resident, peak_bytes, used = 0, 0, 0
    results = {} if keep_results else None
    done_steps = 0
    t0 = time.perf_counter()
    t_report = t0
    try:
        while pending or live:
            now = time.perf_counter() - t0
            progressed = False
            # admission, in arrival order
            while pending and arrivals[pending[0]] <= now and len(live) < max_resident:
                i = pending[0]
                sc = requests[i]
                prm = dict(sc.get("params", {}))
                prm.update(over)
                h = srv.admit(sc["x"], sc["w"], sc["tris"], sc["edges"], **prm)
                if h is None:
                    break  # the head waits until memory frees up
                pending.popleft()
                L = _Live()
                L.req, L.handle, L.step = i, h, 0
                L.t_ready = float(arrivals[i])
                L.x_cur = torch.as_tensor(sc["x"], dtype=torch.float64, device="cuda")
                L.x_prev = None
                L.w = torch.as_tensor(sc["w"], dtype=torch.float64, device="cuda")
                L.out = torch.empty_like(L.x_cur)
                L.iters, L.pairs = [], []
                srv.submit(h, sc["xt"])
                live[h] = L
                used += srv.scene_bytes(len(sc["x"]), len(sc["tris"]), len(sc["edges"]))
                peak_resident = max(peak_resident, len(live))
                peak_bytes = max(peak_bytes, used)
                progressed = True
            # completions
            for h in list(live):
                L = live[h]
                try:
                    r = srv.poll(h, out=L.out)
                except CCError as e:
                    failed.append(dict(request=L.req, step=L.step, code=e.code))
                    srv.release(h)
                    sc = requests[L.req]
                    used -= srv.scene_bytes(len(sc["x"]), len(sc["tris"]), len(sc["edges"]))
                    del live[h]
                    progressed = True
                    if progress is not None:
                        progress(f"request {L.req} ({sc.get('name', '')}) step {L.step} failed: {e}")
                    continue
                if r is None:
                    continue
                t_done = time.perf_counter() - t0
                x_new, st = r
                lat.append(t_done - L.t_ready)
                L.iters.append(st["iters"])
                L.pairs.append(st["pair_updates"])
                iters.append(st["iters"])
                pairs.append(st["pair_updates"])
                done_steps += 1
                L.step += 1
                L.x_prev, L.x_cur = L.x_cur, x_new.clone()
                progressed = True
                if L.step == steps:
                    srv.release(h)
                    sc = requests[L.req]
                    used -= srv.scene_bytes(len(sc["x"]), len(sc["tris"]), len(sc["edges"]))
                    if keep_results:
                        results[L.req] = dict(x=L.x_cur, iters=L.iters, pairs=L.pairs)
                    del live[h]
                    continue
                xt = next_target(L.x_prev, L.x_cur, L.w, requests[L.req]["h"])
                L.t_ready = t_done
                srv.submit(h, xt)
            if not progressed:
                time.sleep(poll_sleep)
            if progress is not None and time.perf_counter() - t_report > 10.0:
                t_report = time.perf_counter()
                progress(f"{done_steps} steps done, {len(live)} resident, {len(pending)} waiting")
    finally:
        for h in list(live):
            srv.release(h)
    wall = time.perf_counter() - t0
    return dict(latency=np.asarray(lat), wall=wall, steps=done_steps, iters=np.asarray(iters),
                pairs=np.asarray(pairs), peak_resident=peak_resident, peak_bytes=peak_bytes,
                results=results, failed=failed)


def run_alone(ctx, sc, steps: int = 10, progress=None, **over):
    """The same request served by plain consecutive collide_step calls: the
    reference for results in the mix, and the per-scene throughput baseline."""
    import torch

    from . import collide_step
    prm = dict(sc.get("params", {}))
    prm.update(over)
    x = torch.as_tensor(sc["x"], dtype=torch.float64, device="cuda")
    w = torch.as_tensor(sc["w"], dtype=torch.float64, device="cuda")
    tris = torch.as_tensor(sc["tris"], dtype=torch.int32, device="cuda")
    edges = torch.as_tensor(sc["edges"], dtype=torch.int32, device="cuda")
    xt = torch.as_tensor(sc["xt"], dtype=torch.float64, device="cuda")
    prev = None
    its = []
    for k in range(steps):
        out, st = collide_step(ctx, x, xt, w, tris, edges, **prm)
        its.append(st["iters"])
        if progress is not None:
            progress(f"{sc.get('name', 'scene')} step {k}: {st['iters']} iterations")
        prev, x = x, out
        if k + 1 < steps:
            xt = next_target(prev, x, w, sc["h"])
    return x, its
