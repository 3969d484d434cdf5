"""Benchmark of the two-way continuous collision-handling step on one MI355X.

One step = one cc_collide_step call: the whole hot path of Alg. 1 (proximity
search, pair pass, constraint colouring, Gauss-Seidel sweep, forward step, path
certificate, every iteration until ||r||_inf < eps) for one scene time step,
with inputs already resident in HBM. Workload: the self-contact folded cloth,
257x257 vertices (131,072 triangles, 197,120 edges) folded into 4 layers
2^-9 m apart, x~ = x + seeded Perlin displacement of 5 layer gaps; FP64.

Prints one JSON line: steps/s (value), contact-pair updates/s, p50/p99 step
latency, the roofline of the dominant kernel (HIP events over the timed region)
and the FP64 oracle timed on the host on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FETCH_SIZE / WRITE_SIZE scale from the plain copy kernel (see profiles/)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_folded_cloth_257.json")


WORKLOADS = {
    1: "cloth over a static sphere, random velocities, ",
    2: "self-contact folded cloth, 4 layers, Perlin target, ",
    3: "8 stacked cube surfaces, rigid velocities, ",
    4: "hair strands on a sphere, wind impulse, ",
    6: "particle pile on a static ground: vertex-vertex and vertex-triangle pairs, ",
    7: "normal flow of two spheres 1 cm apart: target = outward offset of 1 cm along the "
       "vertex normals and 3 cotangent smoothing steps, built on the device each step, ",
}


def ablation(reps: int):
    """The ablations of Sec. 4.3.1, Sec. 4.3.2 and Sec. 5.1 on the workloads that
    converge (folded cloth, particle pile): Gauss-Seidel with 1, 2 and 4 sweeps,
    projected Jacobi with omega 0.5 and 1.0, and the CCD-based step-size scheme in
    place of the CCD-free forward step. One JSON line per run: iterations to the stop
    test and time per step (HIP events, `reps` calls after one untimed)."""
    import torch

    import paper_2211_04045_amd as cc
    import scenes
    torch.cuda.set_device(0)
    ctx = cc.Context(0)
    variants = [dict(backward="gs", gs_sweeps=1), dict(backward="gs", gs_sweeps=2),
                dict(backward="gs", gs_sweeps=4), dict(backward="jacobi", omega=0.5),
                dict(backward="jacobi", omega=1.0),
                # the CCD-based step-size scheme Sec. 5.1 compares the method with
                dict(backward="gs", gs_sweeps=1, ccd_step=True)]
    for cfg in (2, 6):
        sc = scenes.config(cfg)
        dev = "cuda"
        x = torch.as_tensor(sc["x"], device=dev)
        xt = torch.as_tensor(sc["xt"], device=dev)
        w = torch.as_tensor(sc["w"], device=dev)
        tris = torch.as_tensor(sc["tris"], dtype=torch.int32, device=dev)
        edges = torch.as_tensor(sc["edges"], dtype=torch.int32, device=dev)
        for v in variants:
            prm = dict(sc["params"], **v)
            out, st = cc.collide_step(ctx, x, xt, w, tris, edges, **prm)
            stream = torch.cuda.current_stream()
            ms = []
            for i in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                out, st = cc.collide_step(ctx, x, xt, w, tris, edges, **prm)
                e1.record(stream)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            print(json.dumps({"workload": sc["name"], "config": cfg, **v,
                              "iterations_per_step": st["iters"], "status": st["status"],
                              "ms_per_step": round(float(np.median(ms)), 3),
                              "row_updates_per_step": st["row_updates"],
                              "max_colors_used": st["max_colors_used"],
                              "continuous_tests_per_step": st["ccd_fail"],
                              "scaled_steps_per_step": st["n_scaled"]}), flush=True)


def latency_table(reps: int, small: bool, budget_s: float):
    """p50/p99 of the per-call time (HIP events on the calling stream) over `reps`
    calls of collide_step, after one untimed call, for every single-scene workload;
    a workload whose calls would take more than budget_s in all stops early (after
    at least 5 calls) and reports how many calls it timed."""
    import torch

    import paper_2211_04045_amd as cc
    import scenes
    torch.cuda.set_device(0)
    ctx = cc.Context(0)
    for cfg in (1, 2, 3, 4, 6):
        sc = scenes.config(cfg, small=small)
        dev = "cuda"
        x = torch.as_tensor(sc["x"], device=dev)
        xt = torch.as_tensor(sc["xt"], device=dev)
        w = torch.as_tensor(sc["w"], device=dev)
        tris = torch.as_tensor(sc["tris"], dtype=torch.int32, device=dev)
        edges = torch.as_tensor(sc["edges"], dtype=torch.int32, device=dev)
        t_first = time.perf_counter()
        out, st = cc.collide_step(ctx, x, xt, w, tris, edges, **sc["params"])
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t_first
        print(f"# config {cfg}: untimed call {t_first:.2f} s, {st['iters']} iterations",
              file=sys.stderr, flush=True)
        n = reps if t_first * reps <= budget_s else max(5, int(budget_s / max(t_first, 1e-9)))
        n = min(n, reps)
        stream = torch.cuda.current_stream()
        ev = []
        t0 = time.perf_counter()
        for i in range(n):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out, st = cc.collide_step(ctx, x, xt, w, tris, edges, **sc["params"])
            e1.record(stream)
            ev.append((e0, e1))
            if t_first > 1.0 or (i + 1) % 10 == 0:
                torch.cuda.synchronize()
                print(f"# config {cfg}: {i + 1} calls", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        # resident set of the step: state, topology, pairs and trees (bytes, estimated
        # by the library's own admission formula) against the 256 MB last-level cache
        foot = int(cc._lib.load().cc_scene_bytes(len(sc["x"]), len(sc["tris"]), len(sc["edges"])))
        print(json.dumps({
            "workload": sc["name"], "config": cfg, "verts": int(len(sc["x"])),
            "tris": int(len(sc["tris"])), "edges": int(len(sc["edges"])), "calls": n,
            "iterations_per_step": st["iters"], "status": st["status"],
            "p50_ms": round(float(np.percentile(ms, 50)), 3),
            "p99_ms": round(float(np.percentile(ms, 99)), 3),
            "steps_per_s": round(n / wall, 3),
            "pair_updates_per_step": st["pair_updates"],
            "workspace_bytes_estimate": foot, "fits_256MB_llc": foot < 256 * 2 ** 20}),
            flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--small", action="store_true")
    ap.add_argument("--mixed", action="store_true",
                    help="FP32 backward step (sets, distances, x and CCD stay FP64)")
    ap.add_argument("--jacobi", action="store_true",
                    help="projected Jacobi backward step (Sec. 4.3.2) instead of Gauss-Seidel")
    ap.add_argument("--ccd-step", action="store_true",
                    help="the CCD-based step-size scheme of Sec. 5.1 instead of the CCD-free "
                         "forward step")
    ap.add_argument("--max-iters", type=int, default=0,
                    help="override the workload's iteration cap L (0: the workload's own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=8)
    # serving stream (--config 5)
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=10)
    ap.add_argument("--rate", type=float, default=None,
                    help="Poisson arrival rate (requests/s); default: the frozen SERVE_RATE")
    ap.add_argument("--calibrate", action="store_true",
                    help="measure the closed-batch capacity and print 0.7 of it as a rate")
    ap.add_argument("--compare", type=int, default=24,
                    help="requests served both one by one and as a closed batch")
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-max-iters", type=int, default=200,
                    help="iteration cap L of the served steps (the same in every path compared)")
    # HBM traffic from rocprofv3 counters
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, run one plain copy of known size (the "
                         "scale reference for FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--digest-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of "
                         "a --copy-probe run into per-kernel HBM bytes per launch")
    ap.add_argument("--latency", type=int, default=0, metavar="R",
                    help="per-call latency (HIP events) of R calls on each single-scene "
                         "workload (configs 1, 2, 3, 4, 6): one JSON line per workload")
    ap.add_argument("--ablation", type=int, default=0, metavar="R",
                    help="backward-step ablations (sweeps, Jacobi) on the converging "
                         "workloads, R timed calls each")
    ap.add_argument("--latency-budget", type=float, default=90.0,
                    help="seconds of timed calls per workload in --latency (at least 5 calls)")
    args = ap.parse_args()
    if args.digest_pmc:
        digest_pmc(*args.digest_pmc)
        return
    if args.latency:
        latency_table(args.latency, args.small, args.latency_budget)
        return
    if args.ablation:
        ablation(args.ablation)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU: sharding the step over "
                                   "several GPUs is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.config == 5:
        serve_bench(args)
        return

    import torch

    import paper_2211_04045_amd as cc
    import scenes

    torch.cuda.set_device(0)
    sc = scenes.config(args.config, small=args.small)
    prm = dict(sc["params"])
    if args.max_iters > 0:
        prm["max_iters"] = args.max_iters
    if args.mixed:
        prm["mixed"] = True
    if args.jacobi:
        prm["backward"] = "jacobi"
    if args.ccd_step:
        prm["ccd_step"] = True
    dev = "cuda"
    x = torch.as_tensor(sc["x"], device=dev)
    w = torch.as_tensor(sc["w"], device=dev)
    tris = torch.as_tensor(sc["tris"], dtype=torch.int32, device=dev)
    edges = torch.as_tensor(sc["edges"], dtype=torch.int32, device=dev)
    ctx = cc.Context(0)
    flow = sc.get("flow")
    xt = None if flow else torch.as_tensor(sc["xt"], device=dev)

    ALL = {"time_kernels": True}

    def step(timing):
        # a normal-flow frame builds its target on the device first (part of the step)
        y = cc.normal_flow_target(ctx, x, tris, **flow) if flow else xt
        return cc.collide_step(ctx, x, y, w, tris, edges, **timing, **prm)

    def dominant(stats):
        # dominant kernel among the single-kernel families (pair pass, traversal,
        # forward, certificate)
        ms = {k: sum(s["kernels"][k]["ms"] for s in stats)
              for k in ("pair", "search", "forward", "cert")}
        return max(ms, key=ms.get)

    warm = []
    for i in range(args.warmup):
        out, st = step(ALL)
        warm.append(st)
        print(f"# warmup {i}: iters={st['iters']} status={st['status']}", file=sys.stderr,
              flush=True)
    # the timed steps carry HIP events around the dominant kernel's launches only
    # (events around every family cost host time the step would not spend)
    dom = dominant(warm) if warm else "search"
    timed = {"time_one": dom}
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    lat, stats = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out, st = step(timed)
        e1.record(stream)
        stats.append(st)
        print(f"# step {i}: iters={st['iters']} pairs={st['pair_updates']}", file=sys.stderr,
              flush=True)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat_ms = [a.elapsed_time(b) for a, b in lat]
    if args.copy_probe:
        copy_probe()

    iters = stats[-1]["iters"]
    pairs = sum(s["pair_updates"] for s in stats)
    rows = sum(s["row_updates"] for s in stats)

    def families_of(sts):
        kern = {}
        for name in sts[0]["kernels"]:
            ms = sum(s["kernels"][name]["ms"] for s in sts)
            n = sum(s["kernels"][name]["launches"] for s in sts)
            by = sum(s["kernels"][name]["bytes"] for s in sts)
            kern[name] = dict(ms=ms, launches=n, bytes=by)
        return kern

    # the dominant kernel as timed live over the timed steps
    kd = families_of(stats)[dom]
    # every family, timed in further steps after the timed region
    fam_steps = max(1, min(2, args.steps))
    fam = [step(ALL)[1] for _ in range(fam_steps)]
    torch.cuda.synchronize()
    kern = families_of(fam)
    avg_s = kd["ms"] / 1e3 / max(kd["launches"], 1)
    bytes_per_launch = kd["bytes"] / max(kd["launches"], 1)
    achieved = bytes_per_launch / avg_s / 1e9
    traffic = None
    if args.config == 2 and not args.small and os.path.exists(TRAFFIC_FILE):
        try:
            tj = json.load(open(TRAFFIC_FILE))
            kname = {"pair": "k_pair_pass", "search": "k_traverse", "forward": "k_forward",
                     "cert": "k_cert"}[dom]
            if tj.get("source_hash") == _src_hash() and kname in tj.get("kernels", {}):
                traffic = round(tj["kernels"][kname]["bytes_per_launch"])
        except Exception:
            traffic = None
    # every timed family against the same peak (the projection and certificate
    # families are the ones the spec bar names)
    families = {}
    for name, kv in kern.items():
        if kv["ms"] > 0 and kv["bytes"] > 0:
            gbs = kv["bytes"] / (kv["ms"] / 1e3) / 1e9
            families[name] = {"achieved_GBps": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 4),
                              "ms_per_step": round(kv["ms"] / fam_steps, 3),
                              "launches_per_step": round(kv["launches"] / fam_steps, 1)}
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": {"pair": "k_pair_pass", "search": "k_traverse",
                           "forward": "k_forward", "cert": "k_cert"}[dom],
                "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_bytes_per_launch": round(bytes_per_launch)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sc, prm, iters, args.cpu_sample_iters)

    value = args.steps / wall
    line = {
        "metric": "collision-handling steps/sec + contact-pair updates/sec; p50/p99 step latency",
        "value": round(value, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if args.mixed else "f64",
        "data": "synthetic",
        "config": {"workload": sc["name"] + " (" + WORKLOADS.get(args.config, "") +
                               ("FP32 backward step, FP64 sets, x and CCD" if args.mixed
                                else "FP64") +
                               (", projected Jacobi backward step" if args.jacobi else "") +
                               (", CCD-based step sizes" if args.ccd_step else "") + ")",
                   "verts": int(len(sc["x"])), "tris": int(len(sc["tris"])),
                   "edges": int(len(sc["edges"])), "iterations_per_step": iters,
                   "parallelism": "single GPU"},
        "pair_updates_per_s": round(pairs / wall, 1),
        "row_updates_per_s": round(rows / wall, 1),
        "iterations_per_s": round(iters * args.steps / wall, 2),
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "roofline": roofline,
        "kernels_ms_per_step": {k: round(v["ms"] / fam_steps, 3) for k, v in kern.items()},
        "family_rooflines": families,
        "autotune": cc.autotune_table(),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


# Poisson arrival rate of the serving stream (requests/s), frozen from one
# calibration run at 70% of the measured closed-batch capacity
# (`bench.py --config 5 --requests 6 --compare 6 --calibrate`, MI355X: the first 6
# requests, 10 steps each at L = 200, closed batch 3.99 steps/s, plain path 1.80).
SERVE_RATE = 0.2796


def serve_bench(args):
    """Serving stream: requests of mixed families and sizes (2K-150K triangles),
    Poisson arrivals, admission by HBM budget, `serve_steps` consecutive steps per
    request with the scene resident in between. Reports completed steps/s of the
    stream, p50/p99 step latency (ready -> result back), and, on the first
    `compare` requests, closed-batch served throughput against the plain
    one-scene-at-a-time path."""
    import torch

    import paper_2211_04045_amd as cc
    import scenes
    from paper_2211_04045_amd import serve

    torch.cuda.set_device(0)
    ctx = cc.Context(0)
    budget = int(args.budget_gib * (1 << 30))
    t0 = time.perf_counter()
    reqs = [scenes.serve_request(i) for i in range(args.requests)]
    print(f"# generated {len(reqs)} requests in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    k = min(args.compare, len(reqs))
    L = args.serve_max_iters
    # warm-up
    serve.run_alone(ctx, reqs[0], steps=1, max_iters=L)
    torch.cuda.synchronize()
    # plain path: one scene after another, consecutive collide_step calls
    def say(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    n_plain = 0
    for i in range(k):
        _, its = serve.run_alone(ctx, reqs[i], steps=args.serve_steps, max_iters=L,
                                 progress=say)
        n_plain += len(its)
        say(f"plain path: request {i} ({reqs[i]['name']}) iterations {its}")
    torch.cuda.synchronize()
    plain = n_plain / (time.perf_counter() - t0)
    print(f"# plain path: {plain:.2f} steps/s over {k} requests", file=sys.stderr, flush=True)
    closed = serve.run_stream(ctx, reqs[:k], np.zeros(k), steps=args.serve_steps,
                              budget_bytes=budget, progress=say, max_iters=L)
    capacity = closed["steps"] / closed["wall"]
    print(f"# closed batch: {capacity:.2f} steps/s", file=sys.stderr, flush=True)
    if args.calibrate:
        print(json.dumps({"calibrated_rate": round(0.7 * capacity / args.serve_steps, 4),
                          "capacity_steps_per_s": round(capacity, 3)}))
        return
    rate = args.rate or SERVE_RATE or 0.7 * capacity / args.serve_steps
    arr = scenes.poisson_arrivals(len(reqs), rate)
    res = serve.run_stream(ctx, reqs, arr, steps=args.serve_steps, budget_bytes=budget,
                           progress=say, max_iters=L)
    lat = res["latency"] * 1e3
    value = res["steps"] / res["wall"]
    fam = np.bincount([r["family"] for r in reqs], minlength=4)[1:]
    line = {
        "metric": "collision-handling steps/sec + contact-pair updates/sec; p50/p99 step latency",
        "value": round(value, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": int(res["steps"]),
        "warmup": 1,
        "ms_per_step": round(1e3 * res["wall"] / res["steps"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serving stream: {len(reqs)} requests x {args.serve_steps} "
                               "steps, families cloth-over-sphere / folded cloth / stacked "
                               "cubes, 2K-150K triangles log-uniform, Poisson arrivals",
                   "requests_per_family": [int(v) for v in fam],
                   "arrival_rate_per_s": round(rate, 4),
                   "max_iters": L,
                   "budget_gib": args.budget_gib,
                   "parallelism": "single GPU"},
        "pair_updates_per_s": round(float(res["pairs"].sum()) / res["wall"], 1),
        "iterations_per_s": round(float(res["iters"].sum()) / res["wall"], 2),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "peak_resident_scenes": res["peak_resident"],
        "peak_resident_gib": round(res["peak_bytes"] / (1 << 30), 3),
        "failed_steps": res["failed"],
        "closed_batch_steps_per_s": round(capacity, 3),
        "plain_path_steps_per_s": round(plain, 3),
        "served_over_plain": round(capacity / plain, 3),
        "compare_requests": k,
    }
    print(json.dumps(line))


COPY_PROBE_BYTES = 1 << 29  # bytes read (and written) by the copy probe


def copy_probe():
    """One plain elementwise copy, COPY_PROBE_BYTES read and written once."""
    import torch
    a = torch.rand(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()


TRAFFIC_KERNELS = ("k_pair_pass", "k_traverse", "k_stripe_gather", "k_forward", "k_cert", "k_gs_contact")


def digest_pmc(fetch_csv, write_csv):
    """Per-kernel HBM bytes per launch from two counter runs of the same command.

    FETCH_SIZE and WRITE_SIZE are read per dispatch (KiB) and summed over the
    counter instances of each dispatch; each is divided by what the same counter
    reads for the copy probe per byte it must move, so the result is in bytes of
    the copy kernel's own accounting."""
    import csv
    from collections import defaultdict

    def per_dispatch(path, counter):
        vals = defaultdict(float)
        names = {}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                d = row["Dispatch_Id"]
                vals[d] += float(row["Counter_Value"])
                names[d] = row["Kernel_Name"]
        return vals, names

    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        vals, names = per_dispatch(path, counter)
        copy = [vals[d] for d in vals if "elementwise" in names[d] or "mul" in names[d].lower()]
        copy = [v for v in copy if v * 1024 > COPY_PROBE_BYTES / 2]
        if not copy:
            raise SystemExit(f"{path}: no copy-probe dispatch found")
        scale = max(copy) * 1024 / COPY_PROBE_BYTES
        for k in TRAFFIC_KERNELS:
            ds = [d for d in vals if ("::" + k + "(") in names[d] or ("::" + k + "<") in names[d]]
            if not ds:
                continue
            # a template kernel: the instance launched most (the autotuner's choice;
            # the other launch shapes run once each on the first search)
            inst = {}
            for d in ds:
                inst.setdefault(names[d].split("(")[0], []).append(d)
            name, ds = max(inst.items(), key=lambda kv: len(kv[1]))
            e = out.setdefault(k, {"launches": len(ds), "instance": name})
            e[counter.lower() + "_bytes_per_launch"] = sum(vals[d] for d in ds) * 1024 / len(ds) / scale
            e[counter.lower() + "_scale"] = scale
    for k, e in out.items():
        e["bytes_per_launch"] = e.get("fetch_size_bytes_per_launch", 0.0) + \
            e.get("write_size_bytes_per_launch", 0.0)
    res = {"source_hash": _src_hash(), "kernels": out,
           "note": "rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, of bench.py --copy-probe; "
                   "scaled by the copy probe's reading per byte moved"}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def _src_hash():
    import hashlib
    h = hashlib.sha1()
    for f in ("step.hip", "geom.hpp", "lbvh.hip", "internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2211_04045_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def cpu_baseline(sc, prm, iters_per_step, sample_iters):
    """The FP64 oracle, single-threaded on the host, over the first `sample_iters`
    iterations of the same step, scaled by the step's iteration count."""
    import oracle
    t_flow = 0.0
    xt = sc.get("xt")
    if xt is None:  # a normal-flow frame: the oracle builds the target too
        t_flow = time.perf_counter()
        xt = oracle.normal_flow(sc["x"], sc["tris"], **sc["flow"])
        t_flow = time.perf_counter() - t_flow
    s = oracle.Scene(sc["w"], sc["tris"], sc["edges"], **prm)
    s.begin(sc["x"], xt)
    t0 = time.perf_counter()
    done = 0
    pairs = 0
    for _ in range(min(sample_iters, iters_per_step)):
        stop, it = s.iterate()
        done += 1
        pairs += it["n_p"]
        if stop:
            break
    dt = time.perf_counter() - t0
    per_iter = dt / done
    return {"value": round(1.0 / (t_flow + per_iter * iters_per_step), 6), "unit": "steps/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"first {done} of {iters_per_step} iterations of one step "
                      f"({dt:.1f} s, {pairs} pair updates), scaled to the full step",
            "pair_updates_per_s": round(pair_rate(pairs, dt), 1),
            "host_nproc": os.cpu_count(),
            "host_cpu": host_cpu_model()}


def pair_rate(pairs, dt):
    return pairs / dt if dt > 0 else 0.0


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
