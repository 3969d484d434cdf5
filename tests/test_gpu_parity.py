"""Parity of the HIP path with the FP64 oracle, through the C ABI.

The bar: contact sets (P', A and the colouring) bit-identical; positions within
1e-6 of the scene's bounding-box diagonal (the design is order independent, so
the observed difference is expected to be exactly zero and is asserted too).
Final states are checked for intersections in exact arithmetic.
"""
import numpy as np
import pytest

import exact
import oracle
import scenes

pytestmark = pytest.mark.gpu

TRACE_KEYS = ["searched", "n_colors", "n_p", "n_pf", "n_a", "ccd_fail", "ccd_hits", "n_back",
              "n_scaled", "d_before", "d_after", "move_max", "r_inf", "fp_pf", "fp_a", "fp_col"]
SET_KEYS = ("searched", "n_p", "n_pf", "n_a", "n_colors", "fp_pf", "fp_a", "fp_col")


@pytest.fixture(scope="module")
def cc():
    import torch  # noqa: F401
    import paper_2211_04045_amd as cc
    return cc


@pytest.fixture(scope="module")
def ctx(cc):
    return cc.Context(0)


def _u64(t):
    return np.sort(t.cpu().numpy().view(np.uint64))


def _diag(x):
    return float(np.linalg.norm(x.max(axis=0) - x.min(axis=0)))


def _lockstep(cc, ctx, sc, max_iters, check_state_every=1, **over):
    p = dict(sc.get("params", {}))
    p.update(over)
    p["max_iters"] = max_iters
    ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"], **p)
    ref.begin(sc["x"], sc["xt"])
    gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"], trace=True, **p)
    gpu.begin(sc["x"], sc["xt"])
    tol = 1e-6 * _diag(sc["x"])
    n = 0
    trace = []
    for l in range(max_iters):
        s_ref, it_ref = ref.iterate()
        s_gpu, it_gpu = gpu.iterate()
        n += 1
        trace.append(it_gpu)
        for k in TRACE_KEYS:
            assert it_gpu[k] == it_ref[k], (sc["name"], l, k, it_gpu[k], it_ref[k])
        if l % check_state_every == 0 or s_ref:
            xr, yr, rr, Dr = ref.state()
            xg, yg, rg, Dg = (t.cpu().numpy() if hasattr(t, "cpu") else t for t in gpu.state())
            assert np.abs(xg - xr).max() <= tol and np.abs(yg - yr).max() <= tol
            assert np.array_equal(xg, xr) and np.array_equal(yg, yr), (sc["name"], l)
            assert np.array_equal(rg, rr) and Dg == Dr
        assert s_gpu == s_ref
        if s_ref:
            break
    gpu.trace = trace
    return n, ref, gpu


def _replay_lockstep(cc, ctx, sc, max_iters, **over):
    """Every iteration starts the oracle from the GPU's state (x, y, r, D, P'): the
    sets P', A and the colouring are decided in FP64 at the same x and must be
    identical; x and y after the iteration must agree within 1e-6 of the
    bounding-box diagonal. For paths whose arithmetic differs from the oracle's by
    rounding only. Returns the iterations run and the worst difference."""
    p = dict(sc.get("params", {}))
    p.update(over)
    p["max_iters"] = max_iters
    ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"], **p)
    gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"], trace=True, **p)
    gpu.begin(sc["x"], sc["xt"])
    ref.begin(sc["x"], sc["xt"])
    tol = 1e-6 * _diag(sc["x"])
    worst = 0.0
    n = 0
    for l in range(max_iters):
        xg, yg, rg, Dg = (t.cpu().numpy() if hasattr(t, "cpu") else t for t in gpu.state())
        Pg = gpu.P().cpu().numpy().view(np.uint64)
        ref.set_state(xg, yg, rg, Dg, Pg)
        s_ref, it_ref = ref.iterate()
        s_gpu, it_gpu = gpu.iterate()
        n += 1
        for k in SET_KEYS:
            assert it_gpu[k] == it_ref[k], (sc["name"], l, k, it_gpu[k], it_ref[k])
        assert it_gpu["ccd_hits"] == 0 and it_gpu["n_back"] == 0
        xr, yr, _, _ = ref.state()
        xg, yg, _, _ = (t.cpu().numpy() if hasattr(t, "cpu") else t for t in gpu.state())
        err = max(np.abs(xg - xr).max(), np.abs(yg - yr).max())
        worst = max(worst, err)
        assert err <= tol, (sc["name"], l, err, tol)
        if s_ref or s_gpu:
            break
    return n, worst


def test_library_loads_on_gpu(cc, ctx):
    assert ctx.h


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 6])
def test_search_set_matches_oracle_small(cc, ctx, cfg):
    sc = scenes.config(cfg, small=True)
    ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"])
    ref.begin(sc["x"], sc["xt"])
    gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"])
    gpu.begin(sc["x"], sc["xt"])
    for dmax in (4e-3, 1e-2):
        want = np.sort(ref.search(sc["x"], dmax))
        got = _u64(gpu.search(sc["x"], dmax))
        assert np.array_equal(got, want), (cfg, dmax, len(got), len(want))


def test_search_set_matches_oracle_full_folded_cloth(cc, ctx):
    sc = scenes.config(2)
    ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"])
    ref.begin(sc["x"], sc["xt"])
    gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"])
    gpu.begin(sc["x"], sc["xt"])
    want = np.sort(ref.search(sc["x"], 4e-3))
    got = _u64(gpu.search(sc["x"], 4e-3))
    assert len(want) > 1_000_000
    assert np.array_equal(got, want)


@pytest.mark.parametrize("cfg", [2, 3, 4, 1, 6])
def test_end_to_end_lockstep_small(cc, ctx, cfg):
    """Each small workload in lockstep to its end (the stop test, or L = 2048 for the
    crumpling cloth over the sphere): every iteration bit-identical; no pair of P' is
    left uncertified (the lemma of Sec. 5 holds for the rounded moves) and nothing is
    sent back; the final state is free in exact arithmetic."""
    sc = scenes.config(cfg, small=True)
    n, ref, gpu = _lockstep(cc, ctx, sc, sc["params"]["max_iters"])
    assert all(t["ccd_fail"] == 0 and t["ccd_hits"] == 0 and t["n_back"] == 0
               for t in gpu.trace)
    x = gpu.state()[0].cpu().numpy()
    assert _intersection_free(x, sc["tris"], sc["edges"])
    print(f"config {cfg} small: {n} iterations, r_inf {gpu.trace[-1]['r_inf']:.3g}")


def test_unguarded_forward_step_lockstep(cc, ctx):
    """CC_UNGUARDED (the forward step exactly as Eq. eq:forward2): on the crumpling
    cloth some rounded moves break the lemma; the certificate's passes, the pairs it
    does not clear and the vertices it sends back are bit-identical to the oracle's,
    and the output is still free in exact arithmetic."""
    sc = scenes.config(1, small=True)
    n, ref, gpu = _lockstep(cc, ctx, sc, 600, unguarded=True)
    assert sum(t["n_back"] for t in gpu.trace) > 0
    assert _intersection_free(gpu.state()[0].cpu().numpy(), sc["tris"], sc["edges"])


@pytest.mark.parametrize("group", [8, 16, 32, 108, 116, 132])
def test_every_traversal_group_size_finds_the_oracle_set(cc, ctx, group):
    """The traversal's launch shapes the autotuner chooses between (lanes per group,
    one or two nodes per step): each, forced, finds exactly the oracle's pair set on
    the full folded cloth and on the small workloads; the tuning table records what
    was measured."""
    lib = cc._lib.load()
    assert lib.cc_autotune_force(0, group) == 0
    try:
        for sc in [scenes.config(2)] + [scenes.config(c, small=True) for c in (1, 3, 4, 6)]:
            ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"])
            ref.begin(sc["x"], sc["xt"])
            gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"])
            gpu.begin(sc["x"], sc["xt"])
            want = np.sort(ref.search(sc["x"], 4e-3))
            got = _u64(gpu.search(sc["x"], 4e-3))
            assert np.array_equal(got, want), (group, sc["name"])
    finally:
        lib.cc_autotune_force(0, 0)
    table = cc.autotune_table()
    assert all(e["choice"] in (8, 16, 32, 108, 116, 132) and min(e["ms"]) > 0 for e in table)


@pytest.mark.parametrize("cfg", [2, 3, 4, 6])
def test_ccd_step_lockstep_small(cc, ctx, cfg):
    """The CCD-based step-size scheme (Sec. 5.1's comparison; CC_CCD_STEP) in lockstep
    to its end: every iteration bit-identical (the passes, the contacts, the scaled
    steps); the final state free in exact arithmetic."""
    sc = scenes.config(cfg, small=True)
    n, ref, gpu = _lockstep(cc, ctx, sc, sc["params"]["max_iters"], ccd_step=True)
    assert all(t["n_back"] == 0 for t in gpu.trace)
    assert _intersection_free(gpu.state()[0].cpu().numpy(), sc["tris"], sc["edges"])
    print(f"ccd step config {cfg} small: {n} iterations, "
          f"{sum(t['n_scaled'] for t in gpu.trace)} scaled steps")


def test_sets_and_colours_explicit(cc, ctx):
    sc = scenes.config(2, small=True)
    n, ref, gpu = _lockstep(cc, ctx, sc, 3)
    assert np.array_equal(_u64(gpu.P()), np.sort(ref.P()))
    kg, cg = gpu.A()
    kr, cr = ref.A()
    og = np.argsort(kg.cpu().numpy().view(np.uint64))
    orr = np.argsort(kr)
    assert np.array_equal(kg.cpu().numpy().view(np.uint64)[og], kr[orr])
    assert np.array_equal(cg.cpu().numpy()[og], cr[orr])
    assert np.array_equal(gpu.Di().cpu().numpy(), ref.Di())


def test_collide_step_matches_oracle_run(cc, ctx):
    sc = scenes.config(2, small=True)
    want, n, _ = oracle.collide_step(sc)
    got, st = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                              **sc["params"])
    assert st["iters"] == n and st["status"] == 0
    assert np.array_equal(got.cpu().numpy(), want)
    # a second call reuses the cached workspace and gives the same answer
    got2, _ = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                              **sc["params"])
    assert np.array_equal(got2.cpu().numpy(), want)


def test_edge_colouring_reuse_follows_its_inputs(cc, ctx):
    # Steps of one scene keep their edge-row colouring while the edges, the rows,
    # the free vertices, the seed and the palette repeat; each change below must
    # colour again and still give the oracle's step.
    base = scenes.config(2, small=True)
    pinned_w = base["w"].copy()
    pinned_w[0] = 0.0
    swapped = base["edges"].copy()
    swapped[5] = swapped[5][::-1]
    cases = [("first", {}, {}), ("repeat", {}, {}), ("pinned vertex", {"w": pinned_w}, {}),
             ("back", {}, {}), ("seed", {}, {"seed": 12345}), ("swapped edge", {"edges": swapped}, {}),
             ("palette", {}, {"max_colors": 512}), ("repeat again", {}, {})]
    for name, sc_over, p_over in cases:
        sc = dict(base, **sc_over)
        prm = dict(sc["params"], **p_over)
        want, n, _ = oracle.collide_step(sc, **p_over)
        got, st = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"], **prm)
        assert st["iters"] == n and st["status"] == 0, name
        assert np.array_equal(got.cpu().numpy(), want), name


def _full_step_sampled(cc, ctx, sc, samples, **over):
    """A full-size workload in the benchmark's launch configuration: the GPU runs the
    whole step (to the stop test or L); at the sampled iterations and at the last one
    the oracle replays that iteration from the GPU's state (x, y, r, D, P'), and the
    sets, D_i and the new state must agree exactly. The GPU's state before each
    iteration is kept on the device so that the last iteration can be replayed once
    it is known. Returns the solver, the iterations run and the trace."""
    p = dict(sc["params"])
    p.update(over)
    gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"], trace=True, **p)
    gpu.begin(sc["x"], sc["xt"])
    ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"], **p)
    ref.begin(sc["x"], sc["xt"])

    def replay(l, before, it_gpu, after):
        x, y, r, D, P = before
        ref.set_state(x.cpu().numpy(), y.cpu().numpy(), r.cpu().numpy(), D,
                      P.cpu().numpy().view(np.uint64))
        _, it_ref = ref.iterate()
        for k in TRACE_KEYS:
            assert it_gpu[k] == it_ref[k], (sc["name"], l, k, it_gpu[k], it_ref[k])
        xr, yr, rr, Dr = ref.state()
        xg, yg, rg, Dg = after
        assert np.array_equal(xg.cpu().numpy(), xr), (sc["name"], l)
        assert np.array_equal(yg.cpu().numpy(), yr), (sc["name"], l)
        assert np.array_equal(rg.cpu().numpy(), rr) and Dg == Dr
        assert np.array_equal(gpu.Di().cpu().numpy(), ref.Di())

    trace = []
    replayed = set()
    for l in range(p["max_iters"]):
        x, y, r, D = gpu.state()
        before = (x, y, r, D, gpu.P().clone())
        stop, it_gpu = gpu.iterate()
        trace.append(it_gpu)
        last = stop or l == p["max_iters"] - 1
        if l in samples or last:
            replay(l, before, it_gpu, gpu.state())
            replayed.add(l)
        if stop:
            break
    print(f"{sc['name']}: {len(trace)} iterations, replayed {sorted(replayed)}, "
          f"r_inf {trace[-1]['r_inf']:.3g}")
    return gpu, len(trace), trace


def test_full_size_folded_cloth_step(cc, ctx):
    """The benchmark workload (folded cloth 257 x 257) to its stop test, sampled
    iterations and the last replayed by the oracle; no uncertified pair; the final
    state is free in exact arithmetic."""
    sc = scenes.config(2)
    gpu, n, trace = _full_step_sampled(cc, ctx, sc, {0, 1, 5, 12})
    assert trace[-1]["r_inf"] < sc["params"].get("eps", 1e-4)
    assert all(t["ccd_fail"] == 0 and t["n_back"] == 0 for t in trace)
    assert _intersection_free(gpu.state()[0].cpu().numpy(), sc["tris"], sc["edges"])


def test_full_size_cloth_over_sphere_whole_step_matches_oracle(cc, ctx):
    """Cloth over the sphere, full size (33 x 33 grid; the crumpling target runs to
    L = 2048): the whole step bit-identical to the oracle's run, no uncertified pair,
    and the final state free in exact arithmetic."""
    sc = scenes.config(1)
    want, n, trace = oracle.collide_step(sc)
    got, st = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                              **sc["params"])
    assert st["iters"] == n
    assert np.array_equal(got.cpu().numpy(), want)
    assert st["ccd_fail"] == 0 and st["n_back"] == 0
    assert all(t["ccd_fail"] == 0 for t in trace)
    assert _intersection_free(want, sc["tris"], sc["edges"])


@pytest.mark.parametrize("cfg,samples", [(3, {0, 1, 150, 1000}), (4, {0, 1, 40})])
def test_full_size_cubes_and_hair_steps(cc, ctx, cfg, samples):
    """Stacked cubes (8 x 16^3 cells) and hair (10,000 strands), full size, to the stop
    test or L: sampled iterations and the last replayed by the oracle, no uncertified
    pair, final state free in exact arithmetic."""
    sc = scenes.config(cfg)
    gpu, n, trace = _full_step_sampled(cc, ctx, sc, samples)
    assert all(t["ccd_fail"] == 0 and t["n_back"] == 0 for t in trace)
    assert _intersection_free(gpu.state()[0].cpu().numpy(), sc["tris"], sc["edges"])


# ------------------------------------------------------------------ edge cases

def test_max_iters_one_is_safe_and_reports_maxiter(cc, ctx):
    sc = scenes.config(2, small=True)
    got, st = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                              max_iters=1)
    want, n, _ = oracle.collide_step(sc, max_iters=1)
    assert st["iters"] == 1 and st["status"] == 1
    assert np.array_equal(got.cpu().numpy(), want)


def test_hair_without_triangles_and_single_primitives(cc, ctx):
    # polylines only
    sc = scenes.config(4, small=True)
    _lockstep(cc, ctx, sc, 200)
    # one triangle and one free vertex (trees of a single leaf)
    x = np.array([[0.2, 0.2, 0.005], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    xt = x.copy()
    xt[0, 2] = -0.005
    one = dict(name="one", x=x, xt=xt, w=np.array([1.0, 0, 0, 0]),
               tris=np.array([[1, 2, 3]], np.int32), edges=np.array([[1, 2]], np.int32),
               params={})
    n, ref, gpu = _lockstep(cc, ctx, one, 50)
    xg = gpu.state()[0].cpu().numpy()
    assert abs(xg[0, 2] - 1e-3) < 1e-15


def test_static_scene_returns_input(cc, ctx):
    # no pair within delta (cube surfaces 5 mm apart, 2.5 cm cells): x~ = x gives x back
    sc = scenes.config(3, small=True)
    got, st = cc.collide_step(ctx, sc["x"], sc["x"], sc["w"], sc["tris"], sc["edges"])
    assert st["iters"] == 1
    assert np.array_equal(got.cpu().numpy(), sc["x"])
    # folded cloth: the fold strips hold pairs below delta, which the step separates;
    # the result is the oracle's
    sc = scenes.config(2, small=True)
    got, st = cc.collide_step(ctx, sc["x"], sc["x"], sc["w"], sc["tris"], sc["edges"])
    want, n, _ = oracle.collide_step(dict(sc, xt=sc["x"]))
    assert st["iters"] == n
    assert np.array_equal(got.cpu().numpy(), want)


def test_errors_are_reported(cc, ctx):
    sc = scenes.config(2, small=True)
    bad = sc["x"].copy()
    bad[3, 1] = np.nan
    with pytest.raises(cc.CCError) as e:
        cc.collide_step(ctx, bad, sc["xt"], sc["w"], sc["tris"], sc["edges"])
    assert e.value.code == -1
    t = sc["tris"].copy()
    t[5, 0] = len(sc["x"])
    with pytest.raises(cc.CCError):
        cc.Solver(ctx, sc["w"], t, sc["edges"])
    with pytest.raises(cc.CCError):
        cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"], gamma=1.0)
    with pytest.raises(cc.CCError):
        cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"], d_min=0.5e-3)
    # palette too small for the active graph -> colour error, not a wrong answer
    with pytest.raises(cc.CCError) as e:
        cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"], max_colors=2)
    assert e.value.code == -5


def test_batched_equals_solo_and_oracle(cc, ctx):
    """Scenes of uneven sizes in one batched call: every result is bit-identical to
    the scene run alone and to the oracle."""
    batch = [scenes.config(2, small=True), scenes.config(3, small=True),
             scenes.config(4, small=True), scenes.config(2, small=True),
             scenes.folded_cloth(layer_rows=4)]
    for sc in batch:
        sc["params"] = dict(sc["params"], max_iters=300)
    res = cc.collide_step_batched(ctx, batch, max_iters=300)
    assert len(res) == len(batch)
    for sc, (x_b, st_b) in zip(batch, res):
        x_s, st_s = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                                    max_iters=300)
        want, n, _ = oracle.collide_step(sc, max_iters=300)
        assert np.array_equal(x_b.cpu().numpy(), x_s.cpu().numpy())
        assert np.array_equal(x_b.cpu().numpy(), want)
        assert st_b["iters"] == st_s["iters"] == n
    # a second call reuses the slots
    res2 = cc.collide_step_batched(ctx, batch, max_iters=300)
    for (a, _), (b, _) in zip(res, res2):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def _next_target(x_prev, x_new, h, w):
    """x~_{n+1} = x_{n+1} + h v + h^2 g with v = (x_{n+1} - x_n)/h; pinned vertices stay."""
    g = np.array([0.0, 0.0, -9.81])
    v = (x_new - x_prev) / h
    xt = x_new + h * v + h * h * g
    xt[w == 0] = x_new[w == 0]
    return xt


def test_served_scenes_in_a_mix_equal_the_same_steps_alone(cc, ctx):
    import time
    srv = cc.Server(ctx, budget_bytes=0)
    mix = [scenes.config(2, small=True), scenes.config(3, small=True),
           scenes.config(4, small=True), scenes.folded_cloth(layer_rows=4)]
    hs = [srv.admit(sc["x"], sc["w"], sc["tris"], sc["edges"], max_iters=400) for sc in mix]
    prev = [sc["x"].copy() for sc in mix]
    cur = [sc["x"].copy() for sc in mix]
    xt = [sc["xt"].copy() for sc in mix]
    for step in range(3):
        for h, t in zip(hs, xt):
            srv.submit(h, t)
        done = [None] * len(mix)
        t0 = time.time()
        while any(d is None for d in done):
            for i, h in enumerate(hs):
                if done[i] is None:
                    done[i] = srv.poll(h)
            assert time.time() - t0 < 120
        for i, sc in enumerate(mix):
            got = done[i][0].cpu().numpy()
            alone, _ = cc.collide_step(ctx, cur[i], xt[i], sc["w"], sc["tris"], sc["edges"],
                                       max_iters=400)
            assert np.array_equal(got, alone.cpu().numpy()), (i, step)
            prev[i], cur[i] = cur[i], got
            xt[i] = _next_target(prev[i], cur[i], 1.0 / 30.0, sc["w"])
    for h in hs:
        srv.release(h)


def test_admission_respects_the_budget(cc, ctx):
    srv = cc.Server(ctx)
    sc = scenes.config(2, small=True)
    need = srv.scene_bytes(len(sc["x"]), len(sc["tris"]), len(sc["edges"]))
    srv2 = cc.Server(ctx, budget_bytes=int(need * 1.5))
    h1 = srv2.admit(sc["x"], sc["w"], sc["tris"], sc["edges"])
    assert h1 is not None
    assert srv2.admit(sc["x"], sc["w"], sc["tris"], sc["edges"]) is None  # over budget
    srv2.release(h1)
    h2 = srv2.admit(sc["x"], sc["w"], sc["tris"], sc["edges"])
    assert h2 is not None
    srv2.release(h2)
    cc.Server(ctx, budget_bytes=0)  # back to unlimited for later tests


def test_stream_serving_results_equal_alone(cc, ctx):
    """Requests of mixed families and sizes, staggered arrivals and a budget that
    holds only some of them at once: every request's final state after 3 steps
    equals the same 3 steps run alone with collide_step."""
    import torch
    from paper_2211_04045_amd import serve
    reqs = [scenes.serve_request(i, t_min=300.0, t_max=3000.0) for i in range(6)]
    need = [cc.Server(ctx).scene_bytes(len(r["x"]), len(r["tris"]), len(r["edges"])) for r in reqs]
    budget = int(sum(sorted(need)[-3:]))  # at most about three resident at once
    arrivals = np.array([0.0, 0.0, 0.01, 0.02, 0.02, 0.05])
    res = serve.run_stream(ctx, reqs, arrivals, steps=3, budget_bytes=budget, keep_results=True,
                           max_iters=300)
    cc.Server(ctx, 0)
    assert res["steps"] == 18 and len(res["latency"]) == 18
    assert res["peak_bytes"] <= budget
    for i, r in enumerate(reqs):
        x_alone, its = serve.run_alone(ctx, r, steps=3, max_iters=300)
        assert its == res["results"][i]["iters"], (i, r["name"])
        assert torch.equal(x_alone, res["results"][i]["x"]), (i, r["name"])


def _intersection_free(x, tris, edges):
    """Exact check of a final state: no edge touches a triangle it shares no vertex
    with, and no two polyline segments touch (binary64 orientations with error
    bounds, exact rational tests where those leave the sign open)."""
    et, ee = exact.touching_pairs(np.asarray(x), np.asarray(tris), np.asarray(edges))
    return not et and not ee


@pytest.mark.parametrize("cfg,iters", [(2, 60), (3, 120), (4, 60), (1, 60), (6, 60)])
def test_mixed_precision_lockstep(cc, ctx, cfg, iters):
    """Mixed precision (FP32 backward step), the oracle replaying each iteration from
    the GPU's state: identical sets, x and y within 1e-6 of the bbox diagonal."""
    sc = scenes.config(cfg, small=True)
    n, worst = _replay_lockstep(cc, ctx, sc, iters, mixed=True)
    print(f"mixed lockstep config {cfg}: worst |x|,|y| difference {worst:.3e} m")


@pytest.mark.parametrize("cfg", [2, 3])
def test_mixed_precision_end_to_end(cc, ctx, cfg):
    """A whole step in mixed precision ends intersection-free (exact test) with no
    continuous-test contact; its distance from the FP64 oracle's result is printed."""
    sc = scenes.config(cfg, small=True)
    p = dict(sc.get("params", {}))
    p["max_iters"] = 400
    out, st = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"], mixed=True, **p)
    x_mixed = out.cpu().numpy()
    assert st["ccd_hits"] == 0
    assert _intersection_free(x_mixed, sc["tris"], sc["edges"])
    x_ref = oracle.collide_step(sc, **p)[0]
    print(f"mixed end-to-end config {cfg}: iterations {st['iters']}, max |x - x_fp64| "
          f"{np.abs(x_mixed - x_ref).max():.3e} m, bbox diagonal {_diag(sc['x']):.3e} m")


@pytest.mark.parametrize("cfg,iters", [(2, 200), (3, 300), (4, 150), (1, 100), (6, 200)])
def test_jacobi_lockstep(cc, ctx, cfg, iters):
    """Projected Jacobi backward step (Sec. 4.3.2), the oracle replaying each iteration
    from the GPU's state: identical sets; the library sums each vertex's updates on a
    2^-56 m integer grid (order independent), the oracle in binary64 in row order, so
    x and y agree within the stated tolerance, not bit for bit."""
    sc = scenes.config(cfg, small=True)
    n, worst = _replay_lockstep(cc, ctx, sc, iters, backward="jacobi")
    print(f"jacobi lockstep config {cfg}: {n} iterations, worst difference {worst:.3e} m")


def test_jacobi_batched_equals_solo(cc, ctx):
    mix = [scenes.config(2, small=True), scenes.config(3, small=True), scenes.config(4, small=True)]
    res = cc.collide_step_batched(ctx, mix, backward="jacobi", max_iters=300)
    for sc, (out, st) in zip(mix, res):
        alone, st1 = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                                     backward="jacobi", max_iters=300)
        assert torch_equal(out, alone) and st["iters"] == st1["iters"]


def torch_equal(a, b):
    import torch
    return torch.equal(a, b)


def _free_gpu(cc, ctx, x, xt, w, tris, edges):
    """The library's input check at begin: True when x is accepted."""
    s = cc.Solver(ctx, w, tris, edges, validate=True)
    try:
        s.begin(x, xt)
        return True
    except cc.CCError as e:
        assert e.code == -9, e
        return False
    finally:
        s.close()


def _free_oracle(x, xt, w, tris, edges):
    s = oracle.Scene(w, tris, edges)
    s.begin(x, xt)
    return s.validate(x, 1e-9) == 0


def _check_cases():
    out = []
    xa, ta, ea = scenes.grid_cloth(4, 4, 5e-3)
    xb = xa.copy()
    xb[:, :2] += (1.3e-3, 0.9e-3)
    xb[:, 2] += 3e-3
    x = np.vstack([xa, xb])
    tris = np.vstack([ta, ta + len(xa)]).astype(np.int32)
    edges = np.vstack([ea, ea + len(xa)]).astype(np.int32)
    w = np.ones(len(x))
    out.append(("patches apart", x, x, w, tris, edges))
    y = x.copy()
    n = len(xa)
    y[n:, 2] += (y[n:, 1] - y[n:, 1].mean()) * 1.5 - 1e-3
    out.append(("patch tilted through", y, y, w, tris, edges))
    # the same crossing with every vertex static: all-static pairs are skipped
    out.append(("static crossing", y, y, np.zeros(len(y)), tris, edges))
    tri = np.array([[0, 1, 2]], np.int32)
    ned = np.array([[0, 1], [1, 2], [0, 2], [3, 4]], np.int32)
    xn = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0.25, 0.25, -0.5], [0.25, 0.25, 0.5]])
    out.append(("needle through", xn, xn, np.ones(5), tri, ned))
    xm = xn.copy()
    xm[4, 2] = -0.1
    out.append(("needle below", xm, xm, np.ones(5), tri, ned))
    # a vertex hovering 0.5 nm / 2 nm above the triangle
    for h, name in ((5e-10, "vertex at 0.5 nm"), (2e-9, "vertex at 2 nm")):
        xv = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.3, h]])
        out.append((name, xv, xv, np.ones(4), tri, np.array([[0, 1], [1, 2], [0, 2]], np.int32)))
    # soups of small random triangles: some seeds free, some not
    for seed in range(24):
        rng = np.random.default_rng(700 + seed)
        nt = 40
        c = rng.uniform(0, 1, size=(nt, 1, 3))
        xs = (c + rng.normal(size=(nt, 3, 3)) * 0.035).reshape(-1, 3)
        ts = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
        es = scenes.edges_from_tris(ts).astype(np.int32)
        out.append((f"soup {seed}", xs, xs, np.ones(len(xs)), ts, es))
    for cfg in (1, 2, 3, 4):
        sc = scenes.config(cfg, small=True)
        out.append((f"config {cfg}", sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"]))
    return out


def test_input_check_agrees_with_oracle(cc, ctx):
    """CC_VALIDATE_INPUT against the oracle's check on free, crossing, touching,
    static and random-soup inputs: the same verdict on every case."""
    verdicts = {}
    for name, x, xt, w, tris, edges in _check_cases():
        want = _free_oracle(x, xt, w, tris, edges)
        got = _free_gpu(cc, ctx, x, xt, w, tris, edges)
        assert got == want, name
        verdicts[name] = got
    assert verdicts["patches apart"] and not verdicts["patch tilted through"]
    assert verdicts["static crossing"]
    assert not verdicts["needle through"] and verdicts["needle below"]
    assert not verdicts["vertex at 0.5 nm"] and verdicts["vertex at 2 nm"]
    soups = [v for k, v in verdicts.items() if k.startswith("soup")]
    assert any(soups) and not all(soups)
    assert all(verdicts[f"config {c}"] for c in (1, 2, 3, 4))


def test_input_check_in_a_batch_rejects_only_the_bad_scene(cc, ctx):
    """In one multi-scene call a crossing scene fails with CC_ENOTFREE; the
    others' results equal their solo runs."""
    good = [scenes.config(2, small=True), scenes.config(3, small=True)]
    (_, y, _, w, tris, edges) = _check_cases()[1]
    bad = dict(x=y, xt=y, w=w, tris=tris, edges=edges, params={})
    with pytest.raises(cc.CCError) as e:
        cc.collide_step_batched(ctx, [good[0], bad, good[1]], validate=True)
    assert e.value.code == -9
    res = cc.collide_step_batched(ctx, good, validate=True)
    for sc, (xb, _) in zip(good, res):
        xs, _ = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"])
        assert np.array_equal(xb.cpu().numpy(), xs.cpu().numpy())


# --------------------------------------------------- vertex-vertex pairs (sand)

def test_search_set_matches_oracle_full_sand_pile(cc, ctx):
    """The full particle pile (30,720 particles on a static ground): every
    vertex-vertex and vertex-triangle pair below D_max, identical to the oracle's."""
    sc = scenes.config(6)
    ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"])
    ref.begin(sc["x"], sc["xt"])
    gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"])
    gpu.begin(sc["x"], sc["xt"])
    want = np.sort(ref.search(sc["x"], 4e-3))
    got = _u64(gpu.search(sc["x"], 4e-3))
    assert (want >> np.uint64(62) == 1).sum() > 100_000  # vertex-vertex keys
    assert np.array_equal(got, want)


def test_full_size_sand_pile_step_matches_oracle(cc, ctx):
    """One whole step of the full particle pile: iterations and result bit-identical
    to the oracle; no two particles coincide and none is below the ground."""
    sc = scenes.config(6)
    want, n, _ = oracle.collide_step(sc)
    got, st = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                              **sc["params"])
    x = got.cpu().numpy()
    assert st["iters"] == n and st["status"] == 0 and st["ccd_hits"] == 0
    assert np.array_equal(x, want)
    from scipy.spatial import cKDTree
    npart = int((sc["w"] > 0).sum())
    d, _ = cKDTree(x[:npart]).query(x[:npart], k=2)
    assert d[:, 1].min() > 0.5e-3
    inside = (np.abs(x[:npart, :2]) < 0.055).all(axis=1)
    assert (x[:npart][inside, 2] > 0).all()


def test_batched_particles_and_meshes_equal_solo_and_oracle(cc, ctx):
    """Particle piles next to meshes in one multi-scene call: particle lists and the
    particle tree are per scene (no pair across scenes), every result bit-identical
    to the scene alone and to the oracle."""
    batch = [scenes.config(6, small=True), scenes.config(2, small=True),
             scenes.sand_pile(8, 8, 6, seed=77), scenes.config(4, small=True),
             scenes.sand_pile(5, 4, 3, seed=78)]
    res = cc.collide_step_batched(ctx, batch, max_iters=300)
    for sc, (x_b, st_b) in zip(batch, res):
        x_s, st_s = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                                    max_iters=300)
        want, n, _ = oracle.collide_step(sc, max_iters=300)
        assert np.array_equal(x_b.cpu().numpy(), x_s.cpu().numpy()), sc["name"]
        assert np.array_equal(x_b.cpu().numpy(), want), sc["name"]
        assert st_b["iters"] == st_s["iters"] == n


def test_mixed_precision_sand_pile_end_to_end(cc, ctx):
    sc = scenes.config(6, small=True)
    out, st = cc.collide_step(ctx, sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"],
                              mixed=True, max_iters=400)
    x = out.cpu().numpy()
    assert st["ccd_hits"] == 0
    assert _intersection_free(x, sc["tris"], sc["edges"])
    npart = int((sc["w"] > 0).sum())
    d = np.linalg.norm(x[:npart, None] - x[None, :npart], axis=-1)
    assert d[np.triu_indices(npart, 1)].min() > 0.5e-3


@pytest.mark.parametrize("cfg,iters", [(2, 60), (4, 60), (6, 60)])
def test_ccd_on_every_pair_lockstep(cc, ctx, cfg, iters):
    """CC_CCD_ALL: every pair of P' takes the continuous test each iteration; counts
    and state bit-identical to the oracle's, and no pair is ever in contact."""
    sc = scenes.config(cfg, small=True)
    p = dict(sc.get("params", {}), max_iters=iters, ccd_all=True)
    ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"], **p)
    gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"], trace=True, **p)
    ref.begin(sc["x"], sc["xt"])
    gpu.begin(sc["x"], sc["xt"])
    tested = 0
    for l in range(iters):
        s_ref, it_ref = ref.iterate()
        s_gpu, it_gpu = gpu.iterate()
        for k in TRACE_KEYS:
            assert it_gpu[k] == it_ref[k], (cfg, l, k)
        assert it_gpu["ccd_fail"] == it_gpu["n_pf"] and it_gpu["ccd_hits"] == 0
        tested += it_gpu["ccd_fail"]
        xr = ref.state()[0]
        xg = gpu.state()[0].cpu().numpy()
        assert np.array_equal(xg, xr)
        if s_ref:
            break
    assert tested > 0


def test_input_check_rejects_missing_triangle_sides(cc, ctx):
    """Under the input check a mesh whose edges miss a triangle side is rejected
    when it is taken in (edge-edge pairs would be incomplete)."""
    sc = scenes.config(2, small=True)
    edges = sc["edges"][1:]
    with pytest.raises(cc.CCError) as e:
        cc.Solver(ctx, sc["w"], sc["tris"], edges, validate=True)
    assert e.value.code == -1
    s = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"], validate=True)
    s.begin(sc["x"], sc["xt"])
    s.close()


@pytest.mark.parametrize("cfg,backward,sweeps", [(2, "gs", 3), (3, "gs", 2), (2, "jacobi", 2),
                                                 (6, "gs", 4)])
def test_several_sweeps_lockstep(cc, ctx, cfg, backward, sweeps):
    """More than one sweep per backward step (the ablation of Sec. 4.3.1; Jacobi
    sweeps likewise): every iteration bit-identical to the oracle (Jacobi: within
    the tolerance, as in its lockstep)."""
    sc = scenes.config(cfg, small=True)
    if backward == "jacobi":
        n, _ = _replay_lockstep(cc, ctx, sc, 150, gs_sweeps=sweeps, backward=backward)
    else:
        n, ref, gpu = _lockstep(cc, ctx, sc, 150, gs_sweeps=sweeps, backward=backward)
    assert n >= 1


# ------------------------------------------------------- normal-flow target

def _flow_meshes():
    xs, ts = scenes.icosphere(3, 0.1)[:2]
    rng = np.random.default_rng(31)
    xr = xs + rng.normal(size=xs.shape) * 2e-3
    xg, tg, _ = scenes.grid_cloth(17, 9, 0.01)
    xt_, tt_, _ = scenes.torus(48, 16, 0.1, 0.02)
    return [("icosphere", xs, ts), ("rough icosphere", xr, ts), ("grid", xg, tg),
            ("torus", xt_, tt_)]


@pytest.mark.parametrize("beta,alpha,iters", [(0.004, 2e-6, 3), (-0.03, 1e-5, 3), (0.0, 5e-6, 1),
                                              (0.01, 0.0, 0)])
def test_normal_flow_target_matches_oracle(cc, ctx, beta, alpha, iters):
    """The target of the globally injective normal flow, bit-identical to the oracle's on
    spheres, a rough sphere, an open grid and a torus."""
    for name, x, t in _flow_meshes():
        got = cc.normal_flow_target(ctx, x, t, beta, alpha, iters).cpu().numpy()
        want = oracle.normal_flow(x, t, beta, alpha, iters)
        assert np.array_equal(got, want), name


def test_normal_flow_target_rejects_bad_input(cc, ctx):
    x, t = scenes.icosphere(1, 1.0)[:2]
    bad = t.copy()
    bad[0, 0] = len(x)
    with pytest.raises(cc.CCError):
        cc.normal_flow_target(ctx, x, bad, 0.1, 0.1, 3)
    with pytest.raises(cc.CCError):
        cc.normal_flow_target(ctx, x, t, float("nan"), 0.1, 3)


def test_normal_flow_frame_matches_oracle(cc, ctx):
    """One frame of the normal-flow workload (small torus, inward flow through the
    tube): the target and the collision step's result bit-identical to the oracle's,
    and the result intersection free."""
    sc = scenes.config(7, small=True)
    f = sc["flow"]
    y = cc.normal_flow_target(ctx, sc["x"], sc["tris"], **f)
    want_y = oracle.normal_flow(sc["x"], sc["tris"], **f)
    assert np.array_equal(y.cpu().numpy(), want_y)
    got, st = cc.collide_step(ctx, sc["x"], y, sc["w"], sc["tris"], sc["edges"], **sc["params"])
    want, n, _ = oracle.collide_step(dict(sc, xt=want_y))
    assert st["iters"] == n and np.array_equal(got.cpu().numpy(), want)
    assert _intersection_free(got.cpu().numpy(), sc["tris"], sc["edges"])


def test_normal_flow_frame_full_size_matches_oracle(cc, ctx):
    """The full normal-flow frame (two icospheres of 10,242 vertices growing into each
    other): target and result bit-identical to the oracle's; the spheres stop face to
    face, about delta apart."""
    sc = scenes.config(7)
    f = sc["flow"]
    y = cc.normal_flow_target(ctx, sc["x"], sc["tris"], **f)
    want_y = oracle.normal_flow(sc["x"], sc["tris"], **f)
    assert np.array_equal(y.cpu().numpy(), want_y)
    got, st = cc.collide_step(ctx, sc["x"], y, sc["w"], sc["tris"], sc["edges"], **sc["params"])
    want, n, _ = oracle.collide_step(dict(sc, xt=want_y))
    x = got.cpu().numpy()
    assert st["iters"] == n and st["status"] == 0 and np.array_equal(x, want)
    h = len(x) // 2
    assert 0.5e-3 < x[h:, 0].min() - x[:h, 0].max() < 2e-3


def _particle_cluster(k, radius, seed):
    """k particles in a ball of the given radius (pairwise more than 2e-5 m apart),
    each heading 2e-4 m (std) in a random direction: every pair is a contact row."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < k:
        p = rng.uniform(-radius, radius, 3)
        if np.linalg.norm(p) <= radius and all(np.linalg.norm(p - q) > 2e-5 for q in pts):
            pts.append(p)
    x = np.array(pts)
    return x, x + rng.normal(0.0, 2e-4, x.shape)


def _particle_dimers(nd, seed, spacing=5e-3, gap=5e-4):
    """nd particle pairs gap apart on a lattice spacing apart, moving 0.4 mm towards
    each other: nd contact rows over 2 nd vertices."""
    rng = np.random.default_rng(seed)
    m = int(np.ceil(nd ** (1 / 3)))
    c = np.stack(np.meshgrid(*[np.arange(m)] * 3, indexing="ij"), -1).reshape(-1, 3)[:nd] * spacing
    u = rng.normal(size=(nd, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    x = np.concatenate([c + 0.5 * gap * u, c - 0.5 * gap * u])
    xt = x.copy()
    xt[:nd] -= 4e-4 * u
    xt[nd:] += 4e-4 * u
    return x, xt


@pytest.mark.parametrize("kind", ["cluster", "cluster_wide", "dimers_lds", "dimers_many",
                                  "dimers_overflow", "wide_overflow"])
def test_small_contact_set_colouring_paths_lockstep(cc, ctx, kind):
    # Contact sets of at most 4096 rows are coloured by one block with the vertex state
    # in LDS: one colour word per vertex (64 colours) for up to 4096 vertices, or, after
    # a colouring of more than 56 colours, two words (128 colours) for up to 2944. A set
    # that needs more colours than the words hold, or touches more free vertices than
    # fit, is finished by the same block with the global-memory rounds. The cases:
    # - cluster: 90 particles, about 136 colours: beyond both layouts;
    # - cluster_wide: 50 particles, 80 colours: the first iteration overflows the one-word
    #   layout (global rounds), the next ones complete in LDS with two words;
    # - dimers_lds, dimers_many: 900 and 1500 dimers (1800 and 3000 free vertices, one
    #   colour) complete in LDS with one word;
    # - dimers_overflow: 2100 dimers, 4200 free vertices: more than 4096 fit, so the block
    #   colours them with the global-memory rounds;
    # - wide_overflow: the 50-particle cluster 1 m from 1500 dimers: the later iterations
    #   take two words (more than 56 colours) over 3050 free vertices, more than 2944
    #   fit, so the block colours them with the global-memory rounds.
    if kind == "cluster":
        x, xt = _particle_cluster(90, 4.5e-4, 5)
    elif kind == "cluster_wide":
        x, xt = _particle_cluster(50, 4.5e-4, 5)
    elif kind == "wide_overflow":
        xc, xtc = _particle_cluster(50, 4.5e-4, 5)
        xd, xtd = _particle_dimers(1500, 7)
        x = np.concatenate([xc + 1.0, xd])
        xt = np.concatenate([xtc + 1.0, xtd])
    else:
        nd = {"dimers_lds": 900, "dimers_many": 1500, "dimers_overflow": 2100}[kind]
        x, xt = _particle_dimers(nd, 7)
    sc = {"name": kind, "x": x, "xt": xt, "w": np.ones(len(x)),
          "tris": np.zeros((0, 3), np.int32), "edges": np.zeros((0, 2), np.int32), "params": {}}
    n, ref, gpu = _lockstep(cc, ctx, sc, 6)
    assert n >= 2
    cols = [t["n_colors"] for t in gpu.trace]
    if kind == "cluster":
        assert cols[0] > 128
    elif kind == "cluster_wide":
        assert 64 < cols[0] <= 127 and all(56 < c <= 127 for c in cols[1:3])
    elif kind == "dimers_overflow":
        assert len(x) > 4096 and gpu.trace[0]["n_a"] <= 4096
    elif kind == "wide_overflow":
        assert len(x) > 2944 and all(56 < c <= 127 for c in cols[1:3])
        assert all(t["n_a"] <= 4096 for t in gpu.trace)
