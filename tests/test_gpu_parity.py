"""Parity of the HIP path with the FP64 oracle, through the C ABI.

The bar: contact sets (P', A and the colouring) bit-identical; positions within
1e-6 of the scene's bounding-box diagonal (the design is order independent, so
the observed difference is expected to be exactly zero and is asserted too).
"""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu

TRACE_KEYS = ["searched", "n_colors", "n_p", "n_pf", "n_a", "ccd_fail", "d_before", "d_after",
              "move_max", "r_inf", "fp_pf", "fp_a", "fp_col"]


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
    for l in range(max_iters):
        s_ref, it_ref = ref.iterate()
        s_gpu, it_gpu = gpu.iterate()
        n += 1
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
    return n, ref, gpu


def test_library_loads_on_gpu(cc, ctx):
    assert ctx.h


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
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


@pytest.mark.parametrize("cfg,iters", [(2, 200), (3, 400), (4, 200), (1, 120)])
def test_end_to_end_lockstep_small(cc, ctx, cfg, iters):
    sc = scenes.config(cfg, small=True)
    _lockstep(cc, ctx, sc, iters)


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


def test_full_size_folded_cloth_lockstep_samples(cc, ctx):
    """Full-size workload in the benchmark's configuration: the GPU runs the step;
    at sampled iterations the oracle replays one iteration from the GPU's state and
    the sets, D_i and the new state must agree exactly."""
    sc = scenes.config(2)
    p = dict(sc["params"])
    gpu = cc.Solver(ctx, sc["w"], sc["tris"], sc["edges"], trace=True, **p)
    gpu.begin(sc["x"], sc["xt"])
    ref = oracle.Scene(sc["w"], sc["tris"], sc["edges"], **p)
    ref.begin(sc["x"], sc["xt"])
    samples = {0, 1, 5}
    for l in range(6):
        if l in samples:
            x, y, r, D = gpu.state()
            P = gpu.P()
            ref.set_state(x.cpu().numpy(), y.cpu().numpy(), r.cpu().numpy(), D,
                          P.cpu().numpy().view(np.uint64))
            _, it_ref = ref.iterate()
        stop, it_gpu = gpu.iterate()
        if l in samples:
            for k in TRACE_KEYS:
                assert it_gpu[k] == it_ref[k], (l, k, it_gpu[k], it_ref[k])
            xr, yr, rr, Dr = ref.state()
            xg, yg, rg, Dg = gpu.state()
            assert np.array_equal(xg.cpu().numpy(), xr)
            assert np.array_equal(yg.cpu().numpy(), yr)
            assert np.array_equal(rg.cpu().numpy(), rr) and Dg == Dr
            assert np.array_equal(gpu.Di().cpu().numpy(), ref.Di())
        if stop:
            break


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
