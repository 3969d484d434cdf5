"""The normal-flow target without allocation (cc_normal_flow_target_noalloc), called
through the C ABI, against the allocating entry point cc_normal_flow_target."""
import ctypes as C

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2211_04045_amd as cc
    from paper_2211_04045_amd import _lib
    lib = _lib.load()
    lib.cc_normal_flow_target_noalloc.restype = C.c_int
    lib.cc_normal_flow_target_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                                  C.c_int32, C.c_double, C.c_double, C.c_int32,
                                                  C.c_void_p, C.c_void_p]
    return torch, cc, lib, cc.Context(0)


def _mesh(subdiv, seed):
    x, tris, _ = scenes.icosphere(subdiv, 0.05)
    rng = np.random.default_rng(seed)
    return x + rng.normal(size=x.shape) * 1e-4, tris


def _noalloc(env, x, tris, beta, alpha, iters):
    torch, cc, lib, ctx = env
    xd = torch.as_tensor(x, dtype=torch.float64, device="cuda")
    td = torch.as_tensor(tris, dtype=torch.int32, device="cuda")
    y = torch.full_like(xd, float("nan"))
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.cc_normal_flow_target_noalloc(ctx.h, C.c_void_p(xd.data_ptr()), len(x),
                                           C.c_void_p(td.data_ptr()), len(tris), beta, alpha,
                                           iters, C.c_void_p(y.data_ptr()), stream)
    return rc, y.cpu().numpy()


def test_noalloc_target_equals_the_allocating_entry_point_twice(env):
    torch, cc, lib, ctx = env
    # a larger mesh, then a smaller one: the second call must not see the first's
    # counts or lists in the shared scratch array
    for subdiv, seed, iters in ((5, 1, 3), (3, 2, 2), (4, 3, 0)):
        x, tris = _mesh(subdiv, seed)
        rc, got = _noalloc(env, x, tris, 0.004, 2e-6, iters)
        assert rc == 0
        want = cc.normal_flow_target(ctx, x, tris, 0.004, 2e-6, iters).cpu().numpy()
        assert np.array_equal(got, want), subdiv


def test_noalloc_target_rejects_sizes_beyond_its_limit_and_bad_indices(env):
    torch, cc, lib, ctx = env
    x, tris = _mesh(2, 4)
    big = np.zeros((131073, 3))
    rc, _ = _noalloc(env, big, tris, 0.004, 2e-6, 1)
    assert rc == -1
    bad = tris.copy()
    bad[7, 1] = len(x)
    rc, _ = _noalloc(env, x, bad, 0.004, 2e-6, 1)
    assert rc == -1
    # and the next good call is unaffected
    rc, got = _noalloc(env, x, tris, 0.004, 2e-6, 1)
    want = cc.normal_flow_target(ctx, x, tris, 0.004, 2e-6, 1).cpu().numpy()
    assert rc == 0 and np.array_equal(got, want)
