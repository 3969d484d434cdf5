"""The C-ABI library loads and exports every function include/cc.h declares
(CPU only: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "cc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|size_t|const char\*)\s+(cc_\w+)\s*\(", src, re.M)))


def test_header_declares_the_step_and_solver_api():
    names = declared()
    for n in ("cc_collide_step", "cc_context_create", "cc_solver_iterate", "cc_solver_search"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2211_04045_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared():
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTED) == declared()


def test_default_params_are_table_2():
    from paper_2211_04045_amd import params
    p = params()
    assert (p.delta, p.d_min, p.d_max, p.sigma, p.gamma, p.eps) == (1e-3, 2e-3, 4e-3, 1.1, 0.9, 1e-4)
    assert p.gs_sweeps == 1 and p.max_colors == 1024
    # the oracle's defaults are the same numbers (declared independently)
    import oracle
    for k in ("delta", "d_min", "d_max", "sigma", "gamma", "eps", "kappa", "gs_sweeps",
              "max_colors", "seed", "omega", "backward"):
        assert getattr(p, k) == oracle.DEFAULTS[k], k


def test_strerror_names_every_code():
    from paper_2211_04045_amd import _lib
    lib = _lib.load()
    for code in range(0, -10, -1):
        assert lib.cc_strerror(code) != b"unknown error"


def test_edges_from_tris_host_matches_generator():
    """The library's host edge builder against the input generator's numpy one
    (two independent implementations) on a grid, an icosphere and a cube surface."""
    import numpy as np
    import paper_2211_04045_amd as cc
    import scenes
    for tris in (scenes.grid_cloth(7, 5, 0.01)[1], scenes.icosphere(2, 1.0)[1],
                 scenes.box_surface(3, 1.0)[1]):
        got = cc.edges_from_tris(tris)
        want = scenes.edges_from_tris(np.asarray(tris))
        want = np.sort(np.sort(want, axis=1).view([("a", want.dtype), ("b", want.dtype)]), axis=0)
        assert np.array_equal(got, want.view(got.dtype).reshape(-1, 2))
    assert cc.edges_from_tris(np.zeros((0, 3), np.int32)).shape == (0, 2)
    with pytest.raises(cc.CCError):
        cc.edges_from_tris(np.array([[0, 1, 1]], np.int32))


def test_scene_bytes_grows_with_size():
    import paper_2211_04045_amd as cc
    lib = cc._lib.load()
    a = lib.cc_scene_bytes(1000, 2000, 3000)
    assert a > 0
    assert lib.cc_scene_bytes(2000, 2000, 3000) > a
    assert lib.cc_scene_bytes(1000, 4000, 3000) > a
    assert lib.cc_scene_bytes(1000, 2000, 6000) > a
    assert lib.cc_scene_bytes(-1, 0, 0) == 0


def test_timing_flags_select_one_family():
    """time_one= sets CC_TIME_ONE and the family index (cc_params.time_kind); the
    default times nothing, and the flag's bit matches the header."""
    import paper_2211_04045_amd as cc
    from paper_2211_04045_amd import _lib
    src = open(os.path.join(ROOT, "include", "cc.h")).read()
    assert int(re.search(r"#define CC_TIME_ONE (\d+)u", src).group(1)) == _lib.CC_TIME_ONE
    p = cc.params()
    assert not (p.flags & _lib.CC_TIME_ONE) and not (p.flags & _lib.CC_TIME_KERNELS)
    assert p.time_kind == 0
    for i, name in enumerate(_lib.K_NAMES):
        q = cc.params(time_one=name)
        assert q.flags & _lib.CC_TIME_ONE and q.time_kind == i
    assert not (cc.params(time_one="pair", **{}).flags & _lib.CC_TIME_KERNELS)
    assert not (cc.params(time_one=None).flags & _lib.CC_TIME_ONE)
