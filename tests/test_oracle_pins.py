"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
exact rational minimisation, closed forms derived from the constraint
definitions (Sec. 4.1, Sec. 4.2), finite differences of exact distances, worked
cases and invariants of the randomised palette colouring (proper, a function of
the row set), brute-force sets, sampled minimum distances along a piece, the
safety lemma of Sec. 5 checked in exact arithmetic, and exact intersection tests
of whole steps' final states."""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest

import exact
import oracle
import scenes

DELTA = 1e-3


def rel_close(a, b, rtol=1e-12, atol=1e-30):
    return abs(float(a) - float(b)) <= atol + rtol * abs(float(b))


# ------------------------------------------------------------------ distances

def _rand_pts(rng, k, scale=0.01):
    return [rng.normal(size=3) * scale for _ in range(k)]


def test_pt_tri_distance_matches_exact_rational():
    rng = np.random.default_rng(1)
    for trial in range(300):
        p, a, b, c = _rand_pts(rng, 4)
        if trial % 5 == 0:  # point close to the triangle plane
            n = np.cross(b - a, c - a)
            p = a + 0.3 * (b - a) + 0.2 * (c - a) + n / np.linalg.norm(n) * 1e-4
        d2, bary = oracle.pt_tri_d2(p, a, b, c)
        ex = exact.pt_tri_d2(p, a, b, c)
        assert rel_close(d2, ex, rtol=1e-10, atol=1e-24), (trial, d2, float(ex))
        q = bary[0] * a + bary[1] * b + bary[2] * c
        assert abs(bary.sum() - 1) < 1e-12 and (bary >= -1e-15).all()
        assert rel_close(np.dot(p - q, p - q), d2, rtol=1e-9, atol=1e-24)


def test_pt_tri_degenerate_triangles():
    p = np.array([0.3, 0.4, 0.1])
    a = np.array([0.0, 0, 0])
    b = np.array([1.0, 0, 0])
    for c in (np.array([2.0, 0, 0]), a.copy(), np.array([0.5, 0, 0])):
        d2, _ = oracle.pt_tri_d2(p, a, b, c)
        assert rel_close(d2, exact.pt_tri_d2(p, a, b, c))
    # all three corners coincide
    d2, _ = oracle.pt_tri_d2(p, a, a, a)
    assert rel_close(d2, np.dot(p, p))


def test_vertex_over_triangle_interior_is_height():
    a, b, c = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    for h in (1e-3, 0.25, -0.5):
        d2, bary = oracle.pt_tri_d2(np.array([0.25, 0.25, h]), a, b, c)
        assert d2 == h * h
        assert np.allclose(bary, [0.5, 0.25, 0.25])


def test_seg_seg_distance_matches_exact_rational():
    rng = np.random.default_rng(2)
    for trial in range(300):
        a, b, c, e = _rand_pts(rng, 4)
        if trial % 7 == 0:  # parallel
            e = c + (b - a) * 0.7
        if trial % 11 == 0:  # collinear overlapping
            c = a + 0.3 * (b - a)
            e = a + 1.4 * (b - a)
        if trial % 13 == 0:  # zero-length segment
            e = c.copy()
        d2, st = oracle.seg_seg_d2(a, b, c, e)
        ex = exact.seg_seg_d2(a, b, c, e)
        assert rel_close(d2, ex, rtol=1e-10, atol=1e-24), (trial, d2, float(ex))
        p = a + st[0] * (b - a)
        q = c + st[1] * (e - c)
        assert rel_close(np.dot(p - q, p - q), d2, rtol=1e-9, atol=1e-24)


def test_perpendicular_crossing_segments_offset():
    d2, st = oracle.seg_seg_d2([-1.0, 0, 0], [1.0, 0, 0], [0.0, -1, 0.125], [0.0, 1, 0.125])
    assert d2 == 0.125 ** 2 and np.allclose(st, [0.5, 0.5])


# -------------------------------------------------------------- constraints

def _scene(n, w=None, tris=(), edges=(), **kw):
    w = np.ones(n) if w is None else np.asarray(w, float)
    return oracle.Scene(w, np.asarray(tris, np.int32).reshape(-1, 3),
                        np.asarray(edges, np.int32).reshape(-1, 2), **kw)


def _fd_grad(f, x, idx, h=1e-9):
    g = np.zeros((4, 3))
    for i, v in enumerate(idx):
        for k in range(3):
            xp = x.copy(); xm = x.copy()
            xp[v, k] += h; xm[v, k] -= h
            g[i, k] = (f(xp) - f(xm)) / (2 * h)
    return g


def _ref_volume_ratio(xs_ref):
    """V(y)/V(r) - 1 for fixed reference corners, via numpy's determinant."""
    r = np.asarray(xs_ref)
    vr = np.linalg.det(np.stack([r[1] - r[0], r[2] - r[0], r[3] - r[0]]))
    return lambda ys: np.linalg.det(np.stack([ys[1] - ys[0], ys[2] - ys[0], ys[3] - ys[0]])) / vr - 1


def test_vt_volume_constraint_closed_form_and_gradient():
    # the volume form (Sec. 4.1, Fig. fig:vt) for a vertex over the face: its closest
    # point is the interior projection, the separating direction is the normal
    rng = np.random.default_rng(3)
    s = _scene(4, tris=[(1, 2, 3)], delta=DELTA)
    checked = 0
    for trial in range(200):
        tri = rng.normal(size=(3, 3)) * 0.01
        n = np.cross(tri[1] - tri[0], tri[2] - tri[0]); n /= np.linalg.norm(n)
        bc = rng.dirichlet([2, 2, 2]) * 0.9 + 0.1 / 3
        p = bc @ tri + n * rng.uniform(-1, 1) * 0.8e-3
        x = np.vstack([p, tri])
        d = math.sqrt(exact.pt_tri_d2(p, *tri))
        if not d < DELTA:
            continue
        row = s.contact_row(x, oracle.vt_key(0, 0))
        assert row["kind"] == 0
        h = abs(np.dot(p - tri[0], n))
        # c0 = V(x)/V(r) - 1 = |h| / (|h| + delta - d) - 1 (derived from the definition of r)
        assert rel_close(row["c0"] + 1, h / (h + DELTA - d), rtol=1e-7, atol=1e-12)
        # gradient: finite differences of the volume ratio with the reference held fixed;
        # r from the paper's definition with the closest point and side of x
        side = 1.0 if np.dot(p - tri[0], n) >= 0 else -1.0
        g = 0.5 * (DELTA - d)
        ref = [p + g * side * n] + [t - g * side * n for t in tri]
        fd = _fd_grad(_ref_volume_ratio(ref), x, [0, 1, 2, 3], h=1e-7)
        assert np.allclose(row["J"], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
        # the vertex is pushed to x's side of the triangle
        assert np.dot(row["J"][0], side * n) > 0
        # A = sum_v w_v |J_v|^2 with unit masses
        assert rel_close(1 / row["inv_a"], (row["J"] ** 2).sum(), rtol=1e-12)
        checked += 1
    assert checked > 100


def _exact_dist(kind, xs):
    """Exact rational distance of a vertex-triangle (0) or edge-edge (1) pair, as a float."""
    d2 = exact.pt_tri_d2(*xs) if kind == 0 else exact.seg_seg_d2(*xs)
    return math.sqrt(float(d2))


@pytest.mark.parametrize("kind", [0, 1])
def test_gap_form_when_the_closest_point_is_on_the_boundary(kind):
    # a vertex beside the face (closest point on an edge or a corner) or edges whose
    # closest points include an endpoint: the separating direction is not the normal,
    # and the row is the gap constraint c = d/delta - 1 (Sec. 4.1 names it), whose
    # Jacobian is the gradient of the distance over delta: finite differences of the
    # exact rational distance pin it independently
    rng = np.random.default_rng(11 + kind)
    s = _scene(4, tris=[(1, 2, 3)], edges=[(0, 1), (2, 3)], delta=DELTA)
    checked = 0
    for trial in range(300):
        if kind == 0:
            tri = rng.normal(size=(3, 3)) * 0.01
            n = np.cross(tri[1] - tri[0], tri[2] - tri[0]); n /= np.linalg.norm(n)
            e = rng.integers(3)
            a, b = tri[e], tri[(e + 1) % 3]
            c = tri[(e + 2) % 3]
            t = rng.uniform(-0.2, 1.2)
            q = a + t * (b - a)
            # outward in the plane, away from the third corner, plus a normal offset
            m = (q - c) - np.dot(q - c, b - a) / np.dot(b - a, b - a) * (b - a)
            m /= np.linalg.norm(m)
            p = q + m * rng.uniform(0.1, 0.7) * 1e-3 + n * rng.uniform(-0.5, 0.5) * 1e-3
            x = np.vstack([p, tri])
            key = oracle.vt_key(0, 0)
        else:
            a = rng.normal(size=3) * 0.01
            d1 = rng.normal(size=3) * 0.01
            d2 = rng.normal(size=3) * 0.01
            u = rng.normal(size=3); u /= np.linalg.norm(u)
            # the end of edge 1 near an interior point of edge 2
            c = a + d1 + u * rng.uniform(0.1, 0.9) * 1e-3 - rng.uniform(0.2, 0.8) * d2
            x = np.vstack([a, a + d1, c, c + d2])
            key = oracle.ee_key(0, 1)
        d = _exact_dist(kind, x)
        if not d < DELTA:
            continue
        row = s.contact_row(x, key)
        if row["kind"] == 0:
            continue  # the closest points happen to be interior
        assert row["kind"] == 1
        assert rel_close(row["c0"], d / DELTA - 1, rtol=1e-9, atol=1e-12)
        fd = _fd_grad(lambda ys: _exact_dist(kind, ys) / DELTA, x, [0, 1, 2, 3], h=1e-8)
        assert np.allclose(row["J"], fd, rtol=1e-4, atol=1e-5 * np.abs(fd).max())
        checked += 1
    assert checked > 100


def test_ee_volume_constraint_closed_form_and_gradient():
    rng = np.random.default_rng(4)
    s = _scene(4, edges=[(0, 1), (2, 3)], delta=DELTA)
    checked = 0
    for trial in range(200):
        a = rng.normal(size=3) * 0.01
        d1 = rng.normal(size=3) * 0.01
        d2 = rng.normal(size=3) * 0.01
        m = np.cross(d1, d2); m /= np.linalg.norm(m)
        s0, t0 = rng.uniform(0, 1, 2)
        off = m * rng.uniform(-1, 1) * 0.9e-3
        c = a + s0 * d1 - t0 * d2 - off
        x = np.vstack([a, a + d1, c, c + d2])
        d = math.sqrt(exact.seg_seg_d2(*x))
        if not d < DELTA:
            continue
        row = s.contact_row(x, oracle.ee_key(0, 1))
        assert row["kind"] == 0
        h = abs(np.dot(x[0] - x[2], m))
        assert rel_close(row["c0"] + 1, h / (h + DELTA - d), rtol=1e-7, atol=1e-12)
        side = 1.0 if np.dot(x[0] - x[2], m) >= 0 else -1.0
        g = 0.5 * (DELTA - d)
        ref = [x[0] + g * side * m, x[1] + g * side * m, x[2] - g * side * m, x[3] - g * side * m]
        fd = _fd_grad(_ref_volume_ratio(ref), x, [0, 1, 2, 3], h=1e-7)
        assert np.allclose(row["J"], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
        checked += 1
    assert checked > 100


def test_gap_fallback_for_parallel_edges_and_static_triangle():
    s = _scene(4, w=[1, 1, 0, 0], edges=[(0, 1), (2, 3)], delta=DELTA)
    x = np.array([[0, 0, 0.4e-3], [0.01, 0, 0.4e-3], [0.002, 0, 0], [0.008, 0, 0]], float)
    row = s.contact_row(x, oracle.ee_key(0, 1))
    assert row["kind"] == 1
    assert rel_close(row["c0"], 0.4e-3 / DELTA - 1)
    u = np.array([0, 0, 1.0])
    assert np.allclose(row["J"].sum(axis=0), 0, atol=1e-9)
    assert np.dot(row["J"][0] + row["J"][1], u) > 0
    # closed form: J_a + J_b = u/delta (the segment-1 weights sum to one)
    assert np.allclose(row["J"][0] + row["J"][1], u / DELTA)


def test_vt_static_triangle_interior_closed_form():
    # free vertex above the interior of a static triangle: c0 = d/(d + delta - d) - 1 and
    # J_a = n / (delta) * (|N| / |N|) ... i.e. J_a . n = 1/delta
    s = _scene(4, w=[1, 0, 0, 0], tris=[(1, 2, 3)], delta=DELTA)
    for hgt in (1e-5, 3e-4, 9e-4):
        x = np.array([[0.2, 0.2, hgt], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
        row = s.contact_row(x, oracle.vt_key(0, 0))
        assert rel_close(row["c0"], hgt / DELTA - 1, rtol=1e-9)
        assert rel_close(row["J"][0, 2], 1 / DELTA, rtol=1e-9)
        assert abs(row["J"][0, 0]) < 1e-9 and abs(row["J"][0, 1]) < 1e-9


# ------------------------------------------------------------- search, colour

def _two_patches(nx=3, spacing=5e-3, gap=3e-3, shift=(1.3e-3, 0.9e-3), move=8e-3,
                 twist=0.0, seed=5):
    xa, ta, ea = scenes.grid_cloth(nx, nx, spacing)
    xb = xa.copy()
    xb[:, 0] += shift[0]
    xb[:, 1] += shift[1]
    xb[:, 2] += gap
    if twist:
        c, s_ = math.cos(twist), math.sin(twist)
        ctr = xb[:, :2].mean(axis=0)
        d = xb[:, :2] - ctr
        xb[:, :2] = ctr + d @ np.array([[c, s_], [-s_, c]])
    x = np.vstack([xa, xb])
    tris = np.vstack([ta, ta + len(xa)])
    edges = np.vstack([ea, ea + len(xa)])
    rng = np.random.default_rng(seed)
    xt = x.copy()
    xt[: len(xa), 2] += move
    xt[len(xa):, 2] -= move
    xt += rng.normal(size=xt.shape) * 2e-4
    return x, xt, tris.astype(np.int32), edges.astype(np.int32)


def _universe_keys(n, tris, edges):
    keys = set()
    for a in range(n):
        for f, t in enumerate(tris):
            if a not in t:
                keys.add(oracle.vt_key(a, f))
    for e in range(len(edges)):
        for g in range(e + 1, len(edges)):
            if not set(edges[e]) & set(edges[g]):
                keys.add(oracle.ee_key(e, g))
    # vertex-vertex: two vertices that no triangle and no edge refer to
    used = set(int(v) for t in tris for v in t) | set(int(v) for e in edges for v in e)
    part = [a for a in range(n) if a not in used]
    for i, a in enumerate(part):
        for b in part[i + 1:]:
            keys.add(oracle.vv_key(a, b))
    return keys


def _pair_exact(k, X, tris, edges):
    """Vertices of pair key k and its squared distance at X in exact arithmetic."""
    a, f = (k >> 32) & 0x3FFFFFFF, k & 0xFFFFFFFF
    if k >> 63:
        v = [*edges[a], *edges[f]]
        return v, exact.seg_seg_d2(*(X[i] for i in v))
    if (k >> 62) & 1:
        v = [a, f]
        return v, sum((Fr(float(X[a, c])) - Fr(float(X[f, c]))) ** 2 for c in range(3))
    v = [a, *tris[f]]
    return v, exact.pt_tri_d2(*(X[i] for i in v))


def test_search_grid_equals_brute_force_and_exact_threshold():
    x, xt, tris, edges = _two_patches()
    s = oracle.Scene(np.ones(len(x)), tris, edges)
    for dmax in (2e-3, 4e-3, 6e-3):
        g = set(int(k) for k in s.search(x, dmax))
        b = set(int(k) for k in s.search(x, dmax, brute=True))
        assert g == b
        # independent check: universe built here, threshold decided in exact arithmetic
        want = set()
        for k in _universe_keys(len(x), tris, edges):
            ee = k >> 63
            a, f = (k >> 32) & 0x7FFFFFFF, k & 0xFFFFFFFF
            v = [*edges[a], *edges[f]] if ee else [a, *tris[f]]
            d2 = (exact.seg_seg_d2 if ee else exact.pt_tri_d2)(*(x[i] for i in v))
            if d2 < Fr(dmax) * Fr(dmax):
                want.add(k)
        # sets may differ only on pairs whose distance is within rounding of dmax
        for k in want ^ g:
            ee = k >> 63
            a, f = (k >> 32) & 0x7FFFFFFF, k & 0xFFFFFFFF
            v = [*edges[a], *edges[f]] if ee else [a, *tris[f]]
            d2 = float((exact.seg_seg_d2 if ee else exact.pt_tri_d2)(*(x[i] for i in v)))
            assert abs(d2 - dmax * dmax) < 1e-12 * dmax * dmax


def test_search_drops_all_static_pairs():
    x, xt, tris, edges = _two_patches(gap=1e-3)
    w = np.zeros(len(x))
    s = oracle.Scene(w, tris, edges)
    s.begin(x, x)
    assert len(s.search(x, 4e-3)) == 0


PHI = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def _random_rows(rng, n, m):
    rows = rng.integers(0, n, size=(m, 4)).astype(np.int32)
    rows[rng.uniform(size=(m, 4)) < 0.2] = -1
    for r in rows:  # a constraint lists a vertex once
        seen = set()
        for k in range(4):
            if r[k] in seen:
                r[k] = -1
            elif r[k] >= 0:
                seen.add(int(r[k]))
    return rows


def _proper(rows, col, w):
    at = {}
    for r, vs in enumerate(rows):
        for v in vs:
            if v >= 0 and w[v] > 0:
                at.setdefault(int(v), []).append(int(col[r]))
    return all(len(cs) == len(set(cs)) for cs in at.values())


def test_colouring_is_proper_and_independent_of_row_order():
    """Rows sharing a free vertex get different colours; the colour of a row is a
    function of the row set (permuting the rows permutes the colours)."""
    rng = np.random.default_rng(6)
    n = 60
    w = np.where(rng.uniform(size=n) < 0.8, 1.0, 0.0)
    s = _scene(n, w=w)
    for trial in range(20):
        m = int(rng.integers(1, 400))
        rows = _random_rows(rng, n, m)
        keys = rng.choice(2 ** 62, size=m, replace=False).astype(np.uint64)
        col, nc = s.color(rows, keys)
        assert _proper(rows, col, w)
        assert nc == col.max() + 1
        perm = rng.permutation(m)
        col2, nc2 = s.color(rows[perm], keys[perm])
        assert np.array_equal(col2, col[perm]) and nc2 == nc


def _neighbours(rows, w):
    at = {}
    for r, vs in enumerate(rows):
        for v in vs:
            if v >= 0 and w[v] > 0:
                at.setdefault(int(v), set()).add(r)
    nb = [set() for _ in rows]
    for rs in at.values():
        for r in rs:
            nb[r] |= rs - {r}
    return nb


def test_greedy_colouring_is_proper_first_fit_and_follows_its_order():
    """The edge rows' colouring: proper; first fit (every colour below a row's own is
    taken by a neighbour, the defining property of a greedy colouring); no more
    colours than the largest neighbourhood plus one; a function of the row set; and
    equal to a plain greedy pass, written here, over the rows in decreasing
    priority."""
    rng = np.random.default_rng(16)
    n = 50
    w = np.where(rng.uniform(size=n) < 0.8, 1.0, 0.0)
    s = _scene(n, w=w)
    seed = oracle.DEFAULTS["seed"]
    for trial in range(20):
        m = int(rng.integers(1, 300))
        rows = _random_rows(rng, n, m)
        keys = rng.choice(2 ** 31, size=m, replace=False).astype(np.uint64)
        col, nc = s.color_greedy(rows, keys)
        nb = _neighbours(rows, w)
        assert _proper(rows, col, w)
        assert nc == col.max() + 1
        for r in range(m):
            assert {int(col[q]) for q in nb[r]} >= set(range(int(col[r])))
        assert nc <= max(len(x) for x in nb) + 1
        perm = rng.permutation(m)
        col2, nc2 = s.color_greedy(rows[perm], keys[perm])
        assert np.array_equal(col2, col[perm]) and nc2 == nc
        order = sorted(range(m), key=lambda r: -s.greedy_prio(int(keys[r]), seed))
        want = [-1] * m
        for r in order:
            used = {want[q] for q in nb[r]}
            c = 0
            while c in used:
                c += 1
            want[r] = c
        assert list(col) == want


def test_greedy_priority_is_unique_and_seeded():
    """The greedy order: distinct keys get distinct priorities (the key fills the low
    32 bits), and another seed gives another order."""
    s = _scene(4)
    seed = oracle.DEFAULTS["seed"]
    keys = list(range(5000))
    p = [s.greedy_prio(k, seed) for k in keys]
    assert len(set(p)) == len(keys)
    assert all(pk & 0xFFFFFFFF == k for pk, k in zip(p, keys))
    q = [s.greedy_prio(k, seed + 1) for k in keys]
    assert np.argsort(p).tolist() != np.argsort(q).tolist()


def test_colouring_small_cases():
    """Worked cases of the rule: a row alone, or at static vertices only, takes
    colour 0; k rows at one free vertex take k different colours; two rows at one
    free vertex whose first-round picks differ keep them (palette 2, pick
    h mod 2 with h = mix64(mix64(key ^ seed) + 1 * phi))."""
    seed = oracle.DEFAULTS["seed"]
    w = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 1.0, 1.0])
    s = _scene(len(w), w=w)
    col, _ = s.color(np.array([[0, 1, 2, -1]]), np.array([7], np.uint64))
    assert list(col) == [0]
    col, _ = s.color(np.array([[3, 4, -1, -1], [3, 4, -1, -1]]), np.array([1, 2], np.uint64))
    assert list(col) == [0, 0]
    k = 9
    rows = np.array([[5, -1, -1, -1]] * k)
    col, nc = s.color(rows, np.arange(1, k + 1, dtype=np.uint64))
    assert sorted(col) == sorted(set(col)) and len(set(col)) == k
    def first_pick(key):
        h = oracle.mix64((oracle.mix64(key ^ seed) + PHI) & M64)
        return h % 2
    keys = None
    for a in range(1, 200):
        for b in range(a + 1, 200):
            if first_pick(a) != first_pick(b):
                keys = (a, b)
                break
        if keys:
            break
    col, _ = s.color(np.array([[6, 0, -1, -1], [6, 1, -1, -1]]), np.array(keys, np.uint64))
    assert list(col) == [first_pick(keys[0]), first_pick(keys[1])]


# -------------------------------------------------------------- full step

def test_vertex_through_static_triangle_settles_at_delta():
    x = np.array([[0.2, 0.2, 0.005], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    xt = x.copy()
    xt[0, 2] = -0.005
    s = oracle.Scene(np.array([1.0, 0, 0, 0]), [[1, 2, 3]], [[1, 2], [2, 3], [1, 3]], max_iters=100)
    out, n, tr = s.run(x, xt, trace_cap=100)
    assert abs(out[0, 2] - DELTA) < 1e-15  # the fixed point of the renewed linearisation
    assert out[0, 2] > 0  # same side as x^t (Fig. fig:different_linearization)
    assert np.array_equal(out[1:], x[1:])
    assert tr[-1]["r_inf"] < 1e-4


def test_free_flight_iteration_count_and_exact_target():
    # one free vertex, nothing within D_max ever: every iteration moves 0.45 D_max
    x = np.array([[0.0, 0, 0.5], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    xt = x.copy()
    S = 0.0137
    xt[0, 0] += S
    s = oracle.Scene(np.array([1.0, 0, 0, 0]), [[1, 2, 3]], [[1, 2], [2, 3], [1, 3]], max_iters=100)
    out, n, tr = s.run(x, xt, trace_cap=100)
    assert n == math.ceil(S / (0.45 * 4e-3))
    assert np.array_equal(out, xt)
    assert all(t["searched"] for t in tr)  # D drops to 0.1 D_max < D_min each time


def test_static_input_returns_input_after_one_iteration():
    x, xt, tris, edges = _two_patches(gap=3e-3)
    s = oracle.Scene(np.ones(len(x)), tris, edges, max_iters=10)
    out, n, tr = s.run(x, x, trace_cap=10)
    assert n == 1 and np.array_equal(out, x)


def test_single_row_projection_is_exact():
    # one active row, static triangle: after the backward step the linearised
    # constraint holds with equality (complementarity of the LCP, Eq. eqn:LCP)
    x = np.array([[0.2, 0.2, 0.0005], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    xt = x.copy()
    xt[0, 2] = -0.004
    s = oracle.Scene(np.array([1.0, 0, 0, 0]), [[1, 2, 3]], [[1, 2], [2, 3], [1, 3]], max_iters=1)
    s.begin(x, xt)
    s.iterate()
    _, y, _, _ = s.state()
    row = s.contact_row(x, oracle.vt_key(0, 0))
    res = row["c0"] + sum(np.dot(row["J"][k], y[row["v"][k]] - x[row["v"][k]]) for k in range(4))
    assert abs(res) < 1e-12
    assert rel_close(y[0, 2], DELTA, rtol=1e-12)


def test_edge_length_row_limits_stretch_to_sigma():
    # vertex 0 pushed out of a static triangle; its short edge to free vertex 4 would
    # stretch beyond sigma * L; the edge row pulls vertex 4 along
    x = np.array([[0.2, 0.2, 0.0005], [0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.2, 0.0015]], float)
    xt = x.copy()
    xt[0, 2] = -0.003
    xt[4, 2] = -0.004  # target edge points along the coming push, L = 1 mm
    s = oracle.Scene(np.array([1.0, 0, 0, 0, 1.0]), [[1, 2, 3]],
                     [[1, 2], [2, 3], [1, 3], [0, 4]], max_iters=1)
    s.begin(x, xt)
    s.iterate()
    _, y, _, _ = s.state()
    e = xt[0] - xt[4]
    g = e / np.dot(e, e)
    assert rel_close(np.dot(g, y[0] - y[4]), 1.1, rtol=1e-12)


def _safety_run(x, xt, tris, edges, w, iters, **kw):
    s = oracle.Scene(w, tris, edges, max_iters=iters, **kw)
    s.begin(x, xt)
    U = _universe_keys(len(x), tris, edges)
    traj = [x.copy()]
    for l in range(iters):
        X0, _, R0, D0 = s.state()
        stop, it = s.iterate()
        X1, _, R1, D1 = s.state()
        Di = s.Di()
        mv = np.linalg.norm(X1 - X0, axis=1)
        # forward bound (Eq. eq:forward2) and r bookkeeping
        assert (mv <= 0.45 * Di * (1 + 1e-12) + 1e-18).all()
        assert ((R1 >= 0) & (R1 <= R0)).all()
        assert D1 == it["d_before"] - 2 * it["move_max"]
        # P' contains every pair below D^(l) (Sec. 3.1 reuse bound)
        Pf = set(int(k) for k in s.P())
        for k in U:
            v, d2 = _pair_exact(k, X0, tris, edges)
            D = Fr(it["d_before"])
            if d2 < D * D * Fr(1 - 1e-12):
                assert k in Pf
            # the lemma of Sec. 5 in exact arithmetic: no vertex of the pair moved
            # half the pair distance, so the linear piece stays in the free region
            m2 = max(sum((Fr(float(X1[i, c])) - Fr(float(X0[i, c]))) ** 2 for c in range(3))
                     for i in v)
            assert 4 * m2 < d2
        traj.append(X1)
        if stop:
            break
    return traj, s


@pytest.mark.parametrize("twist", [0.0, 0.7])
def test_two_patches_pass_through_is_resolved_safely(twist):
    x, xt, tris, edges = _two_patches(twist=twist)
    traj, s = _safety_run(x, xt, tris, edges, np.ones(len(x)), iters=40)
    xf = traj[-1]
    assert not exact.mesh_self_intersects(xf, tris.tolist(), edges.tolist())
    # the patches kept their order along z (linearisation at x, Sec. 4)
    n = len(x) // 2
    assert xf[:n, 2].mean() < xf[n:, 2].mean()


def test_hair_like_polylines_stay_separated():
    # two crossing polylines, one driven through the other
    t = np.linspace(0, 1, 6)
    la = np.stack([t * 0.02, np.zeros_like(t), np.zeros_like(t)], 1)
    lb = np.stack([np.full_like(t, 0.01), t * 0.02 - 0.01, np.full_like(t, 2e-3)], 1)
    x = np.vstack([la, lb])
    edges = np.array([(i, i + 1) for i in range(5)] + [(6 + i, 7 + i) for i in range(5)], np.int32)
    xt = x.copy()
    xt[6:, 2] -= 6e-3
    w = np.ones(len(x))
    w[[0, 6]] = 0
    xt[[0, 6]] = x[[0, 6]]
    traj, s = _safety_run(x, xt, np.zeros((0, 3), np.int32), edges, w, iters=60)
    xf = traj[-1]
    for e in range(5):
        for g in range(5, 10):
            d2 = exact.seg_seg_d2(*(xf[i] for i in (*edges[e], *edges[g])))
            assert d2 > 0


# ------------------------------------------------------------ continuous test

def _rand_frame(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q


def test_ccd_vertex_through_triangle_hits_at_the_crossing_time():
    rng = np.random.default_rng(11)
    for trial in range(100):
        R = _rand_frame(rng)
        tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float) * 0.01
        bc = rng.dirichlet([2, 2, 2])
        p_cross = bc @ tri
        t_star = rng.uniform(0.1, 0.9)
        vel = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), -1.0]) * 0.004
        p0 = p_cross - t_star * vel
        q = np.vstack([p0, tri]) @ R.T + rng.normal(size=3) * 0.02
        dq = np.vstack([vel, np.zeros((3, 3))]) @ R.T
        hit, t = oracle.ccd_hit(q, dq, ee=False)
        assert hit and abs(t - t_star) < 1e-6, (trial, hit, t, t_star)


def test_ccd_edges_crossing_hit_and_clear_misses_do_not():
    rng = np.random.default_rng(12)
    for trial in range(100):
        R = _rand_frame(rng)
        t_star = rng.uniform(0.1, 0.9)
        e1 = np.array([[-1, 0, 0], [1, 0, 0]], float) * 0.005
        e2 = np.array([[0, -1, 0], [0, 1, 0]], float) * 0.005
        s = rng.uniform(-0.6, 0.6)
        e2[:, 0] += s * 0.005
        vel = np.array([0.0, 0.0, -0.004])
        e1_0 = e1 - t_star * vel
        q = np.vstack([e1_0, e2]) @ R.T
        dq = np.vstack([vel, vel, [0, 0, 0], [0, 0, 0]]) @ R.T
        hit, t = oracle.ccd_hit(q, dq, ee=True)
        assert hit and abs(t - t_star) < 1e-6
        # the same motion shifted sideways beyond the other edge's end never touches
        q_miss = q.copy()
        q_miss[2:] += (np.array([0.02, 0, 0]) @ R.T)
        hit, _ = oracle.ccd_hit(q_miss, dq, ee=True)
        ts = np.linspace(0, 1, 4001)
        dmin = min(oracle.seg_seg_d2(*(q_miss + t_ * dq))[0] for t_ in ts) ** 0.5
        assert dmin > 1e-3 and not hit


def test_ccd_contact_at_the_end_of_the_piece():
    # the vertex arrives exactly on the triangle at t = 1; stopping 0.1 mm short misses
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float) * 0.01
    q = np.vstack([[0.004, 0.004, 0.002], tri])
    dq = np.zeros((4, 3))
    dq[0] = [0.0, 0.0, -0.002]
    hit, t = oracle.ccd_hit(q, dq, ee=False)
    assert hit and abs(t - 1.0) < 1e-12
    dq[0] = [0.0, 0.0, -0.0019]
    hit, _ = oracle.ccd_hit(q, dq, ee=False)
    assert not hit


# ---------------------------------------------------------------- projected Jacobi
# (Sec. 4.3.2: one projected Jacobi iteration in place of the Gauss-Seidel sweep,
# with an under-relaxation factor omega; the per-vertex sums are plain binary64 sums
# in row order)

def test_jacobi_single_row_settles_at_delta():
    # one contact row: Jacobi with omega = 1 is the same projection
    x = np.array([[0.2, 0.2, 0.005], [0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    xt = x.copy()
    xt[0, 2] = -0.005
    s = oracle.Scene(np.array([1.0, 0, 0, 0]), [[1, 2, 3]], [[1, 2], [2, 3], [1, 3]],
                     max_iters=100, backward="jacobi", omega=1.0)
    out, n, tr = s.run(x, xt, trace_cap=100)
    assert abs(out[0, 2] - DELTA) < 1e-15
    assert np.array_equal(out[1:], x[1:])
    assert all(t["n_colors"] == 0 for t in tr)  # no colouring


def test_jacobi_opposite_rows_cancel_exactly():
    # a free vertex midway between two static parallel triangles, 0.5 mm from each:
    # the two rows push with equal and opposite updates from the same y, their
    # fixed-point sum is exactly zero, and the vertex stays where it is (Gauss-Seidel
    # would move it: the second row sees the first row's push)
    h = 0.5e-3
    x = np.array([[0.2, 0.2, 0.0],
                  [0, 0, -h], [1, 0, -h], [0, 1, -h],
                  [0, 0, h], [1, 0, h], [0, 1, h]], float)
    w = np.array([1.0, 0, 0, 0, 0, 0, 0])
    tris = [[1, 2, 3], [4, 5, 6]]
    jac = oracle.Scene(w, tris, [], max_iters=5, backward="jacobi", omega=1.0, edge_len=0)
    out, n, tr = jac.run(x, x.copy(), trace_cap=5)
    assert tr[0]["n_a"] == 2
    assert np.array_equal(out, x)
    gs = oracle.Scene(w, tris, [], max_iters=5, edge_len=0)
    gs.begin(x, x.copy())
    gs.iterate()
    assert gs.state()[1][0, 2] != 0.0  # the sequential sweep is not symmetric


def test_jacobi_result_depends_on_row_order_only_by_rounding():
    # the same step with the pair list handed over in two different orders: every row
    # reads the same y, so the orders differ only in the rounding of the sums
    x, xt, tris, edges = _two_patches()
    w = np.ones(len(x))
    outs = []
    for order in (1, -1):
        s = oracle.Scene(w, tris, edges, max_iters=30, backward="jacobi", omega=0.5)
        s.begin(x, xt)
        s.iterate()  # first iteration: search, then P' in the search's order
        X, Y, R, D = s.state()
        P = s.P()[::order].copy()
        s.set_state(X, Y, R, D, P)
        for _ in range(5):
            s.iterate()
        outs.append(s.state())
    for a, b in zip(outs[0], outs[1]):
        assert np.allclose(np.asarray(a), np.asarray(b), rtol=0, atol=1e-15)


@pytest.mark.parametrize("omega", [0.5, 1.0])
def test_jacobi_two_patches_pass_through_is_resolved_safely(omega):
    x, xt, tris, edges = _two_patches()
    traj, s = _safety_run(x, xt, tris, edges, np.ones(len(x)), iters=60, backward="jacobi",
                          omega=omega)
    xf = traj[-1]
    assert not exact.mesh_self_intersects(xf, tris.tolist(), edges.tolist())
    n = len(x) // 2
    assert xf[:n, 2].mean() < xf[n:, 2].mean()


# ---------------------------------------------------------------- input check
# (x^t must lie in the free space, Sec. 3; the check is an option of the step)

def test_seg_tri_meet_matches_exact_rational():
    rng = np.random.default_rng(7)
    n_meet = 0
    for _ in range(3000):
        a, b, c = rng.normal(size=(3, 3))
        p, q = rng.normal(size=(2, 3)) * 0.8
        want = exact.seg_tri_intersect(p, q, a, b, c)
        got = oracle.seg_tri_meet(p, q, a, b, c)
        assert got == want
        n_meet += want
    assert 100 < n_meet < 2900  # both outcomes well represented


def test_seg_tri_meet_touching_and_coplanar_cases():
    a, b, c = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    # an endpoint on the triangle's interior: touching
    assert oracle.seg_tri_meet([0.2, 0.2, 0.0], [0.2, 0.2, 1.0], a, b, c)
    # an endpoint on a side
    assert oracle.seg_tri_meet([0.5, 0.0, 0.0], [0.5, -1.0, 1.0], a, b, c)
    # just above the plane, off the triangle
    assert not oracle.seg_tri_meet([0.2, 0.2, 1e-6], [0.2, 0.2, 1.0], a, b, c)
    # in the plane, crossing the triangle / far away in the plane
    assert oracle.seg_tri_meet([-1.0, 0.3, 0.0], [2.0, 0.3, 0.0], a, b, c)
    assert not oracle.seg_tri_meet([2.0, 2.0, 0.0], [3.0, 2.5, 0.0], a, b, c)


def test_validate_scenes():
    tol = 1e-9
    # separated patches and the small folded cloth / cubes at x^t: free
    x, xt, tris, edges = _two_patches()
    s = oracle.Scene(np.ones(len(x)), tris, edges)
    s.begin(x, xt)
    assert s.validate(x, tol) == 0
    for cfg in (2, 3):
        sc = scenes.config(cfg, small=True)
        s = oracle.Scene(sc["w"], sc["tris"], sc["edges"])
        s.begin(sc["x"], sc["xt"])
        assert s.validate(sc["x"], tol) == 0
    # the upper patch tilted through the lower one: not free (the exact test agrees)
    n = len(x) // 2
    y = x.copy()
    y[n:, 2] += (y[n:, 1] - y[n:, 1].mean()) * 1.5 - 1e-3
    assert exact.mesh_self_intersects(y, tris.tolist(), edges.tolist())
    s = oracle.Scene(np.ones(len(x)), tris, edges)
    s.begin(y, y)
    assert s.validate(y, tol) == 1
    # a needle through a large triangle, far from its corners and sides: only the
    # edge-triangle part of the check can see it
    xn = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0.25, 0.25, -0.5], [0.25, 0.25, 0.5]])
    s = oracle.Scene(np.ones(5), [[0, 1, 2]], [[0, 1], [1, 2], [0, 2], [3, 4]])
    s.begin(xn, xn)
    assert s.search(xn, 0.2).size == 0  # no vertex-triangle or edge-edge pair nearby
    assert s.validate(xn, tol) == 1
    xn[4, 2] = -0.1  # now below the triangle: free
    s.begin(xn, xn)
    assert s.validate(xn, tol) == 0


# ------------------------------------------------- vertex-vertex pairs (sand)

def test_vv_search_grid_equals_brute_force_and_exact_threshold():
    """Particles (vertices in no triangle or edge) pair with each other only; the
    grid search equals the all-pairs loop and a threshold decided in exact
    arithmetic over a universe built here."""
    rng = np.random.default_rng(11)
    xp = rng.uniform(0.0, 0.012, size=(60, 3))
    xm, tm, em = scenes.grid_cloth(3, 3, 4e-3)
    x = np.vstack([xp, xm + [0.002, 0.002, 0.006]])
    tris, edges = tm + len(xp), em + len(xp)
    s = oracle.Scene(np.ones(len(x)), tris, edges)
    assert np.array_equal(s.particles(), np.arange(len(xp)))
    U = _universe_keys(len(x), tris.tolist(), edges.tolist())
    for dmax in (2e-3, 4e-3):
        g = set(int(k) for k in s.search(x, dmax))
        assert g == set(int(k) for k in s.search(x, dmax, brute=True))
        want = set(k for k in U if _pair_exact(k, x, tris, edges)[1] < Fr(dmax) ** 2)
        assert g == want
        vv = [k for k in g if (k >> 62) & 1 and not k >> 63]
        assert vv and all(((k >> 32) & 0x3FFFFFFF) < (k & 0xFFFFFFFF) < len(xp) for k in vv)


def test_vv_row_closed_form_and_gradient():
    """c = |x_a - x_b|/delta - 1 (Sec. 4.1) at x: c0, J = grad c by central
    differences, A = (w_a + w_b)/delta^2 (|u| = 1)."""
    rng = np.random.default_rng(12)
    for _ in range(5):
        x = rng.normal(size=(2, 3)) * 4e-4
        w = rng.uniform(0.5, 2.0, size=2)
        s = _scene(2, w=w)
        k = oracle.vv_key(0, 1)
        r = s.contact_row(x, k)
        assert r["kind"] == 1 and list(r["v"]) == [0, 1, -1, -1]
        d = np.linalg.norm(x[0] - x[1])
        assert rel_close(r["c0"], d / DELTA - 1)
        f = lambda y: np.linalg.norm(y[0] - y[1]) / DELTA - 1  # noqa: E731
        g = _fd_grad(f, x, [0, 1], h=1e-10)
        assert np.allclose(r["J"][:2], g[:2], rtol=1e-5, atol=1e-3)
        assert np.array_equal(r["J"][2:], np.zeros((2, 3)))
        assert rel_close(1.0 / r["inv_a"], (w[0] + w[1]) / DELTA ** 2, rtol=1e-12)
    # coincident particles carry no row
    assert _scene(2).contact_row(np.zeros((2, 3)), oracle.vv_key(0, 1))["kind"] == 2


def test_particle_through_static_particle_settles_at_delta():
    """A particle driven straight through a static one stops at distance delta on
    its own side (the renewed linearisation's fixed point), like the vertex and the
    static triangle."""
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.005]])
    xt = x.copy()
    xt[1, 2] = -0.005
    s = oracle.Scene(np.array([0.0, 1.0]), np.zeros((0, 3), np.int32),
                     np.zeros((0, 2), np.int32), max_iters=200)
    out, n, tr = s.run(x, xt, trace_cap=200)
    assert abs(out[1, 2] - DELTA) < 1e-15
    assert out[1, 0] == 0.0 and out[1, 1] == 0.0
    assert np.array_equal(out[0], x[0])
    assert tr[-1]["r_inf"] < 1e-4


def _vv_min_dist2_exact(q, dq):
    """Exact minimum over t in [0,1] of |(q0 - q1) + t (dq0 - dq1)|^2."""
    p = [Fr(float(q[0, c])) - Fr(float(q[1, c])) for c in range(3)]
    d = [Fr(float(dq[0, c])) - Fr(float(dq[1, c])) for c in range(3)]
    dd = sum(v * v for v in d)
    t = Fr(0) if dd == 0 else min(max(-sum(a * b for a, b in zip(p, d)) / dd, Fr(0)), Fr(1))
    return sum((a + t * b) ** 2 for a, b in zip(p, d)), t


def test_ccd_vv_closest_approach():
    """The vertex-vertex continuous test against the exact closest approach: head-on
    crossings hit at the meeting time, passes 2 eta apart miss, eta/2 apart hit."""
    rng = np.random.default_rng(13)
    eta = 1e-12
    for _ in range(20):
        R = _rand_frame(rng)
        c = rng.normal(size=3) * 1e-2
        t0 = rng.uniform(0.1, 0.9)
        for off, want in ((0.0, True), (2 * eta, False), (0.5 * eta, True), (1e-9, False)):
            a0 = c + R @ np.array([-1e-3, off, 0.0])
            b0 = c + R @ np.array([1e-3, 0.0, 0.0])
            va = R @ np.array([1e-3 / t0, 0.0, 0.0])
            q = np.stack([a0, b0])
            dq = np.stack([va, -va])
            d2, t = _vv_min_dist2_exact(q, dq)
            hit, th = oracle.ccd_hit(q, dq, 2, eta)
            if abs(float(d2) - eta * eta) > 1e-3 * eta * eta:
                assert hit == (d2 <= Fr(eta) ** 2) == want
            if hit:
                assert abs(th - float(t)) < 1e-9
    # parallel motion: t = 0
    q = np.array([[0.0, 0, 0], [1e-3, 0, 0]])
    assert oracle.ccd_hit(q, np.ones((2, 3)), 2)[0] is False


def test_sand_pile_is_resolved_safely():
    """A small particle pile falling on a static ground: every iteration keeps the
    lemma of Sec. 5 and the reuse bound in exact arithmetic, and the end state has
    no two particles coincident and every particle above the ground."""
    sc = scenes.sand_pile(3, 3, 3, ground=3)
    x, xt, w, tris, edges = sc["x"], sc["xt"], sc["w"], sc["tris"], sc["edges"]
    traj, s = _safety_run(x, xt, tris, edges, w, iters=80)
    assert len(traj) <= 80  # the stop test held before the cap
    xf = traj[-1]
    n = 27
    for a in range(n):
        for b in range(a + 1, n):
            assert _pair_exact(oracle.vv_key(a, b), xf, tris, edges)[1] > 0
        assert xf[a, 2] > 0


def test_ccd_all_checks_every_pair_and_changes_nothing():
    """With the continuous test on every pair of P' (a check of the lemma of Sec. 5),
    every pair is tested, none is in contact, and the path is the same."""
    x, xt, tris, edges = _two_patches()
    a = oracle.Scene(np.ones(len(x)), tris, edges, max_iters=60)
    b = oracle.Scene(np.ones(len(x)), tris, edges, max_iters=60, ccd_all=1)
    xa, na, ta = a.run(x, xt, trace_cap=60)
    xb, nb, tb = b.run(x, xt, trace_cap=60)
    assert na == nb and np.array_equal(xa, xb)
    for ia, ib in zip(ta, tb):
        assert ib["ccd_fail"] == ib["n_pf"] and ib["ccd_hits"] == 0
        assert ia["ccd_fail"] <= ib["ccd_fail"]


# ------------------------------------------------------------ normal flow

def test_normal_flow_flat_grid_moves_interior_by_beta_exactly():
    """Flat dyadic grid: the vertex normals are (0, 0, 1) exactly and the cotangent
    Laplacian of a flat interior vertex vanishes (linear precision), so vertices
    three rings from the border move by exactly beta after three smoothing steps."""
    n = 9
    x, tris, _ = scenes.grid_cloth(n, n, 0.25)
    beta, alpha = 2.0 ** -7, 2.0 ** -10
    y = oracle.normal_flow(x, tris, beta, alpha, 3)
    ij = np.arange(n * n)
    i, j = ij // n, ij % n
    deep = (i >= 3) & (i <= n - 4) & (j >= 3) & (j <= n - 4)
    assert deep.sum() == 9
    assert np.array_equal(y[deep], x[deep] + [0.0, 0.0, beta])
    # the border is smoothed inwards (boundary vertices have a non-zero Laplacian)
    assert np.abs(y[~deep][:, :2] - x[~deep][:, :2]).max() > 0


def test_normal_flow_equilateral_triangle_closed_form():
    """One equilateral triangle of side s: cot 60 = 1/sqrt(3), barycentric area
    sqrt(3) s^2 / 12, so one step moves a corner by alpha * (2 / sqrt(3)) * (centroid
    offset * 3) / (2 * area / 3)."""
    s_ = 0.3
    x = np.array([[0.0, 0.0, 0.0], [s_, 0.0, 0.0], [0.5 * s_, 0.5 * np.sqrt(3.0) * s_, 0.0]])
    alpha = 1e-3
    y = oracle.normal_flow(x, [[0, 1, 2]], 0.0, alpha, 1)
    A = np.sqrt(3.0) * s_ * s_ / 4.0 / 3.0
    for v in range(3):
        q, r = [u for u in range(3) if u != v]
        L = ((x[q] - x[v]) + (x[r] - x[v])) / np.sqrt(3.0)
        want = x[v] + alpha * L / (2.0 * A)
        assert np.allclose(y[v], want, rtol=0, atol=1e-15)


def test_normal_flow_sphere_normals_and_mean_curvature():
    """Icosphere of radius R: vertex normals are radial to within the mesh's
    facet angle, y_0 sits beta outside, and the cotangent Laplacian of the positions
    is the mean-curvature normal -2/R n (to discretisation error)."""
    R = 0.1
    xs, ts = scenes.icosphere(3, R)[:2]
    nrm = xs / np.linalg.norm(xs, axis=1, keepdims=True)
    beta = 2e-3
    y0 = oracle.normal_flow(xs, ts, beta, 0.0, 0)
    assert np.allclose(np.linalg.norm(y0, axis=1), R + beta, rtol=0, atol=2e-5)
    d = y0 - xs
    assert np.degrees(np.arccos(np.clip((d / beta * nrm).sum(1), -1, 1))).max() < 2.0
    a = 1e-8
    L = (oracle.normal_flow(xs, ts, 0.0, a, 1) - xs) / a
    ln = (L * nrm).sum(1)
    assert abs(ln.mean() - (-2.0 / R)) < 0.01 * (2.0 / R)
    assert np.linalg.norm(L - ln[:, None] * nrm, axis=1).max() < 0.05 * (2.0 / R)


def test_normal_flow_rejects_bad_index():
    with pytest.raises(ValueError):
        oracle.normal_flow(np.zeros((3, 3)), [[0, 1, 3]], 0.1, 0.1, 1)


# ------------------------------------------------------ continuous test: ends, coplanar

def test_ccd_contact_within_eta_at_either_end_of_the_piece():
    # a vertex 0.5 pm above the face at t = 0 (below eta = 1 pm), moving away: a
    # contact at t = 0; the mirrored motion arriving 0.5 pm above the face at t = 1
    # reaches eta just before the end of the piece; V(t) keeps its sign on both
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float) * 0.01
    q = np.vstack([[0.003, 0.003, 5e-13], tri])
    dq = np.zeros((4, 3))
    dq[0] = [0.0, 0.0, 1e-3]
    hit, t = oracle.ccd_hit(q, dq, ee=False)
    assert hit and t == 0.0
    q2 = np.vstack([[0.003, 0.003, 1e-3 + 5e-13], tri])
    dq[0] = [0.0, 0.0, -1e-3]
    hit, t = oracle.ccd_hit(q2, dq, ee=False)
    assert hit and 1.0 - 1e-9 < t <= 1.0
    # 2 pm instead: no contact on either piece
    q[0, 2] = 2e-12
    dq[0] = [0.0, 0.0, 1e-3]
    assert not oracle.ccd_hit(q, dq, ee=False)[0]


def test_ccd_coplanar_pieces():
    # the four points stay in one plane (V(t) = 0 for every t), so the coplanarity
    # cubic carries no information: a vertex sliding in the face's plane across an
    # edge into the face, and an edge sliding in the plane of another across it, are
    # contacts; the same slides stopping 0.1 mm short are not
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float) * 0.01
    q = np.vstack([[0.003, -0.002, 0.0], tri])
    dq = np.zeros((4, 3))
    dq[0] = [0.0, 0.004, 0.0]
    hit, t = oracle.ccd_hit(q, dq, ee=False)
    assert hit and abs(t - 0.5) < 1e-6
    dq[0] = [0.0, 0.0019, 0.0]
    assert not oracle.ccd_hit(q, dq, ee=False)[0]
    e = np.array([[-0.005, 0.0, 0.0], [0.005, 0.0, 0.0], [0.0, -0.005, 0.0], [0.0, -0.003, 0.0]])
    dq = np.zeros((4, 3))
    dq[2] = dq[3] = [0.0, 0.006, 0.0]
    hit, t = oracle.ccd_hit(e, dq, ee=True)
    assert hit and abs(t - 0.5) < 1e-6
    dq[2] = dq[3] = [0.0, 0.0029, 0.0]
    assert not oracle.ccd_hit(e, dq, ee=True)[0]


def test_ccd_clearance_matches_sampled_minimum_distance():
    # random short pieces of random vertex-triangle and edge-edge pairs: a piece is
    # cleared exactly when the distance stays above eta; the minimum over a fine
    # sampling of t (an upper bound of the true minimum) must exceed eta on cleared
    # pieces, and pieces whose sampled minimum is far below eta must hit
    rng = np.random.default_rng(21)
    for trial in range(300):
        ee = bool(trial % 2)
        q = rng.normal(size=(4, 3)) * 0.003
        dq = rng.normal(size=(4, 3)) * 0.003
        hit, t = oracle.ccd_hit(q, dq, ee=ee)
        ts = np.linspace(0, 1, 2001)
        f = oracle.seg_seg_d2 if ee else oracle.pt_tri_d2
        d = np.array([f(*(q + t_ * dq))[0] for t_ in ts]) ** 0.5
        if d.min() < 1e-13:
            assert hit
        if not hit:
            assert d.min() > 1e-12


# ------------------------------------------------------ whole steps: safety in FP64

def _run_checked(sc, **over):
    p = dict(sc["params"])
    p.update(over)
    s = oracle.Scene(sc["w"], sc["tris"], sc["edges"], **p)
    out, n, tr = s.run(sc["x"], sc["xt"], trace_cap=p.get("max_iters", 512))
    return s, out, n, tr


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 6])
def test_small_configs_run_to_their_end_intersection_free(cfg):
    # the whole step, to the stop test or L, on the small variant of each workload:
    # no pair of P' is left uncertified by the motion bound in any iteration (the
    # lemma of Sec. 5 holds for the rounded positions), nothing is sent back, and the
    # final state is free in exact arithmetic with no pair within eta
    sc = scenes.config(cfg, small=True)
    s, out, n, tr = _run_checked(sc)
    assert all(t["ccd_fail"] == 0 and t["ccd_hits"] == 0 and t["n_back"] == 0 for t in tr)
    et, ee = exact.touching_pairs(out, sc["tris"], sc["edges"])
    assert et == [] and ee == []
    assert len(s.search(out, 1e-12)) == 0


def test_mid_size_cube_scene_runs_to_its_end_intersection_free():
    # 4 cubes of 8^3 cells: the scene whose former output met itself
    sc = scenes.stacked_cubes(4, 8)
    s, out, n, tr = _run_checked(sc)
    assert all(t["ccd_fail"] == 0 and t["n_back"] == 0 for t in tr)
    et, ee = exact.touching_pairs(out, sc["tris"], sc["edges"])
    assert et == [] and ee == []


def test_lemma_holds_exactly_near_contact_on_the_crumpling_cloth():
    # cloth over the sphere (small): over the first 150 iterations, every pair whose
    # distance fell below D^(l) satisfies the lemma of Sec. 5 in exact rational
    # arithmetic for the rounded positions; this window covers pairs driven from
    # millimetres down to the 1e-11 m scale where the forward step's check of the
    # rounded move freezes their vertices
    sc = scenes.config(1, small=True)
    p = dict(sc["params"])
    p["max_iters"] = 150
    s = oracle.Scene(sc["w"], sc["tris"], sc["edges"], **p)
    s.begin(sc["x"], sc["xt"])
    tris, edges = sc["tris"], sc["edges"]
    smallest = 1.0
    for l in range(p["max_iters"]):
        X0 = s.state()[0]
        stop, it = s.iterate()
        X1 = s.state()[0]
        m = np.linalg.norm(X1 - X0, axis=1)
        for k in s.P():
            k = int(k)
            a, b = (k >> 32) & 0x3FFFFFFF, k & 0xFFFFFFFF
            if k & oracle.KEY_EE:
                v = [*edges[a], *edges[b]]
                d = oracle.seg_seg_d2(*X0[v])[0] ** 0.5
            else:
                v = [a, *tris[b]]
                d = oracle.pt_tri_d2(*X0[v])[0] ** 0.5
            smallest = min(smallest, d)
            mm = max(m[i] for i in v)
            if d > 1e-6 and 2.0 * mm < 0.999 * d:
                continue  # far from the rounding level: the binary64 check is decisive
            v, d2 = _pair_exact(k, X0, tris, edges)
            m2 = max(sum((Fr(float(X1[i, c])) - Fr(float(X0[i, c]))) ** 2 for c in range(3))
                     for i in v)
            assert 4 * m2 < d2, (l, hex(k))
        if stop:
            break
    assert smallest < 1e-9  # the window reaches the near-contact regime


def test_unguarded_forward_step_is_caught_by_the_certificate():
    # the forward step exactly as Eq. eq:forward2, without the check of the rounded
    # move: on the crumpling cloth some rounded moves break the lemma; the certificate
    # finds those pieces, sends their vertices back to x^(l), and the output is still
    # free in exact arithmetic
    sc = scenes.config(1, small=True)
    s, out, n, tr = _run_checked(sc, max_iters=600, unguarded=1)
    assert sum(t["n_back"] for t in tr) > 0
    et, ee = exact.touching_pairs(out, sc["tris"], sc["edges"])
    assert et == [] and ee == []


# ------------------------------------------- CCD-based step-size scheme (Sec. 5.1)

def test_ccd_step_stops_a_vertex_short_of_the_contact():
    # a free vertex 1.5 mm above a static triangle, its target 2 mm below it; the row
    # is not active (d > delta), so y stays the target. The CCD-based step bounds the
    # vertex by 0.45 D^(l) = 1.8 mm, finds the contact at 1.5 mm of that piece and
    # scales the step by gamma t*: the vertex stops at (1 - gamma) 1.5 mm above the
    # face. The CCD-free step moves it by 0.45 D_i = 0.675 mm.
    h0 = 1.5e-3
    x = np.array([[0.002, 0.002, h0], [0, 0, 0], [0.01, 0, 0], [0, 0.01, 0]], float)
    xt = x.copy()
    xt[0, 2] = -2e-3
    w = np.array([1.0, 0, 0, 0])
    ccd = oracle.Scene(w, [[1, 2, 3]], [], max_iters=1, ccd_step=1, edge_len=0)
    ccd.begin(x, xt)
    _, it = ccd.iterate()
    z = ccd.state()[0][0, 2]
    assert it["n_scaled"] == 1 and it["ccd_hits"] == 1 and it["n_back"] == 0
    assert abs(z - (1.0 - 0.9) * h0) < 1e-9
    free = oracle.Scene(w, [[1, 2, 3]], [], max_iters=1, edge_len=0)
    free.begin(x, xt)
    free.iterate()
    assert abs(free.state()[0][0, 2] - (h0 - 0.45 * h0)) < 1e-15


@pytest.mark.parametrize("cfg", [2, 3, 4, 6])
def test_ccd_step_small_configs_end_intersection_free(cfg):
    # the CCD-based scheme on the small workloads: its final states are free in exact
    # arithmetic, nothing had to be sent back, and it needs no more iterations than
    # the CCD-free scheme (its steps are bounded by D^(l), not by D_i)
    sc = scenes.config(cfg, small=True)
    s, out, n, tr = _run_checked(sc, ccd_step=1)
    assert all(t["n_back"] == 0 for t in tr)
    et, ee = exact.touching_pairs(out, sc["tris"], sc["edges"])
    assert et == [] and ee == []
    n_free = _run_checked(sc)[2]
    assert n <= n_free
