"""Exact rational geometry used to pin the oracle (Fractions, no floating point).

Distances are found by enumerating every KKT candidate of the convex quadratic
program min |q - p|^2 over the simplex or the parameter square, solved exactly;
this is a different method from the candidate list the oracle evaluates in
binary64.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from itertools import combinations


def F3(v):
    return [Fr(float(c)) for c in v]


def sub(a, b):
    return [a[0] - b[0], a[1] - b[1], a[2] - b[2]]


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _seg_point_param(p, u, v):
    uv = sub(v, u)
    l2 = dot(uv, uv)
    if l2 == 0:
        return Fr(0)
    t = dot(sub(p, u), uv) / l2
    return min(Fr(1), max(Fr(0), t))


def _point_on(a, dirs, params):
    q = list(a)
    for d, s in zip(dirs, params):
        q = [q[k] + s * d[k] for k in range(3)]
    return q


def pt_tri_d2(p, a, b, c):
    """Exact min over u,v>=0, u+v<=1 of |a + u(b-a) + v(c-a) - p|^2."""
    p, a, b, c = F3(p), F3(a), F3(b), F3(c)
    e1, e2, r = sub(b, a), sub(c, a), sub(p, a)
    cands = []
    # interior stationary point
    A, B, C = dot(e1, e1), dot(e1, e2), dot(e2, e2)
    det = A * C - B * B
    if det != 0:
        d1, d2 = dot(e1, r), dot(e2, r)
        u = (d1 * C - d2 * B) / det
        v = (A * d2 - B * d1) / det
        if u >= 0 and v >= 0 and u + v <= 1:
            cands.append(_point_on(a, [e1, e2], [u, v]))
    # edges (1D exact QPs) and corners
    for u0, v0 in ((a, b), (b, c), (c, a)):
        t = _seg_point_param(p, u0, v0)
        cands.append(_point_on(u0, [sub(v0, u0)], [t]))
    for q in (a, b, c):
        cands.append(q)
    return min(dot(sub(p, q), sub(p, q)) for q in cands)


def seg_seg_d2(a, b, c, e):
    """Exact min over (s,t) in [0,1]^2 of |a + s(b-a) - c - t(e-c)|^2."""
    a, b, c, e = F3(a), F3(b), F3(c), F3(e)
    d1, d2, r = sub(b, a), sub(e, c), sub(a, c)
    A, B, C = dot(d1, d1), dot(d1, d2), dot(d2, d2)
    D, E = dot(d1, r), dot(d2, r)
    pairs = []
    det = A * C - B * B
    if det != 0:
        s = (B * E - C * D) / det
        t = (A * E - B * D) / det
        if 0 <= s <= 1 and 0 <= t <= 1:
            pairs.append((s, t))
    # boundary of the square: one parameter fixed at 0 or 1, exact 1D minimiser
    for s0 in (Fr(0), Fr(1)):
        p = _point_on(a, [d1], [s0])
        pairs.append((s0, _seg_point_param(p, c, e)))
    for t0 in (Fr(0), Fr(1)):
        q = _point_on(c, [d2], [t0])
        pairs.append((_seg_point_param(q, a, b), t0))
    best = None
    for s, t in pairs:
        p = _point_on(a, [d1], [s])
        q = _point_on(c, [d2], [t])
        dd = dot(sub(p, q), sub(p, q))
        best = dd if best is None else min(best, dd)
    return best


def orient3d(a, b, c, d):
    return dot(sub(b, a), cross(sub(c, a), sub(d, a)))


def seg_tri_intersect(p, q, a, b, c):
    """Exact test: does the closed segment [p,q] touch the closed triangle (a,b,c)?
    Non-degenerate triangles only."""
    p, q, a, b, c = F3(p), F3(q), F3(a), F3(b), F3(c)
    s1, s2 = orient3d(a, b, c, p), orient3d(a, b, c, q)
    if s1 == 0 and s2 == 0:
        # coplanar: touch if either endpoint inside or the segment crosses an edge;
        # exact distance 0 decides it
        return (pt_tri_d2(p, a, b, c) == 0 or pt_tri_d2(q, a, b, c) == 0 or
                any(seg_seg_d2(p, q, u, v) == 0 for u, v in ((a, b), (b, c), (c, a))))
    if (s1 > 0 and s2 > 0) or (s1 < 0 and s2 < 0):
        return False
    o1 = orient3d(p, q, a, b)
    o2 = orient3d(p, q, b, c)
    o3 = orient3d(p, q, c, a)
    return (o1 >= 0 and o2 >= 0 and o3 >= 0) or (o1 <= 0 and o2 <= 0 and o3 <= 0)


def mesh_self_intersects(x, tris, edges):
    """Exact: any edge touching a triangle it shares no vertex with, or any two
    edges sharing no vertex at distance 0 (polylines)."""
    for e in edges:
        for t in tris:
            if set(e) & set(t):
                continue
            if seg_tri_intersect(x[e[0]], x[e[1]], x[t[0]], x[t[1]], x[t[2]]):
                return True
    for e, g in combinations(range(len(edges)), 2):
        if set(edges[e]) & set(edges[g]):
            continue
        if seg_seg_d2(*(x[i] for i in (*edges[e], *edges[g]))) == 0:
            return True
    return False


# ------------------------------------------------------------------ fast exact test
#
# The same exact predicate as mesh_self_intersects, for meshes of thousands of
# elements: candidate pairs come from axis-aligned boxes on a uniform grid, each
# orientation is evaluated in binary64 together with a bound on its rounding error,
# and only pairs whose signs the bound leaves undecided are evaluated in Fractions.

def _orient_fp(a, b, c, d):
    """det[b-a, c-a, d-a] in binary64 and a bound on its rounding error (vectorised)."""
    import numpy as np
    u, v, w = b - a, c - a, d - a
    det = (u[:, 0] * (v[:, 1] * w[:, 2] - v[:, 2] * w[:, 1])
           + u[:, 1] * (v[:, 2] * w[:, 0] - v[:, 0] * w[:, 2])
           + u[:, 2] * (v[:, 0] * w[:, 1] - v[:, 1] * w[:, 0]))
    perm = (np.abs(u[:, 0]) * (np.abs(v[:, 1] * w[:, 2]) + np.abs(v[:, 2] * w[:, 1]))
            + np.abs(u[:, 1]) * (np.abs(v[:, 2] * w[:, 0]) + np.abs(v[:, 0] * w[:, 2]))
            + np.abs(u[:, 2]) * (np.abs(v[:, 0] * w[:, 1]) + np.abs(v[:, 1] * w[:, 0])))
    # the differences b-a etc. are rounded too: bound the error by the magnitudes of
    # the inputs as well (a generous multiple of the unit roundoff)
    mag = np.maximum.reduce([np.abs(a).max(1), np.abs(b).max(1), np.abs(c).max(1),
                             np.abs(d).max(1)])
    err = 1e-14 * perm + 1e-14 * mag * (np.abs(u).max(1) + np.abs(v).max(1) +
                                        np.abs(w).max(1)) ** 2
    return det, err


def _box_pairs(lo1, hi1, lo2, hi2, margin):
    """Index pairs (i, j) whose boxes [lo1[i]-m, hi1[i]+m] and [lo2[j], hi2[j]] overlap."""
    import numpy as np
    if len(lo1) == 0 or len(lo2) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    lo1 = lo1 - margin
    hi1 = hi1 + margin
    ext = max(float((hi1 - lo1).max()), float((hi2 - lo2).max()), 1e-12)
    h = ext
    org = np.minimum(lo1.min(0), lo2.min(0))
    dim = np.floor((np.maximum(hi1.max(0), hi2.max(0)) - org) / h).astype(np.int64) + 1

    def cells(lo, hi):
        c0 = np.floor((lo - org) / h).astype(np.int64)
        c1 = np.floor((hi - org) / h).astype(np.int64)
        ids, own = [], []
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    c = c0 + np.array([dx, dy, dz])
                    ok = (c <= c1).all(1)
                    cid = (c[:, 0] * dim[1] + c[:, 1]) * dim[2] + c[:, 2]
                    ids.append(cid[ok])
                    own.append(np.nonzero(ok)[0])
        return np.concatenate(ids), np.concatenate(own)

    c2, o2 = cells(lo2, hi2)
    order = np.argsort(c2, kind="stable")
    c2, o2 = c2[order], o2[order]
    c1, o1 = cells(lo1, hi1)
    start = np.searchsorted(c2, c1, "left")
    stop = np.searchsorted(c2, c1, "right")
    cnt = stop - start
    ii = np.repeat(o1, cnt)
    base = np.repeat(start - np.cumsum(cnt) + cnt, cnt)
    jj = o2[base + np.arange(cnt.sum())]
    key = np.unique(ii * len(lo2) + jj)
    ii, jj = key // len(lo2), key % len(lo2)
    ok = ((lo1[ii] <= hi2[jj]) & (lo2[jj] <= hi1[ii])).all(1)
    return ii[ok], jj[ok]


def _seg_seg_dist_fp(a, b, c, e):
    """Binary64 segment-segment distances (vectorised): the minimum over the interior
    stationary point (when it lies in the unit square) and the four endpoint-to-
    segment distances."""
    import numpy as np

    def pt_seg(p, u, v):
        uv = v - u
        l2 = (uv * uv).sum(1)
        t = np.where(l2 > 0, ((p - u) * uv).sum(1) / np.where(l2 > 0, l2, 1), 0.0)
        t = np.clip(t, 0.0, 1.0)
        return np.linalg.norm(p - (u + t[:, None] * uv), axis=1)

    d1, d2, r = b - a, e - c, a - c
    A, B, C = (d1 * d1).sum(1), (d1 * d2).sum(1), (d2 * d2).sum(1)
    D, E = (d1 * r).sum(1), (d2 * r).sum(1)
    den = A * C - B * B
    ok = den > 0
    dd = np.where(ok, den, 1.0)
    s, t = (B * E - C * D) / dd, (A * E - B * D) / dd
    inside = ok & (s >= 0) & (s <= 1) & (t >= 0) & (t <= 1)
    dint = np.linalg.norm((a + s[:, None] * d1) - (c + t[:, None] * d2), axis=1)
    best = np.minimum.reduce([pt_seg(a, c, e), pt_seg(b, c, e), pt_seg(c, a, b),
                              pt_seg(e, a, b)])
    return np.where(inside, np.minimum(best, dint), best)


def touching_pairs(x, tris, edges, margin=1e-9):
    """Exact edge-triangle touches (closed edge and closed triangle sharing no vertex)
    and, for edges in no triangle, exact edge-edge touches. Returns two lists of
    index pairs (edge, triangle) and (edge, edge). Same predicate as
    mesh_self_intersects."""
    import numpy as np
    x = np.asarray(x, np.float64)
    tris = np.asarray(tris, np.int64).reshape(-1, 3)
    edges = np.asarray(edges, np.int64).reshape(-1, 2)
    et = []
    if len(tris) and len(edges):
        P, Q = x[edges[:, 0]], x[edges[:, 1]]
        A, B, C = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
        ie, it = _box_pairs(np.minimum(P, Q), np.maximum(P, Q),
                            np.minimum(np.minimum(A, B), C), np.maximum(np.maximum(A, B), C),
                            margin)
        share = np.zeros(len(ie), bool)
        for k in range(2):
            for m in range(3):
                share |= edges[ie, k] == tris[it, m]
        ie, it = ie[~share], it[~share]
        p, q, a, b, c = P[ie], Q[ie], A[it], B[it], C[it]
        sp, ep = _orient_fp(a, b, c, p)
        sq, eq = _orient_fp(a, b, c, q)
        sure_p, sure_q = np.abs(sp) > ep, np.abs(sq) > eq
        apart = sure_p & sure_q & (np.sign(sp) == np.sign(sq))
        o = [_orient_fp(p, q, a, b), _orient_fp(p, q, b, c), _orient_fp(p, q, c, a)]
        sure_o = np.all([np.abs(d) > e for d, e in o], axis=0)
        sg = np.stack([np.sign(d) for d, _ in o], 1)
        mixed = sure_o & (sg.max(1) > 0) & (sg.min(1) < 0)
        crossing = sure_p & sure_q & (np.sign(sp) != np.sign(sq)) & sure_o & ~mixed
        undecided = ~(apart | mixed | crossing)
        for k in np.nonzero(crossing)[0]:
            et.append((int(ie[k]), int(it[k])))
        for k in np.nonzero(undecided)[0]:
            e, t = edges[ie[k]], tris[it[k]]
            if seg_tri_intersect(x[e[0]], x[e[1]], x[t[0]], x[t[1]], x[t[2]]):
                et.append((int(ie[k]), int(it[k])))
    ee = []
    if len(edges):
        in_tri = np.zeros(len(x), bool)
        if len(tris):
            in_tri[tris.ravel()] = True
        poly = np.nonzero(~(in_tri[edges[:, 0]] & in_tri[edges[:, 1]]))[0]
        if len(poly) > 1:
            pe = edges[poly]
            P, Q = x[pe[:, 0]], x[pe[:, 1]]
            lo, hi = np.minimum(P, Q), np.maximum(P, Q)
            i1, i2 = _box_pairs(lo, hi, lo, hi, margin)
            ok = i1 < i2
            i1, i2 = i1[ok], i2[ok]
            share = np.zeros(len(i1), bool)
            for k in range(2):
                for m in range(2):
                    share |= pe[i1, k] == pe[i2, m]
            i1, i2 = i1[~share], i2[~share]
            # a binary64 distance clearly above the rounding level cannot be 0
            a, b = x[pe[i1, 0]], x[pe[i1, 1]]
            c, e = x[pe[i2, 0]], x[pe[i2, 1]]
            near = _seg_seg_dist_fp(a, b, c, e) <= 1e-9
            for k in np.nonzero(near)[0]:
                e1, g1 = pe[i1[k]], pe[i2[k]]
                if seg_seg_d2(x[e1[0]], x[e1[1]], x[g1[0]], x[g1[1]]) == 0:
                    ee.append((int(poly[i1[k]]), int(poly[i2[k]])))
    return et, ee
