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
