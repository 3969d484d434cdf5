"""Seeded synthetic scenes for the two-way collision-handling step.

This module only builds inputs: positions x^t, targets x~, inverse masses,
triangles and edges. It holds none of the method's arithmetic, and both the
oracle tests and the GPU path take their inputs from here.

Units are metres and seconds. Every scene is a dict with
  x      (N,3) float64  intersection-free state x^t
  xt     (N,3) float64  time-integrated target x~ (the y^{[k+1]} of Alg. 1)
  w      (N,)  float64  inverse lumped mass (0 = static / pinned)
  tris   (F,3) int32
  edges  (E,2) int32    every triangle edge plus polyline segments
  params dict           overrides of the default parameters (Table 2)
  name   str
"""
from __future__ import annotations

import math

import numpy as np

GRAVITY = np.array([0.0, 0.0, -9.81])


# ----------------------------------------------------------------- topology

def edges_from_tris(tris: np.ndarray) -> np.ndarray:
    """Unique undirected edges (i<j) of a triangle list, sorted."""
    if len(tris) == 0:
        return np.zeros((0, 2), np.int32)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = np.unique(e, axis=0)
    return e.astype(np.int32)


def grid_cloth(nu: int, nv: int, spacing: float):
    """Regular nu x nv vertex grid in the plane z=0, one diagonal per quad.

    Returns (uv positions (N,3) with z=0, tris, edges); vertex id = row*nu + col.
    """
    cols, rows = np.meshgrid(np.arange(nu), np.arange(nv))
    x = np.stack([cols.ravel() * spacing, rows.ravel() * spacing,
                  np.zeros(nu * nv)], axis=1).astype(np.float64)
    tris = []
    for r in range(nv - 1):
        for c in range(nu - 1):
            v00 = r * nu + c
            v01 = v00 + 1
            v10 = v00 + nu
            v11 = v10 + 1
            tris.append((v00, v01, v11))
            tris.append((v00, v11, v10))
    tris = np.asarray(tris, np.int32).reshape(-1, 3)
    return x, tris, edges_from_tris(tris)


def icosphere(subdiv: int, radius: float):
    """Icosahedron refined `subdiv` times by edge midpoints, projected to the sphere."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(v, np.float64) / np.linalg.norm(v) for v in verts]
    for _ in range(subdiv):
        cache = {}
        new_faces = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    x = np.asarray(verts) * radius
    tris = np.asarray(faces, np.int32)
    return x, tris, edges_from_tris(tris)


def box_surface(cells: int, size: float):
    """Boundary surface of a cube [0,size]^3 cut into cells^3 cells (tet-mesh surface)."""
    n = cells + 1
    idx = {}
    verts = []

    def vid(i, j, k):
        key = (i, j, k)
        if key not in idx:
            idx[key] = len(verts)
            verts.append((i * size / cells, j * size / cells, k * size / cells))
        return idx[key]

    tris = []
    # each face: fixed axis value 0 or cells; outward orientation
    for axis in range(3):
        for side in (0, cells):
            a1, a2 = [a for a in range(3) if a != axis]
            for u in range(cells):
                for v in range(cells):
                    def P(du, dv):
                        c = [0, 0, 0]
                        c[axis] = side
                        c[a1] = u + du
                        c[a2] = v + dv
                        return vid(*c)
                    q00, q10, q11, q01 = P(0, 0), P(1, 0), P(1, 1), P(0, 1)
                    # orientation: flip on one side so normals point outward
                    flip = (side == 0) ^ (axis == 1)
                    if flip:
                        tris.append((q00, q11, q10))
                        tris.append((q00, q01, q11))
                    else:
                        tris.append((q00, q10, q11))
                        tris.append((q00, q11, q01))
    assert len(verts) == 6 * n * n - 12 * n + 8
    x = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int32)
    return x, tris, edges_from_tris(tris)


def lumped_inverse_mass(x: np.ndarray, tris: np.ndarray, edges: np.ndarray,
                        free: np.ndarray) -> np.ndarray:
    """Area-lumped (triangles) or length-lumped (edges, when no triangles) masses,
    inverted and normalised so that the mean over free vertices is 1; 0 where not free."""
    n = len(x)
    m = np.zeros(n)
    if len(tris):
        a = x[tris[:, 1]] - x[tris[:, 0]]
        b = x[tris[:, 2]] - x[tris[:, 0]]
        area = 0.5 * np.linalg.norm(np.cross(a, b), axis=1)
        for k in range(3):
            np.add.at(m, tris[:, k], area / 3.0)
    else:
        ln = np.linalg.norm(x[edges[:, 1]] - x[edges[:, 0]], axis=1)
        for k in range(2):
            np.add.at(m, edges[:, k], ln / 2.0)
    w = np.zeros(n)
    ok = free & (m > 0)
    w[ok] = 1.0 / m[ok]
    if ok.any():
        w[ok] /= w[ok].mean()
    return w


# ----------------------------------------------------------------- noise

class Perlin3:
    """Improved gradient noise (Perlin 2002) with a seeded permutation table.

    Written from the published construction: a 256-entry permutation, 12 edge
    gradients, quintic fade 6t^5-15t^4+10t^3 and trilinear blending.
    """

    _G = np.array([(1, 1, 0), (-1, 1, 0), (1, -1, 0), (-1, -1, 0),
                   (1, 0, 1), (-1, 0, 1), (1, 0, -1), (-1, 0, -1),
                   (0, 1, 1), (0, -1, 1), (0, 1, -1), (0, -1, -1)], np.float64)

    def __init__(self, rng: np.random.Generator):
        p = rng.permutation(256)
        self.perm = np.concatenate([p, p]).astype(np.int64)

    @staticmethod
    def _fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    def __call__(self, p: np.ndarray) -> np.ndarray:
        p = np.asarray(p, np.float64)
        fl = np.floor(p)
        i = fl.astype(np.int64) & 255
        f = p - fl
        u = self._fade(f)
        perm = self.perm
        out = np.zeros(len(p))
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    h = perm[perm[perm[i[:, 0] + dx] + i[:, 1] + dy] + i[:, 2] + dz] % 12
                    g = self._G[h]
                    d = f - np.array([dx, dy, dz], np.float64)
                    dot = (g * d).sum(axis=1)
                    wx = u[:, 0] if dx else 1.0 - u[:, 0]
                    wy = u[:, 1] if dy else 1.0 - u[:, 1]
                    wz = u[:, 2] if dz else 1.0 - u[:, 2]
                    out += wx * wy * wz * dot
        return out


# ----------------------------------------------------------------- scenes

def _merge(parts):
    xs, ts, es = [], [], []
    off = 0
    for x, t, e in parts:
        xs.append(x)
        ts.append(t + off)
        es.append(e + off)
        off += len(x)
    return np.concatenate(xs), np.concatenate(ts).astype(np.int32), \
        np.concatenate(es).astype(np.int32)


def cloth_over_sphere(n: int = 33, spacing: float = 0.01, subdiv: int = 3,
                      radius: float = 0.10, height: float = 0.12,
                      h: float = 1.0 / 30.0, vstd: float = 0.5, seed: int = 1001):
    """An n x n cloth 2 cm above a static icosphere; x~ = x + h(v + g h), v ~ N(0, vstd^2)."""
    xc, tc, ec = grid_cloth(n, n, spacing)
    xc[:, 0] -= 0.5 * (n - 1) * spacing
    xc[:, 1] -= 0.5 * (n - 1) * spacing
    xc[:, 2] = height
    xs, ts, es = icosphere(subdiv, radius)
    x, tris, edges = _merge([(xc, tc, ec), (xs, ts, es)])
    nc = len(xc)
    free = np.zeros(len(x), bool)
    free[:nc] = True
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, vstd, size=(nc, 3))
    xt = x.copy()
    xt[:nc] = x[:nc] + h * (v + GRAVITY * h)
    w = lumped_inverse_mass(x, tris, edges, free)
    return dict(name=f"cloth_sphere_{n}x{n}", x=x, xt=xt, w=w, tris=tris,
                edges=edges, params=dict(max_iters=2048))


def folded_cloth(layer_rows: int = 64, cols: int | None = None,
                 spacing: float = 2.0 ** -8, gap: float = 2.0 ** -9,
                 amp_gaps: float = 5.0, wavelength: float = 0.08,
                 seed: int = 1002, noise_space: str = "world"):
    """A (4*layer_rows+1)-row cloth z-folded into 4 layers `gap` apart.

    Grid row r belongs to layer k = min(r // layer_rows, 3), u = r - k*layer_rows,
    at height z = k*gap and y = u*s (k even) or (layer_rows-u)*s (k odd).
    x~ = x + A * (P_x, P_y, P_z), three independent seeded Perlin fields at
    wavelength `wavelength`, A = amp_gaps * gap. noise_space "world" samples the
    fields at the folded positions x (a smooth displacement field, the default);
    "material" samples them at the unfolded grid coordinates, so stacked layers
    receive unrelated displacements and are driven through each other (a stress
    variant).
    """
    nv = 4 * layer_rows + 1
    nu = nv if cols is None else cols
    uv, tris, edges = grid_cloth(nu, nv, spacing)
    rows = np.arange(nu * nv) // nu
    k = np.minimum(rows // layer_rows, 3)
    u = rows - k * layer_rows
    yy = np.where(k % 2 == 0, u, layer_rows - u) * spacing
    x = np.stack([uv[:, 0], yy, k * gap], axis=1)
    rng = np.random.default_rng(seed)
    fields = [Perlin3(rng) for _ in range(3)]
    offs = rng.uniform(0.0, 64.0, size=(3, 3))
    amp = amp_gaps * gap
    disp = np.zeros_like(x)
    base = x if noise_space == "world" else uv
    for c in range(3):
        q = base / wavelength + offs[c]
        disp[:, c] = amp * fields[c](q)
    xt = x + disp
    free = np.ones(len(x), bool)
    w = lumped_inverse_mass(uv, tris, edges, free)
    return dict(name=f"folded_cloth_{nu}x{nv}", x=x, xt=xt, w=w, tris=tris,
                edges=edges, params=dict(max_iters=2048))


def stacked_cubes(n_cubes: int = 8, cells: int = 16, size: float = 0.10,
                  gap: float = 0.005, h: float = 0.1, seed: int = 1003):
    """n_cubes cube surfaces stacked vertically `gap` apart, each with a seeded
    rigid velocity (uniform direction, speed U[2,5] m/s); x~ = x + h(v + g h)."""
    parts = []
    rng = np.random.default_rng(seed)
    vel = []
    for c in range(n_cubes):
        xb, tb, eb = box_surface(cells, size)
        xb = xb.copy()
        xb[:, 2] += c * (size + gap)
        parts.append((xb, tb, eb))
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        vel.append(d * rng.uniform(2.0, 5.0))
    x, tris, edges = _merge(parts)
    nper = len(parts[0][0])
    v = np.repeat(np.asarray(vel), nper, axis=0)
    xt = x + h * (v + GRAVITY * h)
    w = lumped_inverse_mass(x, tris, edges, np.ones(len(x), bool))
    return dict(name=f"cubes_{n_cubes}x{cells}", x=x, xt=xt, w=w, tris=tris,
                edges=edges, params=dict(max_iters=2048))


def hair(n_strands: int = 10000, segs: int = 32, seg_len: float = 0.005,
         radius: float = 0.10, h: float = 1.0 / 30.0, wind: float = 2.0,
         seed: int = 1004, wind_seed: int = 1005):
    """Polyline strands rooted at Fibonacci points of a sphere.

    Each strand grows along its root normal, bent by a smooth seeded noise field;
    roots are pinned (w=0, x~=x). Free vertices get x~ = x + h*(s/l)*v_w + h^2 g,
    with v_w a seeded unit direction times `wind` m/s, +-10% per vertex, and s/l the
    vertex's arc-length fraction along the strand.
    """
    i = np.arange(n_strands) + 0.5
    phi = np.arccos(1.0 - 2.0 * i / n_strands)
    theta = math.pi * (1.0 + 5.0 ** 0.5) * i
    nrm = np.stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi),
                    np.cos(phi)], axis=1)
    rng = np.random.default_rng(seed)
    fields = [Perlin3(rng) for _ in range(3)]
    pts = np.zeros((n_strands, segs + 1, 3))
    pts[:, 0] = nrm * radius
    d = nrm.copy()
    for s in range(segs):
        p = pts[:, s]
        q = p / 0.05
        bend = np.stack([fields[c](q) for c in range(3)], axis=1)
        d = d + 0.35 * bend
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        # keep growing outward
        out = (d * nrm).sum(axis=1, keepdims=True)
        d = np.where(out < 0.3, d + (0.3 - out) * nrm, d)
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        pts[:, s + 1] = p + seg_len * d
    x = pts.reshape(-1, 3)
    base = (np.arange(n_strands) * (segs + 1))[:, None]
    e = np.stack([np.arange(segs), np.arange(segs) + 1], axis=1)[None]
    edges = (base[:, :, None] + e).reshape(-1, 2).astype(np.int32)
    free = np.ones(len(x), bool)
    free[base[:, 0]] = False
    w = lumped_inverse_mass(x, np.zeros((0, 3), np.int32), edges, free)
    wr = np.random.default_rng(wind_seed)
    vw = wr.normal(size=3)
    vw = vw / np.linalg.norm(vw) * wind
    frac = np.tile(np.arange(segs + 1) / segs, n_strands)
    jitter = wr.uniform(0.9, 1.1, size=len(x))
    xt = x + (h * frac * jitter)[:, None] * vw + h * h * GRAVITY
    xt[~free] = x[~free]
    return dict(name=f"hair_{n_strands}x{segs}", x=x, xt=xt, w=w,
                tris=np.zeros((0, 3), np.int32), edges=edges,
                params=dict(max_iters=2048, delta=1e-3))


def sand_pile(nx: int = 32, ny: int = 32, nz: int = 30, spacing: float = 2e-3,
              jitter: float = 2e-4, h: float = 0.01, fall: float = 1.0, vstd: float = 0.5,
              seed: int = 1006, ground: int = 9):
    """A column of nx*ny*nz particles (vertices in no triangle or edge) on a jittered
    lattice `spacing` apart, its lowest layer one spacing above a static ground grid
    (ground x ground vertices, w = 0, x~ = x, 12 spacings beyond the column on every
    side). Particles: w = 1, x~ = x + h(v + g h) with v = (0, 0, -fall) +
    N(0, vstd^2) per component; the relative motion is several spacings per step, so
    grains collide with each other and with the ground."""
    rng = np.random.default_rng(seed)
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    p = np.stack([ii, jj, kk], axis=-1).reshape(-1, 3).astype(np.float64) * spacing
    p[:, 0] -= 0.5 * (nx - 1) * spacing
    p[:, 1] -= 0.5 * (ny - 1) * spacing
    p[:, 2] += spacing
    p += rng.uniform(-jitter, jitter, size=p.shape)
    ng = ground
    gs = (max(nx, ny) + 24) * spacing / (ng - 1)
    xg, tg, eg = grid_cloth(ng, ng, gs)
    xg[:, 0] -= 0.5 * (ng - 1) * gs
    xg[:, 1] -= 0.5 * (ng - 1) * gs
    np_ = len(p)
    x = np.concatenate([p, xg])
    tris = (tg + np_).astype(np.int32)
    edges = (eg + np_).astype(np.int32)
    v = rng.normal(0.0, vstd, size=(np_, 3))
    v[:, 2] -= fall
    xt = x.copy()
    xt[:np_] = p + h * (v + GRAVITY * h)
    w = np.zeros(len(x))
    w[:np_] = 1.0
    return dict(name=f"sand_{nx}x{ny}x{nz}", x=x, xt=xt, w=w, tris=tris, edges=edges,
                params=dict(max_iters=2048))


def torus(nu: int, nv: int, R: float, r: float):
    """Torus surface: nu vertices around the ring, nv around the tube, two triangles
    per quad, outward-facing (counter-clockwise seen from outside)."""
    u = np.arange(nu) * (2.0 * np.pi / nu)
    v = np.arange(nv) * (2.0 * np.pi / nv)
    uu, vv = np.meshgrid(u, v, indexing="ij")
    x = np.stack([(R + r * np.cos(vv)) * np.cos(uu), (R + r * np.cos(vv)) * np.sin(uu),
                  r * np.sin(vv)], axis=-1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = (i * nv + j).ravel()
    b = (((i + 1) % nu) * nv + j).ravel()
    c = (((i + 1) % nu) * nv + (j + 1) % nv).ravel()
    d = (i * nv + (j + 1) % nv).ravel()
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]).astype(np.int32)
    return x, tris, edges_from_tris(tris).astype(np.int32)


def normal_flow_spheres(subdiv: int = 5, radius: float = 0.05, gap: float = 0.01,
                        beta_gaps: float = 1.0, smooth: float = 0.1, iters: int = 3):
    """Globally injective normal flow (a stand-in for the benchmark meshes of the
    paper's normal-flow examples, which are not available): two icospheres `gap`
    apart, a positive flow that moves both surfaces outward by beta = beta_gaps * gap,
    so the spheres grow into each other and must stop face to face; then
    alpha = smooth * (shortest edge)^2 and `iters` Jacobi smoothing steps (small
    enough for the explicit steps not to overshoot). The target is computed by the flow
    code (library or oracle) from these parameters."""
    xs, ts = icosphere(subdiv, radius)[:2]
    es = edges_from_tris(ts)
    a = xs - [radius + 0.5 * gap, 0.0, 0.0]
    b = xs + [radius + 0.5 * gap, 0.0, 0.0]
    x, tris, edges = _merge([(a, ts, es), (b, ts, es)])
    el = np.linalg.norm(x[edges[:, 0]] - x[edges[:, 1]], axis=1).min()
    w = lumped_inverse_mass(x, tris, edges, np.ones(len(x), bool))
    return dict(name=f"normal_flow_spheres_s{subdiv}", x=x, w=w, tris=tris, edges=edges,
                flow=dict(beta=beta_gaps * gap, alpha=smooth * el * el, iters=iters),
                params=dict(max_iters=2048))


def config(i: int, small: bool = False):
    """The single-scene workloads (1-4; 6: the particle pile; 7: normal flow of two spheres,
    whose target comes from the flow code), full size or a
    small variant of the same structure (the small variants finish in seconds on the
    oracle)."""
    if i == 1:
        return cloth_over_sphere(n=17 if small else 33)
    if i == 2:
        return folded_cloth(layer_rows=8 if small else 64)
    if i == 3:
        return stacked_cubes(n_cubes=2 if small else 8, cells=4 if small else 16)
    if i == 4:
        return hair(n_strands=64 if small else 10000, segs=8 if small else 32)
    if i == 6:
        return sand_pile(*((6, 6, 5) if small else (32, 32, 30)))
    if i == 7:
        return normal_flow_spheres(3 if small else 5)
    raise ValueError(i)


def serve_request(i: int, t_min: float = 2000.0, t_max: float = 150000.0):
    """Request i of the serving stream: family uniform in {cloth over sphere,
    folded cloth, stacked cubes}, target triangle count log-uniform in
    [t_min, t_max] rounded to the nearest size the family can realise; seed 1005+i.
    Returns the scene dict with its time step h."""
    rng = np.random.default_rng(1005 + i)
    fam = int(rng.integers(1, 4))
    T = float(np.exp(rng.uniform(np.log(t_min), np.log(t_max))))
    if fam == 1:
        n = max(3, int(round(1.0 + np.sqrt(T / 2.0))))
        sc = cloth_over_sphere(n=n, seed=1005 + i)
        h = 1.0 / 30.0
    elif fam == 2:
        rows = max(1, int(round(np.sqrt(T / 2.0) / 4.0)))
        sc = folded_cloth(layer_rows=rows, seed=1005 + i)
        h = 1.0 / 30.0
    else:
        c = max(1, int(round(np.sqrt(T / 96.0))))
        sc = stacked_cubes(n_cubes=8, cells=c, seed=1005 + i)
        h = 0.1
    sc["family"] = fam
    sc["h"] = h
    sc["name"] = f"req{i}_" + sc["name"]
    return sc


def poisson_arrivals(n: int, rate: float, seed: int = 2005) -> np.ndarray:
    """Arrival times (s) of n requests of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
