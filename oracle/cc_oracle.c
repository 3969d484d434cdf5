/*
 * FP64 CPU oracle of the two-way continuous collision handling step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline leg of the
 * benchmark). It shares no code with the HIP library.
 *
 * Built with -O2 -ffp-contract=off and no fast-math: every expression is
 * evaluated in IEEE binary64, left to right, with correctly rounded sqrt and
 * division.
 *
 * Layout of the step (Alg. 1 of the paper):
 *   x <- x^[k], y <- y^[k+1], D <- 0, r <- 1, P <- {}
 *   for l = 0 .. L-1:
 *     if D < D_min: P <- proximity search at x with bound D_max; D <- D_max  (Sec. 3.1)
 *     pair pass: distances at x; P <- {d < D}; A <- {d < delta}; D_i      (Sec. 3.1, Sec. 5)
 *     backward: one projected Gauss-Seidel sweep over A, then edges       (Sec. 4)
 *     forward:  alpha_i, x_i, r_i                                          (Eq. eq:forward2)
 *     D <- D - 2 max_i ||x_i^(l+1) - x_i^(l)||; stop if ||r||_inf < eps   (Alg. 1)
 *
 * Readings (the paper is silent or ambiguous; each is also listed in the
 * repository's design notes):
 *  - L counts loop iterations: at most max_iters forward steps.
 *  - Set tests compare squared distances with squared thresholds:
 *    P' = {d^2 < D^2}, A = {d^2 < delta^2}, search = {d^2 < D_max^2}.
 *  - D_i = min(D, min over pairs of P' touching i of d) (a vertex in no pair
 *    gets D_i = D, the bound in the equation of Sec. 5).
 *  - alpha_i = 1 when y_i = x_i; when alpha_i = 1 the vertex is set to y_i.
 *  - The multipliers start at zero in every backward step and y carries the
 *    accumulated effect (Sec. 4: y initialised with y^(l)).
 *  - Constraints are coloured on the graph "shares a vertex with w > 0" (Sec. 4.3
 *    colours constraints, not vertices): contact rows by a randomised palette
 *    colouring whose choices are hashes of the row key, the seed and the round
 *    (orc_color_rows), edge-length rows greedily in the order of a hash of their
 *    key and the seed (orc_color_rows_greedy);
 *    the key of a contact is its pair key, the key of an edge-length row its
 *    input edge index. Contacts are swept colour by colour, then edge-length rows
 *    colour by colour.
 *  - Edge-edge contacts use the tetrahedron (a,b,c,e) in the volume form; near
 *    parallel edges and near degenerate triangles fall back to the gap
 *    constraint c = d/delta - 1 (the alternative named in Sec. 4.1).
 *  - Edge-length constraints are linearised once at y^[k+1] (Sec. 4.2) for
 *    every edge with a free end and non-zero target length.
 *  - Every vertex is a point primitive for vertex-triangle pairs; edge-edge
 *    pairs share no vertex; pairs whose vertices are all static (w = 0 and
 *    x~ = x) are dropped.
 *  - Vertex-vertex pairs (the third pair type of Sec. 4.1, c = |x_i - x_a|/delta
 *    - 1, for sand) join two particles: vertices that are a corner of no triangle
 *    and an end of no edge. The row is that constraint linearised at x^(l); the
 *    continuous test of such a pair is the closest approach of the two points.
 */
#include "cc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KEY_EE (1ull << 63)
#define KEY_VV (1ull << 62)
/* distance at which the continuous test reports contact (metres) */
/* eta: primitives closer than eta (metres) count as touching. Binary64 distances of
 * scenes whose coordinates stay within +-10 m are exact to far better than eta. */
#define ORC_ETA 1e-12
/* CCD-based step (Sec. 5.1): passes that scale steps before contacts send back */
#define ORC_STEP_PASSES 16

struct orc_scene {
  int32_t n, nt, ne;
  double* w;
  int32_t* tris;
  int32_t* edges;
  int32_t np;       /* particles: vertices in no triangle and no edge */
  int32_t* part;    /* their ids, increasing */
  uint8_t* stat;
  orc_params p;
  /* state */
  double *x, *y, *xt, *r, *xold, *rold;
  uint8_t* back; /* certificate: vertex returned to x^(l) in this iteration */
  double* alpha; /* the forward step's alpha of each vertex */
  double* scale; /* CCD-based step: factor of a vertex's step from the pass's contacts */
  double D;
  uint64_t* P;
  int64_t nP, capP;
  /* last pair pass */
  uint64_t* A;
  int32_t* acol;
  int64_t nA;
  double* Di;
  double* move2;
  /* edge-length rows, fixed for the step */
  int32_t n_er;
  int32_t* er_e;    /* input edge index of the row (its colouring key) */
  int32_t* er_v;    /* 2 per row */
  double* er_g;     /* 3 per row: (y_i - y_j)/L^2 at y^[k+1] */
  double* er_inv;   /* 1/A */
  int32_t* er_col;
  int32_t n_ecol;
};

uint64_t orc_mix64(uint64_t z) {
  /* splitmix64 output function (Steele, Lea, Flood 2014): a bijection on 64 bits */
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------ vectors */

static void sub3(double* o, const double* a, const double* b) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(double* o, const double* a, const double* b) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------- distances */

/* Squared distance from p to the segment [u,v]; *t = parameter of the closest
 * point (0 for a zero-length segment). */
static double pt_seg_d2(const double* p, const double* u, const double* v, double* t) {
  double uv[3], up[3], q[3], d[3];
  sub3(uv, v, u);
  sub3(up, p, u);
  double l2 = dot3(uv, uv);
  double s = 0.0;
  if (l2 > 0.0) {
    s = dot3(up, uv) / l2;
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
  }
  q[0] = u[0] + s * uv[0];
  q[1] = u[1] + s * uv[1];
  q[2] = u[2] + s * uv[2];
  sub3(d, p, q);
  *t = s;
  return dot3(d, d);
}

/* Squared point-triangle distance. The minimum of |p - q|^2 over the triangle
 * is reached either at the orthogonal projection (when it falls inside) or on
 * one of the three edges; the candidate list is tried in this order and the
 * first strict minimum kept. bary = weights of the closest point on (a,b,c). */
static double pt_tri_d2w(const double* p, const double* a, const double* b,
                         const double* c, double* bary, int* which) {
  double ab[3], ac[3], ap[3], n[3], t1[3], t2[3];
  sub3(ab, b, a);
  sub3(ac, c, a);
  sub3(ap, p, a);
  cross3(n, ab, ac);
  double nn = dot3(n, n);
  double best = INFINITY;
  double bw[3] = {1.0, 0.0, 0.0};
  int win = -1;
  if (nn > 0.0) {
    cross3(t1, ap, ac);
    cross3(t2, ab, ap);
    double wb = dot3(t1, n) / nn;
    double wc = dot3(t2, n) / nn;
    double wa = 1.0 - wb - wc;
    if (wa >= 0.0 && wb >= 0.0 && wc >= 0.0) {
      double h = dot3(ap, n);
      best = h * h / nn;
      win = 0;
      bw[0] = wa;
      bw[1] = wb;
      bw[2] = wc;
    }
  }
  double t, e2;
  e2 = pt_seg_d2(p, a, b, &t);
  if (e2 < best) {
    best = e2;
    win = 1;
    bw[0] = 1.0 - t;
    bw[1] = t;
    bw[2] = 0.0;
  }
  e2 = pt_seg_d2(p, b, c, &t);
  if (e2 < best) {
    best = e2;
    win = 2;
    bw[0] = 0.0;
    bw[1] = 1.0 - t;
    bw[2] = t;
  }
  e2 = pt_seg_d2(p, c, a, &t);
  if (e2 < best) {
    best = e2;
    win = 3;
    bw[0] = t;
    bw[1] = 0.0;
    bw[2] = 1.0 - t;
  }
  if (bary) {
    bary[0] = bw[0];
    bary[1] = bw[1];
    bary[2] = bw[2];
  }
  if (which) *which = win;
  return best;
}

double orc_pt_tri_d2(const double* p, const double* a, const double* b, const double* c,
                     double* bary) {
  return pt_tri_d2w(p, a, b, c, bary, NULL);
}

/* Squared segment-segment distance between [a,b] and [c,e]. The minimum over
 * the parameter square is the interior stationary point (when the lines are not
 * parallel and it lies inside) or lies on the boundary of the square, i.e. is an
 * endpoint-to-segment distance; candidates in this order, first strict minimum.
 * st = (s, t) with closest points a + s(b-a) and c + t(e-c). */
static double seg_seg_d2w(const double* a, const double* b, const double* c,
                          const double* e, double* st, int* which) {
  double d1[3], d2[3], r[3];
  sub3(d1, b, a);
  sub3(d2, e, c);
  sub3(r, a, c);
  double A = dot3(d1, d1), B = dot3(d1, d2), C = dot3(d2, d2);
  double Dd = dot3(d1, r), Ee = dot3(d2, r);
  double den = A * C - B * B;
  double best = INFINITY, bs = 0.0, bt = 0.0;
  int win = -1;
  if (den > 0.0) {
    double s = (B * Ee - C * Dd) / den;
    double t = (A * Ee - B * Dd) / den;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
      double p[3], q[3], d[3];
      p[0] = a[0] + s * d1[0];
      p[1] = a[1] + s * d1[1];
      p[2] = a[2] + s * d1[2];
      q[0] = c[0] + t * d2[0];
      q[1] = c[1] + t * d2[1];
      q[2] = c[2] + t * d2[2];
      sub3(d, p, q);
      best = dot3(d, d);
      win = 0;
      bs = s;
      bt = t;
    }
  }
  double u, e2;
  e2 = pt_seg_d2(a, c, e, &u);
  if (e2 < best) { best = e2; bs = 0.0; bt = u; win = 1; }
  e2 = pt_seg_d2(b, c, e, &u);
  if (e2 < best) { best = e2; bs = 1.0; bt = u; win = 2; }
  e2 = pt_seg_d2(c, a, b, &u);
  if (e2 < best) { best = e2; bs = u; bt = 0.0; win = 3; }
  e2 = pt_seg_d2(e, a, b, &u);
  if (e2 < best) { best = e2; bs = u; bt = 1.0; win = 4; }
  if (st) {
    st[0] = bs;
    st[1] = bt;
  }
  if (which) *which = win;
  return best;
}

double orc_seg_seg_d2(const double* a, const double* b, const double* c, const double* e,
                      double* st) {
  return seg_seg_d2w(a, b, c, e, st, NULL);
}

/* ------------------------------------------------------------------ pairs */

/* Vertex ids of a pair: VT key (a<<32 | f) -> (a, tri f); EE key -> (edge e, edge g). */
/* Vertices of a pair: vertex-triangle (a, i, j, k), edge-edge (a, b, c, e),
 * vertex-vertex (a, b, -1, -1). */
static void pair_verts(const orc_scene* s, uint64_t key, int32_t* v) {
  uint32_t pa = (uint32_t)((key >> 32) & 0x3fffffffu);
  uint32_t pb = (uint32_t)(key & 0xffffffffu);
  if (key & KEY_VV) {
    v[0] = (int32_t)pa;
    v[1] = (int32_t)pb;
    v[2] = -1;
    v[3] = -1;
  } else if (key & KEY_EE) {
    v[0] = s->edges[2 * pa];
    v[1] = s->edges[2 * pa + 1];
    v[2] = s->edges[2 * pb];
    v[3] = s->edges[2 * pb + 1];
  } else {
    v[0] = (int32_t)pa;
    v[1] = s->tris[3 * pb];
    v[2] = s->tris[3 * pb + 1];
    v[3] = s->tris[3 * pb + 2];
  }
}

static double pair_d2(const orc_scene* s, const double* x, uint64_t key, int32_t* v) {
  pair_verts(s, key, v);
  if (key & KEY_VV) {
    double d[3];
    sub3(d, x + 3 * v[0], x + 3 * v[1]);
    return dot3(d, d);
  }
  const double *x0 = x + 3 * v[0], *x1 = x + 3 * v[1], *x2 = x + 3 * v[2], *x3 = x + 3 * v[3];
  if (key & KEY_EE) return orc_seg_seg_d2(x0, x1, x2, x3, NULL);
  return orc_pt_tri_d2(x0, x1, x2, x3, NULL);
}

/* ---------------------------------------------------- contact constraints */

/* Signed volume det[q1-q0, q2-q0, q3-q0] (the 1/6 cancels in the ratio). */
static double det4(const double* q0, const double* q1, const double* q2, const double* q3) {
  double e1[3], e2[3], e3[3], c[3];
  sub3(e1, q1, q0);
  sub3(e2, q2, q0);
  sub3(e3, q3, q0);
  cross3(c, e2, e3);
  return dot3(e1, c);
}

/* Gradient of det4 with respect to q0..q3 (G is 4x3). */
static void grad4(const double* q0, const double* q1, const double* q2, const double* q3,
                  double* G) {
  double e1[3], e2[3], e3[3];
  sub3(e1, q1, q0);
  sub3(e2, q2, q0);
  sub3(e3, q3, q0);
  cross3(G + 3, e2, e3);
  cross3(G + 6, e3, e1);
  cross3(G + 9, e1, e2);
  for (int k = 0; k < 3; ++k) G[k] = -((G[3 + k] + G[6 + k]) + G[9 + k]);
}

/* Contact constraint row linearised at x (Sec. 4, paragraph "Linearization"):
 * c_lin(y) = c0 + sum_v J_v . (y_v - x_v).
 *
 * Vertex-triangle (Sec. 4.1, Fig. fig:vt and Eq. eq:volume_by_det): the
 * reference shape r moves the vertex by +g n and the triangle by -g n with
 * g = (delta - d)/2 and n the unit triangle normal oriented towards the vertex;
 * c = V(x)/V(r) - 1 with r held constant, so J_v = grad_v V(x) / V(r).
 * Edge-edge (same idea, Sec. 4.1): n = unit (b-a) x (e-c) oriented from edge 2
 * to edge 1; edge 1 moves +g n, edge 2 moves -g n; tetrahedron (a,b,c,e).
 * Gap fallback (near-parallel edges, near-degenerate triangle): with closest
 * points p, q and u = (p-q)/|p-q|, c = d/delta - 1 and J_v = omega_v u / delta,
 * omega = (1, -b_i, -b_j, -b_k) or (1-s, s, -(1-t), -t). */
int orc_contact_row(const orc_scene* s, const double* x, uint64_t key, int32_t* v,
                    double* c0, double* J, double* inv_a) {
  const double delta = s->p.delta, kappa2 = s->p.kappa * s->p.kappa;
  pair_verts(s, key, v);
  if (key & KEY_VV) {
    /* c = |x_a - x_b|/delta - 1 (Sec. 4.1) at x^(l): J_a = u/delta, J_b = -u/delta
     * with u the unit vector from b to a; coincident points give no row */
    double diff[3];
    sub3(diff, x + 3 * v[0], x + 3 * v[1]);
    double d = sqrt(dot3(diff, diff));
    memset(J, 0, 12 * sizeof(double));
    if (d == 0.0) {
      *inv_a = 0.0;
      return 2;
    }
    double u[3] = {diff[0] / d, diff[1] / d, diff[2] / d};
    const double om[2] = {1.0, -1.0};
    for (int i = 0; i < 2; ++i) {
      double co = om[i] / delta;
      for (int k = 0; k < 3; ++k) J[3 * i + k] = co * u[k];
    }
    double A = s->w[v[0]] * dot3(J, J);
    A = A + s->w[v[1]] * dot3(J + 3, J + 3);
    *c0 = d / delta - 1.0;
    *inv_a = A > 0.0 ? 1.0 / A : 0.0;
    return *inv_a > 0.0 ? 1 : 2;
  }
  const double* xs[4] = {x + 3 * v[0], x + 3 * v[1], x + 3 * v[2], x + 3 * v[3]};
  double om[4], d2, bw[3], st[2];
  int volume_ok, which;
  double N[3], side;
  if (key & KEY_EE) {
    d2 = seg_seg_d2w(xs[0], xs[1], xs[2], xs[3], st, &which);
    om[0] = 1.0 - st[0];
    om[1] = st[0];
    om[2] = -(1.0 - st[1]);
    om[3] = -st[1];
    double d1v[3], d2v[3], ac[3];
    sub3(d1v, xs[1], xs[0]);
    sub3(d2v, xs[3], xs[2]);
    cross3(N, d1v, d2v);
    double mm = dot3(N, N);
    double l1 = dot3(d1v, d1v), l2 = dot3(d2v, d2v);
    volume_ok = mm > kappa2 * (l1 * l2);
    sub3(ac, xs[0], xs[2]);
    side = dot3(ac, N) >= 0.0 ? 1.0 : -1.0;
  } else {
    d2 = pt_tri_d2w(xs[0], xs[1], xs[2], xs[3], bw, &which);
    om[0] = 1.0;
    om[1] = -bw[0];
    om[2] = -bw[1];
    om[3] = -bw[2];
    double e1[3], e2[3], e3[3], ai[3];
    sub3(e1, xs[2], xs[1]);
    sub3(e2, xs[3], xs[1]);
    sub3(e3, xs[3], xs[2]);
    cross3(N, e1, e2);
    double nn = dot3(N, N);
    double l = dot3(e1, e1), m2 = dot3(e2, e2), m3 = dot3(e3, e3);
    if (m2 > l) l = m2;
    if (m3 > l) l = m3;
    volume_ok = nn > kappa2 * (l * l);
    sub3(ai, xs[0], xs[1]);
    side = dot3(ai, N) >= 0.0 ? 1.0 : -1.0;
  }
  /* the reference shape separates the closest points along n, which is their
   * separating direction only when both closest points are interior (the vertex
   * over the face, or the common perpendicular of the edges); otherwise the gap
   * form */
  if (which != 0) volume_ok = 0;
  double d = sqrt(d2);
  double c = 0.0, Jl[12];
  int kind;
  if (volume_ok) {
    double g = 0.5 * (delta - d);
    double scale = side / sqrt(dot3(N, N));
    double off[3] = {g * (N[0] * scale), g * (N[1] * scale), g * (N[2] * scale)};
    double r[4][3];
    /* vertex (VT) or edge 1 (EE) moves +g n; the other simplex moves -g n */
    int plus1 = (key & KEY_EE) ? 1 : 0;
    for (int k = 0; k < 3; ++k) {
      r[0][k] = xs[0][k] + off[k];
      r[1][k] = plus1 ? xs[1][k] + off[k] : xs[1][k] - off[k];
      r[2][k] = xs[2][k] - off[k];
      r[3][k] = xs[3][k] - off[k];
    }
    double vr = det4(r[0], r[1], r[2], r[3]);
    if (vr == 0.0) {
      *inv_a = 0.0;
      return 2;
    }
    double vx = det4(xs[0], xs[1], xs[2], xs[3]);
    c = vx / vr - 1.0;
    double G[12];
    grad4(xs[0], xs[1], xs[2], xs[3], G);
    for (int i = 0; i < 12; ++i) Jl[i] = G[i] / vr;
    kind = 0;
  } else {
    double diff[3];
    if (key & KEY_EE) {
      double p[3], q[3], d1v[3], d2v[3];
      sub3(d1v, xs[1], xs[0]);
      sub3(d2v, xs[3], xs[2]);
      for (int k = 0; k < 3; ++k) {
        p[k] = xs[0][k] + st[0] * d1v[k];
        q[k] = xs[2][k] + st[1] * d2v[k];
      }
      sub3(diff, p, q);
    } else {
      double p[3];
      for (int k = 0; k < 3; ++k)
        p[k] = (bw[0] * xs[1][k] + bw[1] * xs[2][k]) + bw[2] * xs[3][k];
      sub3(diff, xs[0], p);
    }
    double dd = sqrt(dot3(diff, diff));
    if (dd == 0.0) {
      *inv_a = 0.0;
      return 2;
    }
    double u[3] = {diff[0] / dd, diff[1] / dd, diff[2] / dd};
    c = d / delta - 1.0;
    for (int i = 0; i < 4; ++i) {
      double co = om[i] / delta;
      for (int k = 0; k < 3; ++k) Jl[3 * i + k] = co * u[k];
    }
    kind = 1;
  }
  double A = 0.0;
  for (int i = 0; i < 4; ++i) A = A + s->w[v[i]] * dot3(Jl + 3 * i, Jl + 3 * i);
  *c0 = c;
  memcpy(J, Jl, sizeof Jl);
  *inv_a = A > 0.0 ? 1.0 / A : 0.0;
  return *inv_a > 0.0 ? kind : 2;
}

/* --------------------------------------------------------------- search */

typedef struct {
  int64_t cell;
  int32_t prim;
} cell_entry;

static int cmp_cell(const void* a, const void* b) {
  const cell_entry *x = (const cell_entry*)a, *y = (const cell_entry*)b;
  if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
  return (x->prim > y->prim) - (x->prim < y->prim);
}
static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

typedef struct {
  double lo[3], h;
  int64_t dim[3];
  cell_entry* ent;
  int64_t n;
} grid_t;

static int64_t cell_of(const grid_t* g, int64_t i, int64_t j, int64_t k) {
  return (i * g->dim[1] + j) * g->dim[2] + k;
}
static int64_t clampi(int64_t v, int64_t hi) { return v < 0 ? 0 : (v >= hi ? hi - 1 : v); }
static void cell_range(const grid_t* g, const double* lo, const double* hi, int64_t* c0,
                       int64_t* c1) {
  for (int k = 0; k < 3; ++k) {
    c0[k] = clampi((int64_t)floor((lo[k] - g->lo[k]) / g->h), g->dim[k]);
    c1[k] = clampi((int64_t)floor((hi[k] - g->lo[k]) / g->h), g->dim[k]);
  }
}

/* Uniform grid over the primitives `ids` with boxes inflated by `infl`. */
static void grid_build(grid_t* g, const double* x, const int32_t* idx, int32_t stride,
                       int32_t count, double infl, const double* slo, double h,
                       const int64_t* dim) {
  memcpy(g->lo, slo, sizeof g->lo);
  g->h = h;
  memcpy(g->dim, dim, sizeof g->dim);
  int64_t cap = 0;
  g->ent = NULL;
  g->n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    int64_t n = 0;
    for (int32_t f = 0; f < count; ++f) {
      double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int c = 0; c < stride; ++c) {
        const double* q = x + 3 * idx[stride * f + c];
        for (int k = 0; k < 3; ++k) {
          if (q[k] < lo[k]) lo[k] = q[k];
          if (q[k] > hi[k]) hi[k] = q[k];
        }
      }
      for (int k = 0; k < 3; ++k) {
        lo[k] -= infl;
        hi[k] += infl;
      }
      int64_t a[3], b[3];
      cell_range(g, lo, hi, a, b);
      for (int64_t i = a[0]; i <= b[0]; ++i)
        for (int64_t j = a[1]; j <= b[1]; ++j)
          for (int64_t k = a[2]; k <= b[2]; ++k) {
            if (pass == 1) {
              g->ent[n].cell = cell_of(g, i, j, k);
              g->ent[n].prim = f;
            }
            ++n;
          }
    }
    if (pass == 0) {
      cap = n;
      g->ent = (cell_entry*)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(cell_entry));
    } else {
      g->n = n;
    }
  }
  qsort(g->ent, (size_t)g->n, sizeof(cell_entry), cmp_cell);
}

static int64_t grid_lower(const grid_t* g, int64_t cell) {
  int64_t lo = 0, hi = g->n;
  while (lo < hi) {
    int64_t m = (lo + hi) / 2;
    if (g->ent[m].cell < cell) lo = m + 1; else hi = m;
  }
  return lo;
}

static int all_static(const orc_scene* s, const int32_t* v) {
  for (int k = 0; k < 4; ++k)
    if (v[k] >= 0 && !s->stat[v[k]]) return 0;
  return 1;
}

typedef struct {
  uint64_t* out;
  int64_t n, cap;
} keybuf;
static void kb_push(keybuf* b, uint64_t k) {
  if (b->n < b->cap && b->out) b->out[b->n] = k;
  b->n++;
}

/* The pair universe (Sec. 5: two non-adjacent simplices): vertex-triangle (a,f)
 * with a not a corner of f, edge-edge (e,g) with e<g sharing no vertex, and
 * vertex-vertex (a,b) with a<b, both particles. */
static int vt_ok(const orc_scene* s, int32_t a, int32_t f) {
  const int32_t* t = s->tris + 3 * f;
  return a != t[0] && a != t[1] && a != t[2];
}
static int ee_ok(const orc_scene* s, int32_t e, int32_t g) {
  const int32_t *p = s->edges + 2 * e, *q = s->edges + 2 * g;
  return e < g && p[0] != q[0] && p[0] != q[1] && p[1] != q[0] && p[1] != q[1];
}

static void test_pair(orc_scene* s, const double* x, uint64_t key, double dmax2, keybuf* kb) {
  int32_t v[4];
  pair_verts(s, key, v);
  if (all_static(s, v)) return;
  if (pair_d2(s, x, key, v) < dmax2) kb_push(kb, key);
}

/* Grid over the scene at x: cell size >= dmax and >= the mean edge extent, the
 * scene's box widened by 2 dmax, at most 4096 cells per axis. */
static void grid_dims(const orc_scene* s, const double* x, double dmax, double* glo, double* h_out,
                      int64_t* dim) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = 0; i < s->n; ++i)
      for (int k = 0; k < 3; ++k) {
        if (x[3 * i + k] < lo[k]) lo[k] = x[3 * i + k];
        if (x[3 * i + k] > hi[k]) hi[k] = x[3 * i + k];
      }
    double ext = 0.0;
    int64_t cnt = 0;
    for (int32_t e = 0; e < s->ne; ++e) {
      double d[3];
      sub3(d, x + 3 * s->edges[2 * e + 1], x + 3 * s->edges[2 * e]);
      ext += fabs(d[0]) > fabs(d[1]) ? (fabs(d[0]) > fabs(d[2]) ? fabs(d[0]) : fabs(d[2]))
                                     : (fabs(d[1]) > fabs(d[2]) ? fabs(d[1]) : fabs(d[2]));
      ++cnt;
    }
    double h = dmax;
    if (cnt && ext / (double)cnt > h) h = ext / (double)cnt;
    for (int k = 0; k < 3; ++k) {
      glo[k] = lo[k] - 2.0 * dmax;
      double span = (hi[k] + 2.0 * dmax) - glo[k];
      dim[k] = (int64_t)floor(span / h) + 1;
      if (dim[k] > 4096) dim[k] = 4096;
    }
    /* keep every cell id inside int64 */
    double hh = h;
    for (int k = 0; k < 3; ++k) {
      double span = (hi[k] + 2.0 * dmax) - glo[k];
      if (span / hh > (double)dim[k]) hh = span / (double)(dim[k] - 1);
    }
    h = hh;
    *h_out = h;
}

/* --------------------------------------------------------------- validation */

/* Sign of det[b-a, c-a, d-a] (d against the plane of a, b, c); 0 when the FP64
 * value lies within 1e-12 of the sum of the absolute products (touching). */
static int orient_band(const double* a, const double* b, const double* c, const double* d) {
  double u[3], v[3], w[3], n[3];
  sub3(u, b, a);
  sub3(v, c, a);
  sub3(w, d, a);
  cross3(n, u, v);
  double o = dot3(n, w);
  double perm = (fabs(u[1] * v[2]) + fabs(u[2] * v[1])) * fabs(w[0]) +
                (fabs(u[2] * v[0]) + fabs(u[0] * v[2])) * fabs(w[1]) +
                (fabs(u[0] * v[1]) + fabs(u[1] * v[0])) * fabs(w[2]);
  double band = 1e-12 * perm;
  return o > band ? 1 : (o < -band ? -1 : 0);
}

/* Does segment pq meet triangle abc (crossing or touching)? Off the plane: the
 * endpoints are not strictly on one side and the line pq passes through the
 * closed triangle (the three orientations of pq against its sides agree). In the
 * plane (both endpoints within the band): the FP64 distance is at most tol. */
int orc_seg_tri_meet(const double* p, const double* q, const double* a, const double* b,
                     const double* c, double tol) {
  int sp = orient_band(a, b, c, p), sq = orient_band(a, b, c, q);
  if (sp == 0 && sq == 0) {
    double d2 = orc_seg_seg_d2(p, q, a, b, NULL), t;
    t = orc_seg_seg_d2(p, q, b, c, NULL);
    if (t < d2) d2 = t;
    t = orc_seg_seg_d2(p, q, c, a, NULL);
    if (t < d2) d2 = t;
    t = orc_pt_tri_d2(p, a, b, c, NULL);
    if (t < d2) d2 = t;
    t = orc_pt_tri_d2(q, a, b, c, NULL);
    if (t < d2) d2 = t;
    return d2 <= tol * tol;
  }
  if (sp * sq > 0) return 0;
  int s1 = orient_band(p, q, a, b), s2 = orient_band(p, q, b, c), s3 = orient_band(p, q, c, a);
  return (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
}

/* The input check (x^t must be in the free space, Sec. 3): 1 when some vertex-
 * triangle or edge-edge pair of the universe is closer than tol, or some edge
 * meets a triangle it shares no vertex with (pairs whose vertices are all static
 * are skipped, as in the step); 0 otherwise. */
int orc_validate(orc_scene* s, const double* x, double tol) {
  if (orc_search(s, x, tol, 0, NULL, 0) > 0) return 1;
  if (s->nt == 0 || s->ne == 0) return 0;
  int64_t dim[3];
  double glo[3], h;
  grid_dims(s, x, tol, glo, &h, dim);
  grid_t g;
  grid_build(&g, x, s->tris, 3, s->nt, tol, glo, h, dim);
  int32_t* seen = (int32_t*)malloc((size_t)s->nt * sizeof(int32_t));
  for (int32_t f = 0; f < s->nt; ++f) seen[f] = -1;
  int bad = 0;
  for (int32_t e = 0; e < s->ne && !bad; ++e) {
    const int32_t* ev = s->edges + 2 * e;
    const double *p = x + 3 * ev[0], *q = x + 3 * ev[1];
    double blo[3], bhi[3];
    for (int k = 0; k < 3; ++k) {
      blo[k] = p[k] < q[k] ? p[k] : q[k];
      bhi[k] = p[k] < q[k] ? q[k] : p[k];
    }
    int64_t c0[3], c1[3];
    cell_range(&g, blo, bhi, c0, c1);
    for (int64_t i0 = c0[0]; i0 <= c1[0] && !bad; ++i0)
      for (int64_t j0 = c0[1]; j0 <= c1[1] && !bad; ++j0)
        for (int64_t k0 = c0[2]; k0 <= c1[2] && !bad; ++k0) {
          int64_t cell = cell_of(&g, i0, j0, k0);
          for (int64_t i = grid_lower(&g, cell); i < g.n && g.ent[i].cell == cell; ++i) {
            int32_t f = g.ent[i].prim;
            if (seen[f] == e) continue;
            seen[f] = e;
            const int32_t* t = s->tris + 3 * f;
            if (ev[0] == t[0] || ev[0] == t[1] || ev[0] == t[2] || ev[1] == t[0] || ev[1] == t[1] ||
                ev[1] == t[2])
              continue;
            if (s->stat[ev[0]] && s->stat[ev[1]] && s->stat[t[0]] && s->stat[t[1]] && s->stat[t[2]])
              continue;
            if (orc_seg_tri_meet(p, q, x + 3 * t[0], x + 3 * t[1], x + 3 * t[2], tol)) {
              bad = 1;
              break;
            }
          }
        }
  }
  free(seen);
  free(g.ent);
  return bad;
}

int64_t orc_search(orc_scene* s, const double* x, double dmax, int brute, uint64_t* out,
                   int64_t cap) {
  keybuf kb = {out, 0, cap};
  double dmax2 = dmax * dmax;
  if (brute) {
    for (int32_t a = 0; a < s->n; ++a)
      for (int32_t f = 0; f < s->nt; ++f)
        if (vt_ok(s, a, f)) test_pair(s, x, ((uint64_t)a << 32) | (uint32_t)f, dmax2, &kb);
    for (int32_t e = 0; e < s->ne; ++e)
      for (int32_t g = e + 1; g < s->ne; ++g)
        if (ee_ok(s, e, g))
          test_pair(s, x, KEY_EE | ((uint64_t)e << 32) | (uint32_t)g, dmax2, &kb);
    for (int32_t i = 0; i < s->np; ++i)
      for (int32_t j = i + 1; j < s->np; ++j)
        test_pair(s, x, KEY_VV | ((uint64_t)s->part[i] << 32) | (uint32_t)s->part[j], dmax2, &kb);
  } else {
    int64_t dim[3];
    double glo[3], h;
    grid_dims(s, x, dmax, glo, &h, dim);
    if (s->nt > 0) {
      grid_t g;
      grid_build(&g, x, s->tris, 3, s->nt, dmax, glo, h, dim);
      for (int32_t a = 0; a < s->n; ++a) {
        int64_t c0[3], c1[3];
        cell_range(&g, x + 3 * a, x + 3 * a, c0, c1);
        int64_t cell = cell_of(&g, c0[0], c0[1], c0[2]);
        for (int64_t i = grid_lower(&g, cell); i < g.n && g.ent[i].cell == cell; ++i) {
          int32_t f = g.ent[i].prim;
          if (vt_ok(s, a, f)) test_pair(s, x, ((uint64_t)a << 32) | (uint32_t)f, dmax2, &kb);
        }
      }
      free(g.ent);
    }
    if (s->ne > 1) {
      grid_t g;
      grid_build(&g, x, s->edges, 2, s->ne, dmax, glo, h, dim);
      int32_t* seen = (int32_t*)malloc((size_t)s->ne * sizeof(int32_t));
      for (int32_t e = 0; e < s->ne; ++e) seen[e] = -1;
      for (int32_t e = 0; e < s->ne; ++e) {
        double blo[3], bhi[3];
        const double *p = x + 3 * s->edges[2 * e], *q = x + 3 * s->edges[2 * e + 1];
        for (int k = 0; k < 3; ++k) {
          blo[k] = p[k] < q[k] ? p[k] : q[k];
          bhi[k] = p[k] < q[k] ? q[k] : p[k];
        }
        int64_t c0[3], c1[3];
        cell_range(&g, blo, bhi, c0, c1);
        for (int64_t i0 = c0[0]; i0 <= c1[0]; ++i0)
          for (int64_t j0 = c0[1]; j0 <= c1[1]; ++j0)
            for (int64_t k0 = c0[2]; k0 <= c1[2]; ++k0) {
              int64_t cell = cell_of(&g, i0, j0, k0);
              for (int64_t i = grid_lower(&g, cell); i < g.n && g.ent[i].cell == cell; ++i) {
                int32_t gg = g.ent[i].prim;
                if (seen[gg] == e) continue;
                seen[gg] = e;
                if (ee_ok(s, e, gg))
                  test_pair(s, x, KEY_EE | ((uint64_t)e << 32) | (uint32_t)gg, dmax2, &kb);
              }
            }
      }
      free(seen);
      free(g.ent);
    }
    if (s->np > 1) {
      /* particles: each particle's cell against the particles whose box, widened
       * by dmax, covers it; the pair is taken once, from its lower vertex */
      grid_t g;
      grid_build(&g, x, s->part, 1, s->np, dmax, glo, h, dim);
      for (int32_t i = 0; i < s->np; ++i) {
        const int32_t a = s->part[i];
        int64_t c0[3], c1[3];
        cell_range(&g, x + 3 * a, x + 3 * a, c0, c1);
        int64_t cell = cell_of(&g, c0[0], c0[1], c0[2]);
        for (int64_t k = grid_lower(&g, cell); k < g.n && g.ent[k].cell == cell; ++k) {
          const int32_t b = s->part[g.ent[k].prim];
          if (a < b) test_pair(s, x, KEY_VV | ((uint64_t)a << 32) | (uint32_t)b, dmax2, &kb);
        }
      }
      free(g.ent);
    }
  }
  if (out && kb.n <= cap) qsort(out, (size_t)kb.n, sizeof(uint64_t), cmp_u64);
  return kb.n;
}

/* ------------------------------------------------------------------- CCD */

/* Continuous test of one pair along the linear piece q_k(t) = q_k + t dq_k,
 * t in [0,1] (q in the tetrahedron order of the contact row: vertex then
 * triangle, or edge 1 then edge 2); contact means a distance <= eta. The
 * primitives' distance is probed at t = 0; then at the times where the four points
 * are coplanar, V(t) = det[q1-q0, q2-q0, q3-q0](t) = 0, a cubic
 * a3 t^3 + a2 t^2 + a1 t + a0 whose critical points split [0,1] into monotone
 * pieces (a piece whose end values differ in sign is bisected to its root), and at
 * those critical points; a piece with no contact at these times is then swept by
 * conservative advancement (below), and probed at t = 1. Returns 1 on a contact
 * and stores its time. */
static double cubic_at(const double* a, double t) { return ((a[3] * t + a[2]) * t + a[1]) * t + a[0]; }

/* Vertex-vertex: the closest approach of two points moving linearly, at
 * t* = clamp(-(p.dp)/(dp.dp), 0, 1) with p = q_a - q_b, dp = dq_a - dq_b (t* = 0
 * when the points move together); contact when their distance there is <= eta. */
static int ccd_hit_vv(const double* q, const double* dq, double eta, double* t_hit) {
  double p[3], dp[3];
  sub3(p, q, q + 3);
  sub3(dp, dq, dq + 3);
  double dd = dot3(dp, dp);
  double t = 0.0;
  if (dd > 0.0) {
    t = -dot3(p, dp) / dd;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
  }
  double a[3], b[3], e[3];
  for (int m = 0; m < 3; ++m) {
    a[m] = q[m] + t * dq[m];
    b[m] = q[3 + m] + t * dq[3 + m];
  }
  sub3(e, a, b);
  if (dot3(e, e) <= eta * eta) {
    if (t_hit) *t_hit = t;
    return 1;
  }
  return 0;
}

#define ORC_CA_STEPS 1024

/* squared distance of the two primitives at time t of the piece */
static double ccd_dist2(const double* q, const double* dq, int ee, double t) {
  double p[4][3];
  for (int k = 0; k < 4; ++k)
    for (int m = 0; m < 3; ++m) p[k][m] = q[3 * k + m] + t * dq[3 * k + m];
  return ee ? orc_seg_seg_d2(p[0], p[1], p[2], p[3], NULL)
            : orc_pt_tri_d2(p[0], p[1], p[2], p[3], NULL);
}

static int ccd_probe(const double* q, const double* dq, int ee, double t, double eta2) {
  return ccd_dist2(q, dq, ee, t) <= eta2;
}

int orc_ccd_hit(const double* q, const double* dq, int kind, double eta, double* t_hit) {
  if (kind == 2) return ccd_hit_vv(q, dq, eta, t_hit);
  const int ee = kind;
  const double eta2 = eta * eta;
  /* the start of the piece */
  if (ccd_probe(q, dq, ee, 0.0, eta2)) {
    if (t_hit) *t_hit = 0.0;
    return 1;
  }
  double e1[3], e2[3], e3[3], f1[3], f2[3], f3[3], c[3], a[4];
  for (int m = 0; m < 3; ++m) {
    e1[m] = q[3 + m] - q[m];
    e2[m] = q[6 + m] - q[m];
    e3[m] = q[9 + m] - q[m];
    f1[m] = dq[3 + m] - dq[m];
    f2[m] = dq[6 + m] - dq[m];
    f3[m] = dq[9 + m] - dq[m];
  }
  double c23[3], f2e3[3], e2f3[3], f2f3[3];
  cross3(c23, e2, e3);
  cross3(f2e3, f2, e3);
  cross3(e2f3, e2, f3);
  cross3(f2f3, f2, f3);
  a[0] = dot3(e1, c23);
  a[1] = dot3(f1, c23) + dot3(e1, f2e3) + dot3(e1, e2f3);
  a[2] = dot3(f1, f2e3) + dot3(f1, e2f3) + dot3(e1, f2f3);
  a[3] = dot3(f1, f2f3);
  (void)c;
  /* knots: 0, critical points inside (0,1) in increasing order, 1 */
  double knot[4];
  int nk = 0;
  knot[nk++] = 0.0;
  double A = 3.0 * a[3], B = 2.0 * a[2], C = a[1];
  double crit[2];
  int nc = 0;
  if (A == 0.0) {
    if (B != 0.0) crit[nc++] = -C / B;
  } else {
    double disc = B * B - 4.0 * A * C;
    if (disc >= 0.0) {
      double sq = sqrt(disc);
      double r1 = (-B - sq) / (2.0 * A), r2 = (-B + sq) / (2.0 * A);
      crit[nc++] = r1 < r2 ? r1 : r2;
      crit[nc++] = r1 < r2 ? r2 : r1;
    }
  }
  for (int i = 0; i < nc; ++i)
    if (crit[i] > 0.0 && crit[i] < 1.0 && crit[i] > knot[nk - 1]) knot[nk++] = crit[i];
  knot[nk++] = 1.0;
  for (int i = 0; i + 1 < nk; ++i) {
    double lo = knot[i], hi = knot[i + 1];
    double vlo = cubic_at(a, lo), vhi = cubic_at(a, hi);
    double t = -1.0;
    if (vlo == 0.0) {
      t = lo;
    } else if (vhi == 0.0) {
      t = hi;
    } else if ((vlo < 0.0) != (vhi < 0.0)) {
      for (int it = 0; it < 64; ++it) {
        double mid = 0.5 * (lo + hi);
        double vm = cubic_at(a, mid);
        if (vm == 0.0) {
          lo = mid;
          hi = mid;
          break;
        }
        if ((vm < 0.0) == (vlo < 0.0)) lo = mid; else hi = mid;
      }
      t = 0.5 * (lo + hi);
    }
    if (t >= 0.0 && ccd_probe(q, dq, ee, t, eta2)) {
      if (t_hit) *t_hit = t;
      return 1;
    }
    /* a grazing contact leaves no sign change: probe the critical point too */
    if (i + 2 < nk && ccd_probe(q, dq, ee, knot[i + 1], eta2)) {
      if (t_hit) *t_hit = knot[i + 1];
      return 1;
    }
  }
  /* Clearance by conservative advancement (Mirtich's method): the distance of the
   * two primitives changes with t at most at rate Lc = max |dq| over the first
   * primitive's points + max |dq| over the second's, so from a time t with distance
   * d > eta no contact occurs before t + (d - eta) / Lc. This also covers a piece
   * that stays coplanar (V(t) = 0 throughout), which the cubic does not see. A
   * piece not cleared within ORC_CA_STEPS advances counts as a contact. */
  double l1 = 0.0, l2 = 0.0;
  for (int k = 0; k < 4; ++k) {
    const double mk = sqrt(dot3(dq + 3 * k, dq + 3 * k));
    if (k < (ee ? 2 : 1)) {
      if (mk > l1) l1 = mk;
    } else if (mk > l2) {
      l2 = mk;
    }
  }
  const double lc = l1 + l2;
  double t = 0.0;
  int cleared = !(lc > 0.0);
  for (int step = 0; step < ORC_CA_STEPS && !cleared; ++step) {
    const double d = sqrt(ccd_dist2(q, dq, ee, t));
    if (d <= eta) {
      if (t_hit) *t_hit = t;
      return 1;
    }
    t = t + (d - eta) / lc;
    if (t >= 1.0) cleared = 1;
  }
  if (!cleared) {
    if (t_hit) *t_hit = t;
    return 1;
  }
  /* the end of the piece (the advancement leaves a distance of at least eta there) */
  if (ccd_probe(q, dq, ee, 1.0, eta2)) {
    if (t_hit) *t_hit = 1.0;
    return 1;
  }
  return 0;
}



/* ------------------------------------------------------------- colouring */

/* Randomised palette colouring, after the colouring the backward step of
 * Sec. 4.3 takes (rows of one colour share no free vertex and are projected in
 * parallel), with its random choices made functions of the row's key, the seed
 * and the round so that the colours depend only on the row set. In round
 * t = 1, 2, ... every uncoloured row r
 *   - finds u_v, the number of uncoloured rows at each of its free vertices v
 *     (r included), and its palette size m_r = max(1, max_v u_v) + f_r, where f_r
 *     counts the rounds r has failed;
 *   - picks the (h mod m_r)-th smallest colour (counting from 0) not used by the
 *     coloured rows at its free vertices, h = mix64(mix64(key ^ seed) + t * phi),
 *     phi = 0x9E3779B97F4A7C15 (wrapping arithmetic);
 * then every row whose pick no other uncoloured row sharing a free vertex made in
 * this round keeps it; the others fail and try again. A pick beyond the palette
 * limit, or more than ORC_MAX_ROUNDS rounds, is an error. */
#define ORC_MAX_ROUNDS 4096
#define ORC_PHI 0x9E3779B97F4A7C15ull

typedef struct {
  int64_t key; /* vertex * 2048 + colour */
  int64_t row;
} claim_t;

static int cmp_claim(const void* a, const void* b) {
  const claim_t *x = (const claim_t*)a, *y = (const claim_t*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->row > y->row) - (x->row < y->row);
}

static int free_vertex(const orc_scene* s, int32_t v) { return v >= 0 && s->w[v] > 0.0; }

int32_t orc_color_rows(const orc_scene* s, int64_t nrows, const int32_t* rv,
                       const uint64_t* keys, int32_t* colors) {
  const int W = (s->p.max_colors + 63) / 64;
  const size_t NR = (size_t)(nrows > 0 ? nrows : 1);
  uint64_t* prio = (uint64_t*)malloc(NR * sizeof(uint64_t));
  int32_t* fails = (int32_t*)calloc(NR, sizeof(int32_t));
  int32_t* pick = (int32_t*)malloc(NR * sizeof(int32_t));
  uint8_t* lost = (uint8_t*)malloc(NR);
  int32_t* unc = (int32_t*)calloc((size_t)s->n, sizeof(int32_t));
  uint64_t* mask = (uint64_t*)calloc((size_t)s->n * (size_t)W, sizeof(uint64_t));
  claim_t* cl = (claim_t*)malloc(NR * 4 * sizeof(claim_t));
  int32_t ncol = 0, err = 0;
  for (int64_t r = 0; r < nrows; ++r) {
    prio[r] = orc_mix64(keys[r] ^ s->p.seed);
    colors[r] = -1;
  }
  int64_t left = nrows;
  for (uint64_t t = 1; left > 0 && !err; ++t) {
    if (t > ORC_MAX_ROUNDS) {
      err = 1;
      break;
    }
    /* uncoloured rows at each free vertex */
    for (int32_t v = 0; v < s->n; ++v) unc[v] = 0;
    for (int64_t r = 0; r < nrows; ++r) {
      if (colors[r] >= 0) continue;
      for (int k = 0; k < 4; ++k)
        if (free_vertex(s, rv[4 * r + k])) unc[rv[4 * r + k]] += 1;
    }
    /* picks */
    int64_t ncl = 0;
    for (int64_t r = 0; r < nrows && !err; ++r) {
      if (colors[r] >= 0) continue;
      int32_t m = 1;
      for (int k = 0; k < 4; ++k) {
        const int32_t v = rv[4 * r + k];
        if (free_vertex(s, v) && unc[v] > m) m = unc[v];
      }
      m += fails[r];
      const uint64_t h = orc_mix64(prio[r] + t * ORC_PHI);
      const int64_t want = (int64_t)(h % (uint64_t)m);
      int32_t c = -1;
      int64_t seen = 0;
      for (int32_t q = 0; q < s->p.max_colors; ++q) {
        int used = 0;
        for (int k = 0; k < 4; ++k) {
          const int32_t v = rv[4 * r + k];
          if (free_vertex(s, v) && ((mask[(size_t)v * W + q / 64] >> (q % 64)) & 1ull)) used = 1;
        }
        if (used) continue;
        if (seen == want) {
          c = q;
          break;
        }
        ++seen;
      }
      if (c < 0) {
        err = 1;
        break;
      }
      pick[r] = c;
      for (int k = 0; k < 4; ++k) {
        const int32_t v = rv[4 * r + k];
        if (free_vertex(s, v)) {
          cl[ncl].key = (int64_t)v * 2048 + c;
          cl[ncl].row = r;
          ++ncl;
        }
      }
    }
    if (err) break;
    /* rows whose pick another row at a shared free vertex made too */
    for (int64_t r = 0; r < nrows; ++r) lost[r] = 0;
    qsort(cl, (size_t)ncl, sizeof(claim_t), cmp_claim);
    for (int64_t i = 0; i < ncl;) {
      int64_t j = i + 1;
      while (j < ncl && cl[j].key == cl[i].key) ++j;
      if (j - i > 1)
        for (int64_t q = i; q < j; ++q) lost[cl[q].row] = 1;
      i = j;
    }
    /* commit */
    for (int64_t r = 0; r < nrows; ++r) {
      if (colors[r] >= 0) continue;
      if (lost[r]) {
        fails[r] += 1;
        continue;
      }
      const int32_t c = pick[r];
      colors[r] = c;
      if (c + 1 > ncol) ncol = c + 1;
      for (int k = 0; k < 4; ++k) {
        const int32_t v = rv[4 * r + k];
        if (free_vertex(s, v)) mask[(size_t)v * W + c / 64] |= 1ull << (c % 64);
      }
      --left;
    }
  }
  free(prio); free(fails); free(pick); free(lost); free(unc); free(mask); free(cl);
  return err ? -1 : ncol;
}

/* Greedy colouring in priority order, for the edge-length rows (colours kept for
 * a scene's steps, so their number, which sets the sweeps per backward step, counts
 * more than the time to find them): the rows are taken in decreasing priority,
 * prio = (high 32 bits of mix64(key ^ seed)) << 32 | key (keys below 2^32, so no two
 * rows tie), and each takes the smallest colour not used by an already coloured row
 * at one of its free vertices. Returns the colour count, or -1 past max_colors. */
typedef struct {
  uint64_t prio;
  int64_t row;
} prio_row_t;

static int cmp_prio_desc(const void* a, const void* b) {
  const prio_row_t *x = (const prio_row_t*)a, *y = (const prio_row_t*)b;
  if (x->prio != y->prio) return x->prio > y->prio ? -1 : 1;
  return 0;
}

uint64_t orc_greedy_prio(uint64_t key, uint64_t seed) {
  return (orc_mix64(key ^ seed) & 0xFFFFFFFF00000000ull) | (key & 0xFFFFFFFFull);
}

int32_t orc_color_rows_greedy(const orc_scene* s, int64_t nrows, const int32_t* rv,
                              const uint64_t* keys, int32_t* colors) {
  const int W = (s->p.max_colors + 63) / 64;
  const size_t NR = (size_t)(nrows > 0 ? nrows : 1);
  prio_row_t* order = (prio_row_t*)malloc(NR * sizeof(prio_row_t));
  uint64_t* mask = (uint64_t*)calloc((size_t)s->n * (size_t)W, sizeof(uint64_t));
  for (int64_t r = 0; r < nrows; ++r) {
    order[r].prio = orc_greedy_prio(keys[r], s->p.seed);
    order[r].row = r;
    colors[r] = -1;
  }
  qsort(order, (size_t)nrows, sizeof(prio_row_t), cmp_prio_desc);
  int32_t ncol = 0, err = 0;
  for (int64_t i = 0; i < nrows && !err; ++i) {
    const int64_t r = order[i].row;
    int32_t c = -1;
    for (int32_t q = 0; q < s->p.max_colors; ++q) {
      int used = 0;
      for (int k = 0; k < 4; ++k) {
        const int32_t v = rv[4 * r + k];
        if (free_vertex(s, v) && ((mask[(size_t)v * W + q / 64] >> (q % 64)) & 1ull)) used = 1;
      }
      if (!used) {
        c = q;
        break;
      }
    }
    if (c < 0) {
      err = 1;
      break;
    }
    colors[r] = c;
    if (c + 1 > ncol) ncol = c + 1;
    for (int k = 0; k < 4; ++k) {
      const int32_t v = rv[4 * r + k];
      if (free_vertex(s, v)) mask[(size_t)v * W + c / 64] |= 1ull << (c % 64);
    }
  }
  free(order);
  free(mask);
  return err ? -1 : ncol;
}

/* ------------------------------------------------------------- scene */

orc_scene* orc_create(int32_t n, const double* w, const int32_t* tris, int32_t nt,
                      const int32_t* edges, int32_t ne, const orc_params* p) {
  orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
  s->n = n;
  s->nt = nt;
  s->ne = ne;
  s->p = *p;
  size_t N = (size_t)(n > 0 ? n : 1);
  s->w = (double*)malloc(N * sizeof(double));
  memcpy(s->w, w, (size_t)n * sizeof(double));
  s->tris = (int32_t*)malloc((size_t)(nt > 0 ? nt : 1) * 3 * sizeof(int32_t));
  if (nt) memcpy(s->tris, tris, (size_t)nt * 3 * sizeof(int32_t));
  s->edges = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * 2 * sizeof(int32_t));
  if (ne) memcpy(s->edges, edges, (size_t)ne * 2 * sizeof(int32_t));
  s->stat = (uint8_t*)calloc(N, 1);
  /* particles: vertices no triangle or edge refers to */
  for (int32_t f = 0; f < 3 * nt; ++f) s->stat[tris[f]] = 1;
  for (int32_t e = 0; e < 2 * ne; ++e) s->stat[edges[e]] = 1;
  s->part = (int32_t*)malloc(N * sizeof(int32_t));
  s->np = 0;
  for (int32_t i = 0; i < n; ++i)
    if (!s->stat[i]) s->part[s->np++] = i;
  memset(s->stat, 0, N);
  s->x = (double*)malloc(N * 3 * sizeof(double));
  s->y = (double*)malloc(N * 3 * sizeof(double));
  s->xt = (double*)malloc(N * 3 * sizeof(double));
  s->xold = (double*)malloc(N * 3 * sizeof(double));
  s->r = (double*)malloc(N * sizeof(double));
  s->rold = (double*)malloc(N * sizeof(double));
  s->back = (uint8_t*)malloc(N);
  s->alpha = (double*)malloc(N * sizeof(double));
  s->scale = (double*)malloc(N * sizeof(double));
  s->Di = (double*)malloc(N * sizeof(double));
  s->move2 = (double*)malloc(N * sizeof(double));
  s->er_e = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(int32_t));
  s->er_v = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * 2 * sizeof(int32_t));
  s->er_g = (double*)malloc((size_t)(ne > 0 ? ne : 1) * 3 * sizeof(double));
  s->er_inv = (double*)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(double));
  s->er_col = (int32_t*)malloc((size_t)(ne > 0 ? ne : 1) * sizeof(int32_t));
  return s;
}

int32_t orc_particles(const orc_scene* s, int32_t* ids) {
  if (ids) memcpy(ids, s->part, (size_t)s->np * sizeof(int32_t));
  return s->np;
}

void orc_destroy(orc_scene* s) {
  if (!s) return;
  free(s->w); free(s->tris); free(s->edges); free(s->part); free(s->stat);
  free(s->x); free(s->y); free(s->xt); free(s->xold); free(s->r); free(s->rold);
  free(s->back); free(s->alpha); free(s->scale);
  free(s->Di); free(s->move2); free(s->P); free(s->A); free(s->acol);
  free(s->er_e); free(s->er_v); free(s->er_g); free(s->er_inv); free(s->er_col);
  free(s);
}

static void ensure_P(orc_scene* s, int64_t n) {
  if (n <= s->capP) return;
  s->capP = n + n / 2 + 16;
  s->P = (uint64_t*)realloc(s->P, (size_t)s->capP * sizeof(uint64_t));
  s->A = (uint64_t*)realloc(s->A, (size_t)s->capP * sizeof(uint64_t));
  s->acol = (int32_t*)realloc(s->acol, (size_t)s->capP * sizeof(int32_t));
}

/* Edge-length rows (Sec. 4.2): c = sigma - |x_i - x_j| / |y_i - y_j| linearised at
 * y = y^[k+1]: c_lin(y) = sigma - g . (y_i - y_j) with g = (y^_i - y^_j)/L^2,
 * J_i = -g, J_j = +g, A = (w_i + w_j) |g|^2. */
static int setup_edges(orc_scene* s) {
  s->n_er = 0;
  s->n_ecol = 0;
  if (!s->p.edge_len) return 0;
  for (int32_t e = 0; e < s->ne; ++e) {
    int32_t i = s->edges[2 * e], j = s->edges[2 * e + 1];
    if (!(s->w[i] > 0.0 || s->w[j] > 0.0)) continue;
    double d[3];
    sub3(d, s->xt + 3 * i, s->xt + 3 * j);
    double l2 = dot3(d, d);
    if (!(l2 > 0.0)) continue;
    int32_t r = s->n_er++;
    s->er_e[r] = e;
    s->er_v[2 * r] = i;
    s->er_v[2 * r + 1] = j;
    double* g = s->er_g + 3 * r;
    g[0] = d[0] / l2;
    g[1] = d[1] / l2;
    g[2] = d[2] / l2;
    double A = (s->w[i] + s->w[j]) * dot3(g, g);
    s->er_inv[r] = 1.0 / A;
  }
  if (s->n_er == 0) return 0;
  int32_t* rv = (int32_t*)malloc((size_t)s->n_er * 4 * sizeof(int32_t));
  uint64_t* keys = (uint64_t*)malloc((size_t)s->n_er * sizeof(uint64_t));
  for (int32_t r = 0; r < s->n_er; ++r) {
    rv[4 * r] = s->er_v[2 * r];
    rv[4 * r + 1] = s->er_v[2 * r + 1];
    rv[4 * r + 2] = -1;
    rv[4 * r + 3] = -1;
    keys[r] = (uint64_t)s->er_e[r];
  }
  int32_t nc = orc_color_rows_greedy(s, s->n_er, rv, keys, s->er_col);
  free(rv);
  free(keys);
  if (nc < 0) return -1;
  s->n_ecol = nc;
  return 0;
}

int orc_begin(orc_scene* s, const double* x_prev, const double* x_tilde) {
  size_t n3 = (size_t)s->n * 3;
  memcpy(s->x, x_prev, n3 * sizeof(double));
  memcpy(s->xt, x_tilde, n3 * sizeof(double));
  memcpy(s->y, x_tilde, n3 * sizeof(double));
  for (int32_t i = 0; i < s->n; ++i) {
    s->r[i] = 1.0;
    s->stat[i] = s->w[i] == 0.0 && x_prev[3 * i] == x_tilde[3 * i] &&
                 x_prev[3 * i + 1] == x_tilde[3 * i + 1] && x_prev[3 * i + 2] == x_tilde[3 * i + 2];
  }
  s->D = 0.0;
  s->nP = 0;
  s->nA = 0;
  return setup_edges(s);
}

static uint64_t fp_key(uint64_t k) { return orc_mix64(k ^ 0x6A09E667F3BCC909ull); }

/* Projected Jacobi backward step (Sec. 4.3.2: one projected Jacobi iteration in
 * place of the Gauss-Seidel sweep, with an under-relaxation factor). Every row
 * (contacts of A, then the edge-length rows; no colouring) is evaluated from the
 * same y: w = c0 + J.(y - x) (contacts) or sigma - g.(y_i - y_j) (edges),
 * lambda' = max(0, lambda - w/A), dl = lambda' - lambda, and the update w_v dl J_v of
 * each of its free vertices is added, in binary64 and in row order, to that
 * vertex's sum; then y_v += omega * sum_v. gs_sweeps such iterations run per
 * backward step, lambda carried between them. */
static int backward_jacobi(orc_scene* s, int64_t na, orc_iter* it) {
  const orc_params* p = &s->p;
  const int64_t NA = na > 0 ? na : 1;
  int32_t* rv = (int32_t*)malloc((size_t)NA * 4 * sizeof(int32_t));
  double* rc0 = (double*)malloc((size_t)NA * sizeof(double));
  double* rJ = (double*)malloc((size_t)NA * 12 * sizeof(double));
  double* rinv = (double*)malloc((size_t)NA * sizeof(double));
  double* lam = (double*)calloc((size_t)NA, sizeof(double));
  double* elam = (double*)calloc((size_t)(s->n_er > 0 ? s->n_er : 1), sizeof(double));
  double* acc = (double*)calloc((size_t)(s->n > 0 ? s->n : 1) * 3, sizeof(double));
  for (int64_t q = 0; q < na; ++q)
    orc_contact_row(s, s->x, s->A[q], rv + 4 * q, rc0 + q, rJ + 12 * q, rinv + q);
  it->n_colors = 0;
  for (int64_t q = 0; q < na; ++q) s->acol[q] = 0;  /* no colouring: every row in colour 0 */
  for (int sw = 0; sw < p->gs_sweeps; ++sw) {
    for (int64_t q = 0; q < na; ++q) {
      if (!(rinv[q] > 0.0)) continue;
      const double* J = rJ + 12 * q;
      double wr = rc0[q];
      for (int k = 0; k < 4; ++k) {
        const int32_t vv = rv[4 * q + k];
        if (vv < 0) continue;
        double dy[3];
        sub3(dy, s->y + 3 * vv, s->x + 3 * vv);
        wr = wr + dot3(J + 3 * k, dy);
      }
      double ln = lam[q] - wr * rinv[q];
      if (ln < 0.0) ln = 0.0;
      double dl = ln - lam[q];
      lam[q] = ln;
      for (int k = 0; k < 4; ++k) {
        const int32_t vv = rv[4 * q + k];
        if (vv < 0 || !(s->w[vv] > 0.0)) continue;
        double co = s->w[vv] * dl;
        for (int m = 0; m < 3; ++m) acc[3 * vv + m] = acc[3 * vv + m] + co * J[3 * k + m];
      }
    }
    for (int32_t q = 0; q < s->n_er; ++q) {
      const int32_t i = s->er_v[2 * q], j = s->er_v[2 * q + 1];
      const double* g = s->er_g + 3 * q;
      double dy[3];
      sub3(dy, s->y + 3 * i, s->y + 3 * j);
      double wr = p->sigma - dot3(g, dy);
      double ln = elam[q] - wr * s->er_inv[q];
      if (ln < 0.0) ln = 0.0;
      double dl = ln - elam[q];
      elam[q] = ln;
      if (s->w[i] > 0.0) {
        double co = s->w[i] * dl;
        for (int m = 0; m < 3; ++m) acc[3 * i + m] = acc[3 * i + m] - co * g[m];
      }
      if (s->w[j] > 0.0) {
        double co = s->w[j] * dl;
        for (int m = 0; m < 3; ++m) acc[3 * j + m] = acc[3 * j + m] + co * g[m];
      }
    }
    for (int64_t c = 0; c < 3 * (int64_t)s->n; ++c) {
      s->y[c] = s->y[c] + p->omega * acc[c];
      acc[c] = 0.0;
    }
  }
  free(rv); free(rc0); free(rJ); free(rinv); free(lam); free(elam); free(acc);
  return 0;
}

int orc_iterate(orc_scene* s, orc_iter* info) {
  const orc_params* p = &s->p;
  orc_iter it;
  memset(&it, 0, sizeof it);
  /* Alg. 1: search when the reuse bound has dropped below D_min (Sec. 3.1) */
  if (s->D < p->d_min) {
    int64_t n = orc_search(s, s->x, p->d_max, 0, NULL, 0);
    ensure_P(s, n);
    s->nP = orc_search(s, s->x, p->d_max, 0, s->P, s->capP);
    s->D = p->d_max;
    it.searched = 1;
  }
  const double D = s->D, D2 = D * D, dl2 = p->delta * p->delta;
  it.d_before = D;
  it.n_p = s->nP;

  /* pair pass: distances at x^(l); filter P by D (Sec. 3.1); activate below delta
   * (Sec. 4.1); per-vertex bound D_i (Sec. 5) */
  for (int32_t i = 0; i < s->n; ++i) s->Di[i] = D;
  int64_t npf = 0, na = 0;
  double* dpf = (double*)malloc((size_t)(s->nP > 0 ? s->nP : 1) * sizeof(double));
  for (int64_t q = 0; q < s->nP; ++q) {
    uint64_t key = s->P[q];
    int32_t v[4];
    double d2 = pair_d2(s, s->x, key, v);
    if (!(d2 < D2)) continue;
    dpf[npf] = d2;
    s->P[npf++] = key;
    double d = sqrt(d2);
    for (int k = 0; k < 4; ++k)
      if (v[k] >= 0 && d < s->Di[v[k]]) s->Di[v[k]] = d;
    if (d2 < dl2) s->A[na++] = key;
  }
  s->nP = npf;
  s->nA = na;
  it.n_pf = npf;
  it.n_a = na;

  if (p->backward == 1) {
    int rc = backward_jacobi(s, na, &it);
    if (rc != 0) {
      free(dpf);
      return rc;
    }
  } else {
  /* backward (Sec. 4): rows linearised at x^(l), coloured, one projected sweep */
  int32_t* rv = (int32_t*)malloc((size_t)(na > 0 ? na : 1) * 4 * sizeof(int32_t));
  double* rc0 = (double*)malloc((size_t)(na > 0 ? na : 1) * sizeof(double));
  double* rJ = (double*)malloc((size_t)(na > 0 ? na : 1) * 12 * sizeof(double));
  double* rinv = (double*)malloc((size_t)(na > 0 ? na : 1) * sizeof(double));
  double* lam = (double*)calloc((size_t)(na > 0 ? na : 1), sizeof(double));
  double* elam = (double*)calloc((size_t)(s->n_er > 0 ? s->n_er : 1), sizeof(double));
  for (int64_t q = 0; q < na; ++q)
    orc_contact_row(s, s->x, s->A[q], rv + 4 * q, rc0 + q, rJ + 12 * q, rinv + q);
  int32_t ncol = orc_color_rows(s, na, rv, s->A, s->acol);
  if (ncol < 0) {
    free(dpf); free(rv); free(rc0); free(rJ); free(rinv); free(lam); free(elam);
    return -2;
  }
  it.n_colors = ncol;
  for (int sw = 0; sw < p->gs_sweeps; ++sw) {
    for (int32_t c = 0; c < ncol; ++c)
      for (int64_t q = 0; q < na; ++q) {
        if (s->acol[q] != c || !(rinv[q] > 0.0)) continue;
        const double* J = rJ + 12 * q;
        double wr = rc0[q];
        for (int k = 0; k < 4; ++k) {
          const int32_t vv = rv[4 * q + k];
          if (vv < 0) continue;
          double dy[3];
          sub3(dy, s->y + 3 * vv, s->x + 3 * vv);
          wr = wr + dot3(J + 3 * k, dy);
        }
        double ln = lam[q] - wr * rinv[q];
        if (ln < 0.0) ln = 0.0;
        double dl = ln - lam[q];
        lam[q] = ln;
        for (int k = 0; k < 4; ++k) {
          const int32_t vv = rv[4 * q + k];
          if (vv < 0 || !(s->w[vv] > 0.0)) continue;
          double co = s->w[vv] * dl;
          for (int m = 0; m < 3; ++m) s->y[3 * vv + m] = s->y[3 * vv + m] + co * J[3 * k + m];
        }
      }
    for (int32_t c = 0; c < s->n_ecol; ++c)
      for (int32_t q = 0; q < s->n_er; ++q) {
        if (s->er_col[q] != c) continue;
        const int32_t i = s->er_v[2 * q], j = s->er_v[2 * q + 1];
        const double* g = s->er_g + 3 * q;
        double dy[3];
        sub3(dy, s->y + 3 * i, s->y + 3 * j);
        double wr = p->sigma - dot3(g, dy);
        double ln = elam[q] - wr * s->er_inv[q];
        if (ln < 0.0) ln = 0.0;
        double dl = ln - elam[q];
        elam[q] = ln;
        if (s->w[i] > 0.0) {
          double co = s->w[i] * dl;
          for (int m = 0; m < 3; ++m) s->y[3 * i + m] = s->y[3 * i + m] - co * g[m];
        }
        if (s->w[j] > 0.0) {
          double co = s->w[j] * dl;
          for (int m = 0; m < 3; ++m) s->y[3 * j + m] = s->y[3 * j + m] + co * g[m];
        }
      }
  }

  free(rv); free(rc0); free(rJ); free(rinv); free(lam); free(elam);
  }

  /* forward (Sec. 5, Eq. eq:forward2) */
  const double hg = 0.5 * p->gamma;
  double mmax = 0.0;
  memcpy(s->xold, s->x, (size_t)s->n * 3 * sizeof(double));
  memcpy(s->rold, s->r, (size_t)s->n * sizeof(double));
  for (int32_t i = 0; i < s->n; ++i) {
    double* xi = s->x + 3 * i;
    const double* yi = s->y + 3 * i;
    /* the CCD-based scheme bounds every vertex by D^(l) alone (the pairs it cannot
     * meet in one step); its contacts along P' are found afterwards */
    const double bound = p->ccd_step ? D : s->Di[i];
    double dx[3];
    sub3(dx, yi, xi);
    double n2 = dot3(dx, dx);
    double alpha = 1.0;
    if (n2 > 0.0) {
      double a = (hg * bound) / sqrt(n2);
      if (a < 1.0) alpha = a;
    }
    double xn[3];
    if (alpha == 1.0) {
      xn[0] = yi[0];
      xn[1] = yi[1];
      xn[2] = yi[2];
    } else {
      xn[0] = xi[0] + alpha * dx[0];
      xn[1] = xi[1] + alpha * dx[1];
      xn[2] = xi[2] + alpha * dx[2];
    }
    double mv[3];
    sub3(mv, xn, xi);
    double m2 = dot3(mv, mv);
    /* the lemma of Sec. 5 for the rounded move: the vertex advances only when
     * 2 |x_new - x| < D_i - eta, eta = ORC_ETA covering the rounding of the
     * distances; otherwise it stays (alpha = 0). In exact arithmetic with
     * gamma < 1 the test fails only when D_i <= eta / (1 - gamma). */
    const double sb = bound - ORC_ETA;
    if (!p->unguarded && !(sb > 0.0 && 4.0 * m2 < sb * sb)) {
      xn[0] = xi[0];
      xn[1] = xi[1];
      xn[2] = xi[2];
      m2 = 0.0;
      alpha = 0.0;
    }
    s->move2[i] = m2;
    s->alpha[i] = alpha;
    double mvn = sqrt(m2);
    if (mvn > mmax) mmax = mvn;
    xi[0] = xn[0];
    xi[1] = xn[1];
    xi[2] = xn[2];
    s->r[i] = s->r[i] * (1.0 - alpha);
  }

  /* path certificate on P' along x^(l) -> x^(l+1) (Sec. 5 and Sec. 5.1). A pair
   * is certified when no vertex of it moved half the pair distance (the lemma:
   * 4 max_v |dx_v|^2 < d^2); the others take the continuous test of the piece.
   * A pair the test does not clear sends its vertices back to x^(l) (alpha = 0,
   * r unchanged). That changes the piece of every pair sharing those vertices, so
   * the pass repeats until it returns no new vertex (the returned set only grows).
   * With ccd_all every pair takes the continuous test in every pass; a pair the
   * motion bound certifies is never sent back.
   * The CCD-based scheme of Sec. 5.1 (ccd_step) answers its first ORC_STEP_PASSES
   * passes differently: a pair in contact at time t* of its piece scales the steps
   * of its moving vertices by gamma t* (a vertex takes the smallest factor of its pairs;
   * alpha <- alpha factor, x <- x^(l) + alpha (y - x^(l)), r <- r^(l) (1 - alpha)),
   * and the passes go on while they find contacts. */
  int64_t fail = 0, hits = 0, nback = 0, nscaled = 0;
  memset(s->back, 0, (size_t)s->n);
  for (int32_t i = 0; i < s->n; ++i) s->scale[i] = 1.0;
  for (int pass = 0;; ++pass) {
    const int scaling = p->ccd_step && pass < ORC_STEP_PASSES;
    int64_t newly = 0;
    for (int64_t q = 0; q < npf; ++q) {
      int32_t v[4];
      pair_verts(s, s->P[q], v);
      const int nv = (s->P[q] & KEY_VV) ? 2 : 4;
      double mv = s->move2[v[0]];
      for (int k = 1; k < nv; ++k)
        if (s->move2[v[k]] > mv) mv = s->move2[v[k]];
      const int bound_ok = 4.0 * mv < dpf[q];
      if (bound_ok && !p->ccd_all) continue;
      ++fail;
      double qq[12], dq[12];
      for (int k = 0; k < nv; ++k)
        for (int m = 0; m < 3; ++m) {
          qq[3 * k + m] = s->xold[3 * v[k] + m];
          dq[3 * k + m] = s->x[3 * v[k] + m] - s->xold[3 * v[k] + m];
        }
      const int kind = (s->P[q] & KEY_VV) ? 2 : ((s->P[q] & KEY_EE) ? 1 : 0);
      double th = 0.0;
      if (!orc_ccd_hit(qq, dq, kind, ORC_ETA, &th)) continue;
      ++hits;
      if (bound_ok) continue;
      if (scaling) {
        const double f = p->gamma * th;
        for (int k = 0; k < nv; ++k)
          if (f < s->scale[v[k]]) s->scale[v[k]] = f;
        ++newly;
      } else {
        for (int k = 0; k < nv; ++k)
          if (!s->back[v[k]]) {
            s->back[v[k]] = 2;
            ++newly;
          }
      }
    }
    if (newly == 0) break;
    if (scaling) {
      for (int32_t i = 0; i < s->n; ++i) {
        if (!(s->scale[i] < 1.0)) continue;
        const double a = s->alpha[i] * s->scale[i];
        s->scale[i] = 1.0;
        if (s->move2[i] == 0.0) continue; /* no step to scale */
        s->alpha[i] = a;
        double* xi = s->x + 3 * i;
        const double *x0 = s->xold + 3 * i, *yi = s->y + 3 * i;
        double dx[3], mvv[3];
        sub3(dx, yi, x0);
        for (int m = 0; m < 3; ++m) xi[m] = x0[m] + a * dx[m];
        sub3(mvv, xi, x0);
        s->move2[i] = dot3(mvv, mvv);
        s->r[i] = s->rold[i] * (1.0 - a);
        ++nscaled;
      }
      continue;
    }
    nback += newly;
    for (int32_t i = 0; i < s->n; ++i) {
      if (s->back[i] != 2) continue;
      s->back[i] = 1;
      memcpy(s->x + 3 * i, s->xold + 3 * i, 3 * sizeof(double));
      s->r[i] = s->rold[i];
      s->move2[i] = 0.0;
    }
  }
  it.ccd_fail = fail;
  it.ccd_hits = hits;
  it.n_back = nback;
  it.n_scaled = nscaled;
  double rinf = 0.0;
  for (int32_t i = 0; i < s->n; ++i)
    if (s->r[i] > rinf) rinf = s->r[i];

  s->D = D - 2.0 * mmax;
  it.d_after = s->D;
  it.move_max = mmax;
  it.r_inf = rinf;
  for (int64_t q = 0; q < npf; ++q) it.fp_pf += fp_key(s->P[q]);
  for (int64_t q = 0; q < na; ++q) {
    it.fp_a += fp_key(s->A[q]);
    it.fp_col += orc_mix64(fp_key(s->A[q]) ^ (uint64_t)s->acol[q]);
  }
  free(dpf);
  if (info) *info = it;
  return rinf < p->eps ? 1 : 0;
}

int orc_run(orc_scene* s, double* x_out, orc_iter* trace, int32_t trace_cap) {
  int l = 0;
  for (; l < s->p.max_iters; ++l) {
    orc_iter it;
    int rc = orc_iterate(s, &it);
    if (rc < 0) return rc;
    if (trace && l < trace_cap) trace[l] = it;
    if (rc == 1) {
      ++l;
      break;
    }
  }
  if (x_out) memcpy(x_out, s->x, (size_t)s->n * 3 * sizeof(double));
  return l;
}

void orc_get_state(const orc_scene* s, double* x, double* y, double* r, double* D) {
  size_t n3 = (size_t)s->n * 3;
  if (x) memcpy(x, s->x, n3 * sizeof(double));
  if (y) memcpy(y, s->y, n3 * sizeof(double));
  if (r) memcpy(r, s->r, (size_t)s->n * sizeof(double));
  if (D) *D = s->D;
}

int orc_set_state(orc_scene* s, const double* x, const double* y, const double* r, double D,
                  const uint64_t* P, int64_t nP) {
  size_t n3 = (size_t)s->n * 3;
  memcpy(s->x, x, n3 * sizeof(double));
  memcpy(s->y, y, n3 * sizeof(double));
  memcpy(s->r, r, (size_t)s->n * sizeof(double));
  s->D = D;
  ensure_P(s, nP);
  if (nP) memcpy(s->P, P, (size_t)nP * sizeof(uint64_t));
  s->nP = nP;
  return 0;
}

int64_t orc_get_P(const orc_scene* s, uint64_t* out, int64_t cap) {
  if (out && cap >= s->nP) memcpy(out, s->P, (size_t)s->nP * sizeof(uint64_t));
  return s->nP;
}

int64_t orc_get_A(const orc_scene* s, uint64_t* keys, int32_t* colors, int64_t cap) {
  if (keys && cap >= s->nA) memcpy(keys, s->A, (size_t)s->nA * sizeof(uint64_t));
  if (colors && cap >= s->nA) memcpy(colors, s->acol, (size_t)s->nA * sizeof(int32_t));
  return s->nA;
}

void orc_get_Di(const orc_scene* s, double* out) {
  memcpy(out, s->Di, (size_t)s->n * sizeof(double));
}

/* ----------------------------------------------------------- normal flow */

/* Target of the globally injective normal flow (Sec. 7.4, Eq. eq:normal flow):
 * y_0 = x + beta n with n the vertex normal field at x, then `iters` Jacobi steps
 * y_{i+1}(v) = y_i(v) + alpha L y_i(v) with L the cotangent Laplace-Beltrami
 * operator of the mesh at y_i. Readings: n_v = normalised sum, over the triangles
 * at v in increasing index, of (x_b - x_a) x (x_c - x_a) (area weighted; 0 when the
 * sum vanishes); L y(v) = (1 / (2 A_v)) sum over the triangles at v of
 * [cot_r (y_q - y_v) + cot_q (y_r - y_v)], (v, q, r) the triangle rotated to start
 * at v, cot_q the cotangent of its angle at q (0 for a degenerate triangle),
 * A_v = sum of a third of those triangles' areas (barycentric area; a vertex with
 * A_v = 0 does not move). */
static void nf_rotate(const int32_t* t, int32_t v, int32_t* q, int32_t* r) {
  if (t[0] == v) {
    *q = t[1];
    *r = t[2];
  } else if (t[1] == v) {
    *q = t[2];
    *r = t[0];
  } else {
    *q = t[0];
    *r = t[1];
  }
}

/* cotangent of the angle at b of triangle (a, b, c) */
static double nf_cot(const double* a, const double* b, const double* c) {
  double u[3], w[3], k[3];
  sub3(u, a, b);
  sub3(w, c, b);
  cross3(k, u, w);
  double s = sqrt(dot3(k, k));
  if (s == 0.0) return 0.0;
  return dot3(u, w) / s;
}

int orc_normal_flow(int32_t n, const double* x, const int32_t* tris, int32_t nt, double beta,
                    double alpha, int32_t iters, double* y_out) {
  if (n < 0 || nt < 0 || iters < 0) return -1;
  /* incident triangles of each vertex, in increasing index */
  int32_t* cnt = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  for (int32_t f = 0; f < 3 * nt; ++f) {
    if (tris[f] < 0 || tris[f] >= n) {
      free(cnt);
      return -1;
    }
    cnt[tris[f] + 1] += 1;
  }
  for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  int32_t* inc = (int32_t*)malloc((size_t)(3 * nt > 0 ? 3 * nt : 1) * sizeof(int32_t));
  int32_t* cur = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int32_t v = 0; v < n; ++v) cur[v] = cnt[v];
  for (int32_t f = 0; f < nt; ++f)
    for (int k = 0; k < 3; ++k) inc[cur[tris[3 * f + k]]++] = f;
  double* ya = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
  double* yb = (double*)malloc((size_t)(n > 0 ? n : 1) * 3 * sizeof(double));
  /* y_0 = x + beta n */
  for (int32_t v = 0; v < n; ++v) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int32_t i = cnt[v]; i < cnt[v + 1]; ++i) {
      const int32_t* t = tris + 3 * inc[i];
      double e1[3], e2[3], N[3];
      sub3(e1, x + 3 * t[1], x + 3 * t[0]);
      sub3(e2, x + 3 * t[2], x + 3 * t[0]);
      cross3(N, e1, e2);
      for (int k = 0; k < 3; ++k) s[k] = s[k] + N[k];
    }
    double len = sqrt(dot3(s, s));
    for (int k = 0; k < 3; ++k) {
      double nk = len > 0.0 ? s[k] / len : 0.0;
      ya[3 * v + k] = x[3 * v + k] + beta * nk;
    }
  }
  /* Jacobi smoothing steps */
  for (int32_t it = 0; it < iters; ++it) {
    for (int32_t v = 0; v < n; ++v) {
      double L[3] = {0.0, 0.0, 0.0}, A = 0.0;
      const double* p = ya + 3 * v;
      for (int32_t i = cnt[v]; i < cnt[v + 1]; ++i) {
        int32_t q, r;
        nf_rotate(tris + 3 * inc[i], v, &q, &r);
        const double *yq = ya + 3 * q, *yr = ya + 3 * r;
        const double cq = nf_cot(p, yq, yr), cr = nf_cot(p, yr, yq);
        double dq[3], dr[3], k3[3];
        sub3(dq, yq, p);
        sub3(dr, yr, p);
        for (int k = 0; k < 3; ++k) {
          L[k] = L[k] + cr * dq[k];
          L[k] = L[k] + cq * dr[k];
        }
        cross3(k3, dq, dr);
        A = A + (0.5 * sqrt(dot3(k3, k3))) / 3.0;
      }
      for (int k = 0; k < 3; ++k)
        yb[3 * v + k] = A > 0.0 ? p[k] + alpha * (L[k] / (2.0 * A)) : p[k];
    }
    double* t = ya;
    ya = yb;
    yb = t;
  }
  memcpy(y_out, ya, (size_t)n * 3 * sizeof(double));
  free(cnt); free(inc); free(cur); free(ya); free(yb);
  return 0;
}
