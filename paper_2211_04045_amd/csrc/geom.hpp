// Device geometry of the two-way collision step: distances, contact rows.
//
// Compiled with -ffp-contract=off: every expression below is evaluated as
// written, left to right, in binary64 with correctly rounded sqrt and
// division, so that the results do not depend on the compiler's choice of
// fused operations. The operation order is the project's written geometry
// specification; see the design notes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cc {

struct V3 {
  double x, y, z;
};

__device__ __forceinline__ V3 ld3(const double* __restrict__ p, int32_t i) {
  const double* q = p + 3 * (int64_t)i;
  return V3{q[0], q[1], q[2]};
}
__device__ __forceinline__ void st3(double* __restrict__ p, int32_t i, V3 v) {
  double* q = p + 3 * (int64_t)i;
  q[0] = v.x;
  q[1] = v.y;
  q[2] = v.z;
}
__device__ __forceinline__ V3 vsub(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double vdot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 vcross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// u + s*v per component
__device__ __forceinline__ V3 vaxpy(V3 u, double s, V3 v) {
  return V3{u.x + s * v.x, u.y + s * v.y, u.z + s * v.z};
}

// |p - q|^2 for the closest point q of segment [u,v]; t its parameter.
__device__ __forceinline__ double pt_seg_d2(V3 p, V3 u, V3 v, double& t) {
  V3 uv = vsub(v, u);
  V3 up = vsub(p, u);
  double l2 = vdot(uv, uv);
  double s = 0.0;
  if (l2 > 0.0) {
    s = vdot(up, uv) / l2;
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
  }
  V3 q = vaxpy(u, s, uv);
  V3 d = vsub(p, q);
  t = s;
  return vdot(d, d);
}

// Point-triangle: interior projection candidate (when inside), then edges
// (a,b), (b,c), (c,a); first strict minimum. bw = closest point weights; which =
// the winning candidate (0 interior, 1..3 the edges, -1 none).
__device__ __forceinline__ double pt_tri_d2(V3 p, V3 a, V3 b, V3 c, double bw[3], int& which) {
  V3 ab = vsub(b, a), ac = vsub(c, a), ap = vsub(p, a);
  V3 n = vcross(ab, ac);
  double nn = vdot(n, n);
  double best = __builtin_inf();
  which = -1;
  bw[0] = 1.0;
  bw[1] = 0.0;
  bw[2] = 0.0;
  if (nn > 0.0) {
    V3 t1 = vcross(ap, ac);
    V3 t2 = vcross(ab, ap);
    double wb = vdot(t1, n) / nn;
    double wc = vdot(t2, n) / nn;
    double wa = 1.0 - wb - wc;
    if (wa >= 0.0 && wb >= 0.0 && wc >= 0.0) {
      double h = vdot(ap, n);
      best = h * h / nn;
      which = 0;
      bw[0] = wa;
      bw[1] = wb;
      bw[2] = wc;
    }
  }
  double t, e2;
  e2 = pt_seg_d2(p, a, b, t);
  if (e2 < best) {
    best = e2;
    which = 1;
    bw[0] = 1.0 - t;
    bw[1] = t;
    bw[2] = 0.0;
  }
  e2 = pt_seg_d2(p, b, c, t);
  if (e2 < best) {
    best = e2;
    which = 2;
    bw[0] = 0.0;
    bw[1] = 1.0 - t;
    bw[2] = t;
  }
  e2 = pt_seg_d2(p, c, a, t);
  if (e2 < best) {
    best = e2;
    which = 3;
    bw[0] = t;
    bw[1] = 0.0;
    bw[2] = 1.0 - t;
  }
  return best;
}
__device__ __forceinline__ double pt_tri_d2(V3 p, V3 a, V3 b, V3 c, double bw[3]) {
  int which;
  return pt_tri_d2(p, a, b, c, bw, which);
}

// Segment-segment: interior stationary point (non-parallel, inside the unit
// square), then endpoint candidates a|ce, b|ce, c|ab, e|ab; first strict minimum.
// which = the winning candidate (0 interior, 1..4 the endpoint candidates).
__device__ __forceinline__ double seg_seg_d2(V3 a, V3 b, V3 c, V3 e, double& bs, double& bt,
                                             int& which) {
  V3 d1 = vsub(b, a), d2 = vsub(e, c), r = vsub(a, c);
  double A = vdot(d1, d1), B = vdot(d1, d2), C = vdot(d2, d2);
  double Dd = vdot(d1, r), Ee = vdot(d2, r);
  double den = A * C - B * B;
  double best = __builtin_inf();
  which = -1;
  bs = 0.0;
  bt = 0.0;
  if (den > 0.0) {
    double s = (B * Ee - C * Dd) / den;
    double t = (A * Ee - B * Dd) / den;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
      V3 p = vaxpy(a, s, d1);
      V3 q = vaxpy(c, t, d2);
      V3 d = vsub(p, q);
      best = vdot(d, d);
      which = 0;
      bs = s;
      bt = t;
    }
  }
  double u, e2;
  e2 = pt_seg_d2(a, c, e, u);
  if (e2 < best) { best = e2; bs = 0.0; bt = u; which = 1; }
  e2 = pt_seg_d2(b, c, e, u);
  if (e2 < best) { best = e2; bs = 1.0; bt = u; which = 2; }
  e2 = pt_seg_d2(c, a, b, u);
  if (e2 < best) { best = e2; bs = u; bt = 0.0; which = 3; }
  e2 = pt_seg_d2(e, a, b, u);
  if (e2 < best) { best = e2; bs = u; bt = 1.0; which = 4; }
  return best;
}
__device__ __forceinline__ double seg_seg_d2(V3 a, V3 b, V3 c, V3 e, double& bs, double& bt) {
  int which;
  return seg_seg_d2(a, b, c, e, bs, bt, which);
}

// Pair keys: bit 63 = edge-edge, bit 62 = vertex-vertex; bits 61..32 = first
// primitive (vertex or edge), bits 31..0 = second primitive (triangle, edge or
// vertex). Primitive ids are below 2^30.
constexpr uint64_t KEY_EE = 1ull << 63;
constexpr uint64_t KEY_VV = 1ull << 62;
__device__ __forceinline__ bool key_is_ee(uint64_t k) { return (k & KEY_EE) != 0; }
__device__ __forceinline__ bool key_is_vv(uint64_t k) { return (k & KEY_VV) != 0; }
__device__ __forceinline__ uint32_t key_a(uint64_t k) { return (uint32_t)((k >> 32) & 0x3fffffffu); }
__device__ __forceinline__ uint32_t key_b(uint64_t k) { return (uint32_t)(k & 0xffffffffu); }

struct Topo {
  const int32_t* __restrict__ tris;
  const int32_t* __restrict__ edges;
};

// The pair's four vertices; a vertex-vertex pair (a, b) lists (a, b, a, b), so
// that loads, minima and maxima over the four need no special case (sums and
// updates take the first two only).
__device__ __forceinline__ void pair_verts(const Topo& T, uint64_t k, int32_t v[4]) {
  uint32_t a = key_a(k), b = key_b(k);
  if (key_is_vv(k)) {
    v[0] = (int32_t)a;
    v[1] = (int32_t)b;
    v[2] = (int32_t)a;
    v[3] = (int32_t)b;
  } else if (key_is_ee(k)) {
    v[0] = T.edges[2 * a];
    v[1] = T.edges[2 * a + 1];
    v[2] = T.edges[2 * b];
    v[3] = T.edges[2 * b + 1];
  } else {
    v[0] = (int32_t)a;
    v[1] = T.tris[3 * b];
    v[2] = T.tris[3 * b + 1];
    v[3] = T.tris[3 * b + 2];
  }
}

__device__ __forceinline__ double pair_d2(uint64_t key, V3 p0, V3 p1, V3 p2, V3 p3) {
  if (key_is_vv(key)) {
    const V3 d = vsub(p0, p1);
    return vdot(d, d);
  }
  if (key_is_ee(key)) {
    double s, t;
    return seg_seg_d2(p0, p1, p2, p3, s, t);
  }
  double bw[3];
  return pt_tri_d2(p0, p1, p2, p3, bw);
}

// det[q1-q0, q2-q0, q3-q0]
__device__ __forceinline__ double det4(V3 q0, V3 q1, V3 q2, V3 q3) {
  V3 e1 = vsub(q1, q0), e2 = vsub(q2, q0), e3 = vsub(q3, q0);
  return vdot(e1, vcross(e2, e3));
}

struct Row {
  double c0;
  double inv_a;  // 0 = inactive
  V3 J[4];
};

// Contact row at x: volume form (Sec. 4.1: reference shape separated by delta
// along the normal, c = V(x)/V(r) - 1, J = grad V(x) / V(r)) when both closest
// points are interior (the normal is then their separating direction) and the
// tetrahedron is not near degenerate; otherwise the gap form c = d/delta - 1,
// J_v = omega_v u / delta. w = inverse masses of the four vertices.
__device__ __forceinline__ void contact_row(bool ee, const V3 xs[4], const double w[4],
                                            double delta, double kappa2, Row& R) {
  double om[4], d2, bw[3], s0 = 0.0, t0 = 0.0;
  bool volume_ok;
  int which;
  V3 N;
  double side;
  if (ee) {
    d2 = seg_seg_d2(xs[0], xs[1], xs[2], xs[3], s0, t0, which);
    om[0] = 1.0 - s0;
    om[1] = s0;
    om[2] = -(1.0 - t0);
    om[3] = -t0;
    V3 d1v = vsub(xs[1], xs[0]), d2v = vsub(xs[3], xs[2]);
    N = vcross(d1v, d2v);
    double mm = vdot(N, N);
    double l1 = vdot(d1v, d1v), l2 = vdot(d2v, d2v);
    volume_ok = mm > kappa2 * (l1 * l2);
    V3 ac = vsub(xs[0], xs[2]);
    side = vdot(ac, N) >= 0.0 ? 1.0 : -1.0;
  } else {
    d2 = pt_tri_d2(xs[0], xs[1], xs[2], xs[3], bw, which);
    om[0] = 1.0;
    om[1] = -bw[0];
    om[2] = -bw[1];
    om[3] = -bw[2];
    V3 e1 = vsub(xs[2], xs[1]), e2 = vsub(xs[3], xs[1]), e3 = vsub(xs[3], xs[2]);
    N = vcross(e1, e2);
    double nn = vdot(N, N);
    double l = vdot(e1, e1), m2 = vdot(e2, e2), m3 = vdot(e3, e3);
    if (m2 > l) l = m2;
    if (m3 > l) l = m3;
    volume_ok = nn > kappa2 * (l * l);
    V3 ai = vsub(xs[0], xs[1]);
    side = vdot(ai, N) >= 0.0 ? 1.0 : -1.0;
  }
  if (which != 0) volume_ok = false;
  double d = sqrt(d2);
  R.inv_a = 0.0;
  if (volume_ok) {
    double g = 0.5 * (delta - d);
    double scale = side / sqrt(vdot(N, N));
    V3 off = V3{g * (N.x * scale), g * (N.y * scale), g * (N.z * scale)};
    V3 r0 = V3{xs[0].x + off.x, xs[0].y + off.y, xs[0].z + off.z};
    V3 r1 = ee ? V3{xs[1].x + off.x, xs[1].y + off.y, xs[1].z + off.z}
               : V3{xs[1].x - off.x, xs[1].y - off.y, xs[1].z - off.z};
    V3 r2 = V3{xs[2].x - off.x, xs[2].y - off.y, xs[2].z - off.z};
    V3 r3 = V3{xs[3].x - off.x, xs[3].y - off.y, xs[3].z - off.z};
    double vr = det4(r0, r1, r2, r3);
    if (vr == 0.0) return;
    double vx = det4(xs[0], xs[1], xs[2], xs[3]);
    R.c0 = vx / vr - 1.0;
    V3 e1 = vsub(xs[1], xs[0]), e2 = vsub(xs[2], xs[0]), e3 = vsub(xs[3], xs[0]);
    V3 G1 = vcross(e2, e3), G2 = vcross(e3, e1), G3 = vcross(e1, e2);
    V3 G0 = V3{-((G1.x + G2.x) + G3.x), -((G1.y + G2.y) + G3.y), -((G1.z + G2.z) + G3.z)};
    R.J[0] = V3{G0.x / vr, G0.y / vr, G0.z / vr};
    R.J[1] = V3{G1.x / vr, G1.y / vr, G1.z / vr};
    R.J[2] = V3{G2.x / vr, G2.y / vr, G2.z / vr};
    R.J[3] = V3{G3.x / vr, G3.y / vr, G3.z / vr};
  } else {
    V3 diff;
    if (ee) {
      V3 d1v = vsub(xs[1], xs[0]), d2v = vsub(xs[3], xs[2]);
      V3 p = vaxpy(xs[0], s0, d1v);
      V3 q = vaxpy(xs[2], t0, d2v);
      diff = vsub(p, q);
    } else {
      V3 p = V3{(bw[0] * xs[1].x + bw[1] * xs[2].x) + bw[2] * xs[3].x,
                (bw[0] * xs[1].y + bw[1] * xs[2].y) + bw[2] * xs[3].y,
                (bw[0] * xs[1].z + bw[1] * xs[2].z) + bw[2] * xs[3].z};
      diff = vsub(xs[0], p);
    }
    double dd = sqrt(vdot(diff, diff));
    if (dd == 0.0) return;
    V3 u = V3{diff.x / dd, diff.y / dd, diff.z / dd};
    R.c0 = d / delta - 1.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double co = om[i] / delta;
      R.J[i] = V3{co * u.x, co * u.y, co * u.z};
    }
  }
  double A = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) A = A + w[i] * vdot(R.J[i], R.J[i]);
  R.inv_a = A > 0.0 ? 1.0 / A : 0.0;
}

// Vertex-vertex row (Sec. 4.1): c = |x_a - x_b|/delta - 1 at x, J_a = u/delta,
// J_b = -u/delta with u the unit vector from b to a; slots 2 and 3 carry zero.
// Coincident points give no row.
__device__ __forceinline__ void contact_row_vv(const V3 xs[4], const double w[4], double delta,
                                               Row& R) {
  R.inv_a = 0.0;
  const V3 diff = vsub(xs[0], xs[1]);
  const double d = sqrt(vdot(diff, diff));
  R.J[2] = V3{0.0, 0.0, 0.0};
  R.J[3] = V3{0.0, 0.0, 0.0};
  if (d == 0.0) return;
  const V3 u = V3{diff.x / d, diff.y / d, diff.z / d};
  const double c0 = 1.0 / delta, c1 = -1.0 / delta;
  R.J[0] = V3{c0 * u.x, c0 * u.y, c0 * u.z};
  R.J[1] = V3{c1 * u.x, c1 * u.y, c1 * u.z};
  double A = w[0] * vdot(R.J[0], R.J[0]);
  A = A + w[1] * vdot(R.J[1], R.J[1]);
  R.c0 = d / delta - 1.0;
  R.inv_a = A > 0.0 ? 1.0 / A : 0.0;
}

// Continuous test of one pair along the linear piece q_k(t) = q_k + t dq_k,
// t in [0,1] (points in the contact-row order); contact means a distance <= eta.
// The distance is probed at t = 0; at the times where the four points are
// coplanar, V(t) = det[q1-q0, q2-q0, q3-q0](t) = 0, a cubic a3 t^3 + a2 t^2 + a1 t
// + a0 whose critical points split [0,1] into monotone pieces (a sign change is
// bisected to the root), and at those critical points; then the piece is swept by
// conservative advancement (Mirtich's method: the distance changes at most at rate
// Lc = max |dq| over the first primitive + max |dq| over the second, so from a time
// t with distance d > eta no contact occurs before t + (d - eta) / Lc; this also
// covers a piece that stays coplanar, which the cubic cannot see; a piece not
// cleared within kCaSteps advances counts as a contact) and probed at t = 1.
// Returns the time of the contact found (the earliest probe or advance that found
// it), or -1 when the piece is clear. FP64 throughout.
constexpr int kCaSteps = 1024;

__device__ __forceinline__ double cubic_at(const double a[4], double t) {
  return ((a[3] * t + a[2]) * t + a[1]) * t + a[0];
}

__device__ __forceinline__ double ccd_dist2(const V3 q[4], const V3 dq[4], bool ee, double t) {
  V3 p0 = vaxpy(q[0], t, dq[0]), p1 = vaxpy(q[1], t, dq[1]);
  V3 p2 = vaxpy(q[2], t, dq[2]), p3 = vaxpy(q[3], t, dq[3]);
  return pair_d2(ee ? KEY_EE : 0ull, p0, p1, p2, p3);
}

__device__ __forceinline__ bool ccd_probe(const V3 q[4], const V3 dq[4], bool ee, double t,
                                          double eta2) {
  return ccd_dist2(q, dq, ee, t) <= eta2;
}

__device__ __noinline__ double ccd_hit(const V3 q[4], const V3 dq[4], bool ee, double eta) {
  const double eta2 = eta * eta;
  if (ccd_probe(q, dq, ee, 0.0, eta2)) return 0.0;
  V3 e1 = vsub(q[1], q[0]), e2 = vsub(q[2], q[0]), e3 = vsub(q[3], q[0]);
  V3 f1 = vsub(dq[1], dq[0]), f2 = vsub(dq[2], dq[0]), f3 = vsub(dq[3], dq[0]);
  V3 c23 = vcross(e2, e3), f2e3 = vcross(f2, e3), e2f3 = vcross(e2, f3), f2f3 = vcross(f2, f3);
  double a[4];
  a[0] = vdot(e1, c23);
  a[1] = vdot(f1, c23) + vdot(e1, f2e3) + vdot(e1, e2f3);
  a[2] = vdot(f1, f2e3) + vdot(f1, e2f3) + vdot(e1, f2f3);
  a[3] = vdot(f1, f2f3);
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
    if (t >= 0.0 && ccd_probe(q, dq, ee, t, eta2)) return t;
    if (i + 2 < nk && ccd_probe(q, dq, ee, knot[i + 1], eta2)) return knot[i + 1];
  }
  // conservative advancement over the piece
  double l1 = 0.0, l2 = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double mk = sqrt(vdot(dq[k], dq[k]));
    if (k < (ee ? 2 : 1)) {
      if (mk > l1) l1 = mk;
    } else if (mk > l2) {
      l2 = mk;
    }
  }
  const double lc = l1 + l2;
  double t = 0.0;
  bool cleared = !(lc > 0.0);
  for (int step = 0; step < kCaSteps && !cleared; ++step) {
    const double d = sqrt(ccd_dist2(q, dq, ee, t));
    if (d <= eta) return t;
    t = t + (d - eta) / lc;
    if (t >= 1.0) cleared = true;
  }
  if (!cleared) return t;
  return ccd_probe(q, dq, ee, 1.0, eta2) ? 1.0 : -1.0;
}

// Sign of det[b-a, c-a, d-a] (d against the plane of a, b, c); 0 when the FP64
// value lies within 1e-12 of the sum of the absolute products (touching).
__device__ __forceinline__ int orient_band(V3 a, V3 b, V3 c, V3 d) {
  const V3 u = vsub(b, a), v = vsub(c, a), w = vsub(d, a);
  const double o = vdot(vcross(u, v), w);
  const double perm = (fabs(u.y * v.z) + fabs(u.z * v.y)) * fabs(w.x) +
                      (fabs(u.z * v.x) + fabs(u.x * v.z)) * fabs(w.y) +
                      (fabs(u.x * v.y) + fabs(u.y * v.x)) * fabs(w.z);
  const double band = 1e-12 * perm;
  return o > band ? 1 : (o < -band ? -1 : 0);
}

// Does segment pq meet triangle abc (crossing or touching)? Off the plane: the
// endpoints are not strictly on one side and the line pq passes through the closed
// triangle; in the plane: the FP64 distance is at most tol.
__device__ __forceinline__ bool seg_tri_meet(V3 p, V3 q, V3 a, V3 b, V3 c, double tol) {
  const int sp = orient_band(a, b, c, p), sq = orient_band(a, b, c, q);
  if (sp == 0 && sq == 0) {
    double s_, t_, bw[3];
    double d2 = seg_seg_d2(p, q, a, b, s_, t_), t;
    t = seg_seg_d2(p, q, b, c, s_, t_);
    if (t < d2) d2 = t;
    t = seg_seg_d2(p, q, c, a, s_, t_);
    if (t < d2) d2 = t;
    t = pt_tri_d2(p, a, b, c, bw);
    if (t < d2) d2 = t;
    t = pt_tri_d2(q, a, b, c, bw);
    if (t < d2) d2 = t;
    return d2 <= tol * tol;
  }
  if (sp * sq > 0) return false;
  const int s1 = orient_band(p, q, a, b), s2 = orient_band(p, q, b, c), s3 = orient_band(p, q, c, a);
  return (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
}

// Vertex-vertex continuous test: the closest approach of two linearly moving
// points, at t = clamp(-(p.dp)/(dp.dp), 0, 1) with p = qa - qb, dp = dqa - dqb
// (t = 0 when they move together); contact when their distance there is <= eta.
// Returns that time on a contact, else -1.
__device__ __forceinline__ double ccd_hit_vv(V3 qa, V3 qb, V3 dqa, V3 dqb, double eta2) {
  const V3 p = vsub(qa, qb), dp = vsub(dqa, dqb);
  const double dd = vdot(dp, dp);
  double t = 0.0;
  if (dd > 0.0) {
    t = -vdot(p, dp) / dd;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
  }
  const V3 e = vsub(vaxpy(qa, t, dqa), vaxpy(qb, t, dqb));
  return vdot(e, e) <= eta2 ? t : -1.0;
}

// splitmix64 output function (Steele, Lea, Flood 2014); a bijection on 64 bits.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t fp_key(uint64_t k) { return mix64(k ^ 0x6A09E667F3BCC909ull); }

}  // namespace cc
