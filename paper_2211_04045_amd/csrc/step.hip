// Per-iteration kernels of the two-way step (Alg. 1): setup, pair pass,
// constraint colouring, projected Gauss-Seidel colour passes, forward step and
// the path certificate.
//
// Everything that decides a set or a position is FP64 and order independent:
// minima and maxima are taken on the bit patterns of non-negative doubles
// (exact, any order), rows of one colour touch disjoint free vertices (no
// atomics, no summation order), colours depend only on the row set.
#include "geom.hpp"
#include "internal.hpp"

namespace cc {

constexpr int kThreads = 256;

static inline unsigned nblk(int64_t n, int t = kThreads) {
  return (unsigned)((n + t - 1) / t);
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// Wave-aggregated append: returns this lane's slot (valid if pred).
__device__ __forceinline__ unsigned long long wave_append(bool pred, unsigned long long* counter) {
  uint64_t m = __ballot(pred);
  unsigned long long base = 0;
  const int lane = __lane_id();
  const int leader = m ? __ffsll((long long)m) - 1 : 0;
  if (m && lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  return base + (unsigned long long)__popcll(m & lanes_below());
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned long long u = __shfl_xor(v, o);
    v = u > v ? u : v;
  }
  return v;
}

// ------------------------------------------------------------- validation

__global__ void k_validate(const int32_t* __restrict__ tris, int32_t nt,
                           const int32_t* __restrict__ edges, int32_t ne, int32_t n,
                           const double* __restrict__ xa, const double* __restrict__ xb,
                           Counters* c) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long err = 0;
  if (g < nt) {
    int32_t i = tris[3 * g], j = tris[3 * g + 1], k = tris[3 * g + 2];
    if (i < 0 || j < 0 || k < 0 || i >= n || j >= n || k >= n || i == j || j == k || i == k)
      err |= 4ull;
  } else if (g < (int64_t)nt + ne) {
    int64_t e = g - nt;
    int32_t i = edges[2 * e], j = edges[2 * e + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) err |= 4ull;
  } else if (g < (int64_t)nt + ne + n) {
    int64_t v = g - nt - ne;
    if (xa)
      for (int k = 0; k < 3; ++k)
        if (!isfinite(xa[3 * v + k])) err |= 8ull;
    if (xb)
      for (int k = 0; k < 3; ++k)
        if (!isfinite(xb[3 * v + k])) err |= 8ull;
  }
  if (err) atomicOr(&c->err, err);
}

int launch_validate(cc_solver* s, const double* xa, const double* xb, hipStream_t st) {
  int64_t m = (int64_t)s->nt + s->ne + s->n;
  CC_HIP(hipMemsetAsync(&s->dc->err, 0, sizeof(unsigned long long), st));
  if (m > 0)
    k_validate<<<nblk(m), kThreads, 0, st>>>(s->tris, s->nt, s->edges, s->ne, s->n, xa, xb, s->dc);
  CC_HIP(hipGetLastError());
  CC_HIP(hipMemcpyAsync(&s->hc->err, &s->dc->err, sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (s->hc->err & 12ull) return CC_EINVAL;
  return CC_OK;
}

// ------------------------------------------------------------- setup (Alg. 1 init)

__global__ void k_setup(const double* __restrict__ xp, const double* __restrict__ xt_in,
                        const double* __restrict__ w, int32_t n, double* __restrict__ x,
                        double* __restrict__ y, double* __restrict__ xt, double* __restrict__ r,
                        uint8_t* __restrict__ stat) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V3 a = ld3(xp, i), b = ld3(xt_in, i);
  st3(x, i, a);
  st3(y, i, b);
  st3(xt, i, b);
  r[i] = 1.0;
  stat[i] = (w[i] == 0.0 && a.x == b.x && a.y == b.y && a.z == b.z) ? 1 : 0;
}

// Edge-length rows (Sec. 4.2): c = sigma - |x_i - x_j| / |y^_i - y^_j| linearised at
// y^ = y^[k+1]: c_lin(y) = sigma - g.(y_i - y_j), g = (y^_i - y^_j)/L^2,
// A = (w_i + w_j)|g|^2. Edges without a free end or with L = 0 carry no row.
__global__ void k_edge_rows(const int32_t* __restrict__ edges, int32_t ne,
                            const double* __restrict__ w, const double* __restrict__ xt,
                            double* __restrict__ eg, double* __restrict__ einv,
                            int32_t* __restrict__ list, Counters* c) {
  int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = false;
  if (e < ne) {
    int32_t i = edges[2 * e], j = edges[2 * e + 1];
    double inv = 0.0;
    if (w[i] > 0.0 || w[j] > 0.0) {
      V3 d = vsub(ld3(xt, i), ld3(xt, j));
      double l2 = vdot(d, d);
      if (l2 > 0.0) {
        V3 g = V3{d.x / l2, d.y / l2, d.z / l2};
        double A = (w[i] + w[j]) * vdot(g, g);
        inv = 1.0 / A;
        st3(eg, e, g);
        valid = true;
      }
    }
    einv[e] = inv;
  }
  unsigned long long pos = wave_append(valid, &c->n_rows);
  if (valid) list[pos] = e;
}

int launch_setup(cc_solver* s, const double* x_prev, const double* x_tilde, hipStream_t st) {
  if (s->n > 0)
    k_setup<<<nblk(s->n), kThreads, 0, st>>>(x_prev, x_tilde, s->w, s->n, s->x, s->y, s->xt,
                                              s->r, s->stat);
  CC_HIP(hipMemsetAsync(&s->dc->n_rows, 0, sizeof(unsigned long long), st));
  if (s->ne > 0 && (s->p.flags & CC_EDGE_LEN))
    k_edge_rows<<<nblk(s->ne), kThreads, 0, st>>>(s->edges, s->ne, s->w, s->xt, s->eg, s->einv,
                                                   s->elist0, s->dc);
  CC_HIP(hipGetLastError());
  CC_HIP(hipMemcpyAsync(&s->hc->n_rows, &s->dc->n_rows, sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  s->n_erows = (int32_t)s->hc->n_rows;
  return CC_OK;
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

int launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st) {
  if (n > 0) k_fill_u64<<<nblk(n), kThreads, 0, st>>>(p, n, v);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- pair pass

struct PairPassArgs {
  const uint64_t* P;
  int64_t nP;
  const double* x;
  Topo T;
  double D2, dl2;
  uint64_t* Pout;
  double* dPout;
  uint64_t* Akeys;
  int4* Averts;
  int64_t capA;
  unsigned long long* Di;
  Counters* c;
  int trace;
};

// Distances at x^(l) for every p in P; P' = {d^2 < D^2} (Sec. 3.1 filter),
// A = {d^2 < delta^2} (Sec. 4.1 activation), D_i = min over P' of d (Sec. 5).
__global__ void __launch_bounds__(kThreads) k_pair_pass(PairPassArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = i < a.nP;
  uint64_t key = valid ? a.P[i] : 0ull;
  int32_t v[4] = {0, 0, 0, 0};
  double d2 = __builtin_inf();
  if (valid) {
    pair_verts(a.T, key, v);
    d2 = pair_d2(key_is_ee(key), ld3(a.x, v[0]), ld3(a.x, v[1]), ld3(a.x, v[2]), ld3(a.x, v[3]));
  }
  bool keep = valid && d2 < a.D2;
  bool act = keep && d2 < a.dl2;
  unsigned long long pk = wave_append(keep, &a.c->n_out);
  if (keep) {
    a.Pout[pk] = key;
    a.dPout[pk] = d2;
    unsigned long long bits = (unsigned long long)__double_as_longlong(sqrt(d2));
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (bits < a.Di[v[k]]) atomicMin(&a.Di[v[k]], bits);
  }
  unsigned long long pa = wave_append(act, &a.c->n_act);
  if (act && (int64_t)pa < a.capA) {
    a.Akeys[pa] = key;
    a.Averts[pa] = make_int4(v[0], v[1], v[2], v[3]);
  }
  if (a.trace) {
    unsigned long long f1 = keep ? fp_key(key) : 0ull, f2 = act ? fp_key(key) : 0ull;
    f1 = wave_sum_u64(f1);
    f2 = wave_sum_u64(f2);
    if (__lane_id() == 0) {
      if (f1) atomicAdd(&a.c->fp_pf, f1);
      if (f2) atomicAdd(&a.c->fp_a, f2);
    }
  }
}

int launch_pair_pass(cc_solver* s, double D2, double dl2, bool trace, hipStream_t st) {
  PairPassArgs a;
  a.P = s->P;
  a.nP = s->nP;
  a.x = s->x;
  a.T = Topo{s->tris, s->edges};
  a.D2 = D2;
  a.dl2 = dl2;
  a.Pout = s->P2;
  a.dPout = s->dP2;
  a.Akeys = s->Akeys;
  a.Averts = s->Averts;
  a.capA = s->capA;
  a.Di = s->Di;
  a.c = s->dc;
  a.trace = trace ? 1 : 0;
  if (s->nP > 0) k_pair_pass<<<nblk(s->nP), kThreads, 0, st>>>(a);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- colouring

// A row source: contact rows (key = pair key, 4 vertices) or edge-length rows
// (key = edge index, 2 vertices).
struct RowSrc {
  const uint64_t* keys;
  const int4* verts;
  const int32_t* edges;
  int is_edge;
  __device__ __forceinline__ void get(int32_t r, uint64_t& key, int32_t v[4]) const {
    if (is_edge) {
      key = (uint64_t)(uint32_t)r;
      v[0] = edges[2 * r];
      v[1] = edges[2 * r + 1];
      v[2] = -1;
      v[3] = -1;
    } else {
      key = keys[r];
      int4 q = verts[r];
      v[0] = q.x;
      v[1] = q.y;
      v[2] = q.z;
      v[3] = q.w;
    }
  }
};

struct JpArgs {
  RowSrc src;
  const int32_t* list;
  int64_t nlist;
  const double* w;
  uint64_t seed;
  unsigned long long* vcur;
  unsigned long long* vnext;
  unsigned long long* masks;
  int maxc;
  int32_t* colors;
  int32_t* list_out;
  Counters* c;
};

__device__ __forceinline__ bool is_free(const double* w, int32_t v) { return v >= 0 && w[v] > 0.0; }

// Round part 1: every uncoloured row offers its priority to its free vertices.
__global__ void __launch_bounds__(kThreads) k_jp_max(JpArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.nlist) return;
  int32_t r = a.list[t];
  uint64_t key;
  int32_t v[4];
  a.src.get(r, key, v);
  unsigned long long pr = (unsigned long long)mix64(key ^ a.seed);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k]) && pr > a.vcur[v[k]]) atomicMax(&a.vcur[v[k]], pr);
}

// Round part 2: a row holding the maximum at all its free vertices takes the
// smallest colour not used at those vertices (Jones-Plassmann); the others go to
// the next round's list. The other priority buffer is cleared for the next round.
__global__ void __launch_bounds__(kThreads) k_jp_pick(JpArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = t < a.nlist;
  bool lose = false;
  int32_t r = 0;
  if (valid) {
    r = a.list[t];
    uint64_t key;
    int32_t v[4];
    a.src.get(r, key, v);
    unsigned long long pr = (unsigned long long)mix64(key ^ a.seed);
    bool win = true;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (is_free(a.w, v[k])) {
        if (a.vcur[v[k]] != pr) win = false;
        a.vnext[v[k]] = 0ull;
      }
    if (win) {
      int col = -1;
      const int W = (a.maxc + 63) / 64;
      for (int wd = 0; wd < W && col < 0; ++wd) {
        unsigned long long used = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (is_free(a.w, v[k])) used |= a.masks[(int64_t)v[k] * kMaskWords + wd];
        if (~used) col = 64 * wd + (__ffsll((long long)~used) - 1);
      }
      if (col < 0 || col >= a.maxc) {
        atomicOr(&a.c->err, 1ull);
        col = 0;
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (is_free(a.w, v[k]))
            atomicOr(&a.masks[(int64_t)v[k] * kMaskWords + col / 64], 1ull << (col % 64));
      }
      a.colors[r] = col;
      atomicMax(&a.c->ncol, (unsigned long long)(col + 1));
    } else {
      lose = true;
    }
  }
  unsigned long long pos = wave_append(lose, &a.c->n_left);
  if (lose) a.list_out[pos] = r;
}

__global__ void k_iota(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

__global__ void k_col_hist(const int32_t* __restrict__ list, int64_t n,
                           const int32_t* __restrict__ colors, int32_t* __restrict__ cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[colors[list ? list[i] : i]], 1);
}

__global__ void k_col_scatter(const int32_t* __restrict__ list, int64_t n,
                              const int32_t* __restrict__ colors, int32_t* __restrict__ cursor,
                              int32_t* __restrict__ order) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t r = list ? list[i] : (int32_t)i;
  int32_t pos = atomicAdd(&cursor[colors[r]], 1);
  order[pos] = r;
}

// Colour the contact rows (A) or the edge-length rows and bucket them by colour.
int color_rows(cc_solver* s, bool edges, hipStream_t st) {
  const int64_t nrows = edges ? s->n_erows : s->nA;
  int32_t* colors = edges ? s->ecol : s->Acol;
  int32_t* order = edges ? s->eorder : s->Aorder;
  std::vector<int32_t>& off = edges ? s->ecol_off : s->col_off;
  off.assign(1, 0);
  if (edges) s->n_ecolors = 0; else s->n_colors = 0;
  if (nrows == 0) return CC_OK;
  // contacts: rows 0..nA-1 (identity base list); edges: the valid-edge list of the
  // step, kept intact in elist0 while elist1/elist2 carry the rounds
  int32_t *cur, *nxt, *base_list;
  if (edges) {
    CC_HIP(hipMemcpyAsync(s->elist1, s->elist0, sizeof(int32_t) * nrows, hipMemcpyDeviceToDevice, st));
    base_list = s->elist0;
    cur = s->elist1;
    nxt = s->elist2;
  } else {
    k_iota<<<nblk(nrows), kThreads, 0, st>>>(s->list0, nrows);
    base_list = nullptr;
    cur = s->list0;
    nxt = s->list1;
  }
  CC_HIP(hipMemsetAsync(s->vmax0, 0, sizeof(unsigned long long) * s->n, st));
  CC_HIP(hipMemsetAsync(s->vmax1, 0, sizeof(unsigned long long) * s->n, st));
  CC_HIP(hipMemsetAsync(s->masks, 0, sizeof(unsigned long long) * s->n * kMaskWords, st));
  CC_HIP(hipMemsetAsync(&s->dc->ncol, 0, sizeof(unsigned long long), st));
  CC_HIP(hipMemsetAsync(&s->dc->err, 0, sizeof(unsigned long long), st));
  JpArgs a;
  a.src = RowSrc{s->Akeys, s->Averts, s->edges, edges ? 1 : 0};
  a.w = s->w;
  a.seed = s->p.seed;
  a.masks = s->masks;
  a.maxc = s->p.max_colors;
  a.colors = colors;
  a.c = s->dc;
  int64_t ncur = nrows;
  int round = 0;
  while (ncur > 0) {
    a.list = cur;
    a.nlist = ncur;
    a.vcur = (round & 1) ? s->vmax1 : s->vmax0;
    a.vnext = (round & 1) ? s->vmax0 : s->vmax1;
    a.list_out = nxt;
    CC_HIP(hipMemsetAsync(&s->dc->n_left, 0, sizeof(unsigned long long), st));
    k_jp_max<<<nblk(ncur), kThreads, 0, st>>>(a);
    k_jp_pick<<<nblk(ncur), kThreads, 0, st>>>(a);
    CC_HIP(hipGetLastError());
    CC_HIP(hipMemcpyAsync(s->hc, s->dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    if (s->hc->err & 1ull) return CC_ECOLOR;
    int64_t left = (int64_t)s->hc->n_left;
    if (left >= ncur) return CC_EHIP;  // no progress is impossible for unique priorities
    ncur = left;
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
    ++round;
  }
  const int32_t ncol = (int32_t)s->hc->ncol;
  CC_HIP(hipMemsetAsync(s->col_cnt, 0, sizeof(int32_t) * (ncol + 1), st));
  k_col_hist<<<nblk(nrows), kThreads, 0, st>>>(base_list, nrows, colors, s->col_cnt);
  std::vector<int32_t> cnt(ncol);
  CC_HIP(hipMemcpyAsync(cnt.data(), s->col_cnt, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  off.assign(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) off[c + 1] = off[c] + cnt[c];
  CC_HIP(hipMemcpyAsync(s->col_cnt, off.data(), sizeof(int32_t) * ncol, hipMemcpyHostToDevice, st));
  k_col_scatter<<<nblk(nrows), kThreads, 0, st>>>(base_list, nrows, colors, s->col_cnt, order);
  CC_HIP(hipGetLastError());
  if (edges) s->n_ecolors = ncol; else s->n_colors = ncol;
  return CC_OK;
}

// ------------------------------------------------------------- Gauss-Seidel

struct GsArgs {
  const int32_t* order;
  int32_t cnt;
  const uint64_t* Akeys;
  const int4* Averts;
  const int32_t* edges;
  const double* eg;
  const double* einv;
  const double* x;
  double* y;
  const double* w;
  double* lam;
  double delta, kappa2, sigma;
};

// One projected Gauss-Seidel update per contact row of this colour (Sec. 4.3):
// residual w = c0 + sum J.(y - x), lambda <- max(0, lambda - w/A), y += w_v dl J_v.
__global__ void __launch_bounds__(kThreads) k_gs_contact(GsArgs a) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.cnt) return;
  int32_t r = a.order[t];
  uint64_t key = a.Akeys[r];
  int4 q = a.Averts[r];
  int32_t v[4] = {q.x, q.y, q.z, q.w};
  V3 xs[4];
  double ws[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    xs[k] = ld3(a.x, v[k]);
    ws[k] = a.w[v[k]];
  }
  Row R;
  contact_row(key_is_ee(key), xs, ws, a.delta, a.kappa2, R);
  if (!(R.inv_a > 0.0)) return;
  double wr = R.c0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    V3 dy = vsub(ld3(a.y, v[k]), xs[k]);
    wr = wr + vdot(R.J[k], dy);
  }
  double lam = a.lam[r];
  double ln = lam - wr * R.inv_a;
  if (ln < 0.0) ln = 0.0;
  double dl = ln - lam;
  a.lam[r] = ln;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!(ws[k] > 0.0)) continue;
    double co = ws[k] * dl;
    V3 yv = ld3(a.y, v[k]);
    yv = V3{yv.x + co * R.J[k].x, yv.y + co * R.J[k].y, yv.z + co * R.J[k].z};
    st3(a.y, v[k], yv);
  }
}

// Edge-length rows of this colour (Sec. 4.2), same projected update.
__global__ void __launch_bounds__(kThreads) k_gs_edge(GsArgs a) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.cnt) return;
  int32_t e = a.order[t];
  int32_t i = a.edges[2 * e], j = a.edges[2 * e + 1];
  V3 g = ld3(a.eg, e);
  V3 yi = ld3(a.y, i), yj = ld3(a.y, j);
  V3 dy = vsub(yi, yj);
  double wr = a.sigma - vdot(g, dy);
  double lam = a.lam[e];
  double ln = lam - wr * a.einv[e];
  if (ln < 0.0) ln = 0.0;
  double dl = ln - lam;
  a.lam[e] = ln;
  double wi = a.w[i], wj = a.w[j];
  if (wi > 0.0) {
    double co = wi * dl;
    st3(a.y, i, V3{yi.x - co * g.x, yi.y - co * g.y, yi.z - co * g.z});
  }
  if (wj > 0.0) {
    double co = wj * dl;
    st3(a.y, j, V3{yj.x + co * g.x, yj.y + co * g.y, yj.z + co * g.z});
  }
}

int launch_gs(cc_solver* s, hipStream_t st) {
  GsArgs a;
  a.Akeys = s->Akeys;
  a.Averts = s->Averts;
  a.edges = s->edges;
  a.eg = s->eg;
  a.einv = s->einv;
  a.x = s->x;
  a.y = s->y;
  a.w = s->w;
  a.delta = s->p.delta;
  a.kappa2 = s->kappa2;
  a.sigma = s->p.sigma;
  if (s->nA > 0) CC_HIP(hipMemsetAsync(s->lamA, 0, sizeof(double) * s->nA, st));
  if (s->n_erows > 0) CC_HIP(hipMemsetAsync(s->lamE, 0, sizeof(double) * s->ne, st));
  for (int sw = 0; sw < s->p.gs_sweeps; ++sw) {
    a.lam = s->lamA;
    for (int c = 0; c < s->n_colors; ++c) {
      a.order = s->Aorder + s->col_off[c];
      a.cnt = s->col_off[c + 1] - s->col_off[c];
      if (a.cnt > 0) k_gs_contact<<<nblk(a.cnt), kThreads, 0, st>>>(a);
    }
    a.lam = s->lamE;
    for (int c = 0; c < s->n_ecolors; ++c) {
      a.order = s->eorder + s->ecol_off[c];
      a.cnt = s->ecol_off[c + 1] - s->ecol_off[c];
      if (a.cnt > 0) k_gs_edge<<<nblk(a.cnt), kThreads, 0, st>>>(a);
    }
  }
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- forward step

// Eq. eq:forward2: alpha_i = min(0.5 gamma D_i / |y_i - x_i|, 1) (1 when y_i = x_i),
// x_i <- y_i if alpha_i = 1 else x_i + alpha_i (y_i - x_i), r_i <- r_i (1 - alpha_i);
// max ||x_i^(l+1) - x_i^(l)|| and ||r||_inf for Alg. 1.
__global__ void __launch_bounds__(kThreads) k_forward(double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const unsigned long long* __restrict__ Di,
                                                      double* __restrict__ r,
                                                      double* __restrict__ move2, int32_t n,
                                                      double hg, Counters* c) {
  __shared__ unsigned long long sm[2][kThreads / 64];
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long mb = 0, rb = 0;
  if (i < n) {
    V3 xi = ld3(x, i), yi = ld3(y, i);
    V3 dx = vsub(yi, xi);
    double n2 = vdot(dx, dx);
    double alpha = 1.0;
    if (n2 > 0.0) {
      double a = (hg * __longlong_as_double((long long)Di[i])) / sqrt(n2);
      if (a < 1.0) alpha = a;
    }
    V3 xn = (alpha == 1.0) ? yi : vaxpy(xi, alpha, dx);
    V3 mv = vsub(xn, xi);
    double m2 = vdot(mv, mv);
    move2[i] = m2;
    st3(x, i, xn);
    double ri = r[i] * (1.0 - alpha);
    r[i] = ri;
    mb = (unsigned long long)__double_as_longlong(sqrt(m2));
    rb = (unsigned long long)__double_as_longlong(ri);
  }
  mb = wave_max_u64(mb);
  rb = wave_max_u64(rb);
  const int wv = threadIdx.x >> 6;
  if (__lane_id() == 0) {
    sm[0][wv] = mb;
    sm[1][wv] = rb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kThreads / 64; ++k) {
      mb = sm[0][k] > mb ? sm[0][k] : mb;
      rb = sm[1][k] > rb ? sm[1][k] : rb;
    }
    mb = sm[0][0] > mb ? sm[0][0] : mb;
    rb = sm[1][0] > rb ? sm[1][0] : rb;
    if (mb) atomicMax(&c->mmax_bits, mb);
    if (rb) atomicMax(&c->rinf_bits, rb);
  }
}

int launch_forward(cc_solver* s, hipStream_t st) {
  const double hg = 0.5 * s->p.gamma;
  if (s->n > 0)
    k_forward<<<nblk(s->n), kThreads, 0, st>>>(s->x, s->y, s->Di, s->r, s->move2, s->n, hg, s->dc);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- certificate

// Lemma of Sec. 5: the linear piece x^(l) -> x^(l+1) stays free for pair p when
// no vertex of p moved half its distance, i.e. 4 max_v |dx_v|^2 < d_p^2.
__global__ void __launch_bounds__(kThreads) k_cert(const uint64_t* __restrict__ P,
                                                   const double* __restrict__ dP, int64_t nP,
                                                   Topo T, const double* __restrict__ move2,
                                                   Counters* c) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (i < nP) {
    int32_t v[4];
    pair_verts(T, P[i], v);
    double mv = move2[v[0]];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      double m = move2[v[k]];
      if (m > mv) mv = m;
    }
    bad = !(4.0 * mv < dP[i]);
  }
  uint64_t m = __ballot(bad);
  if (m && __lane_id() == __ffsll((long long)m) - 1)
    atomicAdd(&c->fail, (unsigned long long)__popcll(m));
}

int launch_cert(cc_solver* s, hipStream_t st) {
  if (s->nP > 0)
    k_cert<<<nblk(s->nP), kThreads, 0, st>>>(s->P, s->dP, s->nP, Topo{s->tris, s->edges},
                                              s->move2, s->dc);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

__global__ void k_fp_col(const uint64_t* __restrict__ keys, const int32_t* __restrict__ col,
                         int64_t n, Counters* c) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long f = i < n ? mix64(fp_key(keys[i]) ^ (uint64_t)col[i]) : 0ull;
  f = wave_sum_u64(f);
  if (__lane_id() == 0 && f) atomicAdd(&c->fp_col, f);
}

int launch_fp_col(cc_solver* s, hipStream_t st) {
  if (s->nA > 0) k_fp_col<<<nblk(s->nA), kThreads, 0, st>>>(s->Akeys, s->Acol, s->nA, s->dc);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

}  // namespace cc
