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

constexpr int kHash = 2048;         // LDS slots for the per-block D_i minimum
constexpr int kPairsPerThread = 4;  // pairs per thread in the pair pass

// Exclusive block-wide prefix sum of one int per thread; *total gets the sum.
__device__ __forceinline__ int block_excl_scan(int v, int* sm, int* total) {
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  int incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) sm[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      int t = sm[w];
      sm[w] = run;
      run += t;
    }
    sm[kThreads / 64] = run;
  }
  __syncthreads();
  int res = sm[wv] + incl - v;
  *total = sm[kThreads / 64];
  __syncthreads();
  return res;
}

// Push the block's per-vertex minima to the global D_i and clear the table.
__device__ __forceinline__ void flush_min_table(int32_t* hkey, unsigned long long* hval,
                                                unsigned long long* Di) {
  __syncthreads();
  for (int t = threadIdx.x; t < kHash; t += kThreads) {
    int32_t vv = hkey[t];
    if (vv >= 0) {
      unsigned long long b = hval[t];
      if (b < Di[vv]) atomicMin(&Di[vv], b);
      hkey[t] = -1;
      hval[t] = ~0ull;
    }
  }
  __syncthreads();
}

// Distances at x^(l) for every p in P; P' = {d^2 < D^2} (Sec. 3.1 filter),
// A = {d^2 < delta^2} (Sec. 4.1 activation), D_i = min over P' of d (Sec. 5).
// Each block handles kThreads*kPairsPerThread consecutive pairs. The minimum is
// first taken in an LDS hash table keyed by vertex (flushed after every 256 pairs,
// so it is never more than half full), then one global atomic per distinct vertex
// (min is exact and order independent on the bit patterns of non-negative
// doubles). P' and A are compacted with one counter atomic per block.
__global__ void __launch_bounds__(kThreads) k_pair_pass(PairPassArgs a) {
  __shared__ int32_t hkey[kHash];
  __shared__ unsigned long long hval[kHash];
  __shared__ int ssc[kThreads / 64 + 1];
  __shared__ unsigned long long sbase[2];
  for (int t = threadIdx.x; t < kHash; t += kThreads) {
    hkey[t] = -1;
    hval[t] = ~0ull;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * (kThreads * kPairsPerThread);
  uint64_t keys[kPairsPerThread];
  double d2s[kPairsPerThread];
  int4 vs[kPairsPerThread];
  unsigned keepm = 0, actm = 0;
  unsigned long long f1 = 0, f2 = 0;
#pragma unroll
  for (int k = 0; k < kPairsPerThread; ++k) {
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    keys[k] = 0;
    d2s[k] = 0.0;
    vs[k] = make_int4(0, 0, 0, 0);
    if (i < a.nP) {
      uint64_t key = a.P[i];
      int32_t v[4];
      pair_verts(a.T, key, v);
      double d2 = pair_d2(key_is_ee(key), ld3(a.x, v[0]), ld3(a.x, v[1]), ld3(a.x, v[2]),
                          ld3(a.x, v[3]));
      keys[k] = key;
      d2s[k] = d2;
      vs[k] = make_int4(v[0], v[1], v[2], v[3]);
      if (d2 < a.D2) {
        keepm |= 1u << k;
        if (a.trace) f1 += fp_key(key);
        if (d2 < a.dl2) {
          actm |= 1u << k;
          if (a.trace) f2 += fp_key(key);
        }
        unsigned long long bits = (unsigned long long)__double_as_longlong(sqrt(d2));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t h = ((uint32_t)v[q] * 2654435761u) >> 21;  // 11 bits
          for (;;) {
            int32_t prev = atomicCAS(&hkey[h], -1, v[q]);
            if (prev == -1 || prev == v[q]) {
              atomicMin(&hval[h], bits);
              break;
            }
            h = (h + 1) & (kHash - 1);
          }
        }
      }
    }
    flush_min_table(hkey, hval, a.Di);
  }
  // block-level compaction of P' and A
  int nk = __popc(keepm), na = __popc(actm), tk = 0, ta = 0;
  int ok = block_excl_scan(nk, ssc, &tk);
  int oa = block_excl_scan(na, ssc, &ta);
  if (threadIdx.x == 0) {
    sbase[0] = tk ? atomicAdd(&a.c->n_out, (unsigned long long)tk) : 0ull;
    sbase[1] = ta ? atomicAdd(&a.c->n_act, (unsigned long long)ta) : 0ull;
  }
  __syncthreads();
  unsigned long long pk = sbase[0] + (unsigned long long)ok;
  unsigned long long pa = sbase[1] + (unsigned long long)oa;
#pragma unroll
  for (int k = 0; k < kPairsPerThread; ++k) {
    if (keepm & (1u << k)) {
      a.Pout[pk] = keys[k];
      a.dPout[pk] = d2s[k];
      ++pk;
    }
    if (actm & (1u << k)) {
      if ((int64_t)pa < a.capA) {
        a.Akeys[pa] = keys[k];
        a.Averts[pa] = vs[k];
      }
      ++pa;
    }
  }
  if (a.trace) {
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
  if (s->nP > 0) k_pair_pass<<<nblk(s->nP, kThreads * kPairsPerThread), kThreads, 0, st>>>(a);
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

constexpr int kRoundsPerSync = 8;  // colouring rounds launched between host reads
constexpr int kTailRows = 4096;     // below this many rows one block finishes the rounds
constexpr int kTailThreads = 1024;

struct JpArgs {
  RowSrc src;
  const double* w;
  uint64_t seed;
  unsigned long long* masks;
  int maxc;
  int32_t* colors;
  Counters* c;
};

__device__ __forceinline__ bool is_free(const double* w, int32_t v) { return v >= 0 && w[v] > 0.0; }

template <bool kAtomicLoads>
__device__ __forceinline__ unsigned long long ld_u64(const unsigned long long* p) {
  if (kAtomicLoads) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}

// Round part 1: an uncoloured row offers its priority to its free vertices.
// (The pre-check only skips atomics that cannot raise the value: in a fresh
// kernel the buffer only grows; inside the single-block tail it is read with
// atomic loads so that no stale cache line can hide a lower value.)
template <bool kAtomicLoads>
__device__ __forceinline__ void jp_offer(const JpArgs& a, int32_t r, unsigned long long* vcur) {
  uint64_t key;
  int32_t v[4];
  a.src.get(r, key, v);
  unsigned long long pr = (unsigned long long)mix64(key ^ a.seed);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k]) && pr > ld_u64<kAtomicLoads>(&vcur[v[k]])) atomicMax(&vcur[v[k]], pr);
}

// Round part 2: a row holding the maximum at all its free vertices takes the
// smallest colour not used at those vertices (Jones-Plassmann); it returns true
// when the row stays uncoloured. The other priority buffer is cleared at the
// row's vertices for the next round.
template <bool kAtomicLoads>
__device__ __forceinline__ bool jp_pick(const JpArgs& a, int32_t r,
                                        const unsigned long long* vcur,
                                        unsigned long long* vnext) {
  uint64_t key;
  int32_t v[4];
  a.src.get(r, key, v);
  unsigned long long pr = (unsigned long long)mix64(key ^ a.seed);
  bool win = true;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k])) {
      if (ld_u64<kAtomicLoads>(&vcur[v[k]]) != pr) win = false;
      vnext[v[k]] = 0ull;
    }
  if (!win) return true;
  int col = -1;
  const int W = (a.maxc + 63) / 64;
  for (int wd = 0; wd < W && col < 0; ++wd) {
    unsigned long long used = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (is_free(a.w, v[k])) used |= ld_u64<kAtomicLoads>(&a.masks[(int64_t)v[k] * kMaskWords + wd]);
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
  return false;
}

// One round over a list whose length lives on the device (rounds are launched
// ahead of the host knowing how many rows are left).
__global__ void __launch_bounds__(kThreads) k_jp_max(JpArgs a, const int32_t* list,
                                                     const unsigned long long* nlist,
                                                     unsigned long long* vcur) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)*nlist) return;
  jp_offer<false>(a, list[t], vcur);
}

__global__ void __launch_bounds__(kThreads) k_jp_pick(JpArgs a, const int32_t* list,
                                                      const unsigned long long* nlist,
                                                      const unsigned long long* vcur,
                                                      unsigned long long* vnext,
                                                      int32_t* list_out,
                                                      unsigned long long* nout) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = t < (int64_t)*nlist;
  int32_t r = valid ? list[t] : 0;
  bool lose = valid && jp_pick<false>(a, r, vcur, vnext);
  unsigned long long pos = wave_append(lose, nout);
  if (lose) list_out[pos] = r;
}

// The remaining rounds in one block: global atomics for the priorities and
// masks, atomic loads to read them back, block barriers between the phases.
__global__ void __launch_bounds__(kTailThreads) k_jp_tail(JpArgs a, int32_t* la, int32_t* lb,
                                                          const unsigned long long* nlist,
                                                          unsigned long long* v0,
                                                          unsigned long long* v1, int parity) {
  __shared__ int32_t ncur, nnext;
  if (threadIdx.x == 0) {
    ncur = (int32_t)*nlist;
    nnext = 0;
  }
  __syncthreads();
  int32_t* cur = la;
  int32_t* nxt = lb;
  int round = parity;
  while (ncur > 0) {
    unsigned long long* vcur = (round & 1) ? v1 : v0;
    unsigned long long* vnext = (round & 1) ? v0 : v1;
    for (int32_t t = threadIdx.x; t < ncur; t += kTailThreads) jp_offer<true>(a, cur[t], vcur);
    __syncthreads();
    for (int32_t t = threadIdx.x; t < ncur; t += kTailThreads) {
      int32_t r = cur[t];
      if (jp_pick<true>(a, r, vcur, vnext)) nxt[atomicAdd(&nnext, 1)] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      ncur = nnext;
      nnext = 0;
    }
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
    ++round;
    __syncthreads();
  }
}

__global__ void k_iota(int32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// Colour buckets: per-block histograms in LDS, one global atomic per block and colour.
__global__ void __launch_bounds__(kThreads) k_bucket_count(const int32_t* __restrict__ list,
                                                           int64_t n,
                                                           const int32_t* __restrict__ colors,
                                                           int32_t ncol, int32_t* __restrict__ cnt) {
  __shared__ int32_t h[kMaxColors];
  for (int c = threadIdx.x; c < ncol; c += kThreads) h[c] = 0;
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&h[colors[list ? list[i] : i]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += kThreads)
    if (h[c]) atomicAdd(&cnt[c], h[c]);
}

__global__ void __launch_bounds__(kThreads) k_bucket_scatter(const int32_t* __restrict__ list,
                                                             int64_t n,
                                                             const int32_t* __restrict__ colors,
                                                             int32_t ncol,
                                                             int32_t* __restrict__ cursor,
                                                             int32_t* __restrict__ order) {
  __shared__ int32_t h[kMaxColors];
  for (int c = threadIdx.x; c < ncol; c += kThreads) h[c] = 0;
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t r = 0, c = 0, rank = 0;
  if (i < n) {
    r = list ? list[i] : (int32_t)i;
    c = colors[r];
    rank = atomicAdd(&h[c], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < ncol; k += kThreads)
    if (h[k]) h[k] = atomicAdd(&cursor[k], h[k]);
  __syncthreads();
  if (i < n) order[h[c] + rank] = r;
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
  CC_HIP(hipMemsetAsync(s->rcnt, 0, sizeof(unsigned long long) * (kMaxRounds + 1), st));
  CC_TRY(launch_fill_u64(s->rcnt, 1, (unsigned long long)nrows, st));
  JpArgs a;
  a.src = RowSrc{s->Akeys, s->Averts, s->edges, edges ? 1 : 0};
  a.w = s->w;
  a.seed = s->p.seed;
  a.masks = s->masks;
  a.maxc = s->p.max_colors;
  a.colors = colors;
  a.c = s->dc;
  int64_t known = nrows;  // upper bound of the current list length
  int round = 0;
  for (;;) {
    if (known <= kTailRows) {
      k_jp_tail<<<1, kTailThreads, 0, st>>>(a, cur, nxt, s->rcnt + round, s->vmax0, s->vmax1,
                                            round & 1);
      break;
    }
    if (round + kRoundsPerSync > kMaxRounds) return CC_ECOLOR;
    for (int b = 0; b < kRoundsPerSync; ++b) {
      unsigned long long* vcur = (round & 1) ? s->vmax1 : s->vmax0;
      unsigned long long* vnext = (round & 1) ? s->vmax0 : s->vmax1;
      k_jp_max<<<nblk(known), kThreads, 0, st>>>(a, cur, s->rcnt + round, vcur);
      k_jp_pick<<<nblk(known), kThreads, 0, st>>>(a, cur, s->rcnt + round, vcur, vnext, nxt,
                                                  s->rcnt + round + 1);
      int32_t* t = cur;
      cur = nxt;
      nxt = t;
      ++round;
    }
    CC_HIP(hipGetLastError());
    CC_HIP(hipMemcpyAsync(&s->hc->n_left, s->rcnt + round, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    known = (int64_t)s->hc->n_left;
    if (known == 0) break;
  }
  CC_HIP(hipGetLastError());
  CC_HIP(hipMemcpyAsync(s->hc, s->dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (s->hc->err & 1ull) return CC_ECOLOR;
  const int32_t ncol = (int32_t)s->hc->ncol;
  CC_HIP(hipMemsetAsync(s->col_cnt, 0, sizeof(int32_t) * (ncol + 1), st));
  k_bucket_count<<<nblk(nrows), kThreads, 0, st>>>(base_list, nrows, colors, ncol, s->col_cnt);
  std::vector<int32_t> cnt(ncol);
  CC_HIP(hipMemcpyAsync(cnt.data(), s->col_cnt, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  off.assign(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) off[c + 1] = off[c] + cnt[c];
  CC_HIP(hipMemcpyAsync(s->col_cnt, off.data(), sizeof(int32_t) * ncol, hipMemcpyHostToDevice, st));
  k_bucket_scatter<<<nblk(nrows), kThreads, 0, st>>>(base_list, nrows, colors, ncol, s->col_cnt,
                                                    order);
  CC_HIP(hipMemcpyAsync(edges ? s->ecoff_dev : s->coff_dev, off.data(), sizeof(int32_t) * (ncol + 1),
                        hipMemcpyHostToDevice, st));
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

constexpr int kGsTailRows = 2048;   // colours smaller than this run in one block
constexpr int kGsTailThreads = 1024;

// One projected Gauss-Seidel update of a contact row (Sec. 4.3): the row is
// linearised at x^(l) (Sec. 4), residual w = c0 + sum J.(y - x),
// lambda <- max(0, lambda - w/A), y_v += w_v dl J_v at its free vertices.
__device__ __forceinline__ void gs_contact_update(const GsArgs& a, int32_t r) {
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

// Edge-length row (Sec. 4.2), same projected update.
__device__ __forceinline__ void gs_edge_update(const GsArgs& a, int32_t e) {
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

// One colour, one row per thread (rows of a colour share no free vertex).
__global__ void __launch_bounds__(kThreads) k_gs_contact(GsArgs a) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < a.cnt) gs_contact_update(a, a.order[t]);
}

__global__ void __launch_bounds__(kThreads) k_gs_edge(GsArgs a) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < a.cnt) gs_edge_update(a, a.order[t]);
}

// A run of small colours [c0, c1) in one block, colour after colour with a block
// barrier between them; `off` holds the colour bucket offsets on the device.
__global__ void __launch_bounds__(kGsTailThreads) k_gs_tail(GsArgs a, const int32_t* off,
                                                            int32_t c0, int32_t c1, int is_edge) {
  for (int32_t c = c0; c < c1; ++c) {
    const int32_t b = off[c], e = off[c + 1];
    for (int32_t t = b + threadIdx.x; t < e; t += kGsTailThreads) {
      if (is_edge) gs_edge_update(a, a.order[t]);
      else gs_contact_update(a, a.order[t]);
    }
    __syncthreads();
  }
}

static void gs_colours(const GsArgs& base, const int32_t* order, const std::vector<int32_t>& off,
                       const int32_t* off_dev, int32_t ncol, bool edge, hipStream_t st) {
  GsArgs a = base;
  int32_t c = 0;
  while (c < ncol) {
    int32_t cnt = off[c + 1] - off[c];
    if (cnt >= kGsTailRows) {
      a.order = order + off[c];
      a.cnt = cnt;
      if (edge) k_gs_edge<<<nblk(cnt), kThreads, 0, st>>>(a);
      else k_gs_contact<<<nblk(cnt), kThreads, 0, st>>>(a);
      ++c;
      continue;
    }
    int32_t c1 = c;
    while (c1 < ncol && off[c1 + 1] - off[c1] < kGsTailRows) ++c1;
    a.order = order;
    a.cnt = 0;
    k_gs_tail<<<1, kGsTailThreads, 0, st>>>(a, off_dev, c, c1, edge ? 1 : 0);
    c = c1;
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
    gs_colours(a, s->Aorder, s->col_off, s->coff_dev, s->n_colors, false, st);
    a.lam = s->lamE;
    gs_colours(a, s->eorder, s->ecol_off, s->ecoff_dev, s->n_ecolors, true, st);
  }
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- forward step

// Eq. eq:forward2: alpha_i = min(0.5 gamma D_i / |y_i - x_i|, 1) (1 when y_i = x_i),
// x_i <- y_i if alpha_i = 1 else x_i + alpha_i (y_i - x_i), r_i <- r_i (1 - alpha_i);
// max ||x_i^(l+1) - x_i^(l)|| and ||r||_inf for Alg. 1.
__global__ void __launch_bounds__(kThreads) k_forward(double* __restrict__ x,
                                                      double* __restrict__ xold,
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
    st3(xold, i, xi);
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
    k_forward<<<nblk(s->n), kThreads, 0, st>>>(s->x, s->xold, s->y, s->Di, s->r, s->move2, s->n, hg,
                                                s->dc);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- certificate

// Lemma of Sec. 5: the linear piece x^(l) -> x^(l+1) stays free for pair p when
// no vertex of p moved half its distance, i.e. 4 max_v |dx_v|^2 < d_p^2. A pair the
// bound does not certify gets the continuous test of the piece (ccd_hit).
__global__ void __launch_bounds__(kThreads) k_cert(const uint64_t* __restrict__ P,
                                                   const double* __restrict__ dP, int64_t nP,
                                                   Topo T, const double* __restrict__ move2,
                                                   const double* __restrict__ xold,
                                                   const double* __restrict__ x, double eta2,
                                                   Counters* c) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false, hit = false;
  if (i < nP) {
    int32_t v[4];
    uint64_t key = P[i];
    pair_verts(T, key, v);
    double mv = move2[v[0]];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      double m = move2[v[k]];
      if (m > mv) mv = m;
    }
    bad = !(4.0 * mv < dP[i]);
    if (bad) {
      V3 q[4], dq[4];
      for (int k = 0; k < 4; ++k) {
        q[k] = ld3(xold, v[k]);
        dq[k] = vsub(ld3(x, v[k]), q[k]);
      }
      hit = ccd_hit(q, dq, key_is_ee(key), eta2);
    }
  }
  uint64_t m = __ballot(bad);
  if (m && __lane_id() == __ffsll((long long)m) - 1)
    atomicAdd(&c->fail, (unsigned long long)__popcll(m));
  uint64_t h = __ballot(hit);
  if (h && __lane_id() == __ffsll((long long)h) - 1)
    atomicAdd(&c->hits, (unsigned long long)__popcll(h));
}

int launch_cert(cc_solver* s, hipStream_t st) {
  const double eta = kCcdEta;
  if (s->nP > 0)
    k_cert<<<nblk(s->nP), kThreads, 0, st>>>(s->P, s->dP, s->nP, Topo{s->tris, s->edges},
                                              s->move2, s->xold, s->x, eta * eta, s->dc);
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
