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

// The block-wide form of wave_append, for kernels whose every thread reaches it:
// one global atomic per block. A device-wide atomic on one address is serialised
// over the whole GPU (about 12 ns each on MI355X), so one per wave over a grid of
// a few thousand waves costs tens of microseconds. *total gets the block's count.
__device__ __forceinline__ unsigned long long block_append(bool pred,
                                                           unsigned long long* counter,
                                                           int* total) {
  __shared__ int s_cnt[kThreads / 64];
  __shared__ unsigned long long s_base;
  const uint64_t m = __ballot(pred);
  const int wv = threadIdx.x >> 6;
  if (__lane_id() == 0) s_cnt[wv] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      const int t = s_cnt[w];
      s_cnt[w] = run;
      run += t;
    }
    s_base = run ? atomicAdd(counter, (unsigned long long)run) : 0ull;
    s_cnt[0] = run;  // wave 0's offset is 0: the slot carries the total meanwhile
  }
  __syncthreads();
  const int off = wv == 0 ? 0 : s_cnt[wv];
  *total = s_cnt[0];
  const unsigned long long pos = s_base + (unsigned long long)off +
                                 (unsigned long long)__popcll(m & lanes_below());
  __syncthreads();  // the slots are free again when the function returns
  return pos;
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

// ------------------------------------------------------------- segments

// Scene-local key of a row, so that colouring priorities do not depend on where
// a scene sits in the solver's arrays: vertex-triangle (v << 32 | f) and
// edge-edge (e << 32 | g), vertex-vertex (a << 32 | b) pair keys and edge-row
// keys (e) lose their segment's bases. A scene alone at base 0 keeps its keys.
__device__ __forceinline__ uint64_t local_pair_key(uint64_t key, const SegDev& sg) {
  const uint32_t hi = key_a(key), lo = (uint32_t)key;
  if (key_is_vv(key))
    return KEY_VV | ((uint64_t)(hi - (uint32_t)sg.vb) << 32) | (uint32_t)(lo - (uint32_t)sg.vb);
  if (key_is_ee(key))
    return KEY_EE | ((uint64_t)(hi - (uint32_t)sg.eb) << 32) | (uint32_t)(lo - (uint32_t)sg.eb);
  return ((uint64_t)(hi - (uint32_t)sg.vb) << 32) | (uint32_t)(lo - (uint32_t)sg.fb);
}

// Small LDS table of per-segment counters for one block: slot keys are segment
// ids (-1 = empty), linear probing; a segment that finds no slot adds straight
// to the global record.
constexpr int kSegSlots = 32;

__device__ __forceinline__ int seg_slot(int32_t* skey, int32_t sg) {
  uint32_t h = ((uint32_t)sg * 2654435761u) >> 27;  // 5 bits
  for (int t = 0; t < kSegSlots; ++t) {
    int32_t prev = atomicCAS(&skey[h], -1, sg);
    if (prev == -1 || prev == sg) return (int)h;
    h = (h + 1) & (kSegSlots - 1);
  }
  return -1;
}

// ------------------------------------------------------------- validation

// Topology of segment `sg` in: local vertex ids are checked against the scene's
// vertex count and stored solver-wide (+ vb); edges record their segment.
__global__ void k_topo_in(const int32_t* __restrict__ tin, const int32_t* __restrict__ ein,
                          int32_t nf, int32_t ne, int32_t nv, int32_t vb, int32_t sg,
                          int32_t* __restrict__ tris, int32_t* __restrict__ edges,
                          int32_t* __restrict__ eseg, Counters* c) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long err = 0;
  if (g < nf) {
    int32_t i = tin[3 * g], j = tin[3 * g + 1], k = tin[3 * g + 2];
    if (i < 0 || j < 0 || k < 0 || i >= nv || j >= nv || k >= nv || i == j || j == k || i == k)
      err |= 4ull;
    tris[3 * g] = i + vb;
    tris[3 * g + 1] = j + vb;
    tris[3 * g + 2] = k + vb;
  } else if (g < (int64_t)nf + ne) {
    int64_t e = g - nf;
    int32_t i = ein[2 * e], j = ein[2 * e + 1];
    if (i < 0 || j < 0 || i >= nv || j >= nv || i == j) err |= 4ull;
    edges[2 * e] = i + vb;
    edges[2 * e + 1] = j + vb;
    eseg[e] = sg;
  }
  if (err) atomicOr(&c->err, err);
}

__global__ void k_check_finite(const double* __restrict__ xa, const double* __restrict__ xb,
                               int32_t n, Counters* c) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  unsigned long long err = 0;
  for (int k = 0; k < 3; ++k) {
    if (xa && !isfinite(xa[3 * v + k])) err |= 8ull;
    if (xb && !isfinite(xb[3 * v + k])) err |= 8ull;
  }
  if (err) atomicOr(&c->err, err);
}

static int read_err(cc_solver* s, hipStream_t st) {
  CC_HIP(hipGetLastError());
  CC_HIP(hipMemcpyAsync(&s->hc->err, &s->dc->err, sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  return (s->hc->err & 12ull) ? CC_EINVAL : CC_OK;
}

int launch_topo_in(cc_solver* s, int32_t sg, const int32_t* tris, const int32_t* edges,
                   hipStream_t st) {
  const Seg& g = s->segs[sg];
  const int64_t m = (int64_t)g.nf + g.ne;
  CC_HIP(hipMemsetAsync(&s->dc->err, 0, sizeof(unsigned long long), st));
  if (m > 0)
    k_topo_in<<<nblk(m), kThreads, 0, st>>>(tris, edges, g.nf, g.ne, g.nv, g.vb, sg,
                                             s->tris + 3 * (int64_t)g.fb,
                                             s->edges + 2 * (int64_t)g.eb, s->eseg + g.eb, s->dc);
  return read_err(s, st);
}

int launch_check_finite(cc_solver* s, const double* xa, const double* xb, int32_t n,
                        hipStream_t st) {
  CC_HIP(hipMemsetAsync(&s->dc->err, 0, sizeof(unsigned long long), st));
  if (n > 0) k_check_finite<<<nblk(n), kThreads, 0, st>>>(xa, xb, n, s->dc);
  return read_err(s, st);
}

// Clear the flag of every vertex a triangle or edge of the segment refers to.
__global__ void k_mark_refs(const int32_t* __restrict__ tris, int64_t n3,
                            const int32_t* __restrict__ edges, int64_t n2,
                            uint8_t* __restrict__ flag) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n3) flag[tris[g]] = 0;
  else if (g < n3 + n2) flag[edges[g - n3]] = 0;
}

// Particles of segment sg (vertices in no triangle and no edge: the vertex-vertex
// pair universe), listed in increasing order at plist[vb, vb + np). The static
// flags of the segment's vertices serve as scratch (begin sets them).
int launch_particles(cc_solver* s, int32_t sg, hipStream_t st) {
  Seg& g = s->segs[sg];
  g.np = 0;
  if (g.nv == 0) return CC_OK;
  CC_HIP(hipMemsetAsync(s->stat + g.vb, 1, (size_t)g.nv, st));
  const int64_t m = 3 * (int64_t)g.nf + 2 * (int64_t)g.ne;
  if (m > 0)
    k_mark_refs<<<nblk(m), kThreads, 0, st>>>(s->tris + 3 * (int64_t)g.fb, 3 * (int64_t)g.nf,
                                               s->edges + 2 * (int64_t)g.eb, 2 * (int64_t)g.ne,
                                               s->stat);
  CC_HIP(hipGetLastError());
  std::vector<uint8_t> flag((size_t)g.nv);
  CC_HIP(hipMemcpyAsync(flag.data(), s->stat + g.vb, (size_t)g.nv, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> ids;
  for (int32_t i = 0; i < g.nv; ++i)
    if (flag[(size_t)i]) ids.push_back(g.vb + i);
  g.np = (int32_t)ids.size();
  if (g.np > 0) {
    CC_HIP(hipMemcpyAsync(s->plist + g.vb, ids.data(), sizeof(int32_t) * ids.size(),
                          hipMemcpyHostToDevice, st));
    CC_HIP(hipStreamSynchronize(st));
  }
  return CC_OK;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

int launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n > 0) k_fill_i32<<<nblk(n), kThreads, 0, st>>>(p, n, v);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- setup (Alg. 1 init)

// One segment's vertices (pointers already offset to the segment): x <- x^[k],
// y <- y^[k+1], r <- 1, static flag. x_prev may be the segment's own x.
__global__ void k_setup(const double* xp, const double* __restrict__ xt_in,
                        const double* __restrict__ w, int32_t n, double* x,
                        double* __restrict__ y, double* __restrict__ xt, double* __restrict__ r,
                        uint8_t* __restrict__ stat, float* __restrict__ dy) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  V3 a = ld3(xp, i), b = ld3(xt_in, i);
  st3(x, i, a);
  st3(y, i, b);
  st3(xt, i, b);
  dy[3 * (int64_t)i] = (float)(b.x - a.x);
  dy[3 * (int64_t)i + 1] = (float)(b.y - a.y);
  dy[3 * (int64_t)i + 2] = (float)(b.z - a.z);
  r[i] = 1.0;
  stat[i] = (w[i] == 0.0 && a.x == b.x && a.y == b.y && a.z == b.z) ? 1 : 0;
}

// Edge-length rows (Sec. 4.2) of one segment's edges: c = sigma - |x_i - x_j| /
// |y^_i - y^_j| linearised at y^ = y^[k+1]: c_lin(y) = sigma - g.(y_i - y_j),
// g = (y^_i - y^_j)/L^2, A = (w_i + w_j)|g|^2. Edges without a free end or with
// L = 0 carry no row. Valid rows are appended to `list` (to be coloured).
__global__ void k_edge_rows(const int32_t* __restrict__ edges, int32_t eb, int32_t ne,
                            const double* __restrict__ w, const double* __restrict__ xt,
                            double* __restrict__ eg, double* __restrict__ einv,
                            int32_t* __restrict__ list, Counters* c,
                            unsigned long long* seg_rows) {
  int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = false;
  if (e < ne) {
    const int32_t ge = eb + e;
    int32_t i = edges[2 * ge], j = edges[2 * ge + 1];
    double inv = 0.0;
    if (w[i] > 0.0 || w[j] > 0.0) {
      V3 d = vsub(ld3(xt, i), ld3(xt, j));
      double l2 = vdot(d, d);
      if (l2 > 0.0) {
        V3 g = V3{d.x / l2, d.y / l2, d.z / l2};
        double A = (w[i] + w[j]) * vdot(g, g);
        inv = 1.0 / A;
        st3(eg, ge, g);
        valid = true;
      }
    }
    einv[ge] = inv;
  }
  int nblock = 0;
  const unsigned long long pos = block_append(valid, &c->n_rows, &nblock);
  if (valid) list[pos] = eb + e;
  if (threadIdx.x == 0 && nblock) atomicAdd(seg_rows, (unsigned long long)nblock);
}

// Begin of one segment: state arrays and its edge-length rows (appended to
// elist0 at the counter dc->n_rows, which the caller zeroes once per batch of
// begins; the segment's own row count goes to its record).
int launch_setup(cc_solver* s, int32_t sg, const double* x_prev, const double* x_tilde,
                 hipStream_t st) {
  const Seg& g = s->segs[sg];
  const int64_t vb = g.vb;
  if (g.nv > 0)
    k_setup<<<nblk(g.nv), kThreads, 0, st>>>(x_prev, x_tilde, s->w + vb, g.nv, s->x + 3 * vb,
                                              s->y + 3 * vb, s->xt + 3 * vb, s->r + vb,
                                              s->stat + vb, s->dy + 3 * vb);
  CC_HIP(hipMemsetAsync(&s->seg_dev[sg].n_rows, 0, sizeof(unsigned long long), st));
  if (g.ne > 0 && (s->p.flags & CC_EDGE_LEN))
    k_edge_rows<<<nblk(g.ne), kThreads, 0, st>>>(s->edges, g.eb, g.ne, s->w, s->xt, s->eg,
                                                  s->einv, s->elist0, s->dc,
                                                  &s->seg_dev[sg].n_rows);
  else if (g.ne > 0)
    CC_HIP(hipMemsetAsync(s->einv + g.eb, 0, sizeof(double) * g.ne, st));
  CC_HIP(hipGetLastError());
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

// D_i <- D^(l) of the vertex's segment (Sec. 5: a vertex in no pair moves at
// most 0.45 D^(l)); vertices of segments that do not iterate are left alone.
// The iteration's counters start from zero here as well.
__global__ void k_di_init(const int32_t* __restrict__ vseg, const SegDev* __restrict__ seg,
                          int32_t n, unsigned long long* __restrict__ Di, Counters* c) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int kWords = (int)(sizeof(Counters) / sizeof(unsigned long long));
  if (v < kWords) reinterpret_cast<unsigned long long*>(c)[v] = 0ull;
  if (v >= n) return;
  const int32_t sg = vseg[v];
  if (sg < 0 || !(seg[sg].flags & kSegActive)) return;
  Di[v] = (unsigned long long)__double_as_longlong(seg[sg].D);
}

int launch_di_init(cc_solver* s, hipStream_t st) {
  static_assert(sizeof(Counters) % sizeof(unsigned long long) == 0 &&
                    sizeof(Counters) / sizeof(unsigned long long) <= kThreads,
                "one block clears the counters");
  k_di_init<<<nblk(s->n > 0 ? s->n : 1), kThreads, 0, st>>>(s->vseg, s->seg_dev, s->n, s->Di,
                                                             s->dc);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- pair pass

struct PairPassArgs {
  const uint64_t* P;
  int64_t nP;
  int64_t n_old;  // [0, n_old): last P'; [n_old, nP): appended by this iteration's search
  int64_t d_from;    // pairs i >= d_from read d^2 from dPin instead of computing it
  const double* dPin;
  const uint8_t* mvd;  // moved flags of the last forward step (null: every distance is taken)
  const double* x;
  Topo T;
  const int32_t* vseg;
  SegDev* seg;
  double dl2;
  uint64_t* Pout;
  double* dPout;
  uint64_t* Akeys;
  int4* Averts;
  int64_t capA;
  unsigned long long* Di;
  Counters* c;
  int trace;
  int in_place;  // every pair is kept (fresh from a search of every scene): P' is P, unwritten
  int32_t one_seg;  // >= 0: every pair of P belongs to this (the only) segment, whose
                    // counts the host takes from n_out and n_act (none are kept here)
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

// Add a thread's per-segment counts to the block's LDS table (or straight to
// the segment's record when the table has no slot for it).
__device__ __forceinline__ void seg_count_flush(int32_t* gkey, unsigned long long (*gcnt)[3],
                                                SegDev* seg, int32_t sg,
                                                unsigned long long* cnt) {
  if (sg < 0 || cnt[0] == 0) return;
  const int slot = seg_slot(gkey, sg);
  if (slot >= 0) {
    atomicAdd(&gcnt[slot][0], cnt[0]);
    if (cnt[1]) atomicAdd(&gcnt[slot][1], cnt[1]);
    if (cnt[2]) atomicAdd(&gcnt[slot][2], cnt[2]);
  } else {
    atomicAdd(&seg[sg].n_p, cnt[0]);
    if (cnt[1]) atomicAdd(&seg[sg].n_pf, cnt[1]);
    if (cnt[2]) atomicAdd(&seg[sg].n_a, cnt[2]);
  }
  cnt[0] = cnt[1] = cnt[2] = 0;
}

// The block's minimum of d for vertex v in its LDS table (open addressing over kHash
// slots, the slots taken listed in occ); past kProbe probes it goes straight to the
// global D_i. Minima of the bit patterns of non-negative doubles are exact and
// independent of order, so either path gives the same D_i.
constexpr int kProbe = 32;
__device__ __forceinline__ void min_insert(int32_t* hkey, unsigned long long* hval,
                                           int16_t* occ, int* nocc, unsigned long long* Di,
                                           int32_t v, unsigned long long bits) {
  uint32_t h = ((uint32_t)v * 2654435761u) >> 21;  // 11 bits
#pragma unroll 1
  for (int p = 0; p < kProbe; ++p) {
    const int32_t prev = atomicCAS(&hkey[h], -1, v);
    if (prev == -1 || prev == v) {
      if (prev == -1) occ[atomicAdd(nocc, 1)] = (int16_t)h;
      atomicMin(&hval[h], bits);
      return;
    }
    h = (h + 1) & (kHash - 1);
  }
  atomicMin(&Di[v], bits);
}

// Distances at x^(l) for every p in P; P' = {d^2 < D^2} (Sec. 3.1 filter),
// A = {d^2 < delta^2} (Sec. 4.1 activation), D_i = min over P' of d (Sec. 5).
// D is the pair's segment's; pairs of segments that do not iterate, and pairs of
// last iteration's P' whose segment was searched again, are dropped unevaluated.
// Each block handles kThreads*kPairsPerThread consecutive pairs. The minimum is
// first taken in an LDS hash table keyed by vertex, then one global atomic per
// distinct vertex of the block, at its end, over the list of slots taken (min is
// exact and order independent on the bit patterns of non-negative doubles). P' and
// A are compacted with one counter atomic per block; the per-segment counts go
// through a small LDS table.
// kCompute = false when every pair carries its distance (d_from = 0: a pair pass
// right after a search of every scene): no positions are loaded and no distance is
// taken, and the kernel needs far fewer registers (more waves per SIMD to cover the
// key -> topology chain).
template <bool kCompute>
__global__ void __launch_bounds__(kThreads) k_pair_pass(PairPassArgs a) {
  __shared__ int32_t hkey[kHash];
  __shared__ unsigned long long hval[kHash];
  __shared__ int16_t occ[kHash];
  __shared__ int nocc;
  __shared__ int ssc[kThreads / 64 + 1];
  __shared__ unsigned long long sbase[2];
  __shared__ int32_t gkey[kSegSlots];
  __shared__ unsigned long long gcnt[kSegSlots][3];
  for (int t = threadIdx.x; t < kHash; t += kThreads) {
    hkey[t] = -1;
    hval[t] = ~0ull;
  }
  if (threadIdx.x == 0) nocc = 0;
  if (threadIdx.x < kSegSlots) {
    gkey[threadIdx.x] = -1;
    gcnt[threadIdx.x][0] = gcnt[threadIdx.x][1] = gcnt[threadIdx.x][2] = 0ull;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * (kThreads * kPairsPerThread);
  uint64_t keys[kPairsPerThread];
  double d2s[kPairsPerThread];
  int4 vs[kPairsPerThread];
  unsigned keepm = 0, actm = 0;
  unsigned long long f1 = 0, f2 = 0;
  int32_t csg = -1;                        // segment of the counts held in registers
  unsigned long long cnt[3] = {0, 0, 0};  // evaluated, in P', in A
  // Every load of the thread's pairs is issued before any distance is taken
  // (keys and stored distances, then topology, then segment ids, moved flags and
  // the four vertices' positions), so the dependent gathers of the pairs overlap
  // instead of running one after the other. A pair of last iteration's P' none of
  // whose vertices the forward step moved keeps its stored distance: the same
  // function of the same positions.
  int32_t pv[kPairsPerThread][4];
  int32_t psg[kPairsPerThread];
  V3 px[kPairsPerThread][4];
  double dst[kPairsPerThread];
  bool fresh[kPairsPerThread];  // the distance is taken from the positions
#pragma unroll
  for (int k = 0; k < kPairsPerThread; ++k) {
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    keys[k] = i < a.nP ? a.P[i] : 0ull;
    dst[k] = i < a.nP && (a.mvd || i >= a.d_from) ? a.dPin[i] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < kPairsPerThread; ++k) {
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    if (i < a.nP) pair_verts(a.T, keys[k], pv[k]);
    else pv[k][0] = pv[k][1] = pv[k][2] = pv[k][3] = 0;
  }
#pragma unroll
  for (int k = 0; k < kPairsPerThread; ++k) {
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    psg[k] = a.one_seg >= 0 ? a.one_seg : a.vseg[pv[k][0]];
    fresh[k] = kCompute && i < a.d_from;
    if (fresh[k] && a.mvd)
      fresh[k] = (a.mvd[pv[k][0]] | a.mvd[pv[k][1]] | a.mvd[pv[k][2]] | a.mvd[pv[k][3]]) != 0;
    if (kCompute && k == 0 && fresh[k]) {
#pragma unroll
      for (int q = 0; q < 4; ++q) px[k][q] = ld3(a.x, pv[k][q]);
    }
  }
#pragma unroll
  for (int k = 0; k < kPairsPerThread; ++k) {
    // the next pair's positions are loaded while this pair's distance is taken
    if (kCompute && k + 1 < kPairsPerThread && fresh[k + 1]) {
#pragma unroll
      for (int q = 0; q < 4; ++q) px[k + 1][q] = ld3(a.x, pv[k + 1][q]);
    }
    const int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
    const uint64_t key = keys[k];
    keys[k] = 0;
    d2s[k] = 0.0;
    vs[k] = make_int4(0, 0, 0, 0);
    if (i < a.nP) {
      const int32_t* v = pv[k];
      const int32_t sg = psg[k];  // -1: a removed scene's pair
      const int32_t fl = sg >= 0 ? a.seg[sg].flags : 0;
      const bool live = (fl & kSegActive) && !(i < a.n_old && (fl & kSegSearched));
      if (live) {
        const double d2 =
            (kCompute && fresh[k]) ? pair_d2(key, px[k][0], px[k][1], px[k][2], px[k][3]) : dst[k];
        keys[k] = key;
        d2s[k] = d2;
        vs[k] = make_int4(v[0], v[1], v[2], v[3]);
        const bool keep = d2 < a.seg[sg].D2, act = keep && d2 < a.dl2;
        if (sg != csg && a.one_seg < 0) {
          seg_count_flush(gkey, gcnt, a.seg, csg, cnt);
          csg = sg;
        }
        if (a.one_seg < 0) {
          cnt[0] += 1;
          cnt[1] += keep ? 1 : 0;
          cnt[2] += act ? 1 : 0;
        }
        if (keep) {
          keepm |= 1u << k;
          if (a.trace) f1 += fp_key(key);
          if (act) {
            actm |= 1u << k;
            if (a.trace) f2 += fp_key(key);
          }
          unsigned long long bits = (unsigned long long)__double_as_longlong(sqrt(d2));
#pragma unroll
          for (int q = 0; q < 4; ++q) min_insert(hkey, hval, occ, &nocc, a.Di, v[q], bits);
        }
      }
    }
  }
  seg_count_flush(gkey, gcnt, a.seg, csg, cnt);
  __syncthreads();
  for (int t = threadIdx.x; t < nocc; t += kThreads) {
    const int h = occ[t];
    atomicMin(&a.Di[hkey[h]], hval[h]);  // no read first: the wave does not wait on it
  }
  // block-level compaction of P' and A
  int nk = __popc(keepm), na = __popc(actm), tk = 0, ta = 0;
  int ok = block_excl_scan(nk, ssc, &tk);
  int oa = block_excl_scan(na, ssc, &ta);
  if (threadIdx.x == 0) {
    // P' kept in place is P (each pair's stored d^2 came from the search, which kept
    // d^2 < D_max^2 by the same comparison): neither offsets nor a count
    sbase[0] = (!a.in_place && tk) ? atomicAdd(&a.c->n_out, (unsigned long long)tk) : 0ull;
    sbase[1] = ta ? atomicAdd(&a.c->n_act, (unsigned long long)ta) : 0ull;
  }
  if (threadIdx.x < kSegSlots && gkey[threadIdx.x] >= 0) {
    SegDev& sd = a.seg[gkey[threadIdx.x]];
    atomicAdd(&sd.n_p, gcnt[threadIdx.x][0]);
    if (gcnt[threadIdx.x][1]) atomicAdd(&sd.n_pf, gcnt[threadIdx.x][1]);
    if (gcnt[threadIdx.x][2]) atomicAdd(&sd.n_a, gcnt[threadIdx.x][2]);
  }
  __syncthreads();
  unsigned long long pk = sbase[0] + (unsigned long long)ok;
  unsigned long long pa = sbase[1] + (unsigned long long)oa;
#pragma unroll
  for (int k = 0; k < kPairsPerThread; ++k) {
    if (keepm & (1u << k)) {
      if (!a.in_place) {
        a.Pout[pk] = keys[k];
        a.dPout[pk] = d2s[k];
      }
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

int launch_pair_pass(cc_solver* s, int64_t n_old, int64_t d_from, double dl2, bool trace,
                     bool in_place, hipStream_t st) {
  PairPassArgs a;
  a.P = s->P;
  a.nP = s->nP;
  a.n_old = n_old;
  a.d_from = d_from;
  a.dPin = s->dP;
  a.mvd = s->mv_gen == s->gen ? s->mvd : nullptr;
  a.x = s->x;
  a.T = Topo{s->tris, s->edges};
  a.vseg = s->vseg;
  a.seg = s->seg_dev;
  a.dl2 = dl2;
  a.Pout = s->P2;
  a.dPout = s->dP2;
  a.Akeys = s->Akeys;
  a.Averts = s->Averts;
  a.capA = s->capA;
  a.Di = s->Di;
  a.c = s->dc;
  a.trace = trace ? 1 : 0;
  a.in_place = in_place ? 1 : 0;
  // one scene and no removed scene's pairs left in P: the segment of a pair is known
  // without its vertex's segment id
  a.one_seg = single_live_seg(s) ? 0 : -1;
  if (s->nP > 0) {
    const unsigned g = nblk(s->nP, kThreads * kPairsPerThread);
    if (d_from > 0) k_pair_pass<true><<<g, kThreads, 0, st>>>(a);
    else k_pair_pass<false><<<g, kThreads, 0, st>>>(a);
  }
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- colouring

// A row source: contact rows (key = pair key, 4 vertices) or edge-length rows
// (key = edge index, 2 vertices). The key returned is the scene-local one.
struct RowSrc {
  const uint64_t* keys;
  const int4* verts;
  const int32_t* edges;
  const int32_t* vseg;
  const int32_t* eseg;
  const SegDev* seg;
  int is_edge;
  __device__ __forceinline__ void get(int32_t r, uint64_t& key, int32_t v[4]) const {
    if (is_edge) {
      key = (uint64_t)(uint32_t)(r - seg[eseg[r]].eb);
      v[0] = edges[2 * r];
      v[1] = edges[2 * r + 1];
      v[2] = -1;
      v[3] = -1;
    } else {
      int4 q = verts[r];
      const uint64_t k = keys[r];
      v[0] = q.x;
      v[1] = q.y;
      v[2] = key_is_vv(k) ? -1 : q.z;  // a vertex-vertex row has two vertices
      v[3] = key_is_vv(k) ? -1 : q.w;
      key = local_pair_key(k, seg[vseg[q.x]]);
    }
  }
};

constexpr int kRoundsPerSync = 8;  // colouring rounds launched between host reads
constexpr int kTailRows = 4096;     // below this many rows one block finishes the rounds
constexpr int kTailThreads = 1024;
constexpr uint64_t kPhi = 0x9E3779B97F4A7C15ull;  // round step of the colouring hash

// Randomised palette colouring (Sec. 4.3 colours the constraints; the random
// choices are hashes of the row key, the seed and the round, so the colours depend
// only on the row set). A round over the uncoloured rows:
//   count:   unc[v] = uncoloured rows at free vertex v;
//   pick:    palette m = max(1, max_v unc[v]) + failed rounds of the row; the row
//            picks the (h mod m)-th smallest colour its coloured neighbours leave
//            free, h = mix64(mix64(key ^ seed) + t * phi), and claims it at its
//            free vertices (a second claim of a colour at a vertex marks a clash);
//   resolve: a row without a clash keeps its colour, the others fail and stay;
//   clear:   the round's counts and claims are reset.
struct PcArgs {
  RowSrc src;
  const double* w;
  uint64_t seed;
  unsigned long long* masks;   // colours used at each vertex (kMaskWords per vertex)
  unsigned long long* claims;  // per vertex: kMaskWords words of claims, then of clashes
  unsigned long long* unc;     // uncoloured rows per vertex (this round)
  int32_t* fails;              // per row: failed rounds
  int32_t* pick;               // per row: this round's pick
  int maxc;
  int32_t* colors;
  Counters* c;
  unsigned long long* lslot;  // one-block colouring of contact rows: each row's
  int32_t* lvert;             // block-local vertex slots, and each slot's vertex
};

__device__ __forceinline__ bool is_free(const double* w, int32_t v) { return v >= 0 && w[v] > 0.0; }

template <bool kAtomicLoads>
__device__ __forceinline__ unsigned long long ld_u64(const unsigned long long* p) {
  if (kAtomicLoads) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return *p;
}

__device__ __forceinline__ unsigned long long* claim_word(const PcArgs& a, int32_t v, int which,
                                                          int wd) {
  return a.claims + ((int64_t)v * 2 + which) * kMaskWords + wd;
}

__device__ __forceinline__ void pc_count(const PcArgs& a, int32_t r) {
  uint64_t key;
  int32_t v[4];
  a.src.get(r, key, v);
  a.colors[r] = 0;  // an uncoloured row reads as colour 0 should the rounds run out
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k])) atomicAdd(&a.unc[v[k]], 1ull);
}

template <bool kAtomicLoads>
__device__ __forceinline__ void pc_pick(const PcArgs& a, int32_t r, uint64_t t) {
  uint64_t key;
  int32_t v[4];
  a.src.get(r, key, v);
  unsigned long long m = 1;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k])) {
      const unsigned long long u = ld_u64<kAtomicLoads>(&a.unc[v[k]]);
      if (u > m) m = u;
    }
  m += (unsigned long long)a.fails[r];
  const uint64_t h = mix64(mix64(key ^ a.seed) + t * kPhi);
  unsigned long long want = h % m;
  int col = -1;
  const int W = (a.maxc + 63) / 64;
  for (int wd = 0; wd < W && col < 0; ++wd) {
    unsigned long long used = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (is_free(a.w, v[k])) used |= ld_u64<kAtomicLoads>(&a.masks[(int64_t)v[k] * kMaskWords + wd]);
    unsigned long long fr = ~used;
    const int lim = a.maxc - 64 * wd;  // palette limit inside this word
    if (lim < 64) fr &= (1ull << lim) - 1ull;
    const unsigned long long cnt = (unsigned long long)__popcll(fr);
    if (want >= cnt) {
      want -= cnt;
      continue;
    }
    for (unsigned long long q = 0; q < want; ++q) fr &= fr - 1ull;  // drop the lowest `want`
    col = 64 * wd + (__ffsll((long long)fr) - 1);
  }
  if (col < 0) {
    atomicOr(&a.c->err, 1ull);
    col = 0;
  }
  a.pick[r] = col;
  const unsigned long long bit = 1ull << (col % 64);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k])) {
      const unsigned long long old = atomicOr(claim_word(a, v[k], 0, col / 64), bit);
      if (old & bit) atomicOr(claim_word(a, v[k], 1, col / 64), bit);
    }
}

// Returns true when the row stays uncoloured; *colored gets the colour it took
// (-1 when it stays). The caller raises c->ncol to the colours taken.
template <bool kAtomicLoads>
__device__ __forceinline__ bool pc_resolve(const PcArgs& a, int32_t r, int* colored) {
  *colored = -1;
  uint64_t key;
  int32_t v[4];
  a.src.get(r, key, v);
  const int col = a.pick[r];
  const unsigned long long bit = 1ull << (col % 64);
  bool clash = false;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k]) && (ld_u64<kAtomicLoads>(claim_word(a, v[k], 1, col / 64)) & bit))
      clash = true;
  if (clash) {
    a.fails[r] += 1;
    return true;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k])) atomicOr(&a.masks[(int64_t)v[k] * kMaskWords + col / 64], bit);
  a.colors[r] = col;
  *colored = col;
  return false;
}

__device__ __forceinline__ void pc_clear(const PcArgs& a, int32_t r) {
  uint64_t key;
  int32_t v[4];
  a.src.get(r, key, v);
  const int wd = a.pick[r] / 64;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k])) {
      a.unc[v[k]] = 0ull;
      *claim_word(a, v[k], 0, wd) = 0ull;
      *claim_word(a, v[k], 1, wd) = 0ull;
    }
}

// One phase of a round over a list whose length lives on the device (rounds are
// launched ahead of the host knowing how many rows are left).
__global__ void __launch_bounds__(kThreads) k_pc_count(PcArgs a, const int32_t* list,
                                                       const unsigned long long* nlist) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (int64_t)*nlist) pc_count(a, list[t]);
}

__global__ void __launch_bounds__(kThreads) k_pc_pick(PcArgs a, const int32_t* list,
                                                      const unsigned long long* nlist,
                                                      uint64_t round) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (int64_t)*nlist) pc_pick<false>(a, list[t], round);
}

__global__ void __launch_bounds__(kThreads) k_pc_resolve(PcArgs a, const int32_t* list,
                                                         const unsigned long long* nlist,
                                                         int32_t* list_out,
                                                         unsigned long long* nout) {
  __shared__ int s_max[kThreads / 64];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < (int64_t)*nlist;
  const int32_t r = valid ? list[t] : 0;
  int col = -1;
  const bool stay = valid && pc_resolve<false>(a, r, &col);
  int nblock = 0;
  const unsigned long long pos = block_append(stay, nout, &nblock);
  if (stay) list_out[pos] = r;
  // the block's largest colour taken: one atomic per block
  for (int o = 32; o >= 1; o >>= 1) col = max(col, __shfl_xor(col, o));
  if (__lane_id() == 0) s_max[threadIdx.x >> 6] = col;
  __syncthreads();
  if (threadIdx.x == 0) {
    int mx = s_max[0];
    for (int w = 1; w < kThreads / 64; ++w) mx = max(mx, s_max[w]);
    if (mx >= 0) atomicMax(&a.c->ncol, (unsigned long long)(mx + 1));
  }
}

__global__ void __launch_bounds__(kThreads) k_pc_clear(PcArgs a, const int32_t* list,
                                                       const unsigned long long* nlist) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (int64_t)*nlist) pc_clear(a, list[t]);
}

// Rounds t0, t0 + 1, ... over the list cur[0, *ncur) in one block: global atomics,
// atomic loads to read what other threads wrote, block barriers between the
// phases (ncur and nnext live in LDS).
__device__ void pc_rounds_block(const PcArgs& a, int32_t* cur, int32_t* nxt, int32_t* ncur,
                                int32_t* nnext, uint64_t t0, uint64_t tmax) {
  for (uint64_t t = t0; *ncur > 0; ++t) {
    if (t > tmax) {
      if (threadIdx.x == 0) atomicOr(&a.c->err, 1ull);
      break;
    }
    const int32_t nc = *ncur;
    for (int32_t i = threadIdx.x; i < nc; i += blockDim.x) pc_count(a, cur[i]);
    __syncthreads();
    for (int32_t i = threadIdx.x; i < nc; i += blockDim.x) pc_pick<true>(a, cur[i], t);
    __syncthreads();
    for (int32_t i = threadIdx.x; i < nc; i += blockDim.x) {
      const int32_t r = cur[i];
      int col;
      if (pc_resolve<true>(a, r, &col)) nxt[atomicAdd(nnext, 1)] = r;
      else atomicMax(&a.c->ncol, (unsigned long long)(col + 1));
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < nc; i += blockDim.x) pc_clear(a, cur[i]);
    __syncthreads();
    if (threadIdx.x == 0) {
      *ncur = *nnext;
      *nnext = 0;
    }
    int32_t* tmp = cur;
    cur = nxt;
    nxt = tmp;
    __syncthreads();
  }
}

// The remaining rounds (from round t0) of a list whose length lives on the device.
__global__ void __launch_bounds__(kTailThreads) k_pc_tail(PcArgs a, int32_t* la, int32_t* lb,
                                                          const unsigned long long* nlist,
                                                          uint64_t t0, uint64_t tmax) {
  __shared__ int32_t ncur, nnext;
  if (threadIdx.x == 0) {
    ncur = (int32_t)*nlist;
    nnext = 0;
  }
  __syncthreads();
  pc_rounds_block(a, la, lb, &ncur, &nnext, t0, tmax);
}

constexpr int kSmallPer = kSmallRows / kTailThreads;  // rows per thread
// LDS layouts of the one-block colouring: kLocWords colour words per vertex (colours
// below 64 kLocWords) for at most kLocCap distinct free vertices: one word for 4096
// vertices, two words for 2944. The colour words are sized for the larger of the two
// (the one-word kernel can start again with two words): about 158 KB of LDS with the
// rest of the block's state, within the 160 KB a block may take on gfx950.
constexpr int kLocCap2 = 2944;
static_assert(kSmallRows % kTailThreads == 0, "whole rows per thread");
static_assert(kMaxColors == kTailThreads, "one thread per colour bucket in the scan");

// The same rounds (from round 1) over every contact row [0, nrows) in one block,
// with the per-vertex state in LDS. The rows' free vertices get block-local slots
// through an open-addressing table in LDS (kHashSize entries, linear probing; it
// borrows the claim and clash words, which the rounds clear before use): each
// (row, corner) enters its vertex with a compare-and-swap, each entry it creates
// takes the next slot, and every corner reads its entry's slot. A thread keeps its
// rows (row t + k * kTailThreads) in registers. When more than kLocCap vertices
// take part (or a vertex finds no place within kHashProbes), or a pick would need
// a colour beyond the kLocWords words in LDS, the block runs the global-memory
// rounds from round 1 instead, with the same result (the colours depend only on
// the row set). Then the colour buckets: counts, their exclusive scan to off
// (kMaxColors + 1 entries), the rows in colour order to order; the colour count
// goes to c->ncol.
// The colouring rounds of the one-block colouring, from round 1, with the state of
// each vertex slot in LDS: kW colour words (64 colours each) per slot. A pick beyond
// kW words sets *s_over and abandons the rounds.
template <int kW>
__device__ __forceinline__ void lds_rounds(const PcArgs& a, int32_t nrows, uint64_t tmax,
                                           unsigned* s_unc, unsigned long long (*s_mask)[kW],
                                           unsigned long long (*s_claim)[kW],
                                           unsigned long long (*s_clash)[kW], int32_t* s_live,
                                           int32_t* s_next, int32_t* s_ncol, int32_t* s_over,
                                           const uint64_t (&hk)[kSmallPer],
                                           const int32_t (&lid)[kSmallPer][4],
                                           int32_t (&fails)[kSmallPer], int32_t (&pick)[kSmallPer],
                                           int32_t (&col)[kSmallPer]) {
  const int tid = threadIdx.x;
  const int W = (a.maxc + 63) / 64;
  for (uint64_t t = 1; *s_live > 0; ++t) {
    if (t > tmax) {
      if (tid == 0) atomicOr(&a.c->err, 1ull);
      break;
    }
    unsigned live = 0;
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      if (tid + k * kTailThreads >= nrows || col[k] >= 0) continue;
      live |= 1u << k;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (lid[k][q] >= 0) atomicAdd(&s_unc[lid[k][q]], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      if (!(live & (1u << k))) continue;
      unsigned long long m = 1;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (lid[k][q] >= 0 && (unsigned long long)s_unc[lid[k][q]] > m) m = s_unc[lid[k][q]];
      m += (unsigned long long)fails[k];
      unsigned long long want = mix64(hk[k] + t * kPhi) % m;
      int c = -1;
      bool over = false;
      for (int wd = 0; wd < W && c < 0; ++wd) {
        if (wd >= kW) {
          over = true;
          break;
        }
        unsigned long long used = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (lid[k][q] >= 0) used |= s_mask[lid[k][q]][wd];
        unsigned long long fr = ~used;
        const int lim = a.maxc - 64 * wd;
        if (lim < 64) fr &= (1ull << lim) - 1ull;
        const unsigned long long cnt = (unsigned long long)__popcll(fr);
        if (want >= cnt) {
          want -= cnt;
          continue;
        }
        for (unsigned long long z = 0; z < want; ++z) fr &= fr - 1ull;
        c = 64 * wd + (__ffsll((long long)fr) - 1);
      }
      if (over) {
        *s_over = 1;
        c = 0;  // the round is abandoned
      } else if (c < 0) {
        atomicOr(&a.c->err, 1ull);
        c = 0;
      }
      pick[k] = c;
      const unsigned long long bit = 1ull << (c % 64);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (lid[k][q] < 0) continue;
        const unsigned long long old = atomicOr(&s_claim[lid[k][q]][c / 64], bit);
        if (old & bit) atomicOr(&s_clash[lid[k][q]][c / 64], bit);
      }
    }
    __syncthreads();
    if (*s_over) break;
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      if (!(live & (1u << k))) continue;
      const int c = pick[k];
      const unsigned long long bit = 1ull << (c % 64);
      bool clash = false;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (lid[k][q] >= 0 && (s_clash[lid[k][q]][c / 64] & bit)) clash = true;
      if (clash) {
        fails[k] += 1;
        atomicAdd(s_next, 1);
        continue;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (lid[k][q] >= 0) atomicOr(&s_mask[lid[k][q]][c / 64], bit);
      col[k] = c;
      atomicMax(s_ncol, c + 1);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      if (!(live & (1u << k))) continue;
      const int wd = pick[k] / 64;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (lid[k][q] < 0) continue;
        s_unc[lid[k][q]] = 0u;
        s_claim[lid[k][q]][wd] = 0ull;
        s_clash[lid[k][q]][wd] = 0ull;
      }
    }
    if (tid == 0) {
      *s_live = *s_next;
      *s_next = 0;
    }
    __syncthreads();
  }
}

constexpr int kHashBits = 13, kHashSize = 1 << kHashBits;
// probes before a vertex gives up its place (at most kLocCap1 = kHashSize / 2 vertices
// fit the LDS state, so a table that holds them is at most half full)
constexpr int kHashProbes = 64;
template <int kLocWords, int kLocCap>
__global__ void __launch_bounds__(kTailThreads) k_pc_small(PcArgs a, int32_t nrows, int32_t* la,
                                                           int32_t* lb,
                                                           int32_t* __restrict__ order,
                                                           int32_t* __restrict__ off,
                                                           uint64_t tmax) {
  // the colour words of the slots, sized for either layout (kLocCap slots of kLocWords
  // words, or kLocCap2 slots of two words for a restart)
  constexpr int kWordsMax = kLocCap * kLocWords > 2 * kLocCap2 ? kLocCap * kLocWords : 2 * kLocCap2;
  __shared__ unsigned s_unc[kLocCap > kLocCap2 ? kLocCap : kLocCap2];
  __shared__ unsigned long long s_maskw[kWordsMax], s_claimw[kWordsMax], s_clashw[kWordsMax];
  auto s_mask = reinterpret_cast<unsigned long long(*)[kLocWords]>(s_maskw);
  auto s_claim = reinterpret_cast<unsigned long long(*)[kLocWords]>(s_claimw);
  auto s_clash = reinterpret_cast<unsigned long long(*)[kLocWords]>(s_clashw);
  __shared__ int32_t s_cnt[kMaxColors];
  __shared__ int32_t s_wsum[kTailThreads / 64];
  __shared__ int32_t s_nloc, s_live, s_next, s_ncol, s_over, ncur, nnext;
  static_assert(sizeof(s_claimw) >= sizeof(int32_t) * kHashSize &&
                    sizeof(s_clashw) >= sizeof(int32_t) * kHashSize,
                "the vertex table fits the claim and clash words");
  int32_t* const hkey = reinterpret_cast<int32_t*>(s_claimw);   // vertex id, -1: empty
  int32_t* const hslot = reinterpret_cast<int32_t*>(s_clashw);  // its slot
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_nloc = 0;
    s_live = nrows;
    s_next = 0;
    s_ncol = 0;
    s_over = 0;
  }
  s_cnt[tid] = 0;
  for (int h = tid; h < kHashSize; h += kTailThreads) hkey[h] = -1;
  uint64_t hk[kSmallPer];
  int32_t vid[kSmallPer][4], lid[kSmallPer][4];
  int32_t fails[kSmallPer], pick[kSmallPer], col[kSmallPer];
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int32_t r = tid + k * kTailThreads;
    fails[k] = 0;
    pick[k] = 0;
    col[k] = -1;
    hk[k] = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) vid[k][q] = lid[k][q] = -1;
    if (r < nrows) {
      uint64_t key;
      int32_t v[4];
      a.src.get(r, key, v);
      hk[k] = mix64(key ^ a.seed);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (is_free(a.w, v[q])) vid[k][q] = v[q];
    }
  }
  __syncthreads();
  // every free corner enters its vertex; lid holds the table position for now
  unsigned made = 0;  // bit 4k + q: this corner created its vertex's entry
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t v = vid[k][q];
      if (v < 0) continue;
      uint32_t h = ((uint32_t)v * 2654435761u) >> (32 - kHashBits);
      int n = 0;
      for (; n < kHashProbes; ++n, h = (h + 1) & (kHashSize - 1)) {
        const int32_t old = atomicCAS(&hkey[h], -1, v);
        if (old == -1) made |= 1u << (4 * k + q);
        if (old == -1 || old == v) break;
      }
      if (n == kHashProbes) s_over = 1;  // a crowded table: the global rounds colour
      lid[k][q] = (int32_t)h;
    }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!(made & (1u << (4 * k + q)))) continue;
      const int32_t l = atomicAdd(&s_nloc, 1);
      hslot[lid[k][q]] = l;
      if (l < kLocCap && a.lvert) a.lvert[l] = vid[k][q];
    }
  __syncthreads();
  const bool in_lds = s_nloc <= kLocCap && !s_over;
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (vid[k][q] >= 0) lid[k][q] = in_lds ? hslot[lid[k][q]] : -1;
  __syncthreads();
  // the slots' state starts clear (the table is done with)
  if (in_lds)
    for (int l = tid; l < s_nloc; l += kTailThreads) {
      s_unc[l] = 0u;
#pragma unroll
      for (int wd = 0; wd < kLocWords; ++wd) s_mask[l][wd] = s_claim[l][wd] = s_clash[l][wd] = 0ull;
    }
  __syncthreads();
  if (in_lds) {
    lds_rounds<kLocWords>(a, nrows, tmax, s_unc, s_mask, s_claim, s_clash, &s_live, &s_next,
                          &s_ncol, &s_over, hk, lid, fails, pick, col);
    // more colours than one word holds: the rounds start again from round 1 with two
    // words per slot in the same LDS when the slots fit (kLocCap2 of them)
    if (kLocWords == 1 && s_over && s_nloc <= kLocCap2) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kSmallPer; ++k) {
        col[k] = -1;
        fails[k] = 0;
        pick[k] = 0;
      }
      auto m2 = reinterpret_cast<unsigned long long(*)[2]>(s_maskw);
      auto c2 = reinterpret_cast<unsigned long long(*)[2]>(s_claimw);
      auto k2 = reinterpret_cast<unsigned long long(*)[2]>(s_clashw);
      for (int l = tid; l < s_nloc; l += kTailThreads) {
        s_unc[l] = 0u;
        m2[l][0] = m2[l][1] = c2[l][0] = c2[l][1] = k2[l][0] = k2[l][1] = 0ull;
      }
      __syncthreads();
      if (tid == 0) {
        s_live = nrows;
        s_next = 0;
        s_ncol = 0;
        s_over = 0;
      }
      __syncthreads();
      lds_rounds<2>(a, nrows, tmax, s_unc, m2, c2, k2, &s_live, &s_next, &s_ncol, &s_over, hk,
                    lid, fails, pick, col);
    }
  }
  const bool global_rounds = !in_lds || s_over;
  if (global_rounds) {
    // every row in the list, none failed yet, no colour at its vertices yet
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const int32_t r = tid + k * kTailThreads;
      if (r >= nrows) continue;
      la[r] = r;
      a.fails[r] = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (vid[k][q] >= 0)
          for (int wd = 0; wd < kMaskWords; ++wd) a.masks[(int64_t)vid[k][q] * kMaskWords + wd] = 0ull;
    }
    if (tid == 0) {
      ncur = nrows;
      nnext = 0;
    }
    __syncthreads();
    pc_rounds_block(a, la, lb, &ncur, &nnext, 1, tmax);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
      const int32_t r = tid + k * kTailThreads;
      if (r < nrows) col[k] = __hip_atomic_load(&a.colors[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  // colour buckets (a row left uncoloured by the round limit reads as colour 0)
  int32_t rank[kSmallPer];
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    rank[k] = 0;
    if (tid + k * kTailThreads >= nrows) continue;
    if (col[k] < 0) col[k] = 0;
    rank[k] = atomicAdd(&s_cnt[col[k]], 1);
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  const int32_t cv = s_cnt[tid];
  int32_t incl = cv;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (lane == 63) s_wsum[wv] = incl;
  __syncthreads();
  int32_t before = 0;
  for (int w = 0; w < wv; ++w) before += s_wsum[w];
  const int32_t ex = before + incl - cv;
  __syncthreads();
  s_cnt[tid] = ex;
  off[tid] = ex;
  if (tid == kTailThreads - 1) off[kMaxColors] = ex + cv;
  if (tid == 0 && !global_rounds) a.c->ncol = (unsigned long long)s_ncol;
  // the rows' block-local slots, for a projection that keeps y at them in LDS
  if (tid == 0 && a.lslot) a.c->nloc = global_rounds ? ~0ull : (unsigned long long)s_nloc;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSmallPer; ++k) {
    const int32_t r = tid + k * kTailThreads;
    if (r >= nrows) continue;
    order[s_cnt[col[k]] + rank[k]] = r;
    a.colors[r] = col[k];
    if (a.lslot && !global_rounds) {
      unsigned long long ps = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        ps |= (unsigned long long)(lid[k][q] >= 0 ? (uint32_t)lid[k][q] : 0xffffu) << (16 * q);
      a.lslot[r] = ps;
    }
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

// Exclusive scan of the kMaxColors bucket counts (one block of kMaxColors
// threads): offsets to `off` (kMaxColors + 1 entries) and, as the scatter's
// cursors, back into `cnt`.
__global__ void __launch_bounds__(kMaxColors) k_bucket_offsets(int32_t* __restrict__ cnt,
                                                               int32_t* __restrict__ off) {
  __shared__ int32_t wsum[kMaxColors / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int32_t v = cnt[t];
  int32_t incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    int32_t u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  int32_t before = 0, total = 0;
  for (int w = 0; w < kMaxColors / 64; ++w) {
    if (w < wv) before += wsum[w];
    total += wsum[w];
  }
  const int32_t ex = before + incl - v;
  off[t] = ex;
  cnt[t] = ex;
  if (t == 0) off[kMaxColors] = total;
}

static PcArgs pc_args(cc_solver* s, bool edges) {
  PcArgs a;
  a.src = RowSrc{s->Akeys, s->Averts, s->edges, s->vseg, s->eseg, s->seg_dev, edges ? 1 : 0};
  a.w = s->w;
  a.seed = s->p.seed;
  a.masks = s->masks;
  a.claims = s->claims;
  a.unc = s->vmax0;
  a.fails = edges ? s->efail : s->afail;
  a.pick = edges ? s->epick : s->apick;
  a.maxc = s->p.max_colors;
  a.colors = edges ? s->ecol : s->Acol;
  a.c = s->dc;
  a.lslot = edges ? nullptr : s->Aslot;
  a.lvert = edges ? nullptr : s->lvert;
  return a;
}

int color_small(cc_solver* s, hipStream_t st) {
  s->col_off.assign(1, 0);
  s->n_colors = 0;
  s->col_small = true;
  if (s->nA == 0) return CC_OK;
  if (s->nA > kSmallRows) return CC_EINVAL;
  if (s->pc_dirty) {  // an aborted colouring left counts or claims behind (over any extent)
    CC_HIP(hipMemsetAsync(s->vmax0, 0, sizeof(unsigned long long) * (size_t)s->capV, st));
    CC_HIP(hipMemsetAsync(s->claims, 0, sizeof(unsigned long long) * (size_t)s->capV * 2 * kMaskWords,
                          st));
  }
  // clean again once the iteration's counters show no colouring error
  s->pc_dirty = true;
  // one colour word (4096 vertices) unless the last such colouring used more than 56
  // colours; either way a set that does not fit is still coloured, by the global rounds
  if (s->pc_wide)
    k_pc_small<2, kLocCap2><<<1, kTailThreads, 0, st>>>(pc_args(s, false), (int32_t)s->nA,
                                                        s->list0, s->list1, s->Aorder,
                                                        s->coff_dev, (uint64_t)kMaxRounds);
  else
    k_pc_small<1, kLocCap1><<<1, kTailThreads, 0, st>>>(pc_args(s, false), (int32_t)s->nA,
                                                        s->list0, s->list1, s->Aorder,
                                                        s->coff_dev, (uint64_t)kMaxRounds);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// Colour the contact rows (A, then bucket them by colour) or the edge-length
// rows listed in elist0[0, n_newrows) (the rows of segments being begun; their
// buckets are built over every iterating segment by build_edge_buckets).
int color_rows(cc_solver* s, bool edges, hipStream_t st) {
  const int64_t nrows = edges ? s->n_newrows : s->nA;
  int32_t* colors = edges ? s->ecol : s->Acol;
  if (edges) s->ecache.ok = false;  // the cached colours are overwritten from here on
  if (!edges) {
    s->col_off.assign(1, 0);
    s->n_colors = 0;
    s->col_small = false;
  }
  if (nrows == 0) return CC_OK;
  int32_t *cur, *nxt;
  if (edges) {
    CC_HIP(hipMemcpyAsync(s->elist1, s->elist0, sizeof(int32_t) * nrows, hipMemcpyDeviceToDevice, st));
    cur = s->elist1;
    nxt = s->elist2;
  } else {
    k_iota<<<nblk(nrows), kThreads, 0, st>>>(s->list0, nrows);
    cur = s->list0;
    nxt = s->list1;
  }
  if (s->pc_dirty) {  // an aborted colouring left counts or claims behind (over any extent)
    CC_HIP(hipMemsetAsync(s->vmax0, 0, sizeof(unsigned long long) * (size_t)s->capV, st));
    CC_HIP(hipMemsetAsync(s->claims, 0, sizeof(unsigned long long) * (size_t)s->capV * 2 * kMaskWords,
                          st));
    s->pc_dirty = false;
  }
  CC_HIP(hipMemsetAsync(s->masks, 0, sizeof(unsigned long long) * s->n * kMaskWords, st));
  CC_HIP(hipMemsetAsync(&s->dc->ncol, 0, sizeof(unsigned long long), st));
  CC_HIP(hipMemsetAsync(&s->dc->err, 0, sizeof(unsigned long long), st));
  CC_HIP(hipMemsetAsync(s->rcnt, 0, sizeof(unsigned long long) * (kMaxRounds + 1), st));
  CC_TRY(launch_fill_u64(s->rcnt, 1, (unsigned long long)nrows, st));
  if (edges) CC_TRY(launch_fill_i32(s->efail, s->capE, 0, st));
  else CC_TRY(launch_fill_i32(s->afail, nrows, 0, st));
  const PcArgs a = pc_args(s, edges);
  int64_t known = nrows;  // upper bound of the current list length
  int round = 0;          // rounds done; round t = round + 1 is next
  s->pc_dirty = true;
  for (;;) {
    if (known <= kTailRows) {
      k_pc_tail<<<1, kTailThreads, 0, st>>>(a, cur, nxt, s->rcnt + round, (uint64_t)round + 1,
                                            (uint64_t)kMaxRounds);
      break;
    }
    if (round + kRoundsPerSync > kMaxRounds) return CC_ECOLOR;
    for (int b = 0; b < kRoundsPerSync; ++b) {
      const unsigned g = nblk(known);
      k_pc_count<<<g, kThreads, 0, st>>>(a, cur, s->rcnt + round);
      k_pc_pick<<<g, kThreads, 0, st>>>(a, cur, s->rcnt + round, (uint64_t)round + 1);
      k_pc_resolve<<<g, kThreads, 0, st>>>(a, cur, s->rcnt + round, nxt, s->rcnt + round + 1);
      k_pc_clear<<<g, kThreads, 0, st>>>(a, cur, s->rcnt + round);
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
  if (edges) {
    CC_HIP(hipMemcpyAsync(s->hc, s->dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    if (s->hc->err & 1ull) return CC_ECOLOR;
    s->pc_dirty = false;
    return CC_OK;
  }
  // contact buckets: counts, offsets (one-block scan) and the scatter are queued
  // behind the colouring; one readback brings the colour count and the offsets
  CC_HIP(hipMemsetAsync(s->col_cnt, 0, sizeof(int32_t) * (kMaxColors + 1), st));
  k_bucket_count<<<nblk(nrows), kThreads, 0, st>>>(nullptr, nrows, colors, kMaxColors, s->col_cnt);
  k_bucket_offsets<<<1, kMaxColors, 0, st>>>(s->col_cnt, s->coff_dev);
  k_bucket_scatter<<<nblk(nrows), kThreads, 0, st>>>(nullptr, nrows, colors, kMaxColors,
                                                    s->col_cnt, s->Aorder);
  CC_HIP(hipGetLastError());
  std::vector<int32_t>& off = s->col_off;
  off.resize(kMaxColors + 1);
  CC_HIP(hipMemcpyAsync(s->hc, s->dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
  CC_HIP(hipMemcpyAsync(off.data(), s->coff_dev, sizeof(int32_t) * (kMaxColors + 1),
                        hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (s->hc->err & 1ull) return CC_ECOLOR;
  s->pc_dirty = false;
  const int32_t ncol = (int32_t)s->hc->ncol;
  off.resize(ncol + 1);
  s->n_colors = ncol;
  return CC_OK;
}

// ------------------------------------------------------------- greedy colouring of edge rows

// The edge-length rows' colouring: greedy in decreasing priority, prio = (high 32
// bits of mix64(key ^ seed)) << 32 | key (distinct for distinct keys), each row
// taking the smallest colour not used by an already coloured row at one of its free
// vertices. Found by Jones-Plassmann rounds: a row whose priority is the largest
// among the uncoloured rows at each of its free vertices takes its colour in the
// round; two such rows share no free vertex, and every row with a higher priority
// at its vertices is coloured by then, so the result is the greedy colouring.
__device__ __forceinline__ uint64_t greedy_prio(uint64_t key, uint64_t seed) {
  return (mix64(key ^ seed) & 0xFFFFFFFF00000000ull) | (key & 0xFFFFFFFFull);
}

// Round part 1: the largest priority of the uncoloured rows at each free vertex
// (a.unc, zero between rounds).
__global__ void __launch_bounds__(kThreads) k_jp_max(PcArgs a, const int32_t* list,
                                                    const unsigned long long* nlist) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)*nlist) return;
  uint64_t key;
  int32_t v[4];
  a.src.get(list[t], key, v);
  const uint64_t p = greedy_prio(key, a.seed);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k])) atomicMax(&a.unc[v[k]], (unsigned long long)p);
}

// Round part 2: a row that holds the largest priority at each of its free vertices
// takes the smallest colour free at them and marks it there (no other row taking a
// colour in this round shares those vertices); the others go to list_out. The
// largest colour taken raises c->ncol once per block.
__global__ void __launch_bounds__(kThreads) k_jp_pick(PcArgs a, const int32_t* list,
                                                     const unsigned long long* nlist,
                                                     int32_t* list_out,
                                                     unsigned long long* nout) {
  __shared__ int s_max[kThreads / 64];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < (int64_t)*nlist;
  int32_t r = 0;
  bool stay = false;
  int col = -1;
  if (valid) {
    r = list[t];
    uint64_t key;
    int32_t v[4];
    a.src.get(r, key, v);
    const uint64_t p = greedy_prio(key, a.seed);
    bool top = true;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (is_free(a.w, v[k]) && a.unc[v[k]] != (unsigned long long)p) top = false;
    if (!top) {
      stay = true;
    } else {
      const int words = (a.maxc + 63) / 64;
      for (int wd = 0; wd < words && col < 0; ++wd) {
        unsigned long long u = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (is_free(a.w, v[k])) u |= a.masks[(int64_t)v[k] * kMaskWords + wd];
        if (~u) {
          const int c = wd * 64 + __ffsll((long long)~u) - 1;
          if (c < a.maxc) col = c;
          else break;
        }
      }
      if (col < 0) {
        atomicOr(&a.c->err, 1ull);  // the palette limit: no colour left
      } else {
        a.colors[r] = col;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (is_free(a.w, v[k]))
            atomicOr(&a.masks[(int64_t)v[k] * kMaskWords + col / 64], 1ull << (col % 64));
      }
    }
  }
  int nblock = 0;
  const unsigned long long pos = block_append(stay, nout, &nblock);
  if (stay) list_out[pos] = r;
  for (int o = 32; o >= 1; o >>= 1) col = max(col, __shfl_xor(col, o));
  if (__lane_id() == 0) s_max[threadIdx.x >> 6] = col;
  __syncthreads();
  if (threadIdx.x == 0) {
    int mx = s_max[0];
    for (int w = 1; w < kThreads / 64; ++w) mx = max(mx, s_max[w]);
    if (mx >= 0) atomicMax(&a.c->ncol, (unsigned long long)(mx + 1));
  }
}

// Round part 3: the priorities of the round's rows cleared at their vertices.
__global__ void __launch_bounds__(kThreads) k_jp_clear(PcArgs a, const int32_t* list,
                                                      const unsigned long long* nlist) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)*nlist) return;
  uint64_t key;
  int32_t v[4];
  a.src.get(list[t], key, v);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (is_free(a.w, v[k])) a.unc[v[k]] = 0ull;
}

int color_edges_greedy(cc_solver* s, hipStream_t st) {
  const int64_t nrows = s->n_newrows;
  s->ecache.ok = false;  // the cached colours are overwritten from here on
  if (nrows == 0) return CC_OK;
  CC_HIP(hipMemcpyAsync(s->elist1, s->elist0, sizeof(int32_t) * nrows, hipMemcpyDeviceToDevice, st));
  int32_t *cur = s->elist1, *nxt = s->elist2;
  if (s->pc_dirty) {  // an aborted colouring left counts or claims behind
    CC_HIP(hipMemsetAsync(s->vmax0, 0, sizeof(unsigned long long) * (size_t)s->capV, st));
    CC_HIP(hipMemsetAsync(s->claims, 0, sizeof(unsigned long long) * (size_t)s->capV * 2 * kMaskWords,
                          st));
    s->pc_dirty = false;
  }
  CC_HIP(hipMemsetAsync(s->masks, 0, sizeof(unsigned long long) * s->n * kMaskWords, st));
  CC_HIP(hipMemsetAsync(&s->dc->ncol, 0, sizeof(unsigned long long), st));
  CC_HIP(hipMemsetAsync(&s->dc->err, 0, sizeof(unsigned long long), st));
  CC_HIP(hipMemsetAsync(s->rcnt, 0, sizeof(unsigned long long) * (kMaxRounds + 1), st));
  CC_TRY(launch_fill_u64(s->rcnt, 1, (unsigned long long)nrows, st));
  const PcArgs a = pc_args(s, true);
  int64_t known = nrows;  // upper bound of the current list length
  int round = 0;
  s->pc_dirty = true;  // until the rounds end with every priority cleared
  while (known > 0) {
    if (round + kRoundsPerSync > kMaxRounds) return CC_ECOLOR;
    for (int b = 0; b < kRoundsPerSync; ++b) {
      const unsigned g = nblk(known);
      k_jp_max<<<g, kThreads, 0, st>>>(a, cur, s->rcnt + round);
      k_jp_pick<<<g, kThreads, 0, st>>>(a, cur, s->rcnt + round, nxt, s->rcnt + round + 1);
      k_jp_clear<<<g, kThreads, 0, st>>>(a, cur, s->rcnt + round);
      std::swap(cur, nxt);
      ++round;
    }
    CC_HIP(hipGetLastError());
    CC_HIP(hipMemcpyAsync(&s->hc->n_left, s->rcnt + round, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, st));
    CC_HIP(hipMemcpyAsync(&s->hc->err, &s->dc->err, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    if (s->hc->err & 1ull) return CC_ECOLOR;
    known = (int64_t)s->hc->n_left;
  }
  s->pc_dirty = false;
  return CC_OK;
}

// ------------------------------------------------------------- edge colouring cache

__global__ void k_ecache(const int32_t* __restrict__ edges, const double* __restrict__ einv,
                         const double* __restrict__ w, int32_t ne, int32_t nv,
                         int32_t* __restrict__ cedges, uint8_t* __restrict__ crow,
                         uint8_t* __restrict__ cfree, int store, unsigned long long* mis) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool diff = false;
  if (i < ne) {
    const int32_t a = edges[2 * i], b = edges[2 * i + 1];
    const uint8_t r = einv[i] != 0.0 ? 1 : 0;
    if (store) {
      cedges[2 * i] = a;
      cedges[2 * i + 1] = b;
      crow[i] = r;
    } else {
      diff = cedges[2 * i] != a || cedges[2 * i + 1] != b || crow[i] != r;
    }
  }
  if (i < nv) {
    const uint8_t f = w[i] > 0.0 ? 1 : 0;
    if (store) cfree[i] = f;
    else diff = diff || cfree[i] != f;
  }
  if (__any(diff) && __lane_id() == 0) atomicAdd(mis, 1ull);  // only on a difference
}

int ecache_compare(cc_solver* s, hipStream_t st) {
  auto& c = s->ecache;
  CC_HIP(hipMemsetAsync(&s->dc->ecmis, 0, sizeof(unsigned long long), st));
  const int32_t n = std::max(c.ne, c.nv);
  if (n > 0)
    k_ecache<<<nblk(n), kThreads, 0, st>>>(s->edges, s->einv, s->w, c.ne, c.nv, c.edges, c.row,
                                           c.freev, 0, &s->dc->ecmis);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

int ecache_store(cc_solver* s, hipStream_t st) {
  auto& c = s->ecache;
  c.ok = false;
  const Seg& g = s->segs[0];
  if (g.ne > c.cap_e) {
    if (c.edges) (void)hipFree(c.edges);
    if (c.row) (void)hipFree(c.row);
    c.edges = nullptr;
    c.row = nullptr;
    c.cap_e = 0;
    if (hipMalloc((void**)&c.edges, sizeof(int32_t) * 2 * (size_t)g.ne) != hipSuccess ||
        hipMalloc((void**)&c.row, (size_t)g.ne) != hipSuccess)
      return CC_OK;  // no cache: the next begin colours again
    c.cap_e = g.ne;
  }
  if (g.nv > c.cap_v) {
    if (c.freev) (void)hipFree(c.freev);
    c.freev = nullptr;
    c.cap_v = 0;
    if (hipMalloc((void**)&c.freev, (size_t)g.nv) != hipSuccess) return CC_OK;
    c.cap_v = g.nv;
  }
  const int32_t n = std::max(g.ne, g.nv);
  if (n > 0)
    k_ecache<<<nblk(n), kThreads, 0, st>>>(s->edges, s->einv, s->w, g.ne, g.nv, c.edges, c.row,
                                           c.freev, 1, &s->dc->ecmis);
  CC_HIP(hipGetLastError());
  c.ok = true;
  c.seed = s->p.seed;
  c.maxc = s->p.max_colors;
  c.ne = g.ne;
  c.nv = g.nv;
  c.rows = s->n_newrows;
  return CC_OK;
}

void ecache_free(cc_solver* s) {
  auto& c = s->ecache;
  if (c.edges) (void)hipFree(c.edges);
  if (c.row) (void)hipFree(c.row);
  if (c.freev) (void)hipFree(c.freev);
  c = cc_solver::EdgeColourCache{};
}

// Edge rows of every iterating segment, bucketed by colour (rows of one colour
// share no free vertex, so the order inside a bucket is free).
__device__ __forceinline__ bool erow_live(int32_t e, const int32_t* eseg, const SegDev* seg,
                                          const double* einv) {
  const int32_t sg = eseg[e];
  return sg >= 0 && (seg[sg].flags & kSegActive) && einv[e] > 0.0;
}

__global__ void __launch_bounds__(kThreads) k_ebucket_count(const int32_t* __restrict__ eseg,
                                                            const SegDev* __restrict__ seg,
                                                            const double* __restrict__ einv,
                                                            const int32_t* __restrict__ colors,
                                                            int32_t ne, int32_t* __restrict__ cnt) {
  __shared__ int32_t h[kMaxColors];
  for (int c = threadIdx.x; c < kMaxColors; c += kThreads) h[c] = 0;
  __syncthreads();
  int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne && erow_live(e, eseg, seg, einv)) atomicAdd(&h[colors[e]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < kMaxColors; c += kThreads)
    if (h[c]) atomicAdd(&cnt[c], h[c]);
}

__global__ void __launch_bounds__(kThreads) k_ebucket_scatter(const int32_t* __restrict__ eseg,
                                                              const SegDev* __restrict__ seg,
                                                              const double* __restrict__ einv,
                                                              const int32_t* __restrict__ colors,
                                                              int32_t ne,
                                                              int32_t* __restrict__ cursor,
                                                              int32_t* __restrict__ order,
                                                              const int32_t* __restrict__ edges,
                                                              int2* __restrict__ eij) {
  __shared__ int32_t h[kMaxColors];
  for (int c = threadIdx.x; c < kMaxColors; c += kThreads) h[c] = 0;
  __syncthreads();
  int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = e < ne && erow_live(e, eseg, seg, einv);
  int32_t c = 0, rank = 0;
  if (live) {
    c = colors[e];
    rank = atomicAdd(&h[c], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kMaxColors; k += kThreads)
    if (h[k]) h[k] = atomicAdd(&cursor[k], h[k]);
  __syncthreads();
  if (live) {
    order[h[c] + rank] = e;
    eij[h[c] + rank] = make_int2(edges[2 * e], edges[2 * e + 1]);
  }
}

int build_edge_buckets(cc_solver* s, hipStream_t st) {
  s->ecol_off.assign(1, 0);
  s->n_ecolors = 0;
  s->n_erows = 0;
  s->erows_dirty = false;
  if (s->ne == 0 || !(s->p.flags & CC_EDGE_LEN)) return CC_OK;
  CC_HIP(hipMemsetAsync(s->col_cnt, 0, sizeof(int32_t) * kMaxColors, st));
  k_ebucket_count<<<nblk(s->ne), kThreads, 0, st>>>(s->eseg, s->seg_dev, s->einv, s->ecol, s->ne,
                                                     s->col_cnt);
  std::vector<int32_t> cnt(kMaxColors);
  CC_HIP(hipMemcpyAsync(cnt.data(), s->col_cnt, sizeof(int32_t) * kMaxColors,
                        hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  int32_t ncol = 0;
  for (int c = 0; c < kMaxColors; ++c)
    if (cnt[c]) ncol = c + 1;
  std::vector<int32_t>& off = s->ecol_off;
  off.assign(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) off[c + 1] = off[c] + cnt[c];
  if (ncol == 0) return CC_OK;
  CC_HIP(hipMemcpyAsync(s->col_cnt, off.data(), sizeof(int32_t) * ncol, hipMemcpyHostToDevice, st));
  k_ebucket_scatter<<<nblk(s->ne), kThreads, 0, st>>>(s->eseg, s->seg_dev, s->einv, s->ecol,
                                                       s->ne, s->col_cnt, s->eorder, s->edges,
                                                       s->eij);
  CC_HIP(hipMemcpyAsync(s->ecoff_dev, off.data(), sizeof(int32_t) * (ncol + 1),
                        hipMemcpyHostToDevice, st));
  CC_HIP(hipGetLastError());
  s->n_ecolors = ncol;
  s->n_erows = off[ncol];
  return CC_OK;
}

// ------------------------------------------------------------- Gauss-Seidel

// A contact row of A linearised at x^(l) (Sec. 4): x does not change during the
// backward step, so the row is built once per step and every sweep reads it.
// Slots 2 and 3 of a vertex-vertex row carry vertex id -1.
struct RowRec {
  int4 v;
  double c0, inv_a;
  double w[4];
  V3 J[4];
};
static_assert(sizeof(RowRec) == 8 * kRowWords, "contact row record size");

struct GsArgs {
  const int32_t* order;
  const unsigned long long* lslot;  // small contact sets: the rows' block-local slots
  const int32_t* lvert;             // and each slot's vertex (from the colouring)
  const int2* eij;  // edge rows: the vertices of each bucket position (with order)
  int32_t cnt;
  const RowRec* rows;
  const unsigned long long* err;  // bit 0 set: the colouring failed, the step does nothing
  const uint64_t* Akeys;
  const int4* Averts;
  const int32_t* edges;
  const double* eg;
  const double* einv;
  const double* x;
  double* y;
  float* dy;  // mixed precision: y - x
  const double* w;
  double* lam;
  float* lamf;  // mixed precision multipliers
  double delta, kappa2, sigma;
};

constexpr int kGsTailRows = 2048;   // colours smaller than this run in one block
constexpr int kGsTailThreads = 1024;

struct F3 {
  float x, y, z;
};
__device__ __forceinline__ F3 ldf3(const float* p, int32_t i) {
  const float* q = p + 3 * (int64_t)i;
  return F3{q[0], q[1], q[2]};
}
__device__ __forceinline__ void stf3(float* p, int32_t i, F3 v) {
  float* q = p + 3 * (int64_t)i;
  q[0] = v.x;
  q[1] = v.y;
  q[2] = v.z;
}

// The contact rows of A at x^(l) (contact_row), and the step's multipliers set to
// zero (contact rows and, with edge-length rows in use, the ne edge rows).
__global__ void __launch_bounds__(kThreads) k_contact_rows(const uint64_t* __restrict__ Akeys,
                                                           const int4* __restrict__ Averts,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ w,
                                                           double delta, double kappa2,
                                                           int64_t nA, RowRec* __restrict__ rows,
                                                           double* __restrict__ lamA,
                                                           double* __restrict__ lamE,
                                                           int64_t ne) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ne) lamE[i] = 0.0;
  if (i >= nA) return;
  lamA[i] = 0.0;
  const uint64_t key = Akeys[i];
  const int4 q = Averts[i];
  const int32_t v[4] = {q.x, q.y, q.z, q.w};
  V3 xs[4];
  double ws[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    xs[k] = ld3(x, v[k]);
    ws[k] = w[v[k]];
  }
  Row R{};
  const bool vv = key_is_vv(key);
  if (vv) contact_row_vv(xs, ws, delta, R);
  else contact_row(key_is_ee(key), xs, ws, delta, kappa2, R);
  RowRec o;
  o.v = vv ? make_int4(q.x, q.y, -1, -1) : q;
  o.c0 = R.c0;
  o.inv_a = R.inv_a;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o.w[k] = ws[k];
    o.J[k] = R.J[k];
  }
  rows[i] = o;
}

// One projected Gauss-Seidel update of a contact row (Sec. 4.3) built by
// k_contact_rows: residual w = c0 + sum J.(y - x), lambda <- max(0, lambda - w/A),
// y_v += w_v dl J_v at its free vertices. Mixed precision: the row (FP64) is
// rounded and the projection runs in FP32 on y - x. The caller holds the row's record
// R (an active one: 1/A > 0); the positions at x^(l) are loaded with y.
template <bool kMixed>
__device__ __forceinline__ void gs_contact_apply(const GsArgs& a, int32_t r, const RowRec& R) {
  const int32_t v[4] = {R.v.x, R.v.y, R.v.z, R.v.w};
  const int nk = v[2] < 0 ? 2 : 4;  // a vertex-vertex row has two vertices
  if (kMixed) {
    F3 J[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) J[k] = F3{(float)R.J[k].x, (float)R.J[k].y, (float)R.J[k].z};
    float wr = (float)R.c0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k >= nk) continue;
      F3 d = ldf3(a.dy, v[k]);
      wr = wr + (J[k].x * d.x + J[k].y * d.y + J[k].z * d.z);
    }
    const float lam = a.lamf[r];
    float ln = lam - wr * (float)R.inv_a;
    if (ln < 0.f) ln = 0.f;
    const float dl = ln - lam;
    a.lamf[r] = ln;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k >= nk || !(R.w[k] > 0.0)) continue;
      const float co = (float)R.w[k] * dl;
      F3 d = ldf3(a.dy, v[k]);
      stf3(a.dy, v[k], F3{d.x + co * J[k].x, d.y + co * J[k].y, d.z + co * J[k].z});
    }
    return;
  }
  double wr = R.c0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k >= nk) continue;
    V3 dy = vsub(ld3(a.y, v[k]), ld3(a.x, v[k]));
    wr = wr + vdot(R.J[k], dy);
  }
  double lam = a.lam[r];
  double ln = lam - wr * R.inv_a;
  if (ln < 0.0) ln = 0.0;
  double dl = ln - lam;
  a.lam[r] = ln;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k >= nk || !(R.w[k] > 0.0)) continue;
    double co = R.w[k] * dl;
    V3 yv = ld3(a.y, v[k]);
    yv = V3{yv.x + co * R.J[k].x, yv.y + co * R.J[k].y, yv.z + co * R.J[k].z};
    st3(a.y, v[k], yv);
  }
}

template <bool kMixed>
__device__ __forceinline__ void gs_contact_update(const GsArgs& a, int32_t r) {
  const RowRec R = a.rows[r];
  if (!(R.inv_a > 0.0)) return;
  gs_contact_apply<kMixed>(a, r, R);
}

// Edge-length row (Sec. 4.2), same projected update. Mixed precision: the part
// sigma - g.(x_i - x_j) in FP64, the rest on y - x in FP32.
// Edge row at bucket position t (its edge and two vertices read side by side, so the
// vertices' loads do not wait on the edge's).
template <bool kMixed>
__device__ __forceinline__ void gs_edge_update(const GsArgs& a, int32_t t) {
  const int32_t e = a.order[t];
  const int2 ij = a.eij[t];
  const int32_t i = ij.x, j = ij.y;
  V3 g = ld3(a.eg, e);
  const double wi = a.w[i], wj = a.w[j];
  if (kMixed) {
    const double base = a.sigma - vdot(g, vsub(ld3(a.x, i), ld3(a.x, j)));
    const F3 gf{(float)g.x, (float)g.y, (float)g.z};
    F3 di = ldf3(a.dy, i), dj = ldf3(a.dy, j);
    const float wr = (float)base - (gf.x * (di.x - dj.x) + gf.y * (di.y - dj.y) + gf.z * (di.z - dj.z));
    const float lam = a.lamf[e];
    float ln = lam - wr * (float)a.einv[e];
    if (ln < 0.f) ln = 0.f;
    const float dl = ln - lam;
    a.lamf[e] = ln;
    if (wi > 0.0) {
      const float co = (float)wi * dl;
      stf3(a.dy, i, F3{di.x - co * gf.x, di.y - co * gf.y, di.z - co * gf.z});
    }
    if (wj > 0.0) {
      const float co = (float)wj * dl;
      stf3(a.dy, j, F3{dj.x + co * gf.x, dj.y + co * gf.y, dj.z + co * gf.z});
    }
    return;
  }
  V3 yi = ld3(a.y, i), yj = ld3(a.y, j);
  V3 dy = vsub(yi, yj);
  double wr = a.sigma - vdot(g, dy);
  double lam = a.lam[e];
  double ln = lam - wr * a.einv[e];
  if (ln < 0.0) ln = 0.0;
  double dl = ln - lam;
  a.lam[e] = ln;
  if (wi > 0.0) {
    double co = wi * dl;
    st3(a.y, i, V3{yi.x - co * g.x, yi.y - co * g.y, yi.z - co * g.z});
  }
  if (wj > 0.0) {
    double co = wj * dl;
    st3(a.y, j, V3{yj.x + co * g.x, yj.y + co * g.y, yj.z + co * g.z});
  }
}

__device__ __forceinline__ bool gs_off(const GsArgs& a) { return a.err && (*a.err & 1ull); }

// One colour, one row per thread (rows of a colour share no free vertex).
template <bool kMixed>
__global__ void __launch_bounds__(kThreads) k_gs_contact(GsArgs a) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < a.cnt && !gs_off(a)) gs_contact_update<kMixed>(a, a.order[t]);
}

template <bool kMixed>
__global__ void __launch_bounds__(kThreads) k_gs_edge(GsArgs a) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < a.cnt && !gs_off(a)) gs_edge_update<kMixed>(a, t);
}

// A run of small colours [c0, c1) in one block, colour after colour with a block
// barrier between them; `off` holds the colour bucket offsets on the device. With
// c1p set, the run ends at the colour count the device holds there (the colouring
// of the same step wrote it).
template <bool kMixed>
__global__ void __launch_bounds__(kGsTailThreads) k_gs_tail(GsArgs a, const int32_t* off,
                                                            int32_t c0, int32_t c1, int is_edge,
                                                            const unsigned long long* c1p) {
  if (gs_off(a)) return;
  if (c1p) c1 = (int32_t)*c1p;
  for (int32_t c = c0; c < c1; ++c) {
    const int32_t b = off[c], e = off[c + 1];
    for (int32_t t = b + threadIdx.x; t < e; t += kGsTailThreads) {
      if (is_edge) gs_edge_update<kMixed>(a, t);
      else gs_contact_update<kMixed>(a, a.order[t]);
    }
    __syncthreads();
  }
}

// Every colour of a small contact set (at most kSmallRows rows, colours and buckets on
// the device) in one block. Position p of the colour order is updated by thread
// p mod kGsTailThreads; the thread of position p < kGsTailThreads holds that row's
// record from the start, so a colour costs it only the loads of x and y at the row's
// vertices and the stores. The bucket offsets are staged in LDS.
// When every row has its own thread and the colouring gave the rows' free vertices
// block-local slots (at most kLocCap1), y at those vertices stays in LDS for the
// whole sweep (read once, written back once) and each thread holds x at its row's
// vertices (y - x at its fixed ones, which the sweep does not move): a colour is
// then LDS traffic only. The arithmetic is the same, in the same order.
template <bool kMixed>
__global__ void __launch_bounds__(kGsTailThreads) k_gs_contact_small(
    GsArgs a, const int32_t* __restrict__ off, const unsigned long long* ncolp,
    const unsigned long long* nAp, const unsigned long long* nlocp) {
  __shared__ int32_t s_off[kMaxColors + 1];
  __shared__ double s_y[kLocCap1][3];
  if (gs_off(a)) return;
  const int32_t ncol = (int32_t)*ncolp;
  const int32_t nA = (int32_t)*nAp;
  for (int32_t c = threadIdx.x; c <= ncol; c += kGsTailThreads) s_off[c] = off[c];
  const int32_t p0 = threadIdx.x;
  int32_t r0 = -1;
  RowRec R0;
  if (p0 < nA) {
    r0 = a.order[p0];
    R0 = a.rows[r0];
    if (!(R0.inv_a > 0.0)) r0 = -1;  // an inactive row does nothing
  }
  const unsigned long long nloc = a.lslot ? *nlocp : ~0ull;
  if (!kMixed && nA <= kGsTailThreads && nloc <= (unsigned long long)kLocCap1) {
    const int32_t U = (int32_t)nloc;
    for (int32_t l = threadIdx.x; l < U; l += kGsTailThreads) {
      const V3 yv = ld3(a.y, a.lvert[l]);
      s_y[l][0] = yv.x;
      s_y[l][1] = yv.y;
      s_y[l][2] = yv.z;
    }
    int32_t sl[4] = {-1, -1, -1, -1};
    V3 xc[4];  // x at a free vertex, y - x at a fixed one
    double lam = 0.0;
    const int32_t v[4] = {R0.v.x, R0.v.y, R0.v.z, R0.v.w};
    const int nk = v[2] < 0 ? 2 : 4;
    if (r0 >= 0) {
      const unsigned long long ps = a.lslot[r0];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t q = (int32_t)((ps >> (16 * k)) & 0xffffull);
        sl[k] = q == 0xffff ? -1 : q;
        xc[k] = V3{0.0, 0.0, 0.0};
        if (k >= nk) continue;
        const V3 xk = ld3(a.x, v[k]);
        xc[k] = sl[k] >= 0 ? xk : vsub(ld3(a.y, v[k]), xk);
      }
      lam = a.lam[r0];
    }
    __syncthreads();
    for (int32_t c = 0; c < ncol; ++c) {
      if (r0 >= 0 && p0 >= s_off[c] && p0 < s_off[c + 1]) {
        double wr = R0.c0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (k >= nk) continue;
          const V3 dy = sl[k] >= 0 ? vsub(V3{s_y[sl[k]][0], s_y[sl[k]][1], s_y[sl[k]][2]}, xc[k])
                                   : xc[k];
          wr = wr + vdot(R0.J[k], dy);
        }
        double ln = lam - wr * R0.inv_a;
        if (ln < 0.0) ln = 0.0;
        const double dl = ln - lam;
        lam = ln;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (k >= nk || sl[k] < 0 || !(R0.w[k] > 0.0)) continue;
          const double co = R0.w[k] * dl;
          double* yv = s_y[sl[k]];
          yv[0] = yv[0] + co * R0.J[k].x;
          yv[1] = yv[1] + co * R0.J[k].y;
          yv[2] = yv[2] + co * R0.J[k].z;
        }
      }
      __syncthreads();
    }
    if (r0 >= 0) a.lam[r0] = lam;
    for (int32_t l = threadIdx.x; l < U; l += kGsTailThreads)
      st3(a.y, a.lvert[l], V3{s_y[l][0], s_y[l][1], s_y[l][2]});
    return;
  }
  __syncthreads();
  for (int32_t c = 0; c < ncol; ++c) {
    const int32_t b = s_off[c], e = s_off[c + 1];
    if (r0 >= 0 && p0 >= b && p0 < e) gs_contact_apply<kMixed>(a, r0, R0);
    for (int32_t p = p0 + kGsTailThreads; p < e; p += kGsTailThreads)
      if (p >= b) gs_contact_update<kMixed>(a, a.order[p]);
    __syncthreads();
  }
}

template <bool kMixed>
static void gs_colours(const GsArgs& base, const int32_t* order, const int2* eij,
                       const std::vector<int32_t>& off, const int32_t* off_dev, int32_t ncol,
                       bool edge, hipStream_t st) {
  GsArgs a = base;
  int32_t c = 0;
  while (c < ncol) {
    int32_t cnt = off[c + 1] - off[c];
    if (cnt >= kGsTailRows) {
      a.order = order + off[c];
      a.eij = eij ? eij + off[c] : nullptr;
      a.cnt = cnt;
      if (edge) k_gs_edge<kMixed><<<nblk(cnt), kThreads, 0, st>>>(a);
      else k_gs_contact<kMixed><<<nblk(cnt), kThreads, 0, st>>>(a);
      ++c;
      continue;
    }
    int32_t c1 = c;
    while (c1 < ncol && off[c1 + 1] - off[c1] < kGsTailRows) ++c1;
    a.order = order;
    a.eij = eij;
    a.cnt = 0;
    k_gs_tail<kMixed><<<1, kGsTailThreads, 0, st>>>(a, off_dev, c, c1, edge ? 1 : 0, nullptr);
    c = c1;
  }
}

template <bool kMixed>
static void gs_sweeps(cc_solver* s, GsArgs a, hipStream_t st) {
  for (int sw = 0; sw < s->p.gs_sweeps; ++sw) {
    a.lam = s->lamA;
    a.lamf = (float*)s->lamA;
    if (s->col_small) {
      // colours of a small contact set are known on the device only: one block runs them all
      a.order = s->Aorder;
      a.cnt = 0;
      if (s->nA > 0)
        k_gs_contact_small<kMixed><<<1, kGsTailThreads, 0, st>>>(a, s->coff_dev, &s->dc->ncol,
                                                                  &s->dc->n_act, &s->dc->nloc);
    } else {
      gs_colours<kMixed>(a, s->Aorder, nullptr, s->col_off, s->coff_dev, s->n_colors, false, st);
    }
    a.lam = s->lamE;
    a.lamf = (float*)s->lamE;
    gs_colours<kMixed>(a, s->eorder, s->eij, s->ecol_off, s->ecoff_dev, s->n_ecolors, true, st);
  }
}

int launch_gs(cc_solver* s, hipStream_t st) {
  GsArgs a;
  a.lslot = s->Aslot;
  a.lvert = s->lvert;
  a.eij = s->eij;
  a.Akeys = s->Akeys;
  a.Averts = s->Averts;
  a.rows = reinterpret_cast<const RowRec*>(s->Arow);
  a.err = s->col_small ? &s->dc->err : nullptr;
  a.edges = s->edges;
  a.eg = s->eg;
  a.einv = s->einv;
  a.x = s->x;
  a.y = s->y;
  a.dy = s->dy;
  a.w = s->w;
  a.delta = s->p.delta;
  a.kappa2 = s->kappa2;
  a.sigma = s->p.sigma;
  // contact rows at x, and the multipliers at zero (0.0 and 0.0f are both all-zero bits)
  const int64_t ne = s->n_erows > 0 ? s->ne : 0;
  const int64_t nz = s->nA > ne ? s->nA : ne;
  if (nz > 0)
    k_contact_rows<<<nblk(nz), kThreads, 0, st>>>(s->Akeys, s->Averts, s->x, s->w, s->p.delta,
                                                  s->kappa2, s->nA,
                                                  reinterpret_cast<RowRec*>(s->Arow), s->lamA,
                                                  s->lamE, ne);
  if (s->p.flags & CC_MIXED) gs_sweeps<true>(s, a, st);
  else gs_sweeps<false>(s, a, st);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- projected Jacobi

// Sec. 4.3.2 variant of the backward step: every row is evaluated from the same
// y, its per-vertex updates w_v dl J_v are rounded to a multiple of 2^-56 m and
// added (integer atomics: exact, so the sum does not depend on the order), then
// y += omega * sum. An update of 64 m or more flags an error (bit 4).
constexpr double kJacScale = 72057594037927936.0;  // 2^56

__device__ __forceinline__ void jac_add(long long* acc, double v, Counters* c) {
  if (!(fabs(v) < 64.0)) {
    atomicOr(&c->err, 16ull);
    return;
  }
  atomicAdd((unsigned long long*)acc, (unsigned long long)__double2ll_rn(v * kJacScale));
}

__global__ void __launch_bounds__(kThreads) k_jacobi_contact(GsArgs a, int64_t nA,
                                                             long long* __restrict__ acc,
                                                             Counters* c) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nA) return;
  const uint64_t key = a.Akeys[r];
  const int4 q = a.Averts[r];
  const int32_t v[4] = {q.x, q.y, q.z, q.w};
  V3 xs[4];
  double ws[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    xs[k] = ld3(a.x, v[k]);
    ws[k] = a.w[v[k]];
  }
  Row R;
  const bool vv = key_is_vv(key);
  const int nk = vv ? 2 : 4;
  if (vv) contact_row_vv(xs, ws, a.delta, R);
  else contact_row(key_is_ee(key), xs, ws, a.delta, a.kappa2, R);
  if (!(R.inv_a > 0.0)) return;
  double wr = R.c0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < nk) wr = wr + vdot(R.J[k], vsub(ld3(a.y, v[k]), xs[k]));
  const double lam = a.lam[r];
  double ln = lam - wr * R.inv_a;
  if (ln < 0.0) ln = 0.0;
  const double dl = ln - lam;
  a.lam[r] = ln;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k >= nk || !(ws[k] > 0.0)) continue;
    const double co = ws[k] * dl;
    long long* p = acc + 3 * (int64_t)v[k];
    jac_add(p, co * R.J[k].x, c);
    jac_add(p + 1, co * R.J[k].y, c);
    jac_add(p + 2, co * R.J[k].z, c);
  }
}

__global__ void __launch_bounds__(kThreads) k_jacobi_edge(GsArgs a, int32_t ne,
                                                          const int32_t* __restrict__ eseg,
                                                          const SegDev* __restrict__ seg,
                                                          long long* __restrict__ acc,
                                                          Counters* c) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne || !erow_live(e, eseg, seg, a.einv)) return;
  const int32_t i = a.edges[2 * e], j = a.edges[2 * e + 1];
  const V3 g = ld3(a.eg, e);
  const double wr = a.sigma - vdot(g, vsub(ld3(a.y, i), ld3(a.y, j)));
  const double lam = a.lam[e];
  double ln = lam - wr * a.einv[e];
  if (ln < 0.0) ln = 0.0;
  const double dl = ln - lam;
  a.lam[e] = ln;
  const double wi = a.w[i], wj = a.w[j];
  if (wi > 0.0) {
    const double co = wi * dl;
    long long* p = acc + 3 * (int64_t)i;
    jac_add(p, -(co * g.x), c);
    jac_add(p + 1, -(co * g.y), c);
    jac_add(p + 2, -(co * g.z), c);
  }
  if (wj > 0.0) {
    const double co = wj * dl;
    long long* p = acc + 3 * (int64_t)j;
    jac_add(p, co * g.x, c);
    jac_add(p + 1, co * g.y, c);
    jac_add(p + 2, co * g.z, c);
  }
}

// y += omega * sum (vertices of iterating segments), and the sums back to zero.
__global__ void __launch_bounds__(kThreads) k_jacobi_apply(double* __restrict__ y,
                                                           long long* __restrict__ acc,
                                                           int32_t n, double omega,
                                                           const int32_t* __restrict__ vseg,
                                                           const SegDev* __restrict__ seg) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t sg = vseg[v];
  if (sg < 0 || !(seg[sg].flags & kSegActive)) return;
#pragma unroll
  for (int m = 0; m < 3; ++m) {  // also for a zero sum (y + 0.0, as the definition reads)
    const int64_t k = 3 * (int64_t)v + m;
    y[k] = y[k] + omega * ((double)acc[k] * (1.0 / kJacScale));
    acc[k] = 0;
  }
}

int launch_jacobi(cc_solver* s, hipStream_t st) {
  GsArgs a;
  a.lslot = nullptr;
  a.lvert = nullptr;
  a.rows = nullptr;
  a.err = nullptr;
  a.Akeys = s->Akeys;
  a.Averts = s->Averts;
  a.edges = s->edges;
  a.eg = s->eg;
  a.einv = s->einv;
  a.x = s->x;
  a.y = s->y;
  a.dy = s->dy;
  a.w = s->w;
  a.delta = s->p.delta;
  a.kappa2 = s->kappa2;
  a.sigma = s->p.sigma;
  if (s->nA > 0) CC_HIP(hipMemsetAsync(s->lamA, 0, sizeof(double) * s->nA, st));
  if (s->ne > 0) CC_HIP(hipMemsetAsync(s->lamE, 0, sizeof(double) * s->ne, st));
  const bool edges = s->ne > 0 && (s->p.flags & CC_EDGE_LEN);
  for (int sw = 0; sw < s->p.gs_sweeps; ++sw) {
    a.lam = s->lamA;
    if (s->nA > 0) k_jacobi_contact<<<nblk(s->nA), kThreads, 0, st>>>(a, s->nA, s->jacc, s->dc);
    a.lam = s->lamE;
    if (edges)
      k_jacobi_edge<<<nblk(s->ne), kThreads, 0, st>>>(a, s->ne, s->eseg, s->seg_dev, s->jacc, s->dc);
    if (s->n > 0)
      k_jacobi_apply<<<nblk(s->n), kThreads, 0, st>>>(s->y, s->jacc, s->n, s->p.omega, s->vseg,
                                                      s->seg_dev);
  }
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- forward step

// Eq. eq:forward2: alpha_i = min(0.5 gamma D_i / |y_i - x_i|, 1) (1 when y_i = x_i),
// x_i <- y_i if alpha_i = 1 else x_i + alpha_i (y_i - x_i), r_i <- r_i (1 - alpha_i);
// per segment max ||x_i^(l+1) - x_i^(l)|| and ||r||_inf for Alg. 1 (bit patterns of
// non-negative doubles, block-combined in a small LDS table, then atomicMax).
// The lemma of Sec. 5 for the rounded move: unless `unguarded`, a vertex advances
// only when 2 |x_new - x| < D_i - eta (eta covers the rounding of the distances);
// otherwise it stays (alpha = 0). With gamma < 1 this differs from the equation
// only below D_i = eta / (1 - gamma) and on rounding.
// x^(l), r^(l) (and in mixed precision y - x^(l)) are kept for the certificate,
// which may send a vertex back; its return flag is cleared here.
// Vertices of segments that do not iterate are left alone.
// Mixed precision: y = x + dy with dy in FP32; the step itself is FP64 and the
// new dy is y - x^(l+1) rounded (0 when the vertex reached y).
template <bool kMixed>
__global__ void __launch_bounds__(kThreads) k_forward(double* __restrict__ x,
                                                      double* __restrict__ xold,
                                                      const double* __restrict__ y,
                                                      float* __restrict__ dyf,
                                                      float* __restrict__ dyold,
                                                      const unsigned long long* __restrict__ Di,
                                                      double* __restrict__ r,
                                                      double* __restrict__ rold,
                                                      int32_t* __restrict__ back,
                                                      double* __restrict__ alph,
                                                      unsigned long long* __restrict__ scale,
                                                      double* __restrict__ move2, int32_t n,
                                                      double hg, int guard, int ccd_step,
                                                      const int32_t* __restrict__ vseg,
                                                      SegDev* seg,
                                                      const unsigned long long* err,
                                                      uint8_t* __restrict__ mvd) {
  if (err && (*err & 1ull)) return;  // the colouring of this step failed: x stays
  __shared__ int32_t gkey[kSegSlots];
  __shared__ unsigned long long gmax[kSegSlots][2];
  if (threadIdx.x < kSegSlots) {
    gkey[threadIdx.x] = -1;
    gmax[threadIdx.x][0] = gmax[threadIdx.x][1] = 0ull;
  }
  __syncthreads();
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t sg = i < n ? vseg[i] : -1;
  if (sg >= 0 && (seg[sg].flags & kSegActive)) {
    V3 xi = ld3(x, i), yi, dx;
    if (kMixed) {
      float* d = dyf + 3 * (int64_t)i;
      dx = V3{(double)d[0], (double)d[1], (double)d[2]};
      yi = V3{xi.x + dx.x, xi.y + dx.y, xi.z + dx.z};
      float* o = dyold + 3 * (int64_t)i;
      o[0] = d[0];
      o[1] = d[1];
      o[2] = d[2];
    } else {
      yi = ld3(y, i);
      dx = vsub(yi, xi);
    }
    // the CCD-based scheme bounds every vertex by D^(l) alone; its contacts along P'
    // are found by the certificate's passes
    const double di = ccd_step ? seg[sg].D : __longlong_as_double((long long)Di[i]);
    double n2 = vdot(dx, dx);
    double alpha = 1.0;
    if (n2 > 0.0) {
      double a = (hg * di) / sqrt(n2);
      if (a < 1.0) alpha = a;
    }
    V3 xn = (alpha == 1.0) ? yi : vaxpy(xi, alpha, dx);
    V3 mv = vsub(xn, xi);
    double m2 = vdot(mv, mv);
    const double sb = di - kEta;
    if (guard && !(sb > 0.0 && 4.0 * m2 < sb * sb)) {
      xn = xi;
      m2 = 0.0;
      alpha = 0.0;
    }
    if (kMixed) {
      float* d = dyf + 3 * (int64_t)i;
      d[0] = (float)(yi.x - xn.x);
      d[1] = (float)(yi.y - xn.y);
      d[2] = (float)(yi.z - xn.z);
    }
    move2[i] = m2;
    mvd[i] = (xn.x != xi.x || xn.y != xi.y || xn.z != xi.z) ? 1 : 0;
    back[i] = 0;
    if (ccd_step) {
      alph[i] = alpha;
      scale[i] = kOneBits;
    }
    st3(xold, i, xi);
    st3(x, i, xn);
    const double r0 = r[i];
    rold[i] = r0;
    double ri = r0 * (1.0 - alpha);
    r[i] = ri;
    const unsigned long long mb = (unsigned long long)__double_as_longlong(sqrt(m2));
    const unsigned long long rb = (unsigned long long)__double_as_longlong(ri);
    const int slot = seg_slot(gkey, sg);
    if (slot >= 0) {
      if (mb) atomicMax(&gmax[slot][0], mb);
      if (rb) atomicMax(&gmax[slot][1], rb);
    } else {
      if (mb) atomicMax(&seg[sg].mmax_bits, mb);
      if (rb) atomicMax(&seg[sg].rinf_bits, rb);
    }
  }
  __syncthreads();
  if (threadIdx.x < kSegSlots && gkey[threadIdx.x] >= 0) {
    SegDev& sd = seg[gkey[threadIdx.x]];
    if (gmax[threadIdx.x][0]) atomicMax(&sd.mmax_bits, gmax[threadIdx.x][0]);
    if (gmax[threadIdx.x][1]) atomicMax(&sd.rinf_bits, gmax[threadIdx.x][1]);
  }
}

int launch_forward(cc_solver* s, hipStream_t st) {
  const double hg = 0.5 * s->p.gamma;
  const int guard = (s->p.flags & CC_UNGUARDED) ? 0 : 1;
  const int ccd_step = (s->p.flags & CC_CCD_STEP) ? 1 : 0;
  const unsigned long long* err = s->col_small ? &s->dc->err : nullptr;
  if (s->n > 0 && (s->p.flags & CC_MIXED))
    k_forward<true><<<nblk(s->n), kThreads, 0, st>>>(s->x, s->xold, s->y, s->dy, s->dyold, s->Di,
                                                      s->r, s->rold, s->back, s->alph, s->scale,
                                                      s->move2, s->n, hg, guard, ccd_step,
                                                      s->vseg, s->seg_dev, err, s->mvd);
  else if (s->n > 0)
    k_forward<false><<<nblk(s->n), kThreads, 0, st>>>(s->x, s->xold, s->y, s->dy, s->dyold,
                                                       s->Di, s->r, s->rold, s->back, s->alph,
                                                       s->scale, s->move2, s->n, hg, guard,
                                                       ccd_step, s->vseg, s->seg_dev, err,
                                                       s->mvd);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// ------------------------------------------------------------- certificate

// Lemma of Sec. 5: the linear piece x^(l) -> x^(l+1) stays free for pair p when
// no vertex of p moved half its distance, i.e. 4 max_v |dx_v|^2 < d_p^2. A pair the
// bound does not certify (or every pair with CC_CCD_ALL) is counted for its scene and
// queued (its index in P, bit 63 set when the bound certified it) for the continuous
// test of the piece, which runs in a kernel of its own: the test is rare and large,
// and kept out of this pass it does not lower its occupancy.
__global__ void __launch_bounds__(kThreads) k_cert(const uint64_t* __restrict__ P,
                                                   const double* __restrict__ dP, int64_t nP,
                                                   Topo T, const double* __restrict__ move2,
                                                   const int32_t* __restrict__ vseg, SegDev* seg,
                                                   unsigned long long* __restrict__ queue,
                                                   unsigned long long* nqueue, int all) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool fail = false, bound_ok = false;
  int32_t v[4] = {0, 0, 0, 0};
  if (i < nP) {
    pair_verts(T, P[i], v);
    double mv = move2[v[0]];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      double m = move2[v[k]];
      if (m > mv) mv = m;
    }
    bound_ok = 4.0 * mv < dP[i];
    fail = all || !bound_ok;
  }
  const unsigned long long pos = wave_append(fail, nqueue);
  if (fail) {
    queue[pos] = (unsigned long long)i | (bound_ok ? kQueueCertified : 0ull);
    atomicAdd(&seg[vseg[v[0]]].fail, 1ull);
  }
}

// The continuous test of every queued pair (a grid-stride loop over the queue,
// whose length is read on the device); contacts are counted for the pair's scene.
// A pair the motion bound did not certify and the test does not clear sends its
// vertices back to x^(l): each vertex is marked once (2 = marked in this pass) and
// counted as returned for its scene.
__global__ void __launch_bounds__(kThreads) k_cert_ccd(const uint64_t* __restrict__ P, Topo T,
                                                       const double* __restrict__ xold,
                                                       const double* __restrict__ x, double eta,
                                                       const int32_t* __restrict__ vseg,
                                                       SegDev* seg,
                                                       const unsigned long long* __restrict__ queue,
                                                       const unsigned long long* nqueue,
                                                       int32_t* __restrict__ back,
                                                       unsigned long long* __restrict__ scale,
                                                       double gamma) {
  const int64_t n = (int64_t)*nqueue;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long e = queue[j];
    const uint64_t key = P[e & ~kQueueCertified];
    int32_t v[4];
    pair_verts(T, key, v);
    V3 q[4], dq[4];
    for (int k = 0; k < 4; ++k) {
      q[k] = ld3(xold, v[k]);
      dq[k] = vsub(ld3(x, v[k]), q[k]);
    }
    const double th = key_is_vv(key) ? ccd_hit_vv(q[0], q[1], dq[0], dq[1], eta * eta)
                                     : ccd_hit(q, dq, key_is_ee(key), eta);
    if (!(th >= 0.0)) continue;
    SegDev& sd = seg[vseg[v[0]]];
    atomicAdd(&sd.hits, 1ull);
    if (e & kQueueCertified) continue;
    if (scale) {
      // CCD-based step: the pair's vertices take at most gamma t* of their step
      const unsigned long long fb = (unsigned long long)__double_as_longlong(gamma * th);
      for (int k = 0; k < 4; ++k) atomicMin(&scale[v[k]], fb);
      atomicAdd(&sd.nstep, 1ull);
    } else {
      for (int k = 0; k < 4; ++k)
        if (atomicCAS(&back[v[k]], 0, 2) == 0) atomicAdd(&sd.nback, 1ull);
    }
  }
}

// CCD-based step: every moving vertex whose factor fell below 1 in the last pass takes
// alpha <- alpha * factor, x <- x^(l) + alpha (y - x^(l)) (y itself when alpha is 1),
// r <- r^(l) (1 - alpha), and is counted for its scene.
__global__ void __launch_bounds__(kThreads) k_step_apply(double* __restrict__ x,
                                                         const double* __restrict__ xold,
                                                         const double* __restrict__ y,
                                                         double* __restrict__ r,
                                                         const double* __restrict__ rold,
                                                         double* __restrict__ alph,
                                                         unsigned long long* __restrict__ scale,
                                                         double* __restrict__ move2,
                                                         uint8_t* __restrict__ mvd, int32_t n,
                                                         const int32_t* __restrict__ vseg,
                                                         SegDev* seg) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !(scale[i] < kOneBits)) return;
  const double a = alph[i] * __longlong_as_double((long long)scale[i]);
  scale[i] = kOneBits;
  if (move2[i] == 0.0) return;  // no step to scale
  alph[i] = a;
  const V3 x0 = ld3(xold, i), yi = ld3(y, i);
  const V3 xn = vaxpy(x0, a, vsub(yi, x0));
  const V3 mv = vsub(xn, x0);
  move2[i] = vdot(mv, mv);
  mvd[i] = (xn.x != x0.x || xn.y != x0.y || xn.z != x0.z) ? 1 : 0;
  st3(x, i, xn);
  r[i] = rold[i] * (1.0 - a);
  atomicAdd(&seg[vseg[i]].nscaled, 1ull);
}

// Vertices marked in the last pass go back to x^(l): x, r (and y - x) as before
// the forward step, no move; then ||r||_inf of every iterating segment again.
__global__ void __launch_bounds__(kThreads) k_send_back(double* __restrict__ x,
                                                        const double* __restrict__ xold,
                                                        double* __restrict__ r,
                                                        const double* __restrict__ rold,
                                                        float* __restrict__ dyf,
                                                        const float* __restrict__ dyold,
                                                        double* __restrict__ move2,
                                                        uint8_t* __restrict__ mvd,
                                                        int32_t* __restrict__ back, int32_t n) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || back[i] != 2) return;
  back[i] = 1;
  st3(x, i, ld3(xold, i));
  r[i] = rold[i];
  if (dyf) {
    for (int k = 0; k < 3; ++k) dyf[3 * (int64_t)i + k] = dyold[3 * (int64_t)i + k];
  }
  move2[i] = 0.0;
  mvd[i] = 0;
}

__global__ void k_seg_rinf_clear(SegDev* seg, int32_t ns) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns && (seg[i].flags & kSegActive)) seg[i].rinf_bits = 0ull;
}

__global__ void __launch_bounds__(kThreads) k_seg_rinf(const double* __restrict__ r, int32_t n,
                                                       const int32_t* __restrict__ vseg,
                                                       SegDev* seg) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t sg = i < n ? vseg[i] : -1;
  if (sg < 0 || !(seg[sg].flags & kSegActive)) return;
  const unsigned long long rb = (unsigned long long)__double_as_longlong(r[i]);
  if (rb) atomicMax(&seg[sg].rinf_bits, rb);
}

// One pass of the certificate over the current P'. The pair buffer P2 is free
// between the pair passes and holds the queue (at most |P'| entries).
int launch_cert(cc_solver* s, bool scaling, hipStream_t st) {
  if (s->nP > 0) {
    unsigned long long* queue = (unsigned long long*)s->P2;
    // dc->ncert starts at zero with the iteration's counters (k_di_init) and is
    // cleared by launch_send_back before a further pass
    k_cert<<<nblk(s->nP), kThreads, 0, st>>>(s->P, s->dP, s->nP, Topo{s->tris, s->edges},
                                              s->move2, s->vseg, s->seg_dev, queue, &s->dc->ncert,
                                              (s->p.flags & CC_CCD_ALL) ? 1 : 0);
    const unsigned nb = std::min<unsigned>(nblk(s->nP), 1024u);
    k_cert_ccd<<<nb, kThreads, 0, st>>>(s->P, Topo{s->tris, s->edges}, s->xold, s->x, kEta,
                                         s->vseg, s->seg_dev, queue, &s->dc->ncert, s->back,
                                         scaling ? s->scale : nullptr, s->p.gamma);
  }
  CC_HIP(hipGetLastError());
  return CC_OK;
}

// Send the marked vertices back (or, scaling, scale their steps), recompute
// ||r||_inf, clear the queue length.
int launch_send_back(cc_solver* s, int32_t ns, bool scaling, hipStream_t st) {
  if (s->n > 0) {
    const bool mixed = (s->p.flags & CC_MIXED) != 0;
    if (scaling)
      k_step_apply<<<nblk(s->n), kThreads, 0, st>>>(s->x, s->xold, s->y, s->r, s->rold, s->alph,
                                                     s->scale, s->move2, s->mvd, s->n, s->vseg,
                                                     s->seg_dev);
    else
      k_send_back<<<nblk(s->n), kThreads, 0, st>>>(s->x, s->xold, s->r, s->rold,
                                                    mixed ? s->dy : nullptr, s->dyold, s->move2,
                                                    s->mvd, s->back, s->n);
    k_seg_rinf_clear<<<(ns + 255) / 256, 256, 0, st>>>(s->seg_dev, ns);
    k_seg_rinf<<<nblk(s->n), kThreads, 0, st>>>(s->r, s->n, s->vseg, s->seg_dev);
  }
  k_fill_u64<<<1, 64, 0, st>>>(&s->dc->ncert, 1, 0ull);
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

__global__ void k_y_of_dy(const double* __restrict__ x, const float* __restrict__ dy,
                          double* __restrict__ y, int32_t n) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) y[3 * (int64_t)i + k] = x[3 * (int64_t)i + k] + (double)dy[3 * (int64_t)i + k];
}

__global__ void k_dy_of_y(const double* __restrict__ x, const double* __restrict__ y,
                          float* __restrict__ dy, int32_t n) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) dy[3 * (int64_t)i + k] = (float)(y[3 * (int64_t)i + k] - x[3 * (int64_t)i + k]);
}

int launch_y_of_dy(cc_solver* s, double* y, int32_t n, hipStream_t st) {
  if (n > 0) k_y_of_dy<<<nblk(n), kThreads, 0, st>>>(s->x, s->dy, y, n);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

int launch_dy_of_y(cc_solver* s, const double* y, int32_t n, hipStream_t st) {
  if (n > 0) k_dy_of_y<<<nblk(n), kThreads, 0, st>>>(s->x, y, s->dy, n);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

int launch_fp_col(cc_solver* s, hipStream_t st) {
  if (s->nA > 0) k_fp_col<<<nblk(s->nA), kThreads, 0, st>>>(s->Akeys, s->Acol, s->nA, s->dc);
  CC_HIP(hipGetLastError());
  return CC_OK;
}

}  // namespace cc
