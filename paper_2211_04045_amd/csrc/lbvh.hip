// Proximity search (Sec. 3.1) as a linear BVH broad phase on gfx950.
//
// Two trees, one over triangles (vertex-triangle queries) and one over edges
// (edge-edge queries). Leaf boxes are the primitive's box at x inflated by
// D_max/2 and rounded outward to float, so box overlap of a query (also
// inflated by D_max/2) is implied by distance < D_max; the exact FP64 filter
// d^2 < D_max^2 then decides membership. Build: 30-bit Morton codes of box
// centres (one key space for both trees, tree id in bit 30), a stable LSD
// radix sort written here (8-bit digits, wave ballot ranking), the hierarchy
// of Karras (2012) and a bottom-up refit with arrival counters. Traversal: one
// thread per query, stack in registers, candidates appended through a
// per-lane LDS buffer flushed with one atomic per wave.
#include "geom.hpp"
#include "internal.hpp"

namespace cc {

constexpr int kTile = 4096;      // radix sort tile per block
constexpr int kRsThreads = 256;
constexpr int kStack = 64;
constexpr int kBuf = 8;          // per-lane pending pairs in the traversal
constexpr int kTravThreads = 256;

__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
__device__ __forceinline__ float lo_out(double v) {
  return nextafterf(__double2float_rd(v), -__builtin_inff());
}
__device__ __forceinline__ float hi_out(double v) {
  return nextafterf(__double2float_ru(v), __builtin_inff());
}

// Leaf boxes for all F triangles then E edges; box-centre bounds (ordered ints).
__global__ void k_boxes(const double* __restrict__ x, const int32_t* __restrict__ tris,
                        const int32_t* __restrict__ edges, int32_t nt, int32_t ne, double infl,
                        float4* __restrict__ blo, float4* __restrict__ bhi,
                        uint32_t* __restrict__ bounds) {
  __shared__ uint32_t sb[6];
  if (threadIdx.x < 6) sb[threadIdx.x] = (threadIdx.x < 3) ? 0xffffffffu : 0u;
  __syncthreads();
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nt + ne) {
    V3 lo, hi;
    if (g < nt) {
      V3 a = ld3(x, tris[3 * g]), b = ld3(x, tris[3 * g + 1]), c = ld3(x, tris[3 * g + 2]);
      lo = V3{fmin(fmin(a.x, b.x), c.x), fmin(fmin(a.y, b.y), c.y), fmin(fmin(a.z, b.z), c.z)};
      hi = V3{fmax(fmax(a.x, b.x), c.x), fmax(fmax(a.y, b.y), c.y), fmax(fmax(a.z, b.z), c.z)};
    } else {
      int32_t e = g - nt;
      V3 a = ld3(x, edges[2 * e]), b = ld3(x, edges[2 * e + 1]);
      lo = V3{fmin(a.x, b.x), fmin(a.y, b.y), fmin(a.z, b.z)};
      hi = V3{fmax(a.x, b.x), fmax(a.y, b.y), fmax(a.z, b.z)};
    }
    float4 l = make_float4(lo_out(lo.x - infl), lo_out(lo.y - infl), lo_out(lo.z - infl), 0.f);
    float4 h = make_float4(hi_out(hi.x + infl), hi_out(hi.y + infl), hi_out(hi.z + infl), 0.f);
    blo[g] = l;
    bhi[g] = h;
    float cx = 0.5f * (l.x + h.x), cy = 0.5f * (l.y + h.y), cz = 0.5f * (l.z + h.z);
    atomicMin(&sb[0], f2ord(cx));
    atomicMin(&sb[1], f2ord(cy));
    atomicMin(&sb[2], f2ord(cz));
    atomicMax(&sb[3], f2ord(cx));
    atomicMax(&sb[4], f2ord(cy));
    atomicMax(&sb[5], f2ord(cz));
  }
  __syncthreads();
  if (threadIdx.x < 3) atomicMin(&bounds[threadIdx.x], sb[threadIdx.x]);
  else if (threadIdx.x < 6) atomicMax(&bounds[threadIdx.x], sb[threadIdx.x]);
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__global__ void k_morton(const float4* __restrict__ blo, const float4* __restrict__ bhi,
                         int32_t nt, int32_t ne, const uint32_t* __restrict__ bounds,
                         uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nt + ne) return;
  float4 l = blo[g], h = bhi[g];
  float c[3] = {0.5f * (l.x + h.x), 0.5f * (l.y + h.y), 0.5f * (l.z + h.z)};
  uint32_t q[3];
  for (int k = 0; k < 3; ++k) {
    float lo = ord2f(bounds[k]), hi = ord2f(bounds[3 + k]);
    float span = hi - lo;
    float t = span > 0.f ? (c[k] - lo) / span : 0.f;
    float v = t * 1024.f;
    v = v < 0.f ? 0.f : (v > 1023.f ? 1023.f : v);
    q[k] = (uint32_t)v;
  }
  uint32_t code = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
  keys[g] = code | ((g < nt ? 0u : 1u) << 30);
  vals[g] = (uint32_t)g;
}

// ---------------------------------------------------------------- radix sort

__global__ void k_rs_hist(const uint32_t* __restrict__ keys, int32_t n, int shift,
                          uint32_t* __restrict__ hist, int32_t nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int32_t base = blockIdx.x * kTile;
  for (int i = 0; i < kTile / kRsThreads; ++i) {
    int32_t idx = base + i * kRsThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of m counts in place, one block of 1024 threads.
__global__ void k_scan_1block(uint32_t* __restrict__ a, int64_t m) {
  __shared__ uint32_t part[1024];
  int64_t per = (m + 1023) / 1024;
  int64_t b = threadIdx.x * per, e = b + per < m ? b + per : m;
  uint32_t sum = 0;
  for (int64_t i = b; i < e; ++i) sum += a[i];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
  for (int64_t i = b; i < e; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

__global__ void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                             uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int32_t n,
                             int shift, const uint32_t* __restrict__ hist, int32_t nb) {
  constexpr int W = kRsThreads / 64;
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[W][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  run[threadIdx.x] = hist[threadIdx.x * nb + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  int32_t base = blockIdx.x * kTile;
  for (int c = 0; c < kTile / kRsThreads; ++c) {
    for (int w = 0; w < W; ++w) wc[w][threadIdx.x] = 0;
    __syncthreads();
    int32_t idx = base + c * kRsThreads + threadIdx.x;
    bool valid = idx < n;
    uint32_t key = valid ? kin[idx] : 0u;
    uint32_t val = valid ? vin[idx] : 0u;
    uint32_t dig = (key >> shift) & 0xffu;
    uint64_t m = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot((dig >> b) & 1u);
      m &= ((dig >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rank = (uint32_t)__popcll(m & lt);
    bool leader = valid && ((m >> lane) >> 1) == 0ull;
    if (leader) wc[wave][dig] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[dig] + rank;
      for (int w = 0; w < wave; ++w) pos += wc[w][dig];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < W; ++w) add += wc[w][threadIdx.x];
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- hierarchy

struct TreeView {
  int32_t n;
  const uint32_t* keys;  // sorted codes of this tree
  int32_t* child;
  int32_t* parent;
};

__device__ __forceinline__ int delta_fn(const uint32_t* __restrict__ k, int32_t n, int32_t i,
                                        int32_t j) {
  if (j < 0 || j >= n) return -1;
  uint32_t a = k[i] & 0x3fffffffu, b = k[j] & 0x3fffffffu;
  if (a != b) return __clz(a ^ b);
  return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

__device__ void karras_node(const TreeView& T, int32_t i) {
  const uint32_t* k = T.keys;
  const int32_t n = T.n;
  int d = delta_fn(k, n, i, i + 1) - delta_fn(k, n, i, i - 1) > 0 ? 1 : -1;
  int dmin = delta_fn(k, n, i, i - d);
  int32_t lmax = 2;
  while (delta_fn(k, n, i, i + lmax * d) > dmin) lmax *= 2;
  int32_t l = 0;
  for (int32_t t = lmax / 2; t >= 1; t /= 2)
    if (delta_fn(k, n, i, i + (l + t) * d) > dmin) l += t;
  int32_t j = i + l * d;
  int dnode = delta_fn(k, n, i, j);
  int32_t s = 0;
  int32_t div = 2;
  int32_t t;
  do {
    t = (l + div - 1) / div;
    if (delta_fn(k, n, i, i + (s + t) * d) > dnode) s += t;
    div *= 2;
  } while (t > 1);
  int32_t gam = i + s * d + (d < 0 ? -1 : 0);
  int32_t lo = i < j ? i : j, hi = i < j ? j : i;
  int32_t left = (lo == gam) ? (int32_t)(0x80000000u | (uint32_t)gam) : gam;
  int32_t right = (hi == gam + 1) ? (int32_t)(0x80000000u | (uint32_t)(gam + 1)) : gam + 1;
  T.child[2 * i] = left;
  T.child[2 * i + 1] = right;
  // parent: internal nodes at [0, n-1), leaves at [n-1, 2n-1)
  T.parent[(left < 0) ? (n - 1 + (left & 0x7fffffff)) : left] = i;
  T.parent[(right < 0) ? (n - 1 + (right & 0x7fffffff)) : right] = i;
}

__global__ void k_karras(TreeView ta, TreeView tb) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t na = ta.n > 1 ? ta.n - 1 : 0, nb = tb.n > 1 ? tb.n - 1 : 0;
  if (g < na) {
    karras_node(ta, g);
    if (g == 0) ta.parent[0] = -1;
  } else if (g < na + nb) {
    karras_node(tb, g - na);
    if (g == na) tb.parent[0] = -1;
  }
}

// Sorted leaf boxes and primitive ids of both trees.
__global__ void k_leaves(const uint32_t* __restrict__ sval, const float4* __restrict__ blo,
                         const float4* __restrict__ bhi, int32_t nt, int32_t ne,
                         float4* __restrict__ tlo, float4* __restrict__ thi,
                         int32_t* __restrict__ tprim, float4* __restrict__ elo,
                         float4* __restrict__ ehi, int32_t* __restrict__ eprim) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nt + ne) return;
  uint32_t p = sval[g];
  if (g < nt) {
    tlo[g] = blo[p];
    thi[g] = bhi[p];
    tprim[g] = (int32_t)p;
  } else {
    int32_t i = g - nt;
    elo[i] = blo[p];
    ehi[i] = bhi[p];
    eprim[i] = (int32_t)p - nt;
  }
}

__device__ __forceinline__ float aload(const float* p) {
  return __uint_as_float(
      __hip_atomic_load((const uint32_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

struct RefitView {
  int32_t n;
  const int32_t* child;
  const int32_t* parent;
  const float4* leaf_lo;
  const float4* leaf_hi;
  float4* node_lo;
  float4* node_hi;
  uint32_t* flag;
};

__device__ void refit_leaf(const RefitView& T, int32_t leaf) {
  int32_t node = T.parent[T.n - 1 + leaf];
  while (node >= 0) {
    __threadfence();
    uint32_t old = atomicAdd(&T.flag[node], 1u);
    if (old == 0) return;
    __threadfence();
    float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
    float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
    for (int c = 0; c < 2; ++c) {
      int32_t ch = T.child[2 * node + c];
      const float* L;
      const float* H;
      if (ch < 0) {
        L = (const float*)&T.leaf_lo[ch & 0x7fffffff];
        H = (const float*)&T.leaf_hi[ch & 0x7fffffff];
      } else {
        L = (const float*)&T.node_lo[ch];
        H = (const float*)&T.node_hi[ch];
      }
      for (int k = 0; k < 3; ++k) {
        lo[k] = fminf(lo[k], aload(L + k));
        hi[k] = fmaxf(hi[k], aload(H + k));
      }
    }
    T.node_lo[node] = make_float4(lo[0], lo[1], lo[2], 0.f);
    T.node_hi[node] = make_float4(hi[0], hi[1], hi[2], 0.f);
    node = T.parent[node];
  }
}

__global__ void k_refit(RefitView ta, RefitView tb) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ta.n) {
    if (ta.n > 1) refit_leaf(ta, g);
  } else if (g < ta.n + tb.n) {
    if (tb.n > 1) refit_leaf(tb, g - ta.n);
  }
}

// ---------------------------------------------------------------- traversal

struct TravTree {
  int32_t n;
  const int32_t* child;
  const float4* node_lo;
  const float4* node_hi;
  const float4* leaf_lo;
  const float4* leaf_hi;
  const int32_t* leaf_prim;
};

struct TravArgs {
  TravTree tt, te;
  const double* x;
  const int32_t* tris;
  const int32_t* edges;
  const uint8_t* stat;
  int32_t n, ne;
  double infl, dmax2;
  uint64_t* out;
  double* dout;
  int64_t cap;
  Counters* cnt;
};

__device__ __forceinline__ bool overlap(float4 al, float4 ah, float4 bl, float4 bh) {
  return al.x <= bh.x && bl.x <= ah.x && al.y <= bh.y && bl.y <= ah.y && al.z <= bh.z &&
         bl.z <= ah.z;
}

__global__ void __launch_bounds__(kTravThreads) k_traverse(TravArgs A) {
  __shared__ uint64_t skey[kTravThreads * kBuf];
  __shared__ double sd2[kTravThreads * kBuf];
  const int lane = threadIdx.x & 63;
  int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const bool is_vt = q < A.n;
  const bool active = q < A.n + A.ne;
  const TravTree& T = is_vt ? A.tt : A.te;
  float4 qlo = make_float4(0.f, 0.f, 0.f, 0.f), qhi = qlo;
  int32_t qv[2] = {0, 0};
  V3 qx0{0, 0, 0}, qx1{0, 0, 0};
  int32_t stack[kStack];
  int sp = 0;
  if (active && T.n > 0) {
    if (is_vt) {
      qv[0] = q;
      qx0 = ld3(A.x, q);
      qlo = make_float4(lo_out(qx0.x - A.infl), lo_out(qx0.y - A.infl), lo_out(qx0.z - A.infl), 0.f);
      qhi = make_float4(hi_out(qx0.x + A.infl), hi_out(qx0.y + A.infl), hi_out(qx0.z + A.infl), 0.f);
    } else {
      int32_t e = q - A.n;
      qv[0] = A.edges[2 * e];
      qv[1] = A.edges[2 * e + 1];
      qx0 = ld3(A.x, qv[0]);
      qx1 = ld3(A.x, qv[1]);
      qlo = make_float4(lo_out(fmin(qx0.x, qx1.x) - A.infl), lo_out(fmin(qx0.y, qx1.y) - A.infl),
                        lo_out(fmin(qx0.z, qx1.z) - A.infl), 0.f);
      qhi = make_float4(hi_out(fmax(qx0.x, qx1.x) + A.infl), hi_out(fmax(qx0.y, qx1.y) + A.infl),
                        hi_out(fmax(qx0.z, qx1.z) + A.infl), 0.f);
    }
    stack[sp++] = T.n == 1 ? (int32_t)0x80000000u : 0;
  }
  const int32_t qid = is_vt ? q : q - A.n;
  int cnt = 0;
  while (__any(sp > 0)) {
    if (sp > 0) {
      int32_t node = stack[--sp];
      if (node < 0) {
        int32_t li = node & 0x7fffffff;
        if (overlap(qlo, qhi, T.leaf_lo[li], T.leaf_hi[li])) {
          int32_t prim = T.leaf_prim[li];
          int32_t v1, v2, v3 = -1;
          bool ok;
          if (is_vt) {
            v1 = A.tris[3 * prim];
            v2 = A.tris[3 * prim + 1];
            v3 = A.tris[3 * prim + 2];
            ok = qv[0] != v1 && qv[0] != v2 && qv[0] != v3;
            ok = ok && !(A.stat[qv[0]] && A.stat[v1] && A.stat[v2] && A.stat[v3]);
          } else {
            v1 = A.edges[2 * prim];
            v2 = A.edges[2 * prim + 1];
            ok = prim > qid && qv[0] != v1 && qv[0] != v2 && qv[1] != v1 && qv[1] != v2;
            ok = ok && !(A.stat[qv[0]] && A.stat[qv[1]] && A.stat[v1] && A.stat[v2]);
          }
          if (ok) {
            double d2;
            uint64_t key;
            if (is_vt) {
              double bw[3];
              d2 = pt_tri_d2(qx0, ld3(A.x, v1), ld3(A.x, v2), ld3(A.x, v3), bw);
              key = ((uint64_t)(uint32_t)qid << 32) | (uint32_t)prim;
            } else {
              double s, t;
              d2 = seg_seg_d2(qx0, qx1, ld3(A.x, v1), ld3(A.x, v2), s, t);
              key = KEY_EE | ((uint64_t)(uint32_t)qid << 32) | (uint32_t)prim;
            }
            if (d2 < A.dmax2) {
              skey[threadIdx.x * kBuf + cnt] = key;
              sd2[threadIdx.x * kBuf + cnt] = d2;
              ++cnt;
            }
          }
        }
      } else if (overlap(qlo, qhi, T.node_lo[node], T.node_hi[node])) {
        if (sp + 2 <= kStack) {
          stack[sp++] = T.child[2 * node];
          stack[sp++] = T.child[2 * node + 1];
        } else {
          atomicOr(&A.cnt->err, 2ull);
          sp = 0;
        }
      }
    }
    if (__any(cnt == kBuf)) {
      // wave-wide flush of every lane's pending pairs
      int incl = cnt;
      for (int o = 1; o < 64; o <<= 1) {
        int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
      }
      int total = __shfl(incl, 63);
      unsigned long long base = 0;
      if (lane == 0 && total > 0) base = atomicAdd(&A.cnt->n_out, (unsigned long long)total);
      base = __shfl(base, 0);
      int64_t pos = (int64_t)base + (incl - cnt);
      for (int i = 0; i < cnt; ++i) {
        if (pos + i < A.cap) {
          A.out[pos + i] = skey[threadIdx.x * kBuf + i];
          if (A.dout) A.dout[pos + i] = sd2[threadIdx.x * kBuf + i];
        }
      }
      cnt = 0;
    }
  }
  {
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    int total = __shfl(incl, 63);
    unsigned long long base = 0;
    if (lane == 0 && total > 0) base = atomicAdd(&A.cnt->n_out, (unsigned long long)total);
    base = __shfl(base, 0);
    int64_t pos = (int64_t)base + (incl - cnt);
    for (int i = 0; i < cnt; ++i) {
      if (pos + i < A.cap) {
        A.out[pos + i] = skey[threadIdx.x * kBuf + i];
        if (A.dout) A.dout[pos + i] = sd2[threadIdx.x * kBuf + i];
      }
    }
  }
}

// ---------------------------------------------------------------- host side

template <class T>
static int dalloc(T** p, int64_t n) {
  if (n <= 0) n = 1;
  if (hipMalloc((void**)p, (size_t)n * sizeof(T)) != hipSuccess) return CC_ENOMEM;
  return CC_OK;
}

static int bvh_alloc_one(Bvh& b, int32_t n) {
  b.n = n;
  int32_t ni = n > 1 ? n - 1 : 1;
  CC_TRY(dalloc(&b.leaf_lo, n));
  CC_TRY(dalloc(&b.leaf_hi, n));
  CC_TRY(dalloc(&b.leaf_prim, n));
  CC_TRY(dalloc(&b.child, 2 * ni));
  CC_TRY(dalloc(&b.parent, ni + n));
  CC_TRY(dalloc(&b.node_lo, ni));
  CC_TRY(dalloc(&b.node_hi, ni));
  CC_TRY(dalloc(&b.flag, ni));
  return CC_OK;
}

static void bvh_free_one(Bvh& b) {
  hipFree(b.leaf_lo); hipFree(b.leaf_hi); hipFree(b.leaf_prim); hipFree(b.child);
  hipFree(b.parent); hipFree(b.node_lo); hipFree(b.node_hi); hipFree(b.flag);
  b = Bvh{};
}

int bvh_alloc(cc_solver* s) {
  int64_t m = (int64_t)s->nt + s->ne;
  CC_TRY(bvh_alloc_one(s->tree_t, s->nt));
  CC_TRY(bvh_alloc_one(s->tree_e, s->ne));
  CC_TRY(dalloc(&s->sk0, m));
  CC_TRY(dalloc(&s->sk1, m));
  CC_TRY(dalloc(&s->sv0, m));
  CC_TRY(dalloc(&s->sv1, m));
  CC_TRY(dalloc(&s->ubox_lo, m));
  CC_TRY(dalloc(&s->ubox_hi, m));
  int64_t nb = (m + kTile - 1) / kTile;
  s->rs_hist_cap = 256 * (nb > 0 ? nb : 1);
  CC_TRY(dalloc(&s->rs_hist, s->rs_hist_cap));
  CC_TRY(dalloc(&s->bounds, 6));
  return CC_OK;
}

void bvh_free(cc_solver* s) {
  bvh_free_one(s->tree_t);
  bvh_free_one(s->tree_e);
  hipFree(s->sk0); hipFree(s->sk1); hipFree(s->sv0); hipFree(s->sv1);
  hipFree(s->ubox_lo); hipFree(s->ubox_hi); hipFree(s->rs_hist); hipFree(s->bounds);
  s->sk0 = s->sk1 = s->sv0 = s->sv1 = nullptr;
}

static inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int lbvh_search(cc_solver* s, const double* x, double dmax, uint64_t* out, double* dout,
                int64_t cap, int64_t* nfound, hipStream_t st) {
  const int32_t nt = s->nt, ne = s->ne;
  const int64_t m = (int64_t)nt + ne;
  const double infl = 0.5 * dmax;
  CC_HIP(hipMemsetAsync(&s->dc->n_out, 0, sizeof(unsigned long long), st));
  CC_HIP(hipMemsetAsync(&s->dc->err, 0, sizeof(unsigned long long), st));
  if (m > 0) {
    // bounds init: min = 0xffffffff, max = 0
    uint32_t init[6] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u};
    CC_HIP(hipMemcpyAsync(s->bounds, init, sizeof init, hipMemcpyHostToDevice, st));
    k_boxes<<<blocks(m, 256), 256, 0, st>>>(x, s->tris, s->edges, nt, ne, infl, s->ubox_lo,
                                           s->ubox_hi, s->bounds);
    k_morton<<<blocks(m, 256), 256, 0, st>>>(s->ubox_lo, s->ubox_hi, nt, ne, s->bounds, s->sk0,
                                             s->sv0);
    const int32_t nb = (int32_t)((m + kTile - 1) / kTile);
    uint32_t *ki = s->sk0, *vi = s->sv0, *ko = s->sk1, *vo = s->sv1;
    for (int shift = 0; shift < 32; shift += 8) {
      k_rs_hist<<<nb, kRsThreads, 0, st>>>(ki, (int32_t)m, shift, s->rs_hist, nb);
      k_scan_1block<<<1, 1024, 0, st>>>(s->rs_hist, (int64_t)256 * nb);
      k_rs_scatter<<<nb, kRsThreads, 0, st>>>(ki, vi, ko, vo, (int32_t)m, shift, s->rs_hist, nb);
      uint32_t* t;
      t = ki; ki = ko; ko = t;
      t = vi; vi = vo; vo = t;
    }
    // after 4 passes the sorted data is back in sk0/sv0
    k_leaves<<<blocks(m, 256), 256, 0, st>>>(ki == s->sk0 ? s->sv0 : s->sv1, s->ubox_lo,
                                             s->ubox_hi, nt, ne, s->tree_t.leaf_lo,
                                             s->tree_t.leaf_hi, s->tree_t.leaf_prim,
                                             s->tree_e.leaf_lo, s->tree_e.leaf_hi,
                                             s->tree_e.leaf_prim);
    const uint32_t* sorted = ki;
    TreeView ta{nt, sorted, s->tree_t.child, s->tree_t.parent};
    TreeView tb{ne, sorted + nt, s->tree_e.child, s->tree_e.parent};
    int64_t ninternal = (nt > 1 ? nt - 1 : 0) + (ne > 1 ? ne - 1 : 0);
    if (ninternal > 0) {
      k_karras<<<blocks(ninternal, 256), 256, 0, st>>>(ta, tb);
      if (nt > 1) CC_HIP(hipMemsetAsync(s->tree_t.flag, 0, sizeof(uint32_t) * (nt - 1), st));
      if (ne > 1) CC_HIP(hipMemsetAsync(s->tree_e.flag, 0, sizeof(uint32_t) * (ne - 1), st));
      RefitView ra{nt, s->tree_t.child, s->tree_t.parent, s->tree_t.leaf_lo, s->tree_t.leaf_hi,
                   s->tree_t.node_lo, s->tree_t.node_hi, s->tree_t.flag};
      RefitView rb{ne, s->tree_e.child, s->tree_e.parent, s->tree_e.leaf_lo, s->tree_e.leaf_hi,
                   s->tree_e.node_lo, s->tree_e.node_hi, s->tree_e.flag};
      k_refit<<<blocks(m, 256), 256, 0, st>>>(ra, rb);
    }
    TravArgs A;
    A.tt = TravTree{nt, s->tree_t.child, s->tree_t.node_lo, s->tree_t.node_hi,
                    s->tree_t.leaf_lo, s->tree_t.leaf_hi, s->tree_t.leaf_prim};
    A.te = TravTree{ne, s->tree_e.child, s->tree_e.node_lo, s->tree_e.node_hi,
                    s->tree_e.leaf_lo, s->tree_e.leaf_hi, s->tree_e.leaf_prim};
    A.x = x;
    A.tris = s->tris;
    A.edges = s->edges;
    A.stat = s->stat;
    A.n = s->n;
    A.ne = ne;
    A.infl = infl;
    A.dmax2 = dmax * dmax;
    A.out = out;
    A.dout = dout;
    A.cap = cap;
    A.cnt = s->dc;
    int64_t nq = (int64_t)s->n + ne;
    if (nq > 0) {
      timer_begin(s, CC_K_SEARCH, st);
      k_traverse<<<blocks(nq, kTravThreads), kTravThreads, 0, st>>>(A);
      timer_end(s, st);
    }
  }
  CC_HIP(hipGetLastError());
  CC_HIP(hipMemcpyAsync(s->hc, s->dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (s->hc->err & 2ull) return CC_EOVERFLOW;
  *nfound = (int64_t)s->hc->n_out;
  // algorithmic bytes of the traversal: queries, leaf and node boxes, output keys
  s->st.kernel_bytes[CC_K_SEARCH] += 24.0 * s->n + 8.0 * ne + 36.0 * (double)m +
                                     32.0 * (double)m + 8.0 * (double)*nfound;
  return CC_OK;
}

}  // namespace cc
