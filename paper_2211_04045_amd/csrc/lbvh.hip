// Proximity search (Sec. 3.1) as a linear BVH broad phase on gfx950.
//
// Two trees, one over triangles (vertex-triangle queries) and one over edges
// (edge-edge queries). Leaf boxes are the primitive's box at x inflated by
// D_max/2 and rounded outward to float, so box overlap of a query (also
// inflated by D_max/2) is implied by distance < D_max; the exact FP64 filter
// d^2 < D_max^2 then decides membership. Build: 30-bit Morton codes of box
// centres and vertices (one key space, group id in bits 31..30), a stable LSD
// radix sort written here (8-bit digits, wave ballot ranking) and the
// hierarchy of Karras (2012). Node boxes need no bottom-up walk: an internal
// node covers a contiguous range of sorted leaves, so its box is a range union,
// taken from LDS inside a 256-leaf block or assembled from per-block prefix,
// suffix and a sparse table of block boxes across blocks (no atomics, no
// device-scope fences).
// Each node record (64 B) holds both child boxes and child ids, leaves inline;
// a 4-wide copy (128 B) collapses each node with its children for traversal.
// Traversal: one thread per query, children tested at the parent, candidates
// appended through a per-lane LDS buffer flushed with one atomic per wave.
// Edge queries run in sorted order and visit only leaves after their own, so
// each edge-edge pair is found once.
// Several scenes (segments) are searched together: a segment's rank sits above
// the Morton code in the sort key, so each segment's leaves form one subtree
// of the radix tree, and its queries start at that subtree's root.
#include <algorithm>
#include <cmath>
#include <cstddef>

#include "geom.hpp"
#include "internal.hpp"

namespace cc {

constexpr int kTile = 4096;      // radix sort tile per block
constexpr int kRsThreads = 256;
constexpr int kStack = 100;     // 4-wide DFS: 3 pending entries per level, <= 32 levels
constexpr int kBlk = 256;        // leaves per refit block
constexpr int32_t kLeaf = (int32_t)0x80000000;
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

// Rank r of the selected segment holding compact index g of one kind
// (0 vertices, 1 triangles, 2 edges, 3 particles): off(r) <= g < off(r + 1).
__device__ __forceinline__ int32_t sel_off(const SelDev& d, int kind) {
  return kind == 0 ? d.voff : (kind == 1 ? d.toff : (kind == 2 ? d.eoff : d.poff));
}
__device__ __forceinline__ int32_t find_sel(const SelDev* __restrict__ sel, int32_t nsel,
                                            int kind, int32_t g) {
  int32_t lo = 0, hi = nsel - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (sel_off(sel[mid], kind) <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Leaf boxes of the selected segments' triangles (compact 0..mt), edges
// (mt..mt+me) and particles (mt+me..mt+me+mp), their primitive ids (particles:
// vertex ids), and per-block bounds of the box centres (order-preserving uint
// encoding), reduced by k_bounds_reduce.
__global__ void k_boxes(const double* __restrict__ x, const int32_t* __restrict__ tris,
                        const int32_t* __restrict__ edges, const int32_t* __restrict__ plist,
                        const SelDev* __restrict__ sel, int32_t nsel, int32_t mt, int32_t me,
                        int32_t mp, double infl, float4* __restrict__ blo,
                        float4* __restrict__ bhi, int32_t* __restrict__ gprim,
                        uint32_t* __restrict__ part) {
  __shared__ uint32_t sb[6];
  if (threadIdx.x < 6) sb[threadIdx.x] = (threadIdx.x < 3) ? 0xffffffffu : 0u;
  __syncthreads();
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < mt + me + mp) {
    V3 lo, hi;
    if (g < mt) {
      const int32_t r = find_sel(sel, nsel, 1, g);
      const int32_t f = sel[r].fb + (g - sel[r].toff);
      gprim[g] = f;
      V3 a = ld3(x, tris[3 * f]), b = ld3(x, tris[3 * f + 1]), c = ld3(x, tris[3 * f + 2]);
      lo = V3{fmin(fmin(a.x, b.x), c.x), fmin(fmin(a.y, b.y), c.y), fmin(fmin(a.z, b.z), c.z)};
      hi = V3{fmax(fmax(a.x, b.x), c.x), fmax(fmax(a.y, b.y), c.y), fmax(fmax(a.z, b.z), c.z)};
    } else if (g < mt + me) {
      const int32_t ge = g - mt;
      const int32_t r = find_sel(sel, nsel, 2, ge);
      const int32_t e = sel[r].eb + (ge - sel[r].eoff);
      gprim[g] = e;
      V3 a = ld3(x, edges[2 * e]), b = ld3(x, edges[2 * e + 1]);
      lo = V3{fmin(a.x, b.x), fmin(a.y, b.y), fmin(a.z, b.z)};
      hi = V3{fmax(a.x, b.x), fmax(a.y, b.y), fmax(a.z, b.z)};
    } else {
      const int32_t gp = g - mt - me;
      const int32_t r = find_sel(sel, nsel, 3, gp);
      const int32_t v = plist[sel[r].vb + (gp - sel[r].poff)];
      gprim[g] = v;
      lo = ld3(x, v);
      hi = lo;
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
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sb[threadIdx.x];
}

__global__ void k_bounds_reduce(const uint32_t* __restrict__ part, int32_t nb,
                                uint32_t* __restrict__ bounds) {
  __shared__ uint32_t sb[6];
  if (threadIdx.x < 6) sb[threadIdx.x] = (threadIdx.x < 3) ? 0xffffffffu : 0u;
  __syncthreads();
  uint32_t v[6] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u};
  for (int32_t b = threadIdx.x; b < nb; b += blockDim.x)
    for (int k = 0; k < 6; ++k) {
      uint32_t u = part[6 * b + k];
      v[k] = k < 3 ? (u < v[k] ? u : v[k]) : (u > v[k] ? u : v[k]);
    }
  for (int k = 0; k < 3; ++k) atomicMin(&sb[k], v[k]);
  for (int k = 3; k < 6; ++k) atomicMax(&sb[k], v[k]);
  __syncthreads();
  if (threadIdx.x < 6) bounds[threadIdx.x] = sb[threadIdx.x];
}

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Sort keys: 30-bit Morton code of the triangle boxes (group 0), edge boxes
// (group 1), particle boxes (group 2) and vertices (group 3, the order of the
// vertex queries), the selected segment's rank in the rb bits above it and the
// group above that.
__global__ void k_morton(const float4* __restrict__ blo, const float4* __restrict__ bhi,
                         const double* __restrict__ x, const SelDev* __restrict__ sel,
                         int32_t nsel, int32_t mt, int32_t me, int32_t mp, int32_t mv, int rb,
                         const uint32_t* __restrict__ bounds, uint64_t* __restrict__ keys,
                         uint32_t* __restrict__ vals) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t m = mt + me + mp;
  if (g >= m + mv) return;
  float c[3];
  uint64_t grp;
  int32_t r;
  if (g < m) {
    float4 l = blo[g], h = bhi[g];
    c[0] = 0.5f * (l.x + h.x);
    c[1] = 0.5f * (l.y + h.y);
    c[2] = 0.5f * (l.z + h.z);
    grp = g < mt ? 0u : (g < mt + me ? 1u : 2u);
    r = g < mt ? find_sel(sel, nsel, 1, g)
               : (g < mt + me ? find_sel(sel, nsel, 2, g - mt) : find_sel(sel, nsel, 3, g - mt - me));
  } else {
    const int32_t gv = g - m;
    r = find_sel(sel, nsel, 0, gv);
    V3 p = ld3(x, sel[r].vb + (gv - sel[r].voff));
    c[0] = (float)p.x;
    c[1] = (float)p.y;
    c[2] = (float)p.z;
    grp = 3u;
  }
  // one scale for the three axes (the largest span): cubic Morton cells, so that a
  // thin scene (a cloth a few layers thick) is split across its extent before its
  // thickness and a node's box stays compact
  float span = 0.f;
  for (int k = 0; k < 3; ++k) span = fmaxf(span, ord2f(bounds[3 + k]) - ord2f(bounds[k]));
  uint32_t q[3];
  for (int k = 0; k < 3; ++k) {
    const float lo = ord2f(bounds[k]);
    float t = span > 0.f ? (c[k] - lo) / span : 0.f;
    float v = t * 1024.f;
    v = v < 0.f ? 0.f : (v > 1023.f ? 1023.f : v);
    q[k] = (uint32_t)v;
  }
  uint32_t code = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
  keys[g] = (grp << (30 + rb)) | ((uint64_t)r << 30) | code;
  vals[g] = (uint32_t)g;
}

// ---------------------------------------------------------------- radix sort

__global__ void k_rs_hist(const uint64_t* __restrict__ keys, int32_t n, int shift,
                          uint32_t* __restrict__ hist, int32_t nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int32_t base = blockIdx.x * kTile;
  for (int i = 0; i < kTile / kRsThreads; ++i) {
    int32_t idx = base + i * kRsThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Per digit (one block each): exclusive scan of the per-block counts of that
// digit in place, and the digit's total.
__global__ void __launch_bounds__(kRsThreads) k_rs_scan_digit(uint32_t* __restrict__ hist,
                                                              int32_t nb,
                                                              uint32_t* __restrict__ total) {
  __shared__ uint32_t wsum[kRsThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t* row = hist + (int64_t)blockIdx.x * nb;
  uint32_t carry = 0;
  for (int32_t b0 = 0; b0 < nb; b0 += kRsThreads) {
    int32_t i = b0 + threadIdx.x;
    uint32_t v = i < nb ? row[i] : 0u;
    uint32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t before = 0, chunk = 0;
    for (int w = 0; w < kRsThreads / 64; ++w) {
      if (w < wv) before += wsum[w];
      chunk += wsum[w];
    }
    if (i < nb) row[i] = carry + before + incl - v;
    carry += chunk;
    __syncthreads();
  }
  if (threadIdx.x == 0) total[blockIdx.x] = carry;
}

__global__ void k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                             uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int32_t n,
                             int shift, const uint32_t* __restrict__ hist, int32_t nb,
                             const uint32_t* __restrict__ total) {
  constexpr int W = kRsThreads / 64;
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[W][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  {
    // digit base = exclusive scan of the digit totals
    uint32_t v = total[threadIdx.x], incl = v;
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (lane == 63) wc[0][wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wc[0][w];
    run[threadIdx.x] = before + incl - v + hist[threadIdx.x * nb + blockIdx.x];
    __syncthreads();
  }
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  int32_t base = blockIdx.x * kTile;
  for (int c = 0; c < kTile / kRsThreads; ++c) {
    for (int w = 0; w < W; ++w) wc[w][threadIdx.x] = 0;
    __syncthreads();
    int32_t idx = base + c * kRsThreads + threadIdx.x;
    bool valid = idx < n;
    uint64_t key = valid ? kin[idx] : 0ull;
    uint32_t val = valid ? vin[idx] : 0u;
    uint32_t dig = (uint32_t)(key >> shift) & 0xffu;
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
  const uint64_t* keys;     // sorted keys of this tree
  uint64_t mask;            // key bits below the group (segment rank and Morton code)
  const int32_t* leaf_prim;
  float4* node;             // 4 float4 per internal node
  int32_t* parent;          // internal nodes [0, n-1), then leaves: (parent << 1) | side
  int2* range;
};

__device__ __forceinline__ int delta_fn(const uint64_t* __restrict__ k, uint64_t mask, int32_t n,
                                        int32_t i, int32_t j) {
  if (j < 0 || j >= n) return -1;
  uint64_t a = k[i] & mask, b = k[j] & mask;
  if (a != b) return __clzll((long long)(a ^ b));
  return 64 + __clz((uint32_t)i ^ (uint32_t)j);
}

// Internal node i of the radix tree over sorted keys (Karras 2012): its leaf
// range, split position and children.
__device__ void karras_node(const TreeView& T, int32_t i) {
  const uint64_t* k = T.keys;
  const uint64_t mk = T.mask;
  const int32_t n = T.n;
  int d = delta_fn(k, mk, n, i, i + 1) - delta_fn(k, mk, n, i, i - 1) > 0 ? 1 : -1;
  int dmin = delta_fn(k, mk, n, i, i - d);
  int32_t lmax = 2;
  while (delta_fn(k, mk, n, i, i + lmax * d) > dmin) lmax *= 2;
  int32_t l = 0;
  for (int32_t t = lmax / 2; t >= 1; t /= 2)
    if (delta_fn(k, mk, n, i, i + (l + t) * d) > dmin) l += t;
  int32_t j = i + l * d;
  int dnode = delta_fn(k, mk, n, i, j);
  int32_t s = 0;
  int32_t div = 2;
  int32_t t;
  do {
    t = (l + div - 1) / div;
    if (delta_fn(k, mk, n, i, i + (s + t) * d) > dnode) s += t;
    div *= 2;
  } while (t > 1);
  int32_t gam = i + s * d + (d < 0 ? -1 : 0);
  int32_t lo = i < j ? i : j, hi = i < j ? j : i;
  int32_t cl, cr;
  if (lo == gam) {
    cl = kLeaf | T.leaf_prim[gam];
    T.parent[n - 1 + gam] = (i << 1) | 0;
  } else {
    cl = gam;
    T.parent[gam] = (i << 1) | 0;
  }
  if (hi == gam + 1) {
    cr = kLeaf | T.leaf_prim[gam + 1];
    T.parent[n - 1 + gam + 1] = (i << 1) | 1;
  } else {
    cr = gam + 1;
    T.parent[gam + 1] = (i << 1) | 1;
  }
  T.node[4 * i + 3] = make_float4(__int_as_float(cl), __int_as_float(cr), __int_as_float(gam),
                                  __int_as_float(hi));
  T.range[i] = make_int2(lo, hi);
  if (i == 0) T.parent[0] = -1;
}

__global__ void k_karras(TreeView ta, TreeView tb) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t na = ta.n > 1 ? ta.n - 1 : 0, nb = tb.n > 1 ? tb.n - 1 : 0;
  if (g < na) karras_node(ta, g);
  else if (g < na + nb) karras_node(tb, g - na);
}

struct LeafOut {
  float4 *lo, *hi;
  int32_t* prim;
  int16_t* rank;
};

// Sorted leaf boxes and primitive ids of the three trees; the vertex queries in
// Morton order with their segment ranks; the segment rank of each edge and
// particle leaf.
__global__ void k_leaves(const uint32_t* __restrict__ sval, const uint64_t* __restrict__ skey,
                         const float4* __restrict__ blo, const float4* __restrict__ bhi,
                         const int32_t* __restrict__ gprim, const SelDev* __restrict__ sel,
                         int32_t mt, int32_t me, int32_t mp, int32_t mv, uint32_t rmask,
                         float4* __restrict__ tlo, float4* __restrict__ thi,
                         int32_t* __restrict__ tprim, float4* __restrict__ elo,
                         float4* __restrict__ ehi, int32_t* __restrict__ eprim,
                         int16_t* __restrict__ erank, LeafOut po, int32_t* __restrict__ vorder,
                         int16_t* __restrict__ vrank) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t m = mt + me + mp;
  if (g >= m + mv) return;
  const uint32_t p = sval[g];
  const int32_t r = (int32_t)((uint32_t)(skey[g] >> 30) & rmask);
  if (g >= m) {
    const int32_t q = g - m, gv = (int32_t)p - m;
    vorder[q] = sel[r].vb + (gv - sel[r].voff);
    vrank[q] = (int16_t)r;
  } else if (g >= mt + me) {
    const int32_t i = g - mt - me;
    po.lo[i] = blo[p];
    po.hi[i] = bhi[p];
    po.prim[i] = gprim[p];
    po.rank[i] = (int16_t)r;
  } else if (g < mt) {
    tlo[g] = blo[p];
    thi[g] = bhi[p];
    tprim[g] = gprim[p];
  } else {
    const int32_t i = g - mt;
    elo[i] = blo[p];
    ehi[i] = bhi[p];
    eprim[i] = gprim[p];
    erank[i] = (int16_t)r;
  }
}

// Root of each selected segment's subtree: its leaves are the sorted positions
// [off(r), off(r+1)); an internal node of a radix tree has one end of its range
// at its own index, so the node covering exactly that range is `lo` or `hi`.
// One leaf: the leaf itself (kLeaf | primitive); none: -1.
__device__ __forceinline__ int32_t seg_root(int32_t lo, int32_t cnt, int32_t n,
                                            const int2* __restrict__ range,
                                            const int32_t* __restrict__ prim) {
  if (cnt <= 0) return -1;
  if (cnt == 1) return kLeaf | prim[lo];
  const int32_t hi = lo + cnt - 1;
  if (lo < n - 1) {
    int2 rg = range[lo];
    if (rg.x == lo && rg.y == hi) return lo;
  }
  return hi;
}

__global__ void k_seg_roots(const SelDev* __restrict__ sel, int32_t nsel, int32_t mt,
                            int32_t me, int32_t mp, const int2* __restrict__ trange,
                            const int32_t* __restrict__ tprim, const int2* __restrict__ erange,
                            const int32_t* __restrict__ eprim, const int2* __restrict__ prange,
                            const int32_t* __restrict__ pprim, int32_t* __restrict__ root_t,
                            int32_t* __restrict__ root_e, int32_t* __restrict__ root_p) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nsel) return;
  root_t[r] = seg_root(sel[r].toff, sel[r + 1].toff - sel[r].toff, mt, trange, tprim);
  root_e[r] = seg_root(sel[r].eoff, sel[r + 1].eoff - sel[r].eoff, me, erange, eprim);
  root_p[r] = seg_root(sel[r].poff, sel[r + 1].poff - sel[r].poff, mp, prange, pprim);
}

struct Box6 {
  float lo[3], hi[3];
};

__device__ __forceinline__ Box6 box_empty() {
  const float inf = __builtin_inff();
  return Box6{{inf, inf, inf}, {-inf, -inf, -inf}};
}
__device__ __forceinline__ Box6 box_union(const Box6& a, const Box6& b) {
  Box6 r;
  for (int k = 0; k < 3; ++k) {
    r.lo[k] = fminf(a.lo[k], b.lo[k]);
    r.hi[k] = fmaxf(a.hi[k], b.hi[k]);
  }
  return r;
}
__device__ __forceinline__ Box6 box_ld(const float4* p) {
  float4 l = p[0], h = p[1];
  return Box6{{l.x, l.y, l.z}, {h.x, h.y, h.z}};
}
__device__ __forceinline__ void box_st(float4* p, const Box6& b) {
  p[0] = make_float4(b.lo[0], b.lo[1], b.lo[2], 0.f);
  p[1] = make_float4(b.hi[0], b.hi[1], b.hi[2], 0.f);
}

// Write a node's box into its parent's record (or the root box).
__device__ __forceinline__ void box_to_parent(float4* __restrict__ node, float4* __restrict__ root,
                                              int32_t par, const Box6& b) {
  if (par < 0) {
    box_st(root, b);
    return;
  }
  float* rec = (float*)(node + 4 * (par >> 1)) + 6 * (par & 1);
  rec[0] = b.lo[0];
  rec[1] = b.lo[1];
  rec[2] = b.lo[2];
  rec[3] = b.hi[0];
  rec[4] = b.hi[1];
  rec[5] = b.hi[2];
}

struct RefitView {
  int32_t n;
  const float4* leaf_lo;
  const float4* leaf_hi;
  const int32_t* parent;
  const int2* range;
  float4* node;
  float4* root;
  float4* pre;  // 2 per leaf
  float4* suf;  // 2 per leaf
  float4* blk;  // 2 per block
  float4* wide;     // the 4-wide records (8 float4 per internal node)
  int wide_direct;  // a refit of built records: boxes go into them directly
};

// A box into one slot of a 4-wide record (the slot's first six floats; its
// child id and last leaf position stay as the build wrote them).
__device__ __forceinline__ void wide_slot_st(float4* wide, int32_t r, int slot, const Box6& b) {
  float* f = (float*)(wide + 8 * (int64_t)r + 2 * slot);
  f[0] = b.lo[0];
  f[1] = b.lo[1];
  f[2] = b.lo[2];
  f[3] = b.hi[0];
  f[4] = b.hi[1];
  f[5] = b.hi[2];
}

// A node's (or leaf's) box to where the traversal reads it: the root box, or the
// binary record of its parent (from which a build makes the 4-wide records); in
// a refit of built 4-wide records, the wide record of its grandparent instead
// (slot 2 x the parent's side + its own side), and for a leaf its parent's wide
// record too (slot 2 x its side: a leaf child stays in place).
__device__ __forceinline__ void put_box(const RefitView& T, int32_t par, bool leaf, const Box6& b) {
  if (par < 0 || !T.wide_direct) {
    box_to_parent(T.node, T.root, par, b);
    return;
  }
  const int32_t p = par >> 1, side = par & 1;
  if (leaf) wide_slot_st(T.wide, p, 2 * side, b);
  const int32_t gp = T.parent[p];
  if (gp >= 0) wide_slot_st(T.wide, gp >> 1, 2 * (gp & 1) + side, b);
}

// Refit, part 1 (one 256-leaf block): leaf boxes into their parents, prefix and
// suffix unions inside the block, the block box, and every internal node whose
// leaf range lies inside the block. Those nodes are formed bottom-up: each leaf
// climbs from its parent, and of a node's two children the second to arrive
// (an arrival count in LDS) forms the node's box from its own and its sibling's
// and climbs on, so a thread does as many steps as its leaf is deep in the
// block's part of the tree. (A Karras node's index lies in its leaf range, so
// a node inside the block has its arrival count at its index minus the block's
// first leaf.)
__device__ void refit_block(const RefitView& T, int32_t b) {
  __shared__ float slo[3][kBlk], shi[3][kBlk];
  __shared__ int arrive[kBlk];
  __shared__ float cbox[kBlk][2][6];
  const int32_t B0 = b * kBlk;
  const int32_t cnt = T.n - B0 < kBlk ? T.n - B0 : kBlk;
  const int tid = threadIdx.x;
  arrive[tid] = 0;
  Box6 mine = box_empty();
  if (tid < cnt) {
    float4 l = T.leaf_lo[B0 + tid], h = T.leaf_hi[B0 + tid];
    mine = Box6{{l.x, l.y, l.z}, {h.x, h.y, h.z}};
    put_box(T, T.parent[T.n - 1 + B0 + tid], true, mine);
  }
  for (int k = 0; k < 3; ++k) {
    slo[k][tid] = mine.lo[k];
    shi[k][tid] = mine.hi[k];
  }
  __syncthreads();
  // inclusive prefix union (Hillis-Steele) in registers via LDS exchange
  Box6 pre = mine;
  for (int off = 1; off < kBlk; off <<= 1) {
    Box6 other = box_empty();
    if (tid >= off)
      for (int k = 0; k < 3; ++k) {
        other.lo[k] = slo[k][tid - off];
        other.hi[k] = shi[k][tid - off];
      }
    __syncthreads();
    pre = box_union(pre, other);
    for (int k = 0; k < 3; ++k) {
      slo[k][tid] = pre.lo[k];
      shi[k][tid] = pre.hi[k];
    }
    __syncthreads();
  }
  if (tid < cnt) box_st(T.pre + 2 * (B0 + tid), pre);
  if (tid == cnt - 1) box_st(T.blk + 2 * b, pre);
  // suffix union
  for (int k = 0; k < 3; ++k) {
    slo[k][tid] = mine.lo[k];
    shi[k][tid] = mine.hi[k];
  }
  __syncthreads();
  Box6 suf = mine;
  for (int off = 1; off < kBlk; off <<= 1) {
    Box6 other = box_empty();
    if (tid + off < kBlk)
      for (int k = 0; k < 3; ++k) {
        other.lo[k] = slo[k][tid + off];
        other.hi[k] = shi[k][tid + off];
      }
    __syncthreads();
    suf = box_union(suf, other);
    for (int k = 0; k < 3; ++k) {
      slo[k][tid] = suf.lo[k];
      shi[k][tid] = suf.hi[k];
    }
    __syncthreads();
  }
  if (tid < cnt) box_st(T.suf + 2 * (B0 + tid), suf);
  if (tid >= cnt) return;
  Box6 u = mine;
  int32_t par = T.parent[T.n - 1 + B0 + tid];
  while (par >= 0) {
    const int32_t p = par >> 1, side = par & 1;
    const int2 r = T.range[p];
    if (r.x < B0 || r.y >= B0 + kBlk) break;  // crosses the block: part 2
    const int slot = p - B0;
    for (int k = 0; k < 3; ++k) {
      cbox[slot][side][k] = u.lo[k];
      cbox[slot][side][3 + k] = u.hi[k];
    }
    __threadfence_block();
    if (atomicAdd(&arrive[slot], 1) == 0) break;  // the sibling forms the node
    __threadfence_block();
    Box6 o;
    for (int k = 0; k < 3; ++k) {
      o.lo[k] = cbox[slot][side ^ 1][k];
      o.hi[k] = cbox[slot][side ^ 1][3 + k];
    }
    u = box_union(u, o);
    par = T.parent[p];
    put_box(T, par, false, u);
  }
}

__global__ void __launch_bounds__(kBlk) k_refit_block(RefitView ta, RefitView tb, int32_t nba) {
  if ((int32_t)blockIdx.x < nba) refit_block(ta, blockIdx.x);
  else refit_block(tb, blockIdx.x - nba);
}

// Sparse table over the block boxes: level k, entry b = union of blocks
// b .. b + 2^k - 1 (level 0 is written by refit_block). One block per tree.
__device__ void blk_sparse(const RefitView& T) {
  const int32_t nb = (T.n + kBlk - 1) / kBlk;
  for (int k = 1; (1 << k) <= nb; ++k) {
    const int32_t half = 1 << (k - 1), cnt = nb - (1 << k) + 1;
    const float4* src = T.blk + (int64_t)2 * nb * (k - 1);
    float4* dst = T.blk + (int64_t)2 * nb * k;
    for (int32_t b = threadIdx.x; b < cnt; b += blockDim.x)
      box_st(dst + 2 * b, box_union(box_ld(src + 2 * b), box_ld(src + 2 * (b + half))));
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024) k_blk_sparse(RefitView ta, RefitView tb) {
  if (blockIdx.x == 0) blk_sparse(ta);
  else blk_sparse(tb);
}

// Refit, part 2: internal nodes whose range crosses blocks: suffix of the first
// block, the whole blocks between (two overlapping sparse-table entries), prefix
// of the last block.
__device__ void refit_top(const RefitView& T, int32_t i) {
  int2 r = T.range[i];
  int32_t b0 = r.x / kBlk, b1 = r.y / kBlk;
  if (b0 == b1) return;
  Box6 u = box_union(box_ld(T.suf + 2 * r.x), box_ld(T.pre + 2 * r.y));
  const int32_t lo = b0 + 1, hi = b1 - 1;
  if (lo <= hi) {
    const int32_t nb = (T.n + kBlk - 1) / kBlk;
    const int k = 31 - __clz((uint32_t)(hi - lo + 1));
    const float4* lev = T.blk + (int64_t)2 * nb * k;
    u = box_union(u, box_union(box_ld(lev + 2 * lo), box_ld(lev + 2 * (hi - (1 << k) + 1))));
  }
  put_box(T, T.parent[i], false, u);
}

__global__ void k_refit_top(RefitView ta, RefitView tb) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t na = ta.n > 1 ? ta.n - 1 : 0, nb = tb.n > 1 ? tb.n - 1 : 0;
  if (g < na) refit_top(ta, g);
  else if (g < na + nb) refit_top(tb, g - na);
}

// ---------------------------------------------------------------- traversal

struct TravTree {
  int32_t n;
  const float4* wide;  // 8 float4 per internal node: four grandchild slots
  const float4* root;
  const int32_t* leaf_prim;
};

// 4-wide records: node i with its children collapsed, so one visit tests up to
// four boxes (the binary node's grandchildren, or a leaf child in place) and a
// traversal takes half as many dependent steps. Each slot is two float4: its
// box, child id and the last leaf position of its range.
__global__ void k_wide(const float4* __restrict__ node, float4* __restrict__ wide, int32_t ni) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  const float* rec = (const float*)(node + 4 * i);
  float box[4][6];
  int32_t id[4], hi[4];
  const float inf = __builtin_inff();
  for (int s = 0; s < 2; ++s) {
    const int32_t c = __float_as_int(rec[12 + s]);
    const int32_t chi = __float_as_int(rec[14 + s]);
    if (c < 0) {
      for (int k = 0; k < 6; ++k) box[2 * s][k] = rec[6 * s + k];
      id[2 * s] = c;
      hi[2 * s] = chi;
      for (int k = 0; k < 3; ++k) {
        box[2 * s + 1][k] = inf;
        box[2 * s + 1][3 + k] = -inf;
      }
      id[2 * s + 1] = c;
      hi[2 * s + 1] = chi;
    } else {
      const float* cr = (const float*)(node + 4 * c);
      for (int t = 0; t < 2; ++t) {
        for (int k = 0; k < 6; ++k) box[2 * s + t][k] = cr[6 * t + k];
        id[2 * s + t] = __float_as_int(cr[12 + t]);
        hi[2 * s + t] = __float_as_int(cr[14 + t]);
      }
    }
  }
  // slot-major: per slot two float4 (box lo xyz, hi x | hi yz, child id, last leaf)
  float4* w = wide + 8 * (int64_t)i;
  for (int s = 0; s < 4; ++s) {
    w[2 * s] = make_float4(box[s][0], box[s][1], box[s][2], box[s][3]);
    w[2 * s + 1] = make_float4(box[s][4], box[s][5], __int_as_float(id[s]), __int_as_float(hi[s]));
  }
}

struct TravArgs {
  TravTree tt, te, tp;
  const double* x;
  const int32_t* tris;
  const int32_t* edges;
  const uint8_t* stat;
  const int32_t* vorder;  // vertex queries in Morton order
  const int16_t* vrank;   // their selected-segment ranks
  const int16_t* erank;   // selected-segment rank of each sorted edge leaf
  const int16_t* prank;   // ... of each sorted particle leaf
  const int32_t* root_t;  // per rank: subtree root in the triangle tree
  const int32_t* root_e;  // ... in the edge tree
  const int32_t* root_p;  // ... in the particle tree
  int32_t mv, me, mp;     // vertex, edge and particle queries
  int32_t mv_pad, me_pad; // the first two counts rounded up to whole waves
  double infl, dmax2;
  float fdmax;  // dmax rounded up to FP32 (the Euclidean box test below)
  // found pairs go to kStripes stripes of capS entries (keys, and d^2 in the same
  // function and operand order as the pair pass); null: counted only
  uint64_t* out;
  double* outd;
  int64_t capS;
  unsigned long long* stripe;  // per stripe: [0] runs << 40 | pairs, [1] node records read
  int4* chunks;                // per stripe capC runs: wave, offset in its output, length, start
  int64_t capC;
  long long* wtot;             // per wave: pairs found
  int32_t xcd_chunk;           // blocks per run of consecutive blocks dealt to one XCD
  int32_t nchunks;             // runs of 64 queries (a wave's worth each)
  unsigned long long* next;    // runs taken past the launch's own (zero at the launch)
  Counters* cnt;
};

__device__ __forceinline__ bool overlap6(float4 ql, float4 qh, float lx, float ly, float lz,
                                         float hx, float hy, float hz) {
  return ql.x <= hx && lx <= qh.x && ql.y <= hy && ly <= qh.y && ql.z <= hz && lz <= qh.z;
}

// Boxes that overlap6 accepts but whose un-inflated boxes lie farther apart than
// dmax in the Euclidean norm hold no pair within dmax (a primitive lies in its box,
// and the FP32 boxes contain the FP64 ones). Both boxes carry half of dmax, so the
// separation on an axis is max(0, gap + dmax), taken here as max(0, (ql + dmax) - h,
// l - (qh - dmax)) with the query's bounds moved by dmax once per query (qlp, qhm);
// r2 is (dmax + m)^2 with m = 1e-6 (1 + |query|_inf) m, far above the FP32 rounding of
// these few operations (below 3e-7 |query|_inf + 2e-7 dmax), so a box is dropped only
// when the exact FP64 test would reject every primitive in it.
__device__ __forceinline__ bool far6(float4 qlp, float4 qhm, float lx, float ly, float lz,
                                     float hx, float hy, float hz, float r2) {
  const float sx = fmaxf(0.f, fmaxf(qlp.x - hx, lx - qhm.x));
  const float sy = fmaxf(0.f, fmaxf(qlp.y - hy, ly - qhm.y));
  const float sz = fmaxf(0.f, fmaxf(qlp.z - hz, lz - qhm.z));
  return __builtin_fmaf(sz, sz, __builtin_fmaf(sy, sy, sx * sx)) > r2;
}

__device__ __forceinline__ uint64_t lanes_below_tr() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// Query classes of the traversal: vertex against the triangle tree, edge against
// the edge tree, particle against the particle tree.
constexpr int kQVT = 0, kQEE = 1, kQVV = 2;

// Exact test of one candidate primitive against the query: non-adjacent, not
// all static, FP64 distance below D_max. On success *out is the pair's key
// (vertex-triangle: vertex << 32 | triangle; edge-edge and vertex-vertex:
// canonical, lower id first, with the distance taken in that order; 0 is a valid
// key).
__device__ __forceinline__ bool candidate(const TravArgs& A, int kind, int32_t prim,
                                          int32_t qid, int32_t qv0, int32_t qv1, V3 qx0, V3 qx1,
                                          uint64_t* out, double* out_d2) {
  // (out and out_d2 point at the lane's next LDS buffer slot; written on success)
  double d2;
  uint64_t key;
  // (positions are loaded before the static flags are tested, so both loads follow
  // the topology together)
  if (kind == kQVV) {
    const V3 xb = ld3(A.x, prim);
    if (A.stat[qv0] && A.stat[prim]) return false;
    const V3 d = qid < prim ? vsub(qx0, xb) : vsub(xb, qx0);
    d2 = vdot(d, d);
    key = qid < prim ? (KEY_VV | ((uint64_t)(uint32_t)qid << 32) | (uint32_t)prim)
                     : (KEY_VV | ((uint64_t)(uint32_t)prim << 32) | (uint32_t)qid);
  } else if (kind == kQVT) {
    int32_t v1 = A.tris[3 * prim], v2 = A.tris[3 * prim + 1], v3 = A.tris[3 * prim + 2];
    const V3 xa = ld3(A.x, v1), xb = ld3(A.x, v2), xc = ld3(A.x, v3);
    if (qv0 == v1 || qv0 == v2 || qv0 == v3 ||
        (A.stat[qv0] && A.stat[v1] && A.stat[v2] && A.stat[v3]))
      return false;
    double bw[3];
    d2 = pt_tri_d2(qx0, xa, xb, xc, bw);
    key = ((uint64_t)(uint32_t)qid << 32) | (uint32_t)prim;
  } else {
    int32_t v1 = A.edges[2 * prim], v2 = A.edges[2 * prim + 1];
    const V3 xa = ld3(A.x, v1), xb = ld3(A.x, v2);
    if (qv0 == v1 || qv0 == v2 || qv1 == v1 || qv1 == v2 ||
        (A.stat[qv0] && A.stat[qv1] && A.stat[v1] && A.stat[v2]))
      return false;
    double s, t;
    if (qid < prim) {
      d2 = seg_seg_d2(qx0, qx1, xa, xb, s, t);
      key = KEY_EE | ((uint64_t)(uint32_t)qid << 32) | (uint32_t)prim;
    } else {
      d2 = seg_seg_d2(xa, xb, qx0, qx1, s, t);
      key = KEY_EE | ((uint64_t)(uint32_t)prim << 32) | (uint32_t)qid;
    }
  }
  if (!(d2 < A.dmax2)) return false;
  *out = key;
  *out_d2 = d2;
  return true;
}

constexpr double kRefitSlack = 1.3;         // node reads allowed to a refitted tree
constexpr int kWaves = kTravThreads / 64;  // waves per traversal block
// lanes sharing one traversal (a power of 2 in [8, 32]): a template argument of the
// traversal, picked per device and query count by the autotuner (16 without it)
constexpr int kGroupDefault = 16;
constexpr int kGStack = 100;                // stack entries per traversal (4-wide DFS)
constexpr int kQueue = 128;                 // candidate ring per wave (two rounds of 64)
constexpr int kOut = 192;                   // found pairs held per wave (flushed from 128)
constexpr int kXcdChunk = 32;               // consecutive traversal blocks per XCD
constexpr int kStripes = 64;                // output stripes of the search
constexpr int kStripeWords = 16;            // their counters 128 B apart
constexpr int kRunShift = 40;               // a stripe counter: runs << 40 | pairs
constexpr unsigned long long kPairMask = (1ull << kRunShift) - 1ull;

// The block's place in query order. Blocks are dealt to the 8 XCDs round-robin
// (block b runs on XCD b mod 8), and each XCD has an L2 of its own. Runs of c
// consecutive blocks (neighbouring queries in Morton order, which reach the same
// part of the tree and the same primitives) go to one XCD, and consecutive runs to
// consecutive XCDs, so that an XCD's waves share what its L2 holds while each XCD
// still takes an even share of dense and sparse regions. The last blocks past a
// whole number of rounds (8 c blocks each) keep their order. c = 1 is the identity.
__device__ __forceinline__ int32_t xcd_block(int32_t b, int32_t nb, int32_t c) {
  const int32_t full = nb / (8 * c) * (8 * c);
  if (c <= 1 || b >= full) return b;
  const int32_t x = b & 7, j = b >> 3;
  return ((j / c) * 8 + x) * c + j % c;
}

// A lane mask with every lane of a group of G consecutive lanes set when any lane of
// the group is set in m (scalar arithmetic on a wave-uniform mask).
template <int G>
__device__ __forceinline__ uint64_t group_any(uint64_t m) {
  if (G == 64) return m ? ~0ull : 0ull;
  uint64_t low = 1ull;  // the first lane of every group
  for (int s = G; s < 64; s <<= 1) low |= low << s;
  uint64_t t = m;
  for (int s = 1; s < G; s <<= 1) t |= t >> s;
  t &= low;
  for (int s = 1; s < G; s <<= 1) t |= t << s;
  return t;
}

template <int G, int P>
struct WaveLds {
  int32_t stack[kWaves][64 / G][kGStack];
  float4 nrec[kWaves][64 / G][8 * P];  // the records of the nodes a group takes in one step
  int32_t qlane[kWaves][kQueue];  // candidate: query lane ...
  int32_t qprim[kWaves][kQueue];  // ... and leaf primitive
  int32_t qi[kWaves][3][64];      // query id and its vertices per lane
  uint64_t okey[kWaves][kOut];    // found pairs not yet written out
  double od2[kWaves][kOut];
};

// The wave's held pairs to the output as one run, reserved with one atomic on the
// counts of the wave's next stripe. A device-wide atomic on one address is
// serialised over the whole GPU (about 12 ns each on MI355X); a wave's flushes
// rotate over the stripes, so each count takes about 1/kStripes of them and the
// stripes fill evenly. The run is recorded (wave, its offset in the wave's output,
// length, start) so that the gather can lay out P wave by wave.
template <class LT>
__device__ __forceinline__ void flush_out(LT& L, int wv, int32_t gw, int& no, unsigned& sidx,
                                          long long& wrun, const TravArgs& A) {
  const int lane = __lane_id();
  const unsigned sid = sidx & (kStripes - 1);
  ++sidx;
  unsigned long long old = 0;
  if (lane == 0)
    old = atomicAdd(&A.stripe[sid * kStripeWords],
                    (1ull << kRunShift) | (unsigned long long)no);
  old = __shfl(old, 0);
  const unsigned long long base = old & kPairMask;
  if (A.out) {
    const int64_t s0 = (int64_t)sid * A.capS;
    for (int j = lane; j < no; j += 64) {
      const int64_t pos = (int64_t)base + j;
      if (pos < A.capS) {
        A.out[s0 + pos] = L.okey[wv][j];
        if (A.outd) A.outd[s0 + pos] = L.od2[wv][j];
      }
    }
    const int64_t run = (int64_t)(old >> kRunShift);
    if (lane == 0 && run < A.capC)
      A.chunks[(int64_t)sid * A.capC + run] =
          make_int4((int)gw, (int)wrun, no, (int)base);
  }
  wrun += no;
  no = 0;
  __builtin_amdgcn_wave_barrier();
}

// The exact test of n <= 64 queued candidates, one per lane; found pairs join the
// wave's held pairs (no, wave-uniform), written out from 128 on.
template <class LT>
__device__ __forceinline__ void drain(LT& L, int wv, int32_t gw, int head, int n, int kind, int& no,
                                      unsigned& sidx, long long& wrun, unsigned& ntested,
                                      const TravArgs& A) {
  ntested += (unsigned)n;
  const int lane = __lane_id();
  bool found = false;
  uint64_t key = 0;
  double d2 = 0.0;
  if (lane < n) {
    const int e = (head + lane) & (kQueue - 1);
    const int ql = L.qlane[wv][e];
    const int32_t prim = L.qprim[wv][e];
    const int32_t qv0 = L.qi[wv][1][ql], qv1 = L.qi[wv][2][ql];
    // the query's positions, gathered again (the same values its box was made from)
    const V3 qx0 = ld3(A.x, qv0);
    const V3 qx1 = kind == kQEE ? ld3(A.x, qv1) : qx0;
    found = candidate(A, kind, prim, L.qi[wv][0][ql], qv0, qv1, qx0, qx1, &key, &d2);
  }
  __builtin_amdgcn_wave_barrier();
  const uint64_t m = __ballot(found);
  if (found) {
    const int j = no + __popcll(m & lanes_below_tr());
    L.okey[wv][j] = key;
    L.od2[wv][j] = d2;
  }
  no += __popcll(m);
  __builtin_amdgcn_wave_barrier();
  if (no >= kOut - 64) flush_out(L, wv, gw, no, sidx, wrun, A);
}

// Proximity search (Sec. 3.1). A wave takes 64 consecutive queries of one class
// (vertices against the triangle tree, edges against the edge tree, particles
// against the particle tree), in Morton order, and splits them into groups of
// kGroup lanes. A group walks the union of its lanes' traversals: a node's
// record is read once for the group, each lane tests the node's four children
// against its own query box, a child is entered when some lane of the group
// overlaps it, and the group's stack lives in LDS. A leaf that lanes overlap
// becomes one candidate per such lane in a ring in LDS shared by the wave; every
// 64 candidates the whole wave runs the exact FP64 tests together. Each lane sees
// exactly the leaves its own box overlaps (their ancestors overlap it too), so
// the pair set is that of independent per-query traversals, whatever kGroup is.
// Lanes of different scenes in one group walk their own subtrees in turn.
// The records of the nodes a group takes in one step are staged in LDS (one float4
// per lane) and their children tested in a loop that is not unrolled, so that the
// exact tests are compiled once (a third of the code, fewer registers). The child
// test is issue-bound, so its lane predicates are kept as scalar lane masks.
// (occupancy target: 4 waves per SIMD)
template <int kGroup, int kPop>
__global__ void __launch_bounds__(kTravThreads, 4) k_traverse(TravArgs A) {
  __shared__ WaveLds<kGroup, kPop> L;
  // the wave index is uniform over the wave: held in a scalar register
  const int lane = __lane_id(), wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = lane / kGroup, gl = lane % kGroup;
  const uint64_t gmask = (kGroup == 64 ? ~0ull : ((1ull << kGroup) - 1ull)) << (grp * kGroup);
  const int32_t lb = xcd_block(blockIdx.x, gridDim.x, A.xcd_chunk);
  unsigned nvisit = 0;  // node records this lane's group read (counted by its first lane)
  // runs of 64 queries: first the wave's own (its place in query order), then, when
  // the launch holds fewer waves than runs, the next run not yet taken
  for (int32_t gw = lb * kWaves + wv; gw < A.nchunks;) {
    const int32_t q0 = gw * 64;                         // the run's first padded query
    int kind;
    int32_t idx, ncl;
    if (q0 < A.mv_pad) {
      kind = kQVT;
      idx = q0 + lane;
      ncl = A.mv;
    } else if (q0 < A.mv_pad + A.me_pad) {
      kind = kQEE;
      idx = q0 - A.mv_pad + lane;
      ncl = A.me;
    } else {
      kind = kQVV;
      idx = q0 - A.mv_pad - A.me_pad + lane;
      ncl = A.mp;
    }
    const bool active = idx < ncl;
    const TravTree T = kind == kQVT ? A.tt : (kind == kQEE ? A.te : A.tp);
    float4 qlo = make_float4(0.f, 0.f, 0.f, 0.f), qhi = qlo;
    int32_t qv0 = 0, qv1 = 0, qid = 0, qpos = -1, root = -1;
    V3 qx0{0, 0, 0}, qx1{0, 0, 0};
    if (active) {
      if (kind == kQVT) {
        qid = A.vorder[idx];
        root = A.root_t[A.vrank[idx]];
        qv0 = qid;
        qx0 = ld3(A.x, qid);
        qlo = make_float4(lo_out(qx0.x - A.infl), lo_out(qx0.y - A.infl),
                          lo_out(qx0.z - A.infl), 0.f);
        qhi = make_float4(hi_out(qx0.x + A.infl), hi_out(qx0.y + A.infl),
                          hi_out(qx0.z + A.infl), 0.f);
      } else if (kind == kQVV) {
        qpos = idx;  // sorted position of the query particle in its tree
        qid = T.leaf_prim[qpos];
        root = A.root_p[A.prank[qpos]];
        qv0 = qid;
        qx0 = ld3(A.x, qid);
        qlo = make_float4(lo_out(qx0.x - A.infl), lo_out(qx0.y - A.infl),
                          lo_out(qx0.z - A.infl), 0.f);
        qhi = make_float4(hi_out(qx0.x + A.infl), hi_out(qx0.y + A.infl),
                          hi_out(qx0.z + A.infl), 0.f);
      } else {
        qpos = idx;  // sorted position of the query edge in the edge tree
        qid = T.leaf_prim[qpos];
        root = A.root_e[A.erank[qpos]];
        qv0 = A.edges[2 * qid];
        qv1 = A.edges[2 * qid + 1];
        qx0 = ld3(A.x, qv0);
        qx1 = ld3(A.x, qv1);
        qlo = make_float4(lo_out(fmin(qx0.x, qx1.x) - A.infl), lo_out(fmin(qx0.y, qx1.y) - A.infl),
                          lo_out(fmin(qx0.z, qx1.z) - A.infl), 0.f);
        qhi = make_float4(hi_out(fmax(qx0.x, qx1.x) + A.infl), hi_out(fmax(qx0.y, qx1.y) + A.infl),
                          hi_out(fmax(qx0.z, qx1.z) + A.infl), 0.f);
      }
    }
    L.qi[wv][0][lane] = qid;
    L.qi[wv][1][lane] = qv0;
    L.qi[wv][2][lane] = qv1;
    int head = 0, qn = 0;  // candidate ring: first entry, entries queued (wave-uniform)
    int no = 0;            // found pairs held (wave-uniform)
    unsigned sidx = gw;  // the stripe of the wave's next flush
    long long wrun = 0;                         // pairs the wave has written out
    unsigned ntested = 0;  // candidates tested by the wave
    // a scene with one triangle: its vertices meet the leaf itself (one edge or one
    // particle pairs with nothing)
    {
      const bool single = active && kind == kQVT && root < -1;
      const uint64_t m = __ballot(single);
      if (single) {
        const int e = __popcll(m & lanes_below_tr());
        L.qlane[wv][e] = lane;
        L.qprim[wv][e] = root & 0x7fffffff;
      }
      qn = __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    if (qn == 64) {
      drain(L, wv, gw, head, 64, kind, no, sidx, wrun, ntested, A);
      qn = 0;
      __builtin_amdgcn_wave_barrier();
    }
    // (dmax + m)^2 of the Euclidean box test, m = 1e-6 (1 + |query|_inf)
    float qr2;
    {
      const float qm = fmaxf(fmaxf(fmaxf(fabsf(qlo.x), fabsf(qhi.x)),
                                   fmaxf(fabsf(qlo.y), fabsf(qhi.y))),
                             fmaxf(fabsf(qlo.z), fabsf(qhi.z)));
      const float r = A.fdmax + 1e-6f * (1.f + qm);
      qr2 = r * r;
    }
    const float4 qlp = make_float4(qlo.x + A.fdmax, qlo.y + A.fdmax, qlo.z + A.fdmax, 0.f);
    const float4 qhm = make_float4(qhi.x - A.fdmax, qhi.y - A.fdmax, qhi.z - A.fdmax, 0.f);
    bool todo = active && root >= 0;  // this lane's subtree still to walk
    bool part = false;                // this lane takes part in its group's current walk
    int sp = 0;                       // the group's stack depth (uniform in the group)
    for (;;) {
      // a group with an empty stack starts the next scene's subtree among its lanes
      const uint64_t tm = __ballot(todo) & gmask;
      if (sp == 0) {
        part = false;
        if (tm) {
          const int32_t r = __shfl(root, __ffsll((long long)tm) - 1);
          part = todo && root == r;
          todo = todo && !part;
          if (gl == 0) L.stack[wv][grp][0] = r;
          sp = 1;
        }
      }
      if (!__any(sp > 0)) break;
      __builtin_amdgcn_wave_barrier();
      // kPop nodes leave the group's stack per step, their records loaded together so
      // that their latencies overlap (kPop = 2 halves the chain of dependent loads of a
      // deep walk; the set of nodes visited is the same)
      unsigned vmask = 0;  // the nodes taken (uniform in the group)
      int32_t ni[kPop];
  #pragma unroll
      for (int k = 0; k < kPop; ++k) {
        ni[k] = 0;
        if (sp > 0) {
          --sp;
          ni[k] = L.stack[wv][grp][sp];
          vmask |= 1u << k;
          if (gl == 0) ++nvisit;
        }
      }
      // each lane of the group stages float4s of the records (8 per node) in LDS; all
      // of a lane's loads are issued before the first is stored, so they overlap
      constexpr int kPer = (8 * kPop + kGroup - 1) / kGroup;  // float4s per lane
      float4 rv[kPer];
  #pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int f = i * kGroup + gl;
        rv[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (f < 8 * kPop) {
          int32_t nk = ni[0];
  #pragma unroll
          for (int k = 1; k < kPop; ++k)
            if ((f >> 3) == k) nk = ni[k];
          if ((vmask >> (f >> 3)) & 1u) rv[i] = T.wide[8 * (int64_t)nk + (f & 7)];
        }
      }
  #pragma unroll
      for (int i = 0; i < kPer; ++i) {
        const int f = i * kGroup + gl;
        if (f < 8 * kPop) L.nrec[wv][grp][f] = rv[i];
      }
      __builtin_amdgcn_wave_barrier();
      // per node taken: the lanes that test its children (taken by their group, and
      // taking part in the group's walk), as a lane mask
      const uint64_t pm = __ballot(part);
      uint64_t live[kPop];
  #pragma unroll
      for (int k = 0; k < kPop; ++k) live[k] = __ballot(((vmask >> k) & 1u) != 0) & pm;
  #pragma unroll 1
      for (int slot = 0; slot < 4 * kPop; ++slot) {
        uint64_t lv = live[0];
  #pragma unroll
        for (int k = 1; k < kPop; ++k)
          if ((slot >> 2) == k) lv = live[k];
        const float4 b0 = L.nrec[wv][grp][2 * slot];
        const float4 b1 = L.nrec[wv][grp][2 * slot + 1];
        const int32_t c = __float_as_int(b1.z);
        bool ov = false;
        if (__builtin_amdgcn_inverse_ballot_w64(lv))
          ov = overlap6(qlo, qhi, b0.x, b0.y, b0.z, b0.w, b1.x, b1.y) &&
               __float_as_int(b1.w) > qpos &&
               !far6(qlp, qhm, b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, qr2);
        // lane masks, kept in scalar registers: the lanes that overlap the child, the
        // groups whose child is internal, the groups that enter it, the leaf candidates
        const uint64_t m = __ballot(ov);
        const uint64_t inner = __ballot(c >= 0);
        const uint64_t enter = group_any<kGroup>(m) & inner;
        const uint64_t ml = m & ~inner;
        // internal child: the group enters it
        if (__builtin_amdgcn_inverse_ballot_w64(enter)) {
          if (sp < kGStack) {
            if (gl == 0) L.stack[wv][grp][sp] = c;
            ++sp;
          } else if (gl == 0) {
            atomicOr(&A.cnt->err, 2ull);
          }
        }
        // leaf child: one candidate per overlapping lane
        if (__builtin_amdgcn_inverse_ballot_w64(ml)) {
          const uint32_t below = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(ml >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ml, 0u));
          const int e = (head + qn + (int)below) & (kQueue - 1);
          L.qlane[wv][e] = lane;
          L.qprim[wv][e] = c & 0x7fffffff;
        }
        qn += __popcll(ml);
        __builtin_amdgcn_wave_barrier();
        while (qn >= 64) {
          drain(L, wv, gw, head, 64, kind, no, sidx, wrun, ntested, A);
          head = (head + 64) & (kQueue - 1);
          qn -= 64;
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
    if (qn > 0) drain(L, wv, gw, head, qn, kind, no, sidx, wrun, ntested, A);
    if (no > 0) flush_out(L, wv, gw, no, sidx, wrun, A);
    if (A.out && lane == 0) A.wtot[gw] = wrun;
    unsigned long long nx = 0;
    if (lane == 0) nx = atomicAdd(A.next, 1ull);
    gw = __builtin_amdgcn_readfirstlane((int32_t)(gridDim.x * kWaves) + (int32_t)__shfl(nx, 0));
  }
  // node records read by the wave's groups: the measure of the tree's quality
  unsigned long long nv = nvisit;
  for (int o = 32; o >= 1; o >>= 1) nv += __shfl_xor(nv, o);
  if (lane == 0 && nv)
    atomicAdd(&A.stripe[((blockIdx.x * kWaves + wv) & (kStripes - 1)) * kStripeWords + 1], nv);
}

// Exclusive prefix sum of the waves' pair counts, in place (one block).
__global__ void __launch_bounds__(1024) k_wave_offsets(long long* w, int32_t n) {
  __shared__ long long part[1024];
  const int t = threadIdx.x;
  const int32_t per = (n + 1023) / 1024, b = t * per, e = b + per < n ? b + per : n;
  long long sum = 0;
  for (int32_t i = b; i < e; ++i) sum += w[i];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const long long v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  long long run = part[t] - sum;
  for (int32_t i = b; i < e; ++i) {
    const long long c = w[i];
    w[i] = run;
    run += c;
  }
}

// The stripes' runs to out, wave by wave: P holds each wave's pairs together, in
// the order the wave found them (a wave's 64 queries are neighbours in Morton order,
// so the pairs of one pair-pass block share most of their vertices). One wave per
// run, kGatherWaves runs per block; the run's stripe from the stripes' run counts
// (one wave's scan per block).
constexpr int kGatherWaves = 4;
__global__ void __launch_bounds__(64 * kGatherWaves) k_stripe_gather(
    const unsigned long long* stripe, int64_t capS, int64_t capC, const int4* chunks,
    const long long* woff, const uint64_t* skeys, const double* sd2, uint64_t* out,
    double* outd, int64_t nruns) {
  static_assert(kStripes == 64, "one lane per stripe");
  __shared__ long long off[kStripes + 1];
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < 64) {
    const long long c = (long long)(stripe[lane * kStripeWords] >> kRunShift);
    long long incl = c;
    for (int o = 1; o < 64; o <<= 1) {
      const long long t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    off[lane + 1] = incl;
    if (lane == 0) off[0] = 0;
  }
  __syncthreads();
  const long long r = (long long)blockIdx.x * kGatherWaves + (threadIdx.x >> 6);
  if (r >= nruns) return;
  int lo = 0, hi = kStripes;  // off[lo] <= r < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= r) lo = mid;
    else hi = mid;
  }
  const int4 c = chunks[(int64_t)lo * capC + (r - off[lo])];
  const int64_t dst = woff[c.x] + c.y, src = (int64_t)lo * capS + c.w;
  for (int j = lane; j < c.z; j += 64) {
    out[dst + j] = skeys[src + j];
    if (outd) outd[dst + j] = sd2[src + j];
  }
}

// ------------------------------------------------------- input check (edges)

struct EtArgs {
  TravTree tt;
  const double* x;
  const int32_t* tris;
  const int32_t* edges;
  const uint8_t* stat;
  const int32_t* eprim;   // sorted edge leaves of the selected segments
  const int16_t* erank;   // their selected-segment ranks
  const int32_t* root_t;  // per rank: subtree root in the triangle tree
  int32_t me;
  double infl, tol;
  Counters* cnt;
};

// Edge (e0, e1) at (p, q) against triangle f: skipped when they share a vertex or
// all five vertices are static; otherwise the segment-triangle meeting test.
__device__ __forceinline__ bool et_meet(const EtArgs& A, int32_t f, int32_t e0, int32_t e1, V3 p,
                                        V3 q) {
  const int32_t a = A.tris[3 * f], b = A.tris[3 * f + 1], c = A.tris[3 * f + 2];
  if (e0 == a || e0 == b || e0 == c || e1 == a || e1 == b || e1 == c) return false;
  if (A.stat[e0] && A.stat[e1] && A.stat[a] && A.stat[b] && A.stat[c]) return false;
  return seg_tri_meet(p, q, ld3(A.x, a), ld3(A.x, b), ld3(A.x, c), A.tol);
}

// One lane per edge: walk its segment's triangle subtree (boxes inflated by
// tol/2, the query box by tol/2: every triangle the edge can meet or come within
// tol of is visited) and raise cnt->et on the first meeting.
__global__ void __launch_bounds__(kTravThreads) k_validate_et(EtArgs A) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= A.me) return;
  const int32_t e = A.eprim[q];
  const int32_t root = A.root_t[A.erank[q]];
  if (root == -1) return;  // the segment has no triangle
  const int32_t e0 = A.edges[2 * e], e1 = A.edges[2 * e + 1];
  const V3 p = ld3(A.x, e0), r = ld3(A.x, e1);
  bool bad = false;
  if (root < 0) {
    bad = et_meet(A, root & 0x7fffffff, e0, e1, p, r);
  } else {
    const float4 qlo = make_float4(lo_out(fmin(p.x, r.x) - A.infl), lo_out(fmin(p.y, r.y) - A.infl),
                                   lo_out(fmin(p.z, r.z) - A.infl), 0.f);
    const float4 qhi = make_float4(hi_out(fmax(p.x, r.x) + A.infl), hi_out(fmax(p.y, r.y) + A.infl),
                                   hi_out(fmax(p.z, r.z) + A.infl), 0.f);
    int32_t stack[kStack];
    int sp = 0;
    stack[sp++] = root;
    while (sp > 0 && !bad) {
      const int32_t i = stack[--sp];
      const float4* rec = A.tt.wide + 8 * i;
      for (int slot = 0; slot < 4 && !bad; ++slot) {
        const float4 b0 = rec[2 * slot], b1 = rec[2 * slot + 1];
        if (!overlap6(qlo, qhi, b0.x, b0.y, b0.z, b0.w, b1.x, b1.y)) continue;
        const int32_t c = __float_as_int(b1.z);
        if (c >= 0) {
          if (sp < kStack) stack[sp++] = c;
          else atomicOr(&A.cnt->err, 2ull);
          continue;
        }
        bad = et_meet(A, c & 0x7fffffff, e0, e1, p, r);
      }
    }
  }
  if (bad) atomicOr(&A.cnt->et, 1ull);
}

// Refit of a kept tree: the leaf boxes of the three trees at x, in their sorted
// order (the sort, the hierarchy and the query orders of the last build stay).
__global__ void k_leaf_refresh(const double* __restrict__ x, const int32_t* __restrict__ tris,
                               const int32_t* __restrict__ edges, int32_t mt, int32_t me,
                               int32_t mp, double infl, LeafOut lt, LeafOut le, LeafOut lp) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  V3 lo, hi;
  float4 *plo, *phi;
  int32_t i;
  if (g < mt) {
    i = g;
    const int32_t f = lt.prim[i];
    V3 a = ld3(x, tris[3 * f]), b = ld3(x, tris[3 * f + 1]), c = ld3(x, tris[3 * f + 2]);
    lo = V3{fmin(fmin(a.x, b.x), c.x), fmin(fmin(a.y, b.y), c.y), fmin(fmin(a.z, b.z), c.z)};
    hi = V3{fmax(fmax(a.x, b.x), c.x), fmax(fmax(a.y, b.y), c.y), fmax(fmax(a.z, b.z), c.z)};
    plo = lt.lo;
    phi = lt.hi;
  } else if (g < mt + me) {
    i = g - mt;
    const int32_t e = le.prim[i];
    V3 a = ld3(x, edges[2 * e]), b = ld3(x, edges[2 * e + 1]);
    lo = V3{fmin(a.x, b.x), fmin(a.y, b.y), fmin(a.z, b.z)};
    hi = V3{fmax(a.x, b.x), fmax(a.y, b.y), fmax(a.z, b.z)};
    plo = le.lo;
    phi = le.hi;
  } else if (g < mt + me + mp) {
    i = g - mt - me;
    lo = ld3(x, lp.prim[i]);
    hi = lo;
    plo = lp.lo;
    phi = lp.hi;
  } else {
    return;
  }
  plo[i] = make_float4(lo_out(lo.x - infl), lo_out(lo.y - infl), lo_out(lo.z - infl), 0.f);
  phi[i] = make_float4(hi_out(hi.x + infl), hi_out(hi.y + infl), hi_out(hi.z + infl), 0.f);
}

// ---------------------------------------------------------------- host side

template <class T>
static int dalloc(T** p, int64_t n) {
  if (n <= 0) n = 1;
  if (hipMalloc((void**)p, (size_t)n * sizeof(T)) != hipSuccess) return CC_ENOMEM;
  return CC_OK;
}
template <class T>
static void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

static int bvh_alloc_one(Bvh& b, int32_t cap) {
  b.n = 0;
  int32_t ni = cap > 1 ? cap - 1 : 1;
  int32_t nb = (cap + kBlk - 1) / kBlk;
  CC_TRY(dalloc(&b.leaf_lo, cap));
  CC_TRY(dalloc(&b.leaf_hi, cap));
  CC_TRY(dalloc(&b.leaf_prim, cap));
  CC_TRY(dalloc(&b.node, 4 * (int64_t)ni));
  CC_TRY(dalloc(&b.wide, 8 * (int64_t)ni));
  CC_TRY(dalloc(&b.parent, (int64_t)ni + cap));
  CC_TRY(dalloc(&b.range, ni));
  CC_TRY(dalloc(&b.pre, 2 * (int64_t)cap));
  CC_TRY(dalloc(&b.suf, 2 * (int64_t)cap));
  int nlev = 1;
  while ((1 << nlev) <= nb) ++nlev;  // sparse-table levels over the block boxes
  CC_TRY(dalloc(&b.blk, 2 * (int64_t)(nb > 0 ? nb : 1) * nlev));
  CC_TRY(dalloc(&b.root, 2));
  return CC_OK;
}

static void bvh_free_one(Bvh& b) {
  dfree(b.leaf_lo); dfree(b.leaf_hi); dfree(b.leaf_prim);
  dfree(b.node); dfree(b.wide); dfree(b.parent); dfree(b.range); dfree(b.pre); dfree(b.suf);
  dfree(b.blk); dfree(b.root);
  b = Bvh{};
}

int bvh_alloc(cc_solver* s) {
  ++s->gen;  // fresh tree memory holds no tree
  const int64_t m = (int64_t)s->capF + s->capE + s->capPt;
  const int64_t mall = m + s->capV;  // triangles, edges, particles and vertices share one sort
  CC_TRY(bvh_alloc_one(s->tree_t, s->capF));
  CC_TRY(bvh_alloc_one(s->tree_e, s->capE));
  CC_TRY(bvh_alloc_one(s->tree_p, s->capPt));
  CC_TRY(dalloc(&s->prank, s->capPt));
  CC_TRY(dalloc(&s->root_p, kMaxSeg));
  CC_TRY(dalloc(&s->sk0, mall));
  CC_TRY(dalloc(&s->sk1, mall));
  CC_TRY(dalloc(&s->sv0, mall));
  CC_TRY(dalloc(&s->sv1, mall));
  CC_TRY(dalloc(&s->ubox_lo, m));
  CC_TRY(dalloc(&s->ubox_hi, m));
  CC_TRY(dalloc(&s->gprim, m));
  CC_TRY(dalloc(&s->vorder, s->capV));
  CC_TRY(dalloc(&s->vrank, s->capV));
  CC_TRY(dalloc(&s->erank, s->capE));
  int64_t nb = (mall + kTile - 1) / kTile;
  s->rs_hist_cap = 256 * (nb > 0 ? nb : 1);
  CC_TRY(dalloc(&s->rs_hist, s->rs_hist_cap));
  CC_TRY(dalloc(&s->rs_total, 256));
  CC_TRY(dalloc(&s->bounds, 6));
  CC_TRY(dalloc(&s->bounds_part, 6 * ((m + 255) / 256)));
  CC_TRY(dalloc(&s->sel_dev, kMaxSeg + 1));
  if (!s->sel_host &&
      hipHostMalloc((void**)&s->sel_host, sizeof(SelDev) * (kMaxSeg + 1), hipHostMallocDefault) !=
          hipSuccess)
    return CC_ENOMEM;
  CC_TRY(dalloc(&s->root_t, kMaxSeg));
  CC_TRY(dalloc(&s->root_e, kMaxSeg));
  return CC_OK;
}

void bvh_free(cc_solver* s) {
  bvh_free_one(s->tree_t);
  bvh_free_one(s->tree_e);
  bvh_free_one(s->tree_p);
  dfree(s->prank); dfree(s->root_p);
  dfree(s->sk0); dfree(s->sk1); dfree(s->sv0); dfree(s->sv1);
  dfree(s->ubox_lo); dfree(s->ubox_hi); dfree(s->gprim); dfree(s->rs_hist); dfree(s->bounds);
  dfree(s->bounds_part); dfree(s->vorder); dfree(s->vrank); dfree(s->erank); dfree(s->rs_total);
  dfree(s->sel_dev); dfree(s->root_t); dfree(s->root_e);
  dfree(s->skeys); dfree(s->sd2); dfree(s->chunks); dfree(s->wtot);
  s->capS = 0;
  s->capC = 0;
  s->capW = 0;
}

static inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

static RefitView refit_view(Bvh& b, bool direct) {
  return RefitView{b.n,   b.leaf_lo, b.leaf_hi, b.parent, b.range, b.node,
                   b.root, b.pre,    b.suf,     b.blk,    b.wide,  direct ? 1 : 0};
}

// Node boxes from the leaf boxes (fence-free refit). After a build the 4-wide
// records are then made from the binary ones; a refit of the same tree writes
// the boxes into the built 4-wide records as it forms them.
static int refit_and_widen(cc_solver* s, int32_t mt, int32_t me, int32_t mp, bool built,
                           hipStream_t st) {
  Bvh& bt = s->tree_t;
  Bvh& be = s->tree_e;
  Bvh& bp = s->tree_p;
  RefitView ra = refit_view(bt, !built), rbv = refit_view(be, !built);
  if (mt < 2) ra.n = 0;
  if (me < 2) rbv.n = 0;
  const int32_t nba = (ra.n + kBlk - 1) / kBlk, nbb = (rbv.n + kBlk - 1) / kBlk;
  const int64_t ninternal = (mt > 1 ? mt - 1 : 0) + (me > 1 ? me - 1 : 0);
  if (nba + nbb > 0) {
    k_refit_block<<<nba + nbb, kBlk, 0, st>>>(ra, rbv, nba);
    k_blk_sparse<<<2, 1024, 0, st>>>(ra, rbv);
    k_refit_top<<<blocks(ninternal, 256), 256, 0, st>>>(ra, rbv);
  }
  if (mp > 1) {  // the particle tree, refit on its own
    RefitView rc = refit_view(bp, !built), rnone = refit_view(bp, !built);
    rnone.n = 0;
    const int32_t nbc = (mp + kBlk - 1) / kBlk;
    k_refit_block<<<nbc, kBlk, 0, st>>>(rc, rnone, nbc);
    k_blk_sparse<<<1, 1024, 0, st>>>(rc, rnone);
    k_refit_top<<<blocks(mp - 1, 256), 256, 0, st>>>(rc, rnone);
  }
  if (built) {
    if (mt > 1) k_wide<<<blocks(mt - 1, 256), 256, 0, st>>>(bt.node, bt.wide, mt - 1);
    if (me > 1) k_wide<<<blocks(me - 1, 256), 256, 0, st>>>(be.node, be.wide, me - 1);
    if (mp > 1) k_wide<<<blocks(mp - 1, 256), 256, 0, st>>>(bp.node, bp.wide, mp - 1);
  }
  CC_HIP(hipGetLastError());
  return CC_OK;
}

constexpr size_t kStripeBytes = sizeof(unsigned long long) * kStripes * kStripeWords;

// Stripes of capS pairs (keys and squared distances) and capC runs each; the
// contents go.
static int grow_stripes(cc_solver* s, int64_t capS, int64_t capC) {
  dfree(s->skeys);
  dfree(s->sd2);
  dfree(s->chunks);
  s->capS = 0;
  s->capC = 0;
  CC_TRY(dalloc(&s->skeys, capS * kStripes));
  CC_TRY(dalloc(&s->sd2, capS * kStripes));
  CC_TRY(dalloc(&s->chunks, capC * kStripes));
  s->capS = capS;
  s->capC = capC;
  return CC_OK;
}
// runs of a stripe of capS pairs: all but a wave's last hold at least kOut - 64
static inline int64_t runs_for(int64_t capS) { return capS / 64 + 1024; }

// Blocks of a traversal variant the device holds at once (0 if unknown).
template <int G, int P>
static unsigned resident_blocks() {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_traverse<G, P>, kTravThreads, 0) !=
          hipSuccess)
    return 0;
  return (unsigned)(ncu > 0 && per > 0 ? ncu * per : 0);
}

// The traversal over A.nchunks runs of 64 queries with at most as many blocks as the
// device holds at once: the runs past the launch's own go to the waves that finish
// first (A.next counts them from zero), so none waits for a whole block to end.
template <int G, int P>
static void traverse_variant(const TravArgs& A, hipStream_t st) {
  static unsigned res[64] = {};  // per device (0: not asked yet)
  int dev = 0;
  (void)hipGetDevice(&dev);
  unsigned& r = res[dev & 63];
  if (r == 0) r = resident_blocks<G, P>();
  unsigned nb = (unsigned)(A.nchunks / kWaves);
  if (r > 0 && nb > r) nb = r;
  k_traverse<G, P><<<nb, kTravThreads, 0, st>>>(A);
}

int launch_traverse(int group, const TravArgs& A, int64_t nq, hipStream_t st) {
  if ((int64_t)A.nchunks * 64 < nq || A.nchunks % kWaves != 0) return CC_EINVAL;
  switch (group) {
    case 8: traverse_variant<8, 1>(A, st); break;
    case 32: traverse_variant<32, 1>(A, st); break;
    case 108: traverse_variant<8, 2>(A, st); break;
    case 116: traverse_variant<16, 2>(A, st); break;
    case 132: traverse_variant<32, 2>(A, st); break;
    default: traverse_variant<16, 1>(A, st); break;
  }
  CC_HIP(hipGetLastError());
  return CC_OK;
}

int lbvh_search(cc_solver* s, int32_t nsel, const double* x, double dmax, uint64_t* out,
                double* outd, int64_t cap, int64_t* nfound, hipStream_t st, bool refit_ok) {
  // compact offsets of the selected segments' vertices, triangles, edges and particles
  int32_t mv = 0, mt = 0, me = 0, mp = 0;
  for (int32_t r = 0; r < nsel; ++r) {
    SelDev& d = s->sel_host[r];
    const Seg& g = s->segs[d.seg];
    d.vb = g.vb;
    d.fb = g.fb;
    d.eb = g.eb;
    d.voff = mv;
    d.toff = mt;
    d.eoff = me;
    d.poff = mp;
    mv += g.nv;
    mt += g.nf;
    me += g.ne;
    mp += g.np;
  }
  s->sel_host[nsel] = SelDev{0, 0, 0, -1, mv, mt, me, mp};
  if (mp > s->capPt) return CC_EINVAL;  // the particle capacity follows seg_add
  int rb = 0;
  while ((1 << rb) < nsel) ++rb;
  const double infl = 0.5 * dmax;
  // the search counts into n_out, err and ncand: one fill clears the counters from
  // n_out to ncand (none of those between is pending when a search starts; the
  // colour, edge-row and input-check counters after them are left alone)
  static_assert(offsetof(Counters, n_out) == 0 && offsetof(Counters, ncand) > offsetof(Counters, err) &&
                    offsetof(Counters, n_rows) > offsetof(Counters, ncand) &&
                    offsetof(Counters, et) > offsetof(Counters, ncand),
                "search counters first");
  CC_HIP(hipMemsetAsync(s->dc, 0, offsetof(Counters, ncand) + sizeof(unsigned long long), st));
  *nfound = 0;
  int64_t nfd = 0;     // pairs found (the stripes' counts)
  int64_t nruns = 0;   // runs written into the stripes
  double ncand = 0.0;  // node records read by the traversal
  const int64_t m = (int64_t)mt + me + mp;
  // the tree of the last build serves again (refit) when the same scenes, in the same
  // order, are searched and none of them changed since
  bool refit = refit_ok && s->bvh_gen == s->gen && (int32_t)s->bvh_sel.size() == nsel;
  for (int32_t r = 0; refit && r < nsel; ++r) refit = s->bvh_sel[r] == s->sel_host[r].seg;
  if (refit_ok) {
    s->bvh_gen = s->gen;
    s->bvh_sel.resize(nsel);
    for (int32_t r = 0; r < nsel; ++r) s->bvh_sel[r] = s->sel_host[r].seg;
  } else {
    s->bvh_gen = ~0ull;  // a build for another purpose: the next search builds anew
  }
  Bvh& bt = s->tree_t;
  Bvh& be = s->tree_e;
  Bvh& bp = s->tree_p;
  if (m > 0 && refit) {
    k_leaf_refresh<<<blocks(m, 256), 256, 0, st>>>(
        x, s->tris, s->edges, mt, me, mp, infl, LeafOut{bt.leaf_lo, bt.leaf_hi, bt.leaf_prim, nullptr},
        LeafOut{be.leaf_lo, be.leaf_hi, be.leaf_prim, nullptr},
        LeafOut{bp.leaf_lo, bp.leaf_hi, bp.leaf_prim, nullptr});
    CC_TRY(refit_and_widen(s, mt, me, mp, false, st));
  } else if (m > 0) {
    CC_HIP(hipMemcpyAsync(s->sel_dev, s->sel_host, sizeof(SelDev) * (nsel + 1),
                          hipMemcpyHostToDevice, st));
    const int64_t mall = m + mv;
    const unsigned nbx = blocks(m, 256);
    k_boxes<<<nbx, 256, 0, st>>>(x, s->tris, s->edges, s->plist, s->sel_dev, nsel, mt, me, mp,
                                 infl, s->ubox_lo, s->ubox_hi, s->gprim, s->bounds_part);
    k_bounds_reduce<<<1, 256, 0, st>>>(s->bounds_part, (int32_t)nbx, s->bounds);
    k_morton<<<blocks(mall, 256), 256, 0, st>>>(s->ubox_lo, s->ubox_hi, x, s->sel_dev, nsel, mt,
                                                me, mp, mv, rb, s->bounds, s->sk0, s->sv0);
    const int32_t nb = (int32_t)((mall + kTile - 1) / kTile);
    uint64_t *ki = s->sk0, *ko = s->sk1;
    uint32_t *vi = s->sv0, *vo = s->sv1;
    for (int shift = 0; shift < 32 + rb; shift += 8) {
      k_rs_hist<<<nb, kRsThreads, 0, st>>>(ki, (int32_t)mall, shift, s->rs_hist, nb);
      k_rs_scan_digit<<<256, kRsThreads, 0, st>>>(s->rs_hist, nb, s->rs_total);
      k_rs_scatter<<<nb, kRsThreads, 0, st>>>(ki, vi, ko, vo, (int32_t)mall, shift, s->rs_hist,
                                              nb, s->rs_total);
      std::swap(ki, ko);
      std::swap(vi, vo);
    }
    bt.n = mt;
    be.n = me;
    bp.n = mp;
    k_leaves<<<blocks(mall, 256), 256, 0, st>>>(vi, ki, s->ubox_lo, s->ubox_hi, s->gprim,
                                                s->sel_dev, mt, me, mp, mv, (1u << rb) - 1u,
                                                bt.leaf_lo, bt.leaf_hi, bt.leaf_prim, be.leaf_lo,
                                                be.leaf_hi, be.leaf_prim, s->erank,
                                                LeafOut{bp.leaf_lo, bp.leaf_hi, bp.leaf_prim,
                                                        s->prank},
                                                s->vorder, s->vrank);
    const uint64_t mask = (1ull << (30 + rb)) - 1ull;
    TreeView ta{mt, ki, mask, bt.leaf_prim, bt.node, bt.parent, bt.range};
    TreeView tb{me, ki + mt, mask, be.leaf_prim, be.node, be.parent, be.range};
    TreeView tc{mp, ki + mt + me, mask, bp.leaf_prim, bp.node, bp.parent, bp.range};
    const TreeView tnone{0, nullptr, 0, nullptr, nullptr, nullptr, nullptr};
    int64_t ninternal = (mt > 1 ? mt - 1 : 0) + (me > 1 ? me - 1 : 0);
    if (ninternal > 0) k_karras<<<blocks(ninternal, 256), 256, 0, st>>>(ta, tb);
    if (mp > 1) k_karras<<<blocks(mp - 1, 256), 256, 0, st>>>(tc, tnone);
    k_seg_roots<<<blocks(nsel, 256), 256, 0, st>>>(s->sel_dev, nsel, mt, me, mp, bt.range,
                                                   bt.leaf_prim, be.range, be.leaf_prim, bp.range,
                                                   bp.leaf_prim, s->root_t, s->root_e, s->root_p);
    CC_TRY(refit_and_widen(s, mt, me, mp, true, st));
  }
  if (m > 0) {
    TravArgs A;
    A.tt = TravTree{mt, bt.wide, bt.root, bt.leaf_prim};
    A.te = TravTree{me, be.wide, be.root, be.leaf_prim};
    A.tp = TravTree{mp, bp.wide, bp.root, bp.leaf_prim};
    A.x = x;
    A.tris = s->tris;
    A.edges = s->edges;
    A.stat = s->stat;
    A.vorder = s->vorder;
    A.vrank = s->vrank;
    A.erank = s->erank;
    A.prank = s->prank;
    A.root_t = s->root_t;
    A.root_e = s->root_e;
    A.root_p = s->root_p;
    A.mv = mt > 0 ? mv : 0;  // no triangles: no vertex-triangle queries
    A.me = me;
    A.mp = mp;
    A.infl = infl;
    A.dmax2 = dmax * dmax;
    A.fdmax = (float)dmax;
    if ((double)A.fdmax < dmax) A.fdmax = nextafterf(A.fdmax, __builtin_inff());
    // the stripes: about cap / kStripes each to start with (a quarter more, for the
    // spread of the stripes' counts), grown below when one overflows
    if (out && s->capS == 0) {
      const int64_t c0 = (cap > 0 ? cap : 1) / kStripes;
      CC_TRY(grow_stripes(s, c0 + c0 / 4 + 1024, runs_for(c0 + c0 / 4 + 1024)));
    }
    A.out = out ? s->skeys : nullptr;
    A.outd = out && outd ? s->sd2 : nullptr;
    A.capS = s->capS;
    A.stripe = s->stripe;
    A.chunks = s->chunks;
    A.capC = s->capC;
    A.cnt = s->dc;
    A.xcd_chunk = kXcdChunk;
    A.next = s->stripe + 2;  // a free word of the first stripe's counters (cleared with them)
    A.mv_pad = (A.mv + 63) & ~63;
    A.me_pad = (me + 63) & ~63;
    int64_t nq = (int64_t)A.mv_pad + A.me_pad + mp;
    const int64_t nwaves = (int64_t)blocks(nq, kTravThreads) * kWaves;
    A.nchunks = (int32_t)nwaves;
    if (out && nwaves > s->capW) {
      dfree(s->wtot);
      s->capW = 0;
      CC_TRY(dalloc(&s->wtot, nwaves));
      s->capW = nwaves;
    }
    A.wtot = s->wtot;
    if (nq > 0) {
      // lanes per traversal group: the autotuner's choice for this device and query
      // count, measured on this search's own queries the first time (every variant
      // finds the same pair set; the counters restart before each)
      int group = kGroupDefault;
      if (!(s->p.flags & CC_NO_AUTOTUNE)) {
        const int cls = A.mv >= A.me && A.mv >= A.mp ? 0 : (A.me >= A.mp ? 1 : 2);
        const int32_t size_class = 4 * (int32_t)std::ilogb((double)nq) + cls;
        int dev = 0;
        CC_HIP(hipGetDevice(&dev));
        group = tune_lookup(dev, CC_TUNE_TRAVERSE, size_class);
        if (group < 0) {
          const int cand[6] = {8, 16, 32, 108, 116, 132};
          float ms[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
          int best = 1;
          hipEvent_t e0, e1;
          CC_HIP(hipEventCreate(&e0));
          CC_HIP(hipEventCreate(&e1));
          for (int c = 0; c < 6; ++c) {
            CC_HIP(hipMemsetAsync(s->dc, 0, offsetof(Counters, ncand) + sizeof(unsigned long long),
                                  st));
            CC_HIP(hipMemsetAsync(s->stripe, 0, kStripeBytes, st));
            CC_HIP(hipEventRecord(e0, st));
            CC_TRY(launch_traverse(cand[c], A, nq, st));
            CC_HIP(hipEventRecord(e1, st));
            CC_HIP(hipEventSynchronize(e1));
            CC_HIP(hipEventElapsedTime(&ms[c], e0, e1));
            if (ms[c] < ms[best]) best = c;
          }
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          group = cand[best];
          tune_store(dev, CC_TUNE_TRAVERSE, size_class, group, ms);
          CC_HIP(hipMemsetAsync(s->dc, 0, offsetof(Counters, ncand) + sizeof(unsigned long long),
                                st));
        }
      }
      // a stripe that overflowed is grown to its count and the traversal runs again:
      // it fills every stripe exactly as before (each wave's flushes, and the stripe
      // each goes to, depend on its own queries only)
      for (int attempt = 0;; ++attempt) {
        CC_HIP(hipMemsetAsync(s->stripe, 0, kStripeBytes, st));
        timer_begin(s, CC_K_SEARCH, st);
        CC_TRY(launch_traverse(group, A, nq, st));
        timer_end(s, st);
        // the stripe counts and the counters after them in one copy
        static_assert(kStripeBytes == kMirrorCounters - kMirrorStripe, "stripes, then counters");
        CC_HIP(hipMemcpyAsync(s->hstripe, s->stripe, kStripeBytes + sizeof(Counters),
                              hipMemcpyDeviceToHost, st));
        CC_HIP(hipStreamSynchronize(st));
        if (s->hc->err & 2ull) return CC_EOVERFLOW;  // a traversal stack overflowed
        unsigned long long mx = 0, mr = 0, tot = 0, nvis = 0;
        nruns = 0;
        for (int k = 0; k < kStripes; ++k) {
          const unsigned long long v = s->hstripe[k * kStripeWords];
          mx = std::max(mx, v & kPairMask);
          mr = std::max(mr, v >> kRunShift);
          tot += v & kPairMask;
          nruns += (int64_t)(v >> kRunShift);
          nvis += s->hstripe[k * kStripeWords + 1];
        }
        nfd = (int64_t)tot;
        ncand = (double)nvis;
        if (!out || ((int64_t)mx <= A.capS && (int64_t)mr <= A.capC)) break;
        if (attempt > 0) return CC_EOVERFLOW;  // cannot happen: the counts repeat
        const int64_t ns = std::max<int64_t>(s->capS, (int64_t)mx + (int64_t)mx / 4 + 1024);
        CC_TRY(grow_stripes(s, ns, std::max<int64_t>(runs_for(ns), (int64_t)mr + (int64_t)mr / 4 + 1024)));
        A.out = s->skeys;
        A.outd = outd ? s->sd2 : nullptr;
        A.capS = s->capS;
        A.chunks = s->chunks;
        A.capC = s->capC;
      }
      if (out && nfd > 0 && nfd <= cap) {
        k_wave_offsets<<<1, 1024, 0, st>>>(s->wtot, (int32_t)nwaves);
        k_stripe_gather<<<(unsigned)((nruns + kGatherWaves - 1) / kGatherWaves), 64 * kGatherWaves,
                          0, st>>>(s->stripe, s->capS, s->capC, s->chunks, s->wtot, s->skeys,
                                   s->sd2, out, outd, nruns);
      }
    }
  }
  // (the gather is left queued on the stream: what follows is ordered after it)
  CC_HIP(hipGetLastError());
  *nfound = nfd;
  // tree quality: node records read by the traversal; a refitted tree whose
  // traversal reads 30 % more of them than right after its build is built anew at the
  // next search
  if (refit_ok && m > 0) {
    const double q = ncand;
    if (!refit) s->bvh_q0 = q;
    else if (q > kRefitSlack * s->bvh_q0) s->bvh_gen = ~0ull;
  }
  // algorithmic bytes of the traversal: queries, node records, output keys and their
  // squared distances (8 + 8 bytes per pair found)
  s->st.kernel_bytes[CC_K_SEARCH] += 24.0 * mv + 8.0 * me + 28.0 * mp + 64.0 * (double)m +
                                     16.0 * (double)*nfound;
  return CC_OK;
}

// The input check: a touching search at tol (vertex-triangle and edge-edge pairs
// closer than tol, counted, not stored), then the edge-triangle meeting test over
// the trees that search built.
int lbvh_validate(cc_solver* s, int32_t nsel, const double* x, double tol, int* bad,
                  hipStream_t st) {
  *bad = 0;
  const double kb = s->st.kernel_bytes[CC_K_SEARCH];
  int64_t n = 0;
  const int rc = lbvh_search(s, nsel, x, tol, nullptr, nullptr, 0, &n, st, false);
  s->st.kernel_bytes[CC_K_SEARCH] = kb;  // not a step's search
  CC_TRY(rc);
  if (n > 0) {
    *bad = 1;
    return CC_OK;
  }
  const int32_t mt = s->sel_host[nsel].toff, me = s->sel_host[nsel].eoff;
  if (mt == 0 || me == 0) return CC_OK;
  CC_HIP(hipMemsetAsync(&s->dc->et, 0, sizeof(unsigned long long), st));
  EtArgs A;
  A.tt = TravTree{mt, s->tree_t.wide, s->tree_t.root, s->tree_t.leaf_prim};
  A.x = x;
  A.tris = s->tris;
  A.edges = s->edges;
  A.stat = s->stat;
  A.eprim = s->tree_e.leaf_prim;
  A.erank = s->erank;
  A.root_t = s->root_t;
  A.me = me;
  A.infl = 0.5 * tol;
  A.tol = tol;
  A.cnt = s->dc;
  k_validate_et<<<blocks(me, kTravThreads), kTravThreads, 0, st>>>(A);
  CC_HIP(hipGetLastError());
  CC_HIP(hipMemcpyAsync(s->hc, s->dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (s->hc->err & 2ull) return CC_EOVERFLOW;
  *bad = s->hc->et != 0;
  return CC_OK;
}

}  // namespace cc
