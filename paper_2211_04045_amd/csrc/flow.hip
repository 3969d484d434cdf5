// Target of the globally injective normal flow (Sec. 7.4, Eq. eq:normal flow):
// y_0 = x + beta n, n the area-weighted vertex normals at x, then `iters` Jacobi
// steps y <- y + alpha L y with L the cotangent Laplace-Beltrami operator of the
// mesh at the current y (barycentric areas). The collision step then makes the
// flow globally injective.
//
// Every per-vertex sum runs over the vertex's triangles in increasing index, in
// the written operation order of the geometry code, so the target is the same on
// any launch configuration.
#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <vector>

#include "geom.hpp"
#include "internal.hpp"

namespace cc {

struct FlowWork {
  int32_t capN = 0, capC = 0;
  int32_t* cnt = nullptr;  // n + 1: counts, then the exclusive offsets of the incidence lists
  int32_t* cur = nullptr;  // n: fill cursors
  int32_t* inc = nullptr;  // 3F: incident triangles of each vertex, increasing
  double* tmp = nullptr;   // 3n: the other buffer of the Jacobi steps
  int32_t* err = nullptr;  // 1: bad vertex index
};

namespace {

constexpr int kFlowThreads = 256;
inline unsigned fblk(int64_t n) { return (unsigned)((n + kFlowThreads - 1) / kFlowThreads); }

__global__ void k_nf_count(const int32_t* __restrict__ tris, int64_t n3, int32_t n,
                           int32_t* __restrict__ cnt, int32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const int32_t v = tris[i];
  if (v < 0 || v >= n) {
    atomicOr(err, 1);
    return;
  }
  atomicAdd(&cnt[v + 1], 1);
}

__global__ void k_nf_fill(const int32_t* __restrict__ tris, int64_t n3, int32_t* __restrict__ cur,
                          int32_t* __restrict__ inc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  inc[atomicAdd(&cur[tris[i]], 1)] = (int32_t)(i / 3);
}

// Each vertex's list in increasing triangle index (short lists: insertion sort).
__global__ void k_nf_sort(const int32_t* __restrict__ off, int32_t n, int32_t* __restrict__ inc) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t b = off[v], e = off[v + 1];
  for (int32_t i = b + 1; i < e; ++i) {
    const int32_t f = inc[i];
    int32_t j = i - 1;
    while (j >= b && inc[j] > f) {
      inc[j + 1] = inc[j];
      --j;
    }
    inc[j + 1] = f;
  }
}

// y_0 = x + beta n; n = normalised sum of (x_b - x_a) x (x_c - x_a) (0 when it vanishes).
__global__ void k_nf_offset(const double* __restrict__ x, const int32_t* __restrict__ tris,
                            const int32_t* __restrict__ off, const int32_t* __restrict__ inc,
                            int32_t n, double beta, double* __restrict__ y) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  V3 s{0.0, 0.0, 0.0};
  for (int32_t i = off[v]; i < off[v + 1]; ++i) {
    const int32_t* t = tris + 3 * (int64_t)inc[i];
    const V3 a = ld3(x, t[0]);
    const V3 N = vcross(vsub(ld3(x, t[1]), a), vsub(ld3(x, t[2]), a));
    s = V3{s.x + N.x, s.y + N.y, s.z + N.z};
  }
  const double len = sqrt(vdot(s, s));
  const V3 nv = len > 0.0 ? V3{s.x / len, s.y / len, s.z / len} : V3{0.0, 0.0, 0.0};
  const V3 p = ld3(x, v);
  st3(y, v, V3{p.x + beta * nv.x, p.y + beta * nv.y, p.z + beta * nv.z});
}

// cotangent of the angle at b of triangle (a, b, c); 0 when degenerate
__device__ __forceinline__ double nf_cot(V3 a, V3 b, V3 c) {
  const V3 u = vsub(a, b), w = vsub(c, b);
  const V3 k = vcross(u, w);
  const double s = sqrt(vdot(k, k));
  if (s == 0.0) return 0.0;
  return vdot(u, w) / s;
}

// One Jacobi step: y'(v) = y(v) + alpha (L / (2 A)), L = sum over the triangles at v
// (rotated to (v, q, r)) of cot_r (y_q - y_v) + cot_q (y_r - y_v), A = sum of a third
// of their areas; a vertex with A = 0 keeps y.
__global__ void k_nf_smooth(const double* __restrict__ y, const int32_t* __restrict__ tris,
                            const int32_t* __restrict__ off, const int32_t* __restrict__ inc,
                            int32_t n, double alpha, double* __restrict__ yo) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const V3 p = ld3(y, v);
  V3 L{0.0, 0.0, 0.0};
  double A = 0.0;
  for (int32_t i = off[v]; i < off[v + 1]; ++i) {
    const int32_t* t = tris + 3 * (int64_t)inc[i];
    const int32_t q = t[0] == v ? t[1] : (t[1] == v ? t[2] : t[0]);
    const int32_t r = t[0] == v ? t[2] : (t[1] == v ? t[0] : t[1]);
    const V3 yq = ld3(y, q), yr = ld3(y, r);
    const double cq = nf_cot(p, yq, yr), cr = nf_cot(p, yr, yq);
    const V3 dq = vsub(yq, p), dr = vsub(yr, p);
    L = V3{L.x + cr * dq.x, L.y + cr * dq.y, L.z + cr * dq.z};
    L = V3{L.x + cq * dr.x, L.y + cq * dr.y, L.z + cq * dr.z};
    const V3 k = vcross(dq, dr);
    A = A + (0.5 * sqrt(vdot(k, k))) / 3.0;
  }
  V3 o = p;
  if (A > 0.0) {
    const double d = 2.0 * A;
    o = V3{p.x + alpha * (L.x / d), p.y + alpha * (L.y / d), p.z + alpha * (L.z / d)};
  }
  st3(yo, v, o);
}

template <class T>
int fgrow(T** p, int64_t n) {
  if (*p) (void)hipFree((void*)*p);
  *p = nullptr;
  if (hipMalloc((void**)p, (size_t)(n > 0 ? n : 1) * sizeof(T)) != hipSuccess) return CC_ENOMEM;
  return CC_OK;
}

}  // namespace

void flow_free(FlowWork* w) {
  if (!w) return;
  (void)hipFree(w->cnt);
  (void)hipFree(w->cur);
  (void)hipFree(w->inc);
  (void)hipFree(w->tmp);
  (void)hipFree(w->err);
  delete w;
}

int normal_flow_target(cc_context* ctx, const double* x, int32_t n, const int32_t* tris,
                       int32_t nt, double beta, double alpha, int32_t iters, double* y,
                       hipStream_t st) {
  if (n < 0 || nt < 0 || iters < 0 || (n > 0 && (!x || !y)) || (nt > 0 && !tris)) return CC_EINVAL;
  if (!std::isfinite(beta) || !std::isfinite(alpha)) return CC_EINVAL;
  if ((int64_t)nt * 3 > (int64_t)INT32_MAX) return CC_EINVAL;
  if (n == 0) return CC_OK;
  if (!ctx->flow) ctx->flow = new FlowWork();
  FlowWork& w = *ctx->flow;
  if (n > w.capN) {
    CC_TRY(fgrow(&w.cnt, (int64_t)n + 1));
    CC_TRY(fgrow(&w.cur, n));
    CC_TRY(fgrow(&w.tmp, 3 * (int64_t)n));
    w.capN = n;
  }
  if (3 * nt > w.capC) {
    CC_TRY(fgrow(&w.inc, 3 * (int64_t)nt));
    w.capC = 3 * nt;
  }
  if (!w.err) CC_TRY(fgrow(&w.err, 1));
  const int64_t n3 = 3 * (int64_t)nt;
  CC_HIP(hipMemsetAsync(w.cnt, 0, sizeof(int32_t) * ((size_t)n + 1), st));
  CC_HIP(hipMemsetAsync(w.err, 0, sizeof(int32_t), st));
  if (n3 > 0) k_nf_count<<<fblk(n3), kFlowThreads, 0, st>>>(tris, n3, n, w.cnt, w.err);
  CC_HIP(hipGetLastError());
  std::vector<int32_t> off((size_t)n + 1);
  int32_t herr = 0;
  CC_HIP(hipMemcpyAsync(off.data(), w.cnt, sizeof(int32_t) * off.size(), hipMemcpyDeviceToHost, st));
  CC_HIP(hipMemcpyAsync(&herr, w.err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (herr) return CC_EINVAL;
  for (int32_t v = 0; v < n; ++v) off[(size_t)v + 1] += off[(size_t)v];
  CC_HIP(hipMemcpyAsync(w.cnt, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, st));
  CC_HIP(hipMemcpyAsync(w.cur, w.cnt, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
  if (n3 > 0) {
    k_nf_fill<<<fblk(n3), kFlowThreads, 0, st>>>(tris, n3, w.cur, w.inc);
    k_nf_sort<<<fblk(n), kFlowThreads, 0, st>>>(w.cnt, n, w.inc);
  }
  // the last of the ping-pong writes lands in y
  double* a = (iters % 2 == 0) ? y : w.tmp;
  double* b = (iters % 2 == 0) ? w.tmp : y;
  k_nf_offset<<<fblk(n), kFlowThreads, 0, st>>>(x, tris, w.cnt, w.inc, n, beta, a);
  for (int32_t it = 0; it < iters; ++it) {
    k_nf_smooth<<<fblk(n), kFlowThreads, 0, st>>>(a, tris, w.cnt, w.inc, n, alpha, b);
    std::swap(a, b);
  }
  CC_HIP(hipGetLastError());
  CC_HIP(hipStreamSynchronize(st));  // the host offsets above must outlive their copy
  return CC_OK;
}

// ---- the target without allocation --------------------------------------------
// For callers that cannot allocate device memory (HIP graph capture, tight serving
// loops): the same kernels on a fixed scratch array compiled into the library, one
// copy per device, sized for kNfStaticVerts vertices and kNfStaticTris triangles.
// Its address on each device is looked up once, when a context for that device is
// created, and only that address is handed to kernels and copies.

namespace {

constexpr int32_t kNfStaticVerts = 1 << 17;
constexpr int32_t kNfStaticTris = 1 << 18;
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNfOffCnt = 0;
constexpr size_t kNfOffCur = kNfOffCnt + al256(sizeof(int32_t) * ((size_t)kNfStaticVerts + 1));
constexpr size_t kNfOffInc = kNfOffCur + al256(sizeof(int32_t) * (size_t)kNfStaticVerts);
constexpr size_t kNfOffTmp = kNfOffInc + al256(sizeof(int32_t) * 3 * (size_t)kNfStaticTris);
constexpr size_t kNfOffErr = kNfOffTmp + al256(sizeof(double) * 3 * (size_t)kNfStaticVerts);
constexpr size_t kNfScratchBytes = kNfOffErr + 256;

__global__ void k_nf_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per triangle: a triangle with a vertex outside [0, n) sets the error flag and is
// left out, so no later kernel reads through its indices.
__device__ __forceinline__ bool nf_tri_ok(const int32_t* t, int32_t n) {
  return t[0] >= 0 && t[0] < n && t[1] >= 0 && t[1] < n && t[2] >= 0 && t[2] < n;
}

__global__ void k_nf_count_tri(const int32_t* __restrict__ tris, int32_t nt, int32_t n,
                               int32_t* __restrict__ cnt, int32_t* err) {
  const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nt) return;
  const int32_t* t = tris + 3 * (int64_t)f;
  if (!nf_tri_ok(t, n)) {
    atomicOr(err, 1);
    return;
  }
  for (int k = 0; k < 3; ++k) atomicAdd(&cnt[t[k] + 1], 1);
}

__global__ void k_nf_fill_tri(const int32_t* __restrict__ tris, int32_t nt, int32_t n,
                              int32_t* __restrict__ cur, int32_t* __restrict__ inc) {
  const int32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nt) return;
  const int32_t* t = tris + 3 * (int64_t)f;
  if (!nf_tri_ok(t, n)) return;
  for (int k = 0; k < 3; ++k) inc[atomicAdd(&cur[t[k]], 1)] = f;
}

// In-place inclusive prefix sum of cnt[0..m) (cnt[0] = 0: the offsets) by one block
// of kFlowThreads threads, kFlowThreads entries at a time with a running carry; the
// fill cursors cur[0..m-1) start as a copy of the offsets.
__global__ void __launch_bounds__(kFlowThreads) k_nf_scan(int32_t* __restrict__ cnt, int32_t m,
                                                          int32_t* __restrict__ cur) {
  __shared__ int32_t part[kFlowThreads];
  int32_t carry = 0;
  for (int32_t b = 0; b < m; b += kFlowThreads) {
    const int32_t i = b + (int32_t)threadIdx.x;
    int32_t v = i < m ? cnt[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kFlowThreads; o <<= 1) {
      const int32_t t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    v = part[threadIdx.x] + carry;
    if (i < m) {
      cnt[i] = v;
      if (i + 1 < m) cur[i] = v;
    }
    const int32_t total = part[kFlowThreads - 1];
    __syncthreads();
    carry += total;
  }
}

}  // namespace

// file-scope device array (about 7 MiB per device, held until the process ends); in
// host code its name is only a stand-in: kernels and copies get g_scratch[device]
static __device__ __align__(256) unsigned char scratch[kNfScratchBytes];

static constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device
static std::mutex g_scratch_mu;

int flow_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return CC_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return CC_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CC_EHIP;
  g_scratch[device] = p;
  return CC_OK;
}

int normal_flow_target_static(int device, const double* x, int32_t n, const int32_t* tris,
                              int32_t nt, double beta, double alpha, int32_t iters, double* y,
                              hipStream_t st) {
  if (n < 0 || nt < 0 || iters < 0 || (n > 0 && (!x || !y)) || (nt > 0 && !tris)) return CC_EINVAL;
  if (!std::isfinite(beta) || !std::isfinite(alpha)) return CC_EINVAL;
  if (n > kNfStaticVerts || nt > kNfStaticTris) return CC_EINVAL;
  if (n == 0) return CC_OK;
  void* base = nullptr;
  if (device >= 0 && device < kMaxDevices) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = g_scratch[device];
  }
  if (!base) return CC_ESTATE;  // no context was created for this device
  unsigned char* b = (unsigned char*)base;
  int32_t* cnt = (int32_t*)(b + kNfOffCnt);
  int32_t* cur = (int32_t*)(b + kNfOffCur);
  int32_t* inc = (int32_t*)(b + kNfOffInc);
  double* tmp = (double*)(b + kNfOffTmp);
  int32_t* err = (int32_t*)(b + kNfOffErr);
  // the array keeps the last call's contents: counts and the error flag start at 0
  k_nf_fill_i32<<<fblk((int64_t)n + 1), kFlowThreads, 0, st>>>(cnt, (int64_t)n + 1, 0);
  k_nf_fill_i32<<<1, kFlowThreads, 0, st>>>(err, 1, 0);
  if (nt > 0) k_nf_count_tri<<<fblk(nt), kFlowThreads, 0, st>>>(tris, nt, n, cnt, err);
  k_nf_scan<<<1, kFlowThreads, 0, st>>>(cnt, n + 1, cur);
  if (nt > 0) {
    k_nf_fill_tri<<<fblk(nt), kFlowThreads, 0, st>>>(tris, nt, n, cur, inc);
    k_nf_sort<<<fblk(n), kFlowThreads, 0, st>>>(cnt, n, inc);
  }
  double* a = (iters % 2 == 0) ? y : tmp;
  double* c = (iters % 2 == 0) ? tmp : y;
  k_nf_offset<<<fblk(n), kFlowThreads, 0, st>>>(x, tris, cnt, inc, n, beta, a);
  for (int32_t it = 0; it < iters; ++it) {
    k_nf_smooth<<<fblk(n), kFlowThreads, 0, st>>>(a, tris, cnt, inc, n, alpha, c);
    std::swap(a, c);
  }
  CC_HIP(hipGetLastError());
  int32_t herr = 0;
  CC_HIP(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  return herr ? CC_EINVAL : CC_OK;
}

}  // namespace cc
