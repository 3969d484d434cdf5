// C ABI of the two-way collision-handling step: contexts, solvers and the host
// loop of Alg. 1 that sequences the HIP kernels on the caller's stream.
//
// A solver is a multi-scene engine: scenes (segments) occupy disjoint index
// ranges of one set of device arrays, and every kernel launch of an iteration
// covers all iterating scenes at once. Each scene keeps its own D, its own stop
// test and its own iteration count; its kernels read and write only its own
// ranges (pairs, rows and colours never mix scenes, and colouring priorities use
// scene-local keys), so a scene's result does not depend on which other scenes
// share the engine. cc_collide_step is a one-scene engine.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <mutex>
#include <thread>

#include "internal.hpp"

using namespace cc;

namespace {

template <class T>
int dalloc(T** p, int64_t n) {
  if (n <= 0) n = 1;
  if (hipMalloc((void**)p, (size_t)n * sizeof(T)) != hipSuccess) return CC_ENOMEM;
  return CC_OK;
}
template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}
// Replace *p by an allocation of n elements holding its first `keep` elements.
template <class T>
int dregrow(T** p, int64_t n, int64_t keep, hipStream_t st) {
  T* q = nullptr;
  CC_TRY(dalloc(&q, n));
  if (*p && keep > 0) CC_HIP(hipMemcpyAsync(q, *p, sizeof(T) * keep, hipMemcpyDeviceToDevice, st));
  CC_HIP(hipStreamSynchronize(st));
  dfree(*p);
  *p = q;
  return CC_OK;
}

hipStream_t as_stream(void* st) { return (hipStream_t)st; }

double bits2d(unsigned long long b) {
  double d;
  memcpy(&d, &b, sizeof d);
  return d;
}
unsigned long long d2bits(double d) {
  unsigned long long b;
  memcpy(&b, &d, sizeof b);
  return b;
}

}  // namespace

namespace cc {

int check_params(const cc_params* p) {
  if (!p) return CC_EINVAL;
  if (!(p->delta > 0.0) || !(p->d_min >= p->delta) || !(p->d_max > p->d_min)) return CC_EINVAL;
  if (!(p->sigma >= 1.0) || !(p->gamma > 0.0 && p->gamma < 1.0) || !(p->eps > 0.0)) return CC_EINVAL;
  if (!(p->kappa >= 0.0)) return CC_EINVAL;
  if (p->max_iters < 1 || p->gs_sweeps < 1) return CC_EINVAL;
  if (p->max_colors < 1 || p->max_colors > kMaxColors) return CC_EINVAL;
  if (p->backward != CC_GAUSS_SEIDEL && p->backward != CC_JACOBI) return CC_EINVAL;
  if ((p->flags & CC_TIME_ONE) && (p->time_kind < 0 || p->time_kind >= CC_K_COUNT)) return CC_EINVAL;
  if (p->backward == CC_JACOBI && (!(p->omega > 0.0 && p->omega <= 1.0) || (p->flags & CC_MIXED)))
    return CC_EINVAL;
  if ((p->flags & CC_CCD_STEP) && (p->flags & CC_MIXED)) return CC_EINVAL;
  return CC_OK;
}

// ---------------------------------------------------------------- autotuner

// Launch shapes measured on the first launch of a (device, kernel, size class) and
// kept for the process: every variant computes the same result, so the choice only
// changes the time. Process-wide, shared by every context.
namespace {
std::mutex g_tune_mu;
std::vector<cc_tune_entry> g_tune;
int g_tune_force[1] = {0};  // per kernel: a forced choice (0: none)
}  // namespace

int tune_lookup(int device, int kernel, int32_t size_class) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (kernel >= 0 && kernel < 1 && g_tune_force[kernel] > 0) return g_tune_force[kernel];
  for (const cc_tune_entry& e : g_tune)
    if (e.device == device && e.kernel == kernel && e.size_class == size_class) return e.choice;
  return -1;
}

void tune_store(int device, int kernel, int32_t size_class, int choice, const float ms[8]) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  cc_tune_entry e{};
  e.device = device;
  e.kernel = kernel;
  e.size_class = size_class;
  e.choice = choice;
  for (int i = 0; i < 8; ++i) e.ms[i] = ms[i];
  g_tune.push_back(e);
}

// ---------------------------------------------------------------- ranges

int32_t RangeAlloc::take(int32_t len) {
  if (len <= 0) return 0;
  for (size_t i = 0; i < free_.size(); ++i) {
    if (free_[i].second < len) continue;
    const int32_t start = free_[i].first;
    free_[i].first += len;
    free_[i].second -= len;
    if (free_[i].second == 0) free_.erase(free_.begin() + i);
    return start;
  }
  return -1;
}

void RangeAlloc::give(int32_t start, int32_t len) {
  if (len <= 0) return;
  auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(start, 0));
  it = free_.insert(it, {start, len});
  size_t i = it - free_.begin();
  if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
    free_[i].second += free_[i + 1].second;
    free_.erase(free_.begin() + i + 1);
  }
  if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
    free_[i - 1].second += free_[i].second;
    free_.erase(free_.begin() + i);
  }
}

void RangeAlloc::grow(int32_t new_cap) {
  if (new_cap <= cap) return;
  const int32_t old = cap;
  cap = new_cap;
  give(old, new_cap - old);
}

int32_t RangeAlloc::extent() const {
  if (!free_.empty() && free_.back().first + free_.back().second == cap) return free_.back().first;
  return cap;
}

}  // namespace cc

namespace {

void free_pairs(cc_solver* s) {
  dfree(s->P); dfree(s->P2); dfree(s->dP); dfree(s->dP2);
}
void free_active(cc_solver* s) {
  dfree(s->Akeys); dfree(s->Averts); dfree(s->Acol); dfree(s->Aorder);
  dfree(s->list0); dfree(s->list1); dfree(s->lamA); dfree(s->afail); dfree(s->apick);
  dfree(s->Arow); dfree(s->Aslot); dfree(s->lvert);
}

// Pair buffers of capacity cap; the first `keep` keys of P survive.
int alloc_pairs(cc_solver* s, int64_t cap, int64_t keep, hipStream_t st) {
  s->mv_gen = ~0ull;  // the stored distances do not survive
  CC_TRY(dregrow(&s->P, cap, keep, st));
  dfree(s->P2); dfree(s->dP); dfree(s->dP2);
  s->capP = cap;
  CC_TRY(dalloc(&s->P2, cap));
  CC_TRY(dalloc(&s->dP, cap));
  CC_TRY(dalloc(&s->dP2, cap));
  return CC_OK;
}

int alloc_active(cc_solver* s, int64_t cap) {
  free_active(s);
  s->capA = cap;
  CC_TRY(dalloc(&s->Akeys, cap));
  CC_TRY(dalloc(&s->Averts, cap));
  CC_TRY(dalloc(&s->Acol, cap));
  CC_TRY(dalloc(&s->Aorder, cap));
  CC_TRY(dalloc(&s->list0, cap));
  CC_TRY(dalloc(&s->list1, cap));
  CC_TRY(dalloc(&s->lamA, cap));
  CC_TRY(dalloc(&s->afail, cap));
  CC_TRY(dalloc(&s->apick, cap));
  CC_TRY(dalloc(&s->Arow, cap * kRowWords));
  CC_TRY(dalloc(&s->Aslot, cap));
  CC_TRY(dalloc(&s->lvert, (int64_t)kLocCap1));
  return CC_OK;
}

void free_vertex_arrays(cc_solver* s) {
  dfree(s->w); dfree(s->stat); dfree(s->x); dfree(s->y); dfree(s->xt); dfree(s->xold);
  dfree(s->rold); dfree(s->dyold); dfree(s->back); dfree(s->alph); dfree(s->scale);
  dfree(s->r); dfree(s->move2); dfree(s->mvd); dfree(s->Di); dfree(s->vseg); dfree(s->plist); dfree(s->dy);
  dfree(s->jacc);
  dfree(s->vmax0); dfree(s->claims); dfree(s->masks);
}
void free_edge_arrays(cc_solver* s) {
  dfree(s->edges); dfree(s->eseg); dfree(s->eg); dfree(s->einv); dfree(s->ecol); dfree(s->eorder);
  dfree(s->eij);
  dfree(s->elist0); dfree(s->elist1); dfree(s->elist2); dfree(s->lamE);
  dfree(s->efail); dfree(s->epick);
}

void solver_free(cc_solver* s) {
  free_vertex_arrays(s);
  free_edge_arrays(s);
  dfree(s->tris);
  free_pairs(s);
  free_active(s);
  dfree(s->col_cnt); dfree(s->rcnt); dfree(s->coff_dev); dfree(s->ecoff_dev);
  bvh_free(s);
  if (s->sel_host) (void)hipHostFree(s->sel_host);
  s->sel_host = nullptr;
  ecache_free(s);
  dfree(s->mirror_dev);
  if (s->mirror_host) (void)hipHostFree(s->mirror_host);
  s->mirror_host = nullptr;
  s->dc = nullptr;
  s->hc = nullptr;
  s->seg_dev = nullptr;
  s->seg_host = nullptr;
  s->stripe = nullptr;
  s->hstripe = nullptr;
  for (auto& t : s->timers) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  s->timers.clear();
  for (auto e : s->event_pool) (void)hipEventDestroy(e);
  s->event_pool.clear();
}

// Per-vertex, per-triangle and per-edge arrays at the given capacities; the
// live contents (state, masses, topology, segment ids, edge rows) of the first
// old-capacity elements are kept. Scratch arrays and the search tree are
// reallocated empty.
int resize_arrays(cc_solver* s, int32_t capV, int32_t capF, int32_t capE, hipStream_t st) {
  const int64_t oV = s->capV, oF = s->capF, oE = s->capE;
  s->ecache.ok = false;
  // pair keys hold primitive ids in 30 bits
  if (capV > kMaxIds || capF > kMaxIds || capE > kMaxIds) return CC_ENOMEM;
  if (capV != oV) {
    CC_TRY(dregrow(&s->w, capV, oV, st));
    CC_TRY(dregrow(&s->stat, capV, oV, st));
    CC_TRY(dregrow(&s->x, 3 * (int64_t)capV, 3 * oV, st));
    CC_TRY(dregrow(&s->y, 3 * (int64_t)capV, 3 * oV, st));
    CC_TRY(dregrow(&s->xt, 3 * (int64_t)capV, 3 * oV, st));
    CC_TRY(dregrow(&s->r, capV, oV, st));
    CC_TRY(dregrow(&s->dy, 3 * (int64_t)capV, 3 * oV, st));
    dfree(s->jacc);
    CC_TRY(dalloc(&s->jacc, 3 * (int64_t)capV));
    CC_HIP(hipMemsetAsync(s->jacc, 0, sizeof(long long) * 3 * (size_t)capV, st));
    CC_TRY(dregrow(&s->vseg, capV, oV, st));
    CC_TRY(launch_fill_i32(s->vseg + oV, capV - oV, -1, st));
    CC_TRY(dregrow(&s->plist, capV, oV, st));
    dfree(s->xold); dfree(s->move2); dfree(s->Di); dfree(s->vmax0); dfree(s->claims); dfree(s->masks);
    dfree(s->rold); dfree(s->dyold); dfree(s->back); dfree(s->alph); dfree(s->scale);
    CC_TRY(dalloc(&s->alph, capV));
    CC_TRY(dalloc(&s->scale, capV));
    CC_TRY(launch_fill_u64(s->scale, capV, kOneBits, st));
    CC_TRY(dalloc(&s->rold, capV));
    CC_TRY(dalloc(&s->dyold, 3 * (int64_t)capV));
    CC_TRY(dalloc(&s->back, capV));
    CC_TRY(launch_fill_i32(s->back, capV, 0, st));
    CC_TRY(dalloc(&s->xold, 3 * (int64_t)capV));
    CC_TRY(dalloc(&s->move2, capV));
    dfree(s->mvd);
    CC_TRY(dalloc(&s->mvd, capV));
    s->mv_gen = ~0ull;
    CC_TRY(dalloc(&s->Di, capV));
    CC_TRY(dalloc(&s->vmax0, capV));
    CC_TRY(dalloc(&s->claims, (int64_t)capV * 2 * kMaskWords));
    // the colouring counts and claims start at zero over the whole capacity: a later
    // scene may reach vertices beyond the extent in use now
    CC_HIP(hipMemsetAsync(s->vmax0, 0, sizeof(unsigned long long) * (size_t)capV, st));
    CC_HIP(hipMemsetAsync(s->claims, 0, sizeof(unsigned long long) * (size_t)capV * 2 * kMaskWords, st));
    s->pc_dirty = false;
    CC_TRY(dalloc(&s->masks, (int64_t)capV * kMaskWords));
  }
  if (capF != oF) CC_TRY(dregrow(&s->tris, 3 * (int64_t)capF, 3 * oF, st));
  if (capE != oE) {
    CC_TRY(dregrow(&s->edges, 2 * (int64_t)capE, 2 * oE, st));
    CC_TRY(dregrow(&s->eseg, capE, oE, st));
    CC_TRY(launch_fill_i32(s->eseg + oE, capE - oE, -1, st));
    CC_TRY(dregrow(&s->eg, 3 * (int64_t)capE, 3 * oE, st));
    CC_TRY(dregrow(&s->einv, capE, oE, st));
    CC_TRY(dregrow(&s->ecol, capE, oE, st));
    dfree(s->eorder); dfree(s->elist0); dfree(s->elist1); dfree(s->elist2); dfree(s->lamE);
    dfree(s->eij);
    CC_TRY(dalloc(&s->eorder, capE));
    CC_TRY(dalloc(&s->eij, capE));
    CC_TRY(dalloc(&s->elist0, capE));
    CC_TRY(dalloc(&s->elist1, capE));
    CC_TRY(dalloc(&s->elist2, capE));
    CC_TRY(dalloc(&s->lamE, capE));
    dfree(s->efail); dfree(s->epick);
    CC_TRY(dalloc(&s->efail, capE));
    CC_TRY(dalloc(&s->epick, capE));
    s->erows_dirty = true;
  }
  s->capV = capV;
  s->capF = capF;
  s->capE = capE;
  bvh_free(s);
  CC_TRY(bvh_alloc(s));
  s->ra_v.grow(capV);
  s->ra_f.grow(capF);
  s->ra_e.grow(capE);
  CC_HIP(hipStreamSynchronize(st));
  return CC_OK;
}

int solver_alloc(cc_solver* s, int32_t capV, int32_t capF, int32_t capE, hipStream_t st) {
  CC_TRY(dalloc(&s->col_cnt, kMaxColors + 1));
  CC_TRY(dalloc(&s->rcnt, kMaxRounds + 1));
  CC_TRY(dalloc(&s->coff_dev, kMaxColors + 1));
  CC_TRY(dalloc(&s->ecoff_dev, kMaxColors + 1));
  static_assert(sizeof(Counters) <= kMirrorSeg - kMirrorCounters, "counters fit their slot");
  static_assert(kMirrorCounters >= 64 * 16 * sizeof(unsigned long long), "stripes fit theirs");
  const size_t mbytes = kMirrorSeg + sizeof(SegDev) * kMaxSeg;
  CC_TRY(dalloc(&s->mirror_dev, (int64_t)mbytes));
  if (hipHostMalloc((void**)&s->mirror_host, mbytes, hipHostMallocDefault) != hipSuccess) {
    s->mirror_host = nullptr;
    return CC_ENOMEM;
  }
  memset(s->mirror_host, 0, mbytes);
  s->stripe = reinterpret_cast<unsigned long long*>(s->mirror_dev + kMirrorStripe);
  s->hstripe = reinterpret_cast<unsigned long long*>(s->mirror_host + kMirrorStripe);
  s->dc = reinterpret_cast<Counters*>(s->mirror_dev + kMirrorCounters);
  s->hc = reinterpret_cast<Counters*>(s->mirror_host + kMirrorCounters);
  s->seg_dev = reinterpret_cast<SegDev*>(s->mirror_dev + kMirrorSeg);
  s->seg_host = reinterpret_cast<SegDev*>(s->mirror_host + kMirrorSeg);
  CC_TRY(resize_arrays(s, std::max(capV, 1), std::max(capF, 1), std::max(capE, 1), st));
  const int64_t cap = std::max<int64_t>(4096, 32 * ((int64_t)capV + capE));
  CC_TRY(alloc_pairs(s, cap, 0, st));
  CC_TRY(alloc_active(s, std::max<int64_t>(4096, cap / 8)));
  return CC_OK;
}

void resolve_timers(cc_solver* s) {
  for (auto& t : s->timers) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      s->st.kernel_ms[t.kind] += ms;
      s->st.kernel_launches[t.kind] += 1;
    }
    s->event_pool.push_back(t.a);
    s->event_pool.push_back(t.b);
  }
  s->timers.clear();
}

}  // namespace

namespace cc {

hipEvent_t pool_event(cc_solver* s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void timer_begin(cc_solver* s, int kind, hipStream_t st) {
  s->timer_open = false;
  if (!(s->p.flags & CC_TIME_KERNELS) &&
      !((s->p.flags & CC_TIME_ONE) && kind == s->p.time_kind))
    return;
  Timer t;
  t.kind = kind;
  t.a = pool_event(s);
  t.b = pool_event(s);
  (void)hipEventRecord(t.a, st);
  s->timers.push_back(t);
  s->timer_open = true;
}

void timer_end(cc_solver* s, hipStream_t st) {
  if (!s->timer_open || s->timers.empty()) return;
  (void)hipEventRecord(s->timers.back().b, st);
  s->timer_open = false;
}

// ---------------------------------------------------------------- engine

int engine_create(cc_context* ctx, const cc_params* params, int32_t capV, int32_t capF,
                  int32_t capE, cc_solver** out, hipStream_t st) {
  CC_TRY(check_params(params));
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  cc_solver* s = new cc_solver();
  s->ctx = ctx;
  s->p = *params;
  s->kappa2 = params->kappa * params->kappa;
  int rc = solver_alloc(s, capV, capF, capE, st);
  if (rc != CC_OK) {
    solver_free(s);
    delete s;
    return rc;
  }
  *out = s;
  return CC_OK;
}

void engine_set_params(cc_solver* s, const cc_params* params) {
  s->p = *params;
  s->kappa2 = params->kappa * params->kappa;
}

static void update_extents(cc_solver* s) {
  s->n = s->ra_v.extent();
  s->nt = s->ra_f.extent();
  s->ne = s->ra_e.extent();
}

void release_pending(cc_solver* s) {
  for (const auto& f : s->pending_free) {
    if (f[0] == 0) s->ra_v.give(f[1], f[2]);
    else if (f[0] == 1) s->ra_f.give(f[1], f[2]);
    else s->ra_e.give(f[1], f[2]);
  }
  s->pending_free.clear();
  update_extents(s);
}

// Every side of every triangle of segment sg must be one of its edges, or edge-edge
// pairs would miss contacts; checked when the input check is on (CC_EINVAL).
static int check_tri_edges(cc_solver* s, int32_t sg, hipStream_t st) {
  const Seg& g = s->segs[sg];
  if (g.nf == 0) return CC_OK;
  std::vector<int32_t> t(3 * (size_t)g.nf), e(2 * (size_t)g.ne);
  CC_HIP(hipMemcpyAsync(t.data(), s->tris + 3 * (int64_t)g.fb, sizeof(int32_t) * t.size(),
                        hipMemcpyDeviceToHost, st));
  if (g.ne > 0)
    CC_HIP(hipMemcpyAsync(e.data(), s->edges + 2 * (int64_t)g.eb, sizeof(int32_t) * e.size(),
                          hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  auto key = [](int32_t a, int32_t b) {
    return a < b ? ((uint64_t)(uint32_t)a << 32) | (uint32_t)b : ((uint64_t)(uint32_t)b << 32) | (uint32_t)a;
  };
  std::vector<uint64_t> ek((size_t)g.ne);
  for (int32_t i = 0; i < g.ne; ++i) ek[(size_t)i] = key(e[2 * (size_t)i], e[2 * (size_t)i + 1]);
  std::sort(ek.begin(), ek.end());
  for (int32_t f = 0; f < g.nf; ++f)
    for (int k = 0; k < 3; ++k)
      if (!std::binary_search(ek.begin(), ek.end(),
                              key(t[3 * (size_t)f + k], t[3 * (size_t)f + (k + 1) % 3])))
        return CC_EINVAL;
  return CC_OK;
}

int seg_add(cc_solver* s, int32_t nv, const double* inv_mass, const int32_t* tris, int32_t nf,
            const int32_t* edges, int32_t ne, int32_t max_iters, int32_t* out, hipStream_t st) {
  if (nv < 0 || nf < 0 || ne < 0 || !out) return CC_EINVAL;
  if ((nf > 0 && !tris) || (ne > 0 && !edges)) return CC_EINVAL;
  ++s->gen;
  int32_t sg = -1;
  for (int32_t i = 0; i < (int32_t)s->segs.size(); ++i)
    if (!s->segs[i].live && !s->segs[i].pending) {
      sg = i;
      break;
    }
  if (sg < 0) {
    if ((int32_t)s->segs.size() >= kMaxSeg) return CC_EAGAIN;
    s->segs.push_back(Seg{});
    sg = (int32_t)s->segs.size() - 1;
  }
  int32_t vb = s->ra_v.take(nv), fb = s->ra_f.take(nf), eb = s->ra_e.take(ne);
  if (vb < 0 || fb < 0 || eb < 0) {
    if (vb >= 0) s->ra_v.give(vb, nv);
    if (fb >= 0) s->ra_f.give(fb, nf);
    if (eb >= 0) s->ra_e.give(eb, ne);
    const int32_t cv = vb < 0 ? std::max(s->capV + nv, 2 * s->capV) : s->capV;
    const int32_t cf = fb < 0 ? std::max(s->capF + nf, 2 * s->capF) : s->capF;
    const int32_t ce = eb < 0 ? std::max(s->capE + ne, 2 * s->capE) : s->capE;
    CC_TRY(resize_arrays(s, cv, cf, ce, st));
    vb = s->ra_v.take(nv);
    fb = s->ra_f.take(nf);
    eb = s->ra_e.take(ne);
    if (vb < 0 || fb < 0 || eb < 0) return CC_ENOMEM;
  }
  Seg& g = s->segs[sg];
  g = Seg{};
  g.vb = vb;
  g.nv = nv;
  g.fb = fb;
  g.nf = nf;
  g.eb = eb;
  g.ne = ne;
  g.max_iters = max_iters;
  g.live = true;
  update_extents(s);
  int rc = CC_OK;
  if (nv > 0) {
    if (inv_mass)
      rc = hipMemcpyAsync(s->w + vb, inv_mass, sizeof(double) * nv, hipMemcpyDefault, st) == hipSuccess
               ? CC_OK : CC_EHIP;
    else
      rc = launch_fill_u64((unsigned long long*)(s->w + vb), nv, d2bits(1.0), st);
    if (rc == CC_OK) rc = launch_fill_i32(s->vseg + vb, nv, sg, st);
  }
  if (rc == CC_OK) rc = launch_topo_in(s, sg, tris, edges, st);
  if (rc == CC_OK && (s->p.flags & CC_VALIDATE_INPUT)) rc = check_tri_edges(s, sg, st);
  if (rc == CC_OK) rc = launch_particles(s, sg, st);
  if (rc == CC_OK) {
    // the search arrays hold every live segment's particles
    int64_t np = 0;
    for (const Seg& o : s->segs)
      if (o.live) np += o.np;
    if (np > s->capPt) {
      s->capPt = (int32_t)std::min<int64_t>(std::max<int64_t>(np, 2 * (int64_t)s->capPt), kMaxIds);
      bvh_free(s);
      rc = bvh_alloc(s);
    }
  }
  SegDev& d = s->seg_host[sg];
  memset(&d, 0, sizeof d);
  d.vb = vb;
  d.fb = fb;
  d.eb = eb;
  if (rc == CC_OK)
    rc = hipMemcpyAsync(s->seg_dev + sg, &d, sizeof d, hipMemcpyHostToDevice, st) == hipSuccess
             ? CC_OK : CC_EHIP;
  if (rc == CC_OK) rc = hipStreamSynchronize(st) == hipSuccess ? CC_OK : CC_EHIP;
  if (rc != CC_OK) {
    seg_remove(s, sg, st);
    return rc;
  }
  *out = sg;
  return CC_OK;
}

int seg_remove(cc_solver* s, int32_t sg, hipStream_t st) {
  if (sg < 0 || sg >= (int32_t)s->segs.size() || !s->segs[sg].live) return CC_EINVAL;
  ++s->gen;
  Seg& g = s->segs[sg];
  CC_TRY(launch_fill_i32(s->vseg + g.vb, g.nv, -1, st));
  CC_TRY(launch_fill_i32(s->eseg + g.eb, g.ne, -1, st));
  g.live = false;
  g.active = false;
  g.pending = true;
  s->seg_host[sg].flags = 0;
  CC_HIP(hipMemcpyAsync(s->seg_dev + sg, s->seg_host + sg, sizeof(SegDev), hipMemcpyHostToDevice, st));
  // the ranges return to the allocator once no pair of P can refer to them
  s->pending_free.push_back({0, g.vb, g.nv});
  s->pending_free.push_back({1, g.fb, g.nf});
  s->pending_free.push_back({2, g.eb, g.ne});
  s->pending_segs.push_back(sg);
  s->erows_dirty = true;
  CC_HIP(hipStreamSynchronize(st));
  if (s->nP == 0) {
    release_pending(s);
    for (int32_t q : s->pending_segs) s->segs[q].pending = false;
    s->pending_segs.clear();
  }
  return CC_OK;
}

static void release_all_pending(cc_solver* s) {
  release_pending(s);
  for (int32_t q : s->pending_segs) s->segs[q].pending = false;
  s->pending_segs.clear();
}

// Alg. 1 initialisation of k segments at once: x <- x^[k] (x_prev[i], or the
// segment's resident x when NULL), y <- y^[k+1], D <- 0, r <- 1, the edge-length
// rows at y^[k+1] and their colouring. rc[i] gets each segment's result.
int seg_begin(cc_solver* s, const int32_t* sgs, int32_t k, const double* const* x_prev,
              const double* const* x_tilde, int* rc, hipStream_t st) {
  ++s->gen;  // new positions: the next search builds its tree anew
  CC_HIP(hipMemsetAsync(&s->dc->n_rows, 0, sizeof(unsigned long long), st));
  std::vector<int32_t> ok;
  for (int32_t i = 0; i < k; ++i) {
    const int32_t sg = sgs[i];
    Seg& g = s->segs[sg];
    if (!g.live || (g.nv > 0 && !x_tilde[i])) {
      rc[i] = CC_EINVAL;
      continue;
    }
    const double* xp = x_prev[i] ? x_prev[i] : s->x + 3 * (int64_t)g.vb;
    rc[i] = launch_check_finite(s, xp, x_tilde[i], g.nv, st);
    if (rc[i] != CC_OK) continue;
    rc[i] = launch_setup(s, sg, xp, x_tilde[i], st);
    if (rc[i] == CC_OK && (s->p.flags & CC_VALIDATE_INPUT)) {
      // x^[k] must lie in the free space (Sec. 3): no pair within kFreeTol, no
      // edge through a triangle
      int bad = 0;
      s->sel_host[0].seg = sg;
      rc[i] = lbvh_validate(s, 1, s->x, kFreeTol, &bad, st);
      if (rc[i] == CC_OK && bad) rc[i] = CC_ENOTFREE;
    }
    if (rc[i] == CC_OK) ok.push_back(i);
  }
  // a lone scene whose edges, rows, free vertices, seed and palette repeat those of
  // its last edge colouring keeps that colouring (checked element by element)
  const bool lone = k == 1 && ok.size() == 1 && sgs[0] == 0 && s->segs.size() == 1 &&
                    s->segs[0].vb == 0 && s->segs[0].eb == 0 && s->pending_segs.empty();
  const cc_solver::EdgeColourCache& ec = s->ecache;
  const bool ec_try = lone && ec.ok && ec.seed == s->p.seed && ec.maxc == s->p.max_colors &&
                      ec.ne == s->segs[0].ne && ec.nv == s->segs[0].nv;
  if (ec_try) CC_TRY(ecache_compare(s, st));
  CC_HIP(hipMemcpyAsync(&s->hc->n_rows, &s->dc->n_rows, sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, st));
  if (ec_try)
    CC_HIP(hipMemcpyAsync(&s->hc->ecmis, &s->dc->ecmis, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  s->n_newrows = (int32_t)s->hc->n_rows;
  int crc = CC_OK;
  if (s->p.backward != CC_JACOBI) {  // the Jacobi step needs no colours
    const bool reuse = ec_try && s->hc->ecmis == 0 && s->n_newrows == ec.rows;
    if (!reuse) {
      timer_begin(s, CC_K_COLOR, st);
      crc = color_edges_greedy(s, st);
      timer_end(s, st);
      if (crc == CC_OK && lone) crc = ecache_store(s, st);
    }
  }
  if (crc == CC_OK)
    crc = hipMemcpyAsync(s->seg_host, s->seg_dev, sizeof(SegDev) * s->segs.size(),
                         hipMemcpyDeviceToHost, st) == hipSuccess ? CC_OK : CC_EHIP;
  if (crc == CC_OK) crc = hipStreamSynchronize(st) == hipSuccess ? CC_OK : CC_EHIP;
  resolve_timers(s);
  for (int32_t i : ok) {
    if (crc != CC_OK) {
      rc[i] = crc;
      continue;
    }
    Seg& g = s->segs[sgs[i]];
    g.D = 0.0;
    g.begun = true;
    g.active = true;
    g.n_erows = (int32_t)s->seg_host[sgs[i]].n_rows;
    memset(&g.st, 0, sizeof g.st);
    g.st.status = CC_MAXITER;
    memset(&g.last, 0, sizeof g.last);
  }
  s->erows_dirty = true;
  return crc;
}

// One iteration of Alg. 1 for every iterating segment.
int engine_iterate(cc_solver* s, hipStream_t st) {
  const cc_params& p = s->p;
  const bool trace = (p.flags & CC_TRACE) != 0;
  const int32_t ns = (int32_t)s->segs.size();
  std::vector<int32_t> act, sel;
  std::vector<char> searched(ns, 0);
  for (int32_t i = 0; i < ns; ++i) {
    const Seg& g = s->segs[i];
    if (!(g.live && g.active)) continue;
    act.push_back(i);
    if (g.D < p.d_min) sel.push_back(i);
  }
  if (act.empty()) {
    s->nP = 0;
    release_all_pending(s);
    return CC_OK;
  }
  // proximity search of the segments whose reuse bound fell below D_min (Sec. 3.1)
  int64_t n_old = s->nP;
  int64_t n_search = 0;
  if (!sel.empty()) {
    if (sel.size() == act.size()) n_old = 0;  // every pair of P is replaced
    for (size_t r = 0; r < sel.size(); ++r) s->sel_host[r].seg = sel[r];
    for (int attempt = 0;; ++attempt) {
      int64_t nf = 0;
      CC_TRY(lbvh_search(s, (int32_t)sel.size(), s->x, p.d_max, s->P + n_old, s->dP + n_old,
                         s->capP - n_old, &nf, st, true));
      if (n_old + nf <= s->capP) {
        n_search = nf;
        break;
      }
      if (attempt > 0) return CC_EOVERFLOW;
      const int64_t need = n_old + nf;
      CC_TRY(alloc_pairs(s, need + need / 4 + 1024, n_old, st));
    }
    s->nP = n_old + n_search;
    for (int32_t sg : sel) {
      s->segs[sg].D = p.d_max;
      s->segs[sg].st.searches += 1;
      s->segs[sg].last.searched = 1;
      searched[sg] = 1;
    }
  }
  // segment records
  for (int32_t i = 0; i < ns; ++i) {
    const Seg& g = s->segs[i];
    SegDev& d = s->seg_host[i];
    const unsigned long long rows = d.n_rows;
    memset(&d, 0, sizeof d);
    d.n_rows = rows;
    d.D = g.D;
    d.D2 = g.D * g.D;
    d.vb = g.vb;
    d.fb = g.fb;
    d.eb = g.eb;
    d.flags = ((g.live && g.active) ? kSegActive : 0) | (searched[i] ? kSegSearched : 0);
  }
  CC_HIP(hipMemcpyAsync(s->seg_dev, s->seg_host, sizeof(SegDev) * ns, hipMemcpyHostToDevice, st));
  const bool jacobi = p.backward == CC_JACOBI;
  if (s->erows_dirty && !jacobi) CC_TRY(build_edge_buckets(s, st));
  // pair pass; regrow the active set if it overflowed. After a search of every
  // iterating scene each pair has d < D_max = D and stays in P': P' is P as it is.
  const bool in_place = !sel.empty() && n_old == 0;
  for (int attempt = 0;; ++attempt) {
    CC_TRY(launch_di_init(s, st));  // also clears the counters
    timer_begin(s, CC_K_PAIR, st);
    // pairs the search just found carry their distance at this x already
    CC_TRY(launch_pair_pass(s, n_old, sel.empty() ? s->nP : n_old, p.delta * p.delta, trace,
                            in_place, st));
    timer_end(s, st);
    // the counters and the segment records in one copy
    CC_HIP(hipMemcpyAsync(s->hc, s->dc, kMirrorSeg - kMirrorCounters + sizeof(SegDev) * ns,
                          hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    if ((int64_t)s->hc->n_act <= s->capA) break;
    if (attempt > 0) return CC_EOVERFLOW;
    CC_TRY(alloc_active(s, (int64_t)s->hc->n_act + (int64_t)s->hc->n_act / 4 + 1024));
    // counters of the failed attempt start again from zero
    for (int32_t i = 0; i < ns; ++i) s->seg_host[i].n_p = s->seg_host[i].n_pf = s->seg_host[i].n_a = 0;
    CC_HIP(hipMemcpyAsync(s->seg_dev, s->seg_host, sizeof(SegDev) * ns, hipMemcpyHostToDevice, st));
  }
  const int64_t n_eval = s->nP;
  const int64_t npf = in_place ? n_eval : (int64_t)s->hc->n_out, na = (int64_t)s->hc->n_act;
  if (single_live_seg(s)) {  // the pair pass kept no per-segment counts
    SegDev& d = s->seg_host[0];
    d.n_p = (d.flags & kSegActive) ? (unsigned long long)n_eval : 0ull;
    d.n_pf = (unsigned long long)npf;
    d.n_a = (unsigned long long)na;
  }
  s->mv_gen = ~0ull;  // valid again once this iteration's forward step has completed
  const uint64_t fp_pf = s->hc->fp_pf, fp_a = s->hc->fp_a;
  if (!in_place) {
    std::swap(s->P, s->P2);
    std::swap(s->dP, s->dP2);
  }
  s->nP = npf;
  s->nA = na;
  release_all_pending(s);  // no pair of a removed segment is left in P
  for (int32_t sg : act) {
    Seg& g = s->segs[sg];
    g.last.d_before = g.D;
    g.last.n_p = (int64_t)s->seg_host[sg].n_p;
    g.last.n_pf = (int64_t)s->seg_host[sg].n_pf;
    g.last.n_a = (int64_t)s->seg_host[sg].n_a;
    if (!searched[sg]) g.last.searched = 0;
  }
  // backward step (Sec. 4): coloured Gauss-Seidel, or the Jacobi variant of Sec. 4.3.2
  if (jacobi) {
    s->n_colors = 0;
    s->col_off.assign(1, 0);
    s->col_small = false;
    if (na > 0) CC_HIP(hipMemsetAsync(s->Acol, 0, sizeof(int32_t) * na, st));  // all in colour 0
  } else {
    // a small contact set is coloured and bucketed by one block, and the projection
    // reads its colours on the device: no host round trip before the forward step
    timer_begin(s, CC_K_COLOR, st);
    int rc = na <= kSmallRows ? color_small(s, st) : color_rows(s, false, st);
    timer_end(s, st);
    if (rc != CC_OK) return rc;
  }
  if (trace) {
    CC_HIP(hipMemsetAsync(&s->dc->fp_col, 0, sizeof(unsigned long long), st));
    CC_TRY(launch_fp_col(s, st));
  }
  timer_begin(s, CC_K_GS, st);
  if (jacobi) {
    CC_HIP(hipMemsetAsync(&s->dc->err, 0, sizeof(unsigned long long), st));
    CC_TRY(launch_jacobi(s, st));
  } else {
    CC_TRY(launch_gs(s, st));
  }
  timer_end(s, st);
  // forward step (Sec. 5) and the path certificate
  timer_begin(s, CC_K_FORWARD, st);
  CC_TRY(launch_forward(s, st));
  timer_end(s, st);
  const bool ccd_step = (p.flags & CC_CCD_STEP) != 0;
  timer_begin(s, CC_K_CERT, st);
  CC_TRY(launch_cert(s, ccd_step, st));
  timer_end(s, st);
  const bool small = s->col_small;
  if (trace || jacobi || small)  // the counters and the segment records in one copy
    CC_HIP(hipMemcpyAsync(s->hc, s->dc, kMirrorSeg - kMirrorCounters + sizeof(SegDev) * ns,
                          hipMemcpyDeviceToHost, st));
  else
    CC_HIP(hipMemcpyAsync(s->seg_host, s->seg_dev, sizeof(SegDev) * ns, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  // vertices of pieces the certificate did not clear go back to x^(l); that changes
  // the pieces of the pairs sharing them, so the certificate runs again until it
  // sends no new vertex back (the returned set only grows). The CCD-based step
  // answers its first kStepPasses passes by scaling the steps instead, as long as
  // they find contacts.
  unsigned long long nb_seen = 0, ns_seen = 0;
  for (int pass = 0;; ++pass) {
    const bool scaling = ccd_step && pass < kStepPasses;
    unsigned long long nb = 0, nstep = 0;
    for (int32_t sg : act) {
      nb += s->seg_host[sg].nback;
      nstep += s->seg_host[sg].nstep;
    }
    const bool more = scaling ? nstep != ns_seen : nb != nb_seen;
    if (!more) break;
    nb_seen = nb;
    ns_seen = nstep;
    const bool next_scaling = ccd_step && pass + 1 < kStepPasses;
    timer_begin(s, CC_K_CERT, st);
    CC_TRY(launch_send_back(s, ns, scaling, st));
    CC_TRY(launch_cert(s, next_scaling, st));
    timer_end(s, st);
    CC_HIP(hipMemcpyAsync(s->seg_host, s->seg_dev, sizeof(SegDev) * ns, hipMemcpyDeviceToHost,
                          st));
    CC_HIP(hipStreamSynchronize(st));
  }
  if (jacobi && (s->hc->err & 16ull)) return CC_EOVERFLOW;
  if (small) {
    // the projection and the forward step did nothing if the colouring failed
    if (s->hc->err & 1ull) return CC_ECOLOR;
    s->pc_dirty = false;
    s->n_colors = (int32_t)s->hc->ncol;
    s->pc_wide = s->n_colors > 56;
  }
  // the forward step wrote every iterating vertex's moved flag, and P' holds the
  // distances at the x it started from
  s->mv_gen = s->gen;
  resolve_timers(s);
  bool changed = false;
  for (int32_t sg : act) {
    Seg& g = s->segs[sg];
    const SegDev& d = s->seg_host[sg];
    const double mmax = bits2d(d.mmax_bits), rinf = bits2d(d.rinf_bits);
    cc_iter_info& it = g.last;
    it.n_colors = s->n_colors;
    it.move_max = mmax;
    it.r_inf = rinf;
    it.ccd_fail = (int64_t)d.fail;
    it.ccd_hits = (int64_t)d.hits;
    it.n_back = (int64_t)d.nback;
    it.n_scaled = (int64_t)d.nscaled;
    it.fp_pf = fp_pf;
    it.fp_a = fp_a;
    it.fp_col = trace ? s->hc->fp_col : 0;
    g.D = g.D - 2.0 * mmax;
    it.d_after = g.D;
    g.st.iters += 1;
    g.st.pair_updates += it.n_p;
    g.st.row_updates += (it.n_a + g.n_erows) * (int64_t)p.gs_sweeps;
    g.st.ccd_fail += it.ccd_fail;
    g.st.ccd_hits += it.ccd_hits;
    g.st.n_back += it.n_back;
    g.st.n_scaled += it.n_scaled;
    g.st.r_inf = rinf;
    if (s->n_colors > g.st.max_colors_used) g.st.max_colors_used = s->n_colors;
    if (rinf < p.eps) {
      g.st.status = CC_CONVERGED;
      g.active = false;
      changed = true;
    } else if (g.st.iters >= g.max_iters) {
      g.active = false;
      changed = true;
    }
  }
  if (changed) s->erows_dirty = true;
  // algorithmic bytes (engine totals)
  {
    const double N = s->n, F = s->nt, E = s->ne;
    s->st.iters += 1;
    s->st.pair_updates += n_eval;
    s->st.kernel_bytes[CC_K_PAIR] += 8.0 * n_eval + 16.0 * npf + 24.0 * na + 32.0 * N + 12.0 * F + 8.0 * E;
    s->st.kernel_bytes[CC_K_FORWARD] += 92.0 * N;
    s->st.kernel_bytes[CC_K_CERT] += 16.0 * npf + 8.0 * N + 12.0 * F + 8.0 * E;
    // projection: per contact row its key and vertex ids, x and w of its four
    // vertices, y (or y - x) read and written, the multiplier; per edge row the
    // ids, g, 1/A, w, y read and written (mixed: x as well, y - x in FP32)
    const bool mixed = (p.flags & CC_MIXED) != 0;
    const double row = mixed ? 8 + 16 + 96 + 32 + 48 + 48 + 8 : 8 + 16 + 96 + 32 + 96 + 96 + 16;
    const double erow = mixed ? 8 + 24 + 8 + 16 + 48 + 24 + 24 + 8 : 8 + 24 + 8 + 16 + 48 + 48 + 16;
    s->st.kernel_bytes[CC_K_GS] += (row * na + erow * s->n_erows) * p.gs_sweeps;
  }
  return CC_OK;
}

int engine_active(const cc_solver* s) {
  int k = 0;
  for (const Seg& g : s->segs) k += (g.live && g.active) ? 1 : 0;
  return k;
}

// Statistics of a segment with the engine's kernel timings and bytes.
void seg_stats(const cc_solver* s, int32_t sg, cc_stats* out) {
  *out = s->segs[sg].st;
  for (int k = 0; k < CC_K_COUNT; ++k) {
    out->kernel_ms[k] = s->st.kernel_ms[k];
    out->kernel_launches[k] = s->st.kernel_launches[k];
    out->kernel_bytes[k] = s->st.kernel_bytes[k];
  }
}

}  // namespace cc

namespace {

// Make ctx's one-scene engine hold exactly this scene, as segment 0 at base 0.
int bind_single(cc_context* ctx, cc_solver*& slot, int32_t n, const double* inv_mass,
                const int32_t* tris, int32_t nt, const int32_t* edges, int32_t ne,
                const cc_params* params, hipStream_t st) {
  if (!slot) CC_TRY(engine_create(ctx, params, n, nt, ne, &slot, st));
  cc_solver* s = slot;
  engine_set_params(s, params);
  for (int32_t i = 0; i < (int32_t)s->segs.size(); ++i)
    if (s->segs[i].live) CC_TRY(seg_remove(s, i, st));
  s->nP = 0;
  release_pending(s);
  for (auto& g : s->segs) g.pending = false;
  s->pending_segs.clear();
  int32_t sg = -1;
  CC_TRY(seg_add(s, n, inv_mass, tris, nt, edges, ne, INT_MAX, &sg, st));
  if (sg != 0 || s->segs[0].vb != 0 || s->segs[0].fb != 0 || s->segs[0].eb != 0) return CC_ESTATE;
  memset(&s->st, 0, sizeof s->st);
  s->begun = false;
  return CC_OK;
}

}  // namespace

extern "C" {

void cc_default_params(cc_params* p) {
  if (!p) return;
  p->delta = 1e-3;
  p->d_min = 2e-3;
  p->d_max = 4e-3;
  p->sigma = 1.1;
  p->gamma = 0.9;
  p->eps = 1e-4;
  p->kappa = 1e-3;
  p->max_iters = 512;
  p->gs_sweeps = 1;
  p->max_colors = 1024;
  p->flags = CC_EDGE_LEN;
  p->seed = 0x221104045ull;
  p->omega = 0.5;
  p->backward = CC_GAUSS_SEIDEL;
  p->time_kind = CC_K_SEARCH;
}

const char* cc_strerror(int code) {
  switch (code) {
    case CC_OK: return "ok";
    case CC_EINVAL: return "invalid argument";
    case CC_ENOMEM: return "device allocation failed";
    case CC_EOVERFLOW: return "pair capacity exceeded";
    case CC_EHIP: return "HIP runtime error";
    case CC_ECOLOR: return "colour palette exhausted";
    case CC_ESTATE: return "call out of order";
    case CC_EAGAIN: return "over the HBM budget or the scene limit, retry after a release";
    case CC_EBUSY: return "step still running";
    case CC_ENOTFREE: return "x_prev is not in the free space";
    default: return "unknown error";
  }
}

int cc_edges_from_tris_host(const int32_t* tris, int32_t nt, int32_t* edges, int32_t cap,
                            int32_t* n_edges) {
  if (nt < 0 || cap < 0 || !n_edges || (nt > 0 && !tris)) return CC_EINVAL;
  std::vector<uint64_t> e;
  e.reserve(3 * (size_t)nt);
  for (int32_t t = 0; t < nt; ++t) {
    const int32_t v[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    if (v[0] < 0 || v[1] < 0 || v[2] < 0 || v[0] == v[1] || v[1] == v[2] || v[0] == v[2])
      return CC_EINVAL;
    for (int k = 0; k < 3; ++k) {
      const uint32_t a = (uint32_t)v[k], b = (uint32_t)v[(k + 1) % 3];
      e.push_back(a < b ? ((uint64_t)a << 32) | b : ((uint64_t)b << 32) | a);
    }
  }
  std::sort(e.begin(), e.end());
  e.erase(std::unique(e.begin(), e.end()), e.end());
  if ((int64_t)e.size() > INT_MAX) return CC_EINVAL;
  *n_edges = (int32_t)e.size();
  if (edges && cap >= (int32_t)e.size())
    for (size_t i = 0; i < e.size(); ++i) {
      edges[2 * i] = (int32_t)(e[i] >> 32);
      edges[2 * i + 1] = (int32_t)(uint32_t)e[i];
    }
  return CC_OK;
}

int cc_context_create(int device, cc_context** out) {
  if (!out) return CC_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CC_EHIP;
  // the no-allocation target's scratch array on this device (its entry point reports
  // CC_ESTATE if the lookup failed)
  (void)cc::flow_scratch_init(device);
  cc_context* c = new cc_context();
  c->device = device;
  *out = c;
  return CC_OK;
}

void cc_context_destroy(cc_context* ctx) {
  if (!ctx) return;
  server_destroy(ctx);
  if (ctx->cached) cc_solver_destroy(ctx->cached);
  if (ctx->batched) cc_solver_destroy(ctx->batched);
  cc::flow_free(ctx->flow);
  delete ctx;
}

int cc_normal_flow_target(cc_context* ctx, const double* x, int32_t n_verts,
                          const int32_t* tris, int32_t n_tris, double beta, double alpha,
                          int32_t iters, double* y, void* stream) {
  if (!ctx) return CC_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  return cc::normal_flow_target(ctx, x, n_verts, tris, n_tris, beta, alpha, iters, y,
                                as_stream(stream));
}

int cc_normal_flow_target_noalloc(cc_context* ctx, const double* x, int32_t n_verts,
                                  const int32_t* tris, int32_t n_tris, double beta, double alpha,
                                  int32_t iters, double* y, void* stream) {
  if (!ctx) return CC_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  return cc::normal_flow_target_static(ctx->device, x, n_verts, tris, n_tris, beta, alpha, iters,
                                       y, as_stream(stream));
}

int cc_autotune_entries(cc_tune_entry* out_host, int32_t cap, int32_t* n) {
  if (!n || cap < 0 || (cap > 0 && !out_host)) return CC_EINVAL;
  std::lock_guard<std::mutex> lk(cc::g_tune_mu);
  *n = (int32_t)cc::g_tune.size();
  if (cap >= *n)
    for (int32_t i = 0; i < *n; ++i) out_host[i] = cc::g_tune[(size_t)i];
  return CC_OK;
}

void cc_autotune_reset(void) {
  std::lock_guard<std::mutex> lk(cc::g_tune_mu);
  cc::g_tune.clear();
}

int cc_autotune_force(int32_t kernel, int32_t choice) {
  if (kernel != CC_TUNE_TRAVERSE) return CC_EINVAL;
  if (choice != 0 && choice != 8 && choice != 16 && choice != 32 && choice != 108 &&
      choice != 116 && choice != 132)
    return CC_EINVAL;
  std::lock_guard<std::mutex> lk(cc::g_tune_mu);
  cc::g_tune_force[kernel] = choice;
  return CC_OK;
}

int cc_solver_create(cc_context* ctx, int32_t n, const double* inv_mass, const int32_t* tris,
                     int32_t nt, const int32_t* edges, int32_t ne, const cc_params* params,
                     cc_solver** out, void* stream) {
  if (!ctx || !out || n < 0 || nt < 0 || ne < 0) return CC_EINVAL;
  if ((nt > 0 && !tris) || (ne > 0 && !edges)) return CC_EINVAL;
  CC_TRY(check_params(params));
  cc_solver* s = nullptr;
  int rc = bind_single(ctx, s, n, inv_mass, tris, nt, edges, ne, params, as_stream(stream));
  if (rc != CC_OK) {
    if (s) cc_solver_destroy(s);
    return rc;
  }
  *out = s;
  return CC_OK;
}

void cc_solver_destroy(cc_solver* s) {
  if (!s) return;
  solver_free(s);  // hipFree waits for the work that uses the memory
  delete s;
}

int cc_solver_begin(cc_solver* s, const double* x_prev, const double* x_tilde, void* stream) {
  if (!s || s->segs.empty() || !s->segs[0].live) return CC_EINVAL;
  if (s->segs[0].nv > 0 && (!x_prev || !x_tilde)) return CC_EINVAL;
  int32_t sg = 0;
  int rc = CC_OK;
  memset(&s->st, 0, sizeof s->st);
  CC_TRY(seg_begin(s, &sg, 1, &x_prev, &x_tilde, &rc, as_stream(stream)));
  CC_TRY(rc);
  s->nP = 0;
  s->nA = 0;
  s->n_colors = 0;
  s->D = 0.0;
  s->begun = true;
  return CC_OK;
}

int cc_solver_iterate(cc_solver* s, int32_t* stop, cc_iter_info* info, void* stream) {
  if (!s) return CC_EINVAL;
  if (!s->begun) return CC_ESTATE;
  Seg& g = s->segs[0];
  g.active = true;  // a converged scene may still be stepped by hand
  CC_TRY(engine_iterate(s, as_stream(stream)));
  s->D = g.D;
  const int done = g.last.r_inf < s->p.eps ? 1 : 0;
  if (stop) *stop = done;
  if (info) *info = g.last;
  return CC_OK;
}

int cc_solver_run(cc_solver* s, double* x_out, cc_stats* stats, void* stream) {
  if (!s) return CC_EINVAL;
  if (!s->begun) return CC_ESTATE;
  for (int l = 0; l < s->p.max_iters; ++l) {
    int32_t stop = 0;
    CC_TRY(cc_solver_iterate(s, &stop, nullptr, stream));
    if (stop) break;
  }
  if (x_out && s->segs[0].nv)
    CC_HIP(hipMemcpyAsync(x_out, s->x, sizeof(double) * 3 * s->segs[0].nv, hipMemcpyDefault,
                          as_stream(stream)));
  CC_HIP(hipStreamSynchronize(as_stream(stream)));
  if (stats) seg_stats(s, 0, stats);
  return CC_OK;
}

int cc_collide_step(cc_context* ctx, const double* x_prev, const double* x_tilde,
                    const double* inv_mass, int32_t n, const int32_t* tris, int32_t nt,
                    const int32_t* edges, int32_t ne, const cc_params* params, double* x_next,
                    cc_stats* stats, void* stream) {
  if (!ctx || n < 0 || nt < 0 || ne < 0 || (n > 0 && !x_next)) return CC_EINVAL;
  if ((nt > 0 && !tris) || (ne > 0 && !edges)) return CC_EINVAL;
  if (n > 0 && (x_next == x_prev || x_next == x_tilde)) return CC_EINVAL;
  CC_TRY(check_params(params));
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  CC_TRY(bind_single(ctx, ctx->cached, n, inv_mass, tris, nt, edges, ne, params, as_stream(stream)));
  CC_TRY(cc_solver_begin(ctx->cached, x_prev, x_tilde, stream));
  return cc_solver_run(ctx->cached, x_next, stats, stream);
}

int cc_collide_step_batched(cc_context* ctx, const cc_scene* scenes, int32_t ns,
                            const cc_params* params, cc_stats* stats, void* stream) {
  if (!ctx || ns < 0 || (ns > 0 && !scenes)) return CC_EINVAL;
  if (ns > kMaxSeg) return CC_EINVAL;
  CC_TRY(check_params(params));
  for (int32_t i = 0; i < ns; ++i) {
    const cc_scene& sc = scenes[i];
    if (sc.n_verts < 0 || sc.n_tris < 0 || sc.n_edges < 0) return CC_EINVAL;
    if (sc.n_verts > 0 && (!sc.x_next || !sc.x_prev || !sc.x_tilde)) return CC_EINVAL;
    if (sc.n_verts > 0 && (sc.x_next == sc.x_prev || sc.x_next == sc.x_tilde)) return CC_EINVAL;
  }
  if (ns == 0) return CC_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  hipStream_t st = as_stream(stream);
  int64_t V = 0, F = 0, E = 0;
  for (int32_t i = 0; i < ns; ++i) {
    V += scenes[i].n_verts;
    F += scenes[i].n_tris;
    E += scenes[i].n_edges;
  }
  if (V > INT_MAX / 4 || F > INT_MAX / 4 || E > INT_MAX / 4) return CC_EINVAL;
  if (!ctx->batched)
    CC_TRY(engine_create(ctx, params, (int32_t)V, (int32_t)F, (int32_t)E, &ctx->batched, st));
  cc_solver* s = ctx->batched;
  engine_set_params(s, params);
  for (int32_t i = 0; i < (int32_t)s->segs.size(); ++i)
    if (s->segs[i].live) CC_TRY(seg_remove(s, i, st));
  s->nP = 0;
  release_pending(s);
  for (auto& g : s->segs) g.pending = false;
  s->pending_segs.clear();
  memset(&s->st, 0, sizeof s->st);
  std::vector<int> rc(ns, CC_OK);
  std::vector<int32_t> sg(ns, -1), begin_ids;
  std::vector<const double*> xp, xt;
  std::vector<int32_t> begin_of;
  for (int32_t i = 0; i < ns; ++i) {
    const cc_scene& sc = scenes[i];
    rc[i] = seg_add(s, sc.n_verts, sc.inv_mass, sc.tris, sc.n_tris, sc.edges, sc.n_edges,
                    params->max_iters, &sg[i], st);
    if (rc[i] != CC_OK) continue;
    begin_ids.push_back(sg[i]);
    xp.push_back(sc.x_prev);
    xt.push_back(sc.x_tilde);
    begin_of.push_back(i);
  }
  if (!begin_ids.empty()) {
    std::vector<int> brc(begin_ids.size(), CC_OK);
    int r = seg_begin(s, begin_ids.data(), (int32_t)begin_ids.size(), xp.data(), xt.data(),
                      brc.data(), st);
    for (size_t k = 0; k < begin_ids.size(); ++k) {
      if (brc[k] != CC_OK) rc[begin_of[k]] = brc[k];
      if (brc[k] != CC_OK && s->segs[begin_ids[k]].live) s->segs[begin_ids[k]].active = false;
    }
    if (r != CC_OK) return r;
    while (engine_active(s) > 0) CC_TRY(engine_iterate(s, st));
  }
  for (int32_t i = 0; i < ns; ++i) {
    if (rc[i] != CC_OK) continue;
    const Seg& g = s->segs[sg[i]];
    if (g.nv)
      CC_HIP(hipMemcpyAsync(scenes[i].x_next, s->x + 3 * (int64_t)g.vb, sizeof(double) * 3 * g.nv,
                            hipMemcpyDefault, st));
    if (stats) seg_stats(s, sg[i], &stats[i]);
  }
  CC_HIP(hipStreamSynchronize(st));
  for (int32_t i = 0; i < ns; ++i)
    if (rc[i] != CC_OK) return rc[i];
  return CC_OK;
}

int cc_solver_get_state(cc_solver* s, double* x, double* y, double* r, double* D_host,
                        void* stream) {
  if (!s || s->segs.empty()) return CC_EINVAL;
  hipStream_t st = as_stream(stream);
  const int32_t n = s->segs[0].nv;
  size_t n3 = sizeof(double) * 3 * n;
  if (x && n) CC_HIP(hipMemcpyAsync(x, s->x, n3, hipMemcpyDefault, st));
  if (y && n && (s->p.flags & CC_MIXED)) CC_TRY(launch_y_of_dy(s, y, n, st));
  else if (y && n) CC_HIP(hipMemcpyAsync(y, s->y, n3, hipMemcpyDefault, st));
  if (r && n) CC_HIP(hipMemcpyAsync(r, s->r, sizeof(double) * n, hipMemcpyDefault, st));
  CC_HIP(hipStreamSynchronize(st));
  if (D_host) *D_host = s->segs[0].D;
  return CC_OK;
}

int cc_solver_set_state(cc_solver* s, const double* x, const double* y, const double* r,
                        double D, const uint64_t* P, int64_t n_p, void* stream) {
  if (!s || n_p < 0 || (n_p > 0 && !P)) return CC_EINVAL;
  if (!s->begun) return CC_ESTATE;
  ++s->gen;  // x set from outside: no tree reuse
  hipStream_t st = as_stream(stream);
  const int32_t n = s->segs[0].nv;
  size_t n3 = sizeof(double) * 3 * n;
  if (n_p > s->capP) CC_TRY(alloc_pairs(s, n_p + n_p / 4 + 1024, 0, st));
  if (x && n) CC_HIP(hipMemcpyAsync(s->x, x, n3, hipMemcpyDefault, st));
  if (y && n) CC_HIP(hipMemcpyAsync(s->y, y, n3, hipMemcpyDefault, st));
  if (y && n && (s->p.flags & CC_MIXED)) CC_TRY(launch_dy_of_y(s, y, n, st));
  if (r && n) CC_HIP(hipMemcpyAsync(s->r, r, sizeof(double) * n, hipMemcpyDefault, st));
  if (n_p) CC_HIP(hipMemcpyAsync(s->P, P, sizeof(uint64_t) * n_p, hipMemcpyDefault, st));
  CC_HIP(hipStreamSynchronize(st));
  s->nP = n_p;
  s->segs[0].D = D;
  s->D = D;
  return CC_OK;
}

int cc_solver_get_P(cc_solver* s, uint64_t* keys, int64_t cap, int64_t* n, void* stream) {
  if (!s || !n) return CC_EINVAL;
  *n = s->nP;
  if (keys && cap >= s->nP && s->nP)
    CC_HIP(hipMemcpyAsync(keys, s->P, sizeof(uint64_t) * s->nP, hipMemcpyDefault, as_stream(stream)));
  CC_HIP(hipStreamSynchronize(as_stream(stream)));
  return CC_OK;
}

int cc_solver_get_A(cc_solver* s, uint64_t* keys, int32_t* colors, int64_t cap, int64_t* n,
                    void* stream) {
  if (!s || !n) return CC_EINVAL;
  *n = s->nA;
  hipStream_t st = as_stream(stream);
  if (cap >= s->nA && s->nA) {
    if (keys) CC_HIP(hipMemcpyAsync(keys, s->Akeys, sizeof(uint64_t) * s->nA, hipMemcpyDefault, st));
    if (colors) CC_HIP(hipMemcpyAsync(colors, s->Acol, sizeof(int32_t) * s->nA, hipMemcpyDefault, st));
  }
  CC_HIP(hipStreamSynchronize(st));
  return CC_OK;
}

int cc_solver_get_Di(cc_solver* s, double* out, void* stream) {
  if (!s || s->segs.empty()) return CC_EINVAL;
  const int32_t n = s->segs[0].nv;
  if (!out && n) return CC_EINVAL;
  if (n) CC_HIP(hipMemcpyAsync(out, s->Di, sizeof(double) * n, hipMemcpyDefault, as_stream(stream)));
  CC_HIP(hipStreamSynchronize(as_stream(stream)));
  return CC_OK;
}

int cc_solver_search(cc_solver* s, const double* x, double dmax, uint64_t* keys, int64_t cap,
                     int64_t* n, void* stream) {
  if (!s || s->segs.empty() || !x || !n || !(dmax > 0.0)) return CC_EINVAL;
  hipStream_t st = as_stream(stream);
  const int32_t nv = s->segs[0].nv;
  CC_TRY(launch_check_finite(s, x, nullptr, nv, st));
  // the static flags come from the last begin; without one every vertex counts as free
  if (!s->begun && nv) CC_HIP(hipMemsetAsync(s->stat, 0, nv, st));
  s->sel_host[0].seg = 0;
  CC_TRY(lbvh_search(s, 1, x, dmax, keys, nullptr, keys ? cap : 0, n, st, false));
  CC_HIP(hipStreamSynchronize(st));  // the keys are in place on return
  return CC_OK;
}

int cc_solver_stats(cc_solver* s, cc_stats* out) {
  if (!s || !out || s->segs.empty()) return CC_EINVAL;
  seg_stats(s, 0, out);
  return CC_OK;
}

}  // extern "C"
