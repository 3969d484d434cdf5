// C ABI of the two-way collision-handling step: contexts, resident solvers and
// the host loop of Alg. 1 that sequences the HIP kernels on the caller's stream.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
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
  if (p) hipFree((void*)p);
  p = nullptr;
}

int check_params(const cc_params* p) {
  if (!p) return CC_EINVAL;
  if (!(p->delta > 0.0) || !(p->d_min >= p->delta) || !(p->d_max > p->d_min)) return CC_EINVAL;
  if (!(p->sigma >= 1.0) || !(p->gamma > 0.0 && p->gamma < 1.0) || !(p->eps > 0.0)) return CC_EINVAL;
  if (!(p->kappa >= 0.0)) return CC_EINVAL;
  if (p->max_iters < 1 || p->gs_sweeps < 1) return CC_EINVAL;
  if (p->max_colors < 1 || p->max_colors > kMaxColors) return CC_EINVAL;
  return CC_OK;
}

void free_pairs(cc_solver* s) {
  dfree(s->P); dfree(s->P2); dfree(s->dP); dfree(s->dP2);
}
void free_active(cc_solver* s) {
  dfree(s->Akeys); dfree(s->Averts); dfree(s->Acol); dfree(s->Aorder);
  dfree(s->list0); dfree(s->list1); dfree(s->lamA);
}

int alloc_pairs(cc_solver* s, int64_t cap) {
  free_pairs(s);
  s->capP = cap;
  CC_TRY(dalloc(&s->P, cap));
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
  return CC_OK;
}

void solver_free(cc_solver* s) {
  dfree(s->w); dfree(s->tris); dfree(s->edges); dfree(s->stat);
  dfree(s->x); dfree(s->y); dfree(s->xt); dfree(s->xold); dfree(s->r); dfree(s->move2); dfree(s->Di);
  free_pairs(s);
  free_active(s);
  dfree(s->eg); dfree(s->einv); dfree(s->ecol); dfree(s->eorder);
  dfree(s->elist0); dfree(s->elist1); dfree(s->elist2); dfree(s->lamE);
  dfree(s->vmax0); dfree(s->vmax1); dfree(s->masks); dfree(s->col_cnt); dfree(s->rcnt);
  dfree(s->coff_dev); dfree(s->ecoff_dev);
  bvh_free(s);
  dfree(s->dc);
  if (s->hc) hipHostFree(s->hc);
  s->hc = nullptr;
  for (auto& t : s->timers) {
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  s->timers.clear();
  for (auto e : s->event_pool) hipEventDestroy(e);
  s->event_pool.clear();
}

int solver_alloc(cc_solver* s) {
  const int64_t n = s->n, nt = s->nt, ne = s->ne;
  CC_TRY(dalloc(&s->w, n));
  CC_TRY(dalloc(&s->tris, 3 * nt));
  CC_TRY(dalloc(&s->edges, 2 * ne));
  CC_TRY(dalloc(&s->stat, n));
  CC_TRY(dalloc(&s->x, 3 * n));
  CC_TRY(dalloc(&s->y, 3 * n));
  CC_TRY(dalloc(&s->xt, 3 * n));
  CC_TRY(dalloc(&s->xold, 3 * n));
  CC_TRY(dalloc(&s->r, n));
  CC_TRY(dalloc(&s->move2, n));
  CC_TRY(dalloc(&s->Di, n));
  CC_TRY(dalloc(&s->eg, 3 * ne));
  CC_TRY(dalloc(&s->einv, ne));
  CC_TRY(dalloc(&s->ecol, ne));
  CC_TRY(dalloc(&s->eorder, ne));
  CC_TRY(dalloc(&s->elist0, ne));
  CC_TRY(dalloc(&s->elist1, ne));
  CC_TRY(dalloc(&s->elist2, ne));
  CC_TRY(dalloc(&s->lamE, ne));
  CC_TRY(dalloc(&s->vmax0, n));
  CC_TRY(dalloc(&s->vmax1, n));
  CC_TRY(dalloc(&s->masks, n * kMaskWords));
  CC_TRY(dalloc(&s->col_cnt, kMaxColors + 1));
  CC_TRY(dalloc(&s->rcnt, kMaxRounds + 1));
  CC_TRY(dalloc(&s->coff_dev, kMaxColors + 1));
  CC_TRY(dalloc(&s->ecoff_dev, kMaxColors + 1));
  CC_TRY(bvh_alloc(s));
  CC_TRY(dalloc(&s->dc, 1));
  if (hipHostMalloc((void**)&s->hc, sizeof(Counters), hipHostMallocDefault) != hipSuccess)
    return CC_ENOMEM;
  int64_t cap = std::max<int64_t>(4096, 32 * (n + ne));
  CC_TRY(alloc_pairs(s, cap));
  CC_TRY(alloc_active(s, std::max<int64_t>(4096, cap / 8)));
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

// Make `slot` a solver for this topology: reuse it when the sizes match (topology
// and masses are copied in again), otherwise replace it.
int bind_solver(cc_context* ctx, cc_solver*& slot, int32_t n, const double* inv_mass,
                const int32_t* tris, int32_t nt, const int32_t* edges, int32_t ne,
                const cc_params* params, void* stream) {
  hipStream_t st = as_stream(stream);
  cc_solver* s = slot;
  if (s && s->n == n && s->nt == nt && s->ne == ne) {
    s->p = *params;
    s->kappa2 = params->kappa * params->kappa;
    if (nt) CC_HIP(hipMemcpyAsync(s->tris, tris, sizeof(int32_t) * 3 * nt, hipMemcpyDefault, st));
    if (ne) CC_HIP(hipMemcpyAsync(s->edges, edges, sizeof(int32_t) * 2 * ne, hipMemcpyDefault, st));
    if (n) {
      if (inv_mass)
        CC_HIP(hipMemcpyAsync(s->w, inv_mass, sizeof(double) * n, hipMemcpyDefault, st));
      else
        CC_TRY(launch_fill_u64((unsigned long long*)s->w, n, d2bits(1.0), st));
    }
    return launch_validate(s, nullptr, nullptr, st);
  }
  if (s) cc_solver_destroy(s);
  slot = nullptr;
  CC_TRY(cc_solver_create(ctx, n, inv_mass, tris, nt, edges, ne, params, &s, stream));
  slot = s;
  return CC_OK;
}

int do_search(cc_solver* s, const double* x, double dmax, hipStream_t st) {
  for (int attempt = 0; attempt < 2; ++attempt) {
    int64_t n = 0;
    CC_TRY(lbvh_search(s, x, dmax, s->P, s->capP, &n, st));
    if (n <= s->capP) {
      s->nP = n;
      return CC_OK;
    }
    CC_TRY(alloc_pairs(s, n + n / 4 + 1024));
  }
  return CC_EOVERFLOW;
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
  hipEventCreate(&e);
  return e;
}

void timer_begin(cc_solver* s, int kind, hipStream_t st) {
  if (!(s->p.flags & CC_TIME_KERNELS)) return;
  Timer t;
  t.kind = kind;
  t.a = pool_event(s);
  t.b = pool_event(s);
  hipEventRecord(t.a, st);
  s->timers.push_back(t);
}

void timer_end(cc_solver* s, hipStream_t st) {
  if (!(s->p.flags & CC_TIME_KERNELS) || s->timers.empty()) return;
  hipEventRecord(s->timers.back().b, st);
}

}  // namespace cc

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
    case CC_EAGAIN: return "over the HBM budget, retry after a release";
    case CC_EBUSY: return "step still running";
    default: return "unknown error";
  }
}

int cc_context_create(int device, cc_context** out) {
  if (!out) return CC_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return CC_EHIP;
  cc_context* c = new cc_context();
  c->device = device;
  *out = c;
  return CC_OK;
}

void cc_context_destroy(cc_context* ctx) {
  if (!ctx) return;
  server_destroy(ctx);
  if (ctx->cached) cc_solver_destroy(ctx->cached);
  for (cc_solver* s : ctx->slots)
    if (s) cc_solver_destroy(s);
  for (hipStream_t s : ctx->slot_streams) (void)hipStreamDestroy(s);
  delete ctx;
}

int cc_solver_create(cc_context* ctx, int32_t n, const double* inv_mass, const int32_t* tris,
                     int32_t nt, const int32_t* edges, int32_t ne, const cc_params* params,
                     cc_solver** out, void* stream) {
  if (!ctx || !out || n < 0 || nt < 0 || ne < 0) return CC_EINVAL;
  if ((nt > 0 && !tris) || (ne > 0 && !edges)) return CC_EINVAL;
  CC_TRY(check_params(params));
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  hipStream_t st = as_stream(stream);
  cc_solver* s = new cc_solver();
  s->ctx = ctx;
  s->n = n;
  s->nt = nt;
  s->ne = ne;
  s->p = *params;
  s->kappa2 = params->kappa * params->kappa;
  int rc = solver_alloc(s);
  if (rc == CC_OK) {
    if (nt) rc = hipMemcpyAsync(s->tris, tris, sizeof(int32_t) * 3 * nt, hipMemcpyDefault, st) == hipSuccess ? CC_OK : CC_EHIP;
    if (rc == CC_OK && ne) rc = hipMemcpyAsync(s->edges, edges, sizeof(int32_t) * 2 * ne, hipMemcpyDefault, st) == hipSuccess ? CC_OK : CC_EHIP;
    if (rc == CC_OK && n) {
      if (inv_mass)
        rc = hipMemcpyAsync(s->w, inv_mass, sizeof(double) * n, hipMemcpyDefault, st) == hipSuccess ? CC_OK : CC_EHIP;
      else
        rc = launch_fill_u64((unsigned long long*)s->w, n, d2bits(1.0), st);
    }
    if (rc == CC_OK) rc = launch_validate(s, nullptr, nullptr, st);
  }
  if (rc != CC_OK) {
    solver_free(s);
    delete s;
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
  if (!s || (s->n > 0 && (!x_prev || !x_tilde))) return CC_EINVAL;
  hipStream_t st = as_stream(stream);
  CC_TRY(launch_validate(s, x_prev, x_tilde, st));
  CC_TRY(launch_setup(s, x_prev, x_tilde, st));
  s->D = 0.0;
  s->nP = 0;
  s->nA = 0;
  s->n_colors = 0;
  memset(&s->st, 0, sizeof s->st);
  s->st.status = CC_MAXITER;
  for (auto& t : s->timers) {
    s->event_pool.push_back(t.a);
    s->event_pool.push_back(t.b);
  }
  s->timers.clear();
  timer_begin(s, CC_K_COLOR, st);
  int rc = color_rows(s, true, st);
  timer_end(s, st);
  if (rc != CC_OK) return rc;
  CC_HIP(hipStreamSynchronize(st));
  resolve_timers(s);
  s->begun = true;
  return CC_OK;
}

int cc_solver_iterate(cc_solver* s, int32_t* stop, cc_iter_info* info, void* stream) {
  if (!s) return CC_EINVAL;
  if (!s->begun) return CC_ESTATE;
  hipStream_t st = as_stream(stream);
  const cc_params& p = s->p;
  const bool trace = (p.flags & CC_TRACE) != 0;
  cc_iter_info it;
  memset(&it, 0, sizeof it);
  // Alg. 1: proximity search when the reuse bound fell below D_min (Sec. 3.1)
  if (s->D < p.d_min) {
    int rc = do_search(s, s->x, p.d_max, st);
    if (rc != CC_OK) return rc;
    s->D = p.d_max;
    it.searched = 1;
    s->st.searches += 1;
  }
  it.d_before = s->D;
  it.n_p = s->nP;
  const double D = s->D;
  // pair pass; regrow the active set if it overflowed
  for (int attempt = 0;; ++attempt) {
    CC_HIP(hipMemsetAsync(s->dc, 0, sizeof(Counters), st));
    CC_TRY(launch_fill_u64(s->Di, s->n, d2bits(D), st));
    timer_begin(s, CC_K_PAIR, st);
    CC_TRY(launch_pair_pass(s, D * D, p.delta * p.delta, trace, st));
    timer_end(s, st);
    CC_HIP(hipMemcpyAsync(s->hc, s->dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
    CC_HIP(hipStreamSynchronize(st));
    if ((int64_t)s->hc->n_act <= s->capA) break;
    if (attempt > 0) return CC_EOVERFLOW;
    CC_TRY(alloc_active(s, (int64_t)s->hc->n_act + (int64_t)s->hc->n_act / 4 + 1024));
  }
  const int64_t npf = (int64_t)s->hc->n_out, na = (int64_t)s->hc->n_act;
  it.fp_pf = s->hc->fp_pf;
  it.fp_a = s->hc->fp_a;
  std::swap(s->P, s->P2);
  std::swap(s->dP, s->dP2);
  s->nP = npf;
  s->nA = na;
  it.n_pf = npf;
  it.n_a = na;
  // backward step (Sec. 4)
  timer_begin(s, CC_K_COLOR, st);
  int rc = color_rows(s, false, st);
  timer_end(s, st);
  if (rc != CC_OK) return rc;
  it.n_colors = s->n_colors;
  if (trace) {
    CC_HIP(hipMemsetAsync(&s->dc->fp_col, 0, sizeof(unsigned long long), st));
    CC_TRY(launch_fp_col(s, st));
  }
  timer_begin(s, CC_K_GS, st);
  CC_TRY(launch_gs(s, st));
  timer_end(s, st);
  // forward step (Sec. 5) and the path certificate
  CC_HIP(hipMemsetAsync(&s->dc->mmax_bits, 0, 2 * sizeof(unsigned long long), st));
  CC_HIP(hipMemsetAsync(&s->dc->fail, 0, sizeof(unsigned long long), st));
  CC_HIP(hipMemsetAsync(&s->dc->hits, 0, sizeof(unsigned long long), st));
  timer_begin(s, CC_K_FORWARD, st);
  CC_TRY(launch_forward(s, st));
  timer_end(s, st);
  timer_begin(s, CC_K_CERT, st);
  CC_TRY(launch_cert(s, st));
  timer_end(s, st);
  CC_HIP(hipMemcpyAsync(s->hc, s->dc, sizeof(Counters), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  resolve_timers(s);
  const double mmax = bits2d(s->hc->mmax_bits), rinf = bits2d(s->hc->rinf_bits);
  it.move_max = mmax;
  it.r_inf = rinf;
  it.ccd_fail = (int64_t)s->hc->fail;
  it.ccd_hits = (int64_t)s->hc->hits;
  if (trace) it.fp_col = s->hc->fp_col;
  s->D = D - 2.0 * mmax;
  it.d_after = s->D;
  const int done = rinf < p.eps ? 1 : 0;
  // statistics and algorithmic bytes
  s->st.iters += 1;
  s->st.pair_updates += it.n_p;
  s->st.row_updates += (na + s->n_erows) * (int64_t)p.gs_sweeps;
  s->st.ccd_fail += it.ccd_fail;
  s->st.ccd_hits += it.ccd_hits;
  s->st.r_inf = rinf;
  if (it.n_colors > s->st.max_colors_used) s->st.max_colors_used = it.n_colors;
  if (done) s->st.status = CC_CONVERGED;
  {
    const double N = s->n, F = s->nt, E = s->ne;
    s->st.kernel_bytes[CC_K_PAIR] += 8.0 * it.n_p + 16.0 * npf + 24.0 * na + 32.0 * N + 12.0 * F + 8.0 * E;
    s->st.kernel_bytes[CC_K_FORWARD] += 92.0 * N;
    s->st.kernel_bytes[CC_K_CERT] += 16.0 * npf + 8.0 * N + 12.0 * F + 8.0 * E;
  }
  if (stop) *stop = done;
  if (info) *info = it;
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
  if (x_out && s->n)
    CC_HIP(hipMemcpyAsync(x_out, s->x, sizeof(double) * 3 * s->n, hipMemcpyDefault, as_stream(stream)));
  CC_HIP(hipStreamSynchronize(as_stream(stream)));
  if (stats) *stats = s->st;
  return CC_OK;
}

int cc_collide_step(cc_context* ctx, const double* x_prev, const double* x_tilde,
                    const double* inv_mass, int32_t n, const int32_t* tris, int32_t nt,
                    const int32_t* edges, int32_t ne, const cc_params* params, double* x_next,
                    cc_stats* stats, void* stream) {
  if (!ctx || (n > 0 && !x_next)) return CC_EINVAL;
  if (n > 0 && (x_next == x_prev || x_next == x_tilde)) return CC_EINVAL;
  CC_TRY(check_params(params));
  CC_TRY(bind_solver(ctx, ctx->cached, n, inv_mass, tris, nt, edges, ne, params, stream));
  CC_TRY(cc_solver_begin(ctx->cached, x_prev, x_tilde, stream));
  return cc_solver_run(ctx->cached, x_next, stats, stream);
}

int cc_collide_step_batched(cc_context* ctx, const cc_scene* scenes, int32_t ns,
                            const cc_params* params, cc_stats* stats, void* stream) {
  if (!ctx || ns < 0 || (ns > 0 && !scenes)) return CC_EINVAL;
  CC_TRY(check_params(params));
  for (int32_t i = 0; i < ns; ++i) {
    const cc_scene& sc = scenes[i];
    if (sc.n_verts < 0 || (sc.n_verts > 0 && !sc.x_next)) return CC_EINVAL;
    if (sc.n_verts > 0 && (sc.x_next == sc.x_prev || sc.x_next == sc.x_tilde)) return CC_EINVAL;
  }
  if (ns == 0) return CC_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  hipStream_t cst = as_stream(stream);
  while ((int32_t)ctx->slots.size() < ns) {
    hipStream_t s = nullptr;
    CC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    ctx->slots.push_back(nullptr);
    ctx->slot_streams.push_back(s);
  }
  // the inputs are produced on the caller's stream: every slot stream waits for it
  hipEvent_t ready = nullptr;
  CC_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  CC_HIP(hipEventRecord(ready, cst));
  for (int32_t i = 0; i < ns; ++i) CC_HIP(hipStreamWaitEvent(ctx->slot_streams[i], ready, 0));
  std::vector<int> rc(ns, CC_OK);
  std::atomic<int32_t> next{0};
  auto worker = [&]() {
    if (hipSetDevice(ctx->device) != hipSuccess) return;
    for (int32_t i = next++; i < ns; i = next++) {
      const cc_scene& sc = scenes[i];
      void* st = (void*)ctx->slot_streams[i];
      int r = bind_solver(ctx, ctx->slots[i], sc.n_verts, sc.inv_mass, sc.tris, sc.n_tris,
                          sc.edges, sc.n_edges, params, st);
      if (r == CC_OK) r = cc_solver_begin(ctx->slots[i], sc.x_prev, sc.x_tilde, st);
      if (r == CC_OK) r = cc_solver_run(ctx->slots[i], sc.x_next, stats ? &stats[i] : nullptr, st);
      rc[i] = r;
    }
  };
  const int32_t nthreads = std::min<int32_t>(ns, 16);
  std::vector<std::thread> pool;
  for (int32_t t = 1; t < nthreads; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  // order the caller's stream after every scene
  for (int32_t i = 0; i < ns; ++i) {
    CC_HIP(hipEventRecord(ready, ctx->slot_streams[i]));
    CC_HIP(hipStreamWaitEvent(cst, ready, 0));
  }
  CC_HIP(hipEventDestroy(ready));
  for (int32_t i = 0; i < ns; ++i)
    if (rc[i] != CC_OK) return rc[i];
  return CC_OK;
}

int cc_solver_get_state(cc_solver* s, double* x, double* y, double* r, double* D_host,
                        void* stream) {
  if (!s) return CC_EINVAL;
  hipStream_t st = as_stream(stream);
  size_t n3 = sizeof(double) * 3 * s->n;
  if (x && s->n) CC_HIP(hipMemcpyAsync(x, s->x, n3, hipMemcpyDefault, st));
  if (y && s->n) CC_HIP(hipMemcpyAsync(y, s->y, n3, hipMemcpyDefault, st));
  if (r && s->n) CC_HIP(hipMemcpyAsync(r, s->r, sizeof(double) * s->n, hipMemcpyDefault, st));
  CC_HIP(hipStreamSynchronize(st));
  if (D_host) *D_host = s->D;
  return CC_OK;
}

int cc_solver_set_state(cc_solver* s, const double* x, const double* y, const double* r,
                        double D, const uint64_t* P, int64_t n_p, void* stream) {
  if (!s || n_p < 0 || (n_p > 0 && !P)) return CC_EINVAL;
  if (!s->begun) return CC_ESTATE;
  hipStream_t st = as_stream(stream);
  size_t n3 = sizeof(double) * 3 * s->n;
  if (n_p > s->capP) CC_TRY(alloc_pairs(s, n_p + n_p / 4 + 1024));
  if (x && s->n) CC_HIP(hipMemcpyAsync(s->x, x, n3, hipMemcpyDefault, st));
  if (y && s->n) CC_HIP(hipMemcpyAsync(s->y, y, n3, hipMemcpyDefault, st));
  if (r && s->n) CC_HIP(hipMemcpyAsync(s->r, r, sizeof(double) * s->n, hipMemcpyDefault, st));
  if (n_p) CC_HIP(hipMemcpyAsync(s->P, P, sizeof(uint64_t) * n_p, hipMemcpyDefault, st));
  CC_HIP(hipStreamSynchronize(st));
  s->nP = n_p;
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
  if (!s || (!out && s->n)) return CC_EINVAL;
  if (s->n) CC_HIP(hipMemcpyAsync(out, s->Di, sizeof(double) * s->n, hipMemcpyDefault, as_stream(stream)));
  CC_HIP(hipStreamSynchronize(as_stream(stream)));
  return CC_OK;
}

int cc_solver_search(cc_solver* s, const double* x, double dmax, uint64_t* keys, int64_t cap,
                     int64_t* n, void* stream) {
  if (!s || !x || !n || !(dmax > 0.0)) return CC_EINVAL;
  hipStream_t st = as_stream(stream);
  CC_TRY(launch_validate(s, x, nullptr, st));
  // the static flags come from the last begin; without one every vertex counts as free
  if (!s->begun && s->n) CC_HIP(hipMemsetAsync(s->stat, 0, s->n, st));
  return lbvh_search(s, x, dmax, keys, keys ? cap : 0, n, st);
}

int cc_solver_stats(cc_solver* s, cc_stats* out) {
  if (!s || !out) return CC_EINVAL;
  *out = s->st;
  return CC_OK;
}

}  // extern "C"
