// Serving: resident scenes admitted against an HBM budget, steps run by a worker
// pool with one stream per scene so that the steps of different scenes overlap
// on the device. A scene keeps its state x between steps: each step starts from
// the previous step's result.
#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>

#include "internal.hpp"

namespace {

enum { kIdle = 0, kRunning = 1, kDone = 2 };

struct Served {
  cc_solver* s = nullptr;
  hipStream_t stream = nullptr;
  size_t bytes = 0;
  std::atomic<int> state{kIdle};
  int rc = CC_OK;
  const double* xt = nullptr;
  cc_stats st{};
};

}  // namespace

struct cc_server {
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<int32_t> queue;
  std::vector<std::thread> workers;
  std::vector<Served*> scenes;  // handle -> scene (nullptr = free slot)
  size_t budget = 0, used = 0;
  bool stop = false;
};

namespace {

void worker_loop(cc_context* ctx, cc_server* sv) {
  if (hipSetDevice(ctx->device) != hipSuccess) return;
  for (;;) {
    int32_t h;
    Served* sc;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
      if (sv->stop && sv->queue.empty()) return;
      h = sv->queue.front();
      sv->queue.pop_front();
      sc = sv->scenes[h];
    }
    // one step from the resident state: x_prev is the scene's own x
    void* st = (void*)sc->stream;
    int rc = cc_solver_begin(sc->s, sc->s->x, sc->xt, st);
    if (rc == CC_OK) rc = cc_solver_run(sc->s, nullptr, &sc->st, st);
    sc->rc = rc;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sc->state.store(kDone);
    }
    sv->done_cv.notify_all();
  }
}

cc_server* server_of(cc_context* ctx) {
  if (!ctx->server) ctx->server = new cc_server();
  return ctx->server;
}

void start_workers(cc_context* ctx, cc_server* sv) {
  if (!sv->workers.empty()) return;
  unsigned hw = std::thread::hardware_concurrency();
  int n = (int)(hw ? (hw < 8 ? hw : 8) : 4);
  for (int i = 0; i < n; ++i) sv->workers.emplace_back(worker_loop, ctx, sv);
}

Served* get(cc_server* sv, int32_t h) {
  if (h < 0 || h >= (int32_t)sv->scenes.size()) return nullptr;
  return sv->scenes[h];
}

}  // namespace

namespace cc {

void server_destroy(cc_context* ctx) {
  cc_server* sv = ctx->server;
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  for (auto& t : sv->workers) t.join();
  for (Served* sc : sv->scenes) {
    if (!sc) continue;
    cc_solver_destroy(sc->s);
    (void)hipStreamDestroy(sc->stream);
    delete sc;
  }
  delete sv;
  ctx->server = nullptr;
}

}  // namespace cc

extern "C" {

size_t cc_scene_bytes(int32_t n, int32_t nt, int32_t ne) {
  if (n < 0 || nt < 0 || ne < 0) return 0;
  // the solver's allocations: per-vertex state, colouring masks and sort keys;
  // per-primitive topology, tree records, boxes and sort keys; the initial pair
  // and active-set buffers (32 (n + e) pairs, an eighth of that active); fixed
  // colouring and round buffers.
  const size_t per_v = 8 + 1 + 4 * 24 + 8 + 8 + 8 + 2 * 8 + 16 * 8 + 4 + 16;
  const size_t per_prim = 32 + 8 + 64 + 128 + 8 + 8 + 64 + 32 + 16;
  const size_t per_e = 8 + 24 + 8 + 4 + 4 + 12 + 8;
  const size_t pair_cap = 32 * ((size_t)n + (size_t)ne);
  const size_t pairs = pair_cap * 32 + (pair_cap / 8) * (8 + 16 + 4 + 4 + 8 + 8);
  const size_t fixed = (size_t)(cc::kMaxRounds + 1) * 8 + 4 * (cc::kMaxColors + 1) * 4 + (1 << 20);
  return per_v * (size_t)n + per_prim * ((size_t)nt + ne) + 12 * (size_t)nt + per_e * ne + pairs +
         fixed;
}

int cc_context_set_budget(cc_context* ctx, size_t bytes) {
  if (!ctx) return CC_EINVAL;
  cc_server* sv = server_of(ctx);
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->budget = bytes;
  return CC_OK;
}

int cc_scene_admit(cc_context* ctx, const cc_scene* scene, const cc_params* params,
                   int32_t* handle) {
  if (!ctx || !scene || !params || !handle) return CC_EINVAL;
  if (scene->n_verts < 0 || (scene->n_verts > 0 && !scene->x_prev)) return CC_EINVAL;
  cc_server* sv = server_of(ctx);
  const size_t bytes = cc_scene_bytes(scene->n_verts, scene->n_tris, scene->n_edges);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->budget && sv->used + bytes > sv->budget) return CC_EAGAIN;
    sv->used += bytes;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  Served* sc = new Served();
  sc->bytes = bytes;
  int rc = hipStreamCreateWithFlags(&sc->stream, hipStreamNonBlocking) == hipSuccess ? CC_OK : CC_EHIP;
  if (rc == CC_OK)
    rc = cc_solver_create(ctx, scene->n_verts, scene->inv_mass, scene->tris, scene->n_tris,
                          scene->edges, scene->n_edges, params, &sc->s, (void*)sc->stream);
  if (rc == CC_OK && scene->n_verts) {
    rc = hipMemcpyAsync(sc->s->x, scene->x_prev, sizeof(double) * 3 * scene->n_verts,
                        hipMemcpyDefault, sc->stream) == hipSuccess ? CC_OK : CC_EHIP;
    if (rc == CC_OK) rc = hipStreamSynchronize(sc->stream) == hipSuccess ? CC_OK : CC_EHIP;
  }
  if (rc != CC_OK) {
    if (sc->s) cc_solver_destroy(sc->s);
    if (sc->stream) (void)hipStreamDestroy(sc->stream);
    delete sc;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->used -= bytes;
    return rc;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  int32_t h = -1;
  for (int32_t i = 0; i < (int32_t)sv->scenes.size(); ++i)
    if (!sv->scenes[i]) {
      h = i;
      break;
    }
  if (h < 0) {
    h = (int32_t)sv->scenes.size();
    sv->scenes.push_back(nullptr);
  }
  sv->scenes[h] = sc;
  start_workers(ctx, sv);
  *handle = h;
  return CC_OK;
}

int cc_scene_submit(cc_context* ctx, int32_t handle, const double* x_tilde) {
  if (!ctx || !ctx->server) return CC_EINVAL;
  cc_server* sv = ctx->server;
  std::lock_guard<std::mutex> lk(sv->mu);
  Served* sc = get(sv, handle);
  if (!sc || (sc->s->n > 0 && !x_tilde)) return CC_EINVAL;
  if (sc->state.load() == kRunning) return CC_EBUSY;
  sc->xt = x_tilde;
  sc->rc = CC_OK;
  sc->state.store(kRunning);
  sv->queue.push_back(handle);
  sv->cv.notify_one();
  return CC_OK;
}

int cc_scene_poll(cc_context* ctx, int32_t handle, double* x_next, cc_stats* stats) {
  if (!ctx || !ctx->server) return CC_EINVAL;
  cc_server* sv = ctx->server;
  Served* sc;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sc = get(sv, handle);
  }
  if (!sc) return CC_EINVAL;
  const int st = sc->state.load();
  if (st == kRunning) return CC_EBUSY;
  if (st == kIdle) return CC_ESTATE;
  if (sc->rc != CC_OK) return sc->rc;
  if (x_next && sc->s->n) {
    if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
    CC_HIP(hipMemcpyAsync(x_next, sc->s->x, sizeof(double) * 3 * sc->s->n, hipMemcpyDefault,
                          sc->stream));
    CC_HIP(hipStreamSynchronize(sc->stream));
  }
  if (stats) *stats = sc->st;
  return CC_OK;
}

int cc_scene_release(cc_context* ctx, int32_t handle) {
  if (!ctx || !ctx->server) return CC_EINVAL;
  cc_server* sv = ctx->server;
  Served* sc;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sc = get(sv, handle);
    if (!sc) return CC_EINVAL;
    sv->done_cv.wait(lk, [&] { return sc->state.load() != kRunning; });
    sv->scenes[handle] = nullptr;
    sv->used -= sc->bytes;
  }
  cc_solver_destroy(sc->s);
  (void)hipStreamDestroy(sc->stream);
  delete sc;
  return CC_OK;
}

}  // extern "C"
