// Serving: continuous batching of collision-handling steps over resident scenes.
//
// Admitted scenes live in one multi-scene engine (their state, topology and
// pairs stay on the device between steps). A scheduler thread owns the engine:
// at every iteration boundary it applies queued admissions, releases and step
// submissions, then runs one iteration of Alg. 1 for all running scenes in the
// same kernel launches. A scene whose step ends (converged or at its iteration
// limit) has its state copied to its own result buffer, where cc_scene_poll
// picks it up; a new step can join at the next boundary while others continue.
#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>

#include "internal.hpp"

namespace {

enum { kIdle = 0, kQueued = 1, kRunning = 2, kDone = 3 };

struct Served {
  int32_t seg = -1;
  int32_t nv = 0;
  size_t bytes = 0;
  std::atomic<int> state{kIdle};
  int rc = CC_OK;
  const double* xt = nullptr;
  double* result = nullptr;  // x after the last finished step (device, nv*3)
  cc_stats st{};
};

struct Cmd {
  enum Kind { kAdmit, kRelease } kind;
  Served* sc = nullptr;
  cc_scene scene{};
  int32_t max_iters = 0;
  int rc = CC_OK;
  bool done = false;
};

}  // namespace

struct cc_server {
  std::mutex mu;
  std::condition_variable cv;       // wakes the scheduler
  std::condition_variable done_cv;  // wakes callers waiting on commands and steps
  std::deque<Cmd*> cmds;
  std::deque<Served*> to_begin;
  std::vector<Served*> scenes;  // handle -> scene (nullptr = free)
  cc_solver* eng = nullptr;
  cc_params p{};
  bool have_params = false;
  hipStream_t stream = nullptr;       // the scheduler's
  hipStream_t poll_stream = nullptr;  // result copies for callers
  std::thread sched;
  bool running = false;
  size_t budget = 0, used = 0;
  bool stop = false;
};

namespace {

bool same_params(const cc_params& a, const cc_params& b) {
  return a.delta == b.delta && a.d_min == b.d_min && a.d_max == b.d_max && a.sigma == b.sigma &&
         a.gamma == b.gamma && a.eps == b.eps && a.kappa == b.kappa &&
         a.gs_sweeps == b.gs_sweeps && a.max_colors == b.max_colors &&
         (a.flags & ~(CC_TIME_KERNELS | CC_TIME_ONE)) ==
             (b.flags & ~(CC_TIME_KERNELS | CC_TIME_ONE)) &&
         a.seed == b.seed;
}

int do_admit(cc_context* ctx, cc_server* sv, Cmd* c) {
  Served* sc = c->sc;
  const cc_scene& s = c->scene;
  if (!sv->eng)
    CC_TRY(cc::engine_create(ctx, &sv->p, s.n_verts, s.n_tris, s.n_edges, &sv->eng, sv->stream));
  int32_t sg = -1;
  CC_TRY(cc::seg_add(sv->eng, s.n_verts, s.inv_mass, s.tris, s.n_tris, s.edges, s.n_edges,
                     c->max_iters, &sg, sv->stream));
  cc_solver* e = sv->eng;
  const cc::Seg& g = e->segs[sg];
  int rc = CC_OK;
  if (s.n_verts > 0) {
    rc = cc::launch_check_finite(e, s.x_prev, nullptr, s.n_verts, sv->stream);
    if (rc == CC_OK && hipMalloc((void**)&sc->result, sizeof(double) * 3 * s.n_verts) != hipSuccess)
      rc = CC_ENOMEM;
    if (rc == CC_OK &&
        hipMemcpyAsync(e->x + 3 * (int64_t)g.vb, s.x_prev, sizeof(double) * 3 * s.n_verts,
                       hipMemcpyDefault, sv->stream) != hipSuccess)
      rc = CC_EHIP;
    if (rc == CC_OK && hipStreamSynchronize(sv->stream) != hipSuccess) rc = CC_EHIP;
  }
  if (rc != CC_OK) {
    cc::seg_remove(e, sg, sv->stream);
    if (sc->result) (void)hipFree(sc->result);
    sc->result = nullptr;
    return rc;
  }
  sc->seg = sg;
  sc->nv = s.n_verts;
  return CC_OK;
}

void finish(cc_server* sv, Served* sc, int rc) {
  cc_solver* e = sv->eng;
  if (rc == CC_OK && sc->nv > 0) {
    const cc::Seg& g = e->segs[sc->seg];
    if (hipMemcpyAsync(sc->result, e->x + 3 * (int64_t)g.vb, sizeof(double) * 3 * sc->nv,
                       hipMemcpyDeviceToDevice, sv->stream) != hipSuccess ||
        hipStreamSynchronize(sv->stream) != hipSuccess)
      rc = CC_EHIP;
  }
  if (rc == CC_OK) cc::seg_stats(e, sc->seg, &sc->st);
  sc->rc = rc;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sc->state.store(kDone);
  }
  sv->done_cv.notify_all();
}

void scheduler(cc_context* ctx, cc_server* sv) {
  if (hipSetDevice(ctx->device) != hipSuccess) return;
  std::vector<Served*> running;
  for (;;) {
    std::deque<Cmd*> cmds;
    std::deque<Served*> begins;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv.wait(lk, [&] {
        return sv->stop || !sv->cmds.empty() || !sv->to_begin.empty() || !running.empty();
      });
      if (sv->stop && sv->cmds.empty() && running.empty() && sv->to_begin.empty()) return;
      cmds.swap(sv->cmds);
      begins.swap(sv->to_begin);
    }
    for (Cmd* c : cmds) {
      int rc = CC_OK;
      if (c->kind == Cmd::kAdmit) {
        rc = do_admit(ctx, sv, c);
      } else {
        Served* sc = c->sc;
        if (sc->seg >= 0) rc = cc::seg_remove(sv->eng, sc->seg, sv->stream);
        if (sc->result) (void)hipFree(sc->result);
        sc->result = nullptr;
      }
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        c->rc = rc;
        c->done = true;
      }
      sv->done_cv.notify_all();
    }
    if (!begins.empty()) {
      std::vector<int32_t> segs;
      std::vector<const double*> xp, xt;
      for (Served* sc : begins) {
        segs.push_back(sc->seg);
        xp.push_back(nullptr);  // from the resident state
        xt.push_back(sc->xt);
      }
      std::vector<int> rcs(segs.size(), CC_OK);
      int r = cc::seg_begin(sv->eng, segs.data(), (int32_t)segs.size(), xp.data(), xt.data(),
                            rcs.data(), sv->stream);
      for (size_t k = 0; k < begins.size(); ++k) {
        if (r != CC_OK || rcs[k] != CC_OK) {
          sv->eng->segs[begins[k]->seg].active = false;
          finish(sv, begins[k], rcs[k] != CC_OK ? rcs[k] : r);
        } else {
          running.push_back(begins[k]);
        }
      }
    }
    if (running.empty()) continue;
    int r = cc::engine_iterate(sv->eng, sv->stream);
    std::vector<Served*> still;
    for (Served* sc : running) {
      cc::Seg& g = sv->eng->segs[sc->seg];
      if (r != CC_OK) {
        g.active = false;
        finish(sv, sc, r);
      } else if (!g.active) {
        finish(sv, sc, CC_OK);
      } else {
        still.push_back(sc);
      }
    }
    running.swap(still);
  }
}

cc_server* server_of(cc_context* ctx) {
  if (!ctx->server) ctx->server = new cc_server();
  return ctx->server;
}

int start(cc_context* ctx, cc_server* sv) {
  if (sv->running) return CC_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
  if (!sv->stream) CC_HIP(hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking));
  if (!sv->poll_stream) CC_HIP(hipStreamCreateWithFlags(&sv->poll_stream, hipStreamNonBlocking));
  sv->sched = std::thread(scheduler, ctx, sv);
  sv->running = true;
  return CC_OK;
}

// Queue a command for the scheduler and wait until it has been applied.
int run_cmd(cc_server* sv, Cmd* c) {
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cmds.push_back(c);
  sv->cv.notify_all();
  sv->done_cv.wait(lk, [&] { return c->done; });
  return c->rc;
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
  if (sv->running) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
    }
    sv->cv.notify_all();
    sv->sched.join();
  }
  for (Served* sc : sv->scenes) {
    if (!sc) continue;
    if (sc->result) (void)hipFree(sc->result);
    delete sc;
  }
  if (sv->eng) cc_solver_destroy(sv->eng);
  if (sv->stream) (void)hipStreamDestroy(sv->stream);
  if (sv->poll_stream) (void)hipStreamDestroy(sv->poll_stream);
  delete sv;
  ctx->server = nullptr;
}

}  // namespace cc

extern "C" {

size_t cc_scene_bytes(int32_t n, int32_t nt, int32_t ne) {
  if (n < 0 || nt < 0 || ne < 0) return 0;
  // per vertex: w, x, y, x~, x^(l), r, move, D_i, segment id, static flag,
  // colouring counts, masks, claims, clashes and block slot, sort keys and values,
  // query order;
  // per triangle: topology, boxes, tree records (binary and 4-wide), refit
  // unions, sort keys; per edge: the same plus the edge row and its colouring;
  // pairs: 32 (N + E) of P, P' and their distances, an eighth of that active (with
  // the linearised contact row).
  const size_t per_v = 8 + 4 * 24 + 8 + 8 + 8 + 4 + 1 + 8 + 16 * 8 + 32 * 8 + 4 + 2 * 12 + 4 + 2;
  const size_t per_prim = 32 + 4 + 64 + 128 + 8 + 8 + 64 + 32 + 2 * 12;
  const size_t per_e = 8 + 4 + 24 + 8 + 4 + 4 + 12 + 8 + 2;
  const size_t pair_cap = 32 * ((size_t)n + (size_t)ne);
  const size_t pairs = pair_cap * 32 + (pair_cap / 8) * (8 + 16 + 4 + 4 + 8 + 8 + 8 + 8 * cc::kRowWords);
  // particles (vertices in no triangle or edge): at least n - 3F - 2E of them, each a
  // leaf of the particle tree and a search key
  const int64_t np = std::max<int64_t>(0, (int64_t)n - 3 * (int64_t)nt - 2 * (int64_t)ne);
  return per_v * (size_t)n + per_prim * ((size_t)nt + ne + (size_t)np) + 12 * (size_t)nt +
         per_e * ne + 4 * (size_t)n + pairs;
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
  if (scene->n_verts < 0 || scene->n_tris < 0 || scene->n_edges < 0) return CC_EINVAL;
  if (scene->n_verts > 0 && !scene->x_prev) return CC_EINVAL;
  CC_TRY(cc::check_params(params));
  cc_server* sv = server_of(ctx);
  const size_t bytes = cc_scene_bytes(scene->n_verts, scene->n_tris, scene->n_edges);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->have_params && !same_params(sv->p, *params)) return CC_EINVAL;
    if (sv->budget && sv->used + bytes > sv->budget) return CC_EAGAIN;
    sv->used += bytes;
    if (!sv->have_params) {
      sv->p = *params;
      sv->have_params = true;
    }
  }
  int rc = start(ctx, sv);
  Served* sc = new Served();
  sc->bytes = bytes;
  Cmd c;
  c.kind = Cmd::kAdmit;
  c.sc = sc;
  c.scene = *scene;
  c.max_iters = params->max_iters;
  if (rc == CC_OK) rc = run_cmd(sv, &c);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (rc != CC_OK) {
    sv->used -= bytes;
    delete sc;
    return rc;
  }
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
  *handle = h;
  return CC_OK;
}

int cc_scene_submit(cc_context* ctx, int32_t handle, const double* x_tilde) {
  if (!ctx || !ctx->server) return CC_EINVAL;
  cc_server* sv = ctx->server;
  std::lock_guard<std::mutex> lk(sv->mu);
  Served* sc = get(sv, handle);
  if (!sc || (sc->nv > 0 && !x_tilde)) return CC_EINVAL;
  const int st = sc->state.load();
  if (st == kQueued || st == kRunning) return CC_EBUSY;
  sc->xt = x_tilde;
  sc->rc = CC_OK;
  sc->state.store(kRunning);
  sv->to_begin.push_back(sc);
  sv->cv.notify_all();
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
  if (st == kQueued || st == kRunning) return CC_EBUSY;
  if (st == kIdle) return CC_ESTATE;
  if (sc->rc != CC_OK) return sc->rc;
  if (x_next && sc->nv) {
    if (hipSetDevice(ctx->device) != hipSuccess) return CC_EHIP;
    CC_HIP(hipMemcpyAsync(x_next, sc->result, sizeof(double) * 3 * sc->nv, hipMemcpyDefault,
                          sv->poll_stream));
    CC_HIP(hipStreamSynchronize(sv->poll_stream));
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
    sv->done_cv.wait(lk, [&] {
      const int s = sc->state.load();
      return s != kQueued && s != kRunning;
    });
    sv->scenes[handle] = nullptr;
  }
  Cmd c;
  c.kind = Cmd::kRelease;
  c.sc = sc;
  int rc = run_cmd(sv, &c);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->used -= sc->bytes;
  }
  delete sc;
  return rc;
}

}  // extern "C"
