/*
 * cc.h - C ABI of the MI355X two-way continuous collision handling step.
 *
 * The step (Alg. 1 of "Fast GPU-Based Two-Way Continuous Collision Handling")
 * takes an intersection-free state x^t, a time-integrated target x~ and the mesh
 * topology, and returns an intersection-free x^{t+1}. Inputs and output have the
 * form the paper states for its collision handling module (an x^[k], y^[k+1]
 * pair in, x^[k+1] out; Sec. 7.3). Every iteration runs:
 *   - the proximity search when the reuse bound D has dropped below D_min
 *     (Sec. 3.1): an LBVH over triangles and edges, boxes inflated by D_max/2,
 *     exact FP64 distance filter d < D_max;
 *   - the pair pass: distances at x^(l), P <- {d < D}, A <- {d < delta}, the
 *     per-vertex bounds D_i (Sec. 5);
 *   - the backward step: contact rows linearised at x^(l) (Sec. 4, Sec. 4.1; the
 *     volume form when both closest points are interior, the gap form the section
 *     names otherwise), coloured (Sec. 4.3), one projected Gauss-Seidel sweep,
 *     then the soft unilateral edge-length rows (Sec. 4.2);
 *   - the forward step (Eq. eq:forward2), with the lemma of Sec. 5 checked on the
 *     rounded move (2 |x_new - x| < D_i - eta, else the vertex stays), and the
 *     reductions of Alg. 1;
 *   - the path certificate of the new linear piece over P (lemma of Sec. 5),
 *     with a continuous test (coplanarity cubic, end probes, conservative
 *     advancement) for pairs the bound misses; a pair it does not clear sends its
 *     vertices back to x^(l).
 *
 * Conventions for every function below:
 *   - Array arguments are DEVICE pointers unless the name ends in _host.
 *     Positions are row-major xyz triples of float64 (x[3*i+k]); tris are int32
 *     triples, edges int32 pairs. The caller owns every array it passes; the
 *     library owns only the workspace inside cc_context / cc_solver.
 *   - `stream` is a hipStream_t (NULL = the default stream). Work is stream
 *     ordered; functions that return counts or statistics synchronise `stream`.
 *   - Return value: CC_OK (0) or a negative error code (cc_strerror).
 *     Reaching max_iters is not an error: the result is still safe (Sec. 3,
 *     the method may always report x^(l+1)) and stats.status = CC_MAXITER.
 *   - Not thread safe per context: one host thread per context at a time.
 */
#ifndef CC_H
#define CC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CC_OK = 0,
  CC_EINVAL = -1,    /* bad argument: NULL pointer, negative size, out-of-range or
                        repeated index in a primitive, NaN/Inf position, invalid
                        parameter (d_min < delta, d_max <= d_min, gamma not in (0,1),
                        sigma < 1, eps <= 0, max_iters < 1, gs_sweeps < 1, omega not in
                        (0,1], unknown backward solver, CC_JACOBI or CC_CCD_STEP
                        with CC_MIXED,
                        CC_TIME_ONE with time_kind outside 0..CC_K_COUNT-1) */
  CC_ENOMEM = -2,    /* device allocation failed */
  CC_EOVERFLOW = -3, /* pair capacity exceeded after regrowth */
  CC_EHIP = -4,      /* HIP runtime error */
  CC_ECOLOR = -5,    /* more colours needed than max_colors */
  CC_ESTATE = -6,    /* call out of order (e.g. iterate before begin) */
  CC_EAGAIN = -7,    /* admission would exceed the HBM budget; retry after a release */
  CC_EBUSY = -8,     /* the scene's step is still running */
  CC_ENOTFREE = -9   /* CC_VALIDATE_INPUT: x_prev is not in the free space */
};

enum { CC_CONVERGED = 0, CC_MAXITER = 1 };

/* flags */
#define CC_EDGE_LEN 1u      /* edge-length constraints on (Sec. 4.2); default on */
#define CC_TIME_KERNELS 2u  /* time kernel families with HIP events */
#define CC_TRACE 4u         /* per-iteration set fingerprints */
#define CC_VALIDATE_INPUT 16u /* check at begin that x_prev is in the free space (the
                               paper assumes it, Sec. 3): no vertex-triangle or edge-edge
                               pair closer than 1e-9 m, no edge meeting a triangle it
                               shares no vertex with (FP64 orientations; values within
                               1e-12 of their absolute products count as touching);
                               all-static pairs skipped. Fails with CC_ENOTFREE. Also
                               checks, when a scene is taken in, that its edges hold every
                               side of every triangle (CC_EINVAL otherwise). */
#define CC_CCD_ALL 32u      /* every pair of P' takes the continuous test of the piece, not
                               only those the motion bound (lemma of Sec. 5) leaves
                               uncertified: a check of the path, at its cost */
#define CC_TIME_ONE 64u     /* time one kernel family alone (cc_params.time_kind) with HIP
                               events: the other families run without events around them */
#define CC_MIXED 8u         /* mixed precision: the backward step (constraint values,
                               Jacobians, multipliers and y - x) in FP32; every set
                               decision, distance, D_i, x, the forward step and the
                               continuous test stay FP64 */
#define CC_CCD_STEP 256u    /* the CCD-based step-size scheme that Sec. 5.1 compares the
                               method with (the paper gives no rule; this one): every vertex
                               takes alpha = min(1, 0.5 gamma D^(l) / |y - x|) (the global
                               bound alone, so pairs outside P' cannot meet), then each pair
                               of P' the motion bound does not certify takes the continuous
                               test, and a contact at time t* of its piece scales the steps
                               of its four vertices by gamma t* (a vertex takes the smallest
                               factor; r follows the new alpha); up to 16 such passes while
                               they find contacts, then the certificate's send-back. Not
                               with CC_MIXED */
#define CC_UNGUARDED 128u   /* the forward step exactly as Eq. eq:forward2, without the
                               check of the rounded move (below): the certificate and its
                               response are then the only guard. A test of the
                               certificate; not for production use */

#define CC_NO_AUTOTUNE 512u /* launch shapes at their defaults; without this flag the
                               autotuner measures the variants of a kernel's launch shape
                               the first time a (device, size class) meets it and keeps the
                               fastest for the process (results do not depend on it) */

/* Parameters; defaults are Table 2 of the paper (cc_default_params). */
typedef struct cc_params {
  double delta;      /* activation threshold, 1e-3 m */
  double d_min;      /* proximity search lower bound, 2e-3 m */
  double d_max;      /* proximity search upper bound, 4e-3 m */
  double sigma;      /* edge violation ratio limit, 1.1 */
  double gamma;      /* damping factor on movement, 0.9 */
  double eps;        /* termination threshold on ||r||_inf, 1e-4 */
  double kappa;      /* near-parallel / near-degenerate threshold of the volume form */
  int32_t max_iters; /* L: 512 (dt = 1/100 s) .. 2048 (dt = 1/20 s) */
  int32_t gs_sweeps; /* Gauss-Seidel sweeps per backward step, 1 (Sec. 4.3.1) */
  int32_t max_colors;/* colour palette, <= 1024 */
  uint32_t flags;    /* CC_EDGE_LEN | CC_TIME_KERNELS | CC_TIME_ONE | CC_TRACE | CC_MIXED |
                        CC_VALIDATE_INPUT | CC_CCD_ALL | CC_UNGUARDED | CC_CCD_STEP |
                        CC_NO_AUTOTUNE */
  uint64_t seed;     /* colouring priority seed */
  double omega;      /* CC_JACOBI: under-relaxation factor in (0, 1] (Sec. 4.3.2 names the
                        factor but gives no value; default 0.5) */
  int32_t backward;  /* CC_GAUSS_SEIDEL (default, Sec. 4.3) or CC_JACOBI (Sec. 4.3.2) */
  int32_t time_kind; /* CC_TIME_ONE: the family timed (CC_K_SEARCH .. CC_K_CERT; default 0) */
} cc_params;

/* backward-step solvers */
enum {
  CC_GAUSS_SEIDEL = 0, /* one projected Gauss-Seidel sweep over the colours (the method) */
  CC_JACOBI = 1        /* one projected Jacobi iteration: every row from the same y, the
                          per-vertex updates summed on a 2^-56 m grid (exact, order
                          independent; within rounding of a plain binary64 sum),
                          y += omega * sum; no colouring. FP64 only. */
};

/* Per-iteration record (filled by cc_solver_iterate). Set fingerprints are
 * wrapping sums of a 64-bit mix of each key, so they do not depend on order;
 * they are computed only with CC_TRACE. */
typedef struct cc_iter_info {
  int32_t searched;
  int32_t n_colors;
  int64_t n_p;       /* |P| evaluated by the pair pass */
  int64_t n_pf;      /* |P'| = {d < D} */
  int64_t n_a;       /* |A| = {d < delta} */
  int64_t ccd_fail;  /* pairs of P' that took the continuous test: those the motion
                        bound did not certify (all pairs with CC_CCD_ALL), summed over
                        the certificate's passes */
  int64_t ccd_hits;  /* of those, pairs the continuous test does not clear (it finds
                        them within eta = 1e-12 m along the piece) */
  int64_t n_back;    /* vertices the certificate sent back to x^(l) */
  int64_t n_scaled;  /* CC_CCD_STEP: vertex steps scaled by a contact */
  double d_before;
  double d_after;
  double move_max;
  double r_inf;
  uint64_t fp_pf, fp_a, fp_col;
} cc_iter_info;

/* Kernel families timed with CC_TIME_KERNELS. */
enum {
  CC_K_SEARCH = 0,   /* LBVH build + traversal */
  CC_K_PAIR = 1,     /* pair pass */
  CC_K_COLOR = 2,    /* colouring */
  CC_K_GS = 3,       /* Gauss-Seidel colour passes (contacts and edges) */
  CC_K_FORWARD = 4,  /* forward step + reductions */
  CC_K_CERT = 5,     /* path certificate */
  CC_K_COUNT = 6
};

typedef struct cc_stats {
  int32_t iters;
  int32_t searches;
  int32_t status;        /* CC_CONVERGED or CC_MAXITER */
  int32_t max_colors_used;
  int64_t pair_updates;  /* sum over iterations of |P| in the pair pass */
  int64_t row_updates;   /* sum over iterations of |A| + active edge rows, x sweeps */
  int64_t ccd_fail;
  int64_t ccd_hits;
  int64_t n_back;
  int64_t n_scaled;
  double r_inf;
  double kernel_ms[CC_K_COUNT];        /* with CC_TIME_KERNELS (CC_TIME_ONE: that family) */
  int64_t kernel_launches[CC_K_COUNT];
  double kernel_bytes[CC_K_COUNT];     /* algorithmic bytes moved */
} cc_stats;

typedef struct cc_context cc_context;
typedef struct cc_solver cc_solver;

/* ---- autotuner ---------------------------------------------------------------
 * Kernels whose launch shape is tuned, and the record of one tuning: the device,
 * the kernel, its size class (CC_TUNE_TRAVERSE: 4 floor(log2(queries)) + the
 * dominant query class, 0 vertex-triangle, 1 edge-edge, 2 vertex-vertex), the
 * choice and the measured time of each variant in milliseconds. CC_TUNE_TRAVERSE
 * variants, in the order of ms[]: 8, 16, 32 lanes per traversal group taking one
 * node per step, then 108, 116, 132: the same group sizes taking two nodes per step
 * (their records loaded together). */
enum { CC_TUNE_TRAVERSE = 0 };
typedef struct cc_tune_entry {
  int32_t device, kernel, size_class, choice;
  float ms[8];
} cc_tune_entry;
/* The process-wide tuning table (HOST array out_host, cap entries): *n gets the
 * number of entries; nothing is written when cap is smaller. */
int cc_autotune_entries(cc_tune_entry* out_host, int32_t cap, int32_t* n);
/* Forget every tuning (the next launches measure again). */
void cc_autotune_reset(void);
/* Force a choice for every later launch of the kernel in this process (CC_TUNE_TRAVERSE:
 * 8, 16, 32, 108, 116 or 132 as above; 0 returns to the tuned choices); CC_EINVAL
 * otherwise. */
int cc_autotune_force(int32_t kernel, int32_t choice);

void cc_default_params(cc_params* p);
const char* cc_strerror(int code);

/* The edges of a triangle mesh (HOST arrays): every unordered vertex pair that is
 * a side of some triangle, once, as (min, max), sorted. The edge-edge pairs of
 * the step are drawn from the edge list, so for a triangle mesh it must hold
 * every triangle side (Sec. 5: the pair types are vertex-triangle and
 * edge-edge). *n_edges gets the count; edges_host (2 * cap int32) is written
 * only when cap is large enough (call with cap = 0 to size it). CC_EINVAL on a
 * negative index or a repeated vertex in a triangle. */
int cc_edges_from_tris_host(const int32_t* tris_host, int32_t n_tris, int32_t* edges_host,
                            int32_t cap, int32_t* n_edges);

/* A context binds a device. Destroy releases every workspace. */
int cc_context_create(int device, cc_context** out);
void cc_context_destroy(cc_context* ctx);

/* One collision-handling step: x_next <- TwoWay(x_prev, x_tilde). inv_mass (N)
 * may be NULL (all ones); w = 0 marks static or pinned vertices (scaled lumped
 * mass of Sec. 3; a global scale cancels). `edges` must list every triangle edge
 * for complete edge-edge coverage. x_next must not alias an input. stats may be
 * NULL. The context keeps its workspace between calls. */
int cc_collide_step(cc_context* ctx, const double* x_prev, const double* x_tilde,
                    const double* inv_mass, int32_t n_verts, const int32_t* tris,
                    int32_t n_tris, const int32_t* edges, int32_t n_edges,
                    const cc_params* params, double* x_next, cc_stats* stats,
                    void* stream);

/* One scene of a batch (device pointers as in cc_collide_step). */
typedef struct cc_scene {
  const double* x_prev;
  const double* x_tilde;
  const double* inv_mass;  /* may be NULL (all ones) */
  int32_t n_verts;
  const int32_t* tris;
  int32_t n_tris;
  const int32_t* edges;
  int32_t n_edges;
  double* x_next;          /* output, must not alias the inputs */
} cc_scene;

/* One collision-handling step for each of n_scenes independent scenes of any
 * sizes. Each scene's result equals the result of cc_collide_step on that scene
 * alone, bit for bit. The scenes are segments of one multi-scene engine (a
 * workspace kept in the context between calls): every iteration runs Alg. 1 once
 * for all scenes still iterating, in the same kernel launches, and a scene drops
 * out when it stops (its own stop test or max_iters). The work is issued on
 * `stream`; the call returns when every scene is done. stats (n_scenes entries)
 * may be NULL. An error in any scene is returned (the first in scene order); the
 * other scenes still complete. */
int cc_collide_step_batched(cc_context* ctx, const cc_scene* scenes, int32_t n_scenes,
                            const cc_params* params, cc_stats* stats, void* stream);

/* ---- target of the globally injective normal flow ---------------------------
 * Sec. 7.4, Eq. eq:normal flow: y = x + beta n, n the vertex normals at x (normalised
 * sums of the cross products (x_b - x_a) x (x_c - x_a) of the vertex's triangles, an
 * area weighting; 0 where that sum vanishes), then `iters` Jacobi steps
 * y(v) <- y(v) + alpha (L y)(v) of the cotangent Laplace-Beltrami operator at the
 * current y: (L y)(v) = 1/(2 A_v) sum over the triangles (v, q, r) at v of
 * cot_r (y_q - y_v) + cot_q (y_r - y_v), A_v = a third of their areas (a vertex with
 * A_v = 0 keeps its position). The paper uses three steps. The result is the target
 * y^[k+1] that cc_collide_step then makes intersection free.
 * x (n_verts x 3 FP64), tris (n_tris x 3 int32) and y (n_verts x 3, written) are
 * device pointers; y must not alias x. Sums over a vertex's triangles run in
 * increasing triangle index, so the result does not depend on the launch. The call
 * returns when y is complete (it synchronises `stream`). Errors: CC_EINVAL (NULL
 * pointer with a non-zero size, negative size or iters, non-finite beta or alpha,
 * a vertex index outside [0, n_verts)), CC_ENOMEM, CC_EHIP. */
int cc_normal_flow_target(cc_context* ctx, const double* x, int32_t n_verts,
                          const int32_t* tris, int32_t n_tris, double beta, double alpha,
                          int32_t iters, double* y, void* stream);

/* The same target without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * it). Arguments, layout, result and errors as cc_normal_flow_target; the caller
 * still provides x, tris and y. The work runs in a fixed scratch array compiled
 * into the library (about 7 MiB on each device, held until the process ends), so
 * sizes are limited: n_verts <= 131072 and n_tris <= 262144, else CC_EINVAL. The
 * array's device address is looked up when a context for the device is created
 * (CC_ESTATE if none was). Every call on one device shares that device's array:
 * calls that overlap on one device (other streams or host threads) race. A triangle
 * with an index outside [0, n_verts) is left out of the work and the call returns
 * CC_EINVAL after the stream has synchronised (y is then unspecified). */
int cc_normal_flow_target_noalloc(cc_context* ctx, const double* x, int32_t n_verts,
                                  const int32_t* tris, int32_t n_tris, double beta,
                                  double alpha, int32_t iters, double* y, void* stream);

/* ---- serving: resident scenes admitted by HBM budget ------------------------
 * A resident scene keeps its topology, masses, current state x and its share of
 * the workspace on the device between steps, so each step starts from the
 * previous step's result. All resident scenes are segments of one multi-scene
 * engine owned by a scheduler thread of the context (continuous batching): at
 * each iteration boundary it applies admissions, releases and submitted steps,
 * then runs one iteration for every scene with a step in flight, in shared kernel
 * launches on its own stream. A scene runs one step at a time. Handles are >= 0. */
/* Budget in bytes for the workspaces of resident scenes (0 = unlimited). */
int cc_context_set_budget(cc_context* ctx, size_t hbm_budget_bytes);
/* Bytes a resident scene of this size reserves against the budget. */
size_t cc_scene_bytes(int32_t n_verts, int32_t n_tris, int32_t n_edges);
/* Admit a scene: copies x_prev (its state x^t), inverse masses and topology
 * (scene->x_tilde and x_next are ignored). CC_EAGAIN when over budget. */
int cc_scene_admit(cc_context* ctx, const cc_scene* scene, const cc_params* params,
                   int32_t* handle);
/* Start one step of the scene towards x_tilde (device, N*3) from its resident
 * state. x_tilde must stay valid until cc_scene_poll reports completion.
 * CC_EBUSY if the scene's previous step is still running. */
int cc_scene_submit(cc_context* ctx, int32_t handle, const double* x_tilde);
/* CC_OK when the last submitted step is done: x_next (device, may be NULL) gets the
 * new state and stats (may be NULL) the step's statistics; CC_EBUSY while it runs;
 * the step's error code if it failed. The resident state is the new x either way. */
int cc_scene_poll(cc_context* ctx, int32_t handle, double* x_next, cc_stats* stats);
/* Wait for the scene's step, then free its workspace and budget. */
int cc_scene_release(cc_context* ctx, int32_t handle);

/* ---- resident solver: the same step split into its phases ------------------
 * A solver keeps one scene's topology, state (x, y, r, D, P) and workspace on
 * the device. cc_collide_step is begin + iterate until stop + copy out. */
int cc_solver_create(cc_context* ctx, int32_t n_verts, const double* inv_mass,
                     const int32_t* tris, int32_t n_tris, const int32_t* edges,
                     int32_t n_edges, const cc_params* params, cc_solver** out,
                     void* stream);
void cc_solver_destroy(cc_solver* s);
/* Alg. 1 initialisation (x <- x^[k], y <- y^[k+1], D <- 0, r <- 1, P <- {}) and the
 * edge-length rows at y^[k+1] with their colouring. */
int cc_solver_begin(cc_solver* s, const double* x_prev, const double* x_tilde, void* stream);
/* One loop iteration of Alg. 1. *stop = 1 when ||r||_inf < eps. info may be NULL. */
int cc_solver_iterate(cc_solver* s, int32_t* stop, cc_iter_info* info, void* stream);
/* Iterate until stop or max_iters; copy x to x_out (device). */
int cc_solver_run(cc_solver* s, double* x_out, cc_stats* stats, void* stream);
/* State access (device arrays of N*3, N*3, N; any may be NULL). */
int cc_solver_get_state(cc_solver* s, double* x, double* y, double* r, double* D_host,
                        void* stream);
/* Replace the state and P (keys, device); used to check one iteration in lockstep. */
int cc_solver_set_state(cc_solver* s, const double* x, const double* y, const double* r,
                        double D, const uint64_t* P, int64_t n_p, void* stream);
/* Sets of the last pair pass: P' keys, A keys with their colours, D_i. *n gets the
 * size; nothing is written when cap is smaller. */
int cc_solver_get_P(cc_solver* s, uint64_t* keys, int64_t cap, int64_t* n, void* stream);
int cc_solver_get_A(cc_solver* s, uint64_t* keys, int32_t* colors, int64_t cap, int64_t* n,
                    void* stream);
int cc_solver_get_Di(cc_solver* s, double* out, void* stream);
/* The proximity search alone at state x with bound dmax (LBVH + exact filter). */
int cc_solver_search(cc_solver* s, const double* x, double dmax, uint64_t* keys, int64_t cap,
                     int64_t* n, void* stream);
/* Accumulated statistics since begin. */
int cc_solver_stats(cc_solver* s, cc_stats* out);

#ifdef __cplusplus
}
#endif
#endif
