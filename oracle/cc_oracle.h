/*
 * FP64 CPU oracle of the two-way continuous collision handling step.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. The HIP product path never
 * includes this header, links this library, or shares code with it.
 *
 * What it computes: Alg. 1 of the paper (the two-way method) with the backward
 * step of Sec. 4 (LCP of Eq. eqn:LCP, linearised at x^(l), one projected
 * multi-colour Gauss-Seidel sweep, volume-based contact constraints of
 * Sec. 4.1, soft unilateral edge-length constraints of Sec. 4.2) and the forward
 * step of Sec. 5 (Eq. eq:forward2 with per-vertex bounds D_i). Readings where the
 * paper is silent are listed in the design notes of the repository and in the
 * comments of cc_oracle.c.
 *
 * Arrays are row-major: x[3*i+k], tris[3*f+k], edges[2*e+k].
 * Parity unpinned: the edge-edge volume constraint, the degenerate fallbacks and
 * the colouring priority are readings, not formulas printed in the paper.
 */
#ifndef CC_ORACLE_H
#define CC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
  double delta;      /* activation threshold (Table 2: 1 mm) */
  double d_min;      /* proximity search lower bound (Table 2: 2 mm) */
  double d_max;      /* proximity search upper bound (Table 2: 4 mm) */
  double sigma;      /* edge violation ratio limit (Table 2: 1.1) */
  double gamma;      /* damping factor on movement (Table 2: 0.9) */
  double eps;        /* termination threshold on ||r||_inf (Table 2: 1e-4) */
  double kappa;      /* near-degenerate test for the volume form (reading) */
  int32_t max_iters; /* L */
  int32_t gs_sweeps; /* Gauss-Seidel sweeps per backward step (Sec. 4.3.1: 1) */
  int32_t max_colors;/* colour palette size (<= 1024) */
  int32_t edge_len;  /* 1: edge-length constraints on (Sec. 4.2) */
  uint64_t seed;     /* colouring priority seed */
  double omega;      /* projected Jacobi: under-relaxation factor (Sec. 4.3.2 gives none) */
  int32_t backward;  /* 0: projected Gauss-Seidel over colours (Sec. 4.3, the method);
                        1: projected Jacobi (Sec. 4.3.2) */
  int32_t ccd_all;   /* 1: every pair of P' takes the continuous test, not only those the
                        motion bound leaves uncertified (a check of the lemma of Sec. 5) */
  int32_t unguarded; /* 1: the forward step exactly as Eq. eq:forward2, without the
                        check of the rounded move; the certificate is then the only
                        guard (a test of the certificate's response) */
  int32_t ccd_step;  /* 1: the CCD-based step-size scheme that Sec. 5.1 compares with:
                        every vertex bounded by D^(l) only, then contacts found by the
                        continuous test along P' scale the steps */
} orc_params;

typedef struct orc_iter {
  int32_t searched;      /* proximity search ran this iteration */
  int32_t n_colors;      /* colours of the contact rows */
  int64_t n_p;           /* |P| evaluated by the pair pass */
  int64_t n_pf;          /* |P'| = pairs with d < D^(l) */
  int64_t n_a;           /* |A| = pairs with d < delta */
  int64_t ccd_fail;      /* pairs of P' that took the continuous test: those the motion
                            bound does not certify, or all with ccd_all (summed over
                            the certificate's passes) */
  int64_t ccd_hits;      /* pairs the continuous test does not clear (all passes) */
  int64_t n_back;        /* vertices the certificate returned to x^(l) */
  int64_t n_scaled;      /* CCD-based step: vertex steps scaled by a contact */
  double d_before;       /* D^(l) used by the pair pass */
  double d_after;        /* D^(l+1) */
  double move_max;       /* max_i ||x_i^(l+1) - x_i^(l)|| */
  double r_inf;          /* ||r^(l+1)||_inf */
  uint64_t fp_pf, fp_a, fp_col; /* order-independent set fingerprints */
} orc_iter;

typedef struct orc_scene orc_scene;

/* Create a scene. w: inverse masses (N); tris (F,3); edges (E,2). Copies all. */
orc_scene* orc_create(int32_t n, const double* w, const int32_t* tris, int32_t nt,
                      const int32_t* edges, int32_t ne, const orc_params* p);
void orc_destroy(orc_scene* s);
/* Alg. 1 initialisation: x <- x^[k], y <- y^[k+1], D <- 0, r <- 1, P <- empty. */
int orc_begin(orc_scene* s, const double* x_prev, const double* x_tilde);
/* One iteration of the loop of Alg. 1. Returns 1 if the stop test holds, 0 if not,
 * <0 on error. */
int orc_iterate(orc_scene* s, orc_iter* info);
/* Full step: iterate until the stop test or max_iters. Returns iterations run. */
int orc_run(orc_scene* s, double* x_out, orc_iter* trace, int32_t trace_cap);

/* State access (lockstep checks). */
void orc_get_state(const orc_scene* s, double* x, double* y, double* r, double* D);
int orc_set_state(orc_scene* s, const double* x, const double* y, const double* r,
                  double D, const uint64_t* P, int64_t nP);
int64_t orc_get_P(const orc_scene* s, uint64_t* out, int64_t cap);
int64_t orc_get_A(const orc_scene* s, uint64_t* keys, int32_t* colors, int64_t cap);
void orc_get_Di(const orc_scene* s, double* out);

/* Building blocks (pinned individually by the tests). */
double orc_pt_tri_d2(const double* p, const double* a, const double* b,
                     const double* c, double* bary);
double orc_seg_seg_d2(const double* a, const double* b, const double* c,
                      const double* e, double* st);
/* Pair keys: vertex-triangle a << 32 | f; edge-edge 1 << 63 | e << 32 | g (e < g);
 * vertex-vertex 1 << 62 | a << 32 | b (a < b, both particles). Ids below 2^30. */
/* Contact row at state x for pair key: vertex ids v[4] (-1 = none), c0, J[12], invA.
 * Returns 0 for the volume form, 1 for the gap fallback, 2 if inactive. */
int orc_contact_row(const orc_scene* s, const double* x, uint64_t key,
                    int32_t* v, double* c0, double* J, double* inv_a);
/* Proximity search: every pair of the universe with d < dmax at state x.
 * brute != 0 uses the all-pairs loop instead of the grid. Result sorted by key. */
int64_t orc_search(orc_scene* s, const double* x, double dmax, int brute,
                   uint64_t* out, int64_t cap);
/* Colouring of rows with vertex lists rv[4*r] (-1 = none, each vertex listed once):
 * rows sharing a vertex with w > 0 get different colours; randomised palette
 * rounds whose choices hash the row key, the seed and the round. Returns the
 * number of colours, <0 on error. */
int32_t orc_color_rows(const orc_scene* s, int64_t nrows, const int32_t* rv,
                       const uint64_t* keys, int32_t* colors);
/* Greedy colouring of rows in decreasing orc_greedy_prio(key, seed) order (the
 * edge-length rows' colouring); same arguments and result as orc_color_rows. */
int32_t orc_color_rows_greedy(const orc_scene* s, int64_t nrows, const int32_t* rv,
                              const uint64_t* keys, int32_t* colors);
uint64_t orc_greedy_prio(uint64_t key, uint64_t seed);
uint64_t orc_mix64(uint64_t z);
/* Continuous test of a pair along q_k + t dq_k, t in [0,1] (q, dq: the points in
 * the contact-row order). kind 0: vertex-triangle (4 points), 1: edge-edge (4),
 * 2: vertex-vertex (2). Returns 1 when the primitives come within eta. */
int orc_ccd_hit(const double* q, const double* dq, int kind, double eta, double* t_hit);
/* Number of particles (vertices in no triangle and no edge: the vertex-vertex
 * pair universe) and their ids, increasing (ids may be NULL). */
int32_t orc_particles(const orc_scene* s, int32_t* ids);
/* Segment pq against triangle abc: 1 when they cross or touch (FP64 orientations;
 * values within 1e-12 of their absolute products count as touching; a segment in
 * the triangle's plane decides by its distance <= tol). */
int orc_seg_tri_meet(const double* p, const double* q, const double* a, const double* b,
                     const double* c, double tol);
/* Input check at x (x^t of a step): 1 when a vertex-triangle or edge-edge pair is
 * closer than tol or an edge meets a triangle it shares no vertex with (all-static
 * pairs skipped; the static flags of the last begin are used). */
int orc_validate(orc_scene* s, const double* x, double tol);
/* Target of the globally injective normal flow at x (Sec. 7.4, Eq. eq:normal flow):
 * y_0 = x + beta n (area-weighted vertex normals), then `iters` Jacobi steps of the
 * cotangent Laplacian at the current y with intensity alpha. Returns 0, or -1 on a
 * bad argument. */
int orc_normal_flow(int32_t n, const double* x, const int32_t* tris, int32_t nt, double beta,
                    double alpha, int32_t iters, double* y_out);

#ifdef __cplusplus
}
#endif
#endif
