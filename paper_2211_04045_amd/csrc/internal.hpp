// Internal declarations of the HIP collision-handling library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <utility>
#include <vector>

#include "../../include/cc.h"

namespace cc {

#define CC_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return CC_EHIP;             \
  } while (0)

#define CC_TRY(call)                                  \
  do {                                                \
    int r_ = (call);                                  \
    if (r_ != CC_OK) return r_;                       \
  } while (0)

constexpr int kMaxColors = 1024;
constexpr int kMaskWords = kMaxColors / 64;
constexpr int kMaxRounds = 4096;  // colouring rounds per colouring
// eta (m): primitives closer than eta count as touching (continuous test), and the
// forward step keeps a vertex's rounded move below (D_i - eta) / 2; binary64
// distances of scenes with coordinates within +-10 m are exact to far better
constexpr double kEta = 1e-12;
// certificate queue entry: bit 63 set when the motion bound certified the pair
constexpr unsigned long long kQueueCertified = 1ull << 63;
constexpr unsigned long long kOneBits = 0x3FF0000000000000ull;  // bits of 1.0
constexpr int kStepPasses = 16;  // CCD-based step: passes that scale steps
constexpr int kMaxSeg = 1024;      // scenes (segments) resident in one solver
// the shared readback block: stripe counts (64 x 128 B), counters, segment records
constexpr size_t kMirrorStripe = 0, kMirrorCounters = 8192, kMirrorSeg = 8192 + 256;
constexpr int kSegBits = 10;       // bits of a segment's rank in a search's sort keys
constexpr int32_t kMaxIds = 1 << 30;  // primitive ids of pair keys are 30-bit
constexpr double kFreeTol = 1e-9;  // input check: closest allowed distance (m)
constexpr int kRowWords = 20;      // one linearised contact row: ids, c0, 1/A, w[4], J[4]
constexpr int kSmallRows = 4096;   // contact sets up to this size are coloured by one block
// vertices a one-block colouring holds in LDS with one colour word each
constexpr int kLocCap1 = 4096;

// Per-segment record on the device (one scene of a multi-scene solver). The host
// writes D, D2, bases and flags before an iteration and reads the reductions back.
struct SegDev {
  double D;                     // D^(l) of the segment
  double D2;                    // D^(l) squared (pair filter)
  int32_t vb, fb, eb;           // first vertex, triangle and edge of the segment
  int32_t flags;                // kSegActive | kSegSearched
  unsigned long long mmax_bits; // max ||dx|| of the forward step (double bits)
  unsigned long long rinf_bits; // max r after the forward step
  unsigned long long fail;      // certificate failures
  unsigned long long hits;      // continuous-test contacts
  unsigned long long n_p;       // pairs evaluated by the pair pass
  unsigned long long n_pf;      // |P'|
  unsigned long long n_a;       // |A|
  unsigned long long n_rows;    // valid edge-length rows (setup)
  unsigned long long nback;     // vertices the certificate sent back to x^(l)
  unsigned long long nstep;     // CCD-based step: uncertified pairs in contact (all passes)
  unsigned long long nscaled;   // CCD-based step: vertex steps scaled
  unsigned long long pad[1];
};
static_assert(sizeof(SegDev) == 128, "SegDev is one 128-byte record");
constexpr int32_t kSegActive = 1;    // the segment iterates
constexpr int32_t kSegSearched = 2;  // searched this iteration: its older pairs are dropped

// Device-side counters, reset and read back by the host loop.
struct Counters {
  unsigned long long n_out;     // compaction 1 (P' / search output)
  unsigned long long n_act;     // compaction 2 (A)
  unsigned long long n_left;    // colouring: rows left after this round
  unsigned long long fail;      // certificate failures
  unsigned long long mmax_bits; // max ||dx|| (bits of a non-negative double)
  unsigned long long rinf_bits; // max r
  unsigned long long fp_pf, fp_a, fp_col;
  unsigned long long err;       // bit 0: palette exhausted, bit 1: stack overflow,
                                // bit 2: bad index, bit 3: non-finite input
  unsigned long long ncand;     // search: node records read
  unsigned long long ncol;      // colours used (max colour + 1)
  unsigned long long n_rows;    // edge rows in use
  unsigned long long hits;      // continuous-test contacts among the failures
  unsigned long long et;        // input check: an edge meets a triangle
  unsigned long long ncert;     // certificate: pairs queued for the continuous test
  unsigned long long ecmis;     // edge colouring cache: inputs differing from the last
  unsigned long long nloc;      // one-block colouring: free vertices given block-local
                                // slots (above kLocCap1 when it coloured without them)
};

// Device buffers of a linear BVH over n leaves (n-1 internal nodes), allocated
// for the solver's capacity; n is the leaf count of the last search.
// Node record (4 float4 = 64 B): left box (6 floats), right box (6 floats),
// then child ids (bit 31 set = leaf, low bits = primitive id), the split
// position and the last leaf position of the node's range.
struct Bvh {
  int32_t n = 0;
  float4* leaf_lo = nullptr;     // sorted leaf boxes
  float4* leaf_hi = nullptr;
  int32_t* leaf_prim = nullptr;  // sorted position -> primitive id
  float4* node = nullptr;        // 4 per internal node
  float4* wide = nullptr;        // 8 per internal node: 4-wide traversal records
  int32_t* parent = nullptr;     // n-1 internal then n leaves: (parent << 1) | side
  int2* range = nullptr;         // leaf range of each internal node
  float4* pre = nullptr;         // per leaf: union of its block's leaves up to it
  float4* suf = nullptr;         // per leaf: union from it to the end of its block
  float4* blk = nullptr;         // sparse table of 256-leaf block unions (level-major)
  float4* root = nullptr;        // root box
};

struct Timer {
  int kind;
  hipEvent_t a, b;
};

}  // namespace cc

struct cc_server;  // resident-scene serving state (serve.hip)
namespace cc {
struct FlowWork;  // normal-flow target workspace (flow.hip)
}

struct cc_context {
  int device = 0;
  cc_server* server = nullptr;
  cc_solver* cached = nullptr;   // workspace reused by cc_collide_step
  cc_solver* batched = nullptr;  // multi-scene workspace reused by cc_collide_step_batched
  cc::FlowWork* flow = nullptr;  // normal-flow target workspace
};

namespace cc {

// Host view of one segment: a scene occupying index ranges of the solver's
// vertex, triangle and edge arrays (topology stored with solver-wide vertex ids).
struct Seg {
  int32_t vb = 0, nv = 0, fb = 0, nf = 0, eb = 0, ne = 0;
  int32_t np = 0;  // particles (vertices in no triangle or edge), listed at plist[vb, vb+np)
  int32_t max_iters = 0;
  double D = 0.0;
  bool live = false;     // holds a scene
  bool active = false;   // iterating
  bool begun = false;
  bool pending = false;  // removed; its ranges are not yet free
  int32_t n_erows = 0;
  cc_stats st{};
  cc_iter_info last{};
};

// One selected segment of a proximity search: its bases and the offsets of its
// vertices, triangles, edges and particles in the search's compact arrays.
struct SelDev {
  int32_t vb, fb, eb, seg;
  int32_t voff, toff, eoff, poff;
};

// First-fit allocator of index ranges.
struct RangeAlloc {
  int32_t cap = 0;
  std::vector<std::pair<int32_t, int32_t>> free_;  // (start, length), sorted, coalesced
  int32_t take(int32_t len);                       // start or -1
  void give(int32_t start, int32_t len);
  void grow(int32_t new_cap);
  int32_t extent() const;                          // one past the last used index
};

}  // namespace cc

struct cc_solver {
  cc_context* ctx = nullptr;
  // used extents (one past the highest index any segment holds) and capacities
  int32_t n = 0, nt = 0, ne = 0;
  int32_t capV = 0, capF = 0, capE = 0;
  int32_t capPt = 0;  // particle capacity of the search arrays (grows on demand)
  cc_params p{};
  double kappa2 = 0.0;
  bool begun = false;  // single-scene interface: segment 0 begun
  // segments
  std::vector<cc::Seg> segs;
  cc::SegDev* seg_dev = nullptr;   // kMaxSeg records
  cc::SegDev* seg_host = nullptr;  // pinned mirror
  cc::RangeAlloc ra_v, ra_f, ra_e;
  // ranges of removed segments (kind 0 vertices, 1 triangles, 2 edges; start;
  // length), freed after the next pair pass has dropped their pairs
  std::vector<std::array<int32_t, 3>> pending_free;
  std::vector<int32_t> pending_segs;
  int32_t* vseg = nullptr;  // segment of each vertex (-1 = none)
  int32_t* eseg = nullptr;  // segment of each edge (-1 = none)
  int32_t* plist = nullptr; // per segment, at its vertex base: its particles' vertex ids
  bool erows_dirty = true;  // the union of edge-row colour buckets needs a rebuild
  // tree reuse: gen changes with every change of the scenes or their state from
  // outside the iteration; the last build's scene list and gen
  uint64_t gen = 0, bvh_gen = ~0ull;
  std::vector<int32_t> bvh_sel;
  double bvh_q0 = 0.0;  // node records the traversal read right after the last build
  // topology and masses
  double* w = nullptr;
  int32_t* tris = nullptr;
  int32_t* edges = nullptr;
  uint8_t* stat = nullptr;
  // state
  double *x = nullptr, *y = nullptr, *xt = nullptr, *r = nullptr, *move2 = nullptr;
  // per vertex: the last forward step changed x; valid for the pairs' stored distances
  // while mv_gen equals gen (set when an iteration completes, cleared by anything that
  // moves x or drops the distances from outside)
  uint8_t* mvd = nullptr;
  uint64_t mv_gen = ~0ull;
  float* dy = nullptr;  // mixed precision: y - x in FP32 (3 per vertex)
  long long* jacc = nullptr;  // projected Jacobi: per-vertex update sums, 2^-56 m units
  double* xold = nullptr;  // x^(l) kept by the forward step for the continuous test
  double* rold = nullptr;  // r^(l), for vertices the certificate sends back
  float* dyold = nullptr;  // mixed precision: y - x^(l), likewise
  int32_t* back = nullptr; // certificate: 0, 2 = sent back in this pass, 1 = earlier
  double* alph = nullptr;  // CCD-based step: the forward step's alpha per vertex
  unsigned long long* scale = nullptr;  // ... and the factor of its step (bits of a double)
  unsigned long long* Di = nullptr;
  double D = 0.0;  // single-scene interface: D of segment 0
  // proximity set (double buffered for compaction) and distances of P'
  uint64_t *P = nullptr, *P2 = nullptr;
  double *dP = nullptr, *dP2 = nullptr;
  int64_t capP = 0, nP = 0, capA = 0;
  // active contacts
  uint64_t* Akeys = nullptr;
  int4* Averts = nullptr;
  int32_t* Acol = nullptr;
  int32_t* Aorder = nullptr;
  int32_t *list0 = nullptr, *list1 = nullptr;
  double* lamA = nullptr;
  double* Arow = nullptr;  // contact rows linearised at x (kRowWords doubles each)
  // one-block colouring: each row's four block-local vertex slots (16 bits each,
  // 0xffff: none) and the vertex of each slot
  unsigned long long* Aslot = nullptr;
  int32_t* lvert = nullptr;
  int64_t nA = 0;
  int32_t n_colors = 0;
  std::vector<int32_t> col_off;  // host copy of colour bucket offsets (n_colors+1)
  bool col_small = false;  // this step's contact colours and buckets live on the device only
  bool pc_wide = false;    // the last one-block colouring used more than 56 colours
  // edge-length rows (one per edge; inv_a = 0 marks an unused edge)
  double* eg = nullptr;     // 3 per edge
  double* einv = nullptr;
  int32_t* ecol = nullptr;
  int32_t* eorder = nullptr;
  int2* eij = nullptr;      // per bucket position: the row's two vertices (with eorder)
  int32_t *elist0 = nullptr, *elist1 = nullptr, *elist2 = nullptr;
  double* lamE = nullptr;
  int32_t n_erows = 0, n_ecolors = 0;  // rows in the union buckets, their colours
  int32_t n_newrows = 0;               // rows being coloured at a begin
  std::vector<int32_t> ecol_off;
  // the last edge-row colouring of a lone scene, reused while its inputs repeat:
  // the colouring is a function of the edges, the rows present, the free vertices,
  // the seed and the palette alone
  struct EdgeColourCache {
    bool ok = false;
    uint64_t seed = 0;
    int32_t maxc = 0, ne = 0, nv = 0, rows = 0;
    int32_t* edges = nullptr;   // 2 per edge
    uint8_t* row = nullptr;     // per edge: 1 = carries a row
    uint8_t* freev = nullptr;   // per vertex: 1 = free (w > 0)
    int32_t cap_e = 0, cap_v = 0;
  } ecache;
  // colouring scratch
  unsigned long long *vmax0 = nullptr, *masks = nullptr;  // per vertex: row count, used colours
  unsigned long long* claims = nullptr;  // per vertex: colours claimed this round, and clashes
  int32_t *afail = nullptr, *apick = nullptr;  // per contact row: failed rounds, pick
  int32_t *efail = nullptr, *epick = nullptr;  // per edge row
  bool pc_dirty = true;                        // counts or claims may be non-zero
  unsigned long long* rcnt = nullptr;  // list length per colouring round (kMaxRounds + 1)
  int32_t* col_cnt = nullptr;  // kMaxColors + 1
  int32_t *coff_dev = nullptr, *ecoff_dev = nullptr;  // colour bucket offsets on the device
  // broad phase
  cc::Bvh tree_t, tree_e, tree_p;  // triangles, edges, particles
  uint64_t *sk0 = nullptr, *sk1 = nullptr;
  uint32_t *sv0 = nullptr, *sv1 = nullptr;
  uint32_t* rs_hist = nullptr;
  uint32_t* rs_total = nullptr;  // per-digit totals of one radix pass
  int64_t rs_hist_cap = 0;
  float4 *ubox_lo = nullptr, *ubox_hi = nullptr;  // compact leaf boxes (F then E)
  int32_t* gprim = nullptr;    // compact primitive -> triangle or edge id
  uint32_t* bounds = nullptr;  // box-centre bounds, order-preserving uint encoding
  uint32_t* bounds_part = nullptr;  // per-block partial bounds
  int32_t* vorder = nullptr;   // vertex queries in Morton order (vertex ids)
  int16_t* vrank = nullptr;    // selected-segment rank of each vertex query
  int16_t* erank = nullptr;    // selected-segment rank of each sorted edge leaf
  int16_t* prank = nullptr;    // ... of each sorted particle leaf
  cc::SelDev* sel_dev = nullptr;   // kMaxSeg + 1
  cc::SelDev* sel_host = nullptr;  // pinned
  int32_t* root_t = nullptr;       // per selected segment: root of its triangle subtree
  int32_t* root_e = nullptr;       // ... of its edge subtree
  int32_t* root_p = nullptr;       // ... of its particle subtree
  // search output in kStripes stripes (see lbvh.hip): per stripe its counts (runs
  // << 40 | pairs) and the node records its waves read (kStripeWords words apart), a
  // pinned host mirror, and the stripes' keys and squared distances, capS entries each
  unsigned long long* stripe = nullptr;
  unsigned long long* hstripe = nullptr;
  uint64_t* skeys = nullptr;
  double* sd2 = nullptr;
  int64_t capS = 0;
  // the runs written into the stripes (capC per stripe: wave, offset in the wave's
  // output, length, start in the stripe), and per wave its pair count, then offset
  int4* chunks = nullptr;
  int64_t capC = 0;
  long long* wtot = nullptr;
  int64_t capW = 0;
  // the search's stripe counts, the counters and the segment records share one device
  // block and one pinned host mirror (kMirror* offsets), so that each host round trip
  // reads back what it needs with one copy
  unsigned char* mirror_dev = nullptr;
  unsigned char* mirror_host = nullptr;
  // counters
  cc::Counters* dc = nullptr;
  cc::Counters* hc = nullptr;  // pinned host mirror
  // statistics and timing
  cc_stats st{};
  std::vector<cc::Timer> timers;
  bool timer_open = false;  // the last timer_begin recorded its start event
  std::vector<hipEvent_t> event_pool;
};

namespace cc {

// ---- launchers (each returns CC_OK or an error code) ----
// broad phase (lbvh.hip)
int bvh_alloc(cc_solver* s);
void bvh_free(cc_solver* s);
// Search of the segments listed in s->sel_host[0..nsel) at state x with bound
// dmax; appends pair keys (solver-wide ids) to out and their squared distances at
// x to outd (if not NULL; capacity cap); *n gets the total number found (may
// exceed cap: caller regrows).
// refit_ok: the caller is the iteration loop, whose x only moves between searches;
// the tree of its last build is refitted when the same scenes are searched again.
int lbvh_search(cc_solver* s, int32_t nsel, const double* x, double dmax, uint64_t* out,
                double* outd, int64_t cap, int64_t* n, hipStream_t st, bool refit_ok);
// Input check of the selected segments at x (tolerance tol): *bad = 1 when a
// vertex-triangle or edge-edge pair is closer than tol or an edge meets a
// triangle it shares no vertex with.
int lbvh_validate(cc_solver* s, int32_t nsel, const double* x, double tol, int* bad,
                  hipStream_t st);

// per-iteration kernels (step.hip)
// Copy a scene's topology in (local vertex ids -> solver-wide) and check it;
// CC_EINVAL on an out-of-range or repeated index.
int launch_topo_in(cc_solver* s, int32_t seg, const int32_t* tris, const int32_t* edges,
                   hipStream_t st);
int launch_check_finite(cc_solver* s, const double* xa, const double* xb, int32_t n,
                        hipStream_t st);
int launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
int launch_particles(cc_solver* s, int32_t sg, hipStream_t st);
int normal_flow_target(cc_context* ctx, const double* x, int32_t n, const int32_t* tris,
                       int32_t nt, double beta, double alpha, int32_t iters, double* y,
                       hipStream_t st);
void flow_free(FlowWork* w);
// The normal-flow target on the library's fixed scratch array (no allocation);
// flow_scratch_init looks up that array's address on `device` (current) once.
int flow_scratch_init(int device);
int normal_flow_target_static(int device, const double* x, int32_t n, const int32_t* tris,
                              int32_t nt, double beta, double alpha, int32_t iters, double* y,
                              hipStream_t st);
int launch_setup(cc_solver* s, int32_t seg, const double* x_prev, const double* x_tilde,
                 hipStream_t st);
int launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st);
int launch_di_init(cc_solver* s, hipStream_t st);
// Colouring of a contact set of at most kSmallRows rows in one block; colours,
// buckets and the colour count stay on the device (s->col_small).
int color_small(cc_solver* s, hipStream_t st);
// The solver holds one live scene and no removed scene's pairs are left in P: every
// pair belongs to segment 0, and the pair pass leaves the per-segment counts to the
// host (evaluated = |P|, kept = |P'|, active = |A|).
inline bool single_live_seg(const cc_solver* s) {
  return s->segs.size() == 1 && s->segs[0].live && s->pending_segs.empty();
}
// pairs [0, n_old) are last iteration's P'; [n_old, nP) were appended by a search;
// pairs from d_from on take their squared distance from dP (written by the search)
int launch_pair_pass(cc_solver* s, int64_t n_old, int64_t d_from, double dl2, bool trace,
                     bool in_place, hipStream_t st);
// contacts: colour A; edges: colour the n_newrows rows listed in elist0
int color_rows(cc_solver* s, bool edges, hipStream_t st);
// the edge-length rows' colouring (greedy in priority order) of the n_newrows rows
// listed in elist0
int color_edges_greedy(cc_solver* s, hipStream_t st);
// Edge colouring cache of a lone scene (segment 0 at offset 0): compare the inputs
// with the cached ones (counted into dc->ecmis, cleared here), or store them.
int ecache_compare(cc_solver* s, hipStream_t st);
int ecache_store(cc_solver* s, hipStream_t st);
void ecache_free(cc_solver* s);
int build_edge_buckets(cc_solver* s, hipStream_t st);
int launch_gs(cc_solver* s, hipStream_t st);
int launch_jacobi(cc_solver* s, hipStream_t st);
int launch_forward(cc_solver* s, hipStream_t st);
// one pass of the certificate over P'; vertices of pairs it does not clear are marked
// (scaling: a contact scales the steps of the pair's vertices, the CCD-based step)
int launch_cert(cc_solver* s, bool scaling, hipStream_t st);
// the marked vertices back to x^(l) (scaling: their steps scaled), ||r||_inf again,
// queue cleared (ns segments)
int launch_send_back(cc_solver* s, int32_t ns, bool scaling, hipStream_t st);
int launch_fp_col(cc_solver* s, hipStream_t st);
// mixed precision: y <-> x + dy for vertices [0, n)
int launch_y_of_dy(cc_solver* s, double* y, int32_t n, hipStream_t st);
int launch_dy_of_y(cc_solver* s, const double* y, int32_t n, hipStream_t st);

// serving (serve.hip): stop the scheduler and free every resident scene
void server_destroy(cc_context* ctx);

// engine (api.hip)
int check_params(const cc_params* p);
int engine_create(cc_context* ctx, const cc_params* params, int32_t capV, int32_t capF,
                  int32_t capE, cc_solver** out, hipStream_t st);
void engine_set_params(cc_solver* s, const cc_params* params);
// Add a scene (topology with its own vertex ids 0..nv-1, device pointers) as a
// segment; the arrays grow when its ranges do not fit. *out = segment id.
int seg_add(cc_solver* s, int32_t nv, const double* inv_mass, const int32_t* tris, int32_t nf,
            const int32_t* edges, int32_t ne, int32_t max_iters, int32_t* out, hipStream_t st);
int seg_remove(cc_solver* s, int32_t sg, hipStream_t st);
void release_pending(cc_solver* s);
// Begin k segments' steps (x_prev[i] NULL = the segment's resident x).
int seg_begin(cc_solver* s, const int32_t* sgs, int32_t k, const double* const* x_prev,
              const double* const* x_tilde, int* rc, hipStream_t st);
// One Alg. 1 iteration of every iterating segment.
int engine_iterate(cc_solver* s, hipStream_t st);
int engine_active(const cc_solver* s);
void seg_stats(const cc_solver* s, int32_t sg, cc_stats* out);

// autotuner of launch shapes (api.hip): the choice stored for (device, kernel, size
// class), or -1; tune_store records a measured choice with the times of its variants
int tune_lookup(int device, int kernel, int32_t size_class);
void tune_store(int device, int kernel, int32_t size_class, int choice, const float ms[8]);

// timing helpers (api.hip)
void timer_begin(cc_solver* s, int kind, hipStream_t st);
void timer_end(cc_solver* s, hipStream_t st);

}  // namespace cc
