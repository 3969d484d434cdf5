// Internal declarations of the HIP collision-handling library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
constexpr int kMaxRounds = 65536;  // Jones-Plassmann rounds per colouring
constexpr double kCcdEta = 1e-12;  // distance at which the continuous test reports contact (m)

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
  unsigned long long ncol;      // colours used (max colour + 1)
  unsigned long long n_rows;    // edge rows in use
  unsigned long long hits;      // continuous-test contacts among the failures
  unsigned long long pad[3];
};

// Device buffers of a linear BVH over n leaves (n-1 internal nodes).
// Node record (4 float4 = 64 B): left box (6 floats), right box (6 floats),
// then child ids (bit 31 set = leaf, low bits = primitive id), the split
// position and the last leaf position of the node's range.
struct Bvh {
  int32_t n = 0;
  float4* leaf_lo = nullptr;     // sorted leaf boxes
  float4* leaf_hi = nullptr;
  int32_t* leaf_prim = nullptr;  // sorted position -> primitive id
  int32_t* pos_of = nullptr;     // primitive id -> sorted position
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

struct cc_context {
  int device = 0;
  cc_server* server = nullptr;
  cc_solver* cached = nullptr;  // workspace reused by cc_collide_step
  // batched steps: one solver and one stream per scene slot
  std::vector<cc_solver*> slots;
  std::vector<hipStream_t> slot_streams;
};

struct cc_solver {
  cc_context* ctx = nullptr;
  int32_t n = 0, nt = 0, ne = 0;
  cc_params p{};
  double kappa2 = 0.0;
  bool begun = false;
  // topology and masses
  double* w = nullptr;
  int32_t* tris = nullptr;
  int32_t* edges = nullptr;
  uint8_t* stat = nullptr;
  // state
  double *x = nullptr, *y = nullptr, *xt = nullptr, *r = nullptr, *move2 = nullptr;
  double* xold = nullptr;  // x^(l) kept by the forward step for the continuous test
  unsigned long long* Di = nullptr;
  double D = 0.0;
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
  int64_t nA = 0;
  int32_t n_colors = 0;
  std::vector<int32_t> col_off;  // host copy of colour bucket offsets (n_colors+1)
  // edge-length rows (one per input edge; inv_a = 0 marks an unused edge)
  double* eg = nullptr;     // 3 per edge
  double* einv = nullptr;
  int32_t* ecol = nullptr;
  int32_t* eorder = nullptr;
  int32_t *elist0 = nullptr, *elist1 = nullptr, *elist2 = nullptr;
  double* lamE = nullptr;
  int32_t n_erows = 0, n_ecolors = 0;
  std::vector<int32_t> ecol_off;
  // colouring scratch
  unsigned long long *vmax0 = nullptr, *vmax1 = nullptr, *masks = nullptr;
  unsigned long long* rcnt = nullptr;  // list length per colouring round (kMaxRounds + 1)
  int32_t* col_cnt = nullptr;  // kMaxColors + 1
  int32_t *coff_dev = nullptr, *ecoff_dev = nullptr;  // colour bucket offsets on the device
  // broad phase
  cc::Bvh tree_t, tree_e;
  uint32_t *sk0 = nullptr, *sk1 = nullptr, *sv0 = nullptr, *sv1 = nullptr;
  uint32_t* rs_hist = nullptr;
  uint32_t* rs_total = nullptr;  // per-digit totals of one radix pass
  int64_t rs_hist_cap = 0;
  float4 *ubox_lo = nullptr, *ubox_hi = nullptr;  // unsorted leaf boxes (F then E)
  uint32_t* bounds = nullptr;  // box-centre bounds, order-preserving uint encoding
  uint32_t* bounds_part = nullptr;  // per-block partial bounds
  int32_t* vorder = nullptr;   // vertices in Morton order (vertex-triangle queries)
  // counters
  cc::Counters* dc = nullptr;
  cc::Counters* hc = nullptr;  // pinned host mirror
  // statistics and timing
  cc_stats st{};
  std::vector<cc::Timer> timers;
  std::vector<hipEvent_t> event_pool;
};

namespace cc {

// ---- launchers (each returns CC_OK or an error code) ----
// broad phase (lbvh.hip)
int bvh_alloc(cc_solver* s);
void bvh_free(cc_solver* s);
// Search at state x with bound dmax; appends pair keys to out (capacity cap);
// *n gets the total number found (may exceed cap: caller regrows).
int lbvh_search(cc_solver* s, const double* x, double dmax, uint64_t* out, int64_t cap,
                int64_t* n, hipStream_t st);

// per-iteration kernels (step.hip)
int launch_validate(cc_solver* s, const double* xa, const double* xb, hipStream_t st);
int launch_setup(cc_solver* s, const double* x_prev, const double* x_tilde, hipStream_t st);
int launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st);
int launch_pair_pass(cc_solver* s, double D2, double dl2, bool trace, hipStream_t st);
int color_rows(cc_solver* s, bool edges, hipStream_t st);
int launch_gs(cc_solver* s, hipStream_t st);
int launch_forward(cc_solver* s, hipStream_t st);
int launch_cert(cc_solver* s, hipStream_t st);
int launch_fp_col(cc_solver* s, hipStream_t st);

// serving (serve.hip): stop the worker pool and free every resident scene
void server_destroy(cc_context* ctx);

// timing helpers (api.hip)
void timer_begin(cc_solver* s, int kind, hipStream_t st);
void timer_end(cc_solver* s, hipStream_t st);

}  // namespace cc
