// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <vector>

#include "eipc.h"

namespace eipc {

// status bits raised by kernels into the device status word
enum : uint32_t {
  ST_INTERSECTING = 1u,
  ST_NONFINITE = 2u,
  ST_CCD_CAPPED = 4u,
  ST_HASH_OVERFLOW = 8u,
  ST_BAD_W = 16u,         // a W row with more than 4 weights
  ST_PLAN_OVERFLOW = 32u,  // a planned capacity was exceeded
  ST_BAD_SCENE = 64u,      // a vertex scene id out of range
  ST_DEGENERATE = 128u     // a degenerate or inverted element of the elastic mesh
};

// scratch buffers owned by the context
enum BufId {
  B_X = 0,       // positions, SoA [3][n_vert]
  B_P,           // CCD displacement, SoA
  B_X1,          // CCD end positions, SoA
  B_XV,          // HVP input mapped to vertices, SoA
  B_SCANTMP,     // int64 block sums
  B_SCANTMP_SIDE,  // the same, for scans on the side stream
  B_ACT_PT, B_TYP_PT, B_ACT_EE, B_TYP_EE,
  B_CAND_PT, B_CAND_EE,  // swept candidates (CCD)
  B_HKEY, B_HVAL,        // global block hash
  B_ROWCNT, B_ROWFILL, B_ROWPTR, B_BCOL, B_BSRC, B_BBLK, B_BCOL2, B_BSRC2,
  B_PG_PT, B_PG_EE, B_PX_PT, B_PX_EE,  // per-pair gradient / Hessian in the Q basis
  B_STEP_PT, B_STEP_EE,                // candidates of a planned step
  B_ALPHA,                             // per-scene step bound bits
  B_PLAN_OUT,                          // outputs of the reserving step of a plan
  B_SKEY, B_SHIST, B_SFILL, B_SSTART, B_SACT, B_STYP,  // locality sort of active pairs
  B_SVIDU, B_SVID,                                   // their vertex ids (unsorted, sorted)
  B_SKEY_EE, B_SHIST_EE, B_SFILL_EE, B_SSTART_EE, B_SACT_EE, B_STYP_EE, B_SVIDU_EE, B_SVID_EE,  // the same for EE
  B_CCD_LONG_PT, B_CCD_LONG_EE,                        // CCD pairs deferred to the second pass
  B_LQTMP,                                             // unsorted candidates of large queries (sorted lists)
  B_BP0,                               // broad-phase scratch: 4 slots (kind, swept) x BP_NBUF
  B_NUM = B_BP0 + 4 * 17
};
constexpr int BP_NBUF = 17;

// capacities of one broad phase in a planned (synchronization-free) call
// Buckets of a broad-phase hash of `entries` (item, cell) entries: a cell
// holds tens of entries, so a quarter as many buckets as entries still
// leaves most occupied cells a bucket of their own (power of 2, >= 1024).
inline int64_t hash_buckets(int64_t entries) {
  int64_t b = 1024;
  while (b < entries / 4 && b < (1ll << 31)) b <<= 1;
  return b;
}

struct BPPlan {
  uint32_t nb;        // hash buckets (power of 2)
  int64_t ent_cap;    // item hash entries
  int64_t cand_cap;   // candidate pairs
  int64_t qent_cap;   // query cell entries (append mode)
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  uint32_t epoch = 0;  // arena mode: the call that carved it
};

// kernels timed by the optional event profiler
enum KernelId {
  K_EMBED = 0, K_QUERY_COUNT_PT, K_QUERY_COUNT_EE, K_QUERY_WRITE_PT, K_QUERY_WRITE_EE, K_NARROW_PT, K_NARROW_EE,
  K_BARRIER_PT, K_BARRIER_EE, K_CCD_PT, K_CCD_EE, K_HVP_PT, K_HVP_EE, K_EXPAND_PT, K_EXPAND_EE, K_CCD_LONG_PT,
  K_CCD_LONG_EE, K_NUM
};
extern const char *const kKernelNames[K_NUM];

struct ProfRec {
  int id;
  hipEvent_t start, stop;
};

}  // namespace eipc

struct eipc_ctx {
  int device = 0;
  char err[512] = {0};
  eipc::DevBuf buf[eipc::B_NUM];
  uint32_t *status = nullptr;   // device status word
  double *stats = nullptr;      // device [32] reduction scratch
  int64_t *counters = nullptr;  // device [16] counters
  // Scratch.  Grow mode (no reservation): each buffer is allocated on
  // first need and replaced by a larger one when a call needs more; the
  // replaced buffer is kept (work already enqueued may still use it) until
  // the next synchronizing plan or eipc_destroy, so growth never waits for
  // the device.  Arena mode (reserve_bytes > 0 at creation): one
  // allocation made by eipc_create, carved afresh by every top-level call
  // (nothing in scratch outlives the call that wrote it, except outputs
  // that are valid until the next call); a call that does not fit returns
  // EIPC_ERR_CAPACITY and nothing is ever allocated after creation.
  std::vector<void *> retired;
  char *arena = nullptr;
  size_t arena_bytes = 0, arena_top = 0, arena_high = 0;
  uint32_t epoch = 1;
  int depth = 0;               // nesting of entry points (plan_step calls others)
  bool scratch_short = false;  // this call ran out of its reservation
  // pair lists of the last planned step, for eipc_step_pairs: the pairs
  // it tested per kind, their count word and capacity, and its active
  // lists (indices into them)
  const int32_t *step_pairs[2] = {nullptr, nullptr};
  const int32_t *step_act[2] = {nullptr, nullptr};
  int step_pair_ctr[2] = {0, 0};
  int64_t step_pair_cap[2] = {0, 0}, step_act_cap[2] = {0, 0};
  int64_t hash_cap = 1 << 16;   // global block hash capacity (power of 2, grows)
  int num_cu = 256;
  double cell_scale = 2.0;       // broad-phase cell edge / mean item extent
  int wg_per_cu[4] = {1, 2, 4, 4};  // grid sizes: barrier stage, stored-terms expansion, narrow, CCD
  int ccd_method = 0;                // 0: additive CCD, 1: advancement along the closest direction
  // append-mode broad phase work split [PT, EE]: 0 thread per query,
  // 1 thread per (query, cell), 2 wavefront per (query, cell), 3 bucket join
  // (the default: the fastest on every workload measured, small to batch)
  int query_mode[2] = {3, 3};
  eipc::BPPlan last_plan[4] = {};   // sizes seen by the last unplanned broad phases
  bool prof = false;                        // record per-kernel events
  bool prof_serial = false;                 // planned step: both chains on the caller's stream
  std::vector<eipc::ProfRec> prof_pending;  // recorded, not yet read
  std::vector<hipEvent_t> prof_pool;        // reusable events
  double prof_ms[eipc::K_NUM] = {0};
  int64_t prof_n[eipc::K_NUM] = {0};
  // second stream (default priority) for work that runs beside the step's
  // main chain; joined back through events, also under graph capture
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // device address of this GPU's copy of the library's fixed no-allocation
  // scratch array (looked up once per device at creation)
  void *noalloc_scratch = nullptr;
};

namespace eipc {

eipc_status set_err(eipc_ctx *c, eipc_status st, const char *fmt, ...);

#define EIPC_HIP(ctx, expr)                                                                      \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess)                                                                        \
      return ::eipc::set_err((ctx), EIPC_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define EIPC_TRY(expr)            \
  do {                            \
    eipc_status s_ = (expr);      \
    if (s_ != EIPC_OK) return s_; \
  } while (0)

// scratch allocation (grow mode or arena mode, see eipc_ctx)
eipc_status ensure(eipc_ctx *c, BufId id, size_t bytes, void **out);
// Marks one entry-point call: the outermost call on a context starts a
// fresh carving of the arena.
struct CallScope {
  eipc_ctx *c;
  explicit CallScope(eipc_ctx *c_) : c(c_) {
    if (c && c->depth++ == 0) {
      c->scratch_short = false;
      if (c->arena) {
        c->arena_top = 0;
        ++c->epoch;
      }
    }
  }
  ~CallScope() {
    if (c) --c->depth;
  }
};
template <class T>
inline eipc_status ensure_t(eipc_ctx *c, BufId id, size_t count, T **out) {
  void *p = nullptr;
  eipc_status st = ensure(c, id, count * sizeof(T) + 64, &p);
  *out = (T *)p;
  return st;
}

// event bracket around one kernel launch when profiling is on
struct ProfScope {
  eipc_ctx *c;
  int id;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(eipc_ctx *c_, int id_, hipStream_t s_);
  ~ProfScope();
};

// Positions inside the library: one 32-byte record per vertex (x, y, z,
// unused), so that gathering a vertex touches one cache line.
constexpr int PSTRIDE = 4;
__device__ __forceinline__ void ld_pos(const double *p, int v, double &x, double &y, double &z) {
  const double2 a = *reinterpret_cast<const double2 *>(p + (int64_t)PSTRIDE * v);
  x = a.x;
  y = a.y;
  z = p[(int64_t)PSTRIDE * v + 2];
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b on XCD
// b % 8), each XCD with its own L2.  This maps the physical workgroup to a
// logical one so that each XCD takes runs of `chunk` consecutive logical
// workgroups (XCD k takes runs k, k + 8, ...): neighbouring work in a
// spatially ordered list then shares one L2, while the runs spread the
// load over the XCDs.  A bijection on [0, gridDim.x) (the tail that does
// not fill 8 runs keeps the identity).
__device__ __forceinline__ int xcd_block(int chunk) {
  const int b = blockIdx.x;
  const int full = gridDim.x / (8 * chunk) * (8 * chunk);
  if (b >= full) return b;
  const int k = b & 7, j = b >> 3;
  return ((j / chunk) * 8 + k) * chunk + j % chunk;
}

inline int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  return (int)(g < 1 ? 1 : g);
}

// ---- geometry.hip ----
eipc_status launch_embed(eipc_ctx *c, const eipc_scene *sc, const double *q, const double *off, double *xs,
                         double *x_aos, hipStream_t s);
eipc_status launch_add_soa(eipc_ctx *c, int64_t n, const double *a, const double *b, double *out, hipStream_t s);
eipc_status exclusive_scan(eipc_ctx *c, const int32_t *in, int64_t n, int64_t *out, hipStream_t s);
eipc_status launch_zero(eipc_ctx *c, void *p, size_t bytes, hipStream_t s);
// Candidate pairs of one kind; swept when x1s != nullptr.  Unplanned
// (plan == nullptr): synchronizes, writes the required count to *n_out and
// the pairs when they fit (sorted per query when sort != 0), growing buffer
// grow_id when given.  Planned: no synchronization and no allocation beyond
// the plan's sizes; the count goes to device *d_total and an overflow
// raises ST_PLAN_OVERFLOW.
eipc_status broad_phase(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *x1s,
                        double dhat, int32_t *out, int64_t cap, int64_t *n_out, int sort, hipStream_t s,
                        int grow_id = -1, int32_t **grown = nullptr, const BPPlan *plan = nullptr,
                        int64_t *d_total = nullptr);
// Active subset of `n` pairs (at most `n`; min(n, *d_n) when d_n is given)
// into act/typ of capacity act_cap (< 0: n).  With cand_count, the pairs
// are swept candidates filtered by the candidate predicate at xs first and
// the number passing is added to *cand_count.
eipc_status launch_narrow(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                          int64_t n, double dhat, int32_t *act, int32_t *typ, int64_t *d_count, hipStream_t s,
                          const int64_t *d_n = nullptr, int64_t act_cap = -1, int64_t *cand_count = nullptr);
inline int n_scene_of(const eipc_scene *sc) { return sc->n_scene > 1 ? sc->n_scene : 1; }
inline const int32_t *vscene_of(const eipc_scene *sc) { return sc->n_scene > 1 ? sc->vert_scene : nullptr; }

// ---- barrier.hip ----
struct HessOut {
  int kind;  // 0 none, 1 dense, 2 global hash
  double *dense;
  int64_t *hkey;  // I * n_node + J, -1 empty
  double *hval;
  uint64_t hmask;
};
eipc_status launch_barrier(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                           const int32_t *act, const int32_t *typ, const int64_t *d_count, int64_t max_count,
                           double dhat, double kappa, uint32_t flags, double *energy, double *grad,
                           const HessOut &h, hipStream_t s);
eipc_status launch_dense_mirror(eipc_ctx *c, int n_node, double *dense, hipStream_t s);
// Reduction through W of per-pair gradients and Hessians in the Q basis
// (SoA [9][cap] and [45][cap]) of min(*d_count, cap) pairs with vertex ids
// vid4; grad or h.kind == 0 skip a part.
// Per-pair terms record (doubles, 16-byte aligned): the Q-basis gradient
// gamma [0, 9), the packed Q-basis Hessian X [9, 54), 2 unused.
constexpr int TERM_REC = 56;
// Reduction through W of per-pair term records (rec[i * TERM_REC + e]).
eipc_status launch_expand(eipc_ctx *c, const eipc_scene *sc, int kind, const int4 *vid4, const int64_t *d_count,
                          int64_t cap, const double *rec, bool want_g, bool want_h, double *grad, const HessOut &h,
                          hipStream_t s);
// BSR view of the hashed blocks.  nnzb_cap < 0: sized on the host
// (synchronizes); else fixed capacity, the count only on the device
// (rowptr[n_node]) and out->nnzb = -1.
eipc_status bsr_compact(eipc_ctx *c, int n_node, const HessOut &h, eipc_bsr *out, hipStream_t s,
                        int64_t nnzb_cap = -1);
eipc_status launch_hvp(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *xvs,
                       const int32_t *pairs, const int32_t *act, const int32_t *typ, const int64_t *d_count,
                       int64_t max_count, double dhat, double kappa, uint32_t flags, double *out,
                       double *out_off, hipStream_t s, bool locality_sort = true);
eipc_status launch_pair_eval(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                             int64_t n, double dhat, double kappa, uint32_t flags, int32_t *type, double *sq,
                             double *e, double *g, double *H, hipStream_t s);

// ---- friction.hip ----
// Lag records (EIPC_FRICTION_LAG doubles per pair) at positions xs, and the
// friction energy / reduced gradient / reduced Hessian at xs from them.
eipc_status launch_friction_lag(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                                int64_t n, double dhat, double kappa, uint32_t flags, double *lag, hipStream_t s);
eipc_status launch_friction(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                            int64_t n, const double *lag, double mu, double epsvh, double *energy, double *grad,
                            const HessOut &h, hipStream_t s);

// ---- ccd.hip ----
// Per-pair bound; min into d_alpha_bits[scene] when given.  n pairs at
// most (min(n, *d_n) when d_n is given).
eipc_status launch_ccd(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *ps,
                       const int32_t *pairs, int64_t n, double sfac, double t_max, int64_t max_iter,
                       uint64_t *d_alpha_bits, double *t_out, int64_t *it_out, hipStream_t s,
                       const int64_t *d_n = nullptr);
// Planned step with a step bound: narrow phase of the swept candidates
// (as launch_narrow with cand_count) and the step bound's first pass (as
// launch_ccd into d_alpha_bits) in one sweep; launch_ccd_long then runs
// the pairs that pass deferred (may go on another stream ordered after it).
eipc_status launch_narrow_ccd(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *ps,
                              const int32_t *pairs, int64_t n, const int64_t *d_n, double dhat, int32_t *act,
                              int32_t *typ, int64_t act_cap, int64_t *d_count, int64_t *cand_count, double sfac,
                              double t_max, int64_t max_iter, uint64_t *d_alpha_bits, hipStream_t s);
eipc_status launch_ccd_long(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *ps,
                            const int32_t *pairs, int64_t n, const int64_t *d_n, double sfac, double t_max,
                            int64_t max_iter, uint64_t *d_alpha_bits, hipStream_t s);
eipc_status launch_fp64_selftest(eipc_ctx *c, const double *a, const double *b, double *sq, double *dv, int64_t n,
                                 hipStream_t s);

}  // namespace eipc
