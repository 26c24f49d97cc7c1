/* eipc.h -- C ABI of the MI355X (gfx950) contact-stage library for
 * Embedded IPC (arXiv 2409.16385).
 *
 * The library computes, for one Newton iteration, the contact terms of the
 * embedded IPC objective on a high-resolution surface whose vertices are
 * interpolated from coarse nodes, x = W q + x_off (Sec. III-D, Eq. 13-14):
 * candidate point-triangle (PT) and edge-edge (EE) pairs, the log-barrier
 * energy kappa * sum b(d_k) (Sec. III-B, Eq. 7, 10-11), its gradient and
 * PSD-projected Hessian reduced through the embedding (Eq. 17), Hessian-
 * vector products, and a conservative continuous-collision step bound that
 * clamps the line search (Sec. III-C).
 *
 * Conventions (every entry point):
 *  - Array arguments are DEVICE pointers on the context's GPU, caller
 *    owned, contiguous, unless a comment says "host".  The library never
 *    frees or retains caller memory past a call.
 *  - FP64 for all real data, int32 indices, int64 sizes.
 *  - q and every reduced vector are double[3*n_node], node-major xyz.
 *    Positions are double[3*n_vert] AoS.
 *  - Work is enqueued on `stream` (a hipStream_t, NULL = default stream).
 *    Calls that return a count or a scalar to a host pointer synchronize
 *    that stream before returning.
 *  - Argument errors are returned synchronously and nothing is enqueued.
 *    Data-dependent errors (an intersecting pair, a non-finite value) are
 *    raised by the kernels into a device status word; calls that
 *    synchronize return it, eipc_sync_status() reads it otherwise.
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef EIPC_H
#define EIPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t eipc_status;
enum {
  EIPC_OK = 0,
  EIPC_ERR_ARG = -1,          /* invalid argument (nothing enqueued) */
  EIPC_ERR_CAPACITY = -2,     /* an output buffer is too small; the required size is returned */
  EIPC_ERR_INTERSECTING = -3, /* a candidate pair has distance 0: the input is not intersection-free */
  EIPC_ERR_DEGENERATE = -4,   /* a degenerate or inverted element of the elastic mesh (eipc_elastic) */
  EIPC_ERR_NONFINITE = -5,    /* NaN or Inf in positions or pair quantities */
  EIPC_ERR_HIP = -6,          /* a HIP runtime call failed; see eipc_last_error */
  EIPC_WARN_CCD_CAPPED = 1    /* CCD hit its per-pair iteration cap (the bound is still safe) */
};
/* A planned call that exceeded a capacity of its plan, or whose
 * reduced-Hessian block table filled up, reports EIPC_ERR_CAPACITY through
 * eipc_sync_status; its outputs are then not valid and the caller plans
 * again with a larger margin. */

/* flags for eipc_barrier_reduce / eipc_barrier_hvp */
enum {
  EIPC_ENERGY = 1,  /* total barrier energy */
  EIPC_GRAD = 2,    /* reduced gradient W^T g */
  EIPC_HESS = 4,    /* reduced Hessian W^T H W */
  EIPC_PROJECT = 8, /* use the per-pair PSD projection of H (projected Newton, Sec. III-C) */
  EIPC_MOLLIFY = 16, /* EE mollifier for near-parallel edges (needs x_rest: EIPC_ERR_ARG without it) */
  /* Alternative formulation: the log barrier of Eq. 7 written in the
   * squared distance, b(s) = -(s - dhat^2)^2 ln(s / dhat^2) with s = d^2
   * (the same active set; the friction normal force becomes
   * kappa m |db/dd| = kappa m 2 d |db/ds|). */
  EIPC_SQDIST = 32,
  /* Alternative projection (barrier_reduce, contact_step): the PSD
   * projection of each pair's reduced local block W_k^T H_k W_k (over the
   * pair's distinct nodes) in place of EIPC_PROJECT's projection of the
   * 12x12 H_k.  The same for point-point pairs (and for W = I); another
   * matrix for point-line and interior pairs under a coarse embedding.
   * EIPC_ERR_ARG with barrier_hvp and pair_eval (per-pair outputs). */
  EIPC_PROJECT_REDUCED = 64
};

typedef struct eipc_ctx eipc_ctx;
typedef void *eipc_stream; /* hipStream_t */

/* One scene: a collision surface M_col = (X, S) and its embedding
 * (Sec. III-D).  Row k of W holds the barycentric weights of surface
 * vertex k in its coarse tetrahedron (Eq. 13); an empty row marks a vertex
 * with no DoF (static, or kinematic: prescribed through x_off, as in the
 * position-controlled grippers of Sec. IV-A).  A row with a single weight
 * 1 is a full-space vertex (W = I is full-space IPC, Sec. III-D).  A row
 * holds at most 4 weights (the nodes of one tetrahedron); a longer row is
 * reported as EIPC_ERR_ARG by the next call that synchronizes.
 *
 * A batch of independent scenes is one eipc_scene whose arrays are the
 * concatenations of the scenes' arrays, with indices already offset to the
 * concatenation (global vertex and node numbers), plus n_scene > 1 and
 * vert_scene[v] = the scene of vertex v.  Every face, edge and W row must
 * stay within one scene.  Pairs never join two scenes, outputs per scene
 * (energy, step bound) are arrays of n_scene, and the reduced vectors are
 * the concatenated per-scene vectors.  n_scene <= 65536.  n_scene = 0 or 1
 * is one scene and vert_scene is then ignored. */
typedef struct {
  int32_t n_vert, n_node, n_face, n_edge;
  const int32_t *faces;    /* [n_face*3] vertex indices */
  const int32_t *edges;    /* [n_edge*2] unique undirected edges, a < b */
  const int32_t *W_rowptr; /* [n_vert+1] CSR row pointers */
  const int32_t *W_col;    /* [nnz] node index in [0, n_node) */
  const double *W_val;     /* [nnz] weights */
  const double *x_off;     /* [n_vert*3] added to W q (static / kinematic positions), or NULL */
  const double *x_rest;    /* [n_vert*3] rest positions for the EE mollifier, or NULL */
  int32_t n_scene;         /* scenes in a batch (0 or 1: a single scene) */
  const int32_t *vert_scene; /* [n_vert] scene id per vertex when n_scene > 1 */
} eipc_scene;

/* Reduced Hessian in 3x3 block-sparse rows (both triangles stored, columns
 * sorted).  All pointers are device memory owned by the context, valid
 * until the next call on that context. */
typedef struct {
  int32_t n_rows;         /* = n_node */
  int64_t nnzb;           /* number of stored 3x3 blocks (-1: only on the device, as rowptr[n_rows]) */
  const int32_t *rowptr;  /* [n_rows+1] */
  const int32_t *col;     /* [nnzb] */
  const double *blocks;   /* [nnzb*9] row-major 3x3 */
} eipc_bsr;

/* Context on GPU `device`.  Owns the scratch memory of the calls and the
 * device status word.
 * reserve_bytes == 0 (grow mode): scratch buffers are allocated when a call
 *   first needs them and replaced by larger ones when a later call needs
 *   more.  A replaced buffer is kept, not freed, until the next
 *   eipc_plan_step or eipc_destroy, so no call waits for the device because
 *   of its scratch.
 * reserve_bytes > 0 (arena mode): eipc_create allocates that many bytes
 *   once and every later call carves its scratch from them; no call
 *   allocates device memory after creation.  A call whose scratch does not
 *   fit returns EIPC_ERR_CAPACITY (eipc_last_error names the size) before
 *   it enqueues the kernel that needed it.  Size the reservation from
 *   eipc_scratch_bytes of a grow-mode run of the same workload.
 * Returns EIPC_ERR_ARG for a bad device, EIPC_ERR_HIP if an allocation
 * fails. */
eipc_status eipc_create(eipc_ctx **ctx, int32_t device, size_t reserve_bytes);
/* reserved (host): the arena size, 0 in grow mode.  high_water (host): the
 * most scratch one call has used (arena mode) or the bytes of all scratch
 * buffers held (grow mode). */
eipc_status eipc_scratch_bytes(const eipc_ctx *ctx, size_t *reserved, size_t *high_water);
void eipc_destroy(eipc_ctx *ctx);
const char *eipc_last_error(const eipc_ctx *ctx);
const char *eipc_status_string(eipc_status s);
/* Synchronizes `stream`, returns and clears the device status word. */
eipc_status eipc_sync_status(eipc_ctx *ctx, eipc_stream stream);

/* Embedding map x = W q + off (Eq. 14), written AoS to x[n_vert*3].
 * Each coordinate is accumulated in CSR order from 0.0 (one rounded
 * multiply and one rounded add per term) and off is added last, so x is
 * reproducible bit for bit.  off may be NULL. */
eipc_status eipc_embed(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const double *off, double *x,
                       eipc_stream stream);

/* Candidate pairs of the pair set B (Sec. III-B) at positions W q + x_off:
 * PT pairs (vertex v, face f) with v not in f and EE pairs (edge a, edge b)
 * with a < b and no shared vertex, whose boxes overlap.  The box of a
 * primitive spans its vertices, widened by dhat/2 on every side (closed
 * intervals).  Pairs whose four vertices all have empty W rows are
 * excluded.  Outputs pt[2*k] = v, pt[2*k+1] = f and ee[2*k] = a,
 * ee[2*k+1] = b, sorted by (first, second).
 * *n_pt, *n_ee (host) always receive the required counts; if either
 * exceeds cap_pt / cap_ee the call returns EIPC_ERR_CAPACITY and the
 * lists are not written.  Synchronizes. */
eipc_status eipc_build_candidates(eipc_ctx *ctx, const eipc_scene *sc, const double *q, double dhat, int32_t *pt,
                                  int64_t cap_pt, int32_t *ee, int64_t cap_ee, int64_t *n_pt, int64_t *n_ee,
                                  eipc_stream stream);

/* Barrier terms over the given pairs (Sec. III-B, Eq. 7, 10-11; reduction
 * Eq. 17).  A pair is active when 0 < d < dhat with d the Euclidean
 * distance between the closed primitives; its energy is kappa * b(d)
 * (times the mollifier m(|ea x eb|^2) for EE pairs with EIPC_MOLLIFY).
 * Pass kappa * h^2 to obtain the h^2-scaled barrier term of E_IPC.
 *   energy    device double[n_scene] or NULL: energy per scene (overwritten)
 *   grad_q    device double[3*n_node] or NULL: W^T g (overwritten)
 *   hess_dense device double[(3*n_node)^2] or NULL: W^T H W, row-major
 *   hess_bsr  host struct or NULL: filled with a context-owned BSR view
 * H is the per-pair PSD projection when EIPC_PROJECT is set, else the true
 * pair Hessian.  n_active (host) or NULL receives the number of active
 * pairs.  Synchronizes when n_active or hess_bsr is requested.
 * An active pair with d == 0 raises EIPC_ERR_INTERSECTING.  The reduced
 * Hessian needs n_node < 2^31 / 3 rows; a reduced gradient or Hessian
 * needs n_node < 2^27 (node ids are packed with a 4-bit slot in the
 * reduction), else EIPC_ERR_ARG. */
eipc_status eipc_barrier_reduce(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const int32_t *pt,
                                int64_t n_pt, const int32_t *ee, int64_t n_ee, double dhat, double kappa,
                                uint32_t flags, double *energy, double *grad_q, double *hess_dense,
                                eipc_bsr *hess_bsr, int64_t *n_active, eipc_stream stream);

/* Conservative step bound for the line search (Sec. III-C): the largest
 * alpha <= t_max such that moving x by alpha * p, p = W dq + dx_off, is
 * guaranteed free of new intersections, computed per swept candidate pair
 * by additive conservative advancement with gap factor s (0 < s < 1) and
 * the minimum taken over all pairs whose swept boxes (start and end
 * positions, widened by dhat/2) overlap.  dx_off may be NULL.
 * alpha (host double[n_scene]): the bound per scene; n_cand (host, or
 * NULL) receives the number of swept
 * candidates.  Returns EIPC_WARN_CCD_CAPPED if some pair reached max_iter
 * iterations before its bound was shown to be no smaller than the scene's
 * bound found so far (pairs shown so are not advanced further: the minimum
 * is the same); alpha is still safe.  Synchronizes. */
eipc_status eipc_ccd_max_step(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const double *dq,
                              const double *dx_off, double dhat, double s, double t_max, int64_t max_iter,
                              double *alpha, int64_t *n_cand, eipc_stream stream);

/* Hessian-vector product through the embedding (Eq. 17), recomputing the
 * pair Hessians (nothing is stored per pair):
 *   out = sum_k W_k^T H_k (W_k v + v_off_k)
 * with H_k the true pair Hessian, or its PSD projection with EIPC_PROJECT.
 * v: device double[3*n_node]; v_off: device double[3*n_vert] or NULL.
 * out: device double[3*n_node] (overwritten).  out_off: device
 * double[3*n_vert] or NULL, receives the unreduced per-vertex sums
 * sum_k H_k z_k (the rows of kinematic vertices). */
eipc_status eipc_barrier_hvp(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const int32_t *pt,
                             int64_t n_pt, const int32_t *ee, int64_t n_ee, double dhat, double kappa,
                             uint32_t flags, const double *v, const double *v_off, double *out, double *out_off,
                             eipc_stream stream);

/* ---- lagged friction (Sec. III-B) ---- */

/* Doubles per lag record: lambda, beta[4], normal[3], G x^n[3]. */
#define EIPC_FRICTION_LAG 11

/* Lag records of the friction potential D_k = mu lambda_k^n f0(|u_k|)
 * (Sec. III-B) at the previous time step's positions x^n = W q_n + x_off,
 * one per given pair (typically the active pairs at x^n), written to
 * lag_pt / lag_ee (device double[n][EIPC_FRICTION_LAG]):
 *   lambda   kappa |b'(d^n)|, the magnitude of the barrier's normal force
 *            (times the mollifier m(c^n) for EE pairs with EIPC_MOLLIFY);
 *            0 for a pair that is not active at x^n (it adds no friction);
 *   beta[4]  signed closest-point weights over the pair's vertices (point
 *            minus closest triangle point for PT; closest point on edge a
 *            minus closest point on edge b for EE), G x = sum_a beta_a x_a;
 *   normal   G x^n / |G x^n|, the contact normal at x^n;
 *   G x^n    the relative position at x^n.
 * Single scenes only (n_scene <= 1).  Asynchronous; a pair at zero
 * distance raises EIPC_ERR_INTERSECTING in the status word. */
eipc_status eipc_friction_lag(eipc_ctx *ctx, const eipc_scene *sc, const double *q_n, const int32_t *pt,
                              int64_t n_pt, const int32_t *ee, int64_t n_ee, double dhat, double kappa,
                              uint32_t flags, double *lag_pt, double *lag_ee, eipc_stream stream);

/* Lagged friction at x = W q + x_off over the pairs and lag records of
 * eipc_friction_lag (Sec. III-B, reduced through the embedding as Eq. 17):
 * u_k = P (G x - G x^n) with P = I - n n^T the tangential part of the
 * relative displacement, D = sum_k mu lambda_k f0(|u_k|) with
 *   f1(y) = 2 y/eps_h - y^2/eps_h^2 for y < eps_h, 1 otherwise,
 *   f0(y) = integral of f1 from eps_h to y, plus eps_h,
 * eps_h = eps_v h (the velocity threshold times the time step).  Pass
 * mu h^2 for the h^2-scaled term of E_IPC.  The pair Hessians are positive
 * semidefinite by construction (no projection).  Flags: EIPC_ENERGY,
 * EIPC_GRAD, EIPC_HESS.
 *   energy     device double[1] or NULL     grad_q  device double[3*n_node] or NULL
 *   hess_dense device double[(3*n_node)^2] or NULL (row-major)
 *   hess_bsr   host struct or NULL: context-owned BSR view (synchronizes)
 * Single scenes only. */
eipc_status eipc_friction_reduce(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const int32_t *pt,
                                 int64_t n_pt, const double *lag_pt, const int32_t *ee, int64_t n_ee,
                                 const double *lag_ee, double mu, double eps_h, uint32_t flags, double *energy,
                                 double *grad_q, double *hess_dense, eipc_bsr *hess_bsr, eipc_stream stream);

/* ---- planned contact step: one Newton iteration's contact stage with no
 * host synchronization and no allocation (capturable in a HIP graph) ---- */

/* Capacities of a planned step (element counts). */
typedef struct {
  int64_t cand_pt, cand_ee;   /* proximity candidates (only used when the step bound is not asked for) */
  int64_t swept_pt, swept_ee; /* swept candidates for the step bound */
  int64_t act_pt, act_ee;     /* active pairs */
  int64_t ent[4];             /* broad-phase item cell entries: PT, EE, swept PT, swept EE */
  int64_t qent[4];            /* broad-phase query cell entries, same order */
  int64_t buckets[4];         /* broad-phase hash buckets (powers of 2) */
  int64_t hess_blocks;        /* reduced-Hessian block table (power of 2); 0: no Hessian */
  int64_t nnzb;               /* BSR blocks */
} eipc_plan;

/* Measures a step at (q, dq, dx_off) with the synchronizing entry points
 * and returns capacities of `margin` (>= 1) times what it needed, then
 * reserves the context's scratch for them, so that eipc_contact_step
 * allocates nothing while the plan holds.  with_hess != 0 plans the
 * reduced-Hessian output.  Synchronizes. */
eipc_status eipc_plan_step(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const double *dq,
                           const double *dx_off, double dhat, double margin, int32_t with_hess, eipc_plan *plan,
                           eipc_stream stream);

/* One contact stage (Sec. III-B, III-C; Eq. 7, 10-11, 17): candidates at
 * q (unsorted), active pairs, energy per scene, reduced gradient and
 * (projected with EIPC_PROJECT) reduced Hessian, and the conservative step
 * bound alpha per scene for the search direction dq (+ dx_off), with the
 * semantics of eipc_build_candidates, eipc_barrier_reduce and
 * eipc_ccd_max_step.  When alpha is asked for, one swept broad phase serves
 * both: every candidate at q is a swept candidate (the swept boxes contain
 * the boxes at q), so the candidates at q are the swept candidates that
 * pass the candidate predicate at q, tested pair by pair before the
 * distance.  Enqueues work only: no synchronization, no
 * allocation, no host-side reads of device data, so it can be captured in
 * a HIP graph and replayed with new contents of q and dq.  With alpha
 * (outside profiling mode 2), the point-triangle part runs on a second
 * stream owned by the context (default
 * priority), forked from `stream` after the shared set-up and joined back
 * into it by events before the call returns: all results are ordered on
 * `stream`, and under capture the fork becomes a parallel branch of the
 * graph.  Calls on one context must not overlap (they share that stream
 * and the scratch).
 *   energy   device double[n_scene] or NULL     grad_q  device double[3*n_node] or NULL
 *   hess_bsr host struct or NULL (needs EIPC_HESS and plan->hess_blocks > 0): context-owned
 *            BSR view with nnzb = -1 (the count is rowptr[n_rows] on the device)
 *   alpha    device double[n_scene] or NULL: step bound per scene (dq may be NULL when NULL)
 *   counts   device int64[5] or NULL: PT and EE candidates, active pairs, swept PT and EE
 * Capacity overflow and data errors are reported by eipc_sync_status.
 * A graph captured from this call keeps the context's scratch addresses:
 * it stays valid while only planned steps of the same (or a smaller) plan
 * run on the context; any other entry point or a larger plan may move
 * that scratch, after which the graph must be captured again. */
eipc_status eipc_contact_step(eipc_ctx *ctx, const eipc_scene *sc, const eipc_plan *plan, const double *q,
                              const double *dq, const double *dx_off, double dhat, double kappa, uint32_t flags,
                              double s, double t_max, int64_t max_iter, double *energy, double *grad_q,
                              eipc_bsr *hess_bsr, double *alpha, int64_t *counts, eipc_stream stream);

/* Pair lists of the last eipc_contact_step on this context (test and
 * inspection use; valid until the next call that runs a planned step or
 * carves scratch).  which = 0 / 1: the PT / EE pairs the step tested (its
 * swept candidates when it computed alpha, else its candidates at q);
 * which = 2 / 3: its active PT / EE pairs.  out (device int32[2*cap])
 * receives the pairs as (first, second) rows in the step's unspecified
 * order and *n (host) their number; when *n > cap the call returns
 * EIPC_ERR_CAPACITY and writes nothing.  Lists cut short by a plan
 * overflow are returned as cut.  Synchronizes. */
eipc_status eipc_step_pairs(eipc_ctx *ctx, int32_t which, int32_t *out, int64_t cap, int64_t *n,
                            eipc_stream stream);

/* Launch shape of the library's kernels for this context: the broad-phase
 * cell edge as a multiple of the mean primitive box extent (> 0); the
 * workgroups per compute unit of the grid-stride kernels (pair terms,
 * expansion, narrow phase, CCD; each 1..64, 0 keeps the current value; the
 * array may be NULL); and how the unsorted (planned-step and step-bound)
 * broad phases split their work, query_cells = mode_PT + 4 * mode_EE with
 * mode 0 = one thread per query, 1 = one thread per (query, cell of its
 * box), 2 = one wavefront per (query, cell), 3 = bucket join (the queries
 * hashed like the items, each bucket's pairs tested from LDS) (-1 keeps
 * the current choice; default 15, the bucket join for both).  Used by the batch autotuner;
 * results do not depend on them except for the order of unsorted
 * candidate lists and the rounding order of sums.  A plan must be made
 * again after changing them. */
eipc_status eipc_set_tuning(eipc_ctx *ctx, double cell_scale, const int32_t wg_per_cu[4], int32_t query_cells);

/* Per-pair step bound of the CCD (Sec. III-C; the paper names a conservative
 * advancement CCD and cites C2A for it) used by every call of this context
 * that computes one (eipc_ccd_max_step, eipc_ccd_toi, eipc_contact_step;
 * a plan keeps working):
 *   EIPC_CCD_ADDITIVE (default): additive CCD, each step (0.9 of) the
 *     distance over lp, the largest possible closing speed (the point's
 *     speed plus the fastest triangle vertex, or the fastest vertex of each
 *     edge, after removing the mean motion).
 *   EIPC_CCD_CLOSEST_DIRECTION: the same steps with lp replaced, at every
 *     iterate, by the closing speed along the closest direction n (from the
 *     second primitive's closest point to the first's),
 *     mu = max_{second} n.p - min_{first} n.p <= lp: both primitives stay on
 *     their sides of the separating planes through the closest points, so
 *     the distance cannot fall faster than mu.  mu <= 0 bounds the pair by
 *     t_max.  Fewer, longer steps where the motion is mostly tangential.
 * Both bounds are conservative; their values differ.  EIPC_ERR_ARG for
 * another method. */
#define EIPC_CCD_ADDITIVE 0
#define EIPC_CCD_CLOSEST_DIRECTION 1
eipc_status eipc_set_ccd_method(eipc_ctx *ctx, int32_t method);

/* ---- dense reduced Newton system (adjoint of a converged step) ---- */

/* In-place dense FP64 Cholesky factorization A = L L^T of the reduced
 * Newton matrix of one implicit step, H = M^q + h^2 (Hessian of the step's
 * potentials) (Sec. III-A, Eq. 5-6; Sec. III-B, Eq. 10-12), which is
 * symmetric positive definite at a strict minimum.  A is row-major, leading
 * dimension lda >= n, device memory; only the lower triangle is read and L
 * overwrites it (the strict upper triangle is left unchanged).  *info
 * (host) receives 0 on success, or j+1 when the leading minor of order j+1
 * is not positive definite (the factor is then not usable).
 * Synchronizes. */
eipc_status eipc_cholesky(eipc_ctx *ctx, double *A, int64_t n, int64_t lda, int64_t *info, eipc_stream stream);

/* Solves A X = B with the factor written by eipc_cholesky.  B is row-major
 * [n][nrhs] device memory and is overwritten by X. */
eipc_status eipc_cholesky_solve(eipc_ctx *ctx, const double *L, int64_t n, int64_t lda, double *B, int64_t nrhs,
                                eipc_stream stream);

/* Reduced mass and gravity of one implicit step on a coarse tetrahedral
 * mesh, from interior samples of the body (M = J^T M_x J, Sec. III-A Eq. 1,
 * with the volume aggregation of Eq. 15; f = J^T f_ext, Eq. 16).  Sample s
 * has mass sample_mass (rho times its volume) and barycentric weights
 * sample_w[4 s .. 4 s + 3] in the coarse tet whose nodes are
 * sample_nodes[4 s .. 4 s + 3]; it adds sample_mass w_a w_b to the diagonal
 * of the 3x3 block (a, b) of M and -sample_mass gravity w_a to the z
 * component of node a in f.  Nodes that no sample reaches then get 1e-3 of
 * the mean mass of the reached nodes on their diagonal, so that the Newton
 * matrix stays definite (this reads M: clear M before the call).
 * M: dense [3 n_node x 3 n_node] row-major, leading dimension lda >=
 * 3 n_node; f: [3 n_node] node-major xyz, or NULL.  Both are added to.
 * Device memory, caller owned.  Enqueued on stream.  EIPC_ERR_ARG for bad
 * sizes or pointers. */
eipc_status eipc_reduced_mass(eipc_ctx *ctx, int32_t n_node, int64_t n_sample, const int32_t *sample_nodes,
                              const double *sample_w, double sample_mass, double gravity, double *M, int64_t lda,
                              double *f, eipc_stream stream);

/* elastic models for eipc_elastic */
enum {
  EIPC_ELASTIC_LINEAR = 0,       /* small-strain linear elasticity: psi = mu eps:eps + lam/2 tr(eps)^2 */
  EIPC_ELASTIC_COROTATIONAL = 1  /* linear corotational (Sec. IV-A): psi = mu |F - R|^2 + lam/2 tr(R^T F - I)^2 */
};

/* Elastic energy Phi of the coarse tetrahedra of one implicit step (Sec.
 * III-A; each tet's volume aggregated from samples as in Eq. 15; the
 * paper's bodies are linear corotational, Sec. IV-A) and its derivatives
 * in the reduced coordinates q (the coarse node positions, [3 n_node]).
 * Tet t has nodes tets[4 t .. 4 t + 3], rest node positions rest
 * ([3 n_node]) and volume vol[t] (tets with volume 0 are skipped);
 * F = sum_a x_a g_a^T with g_a the rest shape-function gradients.
 * EIPC_ELASTIC_LINEAR: eps = sym(F) - I, gradient and Hessian exact (the
 * Hessian is the constant stiffness K0).  EIPC_ELASTIC_COROTATIONAL: R the
 * rotation of F's polar decomposition, first Piola stress
 * P = 2 mu (F - R) + lam tr(R^T F - I) R (the exact gradient), Newton
 * matrix the warped stiffness R K0 R^T (positive semidefinite; K0 at the
 * rest shape).  young > 0 and -1 < poisson < 0.5 give the Lame parameters.
 * Adds scale * energy to energy[0], scale * gradient to grad ([3 n_node])
 * and scale * Newton matrix to hess (dense [3 n_node x 3 n_node] row-major,
 * leading dimension lda >= 3 n_node); each may be NULL.  Device memory,
 * caller owned.  Enqueued on stream.  EIPC_ERR_ARG for bad arguments; a
 * degenerate rest tet, or an inverted one (det F <= 0) in the corotational
 * model, adds nothing and raises EIPC_ERR_DEGENERATE through
 * eipc_sync_status. */
eipc_status eipc_elastic(eipc_ctx *ctx, int32_t n_node, int32_t n_tet, const int32_t *tets, const double *rest,
                         const double *vol, double young, double poisson, int32_t model, const double *q,
                         double scale, double *energy, double *grad, double *hess, int64_t lda,
                         eipc_stream stream);

/* ---- optional kernel timing (benchmarks) ---- */

/* Turn per-kernel timing on (1 or 2) or off (0).  While on, the library
 * brackets each launch of its main kernels with HIP events on the launch
 * stream.  With 2, the planned step also runs its PT chain on the caller's
 * stream, before the EE chain instead of beside it, so that each timed kernel
 * has the device to itself (its time then excludes waiting for the other
 * chain's kernels); results are the same.  Any other value: EIPC_ERR_ARG. */
eipc_status eipc_profile(eipc_ctx *ctx, int32_t enable);

/* Synchronizes on the recorded events and returns, for the kernel `name`
 * ("embed", "query_count_pt", "query_count_ee", "query_write_pt",
 * "query_write_ee", "narrow_pt", "narrow_ee", "barrier_pt", "barrier_ee",
 * "expand_pt", "expand_ee", "ccd_pt", "ccd_ee", "ccd_long_pt", "ccd_long_ee",
 * "hvp_pt", "hvp_ee"; in the planned step with a step bound "ccd_*" is the
 * narrow phase fused with the bound's first pass and "ccd_long_*" the pass
 * for pairs needing more advancement steps), the summed milliseconds and the
 * number of timed launches since the last reset.  reset != 0 clears all
 * totals after reading.  ms and launches are host pointers. */
eipc_status eipc_profile_read(eipc_ctx *ctx, const char *name, double *ms, int64_t *launches, int32_t reset);

/* ---- inspection entry points (same kernels as above, for tests) ---- */

/* Active subset of the given pairs (0 < d < dhat).  act_pt / act_ee
 * (device int32[n_pt] / [n_ee]) receive indices into pt / ee, type_pt /
 * type_ee (device int32, same sizes) the distance type, in unspecified
 * order; counts go to the host.  Synchronizes. */
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * product of eipc_barrier_hvp (same arguments, same result up to the
 * rounding order of its sums) with all scratch in a fixed array of
 * EIPC_NOALLOC_SCRATCH_BYTES that the library holds on each GPU from
 * module load until the process ends (its address is looked up once per
 * device by eipc_create).  The call allocates nothing, does not
 * synchronize, and records no memset.  It needs
 *   256 + 2 * (32 * n_vert + 64) + 8 * (n_pt + n_ee)  bytes
 * (each term rounded up to 256; n_pt, n_ee at least 1); larger inputs
 * return EIPC_ERR_CAPACITY with nothing enqueued.  Every call on one GPU,
 * from any context, uses that GPU's one array: calls that overlap in time
 * on one GPU (two streams, two host threads) race and give wrong results,
 * so callers order them on one stream.  Data-dependent errors go to the
 * context's status word as for eipc_barrier_hvp. */
#define EIPC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
eipc_status eipc_barrier_hvp_noalloc(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const int32_t *pt,
                                     int64_t n_pt, const int32_t *ee, int64_t n_ee, double dhat, double kappa,
                                     uint32_t flags, const double *v, const double *v_off, double *out,
                                     double *out_off, eipc_stream stream);

eipc_status eipc_narrow_phase(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const int32_t *pt,
                              int64_t n_pt, const int32_t *ee, int64_t n_ee, double dhat, int32_t *act_pt,
                              int32_t *type_pt, int64_t *n_act_pt, int32_t *act_ee, int32_t *type_ee,
                              int64_t *n_act_ee, eipc_stream stream);

/* Per-pair quantities for `n` pairs of one kind (0 = PT, 1 = EE): distance
 * type, squared distance, energy, 12-gradient and the 12x12 Hessian
 * (projected with EIPC_PROJECT).  Inactive pairs get e = 0, g = 0, H = 0.
 * Outputs are device arrays int32[n], double[n], double[n], double[n*12],
 * double[n*144]; any may be NULL. */
eipc_status eipc_pair_eval(eipc_ctx *ctx, const eipc_scene *sc, const double *q, int32_t kind,
                           const int32_t *pairs, int64_t n, double dhat, double kappa, uint32_t flags,
                           int32_t *type, double *s, double *e, double *g, double *H, eipc_stream stream);

/* Swept candidates of eipc_ccd_max_step (same layout and capacity rules as
 * eipc_build_candidates).  Synchronizes. */
eipc_status eipc_ccd_candidates(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const double *dq,
                                const double *dx_off, double dhat, int32_t *pt, int64_t cap_pt, int32_t *ee,
                                int64_t cap_ee, int64_t *n_pt, int64_t *n_ee, eipc_stream stream);

/* Per-pair step bound of eipc_ccd_max_step for `n` given pairs of one
 * kind; t (device double[n]) and iters (device int64[n] or NULL). */
eipc_status eipc_ccd_toi(eipc_ctx *ctx, const eipc_scene *sc, const double *q, const double *dq,
                         const double *dx_off, int32_t kind, const int32_t *pairs, int64_t n, double s,
                         double t_max, int64_t max_iter, double *t, int64_t *iters, eipc_stream stream);

/* Device FP64 square root and division on n inputs (sqrt(a), a / b), to
 * check that the device rounds them like the host. */
eipc_status eipc_fp64_selftest(eipc_ctx *ctx, const double *a, const double *b, double *sqrt_a, double *a_div_b,
                               int64_t n, eipc_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* EIPC_H */
