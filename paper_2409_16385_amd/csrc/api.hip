// C-ABI entry points (see include/eipc.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include <mutex>

#include "common.h"

namespace eipc {

// Fixed scratch of eipc_barrier_hvp_noalloc: one copy per GPU, held from
// module load until the process ends.  Host code uses its per-device
// address (noalloc_scratch_of), never this name.
static __device__ __align__(256) unsigned char scratch[EIPC_NOALLOC_SCRATCH_BYTES];

// Device address of this GPU's copy of `scratch` (the device must be
// current); looked up once per device.  nullptr when the lookup fails.
static void *noalloc_scratch_of(int device) {
  static std::mutex mu;
  static void *addr[64] = {nullptr};
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    addr[device] = p;
  }
  return addr[device];
}

eipc_status set_err(eipc_ctx *c, eipc_status st, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return st;
}

const char *const kKernelNames[K_NUM] = {"embed",        "query_count_pt", "query_count_ee", "query_write_pt",
                                         "query_write_ee", "narrow_pt",     "narrow_ee",      "barrier_pt",
                                         "barrier_ee",     "ccd_pt",        "ccd_ee",         "hvp_pt",
                                         "hvp_ee",         "expand_pt",     "expand_ee",      "ccd_long_pt",
                                         "ccd_long_ee"};

static hipEvent_t take_event(eipc_ctx *c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(eipc_ctx *c_, int id_, hipStream_t s_) : c(c_), id(id_), s(s_) {
  if (!c->prof) return;
  a = take_event(c);
  b = take_event(c);
  if (a && b) hipEventRecord(a, s);
}

ProfScope::~ProfScope() {
  if (!c->prof || !a || !b) return;
  hipEventRecord(b, s);
  c->prof_pending.push_back(ProfRec{id, a, b});
}

static void prof_collect(eipc_ctx *c) {
  for (auto &r : c->prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
      c->prof_ms[r.id] += ms;
      c->prof_n[r.id] += 1;
    }
    c->prof_pool.push_back(r.start);
    c->prof_pool.push_back(r.stop);
  }
  c->prof_pending.clear();
}

eipc_status ensure(eipc_ctx *c, BufId id, size_t bytes, void **out) {
  DevBuf &b = c->buf[id];
  if (c->arena) {
    // arena: carve at the top when the buffer is not yet part of this call
    // or too small (its earlier space in this call is then left unused)
    if (b.epoch != c->epoch || b.bytes < bytes) {
      const size_t nb = (std::max(bytes, (size_t)256) + 255) & ~(size_t)255;
      if (c->arena_top + nb > c->arena_bytes) {
        c->scratch_short = true;
        return set_err(c, EIPC_ERR_CAPACITY,
                       "scratch reservation of %zu bytes exhausted: this call needs more than %zu bytes",
                       c->arena_bytes, c->arena_top + nb);
      }
      b.p = c->arena + c->arena_top;
      b.bytes = nb;
      b.epoch = c->epoch;
      c->arena_top += nb;
      c->arena_high = std::max(c->arena_high, c->arena_top);
    }
    *out = b.p;
    return EIPC_OK;
  }
  if (b.bytes < bytes) {
    // grow by at least a quarter so that repeated growth stays rare; the
    // old buffer may still be read by enqueued work, so it is retired, not
    // freed (no device synchronization here)
    size_t nb = std::max({bytes, (size_t)4096, b.bytes + b.bytes / 4});
    nb = (nb + 4095) & ~(size_t)4095;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess)
      return set_err(c, EIPC_ERR_HIP, "hipMalloc(%zu) failed: %s", nb, hipGetErrorString(e));
    if (b.p) c->retired.push_back(b.p);
    b.p = p;
    b.bytes = nb;
  }
  *out = b.p;
  return EIPC_OK;
}

// frees retired scratch; the device must be idle on every stream that
// used it (callers synchronize first)
static void free_retired(eipc_ctx *c) {
  for (void *p : c->retired) hipFree(p);
  c->retired.clear();
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

static eipc_status fill_i32(eipc_ctx *c, int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n == 0) return EIPC_OK;
  k_fill_i32<<<(int)std::min<int64_t>(grid_for(n, 256), 4096), 256, 0, s>>>(p, n, v);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

static eipc_status check_scene(eipc_ctx *c, const eipc_scene *sc) {
  if (!c) return EIPC_ERR_ARG;
  if (!sc) return set_err(c, EIPC_ERR_ARG, "scene is NULL");
  if (sc->n_vert < 0 || sc->n_node < 0 || sc->n_face < 0 || sc->n_edge < 0)
    return set_err(c, EIPC_ERR_ARG, "negative scene size");
  if (!sc->W_rowptr || (sc->n_vert > 0 && (!sc->W_col || !sc->W_val)))
    return set_err(c, EIPC_ERR_ARG, "W is NULL");
  if (sc->n_face > 0 && !sc->faces) return set_err(c, EIPC_ERR_ARG, "faces is NULL");
  if (sc->n_edge > 0 && !sc->edges) return set_err(c, EIPC_ERR_ARG, "edges is NULL");
  if (sc->n_scene < 0 || sc->n_scene > 65536) return set_err(c, EIPC_ERR_ARG, "n_scene must be in [0, 65536]");
  if (sc->n_scene > 1 && sc->n_vert > 0 && !sc->vert_scene)
    return set_err(c, EIPC_ERR_ARG, "vert_scene is NULL for a batch");
  return EIPC_OK;
}

static eipc_status fill_u64(eipc_ctx *c, uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return EIPC_OK;
  k_fill_u64<<<(int)std::min<int64_t>(grid_for(n, 256), 4096), 256, 0, s>>>(p, n, v);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

// the EE mollifier needs the rest positions it is defined by
static eipc_status check_mollify(eipc_ctx *c, const eipc_scene *sc, uint32_t flags) {
  if ((flags & EIPC_MOLLIFY) && !sc->x_rest && sc->n_edge > 0)
    return set_err(c, EIPC_ERR_ARG, "EIPC_MOLLIFY needs the scene's rest positions (x_rest is NULL)");
  return EIPC_OK;
}

static eipc_status check_dhat(eipc_ctx *c, double dhat) {
  if (!(dhat > 0.0) || !std::isfinite(dhat)) return set_err(c, EIPC_ERR_ARG, "dhat must be positive and finite");
  return EIPC_OK;
}

// device status -> API status; clears the word
static eipc_status read_status(eipc_ctx *c, hipStream_t s, bool clear = true) {
  uint32_t st = 0;
  EIPC_HIP(c, hipMemcpyAsync(&st, c->status, 4, hipMemcpyDeviceToHost, s));
  EIPC_HIP(c, hipStreamSynchronize(s));
  if (clear && st) EIPC_HIP(c, hipMemsetAsync(c->status, 0, 4, s));
  if (st & ST_BAD_W) return set_err(c, EIPC_ERR_ARG, "a row of W has more than 4 weights");
  if (st & ST_BAD_SCENE) return set_err(c, EIPC_ERR_ARG, "a vertex scene id is out of range");
  if (st & ST_PLAN_OVERFLOW) return set_err(c, EIPC_ERR_CAPACITY, "a capacity of the step plan was exceeded");
  if (st & ST_HASH_OVERFLOW)
    return set_err(c, EIPC_ERR_CAPACITY, "the reduced-Hessian block table is full (blocks were dropped)");
  if (st & ST_DEGENERATE)
    return set_err(c, EIPC_ERR_DEGENERATE, "an element of the elastic mesh is degenerate or inverted");
  if (st & ST_INTERSECTING) return set_err(c, EIPC_ERR_INTERSECTING, "a candidate pair has zero distance");
  if (st & ST_NONFINITE) return set_err(c, EIPC_ERR_NONFINITE, "non-finite position or pair quantity");
  if (st & ST_CCD_CAPPED) return EIPC_WARN_CCD_CAPPED;
  return EIPC_OK;
}

static int64_t pow2_at_least(int64_t v) {
  uint64_t p = 1;
  while ((int64_t)p < v) p <<= 1;
  return (int64_t)std::min<uint64_t>(p, 1ull << 34);
}

// global block hash of the reduced Hessian, cleared (int64 keys, -1 empty)
static eipc_status hess_table(eipc_ctx *c, int64_t cap, HessOut &h, hipStream_t s) {
  EIPC_TRY(ensure_t(c, B_HKEY, (size_t)cap, &h.hkey));
  EIPC_TRY(ensure_t(c, B_HVAL, (size_t)cap * 9, &h.hval));
  EIPC_TRY(fill_u64(c, (uint64_t *)h.hkey, cap, ~0ull, s));
  EIPC_TRY(launch_zero(c, h.hval, sizeof(double) * 9 * cap, s));
  h.kind = 2;
  h.hmask = (uint64_t)(cap - 1);
  return EIPC_OK;
}

static eipc_status narrow_both(eipc_ctx *c, const eipc_scene *sc, const double *xs, const int32_t *pt, int64_t n_pt,
                               const int32_t *ee, int64_t n_ee, double dhat, int32_t **act_pt, int32_t **typ_pt,
                               int32_t **act_ee, int32_t **typ_ee, hipStream_t s) {
  EIPC_TRY(ensure_t(c, B_ACT_PT, (size_t)std::max<int64_t>(n_pt, 1), act_pt));
  EIPC_TRY(ensure_t(c, B_TYP_PT, (size_t)std::max<int64_t>(n_pt, 1), typ_pt));
  EIPC_TRY(ensure_t(c, B_ACT_EE, (size_t)std::max<int64_t>(n_ee, 1), act_ee));
  EIPC_TRY(ensure_t(c, B_TYP_EE, (size_t)std::max<int64_t>(n_ee, 1), typ_ee));
  EIPC_TRY(launch_zero(c, c->counters + 2, 2 * sizeof(int64_t), s));
  EIPC_TRY(launch_narrow(c, sc, 0, xs, pt, n_pt, dhat, *act_pt, *typ_pt, c->counters + 2, s));
  EIPC_TRY(launch_narrow(c, sc, 1, xs, ee, n_ee, dhat, *act_ee, *typ_ee, c->counters + 3, s));
  return EIPC_OK;
}

}  // namespace eipc

using namespace eipc;

extern "C" {

const char *eipc_status_string(eipc_status s) {
  switch (s) {
    case EIPC_OK: return "ok";
    case EIPC_ERR_ARG: return "invalid argument";
    case EIPC_ERR_CAPACITY: return "output capacity too small";
    case EIPC_ERR_INTERSECTING: return "intersecting input (zero distance pair)";
    case EIPC_ERR_DEGENERATE: return "degenerate primitive";
    case EIPC_ERR_NONFINITE: return "non-finite value";
    case EIPC_ERR_HIP: return "HIP runtime error";
    case EIPC_WARN_CCD_CAPPED: return "CCD iteration cap reached (bound still conservative)";
    default: return "unknown status";
  }
}

eipc_status eipc_create(eipc_ctx **out, int32_t device, size_t reserve_bytes) {
  if (!out) return EIPC_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EIPC_ERR_ARG;
  eipc_ctx *c = new (std::nothrow) eipc_ctx();
  if (!c) return EIPC_ERR_HIP;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess || hipMalloc(&c->status, 256) != hipSuccess ||
      hipMalloc(&c->stats, 32 * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->counters, 16 * sizeof(int64_t)) != hipSuccess ||
      hipMemset(c->status, 0, 256) != hipSuccess || hipMemset(c->counters, 0, 16 * sizeof(int64_t)) != hipSuccess) {
    eipc_destroy(c);
    return EIPC_ERR_HIP;
  }
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess) {
    eipc_destroy(c);
    return EIPC_ERR_HIP;
  }
  if (reserve_bytes > 0) {
    const size_t nb = (reserve_bytes + 4095) & ~(size_t)4095;
    if (hipMalloc((void **)&c->arena, nb) != hipSuccess) {
      c->arena = nullptr;
      eipc_destroy(c);
      return EIPC_ERR_HIP;
    }
    c->arena_bytes = nb;
  }
  c->noalloc_scratch = noalloc_scratch_of(device);
  if (!c->noalloc_scratch) {
    eipc_destroy(c);
    return EIPC_ERR_HIP;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    c->num_cu = ncu;
  *out = c;
  return EIPC_OK;
}

void eipc_destroy(eipc_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  prof_collect(c);
  for (auto e : c->prof_pool) hipEventDestroy(e);
  if (c->arena) {
    hipFree(c->arena);
  } else {
    for (auto &b : c->buf)
      if (b.p) hipFree(b.p);
  }
  free_retired(c);
  if (c->status) hipFree(c->status);
  if (c->stats) hipFree(c->stats);
  if (c->counters) hipFree(c->counters);
  if (c->fork_ev) hipEventDestroy(c->fork_ev);
  if (c->join_ev) hipEventDestroy(c->join_ev);
  if (c->side) hipStreamDestroy(c->side);
  delete c;
}

const char *eipc_last_error(const eipc_ctx *c) { return c ? c->err : "no context"; }

eipc_status eipc_scratch_bytes(const eipc_ctx *c, size_t *reserved, size_t *high_water) {
  if (!c || !reserved || !high_water) return EIPC_ERR_ARG;
  *reserved = c->arena_bytes;
  if (c->arena) {
    *high_water = c->arena_high;
  } else {
    size_t t = 0;
    for (const auto &b : c->buf) t += b.bytes;
    *high_water = t;
  }
  return EIPC_OK;
}

eipc_status eipc_profile(eipc_ctx *c, int32_t enable) {
  if (!c) return EIPC_ERR_ARG;
  if (enable < 0 || enable > 2) return set_err(c, EIPC_ERR_ARG, "profile mode must be 0, 1 or 2");
  c->prof = enable != 0;
  c->prof_serial = enable == 2;
  return EIPC_OK;
}

eipc_status eipc_profile_read(eipc_ctx *c, const char *name, double *ms, int64_t *launches, int32_t reset) {
  if (!c || !name || !ms || !launches) return EIPC_ERR_ARG;
  EIPC_HIP(c, hipSetDevice(c->device));
  prof_collect(c);
  int id = -1;
  for (int k = 0; k < K_NUM; ++k)
    if (std::strcmp(name, kKernelNames[k]) == 0) id = k;
  if (id < 0) return set_err(c, EIPC_ERR_ARG, "unknown kernel name %s", name);
  *ms = c->prof_ms[id];
  *launches = c->prof_n[id];
  if (reset)
    for (int k = 0; k < K_NUM; ++k) {
      c->prof_ms[k] = 0.0;
      c->prof_n[k] = 0;
    }
  return EIPC_OK;
}

eipc_status eipc_sync_status(eipc_ctx *c, eipc_stream stream) {
  if (!c) return EIPC_ERR_ARG;
  EIPC_HIP(c, hipSetDevice(c->device));
  return read_status(c, (hipStream_t)stream);
}

eipc_status eipc_embed(eipc_ctx *c, const eipc_scene *sc, const double *q, const double *off, double *x,
                       eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  if ((!q && sc->n_node > 0) || (!x && sc->n_vert > 0)) return set_err(c, EIPC_ERR_ARG, "q or x is NULL");
  EIPC_HIP(c, hipSetDevice(c->device));
  return launch_embed(c, sc, q, off, nullptr, x, (hipStream_t)stream);
}

eipc_status eipc_build_candidates(eipc_ctx *c, const eipc_scene *sc, const double *q, double dhat, int32_t *pt,
                                  int64_t cap_pt, int32_t *ee, int64_t cap_ee, int64_t *n_pt, int64_t *n_ee,
                                  eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (!n_pt || !n_ee || (!q && sc->n_node > 0) || cap_pt < 0 || cap_ee < 0)
    return set_err(c, EIPC_ERR_ARG, "bad candidate arguments");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  double *xs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)PSTRIDE * sc->n_vert + 1, &xs));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  eipc_status s1 = broad_phase(c, sc, 0, xs, nullptr, dhat, pt, cap_pt, n_pt, 1, s);
  if ((s1 != EIPC_OK && s1 != EIPC_ERR_CAPACITY) || c->scratch_short) return s1;
  eipc_status s2 = broad_phase(c, sc, 1, xs, nullptr, dhat, ee, cap_ee, n_ee, 1, s);
  if ((s2 != EIPC_OK && s2 != EIPC_ERR_CAPACITY) || c->scratch_short) return s2;
  eipc_status st = read_status(c, s);
  if (st != EIPC_OK && st != EIPC_WARN_CCD_CAPPED) return st;
  if (s1 == EIPC_ERR_CAPACITY || s2 == EIPC_ERR_CAPACITY)
    return set_err(c, EIPC_ERR_CAPACITY, "candidates need %lld PT / %lld EE slots", (long long)*n_pt,
                   (long long)*n_ee);
  return EIPC_OK;
}

eipc_status eipc_barrier_reduce(eipc_ctx *c, const eipc_scene *sc, const double *q, const int32_t *pt, int64_t n_pt,
                                const int32_t *ee, int64_t n_ee, double dhat, double kappa, uint32_t flags,
                                double *energy, double *grad_q, double *hess_dense, eipc_bsr *hess_bsr,
                                int64_t *n_active, eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (n_pt < 0 || n_ee < 0 || (n_pt > 0 && !pt) || (n_ee > 0 && !ee) || (!q && sc->n_node > 0) ||
      !std::isfinite(kappa))
    return set_err(c, EIPC_ERR_ARG, "bad pair or parameter arguments");
  EIPC_TRY(check_mollify(c, sc, flags));
  const bool want_h = (flags & EIPC_HESS) && (hess_dense || hess_bsr);
  if (want_h && 3 * (int64_t)sc->n_node >= (int64_t)INT32_MAX)
    return set_err(c, EIPC_ERR_ARG, "reduced Hessian output needs 3 * n_node < 2^31");
  if (hess_dense && hess_bsr) return set_err(c, EIPC_ERR_ARG, "ask for one Hessian layout");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  double *xs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)PSTRIDE * sc->n_vert + 1, &xs));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  int32_t *act_pt, *typ_pt, *act_ee, *typ_ee;
  EIPC_TRY(narrow_both(c, sc, xs, pt, n_pt, ee, n_ee, dhat, &act_pt, &typ_pt, &act_ee, &typ_ee, s));
  const int64_t n3 = 3 * (int64_t)sc->n_node;
  for (int attempt = 0;; ++attempt) {
    if (energy) EIPC_TRY(launch_zero(c, energy, sizeof(double) * n_scene_of(sc), s));
    if (grad_q && (flags & EIPC_GRAD)) EIPC_TRY(launch_zero(c, grad_q, sizeof(double) * n3, s));
    HessOut h{0, nullptr, nullptr, nullptr, 0};
    if (want_h && hess_dense) {
      EIPC_TRY(launch_zero(c, hess_dense, sizeof(double) * n3 * n3, s));
      h.kind = 1;
      h.dense = hess_dense;
    } else if (want_h) {
      int64_t cap = std::max<int64_t>(c->hash_cap, pow2_at_least(16 * (int64_t)sc->n_node));
      c->hash_cap = cap;
      EIPC_TRY(hess_table(c, cap, h, s));
    }
    const uint32_t f = flags & (want_h ? ~0u : ~(uint32_t)EIPC_HESS);
    double *g = (flags & EIPC_GRAD) ? grad_q : nullptr;
    // with enough pairs of both kinds, the PT chain runs on the side stream
    // beside the EE chain, as in the planned step (their outputs meet in
    // atomics; their scratch is per kind); small calls stay on one stream,
    // where the fork and join would cost more than the overlap gains
    const bool fork = !c->prof_serial && n_pt > 0 && n_ee > 0 && n_pt + n_ee >= (int64_t)1 << 16;
    if (fork) {
      EIPC_HIP(c, hipEventRecord(c->fork_ev, s));
      EIPC_HIP(c, hipStreamWaitEvent(c->side, c->fork_ev, 0));
    }
    const eipc_status b0 = launch_barrier(c, sc, 0, xs, pt, act_pt, typ_pt, c->counters + 2, n_pt, dhat, kappa, f,
                                          energy, g, h, fork ? c->side : s);
    const eipc_status b1 = b0 != EIPC_OK ? b0
                                         : launch_barrier(c, sc, 1, xs, ee, act_ee, typ_ee, c->counters + 3, n_ee,
                                                          dhat, kappa, f, energy, g, h, s);
    if (fork) {
      // joined also after a failure, so that nothing enqueued on the side
      // stream can overlap the caller's next use of the scratch
      EIPC_HIP(c, hipEventRecord(c->join_ev, c->side));
      EIPC_HIP(c, hipStreamWaitEvent(s, c->join_ev, 0));
    }
    EIPC_TRY(b1);
    if (h.kind == 1) EIPC_TRY(launch_dense_mirror(c, sc->n_node, hess_dense, s));
    if (h.kind == 2) {
      uint32_t st = 0;
      EIPC_HIP(c, hipMemcpyAsync(&st, c->status, 4, hipMemcpyDeviceToHost, s));
      EIPC_HIP(c, hipStreamSynchronize(s));
      if ((st & ST_HASH_OVERFLOW) && attempt < 8) {
        st &= ~ST_HASH_OVERFLOW;
        EIPC_HIP(c, hipMemcpyAsync(c->status, &st, 4, hipMemcpyHostToDevice, s));
        c->hash_cap *= 4;
        continue;
      }
      if (st & ST_HASH_OVERFLOW) return set_err(c, EIPC_ERR_CAPACITY, "reduced Hessian hash overflow");
      EIPC_TRY(bsr_compact(c, sc->n_node, h, hess_bsr, s));
    }
    break;
  }
  if (n_active) {
    int64_t cnt[2];
    EIPC_HIP(c, hipMemcpyAsync(cnt, c->counters + 2, 16, hipMemcpyDeviceToHost, s));
    EIPC_HIP(c, hipStreamSynchronize(s));
    *n_active = cnt[0] + cnt[1];
  }
  if (n_active || hess_bsr) {
    eipc_status st = read_status(c, s);
    if (st != EIPC_OK && st != EIPC_WARN_CCD_CAPPED) return st;
  }
  return EIPC_OK;
}

eipc_status eipc_ccd_max_step(eipc_ctx *c, const eipc_scene *sc, const double *q, const double *dq,
                              const double *dx_off, double dhat, double sfac, double t_max, int64_t max_iter,
                              double *alpha, int64_t *n_cand, eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (!alpha || (sc->n_node > 0 && (!q || !dq)) || !(sfac > 0.0 && sfac < 1.0) || !(t_max > 0.0) ||
      !std::isfinite(t_max) || max_iter < 1)
    return set_err(c, EIPC_ERR_ARG, "bad CCD arguments");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  const int64_t n3 = (int64_t)PSTRIDE * sc->n_vert;
  double *xs, *ps, *x1s;
  EIPC_TRY(ensure_t(c, B_X, (size_t)n3 + 1, &xs));
  EIPC_TRY(ensure_t(c, B_P, (size_t)n3 + 1, &ps));
  EIPC_TRY(ensure_t(c, B_X1, (size_t)n3 + 1, &x1s));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  EIPC_TRY(launch_embed(c, sc, dq, dx_off, ps, nullptr, s));
  EIPC_TRY(launch_add_soa(c, n3, xs, ps, x1s, s));
  int64_t npt = 0, nee = 0;
  int32_t *cpt = nullptr, *cee = nullptr;
  EIPC_TRY(broad_phase(c, sc, 0, xs, x1s, dhat, nullptr, 0, &npt, 0, s, B_CAND_PT, &cpt));
  EIPC_TRY(broad_phase(c, sc, 1, xs, x1s, dhat, nullptr, 0, &nee, 0, s, B_CAND_EE, &cee));
  const int nsc = n_scene_of(sc);
  uint64_t *abits;
  EIPC_TRY(ensure_t(c, B_ALPHA, (size_t)nsc, &abits));
  uint64_t tb;
  std::memcpy(&tb, &t_max, 8);
  EIPC_TRY(fill_u64(c, abits, nsc, tb, s));
  EIPC_TRY(launch_ccd(c, sc, 0, xs, ps, cpt, npt, sfac, t_max, max_iter, abits, nullptr, nullptr, s));
  EIPC_TRY(launch_ccd(c, sc, 1, xs, ps, cee, nee, sfac, t_max, max_iter, abits, nullptr, nullptr, s));
  EIPC_HIP(c, hipMemcpyAsync(alpha, abits, 8 * (size_t)nsc, hipMemcpyDeviceToHost, s));
  EIPC_HIP(c, hipStreamSynchronize(s));
  if (n_cand) *n_cand = npt + nee;
  return read_status(c, s);
}

eipc_status eipc_barrier_hvp(eipc_ctx *c, const eipc_scene *sc, const double *q, const int32_t *pt, int64_t n_pt,
                             const int32_t *ee, int64_t n_ee, double dhat, double kappa, uint32_t flags,
                             const double *v, const double *v_off, double *out, double *out_off,
                             eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (n_pt < 0 || n_ee < 0 || (n_pt > 0 && !pt) || (n_ee > 0 && !ee) || (sc->n_node > 0 && (!q || !v || !out)))
    return set_err(c, EIPC_ERR_ARG, "bad HVP arguments");
  EIPC_TRY(check_mollify(c, sc, flags));
  if (flags & EIPC_PROJECT_REDUCED)
    return set_err(c, EIPC_ERR_ARG, "EIPC_PROJECT_REDUCED projects reduced blocks: not for per-pair outputs");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  const int64_t n3 = (int64_t)PSTRIDE * sc->n_vert;
  double *xs, *xvs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)n3 + 1, &xs));
  EIPC_TRY(ensure_t(c, B_XV, (size_t)n3 + 1, &xvs));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  EIPC_TRY(launch_embed(c, sc, v, v_off, xvs, nullptr, s));
  int32_t *act_pt, *typ_pt, *act_ee, *typ_ee;
  EIPC_TRY(narrow_both(c, sc, xs, pt, n_pt, ee, n_ee, dhat, &act_pt, &typ_pt, &act_ee, &typ_ee, s));
  EIPC_TRY(launch_zero(c, out, sizeof(double) * 3 * (size_t)sc->n_node, s));
  if (out_off) EIPC_TRY(launch_zero(c, out_off, sizeof(double) * 3 * (size_t)sc->n_vert, s));
  EIPC_TRY(launch_hvp(c, sc, 0, xs, xvs, pt, act_pt, typ_pt, c->counters + 2, n_pt, dhat, kappa, flags, out, out_off,
                      s));
  EIPC_TRY(launch_hvp(c, sc, 1, xs, xvs, ee, act_ee, typ_ee, c->counters + 3, n_ee, dhat, kappa, flags, out, out_off,
                      s));
  return EIPC_OK;
}

eipc_status eipc_barrier_hvp_noalloc(eipc_ctx *c, const eipc_scene *sc, const double *q, const int32_t *pt,
                                     int64_t n_pt, const int32_t *ee, int64_t n_ee, double dhat, double kappa,
                                     uint32_t flags, const double *v, const double *v_off, double *out,
                                     double *out_off, eipc_stream stream) {
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (n_pt < 0 || n_ee < 0 || (n_pt > 0 && !pt) || (n_ee > 0 && !ee) || (sc->n_node > 0 && (!q || !v || !out)))
    return set_err(c, EIPC_ERR_ARG, "bad HVP arguments");
  EIPC_TRY(check_mollify(c, sc, flags));
  if (flags & EIPC_PROJECT_REDUCED)
    return set_err(c, EIPC_ERR_ARG, "EIPC_PROJECT_REDUCED projects reduced blocks: not for per-pair outputs");
  // carve the fixed array: counters, positions of q and of v, active lists
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t pos = up(sizeof(double) * PSTRIDE * (size_t)sc->n_vert + 64);
  const size_t lpt = up(sizeof(int32_t) * (size_t)std::max<int64_t>(n_pt, 1));
  const size_t lee = up(sizeof(int32_t) * (size_t)std::max<int64_t>(n_ee, 1));
  const size_t need = 256 + 2 * pos + 2 * lpt + 2 * lee;
  if (need > EIPC_NOALLOC_SCRATCH_BYTES)
    return set_err(c, EIPC_ERR_CAPACITY, "this product needs %zu bytes of scratch; the fixed array holds %zu", need,
                   (size_t)EIPC_NOALLOC_SCRATCH_BYTES);
  if (!c->noalloc_scratch) return set_err(c, EIPC_ERR_HIP, "no address for the fixed scratch array");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  char *base = (char *)c->noalloc_scratch;
  int64_t *cnt = (int64_t *)base;
  double *xs = (double *)(base + 256);
  double *xvs = (double *)(base + 256 + pos);
  int32_t *act_pt = (int32_t *)(base + 256 + 2 * pos);
  int32_t *typ_pt = (int32_t *)(base + 256 + 2 * pos + lpt);
  int32_t *act_ee = (int32_t *)(base + 256 + 2 * pos + 2 * lpt);
  int32_t *typ_ee = (int32_t *)(base + 256 + 2 * pos + 2 * lpt + lee);
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  EIPC_TRY(launch_embed(c, sc, v, v_off, xvs, nullptr, s));
  EIPC_TRY(launch_zero(c, cnt, 2 * sizeof(int64_t), s));  // the array keeps the last call's counts
  EIPC_TRY(launch_narrow(c, sc, 0, xs, pt, n_pt, dhat, act_pt, typ_pt, cnt, s));
  EIPC_TRY(launch_narrow(c, sc, 1, xs, ee, n_ee, dhat, act_ee, typ_ee, cnt + 1, s));
  EIPC_TRY(launch_zero(c, out, sizeof(double) * 3 * (size_t)sc->n_node, s));
  if (out_off) EIPC_TRY(launch_zero(c, out_off, sizeof(double) * 3 * (size_t)sc->n_vert, s));
  EIPC_TRY(launch_hvp(c, sc, 0, xs, xvs, pt, act_pt, typ_pt, cnt, n_pt, dhat, kappa, flags, out, out_off, s, false));
  EIPC_TRY(launch_hvp(c, sc, 1, xs, xvs, ee, act_ee, typ_ee, cnt + 1, n_ee, dhat, kappa, flags, out, out_off, s,
                      false));
  return EIPC_OK;
}

eipc_status eipc_friction_lag(eipc_ctx *c, const eipc_scene *sc, const double *q_n, const int32_t *pt, int64_t n_pt,
                              const int32_t *ee, int64_t n_ee, double dhat, double kappa, uint32_t flags,
                              double *lag_pt, double *lag_ee, eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (n_pt < 0 || n_ee < 0 || (n_pt > 0 && (!pt || !lag_pt)) || (n_ee > 0 && (!ee || !lag_ee)) ||
      (!q_n && sc->n_node > 0) || !(kappa >= 0.0) || !std::isfinite(kappa))
    return set_err(c, EIPC_ERR_ARG, "bad friction-lag arguments");
  if (sc->n_scene > 1) return set_err(c, EIPC_ERR_ARG, "friction takes one scene");
  EIPC_TRY(check_mollify(c, sc, flags));
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  double *xs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)PSTRIDE * sc->n_vert + 1, &xs));
  EIPC_TRY(launch_embed(c, sc, q_n, sc->x_off, xs, nullptr, s));
  EIPC_TRY(launch_friction_lag(c, sc, 0, xs, pt, n_pt, dhat, kappa, flags, lag_pt, s));
  EIPC_TRY(launch_friction_lag(c, sc, 1, xs, ee, n_ee, dhat, kappa, flags, lag_ee, s));
  return EIPC_OK;
}

eipc_status eipc_friction_reduce(eipc_ctx *c, const eipc_scene *sc, const double *q, const int32_t *pt, int64_t n_pt,
                                 const double *lag_pt, const int32_t *ee, int64_t n_ee, const double *lag_ee,
                                 double mu, double eps_h, uint32_t flags, double *energy, double *grad_q,
                                 double *hess_dense, eipc_bsr *hess_bsr, eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  if (n_pt < 0 || n_ee < 0 || (n_pt > 0 && (!pt || !lag_pt)) || (n_ee > 0 && (!ee || !lag_ee)) ||
      (!q && sc->n_node > 0) || !(mu >= 0.0) || !std::isfinite(mu) || !(eps_h > 0.0) || !std::isfinite(eps_h))
    return set_err(c, EIPC_ERR_ARG, "bad friction arguments");
  if (sc->n_scene > 1) return set_err(c, EIPC_ERR_ARG, "friction takes one scene");
  const bool want_h = (flags & EIPC_HESS) && (hess_dense || hess_bsr);
  if (want_h && 3 * (int64_t)sc->n_node >= (int64_t)INT32_MAX)
    return set_err(c, EIPC_ERR_ARG, "reduced Hessian output needs 3 * n_node < 2^31");
  if (hess_dense && hess_bsr) return set_err(c, EIPC_ERR_ARG, "ask for one Hessian layout");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  double *xs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)PSTRIDE * sc->n_vert + 1, &xs));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  const int64_t n3 = 3 * (int64_t)sc->n_node;
  double *e = (flags & EIPC_ENERGY) ? energy : nullptr;
  double *g = (flags & EIPC_GRAD) ? grad_q : nullptr;
  for (int attempt = 0;; ++attempt) {
    if (e) EIPC_TRY(launch_zero(c, e, sizeof(double), s));
    if (g) EIPC_TRY(launch_zero(c, g, sizeof(double) * n3, s));
    HessOut h{0, nullptr, nullptr, nullptr, 0};
    if (want_h && hess_dense) {
      EIPC_TRY(launch_zero(c, hess_dense, sizeof(double) * n3 * n3, s));
      h.kind = 1;
      h.dense = hess_dense;
    } else if (want_h) {
      int64_t cap = std::max<int64_t>(c->hash_cap, pow2_at_least(16 * (int64_t)sc->n_node));
      c->hash_cap = cap;
      EIPC_TRY(hess_table(c, cap, h, s));
    }
    EIPC_TRY(launch_friction(c, sc, 0, xs, pt, n_pt, lag_pt, mu, eps_h, e, g, h, s));
    EIPC_TRY(launch_friction(c, sc, 1, xs, ee, n_ee, lag_ee, mu, eps_h, e, g, h, s));
    if (h.kind == 1) EIPC_TRY(launch_dense_mirror(c, sc->n_node, hess_dense, s));
    if (h.kind == 2) {
      uint32_t st = 0;
      EIPC_HIP(c, hipMemcpyAsync(&st, c->status, 4, hipMemcpyDeviceToHost, s));
      EIPC_HIP(c, hipStreamSynchronize(s));
      if ((st & ST_HASH_OVERFLOW) && attempt < 8) {
        st &= ~ST_HASH_OVERFLOW;
        EIPC_HIP(c, hipMemcpyAsync(c->status, &st, 4, hipMemcpyHostToDevice, s));
        c->hash_cap *= 4;
        continue;
      }
      if (st & ST_HASH_OVERFLOW) return set_err(c, EIPC_ERR_CAPACITY, "reduced Hessian hash overflow");
      EIPC_TRY(bsr_compact(c, sc->n_node, h, hess_bsr, s));
      eipc_status st2 = read_status(c, s);
      if (st2 != EIPC_OK && st2 != EIPC_WARN_CCD_CAPPED) return st2;
    }
    break;
  }
  return EIPC_OK;
}

eipc_status eipc_narrow_phase(eipc_ctx *c, const eipc_scene *sc, const double *q, const int32_t *pt, int64_t n_pt,
                              const int32_t *ee, int64_t n_ee, double dhat, int32_t *act_pt, int32_t *type_pt,
                              int64_t *n_act_pt, int32_t *act_ee, int32_t *type_ee, int64_t *n_act_ee,
                              eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (n_pt < 0 || n_ee < 0 || (n_pt > 0 && (!pt || !act_pt || !type_pt)) || (n_ee > 0 && (!ee || !act_ee || !type_ee)) ||
      !n_act_pt || !n_act_ee)
    return set_err(c, EIPC_ERR_ARG, "bad narrow-phase arguments");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  double *xs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)PSTRIDE * sc->n_vert + 1, &xs));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  EIPC_TRY(launch_zero(c, c->counters + 2, 2 * sizeof(int64_t), s));
  EIPC_TRY(launch_narrow(c, sc, 0, xs, pt, n_pt, dhat, act_pt, type_pt, c->counters + 2, s));
  EIPC_TRY(launch_narrow(c, sc, 1, xs, ee, n_ee, dhat, act_ee, type_ee, c->counters + 3, s));
  int64_t cnt[2];
  EIPC_HIP(c, hipMemcpyAsync(cnt, c->counters + 2, 16, hipMemcpyDeviceToHost, s));
  EIPC_HIP(c, hipStreamSynchronize(s));
  *n_act_pt = cnt[0];
  *n_act_ee = cnt[1];
  eipc_status st = read_status(c, s);
  return st == EIPC_WARN_CCD_CAPPED ? EIPC_OK : st;
}

eipc_status eipc_pair_eval(eipc_ctx *c, const eipc_scene *sc, const double *q, int32_t kind, const int32_t *pairs,
                           int64_t n, double dhat, double kappa, uint32_t flags, int32_t *type, double *sq, double *e,
                           double *g, double *H, eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if ((kind != 0 && kind != 1) || n < 0 || (n > 0 && !pairs)) return set_err(c, EIPC_ERR_ARG, "bad pair arguments");
  EIPC_TRY(check_mollify(c, sc, flags));
  if (flags & EIPC_PROJECT_REDUCED)
    return set_err(c, EIPC_ERR_ARG, "EIPC_PROJECT_REDUCED projects reduced blocks: not for per-pair outputs");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  double *xs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)PSTRIDE * sc->n_vert + 1, &xs));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  return launch_pair_eval(c, sc, kind, xs, pairs, n, dhat, kappa, flags, type, sq, e, g, H, s);
}

eipc_status eipc_ccd_candidates(eipc_ctx *c, const eipc_scene *sc, const double *q, const double *dq,
                                const double *dx_off, double dhat, int32_t *pt, int64_t cap_pt, int32_t *ee,
                                int64_t cap_ee, int64_t *n_pt, int64_t *n_ee, eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (!n_pt || !n_ee || (sc->n_node > 0 && (!q || !dq))) return set_err(c, EIPC_ERR_ARG, "bad CCD arguments");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  const int64_t n3 = (int64_t)PSTRIDE * sc->n_vert;
  double *xs, *ps, *x1s;
  EIPC_TRY(ensure_t(c, B_X, (size_t)n3 + 1, &xs));
  EIPC_TRY(ensure_t(c, B_P, (size_t)n3 + 1, &ps));
  EIPC_TRY(ensure_t(c, B_X1, (size_t)n3 + 1, &x1s));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  EIPC_TRY(launch_embed(c, sc, dq, dx_off, ps, nullptr, s));
  EIPC_TRY(launch_add_soa(c, n3, xs, ps, x1s, s));
  eipc_status s1 = broad_phase(c, sc, 0, xs, x1s, dhat, pt, cap_pt, n_pt, 1, s);
  if ((s1 != EIPC_OK && s1 != EIPC_ERR_CAPACITY) || c->scratch_short) return s1;
  eipc_status s2 = broad_phase(c, sc, 1, xs, x1s, dhat, ee, cap_ee, n_ee, 1, s);
  if ((s2 != EIPC_OK && s2 != EIPC_ERR_CAPACITY) || c->scratch_short) return s2;
  EIPC_HIP(c, hipStreamSynchronize(s));
  if (s1 == EIPC_ERR_CAPACITY || s2 == EIPC_ERR_CAPACITY)
    return set_err(c, EIPC_ERR_CAPACITY, "swept candidates need %lld PT / %lld EE slots", (long long)*n_pt,
                   (long long)*n_ee);
  return EIPC_OK;
}

eipc_status eipc_ccd_toi(eipc_ctx *c, const eipc_scene *sc, const double *q, const double *dq, const double *dx_off,
                         int32_t kind, const int32_t *pairs, int64_t n, double sfac, double t_max, int64_t max_iter,
                         double *t, int64_t *iters, eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  if ((kind != 0 && kind != 1) || n < 0 || (n > 0 && (!pairs || !t)) || !(sfac > 0.0 && sfac < 1.0) ||
      !(t_max > 0.0) || max_iter < 1)
    return set_err(c, EIPC_ERR_ARG, "bad CCD arguments");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  const int64_t n3 = (int64_t)PSTRIDE * sc->n_vert;
  double *xs, *ps;
  EIPC_TRY(ensure_t(c, B_X, (size_t)n3 + 1, &xs));
  EIPC_TRY(ensure_t(c, B_P, (size_t)n3 + 1, &ps));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  EIPC_TRY(launch_embed(c, sc, dq, dx_off, ps, nullptr, s));
  return launch_ccd(c, sc, kind, xs, ps, pairs, n, sfac, t_max, max_iter, nullptr, t, iters, s);
}

eipc_status eipc_fp64_selftest(eipc_ctx *c, const double *a, const double *b, double *sq, double *dv, int64_t n,
                               eipc_stream stream) {
  if (!c || n < 0 || (n > 0 && (!a || !b || !sq || !dv))) return EIPC_ERR_ARG;
  EIPC_HIP(c, hipSetDevice(c->device));
  return launch_fp64_selftest(c, a, b, sq, dv, n, (hipStream_t)stream);
}


eipc_status eipc_set_tuning(eipc_ctx *c, double cell_scale, const int32_t wg_per_cu[4], int32_t query_cells) {
  if (!c) return EIPC_ERR_ARG;
  if (query_cells < -1 || query_cells > 15)
    return set_err(c, EIPC_ERR_ARG, "query_cells must be -1 or mode_pt + 4 * mode_ee with modes in [0, 3]");
  if (!(cell_scale > 0.0) || !std::isfinite(cell_scale)) return set_err(c, EIPC_ERR_ARG, "cell_scale must be > 0");
  if (wg_per_cu)
    for (int k = 0; k < 4; ++k)
      if (wg_per_cu[k] < 0 || wg_per_cu[k] > 64) return set_err(c, EIPC_ERR_ARG, "wg_per_cu must be in [0, 64]");
  c->cell_scale = cell_scale;
  if (wg_per_cu)
    for (int k = 0; k < 4; ++k)
      if (wg_per_cu[k] > 0) c->wg_per_cu[k] = wg_per_cu[k];
  if (query_cells >= 0) {
    c->query_mode[0] = query_cells & 3;
    c->query_mode[1] = query_cells >> 2;
  }
  return EIPC_OK;
}

eipc_status eipc_set_ccd_method(eipc_ctx *c, int32_t method) {
  if (!c) return EIPC_ERR_ARG;
  if (method != EIPC_CCD_ADDITIVE && method != EIPC_CCD_CLOSEST_DIRECTION)
    return set_err(c, EIPC_ERR_ARG, "method must be EIPC_CCD_ADDITIVE or EIPC_CCD_CLOSEST_DIRECTION");
  c->ccd_method = method;
  return EIPC_OK;
}

}  // extern "C"

namespace eipc {

__global__ void k_step_counts(const int64_t *cn, int64_t *out) {
  if (threadIdx.x == 0) {
    out[0] = cn[5];
    out[1] = cn[6];
    out[2] = cn[2] + cn[3];
    out[3] = cn[7];
    out[4] = cn[8];
  }
}

// out[k] = pairs[act[k]] (two int32 per pair)
__global__ void k_gather_pairs(const int32_t *pairs, const int32_t *act, int64_t n, int32_t *out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = act[i];
    out[2 * i] = pairs[2 * k];
    out[2 * i + 1] = pairs[2 * k + 1];
  }
}

static eipc_status check_plan(eipc_ctx *c, const eipc_plan *p) {
  if (!p) return set_err(c, EIPC_ERR_ARG, "plan is NULL");
  if (p->cand_pt < 0 || p->cand_ee < 0 || p->swept_pt < 0 || p->swept_ee < 0 || p->act_pt < 0 || p->act_ee < 0 ||
      p->hess_blocks < 0 || p->nnzb < 0)
    return set_err(c, EIPC_ERR_ARG, "negative plan capacity");
  for (int k = 0; k < 4; ++k) {
    const int64_t b = p->buckets[k];
    if (b < 1 || (b & (b - 1)) || b > (1ll << 31) || p->ent[k] < 1 || p->qent[k] < 1)
      return set_err(c, EIPC_ERR_ARG, "plan buckets must be powers of 2 and entries >= 1");
  }
  if (p->hess_blocks & (p->hess_blocks - 1)) return set_err(c, EIPC_ERR_ARG, "plan hess_blocks must be a power of 2");
  // the block table holds the upper blocks (at most nnzb); at most half full
  if (p->hess_blocks > 0 && p->hess_blocks < 2 * p->nnzb)
    return set_err(c, EIPC_ERR_ARG, "plan hess_blocks must be at least 2 * nnzb");
  return EIPC_OK;
}

}  // namespace eipc

extern "C" {

eipc_status eipc_contact_step(eipc_ctx *c, const eipc_scene *sc, const eipc_plan *plan, const double *q,
                              const double *dq, const double *dx_off, double dhat, double kappa, uint32_t flags,
                              double sfac, double t_max, int64_t max_iter, double *energy, double *grad_q,
                              eipc_bsr *hess_bsr, double *alpha, int64_t *counts, eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  EIPC_TRY(check_plan(c, plan));
  if ((!q && sc->n_node > 0) || !std::isfinite(kappa)) return set_err(c, EIPC_ERR_ARG, "bad step arguments");
  if (alpha && ((!dq && sc->n_node > 0) || !(sfac > 0.0 && sfac < 1.0) || !(t_max > 0.0) || !std::isfinite(t_max) ||
                max_iter < 1))
    return set_err(c, EIPC_ERR_ARG, "bad step-bound arguments");
  EIPC_TRY(check_mollify(c, sc, flags));
  const bool want_h = (flags & EIPC_HESS) && hess_bsr;
  if (want_h && (plan->hess_blocks == 0 || 3 * (int64_t)sc->n_node >= (int64_t)INT32_MAX))
    return set_err(c, EIPC_ERR_ARG, "the plan has no Hessian capacity");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  const int64_t n3v = (int64_t)PSTRIDE * sc->n_vert;
  int64_t *cn = c->counters;  // [2,3] active, [5,6] candidates, [7,8] swept candidates
  const BPPlan bp[4] = {{(uint32_t)plan->buckets[0], plan->ent[0], plan->cand_pt, plan->qent[0]},
                        {(uint32_t)plan->buckets[1], plan->ent[1], plan->cand_ee, plan->qent[1]},
                        {(uint32_t)plan->buckets[2], plan->ent[2], plan->swept_pt, plan->qent[2]},
                        {(uint32_t)plan->buckets[3], plan->ent[3], plan->swept_ee, plan->qent[3]}};
  double *xs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)n3v + 1, &xs));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  EIPC_TRY(launch_zero(c, cn + 2, 7 * sizeof(int64_t), s));
  int32_t *act_pt, *typ_pt, *act_ee, *typ_ee;
  EIPC_TRY(ensure_t(c, B_ACT_PT, (size_t)std::max<int64_t>(plan->act_pt, 1), &act_pt));
  EIPC_TRY(ensure_t(c, B_TYP_PT, (size_t)std::max<int64_t>(plan->act_pt, 1), &typ_pt));
  EIPC_TRY(ensure_t(c, B_ACT_EE, (size_t)std::max<int64_t>(plan->act_ee, 1), &act_ee));
  EIPC_TRY(ensure_t(c, B_TYP_EE, (size_t)std::max<int64_t>(plan->act_ee, 1), &typ_ee));
  // barrier targets, cleared before any pair is added
  const int64_t n3 = 3 * (int64_t)sc->n_node;
  if (energy) EIPC_TRY(launch_zero(c, energy, sizeof(double) * n_scene_of(sc), s));
  double *g = (flags & EIPC_GRAD) ? grad_q : nullptr;
  if (g) EIPC_TRY(launch_zero(c, g, sizeof(double) * n3, s));
  HessOut h{0, nullptr, nullptr, nullptr, 0};
  if (want_h) EIPC_TRY(hess_table(c, plan->hess_blocks, h, s));
  const uint32_t f = flags & (want_h ? ~0u : ~(uint32_t)EIPC_HESS);
  const bool barrier = energy || g || want_h;
  if (alpha) {
    // one swept broad phase per kind; candidates at q filtered from it pair
    // by pair in the same sweep as the step bound's first pass.  The PT
    // chain runs on the side stream beside the EE chain (both on the
    // caller's stream, PT first, when kernels are timed one at a time);
    // they share only targets that are accumulated atomically (energy,
    // gradient, Hessian table, step bounds, status).
    double *ps, *x1s;
    int32_t *cpt, *cee;
    EIPC_TRY(ensure_t(c, B_P, (size_t)n3v + 1, &ps));
    EIPC_TRY(ensure_t(c, B_X1, (size_t)n3v + 1, &x1s));
    EIPC_TRY(launch_embed(c, sc, dq, dx_off, ps, nullptr, s));
    EIPC_TRY(launch_add_soa(c, n3v, xs, ps, x1s, s));
    EIPC_TRY(ensure_t(c, B_CAND_PT, (size_t)2 * std::max<int64_t>(plan->swept_pt, 1), &cpt));
    EIPC_TRY(ensure_t(c, B_CAND_EE, (size_t)2 * std::max<int64_t>(plan->swept_ee, 1), &cee));
    uint64_t tb;
    std::memcpy(&tb, &t_max, 8);
    EIPC_TRY(fill_u64(c, (uint64_t *)alpha, n_scene_of(sc), tb, s));
    EIPC_HIP(c, hipEventRecord(c->fork_ev, s));
    EIPC_HIP(c, hipStreamWaitEvent(c->side, c->fork_ev, 0));
    auto chains = [&]() -> eipc_status {
      for (int kind = 0; kind < 2; ++kind) {
        hipStream_t st = kind == 0 && !c->prof_serial ? c->side : s;
        int32_t *cand = kind == 0 ? cpt : cee;
        int32_t *act = kind == 0 ? act_pt : act_ee, *typ = kind == 0 ? typ_pt : typ_ee;
        const int64_t swept_cap = kind == 0 ? plan->swept_pt : plan->swept_ee;
        const int64_t act_cap = kind == 0 ? plan->act_pt : plan->act_ee;
        EIPC_TRY(broad_phase(c, sc, kind, xs, x1s, dhat, cand, swept_cap, nullptr, 0, st, -1, nullptr,
                             &bp[2 + kind], cn + 7 + kind));
        EIPC_TRY(launch_narrow_ccd(c, sc, kind, xs, ps, cand, swept_cap, cn + 7 + kind, dhat, act, typ, act_cap,
                                   cn + 2 + kind, cn + 5 + kind, sfac, t_max, max_iter, (uint64_t *)alpha, st));
        EIPC_TRY(launch_ccd_long(c, sc, kind, xs, ps, cand, swept_cap, cn + 7 + kind, sfac, t_max, max_iter,
                                 (uint64_t *)alpha, st));
        if (barrier)
          EIPC_TRY(launch_barrier(c, sc, kind, xs, cand, act, typ, cn + 2 + kind, act_cap, dhat, kappa, f, energy,
                                  g, h, st));
      }
      return EIPC_OK;
    };
    c->step_pairs[0] = cpt;
    c->step_pairs[1] = cee;
    c->step_pair_ctr[0] = 7;
    c->step_pair_ctr[1] = 8;
    c->step_pair_cap[0] = plan->swept_pt;
    c->step_pair_cap[1] = plan->swept_ee;
    const eipc_status cst = chains();
    // joined also when a chain failed part-way, so that nothing it enqueued
    // on the side stream can overlap the caller's next use of the scratch
    EIPC_HIP(c, hipEventRecord(c->join_ev, c->side));
    EIPC_HIP(c, hipStreamWaitEvent(s, c->join_ev, 0));
    if (cst != EIPC_OK) return cst;
  } else {
    int32_t *ppt, *pee;
    EIPC_TRY(ensure_t(c, B_STEP_PT, (size_t)2 * std::max<int64_t>(plan->cand_pt, 1), &ppt));
    EIPC_TRY(ensure_t(c, B_STEP_EE, (size_t)2 * std::max<int64_t>(plan->cand_ee, 1), &pee));
    c->step_pairs[0] = ppt;
    c->step_pairs[1] = pee;
    c->step_pair_ctr[0] = 5;
    c->step_pair_ctr[1] = 6;
    c->step_pair_cap[0] = plan->cand_pt;
    c->step_pair_cap[1] = plan->cand_ee;
    EIPC_TRY(broad_phase(c, sc, 0, xs, nullptr, dhat, ppt, plan->cand_pt, nullptr, 0, s, -1, nullptr, &bp[0], cn + 5));
    EIPC_TRY(broad_phase(c, sc, 1, xs, nullptr, dhat, pee, plan->cand_ee, nullptr, 0, s, -1, nullptr, &bp[1], cn + 6));
    EIPC_TRY(launch_narrow(c, sc, 0, xs, ppt, plan->cand_pt, dhat, act_pt, typ_pt, cn + 2, s, cn + 5, plan->act_pt));
    EIPC_TRY(launch_narrow(c, sc, 1, xs, pee, plan->cand_ee, dhat, act_ee, typ_ee, cn + 3, s, cn + 6, plan->act_ee));
    if (barrier) {
      EIPC_TRY(launch_barrier(c, sc, 0, xs, ppt, act_pt, typ_pt, cn + 2, plan->act_pt, dhat, kappa, f, energy, g, h,
                              s));
      EIPC_TRY(launch_barrier(c, sc, 1, xs, pee, act_ee, typ_ee, cn + 3, plan->act_ee, dhat, kappa, f, energy, g, h,
                              s));
    }
  }
  if (want_h) EIPC_TRY(bsr_compact(c, sc->n_node, h, hess_bsr, s, plan->nnzb));
  for (int kind = 0; kind < 2; ++kind) {
    c->step_act[kind] = kind == 0 ? act_pt : act_ee;
    c->step_act_cap[kind] = kind == 0 ? plan->act_pt : plan->act_ee;
  }
  if (counts) {
    k_step_counts<<<1, 64, 0, s>>>(cn, counts);
    EIPC_HIP(c, hipGetLastError());
  }
  return EIPC_OK;
}

eipc_status eipc_step_pairs(eipc_ctx *c, int32_t which, int32_t *out, int64_t cap, int64_t *n,
                            eipc_stream stream) {
  if (!c) return EIPC_ERR_ARG;
  if (which < 0 || which > 3 || !n || cap < 0 || (cap > 0 && !out))
    return set_err(c, EIPC_ERR_ARG, "bad step_pairs arguments");
  const int kind = which & 1;
  if (!c->step_pairs[kind]) return set_err(c, EIPC_ERR_ARG, "no planned step has run on this context");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  int64_t cnt[9];
  EIPC_HIP(c, hipMemcpyAsync(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  EIPC_HIP(c, hipStreamSynchronize(s));
  const bool active = which >= 2;
  const int64_t total = active ? std::min(cnt[2 + kind], c->step_act_cap[kind])
                               : std::min(cnt[c->step_pair_ctr[kind]], c->step_pair_cap[kind]);
  *n = total;
  if (total > cap) return set_err(c, EIPC_ERR_CAPACITY, "the list has %lld pairs", (long long)total);
  if (total == 0) return EIPC_OK;
  if (active) {
    k_gather_pairs<<<std::min(grid_for(total, 256), 4096), 256, 0, s>>>(c->step_pairs[kind], c->step_act[kind],
                                                                       total, out);
    EIPC_HIP(c, hipGetLastError());
  } else {
    EIPC_HIP(c, hipMemcpyAsync(out, c->step_pairs[kind], sizeof(int32_t) * 2 * (size_t)total,
                               hipMemcpyDeviceToDevice, s));
  }
  EIPC_HIP(c, hipStreamSynchronize(s));
  return EIPC_OK;
}

eipc_status eipc_plan_step(eipc_ctx *c, const eipc_scene *sc, const double *q, const double *dq,
                           const double *dx_off, double dhat, double margin, int32_t with_hess, eipc_plan *plan,
                           eipc_stream stream) {
  CallScope call(c);
  EIPC_TRY(check_scene(c, sc));
  EIPC_TRY(check_dhat(c, dhat));
  if (!plan || (!q && sc->n_node > 0) || !(margin >= 1.0) || !std::isfinite(margin))
    return set_err(c, EIPC_ERR_ARG, "bad plan arguments");
  hipStream_t s = (hipStream_t)stream;
  EIPC_HIP(c, hipSetDevice(c->device));
  const int64_t n3v = (int64_t)PSTRIDE * sc->n_vert;
  auto grow = [margin](int64_t v) { return (int64_t)std::ceil(margin * (double)v) + 1024; };
  eipc_plan p{};
  // measure: unplanned broad phases (append mode, buffers grown to fit)
  double *xs;
  EIPC_TRY(ensure_t(c, B_X, (size_t)n3v + 1, &xs));
  EIPC_TRY(launch_embed(c, sc, q, sc->x_off, xs, nullptr, s));
  int64_t npt = 0, nee = 0;
  int32_t *pt = nullptr, *ee = nullptr;
  EIPC_TRY(broad_phase(c, sc, 0, xs, nullptr, dhat, nullptr, 0, &npt, 0, s, B_STEP_PT, &pt));
  EIPC_TRY(broad_phase(c, sc, 1, xs, nullptr, dhat, nullptr, 0, &nee, 0, s, B_STEP_EE, &ee));
  p.cand_pt = grow(npt);
  p.cand_ee = grow(nee);
  for (int k = 0; k < 2; ++k) {
    p.ent[k] = grow(c->last_plan[k].ent_cap);
    p.qent[k] = grow(c->last_plan[k].qent_cap);
  }
  {
    eipc_bsr tmp;
    int64_t n_act = 0;
    const bool h = with_hess && sc->n_node > 0;
    EIPC_TRY(eipc_barrier_reduce(c, sc, q, pt, npt, ee, nee, dhat, 1.0, h ? EIPC_HESS : 0, nullptr, nullptr, nullptr,
                                 h ? &tmp : nullptr, &n_act, stream));
    int64_t na[2];
    EIPC_HIP(c, hipMemcpy(na, c->counters + 2, 16, hipMemcpyDeviceToHost));
    p.act_pt = grow(na[0]);
    p.act_ee = grow(na[1]);
    if (h) {
      // keys (upper blocks) <= nnzb; table at most half full
      p.nnzb = grow(tmp.nnzb);
      p.hess_blocks = pow2_at_least(2 * p.nnzb);
    }
  }
  if (dq) {
    double *ps, *x1s;
    EIPC_TRY(ensure_t(c, B_P, (size_t)n3v + 1, &ps));
    EIPC_TRY(ensure_t(c, B_X1, (size_t)n3v + 1, &x1s));
    EIPC_TRY(launch_embed(c, sc, dq, dx_off, ps, nullptr, s));
    EIPC_TRY(launch_add_soa(c, n3v, xs, ps, x1s, s));
    int64_t spt = 0, see = 0;
    int32_t *cpt = nullptr, *cee = nullptr;
    EIPC_TRY(broad_phase(c, sc, 0, xs, x1s, dhat, nullptr, 0, &spt, 0, s, B_CAND_PT, &cpt));
    EIPC_TRY(broad_phase(c, sc, 1, xs, x1s, dhat, nullptr, 0, &see, 0, s, B_CAND_EE, &cee));
    p.swept_pt = grow(spt);
    p.swept_ee = grow(see);
    for (int k = 2; k < 4; ++k) {
      p.ent[k] = grow(c->last_plan[k].ent_cap);
      p.qent[k] = grow(c->last_plan[k].qent_cap);
    }
  } else {
    p.ent[2] = p.ent[3] = 1;
    p.qent[2] = p.qent[3] = 1;
  }
  for (int k = 0; k < 4; ++k) p.buckets[k] = hash_buckets(p.ent[k]);
  {
    const eipc_status st0 = read_status(c, s);
    if (st0 != EIPC_OK && st0 != EIPC_WARN_CCD_CAPPED) return st0;
  }
  // reserve: planned steps at these sizes (with and without the step
  // bound) perform every allocation
  double *e1, *g1, *a1;
  int64_t *cnt;
  const int nsc = n_scene_of(sc);
  EIPC_TRY(ensure_t(c, B_PLAN_OUT, (size_t)(3 * sc->n_node + 2 * nsc + 8), &e1));
  g1 = e1 + nsc;
  a1 = g1 + 3 * (int64_t)sc->n_node;
  cnt = (int64_t *)(a1 + nsc);
  eipc_bsr hb;
  const uint32_t fl = EIPC_ENERGY | EIPC_GRAD | (p.hess_blocks ? (EIPC_HESS | EIPC_PROJECT) : 0);
  EIPC_TRY(eipc_contact_step(c, sc, &p, q, dq, dx_off, dhat, 1.0, fl, 0.5, 1.0, 1, e1, g1,
                             p.hess_blocks ? &hb : nullptr, nullptr, cnt, stream));
  if (dq)
    EIPC_TRY(eipc_contact_step(c, sc, &p, q, dq, dx_off, dhat, 1.0, fl, 0.5, 1.0, 1, e1, g1,
                               p.hess_blocks ? &hb : nullptr, a1, cnt, stream));
  eipc_status st = read_status(c, s);
  if (st != EIPC_OK && st != EIPC_WARN_CCD_CAPPED) return st;
  // scratch replaced while measuring is no longer used by any stream
  EIPC_HIP(c, hipStreamSynchronize(c->side));
  free_retired(c);
  *plan = p;
  return EIPC_OK;
}

}  // extern "C"
