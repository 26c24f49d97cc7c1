// Conservative CCD step bound: additive conservative advancement per swept
// candidate pair, minimum over pairs by wavefront reduction and one atomic.
#include <algorithm>

#include "common.h"
#include "pair_math.h"

namespace eipc {

// Min of a per-lane value into bits[scene] (all lanes of the wavefront
// call): one atomic per wavefront when the contributing lanes share a scene.
// Values are >= 0, so their IEEE bit patterns order like the values.
__device__ __forceinline__ void agg_scene_min(unsigned long long *bits, bool valid, int scene, int n_scene, double t,
                                              uint32_t *status) {
  const bool ok = valid && (unsigned)scene < (unsigned)n_scene;
  if (valid && !ok) atomicOr(status, ST_BAD_SCENE);
  const uint64_t vm = __ballot(ok);
  if (vm == 0) return;
  const int first = __ffsll((unsigned long long)vm) - 1;
  const int s0 = __shfl(scene, first, 64);
  if (__ballot(ok && scene != s0) == 0) {
    double m = ok ? t : INFINITY;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
    // the bound only decreases: skip the atomic when a plain read already
    // holds a value no larger (a stale read only lets an atomic through)
    const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
    if ((int)(threadIdx.x & 63) == first && mb < ((volatile unsigned long long *)bits)[s0]) atomicMin(&bits[s0], mb);
  } else if (ok) {
    const unsigned long long tb = (unsigned long long)__double_as_longlong(t);
    if (tb < ((volatile unsigned long long *)bits)[scene]) atomicMin(&bits[scene], tb);
  }
}

// Cut-off for a pair of the given scene when only the per-scene minimum is
// wanted: the scene's bound as published so far.  It starts at t_max and
// only ever takes some pair's final bound, so a pair whose bound is shown
// to be no smaller cannot lower the minimum.  A stale read returns an
// earlier, larger value: a weaker cut-off, never a wrong one.  With no
// step allowed (max_iter < 1) every bound is 0 and nothing is cut.
__device__ __forceinline__ double scene_cut(const unsigned long long *bits, int scene, int n_scene, double t_max,
                                            int64_t max_iter) {
  if (max_iter < 1 || (unsigned)scene >= (unsigned)n_scene) return INFINITY;
  return fmin(__longlong_as_double((long long)((const volatile unsigned long long *)bits)[scene]), t_max);
}

// Advancement of one pair after accd_init_cut, up to lim steps, dropping
// the pair as soon as its bound reaches cut (it only grows from there).
// Returns ACCD_OPEN when lim steps left it undecided.
template <int KIND>
__device__ __forceinline__ int accd_run_cut(V3 *x, const V3 *p, double t_c, int64_t max_iter, double cut,
                                            int64_t lim, AccdState &st, int r) {
  while (r == ACCD_OPEN && st.it < lim) {
    if (accd_step<KIND>(x, p, t_c, max_iter, st))
      r = ACCD_DONE;
    else if (st.t >= cut)
      r = ACCD_DROP;
  }
  if (r == ACCD_OPEN && st.it >= max_iter) {  // cap reached: the bound so far
    accd_step<KIND>(x, p, t_c, max_iter, st);
    r = ACCD_DONE;
  }
  return r;
}

template <int KIND>
__global__ __launch_bounds__(256) void k_ccd(int64_t cap, const int64_t *d_n, const int32_t *__restrict__ pairs,
                      const int32_t *__restrict__ faces, const int32_t *__restrict__ edges,
                      const double *__restrict__ xs, const double *__restrict__ ps, int n_vert, double sfac,
                      double t_max, int64_t max_iter, unsigned long long *alpha_bits, double *t_out, int64_t *it_out,
                      const int32_t *__restrict__ vscene, int n_scene, uint32_t *status, bool dir) {
  const int64_t n = d_n ? (*d_n < cap ? *d_n : cap) : cap;
  bool capped = false;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const bool live = i < n;
    double t = t_max;
    int scene = 0;
    if (live) {
      const int a = pairs[2 * i], b = pairs[2 * i + 1];
      int vid[4];
      if (KIND == 0) {
        vid[0] = a;
        vid[1] = faces[3 * (int64_t)b];
        vid[2] = faces[3 * (int64_t)b + 1];
        vid[3] = faces[3 * (int64_t)b + 2];
      } else {
        vid[0] = edges[2 * (int64_t)a];
        vid[1] = edges[2 * (int64_t)a + 1];
        vid[2] = edges[2 * (int64_t)b];
        vid[3] = edges[2 * (int64_t)b + 1];
      }
      if (vscene) scene = vscene[vid[0]];
      V3 x[4], p[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ld_pos(xs, vid[k], x[k].x, x[k].y, x[k].z);
        ld_pos(ps, vid[k], p[k].x, p[k].y, p[k].z);
      }
      int64_t it = 0;
      t = accd<KIND>(x, p, sfac, t_max, max_iter, &it, dir);
      capped = capped || it >= max_iter;
      if (t_out) t_out[i] = t;
      if (it_out) it_out[i] = it;
    }
    if (alpha_bits) agg_scene_min(alpha_bits, live, scene, n_scene, t, status);
  }
  if (__any(capped) && (threadIdx.x & 63) == 0) atomicOr(status, ST_CCD_CAPPED);
}

// Step bound only (no per-pair output), in two passes so that the few
// pairs needing many advancement steps do not hold up whole wavefronts:
// pass 0 gives every pair up to CCD_SHORT steps and defers the pairs still
// undecided to a compacted list; pass 1 runs those from the start with
// the full iteration cap.  Each pair's bound is computed exactly as in
// one uninterrupted run, or the pair is dropped once its bound is shown to
// be no smaller than its scene's bound published so far (scene_cut): the
// minimum comes out the same, bit for bit.
constexpr int64_t CCD_SHORT = 4;

template <int KIND, int PASS>
__global__ __launch_bounds__(256) void k_ccd2(int64_t cap, const int64_t *d_n, const int32_t *__restrict__ pairs,
                       const int32_t *__restrict__ faces, const int32_t *__restrict__ edges,
                       const double *__restrict__ xs, const double *__restrict__ ps, int n_vert, double sfac,
                       double t_max, int64_t max_iter, unsigned long long *alpha_bits, int32_t *__restrict__ longl,
                       int64_t *n_long, const int32_t *__restrict__ vscene, int n_scene, uint32_t *status,
                       bool dir) {
  const int64_t n = PASS == 0 ? (d_n ? (*d_n < cap ? *d_n : cap) : cap) : (*n_long < cap ? *n_long : cap);
  const int lane = threadIdx.x & 63;
  bool capped = false;
  // each workgroup walks a contiguous range of the list: a scene's pairs
  // are adjacent in it, so the first pairs of a range publish their
  // scene's bound early and the cut-off prunes the rest of the range
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + blockDim.x - 1) / blockDim.x * blockDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  for (int64_t base = r0; base < r1; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const bool live = i < r1;
    double t = t_max;
    int scene = 0;
    bool decided = false, deferred = false;
    if (live) {
      const int64_t k = PASS == 0 ? i : (int64_t)longl[i];
      const int a = pairs[2 * k], b = pairs[2 * k + 1];
      int vid[4];
      if (KIND == 0) {
        vid[0] = a;
        vid[1] = faces[3 * (int64_t)b];
        vid[2] = faces[3 * (int64_t)b + 1];
        vid[3] = faces[3 * (int64_t)b + 2];
      } else {
        vid[0] = edges[2 * (int64_t)a];
        vid[1] = edges[2 * (int64_t)a + 1];
        vid[2] = edges[2 * (int64_t)b];
        vid[3] = edges[2 * (int64_t)b + 1];
      }
      if (vscene) scene = vscene[vid[0]];
      V3 x[4], p[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ld_pos(xs, vid[q], x[q].x, x[q].y, x[q].z);
        ld_pos(ps, vid[q], p[q].x, p[q].y, p[q].z);
      }
      AccdState st;
      st.dir = dir;
      const double cut = scene_cut(alpha_bits, scene, n_scene, t_max, max_iter);
      const int64_t lim = PASS == 0 ? (CCD_SHORT < max_iter ? CCD_SHORT : max_iter) : max_iter;
      const int r = accd_run_cut<KIND>(x, p, t_max, max_iter, cut, lim, st,
                                       accd_init_cut<KIND>(x, p, sfac, t_max, cut, st, false, 0.0));
      if (r == ACCD_DONE) {
        t = st.t;
        capped = st.it >= max_iter;
      }
      decided = r != ACCD_OPEN;  // a dropped pair keeps t = t_max
      deferred = !decided;       // pass 0 only: more than CCD_SHORT steps
    }
    if (PASS == 0) {
      const uint64_t dm = __ballot(deferred);
      if (dm) {
        int64_t p0 = 0;
        if (lane == __ffsll((unsigned long long)dm) - 1)
          p0 = (int64_t)atomicAdd((unsigned long long *)n_long, (unsigned long long)__popcll(dm));
        p0 = __shfl(p0, __ffsll((unsigned long long)dm) - 1, 64);
        if (deferred) longl[p0 + __popcll(dm & ((1ull << lane) - 1ull))] = (int32_t)i;
      }
    }
    agg_scene_min(alpha_bits, live && decided, scene, n_scene, t, status);
  }
  if (__any(capped) && lane == 0) atomicOr(status, ST_CCD_CAPPED);
}

// Narrow phase and step-bound pass 0 in one sweep over the swept
// candidates (the planned step with a step bound): each pair's vertices are
// loaded once; the candidate predicate at x and, for the pairs passing it,
// the distance and activity test (active pairs staged per workgroup and
// appended to act/typ with one atomic per flush) come first, then
// advancement as in k_ccd2 pass 0,
// reusing the distance just computed.  The pass-1 list is the same.
// The PT form is held to three waves per SIMD (168 VGPRs, no spill); the EE
// form runs at two, where its 189 VGPRs fit without spilling (at three it
// spilled 68 bytes per lane and was 8 % slower).
constexpr int NCCD_BUF = 1024;  // staged active pairs per workgroup

template <int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KIND == 0 ? 3 : 2))) void k_narrow_ccd(
    int64_t cap, const int64_t *d_n, const int32_t *__restrict__ pairs, const int32_t *__restrict__ faces,
    const int32_t *__restrict__ edges, const double *__restrict__ xs, const double *__restrict__ ps, double dhat2,
    double h, int32_t *__restrict__ act, int32_t *__restrict__ typ, int64_t act_cap, int64_t *count,
    int64_t *cand_count, double sfac, double t_max, int64_t max_iter, unsigned long long *alpha_bits,
    int32_t *__restrict__ longl, int64_t *n_long, const int32_t *__restrict__ vscene, int n_scene,
    uint32_t *status, bool dir) {
  // active pairs are staged in LDS and appended with one atomic per
  // workgroup flush: one atomic per wavefront on the shared counter
  // serialised at the memory side (about a third of a pass's time)
  __shared__ int2 s_act[NCCD_BUF];
  __shared__ int s_nact;
  __shared__ int64_t s_abase;
  const int64_t n = *d_n < cap ? *d_n : cap;
  const int lane = threadIdx.x & 63;
  bool capped = false;
  int64_t n_cand = 0;
  if (threadIdx.x == 0) s_nact = 0;
  __syncthreads();
  // each workgroup walks a contiguous range of the list: a scene's pairs
  // are adjacent in it, so the first pairs of a range publish their
  // scene's bound early and the cut-off prunes the rest of the range
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + blockDim.x - 1) / blockDim.x * blockDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  for (int64_t base = r0; base < r1; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const bool live = i < r1;
    double t = t_max;
    int scene = 0, ty = 0;
    bool decided = false, deferred = false, active = false;
    if (live) {
      const int a = pairs[2 * i], b = pairs[2 * i + 1];
      int vid[4];
      if (KIND == 0) {
        vid[0] = a;
        vid[1] = faces[3 * (int64_t)b];
        vid[2] = faces[3 * (int64_t)b + 1];
        vid[3] = faces[3 * (int64_t)b + 2];
      } else {
        vid[0] = edges[2 * (int64_t)a];
        vid[1] = edges[2 * (int64_t)a + 1];
        vid[2] = edges[2 * (int64_t)b];
        vid[3] = edges[2 * (int64_t)b + 1];
      }
      if (vscene) scene = vscene[vid[0]];
      V3 x[4], p[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ld_pos(xs, vid[q], x[q].x, x[q].y, x[q].z);
        ld_pos(ps, vid[q], p[q].x, p[q].y, p[q].z);
      }
      double s2 = 0.0;
      const bool cand = static_boxes_overlap<KIND>(x, h);
      if (cand) {
        ++n_cand;
        s2 = pair_dist2<KIND>(x, &ty);
        if (!isfinite(s2)) {
          atomicOr(status, ST_NONFINITE);
        } else if (s2 < dhat2) {
          if (s2 <= 0.0)
            atomicOr(status, ST_INTERSECTING);
          else
            active = true;
        }
      }
      AccdState st;
      st.dir = dir;
      const double cut = scene_cut(alpha_bits, scene, n_scene, t_max, max_iter);
      const int64_t lim = CCD_SHORT < max_iter ? CCD_SHORT : max_iter;
      const int r = accd_run_cut<KIND>(x, p, t_max, max_iter, cut, lim, st,
                                       accd_init_cut<KIND>(x, p, sfac, t_max, cut, st, cand, s2));
      if (r == ACCD_DONE) {
        t = st.t;
        capped = st.it >= max_iter;
      }
      decided = r != ACCD_OPEN;  // a dropped pair keeps t = t_max
      deferred = !decided;
    }
    {
      const uint64_t mask = __ballot(active);
      int p0 = 0;
      if (lane == 0 && mask) p0 = atomicAdd(&s_nact, (int)__popcll(mask));
      p0 = __shfl(p0, 0, 64);
      if (active) s_act[p0 + __popcll(mask & ((1ull << lane) - 1ull))] = make_int2((int)i, ty);
      __syncthreads();
      const int na = s_nact;
      __syncthreads();  // every thread has read the count before it changes
      // flush when another round could overfill the stage, and at the end
      if (na > NCCD_BUF - (int)blockDim.x || base + (int64_t)blockDim.x >= r1) {
        if (threadIdx.x == 0) s_abase = na ? (int64_t)atomicAdd((unsigned long long *)count, (unsigned long long)na) : 0;
        __syncthreads();
        const int64_t ab = s_abase;
        for (int k = threadIdx.x; k < na; k += blockDim.x) {
          const int64_t pos = ab + k;
          if (pos < act_cap) {
            act[pos] = s_act[k].x;
            typ[pos] = s_act[k].y;
          } else {
            atomicOr(status, ST_PLAN_OVERFLOW);
          }
        }
        __syncthreads();
        if (threadIdx.x == 0) s_nact = 0;
        __syncthreads();
      }
    }
    {
      const uint64_t dm = __ballot(deferred);
      if (dm) {
        int64_t p0 = 0;
        if (lane == __ffsll((unsigned long long)dm) - 1)
          p0 = (int64_t)atomicAdd((unsigned long long *)n_long, (unsigned long long)__popcll(dm));
        p0 = __shfl(p0, __ffsll((unsigned long long)dm) - 1, 64);
        if (deferred) longl[p0 + __popcll(dm & ((1ull << lane) - 1ull))] = (int32_t)i;
      }
    }
    agg_scene_min(alpha_bits, live && decided, scene, n_scene, t, status);
  }
  if (__any(capped) && lane == 0) atomicOr(status, ST_CCD_CAPPED);
  // the candidate count: one atomic per workgroup
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n_cand += __shfl_xor(n_cand, o, 64);
  __shared__ int64_t s_cand[4];
  if (lane == 0) s_cand[threadIdx.x >> 6] = n_cand;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t tot = s_cand[0] + s_cand[1] + s_cand[2] + s_cand[3];
    if (tot) atomicAdd((unsigned long long *)cand_count, (unsigned long long)tot);
  }
}

eipc_status launch_narrow_ccd(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *ps,
                              const int32_t *pairs, int64_t n, const int64_t *d_n, double dhat, int32_t *act,
                              int32_t *typ, int64_t act_cap, int64_t *d_count, int64_t *cand_count, double sfac,
                              double t_max, int64_t max_iter, uint64_t *d_alpha_bits, hipStream_t s) {
  if (n == 0) return EIPC_OK;
  const int blocks = (int)std::min<int64_t>(grid_for(n, 256), (int64_t)c->wg_per_cu[3] * c->num_cu);
  const int32_t *vsc = vscene_of(sc);
  const int nsc = n_scene_of(sc);
  int64_t *n_long = c->counters + 9 + kind;
  int32_t *longl;
  EIPC_TRY(ensure_t(c, kind == 0 ? B_CCD_LONG_PT : B_CCD_LONG_EE, (size_t)n, &longl));
  EIPC_TRY(launch_zero(c, n_long, 8, s));
  unsigned long long *ab = (unsigned long long *)d_alpha_bits;
  const double d2 = dhat * dhat, h = 0.5 * dhat;
  {
    ProfScope prof(c, kind == 0 ? K_CCD_PT : K_CCD_EE, s);
    if (kind == 0)
      k_narrow_ccd<0><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, d2, h, act, typ,
                                             act_cap, d_count, cand_count, sfac, t_max, max_iter, ab, longl, n_long,
                                             vsc, nsc, c->status, c->ccd_method == 1);
    else
      k_narrow_ccd<1><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, d2, h, act, typ,
                                             act_cap, d_count, cand_count, sfac, t_max, max_iter, ab, longl, n_long,
                                             vsc, nsc, c->status, c->ccd_method == 1);
    EIPC_HIP(c, hipGetLastError());
  }
  return EIPC_OK;
}

eipc_status launch_ccd_long(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *ps,
                            const int32_t *pairs, int64_t n, const int64_t *d_n, double sfac, double t_max,
                            int64_t max_iter, uint64_t *d_alpha_bits, hipStream_t s) {
  if (n == 0) return EIPC_OK;
  const int blocks = (int)std::min<int64_t>(grid_for(n, 256), (int64_t)c->wg_per_cu[3] * c->num_cu);
  const int32_t *vsc = vscene_of(sc);
  const int nsc = n_scene_of(sc);
  int64_t *n_long = c->counters + 9 + kind;
  int32_t *longl;
  EIPC_TRY(ensure_t(c, kind == 0 ? B_CCD_LONG_PT : B_CCD_LONG_EE, (size_t)n, &longl));
  unsigned long long *ab = (unsigned long long *)d_alpha_bits;
  ProfScope prof(c, kind == 0 ? K_CCD_LONG_PT : K_CCD_LONG_EE, s);
  if (kind == 0)
    k_ccd2<0, 1><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, sc->n_vert, sfac, t_max,
                                        max_iter, ab, longl, n_long, vsc, nsc, c->status, c->ccd_method == 1);
  else
    k_ccd2<1, 1><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, sc->n_vert, sfac, t_max,
                                        max_iter, ab, longl, n_long, vsc, nsc, c->status, c->ccd_method == 1);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

eipc_status launch_ccd(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *ps,
                       const int32_t *pairs, int64_t n, double sfac, double t_max, int64_t max_iter,
                       uint64_t *d_alpha_bits, double *t_out, int64_t *it_out, hipStream_t s, const int64_t *d_n) {
  if (n == 0) return EIPC_OK;
  ProfScope prof(c, kind == 0 ? K_CCD_PT : K_CCD_EE, s);
  const int blocks = (int)std::min<int64_t>(grid_for(n, 256), (int64_t)c->wg_per_cu[3] * c->num_cu);
  const int32_t *vsc = vscene_of(sc);
  const int nsc = n_scene_of(sc);
  if (d_alpha_bits && !t_out && !it_out) {
    int64_t *n_long = c->counters + 9 + kind;
    int32_t *longl;
    EIPC_TRY(ensure_t(c, kind == 0 ? B_CCD_LONG_PT : B_CCD_LONG_EE, (size_t)n, &longl));
    EIPC_TRY(launch_zero(c, n_long, 8, s));
    unsigned long long *ab = (unsigned long long *)d_alpha_bits;
    if (kind == 0) {
      k_ccd2<0, 0><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, sc->n_vert, sfac, t_max,
                                          max_iter, ab, longl, n_long, vsc, nsc, c->status, c->ccd_method == 1);
      k_ccd2<0, 1><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, sc->n_vert, sfac, t_max,
                                          max_iter, ab, longl, n_long, vsc, nsc, c->status, c->ccd_method == 1);
    } else {
      k_ccd2<1, 0><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, sc->n_vert, sfac, t_max,
                                          max_iter, ab, longl, n_long, vsc, nsc, c->status, c->ccd_method == 1);
      k_ccd2<1, 1><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, sc->n_vert, sfac, t_max,
                                          max_iter, ab, longl, n_long, vsc, nsc, c->status, c->ccd_method == 1);
    }
  } else if (kind == 0)
    k_ccd<0><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, sc->n_vert, sfac, t_max, max_iter,
                                     (unsigned long long *)d_alpha_bits, t_out, it_out, vsc, nsc, c->status,
                                     c->ccd_method == 1);
  else
    k_ccd<1><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, ps, sc->n_vert, sfac, t_max, max_iter,
                                     (unsigned long long *)d_alpha_bits, t_out, it_out, vsc, nsc, c->status,
                                     c->ccd_method == 1);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

__global__ void k_fp64_selftest(int64_t n, const double *a, const double *b, double *sq, double *dv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  sq[i] = sqrt(a[i]);
  dv[i] = a[i] / b[i];
}

eipc_status launch_fp64_selftest(eipc_ctx *c, const double *a, const double *b, double *sq, double *dv, int64_t n,
                                 hipStream_t s) {
  if (n == 0) return EIPC_OK;
  k_fp64_selftest<<<grid_for(n, 256), 256, 0, s>>>(n, a, b, sq, dv);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

}  // namespace eipc
