// Lagged friction of Sec. III-B: D_k(x, x^n) = mu lambda_k^n f0(|u_k|), its
// reduced gradient and (positive semidefinite by construction) reduced
// Hessian through the embedding (Eq. 17).
//
// Per pair, at the lagged positions x^n: the distance type, lambda =
// kappa |b'(d^n)| (times the mollifier for EE pairs with EIPC_MOLLIFY), the
// signed closest-point weights beta over the four vertices (relative
// position G x = sum_a beta_a x_a: the point minus the closest triangle
// point for PT, the closest point of edge a minus that of edge b for EE),
// the contact normal n = G x^n / |G x^n| and G x^n itself.  At x: the
// tangential displacement u = P (G x - G x^n) with P = I - n n^T, y = |u|,
//   D = mu lambda f0(y),  g_a = beta_a mu lambda (f1(y)/y) u,
//   H_ab = beta_a beta_b mu lambda (f1(y)/y P + (f1'(y) y - f1(y))/y^3 u u^T),
// where f1(y) = 2 y/(eps h) - y^2/(eps h)^2 below eps h and 1 above, f0 its
// integral from eps h plus eps h.  In the translation-free basis Q of the
// barrier kernels (columns 0.5 S[a][alpha] over the four vertices) the
// gradient is gamma_alpha = b_alpha v and the Hessian X[alpha][beta] =
// b_alpha b_beta K with b_alpha = 0.5 sum_a S[a][alpha] beta_a, so the
// barrier's expansion kernel reduces it through W unchanged.
#include <algorithm>

#include "common.h"
#include "pair_math.h"

namespace eipc {

constexpr int FR_T = 256;

template <int KIND>
__device__ __forceinline__ void pair_vid(const int32_t *pairs, int64_t k, const int32_t *faces, const int32_t *edges,
                                         int *vid) {
  const int a = pairs[2 * k], b = pairs[2 * k + 1];
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
}

template <int KIND>
__global__ __launch_bounds__(FR_T) void k_friction_lag(int64_t n, const int32_t *__restrict__ pairs,
                                                       const int32_t *__restrict__ faces,
                                                       const int32_t *__restrict__ edges, const double *__restrict__ xs,
                                                       const double *__restrict__ x_rest, double dhat, double kappa,
                                                       bool moll, bool sq, double *__restrict__ lag,
                                                       uint32_t *status) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    int vid[4];
    pair_vid<KIND>(pairs, k, faces, edges, vid);
    V3 x[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) ld_pos(xs, vid[a], x[a].x, x[a].y, x[a].z);
    int type;
    const double s2 = pair_dist2<KIND>(x, &type);
    double rec[EIPC_FRICTION_LAG];
#pragma unroll
    for (int i = 0; i < EIPC_FRICTION_LAG; ++i) rec[i] = 0.0;
    if (!isfinite(s2)) {
      atomicOr(status, ST_NONFINITE);
    } else if (s2 < dhat * dhat) {
      if (!(s2 > 0.0)) {
        atomicOr(status, ST_INTERSECTING);
      } else {
        const double d = sqrt(s2);
        // db/dd; of the squared-distance barrier 2 d db/ds
        const double b1 = sq ? 2.0 * d * barrier_s(s2, dhat, true).bs1
                             : -2.0 * (d - dhat) * log(d / dhat) - (d - dhat) * (d - dhat) / d;
        double m = 1.0;
        if (KIND == 1 && moll) {
          V3 r[4];
#pragma unroll
          for (int a = 0; a < 4; ++a)
            r[a] = V3{x_rest[3 * (int64_t)vid[a]], x_rest[3 * (int64_t)vid[a] + 1], x_rest[3 * (int64_t)vid[a] + 2]};
          const double eps = mollifier_eps(r);
          const V3 cr = xcross(xsub(x[1], x[0]), xsub(x[3], x[2]));
          const double c = xdot(cr, cr);
          if (c < eps) m = (2.0 - c / eps) * (c / eps);
        }
        double beta[4];
        closest_beta<KIND>(type, x, beta);
        V3 g{0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          g.x += beta[a] * x[a].x;
          g.y += beta[a] * x[a].y;
          g.z += beta[a] * x[a].z;
        }
        const double gn = sqrt(xdot(g, g));
        rec[0] = kappa * m * fabs(b1);
#pragma unroll
        for (int a = 0; a < 4; ++a) rec[1 + a] = beta[a];
        rec[5] = g.x / gn;
        rec[6] = g.y / gn;
        rec[7] = g.z / gn;
        rec[8] = g.x;
        rec[9] = g.y;
        rec[10] = g.z;
      }
    }
#pragma unroll
    for (int i = 0; i < EIPC_FRICTION_LAG; ++i) lag[EIPC_FRICTION_LAG * k + i] = rec[i];
  }
}

// friction gradient and Hessian of each listed pair in the Q basis (the
// layout the expansion kernel reads), its vertex ids, energy summed
template <int KIND>
__global__ __launch_bounds__(FR_T) void k_friction_terms(
    int64_t n, const int32_t *__restrict__ pairs, const int32_t *__restrict__ faces, const int32_t *__restrict__ edges,
    const double *__restrict__ xs, const double *__restrict__ lag, double mu, double epsvh, double *energy,
    double *__restrict__ rec, bool want_g, bool want_h, int4 *__restrict__ vid4, uint32_t *status) {
  __shared__ double s_e[FR_T / 64];
  double e_acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * FR_T; base < n; base += (int64_t)gridDim.x * FR_T) {
    const int64_t i = base + threadIdx.x;
    if (i < n) {
      int vid[4];
      pair_vid<KIND>(pairs, i, faces, edges, vid);
      vid4[i] = make_int4(vid[0], vid[1], vid[2], vid[3]);
      double L[EIPC_FRICTION_LAG];
#pragma unroll
      for (int t = 0; t < EIPC_FRICTION_LAG; ++t) L[t] = lag[EIPC_FRICTION_LAG * i + t];
      const double ml = mu * L[0];
      double g3[3] = {0.0, 0.0, 0.0}, K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, b[3] = {0.0, 0.0, 0.0};
      if (ml != 0.0) {
        V3 w{-L[8], -L[9], -L[10]};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          V3 xa;
          ld_pos(xs, vid[a], xa.x, xa.y, xa.z);
          w.x += L[1 + a] * xa.x;
          w.y += L[1 + a] * xa.y;
          w.z += L[1 + a] * xa.z;
        }
        const double nn[3] = {L[5], L[6], L[7]};
        const double wn = w.x * nn[0] + w.y * nn[1] + w.z * nn[2];
        const double u[3] = {w.x - wn * nn[0], w.y - wn * nn[1], w.z - wn * nn[2]};
        const double y = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double f0, s1, s2;
        if (y < epsvh) {
          f0 = -(y * y * y) / (3.0 * epsvh * epsvh) + (y * y) / epsvh + epsvh / 3.0;
          s1 = 2.0 / epsvh - y / (epsvh * epsvh);              // f1(y)/y
          s2 = y > 0.0 ? -1.0 / (epsvh * epsvh * y) : 0.0;     // (f1' y - f1)/y^3
        } else {
          f0 = y;
          s1 = 1.0 / y;
          s2 = -1.0 / (y * y * y);
        }
        e_acc += ml * f0;
#pragma unroll
        for (int c = 0; c < 3; ++c) g3[c] = ml * s1 * u[c];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) K[3 * r + c] = ml * (s1 * ((r == c ? 1.0 : 0.0) - nn[r] * nn[c]) + s2 * u[r] * u[c]);
#pragma unroll
        for (int al = 0; al < 3; ++al)
          b[al] = 0.5 * (kS[0][al] * L[1] + kS[1][al] * L[2] + kS[2][al] * L[3] + kS[3][al] * L[4]);
      }
      double *rp = rec + (int64_t)TERM_REC * i;
      if (want_g) {
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int c = 0; c < 3; ++c) rp[3 * al + c] = b[al] * g3[c];
      }
      if (want_h) {
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int be = al; be < 3; ++be)
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                if (al == be && c < r) continue;
                rp[9 + pidx(3 * al + r, 3 * be + c)] = b[al] * b[be] * K[3 * r + c];
              }
      }
      if (!isfinite(e_acc)) atomicOr(status, ST_NONFINITE);
    }
  }
  if (energy) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e_acc += __shfl_xor(e_acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_e[threadIdx.x >> 6] = e_acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < FR_T / 64; ++w) t += s_e[w];
      if (t != 0.0) atomicAdd(energy, t);
    }
  }
}

__global__ void k_set_count(int64_t *p, int64_t v) {
  if (threadIdx.x == 0) *p = v;
}

eipc_status launch_friction_lag(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                                int64_t n, double dhat, double kappa, uint32_t flags, double *lag, hipStream_t s) {
  if (n == 0) return EIPC_OK;
  const int blocks = (int)std::min<int64_t>(grid_for(n, FR_T), 8 * (int64_t)c->num_cu);
  const bool moll = (flags & EIPC_MOLLIFY) && sc->x_rest;
  const bool sq = flags & EIPC_SQDIST;
  if (kind == 0)
    k_friction_lag<0><<<blocks, FR_T, 0, s>>>(n, pairs, sc->faces, sc->edges, xs, sc->x_rest, dhat, kappa, moll, sq,
                                              lag, c->status);
  else
    k_friction_lag<1><<<blocks, FR_T, 0, s>>>(n, pairs, sc->faces, sc->edges, xs, sc->x_rest, dhat, kappa, moll, sq,
                                              lag, c->status);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

eipc_status launch_friction(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                            int64_t n, const double *lag, double mu, double epsvh, double *energy, double *grad,
                            const HessOut &h, hipStream_t s) {
  if (n == 0) return EIPC_OK;
  const bool want_g = grad != nullptr, want_h = h.kind != 0;
  double *rec = nullptr;
  int4 *vid4;
  if (want_g || want_h) EIPC_TRY(ensure_t(c, kind == 0 ? B_PX_PT : B_PX_EE, (size_t)TERM_REC * n, &rec));
  EIPC_TRY(ensure_t(c, kind == 0 ? B_SVID : B_SVID_EE, (size_t)n, &vid4));
  const int blocks = (int)std::min<int64_t>(grid_for(n, FR_T), 8 * (int64_t)c->num_cu);
  if (kind == 0)
    k_friction_terms<0><<<blocks, FR_T, 0, s>>>(n, pairs, sc->faces, sc->edges, xs, lag, mu, epsvh, energy, rec,
                                                want_g, want_h, vid4, c->status);
  else
    k_friction_terms<1><<<blocks, FR_T, 0, s>>>(n, pairs, sc->faces, sc->edges, xs, lag, mu, epsvh, energy, rec,
                                                want_g, want_h, vid4, c->status);
  EIPC_HIP(c, hipGetLastError());
  if (!want_g && !want_h) return EIPC_OK;
  int64_t *cnt = c->counters + 12 + kind;
  k_set_count<<<1, 64, 0, s>>>(cnt, n);
  EIPC_HIP(c, hipGetLastError());
  return launch_expand(c, sc, kind, vid4, cnt, n, rec, want_g, want_h, grad, h, s);
}

}  // namespace eipc
