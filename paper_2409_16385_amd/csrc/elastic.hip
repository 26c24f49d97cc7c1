// Elastic and inertial terms of the reduced Newton system of one implicit
// step on the coarse tetrahedral mesh: the reduced mass M = J^T M_x J from
// interior samples of the body (Eq. 1, with the volume aggregation of
// Eq. 15), gravity f = J^T f_ext (Eq. 16), and the elastic energy Phi of
// the coarse tetrahedra (Sec. III-A) in the paper's linear corotational
// model (Sec. IV-A) or its small-strain linearization, with gradient and
// Newton matrix.  The coarse nodes are the reduced coordinates q (three per
// node), so these terms act on q directly; dense outputs are row-major
// [3 n_node x 3 n_node] with a leading dimension, as the Cholesky kernels
// take them.
#include <cmath>

#include "common.h"

namespace eipc {

constexpr int EL_T = 256;

// 3x3 row-major inverse by cofactors; returns the determinant
__device__ __forceinline__ double inv3(const double *m, double *r) {
  const double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8], c02 = m[3] * m[7] - m[4] * m[6];
  const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
  const double id = 1.0 / det;
  r[0] = c00 * id;
  r[1] = (m[2] * m[7] - m[1] * m[8]) * id;
  r[2] = (m[1] * m[5] - m[2] * m[4]) * id;
  r[3] = c01 * id;
  r[4] = (m[0] * m[8] - m[2] * m[6]) * id;
  r[5] = (m[2] * m[3] - m[0] * m[5]) * id;
  r[6] = c02 * id;
  r[7] = (m[1] * m[6] - m[0] * m[7]) * id;
  r[8] = (m[0] * m[4] - m[1] * m[3]) * id;
  return det;
}

// Rotation R of the polar decomposition F = R S (det F > 0) by Newton's
// iteration X <- (X + X^-T) / 2 from X = F, which converges quadratically
// to R; stopped when a step changes X by less than 1e-15 of its size
// (then one more step), at most 60 steps.
__device__ __forceinline__ void polar_rotation(const double *F, double *R) {
  double X[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) X[k] = F[k];
  bool last = false;
  for (int it = 0; it < 60; ++it) {
    double Xi[9];
    inv3(X, Xi);
    double d2 = 0.0, n2 = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double y = 0.5 * (X[3 * r + c] + Xi[3 * c + r]);
        const double dd = y - X[3 * r + c];
        d2 += dd * dd;
        n2 += y * y;
        X[3 * r + c] = y;
      }
    if (last) break;
    if (d2 <= 1e-30 * n2) last = true;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = X[k];
}

// One thread per tet.  MODEL 0: small-strain linear elasticity,
// psi = mu eps:eps + lam/2 tr(eps)^2 with eps = sym(F) - I, P = 2 mu eps +
// lam tr(eps) I, Hessian the constant stiffness K0.  MODEL 1: linear
// corotational, psi = mu |F - R|^2 + lam/2 tr(R^T F - I)^2 with R the polar
// rotation of F, P = 2 mu (F - R) + lam tr(R^T F - I) R, Newton matrix the
// warped stiffness R K0 R^T.  K0's (a, b) block is V (mu (g_b g_a^T +
// (g_a.g_b) I) + lam g_a g_b^T) for the rest shape-function gradients g_a.
template <int MODEL>
__global__ __launch_bounds__(EL_T) void k_elastic(int n_tet, const int32_t *__restrict__ tets,
                                                  const double *__restrict__ rest, const double *__restrict__ vol,
                                                  double mu, double lam, const double *__restrict__ q, double scale,
                                                  double *energy, double *grad, double *hess, int64_t lda,
                                                  uint32_t *status) {
  __shared__ double s_e[EL_T / 64];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (t < n_tet && vol[t] > 0.0) {
    const double V = vol[t];
    int nd[4];
    double X[4][3], x[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      nd[a] = tets[4 * (int64_t)t + a];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        X[a][c] = rest[3 * (int64_t)nd[a] + c];
        x[a][c] = q[3 * (int64_t)nd[a] + c];
      }
    }
    double Dm[9], Di[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) Dm[3 * r + c] = X[c + 1][r] - X[0][r];
    const double det = inv3(Dm, Di);
    bool ok = det != 0.0 && isfinite(det);
    // rest shape-function gradients: g_k = row k-1 of Dm^-1, g_0 = -(g_1 + g_2 + g_3)
    double g[4][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g[1][c] = Di[c];
      g[2][c] = Di[3 + c];
      g[3][c] = Di[6 + c];
      g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    }
    double F[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) F[3 * i + j] = x[0][i] * g[0][j] + x[1][i] * g[1][j] + x[2][i] * g[2][j] + x[3][i] * g[3][j];
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double P[9], psi = 0.0;
    if (MODEL == 0) {
      double eps[9], tr = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) eps[3 * i + j] = 0.5 * (F[3 * i + j] + F[3 * j + i]) - (i == j ? 1.0 : 0.0);
      tr = eps[0] + eps[4] + eps[8];
      double ee = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) ee += eps[k] * eps[k];
      psi = mu * ee + 0.5 * lam * tr * tr;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P[3 * i + j] = 2.0 * mu * eps[3 * i + j] + (i == j ? lam * tr : 0.0);
    } else {
      const double detF = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                          F[2] * (F[3] * F[7] - F[4] * F[6]);
      ok = ok && detF > 0.0 && isfinite(detF);
      if (ok) polar_rotation(F, R);
      double tr = -3.0, dd = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        tr += R[k] * F[k];  // tr(R^T F)
        dd += (F[k] - R[k]) * (F[k] - R[k]);
      }
      psi = mu * dd + 0.5 * lam * tr * tr;
#pragma unroll
      for (int k = 0; k < 9; ++k) P[k] = 2.0 * mu * (F[k] - R[k]) + lam * tr * R[k];
    }
    if (!ok) {
      atomicOr(status, ST_DEGENERATE);
    } else {
      e = scale * V * psi;
      if (grad) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int i = 0; i < 3; ++i)
            atomicAdd(&grad[3 * (int64_t)nd[a] + i],
                      scale * V * (P[3 * i] * g[a][0] + P[3 * i + 1] * g[a][1] + P[3 * i + 2] * g[a][2]));
      }
      if (hess) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const double gab = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
            double blk[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j)
                blk[3 * i + j] = V * (mu * (g[b][i] * g[a][j] + (i == j ? gab : 0.0)) + lam * g[a][i] * g[b][j]);
            if (MODEL == 1) {
              double tmp[9];
#pragma unroll
              for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                  tmp[3 * i + j] = R[3 * i] * blk[j] + R[3 * i + 1] * blk[3 + j] + R[3 * i + 2] * blk[6 + j];
#pragma unroll
              for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                  blk[3 * i + j] = tmp[3 * i] * R[3 * j] + tmp[3 * i + 1] * R[3 * j + 1] + tmp[3 * i + 2] * R[3 * j + 2];
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j)
                atomicAdd(&hess[(3 * (int64_t)nd[a] + i) * lda + 3 * (int64_t)nd[b] + j], scale * blk[3 * i + j]);
          }
      }
    }
  }
  if (energy) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if (lane == 0) s_e[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < EL_T / 64; ++w) s += s_e[w];
      if (s != 0.0) atomicAdd(energy, s);
    }
  }
}

// Sample s (mass m, weights w in its coarse tet's nodes) adds m w_a w_b to
// the diagonal of the 3x3 block (a, b) of M and -m g w_a to node a's z
// component of f.
__global__ __launch_bounds__(EL_T) void k_sample_mass(int64_t n_s, const int32_t *__restrict__ snodes,
                                                      const double *__restrict__ sw, double m, double gravity,
                                                      double *M, int64_t lda, double *f) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_s) return;
  int nd[4];
  double w[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    nd[a] = snodes[4 * s + a];
    w[a] = sw[4 * s + a];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double v = m * w[a] * w[b];
#pragma unroll
      for (int i = 0; i < 3; ++i) atomicAdd(&M[(3 * (int64_t)nd[a] + i) * lda + 3 * (int64_t)nd[b] + i], v);
    }
    if (f) atomicAdd(&f[3 * (int64_t)nd[a] + 2], -m * gravity * w[a]);
  }
}

// Nodes that no sample reaches (zero mass) get 1e-3 of the mean mass of the
// reached nodes on their diagonal.  One workgroup.
__global__ __launch_bounds__(EL_T) void k_mass_fill(int n_node, double *M, int64_t lda) {
  __shared__ double s_sum[EL_T];
  __shared__ int s_cnt[EL_T];
  double sum = 0.0;
  int cnt = 0;
  for (int a = threadIdx.x; a < n_node; a += EL_T) {
    const double d = M[(3 * (int64_t)a) * lda + 3 * (int64_t)a];
    if (d > 0.0) {
      sum += d;
      ++cnt;
    }
  }
  s_sum[threadIdx.x] = sum;
  s_cnt[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = EL_T / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (s_cnt[0] == 0 || s_cnt[0] == n_node) return;
  const double fill = 1e-3 * (s_sum[0] / (double)s_cnt[0]);
  for (int a = threadIdx.x; a < n_node; a += EL_T) {
    const int64_t k = 3 * (int64_t)a;
    if (!(M[k * lda + k] > 0.0)) {
#pragma unroll
      for (int i = 0; i < 3; ++i) M[(k + i) * lda + k + i] = fill;
    }
  }
}

}  // namespace eipc

using namespace eipc;

extern "C" {

eipc_status eipc_reduced_mass(eipc_ctx *c, int32_t n_node, int64_t n_sample, const int32_t *sample_nodes,
                              const double *sample_w, double sample_mass, double gravity, double *M, int64_t lda,
                              double *f, eipc_stream stream) {
  if (!c) return EIPC_ERR_ARG;
  CallScope call(c);
  if (n_node < 0 || n_sample < 0 || lda < 3 * (int64_t)n_node || (n_node > 0 && !M) ||
      (n_sample > 0 && (!sample_nodes || !sample_w)) || !std::isfinite(sample_mass) || !std::isfinite(gravity))
    return set_err(c, EIPC_ERR_ARG, "bad reduced-mass arguments");
  if (n_node == 0) return EIPC_OK;
  EIPC_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  if (n_sample > 0) {
    k_sample_mass<<<(unsigned)((n_sample + EL_T - 1) / EL_T), EL_T, 0, s>>>(n_sample, sample_nodes, sample_w,
                                                                           sample_mass, gravity, M, lda, f);
    EIPC_HIP(c, hipGetLastError());
  }
  k_mass_fill<<<1, EL_T, 0, s>>>(n_node, M, lda);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

eipc_status eipc_elastic(eipc_ctx *c, int32_t n_node, int32_t n_tet, const int32_t *tets, const double *rest,
                         const double *vol, double young, double poisson, int32_t model, const double *q,
                         double scale, double *energy, double *grad, double *hess, int64_t lda,
                         eipc_stream stream) {
  if (!c) return EIPC_ERR_ARG;
  CallScope call(c);
  if (n_node < 0 || n_tet < 0 || (model != EIPC_ELASTIC_LINEAR && model != EIPC_ELASTIC_COROTATIONAL) ||
      (n_tet > 0 && (!tets || !rest || !vol || !q)) || (hess && lda < 3 * (int64_t)n_node) || !(young > 0.0) ||
      !(poisson > -1.0 && poisson < 0.5) || !std::isfinite(scale))
    return set_err(c, EIPC_ERR_ARG, "bad elastic-term arguments");
  if (n_tet == 0) return EIPC_OK;
  EIPC_HIP(c, hipSetDevice(c->device));
  const double lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson));
  const double mu = young / (2.0 * (1.0 + poisson));
  hipStream_t s = (hipStream_t)stream;
  const unsigned blocks = (unsigned)((n_tet + EL_T - 1) / EL_T);
  if (model == EIPC_ELASTIC_LINEAR)
    k_elastic<0><<<blocks, EL_T, 0, s>>>(n_tet, tets, rest, vol, mu, lam, q, scale, energy, grad, hess, lda,
                                         c->status);
  else
    k_elastic<1><<<blocks, EL_T, 0, s>>>(n_tet, tets, rest, vol, mu, lam, q, scale, energy, grad, hess, lda,
                                         c->status);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

}  // extern "C"
