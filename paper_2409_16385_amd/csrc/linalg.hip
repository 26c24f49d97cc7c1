// Dense FP64 Cholesky factorization and solves for the reduced Newton system
// of one implicit step (used by the adjoint of a converged step).
//
// A is row-major with leading dimension lda; only its lower triangle is read
// and the factor L (A = L L^T) overwrites it.  Blocked right-looking
// algorithm on 64x64 tiles: factor the diagonal tile in LDS, solve the panel
// below it against L_kk^T, update the trailing lower tiles with L_ik L_jk^T.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace eipc {

constexpr int NB = 64;
constexpr int NBP = NB + 1;  // LDS row padding

__device__ __forceinline__ double ld_a(const double *A, int64_t lda, int64_t n, int64_t r, int64_t c) {
  return (r < n && c < n) ? A[r * lda + c] : (r == c ? 1.0 : 0.0);
}

__global__ __launch_bounds__(256) void k_chol_diag(double *A, int64_t n, int64_t lda, int64_t k0, int64_t *info) {
  __shared__ double s[NB][NBP];
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    s[r][c] = ld_a(A, lda, n, k0 + r, k0 + c);
  }
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    if (t == 0) {
      const double d = s[j][j];
      if (!(d > 0.0) || !isfinite(d)) {
        if (k0 + j < n) atomicCAS((unsigned long long *)info, 0ull, (unsigned long long)(k0 + j + 1));
        s[j][j] = 1.0;  // keep going with finite values; info reports the failure
      } else {
        s[j][j] = sqrt(d);
      }
    }
    __syncthreads();
    const double djj = s[j][j];
    for (int i = j + 1 + t; i < NB; i += 256) s[i][j] /= djj;
    __syncthreads();
    const int m = NB - j - 1;
    for (int e = t; e < m * m; e += 256) {
      const int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) s[i][l] -= s[i][j] * s[l][j];
    }
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    if (c <= r && k0 + r < n && k0 + c < n) A[(k0 + r) * lda + k0 + c] = s[r][c];
  }
}

// row blocks below the diagonal: X L_kk^T = A_ik  (one thread per row)
__global__ __launch_bounds__(NB) void k_chol_panel(double *A, int64_t n, int64_t lda, int64_t k0) {
  __shared__ double L[NB][NBP];
  __shared__ double X[NB][NBP];
  const int t = threadIdx.x;
  const int64_t r0 = k0 + NB * (1 + (int64_t)blockIdx.x);
  for (int e = t; e < NB * NB; e += NB) {
    const int r = e / NB, c = e % NB;
    L[r][c] = ld_a(A, lda, n, k0 + r, k0 + c);
    X[r][c] = (r0 + r < n && k0 + c < n) ? A[(r0 + r) * lda + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    double acc = X[t][j];
    for (int l = 0; l < j; ++l) acc -= X[t][l] * L[j][l];
    X[t][j] = acc / L[j][j];
  }
  __syncthreads();
  for (int e = t; e < NB * NB; e += NB) {
    const int r = e / NB, c = e % NB;
    if (r0 + r < n && k0 + c < n) A[(r0 + r) * lda + k0 + c] = X[r][c];
  }
}

// trailing update of lower tiles (i, j), k < j <= i:  A_ij -= L_ik L_jk^T
__global__ __launch_bounds__(256) void k_chol_update(double *A, int64_t n, int64_t lda, int64_t k0, int nt_rem) {
  __shared__ double Li[NB][NBP];
  __shared__ double Lj[NB][NBP];
  // linear block index -> (i, j) with j <= i over the remaining tiles
  const int64_t b = blockIdx.x;
  int i = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= b) ++i;
  while ((int64_t)i * (i + 1) / 2 > b) --i;
  const int j = (int)(b - (int64_t)i * (i + 1) / 2);
  if (i >= nt_rem) return;
  const int64_t ri = k0 + NB * (1 + (int64_t)i), rj = k0 + NB * (1 + (int64_t)j);
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e % NB;
    Li[r][c] = (ri + r < n && k0 + c < n) ? A[(ri + r) * lda + k0 + c] : 0.0;
    Lj[r][c] = (rj + r < n && k0 + c < n) ? A[(rj + r) * lda + k0 + c] : 0.0;
  }
  __syncthreads();
  const int tr = t / 16, tc = t % 16;  // 4x4 outputs per thread
  double acc[4][4] = {};
  for (int l = 0; l < NB; ++l) {
    double a[4], bb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = Li[4 * tr + u][l];
      bb[u] = Lj[4 * tc + u][l];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * bb[v];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = ri + 4 * tr + u, cc = rj + 4 * tc + v;
      if (r < n && cc < n && cc <= r) A[r * lda + cc] -= acc[u][v];
    }
}

// forward substitution L y = b for one block row of 64 unknowns, one
// workgroup per right-hand side: partial sums over the solved prefix, then
// the 64x64 triangular solve.
__global__ __launch_bounds__(256) void k_trsv_lower(const double *L, int64_t n, int64_t lda, double *B, int64_t nrhs,
                                                   int64_t r0) {
  __shared__ double part[256];
  __shared__ double y[NB];
  const int t = threadIdx.x;
  const int64_t rhs = blockIdx.x;
  const int rows = (int)std::min<int64_t>(NB, n - r0);
  // part[t]: thread t sums over columns c = t, t + 256, ... < r0 for row (t / 4)?  Use 4 threads per row.
  const int row = t / 4, lane4 = t % 4;
  double acc = 0.0;
  if (row < rows) {
    const double *Lr = L + (r0 + row) * lda;
    for (int64_t c = lane4; c < r0; c += 4) acc += Lr[c] * B[c * nrhs + rhs];
  }
  part[t] = acc;
  __syncthreads();
  if (t < NB) {
    y[t] = (t < rows) ? B[(r0 + t) * nrhs + rhs] - (part[4 * t] + part[4 * t + 1] + part[4 * t + 2] + part[4 * t + 3])
                      : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    for (int i = 0; i < rows; ++i) {
      double s = y[i];
      const double *Lr = L + (r0 + i) * lda + r0;
      for (int c = 0; c < i; ++c) s -= Lr[c] * y[c];
      y[i] = s / Lr[i];
    }
  }
  __syncthreads();
  if (t < rows) B[(r0 + t) * nrhs + rhs] = y[t];
}

// backward substitution L^T x = y for one block row (rows r0..r0+63),
// using the already solved x below it.
__global__ __launch_bounds__(256) void k_trsv_upper(const double *L, int64_t n, int64_t lda, double *B, int64_t nrhs,
                                                   int64_t r0) {
  __shared__ double part[256];
  __shared__ double y[NB];
  const int t = threadIdx.x;
  const int64_t rhs = blockIdx.x;
  const int rows = (int)std::min<int64_t>(NB, n - r0);
  const int row = t / 4, lane4 = t % 4;
  double acc = 0.0;
  if (row < rows) {
    // (L^T x)_row = sum_{c > row} L[c][row] x_c over c >= r0 + NB
    for (int64_t c = r0 + NB + lane4; c < n; c += 4) acc += L[c * lda + r0 + row] * B[c * nrhs + rhs];
  }
  part[t] = acc;
  __syncthreads();
  if (t < NB) {
    y[t] = (t < rows) ? B[(r0 + t) * nrhs + rhs] - (part[4 * t] + part[4 * t + 1] + part[4 * t + 2] + part[4 * t + 3])
                      : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    for (int i = rows - 1; i >= 0; --i) {
      double s = y[i];
      for (int c = i + 1; c < rows; ++c) s -= L[(r0 + c) * lda + r0 + i] * y[c];
      y[i] = s / L[(r0 + i) * lda + r0 + i];
    }
  }
  __syncthreads();
  if (t < rows) B[(r0 + t) * nrhs + rhs] = y[t];
}

}  // namespace eipc

using namespace eipc;

extern "C" {

eipc_status eipc_cholesky(eipc_ctx *c, double *A, int64_t n, int64_t lda, int64_t *info, eipc_stream stream) {
  if (!c || n < 0 || lda < n || (n > 0 && !A) || !info) return c ? set_err(c, EIPC_ERR_ARG, "bad Cholesky arguments")
                                                                  : EIPC_ERR_ARG;
  EIPC_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  int64_t *d_info = c->counters + 12;
  EIPC_TRY(launch_zero(c, d_info, 8, s));
  const int64_t nt = (n + NB - 1) / NB;
  for (int64_t k = 0; k < nt; ++k) {
    const int64_t k0 = k * NB;
    k_chol_diag<<<1, 256, 0, s>>>(A, n, lda, k0, d_info);
    EIPC_HIP(c, hipGetLastError());
    const int64_t rem = nt - k - 1;
    if (rem > 0) {
      k_chol_panel<<<(unsigned)rem, NB, 0, s>>>(A, n, lda, k0);
      EIPC_HIP(c, hipGetLastError());
      const int64_t nblk = rem * (rem + 1) / 2;
      k_chol_update<<<(unsigned)nblk, 256, 0, s>>>(A, n, lda, k0, (int)rem);
      EIPC_HIP(c, hipGetLastError());
    }
  }
  EIPC_HIP(c, hipMemcpyAsync(info, d_info, 8, hipMemcpyDeviceToHost, s));
  EIPC_HIP(c, hipStreamSynchronize(s));
  return EIPC_OK;
}

eipc_status eipc_cholesky_solve(eipc_ctx *c, const double *L, int64_t n, int64_t lda, double *B, int64_t nrhs,
                                eipc_stream stream) {
  if (!c || n < 0 || lda < n || nrhs < 1 || (n > 0 && (!L || !B)))
    return c ? set_err(c, EIPC_ERR_ARG, "bad solve arguments") : EIPC_ERR_ARG;
  EIPC_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t nt = (n + NB - 1) / NB;
  for (int64_t k = 0; k < nt; ++k) {
    k_trsv_lower<<<(unsigned)nrhs, 256, 0, s>>>(L, n, lda, B, nrhs, k * NB);
    EIPC_HIP(c, hipGetLastError());
  }
  for (int64_t k = nt - 1; k >= 0; --k) {
    k_trsv_upper<<<(unsigned)nrhs, 256, 0, s>>>(L, n, lda, B, nrhs, k * NB);
    EIPC_HIP(c, hipGetLastError());
  }
  return EIPC_OK;
}

}  // extern "C"
