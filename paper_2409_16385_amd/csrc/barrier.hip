// Per-pair barrier energy, gradient and (projected) Hessian, reduced through
// the embedding (Eq. 17) with LDS-staged accumulation; Hessian-vector
// products; BSR compaction of the reduced Hessian.
#include <algorithm>

#include "common.h"
#include "pair_math.h"

namespace eipc {

constexpr int BR_THREADS = 256;
constexpr int LTBL = 1024;  // LDS 3x3-block table entries (76 KiB)
constexpr int LGT = 512;    // LDS node-vector table entries (14 KiB)
constexpr int MAX_PROBE = 32;       // LDS tables (a miss falls back to the global table)
constexpr int GLOBAL_PROBE = 4096;  // global block table (at most half full; a miss is reported)

__device__ __forceinline__ uint32_t mix32(uint32_t k) {
  k ^= k >> 16;
  k *= 0x7feb352dU;
  k ^= k >> 15;
  k *= 0x846ca68bU;
  k ^= k >> 16;
  return k;
}

__device__ __forceinline__ uint32_t mix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  return (uint32_t)k;
}

// find-or-insert in an open-addressing table of 64-bit keys (-1 = empty)
__device__ __forceinline__ int64_t table_slot64(long long *keys, uint64_t mask, long long key, int max_probe) {
  uint64_t h = mix64((uint64_t)key) & mask;
  for (int p = 0; p < max_probe; ++p) {
    long long k = ((volatile long long *)keys)[h];
    if (k == key) return (int64_t)h;
    if (k == -1) {
      long long old = (long long)atomicCAS((unsigned long long *)&keys[h], (unsigned long long)-1ll,
                                           (unsigned long long)key);
      if (old == -1 || old == key) return (int64_t)h;
    }
    h = (h + 1) & mask;
  }
  return -1;
}

// find-or-insert in an open-addressing table of int keys (-1 = empty)
__device__ __forceinline__ int table_slot(int *keys, uint32_t mask, int key) {
  uint32_t h = mix32((uint32_t)key) & mask;
  for (int p = 0; p < MAX_PROBE; ++p) {
    int k = ((volatile int *)keys)[h];
    if (k == key) return (int)h;
    if (k == -1) {
      int old = atomicCAS(&keys[h], -1, key);
      if (old == -1 || old == key) return (int)h;
    }
    h = (h + 1) & mask;
  }
  return -1;
}

template <int KIND>
__device__ __forceinline__ void pair_vertices(const int32_t *pairs, int64_t k, const int32_t *faces,
                                              const int32_t *edges, int *vid) {
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

__device__ __forceinline__ V3 load3(const double *xs, int n, int v) {
  V3 r;
  ld_pos(xs, v, r.x, r.y, r.z);
  return r;
}

// global destination of a 3x3 block (I <= J)
__device__ __forceinline__ void global_block_add(const HessOut &h, int n_node, int64_t I, int64_t J,
                                                 const double *B, uint32_t *status) {
  if (h.kind == 1) {
    const int64_t n3 = 3 * (int64_t)n_node;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) atomicAdd(&h.dense[(3 * (int64_t)I + i) * n3 + 3 * J + j], B[3 * i + j]);
  } else if (h.kind == 2) {
    const int64_t slot = table_slot64((long long *)h.hkey, h.hmask, (long long)(I * n_node + J), GLOBAL_PROBE);
    if (slot < 0) {
      atomicOr(status, ST_HASH_OVERFLOW);
      return;
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) atomicAdd(&h.hval[9 * (int64_t)slot + t], B[t]);
  }
}

struct LdsTables {
  long long *bkey;
  double *bval;
  int *gkey;
  double *gval;
};

__device__ __forceinline__ void lds_vec_add(const LdsTables &T, double *grad, int I, double g0, double g1,
                                            double g2) {
  int slot = table_slot(T.gkey, LGT - 1, I);
  if (slot < 0) {
    atomicAdd(&grad[3 * (int64_t)I], g0);
    atomicAdd(&grad[3 * (int64_t)I + 1], g1);
    atomicAdd(&grad[3 * (int64_t)I + 2], g2);
    return;
  }
  atomicAdd(&T.gval[3 * slot], g0);
  atomicAdd(&T.gval[3 * slot + 1], g1);
  atomicAdd(&T.gval[3 * slot + 2], g2);
}

// ---------------------------------------------------------------------------
// Merged expansion.  The 16 (node, weight) slots of a pair (4 vertices x up
// to 4 weights) are taken to the Q basis, z_s = w_s Q[a(s)] (3 numbers),
// sorted by node with a bitonic network, equal nodes merged, and sorted
// again to compact.  Then, for distinct nodes I <= J,
//   block(I, J) = sum_{alpha, beta} z_I[alpha] z_J[beta] X[alpha][beta]
// and the gradient of node I is sum_alpha z_I[alpha] gamma_alpha with
// gamma = G^T gY.  Each block is summed across the wavefront when every
// lane holding one targets the same block, else added per lane.
// ---------------------------------------------------------------------------
constexpr int NO_NODE = 0x7fffffff;

struct NodeSet {
  int node[16];
  double z[16][3];
};

__device__ __forceinline__ void cswap(NodeSet &S, int a, int b, bool up) {
  const bool sw = up ? (S.node[a] > S.node[b]) : (S.node[a] < S.node[b]);
  const int na = S.node[a], nb = S.node[b];
  S.node[a] = sw ? nb : na;
  S.node[b] = sw ? na : nb;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double za = S.z[a][c], zb = S.z[b][c];
    S.z[a][c] = sw ? zb : za;
    S.z[b][c] = sw ? za : zb;
  }
}

__device__ __forceinline__ void sort16(NodeSet &S) {
#pragma unroll
  for (int k = 2; k <= 16; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int l = i ^ j;
        if (l > i) cswap(S, i, l, (i & k) == 0);
      }
}

// Rows hold at most 4 weights (checked when positions are embedded).
template <int KIND>
__device__ __forceinline__ bool gather_nodes(const int *vid, const int32_t *rowptr, const int32_t *col,
                                             const double *val, NodeSet &S, int &m) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int k0 = rowptr[vid[a]];
    const int cnt = rowptr[vid[a] + 1] - k0;
    ok = ok && cnt <= 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool v = k < cnt;
      const double w = v ? val[k0 + k] : 0.0;
      S.node[4 * a + k] = v ? col[k0 + k] : NO_NODE;
#pragma unroll
      for (int al = 0; al < 3; ++al) S.z[4 * a + k][al] = 0.5 * kS[a][al] * w;
    }
  }
  sort16(S);
#pragma unroll
  for (int s = 0; s < 15; ++s) {
    if (S.node[s] == S.node[s + 1] && S.node[s] != NO_NODE) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        S.z[s + 1][c] += S.z[s][c];
        S.z[s][c] = 0.0;
      }
      S.node[s] = NO_NODE;
    }
  }
  sort16(S);
  m = 0;
#pragma unroll
  for (int s = 0; s < 16; ++s) m += S.node[s] != NO_NODE;
  return ok;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct Acc {
  LdsTables T;
  HessOut h;
  int n_node;
  double *grad;
  uint32_t *status;
};

__device__ __forceinline__ void agg_vec(const Acc &A, bool valid, int node, double g0, double g1, double g2) {
  const uint64_t vm = __ballot(valid);
  if (vm == 0) return;
  const int first = __ffsll((unsigned long long)vm) - 1;
  const int k0 = __shfl(node, first, 64);
  const bool uniform = __ballot(valid && node != k0) == 0;
  if (uniform) {
    g0 = wave_sum(valid ? g0 : 0.0);
    g1 = wave_sum(valid ? g1 : 0.0);
    g2 = wave_sum(valid ? g2 : 0.0);
    if ((int)(threadIdx.x & 63) == first) lds_vec_add(A.T, A.grad, node, g0, g1, g2);
  } else if (valid) {
    lds_vec_add(A.T, A.grad, node, g0, g1, g2);
  }
}

// Add a per-lane value into out[scene] (all lanes of the wavefront call):
// one atomic per wavefront when the contributing lanes share a scene.
__device__ __forceinline__ void agg_scene_add(double *out, bool valid, int scene, int n_scene, double v,
                                              uint32_t *status) {
  const bool ok = valid && (unsigned)scene < (unsigned)n_scene;
  if (valid && !ok) atomicOr(status, ST_BAD_SCENE);
  const uint64_t vm = __ballot(ok);
  if (vm == 0) return;
  const int first = __ffsll((unsigned long long)vm) - 1;
  const int s0 = __shfl(scene, first, 64);
  if (__ballot(ok && scene != s0) == 0) {
    const double t = wave_sum(ok ? v : 0.0);
    if ((int)(threadIdx.x & 63) == first && t != 0.0) atomicAdd(&out[s0], t);
  } else if (ok && v != 0.0) {
    atomicAdd(&out[scene], v);
  }
}

// Phase 1: per active pair, energy (reduced per scene), the gradient in
// the Q basis gamma = G^T gY (9) and the Hessian X in the Q basis (45,
// PSD-projected with EIPC_PROJECT), stored SoA: out[e*cap + i].
template <int KIND>
__global__ __launch_bounds__(BR_THREADS) void k_pair_terms(
    const int32_t *__restrict__ pairs, const int32_t *__restrict__ act, const int32_t *__restrict__ typ,
    const int64_t *__restrict__ d_count, const int32_t *__restrict__ faces, const int32_t *__restrict__ edges,
    const double *__restrict__ xs, const double *__restrict__ x_rest, int n_vert, double dhat, double kappa,
    uint32_t flags, double *energy, double *__restrict__ gq, double *__restrict__ Xq, int64_t cap,
    const int32_t *__restrict__ vscene, int n_scene, uint32_t *status, const int4 *__restrict__ vid4) {
  __shared__ double s_e[BR_THREADS / 64];
  const bool want_g = gq != nullptr;
  const bool want_h = Xq != nullptr;
  const bool project = flags & EIPC_PROJECT;
  const bool moll = (KIND == 1) && (flags & EIPC_MOLLIFY) && x_rest;
  const int64_t n = *d_count < cap ? *d_count : cap;
  double e_acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * BR_THREADS; base < n; base += (int64_t)gridDim.x * BR_THREADS) {
    const int64_t i = base + threadIdx.x;
    const bool live = i < n;
    double e_pair = 0.0;
    int scene = 0;
    if (live) {
      const int ty = typ[i];
      int vid[4];
      if (vid4) {
        const int4 v4 = vid4[i];
        vid[0] = v4.x;
        vid[1] = v4.y;
        vid[2] = v4.z;
        vid[3] = v4.w;
      } else {
        pair_vertices<KIND>(pairs, act[i], faces, edges, vid);
      }
      if (vscene) scene = vscene[vid[0]];
      V3 x[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) x[a] = load3(xs, n_vert, vid[a]);
      const double s2 = type_value<KIND>(ty, x);
      double eps = 0.0;
      if (moll) {
        V3 r[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          r[a] = V3{x_rest[3 * (int64_t)vid[a]], x_rest[3 * (int64_t)vid[a] + 1], x_rest[3 * (int64_t)vid[a] + 2]};
        eps = mollifier_eps(r);
      }
      V3 Y[3];
      y_basis<KIND>(x, Y);
      double gE[9], HE[45];
      e_pair = energy_derivs<KIND>(ty, x, Y, s2, dhat, kappa, eps, gE, HE, want_h);
      if (want_g) {
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int J = 0; J < 3; ++J) {
              const int g = gcoef(KIND, J, al);
              if (g != 0) acc += g * gE[3 * J + c];
            }
            gq[(3 * al + c) * cap + i] = acc;
          }
      }
      if (want_h) {
        double M[45];
        to_q_basis<KIND>(HE, M);
        if (project) project_psd9(M);
#pragma unroll
        for (int e = 0; e < 45; ++e) Xq[e * cap + i] = M[e];
      }
    }
    if (energy && vscene) agg_scene_add(energy, live, scene, n_scene, e_pair, status);
    e_acc += e_pair;
  }
  if (energy && !vscene) {
    e_acc = wave_sum(e_acc);
    if ((threadIdx.x & 63) == 0) s_e[threadIdx.x >> 6] = e_acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < BR_THREADS / 64; ++w) t += s_e[w];
      if (t != 0.0) atomicAdd(energy, t);
    }
  }
}

// ---------------------------------------------------------------------------
// Phase 2, reduction through W of gamma and X.  Cooperative expansion: sixteen lanes per pair, lane s holding slot s =
// (vertex s / 4, weight s % 4) of the pair: its node and z_s = w_s Q[a]
// (3 numbers).  The sixteen slots are sorted by node across the lanes
// (bitonic exchange within the 16-lane group), runs of equal nodes summed
// (segmented scan; the last lane of a run keeps the node), so each node of
// the pair sits on one lane.  That lane forms Y_J = sum_beta z_J[beta]
// X[.][beta] (27 numbers) and, for every node I <= J of the group (taken
// by shuffle), the block sum_alpha z_I[alpha] Y_J[alpha], accumulated in
// the workgroup's LDS table as in the per-pair form; the node's gradient
// is sum_alpha z_J[alpha] gamma_alpha.
// ---------------------------------------------------------------------------
// threads per workgroup: 64 pairs per step.  The LDS tables allow one
// workgroup per CU, so its size sets the waves a CU runs: 1,024 threads
// (four per SIMD; the kernel is then held to 128 VGPRs and spills 68 bytes
// per lane) measured faster than 768 (three) and 512 (two)
constexpr int EX_T = 1024;

__device__ __forceinline__ int64_t table_slot64_new(long long *keys, uint64_t mask, long long key, bool &fresh) {
  uint64_t h = mix64((uint64_t)key) & mask;
  fresh = false;
  for (int p = 0; p < MAX_PROBE; ++p) {
    long long k = ((volatile long long *)keys)[h];
    if (k == key) return (int64_t)h;
    if (k == -1) {
      long long old = (long long)atomicCAS((unsigned long long *)&keys[h], (unsigned long long)-1ll,
                                           (unsigned long long)key);
      if (old == -1) {
        fresh = true;
        return (int64_t)h;
      }
      if (old == key) return (int64_t)h;
    }
    h = (h + 1) & mask;
  }
  return -1;
}

template <int KIND>
__global__ __launch_bounds__(EX_T) void k_expand16(
    const int4 *__restrict__ vid4, const int64_t *__restrict__ d_count, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const double *__restrict__ val, int n_node, const double *__restrict__ gq,
    const double *__restrict__ Xq, int64_t cap, double *grad, HessOut h, uint32_t *status) {
  __shared__ long long s_bkey[LTBL];
  __shared__ double s_bval[LTBL * 9];
  __shared__ int s_gkey[LGT];
  __shared__ double s_gval[LGT * 3];
  __shared__ int s_used;
  const bool want_g = gq != nullptr && grad != nullptr;
  const bool want_h = Xq != nullptr && h.kind != 0;
  for (int t = threadIdx.x; t < LTBL; t += EX_T) s_bkey[t] = -1;
  for (int t = threadIdx.x; t < LTBL * 9; t += EX_T) s_bval[t] = 0.0;
  for (int t = threadIdx.x; t < LGT; t += EX_T) s_gkey[t] = -1;
  for (int t = threadIdx.x; t < LGT * 3; t += EX_T) s_gval[t] = 0.0;
  if (threadIdx.x == 0) s_used = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int s = lane & 15;
  const int gbase = lane & ~15;
  constexpr int PPS = EX_T / 16;  // pairs per step
  const int64_t n = *d_count < cap ? *d_count : cap;
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + PPS - 1) / PPS * PPS;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  for (int64_t base = r0; base < r1; base += PPS) {
    const int64_t i = base + (threadIdx.x >> 4);
    const bool active = i < r1;
    // this lane's slot
    int node = NO_NODE;
    double z[3] = {0.0, 0.0, 0.0};
    if (active) {
      const int a = s >> 2, k = s & 3;
      const int4 v4 = vid4[i];
      const int v = a == 0 ? v4.x : (a == 1 ? v4.y : (a == 2 ? v4.z : v4.w));
      const int k0 = rowptr[v];
      if (k < rowptr[v + 1] - k0) {
        node = col[k0 + k];
        const double w = val[k0 + k];
#pragma unroll
        for (int al = 0; al < 3; ++al) z[al] = 0.5 * kS[a][al] * w;
      }
    }
    // sort the group's slots by node (bitonic, ascending; ties keep place)
#pragma unroll
    for (int k = 2; k <= 16; k <<= 1)
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int pn = __shfl_xor(node, j, 64);
        double pz[3];
#pragma unroll
        for (int al = 0; al < 3; ++al) pz[al] = __shfl_xor(z[al], j, 64);
        const bool up = (s & k) == 0, low = (s & j) == 0;
        const bool take = (low == up) ? (pn < node) : (pn > node);
        if (take) {
          node = pn;
#pragma unroll
          for (int al = 0; al < 3; ++al) z[al] = pz[al];
        }
      }
    // sum runs of equal nodes; the run's last lane holds the total
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const int pn = __shfl_up(node, off, 16);
      double pz[3];
#pragma unroll
      for (int al = 0; al < 3; ++al) pz[al] = __shfl_up(z[al], off, 16);
      if (s >= off && pn == node) {
#pragma unroll
        for (int al = 0; al < 3; ++al) z[al] += pz[al];
      }
    }
    const int nn = __shfl_down(node, 1, 16);
    const bool mine = node != NO_NODE && (s == 15 || nn != node);
    if (want_g) {
      double gam[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) gam[e] = active ? gq[e * cap + i] : 0.0;
      double g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = z[0] * gam[c] + z[1] * gam[3 + c] + z[2] * gam[6 + c];
      LdsTables T{s_bkey, s_bval, s_gkey, s_gval};
      Acc A{T, h, n_node, grad, status};
      agg_vec(A, mine, mine ? node : -1, g[0], g[1], g[2]);
    }
    if (want_h) {
      double Y[3][9];
      {
        double X[45];
#pragma unroll
        for (int e = 0; e < 45; ++e) X[e] = active ? Xq[e * cap + i] : 0.0;
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              Y[al][3 * r + c] = z[0] * X[pidx(3 * al + r, c)] + z[1] * X[pidx(3 * al + r, 3 + c)] +
                                 z[2] * X[pidx(3 * al + r, 6 + c)];
      }
#pragma unroll 2
      for (int ii = 0; ii < 16; ++ii) {
        const int src = gbase + ii;
        const int nI = __shfl(node, src, 64);
        const int nI1 = __shfl(node, (src & ~15) | ((ii + 1) & 15), 64);
        const bool mI = nI != NO_NODE && (ii == 15 || nI1 != nI);
        const bool v = mine && mI && nI <= node;
        if (!__any(v)) continue;
        double zI[3];
#pragma unroll
        for (int al = 0; al < 3; ++al) zI[al] = __shfl(z[al], src, 64);
        if (v) {
          double B[9];
#pragma unroll
          for (int t = 0; t < 9; ++t) B[t] = zI[0] * Y[0][t] + zI[1] * Y[1][t] + zI[2] * Y[2][t];
          const long long key = (long long)nI * n_node + node;
          bool fresh;
          const int slot = (int)table_slot64_new(s_bkey, LTBL - 1, key, fresh);
          if (slot < 0) {
            global_block_add(h, n_node, nI, node, B, status);
          } else {
            if (fresh) atomicAdd(&s_used, 1);
#pragma unroll
            for (int t = 0; t < 9; ++t) atomicAdd(&s_bval[9 * slot + t], B[t]);
          }
        }
      }
    }
    __syncthreads();
    const bool last = base + PPS >= r1;
    if (last || s_used > LTBL / 2) {
      for (int t = threadIdx.x; t < LTBL; t += EX_T) {
        const long long key = s_bkey[t];
        if (key != -1) {
          global_block_add(h, n_node, key / n_node, key % n_node, &s_bval[9 * t], status);
          s_bkey[t] = -1;
#pragma unroll
          for (int u = 0; u < 9; ++u) s_bval[9 * t + u] = 0.0;
        }
      }
      for (int t = threadIdx.x; t < LGT; t += EX_T) {
        const int key = s_gkey[t];
        if (key != -1) {
          atomicAdd(&grad[3 * (int64_t)key], s_gval[3 * t]);
          atomicAdd(&grad[3 * (int64_t)key + 1], s_gval[3 * t + 1]);
          atomicAdd(&grad[3 * (int64_t)key + 2], s_gval[3 * t + 2]);
          s_gkey[t] = -1;
          s_gval[3 * t] = s_gval[3 * t + 1] = s_gval[3 * t + 2] = 0.0;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) s_used = 0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Locality order of the active pairs: a counting sort by the first coarse
// node of the pair's first vertex with a DoF, so that a workgroup's range
// of pairs touches few distinct node blocks (its LDS tables then absorb
// most of the accumulation).
// ---------------------------------------------------------------------------
// Per-lane offsets from counters ctr[key], one atomic per distinct key in
// the wavefront (lanes with equal keys are served together).  All lanes
// of the wavefront must call.
__device__ __forceinline__ int wave_key_add(int *ctr, int key, bool valid) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (1ull << lane) - 1ull;
  int res = 0;
  uint64_t pending = __ballot(valid);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int lk = __shfl(key, leader, 64);
    const uint64_t m = __ballot(valid && key == lk) & pending;
    int base = 0;
    if (lane == leader) base = atomicAdd(&ctr[lk], __popcll(m));
    base = __shfl(base, leader, 64);
    if ((m >> lane) & 1ull) res = base + __popcll(m & lt);
    pending &= ~m;
  }
  return res;
}

template <int KIND>
__global__ void k_pair_keys(const int32_t *__restrict__ pairs, const int32_t *__restrict__ act,
                            const int64_t *__restrict__ d_count, int64_t cap, const int32_t *__restrict__ faces,
                            const int32_t *__restrict__ edges, const int32_t *__restrict__ rowptr,
                            const int32_t *__restrict__ col, int n_node, int32_t *__restrict__ key, int32_t *hist,
                            int4 *__restrict__ vidu) {
  const int64_t n = *d_count < cap ? *d_count : cap;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const bool live = i < n;
    int k = 0;
    if (live) {
      int vid[4];
      pair_vertices<KIND>(pairs, act[i], faces, edges, vid);
      k = -1;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int r0 = rowptr[vid[a]];
        if (k < 0 && rowptr[vid[a] + 1] > r0) k = col[r0];
      }
      if ((unsigned)k >= (unsigned)n_node) k = 0;
      key[i] = k;
      vidu[i] = make_int4(vid[0], vid[1], vid[2], vid[3]);
    }
    wave_key_add(hist, k, live);
  }
}

__global__ void k_pair_scatter(const int32_t *__restrict__ act, const int32_t *__restrict__ typ,
                               const int64_t *__restrict__ d_count, int64_t cap, const int32_t *__restrict__ key,
                               const int64_t *__restrict__ start, int32_t *fill, int32_t *__restrict__ act2,
                               int32_t *__restrict__ typ2, const int4 *__restrict__ vidu, int4 *__restrict__ vid2) {
  const int64_t n = *d_count < cap ? *d_count : cap;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const bool live = i < n;
    const int k = live ? key[i] : 0;
    const int off = wave_key_add(fill, k, live);
    if (live) {
      const int64_t pos = start[k] + off;
      act2[pos] = act[i];
      typ2[pos] = typ[i];
      vid2[pos] = vidu[i];
    }
  }
}

static eipc_status sort_active(eipc_ctx *c, const eipc_scene *sc, int kind, const int32_t *pairs, const int32_t *act,
                               const int32_t *typ, const int64_t *d_count, int64_t cap, const int32_t **act2,
                               const int32_t **typ2, const int4 **vid2, hipStream_t s) {
  const int nn = std::max(sc->n_node, 1);
  int32_t *key, *hist, *fill, *a2, *t2;
  int4 *vu, *v2;
  int64_t *start;
  // per kind, so that the two kinds can be sorted concurrently
  const bool e = kind != 0;
  EIPC_TRY(ensure_t(c, e ? B_SKEY_EE : B_SKEY, (size_t)cap, &key));
  EIPC_TRY(ensure_t(c, e ? B_SHIST_EE : B_SHIST, (size_t)nn + 1, &hist));
  EIPC_TRY(ensure_t(c, e ? B_SFILL_EE : B_SFILL, (size_t)nn + 1, &fill));
  EIPC_TRY(ensure_t(c, e ? B_SSTART_EE : B_SSTART, (size_t)nn + 1, &start));
  EIPC_TRY(ensure_t(c, e ? B_SACT_EE : B_SACT, (size_t)cap, &a2));
  EIPC_TRY(ensure_t(c, e ? B_STYP_EE : B_STYP, (size_t)cap, &t2));
  EIPC_TRY(ensure_t(c, e ? B_SVIDU_EE : B_SVIDU, (size_t)cap, &vu));
  EIPC_TRY(ensure_t(c, e ? B_SVID_EE : B_SVID, (size_t)cap, &v2));
  EIPC_TRY(launch_zero(c, hist, sizeof(int32_t) * (nn + 1), s));
  EIPC_TRY(launch_zero(c, fill, sizeof(int32_t) * (nn + 1), s));
  const int blocks = (int)std::min<int64_t>(grid_for(cap, 256), 8 * (int64_t)c->num_cu);
  if (kind == 0)
    k_pair_keys<0><<<blocks, 256, 0, s>>>(pairs, act, d_count, cap, sc->faces, sc->edges, sc->W_rowptr, sc->W_col,
                                          nn, key, hist, vu);
  else
    k_pair_keys<1><<<blocks, 256, 0, s>>>(pairs, act, d_count, cap, sc->faces, sc->edges, sc->W_rowptr, sc->W_col,
                                          nn, key, hist, vu);
  EIPC_HIP(c, hipGetLastError());
  EIPC_TRY(exclusive_scan(c, hist, nn, start, s));
  k_pair_scatter<<<blocks, 256, 0, s>>>(act, typ, d_count, cap, key, start, fill, a2, t2, vu, v2);
  EIPC_HIP(c, hipGetLastError());
  *act2 = a2;
  *typ2 = t2;
  if (vid2) *vid2 = v2;
  return EIPC_OK;
}

eipc_status launch_barrier(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                           const int32_t *act, const int32_t *typ, const int64_t *d_count, int64_t max_count,
                           double dhat, double kappa, uint32_t flags, double *energy, double *grad,
                           const HessOut &h, hipStream_t s) {
  if (max_count == 0) return EIPC_OK;
  const bool want_g = (flags & EIPC_GRAD) && grad;
  const bool want_h = (flags & EIPC_HESS) && h.kind != 0;
  double *gq = nullptr, *Xq = nullptr;
  const int64_t cap = max_count;
  if (want_g) EIPC_TRY(ensure_t(c, kind == 0 ? B_PG_PT : B_PG_EE, (size_t)9 * cap, &gq));
  if (want_h) EIPC_TRY(ensure_t(c, kind == 0 ? B_PX_PT : B_PX_EE, (size_t)45 * cap, &Xq));
  const int4 *vid4 = nullptr;  // vertex ids of the sorted pairs
  if (want_g || want_h) EIPC_TRY(sort_active(c, sc, kind, pairs, act, typ, d_count, cap, &act, &typ, &vid4, s));
  {
    int blocks = (int)std::min<int64_t>(grid_for(max_count, BR_THREADS), (int64_t)c->wg_per_cu[0] * c->num_cu);
    ProfScope ps(c, kind == 0 ? K_BARRIER_PT : K_BARRIER_EE, s);
    const int32_t *vsc = vscene_of(sc);
    const int nsc = n_scene_of(sc);
    if (kind == 0)
      k_pair_terms<0><<<blocks, BR_THREADS, 0, s>>>(pairs, act, typ, d_count, sc->faces, sc->edges, xs, sc->x_rest,
                                                     sc->n_vert, dhat, kappa, flags, energy, gq, Xq, cap, vsc, nsc,
                                                     c->status, vid4);
    else
      k_pair_terms<1><<<blocks, BR_THREADS, 0, s>>>(pairs, act, typ, d_count, sc->faces, sc->edges, xs, sc->x_rest,
                                                     sc->n_vert, dhat, kappa, flags, energy, gq, Xq, cap, vsc, nsc,
                                                     c->status, vid4);
    EIPC_HIP(c, hipGetLastError());
  }
  if (!want_g && !want_h) return EIPC_OK;
  return launch_expand(c, sc, kind, vid4, d_count, cap, gq, Xq, want_g ? grad : nullptr, want_h ? h : HessOut{},
                       s);
}

eipc_status launch_expand(eipc_ctx *c, const eipc_scene *sc, int kind, const int4 *vid4, const int64_t *d_count,
                          int64_t cap, const double *gq, const double *Xq, double *grad, const HessOut &h,
                          hipStream_t s) {
  int blocks = (int)std::min<int64_t>(grid_for(cap, EX_T / 16), (int64_t)c->wg_per_cu[1] * c->num_cu);
  ProfScope ps(c, kind == 0 ? K_EXPAND_PT : K_EXPAND_EE, s);
  if (kind == 0)
    k_expand16<0><<<blocks, EX_T, 0, s>>>(vid4, d_count, sc->W_rowptr, sc->W_col, sc->W_val, sc->n_node, gq, Xq,
                                           cap, grad, h, c->status);
  else
    k_expand16<1><<<blocks, EX_T, 0, s>>>(vid4, d_count, sc->W_rowptr, sc->W_col, sc->W_val, sc->n_node, gq, Xq,
                                           cap, grad, h, c->status);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

// lower 3x3 blocks of the dense reduced Hessian from the upper ones
__global__ void k_dense_mirror(int n_node, double *d) {
  const int64_t n3 = 3 * (int64_t)n_node;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n3 * n3) return;
  const int64_t r = idx / n3, cc = idx % n3;
  if (r / 3 > cc / 3) d[idx] = d[cc * n3 + r];
}

eipc_status launch_dense_mirror(eipc_ctx *c, int n_node, double *dense, hipStream_t s) {
  int64_t n3 = 3 * (int64_t)n_node;
  if (n3 == 0) return EIPC_OK;
  k_dense_mirror<<<grid_for(n3 * n3, 256), 256, 0, s>>>(n_node, dense);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

// ---------------------------------------------------------------------------
// BSR from the global hash of upper blocks: count per row (both
// triangles), scan, fill, sort each row by column, gather values.
// ---------------------------------------------------------------------------
__global__ void k_hash_rowcount(int64_t cap, const int64_t *hkey, int n_node, int32_t *rowcnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cap) return;
  const int64_t key = hkey[t];
  if (key < 0) return;
  const int I = (int)(key / n_node), J = (int)(key % n_node);
  atomicAdd(&rowcnt[I], 1);
  if (I != J) atomicAdd(&rowcnt[J], 1);
}

__global__ void k_hash_rowfill(int64_t cap, const int64_t *hkey, int n_node, const int64_t *rowptr,
                               int32_t *rowfill, int32_t *bcol, int64_t *bsrc, int64_t nnzb_cap) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cap) return;
  const int64_t key = hkey[t];
  if (key < 0) return;
  const int I = (int)(key / n_node), J = (int)(key % n_node);
  int64_t p = rowptr[I] + atomicAdd(&rowfill[I], 1);
  if (p < nnzb_cap) {
    bcol[p] = J;
    bsrc[p] = 2 * t;  // even: as stored
  }
  if (I != J) {
    p = rowptr[J] + atomicAdd(&rowfill[J], 1);
    if (p < nnzb_cap) {
      bcol[p] = I;
      bsrc[p] = 2 * t + 1;  // odd: transposed
    }
  }
}

// Sort each BSR row by column, out of place (bcol, bsrc -> bcol2, bsrc2):
// one wavefront per row.  Columns of a row are distinct, so an entry's
// position is its rank, the number of entries of the row with a smaller
// column.  Rows of up to 64 entries rank by shuffles; longer rows are
// taken 64 entries at a time, each ranked against the whole row by
// wavefront-uniform reads (any length; time grows as len^2 / 64).
// Rows that end beyond the capacity are left alone (overflow is raised).
__global__ void k_row_sort(int n_node, const int64_t *rowptr, const int32_t *bcol, const int64_t *bsrc,
                           int32_t *bcol2, int64_t *bsrc2, int32_t *rowptr32, int64_t nnzb_cap, uint32_t *status) {
  const int lane = threadIdx.x & 63;
  const int r = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (r > n_node) return;
  if (r == n_node) {
    if (lane == 0) {
      const int64_t tot = rowptr[r];
      rowptr32[r] = (int32_t)(tot < nnzb_cap ? tot : nnzb_cap);
      if (tot > nnzb_cap) atomicOr(status, ST_PLAN_OVERFLOW);
    }
    return;
  }
  const int64_t b = rowptr[r], e = rowptr[r + 1];
  if (lane == 0) rowptr32[r] = (int32_t)(b < nnzb_cap ? b : nnzb_cap);
  if (e > nnzb_cap) return;
  const int64_t len = e - b;
  if (len <= 64) {
    const bool v = lane < len;
    const int32_t cv = v ? bcol[b + lane] : 0x7fffffff;
    int rank = 0;
    for (int j = 0; j < len; ++j) rank += __shfl(cv, j, 64) < cv;
    if (v) {
      bcol2[b + rank] = cv;
      bsrc2[b + rank] = bsrc[b + lane];
    }
    return;
  }
  for (int64_t c0 = 0; c0 < len; c0 += 64) {
    const int64_t idx = c0 + lane;
    const bool v = idx < len;
    const int32_t cv = v ? bcol[b + idx] : 0x7fffffff;
    int64_t rank = 0;
    for (int64_t j = 0; j < len; ++j) rank += bcol[b + j] < cv;
    if (v) {
      bcol2[b + rank] = cv;
      bsrc2[b + rank] = bsrc[b + idx];
    }
  }
}

// blocks in BSR order; the count is read from the device (capped)
__global__ void k_bsr_gather(int64_t cap, const int32_t *rowptr32, int n_node, const int64_t *bsrc,
                             const double *hval, double *blocks) {
  const int64_t nnzb = rowptr32[n_node];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnzb && p < cap;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t src = bsrc[p];
    const double *v = hval + 9 * (src >> 1);
    if ((src & 1) == 0) {
#pragma unroll
      for (int t = 0; t < 9; ++t) blocks[9 * p + t] = v[t];
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) blocks[9 * p + 3 * i + j] = v[3 * j + i];
    }
  }
}

eipc_status bsr_compact(eipc_ctx *c, int n_node, const HessOut &h, eipc_bsr *out, hipStream_t s, int64_t nnzb_cap) {
  const int64_t cap = (int64_t)h.hmask + 1;
  int32_t *rowcnt, *rowfill, *bcol, *rowptr32;
  int64_t *rowptr, *bsrc;
  double *blocks;
  EIPC_TRY(ensure_t(c, B_ROWCNT, (size_t)n_node + 1, &rowcnt));
  EIPC_TRY(ensure_t(c, B_ROWFILL, (size_t)n_node + 1, &rowfill));
  EIPC_TRY(ensure_t(c, B_ROWPTR, (size_t)n_node + 1, &rowptr));
  EIPC_TRY(launch_zero(c, rowcnt, sizeof(int32_t) * (n_node + 1), s));
  EIPC_TRY(launch_zero(c, rowfill, sizeof(int32_t) * (n_node + 1), s));
  k_hash_rowcount<<<grid_for(cap, 256), 256, 0, s>>>(cap, h.hkey, n_node, rowcnt);
  EIPC_HIP(c, hipGetLastError());
  EIPC_TRY(exclusive_scan(c, rowcnt, n_node, rowptr, s));
  const bool planned = nnzb_cap >= 0;
  int64_t nnzb = 0;
  if (!planned) {
    EIPC_HIP(c, hipMemcpyAsync(&nnzb, rowptr + n_node, 8, hipMemcpyDeviceToHost, s));
    EIPC_HIP(c, hipStreamSynchronize(s));
    nnzb_cap = nnzb;
  }
  EIPC_TRY(ensure_t(c, B_BCOL, (size_t)std::max<int64_t>(nnzb_cap, 1), &bcol));
  EIPC_TRY(ensure_t(c, B_BSRC, (size_t)std::max<int64_t>(nnzb_cap, 1), &bsrc));
  EIPC_TRY(ensure_t(c, B_BBLK, (size_t)std::max<int64_t>(nnzb_cap, 1) * 9, &blocks));
  int32_t *bcol2;
  int64_t *bsrc2;
  EIPC_TRY(ensure_t(c, B_BCOL2, (size_t)std::max<int64_t>(nnzb_cap, 1), &bcol2));
  EIPC_TRY(ensure_t(c, B_BSRC2, (size_t)std::max<int64_t>(nnzb_cap, 1), &bsrc2));
  rowptr32 = rowcnt;  // counts are no longer needed once scanned
  k_hash_rowfill<<<grid_for(cap, 256), 256, 0, s>>>(cap, h.hkey, n_node, rowptr, rowfill, bcol, bsrc, nnzb_cap);
  EIPC_HIP(c, hipGetLastError());
  k_row_sort<<<grid_for((int64_t)(n_node + 1) * 64, 256), 256, 0, s>>>(n_node, rowptr, bcol, bsrc, bcol2, bsrc2,
                                                                        rowptr32, nnzb_cap, c->status);
  EIPC_HIP(c, hipGetLastError());
  if (nnzb_cap > 0) {
    k_bsr_gather<<<std::min(grid_for(nnzb_cap, 256), 16 * c->num_cu), 256, 0, s>>>(nnzb_cap, rowptr32, n_node, bsrc2,
                                                                                   h.hval, blocks);
    EIPC_HIP(c, hipGetLastError());
  }
  out->n_rows = n_node;
  out->nnzb = planned ? -1 : nnzb;
  out->rowptr = rowptr32;
  out->col = bcol2;
  out->blocks = blocks;
  return EIPC_OK;
}

// ---------------------------------------------------------------------------
// Hessian-vector product: y = H_x z per pair, z = (W v + v_off) on the
// pair's vertices, scattered through W^T (and unreduced into out_off).
// H_x = Q X Q^T:  zeta = Q^T z, eta = X zeta, y = Q eta.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(BR_THREADS) void k_hvp(
    const int32_t *__restrict__ pairs, const int32_t *__restrict__ act, const int32_t *__restrict__ typ,
    const int64_t *__restrict__ d_count, const int32_t *__restrict__ faces, const int32_t *__restrict__ edges,
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ xs, const double *__restrict__ xvs, const double *__restrict__ x_rest, int n_vert,
    int n_node, double dhat, double kappa, uint32_t flags, double *out, double *out_off, uint32_t *status) {
  __shared__ int s_gkey[LGT];
  __shared__ double s_gval[LGT * 3];
  __shared__ int s_used;
  LdsTables T{nullptr, nullptr, s_gkey, s_gval};
  HessOut none{0, nullptr, nullptr, nullptr, 0};
  Acc A{T, none, n_node, out, status};
  const bool moll = (KIND == 1) && (flags & EIPC_MOLLIFY) && x_rest;
  for (int t = threadIdx.x; t < LGT; t += BR_THREADS) s_gkey[t] = -1;
  for (int t = threadIdx.x; t < LGT * 3; t += BR_THREADS) s_gval[t] = 0.0;
  __syncthreads();
  const int64_t n = *d_count;
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + BR_THREADS - 1) / BR_THREADS * BR_THREADS;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  for (int64_t base = r0; base < r1; base += BR_THREADS) {
    const int64_t i = base + threadIdx.x;
    const bool active = i < r1;
    double eta[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int vid[4] = {0, 0, 0, 0};
    if (active) {
      const int64_t k = act[i];
      const int ty = typ[i];
      pair_vertices<KIND>(pairs, k, faces, edges, vid);
      V3 x[4], z[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        x[a] = load3(xs, n_vert, vid[a]);
        z[a] = load3(xvs, n_vert, vid[a]);
      }
      const double s2 = type_value<KIND>(ty, x);
      double eps = 0.0;
      if (moll) {
        V3 r[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          r[a] = V3{x_rest[3 * (int64_t)vid[a]], x_rest[3 * (int64_t)vid[a] + 1], x_rest[3 * (int64_t)vid[a] + 2]};
        eps = mollifier_eps(r);
      }
      V3 Y[3];
      y_basis<KIND>(x, Y);
      double gE[9], HE[45], M[45];
      energy_derivs<KIND>(ty, x, Y, s2, dhat, kappa, eps, gE, HE, true);
      to_q_basis<KIND>(HE, M);
      if (flags & EIPC_PROJECT) project_psd9(M);
      // zeta = Q^T z, eta = X zeta
      double zeta[9];
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        double zx = 0, zy = 0, zz = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const double sg = 0.5 * kS[a][al];
          zx += sg * z[a].x;
          zy += sg * z[a].y;
          zz += sg * z[a].z;
        }
        zeta[3 * al] = zx;
        zeta[3 * al + 1] = zy;
        zeta[3 * al + 2] = zz;
      }
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int cc = 0; cc < 9; ++cc) acc += M[pidx(r, cc)] * zeta[cc];
        eta[r] = acc;
      }
      if (out_off) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          double y0 = 0, y1 = 0, y2 = 0;
#pragma unroll
          for (int al = 0; al < 3; ++al) {
            const double sg = 0.5 * kS[a][al];
            y0 += sg * eta[3 * al];
            y1 += sg * eta[3 * al + 1];
            y2 += sg * eta[3 * al + 2];
          }
          atomicAdd(&out_off[3 * (int64_t)vid[a]], y0);
          atomicAdd(&out_off[3 * (int64_t)vid[a] + 1], y1);
          atomicAdd(&out_off[3 * (int64_t)vid[a] + 2], y2);
        }
      }
    }
    // reduced product through the merged node set: out[I] += z_I^T eta
    NodeSet S;
    int m = 0;
    if (active) gather_nodes<KIND>(vid, rowptr, col, val, S, m);
#pragma unroll
    for (int sl = 0; sl < 16; ++sl) {
      const bool v = active && sl < m;
      if (__any(v)) {
        double g[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
          g[c] = S.z[sl][0] * eta[c] + S.z[sl][1] * eta[3 + c] + S.z[sl][2] * eta[6 + c];
        agg_vec(A, v, v ? S.node[sl] : -1, g[0], g[1], g[2]);
      }
    }
    __syncthreads();
    const bool last = base + BR_THREADS >= r1;
    if (!last) {
      if (threadIdx.x == 0) s_used = 0;
      __syncthreads();
      int cnt = 0;
      for (int t = threadIdx.x; t < LGT; t += BR_THREADS) cnt += s_gkey[t] != -1;
      if (cnt) atomicAdd(&s_used, cnt);
      __syncthreads();
    }
    if (last || s_used > LGT / 2) {
      for (int t = threadIdx.x; t < LGT; t += BR_THREADS) {
        const int key = s_gkey[t];
        if (key != -1) {
          atomicAdd(&out[3 * (int64_t)key], s_gval[3 * t]);
          atomicAdd(&out[3 * (int64_t)key + 1], s_gval[3 * t + 1]);
          atomicAdd(&out[3 * (int64_t)key + 2], s_gval[3 * t + 2]);
          s_gkey[t] = -1;
          s_gval[3 * t] = s_gval[3 * t + 1] = s_gval[3 * t + 2] = 0.0;
        }
      }
    }
    __syncthreads();
  }
}

eipc_status launch_hvp(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *xvs,
                       const int32_t *pairs, const int32_t *act, const int32_t *typ, const int64_t *d_count,
                       int64_t max_count, double dhat, double kappa, uint32_t flags, double *out,
                       double *out_off, hipStream_t s, bool locality_sort) {
  if (max_count == 0) return EIPC_OK;
  // the locality order only cuts the flushes of the LDS tables
  if (locality_sort) EIPC_TRY(sort_active(c, sc, kind, pairs, act, typ, d_count, max_count, &act, &typ, nullptr, s));
  int blocks = (int)std::min<int64_t>(grid_for(max_count, BR_THREADS), 4 * (int64_t)c->num_cu);
  ProfScope ps(c, kind == 0 ? K_HVP_PT : K_HVP_EE, s);
  if (kind == 0)
    k_hvp<0><<<blocks, BR_THREADS, 0, s>>>(pairs, act, typ, d_count, sc->faces, sc->edges, sc->W_rowptr, sc->W_col,
                                            sc->W_val, xs, xvs, sc->x_rest, sc->n_vert, sc->n_node, dhat, kappa,
                                            flags, out, out_off, c->status);
  else
    k_hvp<1><<<blocks, BR_THREADS, 0, s>>>(pairs, act, typ, d_count, sc->faces, sc->edges, sc->W_rowptr, sc->W_col,
                                            sc->W_val, xs, xvs, sc->x_rest, sc->n_vert, sc->n_node, dhat, kappa,
                                            flags, out, out_off, c->status);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

// ---------------------------------------------------------------------------
// per-pair inspection: type, s, e, g (12), H (12x12)
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void k_pair_eval(int64_t n, const int32_t *__restrict__ pairs, const int32_t *__restrict__ faces,
                            const int32_t *__restrict__ edges, const double *__restrict__ xs,
                            const double *__restrict__ x_rest, int n_vert, double dhat, double kappa,
                            uint32_t flags, int32_t *type, double *sq, double *e, double *g, double *H) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int vid[4];
  pair_vertices<KIND>(pairs, i, faces, edges, vid);
  V3 x[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) x[a] = load3(xs, n_vert, vid[a]);
  int ty;
  const double s2 = pair_dist2<KIND>(x, &ty);
  if (type) type[i] = ty;
  if (sq) sq[i] = s2;
  const bool active = s2 > 0.0 && s2 < dhat * dhat;
  double eps = 0.0;
  if (KIND == 1 && (flags & EIPC_MOLLIFY) && x_rest) {
    V3 r[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      r[a] = V3{x_rest[3 * (int64_t)vid[a]], x_rest[3 * (int64_t)vid[a] + 1], x_rest[3 * (int64_t)vid[a] + 2]};
    eps = mollifier_eps(r);
  }
  double gE[9], HE[45], M[45];
  double ev = 0.0;
  if (active) {
    V3 Y[3];
    y_basis<KIND>(x, Y);
    ev = energy_derivs<KIND>(ty, x, Y, s2, dhat, kappa, eps, gE, HE, true);
    to_q_basis<KIND>(HE, M);
    if (flags & EIPC_PROJECT) project_psd9(M);
  }
  if (e) e[i] = ev;
  if (g) {
    double gx[12];
    if (active)
      slot_grad<KIND>(gE, gx);
    else
      for (int t = 0; t < 12; ++t) gx[t] = 0.0;
    for (int t = 0; t < 12; ++t) g[12 * i + t] = gx[t];
  }
  if (H) {
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        double B[9];
        if (active)
          x_block(M, a, b, B);
        else
          for (int t = 0; t < 9; ++t) B[t] = 0.0;
        for (int ii = 0; ii < 3; ++ii)
          for (int jj = 0; jj < 3; ++jj) H[144 * i + (3 * a + ii) * 12 + 3 * b + jj] = B[3 * ii + jj];
      }
  }
}

eipc_status launch_pair_eval(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                             int64_t n, double dhat, double kappa, uint32_t flags, int32_t *type, double *sq,
                             double *e, double *g, double *H, hipStream_t s) {
  if (n == 0) return EIPC_OK;
  if (kind == 0)
    k_pair_eval<0><<<grid_for(n, 64), 64, 0, s>>>(n, pairs, sc->faces, sc->edges, xs, sc->x_rest, sc->n_vert, dhat,
                                                   kappa, flags, type, sq, e, g, H);
  else
    k_pair_eval<1><<<grid_for(n, 64), 64, 0, s>>>(n, pairs, sc->faces, sc->edges, xs, sc->x_rest, sc->n_vert, dhat,
                                                   kappa, flags, type, sq, e, g, H);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

}  // namespace eipc
