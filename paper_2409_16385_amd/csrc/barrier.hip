// Per-pair barrier energy, gradient and (projected) Hessian, reduced through
// the embedding (Eq. 17) with LDS-staged accumulation; Hessian-vector
// products; BSR compaction of the reduced Hessian.
#include <algorithm>

#include "common.h"
#include "pair_math.h"

namespace eipc {

constexpr int BR_THREADS = 256;
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
    long long k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// find-or-insert of key in an LDS open-addressing table of `size` entries
// (all bits set = empty): linear probing from a multiplicative range
// reduction of the key's hash.  All lanes of the wavefront call, `valid`
// marking the lanes that look up; a lane that finds no slot within
// MAX_PROBE probes gets -1.  fresh: this lane inserted the key.
template <typename K>
__device__ __forceinline__ int lds_slot(K *keys, int size, K key, bool valid, bool &fresh) {
  const uint32_t hv = sizeof(K) == 8 ? mix64((uint64_t)key) : mix32((uint32_t)key);
  int h = (int)(((uint64_t)hv * (uint32_t)size) >> 32);
  int slot = -1;
  fresh = false;
  bool pending = valid;
  for (int p = 0; p < MAX_PROBE; ++p) {
    if (!__any(pending)) break;
    if (pending) {
      K k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (k == (K)~(K)0) {
        k = atomicCAS(&keys[h], (K)~(K)0, key);
        if (k == (K)~(K)0) {
          fresh = true;
          k = key;
        }
      }
      if (k == key) {
        slot = h;
        pending = false;
      } else {
        h = h + 1 == size ? 0 : h + 1;
      }
    }
  }
  return slot;
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

// A workgroup's LDS table of node 3-vectors keyed by node.
struct LdsTables {
  uint32_t *gkey;
  double *gval;
};

// ---------------------------------------------------------------------------
// A pair's merged node set in one lane (the Hessian-vector product).  The
// 16 (node, weight) slots of a pair (4 vertices x up to 4 weights) are
// taken to the Q basis, z_s = w_s Q[a(s)] (3 numbers), sorted by node with
// a bitonic network, equal nodes merged, and sorted again to compact.
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

// Add a lane's node 3-vector into the LDS node table (all lanes of the
// wavefront call): summed across the wavefront first when every valid lane
// holds the same node; a table miss goes to the output directly.
__device__ __forceinline__ void agg_vec(const Acc &A, bool valid, int node, double g0, double g1, double g2) {
  const uint64_t vm = __ballot(valid);
  if (vm == 0) return;
  const int first = __ffsll((unsigned long long)vm) - 1;
  const int k0 = __shfl(node, first, 64);
  bool ins = valid;
  if (__ballot(valid && node != k0) == 0) {
    g0 = wave_sum(valid ? g0 : 0.0);
    g1 = wave_sum(valid ? g1 : 0.0);
    g2 = wave_sum(valid ? g2 : 0.0);
    ins = (int)(threadIdx.x & 63) == first;
  }
  bool fresh;
  const int slot = lds_slot<uint32_t>(A.T.gkey, LGT, (uint32_t)node, ins, fresh);
  if (!ins) return;
  if (slot < 0) {
    atomicAdd(&A.grad[3 * (int64_t)node], g0);
    atomicAdd(&A.grad[3 * (int64_t)node + 1], g1);
    atomicAdd(&A.grad[3 * (int64_t)node + 2], g2);
    return;
  }
  atomicAdd(&A.T.gval[3 * slot], g0);
  atomicAdd(&A.T.gval[3 * slot + 1], g1);
  atomicAdd(&A.T.gval[3 * slot + 2], g2);
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

// ---------------------------------------------------------------------------
// Reduction through W (Eq. 17) of per-pair term records (gamma, X in the Q
// basis; TERM_REC doubles per pair).
//
// A workgroup accumulates into LDS over a contiguous range of pairs in
// locality order.  Nodes, not blocks, are looked up: a node's local index
// is its slot in a small open-addressing table of LN slots (installed by
// compare-and-swap), and the blocks of local nodes a <= b live in a dense
// packed upper triangle of LN x LN 3x3 FP64 blocks addressed
// arithmetically, the gradient in LN 3-vectors.  A node that finds no slot
// (the table is full) goes straight to the outputs.  Between steps the
// accumulator is flushed into the outputs once it holds more than LN / 2
// nodes (each touched block once).
// ---------------------------------------------------------------------------
constexpr int EX_T = 512;                // eight wavefronts, two per SIMD
constexpr int EX_PPG = 8;                // pairs per 16-lane group and step
constexpr int EX_STEP = EX_T / 16 * EX_PPG;  // pairs per step (256)
constexpr int LN = 60;                   // local node slots
constexpr int LNB = LN * (LN + 1) / 2;   // their upper 3x3 blocks (129 KiB)
constexpr int LN_PROBE = 16;
constexpr int EX_TRI = 16 * 17 / 2;      // blocks of a pair's (at most 16) merged nodes

struct LocalAcc {
  int *nkey;               // LN: node of the slot, -1 = empty
  double *bval;            // LNB * 9 (rows of the lower slot)
  unsigned char *touched;  // LNB
  double *gval;            // LN * 3
  int *count;              // nodes installed
};

__device__ __forceinline__ int ltri(int a, int b) { return a * LN - (a * (a - 1)) / 2 + (b - a); }  // a <= b

// local slot of node (all lanes of the wavefront call; valid marks the
// lookups); -1 when none is found within LN_PROBE probes
__device__ __forceinline__ int local_index(const LocalAcc &L, int node, bool valid) {
  int h = (int)(((uint64_t)mix32((uint32_t)node) * (uint32_t)LN) >> 32);
  int li = -1;
  bool pending = valid;
  for (int p = 0; p < LN_PROBE; ++p) {
    if (!__any(pending)) break;
    if (pending) {
      int k = __hip_atomic_load(&L.nkey[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (k == -1) {
        k = atomicCAS(&L.nkey[h], -1, node);
        if (k == -1) {
          atomicAdd(L.count, 1);
          k = node;
        }
      }
      if (k == node) {
        li = h;
        pending = false;
      } else {
        h = h + 1 == LN ? 0 : h + 1;
      }
    }
  }
  return li;
}

__device__ __forceinline__ void local_init(const LocalAcc &L) {
  for (int t = threadIdx.x; t < LN; t += blockDim.x) L.nkey[t] = -1;
  for (int t = threadIdx.x; t < LNB * 9; t += blockDim.x) L.bval[t] = 0.0;
  for (int t = threadIdx.x; t < LNB; t += blockDim.x) L.touched[t] = 0;
  for (int t = threadIdx.x; t < LN * 3; t += blockDim.x) L.gval[t] = 0.0;
  if (threadIdx.x == 0) *L.count = 0;
}

// All threads of the workgroup call (between barriers).
__device__ __forceinline__ void local_flush(const LocalAcc &L, const HessOut &h, int n_node, double *grad,
                                            uint32_t *status) {
  // per thread up to FU blocks at a time: first their global slots (table
  // reads), then their adds.  A table read issued after adds would wait
  // for all of them: vector memory operations retire in order.
  constexpr int FU = 4;
  for (int base = 0; base < LNB; base += FU * (int)blockDim.x) {
    int64_t dst[FU];  // kind 2: table slot; kind 1: I * n_node + J; -1: none
    bool tr[FU];
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int idx = base + u * (int)blockDim.x + (int)threadIdx.x;
      dst[u] = -1;
      tr[u] = false;
      if (idx < LNB && L.touched[idx]) {
        // row a of the packed triangle: start(a) = a (2 LN - a + 1) / 2 <= idx
        int a = (int)((2.0 * LN + 1.0 - sqrt((2.0 * LN + 1.0) * (2.0 * LN + 1.0) - 8.0 * idx)) * 0.5);
        if (a < 0) a = 0;
        while (a + 1 < LN && ltri(a + 1, a + 1) <= idx) ++a;
        while (a > 0 && ltri(a, a) > idx) --a;
        const int b = a + (idx - ltri(a, a));
        const int na = L.nkey[a], nb = L.nkey[b];
        tr[u] = na > nb;
        const int64_t I = tr[u] ? nb : na, J = tr[u] ? na : nb;
        if (h.kind == 1) {
          dst[u] = I * n_node + J;
        } else if (h.kind == 2) {
          dst[u] = table_slot64((long long *)h.hkey, h.hmask, (long long)(I * n_node + J), GLOBAL_PROBE);
          if (dst[u] < 0) atomicOr(status, ST_HASH_OVERFLOW);
        }
        if (dst[u] < 0) {
#pragma unroll
          for (int t = 0; t < 9; ++t) L.bval[9 * idx + t] = 0.0;
          L.touched[idx] = 0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int idx = base + u * (int)blockDim.x + (int)threadIdx.x;
      if (dst[u] < 0) continue;
      double B[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) B[3 * r + c] = tr[u] ? L.bval[9 * idx + 3 * c + r] : L.bval[9 * idx + 3 * r + c];
#pragma unroll
      for (int t = 0; t < 9; ++t) L.bval[9 * idx + t] = 0.0;
      L.touched[idx] = 0;
      if (h.kind == 1) {
        const int64_t n3 = 3 * (int64_t)n_node, I = dst[u] / n_node, J = dst[u] % n_node;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) atomicAdd(&h.dense[(3 * I + i) * n3 + 3 * J + j], B[3 * i + j]);
      } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) atomicAdd(&h.hval[9 * dst[u] + t], B[t]);
      }
    }
  }
  __syncthreads();  // nkey is read above and reset below
  for (int li = threadIdx.x; li < LN; li += blockDim.x) {
    const int node = L.nkey[li];
    if (node >= 0 && grad) {
#pragma unroll
      for (int c = 0; c < 3; ++c) atomicAdd(&grad[3 * (int64_t)node + c], L.gval[3 * li + c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) L.gval[3 * li + c] = 0.0;
    L.nkey[li] = -1;
  }
  __syncthreads();
  if (threadIdx.x == 0) *L.count = 0;
}

__device__ __forceinline__ int permute_lane(int v, int dst) { return __builtin_amdgcn_ds_permute(dst << 2, v); }
__device__ __forceinline__ double permute_lane(double v, int dst) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_permute(dst << 2, (int)(unsigned)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_permute(dst << 2, (int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// J with J(J+1)/2 <= t < (J+1)(J+2)/2, for 0 <= t < 256
__device__ __forceinline__ int tri_root(int t) {
  int J = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  if (((J + 1) * (J + 2)) / 2 <= t) ++J;
  if ((J * (J + 1)) / 2 > t) --J;
  return J;
}

// The wavefront's pairs are held by lanes 16g + p, p < EX_PPG (pair i0 +
// g EX_PPG + p, `own` when it exists) and taken in EX_PPG passes: in pass p
// the sixteen lanes of group g (lanes 16g .. 16g+15) serve the pair of lane
// 16g + p, lane s holding slot s = (vertex s / 4, weight s % 4): its node
// and z_s = w_s Q[a] (3 numbers).
// The slots are sorted by node (bitonic on the packed key node * 16 + s),
// runs of equal nodes summed (the run's last lane keeps the total), and the
// m distinct nodes packed in order onto lanes 0 .. m-1 of the group, which
// look up their local indices.  Node I's gradient is sum_alpha z_I[alpha]
// gamma_alpha; the merged nodes are staged in LDS and the m(m+1)/2 blocks
// I <= J dealt to the group's lanes (block t on lane t mod 16, its (I, J)
// from a table),
//   B(I, J) = sum_{alpha, beta} z_I[alpha] z_J[beta] X[alpha][beta].
// All 64 lanes call, in wavefront-uniform control flow.
// A merged node of a pass, staged in LDS for the group's block lanes.
struct NodeRec {
  double z[3];
  int node;  // NO_NODE past the group's m nodes
  int li;    // local index, -1 = none
};

// One block of the pass: B(I, J) = sum_{alpha, beta} z_I[alpha] z_J[beta]
// X[alpha][beta] into the accumulator.  A local block holds the rows of the
// lower local index: when that is J's, B(J, I) = B(I, J)^T is formed
// directly by exchanging the two nodes' roles (X is symmetric), so no
// element is picked by a run-time index.
__device__ __forceinline__ void expand_block(const LocalAcc &L, const HessOut &h, int n_node, uint32_t *status,
                                             const double *Xo, const NodeRec &RI, const NodeRec &RJ) {
  const bool both = RI.li >= 0 && RJ.li >= 0;
  const bool tr = both && RI.li > RJ.li;
  double w[9];
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int be = 0; be < 3; ++be) w[3 * al + be] = (tr ? RJ.z[al] : RI.z[al]) * (tr ? RI.z[be] : RJ.z[be]);
  double B[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) acc += w[3 * al + be] * Xo[pidx(3 * al + r, 3 * be + c)];
      B[3 * r + c] = acc;
    }
  if (both) {
    const int slot = tr ? ltri(RJ.li, RI.li) : ltri(RI.li, RJ.li);
#pragma unroll
    for (int u = 0; u < 9; ++u) atomicAdd(&L.bval[9 * slot + u], B[u]);
    L.touched[slot] = 1;
  } else {
    global_block_add(h, n_node, RI.node, RJ.node, B, status);
  }
}

__device__ __forceinline__ void expand_wave(const LocalAcc &L, const HessOut &h, int n_node, double *grad,
                                            uint32_t *status, const int32_t *__restrict__ rowptr,
                                            const int32_t *__restrict__ col, const double *__restrict__ val,
                                            bool own, const int *vid, const double *__restrict__ rec, int64_t i0,
                                            bool want_g, bool want_h, NodeRec *nstage,
                                            const uint16_t *__restrict__ tri_ij) {
  const int lane = threadIdx.x & 63;
  const int s = lane & 15;
  const int gbase = lane & ~15;
  const int a = s >> 2, k = s & 3;
  const uint64_t own_mask = __ballot(own);
  // The slot data of pass p (row of the slot's vertex, then its node and
  // weight) is loaded one and two passes ahead, so its latency hides behind
  // the previous pass.
  auto slot_vertex = [&](int p) {
    const int owner = gbase + p;
    const int v0 = __shfl(vid[0], owner, 64), v1 = __shfl(vid[1], owner, 64);
    const int v2 = __shfl(vid[2], owner, 64), v3 = __shfl(vid[3], owner, 64);
    return a == 0 ? v0 : (a == 1 ? v1 : (a == 2 ? v2 : v3));
  };
  int row_k0, row_n;  // row of pass p + 1
  int cur_node = NO_NODE;
  double cur_w = 0.0;  // slot of pass p
  {
    const int v = slot_vertex(0);
    const int k0 = rowptr[v];
    const int cnt = rowptr[v + 1] - k0;
    if ((own_mask >> gbase) & 1ull && k < cnt) {
      cur_node = col[k0 + k];
      cur_w = val[k0 + k];
    }
    const int v1 = slot_vertex(1 < EX_PPG ? 1 : 0);
    row_k0 = rowptr[v1];
    row_n = rowptr[v1 + 1] - row_k0;
  }
  for (int p = 0; p < EX_PPG; ++p) {
    // pairs fill the owner lanes in order: an empty pass ends the wavefront's work
    if (((own_mask >> p) & 0x0001000100010001ull) == 0) break;
    const int owner = gbase + p;
    const bool active = (own_mask >> owner) & 1ull;
    // the owner's terms (the sixteen lanes read the same record; a group
    // without a pair reads the wavefront's first and ignores it)
    const double2 *r2 =
        (const double2 *)(rec + (i0 + (active ? (gbase >> 4) * EX_PPG + p : 0)) * TERM_REC);
    double tv[54];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const double2 t2 = r2[q];
      tv[2 * q] = t2.x;
      tv[2 * q + 1] = t2.y;
    }
    if (want_h) {
#pragma unroll
      for (int q = 5; q < 27; ++q) {
        const double2 t2 = r2[q];
        tv[2 * q] = t2.x;
        tv[2 * q + 1] = t2.y;
      }
    }
    // prefetch: the slot of pass p + 1, the row of pass p + 2
    int nxt_node = NO_NODE;
    double nxt_w = 0.0;
    if (p + 1 < EX_PPG) {
      if ((own_mask >> (owner + 1)) & 1ull && k < row_n) {
        nxt_node = col[row_k0 + k];
        nxt_w = val[row_k0 + k];
      }
      if (p + 2 < EX_PPG) {
        const int v2 = slot_vertex(p + 2);
        row_k0 = rowptr[v2];
        row_n = rowptr[v2 + 1] - row_k0;
      }
    }
    int node = cur_node;
    double z[3];
#pragma unroll
    for (int al = 0; al < 3; ++al) z[al] = 0.5 * (double)qsign(a, al) * cur_w;
    cur_node = nxt_node;
    cur_w = nxt_w;
    // sort the group's slots by node: bitonic on the packed key node * 16 +
    // slot (unique in the group, empty slots last), then each position
    // takes its slot's z
    uint32_t pk = node == NO_NODE ? (0xfffffff0u | (uint32_t)s) : (((uint32_t)node << 4) | (uint32_t)s);
#pragma unroll
    for (int kk = 2; kk <= 16; kk <<= 1)
#pragma unroll
      for (int j = kk >> 1; j > 0; j >>= 1) {
        const uint32_t po = (uint32_t)__shfl_xor((int)pk, j, 64);
        const bool up = (s & kk) == 0, low = (s & j) == 0;
        const bool take = (low == up) ? (po < pk) : (po > pk);
        pk = take ? po : pk;
      }
    node = (pk >> 4) == 0x0fffffffu ? NO_NODE : (int)(pk >> 4);
    {
      const int src = gbase + (int)(pk & 15u);
#pragma unroll
      for (int al = 0; al < 3; ++al) z[al] = __shfl(z[al], src, 64);
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
    // pack the distinct nodes onto lanes 0..m-1 of the group, in order (a
    // permutation of the group's lanes)
    const uint32_t gm = (uint32_t)(__ballot(mine) >> gbase) & 0xffffu;
    const int m = __popc(gm);
    const int below = __popc(gm & ((1u << s) - 1u));
    const int dst = gbase + (mine ? below : m + (s - below));
    const int pnode = permute_lane(node, dst);
    double cz[3];
#pragma unroll
    for (int al = 0; al < 3; ++al) cz[al] = permute_lane(z[al], dst);
    const bool has = s < m;
    const int cnode = has ? pnode : NO_NODE;
    const int cli = local_index(L, cnode, has);
    if (want_g && has) {
      double g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = cz[0] * tv[c] + cz[1] * tv[3 + c] + cz[2] * tv[6 + c];
      if (cli >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(&L.gval[3 * cli + c], g[c]);
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(&grad[3 * (int64_t)cnode + c], g[c]);
      }
    }
    if (want_h) {
      // the group's merged nodes go to its LDS stage (the previous pass's
      // reads of it come first in the wavefront's program order)
      NodeRec *ns = nstage + gbase;
      if (has) {
        NodeRec r;
        r.z[0] = cz[0];
        r.z[1] = cz[1];
        r.z[2] = cz[2];
        r.node = cnode;
        r.li = cli;
        ns[s] = r;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const double *Xo = tv + 9;
      const int nb = (m * (m + 1)) >> 1;
      for (int t0 = 0;; t0 += 16) {
        const int t = t0 + s;
        const bool vb = t < nb;
        if (!__any(vb)) break;
        if (vb) {
          const uint32_t ij = tri_ij[t];
          expand_block(L, h, n_node, status, Xo, ns[ij & 15u], ns[ij >> 8]);
        }
      }
    }
  }
}

// Reduction of per-pair term records (pairs in locality order with their
// vertex ids): a workgroup takes a contiguous range, 32 pairs per
// wavefront and step.  Instantiated per pair kind (the code is the same)
// so that the two launches of a step carry their own names in kernel
// traces.
template <int KIND>
__global__ __launch_bounds__(EX_T) void k_expand(
    const int4 *__restrict__ vid4, const int64_t *__restrict__ d_count, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const double *__restrict__ val, int n_node, const double *__restrict__ rec,
    int64_t cap, bool want_g, bool want_h, double *grad, HessOut h, uint32_t *status) {
  __shared__ int s_nkey[LN];
  __shared__ double s_bval[LNB * 9];
  __shared__ double s_gval[LN * 3];
  __shared__ unsigned char s_touched[LNB];
  __shared__ int s_count;
  __shared__ NodeRec s_nodes[EX_T];       // per wavefront: 4 groups x 16
  __shared__ uint16_t s_tri[EX_TRI];      // block t -> I | J << 8, I <= J < 16
  LocalAcc L{s_nkey, s_bval, s_touched, s_gval, &s_count};
  for (int t = threadIdx.x; t < EX_TRI; t += blockDim.x) {
    const int J = tri_root(t);
    s_tri[t] = (uint16_t)((t - ((J * (J + 1)) >> 1)) | (J << 8));
  }
  local_init(L);
  __syncthreads();
  // consecutive ranges on one XCD (workgroups are dealt to the 8 XCDs in turn)
  int rid = blockIdx.x;
  if ((gridDim.x & 7) == 0) rid = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const int64_t n = *d_count < cap ? *d_count : cap;
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + 63) / 64 * 64;
  const int64_t r0 = (int64_t)rid * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int64_t base = r0; base < r1; base += EX_STEP) {
    const int64_t wb = base + 4 * EX_PPG * wave;
    if (wb < r1) {
      const int64_t i = wb + (lane >> 4) * EX_PPG + (lane & 15);
      const bool live = (lane & 15) < EX_PPG && i < r1;
      int vid[4] = {0, 0, 0, 0};
      if (live) {
        const int4 v4 = vid4[i];
        vid[0] = v4.x;
        vid[1] = v4.y;
        vid[2] = v4.z;
        vid[3] = v4.w;
      }
      expand_wave(L, h, n_node, grad, status, rowptr, col, val, live, vid, rec, wb, want_g, want_h,
                  s_nodes + 64 * wave, s_tri);
    }
    __syncthreads();
    if (base + EX_STEP >= r1 || s_count > LN / 2) local_flush(L, h, n_node, want_g ? grad : nullptr, status);
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

// ---------------------------------------------------------------------------
// Per active pair: the energy (Eq. 7, summed per scene), its Q-basis
// gradient and (projected) Hessian, stored as a term record in the pair's
// (locality-order) position for k_expand.
//
// A workgroup takes a contiguous range of the active pairs in tiles of up
// to TERMS_TILE pairs.  Each tile is put in order of pair class (point-point,
// point-line, interior, mollified) by a counting sort in LDS, so that the
// lanes of a wavefront nearly always share one derivative path; each
// wavefront then takes 64 pairs of the tile at a time, one per lane.
// ---------------------------------------------------------------------------
constexpr int TERMS_T = 256;      // four wavefronts, one per SIMD (the 9x9 projection's registers)
constexpr int TERMS_TILE = 2048;  // pairs per class-sorted tile

template <int KIND, bool REDUCED>
__global__ __launch_bounds__(TERMS_T) void k_pair_terms(
    const int32_t *__restrict__ pairs, const int32_t *__restrict__ act, const int32_t *__restrict__ typ,
    const int4 *__restrict__ vid4, const int64_t *__restrict__ d_count, int64_t cap,
    const int32_t *__restrict__ faces, const int32_t *__restrict__ edges, const double *__restrict__ xs,
    const double *__restrict__ x_rest, int n_vert, double dhat, double kappa, uint32_t flags, bool want_g,
    bool want_h, double *energy, double *__restrict__ rec, const int32_t *__restrict__ vscene, int n_scene,
    uint32_t *status, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
    const double *__restrict__ val) {
  __shared__ int s_tile[TERMS_TILE];
  __shared__ int s_cnt[4];
  __shared__ double s_e[TERMS_T / 64];
  const bool expand = want_g || want_h;
  // the reduced-block projection takes the true X and projects after the transform
  const bool reduced = REDUCED && want_h;
  const bool project = (flags & EIPC_PROJECT) && !reduced;
  const bool sq = flags & EIPC_SQDIST;
  const bool moll = (KIND == 1) && (flags & EIPC_MOLLIFY) && x_rest;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  constexpr int NW = TERMS_T / 64;
  const int64_t n = *d_count < cap ? *d_count : cap;
  const int64_t per = ((n + gridDim.x - 1) / gridDim.x + 63) / 64 * 64;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  double e_acc = 0.0;
  for (int64_t tb = r0; tb < r1; tb += TERMS_TILE) {
    const int tn = (int)(r1 - tb < TERMS_TILE ? r1 - tb : TERMS_TILE);
    if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    // class of each pair of the tile and its rank within the class
    constexpr int PER_T = TERMS_TILE / TERMS_T;
    int cls_of[PER_T], rank_of[PER_T];
#pragma unroll
    for (int u = 0; u < PER_T; ++u) {
      const int li = u * TERMS_T + threadIdx.x;
      const bool v = li < tn;
      int cls = 0;
      if (v && expand) {
        const int64_t i = tb + li;
        const int ty = typ[i];
        if (moll) {
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
          V3 x[4], r[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            x[q] = load3(xs, n_vert, vid[q]);
            r[q] = V3{x_rest[3 * (int64_t)vid[q]], x_rest[3 * (int64_t)vid[q] + 1], x_rest[3 * (int64_t)vid[q] + 2]};
          }
          cls = pair_class<KIND>(ty, x, mollifier_eps(r));
        } else {
          cls = type_fn<KIND>(ty);
        }
      }
      cls_of[u] = cls;
      rank_of[u] = wave_key_add(s_cnt, cls, v);
    }
    __syncthreads();
    {
      const int c0 = s_cnt[0], c1 = s_cnt[1], c2 = s_cnt[2];
#pragma unroll
      for (int u = 0; u < PER_T; ++u) {
        const int li = u * TERMS_T + threadIdx.x;
        if (li < tn) {
          const int cls = cls_of[u];
          const int base = cls == 0 ? 0 : (cls == 1 ? c0 : (cls == 2 ? c0 + c1 : c0 + c1 + c2));
          s_tile[base + rank_of[u]] = li | (cls << 16);
        }
      }
    }
    __syncthreads();
    const int nc = (tn + 63) / 64;
    for (int ch = wave; ch < nc; ch += NW) {
      const int pos = ch * 64 + lane;
      const bool live = pos < tn;
      double e_pair = 0.0;
      int scene = 0;
      if (live) {
        const int code = s_tile[pos];
        const int64_t i = tb + (code & 0xffff);
        const int cls = code >> 16;
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
        for (int q = 0; q < 4; ++q) x[q] = load3(xs, n_vert, vid[q]);
        double eps = 0.0;
        if (moll && (cls == CLS_GEN || !expand)) {
          V3 r[4];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            r[q] = V3{x_rest[3 * (int64_t)vid[q]], x_rest[3 * (int64_t)vid[q] + 1], x_rest[3 * (int64_t)vid[q] + 2]};
          eps = mollifier_eps(r);
        }
        if (expand) {
          double tv[54];
          e_pair = pair_qterms<KIND>(cls, ty, x, eps, dhat, kappa, want_g, want_h, project, sq, tv, tv + 9);
          if (reduced) {
            // dot products of the four vertices' rows of W
            int cc[4][4];
            double ww[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const int k0 = rowptr[vid[a]];
              const int n = rowptr[vid[a] + 1] - k0;
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const bool v = k < n;
                cc[a][k] = v ? col[k0 + k] : -1 - (4 * a + k);
                ww[a][k] = v ? val[k0 + k] : 0.0;
              }
            }
            double M4[16];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = a; b < 4; ++b) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                  for (int l = 0; l < 4; ++l) acc += cc[a][k] == cc[b][l] ? ww[a][k] * ww[b][l] : 0.0;
                M4[a * 4 + b] = acc;
                M4[b * 4 + a] = acc;
              }
            reduced_block_projection(M4, tv + 9);
          }
          double2 *r2 = (double2 *)(rec + i * TERM_REC);
          const int nst = want_h ? 27 : 5;
#pragma unroll
          for (int q = 0; q < 27; ++q)
            if (q < nst) r2[q] = make_double2(tv[2 * q], tv[2 * q + 1]);
        } else {
          e_pair = pair_energy<KIND>(ty, x, eps, dhat, kappa, sq);
        }
      }
      if (energy && vscene) agg_scene_add(energy, live, scene, n_scene, e_pair, status);
      e_acc += e_pair;
    }
  }
  if (energy && !vscene) {
    e_acc = wave_sum(e_acc);
    if (lane == 0) s_e[wave] = e_acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += s_e[w];
      if (t != 0.0) atomicAdd(energy, t);
    }
  }
}

eipc_status launch_barrier(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                           const int32_t *act, const int32_t *typ, const int64_t *d_count, int64_t max_count,
                           double dhat, double kappa, uint32_t flags, double *energy, double *grad,
                           const HessOut &h, hipStream_t s) {
  if (max_count == 0) return EIPC_OK;
  // node ids are packed with 4 bits of slot in the expansion's sort
  if (sc->n_node >= (1 << 27)) return set_err(c, EIPC_ERR_ARG, "n_node must be below 2^27");
  const bool want_g = (flags & EIPC_GRAD) && grad;
  const bool want_h = (flags & EIPC_HESS) && h.kind != 0;
  const int64_t cap = max_count;
  const int4 *vid4 = nullptr;  // vertex ids of the sorted pairs
  double *rec = nullptr;
  if (want_g || want_h) {
    EIPC_TRY(sort_active(c, sc, kind, pairs, act, typ, d_count, cap, &act, &typ, &vid4, s));
    EIPC_TRY(ensure_t(c, kind == 0 ? B_PX_PT : B_PX_EE, (size_t)TERM_REC * cap, &rec));
  }
  const int blocks =
      (int)std::max<int64_t>(1, std::min<int64_t>(grid_for(max_count, 64), (int64_t)c->wg_per_cu[0] * c->num_cu));
  const int32_t *vsc = vscene_of(sc);
  const int nsc = n_scene_of(sc);
  {
    ProfScope ps(c, kind == 0 ? K_BARRIER_PT : K_BARRIER_EE, s);
#define EIPC_TERMS_LAUNCH(K, R)                                                                                    \
  k_pair_terms<K, R><<<blocks, TERMS_T, 0, s>>>(pairs, act, typ, vid4, d_count, cap, sc->faces, sc->edges, xs,        \
                                                sc->x_rest, sc->n_vert, dhat, kappa, flags, want_g, want_h, energy, \
                                                rec, vsc, nsc, c->status, sc->W_rowptr, sc->W_col, sc->W_val)
    const bool reduced = want_h && (flags & EIPC_PROJECT_REDUCED);
    if (kind == 0) {
      if (reduced)
        EIPC_TERMS_LAUNCH(0, true);
      else
        EIPC_TERMS_LAUNCH(0, false);
    } else {
      if (reduced)
        EIPC_TERMS_LAUNCH(1, true);
      else
        EIPC_TERMS_LAUNCH(1, false);
    }
#undef EIPC_TERMS_LAUNCH
    EIPC_HIP(c, hipGetLastError());
  }
  if (!want_g && !want_h) return EIPC_OK;
  return launch_expand(c, sc, kind, vid4, d_count, cap, rec, want_g, want_h, want_g ? grad : nullptr,
                       want_h ? h : HessOut{}, s);
}

eipc_status launch_expand(eipc_ctx *c, const eipc_scene *sc, int kind, const int4 *vid4, const int64_t *d_count,
                          int64_t cap, const double *rec, bool want_g, bool want_h, double *grad, const HessOut &h,
                          hipStream_t s) {
  if (sc->n_node >= (1 << 27)) return set_err(c, EIPC_ERR_ARG, "n_node must be below 2^27");
  const int blocks =
      (int)std::max<int64_t>(1, std::min<int64_t>(grid_for(cap, 64), (int64_t)c->wg_per_cu[1] * c->num_cu));
  ProfScope ps(c, kind == 0 ? K_EXPAND_PT : K_EXPAND_EE, s);
  if (kind == 0)
    k_expand<0><<<blocks, EX_T, 0, s>>>(vid4, d_count, sc->W_rowptr, sc->W_col, sc->W_val, sc->n_node, rec, cap,
                                        want_g, want_h, grad, h, c->status);
  else
    k_expand<1><<<blocks, EX_T, 0, s>>>(vid4, d_count, sc->W_rowptr, sc->W_col, sc->W_val, sc->n_node, rec, cap,
                                        want_g, want_h, grad, h, c->status);
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
  __shared__ uint32_t s_gkey[LGT];
  __shared__ double s_gval[LGT * 3];
  __shared__ int s_used;
  LdsTables T{s_gkey, s_gval};
  HessOut none{0, nullptr, nullptr, nullptr, 0};
  Acc A{T, none, n_node, out, status};
  const bool moll = (KIND == 1) && (flags & EIPC_MOLLIFY) && x_rest;
  for (int t = threadIdx.x; t < LGT; t += BR_THREADS) s_gkey[t] = 0xffffffffu;
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
      double eps = 0.0;
      if (moll) {
        V3 r[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          r[a] = V3{x_rest[3 * (int64_t)vid[a]], x_rest[3 * (int64_t)vid[a] + 1], x_rest[3 * (int64_t)vid[a] + 2]};
        eps = mollifier_eps(r);
      }
      // the Hessian of the barrier stage's per-class path
      double gam[9], M[45];
      pair_qterms<KIND>(pair_class<KIND>(ty, x, eps), ty, x, eps, dhat, kappa, false, true,
                        (flags & EIPC_PROJECT) != 0, (flags & EIPC_SQDIST) != 0, gam, M);
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
      for (int t = threadIdx.x; t < LGT; t += BR_THREADS) cnt += s_gkey[t] != 0xffffffffu;
      if (cnt) atomicAdd(&s_used, cnt);
      __syncthreads();
    }
    if (last || s_used > LGT / 2) {
      for (int t = threadIdx.x; t < LGT; t += BR_THREADS) {
        const int key = (int)s_gkey[t];
        if (key != -1) {
          atomicAdd(&out[3 * (int64_t)key], s_gval[3 * t]);
          atomicAdd(&out[3 * (int64_t)key + 1], s_gval[3 * t + 1]);
          atomicAdd(&out[3 * (int64_t)key + 2], s_gval[3 * t + 2]);
          s_gkey[t] = 0xffffffffu;
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
__global__ __launch_bounds__(64) void k_pair_eval(int64_t n, const int32_t *__restrict__ pairs, const int32_t *__restrict__ faces,
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
  // the barrier stage's own per-class path; x-space gradient g_x = Q gamma
  double gam[9], M[45];
  double ev = 0.0;
  if (active) {
    const int cls = pair_class<KIND>(ty, x, eps);
    ev = pair_qterms<KIND>(cls, ty, x, eps, dhat, kappa, true, true, (flags & EIPC_PROJECT) != 0,
                           (flags & EIPC_SQDIST) != 0, gam, M);
  }
  if (e) e[i] = ev;
  if (g) {
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        if (active)
          for (int al = 0; al < 3; ++al) acc += (0.5 * kS[a][al]) * gam[3 * al + c];
        g[12 * i + 3 * a + c] = acc;
      }
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
