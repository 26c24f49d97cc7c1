// Embedding, scans, the spatial-hash broad phase and the narrow phase.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "pair_math.h"

namespace eipc {

// ---------------------------------------------------------------------------
// embedding x = W q + off (Eq. 14): CSR order from 0.0, one rounded multiply
// and one rounded add per term, off added last.  Output SoA (and AoS).
// ---------------------------------------------------------------------------
__global__ void k_embed(int n, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                        const double *__restrict__ val, const double *__restrict__ q,
                        const double *__restrict__ off, double *__restrict__ xs, double *__restrict__ x_aos,
                        const int32_t *__restrict__ vscene, int n_scene, uint32_t *status) {
#pragma clang fp contract(off)
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const int k0 = rowptr[v], k1 = rowptr[v + 1];
  if (k1 - k0 > 4 || k1 < k0) atomicOr(status, ST_BAD_W);
  if (vscene && (unsigned)vscene[v] >= (unsigned)n_scene) atomicOr(status, ST_BAD_SCENE);
  for (int k = k0; k < k1; ++k) {
    const double w = val[k];
    const int64_t c = 3 * (int64_t)col[k];
    a0 = a0 + w * q[c];
    a1 = a1 + w * q[c + 1];
    a2 = a2 + w * q[c + 2];
  }
  if (off) {
    a0 = a0 + off[3 * (int64_t)v];
    a1 = a1 + off[3 * (int64_t)v + 1];
    a2 = a2 + off[3 * (int64_t)v + 2];
  }
  if (xs) {
    double2 *r = reinterpret_cast<double2 *>(xs + (int64_t)PSTRIDE * v);
    r[0] = double2{a0, a1};
    r[1] = double2{a2, 0.0};
  }
  if (x_aos) {
    x_aos[3 * (int64_t)v] = a0;
    x_aos[3 * (int64_t)v + 1] = a1;
    x_aos[3 * (int64_t)v + 2] = a2;
  }
  if (!(isfinite(a0) && isfinite(a1) && isfinite(a2))) atomicOr(status, ST_NONFINITE);
}

eipc_status launch_embed(eipc_ctx *c, const eipc_scene *sc, const double *q, const double *off, double *xs,
                         double *x_aos, hipStream_t s) {
  if (sc->n_vert == 0) return EIPC_OK;
  ProfScope ps(c, K_EMBED, s);
  k_embed<<<grid_for(sc->n_vert, 256), 256, 0, s>>>(sc->n_vert, sc->W_rowptr, sc->W_col, sc->W_val, q, off, xs,
                                                     x_aos, vscene_of(sc), n_scene_of(sc), c->status);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

__global__ void k_add(int64_t n, const double *a, const double *b, double *out) {
#pragma clang fp contract(off)
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

eipc_status launch_add_soa(eipc_ctx *c, int64_t n, const double *a, const double *b, double *out, hipStream_t s) {
  if (n == 0) return EIPC_OK;
  k_add<<<grid_for(n, 256), 256, 0, s>>>(n, a, b, out);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

__global__ void k_zero(uint64_t *p, int64_t n64) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n64; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}
__global__ void k_zero_bytes(uint8_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Fill kernel (used instead of hipMemsetAsync so the sequence can be
// captured into a graph).
eipc_status launch_zero(eipc_ctx *c, void *p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return EIPC_OK;
  int64_t n64 = (int64_t)(bytes / 8);
  if (((uintptr_t)p & 7) == 0 && n64 > 0) {
    int g = (int)std::min<int64_t>(grid_for(n64, 256), 4096);
    k_zero<<<g, 256, 0, s>>>((uint64_t *)p, n64);
    EIPC_HIP(c, hipGetLastError());
    size_t rem = bytes - (size_t)n64 * 8;
    if (rem) {
      k_zero_bytes<<<1, 64, 0, s>>>((uint8_t *)p + n64 * 8, (int64_t)rem);
      EIPC_HIP(c, hipGetLastError());
    }
  } else {
    k_zero_bytes<<<grid_for((int64_t)bytes, 256), 256, 0, s>>>((uint8_t *)p, (int64_t)bytes);
    EIPC_HIP(c, hipGetLastError());
  }
  return EIPC_OK;
}

// ---------------------------------------------------------------------------
// exclusive scan: int32 counts[n] -> int64 offsets[n+1] (offsets[n] = total)
// tiles of 2048 elements (256 threads x 8), block sums scanned by one block
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_E = 8, SCAN_TILE = SCAN_T * SCAN_E;

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *smem, int64_t *total) {
  // inclusive wave scan
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) smem[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      int64_t t = smem[w];
      smem[w] = acc;
      acc += t;
    }
    smem[16] = acc;
  }
  __syncthreads();
  int64_t r = x - v + smem[wid];
  *total = smem[16];
  __syncthreads();
  return r;
}

__global__ void k_scan_partial(const int32_t *in, int64_t n, int64_t *bsum) {
  __shared__ int64_t sm[17];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_E;
  int64_t acc = 0;
#pragma unroll
  for (int e = 0; e < SCAN_E; ++e)
    if (base + e < n) acc += in[base + e];
  int64_t tot;
  block_excl_scan(acc, sm, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_top(int64_t *bsum, int64_t nb) {
  __shared__ int64_t sm[17];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += blockDim.x) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < nb ? bsum[i] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan(v, sm, &tot);
    if (i < nb) bsum[i] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void k_scan_final(const int32_t *in, int64_t n, const int64_t *bsum, int64_t nb, int64_t *out) {
  __shared__ int64_t sm[17];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_E;
  int64_t vals[SCAN_E];
  int64_t acc = 0;
#pragma unroll
  for (int e = 0; e < SCAN_E; ++e) {
    vals[e] = (base + e < n) ? in[base + e] : 0;
    acc += vals[e];
  }
  int64_t tot;
  int64_t ex = block_excl_scan(acc, sm, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int e = 0; e < SCAN_E; ++e) {
    if (base + e < n) out[base + e] = ex;
    ex += vals[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

eipc_status exclusive_scan(eipc_ctx *c, const int32_t *in, int64_t n, int64_t *out, hipStream_t s) {
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb < 1) nb = 1;
  int64_t *bsum;
  EIPC_TRY(ensure_t(c, s == c->side ? B_SCANTMP_SIDE : B_SCANTMP, (size_t)nb + 1, &bsum));
  k_scan_partial<<<(unsigned)nb, SCAN_T, 0, s>>>(in, n, bsum);
  EIPC_HIP(c, hipGetLastError());
  k_scan_top<<<1, 1024, 0, s>>>(bsum, nb);
  EIPC_HIP(c, hipGetLastError());
  k_scan_final<<<(unsigned)nb, SCAN_T, 0, s>>>(in, n, bsum, nb, out);
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

// device-side candidate count for the next stage, clamped to the capacity
// (an overflow is raised for the caller to re-plan)
__global__ void k_copy_count(const int64_t *src, int64_t *dst, int64_t cap, uint32_t *status) {
  const int64_t v = *src;
  if (v > cap) atomicOr(status, ST_PLAN_OVERFLOW);
  *dst = v < cap ? v : cap;
}

// ---------------------------------------------------------------------------
// Broad phase.  Boxes: per primitive, lo = min over its vertices (start and
// end positions when swept) - dhat/2, hi = max + dhat/2.  Items (faces for
// PT, edges for EE) are stored as 64-byte records; the uniform grid is a
// hash from (scene, cell) to the items whose boxes touch the cell.  Grid
// parameters are computed on the device, so the sequence can run without
// host synchronization once capacities are known.
// ---------------------------------------------------------------------------
struct ItemRec {
  double lo[3], hi[3];
  int32_t v[3];
  int32_t tag;  // bit 0: some vertex has a DoF; bits 1..: scene id
};

__device__ __forceinline__ bool has_dof(const int32_t *rowptr, int v) { return rowptr[v + 1] > rowptr[v]; }
__device__ __forceinline__ int scene_of(const int32_t *vscene, int v) { return vscene ? vscene[v] : 0; }

template <int NV>
__device__ __forceinline__ void prim_box(const int *vid, const double *xs, const double *x1s, int n_vert, double h,
                                         double *lo, double *hi) {
#pragma clang fp contract(off)
#pragma unroll
  for (int cax = 0; cax < 3; ++cax) {
    double mn = xs[(int64_t)PSTRIDE * vid[0] + cax], mx = mn;
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      double v = xs[(int64_t)PSTRIDE * vid[a] + cax];
      mn = fmin(mn, v);
      mx = fmax(mx, v);
      if (x1s) {
        double w = x1s[(int64_t)PSTRIDE * vid[a] + cax];
        mn = fmin(mn, w);
        mx = fmax(mx, w);
      }
    }
    lo[cax] = mn - h;
    hi[cax] = mx + h;
  }
}

template <int NV>
__global__ void k_items(int n, const int32_t *__restrict__ idx, const double *__restrict__ xs,
                        const double *__restrict__ x1s, int n_vert, double h, const int32_t *__restrict__ rowptr,
                        const int32_t *__restrict__ vscene, ItemRec *__restrict__ rec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int vid[NV];
#pragma unroll
  for (int a = 0; a < NV; ++a) vid[a] = idx[(int64_t)NV * i + a];
  ItemRec r;
  prim_box<NV>(vid, xs, x1s, n_vert, h, r.lo, r.hi);
  int dof = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.v[a] = a < NV ? vid[a] : -1;
    if (a < NV) dof |= has_dof(rowptr, vid[a]);
  }
  r.tag = dof | (scene_of(vscene, vid[0]) << 1);
  rec[i] = r;
}

__device__ __forceinline__ uint64_t ord_key(double v) {
  uint64_t b = __double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_dec(uint64_t k) {
  uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double(b);
}

// stats (uint64 view): [0..2] min lo (ordered), [3..5] max hi (ordered);
// double view [6..8] sum of item extents.  Items from records, or vertex
// (point) boxes when rec == nullptr.  Grid-stride, reduced per workgroup,
// one atomic per workgroup and value.
constexpr int STAT_T = 256;
__global__ __launch_bounds__(STAT_T) void k_box_stats(int n, const ItemRec *__restrict__ rec,
                                                      const double *__restrict__ xs, const double *__restrict__ x1s,
                                                      int n_vert, double h, uint64_t *st, int with_ext) {
  __shared__ double s_red[STAT_T / 64][9];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, ex[3] = {0, 0, 0};
  for (int i = blockIdx.x * STAT_T + threadIdx.x; i < n; i += gridDim.x * STAT_T) {
    double l[3], u[3];
    if (rec) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        l[a] = rec[i].lo[a];
        u[a] = rec[i].hi[a];
      }
    } else {
      int v = i;
      prim_box<1>(&v, xs, x1s, n_vert, h, l, u);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], l[a]);
      hi[a] = fmax(hi[a], u[a]);
      ex[a] += u[a] - l[a];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], __shfl_xor(lo[a], o, 64));
      hi[a] = fmax(hi[a], __shfl_xor(hi[a], o, 64));
      ex[a] += __shfl_xor(ex[a], o, 64);
    }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      s_red[w][a] = lo[a];
      s_red[w][3 + a] = hi[a];
      s_red[w][6 + a] = ex[a];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < STAT_T / 64; ++k)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = fmin(lo[a], s_red[k][a]);
        hi[a] = fmax(hi[a], s_red[k][3 + a]);
        ex[a] += s_red[k][6 + a];
      }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      atomicMin((unsigned long long *)&st[a], (unsigned long long)ord_key(lo[a]));
      atomicMax((unsigned long long *)&st[3 + a], (unsigned long long)ord_key(hi[a]));
      if (with_ext) atomicAdd((double *)&st[6 + a], ex[a]);
    }
  }
}

// a bounded number of workgroups: each ends with 9 atomics on the same 9
// words, and too few leave each thread hundreds of items on large batches
static int stat_blocks(int n) { return std::max(1, std::min(grid_for(n, STAT_T), 256)); }

__global__ void k_stats_init(uint64_t *st) {
  int t = threadIdx.x;
  if (t < 3) {
    st[t] = ~0ull;
    st[3 + t] = 0ull;
    ((double *)st)[6 + t] = 0.0;
  }
}

struct GridDev {
  double o[3];
  double inv_h;
  int dim[3];
  int bad;  // non-finite boxes
};

constexpr int MAX_ITEM_CELLS = 64;
constexpr int BIG_CELLS = 4096;
constexpr int GRID_AXIS_MAX = 1 << 16;

// cell edge: cell_scale times the mean item box extent (largest axis of the
// mean), at least 1e-6 of the scene span, grown until every axis has at
// most 2^16 cells
__global__ void k_grid_params(const uint64_t *st, int n_items, double cell_scale, GridDev *g, uint32_t *status) {
  if (threadIdx.x != 0) return;
  double lo[3], hi[3], ext[3];
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    lo[a] = ord_dec(st[a]);
    hi[a] = ord_dec(st[3 + a]);
    ext[a] = ((const double *)st)[6 + a];
    ok = ok && isfinite(lo[a]) && isfinite(hi[a]);
  }
  GridDev r;
  r.bad = ok ? 0 : 1;
  if (!ok) {
    atomicOr(status, ST_NONFINITE);
    for (int a = 0; a < 3; ++a) {
      lo[a] = 0.0;
      hi[a] = 0.0;
    }
  }
  double cell = cell_scale * fmax(ext[0], fmax(ext[1], ext[2])) / (double)(n_items > 0 ? n_items : 1);
  double span = fmax(hi[0] - lo[0], fmax(hi[1] - lo[1], hi[2] - lo[2]));
  cell = fmax(cell, span * 1e-6);
  if (!(cell > 0.0) || !isfinite(cell)) cell = 1.0;
  for (int it = 0; it < 64; ++it) {
    bool fits = true;
    for (int a = 0; a < 3; ++a)
      if (floor((hi[a] - lo[a]) / cell) + 1.0 > (double)GRID_AXIS_MAX) fits = false;
    if (fits) break;
    cell *= 2.0;
  }
  for (int a = 0; a < 3; ++a) {
    r.o[a] = lo[a];
    double d = floor((hi[a] - lo[a]) / cell) + 1.0;
    r.dim[a] = (int)fmin(d, (double)GRID_AXIS_MAX);
  }
  r.inv_h = 1.0 / cell;
  *g = r;
}

__device__ __forceinline__ int cell_of(double v, double o, double inv_h, int dim) {
#pragma clang fp contract(off)
  double t = floor((v - o) * inv_h);
  int c = t < 0.0 ? 0 : (t > (double)(dim - 1) ? dim - 1 : (int)t);
  return c;
}
__device__ __forceinline__ uint64_t cell_key(int x, int y, int z, int scene) {
  return (uint64_t)x | ((uint64_t)y << 16) | ((uint64_t)z << 32) | ((uint64_t)scene << 48);
}
__device__ __forceinline__ uint32_t cell_hash(int x, int y, int z, int scene) {
  return ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349663u) ^ ((uint32_t)z * 83492791u) ^
         ((uint32_t)scene * 2654435761u);
}
__device__ __forceinline__ void cell_range(const GridDev &g, const double *lo, const double *hi, int *c0, int *c1) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c0[a] = cell_of(lo[a], g.o[a], g.inv_h, g.dim[a]);
    c1[a] = cell_of(hi[a], g.o[a], g.inv_h, g.dim[a]);
  }
}

// Items covering up to MAX_ITEM_CELLS cells are hashed one thread per
// item; larger ones with at most 64 cells per axis (the reach of the 6-bit
// offsets of an entry) and at most BIG_CELLS cells are hashed one wavefront
// per item (the big list, n_big = {items, cells}); the rest (the large
// list) are tested against every query instead.
__global__ void k_item_cells(int n, const ItemRec *__restrict__ rec, const GridDev *__restrict__ gp, int32_t *cnt,
                             int32_t *large, int64_t *n_large, int32_t *big, int64_t *n_big) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GridDev g = *gp;
  int c0[3], c1[3];
  cell_range(g, rec[i].lo, rec[i].hi, c0, c1);
  const int sx = c1[0] - c0[0] + 1, sy = c1[1] - c0[1] + 1, sz = c1[2] - c0[2] + 1;
  const int64_t nc = (int64_t)sx * sy * sz;
  if (nc <= MAX_ITEM_CELLS) {
    cnt[i] = (int32_t)nc;
    return;
  }
  cnt[i] = 0;
  if (sx <= 64 && sy <= 64 && sz <= 64 && nc <= BIG_CELLS) {
    const int slot = (int)atomicAdd((unsigned long long *)&n_big[0], 1ull);
    big[slot] = i;
    atomicAdd((unsigned long long *)&n_big[1], (unsigned long long)nc);
  } else {
    const int slot = (int)atomicAdd((unsigned long long *)n_large, 1ull);
    large[slot] = i;
  }
}

// the cells of a big item, one lane per cell
__device__ __forceinline__ void big_cell(const int *c0, const int *c1, int c, int &x, int &y, int &z) {
  const int sx = c1[0] - c0[0] + 1, sy = c1[1] - c0[1] + 1;
  x = c0[0] + c % sx;
  y = c0[1] + (c / sx) % sy;
  z = c0[2] + c / (sx * sy);
}

__global__ void k_big_hist(const int32_t *__restrict__ big, const int64_t *__restrict__ n_big,
                           const ItemRec *__restrict__ rec, const GridDev *__restrict__ gp, uint32_t bmask,
                           int32_t *bcnt) {
  const int lane = threadIdx.x & 63;
  const int64_t nbig = n_big[0];
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nbig; w += nw) {
    const int i = big[w];
    const GridDev g = *gp;
    const int sc = rec[i].tag >> 1;
    int c0[3], c1[3];
    cell_range(g, rec[i].lo, rec[i].hi, c0, c1);
    const int nc = (c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
    for (int c = lane; c < nc; c += 64) {
      int x, y, z;
      big_cell(c0, c1, c, x, y, z);
      atomicAdd(&bcnt[cell_hash(x, y, z, sc) & bmask], 1);
    }
  }
}

// Workgroup-local bucket table: the items of a workgroup are neighbours
// in mesh order, so their (item, cell) entries fall into few buckets.  Each
// distinct bucket takes one LDS slot (linear probing on the bucket id), the
// entries are counted there, and one global atomic per slot carries the
// count (histogram) or reserves the bucket's range (fill).  An entry whose
// probe finds neither its bucket nor a free slot within LT_PROBE steps goes
// to the global counters directly; its bucket then never enters the table.
constexpr int LT_T = 256;       // items per workgroup
constexpr int LT_SLOTS = 2048;  // LDS table slots
constexpr int LT_PROBE = 32;

__device__ __forceinline__ int lt_insert(uint32_t *key, uint32_t b) {
  uint32_t h = (b * 2654435761u) >> 21;  // 11 bits
  for (int p = 0; p < LT_PROBE; ++p) {
    const uint32_t old = atomicCAS(&key[h], 0u, b + 1u);
    if (old == 0u || old == b + 1u) return (int)h;
    h = (h + 1) & (LT_SLOTS - 1);
  }
  return -1;
}
__device__ __forceinline__ int lt_find(const uint32_t *key, uint32_t b) {
  uint32_t h = (b * 2654435761u) >> 21;
  for (int p = 0; p < LT_PROBE; ++p) {
    const uint32_t k = key[h];
    if (k == b + 1u) return (int)h;
    if (k == 0u) return -1;
    h = (h + 1) & (LT_SLOTS - 1);
  }
  return -1;
}

__global__ __launch_bounds__(LT_T) void k_item_hist(int n, const ItemRec *__restrict__ rec,
                                                    const GridDev *__restrict__ gp, uint32_t bmask,
                                                    const int32_t *cnt, int32_t *bcnt) {
  __shared__ uint32_t s_key[LT_SLOTS];
  __shared__ int32_t s_cnt[LT_SLOTS];
  for (int k = threadIdx.x; k < LT_SLOTS; k += LT_T) {
    s_key[k] = 0u;
    s_cnt[k] = 0;
  }
  __syncthreads();
  const int i = blockIdx.x * LT_T + threadIdx.x;
  if (i < n && cnt[i] != 0) {
    const GridDev g = *gp;
    const int sc = rec[i].tag >> 1;
    int c0[3], c1[3];
    cell_range(g, rec[i].lo, rec[i].hi, c0, c1);
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x) {
          const uint32_t b = cell_hash(x, y, z, sc) & bmask;
          const int t = lt_insert(s_key, b);
          if (t >= 0)
            atomicAdd(&s_cnt[t], 1);
          else
            atomicAdd(&bcnt[b], 1);
        }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < LT_SLOTS; k += LT_T)
    if (s_key[k] != 0u) atomicAdd(&bcnt[s_key[k] - 1u], s_cnt[k]);
}

// Hash entry: one (item, cell) pair.  The offset of the cell from the
// item's lower cell decides the lower-corner rule without the item's record.
struct Entry {
  uint64_t cell;
  int32_t item;
  int32_t dlo;  // cell minus the item's lower cell, 6 bits per axis
};

__global__ __launch_bounds__(LT_T) void k_item_fill(int n, const ItemRec *__restrict__ rec,
                                                    const GridDev *__restrict__ gp, uint32_t bmask,
                                                    const int32_t *cnt, const int64_t *bstart, int32_t *bfill,
                                                    Entry *ent, int64_t ent_cap, uint32_t *status) {
  __shared__ uint32_t s_key[LT_SLOTS];
  __shared__ int32_t s_cnt[LT_SLOTS];
  __shared__ int32_t s_base[LT_SLOTS];
  for (int k = threadIdx.x; k < LT_SLOTS; k += LT_T) {
    s_key[k] = 0u;
    s_cnt[k] = 0;
  }
  __syncthreads();
  const int i = blockIdx.x * LT_T + threadIdx.x;
  const bool live = i < n && cnt[i] != 0;
  GridDev g;
  int sc = 0, c0[3] = {0, 0, 0}, c1[3] = {-1, -1, -1};
  if (live) {
    g = *gp;
    sc = rec[i].tag >> 1;
    cell_range(g, rec[i].lo, rec[i].hi, c0, c1);
  }
  auto put = [&](int64_t slot, int x, int y, int z) {
    if (slot < ent_cap) {
      Entry en;
      en.cell = cell_key(x, y, z, sc);
      en.item = i;
      en.dlo = (x - c0[0]) | ((y - c0[1]) << 6) | ((z - c0[2]) << 12);
      ent[slot] = en;
    } else {
      atomicOr(status, ST_PLAN_OVERFLOW);
    }
  };
  // count per bucket in LDS (entries that find no slot take their global
  // slot now)
  for (int z = c0[2]; z <= c1[2]; ++z)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int x = c0[0]; x <= c1[0]; ++x) {
        const uint32_t b = cell_hash(x, y, z, sc) & bmask;
        const int t = lt_insert(s_key, b);
        if (t >= 0)
          atomicAdd(&s_cnt[t], 1);
        else
          put(bstart[b] + atomicAdd(&bfill[b], 1), x, y, z);
      }
  __syncthreads();
  // reserve each bucket's range once
  for (int k = threadIdx.x; k < LT_SLOTS; k += LT_T)
    if (s_key[k] != 0u) s_base[k] = atomicAdd(&bfill[s_key[k] - 1u], s_cnt[k]);
  __syncthreads();
  // place: rank within the workgroup's range from the LDS count
  for (int z = c0[2]; z <= c1[2]; ++z)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int x = c0[0]; x <= c1[0]; ++x) {
        const uint32_t b = cell_hash(x, y, z, sc) & bmask;
        const int t = lt_find(s_key, b);
        if (t >= 0) put(bstart[b] + s_base[t] + atomicSub(&s_cnt[t], 1) - 1, x, y, z);
      }
}

__global__ void k_big_fill(const int32_t *__restrict__ big, const int64_t *__restrict__ n_big,
                           const ItemRec *__restrict__ rec, const GridDev *__restrict__ gp, uint32_t bmask,
                           const int64_t *bstart, int32_t *bfill, Entry *ent, int64_t ent_cap, uint32_t *status) {
  const int lane = threadIdx.x & 63;
  const int64_t nbig = n_big[0];
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nbig; w += nw) {
    const int i = big[w];
    const GridDev g = *gp;
    const int sc = rec[i].tag >> 1;
    int c0[3], c1[3];
    cell_range(g, rec[i].lo, rec[i].hi, c0, c1);
    const int nc = (c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
    for (int c = lane; c < nc; c += 64) {
      int x, y, z;
      big_cell(c0, c1, c, x, y, z);
      const uint32_t b = cell_hash(x, y, z, sc) & bmask;
      const int64_t slot = bstart[b] + atomicAdd(&bfill[b], 1);
      if (slot < ent_cap) {
        Entry en;
        en.cell = cell_key(x, y, z, sc);
        en.item = i;
        en.dlo = (x - c0[0]) | ((y - c0[1]) << 6) | ((z - c0[2]) << 12);
        ent[slot] = en;
      } else {
        atomicOr(status, ST_PLAN_OVERFLOW);
      }
    }
  }
}

// The hash of n records (count, histogram, scan, fill), small items one
// thread each and big items one wavefront each.
constexpr int BIG_BLOCKS = 256;

__device__ __forceinline__ bool overlap(const double *qlo, const double *qhi, const ItemRec &r) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (!(qlo[a] <= r.hi[a] && r.lo[a] <= qhi[a])) return false;
  return true;
}

template <int KIND>
__device__ __forceinline__ bool pair_ok(int q, int qa, int qb, bool qdof, int it, const ItemRec &r) {
  if (KIND == 1 && it <= q) return false;
  if (KIND == 0) {
    if (qa == r.v[0] || qa == r.v[1] || qa == r.v[2]) return false;
  } else {
    if (qa == r.v[0] || qa == r.v[1] || qb == r.v[0] || qb == r.v[1]) return false;
  }
  return qdof || (r.tag & 1);
}

// Scan the hash entries [e0, e1) of one bucket for the query's cell
// (x, y, z) (key), with the query's lower cell (qx, qy, qz): entries are
// read four at a time (independent loads), filtered on their own fields
// (cell, EE order, lower-corner rule), then the surviving items' records
// are read together and tested exactly; emit(item) for each candidate.
template <int KIND, class Emit>
__device__ __forceinline__ void scan_bucket(const Entry *__restrict__ ent, const ItemRec *__restrict__ items,
                                            int64_t e0, int64_t e1, uint64_t key, int x, int y, int z, int qx,
                                            int qy, int qz, int q, int qa, int qb, bool qdof, const double *qlo,
                                            const double *qhi, Emit emit) {
  for (int64_t e = e0; e < e1; e += 4) {
    Entry en[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (e + u < e1) {
        en[u] = ent[e + u];
      } else {
        en[u].cell = ~0ull;
        en[u].item = 0;
        en[u].dlo = 0;
      }
    }
    bool pass[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int it = en[u].item;
      const int ix = x - (en[u].dlo & 63), iy = y - ((en[u].dlo >> 6) & 63), iz = z - ((en[u].dlo >> 12) & 63);
      // & rather than &&: no branches between the fields' tests
      pass[u] = (en[u].cell == key) & (KIND == 0 || it > q) & ((ix > qx ? ix : qx) == x) &
                ((iy > qy ? iy : qy) == y) & ((iz > qz ? iz : qz) == z);
    }
    ItemRec r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (pass[u]) r[u] = items[en[u].item];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (pass[u] && (pair_ok<KIND>(q, qa, qb, qdof, en[u].item, r[u]) & overlap(qlo, qhi, r[u]))) emit(en[u].item);
  }
}

constexpr int QT = 128;         // query threads per block
constexpr int XCD_CHUNK = 16;   // consecutive query workgroups kept on one XCD
constexpr int APPEND_BUF = 16;  // per-thread LDS staging for append mode

// append mode: stage a candidate in the thread's LDS slots; flush a full
// buffer with one atomic
__device__ __forceinline__ void stage_pair(int2 *buf, int &nb, int q, int it, unsigned long long *total,
                                           int32_t *out, int64_t cap) {
  buf[nb] = make_int2(q, it);
  if (++nb == APPEND_BUF) {
    const int64_t p = (int64_t)atomicAdd(total, (unsigned long long)APPEND_BUF);
    for (int j = 0; j < APPEND_BUF; ++j)
      if (p + j < cap) {
        out[2 * (p + j)] = buf[j].x;
        out[2 * (p + j) + 1] = buf[j].y;
      }
    nb = 0;
  }
}

// Flush every lane's staged pairs with one atomic for the wavefront (all
// lanes of the wavefront must call).
__device__ __forceinline__ void wave_flush(int2 *buf, int &nbuf, unsigned long long *total, int32_t *out,
                                           int64_t cap) {
  const int lane = threadIdx.x & 63;
  int64_t ex = nbuf;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t yv = __shfl_up(ex, o, 64);
    if (lane >= o) ex += yv;
  }
  const int64_t wsum = __shfl(ex, 63, 64);
  int64_t p0 = 0;
  if (lane == 63 && wsum) p0 = (int64_t)atomicAdd(total, (unsigned long long)wsum);
  p0 = __shfl(p0, 63, 64);
  const int64_t p = p0 + ex - nbuf;
  for (int j = 0; j < nbuf; ++j)
    if (p + j < cap) {
      out[2 * (p + j)] = buf[j].x;
      out[2 * (p + j) + 1] = buf[j].y;
    }
  nbuf = 0;
}

struct QueryArgs {
  const GridDev *g;
  uint32_t bmask;
  const int64_t *bstart;
  const Entry *ent;
  int64_t ent_cap;
  const int32_t *large;
  const int64_t *n_large;
  const ItemRec *items;
  const int32_t *rowptr;
  const int32_t *vscene;
  const int32_t *qlist;    // when set: the queries to run, *n_qlist of them
  const int64_t *n_qlist;
  int32_t *defer;          // when set: queries spanning more than LQ_CELLS cells are
  int64_t *n_defer;        // listed here and skipped (k_query_lq runs them)
  int n_items;             // items in the hash (k_query_lq: a query of more cells tests them all)
};

// Queries whose boxes span more than this many cells run one wavefront
// each (k_query_lq) instead of one thread each.
constexpr int LQ_CELLS = 64;

__device__ __forceinline__ int64_t n_cells(const int *c0, const int *c1) {
  return (int64_t)(c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
}

// box, vertices, DoF flag and scene of query q (a vertex for PT, an edge
// record for EE)
template <int KIND>
__device__ __forceinline__ void query_data(int q, const double *xs, const double *x1s, int n_vert, double h,
                                           const QueryArgs &qa_, double *qlo, double *qhi, int &qa, int &qb,
                                           bool &qdof, int &qsc) {
  if (KIND == 0) {
    qa = q;
    qb = -1;
    prim_box<1>(&qa, xs, x1s, n_vert, h, qlo, qhi);
    qdof = has_dof(qa_.rowptr, qa);
    qsc = scene_of(qa_.vscene, qa);
  } else {
    const ItemRec r = qa_.items[q];
    qa = r.v[0];
    qb = r.v[1];
    qdof = r.tag & 1;
    qsc = r.tag >> 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qlo[a] = r.lo[a];
      qhi[a] = r.hi[a];
    }
  }
}

// modes: 0 count, 1 write (offset per query, sorted per query, capacity
// guarded)
template <int KIND, int MODE>
__global__ __launch_bounds__(QT) void k_query(int nq, const double *__restrict__ xs, const double *__restrict__ x1s,
                                              int n_vert, double h, QueryArgs qa_, int32_t *__restrict__ cnt,
                                              const int64_t *__restrict__ off, int32_t *__restrict__ out, int64_t cap,
                                              unsigned long long *total, uint32_t *status) {
  const GridDev g = *qa_.g;
  const ItemRec *items = qa_.items;
  const int nl = (int)*qa_.n_large;  // read before any store: a later load would wait for the stores
  // workgroups of consecutive queries in runs on one XCD (its L2 then holds
  // their hash entries)
  const int t = xcd_block(XCD_CHUNK) * blockDim.x + threadIdx.x;
  const int q = qa_.qlist ? (t < *qa_.n_qlist ? qa_.qlist[t] : -1) : t;
  const bool live = q >= 0 && q < nq;
  int qa = 0, qb = -1, qsc = 0;
  bool qdof = false;
  double qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
  if (live) query_data<KIND>(q, xs, x1s, n_vert, h, qa_, qlo, qhi, qa, qb, qdof, qsc);
  int c0[3] = {0, 0, 0}, c1[3] = {-1, -1, -1};
  if (live) cell_range(g, qlo, qhi, c0, c1);
  if (live && qa_.defer && n_cells(c0, c1) > LQ_CELLS) {
    // a wavefront counts and writes this query (k_query_lq)
    if (MODE == 0) qa_.defer[atomicAdd((unsigned long long *)qa_.n_defer, 1ull)] = q;
    return;
  }
  const int64_t base = (MODE == 1 && live) ? off[q] : 0;
  int64_t k = 0;
  for (int z = c0[2]; z <= c1[2]; ++z)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int x = c0[0]; x <= c1[0]; ++x) {
        const uint64_t key = cell_key(x, y, z, qsc);
        const uint32_t b = cell_hash(x, y, z, qsc) & qa_.bmask;
        const int64_t e1 = qa_.bstart[b + 1] < qa_.ent_cap ? qa_.bstart[b + 1] : qa_.ent_cap;
        // report only in the cell holding the lower corner of the overlap:
        // max(query low cell, item low cell) == this cell on every axis
        scan_bucket<KIND>(qa_.ent, items, qa_.bstart[b], e1, key, x, y, z, c0[0], c0[1], c0[2], q, qa, qb, qdof,
                          qlo, qhi, [&](int it) {
                            if (MODE == 1 && base + k < cap) {
                              out[2 * (base + k)] = q;
                              out[2 * (base + k) + 1] = it;
                            }
                            ++k;
                          });
      }
  if (live) {
    for (int j = 0; j < nl; ++j) {
      const int it = qa_.large[j];
      const ItemRec r = items[it];
      if ((r.tag >> 1) != qsc) continue;
      if (!pair_ok<KIND>(q, qa, qb, qdof, it, r)) continue;
      if (!overlap(qlo, qhi, r)) continue;
      if (MODE == 1 && base + k < cap) {
        out[2 * (base + k)] = q;
        out[2 * (base + k) + 1] = it;
      }
      ++k;
    }
  }
  if (MODE == 0 && live) cnt[q] = (int32_t)k;
  if (MODE == 1 && live) {
    if (base + k > cap) {
      atomicOr(status, ST_PLAN_OVERFLOW);
    } else if (k > 1) {
      int32_t *seg = out + 2 * base;
      for (int64_t i = 1; i < k; ++i) {
        int32_t v = seg[2 * i + 1];
        int64_t j = i - 1;
        while (j >= 0 && seg[2 * j + 1] > v) {
          seg[2 * (j + 1) + 1] = seg[2 * j + 1];
          --j;
        }
        seg[2 * (j + 1) + 1] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Queries whose boxes span more than LQ_CELLS cells (listed by the
// per-query kernels, or too large to bin or hash): one wavefront per query,
// its cells and the items too large to hash spread over the 64 lanes, so
// that one huge box does not keep a single thread scanning thousands of
// cells.  MODE 0 counts each query's candidates into cnt[q]; MODE 1 writes
// them, unsorted, to tmp at the query's offset (k_seg_rank then puts them
// in order into out); MODE 2 appends them to out (staged per lane).
// ---------------------------------------------------------------------------
template <int KIND, int MODE>
__global__ __launch_bounds__(QT) void k_query_lq(const int32_t *__restrict__ qlist, const int64_t *__restrict__ n_qlist,
                                                 const double *__restrict__ xs, const double *__restrict__ x1s,
                                                 int n_vert, double h, QueryArgs qa_, int32_t *__restrict__ cnt,
                                                 const int64_t *__restrict__ off, int32_t *__restrict__ tmp,
                                                 int32_t *__restrict__ out, int64_t cap, unsigned long long *total) {
  __shared__ int2 s_buf[QT * APPEND_BUF];
  int2 *buf = s_buf + threadIdx.x * APPEND_BUF;
  int nbuf = 0;
  const int lane = threadIdx.x & 63;
  const ItemRec *items = qa_.items;
  const GridDev g = *qa_.g;
  const int n_large = (int)*qa_.n_large;
  const int64_t nl = *n_qlist;
  const int64_t nw = ((int64_t)gridDim.x * QT) >> 6;
  for (int64_t w = ((int64_t)blockIdx.x * QT + threadIdx.x) >> 6; w < nl; w += nw) {
    const int q = qlist[w];
    double qlo[3], qhi[3];
    int qa, qb, qsc;
    bool qdof;
    query_data<KIND>(q, xs, x1s, n_vert, h, qa_, qlo, qhi, qa, qb, qdof, qsc);
    int c0[3], c1[3];
    cell_range(g, qlo, qhi, c0, c1);
    const int64_t nx = c1[0] - c0[0] + 1, ny = c1[1] - c0[1] + 1;
    const int64_t nc = n_cells(c0, c1);
    // a query whose cells outnumber the items by a sixteenth tests every
    // item instead, four independent record loads per lane at a time (the
    // same set: the cell scan reports each overlapping item once, the
    // unhashed ones from their list; a cell costs a chain of dependent
    // loads, an item one coalesced load)
    const bool all_items = qa_.n_items > 0 && 16 * nc > (int64_t)qa_.n_items;
    // this lane's share: cells lane, lane + 64, ..., then large items alike
    auto each = [&](auto emit) {
      if (all_items) {
        for (int i0 = 0; i0 < qa_.n_items; i0 += 256) {
          ItemRec r[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int it = i0 + 64 * u + lane;
            r[u] = items[it < qa_.n_items ? it : 0];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int it = i0 + 64 * u + lane;
            // & rather than &&: every record was read, so nothing needs a branch
            if ((it < qa_.n_items) & ((r[u].tag >> 1) == qsc) & pair_ok<KIND>(q, qa, qb, qdof, it, r[u]) &
                overlap(qlo, qhi, r[u]))
              emit(it);
          }
        }
        return;
      }
      for (int64_t ci = lane; ci < nc; ci += 64) {
        const int x = c0[0] + (int)(ci % nx), y = c0[1] + (int)((ci / nx) % ny), z = c0[2] + (int)(ci / (nx * ny));
        const uint64_t key = cell_key(x, y, z, qsc);
        const uint32_t b = cell_hash(x, y, z, qsc) & qa_.bmask;
        const int64_t e1 = qa_.bstart[b + 1] < qa_.ent_cap ? qa_.bstart[b + 1] : qa_.ent_cap;
        scan_bucket<KIND>(qa_.ent, items, qa_.bstart[b], e1, key, x, y, z, c0[0], c0[1], c0[2], q, qa, qb, qdof,
                          qlo, qhi, emit);
      }
      for (int j = lane; j < n_large; j += 64) {
        const int it = qa_.large[j];
        const ItemRec r = items[it];
        if ((r.tag >> 1) == qsc && pair_ok<KIND>(q, qa, qb, qdof, it, r) && overlap(qlo, qhi, r)) emit(it);
      }
    };
    if constexpr (MODE == 2) {
      each([&](int it) { stage_pair(buf, nbuf, q, it, total, out, cap); });
      wave_flush(buf, nbuf, total, out, cap);
    } else {
      int64_t k = 0;
      each([&](int) { ++k; });
      int64_t ex = k;  // inclusive scan over the lanes
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int64_t yv = __shfl_up(ex, o, 64);
        if (lane >= o) ex += yv;
      }
      if constexpr (MODE == 0) {
        if (lane == 63) cnt[q] = (int32_t)ex;
      } else {
        int64_t p = off[q] + ex - k;
        each([&](int it) {
          if (p < cap) tmp[p] = it;
          ++p;
        });
      }
    }
  }
}

// Sorts the candidates of each listed query (tmp, unsorted, at off[q]) into
// out by rank: the items of one query are distinct, so an item's position
// is the number of smaller items, counted against the query's list staged
// through LDS in tiles.  One workgroup per query.
constexpr int RANK_T = 256, RANK_TILE = 2048;
__global__ __launch_bounds__(RANK_T) void k_seg_rank(const int32_t *__restrict__ qlist,
                                                     const int64_t *__restrict__ n_qlist,
                                                     const int32_t *__restrict__ cnt, const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ tmp, int32_t *__restrict__ out,
                                                     int64_t cap) {
  __shared__ int32_t tile[RANK_TILE];
  const int64_t nl = *n_qlist;
  for (int64_t w = blockIdx.x; w < nl; w += gridDim.x) {
    const int q = qlist[w];
    const int64_t o = off[q], L = cnt[q];
    if (o + L > cap) continue;  // the host checked the total against the capacity
    for (int64_t c0 = 0; c0 < L; c0 += RANK_T) {
      const int64_t i = c0 + threadIdx.x;
      const int32_t v = i < L ? tmp[o + i] : 0x7fffffff;
      int64_t rank = 0;
      for (int64_t t0 = 0; t0 < L; t0 += RANK_TILE) {
        const int tn = (int)(L - t0 < RANK_TILE ? L - t0 : RANK_TILE);
        __syncthreads();
        for (int j = threadIdx.x; j < tn; j += RANK_T) tile[j] = tmp[o + t0 + j];
        __syncthreads();
        for (int j = 0; j < tn; ++j) rank += tile[j] < v;
      }
      if (i < L) {
        out[2 * (o + rank)] = q;
        out[2 * (o + rank) + 1] = v;
      }
    }
  }
}

static uint32_t next_pow2(uint64_t v) {
  uint64_t p = 1;
  while (p < v) p <<= 1;
  return (uint32_t)p;
}

template <int KIND, int MODE>
static void launch_query(int nq, const double *xs, const double *x1s, int n_vert, double h, const QueryArgs &qa,
                         int32_t *cnt, const int64_t *off, int32_t *out, int64_t cap, unsigned long long *total,
                         uint32_t *status, hipStream_t s) {
  k_query<KIND, MODE><<<grid_for(nq, QT), QT, 0, s>>>(nq, xs, x1s, n_vert, h, qa, cnt, off, out, cap, total,
                                                       status);
}

// ---------------------------------------------------------------------------
// Cell-parallel query (append mode): one thread per (query, cell of its
// box), listed in query order so that neighbouring threads share the query
// and its neighbourhood (mesh order is spatially coherent).  Queries
// covering more than MAX_ITEM_CELLS cells run per query (k_query on a
// list).
// ---------------------------------------------------------------------------
struct QEntry {
  uint64_t cell;
  int32_t q;
  int32_t dlo;  // cell minus the query's lower cell, 6 bits per axis
};

template <int KIND>
__global__ void k_qcells(int nq, const double *__restrict__ xs, const double *__restrict__ x1s, int n_vert, double h,
                         QueryArgs qa_, int32_t *qcnt, int32_t *qlarge, int64_t *n_qlarge) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const GridDev g = *qa_.g;
  double qlo[3], qhi[3];
  int qa, qb, qsc;
  bool qdof;
  query_data<KIND>(q, xs, x1s, n_vert, h, qa_, qlo, qhi, qa, qb, qdof, qsc);
  int c0[3], c1[3];
  cell_range(g, qlo, qhi, c0, c1);
  const int64_t nc = (int64_t)(c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
  if (nc > MAX_ITEM_CELLS) {
    const int slot = (int)atomicAdd((unsigned long long *)n_qlarge, 1ull);
    qlarge[slot] = q;
    qcnt[q] = 0;
  } else {
    qcnt[q] = (int32_t)nc;
  }
}

template <int KIND>
__global__ void k_qlist(int nq, const double *__restrict__ xs, const double *__restrict__ x1s, int n_vert, double h,
                        QueryArgs qa_, const int32_t *qcnt, const int64_t *qoff, QEntry *qent, int64_t qent_cap,
                        uint32_t *status) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq || qcnt[q] == 0) return;
  const GridDev g = *qa_.g;
  double qlo[3], qhi[3];
  int qa, qb, qsc;
  bool qdof;
  query_data<KIND>(q, xs, x1s, n_vert, h, qa_, qlo, qhi, qa, qb, qdof, qsc);
  int c0[3], c1[3];
  cell_range(g, qlo, qhi, c0, c1);
  int64_t slot = qoff[q];
  for (int z = c0[2]; z <= c1[2]; ++z)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int x = c0[0]; x <= c1[0]; ++x, ++slot) {
        if (slot < qent_cap)
          qent[slot] = QEntry{cell_key(x, y, z, qsc), q, (x - c0[0]) | ((y - c0[1]) << 6) | ((z - c0[2]) << 12)};
        else
          atomicOr(status, ST_PLAN_OVERFLOW);
      }
}

template <int KIND>
__global__ __launch_bounds__(QT) void k_query_ent(const int64_t *__restrict__ n_qent, int64_t qent_cap,
                                                  const QEntry *__restrict__ qent, const double *__restrict__ xs,
                                                  const double *__restrict__ x1s, int n_vert, double h, QueryArgs qa_,
                                                  int32_t *__restrict__ out, int64_t cap, unsigned long long *total) {
  __shared__ int2 s_buf[QT * APPEND_BUF];
  int2 *buf = s_buf + threadIdx.x * APPEND_BUF;
  int nbuf = 0;
  const ItemRec *items = qa_.items;
  const int nl = (int)*qa_.n_large;  // read before any store: a later load would wait for the stores
  const int64_t n = *n_qent < qent_cap ? *n_qent : qent_cap;
  for (int64_t base = (int64_t)blockIdx.x * QT; base < n; base += (int64_t)gridDim.x * QT) {
    const int64_t t = base + threadIdx.x;
    if (t < n) {
      const QEntry qe = qent[t];
      const int q = qe.q;
      double qlo[3], qhi[3];
      int qa, qb, qsc;
      bool qdof;
      query_data<KIND>(q, xs, x1s, n_vert, h, qa_, qlo, qhi, qa, qb, qdof, qsc);
      const int x = (int)(qe.cell & 0xffff), y = (int)((qe.cell >> 16) & 0xffff), z = (int)((qe.cell >> 32) & 0xffff);
      const int qx = x - (qe.dlo & 63), qy = y - ((qe.dlo >> 6) & 63), qz = z - ((qe.dlo >> 12) & 63);
      const uint32_t b = cell_hash(x, y, z, qsc) & qa_.bmask;
      const int64_t e1 = qa_.bstart[b + 1] < qa_.ent_cap ? qa_.bstart[b + 1] : qa_.ent_cap;
      scan_bucket<KIND>(qa_.ent, items, qa_.bstart[b], e1, qe.cell, x, y, z, qx, qy, qz, q, qa, qb, qdof, qlo, qhi,
                        [&](int it) { stage_pair(buf, nbuf, q, it, total, out, cap); });
      if (qe.dlo == 0) {
        // the query's lower cell also runs the items too large to hash
        for (int j = 0; j < nl; ++j) {
          const int it = qa_.large[j];
          const ItemRec r = items[it];
          if ((r.tag >> 1) != qsc) continue;
          if (!pair_ok<KIND>(q, qa, qb, qdof, it, r)) continue;
          if (!overlap(qlo, qhi, r)) continue;
          stage_pair(buf, nbuf, q, it, total, out, cap);
        }
      }
    }
    if (__any(nbuf >= APPEND_BUF / 2)) wave_flush(buf, nbuf, total, out, cap);
  }
  wave_flush(buf, nbuf, total, out, cap);
}

// Wavefront per (query, cell): the 64 lanes read 64 consecutive entries of
// the cell's bucket at once (coalesced), filter them in parallel and test
// the survivors exactly; the query's data is the same for every lane.
// Candidates are staged per lane in LDS as in k_query.  Query cells are
// taken in query order, one per wavefront at a time.
template <int KIND>
__global__ __launch_bounds__(QT) void k_query_wave(const int64_t *__restrict__ n_qent, int64_t qent_cap,
                                                   const QEntry *__restrict__ qent, const double *__restrict__ xs,
                                                   const double *__restrict__ x1s, int n_vert, double h,
                                                   QueryArgs qa_, int32_t *__restrict__ out, int64_t cap,
                                                   unsigned long long *total) {
  __shared__ int2 s_buf[QT * APPEND_BUF];
  int2 *buf = s_buf + threadIdx.x * APPEND_BUF;
  int nbuf = 0;
  const ItemRec *items = qa_.items;
  const int lane = threadIdx.x & 63;
  const int nl = (int)*qa_.n_large;  // read before any store: a later load would wait for the stores
  const int64_t n = *n_qent < qent_cap ? *n_qent : qent_cap;
  const int64_t wave = ((int64_t)blockIdx.x * QT + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * QT) >> 6;
  for (int64_t t = wave; t < n; t += n_waves) {
    const QEntry qe = qent[t];
    const int q = qe.q;
    double qlo[3], qhi[3];
    int qa, qb, qsc;
    bool qdof;
    query_data<KIND>(q, xs, x1s, n_vert, h, qa_, qlo, qhi, qa, qb, qdof, qsc);
    const int x = (int)(qe.cell & 0xffff), y = (int)((qe.cell >> 16) & 0xffff), z = (int)((qe.cell >> 32) & 0xffff);
    const int qx = x - (qe.dlo & 63), qy = y - ((qe.dlo >> 6) & 63), qz = z - ((qe.dlo >> 12) & 63);
    const uint32_t b = cell_hash(x, y, z, qsc) & qa_.bmask;
    const int64_t e0 = qa_.bstart[b];
    const int64_t e1 = qa_.bstart[b + 1] < qa_.ent_cap ? qa_.bstart[b + 1] : qa_.ent_cap;
    for (int64_t base = e0; base < e1; base += 64) {
      const int64_t e = base + lane;
      if (e < e1) {
        const Entry en = qa_.ent[e];
        const int it = en.item;
        // report only in the cell holding the lower corner of the overlap
        const int ix = x - (en.dlo & 63), iy = y - ((en.dlo >> 6) & 63), iz = z - ((en.dlo >> 12) & 63);
        if (en.cell == qe.cell && (KIND == 0 || it > q) && (ix > qx ? ix : qx) == x && (iy > qy ? iy : qy) == y &&
            (iz > qz ? iz : qz) == z) {
          const ItemRec r = items[it];
          if (pair_ok<KIND>(q, qa, qb, qdof, it, r) && overlap(qlo, qhi, r)) buf[nbuf++] = make_int2(q, it);
        }
      }
      if (__any(nbuf >= APPEND_BUF - 1)) wave_flush(buf, nbuf, total, out, cap);
    }
    if (qe.dlo == 0) {
      // the query's lower cell also runs the items too large to hash
      for (int jb = 0; jb < nl; jb += 64) {
        const int j = jb + lane;
        if (j < nl) {
          const int it = qa_.large[j];
          const ItemRec r = items[it];
          if ((r.tag >> 1) == qsc && pair_ok<KIND>(q, qa, qb, qdof, it, r) && overlap(qlo, qhi, r))
            buf[nbuf++] = make_int2(q, it);
        }
        if (__any(nbuf >= APPEND_BUF - 1)) wave_flush(buf, nbuf, total, out, cap);
      }
    }
  }
  wave_flush(buf, nbuf, total, out, cap);
}

// Wavefront-level candidate staging: every lane of the wavefront calls
// push (ok false where it has nothing); positions come from the ballot, so
// the count stays the same on every lane and needs no atomics.  A flush
// reserves the whole staged run with one global atomic and writes it with
// consecutive lanes on consecutive pairs.
__device__ __forceinline__ void wave_push(bool ok, int2 pr, int2 *wout, int &wcnt) {
  const unsigned long long m = __ballot(ok);
  const int lane = threadIdx.x & 63;
  if (ok) wout[wcnt + __popcll(m & ((1ull << lane) - 1ull))] = pr;
  wcnt += __popcll(m);
}
__device__ __forceinline__ void wave_out_flush(int2 *wout, int &wcnt, unsigned long long *total,
                                               int32_t *out, int64_t cap) {
  if (wcnt == 0) return;
  __builtin_amdgcn_wave_barrier();
  const int lane = threadIdx.x & 63;
  int64_t p0 = 0;
  if (lane == 0) p0 = (int64_t)atomicAdd(total, (unsigned long long)wcnt);
  p0 = __shfl(p0, 0, 64);
  int2 *o2 = reinterpret_cast<int2 *>(out);
  for (int k = lane; k < wcnt; k += 64)
    if (p0 + k < cap) o2[p0 + k] = wout[k];
  __builtin_amdgcn_wave_barrier();
  wcnt = 0;
}

// Per-query append (work split 0) as rounds: in each round every lane
// advances its own query by one group of up to four hash entries (or four
// large items), so wavefront-uniform points come often enough to flush
// all lanes' staged pairs with one atomic per wavefront.  Visits the same
// cells, entries and large items in the same order as k_query.
template <int KIND>
__global__ __launch_bounds__(QT) void k_query_sm(int nq, const double *__restrict__ xs,
                                                 const double *__restrict__ x1s, int n_vert, double h, QueryArgs qa_,
                                                 int32_t *__restrict__ out, int64_t cap, unsigned long long *total) {
  __shared__ int2 s_buf[QT * APPEND_BUF];
  int2 *buf = s_buf + threadIdx.x * APPEND_BUF;
  int nbuf = 0;
  const ItemRec *items = qa_.items;
  const int t = xcd_block(XCD_CHUNK) * blockDim.x + threadIdx.x;
  const int q = qa_.qlist ? (t < *qa_.n_qlist ? qa_.qlist[t] : -1) : t;
  const bool live = q >= 0 && q < nq;
  int qa = 0, qb = -1, qsc = 0;
  bool qdof = false;
  double qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
  int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
  bool deferred = false;
  if (live) {
    query_data<KIND>(q, xs, x1s, n_vert, h, qa_, qlo, qhi, qa, qb, qdof, qsc);
    cell_range(*qa_.g, qlo, qhi, c0, c1);
    if (qa_.defer && n_cells(c0, c1) > LQ_CELLS) {
      qa_.defer[atomicAdd((unsigned long long *)qa_.n_defer, 1ull)] = q;  // run by k_query_lq
      deferred = true;
    }
  }
  const int nl = (int)*qa_.n_large;
  int x = c0[0], y = c0[1], z = c0[2];
  int64_t e = 0, e1 = 0;
  uint64_t key = 0;
  int lj = 0;
  int phase = live && !deferred ? 0 : 3;  // 0 open cell, 1 scan its bucket, 2 large items, 3 done
  auto emit = [&](int it) { buf[nbuf++] = make_int2(q, it); };
  while (__any(phase != 3)) {
    if (phase == 0) {
      key = cell_key(x, y, z, qsc);
      const uint32_t b = cell_hash(x, y, z, qsc) & qa_.bmask;
      e = qa_.bstart[b];
      e1 = qa_.bstart[b + 1] < qa_.ent_cap ? qa_.bstart[b + 1] : qa_.ent_cap;
      phase = 1;
    }
    if (phase == 1) {
      if (e < e1) {
        const int64_t eg = e + 4 < e1 ? e + 4 : e1;
        scan_bucket<KIND>(qa_.ent, items, e, eg, key, x, y, z, c0[0], c0[1], c0[2], q, qa, qb, qdof, qlo, qhi, emit);
        e = eg;
      }
      if (e >= e1) {
        if (++x > c1[0]) {
          x = c0[0];
          if (++y > c1[1]) {
            y = c0[1];
            if (++z > c1[2]) phase = 2;
          }
        }
        if (phase == 1) phase = 0;
      }
    } else if (phase == 2) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = lj + u;
        if (j < nl) {
          const int it = qa_.large[j];
          const ItemRec r = items[it];
          if ((r.tag >> 1) == qsc && pair_ok<KIND>(q, qa, qb, qdof, it, r) && overlap(qlo, qhi, r)) emit(it);
        }
      }
      lj += 4;
      if (lj >= nl) phase = 3;
    }
    if (__any(nbuf > APPEND_BUF - 4)) wave_flush(buf, nbuf, total, out, cap);
  }
  wave_flush(buf, nbuf, total, out, cap);
}

// ---------------------------------------------------------------------------
// Bucket join (work split 3).  The queries are hashed like the items (PT:
// vertex records in a second hash over the same grid and buckets; EE: the
// edge hash itself), so every (query, item) pair that shares a cell lies in
// one bucket of both hashes.  A workgroup takes JT consecutive query
// entries (rows, in bucket order); the item entries of the buckets those
// rows touch form one contiguous window of the item hash, staged in LDS in
// chunks of JWIN entries together with their records.  Each row then tests
// the items of its own bucket from LDS: same cell, lower-corner rule
// (min of the two offsets from the lower cells is zero on every axis),
// adjacency and DoF rule, exact box overlap.  EE joins the edge hash with
// itself: each row pairs with about half of its bucket (the entries after
// it, wrapping to the bucket's start), so that every unordered pair of the
// bucket is tested once, and reports (min, max).  The row that is a query's lower cell also runs the
// items too large to hash, as in the per-query splits; queries too large
// to hash run per query (k_query_sm on a list).
// ---------------------------------------------------------------------------
constexpr int JT = 128;     // rows per workgroup
constexpr int JWIN = 192;   // item entries staged in LDS per chunk (five workgroups per CU)
constexpr int JOUT = 1024;  // candidates staged per wavefront

struct JoinArgs {
  const Entry *rows;        // query entries in bucket order
  const int64_t *n_rows;    // number written (device), clamped to row_cap
  int64_t row_cap;
  const ItemRec *qrec;      // query records (PT: vertex records; EE: items)
  const int64_t *pbstart;   // item-hash bucket offsets (nb + 1)
  const Entry *pent;        // item entries
  int64_t pent_cap;
  const ItemRec *items;
  const int32_t *large;
  const int64_t *n_large;
  uint32_t bmask;
};

__device__ __forceinline__ uint32_t key_bucket(uint64_t key, uint32_t bmask) {
  return cell_hash((int)(key & 0xffff), (int)((key >> 16) & 0xffff), (int)((key >> 32) & 0xffff), (int)(key >> 48)) &
         bmask;
}

// lower-corner rule from the two offsets (cell minus lower cell, 6 bits per
// axis): on every axis one of the two offsets is zero.  With the row's
// nonzero fields as a mask (all ones in each such field) it is one AND per
// partner: (partner offsets & mask) == 0
__device__ __forceinline__ int nonzero_fields(int d) {
  return ((d & 63) != 0 ? 63 : 0) | ((d & (63 << 6)) != 0 ? 63 << 6 : 0) | ((d & (63 << 12)) != 0 ? 63 << 12 : 0);
}

// adjacency, DoF rule and exact box overlap of a (query, item) pair, with
// bitwise logic so that no part of it branches
template <int KIND>
__device__ __forceinline__ bool join_test(const ItemRec &r, int qa, int qb, bool qdof, const double *qlo,
                                          const double *qhi) {
  bool ok = (qa != r.v[0]) & (qa != r.v[1]);
  if (KIND == 0)
    ok &= qa != r.v[2];
  else
    ok &= (qb != r.v[0]) & (qb != r.v[1]);
  ok &= qdof | ((r.tag & 1) != 0);
  ok &= (qlo[0] <= r.hi[0]) & (r.lo[0] <= qhi[0]) & (qlo[1] <= r.hi[1]) & (r.lo[1] <= qhi[1]) &
        (qlo[2] <= r.hi[2]) & (r.lo[2] <= qhi[2]);
  return ok;
}

template <int KIND>
__global__ __launch_bounds__(JT) void k_join(JoinArgs ja, int32_t *__restrict__ out, int64_t cap,
                                             unsigned long long *total) {
  __shared__ Entry s_ent[JWIN];
  __shared__ ItemRec s_rec[JWIN];
  __shared__ int2 s_out[JT / 64][JOUT];
  __shared__ int64_t s_win[2];
  int2 *wout = s_out[threadIdx.x >> 6];
  int wcnt = 0;
  const int64_t nr0 = *ja.n_rows;
  // read here, not after the scan: a late load of it waited for all of the
  // wavefront's stores, which kept finished wavefronts resident
  const int nl = (int)*ja.n_large;
  const int64_t n_rows = nr0 < ja.row_cap ? nr0 : ja.row_cap;
  const int64_t r0 = (int64_t)blockIdx.x * JT;
  if (r0 >= n_rows) return;  // uniform over the workgroup
  const int64_t r1 = r0 + JT < n_rows ? r0 + JT : n_rows;
  const int64_t i = r0 + threadIdx.x;
  const bool live = i < r1;
  // the row: its entry, bucket, record and partner range
  Entry re{0, 0, 0};
  // partners: the entries [pa0, pa1) and then [pb0, pb1) of the row's
  // bucket [bs, be).  PT: the whole bucket.  EE: the next h entries after
  // the row, cyclically (wrapping to the bucket's start), with h = (n - 1)
  // / 2 for a bucket of n entries, plus one for the first half of an even
  // bucket (its partner n / 2 ahead): every unordered pair of the bucket
  // once, and every row about half the bucket, where scanning all later
  // entries left the first rows of a bucket with all of it.
  int64_t pa0 = 0, pa1 = 0, pb0 = 0, pb1 = 0, bs = 0, be = 0;
  double qlo[3] = {0, 0, 0}, qhi[3] = {0, 0, 0};
  int qa = 0, qb = -1, qsc = 0;
  bool qdof = false;
  if (live) {
    re = ja.rows[i];
    const uint32_t b = key_bucket(re.cell, ja.bmask);
    const int64_t e0 = ja.pbstart[b], e1 = ja.pbstart[b + 1];
    be = e1 < ja.pent_cap ? e1 : ja.pent_cap;
    bs = e0 < be ? e0 : be;
    if (KIND == 0) {
      pa0 = bs;
      pa1 = be;
    } else {
      const int64_t n = be - bs, pos = i - bs;
      const int64_t h = (n - 1) / 2 + ((n % 2 == 0 && pos < n / 2) ? 1 : 0);
      pa0 = i + 1;
      pa1 = i + 1 + h < be ? i + 1 + h : be;
      pb0 = bs;
      pb1 = bs + (i + 1 + h - be > 0 ? i + 1 + h - be : 0);
    }
    const ItemRec qr = ja.qrec[re.item];
    qa = qr.v[0];
    qb = qr.v[1];
    qdof = qr.tag & 1;
    qsc = qr.tag >> 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qlo[a] = qr.lo[a];
      qhi[a] = qr.hi[a];
    }
  }
  // window of item entries for the whole tile: first row's bucket start to
  // last row's bucket end (rows are in bucket order)
  const int rmask = nonzero_fields(re.dlo);
  if (threadIdx.x == 0) s_win[0] = bs;
  if (i == r1 - 1) s_win[1] = be;
  __syncthreads();
  const int64_t w0 = s_win[0], w1 = s_win[1];
  for (int64_t c0 = w0; c0 < w1; c0 += JWIN) {
    const int nw = (int)(w1 - c0 < JWIN ? w1 - c0 : JWIN);
    __syncthreads();  // previous chunk consumed
    {
      constexpr int U = (JWIN + JT - 1) / JT;
      Entry e[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = u * JT + threadIdx.x;
        if (k < nw) e[u] = ja.pent[c0 + k];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = u * JT + threadIdx.x;
        if (k < nw) {
          s_ent[k] = e[u];
          s_rec[k] = ja.items[e[u].item];
        }
      }
    }
    __syncthreads();
    // this chunk's part of the two partner ranges, taken as one list
    const int64_t cend = c0 + nw;
    const int64_t a0 = pa0 > c0 ? pa0 : c0, a1 = pa1 < cend ? pa1 : cend;
    const int64_t b0 = pb0 > c0 ? pb0 : c0, b1 = pb1 < cend ? pb1 : cend;
    // chunk-relative: the list's entry tu is ra + tu below na, else rb + tu
    const int na = a1 > a0 ? (int)(a1 - a0) : 0;
    const int ntot = na + (b1 > b0 ? (int)(b1 - b0) : 0);
    const int ra = (int)(a0 - c0), rb = (int)(b0 - c0) - na;
    int t = 0;
    while (__any(t < ntot)) {
      // four partners per lane: their entries and records read from LDS
      // without conditions (a conditional read kept the previous records
      // live in registers: ~45 copies per step and 200 VGPRs), then the
      // same-cell and lower-corner rule and the pair test
      Entry pe[4];
      bool pass[4];
      int idx[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int tu = t + u;
        idx[u] = tu < ntot ? (tu < na ? ra : rb) + tu : 0;
        pe[u] = s_ent[idx[u]];
      }
      ItemRec r[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) r[u] = s_rec[idx[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        pass[u] = (t + u < ntot) & (pe[u].cell == re.cell) & ((pe[u].dlo & rmask) == 0);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // & rather than &&: the test is branch-free, a short circuit would branch
        const bool ok = pass[u] & join_test<KIND>(r[u], qa, qb, qdof, qlo, qhi);
        const int it = pe[u].item;
        const int2 pr = (KIND == 0 || re.item < it) ? make_int2(re.item, it) : make_int2(it, re.item);
        wave_push(ok, pr, wout, wcnt);
      }
      t += 4;
      if (wcnt > JOUT - 4 * 64) wave_out_flush(wout, wcnt, total, out, cap);
    }
  }
  // the query's lower-cell row also runs the items too large to hash
  if (nl > 0) {
    const bool lower = live && re.dlo == 0;
    const int q = re.item;
    for (int jb = 0; __any(lower && jb < nl); jb += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jj = jb + u;
        bool ok = false;
        int it = 0;
        if (lower && jj < nl) {
          it = ja.large[jj];
          const ItemRec r = ja.items[it];
          ok = ((r.tag >> 1) == qsc) & pair_ok<KIND>(q, qa, qb, qdof, it, r) & overlap(qlo, qhi, r);
        }
        wave_push(ok, make_int2(q, it), wout, wcnt);
      }
      if (wcnt > JOUT - 4 * 64) wave_out_flush(wout, wcnt, total, out, cap);
    }
  }
  wave_out_flush(wout, wcnt, total, out, cap);
}

// vertex records for the PT query hash (box of the point, swept when x1s)
__global__ void k_vert_items(int n, const double *__restrict__ xs, const double *__restrict__ x1s, int n_vert,
                             double h, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ vscene,
                             ItemRec *__restrict__ rec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ItemRec r;
  prim_box<1>(&i, xs, x1s, n_vert, h, r.lo, r.hi);
  r.v[0] = i;
  r.v[1] = -1;
  r.v[2] = -1;
  r.tag = (int)has_dof(rowptr, i) | (scene_of(vscene, i) << 1);
  rec[i] = r;
}

// Scratch of one broad phase (kind, swept) kept in the context's buffers.
struct BPScratch {
  ItemRec *items;
  int32_t *cnt, *large, *bcnt, *bfill, *qcnt, *qlarge;
  int64_t *cell_off, *bstart, *qoff, *n_large, *n_qlarge;
  Entry *ent;
  QEntry *qent;
  int32_t *big, *qbig;
  int64_t *n_big, *n_qbig;  // {items, cells}
  ItemRec *vrec;     // bucket join, PT: vertex records
  int64_t *vbstart;  // bucket join, PT: vertex-hash bucket offsets
  GridDev *g;
  uint64_t *st;
  unsigned long long *total;
};

static eipc_status bp_scratch(eipc_ctx *c, int nq, int ni, uint32_t nb, int64_t ent_cap, int slot, BPScratch &b,
                              int64_t qent_cap = 1) {
  const int base = slot * BP_NBUF;
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 0), (size_t)ni, &b.items));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 1), (size_t)ni, &b.cnt));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 2), (size_t)ni, &b.large));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 3), (size_t)ni + 1, &b.cell_off));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 4), (size_t)nb, &b.bcnt));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 5), (size_t)nb, &b.bfill));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 6), (size_t)nb + 1, &b.bstart));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 7), (size_t)std::max<int64_t>(ent_cap, 1), &b.ent));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 8), (size_t)nq, &b.qcnt));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 9), (size_t)nq + 1, &b.qoff));
  char *small;
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 10), 512, &small));
  b.g = (GridDev *)small;
  b.st = (uint64_t *)(small + 128);
  b.n_large = (int64_t *)(small + 256);
  b.total = (unsigned long long *)(small + 264);
  b.n_qlarge = (int64_t *)(small + 272);
  b.n_big = (int64_t *)(small + 280);
  b.n_qbig = (int64_t *)(small + 296);
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 11), (size_t)nq, &b.qlarge));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 12), (size_t)std::max<int64_t>(qent_cap, 1), &b.qent));
  const bool vhash = (slot & 1) == 0 && c->query_mode[0] == 3;
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 13), vhash ? (size_t)nq : 1, &b.vrec));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 14), vhash ? (size_t)nb + 1 : 1, &b.vbstart));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 15), (size_t)ni, &b.big));
  EIPC_TRY(ensure_t(c, (BufId)(B_BP0 + base + 16), vhash ? (size_t)nq : 1, &b.qbig));
  return EIPC_OK;
}

eipc_status broad_phase(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const double *x1s,
                        double dhat, int32_t *out, int64_t cap, int64_t *n_out, int sort, hipStream_t s,
                        int grow_id, int32_t **grown, const BPPlan *plan, int64_t *d_total) {
  const int nq = kind == 0 ? sc->n_vert : sc->n_edge;
  const int ni = kind == 0 ? sc->n_face : sc->n_edge;
  const int slot = kind + 2 * (x1s != nullptr);
  if (n_out) *n_out = 0;
  if (nq == 0 || ni == 0) {
    if (d_total) EIPC_TRY(launch_zero(c, d_total, 8, s));
    if (!plan) c->last_plan[slot] = BPPlan{1024, 1, 0, 1};
    return EIPC_OK;
  }
  const double h = 0.5 * dhat;
  const int32_t *vsc = sc->n_scene > 1 ? sc->vert_scene : nullptr;
  // phase 1: items, statistics, grid parameters, cell counts (always)
  BPScratch b;
  uint32_t nb = plan ? plan->nb : 1024;
  int64_t ent_cap = plan ? plan->ent_cap : 1;
  EIPC_TRY(bp_scratch(c, nq, ni, nb, ent_cap, slot, b, plan ? plan->qent_cap : 1));
  if (kind == 0)
    k_items<3><<<grid_for(ni, 256), 256, 0, s>>>(ni, sc->faces, xs, x1s, sc->n_vert, h, sc->W_rowptr, vsc, b.items);
  else
    k_items<2><<<grid_for(ni, 256), 256, 0, s>>>(ni, sc->edges, xs, x1s, sc->n_vert, h, sc->W_rowptr, vsc, b.items);
  EIPC_HIP(c, hipGetLastError());
  k_stats_init<<<1, 64, 0, s>>>(b.st);
  k_box_stats<<<stat_blocks(ni), STAT_T, 0, s>>>(ni, b.items, nullptr, nullptr, 0, h, b.st, 1);
  if (kind == 0) k_box_stats<<<stat_blocks(nq), STAT_T, 0, s>>>(nq, nullptr, xs, x1s, sc->n_vert, h, b.st, 0);
  k_grid_params<<<1, 64, 0, s>>>(b.st, ni, c->cell_scale, b.g, c->status);
  EIPC_TRY(launch_zero(c, b.n_large, 56, s));
  k_item_cells<<<grid_for(ni, 256), 256, 0, s>>>(ni, b.items, b.g, b.cnt, b.large, b.n_large, b.big, b.n_big);
  EIPC_HIP(c, hipGetLastError());
  EIPC_TRY(exclusive_scan(c, b.cnt, ni, b.cell_off, s));
  if (!plan) {
    // size the hash from the entry count (synchronizes)
    int64_t hv[2];
    int64_t hbig[2];
    GridDev gh;
    EIPC_HIP(c, hipMemcpyAsync(&hv[0], b.cell_off + ni, 8, hipMemcpyDeviceToHost, s));
    EIPC_HIP(c, hipMemcpyAsync(hbig, b.n_big, 16, hipMemcpyDeviceToHost, s));
    EIPC_HIP(c, hipMemcpyAsync(&gh, b.g, sizeof(GridDev), hipMemcpyDeviceToHost, s));
    EIPC_HIP(c, hipStreamSynchronize(s));
    if (gh.bad) {
      EIPC_TRY(launch_zero(c, c->status, 4, s));  // reported here instead
      return set_err(c, EIPC_ERR_NONFINITE, "non-finite primitive boxes");
    }
    hv[0] += hbig[1];
    ent_cap = std::max<int64_t>(hv[0], 1);
    nb = (uint32_t)hash_buckets(hv[0]);
    EIPC_TRY(bp_scratch(c, nq, ni, nb, ent_cap, slot, b));
    c->last_plan[slot].nb = nb;
    c->last_plan[slot].ent_cap = ent_cap;
  }
  const uint32_t bmask = nb - 1;
  EIPC_TRY(launch_zero(c, b.bcnt, sizeof(int32_t) * nb, s));
  EIPC_TRY(launch_zero(c, b.bfill, sizeof(int32_t) * nb, s));
  k_item_hist<<<grid_for(ni, LT_T), LT_T, 0, s>>>(ni, b.items, b.g, bmask, b.cnt, b.bcnt);
  k_big_hist<<<BIG_BLOCKS, 256, 0, s>>>(b.big, b.n_big, b.items, b.g, bmask, b.bcnt);
  EIPC_HIP(c, hipGetLastError());
  EIPC_TRY(exclusive_scan(c, b.bcnt, nb, b.bstart, s));
  k_item_fill<<<grid_for(ni, LT_T), LT_T, 0, s>>>(ni, b.items, b.g, bmask, b.cnt, b.bstart, b.bfill, b.ent, ent_cap,
                                                 c->status);
  k_big_fill<<<BIG_BLOCKS, 256, 0, s>>>(b.big, b.n_big, b.items, b.g, bmask, b.bstart, b.bfill, b.ent, ent_cap,
                                        c->status);
  EIPC_HIP(c, hipGetLastError());
  QueryArgs qa{b.g, bmask, b.bstart, b.ent, ent_cap, b.large, b.n_large, b.items, sc->W_rowptr, vsc, nullptr,
               nullptr, nullptr, nullptr, ni};
  QueryArgs qdef = qa;  // per-query kernels hand queries of many cells to k_query_lq
  qdef.defer = b.qlarge;
  qdef.n_defer = b.n_qlarge;
  const int glq = 2 * c->num_cu;
  const int n_vert = sc->n_vert;
  if (!sort) {
    // single pass, unsorted append; per query, per (query, cell) or as a
    // bucket join
    const int qmode = c->query_mode[kind];
    const bool cellpar = qmode == 1 || qmode == 2;
    int64_t qent_cap = plan ? plan->qent_cap : 1;
    const int gq = grid_for(nq, 256);
    if (qmode == 3) {
      if (kind == 0) {
        // vertex hash over the same grid and buckets as the faces
        k_vert_items<<<gq, 256, 0, s>>>(nq, xs, x1s, n_vert, h, sc->W_rowptr, vsc, b.vrec);
        k_item_cells<<<gq, 256, 0, s>>>(nq, b.vrec, b.g, b.qcnt, b.qlarge, b.n_qlarge, b.qbig, b.n_qbig);
        EIPC_HIP(c, hipGetLastError());
        if (!plan) {
          EIPC_TRY(exclusive_scan(c, b.qcnt, nq, b.qoff, s));
          int64_t tq = 0, tbig[2];
          EIPC_HIP(c, hipMemcpyAsync(&tq, b.qoff + nq, 8, hipMemcpyDeviceToHost, s));
          EIPC_HIP(c, hipMemcpyAsync(tbig, b.n_qbig, 16, hipMemcpyDeviceToHost, s));
          EIPC_HIP(c, hipStreamSynchronize(s));
          qent_cap = std::max<int64_t>(tq + tbig[1], 1);
          c->last_plan[slot].qent_cap = qent_cap;
          EIPC_TRY(bp_scratch(c, nq, ni, nb, ent_cap, slot, b, qent_cap));
        }
        EIPC_TRY(launch_zero(c, b.bcnt, sizeof(int32_t) * nb, s));
        EIPC_TRY(launch_zero(c, b.bfill, sizeof(int32_t) * nb, s));
        k_item_hist<<<grid_for(nq, LT_T), LT_T, 0, s>>>(nq, b.vrec, b.g, bmask, b.qcnt, b.bcnt);
        k_big_hist<<<BIG_BLOCKS, 256, 0, s>>>(b.qbig, b.n_qbig, b.vrec, b.g, bmask, b.bcnt);
        EIPC_HIP(c, hipGetLastError());
        EIPC_TRY(exclusive_scan(c, b.bcnt, nb, b.vbstart, s));
        k_item_fill<<<grid_for(nq, LT_T), LT_T, 0, s>>>(nq, b.vrec, b.g, bmask, b.qcnt, b.vbstart, b.bfill,
                                       reinterpret_cast<Entry *>(b.qent), qent_cap, c->status);
        k_big_fill<<<BIG_BLOCKS, 256, 0, s>>>(b.qbig, b.n_qbig, b.vrec, b.g, bmask, b.vbstart, b.bfill,
                                              reinterpret_cast<Entry *>(b.qent), qent_cap, c->status);
        EIPC_HIP(c, hipGetLastError());
      } else if (!plan) {
        c->last_plan[slot].qent_cap = 1;
      }
    } else if (!cellpar) {
      if (!plan) c->last_plan[slot].qent_cap = 1;
    } else {
    if (kind == 0)
      k_qcells<0><<<gq, 256, 0, s>>>(nq, xs, x1s, n_vert, h, qa, b.qcnt, b.qlarge, b.n_qlarge);
    else
      k_qcells<1><<<gq, 256, 0, s>>>(nq, xs, x1s, n_vert, h, qa, b.qcnt, b.qlarge, b.n_qlarge);
    EIPC_HIP(c, hipGetLastError());
    EIPC_TRY(exclusive_scan(c, b.qcnt, nq, b.qoff, s));
    if (!plan) {
      int64_t tq = 0;
      EIPC_HIP(c, hipMemcpyAsync(&tq, b.qoff + nq, 8, hipMemcpyDeviceToHost, s));
      EIPC_HIP(c, hipStreamSynchronize(s));
      qent_cap = std::max<int64_t>(tq, 1);
      c->last_plan[slot].qent_cap = qent_cap;
      EIPC_TRY(bp_scratch(c, nq, ni, nb, ent_cap, slot, b, qent_cap));
    }
    if (kind == 0)
      k_qlist<0><<<gq, 256, 0, s>>>(nq, xs, x1s, n_vert, h, qa, b.qcnt, b.qoff, b.qent, qent_cap, c->status);
    else
      k_qlist<1><<<gq, 256, 0, s>>>(nq, xs, x1s, n_vert, h, qa, b.qcnt, b.qoff, b.qent, qent_cap, c->status);
    EIPC_HIP(c, hipGetLastError());
    }
    QueryArgs qlq = qa;  // queries too large to bin, run per query
    qlq.qlist = b.qlarge;
    qlq.n_qlist = b.n_qlarge;
    int64_t capa = cap;
    if (plan) {
      capa = plan->cand_cap;
    } else if (grow_id >= 0) {
      capa = (int64_t)(c->buf[grow_id].bytes / 8);
      if (capa > 64) capa -= 16;
      EIPC_TRY(ensure_t(c, (BufId)grow_id, (size_t)std::max<int64_t>(2 * capa, 2), &out));
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
      EIPC_TRY(launch_zero(c, b.total, 8, s));
      {
        ProfScope ps(c, kind == 0 ? K_QUERY_WRITE_PT : K_QUERY_WRITE_EE, s);
        const int ge = (int)std::min<int64_t>(grid_for(qent_cap, QT), 64 * (int64_t)c->num_cu);
        if (qmode == 3) {
          QueryArgs qlj = qa;  // queries too large to hash, run per query
          if (kind == 0) {
            const JoinArgs ja{reinterpret_cast<const Entry *>(b.qent), b.vbstart + nb, qent_cap, b.vrec, b.bstart,
                              b.ent, ent_cap, b.items, b.large, b.n_large, bmask};
            k_join<0><<<grid_for(qent_cap, JT), JT, 0, s>>>(ja, out, capa, b.total);
            qlj.qlist = b.qlarge;
            qlj.n_qlist = b.n_qlarge;
          } else {
            const JoinArgs ja{b.ent, b.bstart + nb, ent_cap, b.items, b.bstart, b.ent, ent_cap, b.items, b.large,
                              b.n_large, bmask};
            k_join<1><<<grid_for(ent_cap, JT), JT, 0, s>>>(ja, out, capa, b.total);
            qlj.qlist = b.large;
            qlj.n_qlist = b.n_large;
          }
          EIPC_HIP(c, hipGetLastError());
          if (kind == 0)
            k_query_lq<0, 2><<<glq, QT, 0, s>>>(qlj.qlist, qlj.n_qlist, xs, x1s, n_vert, h, qa, nullptr, nullptr,
                                                nullptr, out, capa, b.total);
          else
            k_query_lq<1, 2><<<glq, QT, 0, s>>>(qlj.qlist, qlj.n_qlist, xs, x1s, n_vert, h, qa, nullptr, nullptr,
                                                nullptr, out, capa, b.total);
        } else if (!cellpar) {
          // the deferred list is rebuilt by every attempt
          EIPC_TRY(launch_zero(c, b.n_qlarge, 8, s));
          if (kind == 0)
            k_query_sm<0><<<grid_for(nq, QT), QT, 0, s>>>(nq, xs, x1s, n_vert, h, qdef, out, capa, b.total);
          else
            k_query_sm<1><<<grid_for(nq, QT), QT, 0, s>>>(nq, xs, x1s, n_vert, h, qdef, out, capa, b.total);
          EIPC_HIP(c, hipGetLastError());
          if (kind == 0)
            k_query_lq<0, 2><<<glq, QT, 0, s>>>(b.qlarge, b.n_qlarge, xs, x1s, n_vert, h, qa, nullptr, nullptr,
                                                nullptr, out, capa, b.total);
          else
            k_query_lq<1, 2><<<glq, QT, 0, s>>>(b.qlarge, b.n_qlarge, xs, x1s, n_vert, h, qa, nullptr, nullptr,
                                                nullptr, out, capa, b.total);
        } else if (c->query_mode[kind] == 2) {
          const int gw = (int)std::min<int64_t>(grid_for(qent_cap * 64, QT), 32 * (int64_t)c->num_cu);
          if (kind == 0)
            k_query_wave<0><<<gw, QT, 0, s>>>(b.qoff + nq, qent_cap, b.qent, xs, x1s, n_vert, h, qa, out, capa,
                                              b.total);
          else
            k_query_wave<1><<<gw, QT, 0, s>>>(b.qoff + nq, qent_cap, b.qent, xs, x1s, n_vert, h, qa, out, capa,
                                              b.total);
          EIPC_HIP(c, hipGetLastError());
          if (kind == 0)
            k_query_lq<0, 2><<<glq, QT, 0, s>>>(qlq.qlist, qlq.n_qlist, xs, x1s, n_vert, h, qa, nullptr, nullptr,
                                                nullptr, out, capa, b.total);
          else
            k_query_lq<1, 2><<<glq, QT, 0, s>>>(qlq.qlist, qlq.n_qlist, xs, x1s, n_vert, h, qa, nullptr, nullptr,
                                                nullptr, out, capa, b.total);
        } else {
        if (kind == 0)
          k_query_ent<0><<<ge, QT, 0, s>>>(b.qoff + nq, qent_cap, b.qent, xs, x1s, n_vert, h, qa, out, capa,
                                           b.total);
        else
          k_query_ent<1><<<ge, QT, 0, s>>>(b.qoff + nq, qent_cap, b.qent, xs, x1s, n_vert, h, qa, out, capa,
                                           b.total);
        EIPC_HIP(c, hipGetLastError());
        if (kind == 0)
          k_query_lq<0, 2><<<glq, QT, 0, s>>>(qlq.qlist, qlq.n_qlist, xs, x1s, n_vert, h, qa, nullptr, nullptr,
                                              nullptr, out, capa, b.total);
        else
          k_query_lq<1, 2><<<glq, QT, 0, s>>>(qlq.qlist, qlq.n_qlist, xs, x1s, n_vert, h, qa, nullptr, nullptr,
                                              nullptr, out, capa, b.total);
        }
      }
      EIPC_HIP(c, hipGetLastError());
      if (plan) {
        // device-side count for the consumer; overflow is detected there
        k_copy_count<<<1, 1, 0, s>>>((const int64_t *)b.total, d_total, capa, c->status);
        EIPC_HIP(c, hipGetLastError());
        return EIPC_OK;
      }
      int64_t total = 0;
      EIPC_HIP(c, hipMemcpyAsync(&total, b.total, 8, hipMemcpyDeviceToHost, s));
      EIPC_HIP(c, hipStreamSynchronize(s));
      if (n_out) *n_out = total;
      if (total <= capa) {
        if (grown) *grown = out;
        c->last_plan[slot].cand_cap = total;
        return EIPC_OK;
      }
      if (grow_id < 0) return EIPC_ERR_CAPACITY;
      capa = total + total / 4 + 1024;
      EIPC_TRY(ensure_t(c, (BufId)grow_id, (size_t)2 * capa, &out));
    }
    return set_err(c, EIPC_ERR_CAPACITY, "candidate append did not converge");
  }
  {
    ProfScope ps(c, kind == 0 ? K_QUERY_COUNT_PT : K_QUERY_COUNT_EE, s);
    if (kind == 0) {
      launch_query<0, 0>(nq, xs, x1s, n_vert, h, qdef, b.qcnt, nullptr, nullptr, 0, nullptr, c->status, s);
      k_query_lq<0, 0><<<glq, QT, 0, s>>>(b.qlarge, b.n_qlarge, xs, x1s, n_vert, h, qa, b.qcnt, nullptr, nullptr,
                                          nullptr, 0, nullptr);
    } else {
      launch_query<1, 0>(nq, xs, x1s, n_vert, h, qdef, b.qcnt, nullptr, nullptr, 0, nullptr, c->status, s);
      k_query_lq<1, 0><<<glq, QT, 0, s>>>(b.qlarge, b.n_qlarge, xs, x1s, n_vert, h, qa, b.qcnt, nullptr, nullptr,
                                          nullptr, 0, nullptr);
    }
  }
  EIPC_HIP(c, hipGetLastError());
  EIPC_TRY(exclusive_scan(c, b.qcnt, nq, b.qoff, s));
  if (plan) {
    cap = plan->cand_cap;
  } else {
    int64_t total = 0;
    EIPC_HIP(c, hipMemcpyAsync(&total, b.qoff + nq, 8, hipMemcpyDeviceToHost, s));
    EIPC_HIP(c, hipStreamSynchronize(s));
    if (n_out) *n_out = total;
    c->last_plan[slot].cand_cap = total;
    if (grow_id >= 0) {
      EIPC_TRY(ensure_t(c, (BufId)grow_id, (size_t)std::max<int64_t>(2 * total, 2), &out));
      cap = total;
      *grown = out;
    }
    if (total > cap || out == nullptr) return total > cap ? EIPC_ERR_CAPACITY : EIPC_OK;
    if (total == 0) return EIPC_OK;
  }
  {
    int32_t *tmp;
    EIPC_TRY(ensure_t(c, B_LQTMP, (size_t)std::max<int64_t>(cap, 1), &tmp));
    ProfScope ps(c, kind == 0 ? K_QUERY_WRITE_PT : K_QUERY_WRITE_EE, s);
    if (kind == 0) {
      launch_query<0, 1>(nq, xs, x1s, n_vert, h, qdef, b.qcnt, b.qoff, out, cap, nullptr, c->status, s);
      k_query_lq<0, 1><<<glq, QT, 0, s>>>(b.qlarge, b.n_qlarge, xs, x1s, n_vert, h, qa, nullptr, b.qoff, tmp,
                                          nullptr, cap, nullptr);
    } else {
      launch_query<1, 1>(nq, xs, x1s, n_vert, h, qdef, b.qcnt, b.qoff, out, cap, nullptr, c->status, s);
      k_query_lq<1, 1><<<glq, QT, 0, s>>>(b.qlarge, b.n_qlarge, xs, x1s, n_vert, h, qa, nullptr, b.qoff, tmp,
                                          nullptr, cap, nullptr);
    }
    k_seg_rank<<<glq, RANK_T, 0, s>>>(b.qlarge, b.n_qlarge, b.qcnt, b.qoff, tmp, out, cap);
  }
  EIPC_HIP(c, hipGetLastError());
  if (plan) {
    k_copy_count<<<1, 1, 0, s>>>(b.qoff + nq, d_total, cap, c->status);
    EIPC_HIP(c, hipGetLastError());
  }
  return EIPC_OK;
}

// ---------------------------------------------------------------------------
// narrow phase: distance type and d^2 per candidate; active (0 < d < dhat)
// pairs compacted by wavefront ballots into a workgroup stage in LDS and
// appended with one atomic per stage flush.
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ void pair_vids(const int32_t *pairs, int64_t k, const int32_t *faces,
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

constexpr int NARROW_BUF = 1024;  // staged active pairs per workgroup (256 threads)

template <int KIND, bool FILTER>
__global__ void k_narrow(int64_t cap, const int64_t *d_n, const int32_t *__restrict__ pairs,
                         const int32_t *__restrict__ faces, const int32_t *__restrict__ edges,
                         const double *__restrict__ xs, int n_vert, double dhat2, double h,
                         int32_t *__restrict__ act, int32_t *__restrict__ typ, int64_t act_cap, int64_t *count,
                         int64_t *cand_count, uint32_t *status) {
  // active pairs staged in LDS and appended with one atomic per workgroup
  // flush (one atomic per wavefront on the shared counter serialises)
  __shared__ int2 s_act[NARROW_BUF];
  __shared__ int s_nact;
  __shared__ int64_t s_abase;
  const int64_t n = d_n ? (*d_n < cap ? *d_n : cap) : cap;
  const int lane = threadIdx.x & 63;
  int64_t n_cand = 0;
  if (threadIdx.x == 0) s_nact = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    bool active = false;
    int ty = 0;
    if (i < n) {
      int vid[4];
      pair_vids<KIND>(pairs, i, faces, edges, vid);
      V3 x[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) ld_pos(xs, vid[a], x[a].x, x[a].y, x[a].z);
      const bool cand = !FILTER || static_boxes_overlap<KIND>(x, h);
      if (cand) {
        ++n_cand;
        double s2 = pair_dist2<KIND>(x, &ty);
        if (!isfinite(s2)) {
          atomicOr(status, ST_NONFINITE);
        } else if (s2 < dhat2) {
          if (s2 <= 0.0)
            atomicOr(status, ST_INTERSECTING);
          else
            active = true;
        }
      }
    }
    const uint64_t mask = __ballot(active);
    int p0 = 0;
    if (lane == 0 && mask) p0 = atomicAdd(&s_nact, (int)__popcll(mask));
    p0 = __shfl(p0, 0, 64);
    if (active) s_act[p0 + __popcll(mask & ((1ull << lane) - 1ull))] = make_int2((int)i, ty);
    __syncthreads();
    const int na = s_nact;
    __syncthreads();  // every thread has read the count before it changes
    // flush when another round could overfill the stage, and at the end
    if (na > NARROW_BUF - (int)blockDim.x || base + stride >= n) {
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
  if (FILTER) {
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
}

eipc_status launch_narrow(eipc_ctx *c, const eipc_scene *sc, int kind, const double *xs, const int32_t *pairs,
                          int64_t n, double dhat, int32_t *act, int32_t *typ, int64_t *d_count, hipStream_t s,
                          const int64_t *d_n, int64_t act_cap, int64_t *cand_count) {
  if (n == 0) return EIPC_OK;
  const double d2 = dhat * dhat;
  const double h = 0.5 * dhat;
  if (act_cap < 0) act_cap = n;
  const int blocks = (int)std::min<int64_t>(grid_for(n, 256), (int64_t)c->wg_per_cu[2] * c->num_cu);
  ProfScope ps(c, kind == 0 ? K_NARROW_PT : K_NARROW_EE, s);
  if (cand_count) {
    if (kind == 0)
      k_narrow<0, true><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, sc->n_vert, d2, h, act, typ,
                                               act_cap, d_count, cand_count, c->status);
    else
      k_narrow<1, true><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, sc->n_vert, d2, h, act, typ,
                                               act_cap, d_count, cand_count, c->status);
  } else {
    if (kind == 0)
      k_narrow<0, false><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, sc->n_vert, d2, h, act,
                                                typ, act_cap, d_count, nullptr, c->status);
    else
      k_narrow<1, false><<<blocks, 256, 0, s>>>(n, d_n, pairs, sc->faces, sc->edges, xs, sc->n_vert, d2, h, act,
                                                typ, act_cap, d_count, nullptr, c->status);
  }
  EIPC_HIP(c, hipGetLastError());
  return EIPC_OK;
}

}  // namespace eipc
