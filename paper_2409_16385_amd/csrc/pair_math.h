// Per-pair device math for the contact stage (gfx950, FP64).
//
// Two kinds of code live here:
//  * exact code (embedding sums, boxes, distance classification and the
//    squared-distance value, the CCD advancement loop) is compiled with
//    contraction off so each expression is one rounded operation per
//    operator, evaluated as written;
//  * derivative code (distance derivatives, barrier chain rule, mollifier,
//    the 9x9 eigen-projection) lets the compiler fuse multiply-adds.
//
// A pair has four vertex slots: PT (p, t0, t1, t2), EE (a0, a1, b0, b1).
// All pair quantities are translation invariant, so derivatives are taken in
// a 9-dimensional basis of difference vectors
//   PT: Y = (p - t0, t1 - t0, t2 - t0),   EE: Y = (a0 - b0, a1 - a0, b1 - b0)
// and the 12x12 Hessian is H_x = T^T H_Y T with T the fixed 9x12 difference
// map.  Its PSD projection is taken in an orthonormal basis Q (12x9, entries
// +-1/2, Hadamard columns orthogonal to translations):
//   P_x = Q proj(Q^T H_x Q) Q^T,   Q^T H_x Q = G^T H_Y G,  G = T Q.
// Since H_x vanishes on translations this equals the projection of the full
// 12x12 matrix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eipc {

struct V3 {
  double x, y, z;
};

// ---------------------------------------------------------------------------
// exact helpers (contraction off)
// ---------------------------------------------------------------------------
__device__ __forceinline__ V3 xsub(V3 a, V3 b) {
#pragma clang fp contract(off)
  return V3{a.x - b.x, a.y - b.y, a.z - b.z};
}
__device__ __forceinline__ double xdot(V3 a, V3 b) {
#pragma clang fp contract(off)
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
__device__ __forceinline__ V3 xcross(V3 a, V3 b) {
#pragma clang fp contract(off)
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// ---------------------------------------------------------------------------
// distance types and their canonical squared-distance formulas
//   PP      s = r.r                r = x[plus0] - x[minus0]
//   PL      s = |r x e|^2 / e.e    r = x[plus0]-x[minus0], e = x[plus1]-x[minus1]
//   TRIPLE  s = (y0.(y1 x y2))^2 / |y1 x y2|^2,  y_j = x[plus_j] - x[minus_j]
// ---------------------------------------------------------------------------
enum { PT_T0 = 0, PT_T1, PT_T2, PT_E0, PT_E1, PT_E2, PT_T };
enum { EE_A0B0 = 0, EE_A0B1, EE_A1B0, EE_A1B1, EE_AB0, EE_AB1, EE_A0B, EE_A1B, EE_AB };
enum { FN_PP = 0, FN_PL = 1, FN_TRI = 2 };

struct TypeDef {
  int fn, m;
  int plus[3], minus[3];
  int c[3][3];  // local vector j as an integer combination of the Y basis
};

// PT slots p=0, t0=1, t1=2, t2=3;  Y = (p-t0, t1-t0, t2-t0)
constexpr TypeDef kPT[7] = {
    {FN_PP, 1, {0, 0, 0}, {1, 0, 0}, {{1, 0, 0}, {0, 0, 0}, {0, 0, 0}}},       // p - t0
    {FN_PP, 1, {0, 0, 0}, {2, 0, 0}, {{1, -1, 0}, {0, 0, 0}, {0, 0, 0}}},      // p - t1
    {FN_PP, 1, {0, 0, 0}, {3, 0, 0}, {{1, 0, -1}, {0, 0, 0}, {0, 0, 0}}},      // p - t2
    {FN_PL, 2, {0, 2, 0}, {1, 1, 0}, {{1, 0, 0}, {0, 1, 0}, {0, 0, 0}}},       // p on t0t1
    {FN_PL, 2, {0, 3, 0}, {2, 2, 0}, {{1, -1, 0}, {0, -1, 1}, {0, 0, 0}}},     // p on t1t2
    {FN_PL, 2, {0, 1, 0}, {3, 3, 0}, {{1, 0, -1}, {0, 0, -1}, {0, 0, 0}}},     // p on t2t0
    {FN_TRI, 3, {0, 2, 3}, {1, 1, 1}, {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}},      // interior
};
// EE slots a0=0, a1=1, b0=2, b1=3;  Y = (a0-b0, a1-a0, b1-b0)
constexpr TypeDef kEE[9] = {
    {FN_PP, 1, {0, 0, 0}, {2, 0, 0}, {{1, 0, 0}, {0, 0, 0}, {0, 0, 0}}},       // a0 - b0
    {FN_PP, 1, {0, 0, 0}, {3, 0, 0}, {{1, 0, -1}, {0, 0, 0}, {0, 0, 0}}},      // a0 - b1
    {FN_PP, 1, {1, 0, 0}, {2, 0, 0}, {{1, 1, 0}, {0, 0, 0}, {0, 0, 0}}},       // a1 - b0
    {FN_PP, 1, {1, 0, 0}, {3, 0, 0}, {{1, 1, -1}, {0, 0, 0}, {0, 0, 0}}},      // a1 - b1
    {FN_PL, 2, {2, 1, 0}, {0, 0, 0}, {{-1, 0, 0}, {0, 1, 0}, {0, 0, 0}}},      // b0 on a
    {FN_PL, 2, {3, 1, 0}, {0, 0, 0}, {{-1, 0, 1}, {0, 1, 0}, {0, 0, 0}}},      // b1 on a
    {FN_PL, 2, {0, 3, 0}, {2, 2, 0}, {{1, 0, 0}, {0, 0, 1}, {0, 0, 0}}},       // a0 on b
    {FN_PL, 2, {1, 3, 0}, {2, 2, 0}, {{1, 1, 0}, {0, 0, 1}, {0, 0, 0}}},       // a1 on b
    {FN_TRI, 3, {0, 1, 3}, {2, 0, 2}, {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}},      // interior
};

// T: rows of the Y basis over the 4 slots; S: 2*Q (Hadamard signs), Q = S/2
constexpr int kT[2][3][4] = {{{1, -1, 0, 0}, {0, -1, 1, 0}, {0, -1, 0, 1}},
                                        {{1, 0, -1, 0}, {-1, 1, 0, 0}, {0, 0, -1, 1}}};
constexpr int kS[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
// G = T Q: G[J][alpha] = (1/2) sum_a T[J][a] S[a][alpha] (integers)
__host__ __device__ constexpr int gcoef(int kind, int J, int al) {
  return (kT[kind][J][0] * kS[0][al] + kT[kind][J][1] * kS[1][al] + kT[kind][J][2] * kS[2][al] +
          kT[kind][J][3] * kS[3][al]) /
         2;
}

template <int KIND, int TYPE>
__host__ __device__ constexpr TypeDef type_def() {
  if constexpr (KIND == 0)
    return kPT[TYPE];
  else
    return kEE[TYPE];
}

template <int KIND, int TYPE>
__device__ __forceinline__ double type_value_t(const V3 *x) {
#pragma clang fp contract(off)
  constexpr TypeDef t = type_def<KIND, TYPE>();
  V3 y0 = xsub(x[t.plus[0]], x[t.minus[0]]);
  if constexpr (t.fn == FN_PP) {
    return xdot(y0, y0);
  } else if constexpr (t.fn == FN_PL) {
    V3 y1 = xsub(x[t.plus[1]], x[t.minus[1]]);
    V3 c = xcross(y0, y1);
    return xdot(c, c) / xdot(y1, y1);
  } else {
    V3 y1 = xsub(x[t.plus[1]], x[t.minus[1]]);
    V3 y2 = xsub(x[t.plus[2]], x[t.minus[2]]);
    V3 n = xcross(y1, y2);
    double N = xdot(y0, n);
    return (N * N) / xdot(n, n);
  }
}

template <int KIND>
__device__ __forceinline__ double type_value(int type, const V3 *x) {
  if constexpr (KIND == 0) {
    switch (type) {
      case 0: return type_value_t<0, 0>(x);
      case 1: return type_value_t<0, 1>(x);
      case 2: return type_value_t<0, 2>(x);
      case 3: return type_value_t<0, 3>(x);
      case 4: return type_value_t<0, 4>(x);
      case 5: return type_value_t<0, 5>(x);
      default: return type_value_t<0, 6>(x);
    }
  } else {
    switch (type) {
      case 0: return type_value_t<1, 0>(x);
      case 1: return type_value_t<1, 1>(x);
      case 2: return type_value_t<1, 2>(x);
      case 3: return type_value_t<1, 3>(x);
      case 4: return type_value_t<1, 4>(x);
      case 5: return type_value_t<1, 5>(x);
      case 6: return type_value_t<1, 6>(x);
      case 7: return type_value_t<1, 7>(x);
      default: return type_value_t<1, 8>(x);
    }
  }
}

// point-segment sub-feature: 0 endpoint a, 1 endpoint b, 2 interior
__device__ __forceinline__ int point_segment(V3 p, V3 a, V3 b) {
#pragma clang fp contract(off)
  V3 r = xsub(p, a);
  V3 e = xsub(b, a);
  double t = xdot(r, e);
  if (t <= 0.0) return 0;
  double ee = xdot(e, e);
  if (t >= ee) return 1;
  return 2;
}

// PT: interior when the plane projection is strictly inside (Cramer
// numerators against det = |n|^2); else the closest point-segment feature
// over edges t0t1, t1t2, t2t0 (first strict minimum wins).
__device__ __forceinline__ int pt_type(const V3 *x) {
#pragma clang fp contract(off)
  V3 e0 = xsub(x[2], x[1]);
  V3 e1 = xsub(x[3], x[1]);
  V3 r = xsub(x[0], x[1]);
  V3 n = xcross(e0, e1);
  double det = xdot(n, n);
  if (det > 0.0) {
    double a = xdot(e0, e0), b = xdot(e0, e1), c = xdot(e1, e1);
    double d0 = xdot(e0, r), d1 = xdot(e1, r);
    double un = c * d0 - b * d1;
    double vn = a * d1 - b * d0;
    if (un > 0.0 && vn > 0.0 && un + vn < det) return PT_T;
  }
  int best = 0;
  double bs = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ia = 1 + k, ib = 1 + (k + 1) % 3;
    int sub = point_segment(x[0], x[ia], x[ib]);
    int ty = sub == 0 ? (ia - 1) : (sub == 1 ? (ib - 1) : PT_E0 + k);
    double s = type_value<0>(ty, x);
    if (k == 0 || s < bs) {
      best = ty;
      bs = s;
    }
  }
  return best;
}

// EE: interior-interior when not near-parallel (|u x v|^2 > 1e-20 |u|^2
// |v|^2) and both line parameters lie strictly inside (0, 1); else the
// closest endpoint-segment feature in order a0|b, a1|b, b0|a, b1|a.
__device__ __forceinline__ int ee_type(const V3 *x) {
#pragma clang fp contract(off)
  V3 u = xsub(x[1], x[0]);
  V3 v = xsub(x[3], x[2]);
  V3 w = xsub(x[0], x[2]);
  V3 n = xcross(u, v);
  double D = xdot(n, n);
  double a = xdot(u, u), c = xdot(v, v);
  if (D > 1e-20 * a * c) {
    double b = xdot(u, v), d = xdot(u, w), e = xdot(v, w);
    double sn = b * e - c * d;
    double tn = a * e - b * d;
    if (sn > 0.0 && sn < D && tn > 0.0 && tn < D) return EE_AB;
  }
  constexpr int pslot[4] = {0, 1, 2, 3};
  constexpr int sa[4] = {2, 2, 0, 0};
  constexpr int sb[4] = {3, 3, 1, 1};
  constexpr int ty[4][3] = {{EE_A0B0, EE_A0B1, EE_A0B},
                            {EE_A1B0, EE_A1B1, EE_A1B},
                            {EE_A0B0, EE_A1B0, EE_AB0},
                            {EE_A0B1, EE_A1B1, EE_AB1}};
  int best = 0;
  double bs = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int sub = point_segment(x[pslot[k]], x[sa[k]], x[sb[k]]);
    int t = ty[k][sub];
    double s = type_value<1>(t, x);
    if (k == 0 || s < bs) {
      best = t;
      bs = s;
    }
  }
  return best;
}

template <int KIND>
__device__ __forceinline__ int classify(const V3 *x) {
  if constexpr (KIND == 0)
    return pt_type(x);
  else
    return ee_type(x);
}

template <int KIND>
__device__ __forceinline__ double pair_dist2(const V3 *x, int *type_out) {
  int t = classify<KIND>(x);
  *type_out = t;
  return type_value<KIND>(t, x);
}

// ---------------------------------------------------------------------------
// symmetric 9x9 in packed upper storage
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int pidx(int i, int j) {
  return i <= j ? i * 9 - (i * (i - 1)) / 2 + (j - i) : j * 9 - (j * (j - 1)) / 2 + (i - j);
}

__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double comp(V3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// Local derivatives of s for a type in its own local vectors y_0..y_{m-1}:
// gl[3m], Hl[3m][3m] (full, row-major, stride 9).
//   PP:  s = y.y
//   PL:  s = N/D, N = |r x e|^2, D = e.e
//   TRI: s = N^2/D, N = y0.(y1 x y2), D = |y1 x y2|^2
// via  grad s = fN gN + fD gD,
//      hess s = fNN gN gN^T + fND (gN gD^T + gD gN^T) + fDD gD gD^T + fN HN + fD HD.
struct Local {
  double g[9];
  double H[81];
};

__device__ __forceinline__ void skew_into(double *H, int r0, int c0, V3 a, double sgn) {
  // H[r0+i][c0+j] += sgn * [a]_x[i][j]
  H[(r0 + 0) * 9 + c0 + 1] += -sgn * a.z;
  H[(r0 + 0) * 9 + c0 + 2] += sgn * a.y;
  H[(r0 + 1) * 9 + c0 + 0] += sgn * a.z;
  H[(r0 + 1) * 9 + c0 + 2] += -sgn * a.x;
  H[(r0 + 2) * 9 + c0 + 0] += -sgn * a.y;
  H[(r0 + 2) * 9 + c0 + 1] += sgn * a.x;
}

// |y1 x y2|^2: gradient into g[o1..], g[o2..] and Hessian blocks into H.
// The cross product and its norm are formed without contraction, as in the
// squared-distance values: when y1 and y2 are nearly parallel n is far
// smaller than its products, and only the same rounding keeps the
// derivatives consistent with the value (and with the oracle's).
__device__ __forceinline__ double crossnorm2(V3 y1, V3 y2, int o1, int o2, double *g, double *H) {
  V3 n = xcross(y1, y2);
  V3 t1 = cross(y2, n), t2 = cross(n, y1);
  g[o1 + 0] = 2.0 * t1.x; g[o1 + 1] = 2.0 * t1.y; g[o1 + 2] = 2.0 * t1.z;
  g[o2 + 0] = 2.0 * t2.x; g[o2 + 1] = 2.0 * t2.y; g[o2 + 2] = 2.0 * t2.z;
  double a11 = dot(y1, y1), a22 = dot(y2, y2), a12 = dot(y1, y2);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double id = (i == j) ? 1.0 : 0.0;
      H[(o1 + i) * 9 + o1 + j] = 2.0 * (a22 * id - comp(y2, i) * comp(y2, j));
      H[(o2 + i) * 9 + o2 + j] = 2.0 * (a11 * id - comp(y1, i) * comp(y1, j));
      double c = 4.0 * comp(y1, i) * comp(y2, j) - 2.0 * comp(y2, i) * comp(y1, j) - 2.0 * a12 * id;
      H[(o1 + i) * 9 + o2 + j] = c;
      H[(o2 + j) * 9 + o1 + i] = c;
    }
  return xdot(n, n);
}

template <int FN>
__device__ __forceinline__ void local_derivs(const V3 *y, Local &L) {
#pragma unroll
  for (int i = 0; i < 81; ++i) L.H[i] = 0.0;
  if constexpr (FN == FN_PP) {
    L.g[0] = 2.0 * y[0].x; L.g[1] = 2.0 * y[0].y; L.g[2] = 2.0 * y[0].z;
    L.H[0] = 2.0; L.H[10] = 2.0; L.H[20] = 2.0;
    return;
  } else {
    constexpr int nl = FN == FN_PL ? 6 : 9;
    double gN[9] = {0}, gD[9] = {0}, HN[81], HD[81];
#pragma unroll
    for (int i = 0; i < 81; ++i) { HN[i] = 0.0; HD[i] = 0.0; }
    double N, D, fN, fD, fNN, fND, fDD;
    if constexpr (FN == FN_PL) {
      N = crossnorm2(y[0], y[1], 0, 3, gN, HN);
      D = xdot(y[1], y[1]);
      gD[3] = 2.0 * y[1].x; gD[4] = 2.0 * y[1].y; gD[5] = 2.0 * y[1].z;
      HD[3 * 9 + 3] = 2.0; HD[4 * 9 + 4] = 2.0; HD[5 * 9 + 5] = 2.0;
      double iD = 1.0 / D;
      fN = iD;
      fD = -N * iD * iD;
      fNN = 0.0;
      fND = -iD * iD;
      fDD = 2.0 * N * iD * iD * iD;
    } else {
      // the triple product N is small against its terms near the plane:
      // formed as in the value, without contraction
      V3 n = xcross(y[1], y[2]);
      V3 c20 = cross(y[2], y[0]), c01 = cross(y[0], y[1]);
      N = xdot(y[0], n);
      gN[0] = n.x; gN[1] = n.y; gN[2] = n.z;
      gN[3] = c20.x; gN[4] = c20.y; gN[5] = c20.z;
      gN[6] = c01.x; gN[7] = c01.y; gN[8] = c01.z;
      skew_into(HN, 0, 3, y[2], -1.0);
      skew_into(HN, 0, 6, y[1], 1.0);
      skew_into(HN, 3, 6, y[0], -1.0);
#pragma unroll
      for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) HN[i * 9 + j] = HN[j * 9 + i];
      D = crossnorm2(y[1], y[2], 3, 6, gD, HD);
      double iD = 1.0 / D;
      fN = 2.0 * N * iD;
      fD = -(N * N) * iD * iD;
      fNN = 2.0 * iD;
      fND = -2.0 * N * iD * iD;
      fDD = 2.0 * (N * N) * iD * iD * iD;
    }
#pragma unroll
    for (int i = 0; i < nl; ++i) L.g[i] = fN * gN[i] + fD * gD[i];
#pragma unroll
    for (int i = 0; i < nl; ++i)
#pragma unroll
      for (int j = 0; j < nl; ++j)
        L.H[i * 9 + j] = fNN * gN[i] * gN[j] + fND * (gN[i] * gD[j] + gD[i] * gN[j]) + fDD * gD[i] * gD[j] +
                         fN * HN[i * 9 + j] + fD * HD[i * 9 + j];
  }
}

// s-derivatives of one type mapped to the Y basis: gY[9], HY packed[45].
// The local vectors are the value's own differences of the four positions
// x (not combinations of Y), so s and its derivatives see the same inputs.
template <int KIND, int TYPE>
__device__ __forceinline__ void s_derivs_typed(const V3 *x, double *gY, double *HY) {
  constexpr TypeDef t = type_def<KIND, TYPE>();
  V3 y[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) y[j] = (j < t.m) ? xsub(x[t.plus[j]], x[t.minus[j]]) : V3{0, 0, 0};
  Local L;
  local_derivs<t.fn>(y, L);
#pragma unroll
  for (int J = 0; J < 3; ++J)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < t.m; ++j)
        if (t.c[j][J] != 0) acc += t.c[j][J] * L.g[3 * j + i];
      gY[3 * J + i] = acc;
    }
#pragma unroll
  for (int J = 0; J < 3; ++J)
#pragma unroll
    for (int K = J; K < 3; ++K)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          if (J == K && l < i) continue;
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < t.m; ++j)
#pragma unroll
            for (int k = 0; k < t.m; ++k)
              if (t.c[j][J] != 0 && t.c[k][K] != 0) acc += (t.c[j][J] * t.c[k][K]) * L.H[(3 * j + i) * 9 + 3 * k + l];
          HY[pidx(3 * J + i, 3 * K + l)] = acc;
        }
}

// type-dispatched s_derivs_typed over the four positions x
template <int KIND>
__device__ __forceinline__ void s_derivs(int type, const V3 *x, double *gY, double *HY) {
  if constexpr (KIND == 0) {
    switch (type) {
      case 0: s_derivs_typed<0, 0>(x, gY, HY); break;
      case 1: s_derivs_typed<0, 1>(x, gY, HY); break;
      case 2: s_derivs_typed<0, 2>(x, gY, HY); break;
      case 3: s_derivs_typed<0, 3>(x, gY, HY); break;
      case 4: s_derivs_typed<0, 4>(x, gY, HY); break;
      case 5: s_derivs_typed<0, 5>(x, gY, HY); break;
      default: s_derivs_typed<0, 6>(x, gY, HY); break;
    }
  } else {
    switch (type) {
      case 0: s_derivs_typed<1, 0>(x, gY, HY); break;
      case 1: s_derivs_typed<1, 1>(x, gY, HY); break;
      case 2: s_derivs_typed<1, 2>(x, gY, HY); break;
      case 3: s_derivs_typed<1, 3>(x, gY, HY); break;
      case 4: s_derivs_typed<1, 4>(x, gY, HY); break;
      case 5: s_derivs_typed<1, 5>(x, gY, HY); break;
      case 6: s_derivs_typed<1, 6>(x, gY, HY); break;
      case 7: s_derivs_typed<1, 7>(x, gY, HY); break;
      default: s_derivs_typed<1, 8>(x, gY, HY); break;
    }
  }
}

// ---------------------------------------------------------------------------
// barrier (Eq. 7) as a function of s = d^2:  bt(s) = b(sqrt(s))
//   b   = -(d - dhat)^2 ln(d/dhat)
//   b'  = -2 (d - dhat) ln(d/dhat) - (d - dhat)^2 / d
//   b'' = -2 ln(d/dhat) - 4 (d - dhat)/d + (d - dhat)^2/d^2
//   bt' = b'/(2d),  bt'' = (b'' - b'/d) / (4 s)
// ---------------------------------------------------------------------------
struct Barrier {
  double b, bs1, bs2;
};
// sq (alternative formulation): the barrier written in s itself,
//   bt(s) = -(s - shat)^2 ln(s / shat),  shat = dhat^2
__device__ __forceinline__ Barrier barrier_s(double s, double dhat, bool sq) {
  if (sq) {
    const double shat = dhat * dhat;
    const double lr = log(s / shat);
    const double sm = s - shat;
    const double is = 1.0 / s;
    Barrier r;
    r.b = -(sm * sm) * lr;
    r.bs1 = -2.0 * sm * lr - (sm * sm) * is;
    r.bs2 = -2.0 * lr - 4.0 * sm * is + (sm * sm) * is * is;
    return r;
  }
  double d = sqrt(s);
  double lr = log(d / dhat);
  double dm = d - dhat;
  double id = 1.0 / d;
  double b = -(dm * dm) * lr;
  double b1 = -2.0 * dm * lr - (dm * dm) * id;
  double b2 = -2.0 * lr - 4.0 * dm * id + (dm * dm) * id * id;
  Barrier r;
  r.b = b;
  r.bs1 = 0.5 * b1 * id;
  r.bs2 = (b2 - b1 * id) * (0.25 / s);
  return r;
}

// Energy derivatives in the Y basis: e = kappa m(c) bt(s) (m = 1 without
// mollifier).  gE[9], HE packed [45].  eps_x <= 0 disables the mollifier.
// Returns the energy.
// (gs, Hs: the s-derivatives in the Y basis)
template <int KIND>
__device__ __forceinline__ double energy_derivs_gs(const double *gs, const double *Hs, const V3 *Y, double s,
                                                   double dhat, double kappa, double eps_x, double *gE, double *HE,
                                                   bool want_h, bool sq) {
  Barrier br = barrier_s(s, dhat, sq);
  double m = 1.0, m1 = 0.0, m2 = 0.0;
  double gc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double Hc[81];
  bool moll = false;
  if constexpr (KIND == 1) {
    if (eps_x > 0.0) {
      V3 n = xcross(Y[1], Y[2]);
      double c = xdot(n, n);
      if (c < eps_x) {
        moll = true;
        double r = c / eps_x;
        m = (2.0 - r) * r;
        m1 = (2.0 - 2.0 * r) / eps_x;
        m2 = -2.0 / (eps_x * eps_x);
#pragma unroll
        for (int i = 0; i < 81; ++i) Hc[i] = 0.0;
        crossnorm2(Y[1], Y[2], 3, 6, gc, Hc);
      }
    }
  }
  double e = kappa * (m * br.b);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double gb = br.bs1 * gs[i];
    gE[i] = kappa * (moll ? (m * gb + br.b * m1 * gc[i]) : gb);
  }
  if (want_h) {
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
      for (int j = i; j < 9; ++j) {
        double hb = br.bs2 * gs[i] * gs[j] + br.bs1 * Hs[pidx(i, j)];
        double h = hb;
        if (moll) {
          double gbi = br.bs1 * gs[i], gbj = br.bs1 * gs[j];
          h = m * hb + m1 * (gbi * gc[j] + gc[i] * gbj) + br.b * (m2 * gc[i] * gc[j] + m1 * Hc[i * 9 + j]);
        }
        HE[pidx(i, j)] = kappa * h;
      }
  }
  return e;
}

template <int KIND>
__device__ __forceinline__ double energy_derivs(int type, const V3 *x, const V3 *Y, double s, double dhat,
                                                double kappa, double eps_x, double *gE, double *HE, bool want_h,
                                                bool sq) {
  double gs[9], Hs[45];
  s_derivs<KIND>(type, x, gs, Hs);
  return energy_derivs_gs<KIND>(gs, Hs, Y, s, dhat, kappa, eps_x, gE, HE, want_h, sq);
}

// M = G^T H G (packed), G = (T Q) (x) I3 with integer entries gcoef.
template <int KIND>
__device__ __forceinline__ void to_q_basis(const double *H, double *M) {
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int be = al; be < 3; ++be)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (al == be && j < i) continue;
          double acc = 0.0;
#pragma unroll
          for (int J = 0; J < 3; ++J)
#pragma unroll
            for (int K = 0; K < 3; ++K) {
              const int c = gcoef(KIND, J, al) * gcoef(KIND, K, be);
              if (c != 0) acc += c * H[pidx(3 * J + i, 3 * K + j)];
            }
          M[pidx(3 * al + i, 3 * be + j)] = acc;
        }
}

// One Jacobi rotation zeroing a[p][q]; V accumulates the rotations.
// Entries below thr (1e-20 of the matrix norm) are left alone: lanes keep
// sweeping until the whole wavefront has converged, and rotating such
// entries would square values that underflow.
// 1/sqrt(x) and 1/x (x > 0, normal) from the hardware estimates refined by
// two Newton steps (each roughly doubles the correct bits: y <- y (3 - x y^2)
// / 2 and y <- y (2 - x y)), within a few ulp of the correctly rounded
// values at a fraction of their cost.  The Jacobi rotation needs no more:
// its (c, s) stay orthonormal to rounding, and its angle only has to
// shrink the off-diagonal entry, which the sweep loop checks.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
  }
  return y;
}

// packed index of the upper triangle of an N x N symmetric matrix
template <int N>
__host__ __device__ constexpr int pidxn(int i, int j) {
  return i <= j ? i * N - (i * (i - 1)) / 2 + (j - i) : j * N - (j * (j - 1)) / 2 + (i - j);
}

template <int N, int P, int Q>
__device__ __forceinline__ void jacobi_rot(double *a, double *v, double thr) {
  const double apq = a[pidxn<N>(P, Q)];
  const double app = a[pidxn<N>(P, P)];
  const double aqq = a[pidxn<N>(Q, Q)];
  const double h = 0.5 * (aqq - app);
  const double ss = h * h + apq * apq;
  // sqrt(ss) as ss / sqrt(ss); the smallest normal double keeps ss = 0 at 0
  const double r = ss * rsqrt_nr(fmax(ss, 2.2250738585072014e-308));
  const double den = h >= 0.0 ? h + r : h - r;
  // (an infinite den, from entries beyond 1e154, gives t = 0 as apq / den would)
  const double t = (fabs(apq) > thr && den != 0.0 && fabs(den) < INFINITY) ? apq * rcp_nr(den) : 0.0;
  const double c = rsqrt_nr(1.0 + t * t);
  const double s = t * c;
  a[pidxn<N>(P, P)] = app - t * apq;
  a[pidxn<N>(Q, Q)] = aqq + t * apq;
  a[pidxn<N>(P, Q)] = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k == P || k == Q) continue;
    const double akp = a[pidxn<N>(k, P)], akq = a[pidxn<N>(k, Q)];
    a[pidxn<N>(k, P)] = c * akp - s * akq;
    a[pidxn<N>(k, Q)] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double vkp = v[k * N + P], vkq = v[k * N + Q];
    v[k * N + P] = c * vkp - s * vkq;
    v[k * N + Q] = s * vkp + c * vkq;
  }
}

template <int N, int P, int Q>
__device__ __forceinline__ void jacobi_sweep_from(double *a, double *v, double thr) {
  if constexpr (P < N - 1) {
    jacobi_rot<N, P, Q>(a, v, thr);
    if constexpr (Q + 1 < N)
      jacobi_sweep_from<N, P, Q + 1>(a, v, thr);
    else if constexpr (P + 2 < N)
      jacobi_sweep_from<N, P + 1, P + 2>(a, v, thr);
  }
}

// In place on a packed N x N symmetric matrix: a <- V max(L, 0) V^T,
// cyclic Jacobi until the off-diagonal mass is below 1e-30 of the total
// (relative off-norm 1e-15), at most 16 sweeps.  The loop count is uniform
// over the wavefront.
template <int N>
__device__ __forceinline__ void project_psd(double *a) {
  double v[N * N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) v[i * N + j] = (i == j) ? 1.0 : 0.0;
  double fro2 = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) fro2 += (i == j ? 1.0 : 2.0) * a[pidxn<N>(i, j)] * a[pidxn<N>(i, j)];
  const double thr = 1e-20 * sqrt(fro2);
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += a[pidxn<N>(i, j)] * a[pidxn<N>(i, j)];
    const bool done = !(off > 1e-30 * fro2);
    if (__all(done)) break;
    jacobi_sweep_from<N, 0, 1>(a, v, thr);
  }
  double lam[N];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = fmax(a[pidxn<N>(k, k)], 0.0);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += v[i * N + k] * lam[k] * v[j * N + k];
      a[pidxn<N>(i, j)] = acc;
    }
}

__device__ __forceinline__ void project_psd9(double *a) { project_psd<9>(a); }

// Symmetric eigendecomposition of a packed N x N matrix by the same cyclic
// Jacobi sweeps: on return the diagonal of a holds the eigenvalues and the
// columns of v (row-major N x N) the eigenvectors.
template <int N>
__device__ __forceinline__ void jacobi_eig(double *a, double *v) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) v[i * N + j] = (i == j) ? 1.0 : 0.0;
  double fro2 = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) fro2 += (i == j ? 1.0 : 2.0) * a[pidxn<N>(i, j)] * a[pidxn<N>(i, j)];
  const double thr = 1e-20 * sqrt(fro2);
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += a[pidxn<N>(i, j)] * a[pidxn<N>(i, j)];
    if (__all(!(off > 1e-30 * fro2))) break;
    jacobi_sweep_from<N, 0, 1>(a, v, thr);
  }
}

// 3x3 block (a, b) of H_x = Q X Q^T from X packed in the Q basis.
__device__ __forceinline__ void x_block(const double *X, int a, int b, double *B) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) {
          const double x = X[pidx(3 * al + i, 3 * be + j)];
          acc += (kS[a][al] * kS[b][be] > 0) ? x : -x;
        }
      B[i * 3 + j] = 0.25 * acc;
    }
}

// gradient over the 4 slots from the Y basis: g_x[a] = sum_J T[J][a] gY[J]
template <int KIND>
__device__ __forceinline__ void slot_grad(const double *gY, double *gx) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int J = 0; J < 3; ++J)
        if (kT[KIND][J][a] != 0) acc += kT[KIND][J][a] * gY[3 * J + i];
      gx[3 * a + i] = acc;
    }
}

template <int KIND>
__device__ __forceinline__ void y_basis(const V3 *x, V3 *Y) {
  if constexpr (KIND == 0) {
    Y[0] = V3{x[0].x - x[1].x, x[0].y - x[1].y, x[0].z - x[1].z};
    Y[1] = V3{x[2].x - x[1].x, x[2].y - x[1].y, x[2].z - x[1].z};
    Y[2] = V3{x[3].x - x[1].x, x[3].y - x[1].y, x[3].z - x[1].z};
  } else {
    Y[0] = V3{x[0].x - x[2].x, x[0].y - x[2].y, x[0].z - x[2].z};
    Y[1] = V3{x[1].x - x[0].x, x[1].y - x[0].y, x[1].z - x[0].z};
    Y[2] = V3{x[3].x - x[2].x, x[3].y - x[2].y, x[3].z - x[2].z};
  }
}

// mollifier threshold eps_x = 1e-3 |ea_rest|^2 |eb_rest|^2
__device__ __forceinline__ double mollifier_eps(const V3 *r) {
#pragma clang fp contract(off)
  V3 u = xsub(r[1], r[0]);
  V3 v = xsub(r[3], r[2]);
  return 1e-3 * xdot(u, u) * xdot(v, v);
}

// ---------------------------------------------------------------------------
// Pair terms in the Q basis by class of distance type.
//
// With xi the Q-basis coordinates of the pair (x_a = sum_alpha Q[a][alpha]
// xi_alpha + a translation), a type's local vectors are
//   y_j = x[plus_j] - x[minus_j] = sum_alpha E[j][alpha] xi_alpha,
//   E[j][alpha] = (S[plus_j][alpha] - S[minus_j][alpha]) / 2 in {-1, 0, 1},
// so the Q-basis gradient is gamma = (E^T x I3) g_l and the Hessian
// X = (E^T x I3) H_l (E x I3), with g_l, H_l the energy's derivatives in
// the local vectors.  E E^T is the Gram matrix of the types' difference
// rows over the four slots, the same for every type of a class ([2] for
// point-point, [[2,1],[1,2]] for point-line).  With E E^T = L L^T the rows
// of F = L^{-1} E are orthonormal, so F^T x I3 is an isometry and
//   X = (F^T x I3) P (F x I3),  P = (L^T x I3) H_l (L x I3),
//   proj(X) = (F^T x I3) proj(P) (F x I3).
// A point-point pair's H_l = a y y^T + b I is projected in closed form
// (eigenvalues a s + b along y, b across), a point-line pair's 6x6 P by
// Jacobi, and an interior pair's 9x9 X by Jacobi.  Mollified edge-edge
// pairs (whose mollifier involves all four slots) take the general path.
// ---------------------------------------------------------------------------
enum { CLS_PP = 0, CLS_PL = 1, CLS_TRI = 2, CLS_GEN = 3 };

template <int KIND>
__host__ __device__ constexpr int type_fn(int type) {
  return KIND == 0 ? (type < 3 ? FN_PP : (type < 6 ? FN_PL : FN_TRI))
                   : (type < 4 ? FN_PP : (type < 8 ? FN_PL : FN_TRI));
}

// plus/minus slots of the first two local vectors of each point-point and
// point-line type, 2 bits each, 8 bits per type
template <int KIND>
__host__ __device__ constexpr uint64_t slot_codes() {
  uint64_t r = 0;
  const int nt = KIND == 0 ? 6 : 8;
  for (int t = 0; t < nt; ++t) {
    const TypeDef d = KIND == 0 ? kPT[t] : kEE[t];
    const uint64_t c = (uint64_t)d.plus[0] | ((uint64_t)d.minus[0] << 2) | ((uint64_t)d.plus[1] << 4) |
                       ((uint64_t)d.minus[1] << 6);
    r |= c << (8 * t);
  }
  return r;
}

template <int KIND>
__host__ __device__ constexpr bool type_fn_matches_tables() {
  const int nt = KIND == 0 ? 7 : 9;
  for (int t = 0; t < nt; ++t)
    if ((KIND == 0 ? kPT[t].fn : kEE[t].fn) != type_fn<KIND>(t)) return false;
  return true;
}
static_assert(type_fn_matches_tables<0>() && type_fn_matches_tables<1>(), "type classes");

// S[a][alpha] (Hadamard signs) for a runtime slot a
__host__ __device__ constexpr int qsign(int a, int al) {
  return al == 0 ? ((a & 2) ? -1 : 1) : (al == 1 ? ((a & 1) ? -1 : 1) : ((a & 2) ? -1 : 1) * ((a & 1) ? -1 : 1));
}
__host__ __device__ constexpr bool qsign_matches() {
  for (int a = 0; a < 4; ++a)
    for (int al = 0; al < 3; ++al)
      if (qsign(a, al) != kS[a][al]) return false;
  return true;
}
static_assert(qsign_matches(), "Hadamard signs");

__device__ __forceinline__ V3 pick4(const V3 *x, int i) {
  const V3 a = (i & 1) ? x[1] : x[0];
  const V3 b = (i & 1) ? x[3] : x[2];
  return (i & 2) ? b : a;
}

__device__ __forceinline__ void e_row(int p, int m, double *E) {
#pragma unroll
  for (int al = 0; al < 3; ++al) E[al] = 0.5 * (double)(qsign(p, al) - qsign(m, al));
}

// class of a pair: its type's function, or the general path when the
// edge-edge mollifier is active (the same test as in energy_derivs_gs)
template <int KIND>
__device__ __forceinline__ int pair_class(int type, const V3 *x, double eps_x) {
  if constexpr (KIND == 1) {
    if (eps_x > 0.0) {
      V3 Y[3];
      y_basis<1>(x, Y);
      const V3 n = xcross(Y[1], Y[2]);
      if (xdot(n, n) < eps_x) return CLS_GEN;
    }
  }
  return type_fn<KIND>(type);
}

template <int KIND>
__device__ __forceinline__ void grad_to_q(const double *gE, double *gam) {
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
      gam[3 * al + c] = acc;
    }
}

template <int KIND>
__device__ __forceinline__ double terms_pp(int type, const V3 *x, double dhat, double kappa, bool want_g,
                                           bool want_h, bool project, bool sq, double *gam, double *X) {
  const uint32_t code = (uint32_t)(slot_codes<KIND>() >> (8 * type)) & 0xffu;
  const int p0 = code & 3, m0 = (code >> 2) & 3;
  const V3 y = xsub(pick4(x, p0), pick4(x, m0));
  const double s = xdot(y, y);
  const Barrier br = barrier_s(s, dhat, sq);
  double E[3];
  e_row(p0, m0, E);
  if (want_g) {
    const double g[3] = {kappa * (br.bs1 * (2.0 * y.x)), kappa * (br.bs1 * (2.0 * y.y)),
                         kappa * (br.bs1 * (2.0 * y.z))};
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
      for (int c = 0; c < 3; ++c) gam[3 * al + c] = E[al] * g[c];
  }
  if (want_h) {
    // H_l = c1 y y^T + c0 I
    const double a = kappa * (4.0 * br.bs2), b = kappa * (2.0 * br.bs1);
    double c0 = b, c1 = a;
    if (project) {
      const double l1 = fmax(a * s + b, 0.0), l2 = fmax(b, 0.0);
      c0 = l2;
      c1 = (l1 - l2) / s;
    }
    const double yv[3] = {y.x, y.y, y.z};
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
      for (int be = al; be < 3; ++be)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (al == be && c < r) continue;
            const double hl = c1 * yv[r] * yv[c] + (r == c ? c0 : 0.0);
            X[pidx(3 * al + r, 3 * be + c)] = (E[al] * E[be]) * hl;
          }
  }
  return kappa * br.b;
}

template <int KIND>
__device__ __forceinline__ double terms_pl(int type, const V3 *x, double dhat, double kappa, bool want_g,
                                           bool want_h, bool project, bool sq, double *gam, double *X) {
  const uint32_t code = (uint32_t)(slot_codes<KIND>() >> (8 * type)) & 0xffu;
  const int p0 = code & 3, m0 = (code >> 2) & 3, p1 = (code >> 4) & 3, m1 = (code >> 6) & 3;
  V3 y[3];
  y[0] = xsub(pick4(x, p0), pick4(x, m0));
  y[1] = xsub(pick4(x, p1), pick4(x, m1));
  y[2] = V3{0.0, 0.0, 0.0};
  double s;
  {
#pragma clang fp contract(off)
    const V3 cr = xcross(y[0], y[1]);
    s = xdot(cr, cr) / xdot(y[1], y[1]);
  }
  const Barrier br = barrier_s(s, dhat, sq);
  if (!want_g && !want_h) return kappa * br.b;
  Local L;
  local_derivs<FN_PL>(y, L);
  double E[2][3];
  e_row(p0, m0, E[0]);
  e_row(p1, m1, E[1]);
  if (want_g) {
    double gl[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) gl[i] = kappa * (br.bs1 * L.g[i]);
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
      for (int c = 0; c < 3; ++c) gam[3 * al + c] = E[0][al] * gl[c] + E[1][al] * gl[3 + c];
  }
  if (want_h) {
    double H6[21];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i; j < 6; ++j) H6[pidxn<6>(i, j)] = kappa * (br.bs2 * L.g[i] * L.g[j] + br.bs1 * L.H[i * 9 + j]);
    double W[2][3];
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      W[0][al] = E[0][al];
      W[1][al] = E[1][al];
    }
    if (project) {
      // Gram [[2,1],[1,2]] = L L^T, L = [[l00, 0], [l10, l11]]
      constexpr double l00 = 1.4142135623730951, l10 = 0.7071067811865476, l11 = 1.2247448713915890;
      double P[21];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double h00 = H6[pidxn<6>(r, c)], h11 = H6[pidxn<6>(3 + r, 3 + c)];
          const double h01 = H6[pidxn<6>(r, 3 + c)], h10 = H6[pidxn<6>(3 + r, c)];
          if (c >= r) {
            P[pidxn<6>(r, c)] = l00 * l00 * h00 + l00 * l10 * (h01 + h10) + l10 * l10 * h11;
            P[pidxn<6>(3 + r, 3 + c)] = l11 * l11 * h11;
          }
          P[pidxn<6>(r, 3 + c)] = l00 * l11 * h01 + l10 * l11 * h11;
        }
      project_psd<6>(P);
#pragma unroll
      for (int i = 0; i < 21; ++i) H6[i] = P[i];
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        W[0][al] = E[0][al] * (1.0 / l00);
        W[1][al] = (E[1][al] - l10 * W[0][al]) * (1.0 / l11);
      }
    }
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
      for (int be = al; be < 3; ++be)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if (al == be && c < r) continue;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
              for (int k = 0; k < 2; ++k) acc += (W[j][al] * W[k][be]) * H6[pidxn<6>(3 * j + r, 3 * k + c)];
            X[pidx(3 * al + r, 3 * be + c)] = acc;
          }
  }
  return kappa * br.b;
}

template <int KIND>
__device__ __forceinline__ double terms_tri(const V3 *x, double dhat, double kappa, bool want_g, bool want_h,
                                            bool project, bool sq, double *gam, double *X) {
  constexpr int TT = KIND == 0 ? (int)PT_T : (int)EE_AB;
  const double s = type_value_t<KIND, TT>(x);
  if (!want_g && !want_h) return kappa * barrier_s(s, dhat, sq).b;
  double gs[9], Hs[45], gE[9], HE[45];
  s_derivs_typed<KIND, TT>(x, gs, Hs);
  V3 Y[3];
  y_basis<KIND>(x, Y);
  const double e = energy_derivs_gs<KIND>(gs, Hs, Y, s, dhat, kappa, 0.0, gE, HE, want_h, sq);
  if (want_g) grad_to_q<KIND>(gE, gam);
  if (want_h) {
    to_q_basis<KIND>(HE, X);
    if (project) project_psd<9>(X);
  }
  return e;
}

// any type, with the mollifier when eps_x > 0
template <int KIND>
__device__ __forceinline__ double terms_gen(int type, const V3 *x, double eps_x, double dhat, double kappa,
                                            bool want_g, bool want_h, bool project, bool sq, double *gam,
                                            double *X) {
  const double s = type_value<KIND>(type, x);
  V3 Y[3];
  y_basis<KIND>(x, Y);
  double gE[9], HE[45];
  const double e = energy_derivs<KIND>(type, x, Y, s, dhat, kappa, eps_x, gE, HE, want_h, sq);
  if (want_g) grad_to_q<KIND>(gE, gam);
  if (want_h) {
    to_q_basis<KIND>(HE, X);
    if (project) project_psd<9>(X);
  }
  return e;
}

// energy only
template <int KIND>
__device__ __forceinline__ double pair_energy(int type, const V3 *x, double eps_x, double dhat, double kappa,
                                              bool sq) {
  const double s = type_value<KIND>(type, x);
  const Barrier br = barrier_s(s, dhat, sq);
  double m = 1.0;
  if constexpr (KIND == 1) {
    if (eps_x > 0.0) {
      V3 Y[3];
      y_basis<1>(x, Y);
      const V3 n = xcross(Y[1], Y[2]);
      const double c = xdot(n, n);
      if (c < eps_x) {
        const double r = c / eps_x;
        m = (2.0 - r) * r;
      }
    }
  }
  return kappa * (m * br.b);
}

// Energy, Q-basis gradient gamma[9] and Hessian X (packed, 45) of one pair
// of class cls.  Lanes of a wavefront that share the class share the path.
template <int KIND>
__device__ __forceinline__ double pair_qterms(int cls, int type, const V3 *x, double eps_x, double dhat,
                                              double kappa, bool want_g, bool want_h, bool project, bool sq,
                                              double *gam, double *X) {
  if (cls == CLS_PP) return terms_pp<KIND>(type, x, dhat, kappa, want_g, want_h, project, sq, gam, X);
  if (cls == CLS_PL) return terms_pl<KIND>(type, x, dhat, kappa, want_g, want_h, project, sq, gam, X);
  if (cls == CLS_TRI) return terms_tri<KIND>(x, dhat, kappa, want_g, want_h, project, sq, gam, X);
  return terms_gen<KIND>(type, x, eps_x, dhat, kappa, want_g, want_h, project, sq, gam, X);
}

// ---------------------------------------------------------------------------
// CCD: additive conservative advancement for one pair (exact arithmetic,
// same operation sequence as the CPU reference reading):
//   p_i -= mean(p);  l_p = |p0| + max(|p1|,|p2|,|p3|)  (PT)
//                     l_p = max(|p0|,|p1|) + max(|p2|,|p3|) (EE)
//   d = dist(x); g = s d; t = 0; tl = (1 - s) d / l_p
//   loop: x += tl p; d = dist(x); if t > 0 and d < g stop;
//         t += tl; if t > t_c return t_c; tl = 0.9 d / l_p
// ---------------------------------------------------------------------------
// The candidate predicate on the pair's own vertices: the box of the
// query primitive (PT: the vertex, EE: the first edge) against the box of
// the item (the face, the second edge), each spanning its vertices widened
// by h on every side, closed intervals -- the same arithmetic as the broad
// phase's boxes.
template <int KIND>
__device__ __forceinline__ bool static_boxes_overlap(const V3 *x, double h) {
#pragma clang fp contract(off)
  const int nq = KIND == 0 ? 1 : 2;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double qmn = INFINITY, qmx = -INFINITY, imn = INFINITY, imx = -INFINITY;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double v = c == 0 ? x[a].x : (c == 1 ? x[a].y : x[a].z);
      if (a < nq) {
        qmn = fmin(qmn, v);
        qmx = fmax(qmx, v);
      } else {
        imn = fmin(imn, v);
        imx = fmax(imx, v);
      }
    }
    ok = ok & (qmn - h <= imx + h) & (imn - h <= qmx + h);  // & rather than &&: no branch
  }
  return ok;
}

// Narrow phase: distance type and d^2 per pair, active iff 0 < d^2 <
// dhat^2, wavefront-ballot compaction into act/typ (capacity act_cap).
// FILTER: the pairs are swept candidates; only those that pass the
// candidate predicate at the start positions are considered, and their
// number is added to *cand_count.
// Alternative projection: the PSD projection of the pair's reduced local
// block K = Z^T X Z (Z: the 9 x 3m map from the pair's m merged nodes, node
// I's block z_I (x) I3 with z_I = sum_{slots of I} w Q[a]) instead of X.
// With G3 = sum_I z_I z_I^T = V L V^T and R = V L^{1/2}, U = R^+ Z has
// orthonormal rows and Z = (R (x) I3) U, so
//   proj(K) = U^T proj((R^T (x) I3) X (R (x) I3)) U,
// and X is replaced by X_eff = (R^+T (x) I3) proj(X') (R^+ (x) I3) with
// X' = (R^T (x) I3) X (R (x) I3): the reduction B(I, J) = z_I^T X z_J then
// gives proj(K)'s blocks.  G3 = Q^T M Q with M_ab = w_a . w_b, the dot
// products of the four vertices' rows of W; directions of G3 below 1e-12
// of its largest eigenvalue (the z_I have no component there) are dropped.
__device__ __forceinline__ void reduced_block_projection(const double *M4, double *X) {
  // G3 (packed 3x3)
  double G[6];
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int be = al; be < 3; ++be) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc += (0.25 * (double)(qsign(a, al) * qsign(b, be))) * M4[a * 4 + b];
      G[pidxn<3>(al, be)] = acc;
    }
  double V[9];
  jacobi_eig<3>(G, V);
  double lmax = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) lmax = fmax(lmax, G[pidxn<3>(k, k)]);
  double R[9], Rp[9];  // R[al][k], Rp[k][al]
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double lam = G[pidxn<3>(k, k)];
    const bool keep = lam > 1e-12 * lmax;
    const double sq = keep ? sqrt(lam) : 0.0, isq = keep ? 1.0 / sqrt(lam) : 0.0;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
      R[al * 3 + k] = V[al * 3 + k] * sq;
      Rp[k * 3 + al] = V[al * 3 + k] * isq;
    }
  }
  double Xp[45];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = k; l < 3; ++l)
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (k == l && c < r) continue;
          double acc = 0.0;
#pragma unroll
          for (int al = 0; al < 3; ++al)
#pragma unroll
            for (int be = 0; be < 3; ++be) acc += (R[al * 3 + k] * R[be * 3 + l]) * X[pidx(3 * al + r, 3 * be + c)];
          Xp[pidx(3 * k + r, 3 * l + c)] = acc;
        }
  project_psd<9>(Xp);
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int be = al; be < 3; ++be)
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (al == be && c < r) continue;
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) acc += (Rp[k * 3 + al] * Rp[l * 3 + be]) * Xp[pidx(3 * k + r, 3 * l + c)];
          X[pidx(3 * al + r, 3 * be + c)] = acc;
        }
}

// signed closest-point weights of a classified pair at positions x (the
// point minus the closest triangle point for PT, the closest point of edge
// a minus that of edge b for EE: G x = sum_a beta_a x_a), each product and
// sum rounded on its own
template <int KIND>
__device__ __forceinline__ void closest_beta(int type, const V3 *x, double *beta) {
#pragma clang fp contract(off)
  constexpr const TypeDef *defs = KIND == 0 ? kPT : kEE;
  const TypeDef t = defs[type];
  // vertices are picked and weights placed by selects, never by a run-time
  // index into x or beta (which would put both in scratch memory)
  if (t.fn == FN_PP) {
    const int p0 = t.plus[0], m0 = t.minus[0];
#pragma unroll
    for (int a = 0; a < 4; ++a) beta[a] = a == p0 ? 1.0 : (a == m0 ? -1.0 : 0.0);
  } else if (t.fn == FN_PL) {
    // point P = plus[0] against the segment from A = minus[1] to B = plus[1]
    const int p0 = t.plus[0], m1 = t.minus[1], p1 = t.plus[1];
    const V3 y0 = xsub(pick4(x, p0), pick4(x, m1));
    const V3 y1 = xsub(pick4(x, p1), pick4(x, m1));
    const double s = xdot(y0, y1) / xdot(y1, y1);
    const double sg = (KIND == 0 || p0 < 2) ? 1.0 : -1.0;  // the point's side
    const double bp0 = sg, bm1 = -sg * (1.0 - s), bp1 = -sg * s;
#pragma unroll
    for (int a = 0; a < 4; ++a) beta[a] = a == p0 ? bp0 : (a == m1 ? bm1 : (a == p1 ? bp1 : 0.0));
  } else if (KIND == 0) {
    // closest triangle point t0 + u (t1 - t0) + v (t2 - t0)
    const V3 r = xsub(x[0], x[1]), e0 = xsub(x[2], x[1]), e1 = xsub(x[3], x[1]);
    const double a = xdot(e0, e0), b = xdot(e0, e1), c = xdot(e1, e1);
    const double d0 = xdot(e0, r), d1 = xdot(e1, r);
    const double det = a * c - b * b;
    const double u = (c * d0 - b * d1) / det, v = (a * d1 - b * d0) / det;
    beta[0] = 1.0;
    beta[1] = -(1.0 - u - v);
    beta[2] = -u;
    beta[3] = -v;
  } else {
    // closest points a0 + s (a1 - a0) and b0 + t (b1 - b0)
    const V3 u = xsub(x[1], x[0]), v = xsub(x[3], x[2]), w = xsub(x[0], x[2]);
    const double a = xdot(u, u), b = xdot(u, v), c = xdot(v, v), d = xdot(u, w), e = xdot(v, w);
    const double D = a * c - b * b;
    const double s = (b * e - c * d) / D, tt = (a * e - b * d) / D;
    beta[0] = 1.0 - s;
    beta[1] = s;
    beta[2] = -(1.0 - tt);
    beta[3] = -tt;
  }
}

// Rate at which the gap along the pair's current closest direction can
// close under the motion p (conservative advancement after C2A): with n
// the unit vector from the second primitive's closest point to the
// first's, both primitives stay on their sides of the separating planes
// through the closest points, and each point of a primitive is a convex
// combination of its linearly moving vertices, so the distance at any
// later time t' is at least d - mu (t' - t) with
//   mu = max_{b in second} n.p_b - min_{a in first} n.p_a  (<= lp).
template <int KIND>
__device__ __forceinline__ double closing_rate(int type, const V3 *x, const V3 *p) {
#pragma clang fp contract(off)
  double beta[4];
  closest_beta<KIND>(type, x, beta);
  V3 r{0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    r.x += beta[a] * x[a].x;
    r.y += beta[a] * x[a].y;
    r.z += beta[a] * x[a].z;
  }
  const double rn = sqrt(xdot(r, r));
  const V3 n{r.x / rn, r.y / rn, r.z / rn};
  constexpr int nfirst = KIND == 0 ? 1 : 2;
  double amin = INFINITY, bmax = -INFINITY;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double v = n.x * p[a].x + n.y * p[a].y + n.z * p[a].z;
    if (a < nfirst)
      amin = fmin(amin, v);
    else
      bmax = fmax(bmax, v);
  }
  return bmax - amin;
}

// dir: advance with the closing rate along the closest direction (an
// alternative CCD) instead of lp
struct AccdState {
  double lp, g, t, tl;
  int64_t it;
  bool dir;
};

// p made relative to its mean; st.lp = the largest possible rate of
// closing (the point's speed plus the triangle's fastest vertex, or the
// fastest vertex of each edge); st.t = 0, no steps taken.
template <int KIND>
__device__ __forceinline__ void accd_motion(V3 *p, AccdState &st) {
#pragma clang fp contract(off)
  V3 mean;
  mean.x = (((p[0].x + p[1].x) + p[2].x) + p[3].x) * 0.25;
  mean.y = (((p[0].y + p[1].y) + p[2].y) + p[3].y) * 0.25;
  mean.z = (((p[0].z + p[1].z) + p[2].z) + p[3].z) * 0.25;
#pragma unroll
  for (int a = 0; a < 4; ++a) p[a] = xsub(p[a], mean);
  // |p_a| through squared norms: sqrt is monotone and correctly rounded,
  // so sqrt(max(a, b)) == max(sqrt(a), sqrt(b)) exactly
  const double q0 = xdot(p[0], p[0]), q1 = xdot(p[1], p[1]), q2 = xdot(p[2], p[2]), q3 = xdot(p[3], p[3]);
  st.lp = KIND == 0 ? sqrt(q0) + sqrt(fmax(q1, fmax(q2, q3))) : sqrt(fmax(q0, q1)) + sqrt(fmax(q2, q3));
  st.it = 0;
  st.t = 0.0;
}

// Set-up of one pair (p is made relative to its mean).  Returns true when
// the pair is already decided (no relative motion: the bound is t_c).
// known: s2 holds the pair's squared distance at x, already computed (the
// same function of the same x).
template <int KIND>
__device__ __forceinline__ bool accd_init(V3 *x, V3 *p, double s, double t_c, AccdState &st, bool known = false,
                                          double s2 = 0.0) {
#pragma clang fp contract(off)
  accd_motion<KIND>(p, st);
  if (st.lp == 0.0) {
    st.t = t_c;
    return true;
  }
  int ty = 0;
  const double d = sqrt(known ? s2 : pair_dist2<KIND>(x, &ty));
  st.g = s * d;
  double rate = st.lp;
  if (st.dir) {
    if (known) ty = classify<KIND>(x);
    rate = closing_rate<KIND>(ty, x, p);
    if (!(rate > 0.0)) {  // the gap along the closest direction never closes
      st.t = t_c;
      return true;
    }
  }
  st.tl = (1.0 - s) * d / rate;
  return false;
}

// Squared gap between the boxes of the pair's two primitives at x (zero
// when they overlap): a lower bound on the pair's squared distance.
template <int KIND>
__device__ __forceinline__ double box_gap2(const V3 *x) {
#pragma clang fp contract(off)
  const int nq = KIND == 0 ? 1 : 2;
  double g2 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double qmn = INFINITY, qmx = -INFINITY, imn = INFINITY, imx = -INFINITY;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double v = c == 0 ? x[a].x : (c == 1 ? x[a].y : x[a].z);
      if (a < nq) {
        qmn = fmin(qmn, v);
        qmx = fmax(qmx, v);
      } else {
        imn = fmin(imn, v);
        imx = fmax(imx, v);
      }
    }
    const double g = fmax(fmax(imn - qmx, qmn - imx), 0.0);
    g2 = g2 + g * g;
  }
  return g2;
}

enum { ACCD_OPEN = 0, ACCD_DONE = 1, ACCD_DROP = 2 };

// Set-up for the step bound alone (the minimum over pairs), given cut, a
// value that the minimum is already known not to exceed (at most t_c; an
// infinite cut turns the dropping off, up to an infinite first step, which
// the plain set-up decides at t_c, so either way the pair contributes no
// less than t_c).  A pair's
// bound never falls below min(first step, t_c): its first step skips the
// gap test, and later steps only add to st.t.  So a pair whose first step
// is at least cut cannot lower the minimum, and is dropped (ACCD_DROP)
// without further steps.  For a pair whose distance is not yet known the
// test is tried first with the box gap in place of the distance (shrunk by
// a relative 1e-6, far above the rounding error of the gap or of the
// computed distance; rounded products and quotients are monotone, so the
// first step from the gap is no larger than the one from the distance),
// which spares the distance for far pairs.  ACCD_DONE: decided with st.t
// (no relative motion); ACCD_OPEN: advance with accd_step.
template <int KIND>
__device__ __forceinline__ int accd_init_cut(V3 *x, V3 *p, double s, double t_c, double cut, AccdState &st,
                                             bool known, double s2) {
#pragma clang fp contract(off)
  accd_motion<KIND>(p, st);
  if (st.lp == 0.0) {
    st.t = t_c;
    return ACCD_DONE;
  }
  if (!known) {
    const double lb = sqrt(box_gap2<KIND>(x)) * (1.0 - 1e-6);
    if ((1.0 - s) * lb / st.lp >= cut) return ACCD_DROP;
  }
  int ty = 0;
  const double d = sqrt(known ? s2 : pair_dist2<KIND>(x, &ty));
  st.g = s * d;
  double rate = st.lp;
  if (st.dir) {
    // (the box-gap test above used lp >= the closing rate: a first step it
    // drops is no shorter here)
    if (known) ty = classify<KIND>(x);
    rate = closing_rate<KIND>(ty, x, p);
    if (!(rate > 0.0)) {
      st.t = t_c;
      return ACCD_DONE;
    }
  }
  st.tl = (1.0 - s) * d / rate;
  return st.tl >= cut ? ACCD_DROP : ACCD_OPEN;
}

// One advancement step.  Returns true when the pair's bound st.t is final.
template <int KIND>
__device__ __forceinline__ bool accd_step(V3 *x, const V3 *p, double t_c, int64_t max_iter, AccdState &st) {
#pragma clang fp contract(off)
  if (st.it >= max_iter) return true;
  ++st.it;
  // before the first advance (t == 0) the gap test cannot stop the pair,
  // so a first step beyond t_c decides it without its distance
  if (st.t == 0.0 && st.t + st.tl > t_c) {
    st.t = t_c;
    return true;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    x[a].x = x[a].x + st.tl * p[a].x;
    x[a].y = x[a].y + st.tl * p[a].y;
    x[a].z = x[a].z + st.tl * p[a].z;
  }
  int ty;
  const double d = sqrt(pair_dist2<KIND>(x, &ty));
  if (st.t > 0.0 && d < st.g) return true;
  st.t = st.t + st.tl;
  if (st.t > t_c) {
    st.t = t_c;
    return true;
  }
  double rate = st.lp;
  if (st.dir) {
    rate = closing_rate<KIND>(ty, x, p);
    if (!(rate > 0.0)) {
      st.t = t_c;
      return true;
    }
  }
  st.tl = 0.9 * d / rate;
  return false;
}

template <int KIND>
__device__ __forceinline__ double accd(V3 *x, V3 *p, double s, double t_c, int64_t max_iter, int64_t *iters,
                                       bool dir) {
  AccdState st;
  st.dir = dir;
  if (!accd_init<KIND>(x, p, s, t_c, st))
    while (!accd_step<KIND>(x, p, t_c, max_iter, st)) {
    }
  *iters = st.it;
  return st.t;
}

}  // namespace eipc
