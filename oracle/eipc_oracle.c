/* Oracle for the Embedded IPC contact stage (TEST INFRASTRUCTURE ONLY).
 *
 * Plain FP64 CPU code that follows the paper's definitions directly:
 *   embedding x = W q (Sec. III-D, Eq. 13-14; J = dphi/dq, Sec. III-A),
 *   pair set B of all surface point-triangle and edge-edge pairs and the
 *   log barrier b(d) (Sec. III-B, Eq. 7), barrier potential kappa*sum b
 *   (Eq. 10-11), projected Newton (Sec. III-C), the chain rule
 *   grad_q = J^T grad_x, hess_q = J^T hess_x J (Eq. 17) and a conservative
 *   CCD step bound used to clamp the line search (Sec. III-C).
 * Where the paper defers to IPC (distances, mollifier) or is silent (the CCD
 * algorithm, tie-breaks, the eigen-solver) the readings are stated at each
 * function.  Compiled with -ffp-contract=off: every a*b+c below is a rounded
 * multiply followed by a rounded add, evaluated left to right as written.
 *
 * No blocking, fusion or reordering: brute-force loops over the definition.
 */
#include "eipc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small vector helpers (left-to-right sums, no contraction)           */
/* ------------------------------------------------------------------ */
static void sub3(const double *a, const double *b, double *r) {
  r[0] = a[0] - b[0];
  r[1] = a[1] - b[1];
  r[2] = a[2] - b[2];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

/* Neumaier compensated accumulation (the accurate reference sum). */
static void nsum(double *s, double *c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x))
    *c += (*s - t) + x;
  else
    *c += (x - t) + *s;
  *s = t;
}

static int has_dof(const or_scene *sc, int32_t v) { return sc->rowptr[v + 1] > sc->rowptr[v]; }

/* ------------------------------------------------------------------ */
/* Embedding (Eq. 13-14): x_k = sum_j w_kj q_j, then + off_k.          */
/* Accumulated in CSR order from 0.0, multiply then add per term, the  */
/* offset added last.  Used for positions (q, x_off) and displacements */
/* (dq, dx_off) alike.                                                 */
/* ------------------------------------------------------------------ */
void or_embed(const or_scene *sc, const double *q, const double *off, double *x) {
  for (int32_t v = 0; v < sc->n_vert; ++v) {
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int32_t k = sc->rowptr[v]; k < sc->rowptr[v + 1]; ++k) acc = acc + sc->val[k] * q[3 * sc->col[k] + c];
      if (off) acc = acc + off[3 * v + c];
      x[3 * v + c] = acc;
    }
  }
}

/* ------------------------------------------------------------------ */
/* Candidate pairs (the pair set B of Sec. III-B restricted by boxes).  */
/* Box of a primitive: per axis lo = min over its vertices (and, when   */
/* x1 is given, over their end positions too) minus dhat/2, hi = max    */
/* plus dhat/2, with dhat/2 computed once as 0.5*dhat.  A pair is a     */
/* candidate iff the closed boxes overlap on all three axes.  PT ranges */
/* over all (vertex v, face f) with v not in f; EE over all edge pairs  */
/* a < b sharing no vertex.  Pairs whose four vertices all have empty W */
/* rows carry no DoF and are excluded.                                  */
/* ------------------------------------------------------------------ */
static void prim_box(const double *x, const double *x1, const int32_t *vid, int nv, double h,
                     double *lo, double *hi) {
  for (int c = 0; c < 3; ++c) {
    double mn = x[3 * vid[0] + c], mx = mn;
    for (int i = 0; i < nv; ++i) {
      double a = x[3 * vid[i] + c];
      if (a < mn) mn = a;
      if (a > mx) mx = a;
      if (x1) {
        double b = x1[3 * vid[i] + c];
        if (b < mn) mn = b;
        if (b > mx) mx = b;
      }
    }
    lo[c] = mn - h;
    hi[c] = mx + h;
  }
}
static int boxes_overlap(const double *alo, const double *ahi, const double *blo, const double *bhi) {
  for (int c = 0; c < 3; ++c)
    if (!(alo[c] <= bhi[c] && blo[c] <= ahi[c])) return 0;
  return 1;
}

int64_t or_pt_query(const or_scene *sc, const double *x, const double *x1, double dhat, int32_t v,
                    int32_t *out, int64_t cap) {
  double h = 0.5 * dhat, vlo[3], vhi[3], flo[3], fhi[3];
  prim_box(x, x1, &v, 1, h, vlo, vhi);
  int64_t n = 0;
  for (int32_t f = 0; f < sc->n_face; ++f) {
    const int32_t *fv = sc->faces + 3 * f;
    if (fv[0] == v || fv[1] == v || fv[2] == v) continue;
    if (!has_dof(sc, v) && !has_dof(sc, fv[0]) && !has_dof(sc, fv[1]) && !has_dof(sc, fv[2])) continue;
    prim_box(x, x1, fv, 3, h, flo, fhi);
    if (!boxes_overlap(vlo, vhi, flo, fhi)) continue;
    if (n < cap) out[n] = f;
    ++n;
  }
  return n;
}

int64_t or_ee_query(const or_scene *sc, const double *x, const double *x1, double dhat, int32_t ea,
                    int32_t *out, int64_t cap) {
  double h = 0.5 * dhat, alo[3], ahi[3], blo[3], bhi[3];
  const int32_t *a = sc->edges + 2 * ea;
  prim_box(x, x1, a, 2, h, alo, ahi);
  int64_t n = 0;
  for (int32_t eb = ea + 1; eb < sc->n_edge; ++eb) {
    const int32_t *b = sc->edges + 2 * eb;
    if (a[0] == b[0] || a[0] == b[1] || a[1] == b[0] || a[1] == b[1]) continue;
    if (!has_dof(sc, a[0]) && !has_dof(sc, a[1]) && !has_dof(sc, b[0]) && !has_dof(sc, b[1])) continue;
    prim_box(x, x1, b, 2, h, blo, bhi);
    if (!boxes_overlap(alo, ahi, blo, bhi)) continue;
    if (n < cap) out[n] = eb;
    ++n;
  }
  return n;
}

/* All candidates, sorted by (first, second) by construction. */
int or_candidates(const or_scene *sc, const double *x, const double *x1, double dhat, int32_t *pt,
                  int64_t cap_pt, int64_t *n_pt, int32_t *ee, int64_t cap_ee, int64_t *n_ee) {
  int64_t npt = 0, nee = 0;
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(sc->n_face > sc->n_edge ? sc->n_face : sc->n_edge) + 4);
  for (int32_t v = 0; v < sc->n_vert; ++v) {
    int64_t k = or_pt_query(sc, x, x1, dhat, v, buf, sc->n_face);
    for (int64_t i = 0; i < k; ++i, ++npt)
      if (npt < cap_pt) { pt[2 * npt] = v; pt[2 * npt + 1] = buf[i]; }
  }
  for (int32_t ea = 0; ea < sc->n_edge; ++ea) {
    int64_t k = or_ee_query(sc, x, x1, dhat, ea, buf, sc->n_edge);
    for (int64_t i = 0; i < k; ++i, ++nee)
      if (nee < cap_ee) { ee[2 * nee] = ea; ee[2 * nee + 1] = buf[i]; }
  }
  free(buf);
  *n_pt = npt;
  *n_ee = nee;
  return (npt > cap_pt || nee > cap_ee) ? OR_ERR_CAPACITY : OR_OK;
}

/* ------------------------------------------------------------------ */
/* Distances (the paper defers to IPC for d_k; Sec. III-B).            */
/* d is the Euclidean distance between the closed primitives.  It is   */
/* evaluated as s = d^2 through a distance type naming the closest     */
/* feature pair; each type has one canonical value formula:            */
/*   PP     s = r.r                   r = x_i - x_j                    */
/*   PL     s = |r x e|^2 / (e.e)     r = point - a, e = b - a          */
/*   TRIPLE s = (y0.(y1 x y2))^2 / |y1 x y2|^2                          */
/*          PT: y0 = p-t0, y1 = t1-t0, y2 = t2-t0                      */
/*          EE: y0 = a0-b0, y1 = a1-a0, y2 = b1-b0                     */
/* Each local vector y_j is x[plus_j] - x[minus_j] over the 4 vertex    */
/* slots (PT: p,t0,t1,t2; EE: a0,a1,b0,b1).                            */
/* ------------------------------------------------------------------ */
enum { K_PP = 0, K_PL = 1, K_TRIPLE = 2 };
typedef struct {
  int kind, m;
  int plus[3], minus[3];
} locmap;

static const locmap PT_MAP[7] = {
    {K_PP, 1, {0}, {1}},                     /* P-T0 */
    {K_PP, 1, {0}, {2}},                     /* P-T1 */
    {K_PP, 1, {0}, {3}},                     /* P-T2 */
    {K_PL, 2, {0, 2}, {1, 1}},               /* P-E0: p on t0t1 */
    {K_PL, 2, {0, 3}, {2, 2}},               /* P-E1: p on t1t2 */
    {K_PL, 2, {0, 1}, {3, 3}},               /* P-E2: p on t2t0 */
    {K_TRIPLE, 3, {0, 2, 3}, {1, 1, 1}},     /* P-T: interior */
};
static const locmap EE_MAP[9] = {
    {K_PP, 1, {0}, {2}},                     /* a0-b0 */
    {K_PP, 1, {0}, {3}},                     /* a0-b1 */
    {K_PP, 1, {1}, {2}},                     /* a1-b0 */
    {K_PP, 1, {1}, {3}},                     /* a1-b1 */
    {K_PL, 2, {2, 1}, {0, 0}},               /* b0 on edge a */
    {K_PL, 2, {3, 1}, {0, 0}},               /* b1 on edge a */
    {K_PL, 2, {0, 3}, {2, 2}},               /* a0 on edge b */
    {K_PL, 2, {1, 3}, {2, 2}},               /* a1 on edge b */
    {K_TRIPLE, 3, {0, 1, 3}, {2, 0, 2}},     /* interior-interior */
};

static const locmap *map_of(int kind, int type) { return kind == 0 ? &PT_MAP[type] : &EE_MAP[type]; }

static void local_vectors(const locmap *mp, const double *x12, double *y) {
  for (int j = 0; j < mp->m; ++j) sub3(x12 + 3 * mp->plus[j], x12 + 3 * mp->minus[j], y + 3 * j);
}

static double value_of(int kind_fn, const double *y) {
  if (kind_fn == K_PP) return dot3(y, y);
  if (kind_fn == K_PL) {
    double c[3];
    cross3(y, y + 3, c);
    return dot3(c, c) / dot3(y + 3, y + 3);
  }
  double n[3];
  cross3(y + 3, y + 6, n);
  double N = dot3(y, n);
  return (N * N) / dot3(n, n);
}

double or_pair_dist2(int kind, int type, const double *x12) {
  const locmap *mp = map_of(kind, type);
  double y[9];
  local_vectors(mp, x12, y);
  return value_of(mp->kind, y);
}

/* Point-segment sub-classification: 0 = endpoint a, 1 = endpoint b,
 * 2 = interior (lower-dimensional feature preferred on ties). */
static int point_segment(const double *p, const double *a, const double *b) {
  double r[3], e[3];
  sub3(p, a, r);
  sub3(b, a, e);
  double t = dot3(r, e);
  if (t <= 0.0) return 0;
  double ee = dot3(e, e);
  if (t >= ee) return 1;
  return 2;
}

/* PT: interior iff the plane projection is strictly inside the triangle
 * (Cramer numerators against det = |n|^2); otherwise the closest of the
 * three point-segment features, edges in order t0t1, t1t2, t2t0, first
 * strict minimum wins. */
int or_pt_type(const double *p, const double *t0, const double *t1, const double *t2) {
  double e0[3], e1[3], r[3], n[3];
  sub3(t1, t0, e0);
  sub3(t2, t0, e1);
  sub3(p, t0, r);
  cross3(e0, e1, n);
  double det = dot3(n, n);
  if (det > 0.0) {
    double a = dot3(e0, e0), b = dot3(e0, e1), c = dot3(e1, e1);
    double d0 = dot3(e0, r), d1 = dot3(e1, r);
    double un = c * d0 - b * d1;
    double vn = a * d1 - b * d0;
    if (un > 0.0 && vn > 0.0 && un + vn < det) return PT_T;
  }
  const double *tv[3] = {t0, t1, t2};
  static const int vtype[3] = {PT_T0, PT_T1, PT_T2};
  double x12[12];
  memcpy(x12, p, 24);
  memcpy(x12 + 3, t0, 24);
  memcpy(x12 + 6, t1, 24);
  memcpy(x12 + 9, t2, 24);
  int best = -1;
  double best_s = 0.0;
  for (int k = 0; k < 3; ++k) {
    int ia = k, ib = (k + 1) % 3;
    int sub = point_segment(p, tv[ia], tv[ib]);
    int type = sub == 0 ? vtype[ia] : (sub == 1 ? vtype[ib] : PT_E0 + k);
    double s = or_pair_dist2(0, type, x12);
    if (best < 0 || s < best_s) {
      best = type;
      best_s = s;
    }
  }
  return best;
}

/* EE: interior-interior iff the edges are not near-parallel
 * (|u x v|^2 > 1e-20 |u|^2 |v|^2) and both line parameters lie strictly
 * inside (0, 1); otherwise the closest of the four endpoint-segment
 * features in order a0|b, a1|b, b0|a, b1|a, first strict minimum wins. */
int or_ee_type(const double *a0, const double *a1, const double *b0, const double *b1) {
  double u[3], v[3], w[3], n[3];
  sub3(a1, a0, u);
  sub3(b1, b0, v);
  sub3(a0, b0, w);
  cross3(u, v, n);
  double D = dot3(n, n);
  double a = dot3(u, u), c = dot3(v, v);
  if (D > 1e-20 * a * c) {
    double b = dot3(u, v), d = dot3(u, w), e = dot3(v, w);
    double sn = b * e - c * d;
    double tn = a * e - b * d;
    if (sn > 0.0 && sn < D && tn > 0.0 && tn < D) return EE_AB;
  }
  double x12[12];
  memcpy(x12, a0, 24);
  memcpy(x12 + 3, a1, 24);
  memcpy(x12 + 6, b0, 24);
  memcpy(x12 + 9, b1, 24);
  /* (point, seg end 0, seg end 1) and the types for endpoint0/endpoint1/interior */
  const double *pp[4] = {a0, a1, b0, b1};
  const double *sa[4] = {b0, b0, a0, a0};
  const double *sb[4] = {b1, b1, a1, a1};
  static const int ty[4][3] = {{EE_A0B0, EE_A0B1, EE_A0B},
                               {EE_A1B0, EE_A1B1, EE_A1B},
                               {EE_A0B0, EE_A1B0, EE_AB0},
                               {EE_A0B1, EE_A1B1, EE_AB1}};
  int best = -1;
  double best_s = 0.0;
  for (int k = 0; k < 4; ++k) {
    int sub = point_segment(pp[k], sa[k], sb[k]);
    int type = ty[k][sub];
    double s = or_pair_dist2(1, type, x12);
    if (best < 0 || s < best_s) {
      best = type;
      best_s = s;
    }
  }
  return best;
}

/* ------------------------------------------------------------------ */
/* Derivatives of s in local coordinates, then chain rule to 12 coords. */
/* Ratio rule for s = f(N, D):                                          */
/*   grad s = fN gN + fD gD                                             */
/*   hess s = fNN gN gN^T + fND (gN gD^T + gD gN^T) + fDD gD gD^T       */
/*            + fN HN + fD HD                                           */
/* ------------------------------------------------------------------ */
static void skew_add(double *H, int ld, int r0, int c0, const double *a, double sgn) {
  /* H[r0.., c0..] += sgn * [a]_x  where [a]_x b = a x b */
  H[(r0 + 0) * ld + c0 + 1] += sgn * -a[2];
  H[(r0 + 0) * ld + c0 + 2] += sgn * a[1];
  H[(r0 + 1) * ld + c0 + 0] += sgn * a[2];
  H[(r0 + 1) * ld + c0 + 2] += sgn * -a[0];
  H[(r0 + 2) * ld + c0 + 0] += sgn * -a[1];
  H[(r0 + 2) * ld + c0 + 1] += sgn * a[0];
}

/* |y1 x y2|^2 with gradient (w.r.t. y1, y2: 6) and Hessian (6x6). */
static void crossnorm2(const double *y1, const double *y2, double *val, double *g, double *H) {
  double n[3];
  cross3(y1, y2, n);
  *val = dot3(n, n);
  double t1[3], t2[3];
  cross3(y2, n, t1); /* d/dy1 = 2 y2 x n */
  cross3(n, y1, t2); /* d/dy2 = 2 n x y1 */
  for (int i = 0; i < 3; ++i) {
    g[i] = 2.0 * t1[i];
    g[3 + i] = 2.0 * t2[i];
  }
  double a11 = dot3(y1, y1), a22 = dot3(y2, y2), a12 = dot3(y1, y2);
  memset(H, 0, sizeof(double) * 36);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double id = (i == j) ? 1.0 : 0.0;
      H[i * 6 + j] = 2.0 * (a22 * id - y2[i] * y2[j]);
      H[(3 + i) * 6 + 3 + j] = 2.0 * (a11 * id - y1[i] * y1[j]);
      double c = 4.0 * y1[i] * y2[j] - 2.0 * y2[i] * y1[j] - 2.0 * a12 * id;
      H[i * 6 + 3 + j] = c;
      H[(3 + j) * 6 + i] = c;
    }
}

static void local_derivs(int kind_fn, const double *y, double *s, double *gs, double *Hs) {
  int nl = 0;
  if (kind_fn == K_PP) {
    *s = dot3(y, y);
    memset(Hs, 0, sizeof(double) * 9);
    for (int i = 0; i < 3; ++i) {
      gs[i] = 2.0 * y[i];
      Hs[i * 3 + i] = 2.0;
    }
    return;
  }
  double gN[9] = {0}, HN[81] = {0}, gD[9] = {0}, HD[81] = {0};
  double N, D, fN, fD, fNN, fND, fDD;
  if (kind_fn == K_PL) {
    nl = 6;
    /* N = |r x e|^2, D = e.e, s = N / D */
    double g6[6], H36[36];
    crossnorm2(y, y + 3, &N, g6, H36);
    for (int i = 0; i < 6; ++i) gN[i] = g6[i];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) HN[i * nl + j] = H36[i * 6 + j];
    D = dot3(y + 3, y + 3);
    for (int i = 0; i < 3; ++i) {
      gD[3 + i] = 2.0 * y[3 + i];
      HD[(3 + i) * nl + 3 + i] = 2.0;
    }
    *s = N / D;
    fN = 1.0 / D;
    fD = -N / (D * D);
    fNN = 0.0;
    fND = -1.0 / (D * D);
    fDD = 2.0 * N / (D * D * D);
  } else {
    nl = 9;
    /* N = y0.(y1 x y2), D = |y1 x y2|^2, s = N^2 / D */
    double n[3], c20[3], c01[3];
    cross3(y + 3, y + 6, n);
    cross3(y + 6, y, c20);
    cross3(y, y + 3, c01);
    N = dot3(y, n);
    for (int i = 0; i < 3; ++i) {
      gN[i] = n[i];
      gN[3 + i] = c20[i];
      gN[6 + i] = c01[i];
    }
    /* HN: (0,1) = -[y2]x, (0,2) = [y1]x, (1,2) = -[y0]x, symmetric */
    skew_add(HN, nl, 0, 3, y + 6, -1.0);
    skew_add(HN, nl, 0, 6, y + 3, 1.0);
    skew_add(HN, nl, 3, 6, y, -1.0);
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < i; ++j) HN[i * nl + j] = HN[j * nl + i];
    double g6[6], H36[36];
    crossnorm2(y + 3, y + 6, &D, g6, H36);
    for (int i = 0; i < 6; ++i) gD[3 + i] = g6[i];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) HD[(3 + i) * nl + 3 + j] = H36[i * 6 + j];
    *s = (N * N) / D;
    fN = 2.0 * N / D;
    fD = -(N * N) / (D * D);
    fNN = 2.0 / D;
    fND = -2.0 * N / (D * D);
    fDD = 2.0 * (N * N) / (D * D * D);
  }
  for (int i = 0; i < nl; ++i) gs[i] = fN * gN[i] + fD * gD[i];
  for (int i = 0; i < nl; ++i)
    for (int j = 0; j < nl; ++j)
      Hs[i * nl + j] = fNN * gN[i] * gN[j] + fND * (gN[i] * gD[j] + gD[i] * gN[j]) + fDD * gD[i] * gD[j] +
                       fN * HN[i * nl + j] + fD * HD[i * nl + j];
}

/* coefficient of vertex slot a in local vector j: +1, -1 or 0 */
static double coef(const locmap *mp, int j, int a) {
  return (mp->plus[j] == a ? 1.0 : 0.0) - (mp->minus[j] == a ? 1.0 : 0.0);
}

static void to_slots(const locmap *mp, int m, const int *plus, const int *minus, const double *gl,
                     const double *Hl, double *g12, double *H144) {
  locmap tmp;
  tmp.m = m;
  for (int j = 0; j < m; ++j) {
    tmp.plus[j] = plus[j];
    tmp.minus[j] = minus[j];
  }
  (void)mp;
  int nl = 3 * m;
  if (g12) {
    memset(g12, 0, sizeof(double) * 12);
    for (int a = 0; a < 4; ++a)
      for (int j = 0; j < m; ++j) {
        double ca = coef(&tmp, j, a);
        if (ca == 0.0) continue;
        for (int i = 0; i < 3; ++i) g12[3 * a + i] += ca * gl[3 * j + i];
      }
  }
  if (H144) {
    memset(H144, 0, sizeof(double) * 144);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int j = 0; j < m; ++j)
          for (int k = 0; k < m; ++k) {
            double c = coef(&tmp, j, a) * coef(&tmp, k, b);
            if (c == 0.0) continue;
            for (int i = 0; i < 3; ++i)
              for (int l = 0; l < 3; ++l) H144[(3 * a + i) * 12 + 3 * b + l] += c * Hl[(3 * j + i) * nl + 3 * k + l];
          }
  }
}

void or_pair_dist2_derivs(int kind, int type, const double *x12, double *s, double *g12, double *H144) {
  const locmap *mp = map_of(kind, type);
  double y[9], gl[9], Hl[81];
  local_vectors(mp, x12, y);
  local_derivs(mp->kind, y, s, gl, Hl);
  /* the value reported is the canonical value formula */
  *s = value_of(mp->kind, y);
  to_slots(mp, mp->m, mp->plus, mp->minus, gl, Hl, g12, H144);
}

/* ------------------------------------------------------------------ */
/* Barrier (Eq. 7): b(d) = -(d - dhat)^2 ln(d / dhat) on (0, dhat), 0   */
/* elsewhere, with b' and b'' in d.                                     */
/* ------------------------------------------------------------------ */
void or_barrier(double d, double dhat, double *b, double *b1, double *b2) {
  if (!(d > 0.0 && d < dhat)) {
    *b = *b1 = *b2 = 0.0;
    return;
  }
  double lr = log(d / dhat);
  double dm = d - dhat;
  *b = -(dm * dm) * lr;
  *b1 = -2.0 * dm * lr - (dm * dm) / d;
  *b2 = -2.0 * lr - 4.0 * dm / d + (dm * dm) / (d * d);
}

/* Alternative formulation: the same log barrier written in the squared
 * distance, b(s) = -(s - shat)^2 ln(s / shat) with s = d^2, shat = dhat^2
 * (the form IPC implementations evaluate; Eq. 7 states it in d).  The
 * active set is the same (s < shat); b1, b2 are db/ds and d2b/ds2. */
void or_barrier_sq(double s, double shat, double *b, double *b1, double *b2) {
  if (!(s > 0.0 && s < shat)) {
    *b = *b1 = *b2 = 0.0;
    return;
  }
  double lr = log(s / shat);
  double sm = s - shat;
  *b = -(sm * sm) * lr;
  *b1 = -2.0 * sm * lr - (sm * sm) / s;
  *b2 = -2.0 * lr - 4.0 * sm / s + (sm * sm) / (s * s);
}

/* EE mollifier (IPC, which the paper defers to for its contact model):
 * m(c) = (2 - c/eps) c/eps for c < eps, else 1, with c = |ea x eb|^2. */
void or_mollifier(double c, double eps_x, double *m, double *m1, double *m2) {
  if (c < eps_x) {
    double r = c / eps_x;
    *m = (2.0 - r) * r;
    *m1 = (2.0 - 2.0 * r) / eps_x;
    *m2 = -2.0 / (eps_x * eps_x);
  } else {
    *m = 1.0;
    *m1 = 0.0;
    *m2 = 0.0;
  }
}

/* One pair: energy kappa*m*b(d), its 12-gradient and true 12x12 Hessian.
 * rest12 != NULL switches the EE mollifier on (ignored for PT).
 * Returns OR_OK (active), OR_INACTIVE (d >= dhat), OR_ERR_INTERSECTING
 * (d == 0) or OR_ERR_NONFINITE. */
int or_pair_eval(int kind, const double *x12, const double *rest12, double dhat, double kappa, int *type_out,
                 double *s_out, double *e, double *g12, double *H144) {
  return or_pair_eval_f(kind, x12, rest12, dhat, kappa, 0, type_out, s_out, e, g12, H144);
}

int or_pair_eval_f(int kind, const double *x12, const double *rest12, double dhat, double kappa, uint32_t flags,
                   int *type_out, double *s_out, double *e, double *g12, double *H144) {
  int type = kind == 0 ? or_pt_type(x12, x12 + 3, x12 + 6, x12 + 9) : or_ee_type(x12, x12 + 3, x12 + 6, x12 + 9);
  double s = or_pair_dist2(kind, type, x12);
  if (type_out) *type_out = type;
  if (s_out) *s_out = s;
  if (!isfinite(s)) return OR_ERR_NONFINITE;
  if (!(s < dhat * dhat)) return OR_INACTIVE;
  if (s <= 0.0) return OR_ERR_INTERSECTING;
  double gs[12], Hs[144], s2;
  or_pair_dist2_derivs(kind, type, x12, &s2, gs, Hs);
  double b, bs1, bs2;
  if (flags & OR_SQDIST) {
    or_barrier_sq(s, dhat * dhat, &b, &bs1, &bs2);
  } else {
    double d = sqrt(s), b1, b2;
    or_barrier(d, dhat, &b, &b1, &b2);
    /* b as a function of s = d^2 */
    bs1 = b1 / (2.0 * d);
    bs2 = (b2 - b1 / d) / (4.0 * s);
  }
  double m = 1.0, m1 = 0.0, m2 = 0.0, c = 0.0, gc[12] = {0}, Hc[144] = {0};
  int moll = (kind == 1 && rest12 != NULL);
  if (moll) {
    double ur[3], vr[3];
    sub3(rest12 + 3, rest12, ur);
    sub3(rest12 + 9, rest12 + 6, vr);
    double eps_x = 1e-3 * dot3(ur, ur) * dot3(vr, vr);
    double u[3], v[3], g6[6], H36[36];
    sub3(x12 + 3, x12, u);
    sub3(x12 + 9, x12 + 6, v);
    crossnorm2(u, v, &c, g6, H36);
    or_mollifier(c, eps_x, &m, &m1, &m2);
    if (m1 != 0.0 || m2 != 0.0) {
      /* u = x1 - x0, v = x3 - x2 */
      static const int pl[2] = {1, 3}, mi[2] = {0, 2};
      to_slots(NULL, 2, pl, mi, g6, H36, gc, Hc);
    } else {
      moll = 0;
    }
  }
  if (e) *e = kappa * (m * b);
  if (g12) {
    for (int i = 0; i < 12; ++i) {
      double gb = bs1 * gs[i];
      g12[i] = kappa * (m * gb + (moll ? b * m1 * gc[i] : 0.0));
    }
  }
  if (H144) {
    for (int i = 0; i < 12; ++i)
      for (int j = 0; j < 12; ++j) {
        double Hb = bs2 * gs[i] * gs[j] + bs1 * Hs[i * 12 + j];
        double h = m * Hb;
        if (moll) {
          double gbi = bs1 * gs[i], gbj = bs1 * gs[j];
          h += m1 * (gbi * gc[j] + gc[i] * gbj) + b * (m2 * gc[i] * gc[j] + m1 * Hc[i * 12 + j]);
        }
        H144[i * 12 + j] = kappa * h;
      }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* PSD projection for projected Newton (Sec. III-C): P = V max(L,0) V^T */
/* from the symmetric eigendecomposition of A, by the cyclic Jacobi     */
/* method (classical two-sided rotations zeroing a_pq in row order),    */
/* until the off-diagonal Frobenius norm falls below 1e-17 ||A||_F.     */
/* P is the unique Frobenius-nearest PSD matrix, so any converged       */
/* eigensolver gives the same P.  Returns the number of sweeps.         */
/* ------------------------------------------------------------------ */
int or_project_psd(int n, const double *A, double *P) {
  static _Thread_local double a[48 * 48], v[48 * 48];
  if (n < 1 || n > 48) return -1;
  memcpy(a, A, sizeof(double) * n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      a[i * n + j] = 0.5 * (A[i * n + j] + A[j * n + i]);
      v[i * n + j] = (i == j) ? 1.0 : 0.0;
    }
  double fro = 0.0;
  for (int i = 0; i < n * n; ++i) fro += a[i] * a[i];
  fro = sqrt(fro);
  int sweep = 0;
  for (; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
    if (sqrt(off) <= 1e-17 * fro || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (apq == 0.0) continue;
        double tau = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        double t;
        if (fabs(tau) > 1e150)
          t = 0.5 / tau;
        else
          t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) { /* columns p, q */
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) { /* rows p, q */
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = v[k * n + p], vkq = v[k * n + q];
          v[k * n + p] = c * vkp - s * vkq;
          v[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) {
        double lam = a[k * n + k];
        if (lam > 0.0) acc += v[i * n + k] * lam * v[j * n + k];
      }
      P[i * n + j] = acc;
    }
  return sweep;
}

/* ------------------------------------------------------------------ */
/* Reduction through the embedding (Eq. 17): grad_q = J^T grad_x,       */
/* hess_q = J^T hess_x J, per pair with J restricted to the pair's four */
/* vertices.  Summed over pairs in list order (PT list then EE list)    */
/* with Neumaier compensation.                                          */
/* ------------------------------------------------------------------ */
static void pair_vertices(const or_scene *sc, int kind, const int32_t *pr, int32_t *vid) {
  if (kind == 0) {
    vid[0] = pr[0];
    vid[1] = sc->faces[3 * pr[1]];
    vid[2] = sc->faces[3 * pr[1] + 1];
    vid[3] = sc->faces[3 * pr[1] + 2];
  } else {
    vid[0] = sc->edges[2 * pr[0]];
    vid[1] = sc->edges[2 * pr[0] + 1];
    vid[2] = sc->edges[2 * pr[1]];
    vid[3] = sc->edges[2 * pr[1] + 1];
  }
}

int or_barrier_reduce(const or_scene *sc, const double *q, const int32_t *pt, int64_t n_pt, const int32_t *ee,
                      int64_t n_ee, double dhat, double kappa, uint32_t flags, double *energy, double *grad_q,
                      double *hess_q, int64_t *n_active) {
  int64_t nd = 3 * (int64_t)sc->n_node;
  double *x = (double *)malloc(sizeof(double) * 3 * (size_t)sc->n_vert + 8);
  or_embed(sc, q, sc->x_off, x);
  double es = 0.0, ec = 0.0;
  double *gc = grad_q ? (double *)calloc((size_t)nd + 1, sizeof(double)) : NULL;
  double *hc = hess_q ? (double *)calloc((size_t)(nd * nd) + 1, sizeof(double)) : NULL;
  if (grad_q) memset(grad_q, 0, sizeof(double) * nd);
  if (hess_q) memset(hess_q, 0, sizeof(double) * nd * nd);
  int64_t na = 0;
  int status = OR_OK;
  int moll = (flags & OR_MOLLIFY) && sc->x_rest;
  for (int kind = 0; kind < 2; ++kind) {
    const int32_t *list = kind == 0 ? pt : ee;
    int64_t n = kind == 0 ? n_pt : n_ee;
    for (int64_t k = 0; k < n; ++k) {
      int32_t vid[4];
      pair_vertices(sc, kind, list + 2 * k, vid);
      double x12[12], r12[12];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) {
          x12[3 * a + c] = x[3 * vid[a] + c];
          if (moll) r12[3 * a + c] = sc->x_rest[3 * vid[a] + c];
        }
      double e, g[12], H[144], P[144];
      int st = or_pair_eval_f(kind, x12, moll ? r12 : NULL, dhat, kappa, flags, NULL, NULL, &e, g, H);
      if (st == OR_INACTIVE) continue;
      if (st != OR_OK) {
        status = st;
        continue;
      }
      ++na;
      nsum(&es, &ec, e);
      if (hess_q && (flags & OR_PROJECT_REDUCED)) {
        /* the pair's reduced local block over its distinct nodes, then its
         * PSD projection */
        int32_t nodes[16];
        int m = 0;
        for (int a = 0; a < 4; ++a)
          for (int32_t ka = sc->rowptr[vid[a]]; ka < sc->rowptr[vid[a] + 1]; ++ka) {
            int f = 0;
            for (int t = 0; t < m; ++t) f |= nodes[t] == sc->col[ka];
            if (!f) nodes[m++] = sc->col[ka];
          }
        static _Thread_local double K[48 * 48], PK[48 * 48];
        int n3 = 3 * m;
        memset(K, 0, sizeof(double) * n3 * n3);
        for (int a = 0; a < 4; ++a)
          for (int32_t ka = sc->rowptr[vid[a]]; ka < sc->rowptr[vid[a] + 1]; ++ka) {
            int I = 0;
            while (nodes[I] != sc->col[ka]) ++I;
            for (int b = 0; b < 4; ++b)
              for (int32_t kb = sc->rowptr[vid[b]]; kb < sc->rowptr[vid[b] + 1]; ++kb) {
                int J = 0;
                while (nodes[J] != sc->col[kb]) ++J;
                double wab = sc->val[ka] * sc->val[kb];
                for (int i = 0; i < 3; ++i)
                  for (int j = 0; j < 3; ++j) K[(3 * I + i) * n3 + 3 * J + j] += wab * H[(3 * a + i) * 12 + 3 * b + j];
              }
          }
        if (m > 0) or_project_psd(n3, K, PK);
        for (int I = 0; I < m; ++I)
          for (int J = 0; J < m; ++J)
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) {
                int64_t idx = (3 * (int64_t)nodes[I] + i) * nd + 3 * nodes[J] + j;
                nsum(&hess_q[idx], &hc[idx], PK[(3 * I + i) * n3 + 3 * J + j]);
              }
        if (grad_q)
          for (int a = 0; a < 4; ++a)
            for (int32_t ka = sc->rowptr[vid[a]]; ka < sc->rowptr[vid[a] + 1]; ++ka)
              for (int i = 0; i < 3; ++i)
                nsum(&grad_q[3 * sc->col[ka] + i], &gc[3 * sc->col[ka] + i], sc->val[ka] * g[3 * a + i]);
        continue;
      }
      const double *Hu = H;
      if (hess_q && (flags & OR_PROJECT)) {
        or_project_psd(12, H, P);
        Hu = P;
      }
      for (int a = 0; a < 4; ++a)
        for (int32_t ka = sc->rowptr[vid[a]]; ka < sc->rowptr[vid[a] + 1]; ++ka) {
          int32_t I = sc->col[ka];
          double wa = sc->val[ka];
          if (grad_q)
            for (int i = 0; i < 3; ++i) nsum(&grad_q[3 * I + i], &gc[3 * I + i], wa * g[3 * a + i]);
          if (!hess_q) continue;
          for (int b = 0; b < 4; ++b)
            for (int32_t kb = sc->rowptr[vid[b]]; kb < sc->rowptr[vid[b] + 1]; ++kb) {
              int32_t J = sc->col[kb];
              double wab = wa * sc->val[kb];
              for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                  int64_t idx = (3 * (int64_t)I + i) * nd + 3 * J + j;
                  nsum(&hess_q[idx], &hc[idx], wab * Hu[(3 * a + i) * 12 + 3 * b + j]);
                }
            }
        }
    }
  }
  if (grad_q)
    for (int64_t i = 0; i < nd; ++i) grad_q[i] += gc[i];
  if (hess_q)
    for (int64_t i = 0; i < nd * nd; ++i) hess_q[i] += hc[i];
  if (energy) *energy = es + ec;
  if (n_active) *n_active = na;
  free(gc);
  free(hc);
  free(x);
  return status;
}

/* Hessian-vector product through the embedding: out = sum_k W_k^T H_k
 * (W_k v + v_off_k), H_k the true pair Hessian or, with OR_PROJECT, its PSD
 * projection.  out_off (optional) receives the unreduced per-vertex sums
 * of H_k z_k (the kinematic rows). */
int or_barrier_hvp(const or_scene *sc, const double *q, const int32_t *pt, int64_t n_pt, const int32_t *ee,
                   int64_t n_ee, double dhat, double kappa, uint32_t flags, const double *v, const double *v_off,
                   double *out, double *out_off) {
  int64_t nd = 3 * (int64_t)sc->n_node;
  double *x = (double *)malloc(sizeof(double) * 3 * (size_t)sc->n_vert + 8);
  double *xv = (double *)malloc(sizeof(double) * 3 * (size_t)sc->n_vert + 8);
  or_embed(sc, q, sc->x_off, x);
  or_embed(sc, v, v_off, xv);
  double *oc = (double *)calloc((size_t)nd + 1, sizeof(double));
  double *ofc = out_off ? (double *)calloc(3 * (size_t)sc->n_vert + 1, sizeof(double)) : NULL;
  memset(out, 0, sizeof(double) * nd);
  if (out_off) memset(out_off, 0, sizeof(double) * 3 * sc->n_vert);
  int status = OR_OK;
  int moll = (flags & OR_MOLLIFY) && sc->x_rest;
  for (int kind = 0; kind < 2; ++kind) {
    const int32_t *list = kind == 0 ? pt : ee;
    int64_t n = kind == 0 ? n_pt : n_ee;
    for (int64_t k = 0; k < n; ++k) {
      int32_t vid[4];
      pair_vertices(sc, kind, list + 2 * k, vid);
      double x12[12], r12[12], z[12];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) {
          x12[3 * a + c] = x[3 * vid[a] + c];
          z[3 * a + c] = xv[3 * vid[a] + c];
          if (moll) r12[3 * a + c] = sc->x_rest[3 * vid[a] + c];
        }
      double H[144], P[144];
      int st = or_pair_eval_f(kind, x12, moll ? r12 : NULL, dhat, kappa, flags, NULL, NULL, NULL, NULL, H);
      if (st == OR_INACTIVE) continue;
      if (st != OR_OK) {
        status = st;
        continue;
      }
      const double *Hu = H;
      if (flags & OR_PROJECT) {
        or_project_psd(12, H, P);
        Hu = P;
      }
      double y[12];
      for (int i = 0; i < 12; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 12; ++j) acc += Hu[i * 12 + j] * z[j];
        y[i] = acc;
      }
      for (int a = 0; a < 4; ++a) {
        if (out_off)
          for (int i = 0; i < 3; ++i) nsum(&out_off[3 * vid[a] + i], &ofc[3 * vid[a] + i], y[3 * a + i]);
        for (int32_t ka = sc->rowptr[vid[a]]; ka < sc->rowptr[vid[a] + 1]; ++ka) {
          int32_t I = sc->col[ka];
          double wa = sc->val[ka];
          for (int i = 0; i < 3; ++i) nsum(&out[3 * I + i], &oc[3 * I + i], wa * y[3 * a + i]);
        }
      }
    }
  }
  for (int64_t i = 0; i < nd; ++i) out[i] += oc[i];
  if (out_off)
    for (int64_t i = 0; i < 3 * (int64_t)sc->n_vert; ++i) out_off[i] += ofc[i];
  free(oc);
  free(ofc);
  free(x);
  free(xv);
  return status;
}

/* ------------------------------------------------------------------ */
/* Conservative CCD step bound (Sec. III-C: CCD clamps every Newton     */
/* step; the cited conservative-advancement family).  Reading: additive */
/* CCD per pair with zero thickness:                                    */
/*   1. subtract the mean of the four displacements from each;          */
/*   2. l_p = |p0| + max(|p1|,|p2|,|p3|) (PT) or                        */
/*      max(|p0|,|p1|) + max(|p2|,|p3|) (EE); l_p = 0 -> t_c;           */
/*   3. d = dist(x), gap g = s d, t = 0, first step t_l = (1-s) d / l_p;*/
/*   4. repeat: x += t_l p, d = dist(x); stop if t > 0 and d < g;       */
/*      t += t_l; if t > t_c return t_c; t_l = 0.9 d / l_p.             */
/* Capped at max_iter iterations (returns the current t, still safe).   */
/* dist is the unmollified distance of the classified type.             */
/* ------------------------------------------------------------------ */
static double pair_dist(int kind, const double *x12) {
  int type = kind == 0 ? or_pt_type(x12, x12 + 3, x12 + 6, x12 + 9) : or_ee_type(x12, x12 + 3, x12 + 6, x12 + 9);
  return sqrt(or_pair_dist2(kind, type, x12));
}

double or_accd_pair(int kind, const double *x12, const double *p12, double s, double t_c, int64_t max_iter,
                    int64_t *iters) {
  double x[12], p[12], mean[3];
  memcpy(x, x12, sizeof x);
  for (int c = 0; c < 3; ++c) mean[c] = (((p12[c] + p12[3 + c]) + p12[6 + c]) + p12[9 + c]) * 0.25;
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) p[3 * a + c] = p12[3 * a + c] - mean[c];
  double n0 = sqrt(dot3(p, p)), n1 = sqrt(dot3(p + 3, p + 3)), n2 = sqrt(dot3(p + 6, p + 6)),
         n3 = sqrt(dot3(p + 9, p + 9));
  double lp;
  if (kind == 0)
    lp = n0 + fmax(n1, fmax(n2, n3));
  else
    lp = fmax(n0, n1) + fmax(n2, n3);
  if (iters) *iters = 0;
  if (lp == 0.0) return t_c;
  double d = pair_dist(kind, x);
  double g = s * d;
  double t = 0.0;
  double tl = (1.0 - s) * d / lp;
  int64_t it = 0;
  for (;;) {
    if (it >= max_iter) break;
    ++it;
    for (int i = 0; i < 12; ++i) x[i] = x[i] + tl * p[i];
    d = pair_dist(kind, x);
    if (t > 0.0 && d < g) break;
    t = t + tl;
    if (t > t_c) {
      t = t_c;
      break;
    }
    tl = 0.9 * d / lp;
  }
  if (iters) *iters = it;
  return t;
}

/* Alternative CCD (f4): conservative advancement along the closest
 * direction, after C2A (the CCD reference the paper cites).  At positions
 * x with distance d, let n be the unit vector from the second primitive's
 * closest point to the first's (the triangle or edge b, to the point or
 * edge a).  The two closest points span separating planes with normal n:
 * every point of the first primitive lies at or beyond n.c_first and every
 * point of the second at or before n.c_second.  Under linear motion each
 * point of a primitive stays a convex combination of its moving vertices,
 * so for any later time t' the distance is at least
 *   d - mu (t' - t),   mu = max_{b in second} n.p_b - min_{a in first} n.p_a.
 * The steps are those of additive CCD (or_accd_pair) with the motion bound
 * lp replaced by mu at each iterate; mu <= 0 (the gap along n does not
 * close) bounds the pair by t_c.  mu <= lp, so no step is shorter than the
 * additive one from the same iterate. */
static void closest_weights(int kind, int type, const double *x12, double *beta);

static double closing_rate(int kind, const double *x12, const double *p12) {
  int type = kind == 0 ? or_pt_type(x12, x12 + 3, x12 + 6, x12 + 9) : or_ee_type(x12, x12 + 3, x12 + 6, x12 + 9);
  double beta[4], r[3] = {0.0, 0.0, 0.0};
  closest_weights(kind, type, x12, beta);
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) r[c] += beta[a] * x12[3 * a + c];
  double rn = sqrt(dot3(r, r));
  double nv[3] = {r[0] / rn, r[1] / rn, r[2] / rn};
  int nfirst = kind == 0 ? 1 : 2;
  double amin = INFINITY, bmax = -INFINITY;
  for (int a = 0; a < 4; ++a) {
    double v = dot3(nv, p12 + 3 * a);
    if (a < nfirst)
      amin = fmin(amin, v);
    else
      bmax = fmax(bmax, v);
  }
  return bmax - amin;
}

double or_c2a_pair(int kind, const double *x12, const double *p12, double s, double t_c, int64_t max_iter,
                   int64_t *iters) {
  double x[12], p[12], mean[3];
  memcpy(x, x12, sizeof x);
  for (int c = 0; c < 3; ++c) mean[c] = (((p12[c] + p12[3 + c]) + p12[6 + c]) + p12[9 + c]) * 0.25;
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) p[3 * a + c] = p12[3 * a + c] - mean[c];
  if (iters) *iters = 0;
  int moving = 0;
  for (int i = 0; i < 12; ++i) moving |= p[i] != 0.0;
  if (!moving) return t_c;
  double d = pair_dist(kind, x);
  double mu = closing_rate(kind, x, p);
  if (!(mu > 0.0)) return t_c;
  double g = s * d;
  double t = 0.0;
  double tl = (1.0 - s) * d / mu;
  int64_t it = 0;
  for (;;) {
    if (it >= max_iter) break;
    ++it;
    if (t == 0.0 && t + tl > t_c) {
      t = t_c;
      break;
    }
    for (int i = 0; i < 12; ++i) x[i] = x[i] + tl * p[i];
    d = pair_dist(kind, x);
    if (t > 0.0 && d < g) break;
    t = t + tl;
    if (t > t_c) {
      t = t_c;
      break;
    }
    mu = closing_rate(kind, x, p);
    if (!(mu > 0.0)) {
      t = t_c;
      break;
    }
    tl = 0.9 * d / mu;
  }
  if (iters) *iters = it;
  return t;
}

int or_ccd_toi(const or_scene *sc, const double *x, const double *p, int kind, const int32_t *pairs, int64_t n,
               double s, double t_c, int64_t max_iter, double *t_out, int64_t *iters_out) {
  return or_ccd_toi_m(sc, x, p, kind, pairs, n, s, t_c, max_iter, 0, t_out, iters_out);
}

int or_ccd_toi_m(const or_scene *sc, const double *x, const double *p, int kind, const int32_t *pairs, int64_t n,
                 double s, double t_c, int64_t max_iter, int method, double *t_out, int64_t *iters_out) {
  for (int64_t k = 0; k < n; ++k) {
    int32_t vid[4];
    pair_vertices(sc, kind, pairs + 2 * k, vid);
    double x12[12], p12[12];
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) {
        x12[3 * a + c] = x[3 * vid[a] + c];
        p12[3 * a + c] = p[3 * vid[a] + c];
      }
    int64_t it;
    t_out[k] = method == 1 ? or_c2a_pair(kind, x12, p12, s, t_c, max_iter, &it)
                           : or_accd_pair(kind, x12, p12, s, t_c, max_iter, &it);
    if (iters_out) iters_out[k] = it;
  }
  return OR_OK;
}

/* alpha = min(t_max, min over swept-box candidates of the per-pair bound).
 * Swept candidates: the candidate predicate on boxes spanning start x and
 * end x + p (p = W dq + dx_off). */
int or_ccd_max_step(const or_scene *sc, const double *q, const double *dq, const double *dx_off, double dhat,
                    double s, double t_max, int64_t max_iter, double *alpha, int64_t *n_cand, int64_t *n_capped) {
  size_t n3 = 3 * (size_t)sc->n_vert;
  double *x = (double *)malloc(sizeof(double) * n3 + 8);
  double *p = (double *)malloc(sizeof(double) * n3 + 8);
  double *x1 = (double *)malloc(sizeof(double) * n3 + 8);
  or_embed(sc, q, sc->x_off, x);
  or_embed(sc, dq, dx_off, p);
  for (size_t i = 0; i < n3; ++i) x1[i] = x[i] + p[i];
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(sc->n_face > sc->n_edge ? sc->n_face : sc->n_edge) + 4);
  double a = t_max;
  int64_t nc = 0, ncap = 0;
  for (int kind = 0; kind < 2; ++kind) {
    int32_t nq = kind == 0 ? sc->n_vert : sc->n_edge;
    for (int32_t i = 0; i < nq; ++i) {
      int64_t k = kind == 0 ? or_pt_query(sc, x, x1, dhat, i, buf, sc->n_face)
                            : or_ee_query(sc, x, x1, dhat, i, buf, sc->n_edge);
      for (int64_t j = 0; j < k; ++j) {
        int32_t pr[2] = {i, buf[j]};
        double t;
        int64_t it;
        or_ccd_toi(sc, x, p, kind, pr, 1, s, t_max, max_iter, &t, &it);
        if (it >= max_iter) ++ncap;
        if (t < a) a = t;
        ++nc;
      }
    }
  }
  *alpha = a;
  if (n_cand) *n_cand = nc;
  if (n_capped) *n_capped = ncap;
  free(buf);
  free(x);
  free(p);
  free(x1);
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Candidate pairs through a uniform grid, for scenes too large for the */
/* brute-force loops above.  The grid only filters: every item whose    */
/* box shares a cell with the query's box is tested with the same       */
/* closed-box predicate and the same exclusion rules as or_pt_query and */
/* or_ee_query, and the pairs come out in the same (first, second)      */
/* order, so the result is the brute-force result.  Two overlapping     */
/* closed boxes both contain the lower corner of their overlap, and the */
/* cell index floor((v - origin) / cell) is monotone in v, so that      */
/* corner's cell lies in both boxes' cell ranges: no candidate is lost. */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t key;
  int32_t item;
} or_cell_ent;

struct or_grid {
  const or_scene *sc;
  double origin[3], cell;
  int64_t dims[3];
  double *vbox, *fbox, *ebox; /* [n][6]: lo xyz, hi xyz */
  or_cell_ent *fent, *eent;
  int64_t n_fent, n_eent;
};

static int cmp_ent(const void *a, const void *b) {
  const or_cell_ent *x = (const or_cell_ent *)a, *y = (const or_cell_ent *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->item > y->item) - (x->item < y->item);
}
static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static int64_t cell_index(double v, double o, double cell) { return (int64_t)floor((v - o) / cell); }

static void cell_range(const or_grid *g, const double *box, int64_t *lo, int64_t *hi) {
  for (int c = 0; c < 3; ++c) {
    lo[c] = cell_index(box[c], g->origin[c], g->cell);
    hi[c] = cell_index(box[3 + c], g->origin[c], g->cell);
  }
}

static int64_t cell_key(const or_grid *g, int64_t i, int64_t j, int64_t k) {
  return (i * g->dims[1] + j) * g->dims[2] + k;
}

static or_cell_ent *grid_entries(const or_grid *g, const double *boxes, int32_t n, int64_t *n_out) {
  int64_t tot = 0, lo[3], hi[3];
  for (int32_t i = 0; i < n; ++i) {
    cell_range(g, boxes + 6 * (int64_t)i, lo, hi);
    tot += (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
  }
  or_cell_ent *e = (or_cell_ent *)malloc(sizeof(or_cell_ent) * (size_t)(tot + 1));
  int64_t k = 0;
  for (int32_t i = 0; i < n; ++i) {
    cell_range(g, boxes + 6 * (int64_t)i, lo, hi);
    for (int64_t a = lo[0]; a <= hi[0]; ++a)
      for (int64_t b = lo[1]; b <= hi[1]; ++b)
        for (int64_t c = lo[2]; c <= hi[2]; ++c) {
          e[k].key = cell_key(g, a, b, c);
          e[k].item = i;
          ++k;
        }
  }
  qsort(e, (size_t)tot, sizeof(or_cell_ent), cmp_ent);
  *n_out = tot;
  return e;
}

/* cell <= 0: twice the mean largest box extent of the faces and edges */
or_grid *or_grid_build(const or_scene *sc, const double *x, const double *x1, double dhat, double cell) {
  or_grid *g = (or_grid *)calloc(1, sizeof(or_grid));
  g->sc = sc;
  double h = 0.5 * dhat;
  g->vbox = (double *)malloc(sizeof(double) * 6 * (size_t)sc->n_vert + 8);
  g->fbox = (double *)malloc(sizeof(double) * 6 * (size_t)sc->n_face + 8);
  g->ebox = (double *)malloc(sizeof(double) * 6 * (size_t)sc->n_edge + 8);
  for (int32_t v = 0; v < sc->n_vert; ++v) prim_box(x, x1, &v, 1, h, g->vbox + 6 * (int64_t)v, g->vbox + 6 * (int64_t)v + 3);
  for (int32_t f = 0; f < sc->n_face; ++f)
    prim_box(x, x1, sc->faces + 3 * (int64_t)f, 3, h, g->fbox + 6 * (int64_t)f, g->fbox + 6 * (int64_t)f + 3);
  for (int32_t e = 0; e < sc->n_edge; ++e)
    prim_box(x, x1, sc->edges + 2 * (int64_t)e, 2, h, g->ebox + 6 * (int64_t)e, g->ebox + 6 * (int64_t)e + 3);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double ext = 0.0;
  int64_t n_ext = 0;
  const double *sets[3] = {g->vbox, g->fbox, g->ebox};
  const int32_t counts[3] = {sc->n_vert, sc->n_face, sc->n_edge};
  for (int s = 0; s < 3; ++s)
    for (int32_t i = 0; i < counts[s]; ++i) {
      const double *b = sets[s] + 6 * (int64_t)i;
      double m = 0.0;
      for (int c = 0; c < 3; ++c) {
        if (b[c] < lo[c]) lo[c] = b[c];
        if (b[3 + c] > hi[c]) hi[c] = b[3 + c];
        if (b[3 + c] - b[c] > m) m = b[3 + c] - b[c];
      }
      if (s > 0) {
        ext += m;
        ++n_ext;
      }
    }
  if (cell <= 0.0) cell = n_ext > 0 ? 2.0 * ext / (double)n_ext : 1.0;
  if (!(lo[0] <= hi[0])) lo[0] = lo[1] = lo[2] = hi[0] = hi[1] = hi[2] = 0.0;
  /* keep the cell count within int64 keys */
  for (;;) {
    double tot = 1.0;
    for (int c = 0; c < 3; ++c) tot *= floor((hi[c] - lo[c]) / cell) + 1.0;
    if (tot < 1e15) break;
    cell *= 2.0;
  }
  g->cell = cell;
  for (int c = 0; c < 3; ++c) {
    g->origin[c] = lo[c];
    g->dims[c] = cell_index(hi[c], lo[c], cell) + 1;
  }
  g->fent = grid_entries(g, g->fbox, sc->n_face, &g->n_fent);
  g->eent = grid_entries(g, g->ebox, sc->n_edge, &g->n_eent);
  return g;
}

void or_grid_free(or_grid *g) {
  if (!g) return;
  free(g->vbox);
  free(g->fbox);
  free(g->ebox);
  free(g->fent);
  free(g->eent);
  free(g);
}

double or_grid_cell(const or_grid *g) { return g->cell; }

static int64_t lower_key(const or_cell_ent *e, int64_t n, int64_t key) {
  int64_t a = 0, b = n;
  while (a < b) {
    int64_t m = a + (b - a) / 2;
    if (e[m].key < key) a = m + 1; else b = m;
  }
  return a;
}

/* Candidates of queries q0 <= q < q1 of one kind (0: vertex against faces,
 * 1: edge against later edges), in (query, item) order.  Returns the
 * number of pairs; writes the first `cap` to out (2 int32 each). */
int64_t or_grid_pairs(const or_grid *g, int kind, int32_t q0, int32_t q1, int32_t *out, int64_t cap) {
  const or_scene *sc = g->sc;
  const or_cell_ent *ent = kind == 0 ? g->fent : g->eent;
  const int64_t n_ent = kind == 0 ? g->n_fent : g->n_eent;
  const double *qbox = kind == 0 ? g->vbox : g->ebox;
  const double *ibox = kind == 0 ? g->fbox : g->ebox;
  int64_t bufcap = 1024, n = 0;
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)bufcap);
  for (int32_t qi = q0; qi < q1; ++qi) {
    const double *qb = qbox + 6 * (int64_t)qi;
    int64_t lo[3], hi[3], nb = 0;
    cell_range(g, qb, lo, hi);
    for (int64_t a = lo[0]; a <= hi[0]; ++a)
      for (int64_t b = lo[1]; b <= hi[1]; ++b)
        for (int64_t c = lo[2]; c <= hi[2]; ++c) {
          if (a < 0 || b < 0 || c < 0 || a >= g->dims[0] || b >= g->dims[1] || c >= g->dims[2]) continue;
          int64_t key = cell_key(g, a, b, c);
          for (int64_t k = lower_key(ent, n_ent, key); k < n_ent && ent[k].key == key; ++k) {
            if (nb == bufcap) {
              bufcap *= 2;
              buf = (int32_t *)realloc(buf, sizeof(int32_t) * (size_t)bufcap);
            }
            buf[nb++] = ent[k].item;
          }
        }
    qsort(buf, (size_t)nb, sizeof(int32_t), cmp_i32);
    for (int64_t k = 0; k < nb; ++k) {
      int32_t it = buf[k];
      if (k > 0 && buf[k - 1] == it) continue;
      if (kind == 0) {
        const int32_t *fv = sc->faces + 3 * (int64_t)it;
        if (fv[0] == qi || fv[1] == qi || fv[2] == qi) continue;
        if (!has_dof(sc, qi) && !has_dof(sc, fv[0]) && !has_dof(sc, fv[1]) && !has_dof(sc, fv[2])) continue;
      } else {
        if (it <= qi) continue;
        const int32_t *ea = sc->edges + 2 * (int64_t)qi, *eb = sc->edges + 2 * (int64_t)it;
        if (ea[0] == eb[0] || ea[0] == eb[1] || ea[1] == eb[0] || ea[1] == eb[1]) continue;
        if (!has_dof(sc, ea[0]) && !has_dof(sc, ea[1]) && !has_dof(sc, eb[0]) && !has_dof(sc, eb[1])) continue;
      }
      const double *ib = ibox + 6 * (int64_t)it;
      if (!boxes_overlap(qb, qb + 3, ib, ib + 3)) continue;
      if (n < cap) {
        out[2 * n] = qi;
        out[2 * n + 1] = it;
      }
      ++n;
    }
  }
  free(buf);
  return n;
}

/* ------------------------------------------------------------------ */
/* Reduction through the embedding (Eq. 17) into block-sparse rows: the */
/* same pair loop, pair order and Neumaier-compensated sums as          */
/* or_barrier_reduce, with the reduced Hessian kept as the 3x3 blocks   */
/* (I, J) the pairs touch (both triangles) instead of a dense matrix.   */
/* Row I holds its blocks sorted by column (binary search, insertion).  */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t n, cap;
  int32_t *col;
  double *val, *comp; /* [cap][9] */
} or_row;

struct or_bsr {
  int32_t n_rows;
  or_row *rows;
};

static double *row_block(or_row *r, int32_t J, double **comp) {
  int32_t a = 0, b = r->n;
  while (a < b) {
    int32_t m = a + (b - a) / 2;
    if (r->col[m] < J) a = m + 1; else b = m;
  }
  if (a == r->n || r->col[a] != J) {
    if (r->n == r->cap) {
      r->cap = r->cap ? 2 * r->cap : 8;
      r->col = (int32_t *)realloc(r->col, sizeof(int32_t) * (size_t)r->cap);
      r->val = (double *)realloc(r->val, sizeof(double) * 9 * (size_t)r->cap);
      r->comp = (double *)realloc(r->comp, sizeof(double) * 9 * (size_t)r->cap);
    }
    memmove(r->col + a + 1, r->col + a, sizeof(int32_t) * (size_t)(r->n - a));
    memmove(r->val + 9 * (int64_t)(a + 1), r->val + 9 * (int64_t)a, sizeof(double) * 9 * (size_t)(r->n - a));
    memmove(r->comp + 9 * (int64_t)(a + 1), r->comp + 9 * (int64_t)a, sizeof(double) * 9 * (size_t)(r->n - a));
    r->col[a] = J;
    memset(r->val + 9 * (int64_t)a, 0, sizeof(double) * 9);
    memset(r->comp + 9 * (int64_t)a, 0, sizeof(double) * 9);
    ++r->n;
  }
  *comp = r->comp + 9 * (int64_t)a;
  return r->val + 9 * (int64_t)a;
}

or_bsr *or_barrier_reduce_bsr(const or_scene *sc, const double *q, const int32_t *pt, int64_t n_pt,
                              const int32_t *ee, int64_t n_ee, double dhat, double kappa, uint32_t flags,
                              double *energy, double *grad_q, int64_t *n_active, int *status_out) {
  int64_t nd = 3 * (int64_t)sc->n_node;
  double *x = (double *)malloc(sizeof(double) * 3 * (size_t)sc->n_vert + 8);
  or_embed(sc, q, sc->x_off, x);
  or_bsr *B = (or_bsr *)calloc(1, sizeof(or_bsr));
  B->n_rows = sc->n_node;
  B->rows = (or_row *)calloc((size_t)sc->n_node + 1, sizeof(or_row));
  double es = 0.0, ec = 0.0;
  double *gc = grad_q ? (double *)calloc((size_t)nd + 1, sizeof(double)) : NULL;
  if (grad_q) memset(grad_q, 0, sizeof(double) * nd);
  int64_t na = 0;
  int status = OR_OK;
  int moll = (flags & OR_MOLLIFY) && sc->x_rest;
  for (int kind = 0; kind < 2; ++kind) {
    const int32_t *list = kind == 0 ? pt : ee;
    int64_t n = kind == 0 ? n_pt : n_ee;
    for (int64_t k = 0; k < n; ++k) {
      int32_t vid[4];
      pair_vertices(sc, kind, list + 2 * k, vid);
      double x12[12], r12[12];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) {
          x12[3 * a + c] = x[3 * vid[a] + c];
          if (moll) r12[3 * a + c] = sc->x_rest[3 * vid[a] + c];
        }
      double e, g[12], H[144], P[144];
      int st = or_pair_eval_f(kind, x12, moll ? r12 : NULL, dhat, kappa, flags, NULL, NULL, &e, g, H);
      if (st == OR_INACTIVE) continue;
      if (st != OR_OK) {
        status = st;
        continue;
      }
      ++na;
      nsum(&es, &ec, e);
      const double *Hu = H;
      if ((flags & OR_HESS) && (flags & OR_PROJECT)) {
        or_project_psd(12, H, P);
        Hu = P;
      }
      for (int a = 0; a < 4; ++a)
        for (int32_t ka = sc->rowptr[vid[a]]; ka < sc->rowptr[vid[a] + 1]; ++ka) {
          int32_t I = sc->col[ka];
          double wa = sc->val[ka];
          if (grad_q)
            for (int i = 0; i < 3; ++i) nsum(&grad_q[3 * I + i], &gc[3 * I + i], wa * g[3 * a + i]);
          if (!(flags & OR_HESS)) continue;
          for (int b = 0; b < 4; ++b)
            for (int32_t kb = sc->rowptr[vid[b]]; kb < sc->rowptr[vid[b] + 1]; ++kb) {
              int32_t J = sc->col[kb];
              double wab = wa * sc->val[kb];
              double *cmp;
              double *blk = row_block(&B->rows[I], J, &cmp);
              for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) nsum(&blk[3 * i + j], &cmp[3 * i + j], wab * Hu[(3 * a + i) * 12 + 3 * b + j]);
            }
        }
    }
  }
  if (grad_q)
    for (int64_t i = 0; i < nd; ++i) grad_q[i] += gc[i];
  for (int32_t I = 0; I < B->n_rows; ++I) {
    or_row *r = &B->rows[I];
    for (int64_t t = 0; t < 9 * (int64_t)r->n; ++t) r->val[t] += r->comp[t];
  }
  if (energy) *energy = es + ec;
  if (n_active) *n_active = na;
  if (status_out) *status_out = status;
  free(gc);
  free(x);
  return B;
}

int64_t or_bsr_nnzb(const or_bsr *B) {
  int64_t t = 0;
  for (int32_t I = 0; I < B->n_rows; ++I) t += B->rows[I].n;
  return t;
}

void or_bsr_copy(const or_bsr *B, int32_t *rowptr, int32_t *col, double *blocks) {
  int64_t p = 0;
  rowptr[0] = 0;
  for (int32_t I = 0; I < B->n_rows; ++I) {
    const or_row *r = &B->rows[I];
    memcpy(col + p, r->col, sizeof(int32_t) * (size_t)r->n);
    memcpy(blocks + 9 * p, r->val, sizeof(double) * 9 * (size_t)r->n);
    p += r->n;
    rowptr[I + 1] = (int32_t)p;
  }
}

void or_bsr_free(or_bsr *B) {
  if (!B) return;
  for (int32_t I = 0; I < B->n_rows; ++I) {
    free(B->rows[I].col);
    free(B->rows[I].val);
    free(B->rows[I].comp);
  }
  free(B->rows);
  free(B);
}

/* Narrow phase of a pair list (O3 and the indicator of Eq. 7): the
 * distance type and squared distance of every pair, and whether it is
 * active, 0 < d^2 < dhat^2 (d^2 < dhat^2 tested against dhat*dhat). */
void or_narrow(const or_scene *sc, const double *x, int kind, const int32_t *pairs, int64_t n, double dhat,
               int32_t *type, double *s2, uint8_t *active) {
  for (int64_t k = 0; k < n; ++k) {
    int32_t vid[4];
    pair_vertices(sc, kind, pairs + 2 * k, vid);
    double x12[12];
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) x12[3 * a + c] = x[3 * vid[a] + c];
    int t = kind == 0 ? or_pt_type(x12, x12 + 3, x12 + 6, x12 + 9) : or_ee_type(x12, x12 + 3, x12 + 6, x12 + 9);
    double s = or_pair_dist2(kind, t, x12);
    if (type) type[k] = t;
    if (s2) s2[k] = s;
    if (active) active[k] = (uint8_t)(s > 0.0 && s < dhat * dhat);
  }
}

/* ------------------------------------------------------------------ */
/* Lagged friction (Sec. III-B): D_k(x, x^n) = mu lambda_k^n f0(|u_k|),  */
/*   f1(y) = -y^2/(eps_v h)^2 + 2y/(eps_v h) on (0, eps_v h), 1 above;   */
/*   f0(x) = integral of f1 from eps_v h to x, plus eps_v h.            */
/* Readings (the paper defers to IPC):                                  */
/*  - lambda_k^n = kappa |b'(d^n)| (times m(c^n) for a mollified EE     */
/*    pair), the magnitude of the barrier's normal force at x^n;        */
/*  - the closest points at x^n define signed weights beta over the     */
/*    pair's four vertices (point minus closest triangle point for PT,  */
/*    closest point of edge a minus that of edge b for EE), so the      */
/*    relative position is G x = sum_a beta_a x_a, and the contact      */
/*    normal is n = G x^n / |G x^n|;                                    */
/*  - u_k is the part of G (x - x^n) orthogonal to n (its length is     */
/*    the same in any orthonormal tangent frame).                      */
/* Lag record (11 doubles): lambda, beta[4], n[3], G x^n[3].            */
/* ------------------------------------------------------------------ */
void or_friction_f(double y, double epsvh, double *f0, double *f1, double *f1p) {
  if (y < epsvh) {
    double r = y / epsvh;
    *f0 = -(y * y * y) / (3.0 * epsvh * epsvh) + (y * y) / epsvh + epsvh / 3.0;
    *f1 = -(r * r) + 2.0 * r;
    *f1p = -2.0 * y / (epsvh * epsvh) + 2.0 / epsvh;
  } else {
    *f0 = y;
    *f1 = 1.0;
    *f1p = 0.0;
  }
}

/* closest-point weights of a classified pair: G x = sum_a beta_a x_a */
static void closest_weights(int kind, int type, const double *x12, double *beta) {
  const double *p0 = x12, *p1 = x12 + 3, *p2 = x12 + 6, *p3 = x12 + 9;
  for (int a = 0; a < 4; ++a) beta[a] = 0.0;
  if (kind == 0) {
    double w[3] = {0.0, 0.0, 0.0};
    if (type <= PT_T2) {
      w[type] = 1.0;
    } else if (type <= PT_E2) {
      int i = type - PT_E0, j = (i + 1) % 3; /* edges t0t1, t1t2, t2t0 */
      const double *ti = x12 + 3 * (1 + i), *tj = x12 + 3 * (1 + j);
      double e[3], r[3];
      sub3(tj, ti, e);
      sub3(p0, ti, r);
      double s = dot3(r, e) / dot3(e, e);
      w[i] = 1.0 - s;
      w[j] = s;
    } else {
      double e0[3], e1[3], r[3];
      sub3(p2, p1, e0);
      sub3(p3, p1, e1);
      sub3(p0, p1, r);
      double a = dot3(e0, e0), b = dot3(e0, e1), c = dot3(e1, e1);
      double d0 = dot3(e0, r), d1 = dot3(e1, r);
      double det = a * c - b * b;
      double u = (c * d0 - b * d1) / det, v = (a * d1 - b * d0) / det;
      w[0] = 1.0 - u - v;
      w[1] = u;
      w[2] = v;
    }
    beta[0] = 1.0;
    beta[1] = -w[0];
    beta[2] = -w[1];
    beta[3] = -w[2];
  } else {
    double s = 0.0, t = 0.0; /* closest points a0 + s (a1 - a0), b0 + t (b1 - b0) */
    double u[3], v[3];
    sub3(p1, p0, u);
    sub3(p3, p2, v);
    switch (type) {
      case EE_A0B0: s = 0.0; t = 0.0; break;
      case EE_A0B1: s = 0.0; t = 1.0; break;
      case EE_A1B0: s = 1.0; t = 0.0; break;
      case EE_A1B1: s = 1.0; t = 1.0; break;
      case EE_AB0: { double r[3]; sub3(p2, p0, r); s = dot3(r, u) / dot3(u, u); t = 0.0; break; }
      case EE_AB1: { double r[3]; sub3(p3, p0, r); s = dot3(r, u) / dot3(u, u); t = 1.0; break; }
      case EE_A0B: { double r[3]; sub3(p0, p2, r); t = dot3(r, v) / dot3(v, v); s = 0.0; break; }
      case EE_A1B: { double r[3]; sub3(p1, p2, r); t = dot3(r, v) / dot3(v, v); s = 1.0; break; }
      default: {
        double w[3];
        sub3(p0, p2, w);
        double a = dot3(u, u), b = dot3(u, v), c = dot3(v, v), d = dot3(u, w), e = dot3(v, w);
        double D = a * c - b * b;
        s = (b * e - c * d) / D;
        t = (a * e - b * d) / D;
      }
    }
    beta[0] = 1.0 - s;
    beta[1] = s;
    beta[2] = -(1.0 - t);
    beta[3] = -t;
  }
}

/* Lag record of one pair at x^n (see above); returns OR_OK, OR_INACTIVE
 * (lambda = 0: the pair adds no friction) or an error. */
int or_friction_lag(int kind, const double *x12, const double *rest12, double dhat, double kappa, double *lag) {
  return or_friction_lag_f(kind, x12, rest12, dhat, kappa, 0, lag);
}

/* OR_SQDIST: the normal force is kappa m |db/dd| of the squared-distance
 * barrier, 2 d |db/ds| */
int or_friction_lag_f(int kind, const double *x12, const double *rest12, double dhat, double kappa, uint32_t flags,
                      double *lag) {
  for (int i = 0; i < 11; ++i) lag[i] = 0.0;
  int type = kind == 0 ? or_pt_type(x12, x12 + 3, x12 + 6, x12 + 9) : or_ee_type(x12, x12 + 3, x12 + 6, x12 + 9);
  double s = or_pair_dist2(kind, type, x12);
  if (!isfinite(s)) return OR_ERR_NONFINITE;
  if (!(s < dhat * dhat)) return OR_INACTIVE;
  if (s <= 0.0) return OR_ERR_INTERSECTING;
  double d = sqrt(s), b, b1, b2;
  if (flags & OR_SQDIST) {
    or_barrier_sq(s, dhat * dhat, &b, &b1, &b2);
    b1 = 2.0 * d * b1;
  } else {
    or_barrier(d, dhat, &b, &b1, &b2);
  }
  double m = 1.0;
  if (kind == 1 && rest12) {
    double ur[3], vr[3], u[3], v[3], n[3], m1, m2;
    sub3(rest12 + 3, rest12, ur);
    sub3(rest12 + 9, rest12 + 6, vr);
    sub3(x12 + 3, x12, u);
    sub3(x12 + 9, x12 + 6, v);
    cross3(u, v, n);
    or_mollifier(dot3(n, n), 1e-3 * dot3(ur, ur) * dot3(vr, vr), &m, &m1, &m2);
  }
  double beta[4], gx[3] = {0.0, 0.0, 0.0};
  closest_weights(kind, type, x12, beta);
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) gx[c] += beta[a] * x12[3 * a + c];
  double gn = sqrt(dot3(gx, gx));
  lag[0] = kappa * m * fabs(b1);
  for (int a = 0; a < 4; ++a) lag[1 + a] = beta[a];
  for (int c = 0; c < 3; ++c) {
    lag[5 + c] = gx[c] / gn;
    lag[8 + c] = gx[c];
  }
  return OR_OK;
}

/* Friction energy of one lagged pair at x, its 12-gradient and 12x12
 * Hessian (exact; positive semidefinite by construction, no projection):
 *   w = G x - G x^n, u = P w with P = I - n n^T, y = |u|,
 *   D = mu lambda f0(y), grad_a = beta_a mu lambda f1(y)/y u,
 *   H_ab = beta_a beta_b mu lambda P [f1(y)/y I + (f1'(y) y - f1(y))/y^3 u u^T] P
 * (at y = 0 the bracket tends to 2/(eps_v h) I). */
void or_friction_pair(const double *x12, const double *lag, double mu, double epsvh, double *e, double *g12,
                      double *H144) {
  double lam = lag[0];
  const double *beta = lag + 1, *n = lag + 5, *c0 = lag + 8;
  double w[3] = {0.0, 0.0, 0.0}, P[9], u[3];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) w[c] += beta[a] * x12[3 * a + c];
  for (int c = 0; c < 3; ++c) w[c] = w[c] - c0[c];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[3 * i + j] = (i == j ? 1.0 : 0.0) - n[i] * n[j];
  for (int i = 0; i < 3; ++i) u[i] = P[3 * i] * w[0] + P[3 * i + 1] * w[1] + P[3 * i + 2] * w[2];
  double y = sqrt(dot3(u, u)), f0, f1, f1p;
  or_friction_f(y, epsvh, &f0, &f1, &f1p);
  double s1 = y > 0.0 ? f1 / y : 2.0 / epsvh;           /* f1(y)/y */
  double s2 = y > 0.0 ? (f1p * y - f1) / (y * y * y) : 0.0; /* (f1' y - f1)/y^3 */
  if (y > 0.0 && y < epsvh) s2 = -1.0 / (epsvh * epsvh * y); /* the same, without cancellation */
  double ml = mu * lam;
  if (e) *e = ml * f0;
  if (g12)
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) g12[3 * a + c] = beta[a] * (ml * s1 * u[c]);
  if (H144) {
    double M[9], K[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M[3 * i + j] = s1 * (i == j ? 1.0 : 0.0) + s2 * u[i] * u[j];
    /* K = P M P */
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) acc += P[3 * i + k] * M[3 * k + l] * P[3 * l + j];
        K[3 * i + j] = ml * acc;
      }
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) H144[(3 * a + i) * 12 + 3 * b + j] = beta[a] * beta[b] * K[3 * i + j];
  }
}

/* Lag records of pair lists at positions W q_n + x_off (inactive pairs get
 * lambda = 0). */
int or_friction_lag_list(const or_scene *sc, const double *q_n, int kind, const int32_t *pairs, int64_t n,
                         double dhat, double kappa, uint32_t flags, double *lag) {
  double *x = (double *)malloc(sizeof(double) * 3 * (size_t)sc->n_vert + 8);
  or_embed(sc, q_n, sc->x_off, x);
  int moll = (flags & OR_MOLLIFY) && sc->x_rest, status = OR_OK;
  for (int64_t k = 0; k < n; ++k) {
    int32_t vid[4];
    pair_vertices(sc, kind, pairs + 2 * k, vid);
    double x12[12], r12[12];
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) {
        x12[3 * a + c] = x[3 * vid[a] + c];
        if (moll) r12[3 * a + c] = sc->x_rest[3 * vid[a] + c];
      }
    int st = or_friction_lag_f(kind, x12, moll ? r12 : NULL, dhat, kappa, flags, lag + 11 * k);
    if (st != OR_OK && st != OR_INACTIVE) status = st;
  }
  free(x);
  return status;
}

/* Friction energy, reduced gradient and dense reduced Hessian (Eq. 17)
 * over lagged pair lists at positions W q + x_off, summed in list order
 * with Neumaier compensation. */
int or_friction_reduce(const or_scene *sc, const double *q, const int32_t *pt, int64_t n_pt, const double *lag_pt,
                       const int32_t *ee, int64_t n_ee, const double *lag_ee, double mu, double epsvh,
                       double *energy, double *grad_q, double *hess_q) {
  int64_t nd = 3 * (int64_t)sc->n_node;
  double *x = (double *)malloc(sizeof(double) * 3 * (size_t)sc->n_vert + 8);
  or_embed(sc, q, sc->x_off, x);
  double es = 0.0, ec = 0.0;
  double *gc = grad_q ? (double *)calloc((size_t)nd + 1, sizeof(double)) : NULL;
  double *hc = hess_q ? (double *)calloc((size_t)(nd * nd) + 1, sizeof(double)) : NULL;
  if (grad_q) memset(grad_q, 0, sizeof(double) * nd);
  if (hess_q) memset(hess_q, 0, sizeof(double) * nd * nd);
  for (int kind = 0; kind < 2; ++kind) {
    const int32_t *list = kind == 0 ? pt : ee;
    const double *lags = kind == 0 ? lag_pt : lag_ee;
    int64_t n = kind == 0 ? n_pt : n_ee;
    for (int64_t k = 0; k < n; ++k) {
      const double *lag = lags + 11 * k;
      if (lag[0] == 0.0) continue;
      int32_t vid[4];
      pair_vertices(sc, kind, list + 2 * k, vid);
      double x12[12], e, g[12], H[144];
      for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) x12[3 * a + c] = x[3 * vid[a] + c];
      or_friction_pair(x12, lag, mu, epsvh, &e, g, H);
      nsum(&es, &ec, e);
      for (int a = 0; a < 4; ++a)
        for (int32_t ka = sc->rowptr[vid[a]]; ka < sc->rowptr[vid[a] + 1]; ++ka) {
          int32_t I = sc->col[ka];
          double wa = sc->val[ka];
          if (grad_q)
            for (int i = 0; i < 3; ++i) nsum(&grad_q[3 * I + i], &gc[3 * I + i], wa * g[3 * a + i]);
          if (!hess_q) continue;
          for (int b = 0; b < 4; ++b)
            for (int32_t kb = sc->rowptr[vid[b]]; kb < sc->rowptr[vid[b] + 1]; ++kb) {
              int32_t J = sc->col[kb];
              double wab = wa * sc->val[kb];
              for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                  int64_t idx = (3 * (int64_t)I + i) * nd + 3 * J + j;
                  nsum(&hess_q[idx], &hc[idx], wab * H[(3 * a + i) * 12 + 3 * b + j]);
                }
            }
        }
    }
  }
  if (grad_q)
    for (int64_t i = 0; i < nd; ++i) grad_q[i] += gc[i];
  if (hess_q)
    for (int64_t i = 0; i < nd * nd; ++i) hess_q[i] += hc[i];
  if (energy) *energy = es + ec;
  free(gc);
  free(hc);
  free(x);
  return OR_OK;
}
