/* Oracle for the Embedded IPC contact stage: a plain, slow, FP64 CPU
 * implementation used only as test infrastructure (parity tests, the smoke
 * check and the CPU baseline timing).  It shares no code with the HIP
 * library and is never called by the product path.
 *
 * Build: gcc -O2 -ffp-contract=off (no fused multiply-add, IEEE
 * round-to-nearest), so every expression is evaluated exactly as written.
 *
 * Conventions: positions are AoS double[n_vert*3]; q is double[3*n_node]
 * (node-major xyz).  A pair is two int32: (vertex, face) for point-triangle
 * (PT) and (edge_a, edge_b) with edge_a < edge_b for edge-edge (EE).
 */
#ifndef EIPC_ORACLE_H
#define EIPC_ORACLE_H
#include <stdint.h>

typedef struct {
  int32_t n_vert, n_node, n_face, n_edge;
  const int32_t *faces;    /* [n_face*3] */
  const int32_t *edges;    /* [n_edge*2], a < b */
  const int32_t *rowptr;   /* W CSR [n_vert+1]; empty row: no DoF */
  const int32_t *col;      /* [nnz] node index */
  const double *val;       /* [nnz] barycentric weight */
  const double *x_off;     /* [n_vert*3] static/kinematic positions or NULL */
  const double *x_rest;    /* [n_vert*3] rest positions (EE mollifier) or NULL */
} or_scene;

enum { OR_ENERGY = 1, OR_GRAD = 2, OR_HESS = 4, OR_PROJECT = 8, OR_MOLLIFY = 16, OR_SQDIST = 32,
       OR_PROJECT_REDUCED = 64 /* or_barrier_reduce: project each pair's reduced local block W^T H W */ };
enum { OR_OK = 0, OR_INACTIVE = 1, OR_ERR_INTERSECTING = -3, OR_ERR_NONFINITE = -5,
       OR_ERR_CAPACITY = -2 };

/* distance types */
enum { PT_T0 = 0, PT_T1, PT_T2, PT_E0, PT_E1, PT_E2, PT_T };
enum { EE_A0B0 = 0, EE_A0B1, EE_A1B0, EE_A1B1, EE_AB0, EE_AB1, EE_A0B, EE_A1B, EE_AB };

void or_embed(const or_scene *sc, const double *q, const double *off, double *x);

int64_t or_pt_query(const or_scene *sc, const double *x, const double *x1, double dhat,
                    int32_t v, int32_t *out, int64_t cap);
int64_t or_ee_query(const or_scene *sc, const double *x, const double *x1, double dhat,
                    int32_t ea, int32_t *out, int64_t cap);
int or_candidates(const or_scene *sc, const double *x, const double *x1, double dhat,
                  int32_t *pt, int64_t cap_pt, int64_t *n_pt,
                  int32_t *ee, int64_t cap_ee, int64_t *n_ee);

int or_pt_type(const double *p, const double *t0, const double *t1, const double *t2);
int or_ee_type(const double *a0, const double *a1, const double *b0, const double *b1);
double or_pair_dist2(int kind, int type, const double *x12);
void or_pair_dist2_derivs(int kind, int type, const double *x12, double *s, double *g12,
                          double *H144);

void or_barrier(double d, double dhat, double *b, double *b1, double *b2);
void or_mollifier(double c, double eps_x, double *m, double *m1, double *m2);

int or_pair_eval(int kind, const double *x12, const double *rest12, double dhat, double kappa,
                 int *type, double *s, double *e, double *g12, double *H144);
/* or_pair_eval with flags (OR_SQDIST: the barrier in s = d^2, see or_barrier_sq) */
int or_pair_eval_f(int kind, const double *x12, const double *rest12, double dhat, double kappa, uint32_t flags,
                   int *type_out, double *s_out, double *e, double *g12, double *H144);
/* squared-distance barrier b(s) = -(s - shat)^2 ln(s / shat) and its s-derivatives */
void or_barrier_sq(double s, double shat, double *b, double *b1, double *b2);
int or_project_psd(int n, const double *A, double *P);

int or_barrier_reduce(const or_scene *sc, const double *q, const int32_t *pt, int64_t n_pt,
                      const int32_t *ee, int64_t n_ee, double dhat, double kappa,
                      uint32_t flags, double *energy, double *grad_q, double *hess_q,
                      int64_t *n_active);
int or_barrier_hvp(const or_scene *sc, const double *q, const int32_t *pt, int64_t n_pt,
                   const int32_t *ee, int64_t n_ee, double dhat, double kappa, uint32_t flags,
                   const double *v, const double *v_off, double *out, double *out_off);

double or_accd_pair(int kind, const double *x12, const double *p12, double s, double t_c,
                    int64_t max_iter, int64_t *iters);
int or_ccd_toi(const or_scene *sc, const double *x, const double *p, int kind,
               const int32_t *pairs, int64_t n, double s, double t_c, int64_t max_iter,
               double *t_out, int64_t *iters_out);
/* method 0: additive CCD (or_accd_pair); 1: conservative advancement along
 * the closest direction (or_c2a_pair) */
int or_ccd_toi_m(const or_scene *sc, const double *x, const double *p, int kind, const int32_t *pairs, int64_t n,
                 double s, double t_c, int64_t max_iter, int method, double *t_out, int64_t *iters_out);
double or_c2a_pair(int kind, const double *x12, const double *p12, double s, double t_c, int64_t max_iter,
                   int64_t *iters);
int or_ccd_max_step(const or_scene *sc, const double *q, const double *dq, const double *dx_off,
                    double dhat, double s, double t_max, int64_t max_iter, double *alpha,
                    int64_t *n_cand, int64_t *n_capped);

void or_narrow(const or_scene *sc, const double *x, int kind, const int32_t *pairs, int64_t n, double dhat,
               int32_t *type, double *s2, uint8_t *active);

/* uniform-grid broad phase (same pairs and order as or_candidates) */
typedef struct or_grid or_grid;
or_grid *or_grid_build(const or_scene *sc, const double *x, const double *x1, double dhat, double cell);
int64_t or_grid_pairs(const or_grid *g, int kind, int32_t q0, int32_t q1, int32_t *out, int64_t cap);
double or_grid_cell(const or_grid *g);
void or_grid_free(or_grid *g);

/* reduction with the reduced Hessian as block-sparse rows */
typedef struct or_bsr or_bsr;
or_bsr *or_barrier_reduce_bsr(const or_scene *sc, const double *q, const int32_t *pt, int64_t n_pt,
                              const int32_t *ee, int64_t n_ee, double dhat, double kappa, uint32_t flags,
                              double *energy, double *grad_q, int64_t *n_active, int *status);
int64_t or_bsr_nnzb(const or_bsr *B);
void or_bsr_copy(const or_bsr *B, int32_t *rowptr, int32_t *col, double *blocks);
void or_bsr_free(or_bsr *B);

/* lagged friction (Sec. III-B); lag record: lambda, beta[4], n[3], G x^n[3] */
void or_friction_f(double y, double epsvh, double *f0, double *f1, double *f1p);
int or_friction_lag(int kind, const double *x12, const double *rest12, double dhat, double kappa, double *lag);
int or_friction_lag_f(int kind, const double *x12, const double *rest12, double dhat, double kappa,
                      uint32_t flags, double *lag);
void or_friction_pair(const double *x12, const double *lag, double mu, double epsvh, double *e, double *g12,
                      double *H144);
int or_friction_lag_list(const or_scene *sc, const double *q_n, int kind, const int32_t *pairs, int64_t n,
                         double dhat, double kappa, uint32_t flags, double *lag);
int or_friction_reduce(const or_scene *sc, const double *q, const int32_t *pt, int64_t n_pt, const double *lag_pt,
                       const int32_t *ee, int64_t n_ee, const double *lag_ee, double mu, double epsvh,
                       double *energy, double *grad_q, double *hess_q);
#endif
