/*
 * FP64 CPU oracle for the batched LAD-LASSO solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code with the HIP path.
 *
 * Problem (Abstract; Sections 2.1, 2.2, 3.1):
 *     minimise  f(b) = sum_i |y_i - x_i . b| + lambda * sum_j |b_j|
 * over b in R^p, for X (n x p, row-major), y (n), lambda >= 0.
 *
 * Parity status of each entry point (what pins it is listed in the tests):
 *   orc_objective, orc_weighted_median, orc_coord_update, orc_brute_force,
 *   orc_lp_simplex, orc_certify, orc_solve (its result, with either section
 *   search), orc_backward, orc_solve_batch:
 *       pinned (brute force on tiny inputs, an independent LP solver,
 *       closed forms, LP duality, finite differences, single solves).
 *   orc_quadrature_update: pinned against the section minimum found by
 *       brute force over the section's kinks, to the search's bracket.
 *   The intermediate iterates of orc_solve's paper-method stages (the
 *   sequence of CCD sweeps and ternary probes) are "parity unpinned": the
 *   paper gives the search only as an outline (Sections 3.5-3.6), so only
 *   its certified end point is checked.
 */
#ifndef LADL_ORACLE_H
#define LADL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_P 64

typedef struct {
    int n, p;
    const double *X; /* row-major n x p */
    const double *y; /* n */
    double lambda;
} orc_prob;

typedef struct {
    double tol_f;      /* CCD stops when a sweep lowers f by <= tol_f * f          */
    double tol_s;      /* ternary bracket stops at hi-lo <= tol_s*(1+|lo|+|hi|)    */
    double lambda_min; /* effective lambda = max(lambda, lambda_min)               */
    int max_sweeps;    /* CCD sweep cap                                            */
    int max_ternary;   /* ternary iteration cap                                    */
    int max_rounds;    /* ternary rounds over successive axes; <0 means p          */
    int max_pivots;    /* edge-descent finisher pivot cap                          */
    int use_finisher;  /* 1: run the finisher when the paper's stages fail         */
    double chop_range; /* initial chop half-width, a fraction of max(1, |b_k|)     */
    int section;       /* 1-D section minimiser: ORC_SECTION_*                     */
    double tol_q;      /* quadrature bracket stops at hi-lo <= tol_q*(1+|lo|+|hi|) */
    int golden;        /* 1: golden-section split of the chop's bracket, else thirds */
} orc_opts;

/* how CCD minimises each 1-D section */
enum {
    ORC_SECTION_MEDIAN = 0,     /* exact lower weighted median of the kinks        */
    ORC_SECTION_QUADRATURE = 1  /* quadrature search on section values (Sec. 3.5)  */
};

/* stage codes reported by orc_solve */
enum {
    ORC_STAGE_CCD = 0,      /* first CCD + snap certified                        */
    ORC_STAGE_TERNARY = 1,  /* 1 + round index: a ternary-chop round certified   */
    ORC_STAGE_FINISHER = 100,
    ORC_STAGE_NONE = -1
};

typedef struct {
    double f;          /* objective at b                                         */
    int stage;         /* see enum above                                         */
    int certified;     /* KKT certificate holds                                  */
    int unique;        /* certificate holds with margin and X_{Z,S} well posed   */
    int nS;            /* |S|                                                    */
    uint64_t S_mask;   /* bit j set iff b_j != 0                                 */
    int Z[ORC_MAX_P];  /* zero-residual rows of the vertex, ascending, -1 padded */
    double umax;       /* max_{i in Z} |u_i|                                     */
    double cmax;       /* max_{j not in S} |c_j| - lambda   (<= 0 when feasible) */
    double gap;        /* f(b) - y.u (LP duality gap)                            */
    double margin_uc;  /* min(1 - max|u_Z|, min_{j not in S} (lambda-|c_j|)/(lambda+sum_{i in Z}|x_ij|)):
                          the dual slacks against the size of the terms through
                          which an error of u_Z enters them                  */
    double margin_r;   /* min over rows off Z of |r_i| / (|y_i| + sum_j |x_ij b_j|) */
    long sweeps, updates, probes, pivots;
    double f_ccd;      /* objective after the first CCD                          */
} orc_info;

void orc_default_opts(orc_opts *o);

/* Section 3.1 objective, Neumaier-compensated. */
double orc_objective(const orc_prob *P, const double *b);

/* Lower weighted median of m keys t with weights w > 0, ties ordered by
 * index: the first key in (t, index) order whose cumulative weight reaches
 * half the total.  Returns its index in 0..m-1 (or -1 if m == 0). */
int orc_weighted_median(int m, const double *t, const double *w);

/* One exact coordinate minimisation of f along axis j (Section 3.3 with the
 * 1-D section minimised exactly, Section 3.5).  Updates b[j] and r = y - Xb.
 * Returns the change of b[j]. */
double orc_coord_update(const orc_prob *P, double lambda, double *b, double *r, int j);

/* One coordinate minimisation of f along axis j by the quadrature search of
 * the section's values (Sections 1, 3.5 and 5; the bracket, the halving rule
 * and the stopping rule are written out in the source).  Updates b[j] and
 * r = y - Xb unless the search finds no value below f at the current b_j.
 * Returns the change of b[j]; *evals (nullable) is increased by the number
 * of section values computed. */
double orc_quadrature_update(const orc_prob *P, double lambda, double tol_q, double *b, double *r, int j,
                             long *evals);

/* Cyclic coordinate descent with one optional frozen axis (-1 = none).
 * Returns the number of sweeps; *f receives the objective. */
int orc_ccd(const orc_prob *P, const orc_opts *o, double lambda, double *b, double *r, int frozen,
            double *f, long *updates);

/* Vertex snap + KKT certificate at b (Sections 3.2 and LP duality).
 * On success b is replaced by the vertex X_{Z,S} b_S = y_Z, info is filled
 * and 1 is returned if the certificate holds. u (n, nullable) receives the
 * dual vector. */
int orc_certify(const orc_prob *P, double lambda, double *b, double *u, orc_info *info);

/* The paper's method + build-added finisher; b_init nullable (zeros). */
int orc_solve(const orc_prob *P, const orc_opts *o, const double *b_init, double *b, orc_info *info);

/* Section 3.2: evaluate f at every intersection of p hyperplanes drawn from
 * {x_i.b = y_i} U {b_j = 0}; returns min f, writes the minimiser. */
double orc_brute_force(const orc_prob *P, double lambda, double *b_best, long *n_vertices);

/* Section 3.1: the LP with split coefficients and split residuals solved by
 * a dense-tableau primal simplex.  Writes b and the dual u (n, nullable).
 * Returns the optimal objective, or NaN on failure. */
double orc_lp_simplex(const orc_prob *P, double lambda, double *b, double *u, long *pivots);

/* Closed-form gradient of L(b*) through the optimal vertex:
 * w = X_{Z,S}^{-T} g_S, dy_Z = w, dX_{Z,S} = -w b_S^T, zero elsewhere.
 * Z: nS row ids; S from b's non-zeros. Returns 0 on success. */
int orc_backward(const orc_prob *P, const double *b, const int *Z, const double *g, double *dy, double *dX);

/* Batch driver: num_solves solves, each a lambda path of path_len steps
 * (warm-started), spread over nthreads threads.  Layout as in the HIP
 * library: X packed row-major blocks at x_off[k], y at row_off[k], lambda at
 * lam[s*path_len + t], outputs of (s,t) at b + path_len*b_off[s] + t*p_s and
 * index s*path_len + t for the scalars, zrows padded to 32 per output,
 * margin_out (nullable) 2 doubles per output: margin_uc, margin_r.
 * Returns wall seconds of the solve loop. */
double orc_solve_batch(int num_solves, const int32_t *problem, const int64_t *row_off,
                       const int64_t *x_off, const int32_t *p_arr, const double *X, const double *y,
                       const double *lam, int path_len, const int64_t *b_off, const orc_opts *o,
                       int nthreads, double *b_out, double *f_out, int32_t *stage_out,
                       uint32_t *smask_out, int32_t *zrows_out, int32_t *cert_out, int64_t *counters_out,
                       double *margin_out);

#ifdef __cplusplus
}
#endif
#endif
