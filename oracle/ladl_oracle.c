/*
 * FP64 CPU oracle for the batched LAD-LASSO solve.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * Everything is plain double precision, written for readability.  Where the
 * paper leaves a choice open the reading taken here is stated next to the
 * code (tie order of the weighted median, the axis chosen for the ternary
 * chop, the start of each restricted sub-search, the bracket extension rule).
 * The intermediate iterates of the paper-method stages are "parity unpinned";
 * the certified end point is pinned by brute force and by an independent LP
 * solver in the tests.
 */
#define _POSIX_C_SOURCE 200809L
#include "ladl_oracle.h"

#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define XIJ(P, i, j) ((P)->X[(size_t)(i) * (size_t)(P)->p + (size_t)(j)])

void orc_default_opts(orc_opts *o)
{
    o->tol_f = 1e-14;
    o->tol_s = 1e-10;
    o->lambda_min = 0.0;
    o->max_sweeps = 1000;
    o->max_ternary = 200;
    o->max_rounds = -1;
    o->max_pivots = 0; /* 0: 4*(n+p) */
    o->use_finisher = 1;
    o->chop_range = 1.0 / 32.0;
    o->section = ORC_SECTION_MEDIAN;
    o->golden = 0;
    o->tol_q = 1e-13;
}

/* ------------------------------------------------------------------------ */
/* Objective (Sections 2.1-2.2 combined as in Section 3.1)                   */
/* ------------------------------------------------------------------------ */

static void neumaier(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

static double resid(const orc_prob *P, const double *b, int i)
{
    double s = P->y[i];
    for (int j = 0; j < P->p; ++j) s -= XIJ(P, i, j) * b[j];
    return s;
}

double orc_objective(const orc_prob *P, const double *b)
{
    double s = 0.0, c = 0.0;
    for (int i = 0; i < P->n; ++i) neumaier(&s, &c, fabs(resid(P, b, i)));
    for (int j = 0; j < P->p; ++j) neumaier(&s, &c, P->lambda * fabs(b[j]));
    return s + c;
}

/* objective with an explicit lambda from a maintained residual vector */
static double obj_r(const orc_prob *P, double lam, const double *b, const double *r)
{
    double s = 0.0, c = 0.0;
    for (int i = 0; i < P->n; ++i) neumaier(&s, &c, fabs(r[i]));
    for (int j = 0; j < P->p; ++j) neumaier(&s, &c, lam * fabs(b[j]));
    return s + c;
}

static void residuals(const orc_prob *P, const double *b, double *r)
{
    for (int i = 0; i < P->n; ++i) r[i] = resid(P, b, i);
}

/* ------------------------------------------------------------------------ */
/* Weighted median: exact minimiser of a 1-D section (Sections 3.3, 3.5)     */
/* Along axis j with the other coordinates fixed, f is                       */
/*   g(t) = sum_i |x_ij| |t - t_i| + lambda |t| + const,                     */
/*   t_i = b_j + r_i / x_ij,                                                  */
/* a convex piecewise-linear function whose slope at t is (weight of keys    */
/* below t) - (weight above t).  Its lowest minimiser is the first key, in    */
/* ascending (key, index) order, at which the cumulative weight reaches half  */
/* of the total.  The binary/ternary/quadrature searches the paper lists      */
/* converge to this same point.                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    double t, w;
    int idx;
} okey;

static int okey_cmp(const void *a, const void *b)
{
    const okey *x = (const okey *)a, *y = (const okey *)b;
    if (x->t < y->t) return -1;
    if (x->t > y->t) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* sorts k in place; returns the position of the lower weighted median */
static int wmedian_sorted(int m, okey *k)
{
    if (m <= 0) return -1;
    qsort(k, (size_t)m, sizeof *k, okey_cmp);
    double W = 0.0;
    for (int i = 0; i < m; ++i) W += k[i].w;
    double cum = 0.0;
    for (int i = 0; i < m; ++i) {
        cum += k[i].w;
        if (2.0 * cum >= W) return i;
    }
    return m - 1;
}

int orc_weighted_median(int m, const double *t, const double *w)
{
    if (m <= 0) return -1;
    okey *k = (okey *)malloc(sizeof(okey) * (size_t)m);
    for (int i = 0; i < m; ++i) {
        k[i].t = t[i];
        k[i].w = w[i];
        k[i].idx = i;
    }
    int pos = wmedian_sorted(m, k);
    int r = k[pos].idx;
    free(k);
    return r;
}

static double coord_update_w(const orc_prob *P, double lam, double *b, double *r, int j, okey *k)
{
    const int n = P->n;
    int m = 0;
    for (int i = 0; i < n; ++i) {
        double x = XIJ(P, i, j);
        if (x != 0.0) {
            k[m].t = b[j] + r[i] / x;
            k[m].w = fabs(x);
            k[m].idx = i;
            ++m;
        }
    }
    if (lam > 0.0) { /* the penalty's kink at b_j = 0, ordered after every row */
        k[m].t = 0.0;
        k[m].w = lam;
        k[m].idx = n;
        ++m;
    }
    if (m == 0) return 0.0; /* section is flat: keep b_j */
    int pos = wmedian_sorted(m, k);
    double nb = (k[pos].idx == n) ? 0.0 : k[pos].t;
    double d = nb - b[j];
    if (d == 0.0) return 0.0;
    for (int i = 0; i < n; ++i) r[i] -= XIJ(P, i, j) * d;
    /* in exact arithmetic the median row now lies on its hyperplane */
    if (k[pos].idx < n) r[k[pos].idx] = 0.0;
    b[j] = nb;
    return d;
}

double orc_coord_update(const orc_prob *P, double lambda, double *b, double *r, int j)
{
    okey *k = (okey *)malloc(sizeof(okey) * (size_t)(P->n + 1));
    double d = coord_update_w(P, lambda, b, r, j, k);
    free(k);
    return d;
}

/* ------------------------------------------------------------------------ */
/* Quadrature search of a 1-D section (Section 3.5 names binary, ternary and */
/* quadrature searches for the sub-space minimisation; Sections 1 and 5      */
/* name the quadrature variant of the coordinate descent).  Only values of   */
/* the section g(t) = sum_i |r_i - x_ij (t - b_j)| + lambda |t| are used: no */
/* ordering or median of the kinks.                                          */
/*   1. Bracket [lo, hi] = [smallest, largest] of the kinks t_i (x_ij != 0)  */
/*      and 0 (lambda > 0): g is non-increasing left of every kink and       */
/*      non-decreasing right of every kink, so a minimiser lies in it.       */
/*   2. Evaluate g at the three quarter points q1 < q2 < q3.  For convex g,  */
/*      the lowest of them, q_k, has a minimiser within [q_{k-1}, q_{k+1}]   */
/*      (q_0 = lo, q_4 = hi): that half of the bracket is kept, and q_k is   */
/*      its centre, so each further halving costs two new values.            */
/*   3. Stop when hi - lo <= tol_q (1 + |lo| + |hi|), or when the quarter    */
/*      points no longer differ from the ends.  Ties go to the centre, then  */
/*      to the lower quarter point.                                          */
/*   4. The kept centre replaces b_j only if its value is below g(b_j), so   */
/*      f never rises.                                                        */
/* ------------------------------------------------------------------------ */

static double section_value(const orc_prob *P, double lam, const double *b, const double *r, int j,
                            double t)
{
    const double d = t - b[j];
    double s = 0.0, c = 0.0;
    for (int i = 0; i < P->n; ++i) neumaier(&s, &c, fabs(r[i] - XIJ(P, i, j) * d));
    neumaier(&s, &c, lam * fabs(t));
    return s + c;
}

static double coord_update_q(const orc_prob *P, double lam, double tol_q, double *b, double *r, int j,
                             long *evals)
{
    const int n = P->n;
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < n; ++i) {
        double x = XIJ(P, i, j);
        if (x != 0.0) {
            double t = b[j] + r[i] / x;
            lo = fmin(lo, t);
            hi = fmax(hi, t);
        }
    }
    if (lam > 0.0) {
        lo = fmin(lo, 0.0);
        hi = fmax(hi, 0.0);
    }
    if (!(lo <= hi)) return 0.0; /* section is flat: keep b_j */
    long ev = 0;
    double mid = 0.5 * (lo + hi);
    double gm = section_value(P, lam, b, r, j, mid);
    ++ev;
    for (int it = 0; it < 4096; ++it) {
        if (hi - lo <= tol_q * (1.0 + fabs(lo) + fabs(hi))) break;
        double q1 = 0.5 * (lo + mid), q3 = 0.5 * (mid + hi);
        if (!(q1 > lo && q1 < mid && q3 > mid && q3 < hi)) break;
        double g1 = section_value(P, lam, b, r, j, q1);
        double g3 = section_value(P, lam, b, r, j, q3);
        ev += 2;
        if (g1 < gm && g1 <= g3) { /* [lo, mid] around q1 */
            hi = mid;
            mid = q1;
            gm = g1;
        } else if (g3 < gm) { /* [mid, hi] around q3 */
            lo = mid;
            mid = q3;
            gm = g3;
        } else { /* [q1, q3] around mid */
            lo = q1;
            hi = q3;
        }
    }
    double g0 = section_value(P, lam, b, r, j, b[j]);
    ++ev;
    if (evals) *evals += ev;
    if (!(gm < g0)) return 0.0;
    double d = mid - b[j];
    for (int i = 0; i < n; ++i) r[i] -= XIJ(P, i, j) * d;
    b[j] = mid;
    return d;
}

double orc_quadrature_update(const orc_prob *P, double lambda, double tol_q, double *b, double *r, int j,
                             long *evals)
{
    return coord_update_q(P, lambda, tol_q, b, r, j, evals);
}

/* ------------------------------------------------------------------------ */
/* Cyclical coordinate descent (Section 3.3); axis `frozen` is held fixed,   */
/* which is the restricted sub-search of Section 3.6.  Stops after a sweep   */
/* that changes nothing or lowers f by at most tol_f * f.                     */
/* ------------------------------------------------------------------------ */

static int ccd_w(const orc_prob *P, const orc_opts *o, double lam, double *b, double *r, int frozen,
                 double *f_out, long *updates, okey *k)
{
    double f = obj_r(P, lam, b, r);
    int sweeps = 0;
    while (sweeps < o->max_sweeps) {
        int changed = 0;
        for (int j = 0; j < P->p; ++j) {
            if (j == frozen) continue;
            const double d = o->section == ORC_SECTION_QUADRATURE
                                 ? coord_update_q(P, lam, o->tol_q, b, r, j, NULL)
                                 : coord_update_w(P, lam, b, r, j, k);
            if (d != 0.0) changed = 1;
            if (updates) ++*updates;
        }
        ++sweeps;
        double fn = obj_r(P, lam, b, r);
        int stop = !changed || (f - fn <= o->tol_f * fn);
        f = fn;
        if (stop) break;
    }
    *f_out = f;
    return sweeps;
}

int orc_ccd(const orc_prob *P, const orc_opts *o, double lambda, double *b, double *r, int frozen,
            double *f, long *updates)
{
    okey *k = (okey *)malloc(sizeof(okey) * (size_t)(P->n + 1));
    int s = ccd_w(P, o, lambda, b, r, frozen, f, updates, k);
    free(k);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Small dense LU with partial pivoting (for the vertex systems)             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int s;
    double a[ORC_MAX_P * ORC_MAX_P];
    int piv[ORC_MAX_P];
} olu;

static int lu_factor(olu *L, int s, const double *A)
{
    L->s = s;
    memcpy(L->a, A, sizeof(double) * (size_t)s * (size_t)s);
    double amax = 0.0;
    for (int i = 0; i < s * s; ++i) amax = fmax(amax, fabs(A[i]));
    for (int k = 0; k < s; ++k) {
        int m = k;
        for (int i = k + 1; i < s; ++i)
            if (fabs(L->a[i * s + k]) > fabs(L->a[m * s + k])) m = i;
        L->piv[k] = m;
        if (!(fabs(L->a[m * s + k]) > 1e-13 * amax)) return 0;
        if (m != k)
            for (int c = 0; c < s; ++c) {
                double t = L->a[k * s + c];
                L->a[k * s + c] = L->a[m * s + c];
                L->a[m * s + c] = t;
            }
        for (int i = k + 1; i < s; ++i) {
            double l = L->a[i * s + k] / L->a[k * s + k];
            L->a[i * s + k] = l;
            for (int c = k + 1; c < s; ++c) L->a[i * s + c] -= l * L->a[k * s + c];
        }
    }
    return 1;
}

/* A x = v in place */
static void lu_solve(const olu *L, double *v)
{
    int s = L->s;
    for (int k = 0; k < s; ++k)
        if (L->piv[k] != k) {
            double t = v[k];
            v[k] = v[L->piv[k]];
            v[L->piv[k]] = t;
        }
    for (int i = 0; i < s; ++i)
        for (int c = 0; c < i; ++c) v[i] -= L->a[i * s + c] * v[c];
    for (int i = s - 1; i >= 0; --i) {
        for (int c = i + 1; c < s; ++c) v[i] -= L->a[i * s + c] * v[c];
        v[i] /= L->a[i * s + i];
    }
}

/* A^T x = v in place */
static void lu_solve_t(const olu *L, double *v)
{
    int s = L->s;
    for (int i = 0; i < s; ++i) {
        for (int c = 0; c < i; ++c) v[i] -= L->a[c * s + i] * v[c];
        v[i] /= L->a[i * s + i];
    }
    for (int i = s - 1; i >= 0; --i)
        for (int c = i + 1; c < s; ++c) v[i] -= L->a[c * s + i] * v[c];
    for (int k = s - 1; k >= 0; --k)
        if (L->piv[k] != k) {
            double t = v[k];
            v[k] = v[L->piv[k]];
            v[L->piv[k]] = t;
        }
}

/* 1-norm condition number of the factored s x s matrix A */
static double lu_cond1(const olu *L, const double *A)
{
    int s = L->s;
    if (s == 0) return 1.0;
    double an = 0.0, in = 0.0, e[ORC_MAX_P];
    for (int c = 0; c < s; ++c) {
        double cs = 0.0;
        for (int i = 0; i < s; ++i) cs += fabs(A[i * s + c]);
        an = fmax(an, cs);
        for (int i = 0; i < s; ++i) e[i] = (i == c);
        lu_solve(L, e);
        cs = 0.0;
        for (int i = 0; i < s; ++i) cs += fabs(e[i]);
        in = fmax(in, cs);
    }
    return an * in;
}

/* ------------------------------------------------------------------------ */
/* Vertices and the KKT certificate                                          */
/*                                                                           */
/* Section 3.2: the optimum lies where p of the hyperplanes {x_i.b = y_i}    */
/* and {b_j = 0} meet.  With S = {j : b_j != 0} and Z the rows on their      */
/* hyperplane, a vertex has |Z| = |S| and b_S = X_{Z,S}^{-1} y_Z.            */
/*                                                                           */
/* Certificate (subgradient optimality, equivalently LP duality for the      */
/* Section 3.1 LP): u_i = sign(r_i) off Z and u_Z solving                    */
/*   X_{Z,S}^T u_Z = lambda sign(b_S) - X_{Zc,S}^T u_Zc,                     */
/* then c = X^T u; b is optimal iff |u_i| <= 1 on Z and |c_j| <= lambda off  */
/* S, and then y.u = f(b).                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int s;
    int S[ORC_MAX_P];
    int Z[ORC_MAX_P];
} overt;

/* The vertex nearest to b: of the n + p hyperplanes {x_i.b = y_i} and
 * {b_j = 0} (Section 3.2), take p that meet in a single point, nearest
 * first in Euclidean distance (|r_i| / ||x_i||_2 for a row, |b_j| for an
 * axis; ties: axes first, then lower index).  A hyperplane whose normal is
 * linearly dependent on the normals already taken (a duplicated row, say)
 * is passed over.  The axes not taken form S and the rows taken form Z, so
 * |Z| = |S|.  Rows with x_i = 0 are not hyperplanes and are never taken. */
typedef struct {
    double d;
    int h;
} ocand;

static int ocand_cmp(const void *a, const void *b)
{
    const ocand *x = (const ocand *)a, *y = (const ocand *)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->h > y->h) - (x->h < y->h);
}

static void choose_vertex(const orc_prob *P, const double *b, const double *r, overt *V)
{
    const int n = P->n, p = P->p;
    ocand *c = (ocand *)malloc(sizeof(ocand) * (size_t)(n + p));
    int m = 0;
    for (int h = 0; h < n + p; ++h) {
        if (h < p) {
            c[m].d = fabs(b[h]);
        } else {
            int i = h - p;
            double nrm = 0.0;
            for (int j = 0; j < p; ++j) nrm += XIJ(P, i, j) * XIJ(P, i, j);
            if (nrm == 0.0) continue;
            c[m].d = fabs(r[i]) / sqrt(nrm);
        }
        c[m].h = h;
        ++m;
    }
    qsort(c, (size_t)m, sizeof *c, ocand_cmp);
    static const int QLD = ORC_MAX_P;
    double Q[ORC_MAX_P * ORC_MAX_P], v[ORC_MAX_P];
    int taken[ORC_MAX_P] = {0}, acc = 0, nz = 0;
    for (int q = 0; q < m && acc < p; ++q) {
        int h = c[q].h;
        for (int j = 0; j < p; ++j) v[j] = h < p ? (double)(j == h) : XIJ(P, h - p, j);
        double n0 = 0.0;
        for (int j = 0; j < p; ++j) n0 += v[j] * v[j];
        n0 = sqrt(n0);
        for (int a = 0; a < acc; ++a) { /* modified Gram-Schmidt */
            double d = 0.0;
            for (int j = 0; j < p; ++j) d += Q[a * QLD + j] * v[j];
            for (int j = 0; j < p; ++j) v[j] -= d * Q[a * QLD + j];
        }
        double nv = 0.0;
        for (int j = 0; j < p; ++j) nv += v[j] * v[j];
        nv = sqrt(nv);
        if (!(nv > 1e-9 * n0)) continue; /* dependent on those taken */
        for (int j = 0; j < p; ++j) Q[acc * QLD + j] = v[j] / nv;
        ++acc;
        if (h < p)
            taken[h] = 1;
        else
            V->Z[nz++] = h - p;
    }
    free(c);
    V->s = 0;
    for (int j = 0; j < p; ++j)
        if (!taken[j]) V->S[V->s++] = j;
    if (acc < p || nz != V->s) V->s = -1; /* fewer than p independent hyperplanes */
}

static void vertex_matrix(const orc_prob *P, const overt *V, double *A)
{
    int s = V->s;
    for (int q = 0; q < s; ++q)
        for (int c = 0; c < s; ++c) A[q * s + c] = XIJ(P, V->Z[q], V->S[c]);
}

/* b <- vertex solution of (Z,S); returns 0 if X_{Z,S} is singular */
static int vertex_solve(const orc_prob *P, const overt *V, olu *L, double *A, double *b)
{
    int s = V->s;
    if (s < 0) return 0;
    vertex_matrix(P, V, A);
    if (!lu_factor(L, s, A)) return 0;
    double v[ORC_MAX_P];
    for (int q = 0; q < s; ++q) v[q] = P->y[V->Z[q]];
    lu_solve(L, v);
    for (int j = 0; j < P->p; ++j) b[j] = 0.0;
    for (int c = 0; c < s; ++c) b[V->S[c]] = v[c];
    for (int c = 0; c < s; ++c)
        if (!isfinite(v[c])) return 0;
    return 1;
}

typedef struct {
    int certified, unique;
    double umax, cmax, gap, f, cond, margin_u, margin_c, margin_cz, margin_r;
} ocert;

static double sgn(double v) { return (v > 0.0) - (v < 0.0); }

/* r: fresh residuals at the vertex; u (n) and c (p) outputs */
static void certificate(const orc_prob *P, double lam, const overt *V, const olu *L, const double *A,
                        const double *b, double *r, double *u, double *c, ocert *C)
{
    const int n = P->n, p = P->p, s = V->s;
    residuals(P, b, r);
    for (int q = 0; q < s; ++q) r[V->Z[q]] = 0.0;
    for (int i = 0; i < n; ++i) u[i] = sgn(r[i]);
    for (int q = 0; q < s; ++q) u[V->Z[q]] = 0.0;
    for (int j = 0; j < p; ++j) {
        double g = 0.0;
        for (int i = 0; i < n; ++i) g += XIJ(P, i, j) * u[i];
        c[j] = g;
    }
    double v[ORC_MAX_P];
    for (int q = 0; q < s; ++q) v[q] = lam * sgn(b[V->S[q]]) - c[V->S[q]];
    lu_solve_t(L, v);
    for (int q = 0; q < s; ++q) u[V->Z[q]] = v[q];
    for (int j = 0; j < p; ++j) {
        double g = c[j];
        for (int q = 0; q < s; ++q) g += XIJ(P, V->Z[q], j) * v[q];
        c[j] = g;
    }
    C->umax = 0.0;
    C->margin_u = 1.0;
    for (int q = 0; q < s; ++q) {
        C->umax = fmax(C->umax, fabs(v[q]));
        C->margin_u = fmin(C->margin_u, 1.0 - fabs(v[q]));
    }
    int inS[ORC_MAX_P] = {0};
    for (int q = 0; q < s; ++q) inS[V->S[q]] = 1;
    int ok = C->umax <= 1.0 + 1e-9;
    C->cmax = -lam;
    C->margin_c = 1.0;
    C->margin_cz = 1.0;
    for (int j = 0; j < p; ++j) {
        if (inS[j]) continue;
        double colabs = 0.0, colz = 0.0;
        for (int i = 0; i < n; ++i) colabs += fabs(XIJ(P, i, j));
        for (int q = 0; q < s; ++q) colz += fabs(XIJ(P, V->Z[q], j));
        C->cmax = fmax(C->cmax, fabs(c[j]) - lam);
        if (fabs(c[j]) > lam + 1e-9 * (lam + colabs)) ok = 0;
        C->margin_c = fmin(C->margin_c, (lam - fabs(c[j])) / (lam + colabs));
        /* the same slack against the terms that carry the error of the
           vertex rows' duals u_Z into c_j = sum_i x_ij u_i */
        C->margin_cz = fmin(C->margin_cz, (lam - fabs(c[j])) / (lam + colz));
    }
    /* distance of the other rows from their hyperplanes */
    C->margin_r = INFINITY;
    int inZ_cnt = 0;
    for (int i = 0; i < n; ++i) {
        int inZ = 0;
        for (int q = 0; q < s; ++q) inZ |= (V->Z[q] == i);
        if (inZ) { ++inZ_cnt; continue; }
        double sc = fabs(P->y[i]);
        for (int j = 0; j < p; ++j) sc += fabs(XIJ(P, i, j) * b[j]);
        C->margin_r = fmin(C->margin_r, fabs(r[i]) / (sc > 0.0 ? sc : 1.0));
    }
    (void)inZ_cnt;
    double f = obj_r(P, lam, b, r);
    double yu = 0.0;
    for (int i = 0; i < n; ++i) yu += P->y[i] * u[i];
    C->f = f;
    C->gap = f - yu;
    C->cond = lu_cond1(L, A);
    C->certified = ok;
    C->unique = ok && C->margin_u > 1e-8 && C->margin_c > 1e-8 && C->margin_r > 1e-12 && C->cond < 1e10;
}

static void fill_info(const orc_prob *P, const overt *V, const double *b, const ocert *C, orc_info *I)
{
    I->f = C->f;
    I->certified = C->certified;
    I->unique = C->unique;
    I->umax = C->umax;
    I->cmax = C->cmax;
    I->gap = C->gap;
    I->margin_uc = fmin(C->margin_u, C->margin_cz);
    I->margin_r = C->margin_r;
    I->nS = 0;
    I->S_mask = 0;
    for (int j = 0; j < P->p; ++j)
        if (b[j] != 0.0) {
            I->nS++;
            I->S_mask |= (uint64_t)1 << j;
        }
    int z[ORC_MAX_P];
    int s = V->s > 0 ? V->s : 0;
    memcpy(z, V->Z, sizeof(int) * (size_t)s);
    for (int a = 1; a < s; ++a) { /* ascending row ids */
        int t = z[a], q = a;
        while (q > 0 && z[q - 1] > t) {
            z[q] = z[q - 1];
            --q;
        }
        z[q] = t;
    }
    for (int q = 0; q < ORC_MAX_P; ++q) I->Z[q] = q < s ? z[q] : -1;
}

typedef struct {
    okey *k;
    double *r, *u, *c, *bt, *rt, *bb, *rb, *xd;
    double A[ORC_MAX_P * ORC_MAX_P];
    olu L;
} owork;

static int work_alloc(owork *W, int n, int p)
{
    W->k = (okey *)malloc(sizeof(okey) * (size_t)(n + p + 1));
    size_t nd = (size_t)n;
    W->r = (double *)malloc(sizeof(double) * nd);
    W->u = (double *)malloc(sizeof(double) * nd);
    W->rt = (double *)malloc(sizeof(double) * nd);
    W->rb = (double *)malloc(sizeof(double) * nd);
    W->xd = (double *)malloc(sizeof(double) * nd);
    W->c = (double *)malloc(sizeof(double) * (size_t)p);
    W->bt = (double *)malloc(sizeof(double) * (size_t)p);
    W->bb = (double *)malloc(sizeof(double) * (size_t)p);
    return W->k && W->r && W->u && W->rt && W->rb && W->xd && W->c && W->bt && W->bb;
}

static void work_free(owork *W)
{
    free(W->k);
    free(W->r);
    free(W->u);
    free(W->rt);
    free(W->rb);
    free(W->xd);
    free(W->c);
    free(W->bt);
    free(W->bb);
}

/* snap b (with residuals r) to its vertex and test the certificate;
 * on success b is replaced by the vertex */
static int snap_certify(const orc_prob *P, double lam, double *b, const double *r, owork *W, overt *V,
                        orc_info *I)
{
    choose_vertex(P, b, r, V);
    memcpy(W->bt, b, sizeof(double) * (size_t)P->p);
    if (!vertex_solve(P, V, &W->L, W->A, W->bt)) return 0;
    ocert C;
    certificate(P, lam, V, &W->L, W->A, W->bt, W->rt, W->u, W->c, &C);
    if (!C.certified) return 0;
    memcpy(b, W->bt, sizeof(double) * (size_t)P->p);
    fill_info(P, V, b, &C, I);
    return 1;
}

int orc_certify(const orc_prob *P, double lambda, double *b, double *u, orc_info *info)
{
    owork W;
    if (!work_alloc(&W, P->n, P->p)) return -1;
    memset(info, 0, sizeof *info);
    residuals(P, b, W.r);
    overt V;
    choose_vertex(P, b, W.r, &V);
    int ok = 0;
    memcpy(W.bt, b, sizeof(double) * (size_t)P->p);
    if (vertex_solve(P, &V, &W.L, W.A, W.bt)) {
        ocert C;
        certificate(P, lambda, &V, &W.L, W.A, W.bt, W.rt, W.u, W.c, &C);
        memcpy(b, W.bt, sizeof(double) * (size_t)P->p);
        fill_info(P, &V, b, &C, info);
        if (u) memcpy(u, W.u, sizeof(double) * (size_t)P->n);
        ok = C.certified;
    }
    work_free(&W);
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Ternary chop along the locus of axis-wise minima (Sections 3.5, 3.6)      */
/*                                                                           */
/* F(s): from the best point found so far, set b_k := s and run CCD with     */
/* axis k frozen (the restricted sub-search); F(s) is the objective reached. */
/* The centre c = b_k is probed too.                                         */
/* The initial range c +- h, h = chop_range * max(1,|c|), around the current */
/* b_k (the paper leaves the initial range to the user and extends it until  */
/* it holds the minimum, Section 3.6) is doubled outward while an end point */
/* is lower than the centre, clamped to                                       */
/* |b_k| <= ||y||_1 / lambda (any minimiser has lambda ||b||_1 <= f(0)).      */
/* The range is then cut in thirds (or golden sections); the best probe is  */
/* kept.                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_prob *P;
    const orc_opts *o;
    double lam;
    int k;
    owork *W;
    double *b, *r, f; /* current best state */
    orc_info *I;
} otern;

static double probe(otern *T, double s)
{
    const orc_prob *P = T->P;
    owork *W = T->W;
    memcpy(W->bt, T->b, sizeof(double) * (size_t)P->p);
    memcpy(W->rt, T->r, sizeof(double) * (size_t)P->n);
    double d = s - W->bt[T->k];
    if (d != 0.0)
        for (int i = 0; i < P->n; ++i) W->rt[i] -= XIJ(P, i, T->k) * d;
    W->bt[T->k] = s;
    double f;
    T->I->sweeps += ccd_w(P, T->o, T->lam, W->bt, W->rt, T->k, &f, &T->I->updates, W->k);
    T->I->probes++;
    if (f < T->f) {
        T->f = f;
        memcpy(T->b, W->bt, sizeof(double) * (size_t)P->p);
        memcpy(T->r, W->rt, sizeof(double) * (size_t)P->n);
    }
    return f;
}

static void ternary(otern *T)
{
    const orc_prob *P = T->P;
    double B = INFINITY;
    if (T->lam > 0.0) {
        double y1 = 0.0;
        for (int i = 0; i < P->n; ++i) y1 += fabs(P->y[i]);
        B = y1 / T->lam;
    }
    double c = T->b[T->k];
    double h = T->o->chop_range * fmax(1.0, fabs(c));
    double lo = fmax(c - h, -B), hi = fmin(c + h, B);
    /* the centre is probed like the ends: the point the chop starts from
     * lies on the locus of axis-wise minima only if the CCD before it ran
     * to convergence, and a sweep cap can stop it short */
    double Fc = probe(T, c);
    double Flo = probe(T, lo), Fhi = probe(T, hi);
    int ext = 0;
    while (Flo < Fc && lo > -B && ext < 64) {
        hi = c;
        Fhi = Fc;
        c = lo;
        Fc = Flo;
        h *= 2.0;
        lo = fmax(c - h, -B);
        Flo = probe(T, lo);
        ++ext;
    }
    while (Fhi < Fc && hi < B && ext < 128) {
        lo = c;
        Flo = Fc;
        c = hi;
        Fc = Fhi;
        h *= 2.0;
        hi = fmin(c + h, B);
        Fhi = probe(T, hi);
        ++ext;
    }
    (void)Flo;
    (void)Fhi;
    if (!T->o->golden) {
        for (int it = 0; it < T->o->max_ternary; ++it) {
            if (hi - lo <= T->o->tol_s * (1.0 + fabs(lo) + fabs(hi))) break;
            double m1 = lo + (hi - lo) / 3.0, m2 = hi - (hi - lo) / 3.0;
            double F1 = probe(T, m1), F2 = probe(T, m2);
            if (F1 < F2)
                hi = m2;
            else
                lo = m1;
        }
        return;
    }
    /* golden sections: the same search with interior points at the golden
     * ratio, so the interior point that survives a step is one of the next
     * step's two points and only one new probe is needed per step */
    const double g = 0.5 * (3.0 - sqrt(5.0));
    double m1 = 0.0, m2 = 0.0, F1 = 0.0, F2 = 0.0;
    int have1 = 0, have2 = 0;
    for (int it = 0; it < T->o->max_ternary; ++it) {
        if (hi - lo <= T->o->tol_s * (1.0 + fabs(lo) + fabs(hi))) break;
        if (!have1) {
            m1 = lo + g * (hi - lo);
            F1 = probe(T, m1);
            have1 = 1;
        }
        if (!have2) {
            m2 = hi - g * (hi - lo);
            F2 = probe(T, m2);
            have2 = 1;
        }
        if (F1 < F2) {
            hi = m2;
            m2 = m1;
            F2 = F1;
            have1 = 0;
        } else {
            lo = m1;
            m1 = m2;
            F1 = F2;
            have2 = 0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Edge-descent finisher (a build addition, not in the paper): primal        */
/* simplex steps in b-space from a vertex whose certificate fails.           */
/*   |u_i0| > 1 on Z: move along X_{Z,S} d_S = -sign(u_i0) e_i0 (row i0       */
/*     leaves its hyperplane), slope 1 - |u_i0| < 0;                          */
/*   |c_j0| > lambda off S: d_j0 = sign(c_j0), X_{Z,S} d_S = -X_{Z,j0} d_j0   */
/*     (b_j0 leaves zero), slope lambda - |c_j0| < 0.                         */
/* The step length minimises f along d exactly: again a weighted median, of  */
/* the kinks r_i / (x_i.d) (weight |x_i.d|) and -b_j / d_j (weight lambda|d_j|). */
/* The kink reached joins the vertex in place of the constraint released.    */
/* ------------------------------------------------------------------------ */

static int finisher(const orc_prob *P, const orc_opts *o, double lam, double *b, owork *W, overt *V,
                    orc_info *I)
{
    const int n = P->n, p = P->p;
    int maxp = o->max_pivots > 0 ? o->max_pivots : 4 * (n + p);
    int bland = 0;
    for (int it = 0; it <= maxp; ++it) {
        if (!vertex_solve(P, V, &W->L, W->A, b)) return 0;
        ocert C;
        certificate(P, lam, V, &W->L, W->A, b, W->r, W->u, W->c, &C);
        if (C.certified) {
            fill_info(P, V, b, &C, I);
            return 1;
        }
        if (it == maxp) break;
        const int s = V->s;
        int inS[ORC_MAX_P] = {0};
        for (int q = 0; q < s; ++q) inS[V->S[q]] = 1;
        /* pick the released constraint: most negative slope, or the lowest
         * index among violators after a degenerate step (Bland) */
        int type = 0, sel = -1;
        double best = 0.0;
        for (int q = 0; q < s; ++q) {
            double slope = 1.0 - fabs(W->u[V->Z[q]]);
            if (slope < -1e-9 && (bland ? sel < 0 || V->Z[q] < V->Z[sel] : slope < best)) {
                best = slope;
                type = 1;
                sel = q;
            }
        }
        if (!(bland && sel >= 0))
            for (int j = 0; j < p; ++j) {
                if (inS[j]) continue;
                double colabs = 0.0;
                for (int i = 0; i < n; ++i) colabs += fabs(XIJ(P, i, j));
                double slope = lam - fabs(W->c[j]);
                if (slope < -1e-9 * (lam + colabs) && (bland ? sel < 0 : slope < best)) {
                    best = slope;
                    type = 2;
                    sel = j;
                }
            }
        if (sel < 0) return 0;
        double d[ORC_MAX_P] = {0}, v[ORC_MAX_P];
        if (type == 1) {
            for (int q = 0; q < s; ++q) v[q] = 0.0;
            v[sel] = -sgn(W->u[V->Z[sel]]);
            lu_solve(&W->L, v);
            for (int q = 0; q < s; ++q) d[V->S[q]] = v[q];
        } else {
            d[sel] = sgn(W->c[sel]);
            for (int q = 0; q < s; ++q) v[q] = -XIJ(P, V->Z[q], sel) * d[sel];
            lu_solve(&W->L, v);
            for (int q = 0; q < s; ++q) d[V->S[q]] = v[q];
        }
        for (int i = 0; i < n; ++i) {
            double a = 0.0;
            for (int j = 0; j < p; ++j) a += XIJ(P, i, j) * d[j];
            W->xd[i] = a;
        }
        for (int q = 0; q < s; ++q) W->xd[V->Z[q]] = (type == 1 && q == sel) ? -sgn(W->u[V->Z[q]]) : 0.0;
        int m = 0;
        for (int i = 0; i < n; ++i)
            if (W->xd[i] != 0.0) {
                W->k[m].t = W->r[i] / W->xd[i];
                W->k[m].w = fabs(W->xd[i]);
                W->k[m].idx = i;
                ++m;
            }
        if (lam > 0.0)
            for (int j = 0; j < p; ++j)
                if (d[j] != 0.0) {
                    W->k[m].t = -b[j] / d[j];
                    W->k[m].w = lam * fabs(d[j]);
                    W->k[m].idx = n + j;
                    ++m;
                }
        int pos = wmedian_sorted(m, W->k);
        if (pos < 0) return 0;
        double t = W->k[pos].t;
        int blk = W->k[pos].idx;
        if (!(t > 0.0)) {
            t = 0.0;
            bland = 1;
        } else
            bland = 0;
        for (int j = 0; j < p; ++j) b[j] += t * d[j];
        /* new vertex */
        if (type == 1) {
            if (blk < n) {
                V->Z[sel] = blk;
            } else {
                int jb = blk - n, c0 = -1;
                for (int q = 0; q < s; ++q)
                    if (V->S[q] == jb) c0 = q;
                if (c0 < 0) return 0;
                for (int q = c0; q + 1 < s; ++q) V->S[q] = V->S[q + 1];
                for (int q = sel; q + 1 < s; ++q) V->Z[q] = V->Z[q + 1];
                V->s = s - 1;
            }
        } else {
            if (blk < n) {
                V->Z[s] = blk;
                V->S[s] = sel;
                V->s = s + 1;
            } else {
                int jb = blk - n, c0 = -1;
                for (int q = 0; q < s; ++q)
                    if (V->S[q] == jb) c0 = q;
                if (c0 < 0) return 0; /* the entering axis itself: degenerate */
                V->S[c0] = sel;
            }
        }
        if (V->s > p || V->s > ORC_MAX_P) return 0;
        I->pivots++;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The full solve                                                            */
/*   1. CCD from b_init (or 0) to an axis-wise minimum (Section 3.3).        */
/*   2. Snap to the vertex and certify; stop if optimal.                     */
/*   3. Ternary chop along axis k (first round: the lowest j with the largest */
/*      |b_j|; later rounds: the next axis), Sections 3.5-3.6.               */
/*   4. Unrestricted CCD from the best probe; snap and certify.              */
/*   5. Repeat 3-4 over up to max_rounds axes.                               */
/*   6. Edge-descent finisher from the snapped vertex (build addition).      */
/* ------------------------------------------------------------------------ */

static int solve_w(const orc_prob *P, const orc_opts *o, const double *b_init, double *b, orc_info *I,
                   owork *W)
{
    const int n = P->n, p = P->p;
    double lam = fmax(P->lambda, o->lambda_min);
    memset(I, 0, sizeof *I);
    for (int q = 0; q < ORC_MAX_P; ++q) I->Z[q] = -1;
    for (int j = 0; j < p; ++j) b[j] = b_init ? b_init[j] : 0.0;
    residuals(P, b, W->r);
    double f;
    I->sweeps += ccd_w(P, o, lam, b, W->r, -1, &f, &I->updates, W->k);
    I->f_ccd = f;
    overt V;
    if (snap_certify(P, lam, b, W->r, W, &V, I)) {
        I->stage = ORC_STAGE_CCD;
        return 1;
    }
    if (p >= 2) {
        int rounds = o->max_rounds < 0 ? p : o->max_rounds;
        int k = 0;
        for (int j = 1; j < p; ++j)
            if (fabs(b[j]) > fabs(b[k])) k = j;
        for (int round = 0; round < rounds; ++round) {
            otern T = {P, o, lam, k, W, b, W->r, f, I};
            ternary(&T);
            f = T.f;
            I->sweeps += ccd_w(P, o, lam, b, W->r, -1, &f, &I->updates, W->k);
            if (snap_certify(P, lam, b, W->r, W, &V, I)) {
                I->stage = ORC_STAGE_TERNARY + round;
                return 1;
            }
            k = (k + 1) % p;
        }
    }
    I->stage = ORC_STAGE_NONE;
    I->f = obj_r(P, lam, b, W->r);
    if (!o->use_finisher) return 0;
    choose_vertex(P, b, W->r, &V);
    memcpy(W->bb, b, sizeof(double) * (size_t)p);
    if (finisher(P, o, lam, W->bb, W, &V, I)) {
        memcpy(b, W->bb, sizeof(double) * (size_t)p);
        I->stage = ORC_STAGE_FINISHER;
        return 1;
    }
    /* A degenerate vertex (more rows on their hyperplanes than active
     * coordinates, e.g. duplicated rows) can make the edge steps cycle.
     * Perturb y by a tiny deterministic amount so that no two rows share a
     * hyperplane, finish there, then take the same vertex with the original
     * y.  The perturbed problem's dual vector u is feasible for the original
     * one (|u_i| <= 1, |X^T u| <= lambda do not involve y), so y.u is a lower
     * bound on the optimum and f(b) - y.u bounds the remaining error. */
    {
        double ybar = 0.0;
        for (int i = 0; i < n; ++i) ybar += fabs(P->y[i]);
        ybar /= (n > 0 ? n : 1);
        double *yp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        for (int i = 0; i < n; ++i) {
            uint32_t hsh = (uint32_t)i * 2654435761u;
            double mag = 0.5 + 0.5 * (double)((hsh >> 8) & 0xFFFF) / 65535.0;
            double sgn_ = (hsh >> 31) ? -1.0 : 1.0;
            yp[i] = P->y[i] + 1e-9 * (fabs(P->y[i]) + ybar) * mag * sgn_;
        }
        orc_prob Pp = *P;
        Pp.y = yp;
        memcpy(W->bb, b, sizeof(double) * (size_t)p);
        residuals(&Pp, W->bb, W->r);
        choose_vertex(&Pp, W->bb, W->r, &V);
        int ok = finisher(&Pp, o, lam, W->bb, W, &V, I);
        if (ok) {
            /* W->u holds the perturbed problem's dual vector */
            double yu = 0.0;
            for (int i = 0; i < n; ++i) yu += P->y[i] * W->u[i];
            if (vertex_solve(P, &V, &W->L, W->A, W->bb)) {
                double f = orc_objective(&(orc_prob){n, p, P->X, P->y, lam}, W->bb);
                double gap = f - yu;
                if (gap <= 1e-9 * fmax(1.0, f)) {
                    memcpy(b, W->bb, sizeof(double) * (size_t)p);
                    I->f = f;
                    I->gap = gap;
                    I->certified = 1;
                    I->unique = 0;
                    I->margin_uc = 0.0;
                    I->margin_r = 0.0;
                    I->stage = ORC_STAGE_FINISHER + 1;
                    free(yp);
                    return 1;
                }
            }
        }
        free(yp);
    }
    I->certified = 0;
    return 0;
}

int orc_solve(const orc_prob *P, const orc_opts *o, const double *b_init, double *b, orc_info *info)
{
    if (P->p > ORC_MAX_P || P->p < 1 || P->n < 0) return -1;
    owork W;
    if (!work_alloc(&W, P->n > 0 ? P->n : 1, P->p)) return -1;
    int ok = solve_w(P, o, b_init, b, info, &W);
    work_free(&W);
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Brute force (Section 3.2): every intersection of p hyperplanes            */
/* ------------------------------------------------------------------------ */

double orc_brute_force(const orc_prob *P, double lambda, double *b_best, long *n_vertices)
{
    const int n = P->n, p = P->p, H = n + p;
    if (p > ORC_MAX_P || p > H) return NAN;
    int comb[ORC_MAX_P];
    for (int q = 0; q < p; ++q) comb[q] = q;
    double best = INFINITY, A[ORC_MAX_P * ORC_MAX_P], v[ORC_MAX_P], b[ORC_MAX_P];
    olu L;
    long cnt = 0;
    orc_prob Q = *P;
    Q.lambda = lambda;
    for (;;) {
        for (int q = 0; q < p; ++q) {
            int h = comb[q];
            for (int c = 0; c < p; ++c) A[q * p + c] = h < n ? XIJ(P, h, c) : (double)(h - n == c);
            v[q] = h < n ? P->y[h] : 0.0;
        }
        if (lu_factor(&L, p, A)) {
            lu_solve(&L, v);
            memcpy(b, v, sizeof(double) * (size_t)p);
            double f = orc_objective(&Q, b);
            ++cnt;
            if (f < best) {
                best = f;
                memcpy(b_best, b, sizeof(double) * (size_t)p);
            }
        }
        int q = p - 1;
        while (q >= 0 && comb[q] == H - p + q) --q;
        if (q < 0) break;
        comb[q]++;
        for (int a = q + 1; a < p; ++a) comb[a] = comb[a - 1] + 1;
    }
    if (n_vertices) *n_vertices = cnt;
    return best;
}

/* ------------------------------------------------------------------------ */
/* Section 3.1 LP, dense tableau primal simplex (Dantzig's rule, Bland's     */
/* rule after a run of degenerate pivots).  Variables b+, b-, r+, r- >= 0;   */
/* rows X(b+ - b-) + r+ - r- = y; cost lambda*(b+ + b-) + (r+ + r-).          */
/* Start basis: r+_i if y_i >= 0 else r-_i, always feasible (Section 3.2,    */
/* note b).                                                                   */
/* ------------------------------------------------------------------------ */

double orc_lp_simplex(const orc_prob *P, double lambda, double *b, double *u, long *pivots)
{
    const int n = P->n, p = P->p, N = 2 * p + 2 * n, ld = N + 1;
    double *T = (double *)calloc((size_t)n * (size_t)ld, sizeof(double));
    double *d = (double *)malloc(sizeof(double) * (size_t)ld);
    double *cost = (double *)malloc(sizeof(double) * (size_t)N);
    int *basis = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!T || !d || !cost || !basis) {
        free(T);
        free(d);
        free(cost);
        free(basis);
        return NAN;
    }
    for (int j = 0; j < 2 * p; ++j) cost[j] = lambda;
    for (int j = 2 * p; j < N; ++j) cost[j] = 1.0;
    for (int i = 0; i < n; ++i) {
        double s = P->y[i] >= 0.0 ? 1.0 : -1.0;
        double *row = T + (size_t)i * ld;
        for (int j = 0; j < p; ++j) {
            row[j] = s * XIJ(P, i, j);
            row[p + j] = -s * XIJ(P, i, j);
        }
        row[2 * p + i] = s;
        row[2 * p + n + i] = -s;
        row[N] = s * P->y[i];
        basis[i] = s > 0 ? 2 * p + i : 2 * p + n + i;
    }
    for (int c = 0; c <= N; ++c) {
        double a = c < N ? cost[c] : 0.0;
        for (int i = 0; i < n; ++i) a -= cost[basis[i]] * T[(size_t)i * ld + c];
        d[c] = a; /* d[N] = -objective */
    }
    long piv = 0, degen = 0, maxpiv = 50L * (n + p) + 1000;
    int ok = 0;
    while (piv < maxpiv) {
        int bland = degen > 20;
        int e = -1;
        double best = -1e-11;
        for (int c = 0; c < N; ++c)
            if (d[c] < best) {
                e = c;
                best = d[c];
                if (bland) break;
            }
        if (e < 0) {
            ok = 1;
            break;
        }
        int l = -1;
        double ratio = INFINITY;
        for (int i = 0; i < n; ++i) {
            double a = T[(size_t)i * ld + e];
            if (a > 1e-11) {
                double q = T[(size_t)i * ld + N] / a;
                if (q < ratio - 1e-14 || (q <= ratio + 1e-14 && l >= 0 && basis[i] < basis[l])) {
                    ratio = q < ratio ? q : ratio;
                    l = i;
                }
            }
        }
        if (l < 0) break; /* unbounded: cannot happen for this LP */
        degen = ratio <= 1e-14 ? degen + 1 : 0;
        double *rl = T + (size_t)l * ld;
        double pv = rl[e];
        for (int c = 0; c <= N; ++c) rl[c] /= pv;
        for (int i = 0; i < n; ++i) {
            if (i == l) continue;
            double *ri = T + (size_t)i * ld;
            double a = ri[e];
            if (a != 0.0)
                for (int c = 0; c <= N; ++c) ri[c] -= a * rl[c];
        }
        double a = d[e];
        for (int c = 0; c <= N; ++c) d[c] -= a * rl[c];
        basis[l] = e;
        ++piv;
    }
    double fopt = NAN;
    if (ok) {
        for (int j = 0; j < p; ++j) b[j] = 0.0;
        for (int i = 0; i < n; ++i) {
            int v = basis[i];
            double val = T[(size_t)i * ld + N];
            if (v < p)
                b[v] += val;
            else if (v < 2 * p)
                b[v - p] -= val;
        }
        if (u)
            for (int i = 0; i < n; ++i) u[i] = 1.0 - d[2 * p + i];
        fopt = -d[N];
    }
    if (pivots) *pivots = piv;
    free(T);
    free(d);
    free(cost);
    free(basis);
    return fopt;
}

/* ------------------------------------------------------------------------ */
/* Gradient through the optimal vertex b_S = X_{Z,S}^{-1} y_Z (Section 3.2   */
/* vertex form): for a loss L with g = dL/db,                                */
/*   w = X_{Z,S}^{-T} g_S,  dL/dy_Z = w,  dL/dX_{Z,S} = -w b_S^T,            */
/* every other entry zero.                                                    */
/* ------------------------------------------------------------------------ */

int orc_backward(const orc_prob *P, const double *b, const int *Z, const double *g, double *dy, double *dX)
{
    const int n = P->n, p = P->p;
    overt V;
    V.s = 0;
    for (int j = 0; j < p; ++j)
        if (b[j] != 0.0) V.S[V.s++] = j;
    for (int q = 0; q < V.s; ++q) V.Z[q] = Z[q];
    for (int i = 0; i < n; ++i) dy[i] = 0.0;
    for (size_t e = 0; e < (size_t)n * (size_t)p; ++e) dX[e] = 0.0;
    if (V.s == 0) return 0;
    double A[ORC_MAX_P * ORC_MAX_P], w[ORC_MAX_P];
    olu L;
    vertex_matrix(P, &V, A);
    if (!lu_factor(&L, V.s, A)) return -1;
    for (int c = 0; c < V.s; ++c) w[c] = g[V.S[c]];
    lu_solve_t(&L, w);
    for (int q = 0; q < V.s; ++q) {
        dy[V.Z[q]] = w[q];
        for (int c = 0; c < V.s; ++c) dX[(size_t)V.Z[q] * p + V.S[c]] = -w[q] * b[V.S[c]];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Thread-pool batch driver                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int num_solves, path_len, nthreads;
    const int32_t *problem, *p_arr;
    const int64_t *row_off, *x_off, *b_off;
    const double *X, *y, *lam;
    const orc_opts *o;
    double *b_out, *f_out;
    int32_t *stage_out, *zrows_out, *cert_out;
    uint32_t *smask_out;
    int64_t *counters_out;
    double *margin_out;
    atomic_int next;
} obatch;

static void *batch_worker(void *arg)
{
    obatch *B = (obatch *)arg;
    int maxn = 1;
    for (int s = 0; s < B->num_solves; ++s) {
        int k = B->problem ? B->problem[s] : s;
        int n = (int)(B->row_off[k + 1] - B->row_off[k]);
        if (n > maxn) maxn = n;
    }
    owork W;
    if (!work_alloc(&W, maxn, ORC_MAX_P)) return NULL;
    double bprev[ORC_MAX_P];
    for (;;) {
        int s = atomic_fetch_add(&B->next, 1);
        if (s >= B->num_solves) break;
        int k = B->problem ? B->problem[s] : s;
        orc_prob P;
        P.n = (int)(B->row_off[k + 1] - B->row_off[k]);
        P.p = B->p_arr[k];
        P.X = B->X + B->x_off[k];
        P.y = B->y + B->row_off[k];
        for (int j = 0; j < P.p; ++j) bprev[j] = 0.0;
        for (int t = 0; t < B->path_len; ++t) {
            size_t o = (size_t)s * (size_t)B->path_len + (size_t)t;
            P.lambda = B->lam[o];
            orc_info I;
            double *b = B->b_out + (size_t)B->path_len * (size_t)B->b_off[s] + (size_t)t * (size_t)P.p;
            int ok = solve_w(&P, B->o, bprev, b, &I, &W);
            memcpy(bprev, b, sizeof(double) * (size_t)P.p);
            B->f_out[o] = I.certified ? I.f : orc_objective(&P, b);
            if (B->stage_out) B->stage_out[o] = I.stage;
            if (B->cert_out) B->cert_out[o] = ok ? (I.unique ? 2 : 1) : 0;
            if (B->smask_out) {
                uint32_t m = 0;
                for (int j = 0; j < P.p && j < 32; ++j)
                    if (b[j] != 0.0) m |= 1u << j;
                B->smask_out[o] = m;
            }
            if (B->zrows_out)
                for (int q = 0; q < 32; ++q) B->zrows_out[o * 32 + q] = (ok && q < ORC_MAX_P) ? I.Z[q] : -1;
            if (B->margin_out) {
                B->margin_out[2 * o] = ok ? I.margin_uc : -1.0;
                B->margin_out[2 * o + 1] = ok ? I.margin_r : -1.0;
            }
            if (B->counters_out) {
                int64_t *c = B->counters_out + o * 4;
                c[0] = I.sweeps;
                c[1] = I.updates;
                c[2] = I.probes;
                c[3] = I.pivots;
            }
        }
    }
    work_free(&W);
    return NULL;
}

double orc_solve_batch(int num_solves, const int32_t *problem, const int64_t *row_off,
                       const int64_t *x_off, const int32_t *p_arr, const double *X, const double *y,
                       const double *lam, int path_len, const int64_t *b_off, const orc_opts *o,
                       int nthreads, double *b_out, double *f_out, int32_t *stage_out,
                       uint32_t *smask_out, int32_t *zrows_out, int32_t *cert_out, int64_t *counters_out,
                       double *margin_out)
{
    obatch B;
    B.num_solves = num_solves;
    B.path_len = path_len;
    B.nthreads = nthreads > 0 ? nthreads : 1;
    B.problem = problem;
    B.p_arr = p_arr;
    B.row_off = row_off;
    B.x_off = x_off;
    B.b_off = b_off;
    B.X = X;
    B.y = y;
    B.lam = lam;
    B.o = o;
    B.b_out = b_out;
    B.f_out = f_out;
    B.stage_out = stage_out;
    B.zrows_out = zrows_out;
    B.cert_out = cert_out;
    B.smask_out = smask_out;
    B.counters_out = counters_out;
    B.margin_out = margin_out;
    atomic_init(&B.next, 0);
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    pthread_t th[256];
    int nt = B.nthreads > 256 ? 256 : B.nthreads;
    for (int t = 1; t < nt; ++t) pthread_create(&th[t], NULL, batch_worker, &B);
    batch_worker(&B);
    for (int t = 1; t < nt; ++t) pthread_join(th[t], NULL);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}
