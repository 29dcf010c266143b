// Plain forward solve: one GPU thread per solve, the problem read straight
// from global memory (row-major X), per-thread scratch in global memory.
// This is the paper's coarse-parallel deployment design (one problem per
// GPU thread, Abstract and Section 5) implemented on gfx950; it runs the
// same method, schedule and tolerances as the wavefront kernel and serves
// as its speed baseline.
//
// Scratch is interleaved across threads (element e of thread t at
// base[e*T + t]) so that threads walking the same element index touch
// consecutive addresses.
#include "ladl_common.hpp"
#include "ladl_kernels.hpp"

#include <climits>

namespace ladl {

template <typename T>
struct IA { // interleaved per-thread array
    T *p;
    int64_t stride;
    __device__ __forceinline__ T &operator[](int i) const { return p[(int64_t)i * stride]; }
};

// scratch layout (elements per thread), NM = largest n of the plan
__host__ __device__ inline int64_t plain_floats(int NM) { return 6 * (int64_t)NM + 2 * ((int64_t)NM + 33) + 2 * 32 * ALD + 5 * 32; }
__host__ __device__ inline int64_t plain_ints(int NM) { return 2 * (int64_t)NM + 33 + 3 * 32; }
__host__ __device__ inline int64_t plain_doubles() { return 32; }

struct PT {
    const float *X, *yg;
    int n, p;
    float lam, ynorm1;
    DevOpt opt;
    IA<float> y, r, rb, rv, rn, xd, ka, kw, A, Q, b, bb, bt, vd, ca;
    IA<int> kid, zf, zs, ss, piv;
    IA<double> gd;
    int c_sweeps, c_updates, c_probes, c_pivots;
    double fv64; // objective of the last evaluated vertex, fp64 residual sums
    __device__ __forceinline__ float x(int i, int j) const { return X[(int64_t)i * p + j]; }
};

__device__ __forceinline__ float sgn1(float v) { return (v > 0.f) ? 1.f : ((v < 0.f) ? -1.f : 0.f); }

__device__ void pt_residuals(PT &t)
{
    for (int i = 0; i < t.n; ++i) {
        float r = t.y[i];
        for (int j = 0; j < t.p; ++j) r = fmaf(-t.x(i, j), t.b[j], r);
        t.r[i] = r;
    }
}

__device__ float pt_objective(PT &t, const IA<float> &r, const IA<float> &b)
{
    float s = 0.f, sb = 0.f;
    for (int i = 0; i < t.n; ++i) s += fabsf(r[i]);
    for (int j = 0; j < t.p; ++j) sb += fabsf(b[j]);
    return s + t.lam * sb;
}

// smallest key a* among ka[0..m) whose cumulative weight (over keys <= a*)
// reaches T (strict: exceeds T); weighted quickselect with three-way
// partitions.  Returns the position of a key equal to a*.
__device__ int pt_select(PT &t, int m, float T, bool strict)
{
    auto reached = [&](float c) { return strict ? (c > T) : (c >= T); };
    auto swp = [&](int i, int j) {
        float a = t.ka[i], w = t.kw[i];
        int d = t.kid[i];
        t.ka[i] = t.ka[j];
        t.kw[i] = t.kw[j];
        t.kid[i] = t.kid[j];
        t.ka[j] = a;
        t.kw[j] = w;
        t.kid[j] = d;
    };
    int lo = 0, hi = m;
    float acc = 0.f;
    while (hi - lo > 16) {
        float a0 = t.ka[lo], a1 = t.ka[(lo + hi) >> 1], a2 = t.ka[hi - 1];
        float piv = fmaxf(fminf(a0, a1), fminf(fmaxf(a0, a1), a2)); // median of three
        // [lo, lt) < piv, [lt, i) == piv, (gt, hi) > piv
        int lt = lo, i = lo, gt = hi - 1;
        float wl = 0.f, we = 0.f;
        while (i <= gt) {
            float a = t.ka[i];
            if (a < piv) {
                wl += t.kw[i];
                swp(lt, i);
                ++lt;
                ++i;
            } else if (a > piv) {
                swp(i, gt);
                --gt;
            } else {
                we += t.kw[i];
                ++i;
            }
        }
        if (reached(acc + wl)) {
            hi = lt;
        } else if (reached(acc + wl + we)) {
            return lt;
        } else {
            acc += wl + we;
            lo = gt + 1;
        }
    }
    // insertion sort of the small remainder, then scan
    for (int i = lo + 1; i < hi; ++i)
        for (int j = i; j > lo && t.ka[j - 1] > t.ka[j]; --j) swp(j - 1, j);
    for (int i = lo; i < hi; ++i) {
        acc += t.kw[i];
        if (reached(acc)) return i;
    }
    return (hi > lo) ? hi - 1 : -1;
}

// exact minimisation along axis j (weighted median of the kinks)
__device__ bool pt_coord_update(PT &t, int j)
{
    float bel = 0.f, at = 0.f, abv = 0.f;
    for (int i = 0; i < t.n; ++i) {
        float r = t.r[i], x = t.x(i, j), ax = fabsf(x);
        bool z = r == 0.f;
        bool neg = __builtin_signbit(r) != __builtin_signbit(x);
        at += z ? ax : 0.f;
        bel += (!z && neg) ? ax : 0.f;
        abv += (!z && !neg) ? ax : 0.f;
    }
    const float bj = t.b[j], lam = t.lam;
    const float W = (bel + at) + (abv + lam);
    if (!(W > 0.f)) return false;
    const float belT = bel + ((bj > 0.f) ? lam : 0.f);
    const float atT = at + ((bj == 0.f) ? lam : 0.f);
    const float half = 0.5f * W;
    int dir;
    if (belT >= half)
        dir = -1;
    else if (belT + atT < half)
        dir = 1;
    else
        return false;
    int m = 0;
    for (int i = 0; i < t.n; ++i) {
        float r = t.r[i], x = t.x(i, j);
        bool neg = __builtin_signbit(r) != __builtin_signbit(x);
        if (x != 0.f && r != 0.f && (dir < 0 ? neg : !neg)) {
            t.ka[m] = fabsf(r) / fabsf(x);
            t.kw[m] = fabsf(x);
            t.kid[m] = i;
            ++m;
        }
    }
    if (lam > 0.f && (dir < 0 ? (bj > 0.f) : (bj < 0.f))) {
        t.ka[m] = fabsf(bj);
        t.kw[m] = lam;
        t.kid[m] = t.n; // the penalty kink, after every row on ties
        ++m;
    }
    if (m == 0) return false;
    const float T = (dir < 0) ? (belT - half) : (half - belT - atT);
    int q = pt_select(t, m, T, dir < 0);
    if (q < 0) return false;
    // prefer a row on ties with the penalty kink
    float as = t.ka[q];
    int owner = t.kid[q];
    if (owner == t.n)
        for (int e = 0; e < m; ++e)
            if (t.ka[e] == as && t.kid[e] < t.n) {
                owner = t.kid[e];
                break;
            }
    float nb = (owner == t.n) ? 0.f : ((dir < 0) ? bj - as : bj + as);
    float d = nb - bj;
    if (d == 0.f || !__builtin_isfinite(d)) return false;
    for (int i = 0; i < t.n; ++i) t.r[i] = fmaf(-t.x(i, j), d, t.r[i]);
    if (owner < t.n) t.r[owner] = 0.f;
    t.b[j] = nb;
    return true;
}

// sum_i |r_i - x_ij d| for three offsets d of b_j at once (one pass over
// the column)
__device__ void pt_section3(PT &t, int j, float d0, float d1, float d2, float &g0, float &g1, float &g2)
{
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (int i = 0; i < t.n; ++i) {
        const float r = t.r[i], x = t.x(i, j);
        s0 += fabsf(fmaf(-x, d0, r));
        s1 += fabsf(fmaf(-x, d1, r));
        s2 += fabsf(fmaf(-x, d2, r));
    }
    g0 = s0;
    g1 = s1;
    g2 = s2;
}

// minimisation along axis j by the quadrature search of the section's
// values (no kink is stored, sorted or selected): bracket [lo, hi] from the
// smallest and largest kink; halve it around the lowest of its quarter
// points; keep the result only if it lowers f
__device__ bool pt_coord_update_quad(PT &t, int j)
{
    const float bj = t.b[j], lam = t.lam;
    float lo = FINF_C, hi = -FINF_C;
    for (int i = 0; i < t.n; ++i) {
        const float x = t.x(i, j);
        if (x != 0.f) {
            const float k = bj + t.r[i] / x;
            lo = fminf(lo, k);
            hi = fmaxf(hi, k);
        }
    }
    if (lam > 0.f) {
        lo = fminf(lo, 0.f);
        hi = fmaxf(hi, 0.f);
    }
    if (!(lo <= hi)) return false;
    float mid = 0.5f * (lo + hi), g0, gm, gu;
    pt_section3(t, j, 0.f, mid - bj, 0.f, g0, gm, gu);
    g0 += lam * fabsf(bj);
    gm += lam * fabsf(mid);
    for (int it = 0; it < QUAD_MAX; ++it) {
        if (hi - lo <= QUAD_TOL * (1.f + fabsf(lo) + fabsf(hi))) break;
        const float q1 = 0.5f * (lo + mid), q3 = 0.5f * (mid + hi);
        if (!(q1 > lo && q1 < mid && q3 > mid && q3 < hi)) break;
        float g1, g3;
        pt_section3(t, j, q1 - bj, q3 - bj, 0.f, g1, g3, gu);
        g1 += lam * fabsf(q1);
        g3 += lam * fabsf(q3);
        if (g1 < gm && g1 <= g3) {
            hi = mid;
            mid = q1;
            gm = g1;
        } else if (g3 < gm) {
            lo = mid;
            mid = q3;
            gm = g3;
        } else {
            lo = q1;
            hi = q3;
        }
    }
    if (!(gm < g0)) return false;
    const float d = mid - bj;
    if (d == 0.f || !__builtin_isfinite(d)) return false;
    for (int i = 0; i < t.n; ++i) t.r[i] = fmaf(-t.x(i, j), d, t.r[i]);
    t.b[j] = mid;
    return true;
}

__device__ float pt_ccd(PT &t, int frozen, float f)
{
    const bool quad = (t.opt.flags & FLAG_QUADRATURE) != 0;
    for (int sw = 0; sw < t.opt.max_sweeps; ++sw) {
        bool changed = false;
        for (int j = 0; j < t.p; ++j) {
            if (j == frozen) continue;
            changed |= quad ? pt_coord_update_quad(t, j) : pt_coord_update(t, j);
            t.c_updates++;
        }
        t.c_sweeps++;
        float fn = pt_objective(t, t.r, t.b);
        bool stop = !changed || (f - fn <= t.opt.tol_f * fn);
        f = fn;
        if (stop) break;
    }
    return f;
}

// nearest vertex (p independent hyperplanes, nearest first)
__device__ int pt_choose_vertex(PT &t)
{
    const int n = t.n, p = t.p;
    for (int i = 0; i < n; ++i) t.zf[i] = 0; // 0 unseen, 1 passed over, 2 taken
    uint32_t cseen = 0, ctaken = 0;
    int acc = 0, nz = 0;
    for (int guard = 0; guard < n + p && acc < p; ++guard) {
        float m = FINF_C;
        int row = -1, col = -1;
        for (int j = 0; j < p; ++j)
            if (!((cseen >> j) & 1u) && fabsf(t.b[j]) < m) {
                m = fabsf(t.b[j]);
                col = j;
            }
        for (int i = 0; i < n; ++i) {
            if (t.zf[i]) continue;
            float nr = t.rn[i];
            if (!(nr > 0.f)) continue;
            float dd = fabsf(t.r[i]) / nr;
            if (dd < m) {
                m = dd;
                row = i;
                col = -1;
            }
        }
        if (m == FINF_C || (row < 0 && col < 0)) break;
        if (row >= 0)
            t.zf[row] = 1;
        else
            cseen |= 1u << col;
        float v[PMAX];
        float n0 = 0.f;
        for (int j = 0; j < p; ++j) {
            v[j] = (row >= 0) ? t.x(row, j) : (j == col ? 1.f : 0.f);
            n0 = fmaf(v[j], v[j], n0);
        }
        for (int a = 0; a < acc; ++a) {
            float dd = 0.f;
            for (int j = 0; j < p; ++j) dd = fmaf(v[j], t.Q[a * ALD + j], dd);
            for (int j = 0; j < p; ++j) v[j] = fmaf(-dd, t.Q[a * ALD + j], v[j]);
        }
        float nv = 0.f;
        for (int j = 0; j < p; ++j) nv = fmaf(v[j], v[j], nv);
        if (!(sqrtf(nv) > 1e-4f * sqrtf(n0))) continue;
        float inv = 1.f / sqrtf(nv);
        for (int j = 0; j < p; ++j) t.Q[acc * ALD + j] = v[j] * inv;
        ++acc;
        if (row >= 0) {
            t.zf[row] = 2;
            t.zs[nz++] = row;
        } else {
            ctaken |= 1u << col;
        }
    }
    int s = 0;
    for (int j = 0; j < p; ++j)
        if (!((ctaken >> j) & 1u)) t.ss[s++] = j;
    for (int i = 0; i < n; ++i) t.zf[i] = (t.zf[i] == 2) ? 1 : 0;
    return (acc == p && s == nz) ? s : -1;
}

__device__ bool pt_lu(PT &t, int s)
{
    float amax = 0.f;
    for (int e = 0; e < s; ++e)
        for (int c = 0; c < s; ++c) amax = fmaxf(amax, fabsf(t.A[e * ALD + c]));
    for (int k = 0; k < s; ++k) {
        int pr = k;
        float vm = fabsf(t.A[k * ALD + k]);
        for (int i = k + 1; i < s; ++i)
            if (fabsf(t.A[i * ALD + k]) > vm) {
                vm = fabsf(t.A[i * ALD + k]);
                pr = i;
            }
        if (!(vm > 1e-7f * amax)) return false;
        t.piv[k] = pr;
        if (pr != k)
            for (int c = 0; c < s; ++c) {
                float tmp = t.A[k * ALD + c];
                t.A[k * ALD + c] = t.A[pr * ALD + c];
                t.A[pr * ALD + c] = tmp;
            }
        float pk = t.A[k * ALD + k];
        for (int i = k + 1; i < s; ++i) {
            float lf = t.A[i * ALD + k] / pk;
            t.A[i * ALD + k] = lf;
            for (int c = k + 1; c < s; ++c) t.A[i * ALD + c] = fmaf(-lf, t.A[k * ALD + c], t.A[i * ALD + c]);
        }
    }
    return true;
}

__device__ void pt_solve(PT &t, int s, float *v)
{
    for (int k = 0; k < s; ++k) {
        int pk = t.piv[k];
        if (pk != k) {
            float tmp = v[k];
            v[k] = v[pk];
            v[pk] = tmp;
        }
    }
    for (int i = 0; i < s; ++i)
        for (int c = 0; c < i; ++c) v[i] = fmaf(-t.A[i * ALD + c], v[c], v[i]);
    for (int i = s - 1; i >= 0; --i) {
        for (int c = i + 1; c < s; ++c) v[i] = fmaf(-t.A[i * ALD + c], v[c], v[i]);
        v[i] = v[i] / t.A[i * ALD + i];
    }
}

__device__ void pt_solve_t(PT &t, int s, float *v)
{
    for (int i = 0; i < s; ++i) {
        for (int c = 0; c < i; ++c) v[i] = fmaf(-t.A[c * ALD + i], v[c], v[i]);
        v[i] = v[i] / t.A[i * ALD + i];
    }
    for (int i = s - 1; i >= 0; --i)
        for (int c = i + 1; c < s; ++c) v[i] = fmaf(-t.A[c * ALD + i], v[c], v[i]);
    for (int k = s - 1; k >= 0; --k) {
        int pk = t.piv[k];
        if (pk != k) {
            float tmp = v[k];
            v[k] = v[pk];
            v[pk] = tmp;
        }
    }
}

// vertex (zs, ss, s): LU of X_{Z,S}, b_S = A^{-1} y_Z with one fp64-residual
// refinement step, b into bt, residuals into rv (zero on Z), f
__device__ bool pt_vertex_eval(PT &t, int s, float &f)
{
    for (int q = 0; q < s; ++q)
        for (int c = 0; c < s; ++c) t.A[q * ALD + c] = t.x(t.zs[q], t.ss[c]);
    if (!pt_lu(t, s)) return false;
    float e[PMAX];
    double v[PMAX];
    for (int q = 0; q < s; ++q) e[q] = t.y[t.zs[q]];
    pt_solve(t, s, e);
    for (int q = 0; q < s; ++q) v[q] = (double)e[q];
    // b_S in fp64 by mixed-precision refinement (fp32 LU, fp64 residuals and
    // accumulation) until the correction is at fp64 rounding level: the
    // certificate reads the signs of the other rows' residuals at this vertex
    for (int it = 0; it < REFINE_MAX; ++it) {
        float cm = 0.f, xm = 0.f;
        for (int q = 0; q < s; ++q) {
            double acc = (double)t.y[t.zs[q]];
            for (int c = 0; c < s; ++c) acc -= (double)t.x(t.zs[q], t.ss[c]) * v[c];
            e[q] = (float)acc;
        }
        pt_solve(t, s, e);
        for (int q = 0; q < s; ++q) {
            v[q] += (double)e[q];
            cm = fmaxf(cm, fabsf(e[q]));
            xm = fmaxf(xm, fabsf((float)v[q]));
        }
        if (cm <= 1e-14f * xm) break;
    }
    for (int j = 0; j < t.p; ++j) t.bt[j] = 0.f;
    for (int c = 0; c < s; ++c) {
        float bc = (float)v[c];
        if (!__builtin_isfinite(bc)) return false;
        t.bt[t.ss[c]] = bc;
    }
    // residuals of the fp64 vertex (stored as fp32): the certificate reads
    // their signs
    double s64 = 0.0;
    for (int i = 0; i < t.n; ++i) {
        double r = (double)t.y[i];
        for (int c = 0; c < s; ++c) r = fma(-(double)t.x(i, t.ss[c]), v[c], r);
        t.rv[i] = t.zf[i] ? 0.f : (float)r;
        s64 += t.zf[i] ? 0.0 : fabs(r);
    }
    for (int c = 0; c < s; ++c) s64 += (double)t.lam * fabs((double)t.bt[t.ss[c]]);
    t.fv64 = s64;
    f = pt_objective(t, t.rv, t.bt);
    return true;
}

__device__ bool pt_certificate(PT &t, int s, float *u, float *c, bool &unique)
{
    const int n = t.n, p = t.p;
    for (int j = 0; j < p; ++j) {
        double g = 0.0;
        for (int i = 0; i < n; ++i) g += (double)t.x(i, j) * (double)sgn1(t.rv[i]);
        t.gd[j] = g;
    }
    uint32_t smask = 0;
    double rhs[PMAX];
    for (int q = 0; q < s; ++q) {
        smask |= 1u << t.ss[q];
        rhs[q] = (double)t.lam * (double)sgn1(t.bt[t.ss[q]]) - t.gd[t.ss[q]];
        u[q] = (float)rhs[q];
    }
    pt_solve_t(t, s, u);
    for (int it = 0; it < REFINE_MAX; ++it) {
        float du[PMAX];
        for (int c = 0; c < s; ++c) {
            double acc = rhs[c];
            for (int q = 0; q < s; ++q) acc -= (double)t.x(t.zs[q], t.ss[c]) * (double)u[q];
            du[c] = (float)acc;
        }
        pt_solve_t(t, s, du);
        float cm = 0.f, um = 1.f;
        for (int c = 0; c < s; ++c) {
            u[c] += du[c];
            cm = fmaxf(cm, fabsf(du[c]));
            um = fmaxf(um, fabsf(u[c]));
        }
        if (cm <= 1e-7f * um) break;
    }
    float umax = 0.f;
    for (int q = 0; q < s; ++q) umax = fmaxf(umax, fabsf(u[q]));
    bool viol = false;
    float mc = FINF_C;
    for (int j = 0; j < p; ++j) {
        double cj = t.gd[j];
        float colz = 0.f; // sum_{i in Z} |x_ij|
        for (int q = 0; q < s; ++q) {
            const float xv = t.x(t.zs[q], j);
            cj += (double)xv * (double)u[q];
            colz += fabsf(xv);
        }
        c[j] = (float)cj;
        if ((smask >> j) & 1u) continue;
        float cabs = fabsf(c[j]), colabs = t.ca[j];
        if (cabs > t.lam * (1.f + TOL_C) + TOL_CA * colabs) viol = true;
        mc = fminf(mc, (t.lam - cabs) / (t.lam + colz));
    }
    const bool cert = umax <= 1.f + TOL_U && !viol;
    // rows off Z: |r_i| against |y_i| + sum_{j in S} |x_ij b_j|
    float mr = FINF_C;
    for (int i = 0; i < n; ++i) {
        if (t.zf[i]) continue;
        float sc = fabsf(t.y[i]);
        for (int q = 0; q < s; ++q) sc = fmaf(fabsf(t.x(i, t.ss[q])), fabsf(t.bt[t.ss[q]]), sc);
        mr = fminf(mr, (sc > 0.f) ? fabsf(t.rv[i]) / sc : fabsf(t.rv[i]));
    }
    unique = cert && (1.f - umax > MARGIN_U) && (mc > MARGIN_C) && (mr > MARGIN_R);
    return cert;
}

__device__ void pt_set_zf(PT &t, int s)
{
    for (int i = 0; i < t.n; ++i) t.zf[i] = 0;
    for (int q = 0; q < s; ++q) t.zf[t.zs[q]] = 1;
}

__device__ int pt_finisher(PT &t, int &s, float &f, float *u, float *c, bool &unique, int maxp)
{
    const int n = t.n, p = t.p;
    const float lam = t.lam;
    double fprev = __builtin_inf();
    int stalls = 0;
    for (int it = 0;; ++it) {
        pt_set_zf(t, s);
        if (!pt_vertex_eval(t, s, f)) return ST_NOTCERT;
        if (pt_certificate(t, s, u, c, unique)) return unique ? ST_CERTIFIED : ST_NONUNIQUE;
        if (it >= maxp) return ST_MAXITER;
        // steepest violated constraint, the violated one of lowest index
        // (Bland's rule) after a step that did not lower f (fp64), and Bland's
        // rule for the rest once STALLS_STICKY steps have stalled
        const bool stalled = !(t.fv64 < fprev - 1e-9 * fabs(fprev));
        stalls += stalled ? 1 : 0;
        const bool bland = stalled || stalls >= STALLS_STICKY;
        fprev = t.fv64;
        uint32_t smask = 0;
        for (int q = 0; q < s; ++q) smask |= 1u << t.ss[q];
        float best = FINF_C;
        int type = 0, sel = -1;
        for (int q = 0; q < s; ++q) {
            float sl = 1.f - fabsf(u[q]);
            if (sl < -TOL_U && (bland ? (sel < 0 || t.zs[q] < t.zs[sel]) : sl < best)) {
                best = sl;
                type = 1;
                sel = q;
            }
        }
        for (int j = 0; j < p && !(bland && sel >= 0); ++j) {
            if ((smask >> j) & 1u) continue;
            float sl = lam - fabsf(c[j]);
            if (fabsf(c[j]) > lam * (1.f + TOL_C) + TOL_CA * t.ca[j] && (bland ? sel < 0 : sl < best)) {
                best = sl;
                type = 2;
                sel = j;
            }
        }
        if (sel < 0) return ST_NOTCERT;
        float dS[PMAX];
        float dj0 = 0.f, usel = 0.f;
        if (type == 1) {
            usel = u[sel];
            for (int q = 0; q < s; ++q) dS[q] = (q == sel) ? -sgn1(usel) : 0.f;
        } else {
            dj0 = sgn1(c[sel]);
            for (int q = 0; q < s; ++q) dS[q] = -t.x(t.zs[q], sel) * dj0;
        }
        pt_solve(t, s, dS);
        for (int j = 0; j < p; ++j) t.vd[j] = 0.f;
        for (int q = 0; q < s; ++q) t.vd[t.ss[q]] = dS[q];
        if (type == 2) t.vd[sel] = dj0;
        const int zsel = (type == 1) ? t.zs[sel] : -1;
        for (int i = 0; i < n; ++i) {
            float a = 0.f;
            for (int j = 0; j < p; ++j) a = fmaf(t.x(i, j), t.vd[j], a);
            if (t.zf[i]) a = (i == zsel) ? -sgn1(usel) : 0.f;
            t.xd[i] = a;
        }
        // the right slope of f along d at t = 0 is `best`; the minimiser is
        // the first kink t > 0 whose cumulative weight reaches -best/2
        const float need = -0.5f * best;
        if (!(need > 0.f)) return ST_NOTCERT;
        int m = 0;
        for (int i = 0; i < n; ++i) {
            float r = t.rv[i], xd = t.xd[i];
            if (r != 0.f && xd != 0.f && __builtin_signbit(r) == __builtin_signbit(xd)) {
                t.ka[m] = fabsf(r) / fabsf(xd);
                t.kw[m] = fabsf(xd);
                t.kid[m] = i;
                ++m;
            }
        }
        if (lam > 0.f)
            for (int j = 0; j < p; ++j) {
                float bj = t.bt[j], dj = t.vd[j];
                if (dj != 0.f && bj != 0.f && __builtin_signbit(bj) != __builtin_signbit(dj)) {
                    t.ka[m] = fabsf(bj) / fabsf(dj);
                    t.kw[m] = lam * fabsf(dj);
                    t.kid[m] = n + j;
                    ++m;
                }
            }
        int q = pt_select(t, m, need, false);
        if (q < 0) return ST_NOTCERT;
        float as = t.ka[q];
        int blk = t.kid[q];
        if (blk >= n)
            for (int e = 0; e < m; ++e)
                if (t.ka[e] == as && t.kid[e] < n) {
                    blk = t.kid[e];
                    break;
                }
        if (!(as > 0.f) || as == FINF_C) return ST_NOTCERT;
        if (type == 1) {
            if (blk < n) {
                t.zs[sel] = blk;
            } else {
                int jb = blk - n, c0 = -1;
                for (int e = 0; e < s; ++e)
                    if (t.ss[e] == jb) c0 = e;
                if (c0 < 0) return ST_NOTCERT;
                for (int e = c0; e + 1 < s; ++e) t.ss[e] = t.ss[e + 1];
                for (int e = sel; e + 1 < s; ++e) t.zs[e] = t.zs[e + 1];
                s -= 1;
            }
        } else {
            if (blk < n) {
                if (s >= 32) return ST_NOTCERT;
                t.zs[s] = blk;
                t.ss[s] = sel;
                s += 1;
            } else {
                int jb = blk - n;
                if (jb == sel) return ST_NOTCERT;
                for (int e = 0; e < s; ++e)
                    if (t.ss[e] == jb) t.ss[e] = sel;
            }
        }
        t.c_pivots++;
    }
    return ST_MAXITER;
}

__device__ float pt_objective64(PT &t, const IA<float> &b)
{
    double s = 0.0;
    for (int i = 0; i < t.n; ++i) {
        double r = (double)t.yg[i];
        for (int j = 0; j < t.p; ++j) r -= (double)t.x(i, j) * (double)b[j];
        s += fabs(r);
    }
    double sb = 0.0;
    for (int j = 0; j < t.p; ++j) sb += fabs((double)b[j]);
    return (float)(s + (double)t.lam * sb);
}

__device__ void pt_solve_item(PT &t, const SolveArgs &a, int s)
{
    const int k = a.problem ? a.problem[s] : s;
    const int64_t r0 = a.row_off[k];
    t.n = (int)(a.row_off[k + 1] - r0);
    t.p = a.p_arr[k];
    t.X = a.X + a.x_off[k];
    t.yg = a.y + r0;
    const int n = t.n, p = t.p;
    bool finite = true;
    float yn = 0.f;
    for (int i = 0; i < n; ++i) {
        float v = t.yg[i];
        t.y[i] = v;
        finite = finite && __builtin_isfinite(v);
        yn += fabsf(v);
        float s2 = 0.f;
        for (int j = 0; j < p; ++j) {
            float x = t.x(i, j);
            finite = finite && __builtin_isfinite(x);
            s2 = fmaf(x, x, s2);
        }
        t.rn[i] = sqrtf(s2);
    }
    t.ynorm1 = yn;
    for (int j = 0; j < p; ++j) {
        float cs = 0.f;
        for (int i = 0; i < n; ++i) cs += fabsf(t.x(i, j));
        t.ca[j] = cs;
    }
    const int64_t bbase = (int64_t)a.path_len * a.b_off[s];
    for (int j = 0; j < p; ++j) {
        float b0 = 0.f;
        if (a.t0 > 0)
            b0 = a.b_out[bbase + (int64_t)(a.t0 - 1) * p + j];
        else if (a.b_init)
            b0 = a.b_init[a.b_off[s] + j];
        t.b[j] = __builtin_isfinite(b0) ? b0 : 0.f;
    }
    float u[PMAX], c[PMAX];
    for (int tt = a.t0; tt < a.t1; ++tt) {
        const int64_t o = (int64_t)s * a.path_len + tt;
        float *bout = a.b_out + bbase + (int64_t)tt * p;
        const float lam_in = a.lam[o];
        t.c_sweeps = t.c_updates = t.c_probes = t.c_pivots = 0;
        int status = ST_NOTCERT;
        float fout;
        int zcount = -1;
        if (!finite || !(lam_in >= 0.f)) {
            status = finite ? ST_BADLAMBDA : ST_NONFINITE;
            for (int j = 0; j < p; ++j) t.b[j] = 0.f;
            fout = __builtin_nanf("");
        } else {
            t.lam = fmaxf(lam_in, t.opt.lambda_min);
            pt_residuals(t);
            float f = pt_objective(t, t.r, t.b);
            bool done = false, unique = false, have_vertex = false;
            int vs = -1;
            float fv = 0.f;
            const bool snap = !(t.opt.flags & FLAG_NO_SNAP);
            const int rounds = (p < 2) ? 0 : ((t.opt.max_rounds < 0) ? p : t.opt.max_rounds);
            const float B = (t.lam > 0.f) ? t.ynorm1 / t.lam : FINF_C;
            Chop q;
            int phase = 0, frozen = -1, round = 0, kax = 0;
            float fbest = FINF_C;
            for (;;) {
                f = pt_ccd(t, frozen, f);
                float sprobe = 0.f;
                bool more;
                if (phase == 0) {
                    if (snap) {
                        vs = pt_choose_vertex(t);
                        have_vertex = vs >= 0;
                        if (have_vertex) {
                            int st = pt_finisher(t, vs, fv, u, c, unique, 0);
                            if (st == ST_CERTIFIED || st == ST_NONUNIQUE) {
                                status = st;
                                done = true;
                                break;
                            }
                        }
                    }
                    if (round >= rounds) break;
                    if (round == 0) {
                        kax = 0;
                        for (int j = 1; j < p; ++j)
                            if (fabsf(t.b[j]) > fabsf(t.b[kax])) kax = j;
                    } else {
                        kax = (kax + 1) % p;
                    }
                    ++round;
                    for (int j = 0; j < p; ++j) t.bb[j] = t.b[j];
                    for (int i = 0; i < n; ++i) t.rb[i] = t.r[i];
                    fbest = f;
                    chop_init(q, t.bb[kax], f, B, t.opt.chop_range);
                    more = chop_next(q, 0.f, sprobe, t.opt);
                } else {
                    t.c_probes++;
                    if (f < fbest) {
                        fbest = f;
                        for (int j = 0; j < p; ++j) t.bb[j] = t.b[j];
                        for (int i = 0; i < n; ++i) t.rb[i] = t.r[i];
                    }
                    more = chop_next(q, f, sprobe, t.opt);
                }
                for (int j = 0; j < p; ++j) t.b[j] = t.bb[j];
                for (int i = 0; i < n; ++i) t.r[i] = t.rb[i];
                if (more) {
                    const float d = sprobe - t.bb[kax];
                    if (d != 0.f)
                        for (int i = 0; i < n; ++i) t.r[i] = fmaf(-t.x(i, kax), d, t.r[i]);
                    t.b[kax] = sprobe;
                    f = pt_objective(t, t.r, t.b);
                    frozen = kax;
                    phase = 1;
                } else {
                    f = fbest;
                    frozen = -1;
                    phase = 0;
                }
            }
            if (!done && snap && have_vertex && !(t.opt.flags & FLAG_NO_FINISHER)) {
                const int maxp = (t.opt.max_pivots > 0) ? t.opt.max_pivots : 4 * p + 32;
                bool perturbed = false;
                for (int attempt = 0; attempt < 2 && !done; ++attempt) {
                    if (attempt == 1) {
                        const float ybar = t.ynorm1 / (float)n;
                        for (int i = 0; i < n; ++i)
                            t.y[i] = t.y[i] + PERTURB_REL * (fabsf(t.y[i]) + ybar) * perturb_dir(i);
                        perturbed = true;
                    }
                    status = pt_finisher(t, vs, fv, u, c, unique, maxp);
                    done = (status == ST_CERTIFIED || status == ST_NONUNIQUE);
                }
                if (done && perturbed) {
                    double yu = 0.0;
                    for (int i = 0; i < n; ++i) yu += (double)t.yg[i] * (double)sgn1(t.rv[i]);
                    for (int e = 0; e < vs; ++e) yu += (double)t.yg[t.zs[e]] * (double)u[e];
                    for (int i = 0; i < n; ++i) t.y[i] = t.yg[i];
                    done = pt_vertex_eval(t, vs, fv);
                    if (done) {
                        float fo = pt_objective64(t, t.bt);
                        done = (double)fo - yu <= 2e-6 * fmax(1.0, (double)fo);
                    }
                    status = done ? ST_NONUNIQUE : ST_NOTCERT;
                } else if (perturbed) {
                    for (int i = 0; i < n; ++i) t.y[i] = t.yg[i]; // for the next path step
                }
            }
            if (done) {
                for (int j = 0; j < p; ++j) t.b[j] = t.bt[j];
                zcount = vs;
            } else if (!snap) {
                status = ST_MAXITER;
            }
            fout = pt_objective64(t, t.b);
        }
        uint32_t act = 0;
        for (int j = 0; j < p; ++j) {
            bout[j] = t.b[j];
            if (t.b[j] != 0.f) act |= 1u << j;
        }
        a.obj_out[o] = fout;
        a.active_out[o] = act;
        a.status_out[o] = status;
        if (a.iters_out) {
            a.iters_out[4 * o + 0] = t.c_sweeps;
            a.iters_out[4 * o + 1] = t.c_updates;
            a.iters_out[4 * o + 2] = t.c_probes;
            a.iters_out[4 * o + 3] = t.c_pivots;
        }
        int32_t *zo = a.zrows_out + (int64_t)ZPAD * o;
        int zz[32];
        int cnt = (zcount > 0) ? zcount : 0;
        for (int e = 0; e < cnt; ++e) zz[e] = t.zs[e];
        for (int e = 1; e < cnt; ++e)
            for (int g = e; g > 0 && zz[g - 1] > zz[g]; --g) {
                int tmp = zz[g];
                zz[g] = zz[g - 1];
                zz[g - 1] = tmp;
            }
        for (int e = 0; e < ZPAD; ++e) zo[e] = (e < cnt) ? zz[e] : -1;
    }
}

__global__ __launch_bounds__(64) void k_plain(SolveArgs a, int NM, int64_t nthreads)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= nthreads) return;
    PT t;
    t.opt = a.opt;
    const int64_t T = nthreads;
    float *fb = a.gws + tid;
    int64_t o = 0;
    auto fa = [&](int64_t len) {
        IA<float> r{fb + o * T, T};
        o += len;
        return r;
    };
    t.y = fa(NM);
    t.r = fa(NM);
    t.rb = fa(NM);
    t.rv = fa(NM);
    t.rn = fa(NM);
    t.xd = fa(NM);
    t.ka = fa(NM + 33);
    t.kw = fa(NM + 33);
    t.A = fa(32 * ALD);
    t.Q = fa(32 * ALD);
    t.b = fa(32);
    t.bb = fa(32);
    t.bt = fa(32);
    t.vd = fa(32);
    t.ca = fa(32);
    int *ib = (int *)(a.gws + plain_floats(NM) * T) + tid;
    int64_t oi = 0;
    auto ia = [&](int64_t len) {
        IA<int> r{ib + oi * T, T};
        oi += len;
        return r;
    };
    t.kid = ia(NM + 33);
    t.zf = ia(NM);
    t.zs = ia(32);
    t.ss = ia(32);
    t.piv = ia(32);
    double *db = (double *)(a.gws + plain_floats(NM) * T + plain_ints(NM) * T) + tid;
    t.gd = IA<double>{db, T};
    for (;;) {
        int q = atomicAdd(a.counter, 1);
        if (q >= a.num_items) break;
        pt_solve_item(t, a, a.order[q]);
    }
}

int64_t plain_scratch_floats(int NM, int64_t nthreads)
{
    // floats + ints + doubles (2 floats each), padded for double alignment
    return (plain_floats(NM) + plain_ints(NM) + 2 * plain_doubles() + 2) * nthreads;
}

hipError_t launch_plain(const SolveArgs &a, int NM, int64_t nthreads, hipStream_t s)
{
    int grid = (int)((nthreads + 63) / 64);
    hipLaunchKernelGGL(k_plain, dim3(grid), dim3(64), 0, s, a, NM, nthreads);
    return hipGetLastError();
}

} // namespace ladl
