// K-fold cross-validation along a lambda path (the paper's use of several
// regularisation settings solved while cross-validating, Section 5): the
// training problems are gathered on the device, solved by the wave kernels
// (ladl_solve_f32 on an inner plan), then scored on the held-out rows.
#include "ladl_common.hpp"
#include "ladl_kernels.hpp"
#include "ladl_wave.hpp"

namespace ladl {

// One wave per training problem q = k*K + f: its rows (base rows outside
// fold f, in order) into the packed row-major block, and its lambda path.
__global__ __launch_bounds__(64) void k_cv_gather(CvArgs a)
{
    const int q = blockIdx.x;
    if (q >= a.num_train) return;
    const int l = lane_id();
    const int k = q / a.folds;
    const int p = a.p_b[k];
    const int64_t r0 = a.tr_off[q];
    const int ntr = (int)(a.tr_off[q + 1] - r0);
    const float *Xb = a.X + a.x_off_b[k];
    const float *yb = a.y + a.row_off_b[k];
    float *Xt = a.Xtr + a.x_off_tr[q];
    const int np = ntr * p;
    for (int e = l; e < np; e += 64) {
        const int i = e / p, j = e - i * p;
        Xt[e] = Xb[(int64_t)a.tr_rows[r0 + i] * p + j];
    }
    for (int i = l; i < ntr; i += 64) a.ytr[r0 + i] = yb[a.tr_rows[r0 + i]];
    for (int t = l; t < a.path_len; t += 64)
        a.lam_tr[(int64_t)q * a.path_len + t] = a.lam[(int64_t)k * a.path_len + t];
}

// One wave per training problem: the held-out absolute error of each path
// step's b over the fold's rows (fp32 residuals, fp64 sums).
__global__ __launch_bounds__(64) void k_cv_validate(CvArgs a)
{
    const int q = blockIdx.x;
    if (q >= a.num_train) return;
    const int l = lane_id();
    const int k = q / a.folds;
    const int p = a.p_b[k];
    const int L = a.path_len;
    const int64_t v0 = a.va_off[q];
    const int nva = (int)(a.va_off[q + 1] - v0);
    const float *Xb = a.X + a.x_off_b[k];
    const float *yb = a.y + a.row_off_b[k];
    const float *bq = a.b + (int64_t)L * a.b_off_tr[q];
    for (int t = 0; t < L; ++t) {
        const float bl = (l < p) ? bq[(int64_t)t * p + l] : 0.f; // lane j: b_j
        double acc = 0.0;
        for (int i0 = 0; i0 < nva; i0 += 64) {
            const int i = i0 + l;
            const int src = (i < nva) ? a.va_rows[v0 + i] : 0;
            const float *xr = Xb + (int64_t)src * p;
            float r = (i < nva) ? yb[src] : 0.f;
            for (int j = 0; j < p; ++j) {
                const float bj = rdlane(bl, j);
                r = (i < nva) ? fmaf(-xr[j], bj, r) : 0.f;
            }
            acc += fabs((double)r);
        }
        acc = wsum_d(acc);
        if (l == 0) a.fold_err[(int64_t)q * L + t] = (float)acc;
    }
}

// One wave per base problem: cv[t] = sum over folds (fp64, fold order), and
// the first t at the minimum (-1 if every value is NaN).
__global__ __launch_bounds__(64) void k_cv_select(CvArgs a)
{
    const int k = blockIdx.x;
    if (k >= a.num_base) return;
    const int l = lane_id();
    const int L = a.path_len, K = a.folds;
    double c = 0.0;
    if (l < L)
        for (int f = 0; f < K; ++f) c += (double)a.fold_err[((int64_t)k * K + f) * L + l];
    const float cf = (l < L) ? (float)c : FINF;
    if (l < L) a.cv_err[(int64_t)k * L + l] = cf;
    const float m = wmin(cf);
    const uint64_t at = ballot(l < L && cf == m);
    if (l == 0) a.best[k] = at ? first_lane(at) : -1;
}

hipError_t launch_cv_gather(const CvArgs &a, hipStream_t s)
{
    if (a.num_train > 0) hipLaunchKernelGGL(k_cv_gather, dim3(a.num_train), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cv_score(const CvArgs &a, hipStream_t s)
{
    if (a.num_train > 0) hipLaunchKernelGGL(k_cv_validate, dim3(a.num_train), dim3(64), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.num_base > 0) hipLaunchKernelGGL(k_cv_select, dim3(a.num_base), dim3(64), 0, s, a);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Subset-stability statistics: for group g, path step t, feature j, the
// fraction of the group's solves (status certified or non-unique) whose b_j
// is non-zero.  Integer counts by atomics, so the result does not depend on
// the order of the solves.  counts holds G * L * 33 ints: 32 feature hits
// and the number of accepted solves.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sel_zero(int32_t *c, int64_t n, int32_t *bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
    if (i == 0) *bad = 0;
}

__global__ __launch_bounds__(256) void k_sel_count(const uint32_t *active, const int32_t *status,
                                                   const int32_t *group, int32_t S, int32_t L, int32_t G,
                                                   int32_t *c, int32_t *bad)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; // output (s, t)
    if (o >= (int64_t)S * L) return;
    const int s = (int)(o / L), t = (int)(o - (int64_t)s * L);
    const int g = group ? group[s] : 0;
    if (g < 0 || g >= G) {
        atomicOr(bad, 1);
        return;
    }
    const int st = status[o];
    if (st != ST_CERTIFIED && st != ST_NONUNIQUE) return;
    int32_t *cg = c + ((int64_t)g * L + t) * 33;
    uint32_t m = active[o];
    while (m) {
        const int j = __builtin_ctz(m);
        m &= m - 1;
        atomicAdd(cg + j, 1);
    }
    atomicAdd(cg + 32, 1);
}

__global__ __launch_bounds__(256) void k_sel_norm(const int32_t *c, int64_t GL, float *freq)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; // (g, t, j)
    if (i >= GL * 32) return;
    const int64_t gt = i / 32;
    const int j = (int)(i - gt * 32);
    const int32_t n = c[gt * 33 + 32];
    freq[i] = n > 0 ? (float)((double)c[gt * 33 + j] / (double)n) : 0.f;
}

hipError_t launch_selection_frequency(const uint32_t *active, const int32_t *status, const int32_t *group,
                                      int32_t num_solves, int32_t path_len, int32_t num_groups, int32_t *counts,
                                      float *freq, int32_t *bad_group, hipStream_t s)
{
    const int64_t GL = (int64_t)num_groups * path_len;
    const int64_t nc = GL * 33, no = (int64_t)num_solves * path_len;
    hipLaunchKernelGGL(k_sel_zero, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, counts, nc, bad_group);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (no > 0)
        hipLaunchKernelGGL(k_sel_count, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, s, active, status, group,
                           num_solves, path_len, num_groups, counts, bad_group);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sel_norm, dim3((unsigned)((GL * 32 + 255) / 256)), dim3(256), 0, s, counts, GL, freq);
    return hipGetLastError();
}

} // namespace ladl
