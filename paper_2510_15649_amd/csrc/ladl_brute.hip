// Exact LAD-LASSO by vertex enumeration (Section 3.2 of the paper): every
// choice of p hyperplanes among the n residual hyperplanes x_i.b = y_i and
// the p axis hyperplanes b_j = 0 that meet in one point is a candidate; f is
// piecewise linear and its minimum is attained at such a point, so the
// smallest f over all candidates is the global minimum.
//
// One wave per (solve, path step).  The C(n+p, p) candidates are split into
// 64 contiguous runs of the lexicographic order, one per lane; each lane
// unranks its first candidate, then steps to the next combination.  The
// p x p system is solved in fp64 registers (Gaussian elimination, partial
// pivoting by selects, p fixed per template instance) and f is evaluated in
// fp64 against X and y held in LDS.  The wave minimum (ties: lowest rank)
// gives the answer.
#include "ladl_common.hpp"
#include "ladl_kernels.hpp"
#include "ladl_wave.hpp"

namespace ladl {

constexpr int BF_NMAX = 64; // n + p <= 64

// C(m, k) for 0 <= k <= m <= 64 (exact in int64 for the sizes allowed)
__device__ __forceinline__ int64_t binom(int m, int k)
{
    if (k < 0 || k > m) return 0;
    int64_t b = 1;
    for (int j = 1; j <= k; ++j) b = b * (m - k + j) / j;
    return b;
}

template <int P>
__global__ __launch_bounds__(64) void k_brute(BruteArgs a)
{
    __shared__ double Xs[BF_NMAX * P];
    __shared__ double ys[BF_NMAX];
    const int l = lane_id();
    const int o = blockIdx.x;
    if (o >= a.count * a.path_len) return;
    const int s = a.order[o / a.path_len];
    const int t = o % a.path_len;
    const int k = a.problem ? a.problem[s] : s;
    const int64_t r0 = a.row_off[k];
    const int n = (int)(a.row_off[k + 1] - r0);
    const float *X = a.X + a.x_off[k];
    for (int e = l; e < n * P; e += 64) Xs[e] = (double)X[e];
    for (int i = l; i < n; i += 64) ys[i] = (double)a.y[r0 + i];
    __syncthreads();
    const int64_t oo = (int64_t)s * a.path_len + t;
    const double lam = (double)a.lam[oo];
    const int N = n + P;
    const int64_t C = binom(N, P);
    int64_t r = C * l / 64;
    const int64_t rend = C * (l + 1) / 64;
    // unrank r (lexicographic order)
    int cmb[P];
    {
        int64_t rr = r;
        int v = 0;
#pragma unroll
        for (int i = 0; i < P; ++i) {
            for (;;) {
                const int64_t c = binom(N - 1 - v, P - 1 - i);
                if (rr < c || v >= N - P + i) break;
                rr -= c;
                ++v;
            }
            cmb[i] = v++;
        }
    }
    double best = __builtin_inf();
    double bb[P];
#pragma unroll
    for (int j = 0; j < P; ++j) bb[j] = 0.0;
    int64_t brank = INT64_MAX;
    double nonsing = 0.0;
    for (; r < rend; ++r) {
        // the system: row q from hyperplane cmb[q]
        double M[P][P + 1];
        double amax = 0.0;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int h = cmb[q];
            const bool row = h < n;
#pragma unroll
            for (int c = 0; c < P; ++c) {
                M[q][c] = row ? Xs[h * P + c] : ((h - n == c) ? 1.0 : 0.0);
                amax = fmax(amax, fabs(M[q][c]));
            }
            M[q][P] = row ? ys[h] : 0.0;
        }
        bool ok = true;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            // partial pivot: the largest |M[q][c]|, q >= c, swapped into row c
            int pr = c;
            double pv = fabs(M[c][c]);
#pragma unroll
            for (int q = c + 1; q < P; ++q) {
                const bool gt = fabs(M[q][c]) > pv;
                pv = gt ? fabs(M[q][c]) : pv;
                pr = gt ? q : pr;
            }
            ok = ok && (pv > 1e-12 * amax);
#pragma unroll
            for (int q = c + 1; q < P; ++q) {
                const bool sw = (pr == q);
#pragma unroll
                for (int e = c; e <= P; ++e) {
                    const double u = M[c][e];
                    M[c][e] = sw ? M[q][e] : u;
                    M[q][e] = sw ? u : M[q][e];
                }
            }
            const double inv = ok ? 1.0 / M[c][c] : 0.0;
#pragma unroll
            for (int q = c + 1; q < P; ++q) {
                const double m = M[q][c] * inv;
#pragma unroll
                for (int e = c + 1; e <= P; ++e) M[q][e] = fma(-m, M[c][e], M[q][e]);
            }
        }
        if (ok) {
            double bv[P];
#pragma unroll
            for (int c = P - 1; c >= 0; --c) {
                double acc = M[c][P];
#pragma unroll
                for (int e = c + 1; e < P; ++e) acc = fma(-M[c][e], bv[e], acc);
                bv[c] = acc / M[c][c];
            }
            double f = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) f += fabs(bv[j]);
            f *= lam;
            for (int i = 0; i < n; ++i) {
                double ri = ys[i];
#pragma unroll
                for (int j = 0; j < P; ++j) ri = fma(-Xs[i * P + j], bv[j], ri);
                f += fabs(ri);
            }
            nonsing += 1.0;
            if (f < best) {
                best = f;
                brank = r;
#pragma unroll
                for (int j = 0; j < P; ++j) bb[j] = bv[j];
            }
        }
        // next combination in lexicographic order
        int i = P - 1;
#pragma unroll
        for (int q = P - 1; q >= 0; --q)
            if (i == q && cmb[q] == N - P + q) i = q - 1;
        if (i < 0) break;
        const int nv = cmb[i] + 1;
#pragma unroll
        for (int q = 0; q < P; ++q) cmb[q] = (q == i) ? nv : ((q > i) ? nv + (q - i) : cmb[q]);
    }
    // wave minimum of f, ties to the lowest rank
    double m = best;
    for (int d = 1; d < 64; d <<= 1) m = fmin(m, __shfl_xor(m, d));
    const uint64_t at = ballot(best == m && brank != INT64_MAX);
    int owner = at ? first_lane(at) : -1; // lanes hold increasing rank ranges
    const double cnt = wsum_d(nonsing);
    float *bout = a.b_out + (int64_t)a.path_len * a.b_off[s] + (int64_t)t * P;
    if (owner < 0) {
        if (l < P) bout[l] = 0.f;
        if (l == 0) a.obj_out[oo] = __builtin_nanf("");
    } else if (l == owner) {
#pragma unroll
        for (int j = 0; j < P; ++j) bout[j] = (float)bb[j];
        a.obj_out[oo] = (float)best;
    }
    if (l == 0 && a.vert_out) a.vert_out[oo] = (int64_t)cnt;
}

hipError_t launch_brute(int p, const BruteArgs &a, hipStream_t s)
{
    const int grid = a.count * a.path_len;
    if (grid <= 0) return hipSuccess;
    switch (p) {
    case 1: hipLaunchKernelGGL(k_brute<1>, dim3(grid), dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_brute<2>, dim3(grid), dim3(64), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_brute<3>, dim3(grid), dim3(64), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_brute<4>, dim3(grid), dim3(64), 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_brute<5>, dim3(grid), dim3(64), 0, s, a); break;
    case 6: hipLaunchKernelGGL(k_brute<6>, dim3(grid), dim3(64), 0, s, a); break;
    case 7: hipLaunchKernelGGL(k_brute<7>, dim3(grid), dim3(64), 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_brute<8>, dim3(grid), dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace ladl
