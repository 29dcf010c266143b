// Tile schedule: the paper's cyclic coordinate descent and ternary chop
// (Sections 3.3-3.6) for small problems (n <= 64), several problems per
// wavefront.  A wave is
// cut into segments of S = 16 or 32 lanes; each segment runs one solve,
// lane i of the segment holding rows i, i + S, ... (RS row slots, n <= S RS).
// The segment's scalars (b_j, lambda, f, the loop state) are computed
// identically in all its lanes: every reduction is an xor butterfly (DPP
// inside a row of 16 lanes, one row exchange across rows), whose two partners
// add the same pair of values, so all lanes of a segment end with the same
// bits and take the same branches; segments diverge from each other only
// through the execution mask.
//
// This stage solves the cold start of each solve (the first step of its
// lambda path) up to the end of the paper's search: coordinate descent to
// an axis-wise minimum, then the ternary chop along the locus of axis-wise
// minima (Sections 3.5-3.6, the rounds the options ask for, each probe a
// coordinate descent with the chop axis frozen), then coordinate descent
// again.  It writes that point; the wavefront kernel starts from it (its
// seed) and runs the rest: a confirming sweep, the snap to a vertex, its
// certificate and the finisher.  Later path steps start from the previous
// step's certified vertex, as without tiles.  Unlike the wavefront kernel,
// which chops only where the certificate of the first descent fails, this
// stage chops every solve: it has no certificate of its own.
// The 1-D minimisation is the exact one: the lower weighted
// median of the kinks t_i = b_j + r_i / x_ij (weight |x_ij|) and 0 (weight
// lambda), found from the current b_j by signs (which side holds the
// median) and then by walking the kinks outward from b_j, nearest first,
// until their cumulative weight reaches the median's.
#include "ladl_common.hpp"
#include "ladl_wave.hpp"

namespace ladl {
namespace {

constexpr int TILE_BLOCK = 64; // one wavefront per workgroup

// ordering of LDS accesses between the lanes of one wavefront (no
// instruction: LDS operations of a wave execute in issue order; this keeps
// the compiler from moving them across)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the value of the same lane in the other row of 16 of a 32-lane segment
// (v_permlane16_swap of gfx950 exchanges the odd rows of its first operand
// with the even rows of its second: with v in both, an even row finds its
// partner in the second result, an odd row in the first)
__device__ __forceinline__ unsigned other_row(unsigned v)
{
    const auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return ((threadIdx.x >> 4) & 1) ? sw[0] : sw[1];
}
__device__ __forceinline__ float other_row(float v) { return bitsf((int)other_row((unsigned)fbits(v))); }
__device__ __forceinline__ int other_row(int v) { return (int)other_row((unsigned)v); }

// xor butterflies over a segment: quad swaps, then the half-row and row
// mirrors (after the quad steps every quad is uniform, so a mirror pairs
// whole quads), then for 32-lane segments the exchange of its two rows
template <int S>
__device__ __forceinline__ float seg_sum(float v)
{
    v += dpp<DPP_XOR1>(0.f, v);
    v += dpp<DPP_XOR2>(0.f, v);
    v += dpp<DPP_HMIRROR>(0.f, v);
    v += dpp<DPP_MIRROR>(0.f, v);
    if constexpr (S == 32) v += other_row(v);
    return v;
}

template <int S>
__device__ __forceinline__ void seg_sum2(float &a, float &b)
{
    a += dpp<DPP_XOR1>(0.f, a);
    b += dpp<DPP_XOR1>(0.f, b);
    a += dpp<DPP_XOR2>(0.f, a);
    b += dpp<DPP_XOR2>(0.f, b);
    a += dpp<DPP_HMIRROR>(0.f, a);
    b += dpp<DPP_HMIRROR>(0.f, b);
    a += dpp<DPP_MIRROR>(0.f, a);
    b += dpp<DPP_MIRROR>(0.f, b);
    if constexpr (S == 32) {
        a += other_row(a);
        b += other_row(b);
    }
}

template <int S>
__device__ __forceinline__ float seg_min(float v)
{
    v = fminf(v, dpp<DPP_XOR1>(FINF, v));
    v = fminf(v, dpp<DPP_XOR2>(FINF, v));
    v = fminf(v, dpp<DPP_HMIRROR>(FINF, v));
    v = fminf(v, dpp<DPP_MIRROR>(FINF, v));
    if constexpr (S == 32) v = fminf(v, other_row(v));
    return v;
}

template <int S>
__device__ __forceinline__ int seg_min_i(int v)
{
    v = min(v, dppi<DPP_XOR1>(INT_MAX, v));
    v = min(v, dppi<DPP_XOR2>(INT_MAX, v));
    v = min(v, dppi<DPP_HMIRROR>(INT_MAX, v));
    v = min(v, dppi<DPP_MIRROR>(INT_MAX, v));
    if constexpr (S == 32) v = min(v, other_row(v));
    return v;
}

// floats of one segment's LDS region: X column-major (pmax columns of S RS
// rows), b, sum_i |x_ij| and the chop's best b (pmax each); padded so that
// the 16-lane segments sharing a half-wave start on different banks
__host__ __device__ constexpr int tile_seg_floats(int S, int RS, int pmax)
{
    const int f = pmax * S * RS + 3 * pmax;
    return (S == 16) ? ((f + 31) / 32) * 32 + 16 : ((f + 31) / 32) * 32;
}

template <int S, int RS>
struct Seg {
    static constexpr int NM = S * RS;
    const float *xs; // X column j: xs[j * NM + i]
    float *bs;       // b_j
    const float *cs; // sum_i |x_ij|
    float *bb;       // the chop's best point
    int n, p, sl;
    float lam;
};

// f = sum |r_i| + lambda sum |b_j| (p <= 32 <= 2 S)
template <int S, int RS>
__device__ __forceinline__ float seg_objective(const Seg<S, RS> &g, const float (&r)[RS])
{
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < RS; ++k) s += fabsf(r[k]);
    float sb = (g.sl < g.p) ? fabsf(g.bs[g.sl]) : 0.f;
    sb += (g.sl + S < g.p) ? fabsf(g.bs[g.sl + S]) : 0.f;
    seg_sum2<S>(s, sb);
    return s + g.lam * sb;
}

// exact minimisation of f along axis j; true if b_j moved
template <int S, int RS>
__device__ __forceinline__ bool seg_update(const Seg<S, RS> &g, float (&r)[RS], int j)
{
    constexpr int NM = Seg<S, RS>::NM;
    float x[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) {
        const int i = g.sl + S * k;
        x[k] = (i < g.n) ? g.xs[j * NM + i] : 0.f;
    }
    const float bj = g.bs[j];
    // weight of the kinks below b_j (r_i x_ij < 0) and at b_j (r_i = 0)
    float bel = 0.f, at = 0.f;
#pragma unroll
    for (int k = 0; k < RS; ++k) {
        const float ax = fabsf(x[k]);
        bel += (r[k] * x[k] < 0.f) ? ax : 0.f;
        at += (r[k] == 0.f) ? ax : 0.f;
    }
    seg_sum2<S>(bel, at);
    const float lam = g.lam;
    const float W = g.cs[j] + lam;
    if (!(W > 0.f)) return false;
    const float belT = bel + ((bj > 0.f) ? lam : 0.f);
    const float atT = at + ((bj == 0.f) ? lam : 0.f);
    const float half = 0.5f * W;
    bool down;
    if (belT >= half)
        down = true;
    else if (belT + atT < half)
        down = false;
    else
        return false; // b_j is the lower weighted median already
    // moving down, the median is the nearest kink below b_j whose
    // cumulative weight (from b_j outward, that kink included) exceeds
    // belT - W/2; moving up, the nearest one above where it reaches
    // W/2 - belT - atT
    const float T = down ? (belT - half) : (half - belT - atT);
    // distances of the kinks on the moving side (none: FINF)
    // (the same float as the wavefront kernel's: r_i rcp(x_ij), the sign
    // flipped when moving down)
    const int flip = down ? (int)0x80000000 : 0;
    float a[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) {
        const float off = bitsf(fbits(r[k] * __builtin_amdgcn_rcpf(x[k])) ^ flip);
        a[k] = (off > 0.f) ? off : FINF; // x = 0: no kink (inf or NaN)
    }
    const bool lcand = (lam > 0.f) && (down ? (bj > 0.f) : (bj < 0.f));
    const float al = fabsf(bj);
    // walk outward: kinks at distances <= lo are counted in cum
    float cum = 0.f, lo = -1.f, mm = FINF;
    for (int it = 0; it <= NM; ++it) {
        float ml = FINF;
#pragma unroll
        for (int k = 0; k < RS; ++k) ml = fminf(ml, (a[k] > lo) ? a[k] : FINF);
        float m = seg_min<S>(ml);
        const bool lnext = lcand && al > lo;
        if (lnext) m = fminf(m, al);
        if (!(m < FINF)) break; // kinks used up (rounding): keep the farthest
        float wl = 0.f;
#pragma unroll
        for (int k = 0; k < RS; ++k) wl += (a[k] == m) ? fabsf(x[k]) : 0.f;
        wl = seg_sum<S>(wl);
        if (lnext && al == m) wl += lam;
        mm = m;
        lo = m;
        cum += wl;
        if (down ? (cum > T) : (cum >= T)) break;
    }
    if (!(mm < FINF)) return false; // nothing on the moving side
    // the median row (lowest index among the kinks at that distance) goes
    // exactly onto its hyperplane; the lambda kink alone moves b_j to 0
    int own = INT_MAX;
#pragma unroll
    for (int k = RS - 1; k >= 0; --k) own = (a[k] == mm) ? (g.sl + S * k) : own;
    own = seg_min_i<S>(own);
    const float nb = (own == INT_MAX) ? 0.f : (down ? bj - mm : bj + mm);
    const float d = nb - bj;
    if (d == 0.f || !__builtin_isfinite(d)) return false;
#pragma unroll
    for (int k = 0; k < RS; ++k) {
        r[k] = fmaf(-x[k], d, r[k]);
        r[k] = (g.sl + S * k == own) ? 0.f : r[k];
    }
    wave_lds_sync();
    if (g.sl == 0) g.bs[j] = nb;
    wave_lds_sync();
    return true;
}

// cyclic coordinate descent with axis `frozen` held (-1: none), stopped as
// the wavefront kernel stops it: a sweep that moves nothing, or lowers f
// by at most tol_f f, or the sweep cap
template <int S, int RS>
__device__ __forceinline__ float seg_ccd(const Seg<S, RS> &g, float (&r)[RS], int frozen, float f,
                                         const DevOpt &opt)
{
    if (g.p == 1 && frozen == 0) return f;
    for (int sw = 0; sw < opt.max_sweeps; ++sw) {
        bool changed = false;
        for (int j = 0; j < g.p; ++j)
            if (j != frozen) changed |= seg_update(g, r, j);
        const float fn = seg_objective(g, r);
        const bool stop = !changed || (f - fn <= opt.tol_f * fn);
        f = fn;
        if (stop) break;
    }
    return f;
}

// b := the saved best point, or (save) the best point := b; the caller
// keeps the matching residuals in registers
template <int S, int RS>
__device__ __forceinline__ void seg_copy_b(const Seg<S, RS> &g, bool save)
{
    wave_lds_sync();
    for (int j = g.sl; j < g.p; j += S) {
        if (save)
            g.bb[j] = g.bs[j];
        else
            g.bs[j] = g.bb[j];
    }
    wave_lds_sync();
}

// descent, the chop rounds along the locus of axis-wise minima, descent:
// the same sequence of probes as the wavefront kernel's search when its
// certificate never succeeds
template <int S, int RS>
__device__ __forceinline__ void seg_search(const Seg<S, RS> &g, float (&r)[RS], float f, float B, const DevOpt &opt)
{
    constexpr int NM = Seg<S, RS>::NM;
    const int p = g.p;
    const int rounds = (p < 2) ? 0 : ((opt.max_rounds < 0) ? p : opt.max_rounds);
    Chop q;
    float rb[RS];
    int phase = 0, frozen = -1, round = 0, kax = 0;
    float fbest = FINF;
    for (;;) {
        f = seg_ccd(g, r, frozen, f, opt);
        float sprobe = 0.f;
        bool more;
        if (phase == 0) {
            if (round >= rounds) break;
            if (round == 0) {
                // the axis of the largest |b_j| (lowest j on ties)
                const float b0 = (g.sl < p) ? fabsf(g.bs[g.sl]) : -1.f;
                const float b1 = (g.sl + S < p) ? fabsf(g.bs[g.sl + S]) : -1.f;
                const float bm = seg_min<S>(-fmaxf(b0, b1));
                int c = INT_MAX;
                c = (b1 == -bm) ? g.sl + S : c;
                c = (b0 == -bm) ? g.sl : c;
                kax = seg_min_i<S>(c);
            } else {
                kax = (kax + 1) % p;
            }
            ++round;
            seg_copy_b(g, true);
#pragma unroll
            for (int kk = 0; kk < RS; ++kk) rb[kk] = r[kk];
            fbest = f;
            chop_init(q, g.bs[kax], f, B, opt.chop_range);
            more = chop_next(q, 0.f, sprobe, opt);
        } else {
            if (f < fbest) {
                fbest = f;
                seg_copy_b(g, true);
#pragma unroll
                for (int kk = 0; kk < RS; ++kk) rb[kk] = r[kk];
            }
            more = chop_next(q, f, sprobe, opt);
        }
        // the next descent starts from the best point; a probe sets b_kax := s
        seg_copy_b(g, false);
#pragma unroll
        for (int kk = 0; kk < RS; ++kk) r[kk] = rb[kk];
        if (more) {
            const float d = sprobe - g.bs[kax];
            if (d != 0.f) {
#pragma unroll
                for (int kk = 0; kk < RS; ++kk) {
                    const int i = g.sl + S * kk;
                    if (i < g.n) r[kk] = fmaf(-g.xs[kax * NM + i], d, r[kk]);
                }
            }
            wave_lds_sync();
            if (g.sl == 0) g.bs[kax] = sprobe;
            wave_lds_sync();
            f = seg_objective(g, r);
            frozen = kax;
            phase = 1;
        } else {
            f = fbest;
            frozen = -1;
            phase = 0;
        }
    }
}

template <int S, int RS>
__global__ __launch_bounds__(TILE_BLOCK) void k_tile(SolveArgs a)
{
    constexpr int NM = S * RS;
    extern __shared__ float lds[];
    const int pm = a.pmax;
    const int sl = threadIdx.x & (S - 1);
    float *xs = lds + (threadIdx.x / S) * tile_seg_floats(S, RS, pm);
    float *bs = xs + pm * NM;
    float *cs = bs + pm;
    float *bb = cs + pm;
    for (;;) {
        int q = 0;
        if (sl == 0) q = atomicAdd(a.counter, 1);
        q = __shfl(q, 0, S);
        if (q >= a.num_items) break;
        const int s = a.order[q];
        const int k = a.problem ? a.problem[s] : s;
        const int64_t r0 = a.row_off[k];
        const int n = (int)(a.row_off[k + 1] - r0);
        const int p = a.p_arr[k];
        const int64_t bbase = (int64_t)a.path_len * a.b_off[s];
        if (n > NM || p > pm) {
            // not a problem of this tile shape (the host never queues one):
            // zero seeds, and the wavefront stage solves it from there
            for (int t = a.t0; t < a.t1; ++t)
                for (int j = sl; j < p; j += S) a.b_out[bbase + (int64_t)t * p + j] = 0.f;
            continue;
        }
        // X (row-major n x p in HBM) into the segment's columns
        const float *Xk = a.X + a.x_off[k];
        bool fin = true;
        wave_lds_sync();
        for (int e = sl; e < n * p; e += S) {
            const float v = Xk[e];
            fin = fin && __builtin_isfinite(v);
            const int i = e / p;
            xs[(e - i * p) * NM + i] = v;
        }
        float yv[RS], ya = 0.f;
#pragma unroll
        for (int kk = 0; kk < RS; ++kk) {
            const int i = sl + S * kk;
            yv[kk] = (i < n) ? a.y[r0 + i] : 0.f;
            fin = fin && __builtin_isfinite(yv[kk]);
            ya += fabsf(yv[kk]);
        }
        const float ynorm1 = seg_sum<S>(ya);
        wave_lds_sync();
        for (int j = 0; j < p; ++j) {
            float c = 0.f;
#pragma unroll
            for (int kk = 0; kk < RS; ++kk) {
                const int i = sl + S * kk;
                c += (i < n) ? fabsf(xs[j * NM + i]) : 0.f;
            }
            c = seg_sum<S>(c);
            if (sl == 0) cs[j] = c;
        }
        const bool ok = seg_min<S>(fin ? 1.f : 0.f) > 0.f;
        // start point of the first step: the previous step of this stage,
        // else b_init, else 0
        for (int j = sl; j < p; j += S) {
            float b0 = 0.f;
            if (a.t0 > 0)
                b0 = a.b_out[bbase + (int64_t)(a.t0 - 1) * p + j];
            else if (a.b_init)
                b0 = a.b_init[a.b_off[s] + j];
            bs[j] = __builtin_isfinite(b0) ? b0 : 0.f;
        }
        wave_lds_sync();
        Seg<S, RS> g{xs, bs, cs, bb, n, p, sl, 0.f};
        for (int t = a.t0; t < a.t1; ++t) {
            const int64_t o = (int64_t)s * a.path_len + t;
            float *bo = a.b_out + bbase + (int64_t)t * p;
            const float lam_in = a.lam[o];
            if (!ok || !(lam_in >= 0.f)) {
                // the wavefront stage reports these; start the next step at 0
                for (int j = sl; j < p; j += S) {
                    bs[j] = 0.f;
                    bo[j] = 0.f;
                }
                wave_lds_sync();
                continue;
            }
            g.lam = fmaxf(lam_in, a.opt.lambda_min);
            float r[RS];
#pragma unroll
            for (int kk = 0; kk < RS; ++kk) r[kk] = yv[kk];
            for (int j = 0; j < p; ++j) {
                const float bj = bs[j];
                if (bj != 0.f) {
#pragma unroll
                    for (int kk = 0; kk < RS; ++kk) {
                        const int i = sl + S * kk;
                        if (i < n) r[kk] = fmaf(-xs[j * NM + i], bj, r[kk]);
                    }
                }
            }
            const float B = (g.lam > 0.f) ? ynorm1 / g.lam : FINF;
            seg_search(g, r, seg_objective(g, r), B, a.opt);
            for (int j = sl; j < p; j += S) bo[j] = bs[j];
        }
        wave_lds_sync();
    }
}

template <int S, int RS>
static hipError_t launch_tile_t(const SolveArgs &a, int grid, hipStream_t s)
{
    const size_t lds = tile_lds_bytes(S, RS, a.pmax);
    hipLaunchKernelGGL((k_tile<S, RS>), dim3(grid), dim3(TILE_BLOCK), lds, s, a);
    return hipGetLastError();
}

template <int S, int RS>
static int tile_blocks_t(int pmax)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile<S, RS>, TILE_BLOCK, tile_lds_bytes(S, RS, pmax)) !=
        hipSuccess)
        return 0;
    return nb;
}

} // namespace

bool tile_shape_for(int nmax, int &S, int &RS)
{
    if (nmax <= 16) {
        S = 16, RS = 1;
    } else if (nmax <= 32) {
        S = 16, RS = 2;
    } else if (nmax <= 64) {
        S = 32, RS = 2;
    } else {
        return false;
    }
    return true;
}

size_t tile_lds_bytes(int S, int RS, int pmax) { return 4 * (size_t)(TILE_BLOCK / S) * tile_seg_floats(S, RS, pmax); }

int tile_solves_per_block(int S) { return TILE_BLOCK / S; }

int tile_max_blocks_per_cu(int S, int RS, int pmax)
{
    if (S == 16 && RS == 1) return tile_blocks_t<16, 1>(pmax);
    if (S == 16 && RS == 2) return tile_blocks_t<16, 2>(pmax);
    if (S == 32 && RS == 2) return tile_blocks_t<32, 2>(pmax);
    return 0;
}

hipError_t launch_tile(int S, int RS, const SolveArgs &a, int grid, hipStream_t s)
{
    if (grid < 1 || a.pmax < 1 || a.pmax > PMAX) return hipErrorInvalidValue;
    if (S == 16 && RS == 1) return launch_tile_t<16, 1>(a, grid, s);
    if (S == 16 && RS == 2) return launch_tile_t<16, 2>(a, grid, s);
    if (S == 32 && RS == 2) return launch_tile_t<32, 2>(a, grid, s);
    return hipErrorInvalidValue;
}

} // namespace ladl
