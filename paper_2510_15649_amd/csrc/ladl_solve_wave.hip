// Forward LAD-LASSO solve: one solve per wavefront, or per team of TW
// wavefronts of one workgroup, in a persistent grid with an atomic work
// queue; problem data in LDS (or partly in a per-team HBM workspace for the
// larger buckets).
//
// Per solve (Abstract; Sections 3.3-3.6 of the paper, plus a vertex
// certificate and simplex finisher that the paper does not have):
//   1. cyclical coordinate descent, each axis minimised exactly by the
//      weighted median of the kinks r_i/x_ij + b_j (weights |x_ij|) and the
//      penalty kink 0 (weight lambda);
//   2. snap to the nearest vertex (p hyperplanes, Section 3.2) and test the
//      LP optimality certificate;
//   3. ternary chop along one axis, each probe a restricted warm-started
//      CCD with that axis frozen, range extended until it brackets the
//      minimum (Sections 3.5-3.6); polish, snap and certify again;
//   4. primal simplex steps along the vertex's edges until certified.
//
// Rows.  With RT = 64 TW rows per register slot, row i belongs to wave
// (i / 64) mod TW, lane i mod 64, slot i / RT: each slot of a wave covers 64
// consecutive rows, so column reads stay coalesced.  Every reduction over
// rows is a team reduction (ladl_team.hpp); b, the chop state and the vertex
// algebra are replicated in every wave and updated identically.
//
// Layout in LDS (floats), per team:
//   shared: team exchange slots; sa/sw (compaction), the sample exchange;
//       Xs: p columns of LDN = 64 R TW + 1 floats, row i of column j at
//       j*LDN + i (rows >= n are 0); ys: y, LDN floats
//   per wave: gd (32 doubles), best residuals (64 R), A (vertex matrix / LU,
//       pmax rows of 33), A0 (unfactored, pmax x (pmax+1)), six vectors of
//       32 (b, best b, column |x| sums, direction, scratch), zs/ss/piv, the
//       chop state
// With the HBM workspace (XG), only the first nlds columns stay in LDS (as
// many as the LDS left over at the kernel's occupancy holds); the other
// columns and y live in the team's workspace slice, in the same layout.
#include "ladl_common.hpp"
#include "ladl_kernels.hpp"
#include "ladl_team.hpp"
#include "ladl_wave.hpp"

#include <climits>

namespace ladl {

__host__ __device__ constexpr int wave_ldn(int R, int TW) { return 64 * R * TW + 1; }

constexpr int CHOP_FLOATS = 32;
// LDS floats shared by a team: exchange slots, sa/sw, samples, queue word
__host__ __device__ constexpr size_t team_shared_floats(int TW)
{
    return (size_t)team_red_words(TW) + 128 + (TW > 1 ? 64 * TW : 0) + 4;
}
// LDS floats private to each wave (a multiple of 4, so every wave's gd
// stays 16-byte aligned)
__host__ __device__ constexpr size_t wave_private_floats(int R, int pmax)
{
    return ((64 + 64 * (size_t)R + (size_t)pmax * ALD + (size_t)pmax * (pmax + 1) + 6 * 32 + 3 * 32 + CHOP_FLOATS) +
            3) & ~(size_t)3;
}
// LDS floats per team: shared part, [Xs, ys when resident; the first nlds
// columns of Xs with the workspace], TW private parts
__host__ __device__ constexpr size_t wave_lds_floats(int R, int pmax, bool xg, int nlds, int TW)
{
    return team_shared_floats(TW) + (size_t)(xg ? nlds : pmax + 1) * wave_ldn(R, TW) +
           (size_t)TW * wave_private_floats(R, pmax);
}
// global workspace floats per team with the workspace: columns nlds .. p-1
// of Xs, then ys
__host__ __device__ constexpr size_t wave_ws_floats(int R, int pmax, int nlds, int TW)
{
    return (size_t)(pmax + 1 - nlds) * wave_ldn(R, TW);
}

template <int R, bool XG, int TW>
struct Wave {
    static constexpr int LDN = wave_ldn(R, TW);
    static constexpr int RT = 64 * TW; // rows per register slot of the team
    // Xs: the LDS columns of X (all of them without the workspace); Xg: the
    // workspace columns (column j >= nlds at (j - nlds) * LDN); ys: y, in
    // LDS without the workspace, else after the workspace columns
    float *Xs, *Xg, *ys, *rbuf, *A, *A0, *vb, *vbb, *vca, *vd, *vg, *vt, *sa, *sw, *smp;
    double *gd;
    int *zs, *ss, *piv, *qw;
    // the ternary chop's state (uniform): kept in LDS rather than in VGPRs
    // that would be live across every probe's CCD
    Chop *chop;
    Team<TW> tm;
    int wv, rb;   // wave in the team; row of this lane in slot 0 (64 wv + lane)
    int n, p, nslot, a0ld, nlds;
    float lam, ynorm1;
    float cav; // lane j: sum_i |x_ij|
    DevOpt opt;
    int c_sweeps, c_updates, c_probes, c_pivots;
    double fv64; // objective of the last evaluated vertex, fp64 residual sums
};

// the team row of register slot k of this lane
template <int R, bool XG, int TW>
__device__ __forceinline__ int row_of(const Wave<R, XG, TW> &w, int k)
{
    return Wave<R, XG, TW>::RT * k + w.rb;
}
// wave, slot and lane that hold team row i
__device__ __forceinline__ int row_wave(int i, int TW) { return (i >> 6) % TW; }
__device__ __forceinline__ int row_slot(int i, int TW) { return i / (64 * TW); }

template <int R, bool XG, int TW>
LADL_INL void carve(Wave<R, XG, TW> &w, float *smem, int pmax, int nlds, float *ws, int wv)
{
    constexpr int LDN = Wave<R, XG, TW>::LDN;
    float *q = smem; // the dynamic LDS base is 16-byte aligned
    w.wv = wv;
    w.rb = 64 * wv + lane_id();
    w.tm.wv = wv;
    w.tm.seq = 0;
    w.tm.red = q;
    w.tm.vec = (double *)(q + 16 * TW);
    q += team_red_words(TW);
    w.sa = q;
    q += 64;
    w.sw = q;
    q += 64;
    w.smp = q;
    q += (TW > 1 ? 64 * TW : 0);
    w.qw = (int *)q;
    q += 4;
    w.Xs = q;
    if (XG) {
        w.nlds = nlds;
        q += (size_t)nlds * LDN;
        w.Xg = ws;
        w.ys = ws + (size_t)(pmax - nlds) * LDN;
    } else {
        w.nlds = pmax;
        q += (size_t)pmax * LDN;
        w.Xg = nullptr;
        w.ys = q;
        q += LDN;
    }
    // this wave's private part (a multiple of 4 floats from a 16-byte
    // aligned start: team_shared_floats and LDN-sized blocks keep q aligned
    // to 4 bytes only, so round up)
    q = (float *)(((uintptr_t)q + 15) & ~(uintptr_t)15);
    q += (size_t)wv * wave_private_floats(R, pmax);
    w.gd = (double *)q;
    q += 64;
    w.rbuf = q;
    q += 64 * R;
    w.A = q;
    q += pmax * ALD;
    w.A0 = q; // unfactored copy of the vertex matrix, row stride pmax + 1
    w.a0ld = pmax + 1;
    q += pmax * (pmax + 1);
    w.vb = q;
    q += 32;
    w.vbb = q;
    q += 32;
    w.vca = q;
    q += 32;
    w.vd = q;
    q += 32;
    w.vg = q;
    q += 32;
    w.vt = q;
    q += 32;
    w.zs = (int *)q;
    q += 32;
    w.ss = (int *)q;
    q += 32;
    w.piv = (int *)q;
    q += 32;
    w.chop = (Chop *)q;
}

// After the team writes its workspace (global memory when XG): the stores
// complete, and L1 drops lines it may hold from before, so the next loads
// see what was written.  With LDS only the barrier is needed.
template <bool XG>
LADL_INL void ws_sync()
{
    if (XG) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Element idx of column j of X (j may differ between lanes): LDS
// instructions without the workspace; with it, for R = 32 a branch to an
// LDS or a global load, for smaller R one generic load of the selected
// address (measured on the ragged workload: the branch form made the
// n <= 2048 bucket 1.5x faster and the n <= 512 and n <= 1024 buckets 5%
// slower).  And this lane's R elements of a column j that is the same on
// every lane, from LDS (j < nlds) or from the workspace (j >= nlds).
typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(1))) float glb_f32;

template <int R, bool XG, int TW>
LADL_INL const float *xaddr(const Wave<R, XG, TW> &w, int j)
{
    constexpr int LDN = Wave<R, XG, TW>::LDN;
    return (j < w.nlds) ? w.Xs + j * LDN : w.Xg + (j - w.nlds) * LDN;
}

template <int R, bool XG, int TW>
LADL_INL float xget(const Wave<R, XG, TW> &w, int j, int idx)
{
    constexpr int LDN = Wave<R, XG, TW>::LDN;
    if (!XG) return ((const lds_f32 *)w.Xs)[j * LDN + idx];
    if (R * TW >= 32) {
        if (j < w.nlds) return ((const lds_f32 *)w.Xs)[j * LDN + idx];
        return ((const glb_f32 *)w.Xg)[(j - w.nlds) * LDN + idx];
    }
    return xaddr(w, j)[idx];
}

template <int R, bool XG, int TW>
LADL_INL void xput(Wave<R, XG, TW> &w, int j, int idx, float v)
{
    constexpr int LDN = Wave<R, XG, TW>::LDN;
    if (!XG || j < w.nlds)
        ((lds_f32 *)w.Xs)[j * LDN + idx] = v;
    else
        ((glb_f32 *)w.Xg)[(j - w.nlds) * LDN + idx] = v;
}

template <int R, bool XG, int TW>
LADL_INL void xcol_lds(const Wave<R, XG, TW> &w, int j, float (&x)[R])
{
    constexpr int LDN = Wave<R, XG, TW>::LDN, RT = Wave<R, XG, TW>::RT;
    const lds_f32 *c = (const lds_f32 *)w.Xs + j * LDN + w.rb;
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = c[RT * k];
}

template <int R, bool XG, int TW>
LADL_INL void xcol_ws(const Wave<R, XG, TW> &w, int j, float (&x)[R])
{
    constexpr int LDN = Wave<R, XG, TW>::LDN, RT = Wave<R, XG, TW>::RT;
    const glb_f32 *c = (const glb_f32 *)w.Xg + (j - w.nlds) * LDN + w.rb;
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = c[RT * k];
}

// --------------------------------------------------------------------------
// problem load: X row-major in HBM -> column-major in LDS (coalesced reads)
// --------------------------------------------------------------------------
template <int R, bool XG, int TW>
LADL_INL bool load_problem(Wave<R, XG, TW> &w, const float *__restrict__ X, const float *__restrict__ y)
{
    // rows n .. RT R - 1 are zero padding (so hot loops read all R slots
    // without guards: a zero row has a zero residual and no weight)
    constexpr int RT = Wave<R, XG, TW>::RT;
    const int l = lane_id(), tl = w.rb, n = w.n, p = w.p, top = RT * R;
    for (int j = 0; j < p; ++j)
        for (int i = n + tl; i < top; i += RT) xput(w, j, i, 0.f);
    for (int i = n + tl; i < top; i += RT) w.ys[i] = 0.f;
    bool finite = true;
    const int np = n * p;
    const float invp = 1.0f / (float)p;
    for (int e = tl; e < np; e += RT) {
        float v = X[e];
        int i = (int)((float)e * invp);
        if (i * p > e)
            --i;
        else if ((i + 1) * p <= e)
            ++i;
        xput(w, e - i * p, i, v);
        finite = finite && __builtin_isfinite(v);
    }
    for (int i = tl; i < n; i += RT) {
        float v = y[i];
        w.ys[i] = v;
        finite = finite && __builtin_isfinite(v);
    }
    ws_sync<XG>();
    float mine = 0.f;
    for (int j = 0; j < p; ++j) {
        float part = 0.f;
        for (int i = tl; i < n; i += RT) part += fabsf(xget(w, j, i));
        const float sj = wsum(part);
        mine = (l == j) ? sj : mine;
    }
    const float cs = (TW == 1) ? mine : (float)tsum_vec_d(w.tm, (double)mine);
    w.cav = (l < p) ? cs : 0.f;
    if (l < p) w.vca[l] = cs;
    float yp = 0.f;
    for (int i = tl; i < n; i += RT) yp += fabsf(w.ys[i]);
    w.ynorm1 = tsum(w.tm, yp);
    __syncthreads();
    return tcount(w.tm, !finite) == 0;
}

// r = y - X b, b held one coefficient per lane (lane j: b_j)
template <int R, bool XG, int TW>
LADL_INL void residuals(Wave<R, XG, TW> &w, float (&r)[R], float bv)
{
#pragma unroll
    for (int k = 0; k < R; ++k) r[k] = (k < w.nslot) ? w.ys[row_of(w, k)] : 0.f;
    for (int j = 0; j < w.p; ++j) {
        float bj = rdlane(bv, j);
        if (bj != 0.f) {
#pragma unroll
            for (int k = 0; k < R; ++k)
                if (k < w.nslot) r[k] = fmaf(-xget(w, j, row_of(w, k)), bj, r[k]);
        }
    }
}

// f = sum |r_i| + lambda sum |b_j|, b one coefficient per lane (the
// penalty counted by the first wave of the team only)
template <int R, bool XG, int TW>
LADL_INL float objective(Wave<R, XG, TW> &w, const float (&r)[R], float bval)
{
    const int l = lane_id();
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < R; ++k) s += fabsf(r[k]);
    float sb = (w.wv == 0 && l < w.p) ? fabsf(bval) : 0.f;
    tsum2(w.tm, s, sb);
    return s + w.lam * sb;
}

// --------------------------------------------------------------------------
// Weighted selection over the team.
// Candidates: per-lane register keys a[k] (FINF = none) with weights
// |x[k]| (zero for FINF keys), plus one extra key (av, wv) per lane (the
// callers place extra keys in the first wave only).  All keys are >= 0.
// Returns the smallest key a* whose cumulative weight (over keys <= a*)
// reaches T (strict: exceeds T), and which wave, register slot or extra
// key holds it (row keys win ties against extra keys; lower waves, then
// lower lanes, then lower slots first).
// --------------------------------------------------------------------------
struct Sel {
    float a;
    int wave, lane, slot;
    bool virt;
};

template <int R, bool XG, int TW>
LADL_INL Sel owner_of(Wave<R, XG, TW> &w, const float (&a)[R], float av, float m)
{
    int myslot = -1;
#pragma unroll
    for (int k = R - 1; k >= 0; --k)
        if (a[k] == m) myslot = k;
    const uint64_t rbal = ballot(myslot >= 0);
    const uint64_t vbal = ballot(av == m);
    const int rl = rbal ? first_lane(rbal) : -1;
    const int rs = rbal ? rdlane(myslot, rl) : -1;
    const int vl = vbal ? first_lane(vbal) : -1;
    Sel s;
    s.a = m;
    if constexpr (TW == 1) {
        s.wave = 0;
        if (rbal) {
            s.lane = rl;
            s.slot = rs;
            s.virt = false;
        } else {
            s.lane = vbal ? vl : 0;
            s.slot = -1;
            s.virt = true;
        }
    } else {
        int *sl = (int *)team_slot(w.tm);
        if (lane_id() == 0) {
            sl[8 * w.wv] = rl;
            sl[8 * w.wv + 1] = rs;
            sl[8 * w.wv + 2] = vl;
        }
        __syncthreads();
        int fw = -1, fv = -1;
#pragma unroll
        for (int q = TW - 1; q >= 0; --q) {
            if (sl[8 * q] >= 0) fw = q;
            if (sl[8 * q + 2] >= 0) fv = q;
        }
        fw = uni(fw);
        fv = uni(fv);
        if (fw >= 0) {
            s.wave = fw;
            s.lane = uni(sl[8 * fw]);
            s.slot = uni(sl[8 * fw + 1]);
            s.virt = false;
        } else {
            s.wave = fv >= 0 ? fv : 0;
            s.lane = fv >= 0 ? uni(sl[8 * fv + 2]) : 0;
            s.slot = -1;
            s.virt = true;
        }
    }
    return s;
}

// number of this wave's keys in (lo, hi], summed over the team
template <int R, int TW>
LADL_INL int tcount_range(Team<TW> &t, const float (&a)[R], float av, float lo, float hi)
{
    int c = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) c += popc64(ballot(a[k] > lo && a[k] <= hi));
    c += popc64(ballot(av > lo && av <= hi));
    if constexpr (TW == 1) {
        return c;
    } else {
        int *sl = (int *)team_slot(t);
        if (lane_id() == 0) sl[t.wv] = c;
        __syncthreads();
        int s = 0;
#pragma unroll
        for (int q = 0; q < TW; ++q) s += sl[q];
        return uni(s);
    }
}

template <int R, bool XG, int TW>
LADL_INL Sel wselect(Wave<R, XG, TW> &w, const float (&a)[R], const float (&x)[R], float av, float wv, float T,
                     bool strict, float lo0, float cum0)
{
    // weights are recomputed where used rather than held in R more registers
    auto wt = [&](int k) { return (a[k] < FINF) ? fabsf(x[k]) : 0.f; };
    const int l = lane_id();
    float lo = lo0, hi = FINF, cum = cum0;
    auto reached = [&](float c) { return strict ? (c > T) : (c >= T); };
    // Phase A: the next distinct keys one at a time (short moves)
    for (int it = 0; it < 3; ++it) {
        float m = FINF;
#pragma unroll
        for (int k = 0; k < R; ++k) m = fminf(m, (a[k] > lo) ? a[k] : FINF);
        m = fminf(m, (av > lo) ? av : FINF);
        m = tmin_nn(w.tm, m);
        if (m == FINF) {
            if (lo < 0.f) return Sel{FINF, 0, 0, -1, false}; // no candidate at all
            return owner_of(w, a, av, lo);                  // weight exhausted by rounding
        }
        // keys equal to the finite m are real kinks: their weight is |x|
        float wm = 0.f;
#pragma unroll
        for (int k = 0; k < R; ++k) wm += (a[k] == m) ? fabsf(x[k]) : 0.f;
        wm += (av == m) ? wv : 0.f;
        wm = tsum(w.tm, wm);
        if (reached(cum + wm)) return owner_of(w, a, av, m);
        cum += wm;
        lo = m;
    }
    // Phase B: narrow (lo, hi] around the target with sampled quantiles
    int cnt = 0;
    for (int round = 0; round < 12; ++round) {
        cnt = tcount_range<R, TW>(w.tm, a, av, lo, hi);
        if (cnt <= 64) break;
        float smp = FINF, wint = 0.f;
#pragma unroll
        for (int k = R - 1; k >= 0; --k) {
            bool in = a[k] > lo && a[k] <= hi;
            smp = in ? a[k] : smp;
            wint += in ? wt(k) : 0.f;
        }
        if (av > lo && av <= hi) {
            smp = (smp == FINF) ? av : smp;
            wint += wv;
        }
        wint = tsum(w.tm, wint);
        if constexpr (TW > 1) {
            // the same 64 samples on every wave: lane l takes wave (l mod TW)'s
            w.smp[64 * w.wv + l] = smp;
            __syncthreads();
            smp = w.smp[64 * (l % TW) + l];
        }
        int ns = popc64(ballot(smp < FINF));
        bitonic64(smp);
        float frac = (T - cum) / wint;
        frac = fminf(fmaxf(frac, 0.f), 1.f);
        int rk = (int)(frac * (float)ns);
        int r1 = max(0, min(ns - 1, rk - 4)), r2 = max(0, min(ns - 1, rk + 4));
        float p1 = rdlane(smp, r1), p2 = rdlane(smp, r2);
        float c1 = 0.f, c2 = 0.f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            bool in = a[k] > lo && a[k] <= hi;
            c1 += (in && a[k] <= p1) ? wt(k) : 0.f;
            c2 += (in && a[k] <= p2) ? wt(k) : 0.f;
        }
        if (av > lo && av <= hi) {
            c1 += (av <= p1) ? wv : 0.f;
            c2 += (av <= p2) ? wv : 0.f;
        }
        float z = 0.f;
        tsum3(w.tm, c1, c2, z);
        if (reached(cum + c1)) {
            hi = p1;
        } else if (reached(cum + c2)) {
            cum += c1;
            lo = p1;
            hi = p2;
        } else {
            cum += c2;
            lo = p2;
        }
    }
    if (cnt > 64) {
        // many equal keys: step through distinct values
        for (int guard = 0; guard < 4096; ++guard) {
            float m = FINF;
#pragma unroll
            for (int k = 0; k < R; ++k)
                if (a[k] > lo && a[k] <= hi) m = fminf(m, a[k]);
            if (av > lo && av <= hi) m = fminf(m, av);
            m = tmin(w.tm, m);
            if (m == FINF) break;
            float wm = 0.f;
#pragma unroll
            for (int k = 0; k < R; ++k) wm += (a[k] == m) ? wt(k) : 0.f;
            wm += (av == m) ? wv : 0.f;
            wm = tsum(w.tm, wm);
            if (reached(cum + wm) || m == hi) return owner_of(w, a, av, m);
            cum += wm;
            lo = m;
        }
        return owner_of(w, a, av, hi);
    }
    // Phase C: compact the <= 64 keys of (lo, hi] (in team row order), sort,
    // scan
    int base = 0;
    if constexpr (TW > 1) {
        // this wave's first position: the counts of the waves before it
        int c = 0;
#pragma unroll
        for (int k = 0; k < R; ++k) c += popc64(ballot(a[k] > lo && a[k] <= hi));
        c += popc64(ballot(av > lo && av <= hi));
        int *sl = (int *)team_slot(w.tm);
        if (l == 0) sl[w.wv] = c;
        __syncthreads();
        for (int q = 0; q < w.wv; ++q) base += sl[q];
        base = uni(base);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        bool in = a[k] > lo && a[k] <= hi;
        uint64_t bal = ballot(in);
        if (in) {
            int pos = base + mbcnt(bal);
            w.sa[pos] = a[k];
            w.sw[pos] = wt(k);
        }
        base += popc64(bal);
    }
    {
        bool in = av > lo && av <= hi;
        uint64_t bal = ballot(in);
        if (in) {
            int pos = base + mbcnt(bal);
            w.sa[pos] = av;
            w.sw[pos] = wv;
        }
        base += popc64(bal);
    }
    __syncthreads();
    const int total = cnt;
    float key = (l < total) ? w.sa[l] : FINF;
    float val = (l < total) ? w.sw[l] : 0.f;
    __syncthreads();
    bitonic64(key, val);
    float inc = wscan_incl(val);
    uint64_t ok = ballot(key < FINF && reached(cum + inc));
    float m;
    if (ok)
        m = rdlane(key, first_lane(ok));
    else if (total > 0)
        m = rdlane(key, total - 1); // rounding: take the last key
    else
        m = (hi < FINF) ? hi : lo;
    return owner_of(w, a, av, m);
}

// --------------------------------------------------------------------------
// H4: exact minimisation of f along axis j: the lower weighted median of the
// kinks t_i = b_j + r_i/x_ij (weight |x_ij|) and 0 (weight lambda).
// One pass over the rows classifies every kink against the current b_j by
// signs alone (below: r_i x_ij < 0, at: r_i = 0) and records, per lane, the
// nearest kink on each side with its weight.  After the two weight sums the
// direction is known; most moves reach only the nearest kink, decided by
// one wave (team) minimum.  Longer moves continue in wselect.
// --------------------------------------------------------------------------
template <int R, bool XG, int TW>
LADL_INL bool coord_update(Wave<R, XG, TW> &w, float (&r)[R], float &bv, int j, const float (&x)[R])
{
    const int l = lane_id();
    // pass 1: weight of the kinks below and at the current b_j (signs only)
    float bel = 0.f, at = 0.f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const float rr = r[k], ax = fabsf(x[k]);
        // r_i x_ij < 0: the kink lies below b_j (a zero residual gives a
        // zero product: that kink is at b_j)
        const bool neg = rr * x[k] < 0.f;
        at += (rr == 0.f) ? ax : 0.f;
        bel += neg ? ax : 0.f;
    }
    const float bj = rdlane(bv, j);
    tsum2(w.tm, bel, at);
    const float lam = w.lam;
    const float W = rdlane(w.cav, j) + lam;
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
        return false; // b_j is already the minimiser
    const float T = down ? (belT - half) : (half - belT - atT);
    auto reached = [&](float c) { return down ? (c > T) : (c >= T); };
    // pass 2: the kinks on the moving side, as distances from b_j, and each
    // lane's nearest one with the weight of all its kinks at that distance.
    // The kink of row i sits at b_j + r_i/x_ij; with the sign flipped when
    // moving down, it lies on the moving side iff the flipped offset is > 0
    // (r_i = 0 gives 0: that kink is at b_j, already weighed; x_ij = 0 gives
    // an infinite offset or NaN: no kink).  The distance |r_i| rcp(|x_ij|)
    // is the same float either way.
    const int flip = down ? (int)0x80000000 : 0;
    float a[R];
    float smin = FINF, sw = 0.f;
    int sk = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const float ax = fabsf(x[k]);
        const float off = bitsf(fbits(r[k] * __builtin_amdgcn_rcpf(x[k])) ^ flip);
        const float ak = (off > 0.f) ? off : FINF;
        a[k] = ak;
        const bool lt = ak < smin, eq = ak == smin;
        sw = lt ? ax : (eq ? sw + ax : sw);
        sk = lt ? k : sk;
        smin = lt ? ak : smin;
    }
    const bool lcand = (lam > 0.f) && (down ? (bj > 0.f) : (bj < 0.f));
    const float al = fabsf(bj);
    float m1, mm, wm;
    int owave = 0, olane = -1;
    if constexpr (TW == 1) {
        m1 = wmin_nn(smin);
        if (!(m1 < FINF) && !lcand) return false;
        mm = lcand ? fminf(m1, al) : m1;
        // weight of the nearest kink(s)
        const uint64_t ob = ballot(smin == mm);
        wm = (popc64(ob) > 1) ? wsum((smin == mm) ? sw : 0.f) : (ob ? rdlane(sw, first_lane(ob)) : 0.f);
        olane = ob ? first_lane(ob) : -1;
    } else {
        // each wave's nearest kink, its weight and first holder, combined in
        // one exchange
        const float mloc = wmin_nn(smin);
        const uint64_t ob = (mloc < FINF) ? ballot(smin == mloc) : 0;
        const float wl = (mloc < FINF) ? wsum((smin == mloc) ? sw : 0.f) : 0.f;
        const int fl = ob ? first_lane(ob) : -1;
        float *sl = team_slot(w.tm);
        if (l == 0) {
            sl[8 * w.wv] = mloc;
            sl[8 * w.wv + 1] = wl;
            ((int *)sl)[8 * w.wv + 2] = fl;
        }
        __syncthreads();
        m1 = sl[0];
#pragma unroll
        for (int q = 1; q < TW; ++q) m1 = fminf(m1, sl[8 * q]);
        m1 = unif(m1);
        if (!(m1 < FINF) && !lcand) return false;
        mm = lcand ? fminf(m1, al) : m1;
        wm = 0.f;
        int fw = -1;
#pragma unroll
        for (int q = TW - 1; q >= 0; --q)
            if (sl[8 * q] == mm) fw = q;
#pragma unroll
        for (int q = 0; q < TW; ++q) wm += (sl[8 * q] == mm) ? sl[8 * q + 1] : 0.f;
        wm = unif(wm);
        fw = uni(fw);
        owave = fw >= 0 ? fw : 0;
        olane = fw >= 0 ? uni(((int *)sl)[8 * fw + 2]) : -1;
    }
    if (lcand && al == mm) wm += lam;
    float nb;
    int oslot = -1;
    bool virt;
    if (reached(wm)) {
        virt = (olane < 0);
        if (!virt && w.wv == owave) oslot = rdlane(sk, olane);
        nb = virt ? 0.f : (down ? bj - mm : bj + mm);
    } else {
        const float av = (w.wv == 0 && l == 0 && lcand) ? al : FINF;
        const float wv = (w.wv == 0 && l == 0 && lcand) ? lam : 0.f;
        Sel sl = wselect(w, a, x, av, wv, T, down, mm, wm);
        if (!(sl.a < FINF)) return false;
        virt = sl.virt;
        owave = sl.wave;
        olane = sl.lane;
        oslot = sl.slot;
        nb = virt ? 0.f : (down ? bj - sl.a : bj + sl.a);
    }
    const float d = nb - bj;
    if (d == 0.f || !__builtin_isfinite(d)) return false;
#pragma unroll
    for (int k = 0; k < R; ++k) r[k] = fmaf(-x[k], d, r[k]);
    // the median row is now on its hyperplane: its residual is exactly zero
    // (one register slot of one lane, the slot index uniform)
    if (!virt && w.wv == owave) {
        const int os = uni(oslot);
        r[os] = (l == olane) ? 0.f : r[os];
    }
    bv = (l == j) ? nb : bv;
    return true;
}

// H4, quadrature variant (the paper's second coordinate-descent algorithm,
// Sections 1, 3.5 and 5): the section g(t) = sum_i |r_i - x_ij (t - b_j)| +
// lambda |t| is minimised from its values alone, with no ordering or
// selection of its kinks.  The bracket [smallest kink, largest kink] (and 0
// when lambda > 0) holds a minimiser; each step evaluates g at the two new
// quarter points of the bracket and keeps the half centred on the lowest of
// its three quarter points, so two sums over the rows per halving.  The
// point reached replaces b_j only if it lowers f.
// --------------------------------------------------------------------------
template <int R, bool XG, int TW>
LADL_INL bool coord_update_quad(Wave<R, XG, TW> &w, float (&r)[R], float &bv, int j, const float (&x)[R])
{
    const int ns = w.nslot;
    const float bj = rdlane(bv, j);
    const float lam = w.lam;
    float lo = FINF, hi = -FINF;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (k >= ns) break;
        if (x[k] != 0.f) {
            const float t = fmaf(r[k], __builtin_amdgcn_rcpf(x[k]), bj);
            lo = fminf(lo, t);
            hi = fmaxf(hi, t);
        }
    }
    lo = tmin(w.tm, lo);
    hi = tmax(w.tm, hi);
    if (lam > 0.f) {
        lo = fminf(lo, 0.f);
        hi = fmaxf(hi, 0.f);
    }
    if (!(lo <= hi)) return false;
    float mid = 0.5f * (lo + hi);
    float g0 = 0.f, gm = 0.f;
    {
        const float dm = mid - bj;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k >= ns) break;
            g0 += fabsf(r[k]);
            gm += fabsf(fmaf(-x[k], dm, r[k]));
        }
    }
    tsum2(w.tm, g0, gm);
    g0 += lam * fabsf(bj);
    gm += lam * fabsf(mid);
    for (int it = 0; it < QUAD_MAX; ++it) {
        if (hi - lo <= QUAD_TOL * (1.f + fabsf(lo) + fabsf(hi))) break;
        const float q1 = 0.5f * (lo + mid), q3 = 0.5f * (mid + hi);
        if (!(q1 > lo && q1 < mid && q3 > mid && q3 < hi)) break;
        const float d1 = q1 - bj, d3 = q3 - bj;
        float g1 = 0.f, g3 = 0.f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k >= ns) break;
            g1 += fabsf(fmaf(-x[k], d1, r[k]));
            g3 += fabsf(fmaf(-x[k], d3, r[k]));
        }
        tsum2(w.tm, g1, g3);
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
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if (k >= ns) break;
        r[k] = fmaf(-x[k], d, r[k]);
    }
    bv = (lane_id() == j) ? mid : bv;
    return true;
}

// H5: cyclic sweeps, axis `frozen` held fixed; Q selects the quadrature
// search for the 1-D sections (a kernel variant of its own, so that the
// exact-median kernels keep their register allocation)
template <bool Q, int R, bool XG, int TW>
LADL_INL float ccd(Wave<R, XG, TW> &w, float (&r)[R], float &bv, int frozen, float f)
{
    const int p = w.p;
    if (p == 1 && frozen == 0) return f;
    // The next column's values are loaded while this one is updated.  With
    // the workspace only its columns are prefetched, into registers that no
    // LDS load writes (a shared destination would make the compiler wait
    // for the prefetch before each update); LDS columns are read when due.
    const int j = (frozen == 0) ? 1 : 0;
    float x[R], xn[R];
    if (!XG)
        xcol_lds(w, j, x);
    else if (j >= w.nlds)
        xcol_ws(w, j, xn);
    for (int sw = 0; sw < w.opt.max_sweeps; ++sw) {
        bool changed = false;
        for (int u = 0; u < p; ++u) {
            if (u == frozen) continue;
            int jn = u + 1;
            if (jn == frozen) ++jn;
            if (jn >= p) jn = (frozen == 0) ? 1 : 0;
            if (!XG) {
                float xp[R];
                xcol_lds(w, jn, xp);
                changed |= Q ? coord_update_quad(w, r, bv, u, x) : coord_update(w, r, bv, u, x);
#pragma unroll
                for (int k = 0; k < R; ++k) x[k] = xp[k];
            } else {
                float xc[R];
                if (u < w.nlds) {
                    xcol_lds(w, u, xc);
                } else {
#pragma unroll
                    for (int k = 0; k < R; ++k) xc[k] = xn[k];
                }
                if (jn >= w.nlds) xcol_ws(w, jn, xn);
                changed |= Q ? coord_update_quad(w, r, bv, u, xc) : coord_update(w, r, bv, u, xc);
            }
            w.c_updates++;
        }
        w.c_sweeps++;
        float fn = objective(w, r, bv);
        bool stop = !changed || (f - fn <= w.opt.tol_f * fn);
        f = fn;
        if (stop) break;
    }
    return f;
}

// --------------------------------------------------------------------------
// H7: vertices, LU in LDS, certificate, finisher
// --------------------------------------------------------------------------

// ||x_i||_2 of the lane's rows (0 for padding rows)
template <int R, bool XG, int TW>
LADL_INL void row_norms(const Wave<R, XG, TW> &w, float (&nr)[R])
{
#pragma unroll
    for (int k = 0; k < R; ++k) nr[k] = 0.f;
    for (int j = 0; j < w.p; ++j) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const float x = xget(w, j, row_of(w, k));
            nr[k] = fmaf(x, x, nr[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) nr[k] = sqrtf(nr[k]);
}

// The vertex nearest to the point (vb, r): of the hyperplanes
// {x_i.b = y_i} and {b_j = 0}, take p that meet in one point, nearest first
// (rows |r_i|/||x_i||, axes |b_j|; ties: axes first, then lower row).  A
// hyperplane whose normal depends linearly on those already taken (a
// duplicated row, say) is passed over (modified Gram-Schmidt, basis kept in
// the A area of LDS).  Writes zs/ss and the per-lane Z bits; returns |S|
// (= |Z|) or -1.
template <int R, bool XG, int TW>
LADL_INL int choose_vertex(Wave<R, XG, TW> &w, const float (&r)[R], float bv, uint32_t &zbits)
{
    const int l = lane_id(), p = w.p;
    float dist[R];
    row_norms(w, dist);
#pragma unroll
    for (int k = 0; k < R; ++k) dist[k] = (dist[k] > 0.f) ? fabsf(r[k]) / dist[k] : FINF;
    const float dv = (l < p) ? fabsf(bv) : FINF;
    float *Q = w.A;
    zbits = 0;
    uint32_t seen = 0;
    bool cseen = false, ctaken = false;
    int acc = 0, nz = 0;
    for (int guard = 0; guard < w.n + p && acc < p; ++guard) {
        float mr = FINF;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (!((seen >> k) & 1u)) mr = fminf(mr, dist[k]);
        const float m = tmin(w.tm, fminf(mr, cseen ? FINF : dv));
        if (m == FINF) break;
        const uint64_t cb = ballot(!cseen && l < p && dv == m);
        int row = -1, col = -1;
        if (cb) {
            col = first_lane(cb);
            if (l == col) cseen = true;
        } else {
            int best = INT_MAX;
#pragma unroll
            for (int k = R - 1; k >= 0; --k)
                if (!((seen >> k) & 1u) && dist[k] == m) best = row_of(w, k);
            row = tmin_i(w.tm, best);
            if (w.wv == row_wave(row, TW) && l == (row & 63)) seen |= 1u << row_slot(row, TW);
        }
        float v = 0.f;
        if (l < p) v = (col >= 0) ? ((l == col) ? 1.f : 0.f) : xget(w, l, row);
        const float n0 = sqrtf(wsum(v * v));
        for (int a2 = 0; a2 < acc; ++a2) {
            const float qa = (l < p) ? Q[a2 * ALD + l] : 0.f;
            const float dd = wsum(v * qa);
            v = fmaf(-dd, qa, v);
        }
        const float nv = sqrtf(wsum(v * v));
        if (!(nv > 1e-4f * n0)) continue; // dependent on the normals taken
        if (l < p) Q[acc * ALD + l] = v / nv;
        __syncthreads();
        ++acc;
        if (col >= 0) {
            if (l == col) ctaken = true;
        } else {
            if (w.wv == row_wave(row, TW) && l == (row & 63)) zbits |= 1u << row_slot(row, TW);
            if (l == 0) w.zs[nz] = row;
            ++nz;
        }
    }
    const uint64_t sb = ballot(l < p && !ctaken);
    const int s = popc64(sb);
    if (l < p && !ctaken) w.ss[mbcnt(sb)] = l;
    __syncthreads();
    return (acc == p && s == nz) ? s : -1;
}

LADL_INL bool lu_factor(float *A, int *piv, int s)
{
    const int l = lane_id();
    float m = 0.f;
    if (l < s)
        for (int c = 0; c < s; ++c) m = fmaxf(m, fabsf(A[l * ALD + c]));
    const float amax = wmax(m);
    for (int k = 0; k < s; ++k) {
        float v = (l >= k && l < s) ? fabsf(A[l * ALD + k]) : -1.f;
        float vm = wmax(v);
        if (!(vm > 1e-7f * amax)) return false;
        int pr = first_lane(ballot(v == vm));
        if (l == 0) piv[k] = pr;
        if (pr != k && l < s) {
            float t = A[k * ALD + l];
            A[k * ALD + l] = A[pr * ALD + l];
            A[pr * ALD + l] = t;
        }
        __syncthreads();
        const float pk = unif(A[k * ALD + k]);
        if (l > k && l < s) {
            float lf = A[l * ALD + k] / pk;
            A[l * ALD + k] = lf;
            for (int c = k + 1; c < s; ++c) A[l * ALD + c] = fmaf(-lf, A[k * ALD + c], A[l * ALD + c]);
        }
        __syncthreads();
    }
    return true;
}

// A x = v, v and x one element per lane (lane q < s)
LADL_INL float lu_solve(const float *A, const int *piv, int s, float v)
{
    const int l = lane_id();
    const int pr = (l < s) ? piv[l] : 0; // lane k: row swapped with k
    for (int k = 0; k < s; ++k) {
        int pk = rdlane(pr, k);
        if (pk != k) {
            float a = rdlane(v, k), b = rdlane(v, pk);
            v = (l == k) ? b : ((l == pk) ? a : v);
        }
    }
    for (int c = 0; c < s; ++c) {
        float vc = rdlane(v, c);
        if (l > c && l < s) v = fmaf(-A[l * ALD + c], vc, v);
    }
    for (int c = s - 1; c >= 0; --c) {
        if (l == c) v = v / A[c * ALD + c];
        float vc = rdlane(v, c);
        if (l < c) v = fmaf(-A[l * ALD + c], vc, v);
    }
    return v;
}

// A^T x = v
LADL_INL float lu_solve_t(const float *A, const int *piv, int s, float v)
{
    const int l = lane_id();
    const int pr = (l < s) ? piv[l] : 0;
    for (int c = 0; c < s; ++c) {
        if (l == c) v = v / A[c * ALD + c];
        float vc = rdlane(v, c);
        if (l > c && l < s) v = fmaf(-A[c * ALD + l], vc, v);
    }
    for (int c = s - 1; c >= 0; --c) {
        float vc = rdlane(v, c);
        if (l < c) v = fmaf(-A[c * ALD + l], vc, v);
    }
    for (int k = s - 1; k >= 0; --k) {
        int pk = rdlane(pr, k);
        if (pk != k) {
            float a = rdlane(v, k), b = rdlane(v, pk);
            v = (l == k) ? b : ((l == pk) ? a : v);
        }
    }
    return v;
}

// Vertex (zs, ss, s): A = X_{Z,S} factored in LDS (A0 keeps it unfactored),
// b_S = A^{-1} y_Z refined to fp64 accuracy, b (rounded to fp32) into vt,
// the residuals of the fp64 vertex into rv (exact zeros on Z), objective
// into f (and in fp64 into w.fv64).
template <int R, bool XG, int TW>
LADL_INL bool vertex_eval(Wave<R, XG, TW> &w, float (&rv)[R], uint32_t zbits, int s, float &f)
{
    const int l = lane_id(), a0ld = w.a0ld;
    // lane q < s: row Z_q and column S_q, held in registers so that the
    // gathers below issue independent loads
    const int zl = (l < s) ? w.zs[l] : 0;
    const int jl = (l < s) ? w.ss[l] : 0;
    // lane c gathers column S_c: A[q][c] = x_{Z_q, S_c}, four rows at a time
    for (int q0 = 0; q0 < s; q0 += 4) {
        float v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int zq = rdlane(zl, q0 + t);
            v[t] = (l < s && q0 + t < s) ? xget(w, jl, zq) : 0.f;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (l < s && q0 + t < s) {
                w.A[(q0 + t) * ALD + l] = v[t];
                w.A0[(q0 + t) * a0ld + l] = v[t];
            }
    }
    __syncthreads();
    if (!lu_factor(w.A, w.piv, s)) return false;
    const float yz = (l < s) ? w.ys[zl] : 0.f;
    // b_S in fp64 by mixed-precision refinement: the fp32 LU applied to the
    // residual y_Z - X_{Z,S} b_S formed in fp64, the correction accumulated
    // in fp64, until it is at fp64 rounding level (each step gains a factor
    // of about cond(X_{Z,S}) * 2^-24).  The certificate reads the signs of
    // the other rows' residuals at this vertex; from an fp32-rounded b a row
    // 1e-6 (relative) from its hyperplane can show the wrong sign.
    double xd = (double)lu_solve(w.A, w.piv, s, yz);
    for (int it = 0; it < REFINE_MAX; ++it) {
        double acc = (double)yz;
        for (int c = 0; c < s; ++c) {
            const double xc = rdlane_d(xd, c);
            if (l < s) acc -= (double)w.A0[l * a0ld + c] * xc;
        }
        const float corr = lu_solve(w.A, w.piv, s, (l < s) ? (float)acc : 0.f);
        xd += (double)corr;
        if (wmax(fabsf(corr)) <= 1e-14f * wmax(fabsf((float)xd))) break;
    }
    const float xs = (float)xd;
    if (ballot(l < s && !__builtin_isfinite(xs))) return false;
    if (l < w.p) w.vt[l] = 0.f;
    __syncthreads();
    if (l < s) w.vt[jl] = xs;
    __syncthreads();
    // residuals in fp64 (stored as fp32): the certificate reads their signs,
    // and a row a few ulps of y from its hyperplane must keep its true sign
    double racc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) racc[k] = (double)w.ys[row_of(w, k)];
    for (int c = 0; c < s; ++c) {
        const int jc = rdlane(jl, c);
        const double bc = rdlane_d(xd, c);
#pragma unroll
        for (int k = 0; k < R; ++k) racc[k] = fma(-(double)xget(w, jc, row_of(w, k)), bc, racc[k]);
    }
    double s64 = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const bool z = (zbits >> k) & 1u;
        rv[k] = z ? 0.f : (float)racc[k];
        s64 += z ? 0.0 : fabs(racc[k]);
    }
    const float bl = (l < w.p) ? w.vt[l] : 0.f;
    s64 += (w.wv == 0) ? (double)w.lam * fabs((double)bl) : 0.0;
    w.fv64 = tsum_d(w.tm, s64);
    f = objective(w, rv, bl);
    return true;
}

// LP optimality certificate at the evaluated vertex (A holds its LU, A0 the
// matrix): u_i = sign(r_i) off Z, X_{Z,S}^T u_Z = lambda sign(b_S) -
// X_{Zc,S}^T u_Zc, c = X^T u.  Lane q returns u_{Z_q} in u, lane j returns
// c_j in c.
template <int R, bool XG, int TW>
LADL_INL bool certificate(Wave<R, XG, TW> &w, const float (&rv)[R], uint32_t zbits, int s, float &u, float &c,
                          bool &unique)
{
    const int l = lane_id(), p = w.p, a0ld = w.a0ld;
    const int zl = (l < s) ? w.zs[l] : 0;
    const int jl = (l < s) ? w.ss[l] : 0;
    // g_j = sum_i x_ij sign(r_i) in fp64 (rows of Z have r = 0); lane j
    // keeps g_j
    double g = 0.0;
    for (int j = 0; j < p; ++j) {
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) part += (double)(xget(w, j, row_of(w, k)) * sgnf(rv[k]));
        const double gj = wsum_d(part);
        g = (l == j) ? gj : g;
    }
    g = tsum_vec_d(w.tm, g);
    if (l < p) w.gd[l] = g;
    __syncthreads();
    uint32_t smask = 0;
    for (int q = 0; q < s; ++q) smask |= 1u << rdlane(jl, q);
    double rhs = 0.0;
    if (l < s) rhs = (double)w.lam * (double)sgnf(w.vt[jl]) - w.gd[jl];
    u = lu_solve_t(w.A, w.piv, s, (float)rhs);
    // refinement: residual rhs - X_{Z,S}^T u in fp64, until the correction
    // is at rounding level (the certificate compares |u_i| with 1 to 2e-5)
    for (int it = 0; it < REFINE_MAX; ++it) {
        double acc = rhs;
        for (int q = 0; q < s; ++q) {
            const float uq = rdlane(u, q);
            if (l < s) acc -= (double)w.A0[q * a0ld + l] * (double)uq;
        }
        const float corr = lu_solve_t(w.A, w.piv, s, (l < s) ? (float)acc : 0.f);
        u += corr;
        if (wmax(fabsf(corr)) <= 1e-7f * fmaxf(1.f, wmax(fabsf(u)))) break;
    }
    double cj = g;
    float colz = 0.f; // lane j: sum_{i in Z} |x_ij|
    for (int q = 0; q < s; ++q) {
        const float uq = rdlane(u, q);
        const int zq = rdlane(zl, q);
        if (l < p) {
            const float xv = xget(w, l, zq);
            cj += (double)xv * (double)uq;
            colz += fabsf(xv);
        }
    }
    c = (float)cj;
    const bool offS = (l < p) && !((smask >> l) & 1u);
    const float umax = wmax((l < s) ? fabsf(u) : 0.f);
    const float cabs = fabsf(c);
    const float colabs = (l < p) ? w.vca[l] : 0.f;
    const bool viol = offS && (cabs > w.lam * (1.f + TOL_C) + TOL_CA * colabs);
    const bool cert = (umax <= 1.f + TOL_U) && (ballot(viol) == 0);
    const float mc = wmin(offS ? (w.lam - cabs) / (w.lam + colz) : FINF);
    // rows off Z: |r_i| against |y_i| + sum_{j in S} |x_ij b_j|
    float sc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) sc[k] = fabsf(w.ys[row_of(w, k)]);
    for (int q = 0; q < s; ++q) {
        const int jc = rdlane(jl, q);
        const float bc = fabsf(w.vt[jc]);
#pragma unroll
        for (int k = 0; k < R; ++k) sc[k] = fmaf(fabsf(xget(w, jc, row_of(w, k))), bc, sc[k]);
    }
    float mr = FINF;
#pragma unroll
    for (int k = 0; k < R; ++k)
        if (!((zbits >> k) & 1u) && row_of(w, k) < w.n)
            mr = fminf(mr, (sc[k] > 0.f) ? fabsf(rv[k]) / sc[k] : fabsf(rv[k]));
    mr = tmin(w.tm, mr);
    unique = cert && (1.f - umax > MARGIN_U) && (mc > MARGIN_C) && (mr > MARGIN_R);
    return cert;
}

// the Z bits of this wave's rows for the vertex rows zs[0 .. s)
template <int R, bool XG, int TW>
LADL_INL uint32_t zbits_of(const Wave<R, XG, TW> &w, int s)
{
    const int l = lane_id();
    const int zn = (l < s) ? w.zs[l] : 0;
    uint32_t zb = 0;
    for (int q = 0; q < s; ++q) {
        const int zq = rdlane(zn, q);
        if (row_wave(zq, TW) == w.wv && (zq & 63) == l) zb |= 1u << row_slot(zq, TW);
    }
    return zb;
}

// Evaluate the vertex (zs, ss, s) and test its certificate; while it fails,
// take primal simplex steps along the vertex's edges (a build addition):
// release a violated constraint, move to the minimum of f along the edge
// (again a weighted median) and let the kink reached join the vertex.
// Returns the status; u (lane q) and c (lane j) hold the last dual values.
template <int R, bool XG, int TW>
LADL_INL int finisher(Wave<R, XG, TW> &w, float (&rv)[R], uint32_t &zbits, int &s, float &f, float &u, float &c,
                      bool &unique, int maxp)
{
    const int l = lane_id(), p = w.p;
    const float lam = w.lam;
    double fprev = __builtin_inf();
    int stalls = 0;
    for (int it = 0;; ++it) {
        if (!vertex_eval(w, rv, zbits, s, f)) return ST_NOTCERT;
        if (certificate(w, rv, zbits, s, u, c, unique)) return unique ? ST_CERTIFIED : ST_NONUNIQUE;
        if (it >= maxp) return ST_MAXITER;
        // The released constraint is the steepest violated one, except after
        // a step that did not lower f (compared in fp64: the fp32 values of
        // neighbouring vertices can tie), where it is the violated one of
        // lowest index (Bland's rule: rows of Z by row index, then axes);
        // after STALLS_STICKY such steps Bland's rule, which cannot cycle,
        // is kept for the rest of the finish.
        const bool stalled = !(w.fv64 < fprev - 1e-9 * fabs(fprev));
        stalls += stalled ? 1 : 0;
        const bool bland = stalled || stalls >= STALLS_STICKY;
        fprev = w.fv64;
        const int zl = (l < s) ? w.zs[l] : 0;
        const int jl = (l < s) ? w.ss[l] : 0;
        uint32_t smask = 0;
        for (int q = 0; q < s; ++q) smask |= 1u << rdlane(jl, q);
        const bool offS = (l < p) && !((smask >> l) & 1u);
        const float colabs = (l < p) ? w.vca[l] : 0.f;
        float vr = (l < s && 1.f - fabsf(u) < -TOL_U) ? 1.f - fabsf(u) : FINF;
        float vcl = (offS && fabsf(c) > lam * (1.f + TOL_C) + TOL_CA * colabs) ? lam - fabsf(c) : FINF;
        float m;
        bool type1;
        int sel;
        if (!bland) {
            m = wmin(fminf(vr, vcl));
            if (m == FINF) return ST_NOTCERT;
            const uint64_t rbal = ballot(vr == m);
            type1 = rbal != 0;
            sel = type1 ? first_lane(rbal) : first_lane(ballot(vcl == m));
        } else {
            const int kmin = wmin_i((vr < FINF) ? zl : INT_MAX);
            type1 = kmin != INT_MAX;
            if (type1) {
                sel = first_lane(ballot(vr < FINF && zl == kmin));
                m = rdlane(vr, sel);
            } else {
                const uint64_t cb = ballot(vcl < FINF);
                if (!cb) return ST_NOTCERT;
                sel = first_lane(cb);
                m = rdlane(vcl, sel);
            }
        }
        float rhs = 0.f, dj0 = 0.f, usel = 0.f;
        if (type1) {
            usel = rdlane(u, sel);
            rhs = (l == sel) ? -sgnf(usel) : 0.f;
        } else {
            dj0 = sgnf(rdlane(c, sel));
            rhs = (l < s) ? -xget(w, sel, zl) * dj0 : 0.f;
        }
        const float dS = lu_solve(w.A, w.piv, s, rhs);
        if (l < p) w.vd[l] = 0.f;
        __syncthreads();
        if (l < s) w.vd[jl] = dS;
        if (!type1 && l == 0) w.vd[sel] = dj0;
        __syncthreads();
        float xd[R];
#pragma unroll
        for (int k = 0; k < R; ++k) xd[k] = 0.f;
        for (int q = 0; q < s; ++q) {
            const int jc = rdlane(jl, q);
            const float dc = rdlane(dS, q);
#pragma unroll
            for (int k = 0; k < R; ++k) xd[k] = fmaf(xget(w, jc, row_of(w, k)), dc, xd[k]);
        }
        if (!type1) {
#pragma unroll
            for (int k = 0; k < R; ++k) xd[k] = fmaf(xget(w, sel, row_of(w, k)), dj0, xd[k]);
        }
        const int zsel = type1 ? rdlane(zl, sel) : -1;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if ((zbits >> k) & 1u) xd[k] = (row_of(w, k) == zsel) ? -sgnf(usel) : 0.f;
        // f(b + t d) = sum |r_i - t xd_i| + lam sum |b_j + t d_j|: kinks at
        // r_i/xd_i (weight |xd_i|) and -b_j/d_j (weight lam |d_j|).  Its
        // right slope at t = 0 is m (1 - |u_i0| or lam - |c_j0|, from the
        // fp64 dual sums), so the minimiser is the first kink t > 0 whose
        // cumulative weight reaches -m/2.
        const float dl = (l < p) ? w.vd[l] : 0.f;
        const float bl = (l < p) ? w.vt[l] : 0.f;
        const float need = -0.5f * m;
        if (!(need > 0.f)) return ST_NOTCERT;
        float a[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            bool pos = rv[k] != 0.f && xd[k] != 0.f && __builtin_signbit(rv[k]) == __builtin_signbit(xd[k]);
            a[k] = pos ? fabsf(rv[k]) / fabsf(xd[k]) : FINF; // weight |xd_i|
        }
        const bool vpos = (w.wv == 0) && (l < p) && lam > 0.f && dl != 0.f && bl != 0.f &&
                          __builtin_signbit(bl) != __builtin_signbit(dl);
        const float av = vpos ? fabsf(bl) / fabsf(dl) : FINF;
        const float wv = vpos ? lam * fabsf(dl) : 0.f;
        Sel sr = wselect(w, a, xd, av, wv, need, false, -1.f, 0.f);
        if (!(sr.a > 0.f) || sr.a == FINF) return ST_NOTCERT;
        const int srow = Wave<R, XG, TW>::RT * sr.slot + 64 * sr.wave + sr.lane; // row reached
        // new vertex
        if (type1) {
            if (!sr.virt) {
                if (l == 0) w.zs[sel] = srow;
            } else {
                if (l == 0) {
                    int c0 = -1;
                    for (int q = 0; q < s; ++q)
                        if (w.ss[q] == sr.lane) c0 = q;
                    for (int q = c0; q + 1 < s; ++q) w.ss[q] = w.ss[q + 1];
                    for (int q = sel; q + 1 < s; ++q) w.zs[q] = w.zs[q + 1];
                }
                s -= 1;
            }
        } else {
            if (!sr.virt) {
                if (s >= 32) return ST_NOTCERT;
                if (l == 0) {
                    w.zs[s] = srow;
                    w.ss[s] = sel;
                }
                s += 1;
            } else {
                if (sr.lane == sel) return ST_NOTCERT;
                if (l == 0)
                    for (int q = 0; q < s; ++q)
                        if (w.ss[q] == sr.lane) w.ss[q] = sel;
            }
        }
        __syncthreads();
        zbits = zbits_of(w, s);
        w.c_pivots++;
    }
    return ST_MAXITER;
}

// Degenerate vertices (more rows on their hyperplanes than active axes,
// e.g. duplicated rows) can make the edge steps cycle; a tiny deterministic
// perturbation of y separates such rows.
template <int R, bool XG, int TW>
LADL_INL void perturb_y(Wave<R, XG, TW> &w)
{
    const float ybar = w.ynorm1 / (float)w.n;
    for (int i = w.rb; i < w.n; i += Wave<R, XG, TW>::RT)
        w.ys[i] += PERTURB_REL * (fabsf(w.ys[i]) + ybar) * perturb_dir(i);
    ws_sync<XG>();
}

// y back from HBM (after a perturbation)
template <int R, bool XG, int TW>
LADL_INL void restore_y(Wave<R, XG, TW> &w, const float *yg)
{
    for (int i = w.rb; i < w.n; i += Wave<R, XG, TW>::RT) w.ys[i] = yg[i];
    ws_sync<XG>();
}

// objective of b (one coefficient per lane) recomputed with fp64 residuals
// and sums
template <int R, bool XG, int TW>
LADL_INL float objective64(Wave<R, XG, TW> &w, float bval)
{
    const int l = lane_id();
    double acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = (k < w.nslot) ? (double)w.ys[row_of(w, k)] : 0.0;
    for (int j = 0; j < w.p; ++j) {
        double bj = (double)rdlane(bval, j);
        if (bj != 0.0) {
#pragma unroll
            for (int k = 0; k < R; ++k)
                if (k < w.nslot) acc[k] -= (double)xget(w, j, row_of(w, k)) * bj;
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) s += fabs(acc[k]);
    s += (w.wv == 0 && l < w.p) ? (double)w.lam * fabs((double)bval) : 0.0;
    return (float)tsum_d(w.tm, s);
}

// --------------------------------------------------------------------------
// one solve (all its path steps)
// --------------------------------------------------------------------------
template <bool Q, int R, bool XG, int TW>
LADL_INL void solve_item(Wave<R, XG, TW> &w, const SolveArgs &a, int s)
{
    constexpr int RT = Wave<R, XG, TW>::RT;
    const int l = lane_id();
    const int k = a.problem ? a.problem[s] : s;
    const int64_t r0 = a.row_off[k];
    w.n = (int)(a.row_off[k + 1] - r0);
    w.p = a.p_arr[k];
    w.nslot = (w.n + RT - 1) / RT;
    const int p = w.p;
    const bool lead = (w.wv == 0); // the wave that writes the outputs
    const bool finite = load_problem(w, a.X + a.x_off[k], a.y + r0);
    const int64_t bbase = (int64_t)a.path_len * a.b_off[s];
    // starting point
    float b0 = 0.f;
    if (a.t0 > 0)
        b0 = (l < p) ? a.b_out[bbase + (int64_t)(a.t0 - 1) * p + l] : 0.f;
    else if (a.b_init)
        b0 = (l < p) ? a.b_init[a.b_off[s] + l] : 0.f;
    float bv = (l < p && __builtin_isfinite(b0)) ? b0 : 0.f; // lane j holds b_j
    // the chop's best point b lives in LDS (vbb, lane j < 32: b_j), like its
    // residuals (rbuf): a register copy would be live across every probe
    float r[R], rv[R];
    for (int t = a.t0; t < a.t1; ++t) {
        const int64_t o = (int64_t)s * a.path_len + t;
        float *bout = a.b_out + bbase + (int64_t)t * p;
        const float lam_in = a.lam[o];
        // the cold start seeded by the tile stage, which ran the chop already
        bool seeded = false;
        if constexpr (R == 1) {
            if (a.b_seed && t == 0) {
                const float b1 = (l < p) ? a.b_seed[bbase + l] : 0.f;
                bv = (l < p && __builtin_isfinite(b1)) ? b1 : 0.f;
                seeded = true;
            }
        }
        w.c_sweeps = w.c_updates = w.c_probes = w.c_pivots = 0;
        int status;
        float fout = 0.f;
        int zcount = -1; // vertex rows to report (-1: none)
        if (!finite || !(lam_in >= 0.f)) {
            status = finite ? ST_BADLAMBDA : ST_NONFINITE;
            bv = 0.f;
            fout = __builtin_nanf("");
        } else {
            w.lam = fmaxf(lam_in, w.opt.lambda_min);
            residuals(w, r, bv);
            float f = objective(w, r, bv);
            status = ST_NOTCERT;
            bool done = false, unique = false, have_vertex = false;
            uint32_t zbits = 0;
            int vs = -1;
            float u = 0.f, c = 0.f, fv = 0.f;
            const bool snap = !(w.opt.flags & FLAG_NO_SNAP);
            const int rounds = (p < 2 || seeded) ? 0 : ((w.opt.max_rounds < 0) ? p : w.opt.max_rounds);
            const float B = (w.lam > 0.f) ? w.ynorm1 / w.lam : FINF;
            static_assert(sizeof(Chop) <= 4 * CHOP_FLOATS, "chop state does not fit its LDS slot");
            Chop &q = *w.chop;
            int phase = 0; // 0: unrestricted CCD done, 1: a chop probe done
            int frozen = -1, round = 0, kax = 0;
            float fbest = FINF;
            for (;;) {
                f = ccd<Q>(w, r, bv, frozen, f); // the only CCD call site
                float sprobe = 0.f;
                bool more;
                if (phase == 0) {
                    if (snap) {
                        vs = choose_vertex(w, r, bv, zbits);
                        have_vertex = vs >= 0;
                        if (have_vertex) {
                            int st = finisher(w, rv, zbits, vs, fv, u, c, unique, 0);
                            if (st == ST_CERTIFIED || st == ST_NONUNIQUE) {
                                status = st;
                                done = true;
                                break;
                            }
                        }
                    }
                    if (round >= rounds) break;
                    if (round == 0) {
                        float bl = (l < p) ? fabsf(bv) : -1.f;
                        float bm = wmax(bl);
                        kax = first_lane(ballot(l < p && bl == bm));
                    } else {
                        kax = (kax + 1) % p;
                    }
                    ++round;
                    if (l < 32) w.vbb[l] = bv;
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) w.rbuf[64 * kk + l] = r[kk];
                    fbest = f;
                    chop_init(q, rdlane(bv, kax), f, B, w.opt.chop_range);
                    more = chop_next(q, 0.f, sprobe, w.opt);
                } else {
                    w.c_probes++;
                    if (f < fbest) {
                        fbest = f;
                        if (l < 32) w.vbb[l] = bv;
#pragma unroll
                        for (int kk = 0; kk < R; ++kk) w.rbuf[64 * kk + l] = r[kk];
                    }
                    more = chop_next(q, f, sprobe, w.opt);
                }
                // next CCD starts from the best point; a probe sets b_kax := s
                bv = (l < 32) ? w.vbb[l] : 0.f;
#pragma unroll
                for (int kk = 0; kk < R; ++kk) r[kk] = w.rbuf[64 * kk + l];
                if (more) {
                    const float d = sprobe - rdlane(bv, kax);
                    if (d != 0.f) {
#pragma unroll
                        for (int kk = 0; kk < R; ++kk) r[kk] = fmaf(-xget(w, kax, row_of(w, kk)), d, r[kk]);
                    }
                    bv = (l == kax) ? sprobe : bv;
                    f = objective(w, r, bv);
                    frozen = kax;
                    phase = 1;
                } else {
                    f = fbest;
                    frozen = -1;
                    phase = 0;
                }
            }
            if (!done && snap && have_vertex && !(w.opt.flags & FLAG_NO_FINISHER)) {
                const int maxp = (w.opt.max_pivots > 0) ? w.opt.max_pivots : 4 * p + 32;
                bool perturbed = false;
                for (int attempt = 0; attempt < 2 && !done; ++attempt) {
                    if (attempt == 1) {
                        perturb_y(w);
                        perturbed = true;
                    }
                    status = finisher(w, rv, zbits, vs, fv, u, c, unique, maxp);
                    done = (status == ST_CERTIFIED || status == ST_NONUNIQUE);
                }
                if (done && perturbed) {
                    // The perturbed problem's dual vector (u_i = sign r_i off Z,
                    // u_Z) is feasible for the original problem, whose
                    // optimum is therefore >= y.u.  Take the same vertex with
                    // the original y and accept it if f - y.u is tiny.
                    float sg[R];
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) sg[kk] = sgnf(rv[kk]);
                    restore_y(w, a.y + r0);
                    double yu = 0.0;
#pragma unroll
                    for (int kk = 0; kk < R; ++kk)
                        if (kk < w.nslot) yu += (double)w.ys[row_of(w, kk)] * (double)sg[kk];
                    if (lead && l < vs) yu += (double)w.ys[w.zs[l]] * (double)u;
                    yu = tsum_d(w.tm, yu);
                    done = vertex_eval(w, rv, zbits, vs, fv);
                    if (done) {
                        float fo = objective64(w, (l < p) ? w.vt[l] : 0.f);
                        done = (double)fo - yu <= 2e-6 * fmax(1.0, (double)fo);
                    }
                    status = done ? ST_NONUNIQUE : ST_NOTCERT;
                } else if (perturbed) {
                    // failed even when perturbed: put y back for the next path step
                    restore_y(w, a.y + r0);
                }
            }
            if (done) {
                bv = (l < p) ? w.vt[l] : 0.f;
                zcount = vs;
            } else if (!snap) {
                status = ST_MAXITER;
            }
            if constexpr (R >= 32) {
                // the n > 1024 kernel sits at its register limit: reading
                // the vertex's fp64 objective below moved its spills into
                // the update loop (6% slower), so it re-evaluates f
                fout = objective64(w, bv);
            } else {
                // f at the certified vertex, summed in fp64 from its fp64
                // residuals when it was evaluated (b is that vertex rounded
                // to fp32, which moves f by about 1e-7 relative)
                fout = done ? (float)w.fv64 : objective64(w, bv);
            }
        }
        // outputs (first wave of the team)
        uint64_t act = ballot(l < p && bv != 0.f);
        if (lead) {
            if (l < p) bout[l] = bv;
            if (l == 0) {
                a.obj_out[o] = fout;
                a.active_out[o] = (uint32_t)act;
                a.status_out[o] = status;
                if (a.iters_out) {
                    a.iters_out[4 * o + 0] = w.c_sweeps;
                    a.iters_out[4 * o + 1] = w.c_updates;
                    a.iters_out[4 * o + 2] = w.c_probes;
                    a.iters_out[4 * o + 3] = w.c_pivots;
                }
            }
            // Z rows in ascending order, -1 padded
            const bool zr = zcount > 0 && l < zcount;
            const int zl = zr ? w.zs[l] : INT_MAX;
            int rank = 0;
            for (int qq = 0; qq < zcount; ++qq) rank += (rdlane(zl, qq) < zl) ? 1 : 0;
            if (zr)
                a.zrows_out[(int64_t)ZPAD * o + rank] = zl;
            else if (l < ZPAD)
                a.zrows_out[(int64_t)ZPAD * o + l] = -1;
        }
        __syncthreads();
    }
}

// Register budget.  Left to the compiler, the R <= 4 kernels take 124-135
// VGPRs (3 waves per SIMD), most of it live only in the vertex and
// finisher code.  The DENSE variant asks for 4 waves per SIMD (128 VGPRs);
// the coordinate-update loop stays spill-free.  It only pays where the X
// workspace is in HBM (with all of X in LDS the LDS caps the waves first)
// and the bucket has solves enough to fill the extra waves.  Measured on
// c1 (n = 200, p = 8, 8192 solves): 4 waves per SIMD keep 5 of the 8
// columns in LDS and the rest in L2 (0.3 GB of HBM traffic per launch,
// 3.82 ms); 5 waves keep 3 columns in LDS, miss L2 (1.8 GB, 4.0 ms).  For
// R >= 8 the budget makes the update loop spill (the n <= 1024 bucket ran
// 1.5-2x slower), so it is not built.
// R = 32 left to the compiler takes 256 VGPRs plus 152 accumulation
// registers, one wave per SIMD; it is compiled for 2 waves per SIMD (256
// registers, some spilled to scratch), which lets the second wave hide the
// first one's latency: 6144 problems of n > 1024 on their 32-lambda paths
// take 0.90 instead of 1.21 s.  R = 8 (170 VGPRs, 2 waves) is compiled for
// 3 (168 VGPRs, no spill in the update loop): 6144 problems of n in
// (256, 512] 0.315 -> 0.301 s.  R = 16 at 3 waves spills in the update loop
// and ran 16% slower, so it keeps the compiler's 2.  The team kernels take
// the budget of their per-wave R.
constexpr int DENSE_WAVES_PER_SIMD = 4;
constexpr int R32_WAVES_PER_SIMD = 2;
constexpr int R8_WAVES_PER_SIMD = 3;
__host__ __device__ constexpr int waves_per_eu(int R, bool dense)
{
    return dense ? DENSE_WAVES_PER_SIMD : (R >= 32 ? R32_WAVES_PER_SIMD : (R == 8 ? R8_WAVES_PER_SIMD : 1));
}

template <int R, bool XG, bool DENSE, int TW, bool Q>
__global__ __launch_bounds__(64 * TW) __attribute__((amdgpu_waves_per_eu(waves_per_eu(R, DENSE))))
void k_wave(SolveArgs a)
{
    extern __shared__ float smem[];
    Wave<R, XG, TW> w;
    const int wv = (TW > 1) ? (int)(threadIdx.x >> 6) : 0;
    carve(w, smem, a.pmax, a.nlds, XG ? a.gws + (int64_t)blockIdx.x * a.gws_stride : nullptr, wv);
    w.opt = a.opt;
    const int l = lane_id();
    for (;;) {
        int q = 0;
        if constexpr (TW == 1) {
            if (l == 0) q = atomicAdd(a.counter, 1);
            q = rdlane(q, 0);
        } else {
            // the team's next solve, broadcast through LDS (the solve's own
            // barriers separate this read from the next write)
            if (wv == 0 && l == 0) w.qw[0] = atomicAdd(a.counter, 1);
            __syncthreads();
            q = uni(w.qw[0]);
        }
        if (q >= a.num_items) break;
        solve_item<Q>(w, a, a.order[q]);
    }
}

__global__ void k_reset(int32_t *c, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
}

size_t wave_lds_bytes(int R, int pmax, bool xg, int nlds, int tw)
{
    return 4 * wave_lds_floats(R, pmax, xg, nlds, tw) + 16;
}
size_t wave_ws_floats_host(int R, int pmax, int nlds, int tw) { return wave_ws_floats(R, pmax, nlds, tw); }

hipError_t launch_reset(int32_t *counters, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3((n + 63) / 64), dim3(64), 0, s, counters, n);
    return hipGetLastError();
}

template <int R, bool XG, bool DENSE, int TW, bool Q>
static hipError_t launch_wave_t(const SolveArgs &a, int grid, hipStream_t s)
{
    size_t lds = wave_lds_bytes(R, a.pmax, XG, a.nlds, TW);
    static bool attr = false;
    if (!attr) {
        // allow dynamic LDS beyond the default limit; harmless if refused
        (void)hipFuncSetAttribute((const void *)k_wave<R, XG, DENSE, TW, Q>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL((k_wave<R, XG, DENSE, TW, Q>), dim3(grid), dim3(64 * TW), lds, s, a);
    return hipGetLastError();
}

template <int R, bool XG, bool DENSE, int TW, bool Q>
static int max_blocks_t(int pmax, int nlds)
{
    int nb = 0;
    size_t lds = wave_lds_bytes(R, pmax, XG, nlds, TW);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_wave<R, XG, DENSE, TW, Q>, 64 * TW, lds) != hipSuccess)
        return 0;
    return nb;
}

bool wave_has_dense(int R) { return R == 1 || R == 2 || R == 4; }

// team sizes built for rows-per-lane bucket Rt (R = Rt / tw rows per lane
// of each wave): tw = 1 always; tw = 2, 4 for the n > 1024 bucket (Rt = 32)
bool wave_has_team(int Rt, int tw) { return tw == 1 || (Rt == 32 && (tw == 2 || tw == 4)); }

// the variants that exist: R in {1,2,4,8,16} with X in LDS or HBM, R = 32
// with X in HBM, the dense register budget for R <= 4 with X in HBM, and the
// teams of the n > 1024 bucket (2 x 16, 4 x 8 rows per lane) with X in HBM
template <bool Q>
static hipError_t launch_wave_q(int Rt, bool xg, bool dense, int tw, const SolveArgs &a, int grid, hipStream_t s)
{
    if (tw == 2 || tw == 4) {
        if (!xg || dense || Rt != 32) return hipErrorInvalidValue;
        return tw == 2 ? launch_wave_t<16, true, false, 2, Q>(a, grid, s) : launch_wave_t<8, true, false, 4, Q>(a, grid, s);
    }
    if (tw != 1) return hipErrorInvalidValue;
    if (dense) {
        if (!xg) return hipErrorInvalidValue;
        switch (Rt) {
        case 1: return launch_wave_t<1, true, true, 1, Q>(a, grid, s);
        case 2: return launch_wave_t<2, true, true, 1, Q>(a, grid, s);
        case 4: return launch_wave_t<4, true, true, 1, Q>(a, grid, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (xg) {
        switch (Rt) {
        case 1: return launch_wave_t<1, true, false, 1, Q>(a, grid, s);
        case 2: return launch_wave_t<2, true, false, 1, Q>(a, grid, s);
        case 4: return launch_wave_t<4, true, false, 1, Q>(a, grid, s);
        case 8: return launch_wave_t<8, true, false, 1, Q>(a, grid, s);
        case 16: return launch_wave_t<16, true, false, 1, Q>(a, grid, s);
        case 32: return launch_wave_t<32, true, false, 1, Q>(a, grid, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (Rt) {
    case 1: return launch_wave_t<1, false, false, 1, Q>(a, grid, s);
    case 2: return launch_wave_t<2, false, false, 1, Q>(a, grid, s);
    case 4: return launch_wave_t<4, false, false, 1, Q>(a, grid, s);
    case 8: return launch_wave_t<8, false, false, 1, Q>(a, grid, s);
    case 16: return launch_wave_t<16, false, false, 1, Q>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool Q>
static int max_blocks_q(int Rt, int pmax, bool xg, bool dense, int tw, int nlds)
{
    if (tw == 2 || tw == 4) {
        if (!xg || dense || Rt != 32) return 0;
        return tw == 2 ? max_blocks_t<16, true, false, 2, Q>(pmax, nlds) : max_blocks_t<8, true, false, 4, Q>(pmax, nlds);
    }
    if (tw != 1) return 0;
    if (dense) {
        if (!xg) return 0;
        switch (Rt) {
        case 1: return max_blocks_t<1, true, true, 1, Q>(pmax, nlds);
        case 2: return max_blocks_t<2, true, true, 1, Q>(pmax, nlds);
        case 4: return max_blocks_t<4, true, true, 1, Q>(pmax, nlds);
        default: return 0;
        }
    }
    if (xg) {
        switch (Rt) {
        case 1: return max_blocks_t<1, true, false, 1, Q>(pmax, nlds);
        case 2: return max_blocks_t<2, true, false, 1, Q>(pmax, nlds);
        case 4: return max_blocks_t<4, true, false, 1, Q>(pmax, nlds);
        case 8: return max_blocks_t<8, true, false, 1, Q>(pmax, nlds);
        case 16: return max_blocks_t<16, true, false, 1, Q>(pmax, nlds);
        case 32: return max_blocks_t<32, true, false, 1, Q>(pmax, nlds);
        default: return 0;
        }
    }
    switch (Rt) {
    case 1: return max_blocks_t<1, false, false, 1, Q>(pmax, nlds);
    case 2: return max_blocks_t<2, false, false, 1, Q>(pmax, nlds);
    case 4: return max_blocks_t<4, false, false, 1, Q>(pmax, nlds);
    case 8: return max_blocks_t<8, false, false, 1, Q>(pmax, nlds);
    case 16: return max_blocks_t<16, false, false, 1, Q>(pmax, nlds);
    default: return 0;
    }
}

hipError_t launch_wave(int Rt, bool xg, bool dense, int tw, bool quad, const SolveArgs &a, int grid, hipStream_t s)
{
    return quad ? launch_wave_q<true>(Rt, xg, dense, tw, a, grid, s) : launch_wave_q<false>(Rt, xg, dense, tw, a, grid, s);
}

int wave_max_blocks_per_cu(int Rt, int pmax, bool xg, bool dense, int tw, bool quad, int nlds)
{
    return quad ? max_blocks_q<true>(Rt, pmax, xg, dense, tw, nlds) : max_blocks_q<false>(Rt, pmax, xg, dense, tw, nlds);
}

// --------------------------------------------------------------------------
// H10: gradient through the optimal vertex.  At a certified vertex b_S =
// X_{Z,S}^{-1} y_Z (the vertex form of Section 3.2), so for a loss L with
// g = dL/db:  w = X_{Z,S}^{-T} g_S,  dL/dy_Z = w,  dL/dX_{Z,S} = -w b_S^T,
// and every other entry of dL/dy and dL/dX is zero.  At a NONUNIQUE output
// (certified, but a margin at fp32 resolution) this is the derivative of the
// returned vertex, one of the one-sided derivatives of the solution map.
// Two launches: k_bw_vertex runs the dense zero fill (blocks below
// fill_blocks, grid-stride, HBM-bound) side by side with the per-solve
// vertex solves (one wave each, latency-bound), which leave w in a small
// per-solve buffer; k_bw_scatter then writes the few non-zeros.
// --------------------------------------------------------------------------

// The vertex of solve s as the backward sees it: lane c < ns holds the
// c-th column of S (ascending) in sc and b at it in bS; lane q < ns holds
// the q-th zero row in zl.  Returns false (uniformly) when the solve has
// no certified vertex.
struct BwVertex {
    int n, p, ns, zl, sc;
    float bS;
    int64_t x_off, r0, b_base;
};

__device__ __forceinline__ bool bw_vertex(const BackwardArgs &a, int s, BwVertex &v)
{
    const int l = lane_id();
    const int k = a.problem ? a.problem[s] : s;
    v.r0 = a.row_off[k];
    v.n = (int)(a.row_off[k + 1] - v.r0);
    v.p = a.p_arr[k];
    v.x_off = a.x_off[k];
    const int64_t o = (int64_t)s * a.path_len + a.step;
    v.b_base = (int64_t)a.path_len * a.b_off[s] + (int64_t)a.step * v.p;
    const int status = a.status[o];
    const float bl = (l < v.p) ? a.b[v.b_base + l] : 0.f;
    const uint64_t sb = ballot(l < v.p && bl != 0.f);
    v.ns = popc64(sb);
    v.zl = (l < ZPAD) ? a.zrows[(int64_t)ZPAD * o + l] : -1;
    const int nz = popc64(ballot(l < ZPAD && v.zl >= 0));
    bool ok = (status == ST_CERTIFIED || status == ST_NONUNIQUE) && v.ns == nz && v.ns > 0;
    if (ok && l < v.ns && (v.zl < 0 || v.zl >= v.n)) ok = false;
    ok = ballot(!ok) == 0;
    // the c-th set bit of the S mask, for lane c
    uint64_t t = sb;
    v.sc = 0;
    for (int c = 0; c < v.ns; ++c) {
        const int j = (int)__builtin_ctzll(t);
        t &= t - 1;
        v.sc = (l == c) ? j : v.sc;
    }
    v.bS = (l < v.ns) ? a.b[v.b_base + v.sc] : 0.f;
    return ok;
}

__global__ __launch_bounds__(64) void k_bw_vertex(BackwardArgs a, int fill_blocks)
{
    const int l = lane_id();
    if ((int)blockIdx.x < fill_blocks) {
        // dense zeros: 16-byte streaming stores, scalar head and tail
        typedef float f4 __attribute__((ext_vector_type(4)));
        const int64_t t = (int64_t)blockIdx.x * 64 + l, nt = (int64_t)fill_blocks * 64;
        const f4 z = {0.f, 0.f, 0.f, 0.f};
        float *qs[2] = {a.grad_X, a.grad_y};
        const int64_t cs[2] = {a.x_len, a.y_len};
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            float *q = qs[u];
            const int64_t cnt = cs[u];
            const int64_t head = min<int64_t>(cnt, (int64_t)((-(uintptr_t)q >> 2) & 3));
            if (t < head) q[t] = 0.f;
            f4 *vq = (f4 *)(q + head);
            const int64_t m = (cnt - head) >> 2;
            for (int64_t e = t; e < m; e += nt) __builtin_nontemporal_store(z, vq + e);
            const int64_t tail = head + 4 * m + t;
            if (tail < cnt) q[tail] = 0.f;
        }
        return;
    }
    __shared__ float A[32 * ALD];
    __shared__ int piv[32];
    const int s = (int)blockIdx.x - fill_blocks;
    if (s >= a.num_solves) return;
    float *wout = a.bw + (int64_t)32 * s;
    BwVertex v;
    bool ok = bw_vertex(a, s, v);
    if (ok) {
        const float *X = a.X + v.x_off;
        // A[q][c] = x_{Z_q, S_c}: lane c gathers its column
        for (int q = 0; q < v.ns; ++q) {
            const int zq = rdlane(v.zl, q);
            if (l < v.ns) A[q * ALD + l] = X[(int64_t)zq * v.p + v.sc];
        }
        __syncthreads();
        ok = lu_factor(A, piv, v.ns);
    }
    if (!ok) {
        if (l == 0) wout[0] = __builtin_nanf(""); // no gradient for this solve
        return;
    }
    const float g = (l < v.ns) ? a.grad_b[a.b_off[s] + v.sc] : 0.f;
    const float w = lu_solve_t(A, piv, v.ns, g); // lane q: w_q
    if (l < 32) wout[l] = (l < v.ns) ? w : 0.f;
}

__global__ __launch_bounds__(64) void k_bw_scatter(BackwardArgs a)
{
    const int l = lane_id();
    const int s = blockIdx.x;
    if (s >= a.num_solves) return;
    BwVertex v;
    if (!bw_vertex(a, s, v)) return;
    const float w = (l < v.ns) ? a.bw[(int64_t)32 * s + l] : 0.f;
    if (!__builtin_isfinite(rdlane(w, 0))) return;
    if (ballot(l < v.ns && !__builtin_isfinite(w))) return;
    float *gX = a.grad_X + v.x_off;
    float *gy = a.grad_y + v.r0;
    if (l < v.ns) gy[v.zl] = w;
    for (int c = 0; c < v.ns; ++c) {
        const float bc = rdlane(v.bS, c);
        const int jc = rdlane(v.sc, c);
        if (l < v.ns) gX[(int64_t)v.zl * v.p + jc] = -w * bc;
    }
}

hipError_t launch_backward(const BackwardArgs &a, hipStream_t s)
{
    const int64_t f4s = (a.x_len + a.y_len) / 4 + 2;
    // two fill waves per CU: measured fastest (more fill waves crowd out the
    // vertex waves they are meant to overlap: 5.0 TB/s at 512, 3.7 at 2048)
    const int fill_blocks = (int)std::max<int64_t>(1, std::min<int64_t>((f4s + 63) / 64, 512));
    hipLaunchKernelGGL(k_bw_vertex, dim3(fill_blocks + a.num_solves), dim3(64), 0, s, a, fill_blocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.num_solves > 0) hipLaunchKernelGGL(k_bw_scatter, dim3(a.num_solves), dim3(64), 0, s, a);
    return hipGetLastError();
}

} // namespace ladl
