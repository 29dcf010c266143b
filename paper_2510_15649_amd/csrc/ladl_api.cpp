// C-ABI of the batched LAD-LASSO library: validation, plans, launches.
#include "ladlasso.h"
#include "ladl_kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

using namespace ladl;

namespace {

thread_local std::string g_detail;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_detail = buf;
    return code;
}

int hipfail(hipError_t e, const char *what)
{
    return fail(LADL_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int KNOWN_FLAGS = LADL_FLAG_GOLDEN | LADL_FLAG_NO_FINISHER | LADL_FLAG_NO_SNAP | LADL_FLAG_QUADRATURE;
constexpr int NMAX_ROWS = 2048;     // rows per problem (32 slots x 64 lanes)
constexpr size_t LDS_RESIDENT_MAX = 40 * 1024; // larger buckets keep X in the global workspace
constexpr int DENSE_MIN_ROUNDS = 2;             // solves per wave above which the dense variant is used
constexpr int TEAM_R32_DEFAULT = 1;             // waves per solve for n > 1024 unless the options say

int rows_per_lane(int n)
{
    int r = (n + 63) / 64, R = 1;
    while (R < r) R <<= 1;
    return R;
}

} // namespace

struct ladl_handle_s {
    int device = 0;
    int num_cu = 0;
    size_t lds_max = 0;
};

struct Bucket {
    int R = 1, pmax = 1;
    int offset = 0, count = 0; // slice of the order array
    int grid = 0;
    bool xg = false;           // X in the global workspace instead of LDS
    bool dense = false;        // the kernel variant built for 4 waves per SIMD
    int tw = 1;                // waves per solve (a team for tw > 1)
    int nlds = 0;              // with the workspace: columns of X kept in LDS
    int per_cu = 0;
    int64_t ws_off = 0;        // this bucket's slice of the workspace
    int nmax = 0;              // largest n in the bucket
    // tile schedule (n <= 64): the tile kernel's coordinate descent first,
    // in segments of tile_s lanes with tile_rs rows per lane, then the wave
    // kernel from its points
    bool tile_ok = false, tile = false;
    int tile_s = 0, tile_rs = 0, tile_grid = 0;
};

struct ladl_plan_s {
    ladl_handle_s *h = nullptr;
    int P = 0, S = 0, L = 1;
    std::vector<int64_t> row_off, x_off, b_off;
    std::vector<int32_t> p, problem;
    int64_t b_len = 0, x_len = 0, y_len = 0;
    ladl_options opt{};
    std::vector<Bucket> buckets;
    bool multi_bucket = false;   // buckets run side by side and share the CUs
    int64_t *d_row_off = nullptr, *d_x_off = nullptr, *d_b_off = nullptr;
    int32_t *d_p = nullptr, *d_problem = nullptr, *d_order = nullptr, *d_counters = nullptr;
    int32_t *d_order_plain = nullptr, *d_counter_plain = nullptr;
    float *d_gws = nullptr;      // plain kernel scratch
    int64_t gws_stride = 0;
    float *d_wws = nullptr;      // wave kernel workspace (buckets with X outside LDS)
    int64_t wws_floats = 0;
    float *d_bw = nullptr;       // backward: 32 floats per solve (plans with each problem once)
    float *d_seed = nullptr;     // tile stage output, laid out like b (b_len floats)
    int32_t *d_bf_order = nullptr; // vertex enumeration: solves grouped by p (built on first use)
    std::vector<std::pair<int, int>> bf_buckets; // (p, count) in d_bf_order order
    // buckets run concurrently on streams forked from the caller's stream
    std::vector<hipStream_t> bstreams;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;
    int nmax = 0, pmax = 0;
    bool problems_once = false; // every problem used by exactly one solve
    // kernel timing: an event pair around each bucket's launch, recorded on
    // the bucket's stream while profiling is on
    bool profiling = false;
    std::vector<std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof;
};

struct ladl_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
};

static int layout_workspace(ladl_plan_t pl);
static void set_schedule(ladl_plan_t pl, Bucket &b, bool xg, bool dense = false, int tw = 1);
static void set_tile(ladl_plan_t pl, Bucket &b, bool on);
static int alloc_seed(ladl_plan_t pl);
// queue counters: the wave kernel's of bucket i at i, the tile kernel's at
// buckets + i
static int num_counters(ladl_plan_t pl) { return 2 * (int)pl->buckets.size(); }

// exported functions: C linkage comes from their declarations in ladlasso.h

const char *ladl_error_string(int code)
{
    switch (code) {
    case LADL_OK: return "LADL_OK";
    case LADL_EINVAL: return "LADL_EINVAL: invalid argument";
    case LADL_EUNSUPPORTED: return "LADL_EUNSUPPORTED: outside supported limits";
    case LADL_EHIP: return "LADL_EHIP: HIP runtime error";
    case LADL_ENOMEM: return "LADL_ENOMEM: allocation failed";
    default: return "unknown ladl error code";
    }
}

const char *ladl_last_error_detail(void) { return g_detail.c_str(); }

void ladl_default_options(ladl_options *o)
{
    if (!o) return;
    o->tol_f = 1e-6f;
    o->tol_s = 9.5367431640625e-07f; // 2^-20
    o->lambda_min = 0.f;
    o->max_sweeps = 8;
    o->max_ternary = 48;
    o->max_rounds = 1;
    o->max_pivots = 0;
    o->flags = LADL_FLAG_GOLDEN;
    o->schedule = -1;
    o->chop_range = 0.03125f;
    o->team = 0;
    o->tile = 0;
}

int ladl_create(ladl_handle_t *handle)
{
    if (!handle) return fail(LADL_EINVAL, "handle pointer is NULL");
    *handle = nullptr;
    auto *h = new (std::nothrow) ladl_handle_s;
    if (!h) return fail(LADL_ENOMEM, "host allocation");
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hipfail(e, "hipGetDevice");
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, h->device);
    if (e != hipSuccess) {
        delete h;
        return hipfail(e, "hipGetDeviceProperties");
    }
    h->num_cu = prop.multiProcessorCount;
    h->lds_max = prop.sharedMemPerBlock;
    if (prop.maxSharedMemoryPerMultiProcessor > h->lds_max) h->lds_max = prop.maxSharedMemoryPerMultiProcessor;
    if (h->lds_max > 160 * 1024) h->lds_max = 160 * 1024;
    *handle = h;
    return LADL_OK;
}

int ladl_destroy(ladl_handle_t h)
{
    delete h;
    return LADL_OK;
}

static int check_options(const ladl_options *o)
{
    if (!(o->tol_f >= 0.f) || !std::isfinite(o->tol_f)) return fail(LADL_EINVAL, "tol_f must be finite and >= 0");
    if (!(o->tol_s > 0.f) || !std::isfinite(o->tol_s)) return fail(LADL_EINVAL, "tol_s must be finite and > 0");
    if (!(o->lambda_min >= 0.f) || !std::isfinite(o->lambda_min))
        return fail(LADL_EINVAL, "lambda_min must be finite and >= 0");
    if (o->max_sweeps < 1 || o->max_sweeps > 100000) return fail(LADL_EINVAL, "max_sweeps out of [1, 100000]");
    if (o->max_ternary < 0 || o->max_ternary > 10000) return fail(LADL_EINVAL, "max_ternary out of [0, 10000]");
    if (o->max_rounds < -1 || o->max_rounds > 64) return fail(LADL_EINVAL, "max_rounds out of [-1, 64]");
    if (o->max_pivots < 0 || o->max_pivots > 100000) return fail(LADL_EINVAL, "max_pivots out of [0, 100000]");
    if (o->flags & ~KNOWN_FLAGS) return fail(LADL_EINVAL, "unknown flag bits 0x%x", o->flags & ~KNOWN_FLAGS);
    if (o->schedule < -1 || o->schedule > 1) return fail(LADL_EINVAL, "unknown schedule %d", o->schedule);
    if (!(o->chop_range > 0.f) || !std::isfinite(o->chop_range))
        return fail(LADL_EINVAL, "chop_range must be finite and > 0");
    if (o->team != 0 && o->team != 1 && o->team != 2 && o->team != 4)
        return fail(LADL_EINVAL, "team must be 0, 1, 2 or 4 (got %d)", o->team);
    if (o->tile < 0 || o->tile > 2) return fail(LADL_EINVAL, "tile must be 0, 1 or 2 (got %d)", o->tile);
    if (o->tile == 2 && (o->flags & LADL_FLAG_QUADRATURE))
        return fail(LADL_EINVAL, "the tile schedule runs the weighted-median update; it excludes LADL_FLAG_QUADRATURE");
    return LADL_OK;
}

static void prof_clear(ladl_plan_s *pl)
{
    for (auto &v : pl->prof)
        for (auto &e : v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    pl->prof.clear();
}

static void plan_free_device(ladl_plan_s *pl)
{
    prof_clear(pl);
    (void)hipFree(pl->d_row_off);
    (void)hipFree(pl->d_x_off);
    (void)hipFree(pl->d_b_off);
    (void)hipFree(pl->d_p);
    (void)hipFree(pl->d_problem);
    (void)hipFree(pl->d_order);
    (void)hipFree(pl->d_counters);
    (void)hipFree(pl->d_order_plain);
    (void)hipFree(pl->d_counter_plain);
    (void)hipFree(pl->d_gws);
    (void)hipFree(pl->d_wws);
    (void)hipFree(pl->d_bw);
    (void)hipFree(pl->d_seed);
    (void)hipFree(pl->d_bf_order);
    for (hipStream_t st : pl->bstreams) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : pl->ev_join) (void)hipEventDestroy(ev);
    if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
    pl->bstreams.clear();
    pl->ev_join.clear();
    pl->ev_fork = nullptr;
}

template <typename T>
static hipError_t upload(T **dst, const std::vector<T> &src)
{
    size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

int ladl_plan_create(ladl_handle_t h, const ladl_layout *lay, const ladl_options *opt, ladl_plan_t *out)
{
    if (!out) return fail(LADL_EINVAL, "plan pointer is NULL");
    *out = nullptr;
    if (!h || !lay) return fail(LADL_EINVAL, "handle or layout is NULL");
    ladl_options o;
    ladl_default_options(&o);
    if (opt) o = *opt;
    int rc = check_options(&o);
    if (rc) return rc;
    const int P = lay->num_problems, S = lay->num_solves, L = lay->path_len;
    if (P < 1) return fail(LADL_EINVAL, "num_problems must be >= 1 (got %d)", P);
    if (S < 1) return fail(LADL_EINVAL, "num_solves must be >= 1 (got %d)", S);
    if (L < 1) return fail(LADL_EINVAL, "path_len must be >= 1 (got %d)", L);
    if ((int64_t)S * L > (int64_t)INT32_MAX / 32) return fail(LADL_EUNSUPPORTED, "too many solve outputs");
    if (!lay->row_off) return fail(LADL_EINVAL, "row_off is NULL");
    if (lay->x_len < 0 || lay->y_len < 0) return fail(LADL_EINVAL, "negative x_len or y_len");
    auto pl = new (std::nothrow) ladl_plan_s;
    if (!pl) return fail(LADL_ENOMEM, "host allocation");
    pl->h = h;
    pl->P = P;
    pl->S = S;
    pl->L = L;
    pl->opt = o;
    pl->x_len = lay->x_len;
    pl->y_len = lay->y_len;
    pl->row_off.assign(lay->row_off, lay->row_off + P + 1);
    pl->p.resize(P);
    pl->x_off.resize(P);
    auto bad = [&](int code, const char *fmt, auto... args) {
        delete pl;
        return fail(code, fmt, args...);
    };
    if (pl->row_off[0] != 0) return bad(LADL_EINVAL, "row_off[0] must be 0 (got %lld)", (long long)pl->row_off[0]);
    for (int k = 0; k < P; ++k) {
        int64_t n = pl->row_off[k + 1] - pl->row_off[k];
        if (n < 1) return bad(LADL_EINVAL, "problem %d has %lld rows (row_off must increase)", k, (long long)n);
        if (n > NMAX_ROWS) return bad(LADL_EUNSUPPORTED, "problem %d has %lld rows (limit %d)", k, (long long)n, NMAX_ROWS);
        int pk = lay->p ? lay->p[k] : lay->p_uniform;
        if (pk < 1 || pk > PMAX) return bad(LADL_EUNSUPPORTED, "problem %d has p = %d (limit 1..%d)", k, pk, PMAX);
        if (!lay->x_off && lay->p && pk != lay->p_uniform)
            return bad(LADL_EINVAL, "x_off is NULL but p[%d] = %d differs from p_uniform", k, pk);
        int64_t xo = lay->x_off ? lay->x_off[k] : pl->row_off[k] * (int64_t)lay->p_uniform;
        if (xo < 0 || xo + n * pk > lay->x_len)
            return bad(LADL_EINVAL, "problem %d: X block [%lld, %lld) outside x_len %lld", k, (long long)xo,
                       (long long)(xo + n * pk), (long long)lay->x_len);
        pl->p[k] = pk;
        pl->x_off[k] = xo;
        pl->nmax = std::max<int>(pl->nmax, (int)n);
        pl->pmax = std::max(pl->pmax, pk);
    }
    if (pl->row_off[P] > lay->y_len)
        return bad(LADL_EINVAL, "row_off[%d] = %lld exceeds y_len %lld", P, (long long)pl->row_off[P],
                   (long long)lay->y_len);
    pl->problem.resize(S);
    std::vector<int> uses(P, 0);
    for (int s = 0; s < S; ++s) {
        int k = lay->problem ? lay->problem[s] : s;
        if (k < 0 || k >= P) return bad(LADL_EINVAL, "problem[%d] = %d out of range", s, k);
        pl->problem[s] = k;
        uses[k]++;
    }
    pl->problems_once = std::all_of(uses.begin(), uses.end(), [](int u) { return u == 1; });
    pl->b_off.resize(S);
    int64_t acc = 0;
    for (int s = 0; s < S; ++s) {
        pl->b_off[s] = acc;
        acc += pl->p[pl->problem[s]];
    }
    pl->b_len = acc * L;
    // queue order: decreasing n*p, then (with a lambda hint) increasing sum
    // of the path's lambdas, since small-lambda solves run the longest
    std::vector<double> lsum(S, 0.0);
    if (lay->lambda_hint)
        for (int s = 0; s < S; ++s)
            for (int t = 0; t < L; ++t) lsum[s] += (double)lay->lambda_hint[(int64_t)s * L + t];
    auto cost_gt = [&](int a, int c) {
        int ka = pl->problem[a], kc = pl->problem[c];
        int64_t ca = (pl->row_off[ka + 1] - pl->row_off[ka]) * pl->p[ka];
        int64_t cc = (pl->row_off[kc + 1] - pl->row_off[kc]) * pl->p[kc];
        if (ca != cc) return ca > cc;
        return lsum[a] < lsum[c];
    };
    // buckets by rows per lane; decreasing cost inside a bucket
    std::vector<int> Rs = {32, 16, 8, 4, 2, 1};
    {
        uint32_t seen = 0;
        for (int s = 0; s < S; ++s) {
            const int k = pl->problem[s];
            seen |= (uint32_t)rows_per_lane((int)(pl->row_off[k + 1] - pl->row_off[k]));
        }
        pl->multi_bucket = __builtin_popcount(seen) > 1;
    }
    std::vector<int32_t> order;
    order.reserve(S);
    for (int R : Rs) {
        Bucket b;
        b.R = R;
        b.offset = (int)order.size();
        std::vector<int32_t> ids;
        for (int s = 0; s < S; ++s) {
            int k = pl->problem[s];
            int n = (int)(pl->row_off[k + 1] - pl->row_off[k]);
            if (rows_per_lane(n) == R) ids.push_back(s);
        }
        if (ids.empty()) continue;
        std::stable_sort(ids.begin(), ids.end(), cost_gt);
        for (int s : ids) {
            const int k = pl->problem[s];
            b.pmax = std::max(b.pmax, (int)pl->p[k]);
            b.nmax = std::max(b.nmax, (int)(pl->row_off[k + 1] - pl->row_off[k]));
        }
        b.count = (int)ids.size();
        order.insert(order.end(), ids.begin(), ids.end());
        const bool xg = o.schedule >= 0 || R >= 32 || wave_lds_bytes(R, b.pmax, false, 0, 1) > LDS_RESIDENT_MAX;
        size_t lds = wave_lds_bytes(R, b.pmax, xg, 0, 1);
        if (lds > h->lds_max)
            return bad(LADL_EUNSUPPORTED, "bucket R=%d p=%d needs %zu bytes of LDS (device limit %zu)", R, b.pmax,
                       lds, h->lds_max);
        // waves per solve: the option, else the static choice (one wave, or
        // a team for the n > 1024 bucket)
        const int tw = (o.team > 0 && wave_has_team(R, o.team)) ? o.team
                                                                 : (o.team == 0 && R >= 32 ? TEAM_R32_DEFAULT : 1);
        set_schedule(pl, b, xg, false, tw);
        // the dense variant where the bucket holds more than DENSE_MIN_ROUNDS
        // full grids of solves: the extra waves then shorten every round
        // (c1, 8192 solves of n = 200, p = 8: 3.82 instead of 4.0 ms)
        if (b.tw == 1 && wave_has_dense(R) &&
            (o.schedule == 1 || (o.schedule == -1 && b.count > DENSE_MIN_ROUNDS * b.grid)))
            set_schedule(pl, b, true, true);
        {
            int ts, trs;
            b.tile_ok = R == 1 && !(o.flags & LADL_FLAG_QUADRATURE) && tile_shape_for(b.nmax, ts, trs);
        }
        set_tile(pl, b, b.tile_ok && o.tile == 2);
        pl->buckets.push_back(b);
    }
    // plain kernel: all solves, decreasing cost
    std::vector<int32_t> order_plain(S);
    std::iota(order_plain.begin(), order_plain.end(), 0);
    std::stable_sort(order_plain.begin(), order_plain.end(), [&](int a, int c) {
        int ka = pl->problem[a], kc = pl->problem[c];
        return (pl->row_off[ka + 1] - pl->row_off[ka]) * pl->p[ka] > (pl->row_off[kc + 1] - pl->row_off[kc]) * pl->p[kc];
    });
    hipError_t e;
    std::vector<int32_t> zeros(2 * pl->buckets.size() + 1, 0);
    if ((e = upload(&pl->d_row_off, pl->row_off)) != hipSuccess || (e = upload(&pl->d_x_off, pl->x_off)) != hipSuccess ||
        (e = upload(&pl->d_b_off, pl->b_off)) != hipSuccess || (e = upload(&pl->d_p, pl->p)) != hipSuccess ||
        (e = upload(&pl->d_problem, pl->problem)) != hipSuccess || (e = upload(&pl->d_order, order)) != hipSuccess ||
        (e = upload(&pl->d_counters, zeros)) != hipSuccess ||
        (e = upload(&pl->d_order_plain, order_plain)) != hipSuccess ||
        (e = upload(&pl->d_counter_plain, std::vector<int32_t>(1, 0))) != hipSuccess) {
        plan_free_device(pl);
        delete pl;
        return hipfail(e, "plan upload");
    }
    if ((rc = layout_workspace(pl)) != LADL_OK || (rc = alloc_seed(pl)) != LADL_OK) {
        plan_free_device(pl);
        delete pl;
        return rc;
    }
    if (pl->problems_once && S > 0 &&
        (e = hipMalloc((void **)&pl->d_bw, sizeof(float) * 32 * (size_t)S)) != hipSuccess) {
        pl->d_bw = nullptr;
        plan_free_device(pl);
        delete pl;
        return hipfail(e, "backward buffer");
    }
    if (pl->buckets.size() > 1) {
        pl->bstreams.resize(pl->buckets.size(), nullptr);
        pl->ev_join.resize(pl->buckets.size(), nullptr);
        e = hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming);
        for (size_t i = 0; e == hipSuccess && i < pl->buckets.size(); ++i) {
            e = hipStreamCreateWithFlags(&pl->bstreams[i], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_join[i], hipEventDisableTiming);
        }
        if (e != hipSuccess) {
            plan_free_device(pl);
            delete pl;
            return hipfail(e, "plan streams");
        }
    }
    *out = pl;
    return LADL_OK;
}

int ladl_plan_destroy(ladl_plan_t pl)
{
    if (!pl) return LADL_OK;
    plan_free_device(pl);
    delete pl;
    return LADL_OK;
}

int64_t ladl_plan_b_len(ladl_plan_t pl) { return pl ? pl->b_len : -1; }

static DevOpt dev_opt(const ladl_options &o)
{
    DevOpt d;
    d.tol_f = o.tol_f;
    d.tol_s = o.tol_s;
    d.lambda_min = o.lambda_min;
    d.max_sweeps = o.max_sweeps;
    d.max_ternary = o.max_ternary;
    d.max_rounds = o.max_rounds;
    d.max_pivots = o.max_pivots;
    d.flags = o.flags;
    d.chop_range = o.chop_range;
    return d;
}

static int check_solve_ptrs(ladl_plan_t pl, const float *X, const float *y, const float *lam, float *b, float *obj,
                            uint32_t *active, int32_t *zr, int32_t *st)
{
    if (!pl) return fail(LADL_EINVAL, "plan is NULL");
    if (!X || !y || !lam || !b || !obj || !active || !zr || !st)
        return fail(LADL_EINVAL, "a required device pointer is NULL");
    if (((uintptr_t)X | (uintptr_t)y | (uintptr_t)lam | (uintptr_t)b | (uintptr_t)obj | (uintptr_t)active |
         (uintptr_t)zr | (uintptr_t)st) & 3)
        return fail(LADL_EINVAL, "device pointers must be 4-byte aligned");
    return LADL_OK;
}

static SolveArgs base_args(ladl_plan_t pl, const float *X, const float *y, const float *lam, const float *b_init,
                           float *b, float *obj, uint32_t *active, int32_t *zr, int32_t *st, int32_t *it, int t0,
                           int t1)
{
    SolveArgs a;
    std::memset(&a, 0, sizeof a);
    a.X = X;
    a.y = y;
    a.lam = lam;
    a.b_init = b_init;
    a.row_off = pl->d_row_off;
    a.x_off = pl->d_x_off;
    a.b_off = pl->d_b_off;
    a.p_arr = pl->d_p;
    a.problem = pl->d_problem;
    a.path_len = pl->L;
    a.t0 = t0;
    a.t1 = t1;
    a.b_out = b;
    a.obj_out = obj;
    a.active_out = active;
    a.zrows_out = zr;
    a.status_out = st;
    a.iters_out = it;
    a.opt = dev_opt(pl->opt);
    return a;
}

// workspace slices for the buckets whose X lives in HBM; grows the buffer
static int layout_workspace(ladl_plan_t pl)
{
    int64_t tot = 0;
    for (Bucket &b : pl->buckets) {
        b.ws_off = tot;
        if (b.xg) tot += (int64_t)b.grid * (int64_t)wave_ws_floats_host(b.R / b.tw, b.pmax, b.nlds, b.tw);
    }
    if (tot > pl->wws_floats || (tot > 0 && !pl->d_wws)) {
        (void)hipFree(pl->d_wws);
        pl->d_wws = nullptr;
        hipError_t e = hipMalloc((void **)&pl->d_wws, sizeof(float) * (size_t)tot);
        if (e != hipSuccess) return hipfail(e, "workspace");
        pl->wws_floats = tot;
    }
    return LADL_OK;
}

static void set_schedule(ladl_plan_t pl, Bucket &b, bool xg, bool dense, int tw)
{
    b.tw = wave_has_team(b.R, tw) ? tw : 1;
    b.xg = xg || dense || b.tw > 1;
    b.dense = dense && b.tw == 1 && wave_has_dense(b.R);
    b.nlds = b.xg ? 0 : b.pmax;
    const int Rw = b.R / b.tw; // row slots per lane of each wave
    const bool quad = (pl->opt.flags & LADL_FLAG_QUADRATURE) != 0;
    b.per_cu = std::max(1, wave_max_blocks_per_cu(b.R, b.pmax, b.xg, b.dense, b.tw, quad, b.nlds));
    // With the workspace, keep in LDS as many leading columns of X as the
    // LDS left over at this occupancy holds.  Where buckets run side by side
    // that LDS is what lets the other buckets' waves share a CU, so there
    // only the n > 1024 bucket takes columns (measured on the ragged
    // workloads: the n <= 2048 bucket 1.5x faster with them; the 4096 row
    // subsets of the correlated dataset 8% slower when every bucket took
    // them).
    const bool take = !pl->multi_bucket || b.R >= 32;
    while (take && b.xg && b.nlds < b.pmax && wave_lds_bytes(Rw, b.pmax, true, b.nlds + 1, b.tw) <= pl->h->lds_max &&
           wave_max_blocks_per_cu(b.R, b.pmax, true, b.dense, b.tw, quad, b.nlds + 1) >= b.per_cu)
        ++b.nlds;
    b.grid = (int)std::min<int64_t>(b.count, (int64_t)b.per_cu * pl->h->num_cu);
}

static void set_tile(ladl_plan_t pl, Bucket &b, bool on)
{
    b.tile = on && b.tile_ok && tile_shape_for(b.nmax, b.tile_s, b.tile_rs);
    if (!b.tile) return;
    const int per_cu = std::max(1, tile_max_blocks_per_cu(b.tile_s, b.tile_rs, b.pmax));
    const int per_block = tile_solves_per_block(b.tile_s);
    b.tile_grid = (int)std::min<int64_t>((b.count + per_block - 1) / per_block, (int64_t)per_cu * pl->h->num_cu);
}

// the tile stage's output buffer, once any bucket takes the tile schedule
static int alloc_seed(ladl_plan_t pl)
{
    const bool any = std::any_of(pl->buckets.begin(), pl->buckets.end(), [](const Bucket &b) { return b.tile; });
    if (!any || pl->d_seed) return LADL_OK;
    hipError_t e = hipMalloc((void **)&pl->d_seed, sizeof(float) * (size_t)std::max<int64_t>(pl->b_len, 1));
    if (e != hipSuccess) {
        pl->d_seed = nullptr;
        return hipfail(e, "tile stage buffer");
    }
    return LADL_OK;
}

static hipError_t launch_bucket(ladl_plan_t pl, size_t bi, const SolveArgs &base, hipStream_t s)
{
    const Bucket &bk = pl->buckets[bi];
    SolveArgs a = base;
    a.order = pl->d_order + bk.offset;
    a.num_items = bk.count;
    a.counter = pl->d_counters + bi;
    a.pmax = bk.pmax;
    a.nlds = bk.nlds;
    if (bk.tile && a.t0 == 0) {
        // the cold start's descent and chop on tiles, then the wave kernel
        // from their points
        if (!pl->d_seed) return hipErrorInvalidValue;
        SolveArgs at = a;
        at.t1 = 1;
        at.b_out = pl->d_seed;
        at.counter = pl->d_counters + pl->buckets.size() + bi;
        hipError_t e = launch_tile(bk.tile_s, bk.tile_rs, at, bk.tile_grid, s);
        if (e != hipSuccess) return e;
        a.b_seed = pl->d_seed;
    }
    if (bk.xg) {
        a.gws = pl->d_wws + bk.ws_off;
        a.gws_stride = (int64_t)wave_ws_floats_host(bk.R / bk.tw, bk.pmax, bk.nlds, bk.tw);
    }
    return launch_wave(bk.R, bk.xg, bk.dense, bk.tw, (pl->opt.flags & LADL_FLAG_QUADRATURE) != 0, a, bk.grid, s);
}

static int enqueue_wave(ladl_plan_t pl, const float *X, const float *y, const float *lam, const float *b_init,
                        float *b, float *obj, uint32_t *active, int32_t *zr, int32_t *st, int32_t *it, int t0,
                        int t1, hipStream_t s, bool capturing = false)
{
    const bool timed = pl->profiling && !capturing;
    hipError_t e = launch_reset(pl->d_counters, num_counters(pl), s);
    if (e != hipSuccess) return hipfail(e, "queue reset launch");
    const bool fork = pl->buckets.size() > 1;
    if (fork && (e = hipEventRecord(pl->ev_fork, s)) != hipSuccess) return hipfail(e, "fork event");
    for (size_t bi = 0; bi < pl->buckets.size(); ++bi) {
        const Bucket &bk = pl->buckets[bi];
        hipStream_t bs = fork ? pl->bstreams[bi] : s;
        if (fork && (e = hipStreamWaitEvent(bs, pl->ev_fork, 0)) != hipSuccess) return hipfail(e, "fork wait");
        (void)bk;
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        if (timed) {
            if ((e = hipEventCreate(&ev.first)) != hipSuccess || (e = hipEventCreate(&ev.second)) != hipSuccess ||
                (e = hipEventRecord(ev.first, bs)) != hipSuccess) {
                if (ev.first) (void)hipEventDestroy(ev.first);
                if (ev.second) (void)hipEventDestroy(ev.second);
                return hipfail(e, "profiling event");
            }
        }
        e = launch_bucket(pl, bi, base_args(pl, X, y, lam, b_init, b, obj, active, zr, st, it, t0, t1), bs);
        if (e != hipSuccess) return hipfail(e, "solve kernel launch");
        if (timed) {
            if ((e = hipEventRecord(ev.second, bs)) != hipSuccess) return hipfail(e, "profiling event");
            pl->prof[bi].push_back(ev);
        }
        if (fork && (e = hipEventRecord(pl->ev_join[bi], bs)) != hipSuccess) return hipfail(e, "join event");
    }
    for (size_t bi = 0; fork && bi < pl->buckets.size(); ++bi)
        if ((e = hipStreamWaitEvent(s, pl->ev_join[bi], 0)) != hipSuccess) return hipfail(e, "join wait");
    return LADL_OK;
}

int ladl_solve_f32(ladl_plan_t pl, const float *X, const float *y, const float *lam, const float *b_init, float *b,
                   float *obj, uint32_t *active, int32_t *zr, int32_t *st, int32_t *it, void *stream)
{
    int rc = check_solve_ptrs(pl, X, y, lam, b, obj, active, zr, st);
    if (rc) return rc;
    return enqueue_wave(pl, X, y, lam, b_init, b, obj, active, zr, st, it, 0, pl->L, (hipStream_t)stream);
}

int ladl_solve_plain_f32(ladl_plan_t pl, const float *X, const float *y, const float *lam, const float *b_init,
                         float *b, float *obj, uint32_t *active, int32_t *zr, int32_t *st, int32_t *it,
                         void *stream)
{
    int rc = check_solve_ptrs(pl, X, y, lam, b, obj, active, zr, st);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // one thread per solve, up to 2^17 threads fetching from the queue
    const int64_t T = std::min<int64_t>(((int64_t)pl->S + 63) / 64 * 64, 131072);
    if (!pl->d_gws || pl->gws_stride != T) {
        (void)hipFree(pl->d_gws);
        pl->d_gws = nullptr;
        hipError_t e = hipMalloc((void **)&pl->d_gws, sizeof(float) * (size_t)plain_scratch_floats(pl->nmax, T));
        if (e != hipSuccess) return hipfail(e, "plain kernel scratch");
        pl->gws_stride = T;
    }
    hipError_t e = launch_reset(pl->d_counter_plain, 1, s);
    if (e != hipSuccess) return hipfail(e, "queue reset launch");
    SolveArgs a = base_args(pl, X, y, lam, b_init, b, obj, active, zr, st, it, 0, pl->L);
    a.order = pl->d_order_plain;
    a.num_items = pl->S;
    a.counter = pl->d_counter_plain;
    a.gws = pl->d_gws;
    a.gws_stride = T;
    e = launch_plain(a, pl->nmax, T, s);
    if (e != hipSuccess) return hipfail(e, "plain kernel launch");
    return LADL_OK;
}

int ladl_backward_f32(ladl_plan_t pl, const float *X, const float *b, const int32_t *zr, const int32_t *st,
                      int32_t step, const float *grad_b, float *grad_y, float *grad_X, void *stream)
{
    if (!pl) return fail(LADL_EINVAL, "plan is NULL");
    if (!X || !b || !zr || !st || !grad_b || !grad_y || !grad_X)
        return fail(LADL_EINVAL, "a required device pointer is NULL");
    if (step < 0 || step >= pl->L) return fail(LADL_EINVAL, "step %d outside the path [0, %d)", step, pl->L);
    if (!pl->problems_once)
        return fail(LADL_EINVAL, "backward needs every problem used by exactly one solve");
    BackwardArgs a;
    std::memset(&a, 0, sizeof a);
    a.X = X;
    a.b = b;
    a.grad_b = grad_b;
    a.zrows = zr;
    a.status = st;
    a.row_off = pl->d_row_off;
    a.x_off = pl->d_x_off;
    a.b_off = pl->d_b_off;
    a.p_arr = pl->d_p;
    a.problem = pl->d_problem;
    a.num_solves = pl->S;
    a.path_len = pl->L;
    a.step = step;
    a.grad_y = grad_y;
    a.grad_X = grad_X;
    a.x_len = pl->x_len;
    a.y_len = pl->y_len;
    a.bw = pl->d_bw;
    hipError_t e = launch_backward(a, (hipStream_t)stream);
    if (e != hipSuccess) return hipfail(e, "backward kernel launch");
    return LADL_OK;
}

int ladl_graph_create(ladl_plan_t pl, const float *X, const float *y, const float *lam, const float *b_init,
                      float *b, float *obj, uint32_t *active, int32_t *zr, int32_t *st, int32_t *it,
                      ladl_graph_t *graph)
{
    if (!graph) return fail(LADL_EINVAL, "graph pointer is NULL");
    *graph = nullptr;
    int rc = check_solve_ptrs(pl, X, y, lam, b, obj, active, zr, st);
    if (rc) return rc;
    auto *g = new (std::nothrow) ladl_graph_s;
    if (!g) return fail(LADL_ENOMEM, "host allocation");
    hipError_t e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        return hipfail(e, "capture stream");
    }
    e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        ladl_graph_destroy(g);
        return hipfail(e, "begin capture");
    }
    // one launch per path step, each warm-started from the previous output
    for (int t = 0; t < pl->L && rc == LADL_OK; ++t)
        rc = enqueue_wave(pl, X, y, lam, b_init, b, obj, active, zr, st, it, t, t + 1, g->cap, true);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(g->cap, &gr);
    g->graph = gr;
    if (rc != LADL_OK || e != hipSuccess) {
        ladl_graph_destroy(g);
        return rc != LADL_OK ? rc : hipfail(e, "end capture");
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        ladl_graph_destroy(g);
        return hipfail(e, "graph instantiate");
    }
    *graph = g;
    return LADL_OK;
}

int ladl_graph_launch(ladl_graph_t g, void *stream)
{
    if (!g || !g->exec) return fail(LADL_EINVAL, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hipfail(e, "graph launch");
    return LADL_OK;
}

int ladl_graph_destroy(ladl_graph_t g)
{
    if (!g) return LADL_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    delete g;
    return LADL_OK;
}

// Tuning cache: one line per decision, "<device name> <R> <pmax> <choice>"
// (the autotuner's candidate number), in the file named by LADL_TUNE_CACHE
// (optional).
static std::string device_name(int dev)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string n = prop.gcnArchName;
    for (char &c : n)
        if (c == ' ') c = '_';
    return n;
}

static int cache_lookup(const std::string &dev, int R, int pmax)
{
    const char *path = std::getenv("LADL_TUNE_CACHE");
    if (!path) return -1;
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char name[256];
    int r, pm, v, found = -1;
    while (std::fscanf(f, "%255s %d %d %d", name, &r, &pm, &v) == 4)
        if (dev == name && r == R && pm == pmax) found = v;
    std::fclose(f);
    return found;
}

static void cache_store(const std::string &dev, int R, int pmax, int v)
{
    const char *path = std::getenv("LADL_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d\n", dev.c_str(), R, pmax, v);
    std::fclose(f);
}

int ladl_autotune(ladl_plan_t pl, const float *X, const float *y, const float *lam, float *b, float *obj,
                  uint32_t *active, int32_t *zr, int32_t *st, void *stream)
{
    int rc = check_solve_ptrs(pl, X, y, lam, b, obj, active, zr, st);
    if (rc) return rc;
    if (pl->opt.schedule >= 0) return LADL_OK; // the caller fixed the schedule
    hipStream_t s = (hipStream_t)stream;
    const std::string dev = device_name(pl->h->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hipfail(e, "tuning events");
    }
    // candidates per bucket: 0 = X in LDS, 1 = X in the HBM workspace,
    // 2 = the HBM workspace with the dense kernel variant, 3 and 4 = the HBM
    // workspace with a team of 2 or 4 waves per solve; for n <= 64 each of
    // these also with the tile stage in front (value + 8)
    auto apply = [&](Bucket &bk, int v) {
        const int w = v & 7;
        set_schedule(pl, bk, w != 0, w == 2, w == 3 ? 2 : (w == 4 ? 4 : 1));
        set_tile(pl, bk, (v & 8) != 0);
    };
    for (size_t bi = 0; bi < pl->buckets.size() && rc == LADL_OK; ++bi) {
        Bucket &bk = pl->buckets[bi];
        const int forced = pl->opt.team; // 0: the team size is tuned too
        bool can[13] = {};
        can[0] = bk.R < 32 && wave_lds_bytes(bk.R, bk.pmax, false, 0, 1) <= pl->h->lds_max;
        can[1] = true;
        can[2] = wave_has_dense(bk.R);
        can[3] = wave_has_team(bk.R, 2);
        can[4] = wave_has_team(bk.R, 4);
        for (int v = 0; v < 5; ++v) {
            const int tw = v == 3 ? 2 : (v == 4 ? 4 : 1);
            if (forced > 0 && tw != forced) can[v] = false;
        }
        // tiles: where the bucket allows them, unless the option fixes them
        for (int v = 0; v < 5; ++v) {
            can[v + 8] = can[v] && bk.tile_ok && pl->opt.tile != 1;
            if (pl->opt.tile == 2 && bk.tile_ok) can[v] = false;
        }
        int ncand = 0;
        for (int v = 0; v < 13; ++v) ncand += can[v] ? 1 : 0;
        if (ncand < 2) continue; // nothing to choose
        int cached = cache_lookup(dev, bk.R, bk.pmax);
        if (cached >= 0 && cached <= 12 && can[cached]) {
            apply(bk, cached);
            continue;
        }
        float best_ms = 1e30f;
        int best_v = (bk.tw == 4 ? 4 : (bk.tw == 2 ? 3 : (bk.dense ? 2 : (bk.xg ? 1 : 0)))) + (bk.tile ? 8 : 0);
        for (int v = 0; v < 13 && rc == LADL_OK; ++v) {
            if (!can[v]) continue;
            apply(bk, v);
            if ((rc = layout_workspace(pl)) != LADL_OK || (rc = alloc_seed(pl)) != LADL_OK) break;
            SolveArgs a = base_args(pl, X, y, lam, nullptr, b, obj, active, zr, st, nullptr, 0, pl->L);
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) { // first run warms up
                if ((e = launch_reset(pl->d_counters, num_counters(pl), s)) != hipSuccess ||
                    (e = hipEventRecord(e0, s)) != hipSuccess || (e = launch_bucket(pl, bi, a, s)) != hipSuccess ||
                    (e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
                    (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
                    rc = hipfail(e, "tuning run");
                    break;
                }
            }
            if (rc == LADL_OK && ms < best_ms) {
                best_ms = ms;
                best_v = v;
            }
        }
        if (rc == LADL_OK) {
            apply(bk, best_v);
            cache_store(dev, bk.R, bk.pmax, best_v);
        }
    }
    if (rc == LADL_OK) rc = layout_workspace(pl);
    if (rc == LADL_OK) rc = alloc_seed(pl);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int ladl_plan_profile(ladl_plan_t pl, int32_t enable)
{
    if (!pl) return fail(LADL_EINVAL, "plan is NULL");
    prof_clear(pl);
    pl->profiling = enable != 0;
    if (pl->profiling) pl->prof.resize(pl->buckets.size());
    return LADL_OK;
}

int ladl_plan_profile_read(ladl_plan_t pl, float *ms, int32_t *launches, int32_t max_buckets, int32_t *num_buckets)
{
    if (!pl || !ms || !launches || !num_buckets) return fail(LADL_EINVAL, "a required pointer is NULL");
    const int nb = (int)pl->buckets.size();
    *num_buckets = nb;
    if (max_buckets < nb) return fail(LADL_EINVAL, "max_buckets %d < %d buckets", max_buckets, nb);
    for (int bi = 0; bi < nb; ++bi) {
        double acc = 0.0;
        int cnt = 0;
        if (bi < (int)pl->prof.size())
            for (auto &ev : pl->prof[bi]) {
                float t = 0.f;
                hipError_t e = hipEventSynchronize(ev.second);
                if (e == hipSuccess) e = hipEventElapsedTime(&t, ev.first, ev.second);
                if (e != hipSuccess) return hipfail(e, "profiling event");
                acc += t;
                ++cnt;
            }
        ms[bi] = (float)acc;
        launches[bi] = cnt;
    }
    return LADL_OK;
}

int ladl_plan_describe(ladl_plan_t pl, char *buf, int64_t len)
{
    if (!pl || !buf || len < 1) return fail(LADL_EINVAL, "bad arguments");
    std::string s;
    char line[256];
    snprintf(line, sizeof line, "problems=%d solves=%d path_len=%d nmax=%d pmax=%d b_len=%lld\n", pl->P, pl->S,
             pl->L, pl->nmax, pl->pmax, (long long)pl->b_len);
    s += line;
    for (const Bucket &b : pl->buckets) {
        char place[64];
        if (b.xg)
            snprintf(place, sizeof place, "HBM workspace, %d columns in LDS%s", b.nlds, b.dense ? " (dense)" : "");
        else
            snprintf(place, sizeof place, "LDS");
        char tile[64];
        if (b.tile)
            snprintf(tile, sizeof tile, "tile=%dx%d grid=%d", b.tile_s, b.tile_rs, b.tile_grid);
        else
            snprintf(tile, sizeof tile, "tile=%s", b.tile_ok ? "off" : "none");
        snprintf(line, sizeof line,
                 "bucket R=%d (n<=%d) pmax=%d solves=%d grid=%d (%d/CU) waves/solve=%d X in %s lds=%zuB %s\n",
                 b.R, 64 * b.R, b.pmax, b.count, b.grid, b.per_cu, b.tw, place,
                 wave_lds_bytes(b.R / b.tw, b.pmax, b.xg, b.nlds, b.tw), tile);
        s += line;
    }
    std::strncpy(buf, s.c_str(), (size_t)len - 1);
    buf[len - 1] = 0;
    return LADL_OK;
}


// --------------------------------------------------------------------------
// K-fold cross-validation along a lambda path
// --------------------------------------------------------------------------
struct ladl_cv_s {
    int P = 0, K = 0, L = 0, Q = 0;
    int64_t x_len = 0, y_len = 0;
    ladl_plan_t inner = nullptr; // one solve per training problem
    int64_t *d_row_off_b = nullptr, *d_x_off_b = nullptr, *d_tr_off = nullptr, *d_va_off = nullptr;
    int64_t *d_x_off_tr = nullptr, *d_b_off_tr = nullptr;
    int32_t *d_p_b = nullptr, *d_tr_rows = nullptr, *d_va_rows = nullptr;
    float *d_Xtr = nullptr, *d_ytr = nullptr, *d_lamtr = nullptr, *d_b = nullptr, *d_obj = nullptr;
    float *d_ferr = nullptr;
    uint32_t *d_act = nullptr;
    int32_t *d_zr = nullptr, *d_st = nullptr;
};

static void cv_free(ladl_cv_s *cv)
{
    if (cv->inner) ladl_plan_destroy(cv->inner);
    void *ptrs[] = {cv->d_row_off_b, cv->d_x_off_b, cv->d_tr_off, cv->d_va_off, cv->d_x_off_tr, cv->d_b_off_tr,
                    cv->d_p_b,       cv->d_tr_rows,  cv->d_va_rows, cv->d_Xtr,   cv->d_ytr,     cv->d_lamtr,
                    cv->d_b,         cv->d_obj,      cv->d_ferr,    cv->d_act,   cv->d_zr,      cv->d_st};
    for (void *q : ptrs) (void)hipFree(q);
    delete cv;
}

template <typename T>
static hipError_t dalloc(T **dst, int64_t count)
{
    return hipMalloc((void **)dst, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
}

int ladl_cv_create(ladl_handle_t h, const ladl_cv_layout *lay, const ladl_options *opt, ladl_cv_t *out)
{
    if (!out) return fail(LADL_EINVAL, "output pointer is NULL");
    *out = nullptr;
    if (!h || !lay || !lay->row_off) return fail(LADL_EINVAL, "handle, layout and row_off are required");
    const int P = lay->num_problems, K = lay->folds, L = lay->path_len;
    if (P < 1) return fail(LADL_EINVAL, "num_problems = %d", P);
    if (K < 2 || K > 64) return fail(LADL_EINVAL, "folds = %d (must be 2..64)", K);
    if (L < 1 || L > 64) return fail(LADL_EINVAL, "path_len = %d (must be 1..64)", L);
    std::vector<int64_t> row_off(lay->row_off, lay->row_off + P + 1), x_off(P);
    std::vector<int32_t> pb(P);
    if (row_off[0] != 0) return fail(LADL_EINVAL, "row_off[0] must be 0");
    for (int k = 0; k < P; ++k) {
        const int64_t n = row_off[k + 1] - row_off[k];
        if (n < 1) return fail(LADL_EINVAL, "problem %d has %lld rows", k, (long long)n);
        const int pk = lay->p ? lay->p[k] : lay->p_uniform;
        if (pk < 1 || pk > PMAX) return fail(LADL_EUNSUPPORTED, "problem %d has p = %d (limit 1..%d)", k, pk, PMAX);
        const int64_t xo = lay->x_off ? lay->x_off[k] : row_off[k] * (int64_t)lay->p_uniform;
        if (xo < 0 || xo + n * pk > lay->x_len)
            return fail(LADL_EINVAL, "problem %d: X block outside x_len %lld", k, (long long)lay->x_len);
        pb[k] = pk;
        x_off[k] = xo;
    }
    if (row_off[P] > lay->y_len) return fail(LADL_EINVAL, "row_off[%d] exceeds y_len", P);
    // fold lists
    const int Q = P * K;
    std::vector<int64_t> tr_off(Q + 1, 0), va_off(Q + 1, 0), x_off_tr(Q, 0), b_off_tr(Q, 0);
    std::vector<int32_t> tr_rows, va_rows, p_tr(Q);
    tr_rows.reserve((size_t)row_off[P] * (K - 1));
    va_rows.reserve((size_t)row_off[P]);
    int64_t xacc = 0, bacc = 0;
    for (int k = 0; k < P; ++k) {
        const int n = (int)(row_off[k + 1] - row_off[k]);
        std::vector<int> lab(n);
        for (int i = 0; i < n; ++i) {
            lab[i] = lay->fold_of_row ? lay->fold_of_row[row_off[k] + i] : i % K;
            if (lab[i] < 0 || lab[i] >= K)
                return fail(LADL_EINVAL, "fold_of_row[%lld] = %d outside 0..%d", (long long)(row_off[k] + i), lab[i],
                            K - 1);
        }
        for (int f = 0; f < K; ++f) {
            const int q = k * K + f;
            for (int i = 0; i < n; ++i) (lab[i] == f ? va_rows : tr_rows).push_back(i);
            tr_off[q + 1] = (int64_t)tr_rows.size();
            va_off[q + 1] = (int64_t)va_rows.size();
            const int64_t ntr = tr_off[q + 1] - tr_off[q];
            if (ntr < 1) return fail(LADL_EINVAL, "fold %d of problem %d leaves no training rows", f, k);
            p_tr[q] = pb[k];
            x_off_tr[q] = xacc;
            b_off_tr[q] = bacc;
            xacc += ntr * pb[k];
            bacc += pb[k];
        }
    }
    auto *cv = new (std::nothrow) ladl_cv_s;
    if (!cv) return fail(LADL_ENOMEM, "host allocation");
    cv->P = P;
    cv->K = K;
    cv->L = L;
    cv->Q = Q;
    cv->x_len = xacc;
    cv->y_len = tr_off[Q];
    ladl_layout il{};
    il.num_problems = Q;
    il.row_off = tr_off.data();
    il.x_off = x_off_tr.data();
    il.p = p_tr.data();
    il.p_uniform = p_tr[0];
    il.x_len = xacc;
    il.y_len = tr_off[Q];
    il.num_solves = Q;
    il.problem = nullptr;
    il.path_len = L;
    il.lambda_hint = nullptr;
    int rc = ladl_plan_create(h, &il, opt, &cv->inner);
    if (rc != LADL_OK) {
        cv->inner = nullptr;
        std::string d = g_detail;
        cv_free(cv);
        return fail(rc, "training problems: %s", d.c_str());
    }
    const int64_t nout = (int64_t)Q * L;
    hipError_t e;
    if ((e = upload(&cv->d_row_off_b, row_off)) != hipSuccess || (e = upload(&cv->d_x_off_b, x_off)) != hipSuccess ||
        (e = upload(&cv->d_p_b, pb)) != hipSuccess || (e = upload(&cv->d_tr_off, tr_off)) != hipSuccess ||
        (e = upload(&cv->d_va_off, va_off)) != hipSuccess || (e = upload(&cv->d_x_off_tr, x_off_tr)) != hipSuccess ||
        (e = upload(&cv->d_b_off_tr, b_off_tr)) != hipSuccess ||
        (e = upload(&cv->d_tr_rows, tr_rows.empty() ? std::vector<int32_t>(1, 0) : tr_rows)) != hipSuccess ||
        (e = upload(&cv->d_va_rows, va_rows.empty() ? std::vector<int32_t>(1, 0) : va_rows)) != hipSuccess ||
        (e = dalloc(&cv->d_Xtr, xacc)) != hipSuccess || (e = dalloc(&cv->d_ytr, tr_off[Q])) != hipSuccess ||
        (e = dalloc(&cv->d_lamtr, nout)) != hipSuccess || (e = dalloc(&cv->d_b, bacc * L)) != hipSuccess ||
        (e = dalloc(&cv->d_obj, nout)) != hipSuccess || (e = dalloc(&cv->d_ferr, nout)) != hipSuccess ||
        (e = dalloc(&cv->d_act, nout)) != hipSuccess || (e = dalloc(&cv->d_zr, nout * ZPAD)) != hipSuccess ||
        (e = dalloc(&cv->d_st, nout)) != hipSuccess) {
        cv_free(cv);
        return hipfail(e, "cross-validation buffers");
    }
    *out = cv;
    return LADL_OK;
}

int ladl_cv_destroy(ladl_cv_t cv)
{
    if (cv) cv_free(cv);
    return LADL_OK;
}

int ladl_cv_run(ladl_cv_t cv, const float *X, const float *y, const float *lam, float *fold_error, float *cv_error,
                int32_t *best, int32_t *fold_status, void *stream)
{
    if (!cv) return fail(LADL_EINVAL, "cross-validation object is NULL");
    if (!X || !y || !lam || !cv_error || !best) return fail(LADL_EINVAL, "a required device pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    CvArgs a;
    std::memset(&a, 0, sizeof a);
    a.X = X;
    a.y = y;
    a.lam = lam;
    a.row_off_b = cv->d_row_off_b;
    a.x_off_b = cv->d_x_off_b;
    a.p_b = cv->d_p_b;
    a.num_base = cv->P;
    a.folds = cv->K;
    a.path_len = cv->L;
    a.num_train = cv->Q;
    a.tr_rows = cv->d_tr_rows;
    a.va_rows = cv->d_va_rows;
    a.tr_off = cv->d_tr_off;
    a.va_off = cv->d_va_off;
    a.x_off_tr = cv->d_x_off_tr;
    a.b_off_tr = cv->d_b_off_tr;
    a.Xtr = cv->d_Xtr;
    a.ytr = cv->d_ytr;
    a.lam_tr = cv->d_lamtr;
    a.b = cv->d_b;
    a.fold_err = fold_error ? fold_error : cv->d_ferr;
    a.cv_err = cv_error;
    a.best = best;
    hipError_t e = launch_cv_gather(a, s);
    if (e != hipSuccess) return hipfail(e, "cross-validation gather");
    int rc = ladl_solve_f32(cv->inner, cv->d_Xtr, cv->d_ytr, cv->d_lamtr, nullptr, cv->d_b, cv->d_obj, cv->d_act,
                            cv->d_zr, fold_status ? fold_status : cv->d_st, nullptr, stream);
    if (rc != LADL_OK) return rc;
    e = launch_cv_score(a, s);
    if (e != hipSuccess) return hipfail(e, "cross-validation scoring");
    return LADL_OK;
}

// --------------------------------------------------------------------------
// Exact solve by vertex enumeration (small problems)
// --------------------------------------------------------------------------
int ladl_brute_force_f32(ladl_plan_t pl, const float *X, const float *y, const float *lam, float *b, float *obj,
                         int64_t *vertices, void *stream)
{
    if (!pl) return fail(LADL_EINVAL, "plan is NULL");
    if (!X || !y || !lam || !b || !obj) return fail(LADL_EINVAL, "a required device pointer is NULL");
    for (int s = 0; s < pl->S; ++s) {
        const int k = pl->problem[s];
        const int n = (int)(pl->row_off[k + 1] - pl->row_off[k]), p = pl->p[k];
        if (p > 8 || n + p > 64)
            return fail(LADL_EUNSUPPORTED, "solve %d: n = %d, p = %d (vertex enumeration needs p <= 8, n + p <= 64)",
                        s, n, p);
        double c = 1.0;
        for (int j = 1; j <= p; ++j) c = c * (n + j) / j;
        if (c > 2147483647.0)
            return fail(LADL_EUNSUPPORTED, "solve %d: C(%d, %d) vertices exceed 2^31", s, n + p, p);
    }
    if (!pl->d_bf_order && pl->S > 0) {
        std::vector<int32_t> ord;
        ord.reserve(pl->S);
        pl->bf_buckets.clear();
        for (int p = 1; p <= 8; ++p) {
            int cnt = 0;
            for (int s = 0; s < pl->S; ++s)
                if (pl->p[pl->problem[s]] == p) {
                    ord.push_back(s);
                    ++cnt;
                }
            if (cnt) pl->bf_buckets.push_back({p, cnt});
        }
        hipError_t e = upload(&pl->d_bf_order, ord);
        if (e != hipSuccess) {
            pl->d_bf_order = nullptr;
            return hipfail(e, "vertex enumeration order");
        }
    }
    hipStream_t st = (hipStream_t)stream;
    int off = 0;
    for (const auto &bk : pl->bf_buckets) {
        BruteArgs a;
        std::memset(&a, 0, sizeof a);
        a.X = X;
        a.y = y;
        a.lam = lam;
        a.row_off = pl->d_row_off;
        a.x_off = pl->d_x_off;
        a.b_off = pl->d_b_off;
        a.problem = pl->d_problem;
        a.order = pl->d_bf_order + off;
        a.count = bk.second;
        a.path_len = pl->L;
        a.b_out = b;
        a.obj_out = obj;
        a.vert_out = vertices;
        hipError_t e = launch_brute(bk.first, a, st);
        if (e != hipSuccess) return hipfail(e, "vertex enumeration launch");
        off += bk.second;
    }
    return LADL_OK;
}

// --------------------------------------------------------------------------
// Subset-stability statistics over a plan's outputs
// --------------------------------------------------------------------------
int ladl_selection_frequency(ladl_plan_t pl, const uint32_t *active, const int32_t *status, const int32_t *group,
                             int32_t num_groups, int32_t *counts, float *freq, int32_t *bad_group, void *stream)
{
    if (!pl) return fail(LADL_EINVAL, "plan is NULL");
    if (!active || !status || !counts || !freq || !bad_group)
        return fail(LADL_EINVAL, "a required device pointer is NULL");
    if (num_groups < 1) return fail(LADL_EINVAL, "num_groups = %d", num_groups);
    hipError_t e = launch_selection_frequency(active, status, group, pl->S, pl->L, num_groups, counts, freq,
                                              bad_group, (hipStream_t)stream);
    if (e != hipSuccess) return hipfail(e, "selection frequency launch");
    return LADL_OK;
}

// --------------------------------------------------------------------------
// helpers for the other host source files (ladl_host.hpp)
// --------------------------------------------------------------------------
namespace ladl {
int host_fail(int code, const char *msg) { return fail(code, "%s", msg); }
int host_hipfail(hipError_t e, const char *what) { return hipfail(e, what); }
int host_check_options(const ladl_options *o) { return check_options(o); }
DevOpt host_dev_opt(const ladl_options &o) { return dev_opt(o); }
} // namespace ladl
