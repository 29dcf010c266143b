// Launch descriptors shared by the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ladl {

constexpr int PMAX = 32;     // features per problem
constexpr int NMAX = 2048;   // rows per problem (32 slots x 64 lanes)
constexpr int ZPAD = 32;     // zero_rows entries per output

struct DevOpt {
    float tol_f, tol_s, lambda_min;
    int max_sweeps, max_ternary, max_rounds, max_pivots, flags;
    float chop_range;
};

// One launch of the forward solve over a list of solves (one bucket).
struct SolveArgs {
    const float *X, *y, *lam, *b_init;
    const int64_t *row_off, *x_off, *b_off;
    const int32_t *p_arr, *problem;
    const int32_t *order; // solve ids of this bucket, decreasing cost
    int32_t num_items;
    int32_t path_len;
    int32_t t0, t1;       // path steps computed by this launch
    int32_t *counter;     // work-queue head (zeroed by k_reset before launch)
    float *b_out, *obj_out;
    uint32_t *active_out;
    int32_t *zrows_out, *status_out, *iters_out;
    float *gws;           // plain kernel: per-thread global scratch; wave kernel: per-team workspace
    int64_t gws_stride;   // floats per thread (plain) or per team (wave)
    DevOpt opt;
    int32_t pmax;         // largest p in the bucket (LDS carve-up)
    int32_t nlds;         // with the workspace: columns of X kept in LDS
    const float *b_seed;  // wave kernel, n <= 64: start of path step 0
                          // (laid out like b_out), or null
};

struct BackwardArgs {
    const float *X, *b, *grad_b;
    const int32_t *zrows, *status;
    const int64_t *row_off, *x_off, *b_off;
    const int32_t *p_arr, *problem;
    int32_t num_solves, path_len, step;
    float *grad_y, *grad_X;
    int64_t x_len, y_len; // floats of grad_X / grad_y, all written (zeros first)
    float *bw;            // 32 floats per solve: w of the vertex solve (NaN: none)
};

// K-fold cross-validation: training problem q = k*folds + f holds the rows
// of base problem k outside fold f (local indices tr_rows[tr_off[q] ..
// tr_off[q+1])); the rows in the fold are va_rows[va_off[q] .. va_off[q+1]).
struct CvArgs {
    const float *X, *y, *lam;            // base problems, lambda [P * path_len]
    const int64_t *row_off_b, *x_off_b;  // base layout
    const int32_t *p_b;
    int32_t num_base, folds, path_len, num_train;
    const int32_t *tr_rows, *va_rows;
    const int64_t *tr_off, *va_off, *x_off_tr, *b_off_tr;
    float *Xtr, *ytr, *lam_tr;           // packed training problems
    const float *b;                      // training solves' b (all steps)
    float *fold_err, *cv_err;
    int32_t *best;
};

// vertex enumeration: the solves in order[0 .. count) all have the same p
struct BruteArgs {
    const float *X, *y, *lam;
    const int64_t *row_off, *x_off, *b_off;
    const int32_t *problem, *order;
    int32_t count, path_len;
    float *b_out, *obj_out;
    int64_t *vert_out; // non-singular vertices examined per output, or null
};

// host-side launchers (defined with their kernels)
// wave kernel: Rt = rows per lane of the bucket (1..32, n <= 64 Rt); tw =
// waves per solve (a team of tw waves, each with Rt / tw row slots per
// lane); xg = X held in a per-team global workspace instead of LDS
// (required for Rt = 32), except its first nlds columns; dense = the
// variant compiled for 4 waves per SIMD (Rt <= 4 with xg, tw = 1); quad:
// the variant whose 1-D sections are minimised by the quadrature search
// (every combination exists in both forms).  LDS and workspace sizes take
// the per-wave R = Rt / tw.
size_t wave_lds_bytes(int R, int pmax, bool xg, int nlds, int tw);
size_t wave_ws_floats_host(int R, int pmax, int nlds, int tw);
bool wave_has_dense(int Rt);
bool wave_has_team(int Rt, int tw);
int wave_max_blocks_per_cu(int Rt, int pmax, bool xg, bool dense, int tw, bool quad, int nlds);
hipError_t launch_reset(int32_t *counters, int n, hipStream_t s);
hipError_t launch_wave(int Rt, bool xg, bool dense, int tw, bool quad, const SolveArgs &a, int grid, hipStream_t s);
hipError_t launch_plain(const SolveArgs &a, int NM, int64_t nthreads, hipStream_t s);
// tile kernel (n <= 64): segments of S lanes with RS row slots per lane, one
// solve per segment, 64 / S solves per one-wave workgroup.  Writes the end
// point of the descent and chop of path steps t0 .. t1 to a.b_out (the host
// runs it on step 0: the wave kernel's seed).
bool tile_shape_for(int nmax, int &S, int &RS);
size_t tile_lds_bytes(int S, int RS, int pmax);
int tile_solves_per_block(int S);
int tile_max_blocks_per_cu(int S, int RS, int pmax);
hipError_t launch_tile(int S, int RS, const SolveArgs &a, int grid, hipStream_t s);
int64_t plain_scratch_floats(int NM, int64_t nthreads);
hipError_t launch_backward(const BackwardArgs &a, hipStream_t s);
hipError_t launch_cv_gather(const CvArgs &a, hipStream_t s);
hipError_t launch_cv_score(const CvArgs &a, hipStream_t s);
hipError_t launch_brute(int p, const BruteArgs &a, hipStream_t s);
hipError_t launch_selection_frequency(const uint32_t *active, const int32_t *status, const int32_t *group,
                                      int32_t num_solves, int32_t path_len, int32_t num_groups, int32_t *counts,
                                      float *freq, int32_t *bad_group, hipStream_t s);

} // namespace ladl
