/*
 * ladlasso.h - batched LAD-LASSO solver for AMD MI355X (gfx950).
 *
 * Each solve minimises, for one problem (X_k, y_k) and one lambda,
 *
 *     f(b) = sum_i |y_i - x_i . b| + lambda * sum_j |b_j|          (Abstract;
 *                                                   Sections 2.1, 2.2, 3.1)
 *
 * by the paper's coordinate descent: exact 1-D minimisation of f along one
 * axis at a time (Section 3.3; the 1-D section minimum is a weighted median
 * of the kinks r_i/x_ij + b_j, Section 3.5), then a ternary chop along the
 * locus of axis-wise minima with the chop axis held fixed in each sub-search
 * and the range extended until it brackets the minimum (Sections 3.5-3.6).
 * The end point is snapped to the vertex where p hyperplanes meet (Section
 * 3.2) and certified by the LP optimality (dual) conditions; when the
 * certificate fails, primal simplex steps along the edges of the vertex
 * finish the solve (an addition to the paper, counted in `iters`).
 *
 * Conventions
 *   - All functions are plain C.  `void* stream` is a hipStream_t (NULL =
 *     the null stream).
 *   - Arrays named "host" are read synchronously during the call and may be
 *     freed afterwards.  All other arrays are DEVICE pointers owned by the
 *     caller; the library never frees or retains them beyond the work it
 *     enqueues, and reads/writes them only from kernels on `stream`.
 *   - A return of LADL_OK from an enqueueing call means the work was
 *     enqueued; per-solve outcomes are reported in `status`.
 *   - Errors: negative return values; nothing is enqueued when a call
 *     fails validation.  ladl_error_string() names the code and
 *     ladl_last_error_detail() holds a message for the last failure of the
 *     calling thread.
 *   - Limits: 1 <= p_k <= 32, 1 <= n_k <= 2048.
 */
#ifndef LADLASSO_H
#define LADLASSO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
enum {
    LADL_OK = 0,
    LADL_EINVAL = -1,       /* bad argument or layout                        */
    LADL_EUNSUPPORTED = -2, /* valid but outside the limits above            */
    LADL_EHIP = -3,         /* a HIP runtime call failed                     */
    LADL_ENOMEM = -4        /* device or host allocation failed              */
};

/* per-solve status written to `status` */
enum {
    LADL_CERTIFIED = 0,    /* optimality certificate holds with margins the
                              fp32 computation resolves: the minimiser, Z
                              and S are unique.  Margins: 1 - |u_i| > 2e-5 on
                              Z; (lambda - |c_j|) / (lambda + sum_{i in Z}
                              |x_ij|) > 2e-5 off S; |r_i| / (|y_i| + sum_j
                              |x_ij b_j|) > 1e-6 off Z                       */
    LADL_NONUNIQUE = 1,    /* certificate holds, but a margin is below those
                              thresholds (a degenerate or nearly degenerate
                              vertex): f is optimal, b may not be the only
                              minimiser                                      */
    LADL_MAXITER = 2,      /* finisher pivot cap reached before certifying   */
    LADL_NONFINITE = 3,    /* NaN or Inf in this problem's X or y            */
    LADL_BADLAMBDA = 4,    /* lambda < 0 or NaN                              */
    LADL_NOTCERTIFIED = 5  /* no certificate: a singular vertex system, or
                              the finisher (and its perturbed retry) ended
                              without one; the best point is returned       */
};

/* option flags */
enum {
    LADL_FLAG_GOLDEN = 1,       /* golden-section split of the ternary
                                   chop's bracket instead of thirds: the same
                                   search (same bracket invariant and limit)
                                   with one interior probe carried over per
                                   step, so about half the probes; set in
                                   the default options (clear it for
                                   thirds)                                   */
    LADL_FLAG_NO_FINISHER = 2,  /* stop after the paper's stages             */
    LADL_FLAG_NO_SNAP = 4,      /* no vertex snap/certificate: b is the last
                                   coordinate-descent point, status MAXITER  */
    LADL_FLAG_QUADRATURE = 8    /* the paper's second variant (Sections 1,
                                   3.5, 5): every 1-D section is minimised
                                   by a quadrature search of its values
                                   (bracket [smallest kink, largest kink],
                                   halved around the lowest of its three
                                   quarter points until its width is at most
                                   2^-22 (1 + |lo| + |hi|); the point is kept
                                   only if it lowers f) instead of the exact
                                   weighted median.  The chop, the snap and
                                   the certificate are unchanged, so results
                                   are certified as before; the search costs
                                   about 25 passes over the column per
                                   update instead of one or two              */
};

typedef struct {
    float tol_f;         /* CCD stops after a sweep that changes nothing or
                            lowers f by <= tol_f * f          (default 1e-6)  */
    float tol_s;         /* ternary chop stops at hi - lo <= tol_s *
                            (1 + |lo| + |hi|)                 (default 2^-20) */
    float lambda_min;    /* effective lambda = max(lambda, lambda_min); the
                            paper's tie-breaking minimum (Section 3.6)
                                                              (default 0)     */
    int32_t max_sweeps;  /* sweeps per CCD run (a cap on the rare slowly
                            zig-zagging probes; the certificate and the
                            finisher do not depend on it)     (default 8)     */
    int32_t max_ternary; /* chop iterations per round         (default 48)    */
    int32_t max_rounds;  /* chop rounds, each on the next axis: 0 none,
                            -1 one per axis                   (default 1)     */
    int32_t max_pivots;  /* finisher pivots; <= 0 means 4p + 32 (default 0)   */
    int32_t flags;       /* LADL_FLAG_*          (default LADL_FLAG_GOLDEN)   */
    int32_t schedule;    /* -1: per bucket, X in LDS when it fits 40 KB per
                            wave, else in an HBM workspace, and for
                            n <= 256 with more than two grids' worth of
                            solves the HBM workspace with the kernel
                            variant built for 4 waves per SIMD
                            (ladl_autotune may change the choice);
                            0: the HBM workspace for every bucket;
                            1: as 0, with the 4-wave variant wherever
                            n <= 256.  With the workspace, the leading
                            columns of X that fit the LDS left over at
                            the kernel's occupancy stay in LDS (when the
                            plan has one bucket, or for n > 1024)
                                                              (default -1)    */
    float chop_range;    /* initial half-width of the chop's range around
                            b_k, as a fraction of max(1, |b_k|); the range
                            is doubled while an end is lower than the
                            centre (Section 3.6)               (default 1/32) */
    int32_t team;        /* waves per solve for problems of n > 1024: 0 the
                            library's choice (ladl_autotune may change it),
                            1 one wavefront, 2 or 4 a team of that many
                            wavefronts of one workgroup, the rows split
                            between them; smaller problems always take one
                            wavefront                          (default 0)    */
    int32_t tile;        /* tile schedule for problems of n <= 64: 0 the
                            library's choice (off unless ladl_autotune
                            measures it faster), 1 off, 2 on.  On, the
                            coordinate descent (Sections 3.3-3.4) of each
                            path step first runs with 4 problems per
                            wavefront (n <= 32, segments of 16 lanes) or 2
                            (n <= 64, 32 lanes) and stops at its first
                            axis-wise minimum; the wavefront kernel then
                            starts each step from that point and runs the
                            rest of the solve.  Results are certified as
                            without it, but may be a different optimal
                            vertex where the optimum is not unique, and
                            `iters` counts the wavefront stage's work only.
                            Excludes LADL_FLAG_QUADRATURE (EINVAL with 2;
                            never chosen with 0)               (default 0)    */
} ladl_options;

/*
 * Batch layout (HOST arrays).  Problem k has n_k = row_off[k+1] - row_off[k]
 * rows and p_k features; its X block is row-major n_k x p_k at
 * X + x_off[k], its y at y + row_off[k].  Solve s runs problem problem[s]
 * along a lambda path of path_len values lambda[s*path_len + t] (t = 0 ..
 * path_len-1), each step warm-started from the previous one.
 * Outputs of (s, t): b at b + path_len*b_off[s] + t*p_s where b_off is the
 * exclusive prefix sum of p over solves; the scalars at index
 * s*path_len + t; zero_rows at 32*(s*path_len + t).
 */
typedef struct {
    int32_t num_problems;
    const int64_t *row_off; /* host [num_problems+1], row_off[0] = 0, non-decreasing */
    const int64_t *x_off;   /* host [num_problems] or NULL: row_off[k] * p_uniform     */
    const int32_t *p;       /* host [num_problems] or NULL: p_uniform                  */
    int32_t p_uniform;
    int64_t x_len;          /* number of floats in X (bounds check)                    */
    int64_t y_len;          /* number of floats in y (bounds check)                    */
    int32_t num_solves;
    const int32_t *problem; /* host [num_solves] or NULL: solve s uses problem s       */
    int32_t path_len;       /* >= 1                                                    */
    const float *lambda_hint; /* host [num_solves * path_len] or NULL: the lambda values
                                 the plan will mostly be run with; used only to order
                                 the work queue (among solves of equal n*p, smaller
                                 lambda first: those take longer), never read on the
                                 device and not required to match later calls       */
} ladl_layout;

typedef struct ladl_handle_s *ladl_handle_t;
typedef struct ladl_plan_s *ladl_plan_t;
typedef struct ladl_graph_s *ladl_graph_t;

/* Create a handle bound to the calling thread's current HIP device. */
int ladl_create(ladl_handle_t *handle);
int ladl_destroy(ladl_handle_t handle);

void ladl_default_options(ladl_options *opt);

/*
 * Validate a layout and build a plan: per-solve metadata uploaded to the
 * device, solves bucketed by rows per lane and sorted by decreasing cost
 * (n_k * p_k, then increasing lambda when lambda_hint is given) for the
 * persistent work queue, and the schedule chosen.  The plan owns device
 * memory: the metadata, the queue counters, a workspace for buckets whose X
 * is not held in LDS (all or part of it, per the schedule), and (when every
 * problem is used by exactly one solve)
 * 128 bytes per solve for the backward.  Calls on one plan share these, so
 * calls on the same plan must not run concurrently on different streams;
 * calls in stream order are fine.
 * Synchronous.  The plan keeps its own copies; layout arrays may be freed.
 */
int ladl_plan_create(ladl_handle_t handle, const ladl_layout *layout, const ladl_options *opt,
                     ladl_plan_t *plan);
int ladl_plan_destroy(ladl_plan_t plan);
/* total floats of one b output array (all solves, all path steps) */
int64_t ladl_plan_b_len(ladl_plan_t plan);

/*
 * Forward solve (the wavefront-per-solve persistent kernels): for every
 * (solve, path step), minimise f(b) = sum_i |y_i - x_i.b| + lambda ||b||_1
 * (the LAD-LASSO objective of the Abstract and Sections 2.1, 2.2, 3.1) by
 * cyclic coordinate descent with exact 1-D section minima (Sections 3.3,
 * 3.5; or the quadrature search with LADL_FLAG_QUADRATURE), the ternary
 * chop along the locus of axis-wise minima (Sections 3.5, 3.6), then the
 * vertex snap, certificate and finisher (Section 3.2's vertex form; the
 * finisher is this library's addition).  Along a path each step starts
 * from the previous step's answer (Section 5's regularisation paths).
 *   X, y       device, layout as described by the plan
 *   lambda     device [num_solves * path_len]
 *   b_init     device, packed like one path step of b (p_s floats per solve
 *              at b_off[s]), or NULL for zeros: starting point of step 0
 *   b          device [ladl_plan_b_len]          (output)
 *   obj        device [num_solves*path_len]      f(b) in fp32 (output)
 *   active     device [num_solves*path_len]      bit j set iff b_j != 0 (output)
 *   zero_rows  device [32*num_solves*path_len]   the vertex's zero-residual
 *              rows (local ids, ascending, -1 padded) (output)
 *   status     device [num_solves*path_len]      LADL_CERTIFIED ... (output)
 *   iters      device [4*num_solves*path_len] or NULL: CCD sweeps, coordinate
 *              updates, ternary probes, finisher pivots (output)
 */
int ladl_solve_f32(ladl_plan_t plan, const float *X, const float *y, const float *lambda,
                   const float *b_init, float *b, float *obj, uint32_t *active, int32_t *zero_rows,
                   int32_t *status, int32_t *iters, void *stream);

/* The same solve by a plain kernel with one GPU thread per solve and X read
 * from global memory: the paper's coarse-parallel design (Abstract,
 * Section 5), kept as the speed baseline.  Same arguments and outputs. */
int ladl_solve_plain_f32(ladl_plan_t plan, const float *X, const float *y, const float *lambda,
                         const float *b_init, float *b, float *obj, uint32_t *active,
                         int32_t *zero_rows, int32_t *status, int32_t *iters, void *stream);

/*
 * Gradient of a loss L through the solution at path step `step` (usually
 * path_len - 1), using b_S = X_{Z,S}^{-1} y_Z at the optimal vertex:
 *   w = X_{Z,S}^{-T} g_S,  dL/dy_Z = w,  dL/dX_{Z,S} = -w b_S^T,
 * every other entry 0 (the vertex form of Section 3.2).  Every certified
 * output (LADL_CERTIFIED or LADL_NONUNIQUE) with |Z| = |S| > 0 and a
 * non-singular X_{Z,S} gets this gradient; at LADL_NONUNIQUE it is the
 * derivative of the returned vertex (one of the one-sided derivatives of
 * the solution map).  Outputs with b = 0, or without a certificate, get
 * zero gradients (b = 0 with a certificate is locally constant).
 *   b, zero_rows, status   device, the forward outputs (all steps)
 *   grad_b     device, packed like one path step of b
 *   grad_y     device, packed like y (output; all y_len floats written,
 *              zeros outside the vertex rows and outside every problem)
 *   grad_X     device, packed like X (output; all x_len floats written,
 *              likewise)
 * Every problem must be used by exactly one solve.
 */
int ladl_backward_f32(ladl_plan_t plan, const float *X, const float *b, const int32_t *zero_rows,
                      const int32_t *status, int32_t step, const float *grad_b, float *grad_y,
                      float *grad_X, void *stream);

/*
 * Lambda path as a HIP graph: path_len launches, one per path step, each
 * warm-started from the previous step's output (the regularisation path of
 * Section 5, computed step by step as ladl_solve_f32 computes it in one
 * launch; the outputs are bit-identical), captured once and replayed
 * by ladl_graph_launch.  The pointers are baked into the graph: refill the
 * same buffers to run new data of the same layout.
 */
int ladl_graph_create(ladl_plan_t plan, const float *X, const float *y, const float *lambda,
                      const float *b_init, float *b, float *obj, uint32_t *active, int32_t *zero_rows,
                      int32_t *status, int32_t *iters, ladl_graph_t *graph);
int ladl_graph_launch(ladl_graph_t graph, void *stream);
int ladl_graph_destroy(ladl_graph_t graph);

/*
 * Time each candidate schedule on this plan's own data (runs the solve
 * several times on `stream`, synchronously) and keep the fastest per
 * bucket in the plan: X resident in LDS, X in the HBM workspace, (for
 * n <= 256) X in the HBM workspace with the 4-waves-per-SIMD kernel
 * variant, (for n > 1024) teams of 2 or 4 wavefronts per solve, and (for
 * n <= 64, options.tile = 0) each of these with the tile stage in front,
 * for the buckets where more than one exists.  The paper leaves the mapping of
 * problems onto the hardware to the application (coarse parallelism,
 * Abstract and Section 5); this picks it by measurement.  The choice is
 * cached in the file named by the environment variable LADL_TUNE_CACHE (if
 * set), keyed by device, rows per lane and p_max.  Optional: plans start
 * with a static choice; a plan created with options.schedule = 0 or 1 is
 * left as it is.
 */
int ladl_autotune(ladl_plan_t plan, const float *X, const float *y, const float *lambda, float *b,
                  float *obj, uint32_t *active, int32_t *zero_rows, int32_t *status, void *stream);

/*
 * Kernel timing per bucket, for measuring the solve kernels on their own
 * streams (the buckets of a plan run side by side on streams forked from
 * the caller's).  ladl_plan_profile(plan, 1) drops earlier records and
 * starts recording: every later ladl_solve_f32 on the plan records a HIP
 * event pair on each bucket's stream around that bucket's kernel (graph
 * launches are not recorded); ladl_plan_profile(plan, 0) stops and drops
 * them.  ladl_plan_profile_read waits for the recorded events and writes,
 * per bucket in the order ladl_plan_describe lists them, the summed kernel
 * time in ms (host float [max_buckets]) and the number of launches (host
 * int32 [max_buckets]); *num_buckets receives the bucket count
 * (LADL_EINVAL if max_buckets is smaller).  Events are created per launch
 * while recording, so leave it off outside measurements.
 */
int ladl_plan_profile(ladl_plan_t plan, int32_t enable);
int ladl_plan_profile_read(ladl_plan_t plan, float *ms, int32_t *launches, int32_t max_buckets,
                           int32_t *num_buckets);

/* Describe the plan's buckets and schedules as text (host buffer). */
int ladl_plan_describe(ladl_plan_t plan, char *buf, int64_t buf_len);

const char *ladl_error_string(int code);
const char *ladl_last_error_detail(void);

/*
 * Exact solve by vertex enumeration (Section 3.2): every choice of p of the
 * n + p hyperplanes {x_i.b = y_i} and {b_j = 0} that meet in one point is
 * evaluated, and the point of least f is returned (the global minimum: f is
 * piecewise linear and attains its minimum at a vertex).  For the paper's
 * evaluation sizes: every solve of the plan needs p <= 8, n + p <= 64 and
 * C(n+p, p) <= 2^31, else LADL_EUNSUPPORTED.  Each (solve, path step) is
 * independent (no warm start).  Vertex systems and f in fp64; ties go to
 * the first vertex in lexicographic order of hyperplane indices (rows
 * 0..n-1, then axes n..n+p-1).
 *   b         device, packed as for ladl_solve_f32 (output)
 *   obj       device [num_solves*path_len]: the minimum f, NaN if no
 *             vertex exists (output)
 *   vertices  device int64 [num_solves*path_len] or NULL: non-singular
 *             vertices evaluated (output)
 * The plan's queue order and schedule are not used; the first call on a
 * plan uploads a per-p order of its solves.
 */
int ladl_brute_force_f32(ladl_plan_t plan, const float *X, const float *y, const float *lambda, float *b,
                         float *obj, int64_t *vertices, void *stream);

/*
 * Subset-stability statistics over a plan's outputs: the paper's end goal
 * of telling informative from non-informative variables by fitting many
 * row subsets (Sections 1 and 5).  Solve s belongs to group group[s]
 * (device int32 [num_solves], or NULL: all in group 0).  For group g, path
 * step t and feature j:
 *   counts[(g*path_len + t)*33 + j]  solves of g whose b_j at step t is
 *                                    non-zero (bit j of active), j < 32
 *   counts[(g*path_len + t)*33 + 32] solves of g counted (status
 *                                    LADL_CERTIFIED or LADL_NONUNIQUE)
 *   freq[(g*path_len + t)*32 + j]    their ratio (0 when none counted)
 * active, status: the outputs of a solve with this plan (device).  counts
 * (int32 [num_groups*path_len*33]) is the caller's and is overwritten.
 * bad_group (device int32 [1]) is set to 1 if a group id lies outside
 * [0, num_groups) (that solve is skipped), else 0.  Exact integer counts:
 * the result does not depend on the order of the solves.
 */
int ladl_selection_frequency(ladl_plan_t plan, const uint32_t *active, const int32_t *status,
                             const int32_t *group, int32_t num_groups, int32_t *counts, float *freq,
                             int32_t *bad_group, void *stream);

/*
 * K-fold cross-validation along a lambda path, all on the device: the
 * paper's interactive use of several regularisation settings solved while
 * cross-validating (Section 5).  For every base problem k and fold f, the
 * rows outside f form a training problem solved along the path (each step
 * warm-started from the previous one, same method and status codes as
 * ladl_solve_f32); the rows in f score every step's b by the held-out
 * absolute error  e[k,f,t] = sum_{i in f} |y_i - x_i . b_{k,f}(lambda_t)|
 * (fp32 residuals, fp64 sums).  The CV curve is cv[k,t] = sum_f e[k,f,t]
 * and best[k] is its first minimiser.
 *
 * The base layout is that of ladl_layout (one solve per problem).  Fold of
 * local row i of problem k: fold_of_row[row_off[k] + i] when given, else
 * i mod folds.  Every fold must leave at least one training row, and a
 * training problem obeys the solver's limits (n <= 2048, p <= 32).
 * The object owns device memory: the training problems' X and y (K - 1
 * times the base data), their solver plan and its outputs.  Calls on one
 * object run in stream order, not concurrently.  Solver options apply to
 * every training solve.
 */
typedef struct ladl_cv_s *ladl_cv_t;

typedef struct {
    int32_t num_problems;
    const int64_t *row_off;     /* host [num_problems+1], as in ladl_layout              */
    const int64_t *x_off;       /* host [num_problems] or NULL                           */
    const int32_t *p;           /* host [num_problems] or NULL: p_uniform                */
    int32_t p_uniform;
    int64_t x_len;              /* floats in X (bounds check)                            */
    int64_t y_len;              /* floats in y (bounds check)                            */
    int32_t folds;              /* K, 2 .. 64                                            */
    const int32_t *fold_of_row; /* host [row_off[num_problems]] or NULL: i mod K          */
    int32_t path_len;           /* L, 1 .. 64                                            */
} ladl_cv_layout;

int ladl_cv_create(ladl_handle_t handle, const ladl_cv_layout *layout, const ladl_options *opt,
                   ladl_cv_t *cv);
int ladl_cv_destroy(ladl_cv_t cv);

/*
 *   X, y        device, the base problems (as for ladl_solve_f32)
 *   lambda      device [num_problems * path_len], the path of each problem
 *   fold_error  device [num_problems * K * path_len] or NULL: e[k,f,t] at
 *               (k*K + f)*path_len + t (output)
 *   cv_error    device [num_problems * path_len]: cv[k,t] (output)
 *   best        device [num_problems]: first t minimising cv[k,t] (output)
 *   fold_status device [num_problems * K * path_len] or NULL: the solver
 *               status of each training solve, same indexing (output)
 * Enqueued on `stream`; nothing is synchronised.
 */
int ladl_cv_run(ladl_cv_t cv, const float *X, const float *y, const float *lambda, float *fold_error,
                float *cv_error, int32_t *best, int32_t *fold_status, void *stream);

/*
 * Allocation-free forward solve, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same solve, kernels and outputs as
 * ladl_solve_f32 on a uniform batch, without a plan: num_problems problems
 * of n rows and p features each, packed back to back (problem k's
 * row-major X block at X + k*n*p, its y at y + k*n), solve k runs problem
 * k along its lambda path lambda[k*path_len .. (k+1)*path_len), and the
 * outputs are laid out as ladl_solve_f32 lays them out (b of (k, t) at
 * b + (k*path_len + t)*p).  opt may be NULL (defaults); it is validated as
 * for a plan, and its schedule, team and tile fields are then ignored: one
 * wavefront per problem, X always held in LDS.
 *
 * Nothing is allocated and no library routine that allocates is called:
 * the work-queue counter and the per-problem metadata live in a fixed
 * device array of about 2.1 MB, one per GPU, held by the library until the
 * process ends, and rewritten by a kernel on `stream` at the start of every
 * call.  All calls on one GPU share that array, so calls that overlap in
 * time on one GPU (on different streams, or from different host threads)
 * race and must not be issued; calls in one stream's order are fine.
 * Limits (LADL_EUNSUPPORTED beyond them, nothing launched):
 * 1 <= num_problems <= LADL_NOALLOC_MAX_PROBLEMS, 1 <= n <=
 * LADL_NOALLOC_MAX_ROWS, 1 <= p <= 32, and one problem's X must fit the LDS
 * of a compute unit (every n <= 1024, p <= 32 does on MI355X).  Other
 * errors as for ladl_solve_f32.
 */
#define LADL_NOALLOC_MAX_PROBLEMS 65536
#define LADL_NOALLOC_MAX_ROWS 1024
int ladl_solve_uniform_noalloc_f32(int32_t num_problems, int32_t n, int32_t p, int32_t path_len,
                                   const ladl_options *opt, const float *X, const float *y, const float *lambda,
                                   const float *b_init, float *b, float *obj, uint32_t *active, int32_t *zero_rows,
                                   int32_t *status, int32_t *iters, void *stream);

#ifdef __cplusplus
}
#endif
#endif
