// Definitions shared by the wavefront kernel and the plain kernel:
// option flags, status codes, certificate tolerances, and the ternary-chop
// state machine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ladl_kernels.hpp"

namespace ladl {

constexpr float FINF_C = __builtin_inff();

constexpr int FLAG_GOLDEN = 1, FLAG_NO_FINISHER = 2, FLAG_NO_SNAP = 4, FLAG_QUADRATURE = 8;
enum { ST_CERTIFIED = 0, ST_NONUNIQUE = 1, ST_MAXITER = 2, ST_NONFINITE = 3, ST_BADLAMBDA = 4, ST_NOTCERT = 5 };

// optimality certificate slack: the dual sums are accumulated in fp64 and
// the dual solve is refined with fp64 residuals, so u and c carry errors of
// order 1e-6; the slack only has to absorb that
constexpr float TOL_U = 2e-5f;   // |u_i| <= 1 + TOL_U on Z
constexpr float TOL_C = 2e-5f;   // |c_j| <= lambda (1 + TOL_C) + TOL_CA * sum_i |x_ij| off S
constexpr float TOL_CA = 1e-8f;
// Margins below which a certified vertex is reported as possibly
// non-unique, each against the fp32 error of the quantity it bounds:
//   1 - max|u_Z| > MARGIN_U          (u_Z refined to ~1e-7 relative)
//   (lambda - |c_j|) / (lambda + sum_{i in Z} |x_ij|) > MARGIN_C, j off S
//                                    (c_j takes the error of u_Z through
//                                     the vertex rows' entries only; the
//                                     other rows enter through exact signs)
//   |r_i| / (|y_i| + sum_j |x_ij b_j|) > MARGIN_R, rows off Z
//                                    (b rounded to fp32 moves r_i by about
//                                     2^-24 sum_j |x_ij b_j|)
// so a margin above the threshold is resolved by the fp32 computation with
// a factor of 10 or more to spare.
constexpr float MARGIN_U = 2e-5f, MARGIN_C = 2e-5f, MARGIN_R = 1e-6f;

constexpr int ALD = 33; // leading dimension of the vertex matrix
// finisher steps that fail to lower f after which Bland's rule is kept
constexpr int STALLS_STICKY = 4;
constexpr int REFINE_MAX = 8; // refinement steps of the vertex and dual solves

#define LADL_INL __device__ __attribute__((always_inline)) inline

// Quadrature search of a 1-D section (the paper's second coordinate-descent
// variant, Sections 1, 3.5 and 5): the bracket [smallest kink, largest kink]
// is halved around the lowest of its three quarter points until its width
// is at most QUAD_TOL (1 + |lo| + |hi|), or QUAD_MAX halvings.  QUAD_TOL is
// 2^-22: a few units in the last place of fp32, below which the fp32 sums
// of the section values no longer order the points reliably.
constexpr float QUAD_TOL = 2.384185791015625e-07f;
constexpr int QUAD_MAX = 64;


// deterministic perturbation direction of row i for degenerate vertices:
// magnitude in [0.5, 1], sign from the hash
LADL_INL float perturb_dir(int i)
{
    uint32_t h = (uint32_t)i * 2654435761u;
    float mag = 0.5f + 0.5f * (float)((h >> 8) & 0xFFFFu) * (1.f / 65535.f);
    return (h >> 31) ? -mag : mag;
}
constexpr float PERTURB_REL = 1.52587890625e-05f; // 2^-16

// --------------------------------------------------------------------------
// H6: ternary chop along axis kax (Sections 3.5-3.6), as a state machine fed
// with one probe value F(s) at a time so that the solve has a single CCD
// call site.  F(s) = f after CCD with b_kax := s and axis kax frozen,
// started from the best point found so far.  The centre c = b_kax is
// probed first: the start point is on the locus of axis-wise minima only
// when the CCD before the chop converged, which a sweep cap can prevent,
// and the bracket test below needs F(c) itself.  The range c +- h,
// h = chop_range * max(1,|c|) (the paper leaves the initial range open and
// extends it until it holds the minimum), is doubled outward while an end
// is lower than the centre (clamped to
// |b_kax| <= ||y||_1 / lambda, which bounds every minimiser), then cut in
// thirds (or golden sections) keeping the better side.
// --------------------------------------------------------------------------
struct Chop {
    float lo, hi, c, h, B, Fc, Flo, Fhi, m1, m2, F1, F2;
    int stage, which, ext, it;
    bool have1, have2;
};

LADL_INL void chop_init(Chop &q, float c, float f, float B, float range)
{
    q.B = B;
    q.c = c;
    q.h = range * fmaxf(1.f, fabsf(c));
    q.lo = fmaxf(c - q.h, -B);
    q.hi = fminf(c + q.h, B);
    q.Fc = f;
    q.Flo = q.Fhi = q.F1 = q.F2 = FINF_C;
    q.m1 = q.m2 = 0.f;
    q.stage = -1;
    q.which = 0;
    q.ext = 0;
    q.it = 0;
    q.have1 = q.have2 = false;
}

// Record the value of the last requested probe (when which != 0) and return
// the next probe point in s; false when the chop is finished.
LADL_INL bool chop_next(Chop &q, float F, float &s, const DevOpt &opt)
{
    switch (q.which) {
    case 1: q.Flo = F; break;
    case 2: q.Fhi = F; break;
    case 3: q.F1 = F; q.have1 = true; break;
    case 4: q.F2 = F; q.have2 = true; break;
    case 5: q.Fc = F; break;
    default: break;
    }
    const bool golden = (opt.flags & FLAG_GOLDEN) != 0;
    const float g = 0.381966011f;
    for (int guard = 0; guard < 8; ++guard) {
        switch (q.stage) {
        case -1: // F(c)
            q.stage = 0;
            q.which = 5;
            s = q.c;
            return true;
        case 0: // F(lo)
            q.stage = 1;
            q.which = 1;
            s = q.lo;
            return true;
        case 1: // F(hi)
            q.stage = 2;
            q.which = 2;
            s = q.hi;
            return true;
        case 2: // extend to the left while F(lo) < F(c)
            if (q.Flo < q.Fc && q.lo > -q.B && q.ext < 64) {
                q.hi = q.c;
                q.Fhi = q.Fc;
                q.c = q.lo;
                q.Fc = q.Flo;
                q.h *= 2.f;
                q.lo = fmaxf(q.c - q.h, -q.B);
                ++q.ext;
                q.which = 1;
                s = q.lo;
                return true;
            }
            q.stage = 3;
            break;
        case 3: // extend to the right while F(hi) < F(c)
            if (q.Fhi < q.Fc && q.hi < q.B && q.ext < 128) {
                q.lo = q.c;
                q.Flo = q.Fc;
                q.c = q.hi;
                q.Fc = q.Fhi;
                q.h *= 2.f;
                q.hi = fminf(q.c + q.h, q.B);
                ++q.ext;
                q.which = 2;
                s = q.hi;
                return true;
            }
            q.stage = 4;
            break;
        default: // chop
            if (q.have1 && q.have2) {
                if (q.F1 < q.F2) {
                    q.hi = q.m2;
                    if (golden) {
                        q.m2 = q.m1;
                        q.F2 = q.F1;
                        q.have1 = false;
                    } else {
                        q.have1 = q.have2 = false;
                    }
                } else {
                    q.lo = q.m1;
                    if (golden) {
                        q.m1 = q.m2;
                        q.F1 = q.F2;
                        q.have2 = false;
                    } else {
                        q.have1 = q.have2 = false;
                    }
                }
                ++q.it;
            }
            if (q.hi - q.lo <= opt.tol_s * (1.f + fabsf(q.lo) + fabsf(q.hi)) || q.it >= opt.max_ternary) return false;
            if (!q.have1) {
                q.m1 = golden ? q.lo + g * (q.hi - q.lo) : q.lo + (q.hi - q.lo) / 3.f;
                q.which = 3;
                s = q.m1;
            } else {
                q.m2 = golden ? q.hi - g * (q.hi - q.lo) : q.hi - (q.hi - q.lo) / 3.f;
                q.which = 4;
                s = q.m2;
            }
            return true;
        }
    }
    return false;
}


} // namespace ladl
