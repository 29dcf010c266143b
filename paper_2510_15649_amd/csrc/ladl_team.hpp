// Teams of TW wavefronts sharing one solve: the rows of a problem are spread
// over the waves of one workgroup, and every reduction over rows combines the
// waves' partial results through LDS.  The waves combine the partials in the
// same fixed order, so every wave obtains the same bits and takes the same
// branches; all other (per-solve, not per-row) state is held by each wave in
// its own copy and updated identically.  With TW = 1 every primitive is the
// plain wavefront operation and no LDS or barrier is involved.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include "ladl_wave.hpp"

namespace ladl {

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float unif(float v) { return bitsf(__builtin_amdgcn_readfirstlane(fbits(v))); }

// words of LDS one team needs for its exchanges: a ring of two slots of 8
// words per wave, plus 32 doubles per wave for per-feature partial sums
__host__ __device__ constexpr int team_red_words(int TW) { return TW > 1 ? 2 * 8 * TW + 64 * TW : 0; }

template <int TW>
struct Team {
    float *red;  // 2 x TW x 8 words (slot ring)
    double *vec; // TW x 32 doubles
    int wv;      // this wave's index in the team
    int seq;     // exchanges so far (identical on every wave)
};

// The slot of the next exchange.  A slot is written again two exchanges
// later; every wave has then passed the barrier of the exchange in between,
// which it reaches only after reading this one, so no read is overtaken.
template <int TW>
__device__ __forceinline__ float *team_slot(Team<TW> &t)
{
    float *s = t.red + (t.seq & 1) * (8 * TW);
    ++t.seq;
    return s;
}

// Barrier of the team's waves (a workgroup barrier; LDS written before it is
// visible after it).  Nothing for a team of one wave.
template <int TW>
__device__ __forceinline__ void team_sync()
{
    if constexpr (TW > 1) __syncthreads();
}

// sums and extrema over the team of values reduced within each wave
template <int TW>
__device__ __forceinline__ float tsum(Team<TW> &t, float v)
{
    const float s = wsum(v);
    if constexpr (TW == 1) {
        return s;
    } else {
        float *sl = team_slot(t);
        if (lane_id() == 0) sl[t.wv] = s;
        __syncthreads();
        float a = 0.f;
#pragma unroll
        for (int q = 0; q < TW; ++q) a += sl[q];
        return unif(a);
    }
}

template <int TW>
__device__ __forceinline__ void tsum2(Team<TW> &t, float &a, float &b)
{
    wsum2(a, b);
    if constexpr (TW > 1) {
        float *sl = team_slot(t);
        if (lane_id() == 0) {
            sl[2 * t.wv] = a;
            sl[2 * t.wv + 1] = b;
        }
        __syncthreads();
        float x = 0.f, y = 0.f;
#pragma unroll
        for (int q = 0; q < TW; ++q) {
            x += sl[2 * q];
            y += sl[2 * q + 1];
        }
        a = unif(x);
        b = unif(y);
    }
}

template <int TW>
__device__ __forceinline__ void tsum3(Team<TW> &t, float &a, float &b, float &c)
{
    wsum3(a, b, c);
    if constexpr (TW > 1) {
        float *sl = team_slot(t);
        if (lane_id() == 0) {
            sl[4 * t.wv] = a;
            sl[4 * t.wv + 1] = b;
            sl[4 * t.wv + 2] = c;
        }
        __syncthreads();
        float x = 0.f, y = 0.f, z = 0.f;
#pragma unroll
        for (int q = 0; q < TW; ++q) {
            x += sl[4 * q];
            y += sl[4 * q + 1];
            z += sl[4 * q + 2];
        }
        a = unif(x);
        b = unif(y);
        c = unif(z);
    }
}

template <int TW>
__device__ __forceinline__ float tmin(Team<TW> &t, float v)
{
    const float m = wmin(v);
    if constexpr (TW == 1) {
        return m;
    } else {
        float *sl = team_slot(t);
        if (lane_id() == 0) sl[t.wv] = m;
        __syncthreads();
        float a = sl[0];
#pragma unroll
        for (int q = 1; q < TW; ++q) a = fminf(a, sl[q]);
        return unif(a);
    }
}

template <int TW>
__device__ __forceinline__ float tmax(Team<TW> &t, float v)
{
    const float m = wmax(v);
    if constexpr (TW == 1) {
        return m;
    } else {
        float *sl = team_slot(t);
        if (lane_id() == 0) sl[t.wv] = m;
        __syncthreads();
        float a = sl[0];
#pragma unroll
        for (int q = 1; q < TW; ++q) a = fmaxf(a, sl[q]);
        return unif(a);
    }
}

// minimum of non-negative floats (see wmin_nn)
template <int TW>
__device__ __forceinline__ float tmin_nn(Team<TW> &t, float v)
{
    const float m = wmin_nn(v);
    if constexpr (TW == 1) {
        return m;
    } else {
        float *sl = team_slot(t);
        if (lane_id() == 0) sl[t.wv] = m;
        __syncthreads();
        float a = sl[0];
#pragma unroll
        for (int q = 1; q < TW; ++q) a = fminf(a, sl[q]);
        return unif(a);
    }
}

template <int TW>
__device__ __forceinline__ int tmin_i(Team<TW> &t, int v)
{
    const int m = wmin_i(v);
    if constexpr (TW == 1) {
        return m;
    } else {
        int *sl = (int *)team_slot(t);
        if (lane_id() == 0) sl[t.wv] = m;
        __syncthreads();
        int a = sl[0];
#pragma unroll
        for (int q = 1; q < TW; ++q) a = min(a, sl[q]);
        return uni(a);
    }
}

// number of lanes of the team where p holds
template <int TW>
__device__ __forceinline__ int tcount(Team<TW> &t, bool p)
{
    const int c = popc64(ballot(p));
    if constexpr (TW == 1) {
        return c;
    } else {
        int *sl = (int *)team_slot(t);
        if (lane_id() == 0) sl[t.wv] = c;
        __syncthreads();
        int a = 0;
#pragma unroll
        for (int q = 0; q < TW; ++q) a += sl[q];
        return uni(a);
    }
}

template <int TW>
__device__ __forceinline__ double tsum_d(Team<TW> &t, double v)
{
    const double s = wsum_d(v);
    if constexpr (TW == 1) {
        return s;
    } else {
        double *sl = (double *)team_slot(t); // 8 words per wave = 4 doubles
        if (lane_id() == 0) sl[4 * t.wv] = s;
        __syncthreads();
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < TW; ++q) a += sl[4 * q];
        return rdlane_d(a, 0);
    }
}

// Per-feature sums: lane j < 32 of every wave holds this wave's partial for
// feature j; returns the team total in lane j (one barrier for all j).
template <int TW>
__device__ __forceinline__ double tsum_vec_d(Team<TW> &t, double part_j)
{
    if constexpr (TW == 1) {
        return part_j;
    } else {
        const int l = lane_id();
        if (l < 32) t.vec[32 * t.wv + l] = part_j;
        __syncthreads();
        double a = 0.0;
        if (l < 32) {
#pragma unroll
            for (int q = 0; q < TW; ++q) a += t.vec[32 * q + l];
        }
        __syncthreads(); // vec is rewritten by the next call
        return a;
    }
}

} // namespace ladl
