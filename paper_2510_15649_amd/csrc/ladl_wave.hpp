// Wavefront primitives for gfx950 (wave64): DPP reductions and scans,
// ballot/mbcnt compaction helpers and a 64-lane bitonic sort.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ladl {

constexpr int WAVE = 64;
constexpr float FINF = __builtin_inff();

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int fbits(float v) { return __builtin_bit_cast(int, v); }
__device__ __forceinline__ float bitsf(int v) { return __builtin_bit_cast(float, v); }

// lane `l` of v; l must be wave-uniform
__device__ __forceinline__ float rdlane(float v, int l) { return bitsf(__builtin_amdgcn_readlane(fbits(v), l)); }
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// DPP move: lanes whose source is outside the row, or whose row/bank is
// masked off, receive `old`.
template <int CTRL, int ROWM = 0xF, int BANKM = 0xF>
__device__ __forceinline__ float dpp(float old, float v)
{
    return bitsf(__builtin_amdgcn_update_dpp(fbits(old), fbits(v), CTRL, ROWM, BANKM, false));
}
template <int CTRL, int ROWM = 0xF, int BANKM = 0xF>
__device__ __forceinline__ int dppi(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWM, BANKM, false);
}

// DPP controls (GFX9 encoding)
constexpr int DPP_XOR1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int DPP_HMIRROR = 0x141; // row_half_mirror
constexpr int DPP_MIRROR = 0x140;  // row_mirror
constexpr int DPP_SHR1 = 0x111, DPP_SHR2 = 0x112, DPP_SHR4 = 0x114, DPP_SHR8 = 0x118;
constexpr int DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;

// Reductions: prefix combine within each row of 16 lanes (row shifts),
// then across rows with the row broadcasts of lanes 15 and 31; lane 63 ends
// with the result, which one readlane makes wave-uniform.  The order of the
// operations is fixed, so results are deterministic.
__device__ __forceinline__ float wsum(float v)
{
    v += dpp<DPP_SHR1>(0.f, v);
    v += dpp<DPP_SHR2>(0.f, v);
    v += dpp<DPP_SHR4>(0.f, v);
    v += dpp<DPP_SHR8>(0.f, v);
    v += dpp<DPP_BCAST15, 0xA>(0.f, v);
    v += dpp<DPP_BCAST31, 0xC>(0.f, v);
    return rdlane(v, 63);
}

// two or three independent sums, interleaved for latency
__device__ __forceinline__ void wsum2(float &a, float &b)
{
    a += dpp<DPP_SHR1>(0.f, a);
    b += dpp<DPP_SHR1>(0.f, b);
    a += dpp<DPP_SHR2>(0.f, a);
    b += dpp<DPP_SHR2>(0.f, b);
    a += dpp<DPP_SHR4>(0.f, a);
    b += dpp<DPP_SHR4>(0.f, b);
    a += dpp<DPP_SHR8>(0.f, a);
    b += dpp<DPP_SHR8>(0.f, b);
    a += dpp<DPP_BCAST15, 0xA>(0.f, a);
    b += dpp<DPP_BCAST15, 0xA>(0.f, b);
    a += dpp<DPP_BCAST31, 0xC>(0.f, a);
    b += dpp<DPP_BCAST31, 0xC>(0.f, b);
    a = rdlane(a, 63);
    b = rdlane(b, 63);
}

__device__ __forceinline__ void wsum3(float &a, float &b, float &c)
{
    a += dpp<DPP_SHR1>(0.f, a);
    b += dpp<DPP_SHR1>(0.f, b);
    c += dpp<DPP_SHR1>(0.f, c);
    a += dpp<DPP_SHR2>(0.f, a);
    b += dpp<DPP_SHR2>(0.f, b);
    c += dpp<DPP_SHR2>(0.f, c);
    a += dpp<DPP_SHR4>(0.f, a);
    b += dpp<DPP_SHR4>(0.f, b);
    c += dpp<DPP_SHR4>(0.f, c);
    a += dpp<DPP_SHR8>(0.f, a);
    b += dpp<DPP_SHR8>(0.f, b);
    c += dpp<DPP_SHR8>(0.f, c);
    a += dpp<DPP_BCAST15, 0xA>(0.f, a);
    b += dpp<DPP_BCAST15, 0xA>(0.f, b);
    c += dpp<DPP_BCAST15, 0xA>(0.f, c);
    a += dpp<DPP_BCAST31, 0xC>(0.f, a);
    b += dpp<DPP_BCAST31, 0xC>(0.f, b);
    c += dpp<DPP_BCAST31, 0xC>(0.f, c);
    a = rdlane(a, 63);
    b = rdlane(b, 63);
    c = rdlane(c, 63);
}

// two sums and two minima in one interleaved pass
__device__ __forceinline__ void wsum2_min2(float &a, float &b, float &c, float &d)
{
    const float I = __builtin_inff();
    a += dpp<DPP_SHR1>(0.f, a);
    b += dpp<DPP_SHR1>(0.f, b);
    c = fminf(c, dpp<DPP_SHR1>(I, c));
    d = fminf(d, dpp<DPP_SHR1>(I, d));
    a += dpp<DPP_SHR2>(0.f, a);
    b += dpp<DPP_SHR2>(0.f, b);
    c = fminf(c, dpp<DPP_SHR2>(I, c));
    d = fminf(d, dpp<DPP_SHR2>(I, d));
    a += dpp<DPP_SHR4>(0.f, a);
    b += dpp<DPP_SHR4>(0.f, b);
    c = fminf(c, dpp<DPP_SHR4>(I, c));
    d = fminf(d, dpp<DPP_SHR4>(I, d));
    a += dpp<DPP_SHR8>(0.f, a);
    b += dpp<DPP_SHR8>(0.f, b);
    c = fminf(c, dpp<DPP_SHR8>(I, c));
    d = fminf(d, dpp<DPP_SHR8>(I, d));
    a += dpp<DPP_BCAST15, 0xA>(0.f, a);
    b += dpp<DPP_BCAST15, 0xA>(0.f, b);
    c = fminf(c, dpp<DPP_BCAST15, 0xA>(I, c));
    d = fminf(d, dpp<DPP_BCAST15, 0xA>(I, d));
    a += dpp<DPP_BCAST31, 0xC>(0.f, a);
    b += dpp<DPP_BCAST31, 0xC>(0.f, b);
    c = fminf(c, dpp<DPP_BCAST31, 0xC>(I, c));
    d = fminf(d, dpp<DPP_BCAST31, 0xC>(I, d));
    a = rdlane(a, 63);
    b = rdlane(b, 63);
    c = rdlane(c, 63);
    d = rdlane(d, 63);
}

__device__ __forceinline__ float wmin(float v)
{
    const float I = __builtin_inff();
    v = fminf(v, dpp<DPP_SHR1>(I, v));
    v = fminf(v, dpp<DPP_SHR2>(I, v));
    v = fminf(v, dpp<DPP_SHR4>(I, v));
    v = fminf(v, dpp<DPP_SHR8>(I, v));
    v = fminf(v, dpp<DPP_BCAST15, 0xA>(I, v));
    v = fminf(v, dpp<DPP_BCAST31, 0xC>(I, v));
    return rdlane(v, 63);
}

__device__ __forceinline__ float wmax(float v)
{
    const float I = -__builtin_inff();
    v = fmaxf(v, dpp<DPP_SHR1>(I, v));
    v = fmaxf(v, dpp<DPP_SHR2>(I, v));
    v = fmaxf(v, dpp<DPP_SHR4>(I, v));
    v = fmaxf(v, dpp<DPP_SHR8>(I, v));
    v = fmaxf(v, dpp<DPP_BCAST15, 0xA>(I, v));
    v = fmaxf(v, dpp<DPP_BCAST31, 0xC>(I, v));
    return rdlane(v, 63);
}

__device__ __forceinline__ int wmin_i(int v)
{
    const int I = 0x7fffffff;
    v = min(v, dppi<DPP_SHR1>(I, v));
    v = min(v, dppi<DPP_SHR2>(I, v));
    v = min(v, dppi<DPP_SHR4>(I, v));
    v = min(v, dppi<DPP_SHR8>(I, v));
    v = min(v, dppi<DPP_BCAST15, 0xA>(I, v));
    v = min(v, dppi<DPP_BCAST31, 0xC>(I, v));
    return rdlane(v, 63);
}

// Minimum of non-negative floats (or +inf): for such values the bit
// patterns order like unsigned integers, so the minimum is ~max(~bits).  The
// unsigned max has identity 0, which is what DPP writes into lanes whose
// source lies outside the row, so every row step is one v_max_u32 with DPP.
__device__ __forceinline__ float wmin_nn(float v)
{
    uint32_t u = ~(uint32_t)fbits(v);
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, DPP_SHR1, 0xF, 0xF, true));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, DPP_SHR2, 0xF, 0xF, true));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, DPP_SHR4, 0xF, 0xF, true));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, DPP_SHR8, 0xF, 0xF, true));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, DPP_BCAST15, 0xA, 0xF, false));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, DPP_BCAST31, 0xC, 0xF, false));
    return bitsf((int)~(uint32_t)__builtin_amdgcn_readlane((int)u, 63));
}

// DPP move of a double (both halves; `old` is +0.0)
template <int CTRL, int ROWM = 0xF>
__device__ __forceinline__ double dppd(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWM, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWM, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double rdlane_d(double v, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// double-precision sums (the optimality certificate and the final
// objective), same fixed order as wsum; the four-way form interleaves
// independent sums for latency
__device__ __forceinline__ double wsum_d(double v)
{
    v += dppd<DPP_SHR1>(v);
    v += dppd<DPP_SHR2>(v);
    v += dppd<DPP_SHR4>(v);
    v += dppd<DPP_SHR8>(v);
    v += dppd<DPP_BCAST15, 0xA>(v);
    v += dppd<DPP_BCAST31, 0xC>(v);
    return rdlane_d(v, 63);
}

__device__ __forceinline__ void wsum_d4(double &a, double &b, double &c, double &d)
{
    a += dppd<DPP_SHR1>(a);
    b += dppd<DPP_SHR1>(b);
    c += dppd<DPP_SHR1>(c);
    d += dppd<DPP_SHR1>(d);
    a += dppd<DPP_SHR2>(a);
    b += dppd<DPP_SHR2>(b);
    c += dppd<DPP_SHR2>(c);
    d += dppd<DPP_SHR2>(d);
    a += dppd<DPP_SHR4>(a);
    b += dppd<DPP_SHR4>(b);
    c += dppd<DPP_SHR4>(c);
    d += dppd<DPP_SHR4>(d);
    a += dppd<DPP_SHR8>(a);
    b += dppd<DPP_SHR8>(b);
    c += dppd<DPP_SHR8>(c);
    d += dppd<DPP_SHR8>(d);
    a += dppd<DPP_BCAST15, 0xA>(a);
    b += dppd<DPP_BCAST15, 0xA>(b);
    c += dppd<DPP_BCAST15, 0xA>(c);
    d += dppd<DPP_BCAST15, 0xA>(d);
    a += dppd<DPP_BCAST31, 0xC>(a);
    b += dppd<DPP_BCAST31, 0xC>(b);
    c += dppd<DPP_BCAST31, 0xC>(c);
    d += dppd<DPP_BCAST31, 0xC>(d);
    a = rdlane_d(a, 63);
    b = rdlane_d(b, 63);
    c = rdlane_d(c, 63);
    d = rdlane_d(d, 63);
}

// inclusive prefix sum across the 64 lanes (row shifts, then row
// broadcasts of lanes 15 and 31)
__device__ __forceinline__ float wscan_incl(float v)
{
    v += dpp<DPP_SHR1>(0.f, v);
    v += dpp<DPP_SHR2>(0.f, v);
    v += dpp<DPP_SHR4>(0.f, v);
    v += dpp<DPP_SHR8>(0.f, v);
    v += dpp<DPP_BCAST15, 0xA>(0.f, v);
    v += dpp<DPP_BCAST31, 0xC>(0.f, v);
    return v;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }
__device__ __forceinline__ int first_lane(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }
// number of set bits of m in lanes below this one
__device__ __forceinline__ int mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ascending sort of (key, val) pairs held one per lane
__device__ __forceinline__ void bitonic64(float &key, float &val)
{
    const int l = lane_id();
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            float ok = __shfl_xor(key, j);
            float ov = __shfl_xor(val, j);
            bool asc = (l & k) == 0;
            bool lower = (l & j) == 0;
            bool take = (asc == lower) ? (ok < key) : (ok > key);
            key = take ? ok : key;
            val = take ? ov : val;
        }
    }
}

__device__ __forceinline__ void bitonic64(float &key)
{
    const int l = lane_id();
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            float ok = __shfl_xor(key, j);
            bool asc = (l & k) == 0;
            bool lower = (l & j) == 0;
            bool take = (asc == lower) ? (ok < key) : (ok > key);
            key = take ? ok : key;
        }
    }
}

__device__ __forceinline__ float sgnf(float v) { return (v > 0.f) ? 1.f : ((v < 0.f) ? -1.f : 0.f); }

} // namespace ladl
