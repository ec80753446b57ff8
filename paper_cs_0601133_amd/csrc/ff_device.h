// Device-side helpers shared by the kernels: modular arithmetic through a
// floating-point inverse of p (Section 2.1.1: a product, a rounding of the
// quotient and one +-p adjustment), and the workgroup-to-tile mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ff {

// (a * b) mod p for a, b < p < 2^31.  The quotient estimate from the
// double-precision inverse is off by at most one, so the remainder lands in
// [-p, 2p) and one correction on each side makes it canonical.
__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, uint32_t p,
                                           double pinv)
{
    const uint64_t ab = (uint64_t)a * b;
    const uint64_t q = (uint64_t)((double)a * (double)b * pinv);
    int64_t r = (int64_t)(ab - q * (uint64_t)p);
    r += (r < 0) ? (int64_t)p : 0;
    r -= (r >= (int64_t)p) ? (int64_t)p : 0;
    return (uint32_t)r;
}

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t p)
{
    uint32_t s = a + b;
    return s >= p ? s - p : s;
}

// Canonical residue of an integer-valued double x with |x| <= 2^53:
// r = x - p*rint(x/p) is exact (an integer of magnitude <= p/2 + 2) and is
// then moved into [0, p).
__device__ __forceinline__ uint32_t canon_f64(double x, double pd, double pinv,
                                              uint32_t p)
{
    const double q = __builtin_rint(x * pinv);
    const double r = __builtin_fma(-q, pd, x);
    int64_t ri = (int64_t)r;
    ri += (ri < 0) ? (int64_t)p : 0;
    ri += (ri < 0) ? (int64_t)p : 0;
    ri -= (ri >= (int64_t)p) ? (int64_t)p : 0;
    ri -= (ri >= (int64_t)p) ? (int64_t)p : 0;
    return (uint32_t)ri;
}

// Centered value of a residue u in [0, p): u or u - p.
__device__ __forceinline__ int32_t center(uint32_t u, uint32_t p, uint32_t half)
{
    return (int32_t)u - (u > half ? (int32_t)p : 0);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This renumbers block b of G so that every XCD receives a contiguous
// range of logical ids, i.e. neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int b, int G)
{
    constexpr int X = 8;
    const int q = G / X, r = G % X;
    const int x = b % X;
    return x * q + (x < r ? x : r) + b / X;
}

// Logical tile id -> (tm, tn) in groups of GM tile rows, so that the
// workgroups resident at one time reuse the same A row panels and B column
// panels.
template <int GM>
__device__ __forceinline__ void grouped_tile(int t, int tiles_m, int tiles_n,
                                             int *tm, int *tn)
{
    const int per_group = GM * tiles_n;
    const int g = t / per_group;
    const int first = g * GM;
    const int gsz = (tiles_m - first) < GM ? (tiles_m - first) : GM;
    const int in = t - g * per_group;
    *tm = first + in % gsz;
    *tn = in / gsz;
}

// Same with the group height chosen at run time.
__device__ __forceinline__ void grouped_tile_rt(int t, int tiles_m, int tiles_n, int gm,
                                                int *tm, int *tn)
{
    const int per_group = gm * tiles_n;
    const int g = t / per_group;
    const int first = g * gm;
    const int gsz = (tiles_m - first) < gm ? (tiles_m - first) : gm;
    const int in = t - g * per_group;
    *tm = first + in % gsz;
    *tn = in / gsz;
}

} // namespace ff
