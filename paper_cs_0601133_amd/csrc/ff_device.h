// Device-side helpers shared by the kernels: modular arithmetic through a
// floating-point inverse of p (Section 2.1.1: a product, a rounding of the
// quotient and one +-p adjustment), and the workgroup-to-tile mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ff {

// (a * b) mod p for a, b < p < 2^31, in binary64 and 32-bit integers.  The
// exact product is hi + lo with hi = fl(ab) and lo = fma(a, b, -hi) (exact,
// |lo| <= 2^8).  q = rint(hi/p) computed with the rounded inverse is within
// one of the nearest integer to hi/p, so hi - qp is an exact small integer
// (the fma rounds nothing) and r = hi - qp + lo lies in (-p, p); one
// correction makes it canonical.
__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, uint32_t p,
                                           double pinv)
{
    const double ad = (double)a, bd = (double)b, pd = (double)p;
    const double hi = ad * bd;
    const double lo = __builtin_fma(ad, bd, -hi);
    const double q = __builtin_rint(hi * pinv);
    const int32_t r = (int32_t)(__builtin_fma(-q, pd, hi) + lo);
    return (uint32_t)(r < 0 ? r + (int32_t)p : r);
}

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t p)
{
    uint32_t s = a + b;
    return s >= p ? s - p : s;
}

// Canonical residue of an integer-valued double x with |x| <= 2^53:
// r = x - p*rint(x/p) is exact with |r| <= p/2 + 2 (the quotient estimate
// from the rounded inverse is off by at most one), so it converts to 32 bits
// exactly; two corrections each side cover p = 2 and 3.
__device__ __forceinline__ uint32_t canon_f64(double x, double pd, double pinv,
                                              uint32_t p)
{
    const double q = __builtin_rint(x * pinv);
    int32_t r = (int32_t)__builtin_fma(-q, pd, x);
    r += r < 0 ? (int32_t)p : 0;
    r += r < 0 ? (int32_t)p : 0;
    r -= r >= (int32_t)p ? (int32_t)p : 0;
    r -= r >= (int32_t)p ? (int32_t)p : 0;
    return (uint32_t)r;
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
