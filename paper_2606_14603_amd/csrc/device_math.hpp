// device_math.hpp -- counter-based random numbers, the Gaussian transform and
// the geometry predicates of the molecule-agent step, for gfx950.
//
// Everything here is a pure function of its arguments and uses only IEEE
// binary32 +, -, *, /, sqrt and explicit fused multiply-add (the library is
// built with -ffp-contract=off, so no other operation is fused; denormals
// are kept, division and square root correctly rounded), so every result is
// reproducible bit for bit from the step definition.  Box-Muller's quotient
// and roots take shorter sequences that equal the correctly rounded
// operation on the arguments they can receive.
#pragma once

#include "engine.hpp"

namespace mabm {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds over a
// 4-word counter; between rounds the 2-word key advances by the golden-ratio
// and sqrt(3)-1 Weyl increments.  A round takes the 32x32->64 products of
// words 0 and 2 with the two round multipliers and mixes their halves with
// words 1 and 3 and the key.
struct U4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ U4 philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                     uint32_t c2, uint32_t c3)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply-add per product gives both halves; after
        // the first round each three-way xor is one three-input bit
        // operation (truth table 0x96).  The first round keeps plain xors:
        // with a step-uniform counter word its word 0 is wave-uniform, and
        // it stays in scalar registers, as does the next round's product.
        const uint64_t pa = uint64_t(kMulA) * c0;
        const uint64_t pb = uint64_t(kMulB) * c2;
        uint32_t n0, n2;
        if (r == 0) {
            n0 = uint32_t(pb >> 32) ^ c1 ^ k0;
            n2 = uint32_t(pa >> 32) ^ c3 ^ k1;
        } else {
            n0 = __builtin_amdgcn_bitop3_b32(uint32_t(pb >> 32), c1, k0, 0x96);
            n2 = __builtin_amdgcn_bitop3_b32(uint32_t(pa >> 32), c3, k1, 0x96);
        }
        c0 = n0;
        c1 = uint32_t(pb);
        c2 = n2;
        c3 = uint32_t(pa);
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(const Tables& T, uint32_t c0, uint32_t c1, uint32_t pur,
                                   uint32_t c3)
{
    return philox(T.key0, T.key1, c0, c1, pur, c3);
}

// 24-bit uniforms on [0,1) and (0,1], exact in binary32.
__device__ __forceinline__ float u01(uint32_t w) { return float(w >> 8) * 0x1p-24f; }
__device__ __forceinline__ float u01_open0(uint32_t w) { return float((w >> 8) + 1u) * 0x1p-24f; }

// a / b for the quotient of ln_unit below: a = m - 1 and b = m + 1 with m
// a float in [0.70, 1.42], so b lies in [1.7, 2.5] and the quotient is zero
// or normal.  The reciprocal estimate of the hardware is refined by one
// Newton step, and the quotient by two corrections with its residual,
// which a fused multiply-add gives exactly.  No operand scaling or
// special-value fix-up is needed in that range; the result equals the
// correctly rounded quotient for every such m (an exhaustive device test
// compares the two over all of them).
__device__ __forceinline__ float div_log_quotient(float a, float b)
{
    float y = __builtin_amdgcn_rcpf(b);
    y = __builtin_fmaf(__builtin_fmaf(-b, y, 1.0f), y, y);
    float q = a * y;
    q = __builtin_fmaf(__builtin_fmaf(-b, q, a), y, q);
    return __builtin_fmaf(__builtin_fmaf(-b, q, a), y, q);
}

// Square root of x = 0 or x in [2^-96, 64] (the Box-Muller radius: x =
// -2 ln u <= 34): the hardware estimate y is within one unit in the last
// place, and the correctly rounded root is the candidate c among y - ulp,
// y, y + ulp with (c - ulp/2)^2 < x < (c + ulp/2)^2.  Since x and the
// products of candidates are multiples of ulp^2, the two bounds are
// decided exactly by the signs of the fused residuals x - (y - ulp) y and
// x - y (y + ulp).  Equal to the correctly rounded root over the whole
// range (exhaustive device test).
__device__ __forceinline__ float sqrt_radius(float x)
{
    const float y = __builtin_amdgcn_sqrtf(x);
    const float below = __uint_as_float(__float_as_uint(y) - 1u);
    const float above = __uint_as_float(__float_as_uint(y) + 1u);
    float r = y;
    if (__builtin_fmaf(-below, y, x) <= 0.0f) r = below;
    if (__builtin_fmaf(-above, y, x) > 0.0f) r = above;
    return r;
}

// ln x for x in (0, 1]: split x = m 2^e, fold m above sqrt 2 down by one
// octave, then ln m = 2 atanh(s) with s = (m-1)/(m+1) and the odd series of
// atanh through s^9 by Horner's rule with fused multiply-adds; e ln 2 is
// added as a 16-bit head (exact product) and a float tail.
__device__ __forceinline__ float ln_unit(float x)
{
    const uint32_t b = __float_as_uint(x);
    int e = int((b >> 23) & 0xFFu) - 127;
    float m = __uint_as_float((b & 0x007FFFFFu) | 0x3F800000u);
    if (m > 0x1.6a09e6p+0f) {  // sqrt 2 rounded to float
        m = m * 0.5f;
        e = e + 1;
    }
    const float s = div_log_quotient(m - 1.0f, m + 1.0f);
    const float s2 = s * s;
    float h = 1.0f / 9.0f;
    h = __builtin_fmaf(h, s2, 1.0f / 7.0f);
    h = __builtin_fmaf(h, s2, 1.0f / 5.0f);
    h = __builtin_fmaf(h, s2, 1.0f / 3.0f);
    h = h * s2;
    const float ln_m = __builtin_fmaf(s, h, s) * 2.0f;
    const float fe = float(e);
    return __builtin_fmaf(fe, 0x1.62e4p-1f, __builtin_fmaf(fe, 0x1.7f7d1cp-20f, ln_m));
}

// sin and cos of 2 pi a, a in [0,1) on the 2^-24 grid: exact quadrant and
// remainder, fold of the remainder above 1/2 (swapping sin and cos), and the
// Maclaurin series of sin (x^9) and cos (x^8) on [0, pi/4] by Horner's rule
// with fused multiply-adds.
__device__ __forceinline__ void sincos_turn(float a, float& sn, float& cs)
{
    const float a4 = a * 4.0f;
    const int quad = int(a4);
    float r = a4 - float(quad);
    const bool fold = r > 0.5f;
    if (fold) r = 1.0f - r;
    const float x = r * 0x1.921fb6p+0f;  // pi/2 rounded to float
    const float x2 = x * x;
    float ps = 1.0f / 362880.0f;
    ps = __builtin_fmaf(ps, x2, -(1.0f / 5040.0f));
    ps = __builtin_fmaf(ps, x2, 1.0f / 120.0f);
    ps = __builtin_fmaf(ps, x2, -(1.0f / 6.0f));
    ps = ps * x2;
    const float sx = __builtin_fmaf(x, ps, x);
    float pc = 1.0f / 40320.0f;
    pc = __builtin_fmaf(pc, x2, -(1.0f / 720.0f));
    pc = __builtin_fmaf(pc, x2, 1.0f / 24.0f);
    pc = __builtin_fmaf(pc, x2, -0.5f);
    const float cx = __builtin_fmaf(pc, x2, 1.0f);
    // quadrant q in 0..3: (sin, cos) = (s1, c1), (c1, -s1), (-s1, -c1),
    // (-c1, s1), with s1, c1 the folded pair; as selects and sign-bit flips
    // (negation is the sign flip), without branches
    const uint32_t q = uint32_t(quad);
    const bool swap = fold != ((q & 1u) != 0u);
    const float sv = swap ? cx : sx;
    const float cv = swap ? sx : cx;
    sn = __uint_as_float(__float_as_uint(sv) ^ ((q & 2u) << 30));
    cs = __uint_as_float(__float_as_uint(cv) ^ (((q + 1u) & 2u) << 30));
}

// The 32-bit event draw: the four low bytes of the MOVE block, word 0
// lowest (Box-Muller reads only the high 24 bits of each word).
__device__ __forceinline__ uint32_t event_bits(const U4& w)
{
    return (w.w0 & 0xFFu) | ((w.w1 & 0xFFu) << 8) | ((w.w2 & 0xFFu) << 16) | ((w.w3 & 0xFFu) << 24);
}

// Three standard normals by Box-Muller from the MOVE block.
__device__ __forceinline__ void normals3(const U4& w, float& z0, float& z1, float& z2)
{
    float sn, cs;
    const float r1 = sqrt_radius(-2.0f * ln_unit(u01_open0(w.w0)));
    sincos_turn(u01(w.w1), sn, cs);
    z0 = r1 * cs;
    z1 = r1 * sn;
    const float r2 = sqrt_radius(-2.0f * ln_unit(u01_open0(w.w2)));
    sincos_turn(u01(w.w3), sn, cs);
    z2 = r2 * cs;
}

__device__ __forceinline__ float sq3(float x, float y, float z) { return x * x + y * y + z * z; }

// compartment: 0 = nucleus (strictly inside R_in) in the nested geometry
__device__ __forceinline__ int compartment(const Tables& T, float x, float y, float z)
{
    if (T.geometry != kNested) return 0;
    return sq3(x, y, z) < T.Rin2 ? 0 : 1;
}

__device__ __forceinline__ float wrap_box(const Tables& T, float v)
{
    if (v < 0.0f) v += T.L;
    if (v >= T.L) v -= T.L;
    return v;
}

// inside the volume and in compartment c (always true in the box)
__device__ __forceinline__ bool admissible(const Tables& T, float x, float y, float z, int c)
{
    if (T.geometry == kBox) return true;
    const float n2 = sq3(x, y, z);
    if (n2 > T.Rout2) return false;
    if (T.geometry == kNested && (n2 < T.Rin2 ? 0 : 1) != c) return false;
    return true;
}

__device__ __forceinline__ uint32_t cell_coord(const Tables& T, float v)
{
    // clamped to [0, G-1] (fmaxf takes the number over a NaN, so a NaN
    // coordinate maps to cell 0), then converted exactly
    const float f = __builtin_floorf((v - T.lo) * T.inv_h);
    return uint32_t(fminf(fmaxf(f, 0.0f), float(T.G - 1u)));
}

// Morton (Z-order) index: the bits of the three 10-bit cell coordinates
// interleaved (x lowest).  Cells adjacent in space are close in this order at
// every scale, which keeps the neighbour search's gathers local.
__device__ __forceinline__ uint32_t spread_bits3(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t gather_bits3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0x030000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}

__device__ __forceinline__ uint32_t cell_key(uint32_t cx, uint32_t cy, uint32_t cz)
{
    return spread_bits3(cx) | (spread_bits3(cy) << 1) | (spread_bits3(cz) << 2);
}

// sort key of the cell holding a position
__device__ __forceinline__ uint32_t cell_of(const Tables& T, float x, float y, float z)
{
    return cell_key(cell_coord(T, x), cell_coord(T, y), cell_coord(T, z));
}

// the exported cell id cx + G (cy + G cz) of a sort key
__device__ __forceinline__ uint32_t linear_cell(const Tables& T, uint32_t key)
{
    return gather_bits3(key) + T.G * (gather_bits3(key >> 1) + T.G * gather_bits3(key >> 2));
}

}  // namespace mabm
