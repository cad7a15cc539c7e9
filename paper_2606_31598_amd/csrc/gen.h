// Device-side block sources: Philox-GUE entries and sinc-DVR entries.
//
// Seeded generation (paper Sec. III) keyed on global (i, j) so the operator
// does not depend on the block partition (Sec. II).  The binary32 Gaussian
// transform below is a fixed sequence of IEEE operations (explicit fmaf, no
// contraction, correctly rounded division and square root), so the entries
// are reproducible bit for bit by any faithful implementation of the same
// definition.  Translation units including this header are built with
// -ffp-contract=off.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace procmv {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): two 32x32->64
// multiplications per round, Weyl key schedule.
struct Philox {
    static constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    static constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
};

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96, the odd-parity function,
// which is symmetric in its inputs); the compiler emits two v_xor_b32 for the
// plain expression.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1,
                                             uint32_t& c2, uint32_t& c3,
                                             uint32_t k0, uint32_t k1)
{
    uint64_t p0 = (uint64_t)Philox::M0 * c0;
    uint64_t p1 = (uint64_t)Philox::M1 * c2;
    uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
}

// Words 0 and 1 of Philox4x32-10 at counter (i, j, 0, 0).  The first two
// rounds are written out with the zero counter words folded away (round 1:
// M1 * 0 = 0; round 2: its c1 is the low half of that zero product).
__device__ __forceinline__ void philox_ij(uint32_t i, uint32_t j, uint32_t k0,
                                          uint32_t k1, uint32_t& x0,
                                          uint32_t& x1)
{
    // round 1: c = (i, j, 0, 0)
    uint64_t p0 = (uint64_t)Philox::M0 * i;
    uint32_t c0 = j ^ k0;
    uint32_t c1 = 0u;
    uint32_t c2 = (uint32_t)(p0 >> 32) ^ k1;
    uint32_t c3 = (uint32_t)p0;
    k0 += Philox::W0;
    k1 += Philox::W1;
    // round 2: c1 = 0
    p0 = (uint64_t)Philox::M0 * c0;
    uint64_t p1 = (uint64_t)Philox::M1 * c2;
    c0 = (uint32_t)(p1 >> 32) ^ k0;
    c2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    k0 += Philox::W0;
    k1 += Philox::W1;
#pragma unroll
    for (int r = 2; r < 10; ++r) {
        philox_round(c0, c1, c2, c3, k0, k1);
        k0 += Philox::W0;
        k1 += Philox::W1;
    }
    x0 = c0;
    x1 = c1;
}

// The same words when i is the same in every lane of the wave (the matrix-core
// tile kernel generates one row per wave and step).  Rounds 1 and 2 then
// depend on the lane only through j, and the three-word XORs of rounds 2 to
// 4 pair their two row-only words first, which the scalar unit does; the
// rest is philox_ij's sequence.  The words are the same bits either way (XOR
// is associative).
__device__ __forceinline__ void philox_row(uint32_t i, uint32_t j, uint32_t k0, uint32_t k1,
                                           uint32_t& x0, uint32_t& x1)
{
    // round 1: c = (i, j, 0, 0)
    uint64_t p0 = (uint64_t)Philox::M0 * i;
    uint32_t c0 = j ^ k0;
    uint32_t c2 = (uint32_t)(p0 >> 32) ^ k1;
    uint32_t c3 = (uint32_t)p0;
    k0 += Philox::W0;
    k1 += Philox::W1;
    // round 2: c1 = 0; c2 and c3 are row-only, c0 lane-only
    p0 = (uint64_t)Philox::M0 * c0;
    uint64_t p1 = (uint64_t)Philox::M1 * c2;
    c0 = (uint32_t)(p1 >> 32) ^ k0;
    c2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    uint32_t c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    k0 += Philox::W0;
    k1 += Philox::W1;
    // round 3: c0 and c1 are row-only
    p0 = (uint64_t)Philox::M0 * c0;
    p1 = (uint64_t)Philox::M1 * c2;
    c0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);
    c2 = c3 ^ ((uint32_t)(p0 >> 32) ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    k0 += Philox::W0;
    k1 += Philox::W1;
    // round 4: c3 is row-only
    p0 = (uint64_t)Philox::M0 * c0;
    p1 = (uint64_t)Philox::M1 * c2;
    c0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    c2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    k0 += Philox::W0;
    k1 += Philox::W1;
#pragma unroll
    for (int r = 4; r < 10; ++r) {
        philox_round(c0, c1, c2, c3, k0, k1);
        k0 += Philox::W0;
        k1 += Philox::W1;
    }
    x0 = c0;
    x1 = c1;
}

// Uniform (2 (x >> 9) + 1) 2^-24 in (0, 1), exact in binary32.
__device__ __forceinline__ float u01(uint32_t x)
{
    return (float)((x >> 9) * 2u + 1u) * 5.9604644775390625e-8f;
}

// Correctly rounded binary32 a / b and sqrt(a) on the generator's domain.
// The quotient is a reciprocal estimate refined by one residual correction
// (q0 = a y, r = a - q0 b exactly by FMA, q = q0 + r y); the root is the
// hardware estimate moved by at most one ulp to the side that leaves the
// smaller residual.  Neither handles denormal, infinite or NaN operands,
// which the generator never produces (b in [1.7, 2.5], a in [1.2e-7, 33.3]);
// procmv_selftest_generator checks both against IEEE division and square
// root for every one of the 2^23 uniforms the generator can draw.
__device__ __forceinline__ float div_gen(float a, float b)
{
    const float y = __builtin_amdgcn_rcpf(b);
    const float q0 = a * y;
    const float r = __builtin_fmaf(-q0, b, a);
    return __builtin_fmaf(r, y, q0);
}

__device__ __forceinline__ float sqrt_gen(float a)
{
    float s = __builtin_amdgcn_sqrtf(a);
    const float sm = __uint_as_float(__float_as_uint(s) - 1u);
    const float sp = __uint_as_float(__float_as_uint(s) + 1u);
    const float rm = __builtin_fmaf(-sm, s, a);
    const float rp = __builtin_fmaf(-sp, s, a);
    s = (rm <= 0.f) ? sm : s;
    s = (rp > 0.f) ? sp : s;
    return s;
}

// ln u for u in (0, 1): u = 2^e m with m in [sqrt(1/2), sqrt(2)];
// ln m = 2 atanh(s), s = (m - 1)/(m + 1), odd series through s^9.  IEEE
// selects the compiler's general division (the self-test's reference).
template <bool IEEE = false>
__device__ __forceinline__ float ln_unit(float u)
{
    uint32_t b = __float_as_uint(u);
    int e = (int)(b >> 23) - 127;
    float m = __uint_as_float((b & 0x007FFFFFu) | 0x3F800000u);
    if (m > 1.41421356237309504880f) {
        m = m * 0.5f;
        e = e + 1;
    }
    float f = m - 1.0f;
    float s = IEEE ? f / (2.0f + f) : div_gen(f, 2.0f + f);
    float s2 = s * s;
    float p = __builtin_fmaf(s2, (float)(2.0 / 9.0), (float)(2.0 / 7.0));
    p = __builtin_fmaf(s2, p, (float)(2.0 / 5.0));
    p = __builtin_fmaf(s2, p, (float)(2.0 / 3.0));
    float lm = __builtin_fmaf(s * s2, p, 2.0f * s);
    float ef = (float)e;
    const float ln2_hi = 0.693147180559945309417f;
    const float ln2_lo = (float)(0.693147180559945309417232121458 -
                                 (double)0.693147180559945309417f);
    return __builtin_fmaf(ef, ln2_hi, __builtin_fmaf(ef, ln2_lo, lm));
}

// sin(2 pi u), cos(2 pi u): exact quarter-turn reduction u = n/4 + r,
// |r| <= 1/8, then the Taylor polynomials of sin(2 pi r) through r^9 and of
// cos(2 pi r) through r^10 (coefficients (2 pi)^k / k!).
__device__ __forceinline__ void sincos_turn(float u, float& sv, float& cv)
{
    float n = __builtin_rintf(4.0f * u);
    float r = __builtin_fmaf(n, -0.25f, u);
    float r2 = r * r;
    float ps = __builtin_fmaf(r2, 42.0586939448976531450f, -76.7058597530613858416f);
    ps = __builtin_fmaf(r2, ps, 81.6052492760750542034f);
    ps = __builtin_fmaf(r2, ps, -41.3417022403997602340f);
    ps = __builtin_fmaf(r2, ps, 6.28318530717958647692f);
    float sr = r * ps;
    float pc = __builtin_fmaf(r2, -26.4262567833743974529f, 60.2446413718766603627f);
    pc = __builtin_fmaf(r2, pc, -85.4568172066937277360f);
    pc = __builtin_fmaf(r2, pc, 64.9393940226682914910f);
    pc = __builtin_fmaf(r2, pc, -19.7392088021787172377f);
    float cr = __builtin_fmaf(r2, pc, 1.0f);
    int q = ((int)n) & 3;
    float s0 = (q & 1) ? cr : sr;
    float c0 = (q & 1) ? sr : cr;
    sv = (q & 2) ? -s0 : s0;
    cv = ((q + 1) & 2) ? -c0 : c0;
}

// The kernels' form of the transform below: the same binary32 results,
// bit for bit, in fewer instructions (procmv_selftest_generator compares
// both forms over every uniform).
//  * The uniform is kept as Z = u 2^32 = (x with its low nine bits replaced
//    by 1 0000 0000): at most 24 significant bits, so the conversion is
//    exact, and Z has u's significand.
//  * -2 ln u takes Z's exponent minus 159 (= 127 + 32) and the series and
//    ln 2 constants times -2; scaling by a power of two commutes with every
//    rounding here (no result is near the binary32 range limits).
//  * sin and cos reach their quadrant signs by XOR of the sign bit.
__device__ __forceinline__ float unit_2p32(uint32_t x)
{
    // 0x100 held in a register lets the mask and the insert be one
    // v_and_or_b32 (a three-operand instruction takes no literal)
    uint32_t c = 0x100u;
    asm("" : "+v"(c));
    return (float)((x & 0xFFFFFE00u) | c);
}

__device__ __forceinline__ float neg2_ln_2p32(float z)
{
    uint32_t b = __float_as_uint(z);
    int e = (int)(b >> 23) - 159;
    float m = __uint_as_float((b & 0x007FFFFFu) | 0x3F800000u);
    if (m > 1.41421356237309504880f) {
        m = m * 0.5f;
        e = e + 1;
    }
    float f = m - 1.0f;
    float s = div_gen(f, 2.0f + f);
    float s2 = s * s;
    float p = __builtin_fmaf(s2, -2.0f * (float)(2.0 / 9.0), -2.0f * (float)(2.0 / 7.0));
    p = __builtin_fmaf(s2, p, -2.0f * (float)(2.0 / 5.0));
    p = __builtin_fmaf(s2, p, -2.0f * (float)(2.0 / 3.0));
    float lm = __builtin_fmaf(s * s2, p, -4.0f * s);
    float ef = (float)e;
    const float ln2_hi = 0.693147180559945309417f;
    const float ln2_lo = (float)(0.693147180559945309417232121458 -
                                 (double)0.693147180559945309417f);
    return __builtin_fmaf(ef, -2.0f * ln2_hi, __builtin_fmaf(ef, -2.0f * ln2_lo, lm));
}

__device__ __forceinline__ void sincos_2p32(float z, float& sv, float& cv)
{
    const float u = z * 0x1p-32f;
    const float n = __builtin_rintf(z * 0x1p-30f);     // 4u
    const float r = __builtin_fmaf(n, -0.25f, u);
    float r2 = r * r;
    float ps = __builtin_fmaf(r2, 42.0586939448976531450f, -76.7058597530613858416f);
    ps = __builtin_fmaf(r2, ps, 81.6052492760750542034f);
    ps = __builtin_fmaf(r2, ps, -41.3417022403997602340f);
    ps = __builtin_fmaf(r2, ps, 6.28318530717958647692f);
    const float sr = r * ps;
    float pc = __builtin_fmaf(r2, -26.4262567833743974529f, 60.2446413718766603627f);
    pc = __builtin_fmaf(r2, pc, -85.4568172066937277360f);
    pc = __builtin_fmaf(r2, pc, 64.9393940226682914910f);
    pc = __builtin_fmaf(r2, pc, -19.7392088021787172377f);
    const float cr = __builtin_fmaf(r2, pc, 1.0f);
    const int q = (int)n;                              // 0 .. 4; 4 is quadrant 0
    const float s0 = (q & 1) ? cr : sr;
    const float c0 = (q & 1) ? sr : cr;
    // s ^ (t & sign) as one v_bitop3_b32: the function S1 ^ (S0 & S2) (table
    // 0x6c) is symmetric in S0 and S2
    const uint32_t sign = 0x80000000u;
    sv = __uint_as_float(__builtin_amdgcn_bitop3_b32((uint32_t)q << 30, __float_as_uint(s0),
                                                     sign, 0x6c));
    cv = __uint_as_float(__builtin_amdgcn_bitop3_b32((uint32_t)(q + 1) << 30,
                                                     __float_as_uint(c0), sign, 0x6c));
}

// Box-Muller: z0 = r cos(2 pi u1), z1 = r sin(2 pi u1), r = sqrt(-2 ln u0),
// u = u01(x) (the definitions above), in the kernels' form.
__device__ __forceinline__ void box_muller(uint32_t x0, uint32_t x1, float& z0,
                                           float& z1)
{
    float r = sqrt_gen(neg2_ln_2p32(unit_2p32(x0)));
    float sv, cv;
    sincos_2p32(unit_2p32(x1), sv, cv);
    z0 = r * cv;
    z1 = r * sv;
}

// Parameters of the Philox-GUE source.
struct GueParams {
    uint32_t k0, k1;      // key = (seed low, seed high)
    float s_off, s_diag;  // binary32 scales sqrt(1/(2D)), sqrt(1/D)
};

// Canonical entry H_ij, i < j.
__device__ __forceinline__ float2 gue_upper(const GueParams& g, uint32_t i,
                                            uint32_t j)
{
    uint32_t x0, x1;
    philox_ij(i, j, g.k0, g.k1, x0, x1);
    float z0, z1;
    box_muller(x0, x1, z0, z1);
    return make_float2(g.s_off * z0, g.s_off * z1);
}

// Diagonal entry H_ii (real).
__device__ __forceinline__ float gue_diag(const GueParams& g, uint32_t i)
{
    uint32_t x0, x1;
    philox_ij(i, i, g.k0, g.k1, x0, x1);
    float z0, z1;
    box_muller(x0, x1, z0, z1);
    return g.s_diag * z0;
}

// Any entry H_ij (conjugated canonical draw below the diagonal).
__device__ __forceinline__ float2 gue_entry(const GueParams& g, uint32_t i,
                                            uint32_t j)
{
    if (i == j) return make_float2(gue_diag(g, i), 0.0f);
    if (i < j) return gue_upper(g, i, j);
    float2 h = gue_upper(g, j, i);
    return make_float2(h.x, -h.y);
}

// Parameters of the sinc-DVR source: binary32 kinetic symbol tk[k] for
// k = |i - j| >= 1 and binary32 potential v[i]; the binary64 constant
// diagonal is applied in the reduction epilogue.
struct DvrParams {
    const float* tk;
    const float* v;
};

__device__ __forceinline__ float dvr_entry(const DvrParams& p, uint32_t i,
                                           uint32_t j)
{
    if (i == j) return p.v[i];
    return p.tk[i > j ? i - j : j - i];
}

}  // namespace procmv
