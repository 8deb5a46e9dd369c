// device_math.hpp -- per-lane arithmetic of the IRT-PS tracer on gfx950.
//
// Everything that decides which surface sample a ray hits is binary32 with a
// fixed operation order: products and sums round one at a time (the library
// is compiled with -ffp-contract=off), every fused multiply-add is an explicit
// fmaf, division and square root are correctly rounded
// (-fhip-fp32-correctly-rounded-divide-sqrt), denormals are kept, and no
// hardware transcendental is used.  The same inputs therefore give the same
// hit on any IEEE-conforming machine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace irtps {
namespace dm {

constexpr float kPi = 0x1.921fb6p+1f;      // binary32 nearest pi
constexpr float kHalfPi = 0x1.921fb6p+0f;
constexpr float kQuarterPi = 0x1.921fb6p-1f;
constexpr float kTwoPi = 0x1.921fb6p+2f;
constexpr float kInvPi = 0x1.45f306p-2f;
constexpr float kInvTwoPi = 0x1.45f306p-3f;
constexpr float kTanEighthPi = 0x1.a8279ap-2f;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies
// whose high halves are mixed with the other two words and the key; the key
// advances by the Weyl increments between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

// The 64-bit product of a (per lane) and m (uniform) in one v_mad_u64_u32,
// whose carry-out goes to VCC.  The compiler splits such a product into
// v_mul_lo_u32 and v_mul_hi_u32; measured on gfx950 with independent chains,
// the pair takes about 12.7 cycles per wave64 and the single instruction 7.9.
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t m) {
    uint64_t p;
    __asm__("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(p) : "v"(a), "s"(m) : "vcc");
    return p;
}

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round != 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t a = mul_wide(c0, 0xD2511F53u);
        const uint64_t b = mul_wide(c2, 0xCD9E8D57u);
        const uint32_t a_lo = (uint32_t)a, a_hi = (uint32_t)(a >> 32);
        const uint32_t b_lo = (uint32_t)b, b_hi = (uint32_t)(b >> 32);
        const uint32_t y0 = b_hi ^ c1 ^ k0;
        const uint32_t y2 = a_hi ^ c3 ^ k1;
        c0 = y0;
        c1 = b_lo;
        c2 = y2;
        c3 = a_lo;
    }
    return U4{c0, c1, c2, c3};
}

// Top 24 bits scaled to [0,1): exact in binary32.
__device__ __forceinline__ float unit24(uint32_t r) { return (float)(r >> 8) * 0x1p-24f; }

// ---------------------------------------------------------------------------
// Quarter-turn sine and cosine, sin(pi f / 2) and cos(pi f / 2) for f in [0,1):
// Taylor series in f^2 (terms (pi/2)^m / m!) rounded to binary32, Horner order.
__device__ __forceinline__ void quarter_sincos(float f, float& s, float& c) {
    const float q = f * f;
    float ps = 0x1.e8f434p-25f;
    ps = fmaf(ps, q, -0x1.e30750p-19f);
    ps = fmaf(ps, q, 0x1.507834p-13f);
    ps = fmaf(ps, q, -0x1.32d2ccp-8f);
    ps = fmaf(ps, q, 0x1.466bc6p-4f);
    ps = fmaf(ps, q, -0x1.4abbcep-1f);
    ps = fmaf(ps, q, 0x1.921fb6p+0f);
    s = ps * f;
    float pc = -0x1.b6e250p-28f;
    pc = fmaf(pc, q, 0x1.f9d38ap-22f);
    pc = fmaf(pc, q, -0x1.a6d1f2p-16f);
    pc = fmaf(pc, q, 0x1.e1f506p-11f);
    pc = fmaf(pc, q, -0x1.55d3c8p-6f);
    pc = fmaf(pc, q, 0x1.03c1f0p-2f);
    pc = fmaf(pc, q, -0x1.3bd3ccp+0f);
    c = fmaf(pc, q, 1.0f);
}

// arctan on |u| <= tan(pi/8): odd series with coefficients (-1)^m/(2m+1), m <= 8.
__device__ __forceinline__ float atan_small(float u) {
    const float q = u * u;
    float p = 0x1.e1e1e2p-5f;
    p = fmaf(p, q, -0x1.111112p-4f);
    p = fmaf(p, q, 0x1.3b13b2p-4f);
    p = fmaf(p, q, -0x1.745d18p-4f);
    p = fmaf(p, q, 0x1.c71c72p-4f);
    p = fmaf(p, q, -0x1.24924ap-3f);
    p = fmaf(p, q, 0x1.99999ap-3f);
    p = fmaf(p, q, -0x1.555556p-2f);
    p = fmaf(p, q, 1.0f);
    return p * u;
}

// Angle of (x, y) in [-pi, pi]: reduce to the first octant, then above
// tan(pi/8) use atan r = pi/4 + atan((r - 1)/(r + 1)).
__device__ __forceinline__ float angle2(float y, float x) {
    const float ax = fabsf(x);
    const float ay = fabsf(y);
    const bool steep = ay > ax;
    const float big = steep ? ay : ax;
    const float small = steep ? ax : ay;
    if (big == 0.0f) return 0.0f;
    const float r = small / big;
    float a;
    if (r > kTanEighthPi) {
        a = kQuarterPi + atan_small((r - 1.0f) / (r + 1.0f));
    } else {
        a = atan_small(r);
    }
    if (steep) a = kHalfPi - a;
    if (x < 0.0f) a = kPi - a;
    if (y < 0.0f) a = -a;
    return a;
}

// ---------------------------------------------------------------------------
// Cosine-weighted direction about unit normal (nx, ny, nz): a uniform point on
// the unit disc (radius sqrt(u1), angle 2 pi u2, the angle split into a quarter
// turn index and a fraction) lifted to the hemisphere (Malley), then carried to
// world space by the branchless orthonormal basis of Duff et al. (JCGT 2017).
struct V3 {
    float x, y, z;
};

// Correctly rounded square root of x = +0 or x in [2^-96, 2^126): the hardware
// estimate s moved one unit in the last place down or up by the signs of the
// fused residuals x - s' s of its two neighbours s' (the rounding correction
// the compiler applies to sqrtf, without the rescaling of tiny operands and the
// zero, infinity and NaN cases, which such x do not need).
__device__ __forceinline__ float sqrt_rn(float x) {
    const float s = __builtin_amdgcn_sqrtf(x);
    const float dn = __uint_as_float(__float_as_uint(s) - 1u);
    const float up = __uint_as_float(__float_as_uint(s) + 1u);
    const float r_dn = fmaf(-dn, s, x);
    const float r_up = fmaf(-up, s, x);
    const float t = r_dn <= 0.0f ? dn : s;
    return r_up > 0.0f ? up : t;
}

// u1 is k 2^-24 with 0 <= k < 2^24, or (k + 1/2) / M with M < 2^16 in the
// quadrature, so both square-root operands are +0 or at least 2^-24.
__device__ __forceinline__ V3 cosine_dir(float nx, float ny, float nz, float u1, float u2) {
    const float radius = sqrt_rn(u1);
    const float height = sqrt_rn(1.0f - u1);
    const float turns = u2 * 4.0f;
    const int quadrant = (int)turns;
    const float frac = turns - (float)quadrant;
    float s, c;
    quarter_sincos(frac, s, c);
    // (cos, sin) of the angle turned by `quadrant` quarter turns: (c, s),
    // (-s, c), (-c, -s), (s, -c); swaps and sign flips only, so exact
    const bool odd = (quadrant & 1) != 0;
    const unsigned flip_x = (unsigned)((quadrant ^ (quadrant >> 1)) & 1) << 31;
    const unsigned flip_y = (unsigned)(quadrant >> 1) << 31;
    const float ex = __uint_as_float(__float_as_uint(odd ? s : c) ^ flip_x);
    const float ey = __uint_as_float(__float_as_uint(odd ? c : s) ^ flip_y);
    const float lx = radius * ex;
    const float ly = radius * ey;

    const float sg = copysignf(1.0f, nz);
    const float a = -1.0f / (sg + nz);
    const float b = (nx * ny) * a;
    const V3 t{1.0f + ((sg * nx) * nx) * a, sg * b, -(sg * nx)};
    const V3 bt{b, sg + (ny * ny) * a, -ny};
    return V3{fmaf(lx, t.x, fmaf(ly, bt.x, height * nx)),
              fmaf(lx, t.y, fmaf(ly, bt.y, height * ny)),
              fmaf(lx, t.z, fmaf(ly, bt.z, height * nz))};
}

// Equirectangular nearest texel of a direction: polar angle from +z picks the
// row, azimuth from +x towards +y the column.
__device__ __forceinline__ void env_texel(float dx, float dy, float dz, int He, int We,
                                          int& row, int& col) {
    const float rxy = sqrtf(fmaf(dx, dx, dy * dy));
    const float polar = angle2(rxy, dz);
    float azim = angle2(dy, dx);
    if (azim < 0.0f) azim = azim + kTwoPi;
    int r = (int)((polar * kInvPi) * (float)He);
    int c = (int)((azim * kInvTwoPi) * (float)We);
    row = r < 0 ? 0 : (r > He - 1 ? He - 1 : r);
    col = c < 0 ? 0 : (c > We - 1 ? We - 1 : c);
}

}  // namespace dm
}  // namespace irtps
