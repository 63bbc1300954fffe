// Device-side input encoding of one path vertex (Sec. 3.6 "Input Encoding",
// Table "parameters", Sec. 5 "High-performance primitives for encoding"),
// shared by the stand-alone encoding kernel and the fused raw-record
// inference kernels.
#pragma once

#include "nrc_internal.h"

namespace nrc {

constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kPi = 3.14159265358979323846f;

// x mod 2 in [0, 2), exact: x/2, floor and 2*floor are exact, and x - 2k has
// fewer significant bits than x.
__device__ inline float mod2(float x) { return x - 2.0f * floorf(x * 0.5f); }

// Antiderivative of the quartic kernel 15/16 (1 - u^2)^2 on [-1, 1], 0 below
// and 1 above.  Clamping u first is branch-free and exact at the ends: with
// u = +-1 every partial sum of the (dyadic) coefficients is exact, giving 1 and 0.
__device__ inline float quartic_cdf(float u) {
    const float uc = fminf(fmaxf(u, -1.0f), 1.0f);
    const float u2 = uc * uc;
    return 0.5f + uc * (0.9375f + u2 * (-0.625f + 0.1875f * u2));
}

// sin(pi r) and cos(pi r) for r in [0, 2) on the transcendental unit, whose
// v_sin_f32 / v_cos_f32 take their argument in revolutions (r / 2).  On this
// range their absolute error is below 1.3e-7, measured against double
// precision over 2^24 points, the same as a degree-10 polynomial.
__device__ inline void sincospi_r(float r, float* sn, float* cs) {
    const float rev = 0.5f * r;
    *sn = __builtin_amdgcn_sinf(rev);
    *cs = __builtin_amdgcn_cosf(rev);
}

// One-blob encoding with 4 bins on [0,1]: mass of a quartic blob of half-width
// one bin centred at 4s over each bin; the edge bins also take the tails.
__device__ inline void one_blob4(float s, float* e) {
    const float c = 4.0f * s;
    const float f1 = quartic_cdf(1.0f - c);
    const float f2 = quartic_cdf(2.0f - c);
    const float f3 = quartic_cdf(3.0f - c);
    e[0] = f1;
    e[1] = f2 - f1;
    e[2] = f3 - f2;
    e[3] = 1.0f - f3;
}

// The Gaussian one-blob the quartic kernel replaces (Sec. 5 "cheap
// primitives"), one bin per standard deviation: bin masses from the normal
// CDF (1 + erf(u / sqrt 2)) / 2; the edge bins also take the tails.
__device__ inline float gauss_cdf(float u) { return 0.5f + 0.5f * erff(u * 0.707106781186547524f); }

__device__ inline void one_blob4_gauss(float s, float* e) {
    const float c = 4.0f * s;
    const float f1 = gauss_cdf(1.0f - c);
    const float f2 = gauss_cdf(2.0f - c);
    const float f3 = gauss_cdf(3.0f - c);
    e[0] = f1;
    e[1] = f2 - f1;
    e[2] = f3 - f2;
    e[3] = 1.0f - f3;
}

// Unit vector -> spherical coordinates normalised to [0,1]^2.
__device__ inline void sph(float x, float y, float z, float& u, float& w) {
    u = acosf(fminf(fmaxf(z, -1.0f), 1.0f)) * kInvPi;
    w = (atan2f(y, x) + kPi) * (0.5f * kInvPi);
}

// Triangle wave of Sec. 5 (figure "cheap primitives"), the stand-in for the
// frequency encoding's sine: tri(x) = 2 |x mod 2 - 1| - 1, period 2, tri(0) = 1.
// The reduction is exact; r - 1 is exact for r >= 1/2 and rounds by at most
// 2^-25 below it, and 2|.| - 1 is exact (Sterbenz), so |error| <= 2^-24.
__device__ inline float tri(float x) { return 2.0f * fabsf(mod2(x) - 1.0f) - 1.0f; }

// sin and cos of pi * 2^d * p for d = 0 .. NOCT-1.  Octaves 0, 3, 6, 9 are
// evaluated directly (sincospi_r of the exactly reduced phase); the two octaves
// after each come from the double-angle identities sin 2a = 2 sin a cos a,
// cos 2a = (cos a - sin a)(cos a + sin a), which at most quadruple the
// absolute rounding error (a few 1e-7).  Each product is rounded as written:
// with contraction the compiler may fuse either octave's product into the
// next octave's sum, and which one it picks depends on the surrounding code,
// so the stand-alone and fused encodings would round differently.
template <int NOCT>
__device__ inline void octaves(float p, float* sn, float* cs) {
    #pragma clang fp contract(off)
    #pragma unroll
    for (int d = 0; d < NOCT; ++d) {
        if (d % 3 == 0) {
            sincospi_r(mod2(p * (float)(1 << d)), &sn[d], &cs[d]);
        } else {
            const float s0 = sn[d - 1], c0 = cs[d - 1];
            sn[d] = 2.0f * s0 * c0;
            cs[d] = (c0 - s0) * (c0 + s0);
        }
    }
}

// The encoded features of one raw record (14 or 16 floats) in five parts, so
// that a caller can spread the work: part 0..2 the frequency encoding of
// position coordinate 0..2 (features 12c .. 12c + 11), part 3 the one-blobs of
// the first two angles (36..43), part 4 those of the last two angles and the
// remaining features (44..63).
//   config preset: per position coordinate sin, cos of 6 octaves (36), one-blob
//   of the direction and normal angles (16), roughness, diffuse and specular
//   albedo (7), five zeros.
//   paper preset: 12 sines per coordinate (36), one-blob of the angles (16),
//   one-blob of 1 - exp(-roughness) (4), albedos (6), two ones.
//   paper-tri preset: as paper with tri(2^d p) in place of sin(2^d pi p).
//   paper-gauss preset: as paper with Gaussian one-blobs.
template <int PRESET, int LAYOUT, int PART>
__device__ inline void encode_part(const float* x, float* o) {
    constexpr bool paper = PRESET != NRC_PRESET_CONFIG;
    constexpr bool gauss = PRESET == NRC_PRESET_PAPER_GAUSS;
    if constexpr (PART <= 2) {
        constexpr int c = PART;
        if (PRESET == NRC_PRESET_PAPER_TRI) {
            #pragma unroll
            for (int d = 0; d < 12; ++d) o[12 * c + d] = tri(x[c] * (float)(1 << d));
        } else if (PRESET == NRC_PRESET_PAPER || PRESET == NRC_PRESET_PAPER_GAUSS) {
            float sn[12], cs[12];
            octaves<12>(x[c], sn, cs);
            #pragma unroll
            for (int d = 0; d < 12; ++d) o[12 * c + d] = sn[d];
        } else {
            float sn[6], cs[6];
            octaves<6>(x[c], sn, cs);
            #pragma unroll
            for (int d = 0; d < 6; ++d) {
                o[12 * c + 2 * d] = sn[d];
                o[12 * c + 2 * d + 1] = cs[d];
            }
        }
    } else {
        constexpr int a0 = PART == 3 ? 0 : 2;      // first angle of this part
        float ang[2];
        if (LAYOUT == NRC_RAW14) {
            ang[0] = x[3 + a0];
            ang[1] = x[4 + a0];
        } else {
            sph(x[3 + 3 * (a0 / 2)], x[4 + 3 * (a0 / 2)], x[5 + 3 * (a0 / 2)], ang[0], ang[1]);
        }
        #pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (gauss) one_blob4_gauss(ang[a], o + 36 + 4 * (a0 + a)); else one_blob4(ang[a], o + 36 + 4 * (a0 + a));
        }
        if constexpr (PART == 4) {
            const float* rest = x + (LAYOUT == NRC_RAW14 ? 7 : 9);
            if (paper) {
                if (gauss) one_blob4_gauss(1.0f - expf(-rest[0]), o + 52); else one_blob4(1.0f - expf(-rest[0]), o + 52);
                #pragma unroll
                for (int j = 0; j < 6; ++j) o[56 + j] = rest[1 + j];
                o[62] = 1.0f;
                o[63] = 1.0f;
            } else {
                #pragma unroll
                for (int j = 0; j < 7; ++j) o[52 + j] = rest[j];
                #pragma unroll
                for (int j = 59; j < 64; ++j) o[j] = 0.0f;
            }
        }
    }
}

// The 64 encoded features of one raw record: all five parts.
template <int PRESET, int LAYOUT>
__device__ inline void encode_record(const float* x, float* o) {
    encode_part<PRESET, LAYOUT, 0>(x, o);
    encode_part<PRESET, LAYOUT, 1>(x, o);
    encode_part<PRESET, LAYOUT, 2>(x, o);
    encode_part<PRESET, LAYOUT, 3>(x, o);
    encode_part<PRESET, LAYOUT, 4>(x, o);
}

}  // namespace nrc
