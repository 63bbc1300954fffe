// Input encoding kernel (Sec. 3.6 "Input Encoding", Table "parameters", and
// Sec. 5 "High-performance primitives for encoding").
//
// One thread per path vertex.  A workgroup of 128 vertices stages its raw
// records through LDS with 16-byte loads, each thread builds its 64-wide
// encoded row in LDS, and the workgroup writes the rows back with 16-byte
// stores, so both HBM streams stay fully coalesced.  The kernel is bound by
// HBM bandwidth: 56 (or 64) bytes in and 128 (FP16/BF16) or 256 (FP32) bytes
// out per vertex.
#include "nrc_internal.h"

namespace nrc {
namespace {

constexpr int kEncBlock = 128;
constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kPi = 3.14159265358979323846f;

template <typename T> __device__ inline T to_t(float x);
template <> __device__ inline float to_t<float>(float x) { return x; }
template <> __device__ inline _Float16 to_t<_Float16>(float x) { return (_Float16)x; }
template <> __device__ inline __bf16 to_t<__bf16>(float x) { return (__bf16)x; }

// x mod 2 in [0, 2), exact: x/2, floor and 2*floor are exact, and x - 2k has
// fewer significant bits than x.
__device__ inline float mod2(float x) { return x - 2.0f * floorf(x * 0.5f); }

// Antiderivative of the quartic kernel 15/16 (1 - u^2)^2 on [-1, 1], clamped
// to 0 below and 1 above.
__device__ inline float quartic_cdf(float u) {
    if (u <= -1.0f) return 0.0f;
    if (u >= 1.0f) return 1.0f;
    const float u2 = u * u;
    return 0.5f + u * (0.9375f + u2 * (-0.625f + 0.1875f * u2));
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

// Unit vector -> spherical coordinates normalised to [0,1]^2.
__device__ inline void sph(float x, float y, float z, float& u, float& w) {
    u = acosf(fminf(fmaxf(z, -1.0f), 1.0f)) * kInvPi;
    w = (atan2f(y, x) + kPi) * (0.5f * kInvPi);
}

template <typename T, int PRESET, int LAYOUT>
__global__ __launch_bounds__(kEncBlock) void k_encode(const float* __restrict__ raw, int64_t n,
                                                      T* __restrict__ enc) {
    constexpr int RW = LAYOUT == NRC_RAW14 ? 14 : 16;
    constexpr int ROW = 64 + 16 / (int)sizeof(T);  // padded LDS row, elements
    constexpr int CPR = 64 * (int)sizeof(T) / 16;  // 16-byte chunks per encoded row
    __shared__ __attribute__((aligned(16))) float sraw[kEncBlock * RW];
    __shared__ __attribute__((aligned(16))) T sout[kEncBlock * ROW];

    const int64_t base = (int64_t)blockIdx.x * kEncBlock;
    const int nrows = (int)min((int64_t)kEncBlock, n - base);
    const float* src = raw + base * RW;
    const int nf = nrows * RW;
    const int nf4 = nf >> 2;
    for (int i = threadIdx.x; i < nf4; i += kEncBlock)
        reinterpret_cast<float4*>(sraw)[i] = reinterpret_cast<const float4*>(src)[i];
    for (int i = (nf4 << 2) + threadIdx.x; i < nf; i += kEncBlock) sraw[i] = src[i];
    __syncthreads();

    const int r = threadIdx.x;
    if (r < nrows) {
        const float* x = sraw + r * RW;
        T* o = sout + r * ROW;
        // Position: frequency encoding with the phase reduced exactly mod 2.
        #pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float p = x[c];
            if (PRESET == NRC_PRESET_PAPER) {
                #pragma unroll
                for (int d = 0; d < 12; ++d) {
                    o[12 * c + d] = to_t<T>(sinpif(mod2(p * (float)(1 << d))));
                }
            } else {
                #pragma unroll
                for (int d = 0; d < 6; ++d) {
                    float sn, cs;
                    sincospif(mod2(p * (float)(1 << d)), &sn, &cs);
                    o[12 * c + 2 * d] = to_t<T>(sn);
                    o[12 * c + 2 * d + 1] = to_t<T>(cs);
                }
            }
        }
        // Direction and normal: spherical coordinates, then one-blob per coordinate.
        float ang[4];
        const float* rest;
        if (LAYOUT == NRC_RAW14) {
            ang[0] = x[3]; ang[1] = x[4]; ang[2] = x[5]; ang[3] = x[6];
            rest = x + 7;
        } else {
            sph(x[3], x[4], x[5], ang[0], ang[1]);
            sph(x[6], x[7], x[8], ang[2], ang[3]);
            rest = x + 9;
        }
        #pragma unroll
        for (int a = 0; a < 4; ++a) {
            float e[4];
            one_blob4(ang[a], e);
            #pragma unroll
            for (int j = 0; j < 4; ++j) o[36 + 4 * a + j] = to_t<T>(e[j]);
        }
        int k = 52;
        if (PRESET == NRC_PRESET_PAPER) {
            float e[4];
            one_blob4(1.0f - expf(-rest[0]), e);
            #pragma unroll
            for (int j = 0; j < 4; ++j) o[k + j] = to_t<T>(e[j]);
            k += 4;
        } else {
            o[k++] = to_t<T>(rest[0]);
        }
        #pragma unroll
        for (int j = 0; j < 6; ++j) o[k + j] = to_t<T>(rest[1 + j]);
        k += 6;
        const float pad = PRESET == NRC_PRESET_PAPER ? 1.0f : 0.0f;
        for (; k < 64; ++k) o[k] = to_t<T>(pad);
    }
    __syncthreads();

    T* dst = enc + base * 64;
    for (int i = threadIdx.x; i < nrows * CPR; i += kEncBlock) {
        const int rr = i / CPR, cc = i - rr * CPR;
        const uint4 v = *reinterpret_cast<const uint4*>(sout + rr * ROW + cc * (16 / (int)sizeof(T)));
        *reinterpret_cast<uint4*>(dst + (int64_t)rr * 64 + cc * (16 / (int)sizeof(T))) = v;
    }
}

template <typename T>
hipError_t dispatch_encode(int preset, int layout, const float* raw, int64_t n, T* enc,
                           hipStream_t s) {
    const int64_t blocks = (n + kEncBlock - 1) / kEncBlock;
    if (blocks == 0) return hipSuccess;
    const dim3 grid((unsigned)blocks), block(kEncBlock);
    if (preset == NRC_PRESET_PAPER) {
        if (layout == NRC_RAW14)
            hipLaunchKernelGGL((k_encode<T, NRC_PRESET_PAPER, NRC_RAW14>), grid, block, 0, s, raw, n, enc);
        else
            hipLaunchKernelGGL((k_encode<T, NRC_PRESET_PAPER, NRC_RAW16>), grid, block, 0, s, raw, n, enc);
    } else {
        if (layout == NRC_RAW14)
            hipLaunchKernelGGL((k_encode<T, NRC_PRESET_CONFIG, NRC_RAW14>), grid, block, 0, s, raw, n, enc);
        else
            hipLaunchKernelGGL((k_encode<T, NRC_PRESET_CONFIG, NRC_RAW16>), grid, block, 0, s, raw, n, enc);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_encode(int precision, int preset, int layout, const float* raw, int64_t n,
                         void* enc, hipStream_t s) {
    switch (precision) {
        case NRC_FP32: return dispatch_encode<float>(preset, layout, raw, n, (float*)enc, s);
        case NRC_FP16: return dispatch_encode<_Float16>(preset, layout, raw, n, (_Float16*)enc, s);
        default: return dispatch_encode<__bf16>(preset, layout, raw, n, (__bf16*)enc, s);
    }
}

}  // namespace nrc
