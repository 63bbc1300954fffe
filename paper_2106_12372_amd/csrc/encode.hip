// Input encoding kernel (Sec. 3.6 "Input Encoding", Table "parameters", and
// Sec. 5 "High-performance primitives for encoding").
//
// One thread per path vertex.  A workgroup of 128 vertices stages its raw
// records through LDS with 16-byte loads, each thread builds its 64-wide
// encoded row in LDS, and the workgroup writes the rows back with 16-byte
// stores, so both HBM streams stay fully coalesced.  The kernel is bound by
// HBM bandwidth: 56 (or 64) bytes in and 128 (FP16/BF16) or 256 (FP32) bytes
// out per vertex.
#include "encode_impl.h"

namespace nrc {
namespace {

constexpr int kEncBlock = 128;

template <typename T> __device__ inline T to_t(float x);
template <> __device__ inline float to_t<float>(float x) { return x; }
template <> __device__ inline _Float16 to_t<_Float16>(float x) { return (_Float16)x; }
template <> __device__ inline __bf16 to_t<__bf16>(float x) { return (__bf16)x; }

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
        float f[64];
        encode_record<PRESET, LAYOUT>(sraw + r * RW, f);
        T* o = sout + r * ROW;
        #pragma unroll
        for (int k = 0; k < 64; ++k) o[k] = to_t<T>(f[k]);
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
#define NRC_ENC_LAUNCH(PR, LA) \
    hipLaunchKernelGGL((k_encode<T, PR, LA>), grid, block, 0, s, raw, n, enc)
    const bool r14 = layout == NRC_RAW14;
    if (preset == NRC_PRESET_PAPER_GAUSS) {
        if (r14) NRC_ENC_LAUNCH(NRC_PRESET_PAPER_GAUSS, NRC_RAW14); else NRC_ENC_LAUNCH(NRC_PRESET_PAPER_GAUSS, NRC_RAW16);
    } else if (preset == NRC_PRESET_PAPER_TRI) {
        if (r14) NRC_ENC_LAUNCH(NRC_PRESET_PAPER_TRI, NRC_RAW14); else NRC_ENC_LAUNCH(NRC_PRESET_PAPER_TRI, NRC_RAW16);
    } else if (preset == NRC_PRESET_PAPER) {
        if (r14) NRC_ENC_LAUNCH(NRC_PRESET_PAPER, NRC_RAW14); else NRC_ENC_LAUNCH(NRC_PRESET_PAPER, NRC_RAW16);
    } else {
        if (r14) NRC_ENC_LAUNCH(NRC_PRESET_CONFIG, NRC_RAW14); else NRC_ENC_LAUNCH(NRC_PRESET_CONFIG, NRC_RAW16);
    }
#undef NRC_ENC_LAUNCH
    return hipGetLastError();
}

}  // namespace

hipError_t launch_encode(int precision, int preset, int layout, const float* raw, int64_t n,
                         void* enc, hipStream_t s) {
    switch (precision) {
        case NRC_FP32:
        case NRC_FP32_VALU: return dispatch_encode<float>(preset, layout, raw, n, (float*)enc, s);
        case NRC_FP16: return dispatch_encode<_Float16>(preset, layout, raw, n, (_Float16*)enc, s);
        default: return dispatch_encode<__bf16>(preset, layout, raw, n, (__bf16*)enc, s);
    }
}

}  // namespace nrc
