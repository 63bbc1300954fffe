// Plain FP32 form of the network on the vector ALUs only, no matrix
// instructions (Sec. 4 and Sec. 5 "Architecture"): NRC_FP32_VALU, the
// precision baseline the matrix-core forms are compared with.  Packed FP32 is
// not used, so its arithmetic peak is 78.6 TFLOP/s (256 CUs x 4 SIMDs x 16
// lanes x 2 FLOP x 2.4 GHz).
//
// Inference: one lane per query; the query's 64 activations live in VGPRs and
// every weight is a wave-uniform operand fetched with scalar loads, so a layer
// is 4096 FMAs per lane with no LDS or cross-lane traffic.
//
// Training: NWV waves own a tile of 64 records.  Activations of every layer
// stay in LDS ([record][feature], padded rows).  In the forward and
// data-backward passes wave w produces features w*64/NWV.. of all 64 records
// (lane = record); for the weight gradient it produces those rows of dW_l for
// all input features (lane = input feature), summing over the tile's records.
// Each tile writes its dW partial in row-major order; the fixed-order
// reduction of the other forms sums them.
#include "encode_impl.h"
#include "nrc_internal.h"

namespace nrc {
namespace {

constexpr int kW = 64;      // the FP32 forms support width 64
constexpr int kLd = 68;     // padded LDS row stride (floats)
constexpr int kTile = 64;   // training records per workgroup
constexpr int kTrainWaves = 16;

// One 64 -> 64 ReLU layer on the activations in h (VGPRs); every weight is a
// wave-uniform operand fetched with scalar loads.
__device__ inline void layer_fp32(float (&h)[kW], const float* __restrict__ wl) {
    float z[kW];
    #pragma unroll
    for (int o = 0; o < kW; ++o) {
        float acc = 0.0f;
        #pragma unroll
        for (int k = 0; k < kW; ++k) acc = fmaf(wl[o * kW + k], h[k], acc);
        z[o] = acc;
    }
    #pragma unroll
    for (int o = 0; o < kW; ++o) h[o] = relu(z[o]);
}

// The network on one record whose 64 input features are in h.
__device__ inline void mlp_fp32(float (&h)[kW], const float* __restrict__ w, int n_hidden,
                                float (&y)[kNOut]) {
    for (int l = 0; l < n_hidden; ++l) layer_fp32(h, w + l * kW * kW);
    const float* wo = w + n_hidden * kW * kW;
    #pragma unroll
    for (int o = 0; o < kNOut; ++o) {
        float acc = 0.0f;
        #pragma unroll
        for (int k = 0; k < kW; ++k) acc = fmaf(wo[o * kW + k], h[k], acc);
        y[o] = acc;
    }
}

// Output of one query: the network output times the reflectance factor.
__device__ inline void store_query(float* __restrict__ rgb, int64_t s, const float (&y)[kNOut],
                                   const float (&r)[kNOut]) {
    rgb[s * 3 + 0] = y[0] * r[0];
    rgb[s * 3 + 1] = y[1] * r[1];
    rgb[s * 3 + 2] = y[2] * r[2];
}

__global__ __launch_bounds__(256) void k_fwd_fp32_valu(const float* __restrict__ w,
                                                  const float* __restrict__ enc, int64_t n,
                                                  float* __restrict__ rgb, int n_hidden, int fcol) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float h[kW];
    const float4* row = reinterpret_cast<const float4*>(enc + s * kEncWidth);
    #pragma unroll
    for (int q = 0; q < 16; ++q) {
        const float4 v = row[q];
        h[4 * q] = v.x; h[4 * q + 1] = v.y; h[4 * q + 2] = v.z; h[4 * q + 3] = v.w;
    }
    float r[kNOut], y[kNOut];
    reflectance_row(h, fcol, r);
    mlp_fp32(h, w, n_hidden, y);
    store_query(rgb, s, y, r);
}

// Inference from raw records with the encoding fused in: each lane encodes its
// record straight into the VGPRs of the first layer's input.
template <int PRESET, int LAYOUT>
__global__ __launch_bounds__(256) void k_fwd_raw_fp32_valu(const float* __restrict__ w,
                                                      const float* __restrict__ raw, int64_t n,
                                                      float* __restrict__ rgb, int n_hidden, int fcol) {
    constexpr int RW = LAYOUT == NRC_RAW14 ? 14 : 16;
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float x[RW];
    const float2* src = reinterpret_cast<const float2*>(raw + s * RW);
    #pragma unroll
    for (int q = 0; q < RW / 2; ++q) {
        const float2 v = src[q];
        x[2 * q] = v.x; x[2 * q + 1] = v.y;
    }
    float h[kW];
    encode_record<PRESET, LAYOUT>(x, h);
    float r[kNOut], y[kNOut];
    reflectance_row(h, fcol, r);
    mlp_fp32(h, w, n_hidden, y);
    store_query(rgb, s, y, r);
}

// UPSTREAM = false: targets given, relative L2 loss (Eq. 5) produces dL/dy.
// UPSTREAM = true : tgt holds an upstream gradient dL/dy directly.
// With the reflectance factorisation (fcol != 0) y is the network output times
// R = alpha + beta; the network's output gradient is dL/dy * R, and dL/denc
// also takes dL/dy_c * f_c on both albedo columns of channel c.
// NWV waves share a tile of 64 records; wave w owns FPW = 64 / NWV features
// (forward and data backward, lane = record) and FPW rows of each dW_l (lane =
// input feature).  More waves per tile give each SIMD more waves to hide the
// latency of LDS and scalar weight loads.
// RAWL >= 0: the training records are given raw (that layout, encoded with
// PRESET): enc points at FP32 [n][14 or 16] records and the first wave's lane s
// encodes sample s into its h_0 row.
template <bool UPSTREAM, bool GENC, int NWV, int RAWL = -1, int PRESET = NRC_PRESET_CONFIG>
__global__ __launch_bounds__(64 * NWV) void k_train_fp32_valu(const float* __restrict__ w,
                                                         const float* __restrict__ enc,
                                                         const float* __restrict__ tgt,
                                                         const int32_t* __restrict__ idx, int64_t n,
                                                         int n_hidden, int n_params, float loss_eps,
                                                         float grad_scale, float* __restrict__ partials,
                                                         float* __restrict__ loss_part,
                                                         int32_t* __restrict__ tile_bad,
                                                         float* __restrict__ genc, int fcol, LcgGather lg) {
    constexpr int FPW = kW / NWV;                          // features (or dW rows) per wave
    constexpr int NT = 64 * NWV;
    extern __shared__ __attribute__((aligned(16))) float smem[];
    float* hs = smem;                                     // (n_hidden+1) x [64][kLd]
    float* dbuf0 = hs + (n_hidden + 1) * kTile * kLd;     // 2 x [64][kLd]
    float* dbuf1 = dbuf0 + kTile * kLd;
    float* dout = dbuf1 + kTile * kLd;                    // [64][4]: dL/d(network output)
    float* fout = dout + kTile * 4;                       // [64][4]: network output

    // The wave index is uniform across the wave; saying so lets weight
    // addresses that depend on it use scalar loads.
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t tile = blockIdx.x;
    const int64_t row = tile * kTile + lane;
    const bool valid = row < n;
    // record read for this slot: idx[row] or the LCG orbit for a gathered batch, else row
    const int64_t src = !valid ? 0 : gather_row(idx, lg, row);
    float* part = partials + tile * (int64_t)n_params;
    const int f0 = FPW * wave;                            // this wave's first feature / dW row

    // Stage the tile's inputs as h_0 (zeros past the end of the batch).
    if constexpr (RAWL >= 0) {
        static_assert(!UPSTREAM && !GENC, "raw records feed the training step only");
        constexpr int RW = RAWL == NRC_RAW14 ? 14 : 16;
        if (wave == 0) {
            float f[64];
            if (valid) {
                const float* rr = enc + src * RW;
                float x[RW];
                #pragma unroll
                for (int k = 0; k < RW; ++k) x[k] = rr[k];
                encode_record<PRESET, RAWL>(x, f);
            } else {
                #pragma unroll
                for (int k = 0; k < 64; ++k) f[k] = 0.0f;
            }
            #pragma unroll
            for (int q = 0; q < 16; ++q)
                *reinterpret_cast<float4*>(hs + lane * kLd + 4 * q) =
                    make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
        }
    } else {
        for (int i = tid; i < kTile * 16; i += NT) {
            const int s = i >> 4, q = i & 15;
            const int64_t r = tile * kTile + s;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < n) v = reinterpret_cast<const float4*>(enc + gather_row(idx, lg, r) * kEncWidth)[q];
            *reinterpret_cast<float4*>(hs + s * kLd + 4 * q) = v;
        }
    }
    __syncthreads();

    // Forward: wave w writes features f0..f0+FPW-1 of every sample (lane = sample).
    // Layer l's weights start at w + l * 64 * 64 (the input layer is 64 x 64
    // too); addressing them from the base pointer, not a running one, keeps the
    // scalar register file from spilling.
    for (int l = 0; l < n_hidden; ++l) {
        const float* wl = w + l * kW * kW;
        const float* hin = hs + l * kTile * kLd + lane * kLd;
        float* hout = hs + (l + 1) * kTile * kLd + lane * kLd;
        float acc[FPW];
        #pragma unroll
        for (int j = 0; j < FPW; ++j) acc[j] = 0.0f;
        #pragma unroll
        for (int k4 = 0; k4 < 16; ++k4) {
            const float4 hv = *reinterpret_cast<const float4*>(hin + 4 * k4);
            #pragma unroll
            for (int j = 0; j < FPW; ++j) {
                const float* wr = wl + (f0 + j) * kW + 4 * k4;
                acc[j] = fmaf(wr[0], hv.x, acc[j]);
                acc[j] = fmaf(wr[1], hv.y, acc[j]);
                acc[j] = fmaf(wr[2], hv.z, acc[j]);
                acc[j] = fmaf(wr[3], hv.w, acc[j]);
            }
        }
        #pragma unroll
        for (int j4 = 0; j4 < FPW / 4; ++j4)
            *reinterpret_cast<float4*>(hout + f0 + 4 * j4) =
                make_float4(relu(acc[4 * j4]), relu(acc[4 * j4 + 1]),
                            relu(acc[4 * j4 + 2]), relu(acc[4 * j4 + 3]));
        __syncthreads();
    }
    const float* wout = w + n_hidden * kW * kW;           // [3][64]
    const float* hlast = hs + n_hidden * kTile * kLd;

    // Output layer, loss and dL/dy (wave 0, lane = sample).
    if (wave == 0) {
        float f[kNOut] = {0.f, 0.f, 0.f};
        const float* hr = hlast + lane * kLd;
        #pragma unroll
        for (int k = 0; k < kW; ++k) {
            const float hv = hr[k];
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) f[o] = fmaf(wout[o * kW + k], hv, f[o]);
        }
        float r[kNOut] = {1.f, 1.f, 1.f};
        if (fcol) {
            const float* h0 = hs + lane * kLd;
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) r[o] = h0[fcol + o] + h0[fcol + 3 + o];
        }
        float d[kNOut] = {0.f, 0.f, 0.f};
        float lterm = 0.0f;
        if (valid) {
            if (UPSTREAM) {
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) d[o] = tgt[src * 3 + o] * grad_scale * r[o];
            } else {
                float y[kNOut];
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) y[o] = f[o] * r[o];
                const float lum = (y[0] + y[1] + y[2]) * (1.0f / 3.0f);
                const float inv_den = 1.0f / fmaf(lum, lum, loss_eps);
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) {
                    const float diff = y[o] - tgt[src * 3 + o];
                    lterm = fmaf(diff * diff, inv_den, lterm);
                    d[o] = 2.0f * diff * inv_den * grad_scale * r[o];
                }
            }
        }
        *reinterpret_cast<float4*>(dout + lane * 4) = make_float4(d[0], d[1], d[2], 0.f);
        if (GENC) *reinterpret_cast<float4*>(fout + lane * 4) = make_float4(f[0], f[1], f[2], 0.f);
        const float tot = wave_sum_compensated(lterm);
        if (lane == 0) loss_part[tile] = tot;
    }
    __syncthreads();

    // delta_H = W_H^T dL/dy, masked by ReLU'(z_H); wave w: features f0..f0+FPW-1.
    {
        const float4 dv = *reinterpret_cast<const float4*>(dout + lane * 4);
        const float* hr = hlast + lane * kLd + f0;
        float* dst = dbuf0 + lane * kLd + f0;
        #pragma unroll
        for (int j = 0; j < FPW; ++j) {
            const int i = f0 + j;
            float g = wout[i] * dv.x;
            g = fmaf(wout[kW + i], dv.y, g);
            g = fmaf(wout[2 * kW + i], dv.z, g);
            dst[j] = hr[j] > 0.0f ? g : 0.0f;
        }
    }
    // dW_H[o][i] = sum_s dL/dy[s][o] h_H[s][i]; wave o < 3, lane = i.
    bool bad = false;   // any non-finite weight-gradient partial in this tile
    if (wave < kNOut) {
        float acc = 0.0f;
        for (int s = 0; s < kTile; ++s) acc = fmaf(dout[s * 4 + wave], hlast[s * kLd + lane], acc);
        __builtin_nontemporal_store(acc, &part[(n_params - kNOut * kW) + wave * kW + lane]);
        bad |= !isfinite(acc);
    }
    __syncthreads();

    float* dcur = dbuf0;
    float* dnxt = dbuf1;
    int off = n_params - kNOut * kW;
    for (int l = n_hidden - 1; l >= 0; --l) {
        const int cols = (l == 0) ? kEncWidth : kW;
        off -= kW * cols;
        const float* wlay = w + off;
        const float* hl = hs + l * kTile * kLd;
        // dW_l rows f0..f0+FPW-1, lane = input feature i.
        {
            float acc[FPW];
            #pragma unroll
            for (int j = 0; j < FPW; ++j) acc[j] = 0.0f;
            for (int s = 0; s < kTile; ++s) {
                const float hv = hl[s * kLd + lane];
                const float* dr = dcur + s * kLd + f0;
                #pragma unroll
                for (int j4 = 0; j4 < FPW / 4; ++j4) {
                    const float4 dv = *reinterpret_cast<const float4*>(dr + 4 * j4);
                    acc[4 * j4] = fmaf(dv.x, hv, acc[4 * j4]);
                    acc[4 * j4 + 1] = fmaf(dv.y, hv, acc[4 * j4 + 1]);
                    acc[4 * j4 + 2] = fmaf(dv.z, hv, acc[4 * j4 + 2]);
                    acc[4 * j4 + 3] = fmaf(dv.w, hv, acc[4 * j4 + 3]);
                }
            }
            #pragma unroll
            for (int j = 0; j < FPW; ++j) {
                // streamed past the caches: read once, by the reduction
                __builtin_nontemporal_store(acc[j], &part[off + (f0 + j) * cols + lane]);
                bad |= !isfinite(acc[j]);
            }
        }
        // delta_l = W_l^T delta_{l+1}, masked (l >= 1); or dL/dh_0 (l == 0).
        if (l >= 1 || GENC) {
            float acc[FPW];
            #pragma unroll
            for (int j = 0; j < FPW; ++j) acc[j] = 0.0f;
            const float* dr = dcur + lane * kLd;
            #pragma unroll
            for (int o4 = 0; o4 < 16; ++o4) {
                const float4 dv = *reinterpret_cast<const float4*>(dr + 4 * o4);
                #pragma unroll
                for (int j = 0; j < FPW; ++j) {
                    const float* wc = wlay + (4 * o4) * cols + f0 + j;
                    acc[j] = fmaf(wc[0], dv.x, acc[j]);
                    acc[j] = fmaf(wc[cols], dv.y, acc[j]);
                    acc[j] = fmaf(wc[2 * cols], dv.z, acc[j]);
                    acc[j] = fmaf(wc[3 * cols], dv.w, acc[j]);
                }
            }
            if (l >= 1) {
                const float* hr = hl + lane * kLd + f0;
                float* dst = dnxt + lane * kLd + f0;
                #pragma unroll
                for (int j = 0; j < FPW; ++j) dst[j] = hr[j] > 0.0f ? acc[j] : 0.0f;
            } else if (valid) {
                // the loss scale of the upstream gradient divided out
                const float inv_scale = 1.0f / grad_scale;
                #pragma unroll
                for (int j = 0; j < FPW; ++j) acc[j] *= inv_scale;
                if (fcol) {
                    // d(f_c R_c)/d(albedo column) = f_c on the diffuse and specular column.
                    #pragma unroll
                    for (int j = 0; j < FPW; ++j) {
                        int c = f0 + j - fcol;
                        if (c >= 0 && c < 6) {
                            c = c >= 3 ? c - 3 : c;
                            acc[j] = fmaf(tgt[src * 3 + c], fout[lane * 4 + c], acc[j]);
                        }
                    }
                }
                #pragma unroll
                for (int j4 = 0; j4 < FPW / 4; ++j4)
                    *reinterpret_cast<float4*>(genc + row * kEncWidth + f0 + 4 * j4) =
                        make_float4(acc[4 * j4], acc[4 * j4 + 1], acc[4 * j4 + 2], acc[4 * j4 + 3]);
            }
        }
        __syncthreads();
        float* t = dcur; dcur = dnxt; dnxt = t;
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0) tile_bad[tile] = any_bad ? 1 : 0;
}

inline size_t train_lds_bytes(int n_hidden) {
    return ((size_t)(n_hidden + 1) * kTile * kLd + 2 * kTile * kLd + 2 * kTile * 4) * sizeof(float);
}

template <bool UP, bool GE, int RAWL = -1, int PRESET = NRC_PRESET_CONFIG>
hipError_t train_launch(const Geo& d, const float* w, const float* enc, const float* tgt, const int32_t* idx,
                        int64_t n, float loss_eps, float grad_scale, float* partials, float* loss_part,
                        int32_t* tile_bad, float* genc, LcgGather lg, hipStream_t s) {
    const int64_t tiles = (n + kTile - 1) / kTile;
    if (tiles == 0) return hipSuccess;
    const size_t lds = train_lds_bytes(d.H);
    auto k = k_train_fp32_valu<UP, GE, kTrainWaves, RAWL, PRESET>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(64 * kTrainWaves), lds, s, w, enc, tgt, idx, n, d.H,
                       d.n_params(), loss_eps, grad_scale, partials, loss_part, tile_bad, genc, d.F, lg);
    return hipGetLastError();
}

template <int PRESET, int LAYOUT>
hipError_t raw_launch(const Geo& d, const float* w, const float* raw, int64_t n, float* rgb, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd_raw_fp32_valu<PRESET, LAYOUT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       w, raw, n, rgb, d.H, d.F);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fwd_fp32_valu(const Geo& d, const float* w, const float* enc, int64_t n, float* rgb,
                                hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd_fp32_valu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, enc, n, rgb, d.H,
                       d.F);
    return hipGetLastError();
}

hipError_t launch_fwd_raw_fp32_valu(const Geo& d, int preset, int layout, const float* w, const float* raw,
                                    int64_t n, float* rgb, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const bool r14 = layout == NRC_RAW14;
    switch (preset) {
        case NRC_PRESET_PAPER:
            return r14 ? raw_launch<NRC_PRESET_PAPER, NRC_RAW14>(d, w, raw, n, rgb, s)
                       : raw_launch<NRC_PRESET_PAPER, NRC_RAW16>(d, w, raw, n, rgb, s);
        case NRC_PRESET_PAPER_TRI:
            return r14 ? raw_launch<NRC_PRESET_PAPER_TRI, NRC_RAW14>(d, w, raw, n, rgb, s)
                       : raw_launch<NRC_PRESET_PAPER_TRI, NRC_RAW16>(d, w, raw, n, rgb, s);
        case NRC_PRESET_PAPER_GAUSS:
            return r14 ? raw_launch<NRC_PRESET_PAPER_GAUSS, NRC_RAW14>(d, w, raw, n, rgb, s)
                       : raw_launch<NRC_PRESET_PAPER_GAUSS, NRC_RAW16>(d, w, raw, n, rgb, s);
        default:
            return r14 ? raw_launch<NRC_PRESET_CONFIG, NRC_RAW14>(d, w, raw, n, rgb, s)
                       : raw_launch<NRC_PRESET_CONFIG, NRC_RAW16>(d, w, raw, n, rgb, s);
    }
}

hipError_t launch_train_fp32_valu_raw(const Geo& d, int preset, int layout, const float* w, const float* raw,
                                      const float* tgt, const int32_t* idx, int64_t n, float loss_eps,
                                      float grad_scale, float* partials, float* loss_part, int32_t* tile_bad,
                                      hipStream_t s, LcgGather lg) {
#define NRC_TRAIN_RAW(PR, LA)                                                                                  \
    return train_launch<false, false, LA, PR>(d, w, raw, tgt, idx, n, loss_eps, grad_scale, partials,        \
                                              loss_part, tile_bad, nullptr, lg, s)
    const bool r14 = layout == NRC_RAW14;
    if (preset == NRC_PRESET_PAPER_GAUSS) {
        if (r14) NRC_TRAIN_RAW(NRC_PRESET_PAPER_GAUSS, NRC_RAW14); else NRC_TRAIN_RAW(NRC_PRESET_PAPER_GAUSS, NRC_RAW16);
    } else if (preset == NRC_PRESET_PAPER_TRI) {
        if (r14) NRC_TRAIN_RAW(NRC_PRESET_PAPER_TRI, NRC_RAW14); else NRC_TRAIN_RAW(NRC_PRESET_PAPER_TRI, NRC_RAW16);
    } else if (preset == NRC_PRESET_PAPER) {
        if (r14) NRC_TRAIN_RAW(NRC_PRESET_PAPER, NRC_RAW14); else NRC_TRAIN_RAW(NRC_PRESET_PAPER, NRC_RAW16);
    }
    if (r14) NRC_TRAIN_RAW(NRC_PRESET_CONFIG, NRC_RAW14);
    NRC_TRAIN_RAW(NRC_PRESET_CONFIG, NRC_RAW16);
#undef NRC_TRAIN_RAW
}

hipError_t launch_train_fp32_valu(const Geo& d, const float* w, const float* enc, const float* tgt,
                                  const int32_t* idx, int64_t n, bool upstream, float loss_eps, float grad_scale,
                                  float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                                  hipStream_t s, LcgGather lg) {
    if (!upstream)
        return train_launch<false, false>(d, w, enc, tgt, idx, n, loss_eps, grad_scale, partials, loss_part,
                                          tile_bad, genc, lg, s);
    if (genc)
        return train_launch<true, true>(d, w, enc, tgt, idx, n, loss_eps, grad_scale, partials, loss_part,
                                        tile_bad, genc, lg, s);
    return train_launch<true, false>(d, w, enc, tgt, idx, n, loss_eps, grad_scale, partials, loss_part, tile_bad,
                                     genc, lg, s);
}

}  // namespace nrc
