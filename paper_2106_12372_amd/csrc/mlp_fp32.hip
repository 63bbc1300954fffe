// Plain FP32 form of the network (Sec. 4 and Sec. 5 "Architecture"): every
// product and sum in single precision, the precision baseline for the 16-bit
// matrix-core forms.
//
// Inference runs on the FP32 matrix cores (v_mfma_f32_16x16x4_f32), whose dense
// rate equals the packed-FP32 vector rate, twice what unpacked vector FMAs
// reach.  A wave takes 64 queries, one per lane: each lane loads (or encodes)
// its query's 64 features, then a 4 x 4 transpose across the four 16-lane
// groups (v_permlane32_swap, v_permlane16_swap) turns them into the B operands
// of four 16-query columns with no LDS round trip.  A layer's accumulators are
// the next layer's B operands as they stand (the weight's K index follows the
// accumulator layout), so activations never leave VGPRs.  The weights of all
// layers sit in LDS as per-lane float4 A fragments, one workgroup per CU.
//
// Training: a workgroup of 16 waves owns a tile of 64 records.  Activations
// of every layer stay in LDS ([sample][feature], padded rows).  Each of the
// tile's three 64 x 64 products per layer (forward, data backward, weight
// gradient) is 16 blocks of 16 x 16, one per wave, each block 16 FP32 matrix
// instructions over a K of 64; operands come from LDS and, for weights, from
// the L2-resident master copy.  Each tile writes its dW partial; a separate
// fixed-order reduction sums the partials (no atomics, so results are
// reproducible).
#include "encode_impl.h"
#include "nrc_internal.h"

namespace nrc {
namespace {

constexpr int kW = 64;      // the FP32 form supports width 64
constexpr int kLd = 68;     // padded LDS row stride (floats)
constexpr int kTile = 64;       // training records per workgroup
constexpr int kQWaves = 8;      // waves per query workgroup (two per SIMD)
constexpr int kQMaxBlocks = 256;    // query workgroups: one per CU (LDS-bound)

typedef float f4 __attribute__((ext_vector_type(4)));

// Output of one query: the network output times the reflectance factor.
__device__ inline void store_query(float* __restrict__ rgb, int64_t s, const float (&y)[kNOut],
                                   const float (&r)[kNOut]) {
    rgb[s * 3 + 0] = y[0] * r[0];
    rgb[s * 3 + 1] = y[1] * r[1];
    rgb[s * 3 + 2] = y[2] * r[2];
}

// Transposes a 4 x 4 block of (16-lane group, register): afterwards register
// c of group g holds what register g of group c held.  permlane32_swap trades
// groups {2,3} of its first operand for groups {0,1} of its second;
// permlane16_swap trades groups {1,3} of its first for groups {0,2} of its
// second.
__device__ inline void xpose4(float& r0, float& r1, float& r2, float& r3) {
    const auto s02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(r0), __float_as_uint(r2), false, false);
    const auto s13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(r1), __float_as_uint(r3), false, false);
    const auto s01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
    const auto s23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
    r0 = __uint_as_float(s01[0]);
    r1 = __uint_as_float(s01[1]);
    r2 = __uint_as_float(s23[0]);
    r3 = __uint_as_float(s23[1]);
}

// Operand layout of v_mfma_f32_16x16x4_f32 (D = A B + C, 16 x 4 by 4 x 16):
// lane 16k + i supplies A[i][k], lane 16k + j supplies B[k][j], and lane
// 16g + j holds D[4g + r][j] in register r.  With j a query and i an output
// neuron of block ob, lane (g, j) ends a layer holding neurons 16 ob + 4g + r.
// The K step s = 4 ob' + r of the next layer therefore takes neuron
// 16 ob' + 4g + r from lane group g, and the A fragment of (ob, ob') gives lane
// (g, i) the float4 W[16 ob + i][16 ob' + 4g .. 16 ob' + 4g + 3], one element
// per r.  Fragments of layer l occupy [16 l, 16 l + 16) (index 4 ob + ob').
__device__ inline void stage_query_frags(f4* sw, const float* __restrict__ w, int H) {
    const int nfr = 16 * H;
    for (int idx = threadIdx.x; idx < nfr * 64; idx += blockDim.x) {
        const int f = idx >> 6, lane = idx & 63, g = lane >> 4, i = lane & 15;
        const int l = f >> 4, ob = (f >> 2) & 3, obp = f & 3;
        const float* src = w + l * kW * kW + (16 * ob + i) * kW + 16 * obp + 4 * g;
        sw[idx] = f4{src[0], src[1], src[2], src[3]};
    }
}

// The output layer's weights a lane needs: wo[o][b] = W_out[o][16b + 4g .. +3],
// the neurons lane group g holds.
__device__ inline void load_out_weights(const float* __restrict__ w, int H, int g, float4 (&wo)[kNOut][4]) {
    const float* base = w + H * kW * kW + 4 * g;
    #pragma unroll
    for (int o = 0; o < kNOut; ++o)
        #pragma unroll
        for (int b = 0; b < 4; ++b) wo[o][b] = *reinterpret_cast<const float4*>(base + o * kW + 16 * b);
}

// The network on the wave's 64 queries.  h: this lane's 64 input features; y:
// this lane's 3 outputs.  The hidden layers run on the matrix cores; the
// 3-row output layer, which would use 3 of an MFMA block's 16 rows, runs on
// the vector ALUs: each lane forms the partial dots over the 16 neurons it
// holds for its four columns' queries, and one transpose per channel gathers
// the four lane groups' partials onto the lane that loaded the query.
__device__ inline void mlp_query_mfma(const f4* __restrict__ sw, int H, int lane,
                                      const float4 (&wo)[kNOut][4], const float (&h)[kW],
                                      float (&y)[kNOut]) {
    float act[4][16];   // [column][K step]: lane group g, step 4b + r = neuron 16b + 4g + r
    #pragma unroll
    for (int b = 0; b < 4; ++b) {
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
            float q0 = h[16 * b + r], q1 = h[16 * b + 4 + r], q2 = h[16 * b + 8 + r], q3 = h[16 * b + 12 + r];
            xpose4(q0, q1, q2, q3);
            act[0][4 * b + r] = q0;
            act[1][4 * b + r] = q1;
            act[2][4 * b + r] = q2;
            act[3][4 * b + r] = q3;
        }
    }
    for (int l = 0; l < H; ++l) {
        const f4* fl = sw + l * 16 * 64 + lane;
        f4 acc[4][4];   // [column][ob]
        #pragma unroll
        for (int c = 0; c < 4; ++c)
            #pragma unroll
            for (int ob = 0; ob < 4; ++ob) acc[c][ob] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        #pragma unroll
        for (int obp = 0; obp < 4; ++obp) {
            #pragma unroll
            for (int ob = 0; ob < 4; ++ob) {
                const f4 a = fl[(4 * ob + obp) * 64];
                #pragma unroll
                for (int r = 0; r < 4; ++r)
                    #pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[c][ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], act[c][4 * obp + r], acc[c][ob], 0, 0, 0);
            }
        }
        #pragma unroll
        for (int c = 0; c < 4; ++c)
            #pragma unroll
            for (int ob = 0; ob < 4; ++ob)
                #pragma unroll
                for (int r = 0; r < 4; ++r) act[c][4 * ob + r] = fmaxf(acc[c][ob][r], 0.0f);
    }
    #pragma unroll
    for (int o = 0; o < kNOut; ++o) {
        float p[4];   // p[c]: this lane group's share of channel o for column c's query
        #pragma unroll
        for (int c = 0; c < 4; ++c) {
            float acc = 0.0f;
            #pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc = fmaf(wo[o][b].x, act[c][4 * b], acc);
                acc = fmaf(wo[o][b].y, act[c][4 * b + 1], acc);
                acc = fmaf(wo[o][b].z, act[c][4 * b + 2], acc);
                acc = fmaf(wo[o][b].w, act[c][4 * b + 3], acc);
            }
            p[c] = acc;
        }
        // afterwards register c of group g holds group c's share for column
        // g's query: the four registers of a lane add up to its own query
        xpose4(p[0], p[1], p[2], p[3]);
        y[o] = (p[0] + p[1]) + (p[2] + p[3]);
    }
}

// Inference: RAW = false reads 64 encoded features per query; RAW = true reads
// raw records and encodes them in the lane (Sec. 3.6).  A wave takes 64
// consecutive queries per tile; lanes past the end compute on the last query
// and store nothing, so every lane joins every matrix instruction.
template <bool RAW, int PRESET, int LAYOUT>
__device__ inline void query_fp32(const float* __restrict__ w, const float* __restrict__ in, int64_t n,
                                  float* __restrict__ rgb, int H, int fcol) {
    extern __shared__ f4 sw[];
    constexpr int RW = LAYOUT == NRC_RAW14 ? 14 : 16;
    stage_query_frags(sw, w, H);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float4 wo[kNOut][4];
    load_out_weights(w, H, lane >> 4, wo);
    __syncthreads();
    const int64_t n_tiles = (n + 63) / 64;
    const int64_t stride = (int64_t)gridDim.x * kQWaves;
    for (int64_t t = (int64_t)blockIdx.x * kQWaves + wave; t < n_tiles; t += stride) {
        int64_t s = t * 64 + lane;
        const bool valid = s < n;
        if (!valid) s = n - 1;
        float h[kW];
        if (RAW) {
            float x[RW];
            const float2* src = reinterpret_cast<const float2*>(in + s * RW);
            #pragma unroll
            for (int q = 0; q < RW / 2; ++q) {
                const float2 v = src[q];
                x[2 * q] = v.x; x[2 * q + 1] = v.y;
            }
            encode_record<PRESET, LAYOUT>(x, h);
        } else {
            const float4* row = reinterpret_cast<const float4*>(in + s * kEncWidth);
            #pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float4 v = row[q];
                h[4 * q] = v.x; h[4 * q + 1] = v.y; h[4 * q + 2] = v.z; h[4 * q + 3] = v.w;
            }
        }
        float r[kNOut], y[kNOut];
        reflectance_row(h, fcol, r);
        mlp_query_mfma(sw, H, lane, wo, h, y);
        if (valid) store_query(rgb, s, y, r);
    }
}

__global__ __launch_bounds__(64 * kQWaves) void k_fwd_fp32(const float* __restrict__ w,
                                                          const float* __restrict__ enc, int64_t n,
                                                          float* __restrict__ rgb, int n_hidden, int fcol) {
    query_fp32<false, NRC_PRESET_CONFIG, NRC_RAW14>(w, enc, n, rgb, n_hidden, fcol);
}

// Inference from raw records with the encoding fused in.
template <int PRESET, int LAYOUT>
__global__ __launch_bounds__(64 * kQWaves) void k_fwd_raw_fp32(const float* __restrict__ w,
                                                              const float* __restrict__ raw, int64_t n,
                                                              float* __restrict__ rgb, int n_hidden, int fcol) {
    query_fp32<true, PRESET, LAYOUT>(w, raw, n, rgb, n_hidden, fcol);
}

// UPSTREAM = false: targets given, relative L2 loss (Eq. 5) produces dL/dy.
// UPSTREAM = true : tgt holds an upstream gradient dL/dy directly.
// With the reflectance factorisation (fcol != 0) y is the network output times
// R = alpha + beta; the network's output gradient is dL/dy * R, and dL/denc
// also takes dL/dy_c * f_c on both albedo columns of channel c.
// NWV = 16 waves share a tile of 64 records.  In the three products of a
// layer wave w owns one 16 x 16 block (block row w / 4, block column w % 4);
// with the MFMA layout above, lane (g, j) supplies K index 16g + t in step t
// of the forward and data-backward products, so each lane's operand run over
// the 16 steps is contiguous in the row-major weights or in an LDS row, or
// strided by a row (the weight gradient orders its K, the samples, for
// conflict-free LDS banks instead).  The output layer (3 rows)
// and the loss stay on the vector ALUs (lane = record, FPW = 4 features per
// wave where a pass is split by feature).
// Activation buffer of the autograd form (ACT): per tile, h_1 .. h_H as
// [layer][record][feature] FP32, then, after every tile's block, the network
// output [tile * 64 + record][4].  kActNone: no buffer; kActStore: forward
// only, writes the buffer and rgb, then exits; kActLoad: the forward pass is
// read from the buffer instead of recomputed.
constexpr int kActNone = 0, kActStore = 1, kActLoad = 2;

template <bool UPSTREAM, bool GENC, int NWV, int ACT = kActNone>
__global__ __launch_bounds__(64 * NWV) void k_train_fp32(const float* __restrict__ w,
                                                         const float* __restrict__ enc,
                                                         const float* __restrict__ tgt,
                                                         const int32_t* __restrict__ idx, int64_t n,
                                                         int n_hidden, int n_params, float loss_eps,
                                                         float grad_scale, float* __restrict__ partials,
                                                         float* __restrict__ loss_part,
                                                         int32_t* __restrict__ tile_bad,
                                                         float* __restrict__ genc, int fcol,
                                                         float* __restrict__ act, float* __restrict__ rgb,
                                                         LcgGather lg) {
    static_assert(NWV == 16, "one 16 x 16 block of each 64 x 64 product per wave");
    constexpr int FPW = kW / NWV;                          // features per wave (output layer)
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
    const int f0 = FPW * wave;                            // this wave's first feature (output layer)
    const int g = lane >> 4, j = lane & 15;               // MFMA lane group and column
    const int bro = wave >> 2, bco = wave & 3;            // this wave's block row and column

    // Stage the tile's inputs as h_0 (zeros past the end of the batch).
    for (int i = tid; i < kTile * 16; i += NT) {
        const int s = i >> 4, q = i & 15;
        const int64_t r = tile * kTile + s;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < n) v = reinterpret_cast<const float4*>(enc + gather_row(idx, lg, r) * kEncWidth)[q];
        *reinterpret_cast<float4*>(hs + s * kLd + 4 * q) = v;
    }
    __syncthreads();

    // Forward: z = W_l h, wave w the block (out features 16 bro.., samples
    // 16 bco..).  A: lane (g, i) takes W_l[16 bro + i][16g + t]; B: lane (g, j)
    // takes h[16 bco + j][16g + t]; D: lane (g, j) ends with out features
    // 16 bro + 4g .. +3 of sample 16 bco + j.  Layer l's weights start at
    // w + l * 64 * 64 (the input layer is 64 x 64 too).
    const int64_t n_tiles = gridDim.x;
    float* act_t = act + tile * (int64_t)(n_hidden * kTile * kW);
    float* act_y = act + n_tiles * (int64_t)(n_hidden * kTile * kW);
    // copy h_1 .. h_H between LDS and the buffer, one float4 at a time
    auto copy_act = [&](bool to_lds) {
        for (int i = tid; i < n_hidden * kTile * 16; i += NT) {
            const int q = i & 15, rs = i >> 4;               // rs = layer * 64 + record
            float4* l = reinterpret_cast<float4*>(hs + (kTile + rs) * kLd) + q;
            float4* gp = reinterpret_cast<float4*>(act_t + rs * kW) + q;
            if (to_lds) *l = *gp; else *gp = *l;
        }
    };
    if (ACT == kActLoad) {
        copy_act(true);
        __syncthreads();
    }
    const int n_fwd = ACT == kActLoad ? 0 : n_hidden;   // layers the forward pass computes
    for (int l = 0; l < n_fwd; ++l) {
        const float* arow = w + l * kW * kW + (16 * bro + j) * kW + 16 * g;
        const float* brow = hs + l * kTile * kLd + (16 * bco + j) * kLd + 16 * g;
        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        #pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
            const float4 a = *reinterpret_cast<const float4*>(arow + 4 * t4);
            const float4 b = *reinterpret_cast<const float4*>(brow + 4 * t4);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
        }
        float* hout = hs + (l + 1) * kTile * kLd + (16 * bco + j) * kLd + 16 * bro + 4 * g;
        *reinterpret_cast<float4*>(hout) = make_float4(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f),
                                                       fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
        __syncthreads();
    }
    const float* wout = w + n_hidden * kW * kW;           // [3][64]
    const float* hlast = hs + n_hidden * kTile * kLd;

    if (ACT == kActStore) {
        copy_act(false);
        if (wave != 0) return;            // wave 0 stores the outputs below and returns too
    }

    // Output layer, loss and dL/dy (wave 0, lane = sample).
    if (wave == 0) {
        float f[kNOut] = {0.f, 0.f, 0.f};
        if (ACT == kActLoad) {
            if (valid) {
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) f[o] = act_y[row * 4 + o];
            }
        } else {
            const float* hr = hlast + lane * kLd;
            #pragma unroll
            for (int k = 0; k < kW; ++k) {
                const float hv = hr[k];
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) f[o] = fmaf(wout[o * kW + k], hv, f[o]);
            }
        }
        float r[kNOut] = {1.f, 1.f, 1.f};
        if (fcol) {
            const float* h0 = hs + lane * kLd;
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) r[o] = h0[fcol + o] + h0[fcol + 3 + o];
        }
        if (ACT == kActStore) {
            if (valid) {
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) {
                    rgb[row * 3 + o] = f[o] * r[o];
                    act_y[row * 4 + o] = f[o];
                }
                act_y[row * 4 + 3] = 0.0f;
            }
            return;
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
        // dW_l[o][i] = sum_s delta[s][o] h_l[s][i], wave w the block (rows
        // 16 bro.., columns 16 bco..).  In step t lane group g takes sample
        // s = 16 (t / 4) + 4g + t % 4, so the four groups read rows 4 apart
        // (16 banks apart at the 68-float stride; rows 16 apart would share
        // banks).  A: lane (g, i) takes delta[s][16 bro + i]; B: lane (g, j)
        // takes h_l[s][16 bco + j]; D: lane (g, j) ends with rows
        // 16 bro + 4g .. +3 of column 16 bco + j.
        {
            const float* da = dcur + 4 * g * kLd + 16 * bro + j;
            const float* hb = hl + 4 * g * kLd + 16 * bco + j;
            f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            #pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int so = (16 * (t >> 2) + (t & 3)) * kLd;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(da[so], hb[so], acc, 0, 0, 0);
            }
            float* dst = part + off + (16 * bro + 4 * g) * cols + 16 * bco + j;
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                // streamed past the caches: read once, by the reduction
                __builtin_nontemporal_store(acc[r], dst + r * cols);
                bad |= !isfinite(acc[r]);
            }
        }
        // delta_l = W_l^T delta_{l+1}, masked (l >= 1); or dL/dh_0 (l == 0).
        // Wave w the block (features 16 bro.., samples 16 bco..).  A: lane (g, i)
        // takes W_l[16g + t][16 bro + i]; B: lane (g, j) takes
        // delta[16 bco + j][16g + t]; D: lane (g, j) ends with features
        // 16 bro + 4g .. +3 of sample 16 bco + j.
        if (l >= 1 || GENC) {
            const float* wa = wlay + 16 * g * cols + 16 * bro + j;
            const float* db = dcur + (16 * bco + j) * kLd + 16 * g;
            f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            #pragma unroll
            for (int t4 = 0; t4 < 4; ++t4) {
                const float4 b = *reinterpret_cast<const float4*>(db + 4 * t4);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[(4 * t4) * cols], b.x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[(4 * t4 + 1) * cols], b.y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[(4 * t4 + 2) * cols], b.z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[(4 * t4 + 3) * cols], b.w, acc, 0, 0, 0);
            }
            const int sm = 16 * bco + j;                  // this lane's sample in the tile
            const int fb = 16 * bro + 4 * g;              // its first feature
            if (l >= 1) {
                const float4 hv = *reinterpret_cast<const float4*>(hl + sm * kLd + fb);
                *reinterpret_cast<float4*>(dnxt + sm * kLd + fb) =
                    make_float4(hv.x > 0.0f ? acc[0] : 0.0f, hv.y > 0.0f ? acc[1] : 0.0f,
                                hv.z > 0.0f ? acc[2] : 0.0f, hv.w > 0.0f ? acc[3] : 0.0f);
            } else {
                const int64_t srow = tile * kTile + sm;
                if (srow < n) {
                    // the loss scale of the upstream gradient divided out
                    const float inv_scale = 1.0f / grad_scale;
                    #pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] *= inv_scale;
                    if (fcol) {
                        // d(f_c R_c)/d(albedo column) = f_c on the diffuse and specular column.
                        const int64_t ssrc = gather_row(idx, lg, srow);
                        #pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            int c = fb + r - fcol;
                            if (c >= 0 && c < 6) {
                                c = c >= 3 ? c - 3 : c;
                                acc[r] = fmaf(tgt[ssrc * 3 + c], fout[sm * 4 + c], acc[r]);
                            }
                        }
                    }
                    *reinterpret_cast<float4*>(genc + srow * kEncWidth + fb) =
                        make_float4(acc[0], acc[1], acc[2], acc[3]);
                }
            }
        }
        __syncthreads();
        float* t = dcur; dcur = dnxt; dnxt = t;
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0) tile_bad[tile] = any_bad ? 1 : 0;
}

// Query grid: one workgroup of kQWaves waves per CU (the fragments of every
// hidden layer, 16 H KB, fill most of the CU's LDS), each wave striding over
// 64-query tiles.
inline size_t query_lds_bytes(const Geo& d) { return (size_t)(16 * d.H) * 64 * sizeof(f4); }
inline int64_t query_blocks(int64_t n) {
    const int64_t tiles = (n + 63) / 64;
    const int64_t b = (tiles + kQWaves - 1) / kQWaves;
    return b < kQMaxBlocks ? b : kQMaxBlocks;
}

template <typename K>
hipError_t launch_query(K kernel, const Geo& d, const float* w, const float* in, int64_t n, float* rgb,
                        hipStream_t s) {
    const int64_t blocks = query_blocks(n);
    if (blocks == 0) return hipSuccess;
    const size_t lds = query_lds_bytes(d);
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(64 * kQWaves), lds, s, w, in, n, rgb, d.H, d.F);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fwd_fp32(const Geo& d, const float* w, const float* enc, int64_t n, float* rgb,
                           hipStream_t s) {
    return launch_query(k_fwd_fp32, d, w, enc, n, rgb, s);
}

hipError_t launch_fwd_raw_fp32(const Geo& d, int preset, int layout, const float* w, const float* raw,
                               int64_t n, float* rgb, hipStream_t s) {
    const bool r14 = layout == NRC_RAW14;
    switch (preset) {
    case NRC_PRESET_PAPER_GAUSS:
        return r14 ? launch_query(k_fwd_raw_fp32<NRC_PRESET_PAPER_GAUSS, NRC_RAW14>, d, w, raw, n, rgb, s)
                   : launch_query(k_fwd_raw_fp32<NRC_PRESET_PAPER_GAUSS, NRC_RAW16>, d, w, raw, n, rgb, s);
    case NRC_PRESET_PAPER_TRI:
        return r14 ? launch_query(k_fwd_raw_fp32<NRC_PRESET_PAPER_TRI, NRC_RAW14>, d, w, raw, n, rgb, s)
                   : launch_query(k_fwd_raw_fp32<NRC_PRESET_PAPER_TRI, NRC_RAW16>, d, w, raw, n, rgb, s);
    case NRC_PRESET_PAPER:
        return r14 ? launch_query(k_fwd_raw_fp32<NRC_PRESET_PAPER, NRC_RAW14>, d, w, raw, n, rgb, s)
                   : launch_query(k_fwd_raw_fp32<NRC_PRESET_PAPER, NRC_RAW16>, d, w, raw, n, rgb, s);
    default:
        return r14 ? launch_query(k_fwd_raw_fp32<NRC_PRESET_CONFIG, NRC_RAW14>, d, w, raw, n, rgb, s)
                   : launch_query(k_fwd_raw_fp32<NRC_PRESET_CONFIG, NRC_RAW16>, d, w, raw, n, rgb, s);
    }
}

size_t fp32_train_lds_bytes(int n_hidden) {
    return ((size_t)(n_hidden + 1) * kTile * kLd + 2 * kTile * kLd + 2 * kTile * 4) * sizeof(float);
}

// Waves per 64-record training tile of the FP32 form.
constexpr int kTrainWaves = 16;

template <bool UP, bool GE, int NWV, int ACT = kActNone>
hipError_t train_fp32_launch(const Geo& d, const float* w, const float* enc, const float* tgt,
                             const int32_t* idx, int64_t n, float loss_eps, float grad_scale,
                             float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                             hipStream_t s, float* act = nullptr, float* rgb = nullptr,
                             LcgGather lg = LcgGather{}) {
    const int64_t tiles = (n + kTile - 1) / kTile;
    if (tiles == 0) return hipSuccess;
    const size_t lds = fp32_train_lds_bytes(d.H);
    auto k = k_train_fp32<UP, GE, NWV, ACT>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(64 * NWV), lds, s, w, enc, tgt, idx, n, d.H,
                       d.n_params(), loss_eps, grad_scale, partials, loss_part, tile_bad, genc, d.F, act, rgb, lg);
    return hipGetLastError();
}

hipError_t launch_train_fp32(const Geo& d, const float* w, const float* enc, const float* tgt,
                             const int32_t* idx, int64_t n, bool upstream, float loss_eps, float grad_scale,
                             float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                             hipStream_t s, const float* act, LcgGather lg) {
    if (!upstream)
        return train_fp32_launch<false, false, kTrainWaves>(d, w, enc, tgt, idx, n, loss_eps, grad_scale,
                                                            partials, loss_part, tile_bad, genc, s, nullptr,
                                                            nullptr, lg);
    float* a = const_cast<float*>(act);
    if (act) {
        if (genc)
            return train_fp32_launch<true, true, kTrainWaves, kActLoad>(d, w, enc, tgt, idx, n, loss_eps, grad_scale,
                                                                        partials, loss_part, tile_bad, genc, s, a);
        return train_fp32_launch<true, false, kTrainWaves, kActLoad>(d, w, enc, tgt, idx, n, loss_eps, grad_scale,
                                                                     partials, loss_part, tile_bad, genc, s, a);
    }
    if (genc)
        return train_fp32_launch<true, true, kTrainWaves>(d, w, enc, tgt, idx, n, loss_eps, grad_scale,
                                                          partials, loss_part, tile_bad, genc, s);
    return train_fp32_launch<true, false, kTrainWaves>(d, w, enc, tgt, idx, n, loss_eps, grad_scale,
                                                       partials, loss_part, tile_bad, genc, s);
}

hipError_t launch_fwd_train_fp32(const Geo& d, const float* w, const float* enc, int64_t n, float* act,
                                 float* rgb, hipStream_t s) {
    return train_fp32_launch<true, false, kTrainWaves, kActStore>(d, w, enc, nullptr, nullptr, n, 0.0f, 1.0f,
                                                                  nullptr, nullptr, nullptr, nullptr, s, act, rgb);
}

}  // namespace nrc
