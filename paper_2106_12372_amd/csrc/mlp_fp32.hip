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

// The output-layer weights a lane supplies as the A operand of the 4 x 4 x 1
// products: wo[b] = W_out[o][16b + 4g .. +3] for o = lane % 4 (the block row
// the lane feeds; row 3 is padding, zero), over the neurons lane group g holds.
__device__ inline void load_out_weights(const float* __restrict__ w, int H, int lane, f4 (&wo)[4]) {
    const int g = lane >> 4, o = lane & 3;
    const float* base = w + H * kW * kW + (o < kNOut ? o : 0) * kW + 4 * g;
    #pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float4 v = *reinterpret_cast<const float4*>(base + 16 * b);
        wo[b] = o < kNOut ? f4{v.x, v.y, v.z, v.w} : f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
}

// The network on the wave's 64 queries.  h: this lane's 64 input features; y:
// this lane's 3 outputs.  The hidden layers run on the 16 x 16 x 4 matrix
// instructions.  The 3-row output layer runs on v_mfma_f32_4x4x1f32, sixteen
// 4 x 4 blocks of K = 1: block 4g + j/4 of lane (g, j) takes A = W_out[o][n]
// from lanes 4(4g + j/4) + o and B = neuron n of the records 16c + 4(j/4) ..
// +3 of column c, so after the 16 neurons n its group holds (in the vector
// form's order) lane (g, j) has in register o the group's partial dot of
// channel o for query 16c + j; each product adds with one rounding, as the
// fmaf chain of the training kernel's output layer.  One transpose per
// channel gathers the four lane groups' partials onto the lane that loaded
// the query.
__device__ inline void mlp_query_mfma(const f4* __restrict__ sw, int H, int lane,
                                      const f4 (&wo)[4], const float (&h)[kW],
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
                for (int r = 0; r < 4; ++r) act[c][4 * ob + r] = relu(acc[c][ob][r]);
    }
    f4 po[4];   // po[c][o]: this lane group's share of channel o for column c's query
    #pragma unroll
    for (int c = 0; c < 4; ++c) po[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    #pragma unroll
    for (int b = 0; b < 4; ++b)
        #pragma unroll
        for (int r = 0; r < 4; ++r)
            #pragma unroll
            for (int c = 0; c < 4; ++c)
                po[c] = __builtin_amdgcn_mfma_f32_4x4x1f32(wo[b][r], act[c][4 * b + r], po[c], 0, 0, 0);
    #pragma unroll
    for (int o = 0; o < kNOut; ++o) {
        float p[4] = {po[0][o], po[1][o], po[2][o], po[3][o]};
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
    __shared__ int claimed;                 // tiles of the workgroup's share handed out so far
    constexpr int RW = LAYOUT == NRC_RAW14 ? 14 : 16;
    if (threadIdx.x == 0) claimed = 0;
    stage_query_frags(sw, w, H);
    const int lane = threadIdx.x & 63;
    f4 wo[4];
    load_out_weights(w, H, lane, wo);
    __syncthreads();
    // The workgroup owns a contiguous share of the tiles and its waves claim
    // them one at a time, so all waves of the CU finish together.
    const int64_t n_tiles = (n + 63) / 64;
    const int64_t per = n_tiles / gridDim.x, extra = n_tiles % gridDim.x;
    const int64_t t_begin = (int64_t)blockIdx.x * per + ((int64_t)blockIdx.x < extra ? blockIdx.x : extra);
    const int64_t t_end = t_begin + per + ((int64_t)blockIdx.x < extra ? 1 : 0);
    for (;;) {
        int k = 0;
        if (lane == 0) k = atomicAdd(&claimed, 1);
        const int64_t t = t_begin + __builtin_amdgcn_readfirstlane(k);
        if (t >= t_end) break;
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
//
// A workgroup owns a tile of 64 records.  Its 4 chain waves hold 16 records
// each (wave w: records 16w .. 16w+15, lane (g, j): record 16w + j) and run
// the forward pass, the loss and the data backward pass with the activations
// in VGPRs in the query kernel's order: a[4b + r] is neuron 16b + 4g + r,
// which is what an accumulator block leaves in the lane and what the next
// product's B operand needs, so a layer is 64 v_mfma_f32_16x16x4_f32 in four
// independent chains with no data movement.  The forward arithmetic is the
// query kernel's, product for product, so the training forward pass equals
// inference bit for bit.  Every h_l and delta_l also goes to LDS record-major
// ([record][feature], 68-float rows, 16-byte stores).  Its 4 weight-gradient
// waves form dW_l = delta_{l+1} h_l^T over the tile's records as soon as
// delta_{l+1} is in LDS, while the chain computes delta_l: one 16-column
// block per wave, each 16 x 16 block 16 matrix instructions over a K of 64
// records, ordered so the four lane groups read LDS rows 4 apart (16 banks
// apart at the 68-float stride).  The output layer (3 rows), the loss and
// dW of the output layer stay on the vector ALUs.
// Activation buffer of the autograd form (ACT): per tile, h_1 .. h_H as
// [layer][record][feature] FP32, then, after every tile's block, the network
// output [tile * 64 + record][4].  kActNone: no buffer; kActStore: forward
// only, writes the buffer and rgb, then exits; kActLoad: the forward pass is
// read from the buffer instead of recomputed.
constexpr int kActNone = 0, kActStore = 1, kActLoad = 2;
constexpr int kChainWaves = 4, kGradWaves = 4;

// Whether the training kernel keeps W_{H-1} transposed in LDS for the first
// backward iteration: H >= 2 (it is staged for the forward pass) and H <= 5
// (with H = 6 the activations fill the LDS).
__host__ __device__ constexpr bool fp32_train_wlast(int n_hidden) { return n_hidden >= 2 && n_hidden <= 5; }

template <int ACT> constexpr int fp32_train_waves() { return ACT == kActStore ? kChainWaves : kChainWaves + kGradWaves; }

// Training records given raw (RAWL = their layout, PRESET = the cache's
// encoding; RAWL < 0: encoded rows): enc then points at the raw records,
// FP32 [n][14 or 16], and the four lanes (g, j) of each chain wave encode
// record j into the record's h_0 row, a share of its features each, before the
// wave reads its operands back from it.
template <bool UPSTREAM, bool GENC, int ACT = kActNone, int RAWL = -1, int PRESET = NRC_PRESET_CONFIG>
__global__ __launch_bounds__(64 * (kChainWaves + kGradWaves)) void k_train_fp32(
        const float* __restrict__ w, const float* __restrict__ enc, const float* __restrict__ tgt,
        const int32_t* __restrict__ idx, int64_t n, int n_hidden, int n_params, float loss_eps,
        float grad_scale, float* __restrict__ partials, float* __restrict__ loss_part,
        int32_t* __restrict__ tile_bad, float* __restrict__ genc, int fcol, float* __restrict__ act,
        float* __restrict__ rgb, LcgGather lg) {
    constexpr int NT = 64 * fp32_train_waves<ACT>();
    extern __shared__ __attribute__((aligned(16))) float smem[];
    __shared__ float wsum[kChainWaves];
    float* hs = smem;                                     // h_0 .. h_H, each [64][kLd]
    float* dbuf0 = hs + (n_hidden + 1) * kTile * kLd;     // deltas, double-buffered [64][kLd]
    float* dbuf1 = dbuf0 + kTile * kLd;
    float* dout = dbuf1 + kTile * kLd;                    // [64][4]: dL/d(network output)
    float* fout = dout + kTile * 4;                       // [64][4]: network output
    // W_{H-1} transposed for the first backward iteration, written while it is
    // staged for the forward pass (2 <= H <= 5, where it fits beside the rest)
    float* wlast = fout + kTile * 4;
    const bool wlast_on = ACT == kActNone && fp32_train_wlast(n_hidden);
    auto hrow = [&](int l) { return hs + l * kTile * kLd; };

    // The wave index is uniform across the wave; saying so lets addresses that
    // depend on it use scalar registers.
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, j = lane & 15;               // MFMA lane group and column
    const bool chain = wave < kChainWaves;
    const int64_t tile = blockIdx.x;
    const int sl = 16 * (chain ? wave : 0) + j;           // a chain lane's record in the tile
    const int64_t row = tile * kTile + sl;
    const bool valid = chain && row < n;
    // record read for this slot: idx[row] or the LCG orbit for a gathered batch, else row
    const int64_t src = valid ? gather_row(idx, lg, row) : 0;
    const bool out_lane = chain && g == 0;                // lanes 0..15 hold a record's outputs
    float* part = partials + tile * (int64_t)n_params;
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

    // ---- h_0, targets and reflectance factor of the lane's record ----------
    float a[16];   // chain: a[4b + r] = neuron 16b + 4g + r of record sl (activations, later deltas)
    float r[kNOut] = {1.f, 1.f, 1.f}, t[kNOut] = {0.f, 0.f, 0.f};
    if constexpr (RAWL >= 0) {
      static_assert(!UPSTREAM && !GENC && ACT == kActNone, "raw records feed the training step only");
      if (chain) {
        constexpr int RW = RAWL == NRC_RAW14 ? 14 : 16;
        float* h0 = hs + sl * kLd;
        // The four lane groups of a record share its encoding: groups 0..2 the
        // frequency encoding of position coordinate g (the same code for the
        // three, features 12g ..12g + 11), group 3 the rest (features 36 ..63).
        float x[RW];
        if (valid) {
            const float* rr = enc + src * RW;
            #pragma unroll
            for (int k = 0; k < RW; ++k) x[k] = rr[k];
        } else {
            #pragma unroll
            for (int k = 0; k < RW; ++k) x[k] = 0.0f;
        }
        float f[64];
        if (g < 3) {
            float xc[RW];
            xc[0] = g == 0 ? x[0] : g == 1 ? x[1] : x[2];
            encode_part<PRESET, RAWL, 0>(xc, f);
            if (!valid) {
                #pragma unroll
                for (int k = 0; k < 12; ++k) f[k] = 0.0f;
            }
            #pragma unroll
            for (int q = 0; q < 3; ++q)
                *reinterpret_cast<float4*>(h0 + 12 * g + 4 * q) =
                    make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
        } else {
            encode_part<PRESET, RAWL, 3>(x, f);
            encode_part<PRESET, RAWL, 4>(x, f);
            if (!valid) {
                #pragma unroll
                for (int k = 36; k < 64; ++k) f[k] = 0.0f;
            }
            #pragma unroll
            for (int q = 9; q < 16; ++q)
                *reinterpret_cast<float4*>(h0 + 4 * q) = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        #pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float4 v = *reinterpret_cast<const float4*>(h0 + 16 * b + 4 * g);
            a[4 * b] = v.x; a[4 * b + 1] = v.y; a[4 * b + 2] = v.z; a[4 * b + 3] = v.w;
        }
        if (out_lane && valid) {
            if (fcol) {
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) r[o] = h0[fcol + o] + h0[fcol + 3 + o];
            }
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) t[o] = tgt[src * 3 + o];
        }
      }
    } else if (chain) {
        // record src (record 0 for slots past the end, whose features are then zeroed)
        const float* er = enc + src * kEncWidth;
        float4 v[4];
        #pragma unroll
        for (int b = 0; b < 4; ++b) v[b] = *reinterpret_cast<const float4*>(er + 16 * b + 4 * g);
        #pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (!valid) v[b] = make_float4(0.f, 0.f, 0.f, 0.f);
            a[4 * b] = v[b].x; a[4 * b + 1] = v[b].y; a[4 * b + 2] = v[b].z; a[4 * b + 3] = v[b].w;
            *reinterpret_cast<float4*>(hs + sl * kLd + 16 * b + 4 * g) = v[b];
        }
        if (out_lane && valid) {
            if (fcol) {
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) r[o] = er[fcol + o] + er[fcol + 3 + o];
            }
            if (ACT != kActStore) {
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) t[o] = tgt[src * 3 + o];
            }
        }
    }
    if (ACT == kActLoad) {
        copy_act(true);
        __syncthreads();
    }

    // ---- forward: z = W_l h_l; lane (g, i) supplies W_l[16 ob + i][16 obp + 4g + r]
    // in K step (obp, r), the query kernel's fragment.  The delta buffers are
    // free until the backward pass, so they double-buffer the layers' weights
    // in LDS ([64][kLd], row-major): the weight-gradient waves (or, in the
    // forward-only form, the chain waves) load W_{l+1} while the chain
    // computes layer l, and a barrier per layer hands it over.
    const int n_fwd = ACT == kActLoad ? 0 : n_hidden;
    constexpr int NS = ACT == kActStore ? NT : 64 * kGradWaves;   // threads that stage weights
    static_assert(kW * 16 == 4 * NS, "four float4 of a layer's weights per staging thread");
    const bool stager = ACT == kActStore || !chain;
    const int st = ACT == kActStore ? tid : tid - 64 * kChainWaves;
    // staging thread st moves float4 st + u NS (u = 0..3): row (st >> 4) + 16 u, column 4 (st & 15)
    const int srow = st >> 4, scol = 4 * (st & 15);
    float4 s0, s1, s2, s3;
    if (n_fwd > 0) {
        if (stager) {
            const float* src = w + srow * kW + scol;
            s0 = *reinterpret_cast<const float4*>(src);
            s1 = *reinterpret_cast<const float4*>(src + 16 * kW);
            s2 = *reinterpret_cast<const float4*>(src + 32 * kW);
            s3 = *reinterpret_cast<const float4*>(src + 48 * kW);
            float* dst = dbuf0 + srow * kLd + scol;
            *reinterpret_cast<float4*>(dst) = s0;
            *reinterpret_cast<float4*>(dst + 16 * kLd) = s1;
            *reinterpret_cast<float4*>(dst + 32 * kLd) = s2;
            *reinterpret_cast<float4*>(dst + 48 * kLd) = s3;
        }
        __syncthreads();
    }
    for (int l = 0; l < n_fwd; ++l) {
        const bool more = l + 1 < n_fwd;
        if (stager && more) {
            const float* src = w + (l + 1) * kW * kW + srow * kW + scol;
            s0 = *reinterpret_cast<const float4*>(src);
            s1 = *reinterpret_cast<const float4*>(src + 16 * kW);
            s2 = *reinterpret_cast<const float4*>(src + 32 * kW);
            s3 = *reinterpret_cast<const float4*>(src + 48 * kW);
        }
        if (chain) {
            const float* wl = (l & 1 ? dbuf1 : dbuf0) + j * kLd + 4 * g;
            f4 fr[16];
            #pragma unroll
            for (int k = 0; k < 16; ++k) fr[k] = *reinterpret_cast<const f4*>(wl + 16 * (k & 3) * kLd + 16 * (k >> 2));
            f4 acc[4];
            #pragma unroll
            for (int ob = 0; ob < 4; ++ob) acc[ob] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            // the four blocks' chains interleaved: consecutive matrix instructions
            // are independent; each accumulator still takes its K steps in order
            #pragma unroll
            for (int obp = 0; obp < 4; ++obp)
                #pragma unroll
                for (int q = 0; q < 4; ++q)
                    #pragma unroll
                    for (int ob = 0; ob < 4; ++ob)
                        acc[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[4 * obp + ob][q], a[4 * obp + q], acc[ob], 0, 0, 0);
            float* ho = hrow(l + 1) + sl * kLd + 4 * g;
            #pragma unroll
            for (int ob = 0; ob < 4; ++ob) {
                #pragma unroll
                for (int q = 0; q < 4; ++q) a[4 * ob + q] = relu(acc[ob][q]);
                *reinterpret_cast<float4*>(ho + 16 * ob) = make_float4(a[4 * ob], a[4 * ob + 1], a[4 * ob + 2], a[4 * ob + 3]);
            }
        }
        if (stager && more) {
            float* dst = (l & 1 ? dbuf0 : dbuf1) + srow * kLd + scol;
            *reinterpret_cast<float4*>(dst) = s0;
            *reinterpret_cast<float4*>(dst + 16 * kLd) = s1;
            *reinterpret_cast<float4*>(dst + 32 * kLd) = s2;
            *reinterpret_cast<float4*>(dst + 48 * kLd) = s3;
            if (wlast_on && l + 2 == n_hidden) {
                // WT[k][o] = W_{H-1}[o][k]: this thread holds rows srow + 16u, columns scol ..+3
                float* t = wlast + scol * kLd + srow;
                const float4 sv[4] = {s0, s1, s2, s3};
                #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    t[16 * u] = sv[u].x;
                    t[kLd + 16 * u] = sv[u].y;
                    t[2 * kLd + 16 * u] = sv[u].z;
                    t[3 * kLd + 16 * u] = sv[u].w;
                }
            }
        }
        __syncthreads();   // W_{l+1} staged; W_l's buffer free
    }

    // ---- output layer on the vector ALUs: each lane's partial dot over its 16
    // neurons, the four lane groups' partials added as (g0 + g1) + (g2 + g3)
    const float* wout = w + n_hidden * kW * kW;           // [3][64]
    float f[kNOut] = {0.f, 0.f, 0.f};
    if (chain) {
        if (ACT == kActLoad) {
            if (out_lane && valid) {
                #pragma unroll
                for (int o = 0; o < kNOut; ++o) f[o] = act_y[row * 4 + o];
            }
        } else {
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) {
                const float* wo = wout + o * kW + 4 * g;
                float p = 0.0f;
                #pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const float4 v = *reinterpret_cast<const float4*>(wo + 16 * b);
                    p = fmaf(v.x, a[4 * b], p);
                    p = fmaf(v.y, a[4 * b + 1], p);
                    p = fmaf(v.z, a[4 * b + 2], p);
                    p = fmaf(v.w, a[4 * b + 3], p);
                }
                const float s1 = p + __shfl_xor(p, 16, 64);
                f[o] = s1 + __shfl_xor(s1, 32, 64);
            }
        }
    }
    if (ACT == kActStore) {
        if (out_lane && valid) {
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) {
                rgb[row * 3 + o] = f[o] * r[o];
                act_y[row * 4 + o] = f[o];
            }
            act_y[row * 4 + 3] = 0.0f;
        }
        __syncthreads();
        copy_act(false);
        return;
    }

    // ---- loss (Eq. 5) and dL/dy in the output lanes --------------------------
    float d[kNOut] = {0.f, 0.f, 0.f};
    float lterm = 0.0f;
    if (out_lane && valid) {
        if (UPSTREAM) {
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) d[o] = t[o] * grad_scale * r[o];
        } else {
            float y[kNOut];
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) y[o] = f[o] * r[o];
            const float lum = (y[0] + y[1] + y[2]) * (1.0f / 3.0f);
            const float inv_den = 1.0f / fmaf(lum, lum, loss_eps);
            #pragma unroll
            for (int o = 0; o < kNOut; ++o) {
                const float diff = y[o] - t[o];
                lterm = fmaf(diff * diff, inv_den, lterm);
                d[o] = 2.0f * diff * inv_den * grad_scale * r[o];
            }
        }
    }
    if (chain) {
        if (out_lane) {
            *reinterpret_cast<float4*>(dout + sl * 4) = make_float4(d[0], d[1], d[2], 0.f);
            if (GENC) *reinterpret_cast<float4*>(fout + sl * 4) = make_float4(f[0], f[1], f[2], 0.f);
        }
    }
    __syncthreads();   // dL/dy and h_0 .. h_H are in LDS

    bool bad = false;   // any non-finite weight-gradient partial in this tile
    float* dcur = dbuf0;
    float* dnxt = dbuf1;
    if (chain) {
        // delta_H = W_H^T dL/dy, masked by ReLU'(z_H), for the lane's 16 neurons
        float dv[kNOut];
        #pragma unroll
        for (int o = 0; o < kNOut; ++o) dv[o] = __shfl(d[o], j, 64);
        const float* hl = hrow(n_hidden) + sl * kLd + 4 * g;
        #pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float4 hv = *reinterpret_cast<const float4*>(hl + 16 * b);
            const float hq[4] = {hv.x, hv.y, hv.z, hv.w};
            #pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * b + 4 * g + q;
                float s = wout[i] * dv[0];
                s = fmaf(wout[kW + i], dv[1], s);
                s = fmaf(wout[2 * kW + i], dv[2], s);
                a[4 * b + q] = hq[q] > 0.0f ? s : 0.0f;
            }
            #pragma unroll
            for (int q = 0; q < 4; ++q) dcur[(16 * b + 4 * g + q) * kLd + sl] = a[4 * b + q];
        }
    } else {
        // dW_H[o][i] = sum_s dL/dy[s][o] h_H[s][i]: one (o, i) per thread
        const int tt = tid - 64 * kChainWaves;
        if (tt < kNOut * kW) {
            const int o = tt >> 6, i = tt & 63;
            const float* hl = hrow(n_hidden);
            float acc = 0.0f;
            for (int s = 0; s < kTile; ++s) acc = fmaf(dout[s * 4 + o], hl[s * kLd + i], acc);
            __builtin_nontemporal_store(acc, &part[(n_params - kNOut * kW) + o * kW + i]);
            bad |= !isfinite(acc);
        }
    }
    __syncthreads();   // delta_H is in LDS

    for (int l = n_hidden - 1; l >= 0; --l) {
        const float* hl = hrow(l);
        if (!chain) {
            // dW_l[o][i] = sum_s delta_{l+1}[s][o] h_l[s][i]; wave nb = wave - 4
            // the column block 16 nb.., all four row blocks.  In step t lane
            // group g takes sample s = 16 (t / 4) + 4g + t % 4.  A: lane (g, i)
            // takes delta[s][16 mb + i]; B: lane (g, j) takes h_l[s][16 nb + j];
            // D: lane (g, j) ends with rows 16 mb + 4g .. +3 of column 16 nb + j.
            const int nb = wave - kChainWaves;
            const float* da = dcur + j * kLd + 4 * g;                 // delta feature-major
            const float* hb = hl + 4 * g * kLd + 16 * nb + j;
            f4 acc[4];
            #pragma unroll
            for (int mb = 0; mb < 4; ++mb) acc[mb] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            #pragma unroll
            for (int t = 0; t < 4; ++t) {
                f4 av[4];
                #pragma unroll
                for (int mb = 0; mb < 4; ++mb) av[mb] = *reinterpret_cast<const f4*>(da + 16 * mb * kLd + 16 * t);
                #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float bv = hb[(16 * t + u) * kLd];
                    #pragma unroll
                    for (int mb = 0; mb < 4; ++mb)
                        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb][u], bv, acc[mb], 0, 0, 0);
                }
            }
            float* dst = part + l * kW * kW + 4 * g * kW + 16 * nb + j;
            #pragma unroll
            for (int mb = 0; mb < 4; ++mb)
                #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // streamed past the caches: read once, by the reduction
                    __builtin_nontemporal_store(acc[mb][q], dst + (16 * mb + q) * kW);
                    bad |= !isfinite(acc[mb][q]);
                }
        } else if (l >= 1 || GENC) {
            // W_l^T delta_{l+1}: lane (g, i) supplies W_l[16 obp + 4g + r][16 ob + i]
            // in K step (obp, r); a holds delta_{l+1} in the same order.
            // W_{l-1}, which the next iteration needs, is staged transposed
            // (WT[k][o] = W[o][k], rows of kLd floats) into the LDS row block of
            // h_{l+1}, which no later step reads: chain thread tid moves
            // W[tid % 64][16 (tid / 64) ..+15], so a wave's stores fall in
            // consecutive banks.  W_l itself comes from the block
            // the previous iteration filled, or, in the first iteration, from
            // the transposed copy the forward pass left (else from the
            // L2-resident master weights).
            const bool stage = l >= 2 || (GENC && l == 1);
            float4 wn[4];
            if (stage) {
                const float4* src = reinterpret_cast<const float4*>(w + (l - 1) * kW * kW + (tid & 63) * kW +
                                                                    16 * (tid >> 6));
                #pragma unroll
                for (int u = 0; u < 4; ++u) wn[u] = src[u];
            }
            f4 acc[4];
            #pragma unroll
            for (int ob = 0; ob < 4; ++ob) acc[ob] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            const float* wtb = l <= n_hidden - 2 ? hrow(l + 2) : wlast_on ? wlast : nullptr;
            if (wtb) {
                // fragment (ob, obp) of lane (g, j): WT[16 ob + j][16 obp + 4g .. +3]
                const float* wt = wtb + j * kLd + 4 * g;
                f4 fr[4][4];
                #pragma unroll
                for (int obp = 0; obp < 4; ++obp)
                    #pragma unroll
                    for (int ob = 0; ob < 4; ++ob)
                        fr[obp][ob] = *reinterpret_cast<const f4*>(wt + 16 * ob * kLd + 16 * obp);
                #pragma unroll
                for (int obp = 0; obp < 4; ++obp)
                    #pragma unroll
                    for (int q = 0; q < 4; ++q)
                        #pragma unroll
                        for (int ob = 0; ob < 4; ++ob)
                            acc[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[obp][ob][q], a[4 * obp + q], acc[ob],
                                                                           0, 0, 0);
            } else {
                const float* wl = w + l * kW * kW + 4 * g * kW + j;
                #pragma unroll
                for (int obp = 0; obp < 4; ++obp)
                    #pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float* wr = wl + (16 * obp + q) * kW;
                        #pragma unroll
                        for (int ob = 0; ob < 4; ++ob)
                            acc[ob] = __builtin_amdgcn_mfma_f32_16x16x4f32(wr[16 * ob], a[4 * obp + q], acc[ob],
                                                                           0, 0, 0);
                    }
            }
            if (stage) {
                float* dst = hrow(l + 1) + 16 * (tid >> 6) * kLd + (tid & 63);
                #pragma unroll
                for (int u = 0; u < 4; ++u) {
                    dst[(4 * u) * kLd] = wn[u].x;
                    dst[(4 * u + 1) * kLd] = wn[u].y;
                    dst[(4 * u + 2) * kLd] = wn[u].z;
                    dst[(4 * u + 3) * kLd] = wn[u].w;
                }
            }

            if (l >= 1) {
                // delta_l = (W_l^T delta_{l+1}) masked by ReLU'(z_l)
                const float* hr = hl + sl * kLd + 4 * g;
                #pragma unroll
                for (int ob = 0; ob < 4; ++ob) {
                    const float4 hv = *reinterpret_cast<const float4*>(hr + 16 * ob);
                    a[4 * ob] = hv.x > 0.0f ? acc[ob][0] : 0.0f;
                    a[4 * ob + 1] = hv.y > 0.0f ? acc[ob][1] : 0.0f;
                    a[4 * ob + 2] = hv.z > 0.0f ? acc[ob][2] : 0.0f;
                    a[4 * ob + 3] = hv.w > 0.0f ? acc[ob][3] : 0.0f;
                    #pragma unroll
                    for (int q = 0; q < 4; ++q) dnxt[(16 * ob + 4 * g + q) * kLd + sl] = a[4 * ob + q];
                }
            } else if (valid) {
                // dL/dh_0 with the loss scale of the upstream gradient divided out
                const float inv_scale = 1.0f / grad_scale;
                #pragma unroll
                for (int ob = 0; ob < 4; ++ob) {
                    const int fb = 16 * ob + 4 * g;               // the lane's first feature
                    float v[4];
                    #pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = acc[ob][q] * inv_scale;
                    if (fcol) {
                        // d(f_c R_c)/d(albedo column) = f_c on the diffuse and specular column.
                        #pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            int c = fb + q - fcol;
                            if (c >= 0 && c < 6) {
                                c = c >= 3 ? c - 3 : c;
                                v[q] = fmaf(tgt[src * 3 + c], fout[sl * 4 + c], v[q]);
                            }
                        }
                    }
                    *reinterpret_cast<float4*>(genc + row * kEncWidth + fb) = make_float4(v[0], v[1], v[2], v[3]);
                }
            }
        }
        if (l >= 1) {
            __syncthreads();   // delta_l is in LDS; delta_{l+1} has been read
            float* tp = dcur; dcur = dnxt; dnxt = tp;
        }
    }
    // The chain waves' loss sums are formed last: nothing before needs them,
    // and the chain waves wait here while the others finish dW_0.
    if (chain) {
        const float tot = wave_sum_compensated(lterm);
        if (lane == 0) wsum[wave] = tot;
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0) {
        // compensated combine of the chain waves' loss sums, in wave order
        float ts = 0.0f, tc = 0.0f;
        for (int wv = 0; wv < kChainWaves; ++wv) {
            const float x = wsum[wv], u = ts + x;
            tc += fabsf(ts) >= fabsf(x) ? (ts - u) + x : (x - u) + ts;
            ts = u;
        }
        loss_part[tile] = ts + tc;
        tile_bad[tile] = any_bad ? 1 : 0;
    }
}

// Query grid: one workgroup of kQWaves waves per CU (the fragments of every
// hidden layer, 16 H KB, fill most of the CU's LDS), its waves claiming the
// 64-query tiles of the workgroup's share.
inline size_t query_lds_bytes(const Geo& d) { return (size_t)(16 * d.H) * 64 * sizeof(f4); }
inline int64_t query_blocks(int64_t n) {
    const int64_t tiles = (n + 63) / 64;
    const int64_t b = (tiles + kQWaves - 1) / kQWaves;
    const int64_t cus = device_cu_count();
    return b < cus ? b : cus;
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
    return ((size_t)(n_hidden + 1) * kTile * kLd + 2 * kTile * kLd + 2 * kTile * 4 +
            (fp32_train_wlast(n_hidden) ? (size_t)kTile * kLd : 0)) * sizeof(float);
}

template <bool UP, bool GE, int ACT = kActNone, int RAWL = -1, int PRESET = NRC_PRESET_CONFIG>
hipError_t train_fp32_launch(const Geo& d, const float* w, const float* enc, const float* tgt,
                             const int32_t* idx, int64_t n, float loss_eps, float grad_scale,
                             float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                             hipStream_t s, float* act = nullptr, float* rgb = nullptr,
                             LcgGather lg = LcgGather{}) {
    const int64_t tiles = (n + kTile - 1) / kTile;
    if (tiles == 0) return hipSuccess;
    const size_t lds = fp32_train_lds_bytes(d.H);
    auto k = k_train_fp32<UP, GE, ACT, RAWL, PRESET>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(64 * fp32_train_waves<ACT>()), lds, s, w, enc, tgt, idx, n,
                       d.H, d.n_params(), loss_eps, grad_scale, partials, loss_part, tile_bad, genc, d.F, act, rgb,
                       lg);
    return hipGetLastError();
}

hipError_t launch_train_fp32(const Geo& d, const float* w, const float* enc, const float* tgt,
                             const int32_t* idx, int64_t n, bool upstream, float loss_eps, float grad_scale,
                             float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                             hipStream_t s, const float* act, LcgGather lg) {
    if (!upstream)
        return train_fp32_launch<false, false>(d, w, enc, tgt, idx, n, loss_eps, grad_scale, partials, loss_part,
                                               tile_bad, genc, s, nullptr, nullptr, lg);
    float* a = const_cast<float*>(act);
    if (act) {
        if (genc)
            return train_fp32_launch<true, true, kActLoad>(d, w, enc, tgt, idx, n, loss_eps, grad_scale, partials,
                                                           loss_part, tile_bad, genc, s, a);
        return train_fp32_launch<true, false, kActLoad>(d, w, enc, tgt, idx, n, loss_eps, grad_scale, partials,
                                                        loss_part, tile_bad, genc, s, a);
    }
    if (genc)
        return train_fp32_launch<true, true>(d, w, enc, tgt, idx, n, loss_eps, grad_scale, partials, loss_part,
                                             tile_bad, genc, s);
    return train_fp32_launch<true, false>(d, w, enc, tgt, idx, n, loss_eps, grad_scale, partials, loss_part,
                                          tile_bad, genc, s);
}

hipError_t launch_train_fp32_raw(const Geo& d, int preset, int layout, const float* w, const float* raw,
                                 const float* tgt, const int32_t* idx, int64_t n, float loss_eps, float grad_scale,
                                 float* partials, float* loss_part, int32_t* tile_bad, hipStream_t s,
                                 LcgGather lg) {
#define NRC_TRAIN_RAW(PR, LA)                                                                                  \
    return train_fp32_launch<false, false, kActNone, LA, PR>(d, w, raw, tgt, idx, n, loss_eps, grad_scale,    \
                                                             partials, loss_part, tile_bad, nullptr, s,       \
                                                             nullptr, nullptr, lg)
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

hipError_t launch_fwd_train_fp32(const Geo& d, const float* w, const float* enc, int64_t n, float* act,
                                 float* rgb, hipStream_t s) {
    return train_fp32_launch<true, false, kActStore>(d, w, enc, nullptr, nullptr, n, 0.0f, 1.0f, nullptr, nullptr,
                                                     nullptr, nullptr, s, act, rgb);
}

}  // namespace nrc
