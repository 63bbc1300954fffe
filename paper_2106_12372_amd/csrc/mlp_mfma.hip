// Matrix-core forms of the network (Sec. 4 "Fully Fused Neural Networks",
// Sec. 5 "Architecture"): FP16 or BF16 operands, FP32 accumulation, on the
// gfx950 v_mfma_f32_16x16x32_{f16,bf16} instructions.
//
// Operand roles: the weight matrix is the A operand (M = output features,
// K = input features) and the activations are the B operand (K = features,
// N = 16 samples).  The accumulator of one layer is, after ReLU and rounding,
// exactly the B operand of the next layer (see the "chained" feature order in
// nrc_internal.h), so activations never leave the VGPRs of their wave and no
// lane exchange is needed between layers.
//
// Inference: a persistent workgroup stages the forward weight fragments in
// LDS once; each wave then streams tiles of 16*COLS queries: coalesced 16-byte
// loads of the encoded rows, H+1 chained layers of MFMA, and a 12-byte RGB
// store per query.  HBM is touched only for the encoded input and the output.
//
// Training: a workgroup of 4 waves owns 64 records (wave w: records
// 16w..16w+15).  The forward pass also writes every layer's activations to
// LDS in feature-major order; the loss gradient of Eq. 5 is formed in the
// output lanes; the data backward pass chains W_l^T products through VGPRs
// the same way as the forward pass; and the weight gradient of each layer,
// a contraction over the tile's 64 records, reads delta and h back from LDS
// with the record index contiguous.  Each tile writes its weight-gradient
// partial sums; a fixed-order reduction follows (no atomics).
#include "nrc_internal.h"

namespace nrc {
namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec8;
template <> struct Vec8<_Float16> { typedef f16x8 type; };
template <> struct Vec8<__bf16> { typedef bf16x8 type; };

__device__ inline f32x4 mfma(f16x8 a, f16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <typename T> __device__ inline T to_t(float x) { return (T)x; }

template <typename V> __device__ inline V zero8() {
    V v;
    #pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = 0;
    return v;
}

// Two accumulator blocks (features 4g..4g+3 and 16+4g..16+4g+3 of a chunk)
// -> one B operand in chained order.
typedef float f32x8 __attribute__((ext_vector_type(8)));
template <typename T, typename V> __device__ inline V pack8(f32x4 lo, f32x4 hi) {
    const f32x8 f = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_convertvector(f, V);
}

typedef short s16x8 __attribute__((ext_vector_type(8)));

// ReLU on a packed FP16/BF16 operand: a negative value has its sign bit set,
// so as a signed 16-bit integer it is negative and max(., 0) maps it to +0;
// non-negative values are unchanged.  Rounding preserves sign, so
// relu(round(x)) == round(relu(x)).
template <typename V> __device__ inline V relu_packed(V v) {
    s16x8 i = __builtin_bit_cast(s16x8, v);
    i = __builtin_elementwise_max(i, (s16x8)(0));
    return __builtin_bit_cast(V, i);
}

__device__ inline f32x4 relu4(f32x4 a) {
    f32x4 r;
    #pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = fmaxf(a[j], 0.0f);
    return r;
}

__device__ inline float wave_sum(float v) {
    #pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Inference
// ---------------------------------------------------------------------------
template <typename T, int W, int COLS>
__global__ __launch_bounds__(256, 2) void k_fwd_mfma(const T* __restrict__ ffr, int n_frags,
                                                     const T* __restrict__ enc, int64_t n,
                                                     float* __restrict__ rgb, int n_hidden) {
    using V = typename Vec8<T>::type;
    constexpr int MB = W / 16, KC = W / 32;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    V* sfr = reinterpret_cast<V*>(smem_raw);
    const V* gfr = reinterpret_cast<const V*>(ffr);
    for (int base = 0; base < n_frags * 64; base += 12 * 256) {
        V tmp[12];
        #pragma unroll
        for (int u = 0; u < 12; ++u) {
            const int i = base + u * 256 + (int)threadIdx.x;
            if (i < n_frags * 64) tmp[u] = gfr[i];
        }
        #pragma unroll
        for (int u = 0; u < 12; ++u) {
            const int i = base + u * 256 + (int)threadIdx.x;
            if (i < n_frags * 64) sfr[i] = tmp[u];
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, ln = lane & 15;
    const Geo geo(W, n_hidden);
    const int64_t n_tiles = (n + 16 * COLS - 1) / (16 * COLS);
    const int64_t tstride = (int64_t)gridDim.x * 4;

    // The next tile's encoded rows are loaded while the current tile computes.
    // Rows past the end of the batch read the last row instead (their outputs
    // are never stored), so the loads need neither branches nor zero fills.
    V nxt[COLS][2];
    auto load_tile = [&](int64_t t) {
        #pragma unroll
        for (int col = 0; col < COLS; ++col) {
            int64_t row = t * 16 * COLS + 16 * col + ln;
            row = row < n ? row : n - 1;
            #pragma unroll
            for (int c = 0; c < 2; ++c)
                nxt[col][c] = *reinterpret_cast<const V*>(enc + row * kEncWidth + 32 * c + 8 * g);
        }
    };
    int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile < n_tiles) load_tile(tile);
    for (; tile < n_tiles; tile += tstride) {
        const int64_t base = tile * 16 * COLS;
        V b[COLS][KC];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) {
            b[col][0] = nxt[col][0];
            b[col][1] = nxt[col][1];
        }
        if (tile + tstride < n_tiles) load_tile(tile + tstride);
        // Layer l: the first K chunk starts from a zero accumulator (an inline
        // constant operand), ReLU is applied to the packed 16-bit result.
        for (int l = 0; l < n_hidden; ++l) {
            const int kc = l == 0 ? 2 : KC;    // the input layer has K = 64
            const V* fl = sfr + geo.fwd_base(l) * 64 + lane;
            f32x4 acc[COLS][MB];
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const V a = fl[(mb * kc) * 64];
                #pragma unroll
                for (int col = 0; col < COLS; ++col) acc[col][mb] = mfma(a, b[col][0], f32x4{0.f, 0.f, 0.f, 0.f});
            }
            #pragma unroll
            for (int c = 1; c < KC; ++c) {
                if (c >= kc) break;
                #pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const V a = fl[(mb * kc + c) * 64];
                    #pragma unroll
                    for (int col = 0; col < COLS; ++col) acc[col][mb] = mfma(a, b[col][c], acc[col][mb]);
                }
            }
            #pragma unroll
            for (int col = 0; col < COLS; ++col)
                #pragma unroll
                for (int c = 0; c < KC; ++c)
                    b[col][c] = relu_packed(pack8<T, V>(acc[col][2 * c], acc[col][2 * c + 1]));
        }
        // Output layer: 3 rows of a 16-row block; lanes 0..15 receive rows 0..3.
        const V* fo = sfr + geo.fwd_base(n_hidden) * 64 + lane;
        f32x4 o[COLS];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) o[col] = mfma(fo[0], b[col][0], f32x4{0.f, 0.f, 0.f, 0.f});
        #pragma unroll
        for (int c = 1; c < KC; ++c)
            #pragma unroll
            for (int col = 0; col < COLS; ++col) o[col] = mfma(fo[c * 64], b[col][c], o[col]);
        if (g == 0) {
            #pragma unroll
            for (int col = 0; col < COLS; ++col) {
                const int64_t row = base + 16 * col + ln;
                if (row < n) {
                    float* dst = rgb + row * 3;
                    dst[0] = o[col][0];
                    dst[1] = o[col][1];
                    dst[2] = o[col][2];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Training: forward + loss gradient + data backward + per-tile weight gradient
// ---------------------------------------------------------------------------
constexpr int kLdt = kTrainTile + 8;  // LDS row stride of the feature-major stores (elements)

// LDS bytes of the activation and delta stores of one training workgroup.
__host__ __device__ constexpr int train_act_bytes(int W, int H) {
    return (kEncWidth + H * W + 2 * W) * kLdt * 2;
}

// STAGE: all weight fragments are copied to LDS once per workgroup (when they
// fit next to the activations); otherwise each layer reads them from global
// memory (L2-resident).
template <typename T, int W, bool UPSTREAM, bool GENC, bool STAGE>
__global__ __launch_bounds__(256) void k_train_mfma(const T* __restrict__ ffr,
                                                    const T* __restrict__ bfr,
                                                    const T* __restrict__ enc,
                                                    const float* __restrict__ tgt, int64_t n,
                                                    int n_hidden, float loss_eps, float grad_scale,
                                                    float* __restrict__ partials,
                                                    float* __restrict__ loss_part,
                                                    int32_t* __restrict__ tile_bad,
                                                    float* __restrict__ genc) {
    using V = typename Vec8<T>::type;
    constexpr int MB = W / 16, KC = W / 32;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ float wsum[4];
    const Geo geo(W, n_hidden);
    T* hT = reinterpret_cast<T*>(smem_raw);              // h_0: 64 rows, h_l: W rows each
    T* dA = hT + (kEncWidth + n_hidden * W) * kLdt;      // delta buffers, W rows each
    T* dB = dA + W * kLdt;
    V* sfw = reinterpret_cast<V*>(smem_raw + train_act_bytes(W, n_hidden));
    V* sbw = sfw + geo.n_fwd_frags() * 64;

    const int P = geo.n_params();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, ln = lane & 15;
    const int64_t tile = blockIdx.x;
    const int sl = 16 * wave + ln;                       // record within the tile
    const int64_t row = tile * kTrainTile + sl;
    const bool valid = row < n;
    float* part = partials + tile * (int64_t)P;

    // Encoded inputs of this wave's 16 records (zeros past the end of the batch).
    V b[KC];
    #pragma unroll
    for (int c = 0; c < 2; ++c)
        b[c] = valid ? *reinterpret_cast<const V*>(enc + row * kEncWidth + 32 * c + 8 * g) : zero8<V>();
    const V* gf;
    const V* gb;
    if (STAGE) {
        // Forward and backward fragments are contiguous in LDS (sbw follows
        // sfw); copy them in rounds of 12 loads per thread, all in flight
        // before the first LDS store.
        const int nf = geo.n_fwd_frags() * 64, total = nf + geo.n_bwd_frags() * 64;
        const V* src_f = reinterpret_cast<const V*>(ffr);
        const V* src_b = reinterpret_cast<const V*>(bfr);
        for (int base = 0; base < total; base += 12 * 256) {
            V tmp[12];
            #pragma unroll
            for (int u = 0; u < 12; ++u) {
                const int i = base + u * 256 + tid;
                if (i < total) tmp[u] = i < nf ? src_f[i] : src_b[i - nf];
            }
            #pragma unroll
            for (int u = 0; u < 12; ++u) {
                const int i = base + u * 256 + tid;
                if (i < total) sfw[i] = tmp[u];
            }
        }
        gf = sfw + lane;
        gb = sbw + lane;
    } else {
        gf = reinterpret_cast<const V*>(ffr) + lane;
        gb = reinterpret_cast<const V*>(bfr) + lane;
    }
    #pragma unroll
    for (int c = 0; c < 2; ++c)
        #pragma unroll
        for (int i = 0; i < 8; ++i) hT[(32 * c + 8 * g + i) * kLdt + sl] = b[c][i];
    if (STAGE) __syncthreads();

    // ---- forward ------------------------------------------------------------
    for (int l = 0; l < n_hidden; ++l) {
        const int kc = l == 0 ? 2 : KC;
        const V* fl = gf + geo.fwd_base(l) * 64;
        f32x4 acc[MB];
        #pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(fl[(mb * kc) * 64], b[0], f32x4{0.f, 0.f, 0.f, 0.f});
        #pragma unroll
        for (int c = 1; c < KC; ++c) {
            if (c >= kc) break;
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(fl[(mb * kc + c) * 64], b[c], acc[mb]);
        }
        #pragma unroll
        for (int c = 0; c < KC; ++c) b[c] = relu_packed(pack8<T, V>(acc[2 * c], acc[2 * c + 1]));
        // h_{l+1} to LDS, feature-major: slot i of chunk c holds feature chained_feature(c, g, i)
        T* ho = hT + (kEncWidth + l * W) * kLdt;
        #pragma unroll
        for (int c = 0; c < KC; ++c)
            #pragma unroll
            for (int i = 0; i < 8; ++i)
                ho[(32 * c + (i < 4 ? 4 * g + i : 12 + 4 * g + i)) * kLdt + sl] = b[c][i];
    }
    f32x4 y;
    {
        const V* fo = gf + geo.fwd_base(n_hidden) * 64;
        y = mfma(fo[0], b[0], f32x4{0.f, 0.f, 0.f, 0.f});
        #pragma unroll
        for (int c = 1; c < KC; ++c) y = mfma(fo[c * 64], b[c], y);
    }

    // ---- loss gradient (Eq. 5), lanes 0..15 of each wave hold y[0..2] -------
    float d0 = 0.f, d1 = 0.f, d2 = 0.f, lterm = 0.f;
    if (g == 0 && valid) {
        if (UPSTREAM) {
            d0 = tgt[row * 3 + 0] * grad_scale;
            d1 = tgt[row * 3 + 1] * grad_scale;
            d2 = tgt[row * 3 + 2] * grad_scale;
        } else {
            const float lum = (y[0] + y[1] + y[2]) * (1.0f / 3.0f);
            const float inv_den = 1.0f / (lum * lum + loss_eps);
            const float e0 = y[0] - tgt[row * 3 + 0];
            const float e1 = y[1] - tgt[row * 3 + 1];
            const float e2 = y[2] - tgt[row * 3 + 2];
            lterm = (e0 * e0 + e1 * e1 + e2 * e2) * inv_den;
            d0 = 2.0f * e0 * inv_den * grad_scale;
            d1 = 2.0f * e1 * inv_den * grad_scale;
            d2 = 2.0f * e2 * inv_den * grad_scale;
        }
    }
    V bd = zero8<V>();
    if (g == 0) {
        bd[0] = to_t<T>(d0); bd[1] = to_t<T>(d1); bd[2] = to_t<T>(d2);
        dA[0 * kLdt + sl] = bd[0];
        dA[1 * kLdt + sl] = bd[1];
        dA[2 * kLdt + sl] = bd[2];
    }
    const float wl = wave_sum(lterm);
    if (lane == 0) wsum[wave] = wl;
    __syncthreads();
    if (tid == 0) loss_part[tile] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];

    bool bad = false;   // any non-finite weight-gradient partial in this tile
    // ---- output layer: dW_H = dL/dy h_H^T, delta_H = W_H^T dL/dy ------------
    const T* hH = hT + (kEncWidth + (n_hidden - 1) * W) * kLdt;
    for (int nb = wave; nb < MB; nb += 4) {
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        #pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            const V a = ln < kNOut ? *reinterpret_cast<const V*>(dA + ln * kLdt + 32 * kc + 8 * g)
                                   : zero8<V>();
            const V bb = *reinterpret_cast<const V*>(hH + (16 * nb + ln) * kLdt + 32 * kc + 8 * g);
            acc = mfma(a, bb, acc);
        }
        if (g == 0) {
            #pragma unroll
            for (int j = 0; j < kNOut; ++j) {
                part[geo.w_off(n_hidden) + j * W + 16 * nb + ln] = acc[j];
                bad |= !isfinite(acc[j]);
            }
        }
    }
    {
        const V* fb = gb + geo.bwd_base(n_hidden) * 64;
        f32x4 acc[MB];
        #pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(fb[mb * 64], bd, f32x4{0.f, 0.f, 0.f, 0.f});
        #pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            #pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int f = 16 * mb + 4 * g + j;
                acc[mb][j] = (float)hH[f * kLdt + sl] > 0.0f ? acc[mb][j] : 0.0f;
            }
        #pragma unroll
        for (int c = 0; c < KC; ++c) {
            b[c] = pack8<T, V>(acc[2 * c], acc[2 * c + 1]);
            #pragma unroll
            for (int i = 0; i < 8; ++i) dB[(32 * c + (i < 4 ? 4 * g + i : 12 + 4 * g + i)) * kLdt + sl] = b[c][i];
        }
    }

    // ---- hidden and input layers ------------------------------------------
    T* dcur = dB;
    T* dnxt = dA;
    for (int l = n_hidden - 1; l >= 0; --l) {
        __syncthreads();
        const int ncols = l == 0 ? kEncWidth : W;
        const int woff = geo.w_off(l);
        const T* hl = hT + (l == 0 ? 0 : (kEncWidth + (l - 1) * W)) * kLdt;
        // dW_l = delta_{l+1} h_l^T, a contraction over the tile's 64 records.
        for (int nb = wave; nb < ncols / 16; nb += 4) {
            V bb[2];
            #pragma unroll
            for (int kc = 0; kc < 2; ++kc)
                bb[kc] = *reinterpret_cast<const V*>(hl + (16 * nb + ln) * kLdt + 32 * kc + 8 * g);
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                f32x4 acc = mfma(*reinterpret_cast<const V*>(dcur + (16 * mb + ln) * kLdt + 8 * g), bb[0],
                                 f32x4{0.f, 0.f, 0.f, 0.f});
                acc = mfma(*reinterpret_cast<const V*>(dcur + (16 * mb + ln) * kLdt + 32 + 8 * g), bb[1], acc);
                #pragma unroll
                for (int j = 0; j < 4; ++j) {
                    part[woff + (16 * mb + 4 * g + j) * ncols + 16 * nb + ln] = acc[j];
                    bad |= !isfinite(acc[j]);
                }
            }
        }
        if (l >= 1) {
            // delta_l = W_l^T delta_{l+1}, masked by ReLU'(z_l).
            const V* fb = gb + geo.bwd_base(l) * 64;
            f32x4 acc[MB];
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(fb[(mb * KC) * 64], b[0], f32x4{0.f, 0.f, 0.f, 0.f});
            #pragma unroll
            for (int c = 1; c < KC; ++c)
                #pragma unroll
                for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(fb[(mb * KC + c) * 64], b[c], acc[mb]);
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                #pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int f = 16 * mb + 4 * g + j;
                    acc[mb][j] = (float)hl[f * kLdt + sl] > 0.0f ? acc[mb][j] : 0.0f;
                }
            #pragma unroll
            for (int c = 0; c < KC; ++c) {
                b[c] = pack8<T, V>(acc[2 * c], acc[2 * c + 1]);
                #pragma unroll
                for (int i = 0; i < 8; ++i)
                    dnxt[(32 * c + (i < 4 ? 4 * g + i : 12 + 4 * g + i)) * kLdt + sl] = b[c][i];
            }
            T* t = dcur; dcur = dnxt; dnxt = t;
        } else if (GENC) {
            // dL/dh_0 = W_0^T delta_1 (64 input features).
            f32x4 acc[4];
            #pragma unroll
            for (int mb = 0; mb < 4; ++mb) acc[mb] = mfma(gb[(mb * KC) * 64], b[0], f32x4{0.f, 0.f, 0.f, 0.f});
            #pragma unroll
            for (int c = 1; c < KC; ++c)
                #pragma unroll
                for (int mb = 0; mb < 4; ++mb) acc[mb] = mfma(gb[(mb * KC + c) * 64], b[c], acc[mb]);
            if (valid) {
                #pragma unroll
                for (int mb = 0; mb < 4; ++mb)
                    *reinterpret_cast<float4*>(genc + row * kEncWidth + 16 * mb + 4 * g) =
                        make_float4(acc[mb][0], acc[mb][1], acc[mb][2], acc[mb][3]);
            }
        }
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0) tile_bad[tile] = any_bad ? 1 : 0;
}

template <typename T, int W>
hipError_t fwd_dispatch(const Geo& d, const void* ffr, const void* enc, int64_t n, float* rgb,
                        hipStream_t s) {
    constexpr int COLS = 4;
    const int64_t tiles = (n + 16 * COLS - 1) / (16 * COLS);
    if (tiles == 0) return hipSuccess;
    const size_t lds = (size_t)d.n_fwd_frags() * 64 * 16;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 2048) blocks = 2048;   // persistent: 2048 workgroups cover the 256 CUs several times
    auto k = k_fwd_mfma<T, W, COLS>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), lds, s, (const T*)ffr, d.n_fwd_frags(),
                       (const T*)enc, n, rgb, d.H);
    return hipGetLastError();
}

template <typename T, int W, bool UP, bool GE>
hipError_t train_launch(const Geo& d, const void* ffr, const void* bfr, const void* enc,
                        const float* tgt, int64_t n, float loss_eps, float grad_scale,
                        float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                        hipStream_t s) {
    const int64_t tiles = (n + kTrainTile - 1) / kTrainTile;
    if (tiles == 0) return hipSuccess;
    const size_t act = (size_t)train_act_bytes(W, d.H);
    const size_t staged = act + (size_t)(d.n_fwd_frags() + d.n_bwd_frags()) * 1024;
    const size_t lds_cap = 160 * 1024 - 64;   // gfx950 LDS per workgroup, minus the static part
    if (staged <= lds_cap) {
        auto k = k_train_mfma<T, W, UP, GE, true>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)staged);
        hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(256), staged, s, (const T*)ffr, (const T*)bfr,
                           (const T*)enc, tgt, n, d.H, loss_eps, grad_scale, partials, loss_part,
                           tile_bad, genc);
    } else {
        auto k = k_train_mfma<T, W, UP, GE, false>;
        (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)act);
        hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(256), act, s, (const T*)ffr, (const T*)bfr,
                           (const T*)enc, tgt, n, d.H, loss_eps, grad_scale, partials, loss_part,
                           tile_bad, genc);
    }
    return hipGetLastError();
}

template <typename T, int W>
hipError_t train_dispatch(const Geo& d, const void* ffr, const void* bfr, const void* enc,
                          const float* tgt, int64_t n, bool upstream, float loss_eps,
                          float grad_scale, float* partials, float* loss_part, int32_t* tile_bad,
                          float* genc, hipStream_t s) {
    if (!upstream)
        return train_launch<T, W, false, false>(d, ffr, bfr, enc, tgt, n, loss_eps, grad_scale,
                                                partials, loss_part, tile_bad, genc, s);
    if (genc)
        return train_launch<T, W, true, true>(d, ffr, bfr, enc, tgt, n, loss_eps, grad_scale,
                                              partials, loss_part, tile_bad, genc, s);
    return train_launch<T, W, true, false>(d, ffr, bfr, enc, tgt, n, loss_eps, grad_scale,
                                           partials, loss_part, tile_bad, genc, s);
}

}  // namespace

size_t mfma_train_lds_bytes(int width, int n_hidden) {
    return (size_t)train_act_bytes(width, n_hidden) + 16;
}
size_t mfma_fwd_lds_bytes(int width, int n_hidden) {
    return (size_t)Geo(width, n_hidden).n_fwd_frags() * 64 * 16;
}

hipError_t launch_fwd_mfma(int precision, const Geo& d, const void* ffr, const void* enc,
                           int64_t n, float* rgb, hipStream_t s) {
    if (precision == NRC_FP16)
        return d.W == 64 ? fwd_dispatch<_Float16, 64>(d, ffr, enc, n, rgb, s)
                         : fwd_dispatch<_Float16, 128>(d, ffr, enc, n, rgb, s);
    return d.W == 64 ? fwd_dispatch<__bf16, 64>(d, ffr, enc, n, rgb, s)
                     : fwd_dispatch<__bf16, 128>(d, ffr, enc, n, rgb, s);
}

hipError_t launch_train_mfma(int precision, const Geo& d, const void* ffr, const void* bfr,
                             const void* enc, const float* tgt, int64_t n, bool upstream,
                             float loss_eps, float grad_scale, float* partials, float* loss_part,
                             int32_t* tile_bad, float* genc, hipStream_t s) {
    if (precision == NRC_FP16)
        return d.W == 64 ? train_dispatch<_Float16, 64>(d, ffr, bfr, enc, tgt, n, upstream, loss_eps,
                                                        grad_scale, partials, loss_part, tile_bad, genc, s)
                         : train_dispatch<_Float16, 128>(d, ffr, bfr, enc, tgt, n, upstream, loss_eps,
                                                         grad_scale, partials, loss_part, tile_bad, genc, s);
    return d.W == 64 ? train_dispatch<__bf16, 64>(d, ffr, bfr, enc, tgt, n, upstream, loss_eps,
                                                  grad_scale, partials, loss_part, tile_bad, genc, s)
                     : train_dispatch<__bf16, 128>(d, ffr, bfr, enc, tgt, n, upstream, loss_eps,
                                                   grad_scale, partials, loss_part, tile_bad, genc, s);
}

}  // namespace nrc
