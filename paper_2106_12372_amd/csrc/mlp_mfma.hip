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
// Training: a workgroup owns 64 records; its 4 chain waves hold 16 records
// each (wave w: records 16w..16w+15).  The forward pass also writes every
// layer's activations to LDS, record-major; the loss gradient of Eq. 5 is
// formed in the output lanes; the data backward pass chains W_l^T products
// through VGPRs the same way as the forward pass, storing each delta_l.  Four
// more waves form the weight gradients: dW_l, a contraction over the tile's
// 64 records, as soon as delta_{l+1} is in LDS, beside the chain's next
// layer, reading delta and h with LDS transpose loads so that the record
// index runs along K.  Each tile writes its weight-gradient partial sums; a
// fixed-order reduction follows (no atomics).
#include <atomic>

#include "encode_impl.h"
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
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T, typename V> __device__ inline V pack8(f32x4 lo, f32x4 hi) {
    if constexpr (sizeof(T) == 2 && !__is_same(T, _Float16)) {
        // BF16: one v_cvt_pk_bf16_f32 per pair (the generic vector conversion
        // is split into single conversions and byte permutes)
        u32x4 r;
        r[0] = __builtin_bit_cast(unsigned int, __builtin_convertvector(f32x2{lo[0], lo[1]}, bf16x2));
        r[1] = __builtin_bit_cast(unsigned int, __builtin_convertvector(f32x2{lo[2], lo[3]}, bf16x2));
        r[2] = __builtin_bit_cast(unsigned int, __builtin_convertvector(f32x2{hi[0], hi[1]}, bf16x2));
        r[3] = __builtin_bit_cast(unsigned int, __builtin_convertvector(f32x2{hi[2], hi[3]}, bf16x2));
        return __builtin_bit_cast(V, r);
    } else {
        const f32x8 f = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        return __builtin_convertvector(f, V);
    }
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

// ---------------------------------------------------------------------------
// Inference
// ---------------------------------------------------------------------------
// Copy n_frags operand fragments (1 KB each) from global memory to LDS with
// the NT threads of the workgroup; every thread issues up to 12 loads before
// its first store.
template <int NT = 256, typename V>
__device__ inline void stage_frags(V* dst, const V* src, int n_frags) {
    const int total = n_frags * 64;
    for (int base = 0; base < total; base += 12 * NT) {
        V tmp[12];
        #pragma unroll
        for (int u = 0; u < 12; ++u) {
            const int i = base + u * NT + (int)threadIdx.x;
            if (i < total) tmp[u] = src[i];
        }
        #pragma unroll
        for (int u = 0; u < 12; ++u) {
            const int i = base + u * NT + (int)threadIdx.x;
            if (i < total) dst[i] = tmp[u];
        }
    }
}

// The whole network on 16*COLS records held as B operands (b[col][0..1] =
// encoded features, natural order); returns the output accumulators (lanes
// 0..15 hold rows 0..3, i.e. the RGB values and a zero row).  Each layer's
// first K chunk starts from a zero accumulator (an inline constant operand)
// and ReLU is applied to the packed 16-bit result.  NH > 0 fixes the number
// of hidden layers at compile time (the loop unrolls); NH = 0 reads n_hidden.
template <typename T, int W, int COLS, int NH = 0>
__device__ inline void mlp_tile(const typename Vec8<T>::type* sfr, typename Vec8<T>::type (&b)[COLS][W / 32],
                                int n_hidden, int lane, f32x4 (&o)[COLS]) {
    using V = typename Vec8<T>::type;
    constexpr int MB = W / 16, KC = W / 32;
    if (NH > 0) n_hidden = NH;
    const Geo geo(W, n_hidden);
    auto layer = [&](int l) {
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
    };
    if constexpr (NH > 0) {
        #pragma unroll
        for (int l = 0; l < NH; ++l) layer(l);
    } else {
        for (int l = 0; l < n_hidden; ++l) layer(l);
    }
    const V* fo = sfr + geo.fwd_base(n_hidden) * 64 + lane;
    #pragma unroll
    for (int col = 0; col < COLS; ++col) o[col] = mfma(fo[0], b[col][0], f32x4{0.f, 0.f, 0.f, 0.f});
    #pragma unroll
    for (int c = 1; c < KC; ++c)
        #pragma unroll
        for (int col = 0; col < COLS; ++col) o[col] = mfma(fo[c * 64], b[col][c], o[col]);
}

// The same network for width 64 and a depth fixed at compile time, with the
// products ordered column block by column block: a layer's eight weight
// fragments are read once into registers, then each column block runs its
// eight products and its epilogue before the next block starts, so the
// epilogue of one block can issue beside the matrix instructions of the next.
// Every accumulator sees the same products in the same order as mlp_tile, so
// the outputs are equal bit for bit.  hook(l, acc) runs after the first column
// block's products of layer l have been issued (acc: that block's first
// accumulator), so vector work placed there can overlap the layer's remaining
// matrix instructions.
template <typename T, int COLS, int NH, typename Hook>
__device__ inline void mlp_tile_colwise(const typename Vec8<T>::type* sfr, typename Vec8<T>::type (&b)[COLS][2],
                                        int lane, f32x4 (&o)[COLS], Hook&& hook) {
    using V = typename Vec8<T>::type;
    constexpr int MB = 4;
    const Geo geo(64, NH);
    #pragma unroll
    for (int l = 0; l < NH; ++l) {
        const V* fl = sfr + geo.fwd_base(l) * 64 + lane;
        V a[MB][2];
        #pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            #pragma unroll
            for (int c = 0; c < 2; ++c) a[mb][c] = fl[(mb * 2 + c) * 64];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) {
            f32x4 acc[MB];
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(a[mb][0], b[col][0], f32x4{0.f, 0.f, 0.f, 0.f});
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = mfma(a[mb][1], b[col][1], acc[mb]);
            if (col == 0) hook(l, acc[0]);
            #pragma unroll
            for (int c = 0; c < 2; ++c) b[col][c] = relu_packed(pack8<T, V>(acc[2 * c], acc[2 * c + 1]));
        }
    }
    const V* fo = sfr + geo.fwd_base(NH) * 64 + lane;
    const V a0 = fo[0], a1 = fo[64];
    #pragma unroll
    for (int col = 0; col < COLS; ++col) o[col] = mfma(a1, b[col][1], mfma(a0, b[col][0], f32x4{0.f, 0.f, 0.f, 0.f}));
}

// Reflectance factor alpha + beta (Sec. 5) of record ln from the B operand
// holding input features 32..63 in natural order (lane 16g + ln: features
// 32 + 8g .. 32 + 8g + 7); valid in lanes 0..15, 1 when fcol == 0.  Config
// preset: diffuse 53..55 sit in lane 32 + ln, slots 5..7, and specular 56..58
// in lane 48 + ln, slots 0..2; paper presets: both in lane 48 + ln, slots 0..5.
template <typename V>
__device__ inline void reflectance_operand(const V& b1, int fcol, int ln, float (&r)[3]) {
    if (fcol == kAlbedoColConfig) {
        #pragma unroll
        for (int c = 0; c < 3; ++c)
            r[c] = __shfl((float)b1[5 + c], 32 + ln, 64) + __shfl((float)b1[c], 48 + ln, 64);
    } else if (fcol == kAlbedoColPaper) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = __shfl((float)b1[c] + (float)b1[3 + c], 48 + ln, 64);
    } else {
        r[0] = r[1] = r[2] = 1.0f;
    }
}

template <int COLS>
__device__ inline void store_rgb(const f32x4 (&o)[COLS], const float (&r)[COLS][3], int64_t base,
                                 int64_t n, int g, int ln, float* __restrict__ rgb) {
    if (g != 0) return;
    #pragma unroll
    for (int col = 0; col < COLS; ++col) {
        const int64_t row = base + 16 * col + ln;
        if (row < n) {
            float* dst = rgb + row * 3;
            dst[0] = o[col][0] * r[col][0];
            dst[1] = o[col][1] * r[col][1];
            dst[2] = o[col][2] * r[col][2];
        }
    }
}

// Inference from encoded rows.  A persistent workgroup stages the forward
// weight fragments in LDS once; each wave streams tiles of 16*COLS records and
// loads the next tile's rows while the current one computes.
template <typename T, int W, int COLS>
__global__ __launch_bounds__(256, 2) void k_fwd_mfma(const T* __restrict__ ffr, int n_frags,
                                                     const T* __restrict__ enc, int64_t n,
                                                     float* __restrict__ rgb, int n_hidden, int fcol) {
    using V = typename Vec8<T>::type;
    constexpr int KC = W / 32;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    V* sfr = reinterpret_cast<V*>(smem_raw);
    stage_frags(sfr, reinterpret_cast<const V*>(ffr), n_frags);
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, ln = lane & 15;
    const int64_t n_tiles = (n + 16 * COLS - 1) / (16 * COLS);
    const int64_t tstride = (int64_t)gridDim.x * 4;

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
        V b[COLS][KC];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) {
            b[col][0] = nxt[col][0];
            b[col][1] = nxt[col][1];
        }
        if (tile + tstride < n_tiles) load_tile(tile + tstride);
        float r[COLS][3];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) reflectance_operand(b[col][1], fcol, ln, r[col]);
        f32x4 o[COLS];
        mlp_tile<T, W, COLS>(sfr, b, n_hidden, lane, o);
        store_rgb<COLS>(o, r, tile * 16 * COLS, n, g, ln, rgb);
    }
}

// Where k_fwd_mfma_fixed's tiles come from: one batch of encoded rows, or
// the request segments of one launch (serving: queued queries of one cache
// that no training step separates; tile t belongs to the segment whose
// cumulative tile range holds it).  locate gives tile t's rows, the
// segment's row count and its output.
struct EncBatch {
    const void* enc;
    int64_t n;
    float* rgb;
    __device__ int64_t n_tiles() const { return (n + 63) / 64; }
    __device__ void locate(int64_t t, const void*& e, int64_t& base, int64_t& cnt, float*& out) const {
        e = enc; base = t * 64; cnt = n; out = rgb;
    }
};
struct EncSegs {
    SegList s;
    __device__ int64_t n_tiles() const { return s.tile_end[s.count - 1]; }
    __device__ void locate(int64_t t, const void*& e, int64_t& base, int64_t& cnt, float*& out) const {
        int sg = 0;
        while (t >= s.tile_end[sg]) ++sg;
        e = s.enc[sg]; base = (t - (sg ? s.tile_end[sg - 1] : 0)) * 64; cnt = s.n[sg]; out = s.rgb[sg];
    }
};

// Inference from encoded rows for the paper's network (width 64, five hidden
// layers) with depth fixed at compile time: one workgroup per CU shares one
// LDS copy of the weights; it owns a contiguous share of the 64-record tiles
// and its waves claim them one at a time (an LDS counter), loading the next
// claimed tile's rows while the current one runs through the network.  Same
// products and epilogue as k_fwd_mfma / k_fwd_mfma_segs, so the outputs are
// equal bit for bit.
template <typename T, int NW, typename Src>
__global__ __launch_bounds__(64 * NW) void k_fwd_mfma_fixed(const T* __restrict__ ffr, Src src, int fcol) {
    using V = typename Vec8<T>::type;
    constexpr int W = 64, NH = 5, COLS = 4, KC = 2;
    constexpr int NF = 2 * (W / 16) + (NH - 1) * (W / 16) * KC + KC;   // forward fragments
    __shared__ V sfr[NF * 64];
    __shared__ int claimed;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, ln = lane & 15;
    if (threadIdx.x == 0) claimed = 0;
    stage_frags<64 * NW>(sfr, reinterpret_cast<const V*>(ffr), NF);
    __syncthreads();

    const int64_t n_tiles = src.n_tiles();
    const int64_t per = n_tiles / gridDim.x, extra = n_tiles % gridDim.x;
    const int64_t t_begin = (int64_t)blockIdx.x * per + ((int64_t)blockIdx.x < extra ? blockIdx.x : extra);
    const int64_t t_end = t_begin + per + ((int64_t)blockIdx.x < extra ? 1 : 0);
    auto claim = [&]() -> int64_t {
        int k = 0;
        if (lane == 0) k = atomicAdd(&claimed, 1);
        return t_begin + __builtin_amdgcn_readfirstlane(k);
    };
    // Two operand buffers, alternating: the next claimed tile's rows load into
    // one while the other runs through the network (no copies between them).
    V ba[COLS][KC], bb[COLS][KC];
    auto load_tile = [&](V (&dst)[COLS][KC], int64_t t) {      // rows past the end read the last row
        const void* e;
        int64_t base, cnt;
        float* out;
        src.locate(t, e, base, cnt, out);
        const T* enc = reinterpret_cast<const T*>(e);
        #pragma unroll
        for (int col = 0; col < COLS; ++col) {
            int64_t row = base + 16 * col + ln;
            row = row < cnt ? row : cnt - 1;
            #pragma unroll
            for (int c = 0; c < KC; ++c)
                dst[col][c] = *reinterpret_cast<const V*>(enc + row * kEncWidth + 32 * c + 8 * g);
        }
    };
    auto run_tile = [&](V (&b)[COLS][KC], int64_t t) {
        // the weights are read from LDS per tile: held in registers across the
        // loop (42 fragments, 168 VGPRs) they would spill
        asm volatile("" ::: "memory");
        float r[COLS][3];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) reflectance_operand(b[col][1], fcol, ln, r[col]);
        f32x4 o[COLS];
        mlp_tile_colwise<T, COLS, NH>(sfr, b, lane, o, [](int, const f32x4&) {});
        const void* e;
        int64_t base, cnt;
        float* out;
        src.locate(t, e, base, cnt, out);
        store_rgb<COLS>(o, r, base, cnt, g, ln, out);
    };
    int64_t tile = claim();
    if (tile >= t_end) return;
    load_tile(ba, tile);
    for (;;) {
        int64_t nt = claim();
        if (nt < t_end) load_tile(bb, nt);
        run_tile(ba, tile);
        if (nt >= t_end) break;
        tile = nt;
        nt = claim();
        if (nt < t_end) load_tile(ba, nt);
        run_tile(bb, tile);
        if (nt >= t_end) break;
        tile = nt;
    }
}

// Inference over several request segments in one launch (serving: queued
// queries of one cache that no training step separates).  Tile t of the
// launch belongs to the segment whose cumulative tile range holds it; within
// a segment the kernel is k_fwd_mfma.
template <typename T, int W, int COLS>
__global__ __launch_bounds__(256, 2) void k_fwd_mfma_segs(const T* __restrict__ ffr, int n_frags, SegList segs,
                                                          int n_hidden, int fcol) {
    using V = typename Vec8<T>::type;
    constexpr int KC = W / 32;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    V* sfr = reinterpret_cast<V*>(smem_raw);
    stage_frags(sfr, reinterpret_cast<const V*>(ffr), n_frags);
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, ln = lane & 15;
    const int64_t n_tiles = segs.tile_end[segs.count - 1];
    const int64_t tstride = (int64_t)gridDim.x * 4;
    // segment of tile t (wave-uniform) and the tile's first row in it
    auto locate = [&](int64_t t, int& sg, int64_t& base) {
        sg = 0;
        while (t >= segs.tile_end[sg]) ++sg;
        base = (t - (sg ? segs.tile_end[sg - 1] : 0)) * 16 * COLS;
    };
    V nxt[COLS][2];
    auto load_tile = [&](int64_t t) {
        int sg;
        int64_t base;
        locate(t, sg, base);
        const T* enc = reinterpret_cast<const T*>(segs.enc[sg]);
        const int64_t n = segs.n[sg];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) {
            int64_t row = base + 16 * col + ln;
            row = row < n ? row : n - 1;
            #pragma unroll
            for (int c = 0; c < 2; ++c)
                nxt[col][c] = *reinterpret_cast<const V*>(enc + row * kEncWidth + 32 * c + 8 * g);
        }
    };
    int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile < n_tiles) load_tile(tile);
    for (; tile < n_tiles; tile += tstride) {
        V b[COLS][KC];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) {
            b[col][0] = nxt[col][0];
            b[col][1] = nxt[col][1];
        }
        if (tile + tstride < n_tiles) load_tile(tile + tstride);
        float r[COLS][3];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) reflectance_operand(b[col][1], fcol, ln, r[col]);
        f32x4 o[COLS];
        mlp_tile<T, W, COLS>(sfr, b, n_hidden, lane, o);
        int sg;
        int64_t base;
        locate(tile, sg, base);
        store_rgb<COLS>(o, r, base, segs.n[sg], g, ln, segs.rgb[sg]);
    }
}

// Inference from raw records with the encoding fused in (Sec. 3.6 encodings,
// Sec. 4 network).  Each wave owns a 64-record tile: lane r encodes record r
// (the next tile's raw floats are loaded while the current tile computes),
// writes its 64 features to the wave's own LDS rows, and the wave reads them
// back as B operands.  HBM traffic per query: the raw record in, RGB out.
// NW waves per workgroup share one copy of the weights in LDS.
template <typename T, int W, int PRESET, int LAYOUT, int NW>
__global__ __launch_bounds__(64 * NW) void k_fwd_raw_mfma(const T* __restrict__ ffr, int n_frags,
                                                         const float* __restrict__ raw, int64_t n,
                                                         float* __restrict__ rgb, int n_hidden, int fcol) {
    using V = typename Vec8<T>::type;
    constexpr int COLS = 4, KC = W / 32;
    constexpr int RW = LAYOUT == NRC_RAW14 ? 14 : 16;
    constexpr int ROW = 72;                     // LDS row stride of an encoded record, elements
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    V* sfr = reinterpret_cast<V*>(smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, ln = lane & 15;
    T* senc = reinterpret_cast<T*>(smem_raw + n_frags * 1024) + wave * 64 * ROW;
    stage_frags<64 * NW>(sfr, reinterpret_cast<const V*>(ffr), n_frags);
    __syncthreads();

    const int64_t n_tiles = (n + 63) / 64;
    const int64_t tstride = (int64_t)gridDim.x * NW;
    float x[RW];
    auto load_raw = [&](int64_t t) {
        int64_t row = t * 64 + lane;
        row = row < n ? row : n - 1;
        const float* src = raw + row * RW;
        if (RW == 16) {
            #pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 v = reinterpret_cast<const float4*>(src)[q];
                x[4 * q] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
            }
        } else {
            #pragma unroll
            for (int q = 0; q < RW / 2; ++q) {
                const float2 v = reinterpret_cast<const float2*>(src)[q];
                x[2 * q] = v.x; x[2 * q + 1] = v.y;
            }
        }
    };
    int64_t tile = (int64_t)blockIdx.x * NW + wave;
    if (tile < n_tiles) load_raw(tile);
    for (; tile < n_tiles; tile += tstride) {
        {
            float f[64];
            encode_record<PRESET, LAYOUT>(x, f);
            T* dst = senc + lane * ROW;
            #pragma unroll
            for (int q = 0; q < 8; ++q) {
                const f32x4 lo = f32x4{f[8 * q], f[8 * q + 1], f[8 * q + 2], f[8 * q + 3]};
                const f32x4 hi = f32x4{f[8 * q + 4], f[8 * q + 5], f[8 * q + 6], f[8 * q + 7]};
                *reinterpret_cast<V*>(dst + 8 * q) = pack8<T, V>(lo, hi);
            }
        }
        if (tile + tstride < n_tiles) load_raw(tile + tstride);
        // LDS writes of all lanes complete before any lane reads another's row.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        V b[COLS][KC];
        #pragma unroll
        for (int col = 0; col < COLS; ++col)
            #pragma unroll
            for (int c = 0; c < 2; ++c)
                b[col][c] = *reinterpret_cast<const V*>(senc + (16 * col + ln) * ROW + 32 * c + 8 * g);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float r[COLS][3];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) reflectance_operand(b[col][1], fcol, ln, r[col]);
        f32x4 o[COLS];
        mlp_tile<T, W, COLS>(sfr, b, n_hidden, lane, o);
        store_rgb<COLS>(o, r, tile * 64, n, g, ln, rgb);
    }
}

// Encodes the lane's record x and stores its 64 features, rounded to T, at
// dst (a 16-byte aligned LDS row), followed by the record's reflectance
// factor alpha + beta (Sec. 5) as 3 floats in the row's 16 spare bytes: the
// rounded diffuse plus the rounded specular albedo per channel, the same
// arithmetic reflectance_operand does on the B operand, here in the lane that
// holds the record instead of three shuffles per channel and column.
// Features 8q .. 8q + 7 of f, rounded to T, into an LDS row.
template <typename T>
__device__ inline void store8(T* dst, const float* f, int q) {
    using V = typename Vec8<T>::type;
    const f32x4 lo = f32x4{f[8 * q], f[8 * q + 1], f[8 * q + 2], f[8 * q + 3]};
    const f32x4 hi = f32x4{f[8 * q + 4], f[8 * q + 5], f[8 * q + 6], f[8 * q + 7]};
    *reinterpret_cast<V*>(dst + 8 * q) = pack8<T, V>(lo, hi);
}

// Features f[0 .. 3], rounded to T, into an LDS row (8-byte aligned); the same
// rounding as store8.
template <typename T>
__device__ inline void store4(T* dst, const float* f) {
    if constexpr (sizeof(T) == 2 && !__is_same(T, _Float16)) {
        uint2 r;
        r.x = __builtin_bit_cast(unsigned int, __builtin_convertvector(f32x2{f[0], f[1]}, bf16x2));
        r.y = __builtin_bit_cast(unsigned int, __builtin_convertvector(f32x2{f[2], f[3]}, bf16x2));
        *reinterpret_cast<uint2*>(dst) = r;
    } else {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        *reinterpret_cast<h4*>(dst) = __builtin_convertvector(f32x4{f[0], f[1], f[2], f[3]}, h4);
    }
}

template <typename T, int PRESET>
__device__ inline void store_reflectance(T* dst, const float* f, int fcol) {
    f32x4 r = f32x4{1.0f, 1.0f, 1.0f, 0.0f};
    constexpr int ac = PRESET == NRC_PRESET_CONFIG ? kAlbedoColConfig : kAlbedoColPaper;
    if (fcol) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = (float)to_t<T>(f[ac + c]) + (float)to_t<T>(f[ac + 3 + c]);
    }
    *reinterpret_cast<f32x4*>(dst + 64) = r;
}

template <typename T, int PRESET, int LAYOUT>
__device__ inline void encode_to_lds(const float* x, T* dst, int fcol) {
    float f[64];
    encode_record<PRESET, LAYOUT>(x, f);
    #pragma unroll
    for (int q = 0; q < 8; ++q) store8<T>(dst, f, q);
    store_reflectance<T, PRESET>(dst, f, fcol);
}

// Orders a wave's LDS accesses: those before complete before those after,
// across the wave's lanes.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fused raw -> encode -> network inference for a depth fixed at compile time
// (NH hidden layers of width 64), software-pipelined: while a wave's matrix
// cores run one tile, its vector ALUs encode the wave's next tile into the
// wave's LDS rows.  The whole tile is one basic block (layers unrolled, loads
// clamped instead of branched), and the weights and encode rows are distinct
// __shared__ arrays, so the compiler may interleave the two instruction
// streams.  Results equal k_fwd_raw_mfma's bit for bit: every record goes
// through the same arithmetic.  (Measured: matrix and vector work of one wave
// overlap only partly on gfx950, about half of the MFMA time.)
template <typename T, int PRESET, int LAYOUT, int NH, int NW>
__global__ __launch_bounds__(64 * NW) void k_fwd_raw_mfma_fixed(const T* __restrict__ ffr,
                                                               const float* __restrict__ raw, int64_t n,
                                                               float* __restrict__ rgb, int fcol) {
    using V = typename Vec8<T>::type;
    constexpr int W = 64, COLS = 4, KC = 2;
    constexpr int RW = LAYOUT == NRC_RAW14 ? 14 : 16;
    static_assert(NH == 5, "the next tile's encoding is spread over five hidden layers");
    constexpr int ROW = 72;                                // LDS row stride of an encoded record
    constexpr int NF = 2 * (W / 16) + (NH - 1) * (W / 16) * KC + KC;   // forward fragments
    __shared__ V sfr[NF * 64];
    __shared__ __attribute__((aligned(16))) T senc_all[NW * 64 * ROW];
    __shared__ int claimed;                                // tiles of the share handed out so far
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, ln = lane & 15;
    T* senc = senc_all + wave * 64 * ROW;
    if (threadIdx.x == 0) claimed = 0;
    stage_frags<64 * NW>(sfr, reinterpret_cast<const V*>(ffr), NF);
    __syncthreads();

    // The workgroup owns a contiguous share of the tiles; its waves claim them
    // one at a time (an LDS counter), so a wave the SIMD's issue arbitration
    // favours takes more tiles and all waves of the CU finish together.
    // (Measured with a fixed tile per wave and stride: the waves of a CU ran at
    // 3.3 to 7.3 us per tile and the pass ended with the slowest.)
    const int64_t n_tiles = (n + 63) / 64;
    const int64_t per = n_tiles / gridDim.x, extra = n_tiles % gridDim.x;
    const int64_t t_begin = (int64_t)blockIdx.x * per + ((int64_t)blockIdx.x < extra ? blockIdx.x : extra);
    const int64_t t_end = t_begin + per + ((int64_t)blockIdx.x < extra ? 1 : 0);
    auto claim = [&]() -> int64_t {
        int k = 0;
        if (lane == 0) k = atomicAdd(&claimed, 1);
        return t_begin + __builtin_amdgcn_readfirstlane(k);
    };
    float x[RW];
    auto load_raw = [&](int64_t t) {      // rows past the end read the last row
        int64_t row = t * 64 + lane;
        row = row < n ? row : n - 1;
        const float* src = raw + row * RW;
        if (RW == 16) {
            #pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 v = reinterpret_cast<const float4*>(src)[q];
                x[4 * q] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
            }
        } else {
            #pragma unroll
            for (int q = 0; q < RW / 2; ++q) {
                const float2 v = reinterpret_cast<const float2*>(src)[q];
                x[2 * q] = v.x; x[2 * q + 1] = v.y;
            }
        }
    };
    int64_t tile = claim();
    if (tile >= t_end) return;
    load_raw(tile);
    encode_to_lds<T, PRESET, LAYOUT>(x, senc + lane * ROW, fcol);
    int64_t nxt = claim();                 // its record is in x while tile computes
    if (nxt < t_end) load_raw(nxt);        // past the share: nothing to read (the encoding is never used)
    while (tile < t_end) {
        const int64_t nn = claim();
        wave_lds_sync();                   // this tile's rows are written
        V b[COLS][KC];
        float r[COLS][3];
        #pragma unroll
        for (int col = 0; col < COLS; ++col) {
            #pragma unroll
            for (int c = 0; c < 2; ++c)
                b[col][c] = *reinterpret_cast<const V*>(senc + (16 * col + ln) * ROW + 32 * c + 8 * g);
            const f32x4 rv = *reinterpret_cast<const f32x4*>(senc + (16 * col + ln) * ROW + 64);
            r[col][0] = rv[0]; r[col][1] = rv[1]; r[col][2] = rv[2];
        }
        wave_lds_sync();                   // and read by every lane before they are rewritten
        // the next tile's encoding (vector ALUs) beside this tile's network
        // (matrix cores): part l of the record's features after layer l's
        // first products, tied to them by an empty asm so the compiler cannot
        // hoist the encoding ahead of the matrix instructions
        float f[64];
        T* row = senc + lane * ROW;
        // Each part reads its own raw fields (a position coordinate, the
        // direction, the rest), used by no other part, so they are tied in place.
        auto hook = [&](int l, const f32x4& dep) {
            const int lo = l <= 2 ? l : l == 3 ? 3 : (LAYOUT == NRC_RAW14 ? 5 : 6);
            const int hi = l <= 2 ? l : l == 3 ? (LAYOUT == NRC_RAW14 ? 4 : 5) : RW - 1;
            #pragma unroll
            for (int k = 0; k < RW; ++k)
                if (k >= lo && k <= hi) asm volatile("" : "+v"(x[k]) : "v"(dep[0]));
            const float* xs = x;
            if (l == 0) {
                encode_part<PRESET, LAYOUT, 0>(xs, f);
                store8<T>(row, f, 0);
            } else if (l == 1) {
                encode_part<PRESET, LAYOUT, 1>(xs, f);
                store8<T>(row, f, 1);
                store8<T>(row, f, 2);
            } else if (l == 2) {
                encode_part<PRESET, LAYOUT, 2>(xs, f);
                store8<T>(row, f, 3);
            } else if (l == 3) {
                encode_part<PRESET, LAYOUT, 3>(xs, f);
                store8<T>(row, f, 4);
            } else if (l == 4) {
                encode_part<PRESET, LAYOUT, 4>(xs, f);
                store8<T>(row, f, 5);
                store8<T>(row, f, 6);
                store8<T>(row, f, 7);
                store_reflectance<T, PRESET>(row, f, fcol);
            }
        };
        f32x4 o[COLS];
        mlp_tile_colwise<T, COLS, NH>(sfr, b, lane, o, hook);
        if (nn < t_end) load_raw(nn);
        store_rgb<COLS>(o, r, tile * 64, n, g, ln, rgb);
        tile = nxt;
        nxt = nn;
    }
}

// ---------------------------------------------------------------------------
// Training: forward + loss gradient + data backward + per-tile weight gradient
// ---------------------------------------------------------------------------
// Records per workgroup: 64 at width 64 (4 chain waves), 32 at width 128 (2
// chain waves), so that every layer's activations and deltas of the tile fit
// in LDS; as many weight-gradient waves again.
template <int W> struct TrainShape {
    static constexpr int TS = W == 64 ? 64 : 32;   // records per tile
    static constexpr int NW = TS / 16;             // chain waves per workgroup
    static constexpr int LDT = TS + 8;             // row stride of dL/dy, elements
    static constexpr int LDR = W == 64 ? 72 : 144; // record row stride of h_l, delta_l
};
// LDS bytes of one training workgroup: h_0 [record][64 + 8], h_1..h_H and
// delta_1..delta_H [record][LDR], then dL/dy [3 (16) rows][record].
__host__ __device__ constexpr int train_lds_bytes(int W, int H) {
    return ((W == 64 ? 64 : 32) * (72 + 2 * H * (W == 64 ? 72 : 144)) + 16 * (W == 64 ? 72 : 40)) * 2;
}

// Activation buffer of the autograd form (ACT): per tile, h_1 .. h_H as
// [layer][record][feature] at the operand precision (the LDS rows without
// their padding), then, after every tile's block, the network output
// [tile * TS + record][4] (FP32).  kActNone: no buffer; kActStore: forward only,
// writes the buffer and rgb, then exits; kActLoad: the forward pass is read
// from the buffer instead of recomputed.
constexpr int kActNone = 0, kActStore = 1, kActLoad = 2;

// Weight-gradient waves beside the chain waves (none in the forward-only form).
template <int W, int ACT> constexpr int train_helpers() { return ACT == kActStore ? 0 : TrainShape<W>::NW; }

// Training records given raw (RAWL = their layout, PRESET = the cache's
// encoding; RAWL < 0: encoded rows): the kernel's enc argument then points at
// the raw records, FP32 [n][14 or 16], and the four lanes (g, j) of each chain
// wave encode record j, a share of its features each, into the record's h_0
// row, where the stand-alone encoding kernel would have written it, before the
// wave reads its operands back.
template <typename T, int W, bool UPSTREAM, bool GENC, int ACT = kActNone, int RAWL = -1,
          int PRESET = NRC_PRESET_CONFIG>
__global__ __launch_bounds__(512) void k_train_mfma(const T* __restrict__ ffr,
                                                    const T* __restrict__ bfr,
                                                    const T* __restrict__ enc,
                                                    const float* __restrict__ tgt,
                                                    const int32_t* __restrict__ idx, int64_t n,
                                                    int n_hidden, float loss_eps, float grad_scale,
                                                    float* __restrict__ partials,
                                                    float* __restrict__ loss_part,
                                                    int32_t* __restrict__ tile_bad,
                                                    float* __restrict__ genc, int fcol,
                                                    T* __restrict__ act, float* __restrict__ rgb,
                                                    LcgGather lg) {
    using V = typename Vec8<T>::type;
    using S = TrainShape<W>;
    constexpr int MB = W / 16, KC = W / 32, TS = S::TS, NW = S::NW, LDT = S::LDT, TK = TS / 32;
    constexpr int LDR = S::LDR, LD0 = 72;
    constexpr int NHW = train_helpers<W, ACT>();             // weight-gradient waves
    constexpr int NT = 64 * (NW + NHW);
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    __shared__ float wsum[4];
    const Geo geo(W, n_hidden);
    // h_l and delta_l record-major (a record's features contiguous, so the
    // chain waves store and read them 8 bytes at a time); dL/dy feature-major.
    T* hT = reinterpret_cast<T*>(smem_raw);                  // h_0 [TS][LD0], h_1 .. h_H [TS][LDR]
    T* dT = hT + TS * LD0 + n_hidden * TS * LDR;             // delta_1 .. delta_H [TS][LDR]
    T* dO = dT + n_hidden * TS * LDR;                        // dL/dy, rows 0..2 [3][LDT]
    auto hrow = [&](int l) { return hT + (l == 0 ? 0 : TS * LD0 + (l - 1) * TS * LDR); };
    auto drow = [&](int l) { return dT + (l - 1) * TS * LDR; };
    auto ldr = [&](int l) { return l == 0 ? LD0 : LDR; };

    const int P = geo.n_params();
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, ln = lane & 15;
    const int64_t tile = blockIdx.x;
    const bool chain = wave < NW;                            // a chain wave owns 16 records
    const int sl = 16 * (chain ? wave : 0) + ln;             // record within the tile
    const int64_t row = tile * TS + sl;
    const bool valid = chain && row < n;
    // record read for this slot: idx[row] or the LCG orbit for a gathered batch, else row
    const int64_t src = !valid ? 0 : gather_row(idx, lg, row);
    float* part = partials + tile * (int64_t)P;
    const V* gf = reinterpret_cast<const V*>(ffr) + lane;
    const V* gb = reinterpret_cast<const V*>(bfr) + lane;
    // A product with a weight operand: the fragment at f[i] (hi), and in the
    // BF16 form also its lo part, one fragment set further on (the pair carries
    // the weight to ~16 significant bits; both operands are BF16).
    constexpr bool SPLIT = __is_same(T, __bf16);
    const int lo_f = geo.n_fwd_frags() * 64, lo_b = geo.n_bwd_frags() * 64;
    auto wf = [&](const V* f, int i, const V& bop, f32x4 c) {
        c = mfma(f[i], bop, c);
        if (SPLIT) c = mfma(f[i + lo_f], bop, c);
        return c;
    };
    auto wb = [&](const V* f, int i, const V& bop, f32x4 c) {
        c = mfma(f[i], bop, c);
        if (SPLIT) c = mfma(f[i + lo_b], bop, c);
        return c;
    };

    // A chained-order operand (features 32c + 4g .. +3 and 32c + 16 + 4g .. +3
    // of record sl) into a record-major store: two 8-byte writes.
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    auto put = [&](T* base, const V& v, int c) {
        const u32x4 u = __builtin_bit_cast(u32x4, v);
        *reinterpret_cast<u32x2*>(base + sl * LDR + 32 * c + 4 * g) = u32x2{u[0], u[1]};
        *reinterpret_cast<u32x2*>(base + sl * LDR + 32 * c + 16 + 4 * g) = u32x2{u[2], u[3]};
    };

    // ---- forward (each wave: its 16 records, activations in VGPRs) ----------
    V b[KC];
    if constexpr (RAWL >= 0) {
        static_assert(!UPSTREAM && !GENC && ACT == kActNone, "raw records feed the training step only");
        constexpr int RW = RAWL == NRC_RAW14 ? 14 : 16;
        if (chain) {
            T* h0 = hT + sl * LD0;
            // BF16: the first layer's weight fragments (hi and lo parts) start
            // loading now, beside the encoding, so they are cached when the
            // layer reads them (the LDS hand-over below orders every later
            // memory access).  Measured: the BF16 step 17.8 -> 16.2 us; FP16,
            // with half the fragments, no faster, so it does not prefetch.
            constexpr int NPRE = SPLIT ? 4 * MB : 0;
            V pre[NPRE > 0 ? NPRE : 1];
            #pragma unroll
            for (int i = 0; i < NPRE; ++i) pre[i] = gf[(i % (2 * MB)) * 64 + (i < 2 * MB ? 0 : lo_f)];
            // The four lane groups of a record share its encoding: groups 0..2
            // the frequency encoding of position coordinate g (the same code
            // for the three, features 12g ..12g + 11), group 3 the rest (36 ..63).
            float x[RW];
            if (valid) {
                const float* rr = reinterpret_cast<const float*>(enc) + src * RW;
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
                for (int q = 0; q < 3; ++q) store4<T>(h0 + 12 * g + 4 * q, f + 4 * q);
            } else {
                encode_part<PRESET, RAWL, 3>(x, f);
                encode_part<PRESET, RAWL, 4>(x, f);
                if (!valid) {
                    #pragma unroll
                    for (int k = 36; k < 64; ++k) f[k] = 0.0f;
                }
                #pragma unroll
                for (int q = 9; q < 16; ++q) store4<T>(h0 + 4 * q, f + 4 * q);
            }
            wave_lds_sync();
            #pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = *reinterpret_cast<const V*>(h0 + 32 * c + 8 * g);
            #pragma unroll
            for (int i = 0; i < NPRE; ++i) asm volatile("" :: "v"(pre[i]));
        } else {
            b[0] = b[1] = zero8<V>();
        }
    } else {
        #pragma unroll
        for (int c = 0; c < 2; ++c) {
            b[c] = valid ? *reinterpret_cast<const V*>(enc + src * kEncWidth + 32 * c + 8 * g) : zero8<V>();
            if (chain) *reinterpret_cast<V*>(hT + sl * LD0 + 32 * c + 8 * g) = b[c];
        }
    }
    float r[3];                      // reflectance factor of record sl (lanes 0..15)
    reflectance_operand(b[1], fcol, ln, r);
    // this record's targets (or upstream gradient), loaded now and used after the forward pass
    float tg[3] = {0.f, 0.f, 0.f};
    if (ACT != kActStore && g == 0 && valid) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) tg[c] = tgt[src * 3 + c];
    }
    // the tile's block of the activation buffer and its network outputs
    const int64_t n_tiles = gridDim.x;
    T* act_t = act + tile * (int64_t)(n_hidden * W * TS);
    float* act_y = reinterpret_cast<float*>(act + n_tiles * (int64_t)(n_hidden * W * TS));
    // copy h_1 .. h_H between the LDS rows and the buffer, 16 bytes at a time
    auto copy_act = [&](bool to_lds) {
        constexpr int CPR = W * (int)sizeof(T) / 16;          // 16-byte chunks per record row
        const int rows = n_hidden * TS;
        for (int i = tid; i < rows * CPR; i += NT) {
            const int rr = i / CPR, q = i - rr * CPR;
            u32x4* l = reinterpret_cast<u32x4*>(hT + TS * LD0 + rr * LDR) + q;
            u32x4* gp = reinterpret_cast<u32x4*>(act_t + rr * W) + q;
            if (to_lds) *l = *gp; else *gp = *l;
        }
    };
    const int n_fwd = (ACT == kActLoad || !chain) ? 0 : n_hidden;   // layers the forward pass computes
    if constexpr (W == 64 && SPLIT) {
        // BF16 at width 64: every layer has the same 8 fragments (4 row blocks
        // x 2 K chunks) and their lo parts.  The next layer's 16 load into
        // registers while this layer computes, so no layer waits for its
        // weights (measured: 15.9 -> 14.9 us per step; FP16, with half the
        // fragments per layer, measured no faster, and the same prefetch in
        // the backward pass gained nothing in either).
        constexpr int NF8 = MB * KC, NFR = 2 * NF8;              // hi parts, then lo parts
        auto load_fw = [&](int l, V (&d)[NFR]) {
            const V* fl = gf + geo.fwd_base(l) * 64;
            #pragma unroll
            for (int i = 0; i < NFR; ++i) d[i] = fl[(i % NF8) * 64 + (i < NF8 ? 0 : lo_f)];
        };
        // the product of wf: hi part, then lo part
        auto mm = [&](const V (&fr)[NFR], int i, const V& bop, f32x4 c) {
            c = mfma(fr[i], bop, c);
            return mfma(fr[NF8 + i], bop, c);
        };
        V fa[NFR], fn[NFR];
        if (n_fwd > 0) load_fw(0, fa);
        for (int l = 0; l < n_fwd; ++l) {
            if (l + 1 < n_fwd) load_fw(l + 1, fn);
            f32x4 acc[MB];
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = mm(fa, mb * KC, b[0], f32x4{0.f, 0.f, 0.f, 0.f});
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = mm(fa, mb * KC + 1, b[1], acc[mb]);
            T* ho = hrow(l + 1);
            #pragma unroll
            for (int c = 0; c < KC; ++c) {
                b[c] = relu_packed(pack8<T, V>(acc[2 * c], acc[2 * c + 1]));
                put(ho, b[c], c);
            }
            #pragma unroll
            for (int i = 0; i < NFR; ++i) fa[i] = fn[i];
        }
    } else
    for (int l = 0; l < n_fwd; ++l) {
        const int kc = l == 0 ? 2 : KC;
        const V* fl = gf + geo.fwd_base(l) * 64;
        f32x4 acc[MB];
        #pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = wf(fl, (mb * kc) * 64, b[0], f32x4{0.f, 0.f, 0.f, 0.f});
        #pragma unroll
        for (int c = 1; c < KC; ++c) {
            if (c >= kc) break;
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = wf(fl, (mb * kc + c) * 64, b[c], acc[mb]);
        }
        T* ho = hrow(l + 1);
        #pragma unroll
        for (int c = 0; c < KC; ++c) {
            b[c] = relu_packed(pack8<T, V>(acc[2 * c], acc[2 * c + 1]));
            put(ho, b[c], c);
        }
    }
    f32x4 y = f32x4{0.f, 0.f, 0.f, 0.f};
    if (ACT == kActLoad) {
        copy_act(true);
        if (g == 0 && valid) {
            #pragma unroll
            for (int c = 0; c < 3; ++c) y[c] = act_y[row * 4 + c];
        }
        __syncthreads();
    } else {
        const V* fo = gf + geo.fwd_base(n_hidden) * 64;
        y = wf(fo, 0, b[0], f32x4{0.f, 0.f, 0.f, 0.f});
        #pragma unroll
        for (int c = 1; c < KC; ++c) y = wf(fo, c * 64, b[c], y);
    }
    if (ACT == kActStore) {
        // the prediction (network output times the reflectance factor) and
        // the buffer for the backward pass; nothing else
        if (g == 0 && valid) {
            #pragma unroll
            for (int c = 0; c < 3; ++c) {
                rgb[row * 3 + c] = y[c] * r[c];
                act_y[row * 4 + c] = y[c];
            }
            act_y[row * 4 + 3] = 0.0f;
        }
        __syncthreads();
        copy_act(false);
        return;
    }

    // ---- loss gradient (Eq. 5); lanes 0..15 of each wave hold y[0..2] -------
    // The prediction is the network output times r; the network's output
    // gradient is the prediction's gradient times r.
    float d0 = 0.f, d1 = 0.f, d2 = 0.f, lterm = 0.f;
    if (g == 0 && valid) {
        if (UPSTREAM) {
            d0 = tg[0] * grad_scale * r[0];
            d1 = tg[1] * grad_scale * r[1];
            d2 = tg[2] * grad_scale * r[2];
        } else {
            const float p0 = y[0] * r[0], p1 = y[1] * r[1], p2 = y[2] * r[2];
            const float lum = (p0 + p1 + p2) * (1.0f / 3.0f);
            const float inv_den = 1.0f / fmaf(lum, lum, loss_eps);
            const float e0 = p0 - tg[0];
            const float e1 = p1 - tg[1];
            const float e2 = p2 - tg[2];
            lterm = fmaf(e2, e2, fmaf(e1, e1, e0 * e0)) * inv_den;
            d0 = 2.0f * e0 * inv_den * grad_scale * r[0];
            d1 = 2.0f * e1 * inv_den * grad_scale * r[1];
            d2 = 2.0f * e2 * inv_den * grad_scale * r[2];
        }
    }
    V bd = zero8<V>();
    if (g == 0 && chain) {
        bd[0] = to_t<T>(d0); bd[1] = to_t<T>(d1); bd[2] = to_t<T>(d2);
        dO[0 * LDT + sl] = bd[0];
        dO[1 * LDT + sl] = bd[1];
        dO[2 * LDT + sl] = bd[2];
    }
    const float wl = wave_sum_compensated(lterm);
    if (lane == 0 && chain) wsum[wave] = wl;

    // ---- weight gradients: dW_l = delta_{l+1} h_l^T over the tile's records --
    // Computed by the helper waves (hw = 0 .. NHW-1) while the chain waves run
    // the data backward pass: dW_l as soon as delta_{l+1} is in LDS.  The 16x16
    // result blocks are stored in the accumulator's own layout, one float4 per
    // lane: slot w_off(l) + ((mb * NB + nb) * 64 + lane) * 4 + j holds
    // dW_l[16 mb + 4 g + j][16 nb + ln].  The output layer is row-major.
    bool bad = false;
    auto dw_layer = [&](int l, int hw) {
        const int ncols = l == 0 ? kEncWidth : W;
        const int NB = ncols / 16;
        const T* hl = hrow(l);
        const int lh = ldr(l);
        const T* dl = l == n_hidden ? dO : drow(l + 1);
        const int woff = geo.w_off(l);
        // Operand of records 32 kc + 8 g .. +7 (K slots 8 g .. 8 g + 7) for
        // feature 16 blk + ln from a record-major store, by two LDS transpose
        // reads: in each 16-lane group, lane i receives element i % 4 of the
        // 8-byte segments that lanes i / 4, i / 4 + 4, i / 4 + 8, i / 4 + 12
        // address, so lane i addresses record rec0 + i / 4, features
        // 16 blk + 4 (i % 4) .. +3.
        auto gather = [&](const T* base, int stride, int blk, int kc) {
            typedef short s16x4 __attribute__((ext_vector_type(4)));
            typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
            const T* p = base + (32 * kc + 8 * g + (ln >> 2)) * stride + 16 * blk + 4 * (ln & 3);
            const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)p);
            const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p + 4 * stride));
            return __builtin_bit_cast(V, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
        };
        for (int nb = hw; nb < NB; nb += NHW) {
            V bb[TK];
            #pragma unroll
            for (int kc = 0; kc < TK; ++kc) bb[kc] = gather(hl, lh, nb, kc);
            if (l == n_hidden) {
                f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
                #pragma unroll
                for (int kc = 0; kc < TK; ++kc) {
                    const V a = ln < kNOut ? *reinterpret_cast<const V*>(dl + ln * LDT + 32 * kc + 8 * g)
                                           : zero8<V>();
                    acc = mfma(a, bb[kc], acc);
                }
                if (g == 0) {
                    #pragma unroll
                    for (int j = 0; j < kNOut; ++j) {
                        part[woff + j * W + 16 * nb + ln] = acc[j];
                        bad |= !isfinite(acc[j]);
                    }
                }
            } else {
                #pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    f32x4 acc = mfma(gather(dl, LDR, mb, 0), bb[0], f32x4{0.f, 0.f, 0.f, 0.f});
                    #pragma unroll
                    for (int kc = 1; kc < TK; ++kc) acc = mfma(gather(dl, LDR, mb, kc), bb[kc], acc);
                    // streamed past the caches: read once, by the reduction
                    __builtin_nontemporal_store(acc, reinterpret_cast<f32x4*>(part + woff + ((mb * NB + nb) * 64 + lane) * 4));
                    #pragma unroll
                    for (int j = 0; j < 4; ++j) bad |= !isfinite(acc[j]);
                }
            }
        }
    };
    __syncthreads();   // dL/dy and h_0 .. h_H are in LDS

    // ---- data backward: the whole delta chain in VGPRs, each delta kept in LDS
    // delta_l = (W_l^T delta_{l+1}) masked by ReLU'(z_l); W_H^T acts on dL/dy.
    for (int l = n_hidden; l >= 1; --l) {
      if (!chain) {
        dw_layer(l, wave - NW);
      } else {
        const T* hl = hrow(l);
        f32x4 acc[MB];
        if (l == n_hidden) {
            const V* fb = gb + geo.bwd_base(n_hidden) * 64;
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = wb(fb, mb * 64, bd, f32x4{0.f, 0.f, 0.f, 0.f});
        } else {
            const V* fb = gb + geo.bwd_base(l) * 64;
            #pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb] = wb(fb, (mb * KC) * 64, b[0], f32x4{0.f, 0.f, 0.f, 0.f});
            #pragma unroll
            for (int c = 1; c < KC; ++c)
                #pragma unroll
                for (int mb = 0; mb < MB; ++mb) acc[mb] = wb(fb, (mb * KC + c) * 64, b[c], acc[mb]);
        }
        #pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            typedef T t4 __attribute__((ext_vector_type(4)));
            const t4 hv = *reinterpret_cast<const t4*>(hl + sl * LDR + 16 * mb + 4 * g);
            #pragma unroll
            for (int j = 0; j < 4; ++j) acc[mb][j] = (float)hv[j] > 0.0f ? acc[mb][j] : 0.0f;
        }
        T* dl = drow(l);
        #pragma unroll
        for (int c = 0; c < KC; ++c) {
            b[c] = pack8<T, V>(acc[2 * c], acc[2 * c + 1]);
            put(dl, b[c], c);
        }
      }
      __syncthreads();   // delta_l is in LDS
    }
    if (!chain) dw_layer(0, wave - NW);
    if (GENC && chain) {
        // dL/dh_0 = W_0^T delta_1 (64 input features), with the loss scale
        // of the upstream gradient divided out.
        f32x4 acc[4];
        #pragma unroll
        for (int mb = 0; mb < 4; ++mb) acc[mb] = wb(gb, (mb * KC) * 64, b[0], f32x4{0.f, 0.f, 0.f, 0.f});
        #pragma unroll
        for (int c = 1; c < KC; ++c)
            #pragma unroll
            for (int mb = 0; mb < 4; ++mb) acc[mb] = wb(gb, (mb * KC + c) * 64, b[c], acc[mb]);
        const float inv_scale = 1.0f / grad_scale;
        #pragma unroll
        for (int mb = 0; mb < 4; ++mb)
            #pragma unroll
            for (int j = 0; j < 4; ++j) acc[mb][j] *= inv_scale;
        if (fcol) {
            // d(f_c R_c)/d(albedo column) = f_c: lane (g, ln) holds input
            // features 48 + 4g .. 48 + 4g + 3 of record sl in acc[3].
            float f[3];
            #pragma unroll
            for (int c = 0; c < 3; ++c) f[c] = __shfl(y[c], ln, 64);
            if (valid) {
                #pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int c = 48 + 4 * g + j - fcol;
                    if (c >= 0 && c < 6) {
                        c = c >= 3 ? c - 3 : c;
                        const float fc = c == 0 ? f[0] : c == 1 ? f[1] : f[2];
                        acc[3][j] = fmaf(tgt[src * 3 + c], fc, acc[3][j]);
                    }
                }
            }
        }
        if (valid) {
            #pragma unroll
            for (int mb = 0; mb < 4; ++mb)
                *reinterpret_cast<float4*>(genc + row * kEncWidth + 16 * mb + 4 * g) =
                    make_float4(acc[mb][0], acc[mb][1], acc[mb][2], acc[mb][3]);
        }
    }
    if (tid == 0) {
        // compensated combine of the waves' sums, in wave order
        float t = 0.0f, c = 0.0f;
        for (int w = 0; w < NW; ++w) {
            const float x = wsum[w], u = t + x;
            c += fabsf(t) >= fabsf(x) ? (t - u) + x : (x - u) + t;
            t = u;
        }
        loss_part[tile] = t + c;
    }
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0) tile_bad[tile] = any_bad ? 1 : 0;
}

// Workgroups of the persistent inference kernels that are resident at once:
// as many per CU as their weight copies fit in the 160 KB of LDS, at most four
// (the kernels' register budget allows two waves per SIMD per workgroup
// size), so the grid is covered in one round of dispatch.
inline int64_t resident_fwd_blocks(size_t lds) {
    int64_t per_cu = (int64_t)((160 * 1024) / (lds > 0 ? lds : 1));
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 4) per_cu = 4;
    return per_cu * device_cu_count();
}

// Waves per workgroup of k_fwd_mfma_fixed (one workgroup per CU).
constexpr int kEncWaves = 12;

template <typename T, typename Src>
hipError_t fwd_fixed_launch(const void* ffr, const Src& src, int64_t tiles, int fcol, hipStream_t s) {
    constexpr int NW = kEncWaves;
    int64_t blocks = (tiles + NW - 1) / NW;
    if (blocks > device_cu_count()) blocks = device_cu_count();
    hipLaunchKernelGGL((k_fwd_mfma_fixed<T, NW, Src>), dim3((unsigned)blocks), dim3(64 * NW), 0, s,
                       (const T*)ffr, src, fcol);
    return hipGetLastError();
}

template <typename T, int W>
hipError_t fwd_segs_dispatch(const Geo& d, const void* ffr, const SegList& segs, hipStream_t s) {
    constexpr int COLS = 4;
    const int64_t tiles = segs.tile_end[segs.count - 1];
    if (tiles == 0) return hipSuccess;
    if (W == 64 && d.H == 5) return fwd_fixed_launch<T>(ffr, EncSegs{segs}, tiles, d.F, s);
    const size_t lds = (size_t)d.n_fwd_frags() * 64 * 16;
    int64_t blocks = (tiles + 3) / 4;
    const int64_t resident = resident_fwd_blocks(lds);
    if (blocks > resident) blocks = resident;
    auto k = k_fwd_mfma_segs<T, W, COLS>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), lds, s, (const T*)ffr, d.n_fwd_frags(), segs, d.H,
                       d.F);
    return hipGetLastError();
}


template <typename T, int W>
hipError_t fwd_dispatch(const Geo& d, const void* ffr, const void* enc, int64_t n, float* rgb,
                        hipStream_t s) {
    constexpr int COLS = 4;
    const int64_t tiles = (n + 16 * COLS - 1) / (16 * COLS);
    if (tiles == 0) return hipSuccess;
    if (W == 64 && d.H == 5) return fwd_fixed_launch<T>(ffr, EncBatch{enc, n, rgb}, tiles, d.F, s);
    const size_t lds = (size_t)d.n_fwd_frags() * 64 * 16;
    int64_t blocks = (tiles + 3) / 4;
    const int64_t resident = resident_fwd_blocks(lds);
    if (blocks > resident) blocks = resident;
    auto k = k_fwd_mfma<T, W, COLS>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), lds, s, (const T*)ffr, d.n_fwd_frags(),
                       (const T*)enc, n, rgb, d.H, d.F);
    return hipGetLastError();
}

// Waves per workgroup of the fused kernel: 12 waves share one LDS copy of the
// weights (42 KB) beside their 12 encode buffers (110 KB), so one workgroup
// fits per CU, three waves per SIMD; the persistent grid has one workgroup
// per CU.  (Measured: with twice as many workgroups as CUs the second half
// waited ~10 us after the first half had finished before it was dispatched,
// and the 1080p pass took ~78 us instead of ~45.)
constexpr int kRawWaves = 12;

template <typename T, int W, int PRESET, int LAYOUT, int NW = kRawWaves>
hipError_t fwd_raw_launch(const Geo& d, const void* ffr, const float* raw, int64_t n, float* rgb,
                          hipStream_t s, int max_blocks) {
    const int64_t tiles = (n + 63) / 64;
    if (tiles == 0) return hipSuccess;
    const size_t lds = (size_t)d.n_fwd_frags() * 1024 + (size_t)NW * 64 * 72 * sizeof(T);
    int64_t blocks = (tiles + NW - 1) / NW;
    if (blocks > max_blocks) blocks = max_blocks;
    auto k = k_fwd_raw_mfma<T, W, PRESET, LAYOUT, NW>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * NW), lds, s, (const T*)ffr, d.n_fwd_frags(), raw,
                       n, rgb, d.H, d.F);
    return hipGetLastError();
}

// The fixed-depth, software-pipelined kernel for the paper's 5 hidden layers.
template <typename T, int PRESET, int LAYOUT>
hipError_t fwd_raw_fixed_launch(const Geo& d, const void* ffr, const float* raw, int64_t n, float* rgb,
                                hipStream_t s) {
    const int max_blocks = device_cu_count();
    constexpr int NW = kRawWaves;
    const int64_t tiles = (n + 63) / 64;
    if (tiles == 0) return hipSuccess;
    int64_t blocks = (tiles + NW - 1) / NW;
    if (blocks > max_blocks) blocks = max_blocks;
    hipLaunchKernelGGL((k_fwd_raw_mfma_fixed<T, PRESET, LAYOUT, 5, NW>), dim3((unsigned)blocks),
                       dim3(64 * NW), 0, s, (const T*)ffr, raw, n, rgb, d.F);
    return hipGetLastError();
}

// Runtime-depth fused kernel: 12 waves per workgroup when the weights and 12
// encode buffers fit in the 160 KB of LDS, else 8 (deeper networks).
template <typename T, int W, int PRESET, int LAYOUT>
hipError_t fwd_raw_generic(const Geo& d, const void* ffr, const float* raw, int64_t n, float* rgb,
                           hipStream_t s) {
    const size_t lds12 = (size_t)d.n_fwd_frags() * 1024 + (size_t)12 * 64 * 72 * sizeof(T);
    const size_t lds8 = (size_t)d.n_fwd_frags() * 1024 + (size_t)8 * 64 * 72 * sizeof(T);
    const int cus = device_cu_count();
    if (lds12 <= 160 * 1024) return fwd_raw_launch<T, W, PRESET, LAYOUT, 12>(d, ffr, raw, n, rgb, s, cus);
    return fwd_raw_launch<T, W, PRESET, LAYOUT, 8>(d, ffr, raw, n, rgb, s,
                                                   cus * (int)((160 * 1024) / lds8 > 0 ? (160 * 1024) / lds8 : 1));
}

template <typename T, int W>
hipError_t fwd_raw_dispatch(const Geo& d, int preset, int layout, const void* ffr, const float* raw,
                            int64_t n, float* rgb, hipStream_t s) {
    if (W == 64 && d.H == 5) {
        if (preset == NRC_PRESET_PAPER_GAUSS)
            return layout == NRC_RAW14 ? fwd_raw_fixed_launch<T, NRC_PRESET_PAPER_GAUSS, NRC_RAW14>(d, ffr, raw, n, rgb, s)
                                       : fwd_raw_fixed_launch<T, NRC_PRESET_PAPER_GAUSS, NRC_RAW16>(d, ffr, raw, n, rgb, s);
        if (preset == NRC_PRESET_PAPER_TRI)
            return layout == NRC_RAW14 ? fwd_raw_fixed_launch<T, NRC_PRESET_PAPER_TRI, NRC_RAW14>(d, ffr, raw, n, rgb, s)
                                       : fwd_raw_fixed_launch<T, NRC_PRESET_PAPER_TRI, NRC_RAW16>(d, ffr, raw, n, rgb, s);
        if (preset == NRC_PRESET_PAPER)
            return layout == NRC_RAW14 ? fwd_raw_fixed_launch<T, NRC_PRESET_PAPER, NRC_RAW14>(d, ffr, raw, n, rgb, s)
                                       : fwd_raw_fixed_launch<T, NRC_PRESET_PAPER, NRC_RAW16>(d, ffr, raw, n, rgb, s);
        return layout == NRC_RAW14 ? fwd_raw_fixed_launch<T, NRC_PRESET_CONFIG, NRC_RAW14>(d, ffr, raw, n, rgb, s)
                                   : fwd_raw_fixed_launch<T, NRC_PRESET_CONFIG, NRC_RAW16>(d, ffr, raw, n, rgb, s);
    }
    if (preset == NRC_PRESET_PAPER_GAUSS)
        return layout == NRC_RAW14 ? fwd_raw_generic<T, W, NRC_PRESET_PAPER_GAUSS, NRC_RAW14>(d, ffr, raw, n, rgb, s)
                                   : fwd_raw_generic<T, W, NRC_PRESET_PAPER_GAUSS, NRC_RAW16>(d, ffr, raw, n, rgb, s);
    if (preset == NRC_PRESET_PAPER_TRI)
        return layout == NRC_RAW14 ? fwd_raw_generic<T, W, NRC_PRESET_PAPER_TRI, NRC_RAW14>(d, ffr, raw, n, rgb, s)
                                   : fwd_raw_generic<T, W, NRC_PRESET_PAPER_TRI, NRC_RAW16>(d, ffr, raw, n, rgb, s);
    if (preset == NRC_PRESET_PAPER)
        return layout == NRC_RAW14 ? fwd_raw_generic<T, W, NRC_PRESET_PAPER, NRC_RAW14>(d, ffr, raw, n, rgb, s)
                                   : fwd_raw_generic<T, W, NRC_PRESET_PAPER, NRC_RAW16>(d, ffr, raw, n, rgb, s);
    return layout == NRC_RAW14 ? fwd_raw_generic<T, W, NRC_PRESET_CONFIG, NRC_RAW14>(d, ffr, raw, n, rgb, s)
                               : fwd_raw_generic<T, W, NRC_PRESET_CONFIG, NRC_RAW16>(d, ffr, raw, n, rgb, s);
}

template <typename T, int W, bool UP, bool GE, int ACT = kActNone, int RAWL = -1, int PRESET = NRC_PRESET_CONFIG>
hipError_t train_launch(const Geo& d, const void* ffr, const void* bfr, const void* enc,
                        const float* tgt, const int32_t* idx, int64_t n, float loss_eps, float grad_scale,
                        float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                        hipStream_t s, void* act = nullptr, float* rgb = nullptr, LcgGather lg = LcgGather{}) {
    using S = TrainShape<W>;
    const int64_t tiles = (n + S::TS - 1) / S::TS;
    if (tiles == 0) return hipSuccess;
    const size_t lds = (size_t)train_lds_bytes(W, d.H);
    auto k = k_train_mfma<T, W, UP, GE, ACT, RAWL, PRESET>;
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(64 * (S::NW + train_helpers<W, ACT>())), lds, s, (const T*)ffr, (const T*)bfr,
                       (const T*)enc, tgt, idx, n, d.H, loss_eps, grad_scale, partials, loss_part, tile_bad,
                       genc, d.F, (T*)act, rgb, lg);
    return hipGetLastError();
}

template <typename T, int W>
hipError_t train_dispatch(const Geo& d, const void* ffr, const void* bfr, const void* enc,
                          const float* tgt, const int32_t* idx, int64_t n, bool upstream, float loss_eps,
                          float grad_scale, float* partials, float* loss_part, int32_t* tile_bad,
                          float* genc, hipStream_t s, const void* act, LcgGather lg) {
    if (!upstream)
        return train_launch<T, W, false, false>(d, ffr, bfr, enc, tgt, idx, n, loss_eps, grad_scale,
                                                partials, loss_part, tile_bad, genc, s, nullptr, nullptr, lg);
    if (act) {
        if (genc)
            return train_launch<T, W, true, true, kActLoad>(d, ffr, bfr, enc, tgt, idx, n, loss_eps, grad_scale,
                                                            partials, loss_part, tile_bad, genc, s, (void*)act);
        return train_launch<T, W, true, false, kActLoad>(d, ffr, bfr, enc, tgt, idx, n, loss_eps, grad_scale,
                                                         partials, loss_part, tile_bad, genc, s, (void*)act);
    }
    if (genc)
        return train_launch<T, W, true, true>(d, ffr, bfr, enc, tgt, idx, n, loss_eps, grad_scale,
                                              partials, loss_part, tile_bad, genc, s);
    return train_launch<T, W, true, false>(d, ffr, bfr, enc, tgt, idx, n, loss_eps, grad_scale,
                                           partials, loss_part, tile_bad, genc, s);
}

// The training step on raw records (width 64, as the fused query path).
template <typename T>
hipError_t train_raw_dispatch(const Geo& d, int preset, int layout, const void* ffr, const void* bfr,
                              const float* raw, const float* tgt, const int32_t* idx, int64_t n, float loss_eps,
                              float grad_scale, float* partials, float* loss_part, int32_t* tile_bad,
                              hipStream_t s, LcgGather lg) {
#define NRC_TRAIN_RAW(PR, LA)                                                                                 \
    return train_launch<T, 64, false, false, kActNone, LA, PR>(d, ffr, bfr, raw, tgt, idx, n, loss_eps,      \
                                                               grad_scale, partials, loss_part, tile_bad,     \
                                                               nullptr, s, nullptr, nullptr, lg)
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

}  // namespace

int device_cu_count() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = -1;
    if (dev >= 0) {
        const int c = cache[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev < 0 ? 0 : dev) != hipSuccess || cus <= 0)
        cus = 256;   // MI355X
    if (dev >= 0) cache[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

size_t mfma_train_lds_bytes(int width, int n_hidden) {
    return (size_t)train_lds_bytes(width, n_hidden) + 16;
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

hipError_t launch_fwd_mfma_segs(int precision, const Geo& d, const void* ffr, const SegList& segs,
                                hipStream_t s) {
    if (segs.count < 1 || segs.count > kMaxSegs) return hipErrorInvalidValue;
    if (precision == NRC_FP16)
        return d.W == 64 ? fwd_segs_dispatch<_Float16, 64>(d, ffr, segs, s)
                         : fwd_segs_dispatch<_Float16, 128>(d, ffr, segs, s);
    return d.W == 64 ? fwd_segs_dispatch<__bf16, 64>(d, ffr, segs, s)
                     : fwd_segs_dispatch<__bf16, 128>(d, ffr, segs, s);
}

// Width 64 only: the fused kernel keeps the weights and four 64-record encode
// buffers in LDS side by side.
hipError_t launch_fwd_raw_mfma(int precision, const Geo& d, int preset, int layout, const void* ffr,
                               const float* raw, int64_t n, float* rgb, hipStream_t s) {
    if (precision == NRC_FP16) return fwd_raw_dispatch<_Float16, 64>(d, preset, layout, ffr, raw, n, rgb, s);
    return fwd_raw_dispatch<__bf16, 64>(d, preset, layout, ffr, raw, n, rgb, s);
}

hipError_t launch_train_mfma(int precision, const Geo& d, const void* ffr, const void* bfr,
                             const void* enc, const float* tgt, const int32_t* idx, int64_t n, bool upstream,
                             float loss_eps, float grad_scale, float* partials, float* loss_part,
                             int32_t* tile_bad, float* genc, hipStream_t s, const void* act, LcgGather lg) {
    if (precision == NRC_FP16)
        return d.W == 64 ? train_dispatch<_Float16, 64>(d, ffr, bfr, enc, tgt, idx, n, upstream, loss_eps,
                                                        grad_scale, partials, loss_part, tile_bad, genc, s, act, lg)
                         : train_dispatch<_Float16, 128>(d, ffr, bfr, enc, tgt, idx, n, upstream, loss_eps,
                                                         grad_scale, partials, loss_part, tile_bad, genc, s, act,
                                                         lg);
    return d.W == 64 ? train_dispatch<__bf16, 64>(d, ffr, bfr, enc, tgt, idx, n, upstream, loss_eps,
                                                  grad_scale, partials, loss_part, tile_bad, genc, s, act, lg)
                     : train_dispatch<__bf16, 128>(d, ffr, bfr, enc, tgt, idx, n, upstream, loss_eps,
                                                   grad_scale, partials, loss_part, tile_bad, genc, s, act, lg);
}

hipError_t launch_train_mfma_raw(int precision, const Geo& d, int preset, int layout, const void* ffr,
                                 const void* bfr, const float* raw, const float* tgt, const int32_t* idx,
                                 int64_t n, float loss_eps, float grad_scale, float* partials, float* loss_part,
                                 int32_t* tile_bad, hipStream_t s, LcgGather lg) {
    if (d.W != 64) return hipErrorInvalidValue;
    if (precision == NRC_FP16)
        return train_raw_dispatch<_Float16>(d, preset, layout, ffr, bfr, raw, tgt, idx, n, loss_eps, grad_scale,
                                            partials, loss_part, tile_bad, s, lg);
    return train_raw_dispatch<__bf16>(d, preset, layout, ffr, bfr, raw, tgt, idx, n, loss_eps, grad_scale,
                                      partials, loss_part, tile_bad, s, lg);
}

template <typename T, int W>
hipError_t fwd_train_dispatch(const Geo& d, const void* ffr, const void* enc, int64_t n, void* act, float* rgb,
                              hipStream_t s) {
    return train_launch<T, W, true, false, kActStore>(d, ffr, nullptr, enc, nullptr, nullptr, n, 0.0f, 1.0f,
                                                      nullptr, nullptr, nullptr, nullptr, s, act, rgb);
}

hipError_t launch_fwd_train_mfma(int precision, const Geo& d, const void* ffr, const void* enc, int64_t n,
                                 void* act, float* rgb, hipStream_t s) {
    if (precision == NRC_FP16)
        return d.W == 64 ? fwd_train_dispatch<_Float16, 64>(d, ffr, enc, n, act, rgb, s)
                         : fwd_train_dispatch<_Float16, 128>(d, ffr, enc, n, act, rgb, s);
    return d.W == 64 ? fwd_train_dispatch<__bf16, 64>(d, ffr, enc, n, act, rgb, s)
                     : fwd_train_dispatch<__bf16, 128>(d, ffr, enc, n, act, rgb, s);
}

}  // namespace nrc
