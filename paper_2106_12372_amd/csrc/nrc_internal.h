// Internal declarations of the MI355X radiance-cache library: network
// dimensions, weight-fragment layout for the gfx950 matrix cores, and the host
// launch wrappers each kernel source file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/nrc.h"

namespace nrc {

constexpr int kMaxLayers = 9;   // up to 8 hidden layers + output
constexpr int kEncWidth = 64;   // encoded input width (Sec. 3.6)
constexpr int kNOut = 3;        // RGB
// First column of the diffuse albedo in the encoded row; the specular albedo
// follows it (Sec. 3.6 concatenation order): after the roughness at 52 in the
// config preset, after the roughness one-blob at 52..55 in the paper presets.
constexpr int kAlbedoColConfig = 53;
constexpr int kAlbedoColPaper = 56;
__host__ __device__ inline int albedo_col(int preset) {
    return preset == NRC_PRESET_CONFIG ? kAlbedoColConfig : kAlbedoColPaper;
}
// The two FP32 forms (matrix cores, vector ALUs): FP32 encoded input, no
// reduced-precision weight copies, row-major weight-gradient partials.
__host__ __device__ inline bool fp32_form(int precision) {
    return precision == NRC_FP32 || precision == NRC_FP32_VALU;
}
// Training records per workgroup tile: 64, except 32 for the width-128
// matrix-core form (its activations and deltas must fit in LDS).
__host__ __device__ inline int train_tile(int precision, int width) {
    return (!fp32_form(precision) && width == 128) ? 32 : 64;
}

// One matrix-core operand fragment: 64 lanes x 8 16-bit elements.
constexpr int kFragElems = 64 * 8;
// Copies of the training weight fragments: the BF16 form keeps each weight as
// a pair hi = bf16(w), lo = bf16(w - hi) (the lo set follows the hi set in the
// same array), and its training products take both, so training sees the
// weights to about 16 significant bits while its operands stay BF16; queries
// use the hi set.  FP16 keeps one copy.
__host__ __device__ inline int train_frag_copies(int precision) { return precision == NRC_BF16 ? 2 : 1; }

// Shapes and offsets of the network (Sec. 5 "Architecture"), computed
// arithmetically so that kernels never index an array by a runtime layer.
//   Layer l maps h_l (cols(l) features) to z_{l+1} (rows(l) features):
//   l = 0: [W][64]; l = 1..H-1: [W][W]; l = H (output): [3][W].
// Weights are one flat FP32 array, layer after layer, each row-major [out][in].
// Forward fragments of layer l: A operand of z = W_l h (M = rows, K = cols),
//   fwd_mb(l) blocks of 16 rows x fwd_kc(l) chunks of 32 columns.
// Backward fragments of layer l: A operand of g = W_l^T delta (M = cols,
//   K = rows), bwd_mb(l) x bwd_kc(l).
//   F: reflectance factorisation (Sec. 5): 0 = off, otherwise the albedo
//   column (kAlbedoColConfig or kAlbedoColPaper); the prediction is the network
//   output times enc[F + c] + enc[F + 3 + c] per channel c.
struct Geo {
    int W, H, F = 0;
    __host__ __device__ Geo(int width, int n_hidden) : W(width), H(n_hidden) {}
    __host__ __device__ int MB() const { return W >> 4; }
    __host__ __device__ int KC() const { return W >> 5; }
    __host__ __device__ int rows(int l) const { return l == H ? kNOut : W; }
    __host__ __device__ int cols(int l) const { return l == 0 ? kEncWidth : W; }
    __host__ __device__ int w_off(int l) const { return l == 0 ? 0 : kEncWidth * W + (l - 1) * W * W; }
    __host__ __device__ int n_params() const { return w_off(H) + kNOut * W; }
    __host__ __device__ int fwd_kc(int l) const { return l == 0 ? 2 : KC(); }
    __host__ __device__ int fwd_mb(int l) const { return l == H ? 1 : MB(); }
    __host__ __device__ int fwd_base(int l) const { return l == 0 ? 0 : 2 * MB() + (l - 1) * MB() * KC(); }
    __host__ __device__ int n_fwd_frags() const { return fwd_base(H) + KC(); }
    __host__ __device__ int bwd_kc(int l) const { return l == H ? 1 : KC(); }
    __host__ __device__ int bwd_mb(int l) const { return l == 0 ? 4 : MB(); }
    __host__ __device__ int bwd_base(int l) const { return l == 0 ? 0 : 4 * KC() + (l - 1) * MB() * KC(); }
    __host__ __device__ int n_bwd_frags() const { return bwd_base(H) + MB(); }
};

// ---------------------------------------------------------------------------
// Feature <-> operand-slot maps of v_mfma_f32_16x16x32_{f16,bf16}.
//
// B operand (K x N = 32 x 16): lane l holds column n = l % 16 and the eight
// K rows 8*(l/16) .. 8*(l/16)+7.  The accumulator (M x N = 16 x 16): lane l
// holds column n = l % 16 and rows 4*(l/16) .. 4*(l/16)+3.  A layer's two
// adjacent 16-row accumulator blocks therefore hand each lane features
// {4g..4g+3} and {16+4g..16+4g+3} (g = l/16) of one 32-feature chunk, which
// become that lane's eight B slots of the next product directly if the next
// weight matrix's K index is permuted the same way ("chained" order).  Inputs
// read from memory use the natural order 8g..8g+7.
// ---------------------------------------------------------------------------
__host__ __device__ inline int chained_feature(int c, int g, int i) {
    return 32 * c + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
}
__host__ __device__ inline int natural_feature(int c, int g, int i) { return 32 * c + 8 * g + i; }
__host__ __device__ inline void chained_slot(int k, int& c, int& g, int& i) {
    c = k >> 5;
    const int r = k & 31;
    if (r < 16) { g = r >> 2; i = r & 3; } else { g = (r - 16) >> 2; i = 4 + ((r - 16) & 3); }
}
__host__ __device__ inline void natural_slot(int k, int& c, int& g, int& i) {
    c = k >> 5;
    const int r = k & 31;
    g = r >> 3;
    i = r & 7;
}

// Position of weight W_l[o][k] in the forward fragment array (element index),
// and of the same weight in the backward (transposed) fragment array.
__host__ __device__ inline int64_t fwd_frag_index(const Geo& d, int l, int o, int k) {
    int c, g, i;
    if (l == 0) natural_slot(k, c, g, i); else chained_slot(k, c, g, i);
    const int mb = o >> 4, lane = 16 * g + (o & 15);
    return ((int64_t)(d.fwd_base(l) + mb * d.fwd_kc(l) + c) * 64 + lane) * 8 + i;
}
__host__ __device__ inline int64_t bwd_frag_index(const Geo& d, int l, int o, int k) {
    int c, g, i;
    chained_slot(o, c, g, i);  // K index of the transposed product is the row o
    const int mb = k >> 4, lane = 16 * g + (k & 15);
    return ((int64_t)(d.bwd_base(l) + mb * d.bwd_kc(l) + c) * 64 + lane) * 8 + i;
}

// alpha + beta per channel from an encoded row held in registers (one lane per
// record); fcol is 0 (no factorisation, factor 1), kAlbedoColConfig or
// kAlbedoColPaper.  The selects keep every register index compile-time.
__device__ inline void reflectance_row(const float (&h)[kEncWidth], int fcol, float (&r)[kNOut]) {
    #pragma unroll
    for (int c = 0; c < kNOut; ++c)
        r[c] = fcol == kAlbedoColPaper    ? h[kAlbedoColPaper + c] + h[kAlbedoColPaper + 3 + c]
               : fcol == kAlbedoColConfig ? h[kAlbedoColConfig + c] + h[kAlbedoColConfig + 3 + c]
                                          : 1.0f;
}

// ReLU as the IEEE maximum of x and +0: one v_maximum3_f32 on gfx950, where
// fmaxf's rule for NaN operands first needs a canonicalising max.  A NaN
// propagates instead of becoming 0; -0 becomes +0.
__device__ inline float relu(float x) { return __builtin_elementwise_maximum(x, 0.0f); }

// Neumaier-compensated sum of one float per lane over the 64 lanes of a wave,
// in a fixed butterfly order; every lane ends with the same value.  Each pair
// sum is formed with the lower lane's operand first and carries both lanes'
// compensation terms, so the two partners of a pair compute identical bits.
__device__ inline float wave_sum_compensated(float v) {
    const int lane = __lane_id();
    float s = v, c = 0.0f;
    #pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float os = __shfl_xor(s, off, 64), oc = __shfl_xor(c, off, 64);
        const bool lo = (lane & off) == 0;
        const float a = lo ? s : os, b = lo ? os : s;
        const float t = a + b;
        const float e = fabsf(a) >= fabsf(b) ? (a - t) + b : (b - t) + a;
        c = ((lo ? c : oc) + (lo ? oc : c)) + e;
        s = t;
    }
    return s + c;
}

// Request segments of one multi-segment inference launch (serving): segment
// k has n[k] > 0 encoded rows at enc[k] and writes rgb[k]; tile_end[k] is the
// cumulative count of 64-record tiles through segment k.
constexpr int kMaxSegs = 16;
struct SegList {
    int count;
    int64_t tile_end[kMaxSegs];
    const void* enc[kMaxSegs];
    float* rgb[kMaxSegs];
    int64_t n[kMaxSegs];
};

// The record shuffle's LCG as affine maps x -> a x + c (mod 2^32): their
// composition, powers (jump-ahead by repeated squaring) and application.
struct Affine {
    uint32_t a, c;
};
// g after f.
__host__ __device__ inline Affine compose(Affine f, Affine g) { return {g.a * f.a, g.a * f.c + g.c}; }
// f applied j times.
__host__ __device__ inline Affine power(Affine f, uint64_t j) {
    Affine r{1u, 0u};
    while (j) {
        if (j & 1) r = compose(r, f);
        f = compose(f, f);
        j >>= 1;
    }
    return r;
}
__host__ __device__ inline uint32_t apply(Affine f, uint32_t x) { return f.a * x + f.c; }

// A training batch read straight from the LCG orbit: batch slot r is record
// (step^r (x0)) & mask.  Used by a frame over a power-of-two record count,
// where the orbit skips no value, so no permutation is stored.  mask == 0:
// not used.
struct LcgGather {
    Affine step;
    uint32_t x0, mask;
};

// Record read by batch slot r: idx[r] for an index list, the LCG orbit, or r.
__device__ inline int64_t gather_row(const int32_t* idx, const LcgGather& lg, int64_t r) {
    if (idx) return idx[r];
    if (lg.mask) return (int64_t)(apply(power(lg.step, (uint64_t)r), lg.x0) & lg.mask);
    return r;
}

struct AdamHyper {
    float lr, beta1, beta2, eps;
};

// EMA weight set (Eq. 2): alpha = 0 disables it.  e: running sum E,
// wbar: bias-corrected W_bar (FP32), effr: W_bar's forward fragments.
struct EmaArgs {
    float alpha;
    float* e;
    float* wbar;
    void* effr;
};

// ---------------------------------------------------------------------------
// Host launch wrappers (return hipError_t of the launch).
// ---------------------------------------------------------------------------
// encode.hip
// Compute units of the current device (cached per device): persistent grids
// are sized to what is resident at once, so no workgroup waits for a second
// round of dispatch.
int device_cu_count();

hipError_t launch_encode(int precision, int preset, int layout, const float* raw, int64_t n,
                         void* enc, hipStream_t s);
// mlp_fp32.hip
hipError_t launch_fwd_fp32(const Geo& d, const float* w, const float* enc, int64_t n, float* rgb,
                           hipStream_t s);
// idx (may be NULL): the batch is records idx[0..n) of enc / tgt.
hipError_t launch_train_fp32(const Geo& d, const float* w, const float* enc, const float* tgt,
                             const int32_t* idx, int64_t n, bool upstream, float loss_eps, float grad_scale,
                             float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                             hipStream_t s, const float* act = nullptr, LcgGather lg = LcgGather{});
hipError_t launch_fwd_train_fp32(const Geo& d, const float* w, const float* enc, int64_t n, float* act,
                                 float* rgb, hipStream_t s);
// The training steps of the three forms on raw records (layout, the cache's
// preset): each kernel encodes its records as the encoding kernel would, so the
// results equal encode-then-train bit for bit.  FP16/BF16: width 64 only.
hipError_t launch_train_fp32_raw(const Geo& d, int preset, int layout, const float* w, const float* raw,
                                 const float* tgt, const int32_t* idx, int64_t n, float loss_eps, float grad_scale,
                                 float* partials, float* loss_part, int32_t* tile_bad, hipStream_t s,
                                 LcgGather lg);
hipError_t launch_train_fp32_valu_raw(const Geo& d, int preset, int layout, const float* w, const float* raw,
                                      const float* tgt, const int32_t* idx, int64_t n, float loss_eps,
                                      float grad_scale, float* partials, float* loss_part, int32_t* tile_bad,
                                      hipStream_t s, LcgGather lg);
hipError_t launch_train_mfma_raw(int precision, const Geo& d, int preset, int layout, const void* ffr,
                                 const void* bfr, const float* raw, const float* tgt, const int32_t* idx,
                                 int64_t n, float loss_eps, float grad_scale, float* partials, float* loss_part,
                                 int32_t* tile_bad, hipStream_t s, LcgGather lg);
hipError_t launch_fwd_raw_fp32(const Geo& d, int preset, int layout, const float* w, const float* raw,
                               int64_t n, float* rgb, hipStream_t s);
// mlp_fp32_valu.hip (NRC_FP32_VALU: vector ALUs only)
hipError_t launch_fwd_fp32_valu(const Geo& d, const float* w, const float* enc, int64_t n, float* rgb,
                                hipStream_t s);
hipError_t launch_fwd_raw_fp32_valu(const Geo& d, int preset, int layout, const float* w, const float* raw,
                                    int64_t n, float* rgb, hipStream_t s);
hipError_t launch_train_fp32_valu(const Geo& d, const float* w, const float* enc, const float* tgt,
                                  const int32_t* idx, int64_t n, bool upstream, float loss_eps, float grad_scale,
                                  float* partials, float* loss_part, int32_t* tile_bad, float* genc,
                                  hipStream_t s, LcgGather lg = LcgGather{});
// mlp_mfma.hip
hipError_t launch_fwd_raw_mfma(int precision, const Geo& d, int preset, int layout, const void* ffr,
                               const float* raw, int64_t n, float* rgb, hipStream_t s);
hipError_t launch_fwd_mfma(int precision, const Geo& d, const void* ffr, const void* enc,
                           int64_t n, float* rgb, hipStream_t s);
hipError_t launch_fwd_mfma_segs(int precision, const Geo& d, const void* ffr, const SegList& segs,
                                hipStream_t s);
// act (may be NULL, upstream only): activation buffer written by
// launch_fwd_train_mfma; the forward pass is then read instead of recomputed.
hipError_t launch_train_mfma(int precision, const Geo& d, const void* ffr, const void* bfr,
                             const void* enc, const float* tgt, const int32_t* idx, int64_t n, bool upstream,
                             float loss_eps, float grad_scale, float* partials, float* loss_part,
                             int32_t* tile_bad, float* genc, hipStream_t s, const void* act = nullptr,
                             LcgGather lg = LcgGather{});
// Forward pass of the autograd form: rgb[n][3] and the activation buffer
// (act_bytes_mfma / act_bytes_fp32 bytes) for a later backward.
hipError_t launch_fwd_train_mfma(int precision, const Geo& d, const void* ffr, const void* enc, int64_t n,
                                 void* act, float* rgb, hipStream_t s);
size_t fp32_train_lds_bytes(int n_hidden);
size_t mfma_train_lds_bytes(int width, int n_hidden);
size_t mfma_fwd_lds_bytes(int width, int n_hidden);
// optim.hip
int reduce_blocks(int n_params);
// `native`: the partials use the matrix-core accumulator layout (see
// k_train_mfma) instead of row-major [out][in].
hipError_t launch_reduce(const Geo& d, bool native, const float* partials, int n_tiles,
                         float inv_scale, float* grad, const float* loss_part, float inv_count,
                         float* loss_out, hipStream_t s);
hipError_t launch_reduce_adam(int precision, const Geo& d, bool native, const float* partials, int n_tiles,
                              const int32_t* tile_bad, const float* loss_part, float inv_count,
                              float* loss_out, float inv_scale, float* w, float* m, float* v,
                              int32_t* tslots, int parity, AdamHyper hp, EmaArgs ema,
                              int32_t* skipped_out, void* ffr, void* bfr, hipStream_t s);
// shuffle.hip: the record shuffle's LCG, x -> (a x + c) mod 2^k, with
// Knuth's MMIX multiplier and increment reduced mod 2^32 (a = 5 mod 8, c odd:
// full period 2^k for every k <= 32).
constexpr uint32_t kLcgA = 1284865837u;
constexpr uint32_t kLcgC = 4150755663u;
void shuffle_shape(int64_t n, uint64_t& m, int& rounds, int& spans);
size_t shuffle_scratch_bytes();
// perm[0..n) = the orbit from seed mod m with values >= n skipped; counts is
// shuffle_scratch_bytes() of device scratch.
hipError_t launch_shuffle(int64_t n, uint64_t seed, int32_t* perm, int32_t* counts, hipStream_t s);
hipError_t launch_self_train(const float* radiance, const float* throughput, const float* tail_rgb,
                             const int32_t* tail_index, int64_t n, int64_t n_tail, float* target,
                             hipStream_t s);
// validate.hip: per-channel error norms in FP64 (out[3][4], see nrc.h).
size_t error_norms_scratch_bytes();
hipError_t launch_error_norms(const float* got, const double* ref, int64_t n, double* scratch, double* out,
                              hipStream_t s);
// Writes W's forward fragments to ffr and ffr2 (each may be NULL) and its
// backward fragments to bfr (may be NULL).
hipError_t launch_build_frags(int precision, const Geo& d, const float* w, void* ffr, void* bfr,
                              void* ffr2, hipStream_t s);

}  // namespace nrc
