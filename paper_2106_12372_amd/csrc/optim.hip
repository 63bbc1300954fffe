// Weight-gradient reduction and the Adam update (Sec. 5 "Optimizer").
//
// k_reduce<ADAM>: a workgroup owns 32 consecutive weights; its 8 groups of 32
// lanes each sum every 8th tile's partial for one weight (coalesced 128-byte
// rows), with Neumaier compensation, and the 8 group sums are combined in a
// fixed order, so the reduced gradient does not depend on scheduling.
// Without ADAM the gradient is written out (backward of the autograd form).
// With ADAM the workgroup first ORs the per-tile non-finite flags the training
// kernel wrote: if any is set the whole step is skipped (weights, moments and
// step count stay as they are); otherwise each weight's FP32 master copy and
// Adam moments are updated and its FP16/BF16 copies in both matrix-core
// fragment layouts are refreshed.  The step count lives in two device slots
// used in alternation (read one, write the other), so no thread of the launch
// reads a value another thread of the same launch writes.  Workgroup 0 also
// reduces the per-tile loss partials.
#include "nrc_internal.h"

namespace nrc {
namespace {

constexpr int kRedBlock = 256;

__device__ inline void neumaier_add(float& s, float& c, float x) {
    const float t = s + x;
    if (fabsf(s) >= fabsf(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
}

// Layer holding flat index p (weights and partial slots share the ranges).
__device__ inline int layer_of(const Geo& d, int p) {
    if (p < d.w_off(1)) return 0;
    if (p >= d.w_off(d.H)) return d.H;
    return 1 + (p - d.w_off(1)) / (d.W * d.W);
}

// Weight index held by partial slot s in the matrix-core accumulator layout:
// slot w_off(l) + ((mb * NB + nb) * 64 + lane) * 4 + j holds
// dW_l[16 mb + 4 (lane / 16) + j][16 nb + lane % 16]; the output layer is
// row-major.
__device__ inline int param_of_slot(const Geo& d, int s) {
    const int l = layer_of(d, s);
    if (l == d.H) return s;
    const int r = s - d.w_off(l);
    const int cols = d.cols(l), NB = cols >> 4;
    const int j = r & 3, lane = (r >> 2) & 63, blk = r >> 8;
    const int mb = blk / NB, nb = blk - mb * NB;
    return d.w_off(l) + (16 * mb + 4 * (lane >> 4) + j) * cols + 16 * nb + (lane & 15);
}

// Locate weight p (flat index) as (layer, row, column).
__device__ inline void locate(const Geo& d, int p, int& l, int& o, int& k) {
    l = layer_of(d, p);
    const int r = p - d.w_off(l);
    const int cols = d.cols(l);
    o = r / cols;
    k = r - o * cols;
}

// Forward and backward fragment slots of weight p.
__device__ inline void frag_slots(const Geo& d, int p, int64_t& fi, int64_t& bi) {
    int l, o, k;
    locate(d, p, l, o, k);
    fi = fwd_frag_index(d, l, o, k);
    bi = bwd_frag_index(d, l, o, k);
}

// A weight into its forward and backward fragment slots fi, bi.  split: also
// the lo part w - hi into the second copy that follows each array (the BF16
// form's training fragments).
template <typename T>
__device__ inline void put_frags(const Geo& d, int64_t fi, int64_t bi, float w, T* ffr, T* bfr, bool split) {
    const T v = (T)w;
    if (ffr) ffr[fi] = v;
    if (bfr) bfr[bi] = v;
    if (split) {
        const T lo = (T)(w - (float)v);
        if (ffr) ffr[(int64_t)d.n_fwd_frags() * kFragElems + fi] = lo;
        if (bfr) bfr[(int64_t)d.n_bwd_frags() * kFragElems + bi] = lo;
    }
}

template <typename T>
__device__ inline void write_frags(const Geo& d, int p, float w, T* ffr, T* bfr, bool split = false) {
    int64_t fi, bi;
    frag_slots(d, p, fi, bi);
    put_frags<T>(d, fi, bi, w, ffr, bfr, split);
}

constexpr int kRedParams = 32;   // weights per workgroup
constexpr int kRedGroups = 8;    // tile groups per workgroup

template <typename T, bool ADAM, bool NATIVE>
__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ partials, int n_tiles,
                                                const int32_t* __restrict__ tile_bad,
                                                const float* __restrict__ loss_part, float inv_count,
                                                float* __restrict__ loss_out, float inv_scale,
                                                float* __restrict__ grad_out, float* __restrict__ w,
                                                float* __restrict__ m, float* __restrict__ v,
                                                int32_t* __restrict__ tslots, int parity, AdamHyper hp,
                                                EmaArgs ema, int32_t* __restrict__ skipped_out,
                                                T* __restrict__ ffr, T* __restrict__ bfr, int width,
                                                int n_hidden) {
    __shared__ float s_sum[kRedGroups][kRedParams];
    __shared__ float s_cmp[kRedGroups][kRedParams];
    __shared__ int s_skip;
    const Geo d(width, n_hidden);
    const int P = d.n_params();
    const int tid = threadIdx.x, lane = tid & 63;
    const int pl = tid % kRedParams, grp = tid / kRedParams;
    const int sidx = blockIdx.x * kRedParams + pl;          // partial slot (coalesced across lanes)

    // Wave 0 ORs the per-tile non-finite flags; the first 256 are loaded now
    // and combined after the sums, so no load waits on another.
    int bad4[4] = {0, 0, 0, 0};
    if (ADAM && tid < 64) {
        #pragma unroll
        for (int u = 0; u < 4; ++u)
            if (tid + 64 * u < n_tiles) bad4[u] = tile_bad[tid + 64 * u];
    }
    // The update's operands for this thread's weight are loaded before the
    // partials, so their latency overlaps the sums.
    const bool owner = grp == 0 && sidx < P;
    const int p = NATIVE ? param_of_slot(d, owner ? sidx : 0) : sidx;
    float w0 = 0.0f, m0 = 0.0f, v0 = 0.0f, e0 = 0.0f;
    int t_old = 0;
    if (ADAM && owner) {
        w0 = w[p];
        m0 = m[p];
        v0 = v[p];
        if (ema.alpha > 0.0f) e0 = ema.e[p];
        t_old = tslots[parity];
    }
    // Workgroup 0's second wave loads the first 256 per-tile loss terms now,
    // for the same reason.
    const bool loss_wave = blockIdx.x == 0 && tid >= 64 && tid < 128 && loss_out != nullptr;
    float lv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (loss_wave) {
        #pragma unroll
        for (int u = 0; u < 4; ++u)
            if (lane + 64 * u < n_tiles) lv[u] = loss_part[lane + 64 * u];
    }
    // Bias corrections of the step this update would make (a skipped step
    // updates nothing) and the weight's fragment slots, evaluated while the
    // partials are in flight.
    const float t_next = (float)(t_old + 1);
    float bc1 = 1.0f, bc2 = 1.0f, bce = 1.0f;
    int64_t fi = 0, bi = 0;
    if (ADAM && owner) {
        bc1 = 1.0f - powf(hp.beta1, t_next);
        bc2 = 1.0f - powf(hp.beta2, t_next);
        if (ema.alpha > 0.0f) bce = 1.0f - powf(ema.alpha, t_next);
        if (ffr != nullptr || ema.effr != nullptr) frag_slots(d, p, fi, bi);
    }
    float s = 0.0f, c = 0.0f;
    if (sidx < P) {
        // 32 (then 16) loads in flight per thread before the (order-preserving) sums
        int t = grp;
        for (; t + 31 * kRedGroups < n_tiles; t += 32 * kRedGroups) {
            float x[32];
            #pragma unroll
            for (int u = 0; u < 32; ++u)
                x[u] = __builtin_nontemporal_load(&partials[(int64_t)(t + u * kRedGroups) * P + sidx]);
            #pragma unroll
            for (int u = 0; u < 32; ++u) neumaier_add(s, c, x[u]);
        }
        for (; t + 15 * kRedGroups < n_tiles; t += 16 * kRedGroups) {
            float x[16];
            #pragma unroll
            for (int u = 0; u < 16; ++u)
                x[u] = __builtin_nontemporal_load(&partials[(int64_t)(t + u * kRedGroups) * P + sidx]);
            #pragma unroll
            for (int u = 0; u < 16; ++u) neumaier_add(s, c, x[u]);
        }
        for (; t < n_tiles; t += kRedGroups)
            neumaier_add(s, c, __builtin_nontemporal_load(&partials[(int64_t)t * P + sidx]));
    }
    if (ADAM && tid < 64) {
        int any = bad4[0] | bad4[1] | bad4[2] | bad4[3];
        for (int t = tid + 256; t < n_tiles; t += 64) any |= tile_bad[t];
        #pragma unroll
        for (int off = 32; off >= 1; off >>= 1) any |= __shfl_xor(any, off, 64);
        if (tid == 0) s_skip = any;
    }
    s_sum[grp][pl] = s;
    s_cmp[grp][pl] = c;
    __syncthreads();

    if (loss_wave) {
        // compensated sum of the per-tile loss terms, then a compensated
        // combine of the 64 lane sums in a fixed order
        float ls = 0.0f, lc = 0.0f;
        #pragma unroll
        for (int u = 0; u < 4; ++u)
            if (lane + 64 * u < n_tiles) neumaier_add(ls, lc, lv[u]);
        for (int t = lane + 256; t < n_tiles; t += 64) neumaier_add(ls, lc, loss_part[t]);
        #pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float os = __shfl_xor(ls, off, 64), oc = __shfl_xor(lc, off, 64);
            // both partners form the same pair sum (the lower lane's operand first)
            const bool lo = (lane & off) == 0;
            float a = lo ? ls : os, ac = lo ? lc : oc;
            neumaier_add(a, ac, lo ? os : ls);
            ac += lo ? oc : lc;
            ls = a;
            lc = ac;
        }
        if (lane == 0) *loss_out = (ls + lc) * inv_count;
    }
    if (!owner) return;   // workgroup 0's thread 0 has slot 0 and stays
    float gv = 0.0f;
    {
        float S = 0.0f, C = 0.0f;
        #pragma unroll
        for (int k = 0; k < kRedGroups; ++k) {
            neumaier_add(S, C, s_sum[k][pl]);
            C += s_cmp[k][pl];
        }
        gv = (S + C) * inv_scale;
    }
    if (!ADAM) {
        grad_out[p] = gv;
        return;
    }
    const int skip = s_skip;
    const int t_new = skip ? t_old : t_old + 1;
    if (blockIdx.x == 0 && tid == 0) {
        tslots[parity ^ 1] = t_new;
        if (skipped_out) *skipped_out = skip;
    }
    if (skip) return;
    // explicit fused multiply-adds: the rounding does not depend on which
    // product the compiler would contract
    const float m1 = fmaf(hp.beta1, m0, (1.0f - hp.beta1) * gv);
    const float v1 = fmaf(hp.beta2, v0, ((1.0f - hp.beta2) * gv) * gv);
    const float w1 = w0 - hp.lr * (m1 / bc1) / (sqrtf(v1 / bc2) + hp.eps);
    w[p] = w1;
    m[p] = m1;
    v[p] = v1;
    if (ffr != nullptr) put_frags<T>(d, fi, bi, w1, ffr, bfr, __is_same(T, __bf16));
    if (ema.alpha > 0.0f) {
        // Eq. 2, bias-corrected: E_t = a E_{t-1} + (1 - a) W_t, W_bar_t = E_t / (1 - a^t).
        const float e1 = fmaf(ema.alpha, e0, (1.0f - ema.alpha) * w1);
        const float wb = e1 / bce;
        ema.e[p] = e1;
        ema.wbar[p] = wb;
        if (ema.effr != nullptr) put_frags<T>(d, fi, bi, wb, (T*)ema.effr, (T*)nullptr, false);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_build_frags(const float* __restrict__ w, T* __restrict__ ffr,
                                                     T* __restrict__ bfr, T* __restrict__ ffr2,
                                                     int width, int n_hidden) {
    const Geo d(width, n_hidden);
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= d.n_params()) return;
    write_frags<T>(d, p, w[p], ffr, bfr, __is_same(T, __bf16) && bfr != nullptr);
    if (ffr2) write_frags<T>(d, p, w[p], ffr2, (T*)nullptr);
}

}  // namespace

int reduce_blocks(int n_params) { return (n_params + kRedParams - 1) / kRedParams; }

hipError_t launch_reduce(const Geo& d, bool native, const float* partials, int n_tiles,
                         float inv_scale, float* grad, const float* loss_part, float inv_count,
                         float* loss_out, hipStream_t s) {
    const dim3 grid(reduce_blocks(d.n_params())), block(256);
    auto k = native ? k_reduce<_Float16, false, true> : k_reduce<_Float16, false, false>;
    hipLaunchKernelGGL(k, grid, block, 0, s, partials, n_tiles, (const int32_t*)nullptr, loss_part,
                       inv_count, loss_out, inv_scale, grad, (float*)nullptr, (float*)nullptr,
                       (float*)nullptr, (int32_t*)nullptr, 0, AdamHyper{}, EmaArgs{},
                       (int32_t*)nullptr, (_Float16*)nullptr, (_Float16*)nullptr, d.W, d.H);
    return hipGetLastError();
}

hipError_t launch_reduce_adam(int precision, const Geo& d, bool native, const float* partials,
                              int n_tiles, const int32_t* tile_bad, const float* loss_part,
                              float inv_count, float* loss_out, float inv_scale, float* w, float* m,
                              float* v, int32_t* tslots, int parity, AdamHyper hp, EmaArgs ema,
                              int32_t* skipped_out, void* ffr, void* bfr, hipStream_t s) {
    const dim3 grid(reduce_blocks(d.n_params())), block(256);
    if (precision == NRC_BF16) {
        auto k = native ? k_reduce<__bf16, true, true> : k_reduce<__bf16, true, false>;
        hipLaunchKernelGGL(k, grid, block, 0, s, partials, n_tiles, tile_bad, loss_part, inv_count,
                           loss_out, inv_scale, (float*)nullptr, w, m, v, tslots, parity, hp, ema,
                           skipped_out, (__bf16*)ffr, (__bf16*)bfr, d.W, d.H);
    } else {
        // FP32 caches have no reduced-precision copies (ffr, bfr, ema.effr are NULL).
        auto k = native ? k_reduce<_Float16, true, true> : k_reduce<_Float16, true, false>;
        hipLaunchKernelGGL(k, grid, block, 0, s, partials, n_tiles, tile_bad, loss_part, inv_count,
                           loss_out, inv_scale, (float*)nullptr, w, m, v, tslots, parity, hp, ema,
                           skipped_out, (_Float16*)ffr, (_Float16*)bfr, d.W, d.H);
    }
    return hipGetLastError();
}

hipError_t launch_build_frags(int precision, const Geo& d, const float* w, void* ffr, void* bfr,
                              void* ffr2, hipStream_t s) {
    const dim3 grid((d.n_params() + 255) / 256), block(256);
    if (precision == NRC_FP16)
        hipLaunchKernelGGL(k_build_frags<_Float16>, grid, block, 0, s, w, (_Float16*)ffr,
                           (_Float16*)bfr, (_Float16*)ffr2, d.W, d.H);
    else if (precision == NRC_BF16)
        hipLaunchKernelGGL(k_build_frags<__bf16>, grid, block, 0, s, w, (__bf16*)ffr, (__bf16*)bfr,
                           (__bf16*)ffr2, d.W, d.H);
    return hipGetLastError();
}

}  // namespace nrc
