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

// Locate weight p (flat index) as (layer, row, column).
__device__ inline void locate(const Geo& d, int p, int& l, int& o, int& k) {
    if (p < d.w_off(1)) {
        l = 0;
    } else if (p >= d.w_off(d.H)) {
        l = d.H;
    } else {
        l = 1 + (p - d.w_off(1)) / (d.W * d.W);
    }
    const int r = p - d.w_off(l);
    const int cols = d.cols(l);
    o = r / cols;
    k = r - o * cols;
}

template <typename T>
__device__ inline void write_frags(const Geo& d, int p, float w, T* ffr, T* bfr) {
    int l, o, k;
    locate(d, p, l, o, k);
    const T v = (T)w;
    ffr[fwd_frag_index(d, l, o, k)] = v;
    bfr[bwd_frag_index(d, l, o, k)] = v;
}

constexpr int kRedParams = 32;   // weights per workgroup
constexpr int kRedGroups = 8;    // tile groups per workgroup

template <typename T, bool ADAM>
__global__ __launch_bounds__(256) void k_reduce(const float* __restrict__ partials, int n_tiles,
                                                const int32_t* __restrict__ tile_bad,
                                                const float* __restrict__ loss_part, float inv_count,
                                                float* __restrict__ loss_out, float inv_scale,
                                                float* __restrict__ grad_out, float* __restrict__ w,
                                                float* __restrict__ m, float* __restrict__ v,
                                                int32_t* __restrict__ tslots, int parity, AdamHyper hp,
                                                int32_t* __restrict__ skipped_out, T* __restrict__ ffr,
                                                T* __restrict__ bfr, int width, int n_hidden) {
    __shared__ float s_sum[kRedGroups][kRedParams];
    __shared__ float s_cmp[kRedGroups][kRedParams];
    __shared__ int s_skip;
    const Geo d(width, n_hidden);
    const int P = d.n_params();
    const int tid = threadIdx.x, lane = tid & 63;
    const int pl = tid % kRedParams, grp = tid / kRedParams;
    const int p = blockIdx.x * kRedParams + pl;

    if (ADAM && tid < 64) {
        int any = 0;
        for (int t = tid; t < n_tiles; t += 64) any |= tile_bad[t];
        #pragma unroll
        for (int off = 32; off >= 1; off >>= 1) any |= __shfl_xor(any, off, 64);
        if (tid == 0) s_skip = any;
    }
    float s = 0.0f, c = 0.0f;
    if (p < P) {
        int t = grp;
        for (; t + 3 * kRedGroups < n_tiles; t += 4 * kRedGroups) {
            float x[4];
            #pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = partials[(int64_t)(t + u * kRedGroups) * P + p];
            #pragma unroll
            for (int u = 0; u < 4; ++u) neumaier_add(s, c, x[u]);
        }
        for (; t < n_tiles; t += kRedGroups) neumaier_add(s, c, partials[(int64_t)t * P + p]);
    }
    s_sum[grp][pl] = s;
    s_cmp[grp][pl] = c;
    __syncthreads();

    if (blockIdx.x == 0 && tid >= 64 && tid < 128 && loss_out != nullptr) {
        float ls = 0.0f, lc = 0.0f;
        for (int t = lane; t < n_tiles; t += 64) neumaier_add(ls, lc, loss_part[t]);
        float lv = ls + lc;
        #pragma unroll
        for (int off = 32; off >= 1; off >>= 1) lv += __shfl_xor(lv, off, 64);
        if (lane == 0) *loss_out = lv * inv_count;
    }
    if (grp != 0 || p >= P) return;   // workgroup 0's thread 0 has p = 0 and stays
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
    const int t_old = tslots[parity];
    const int t_new = skip ? t_old : t_old + 1;
    if (blockIdx.x == 0 && tid == 0) {
        tslots[parity ^ 1] = t_new;
        if (skipped_out) *skipped_out = skip;
    }
    if (skip) return;
    const float m1 = hp.beta1 * m[p] + (1.0f - hp.beta1) * gv;
    const float v1 = hp.beta2 * v[p] + (1.0f - hp.beta2) * gv * gv;
    const float bc1 = 1.0f - powf(hp.beta1, (float)t_new);
    const float bc2 = 1.0f - powf(hp.beta2, (float)t_new);
    const float w1 = w[p] - hp.lr * (m1 / bc1) / (sqrtf(v1 / bc2) + hp.eps);
    w[p] = w1;
    m[p] = m1;
    v[p] = v1;
    if (ffr != nullptr) write_frags<T>(d, p, w1, ffr, bfr);
}

template <typename T>
__global__ __launch_bounds__(256) void k_build_frags(const float* __restrict__ w, T* __restrict__ ffr,
                                                     T* __restrict__ bfr, int width, int n_hidden) {
    const Geo d(width, n_hidden);
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= d.n_params()) return;
    write_frags<T>(d, p, w[p], ffr, bfr);
}

}  // namespace

int reduce_blocks(int n_params) { return (n_params + kRedParams - 1) / kRedParams; }

hipError_t launch_reduce(const Geo& d, const float* partials, int n_tiles, float inv_scale,
                         float* grad, const float* loss_part, float inv_count, float* loss_out,
                         hipStream_t s) {
    hipLaunchKernelGGL((k_reduce<_Float16, false>), dim3(reduce_blocks(d.n_params())), dim3(256), 0, s,
                       partials, n_tiles, (const int32_t*)nullptr, loss_part, inv_count, loss_out,
                       inv_scale, grad, (float*)nullptr, (float*)nullptr, (float*)nullptr,
                       (int32_t*)nullptr, 0, AdamHyper{}, (int32_t*)nullptr, (_Float16*)nullptr,
                       (_Float16*)nullptr, d.W, d.H);
    return hipGetLastError();
}

hipError_t launch_reduce_adam(int precision, const Geo& d, const float* partials, int n_tiles,
                              const int32_t* tile_bad, const float* loss_part, float inv_count,
                              float* loss_out, float inv_scale, float* w, float* m, float* v,
                              int32_t* tslots, int parity, AdamHyper hp, int32_t* skipped_out,
                              void* ffr, void* bfr, hipStream_t s) {
    const dim3 grid(reduce_blocks(d.n_params())), block(256);
    if (precision == NRC_BF16)
        hipLaunchKernelGGL((k_reduce<__bf16, true>), grid, block, 0, s, partials, n_tiles, tile_bad,
                           loss_part, inv_count, loss_out, inv_scale, (float*)nullptr, w, m, v, tslots,
                           parity, hp, skipped_out, (__bf16*)ffr, (__bf16*)bfr, d.W, d.H);
    else
        hipLaunchKernelGGL((k_reduce<_Float16, true>), grid, block, 0, s, partials, n_tiles, tile_bad,
                           loss_part, inv_count, loss_out, inv_scale, (float*)nullptr, w, m, v, tslots,
                           parity, hp, skipped_out,
                           precision == NRC_FP16 ? (_Float16*)ffr : (_Float16*)nullptr,
                           precision == NRC_FP16 ? (_Float16*)bfr : (_Float16*)nullptr, d.W, d.H);
    return hipGetLastError();
}

hipError_t launch_build_frags(int precision, const Geo& d, const float* w, void* ffr, void* bfr,
                              hipStream_t s) {
    const dim3 grid((d.n_params() + 255) / 256), block(256);
    if (precision == NRC_FP16)
        hipLaunchKernelGGL(k_build_frags<_Float16>, grid, block, 0, s, w, (_Float16*)ffr,
                           (_Float16*)bfr, d.W, d.H);
    else if (precision == NRC_BF16)
        hipLaunchKernelGGL(k_build_frags<__bf16>, grid, block, 0, s, w, (__bf16*)ffr, (__bf16*)bfr,
                           d.W, d.H);
    return hipGetLastError();
}

}  // namespace nrc
