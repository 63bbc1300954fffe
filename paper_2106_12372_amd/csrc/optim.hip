// Weight-gradient reduction and the Adam update (Sec. 5 "Optimizer").
//
// k_reduce: one thread per weight sums that weight's per-tile partials in a
// fixed tile order with Neumaier compensation, so the reduced gradient does
// not depend on scheduling, and flags non-finite results per workgroup.  The
// first wave of workgroup 0 also reduces the per-tile loss partials.
//
// k_adam: one thread per weight.  If any workgroup flagged a non-finite
// gradient the whole step is skipped (weights, moments and step count stay as
// they are).  Otherwise the FP32 master weight and its moments are updated
// and the reduced-precision copies in both matrix-core fragment layouts are
// refreshed in place.  The step count lives in two device slots used in
// alternation (read one, write the other), so no thread of the launch ever
// reads a value another thread of the same launch writes.
#include "nrc_internal.h"

namespace nrc {
namespace {

constexpr int kRedBlock = 256;

__device__ inline void neumaier_add(float& s, float& c, float x) {
    const float t = s + x;
    if (fabsf(s) >= fabsf(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
}

__global__ __launch_bounds__(kRedBlock) void k_reduce(const float* __restrict__ partials,
                                                      int n_tiles, int P, float inv_scale,
                                                      float* __restrict__ grad,
                                                      int32_t* __restrict__ flags,
                                                      const float* __restrict__ loss_part,
                                                      float inv_count, float* __restrict__ loss_out) {
    const int p = blockIdx.x * kRedBlock + threadIdx.x;
    int bad = 0;
    if (p < P) {
        float s = 0.0f, c = 0.0f;
        int t = 0;
        for (; t + 8 <= n_tiles; t += 8) {
            float x[8];
            #pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = partials[(int64_t)(t + u) * P + p];
            #pragma unroll
            for (int u = 0; u < 8; ++u) neumaier_add(s, c, x[u]);
        }
        for (; t < n_tiles; ++t) neumaier_add(s, c, partials[(int64_t)t * P + p]);
        const float gv = (s + c) * inv_scale;
        grad[p] = gv;
        bad = !isfinite(gv);
    }
    const int any = __syncthreads_or(bad);
    if (threadIdx.x == 0) flags[blockIdx.x] = any ? 1 : 0;
    if (blockIdx.x == 0 && threadIdx.x < 64 && loss_out != nullptr) {
        float s = 0.0f, c = 0.0f;
        for (int t = threadIdx.x; t < n_tiles; t += 64) neumaier_add(s, c, loss_part[t]);
        float v = s + c;
        #pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (threadIdx.x == 0) *loss_out = v * inv_count;
    }
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

template <typename T>
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m,
                                              float* __restrict__ v, int32_t* __restrict__ tslots,
                                              int parity, const float* __restrict__ grad,
                                              const int32_t* __restrict__ flags, int n_flags,
                                              AdamHyper hp, int32_t* __restrict__ skipped_out,
                                              T* __restrict__ ffr, T* __restrict__ bfr, int width,
                                              int n_hidden) {
    __shared__ int s_skip;
    if (threadIdx.x < 64) {
        int any = 0;
        for (int i = threadIdx.x; i < n_flags; i += 64) any |= flags[i];
        #pragma unroll
        for (int off = 32; off >= 1; off >>= 1) any |= __shfl_xor(any, off, 64);
        if (threadIdx.x == 0) s_skip = any;
    }
    __syncthreads();
    const int skip = s_skip;
    const int t_old = tslots[parity];
    const int t_new = skip ? t_old : t_old + 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        tslots[parity ^ 1] = t_new;
        if (skipped_out) *skipped_out = skip;
    }
    if (skip) return;
    const Geo d(width, n_hidden);
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= d.n_params()) return;
    const float g = grad[p];
    const float m1 = hp.beta1 * m[p] + (1.0f - hp.beta1) * g;
    const float v1 = hp.beta2 * v[p] + (1.0f - hp.beta2) * g * g;
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

int reduce_blocks(int n_params) { return (n_params + kRedBlock - 1) / kRedBlock; }

hipError_t launch_reduce(const float* partials, int n_tiles, int n_params, float inv_scale,
                         float* grad, int32_t* flags, const float* loss_part, float inv_count,
                         float* loss_out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(reduce_blocks(n_params)), dim3(kRedBlock), 0, s, partials,
                       n_tiles, n_params, inv_scale, grad, flags, loss_part, inv_count, loss_out);
    return hipGetLastError();
}

hipError_t launch_adam(int precision, const Geo& d, float* w, float* m, float* v, int32_t* tslots,
                       int parity, const float* grad, const int32_t* flags, int n_flags,
                       AdamHyper hp, int32_t* skipped_out, void* ffr, void* bfr, hipStream_t s) {
    const dim3 grid((d.n_params() + 255) / 256), block(256);
    if (precision == NRC_FP16)
        hipLaunchKernelGGL(k_adam<_Float16>, grid, block, 0, s, w, m, v, tslots, parity, grad, flags,
                           n_flags, hp, skipped_out, (_Float16*)ffr, (_Float16*)bfr, d.W, d.H);
    else if (precision == NRC_BF16)
        hipLaunchKernelGGL(k_adam<__bf16>, grid, block, 0, s, w, m, v, tslots, parity, grad, flags,
                           n_flags, hp, skipped_out, (__bf16*)ffr, (__bf16*)bfr, d.W, d.H);
    else
        hipLaunchKernelGGL(k_adam<_Float16>, grid, block, 0, s, w, m, v, tslots, parity, grad, flags,
                           n_flags, hp, skipped_out, (_Float16*)nullptr, (_Float16*)nullptr, d.W, d.H);
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
