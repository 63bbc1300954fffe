// Training-record shuffle (Sec. 3.5) and self-training targets (Sec. 3.2).
//
// The shuffled order is the orbit x_0 = seed mod m, x_{i+1} = (a x_i + c) mod m
// of a full-period linear congruential generator on m = 2^k >= n, with values
// >= n skipped.  Sequential by definition, it is computed in parallel: any
// x_j follows from x_0 by the j-fold composition of the affine map
// x -> a x + c, formed by repeated squaring.  Since m divides 2^32, all
// arithmetic is in wrapping 32-bit integers and masked to k bits at the end.
//
// Positions j of the orbit are split into spans of 256 * R; a workgroup owns
// one span and walks it in R rounds of 256 consecutive positions.  In general
// two kernels: k_lcg_count counts the kept values of each span; k_lcg_write
// adds the counts of the spans before its own (at most 1024) and writes its
// kept values in orbit order, compacting each round with wave ballots so that
// the stores stay consecutive.  When n is a power of two, m = n and no value
// is skipped, so position j of the permutation is x_j itself: one kernel,
// k_lcg_full, writes it directly.
#include "nrc_internal.h"

namespace nrc {
namespace {

constexpr int kShufBlock = 256;
constexpr int kMaxSpans = 1024;

__device__ inline int block_sum(int v, int* red) {
    #pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const int t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kShufBlock) void k_lcg_count(Affine step, Affine stride, uint32_t x0,
                                                          uint32_t mask, uint64_t m, uint32_t n,
                                                          int rounds, int32_t* __restrict__ counts) {
    __shared__ int red[4];
    const uint64_t span = (uint64_t)rounds * kShufBlock;
    uint64_t pos = blockIdx.x * span + threadIdx.x;
    uint32_t x = apply(power(step, pos), x0);
    int cnt = 0;
    for (int r = 0; r < rounds; ++r, pos += kShufBlock) {
        cnt += (pos < m && (x & mask) < n) ? 1 : 0;
        x = apply(stride, x);
    }
    const int t = block_sum(cnt, red);
    if (threadIdx.x == 0) counts[blockIdx.x] = t;
}

__global__ __launch_bounds__(kShufBlock) void k_lcg_write(Affine step, Affine stride, uint32_t x0,
                                                          uint32_t mask, uint64_t m, uint32_t n,
                                                          int rounds, const int32_t* __restrict__ counts,
                                                          int32_t* __restrict__ perm) {
    __shared__ int red[4];
    __shared__ int wtot[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int before = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += kShufBlock) before += counts[b];
    int base = block_sum(before, red);
    const uint64_t span = (uint64_t)rounds * kShufBlock;
    uint64_t pos = blockIdx.x * span + threadIdx.x;
    uint32_t x = apply(power(step, pos), x0);
    for (int r = 0; r < rounds; ++r, pos += kShufBlock) {
        const uint32_t v = x & mask;
        const bool keep = pos < m && v < n;
        const uint64_t ballot = __ballot(keep);
        const int below = __popcll(ballot & ((1ull << lane) - 1ull));
        if (lane == 0) wtot[wave] = __popcll(ballot);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wtot[w];
        if (keep && off + below < (int)n) perm[off + below] = (int32_t)v;   // full period: always < n
        base += wtot[0] + wtot[1] + wtot[2] + wtot[3];
        __syncthreads();
        x = apply(stride, x);
    }
}

// n = m: perm[j] = x_j for every orbit position j < m.
__global__ __launch_bounds__(kShufBlock) void k_lcg_full(Affine step, Affine stride, uint32_t x0,
                                                         uint32_t mask, uint64_t m, int rounds,
                                                         int32_t* __restrict__ perm) {
    const uint64_t span = (uint64_t)rounds * kShufBlock;
    uint64_t pos = blockIdx.x * span + threadIdx.x;
    uint32_t x = apply(power(step, pos), x0);
    for (int r = 0; r < rounds; ++r, pos += kShufBlock) {
        if (pos < m) perm[pos] = (int32_t)(x & mask);
        x = apply(stride, x);
    }
}

__global__ __launch_bounds__(256) void k_self_train(const float* __restrict__ radiance,
                                                    const float* __restrict__ throughput,
                                                    const float* __restrict__ tail_rgb,
                                                    const int32_t* __restrict__ tail_index, int64_t n,
                                                    int64_t n_tail, float* __restrict__ target) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t k = tail_index[i];
    const bool ok = k >= 0 && k < n_tail;
    const int64_t kk = ok ? k : 0;          // never read outside tail_rgb
    #pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float tail = ok ? tail_rgb[kk * 3 + c] : __builtin_nanf("");
        target[i * 3 + c] = fmaf(throughput[i * 3 + c], tail, radiance[i * 3 + c]);
    }
}

}  // namespace

// Orbit geometry of n records: modulus m = 2^k >= n, rounds per workgroup and
// number of workgroups (at most kMaxSpans).
void shuffle_shape(int64_t n, uint64_t& m, int& rounds, int& spans) {
    m = 1;
    while (m < (uint64_t)n) m <<= 1;
    const uint64_t per_round = (uint64_t)kShufBlock * kMaxSpans;
    rounds = (int)((m + per_round - 1) / per_round);
    spans = (int)((m + (uint64_t)rounds * kShufBlock - 1) / ((uint64_t)rounds * kShufBlock));
}

size_t shuffle_scratch_bytes() { return kMaxSpans * sizeof(int32_t); }

hipError_t launch_shuffle(int64_t n, uint64_t seed, int32_t* perm, int32_t* counts, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    uint64_t m;
    int rounds, spans;
    shuffle_shape(n, m, rounds, spans);
    const Affine step{kLcgA, kLcgC};
    const Affine stride = power(step, kShufBlock);
    const uint32_t mask = (uint32_t)(m - 1);
    const uint32_t x0 = (uint32_t)(seed & mask);
    if (m == (uint64_t)n) {
        hipLaunchKernelGGL(k_lcg_full, dim3(spans), dim3(kShufBlock), 0, s, step, stride, x0, mask, m, rounds,
                           perm);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_lcg_count, dim3(spans), dim3(kShufBlock), 0, s, step, stride, x0, mask, m,
                       (uint32_t)n, rounds, counts);
    hipLaunchKernelGGL(k_lcg_write, dim3(spans), dim3(kShufBlock), 0, s, step, stride, x0, mask, m,
                       (uint32_t)n, rounds, (const int32_t*)counts, perm);
    return hipGetLastError();
}

hipError_t launch_self_train(const float* radiance, const float* throughput, const float* tail_rgb,
                             const int32_t* tail_index, int64_t n, int64_t n_tail, float* target,
                             hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_self_train, dim3((unsigned)blocks), dim3(256), 0, s, radiance, throughput,
                       tail_rgb, tail_index, n, n_tail, target);
    return hipGetLastError();
}

}  // namespace nrc
