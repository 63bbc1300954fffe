// Validation-error reductions in FP64 on the device: per-channel norms of the
// difference between a batch of FP32 predictions and FP64 reference values,
// the inputs of the per-channel relative errors that measure the precision
// forms (normwise in the L2 and the max norm).  Two kernels: each
// workgroup reduces a fixed contiguous chunk of the records with a fixed
// tree, then one workgroup combines the chunk results in chunk order, so the
// sums are bitwise reproducible.
#include "nrc_internal.h"

namespace nrc {
namespace {

constexpr int kValBlock = 256;
constexpr int kValMaxChunks = 1024;
constexpr int kValStats = 12;   // per channel: sum d^2, sum r^2, max |d|, max |r|

// Fixed-order tree over the workgroup: sums for s < 2 of each channel, maxima
// for s >= 2.
__device__ inline void block_reduce(double (&v)[kValStats], double (*red)[kValBlock]) {
    const int t = threadIdx.x;
    #pragma unroll
    for (int k = 0; k < kValStats; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int off = kValBlock / 2; off >= 1; off >>= 1) {
        if (t < off) {
            #pragma unroll
            for (int k = 0; k < kValStats; ++k) {
                const double a = red[k][t], b = red[k][t + off];
                red[k][t] = (k & 3) < 2 ? a + b : fmax(a, b);
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kValBlock) void k_error_chunks(const float* __restrict__ got,
                                                            const double* __restrict__ ref, int64_t n,
                                                            int64_t chunk, double* __restrict__ part) {
    __shared__ double red[kValStats][kValBlock];
    double v[kValStats] = {};
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kValBlock) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double r = ref[i * 3 + c];
            const double d = (double)got[i * 3 + c] - r;
            v[4 * c + 0] = fma(d, d, v[4 * c + 0]);
            v[4 * c + 1] = fma(r, r, v[4 * c + 1]);
            v[4 * c + 2] = fmax(v[4 * c + 2], fabs(d));
            v[4 * c + 3] = fmax(v[4 * c + 3], fabs(r));
        }
    }
    block_reduce(v, red);
    if (threadIdx.x < kValStats) part[blockIdx.x * kValStats + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kValBlock) void k_error_final(const double* __restrict__ part, int chunks,
                                                           double* __restrict__ out) {
    __shared__ double red[kValStats][kValBlock];
    double v[kValStats] = {};
    for (int b = threadIdx.x; b < chunks; b += kValBlock) {
        #pragma unroll
        for (int k = 0; k < kValStats; ++k) {
            const double x = part[b * kValStats + k];
            v[k] = (k & 3) < 2 ? v[k] + x : fmax(v[k], x);
        }
    }
    block_reduce(v, red);
    if (threadIdx.x < kValStats) out[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace

size_t error_norms_scratch_bytes() { return (size_t)kValMaxChunks * kValStats * sizeof(double); }

hipError_t launch_error_norms(const float* got, const double* ref, int64_t n, double* scratch, double* out,
                              hipStream_t s) {
    int64_t chunk = (n + kValMaxChunks - 1) / kValMaxChunks;
    if (chunk < kValBlock) chunk = kValBlock;
    const int chunks = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_error_chunks, dim3(chunks), dim3(kValBlock), 0, s, got, ref, n, chunk, scratch);
    hipLaunchKernelGGL(k_error_final, dim3(1), dim3(kValBlock), 0, s, (const double*)scratch, chunks, out);
    return hipGetLastError();
}

}  // namespace nrc
