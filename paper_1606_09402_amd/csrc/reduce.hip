// Deterministic FP64 reductions: ||A||_F^2 as a sum of squares (Algorithm 1,
// Section 3.3 asks for the squares to be summed directly), and small fixed-order
// finalisations of per-workgroup partial sums.  No floating-point atomics are used,
// so repeated runs give identical bits.
#include "kernels.h"

namespace qb {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;   // partial sums per pass (fixed => deterministic)

QB_DEV double block_sum(double v, double* sh) {
    // wave reduction by xor-shuffles, then across the 4 waves through LDS
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) t += sh[w];
    }
    __syncthreads();
    return t;
}

// Partial sums of squares of a row-major m x n matrix with row stride lda.  Workgroup
// g owns rows g, g + G, ... ; within a row the threads stride over columns.
__global__ void __launch_bounds__(kRedThreads)
sumsq_dense_partial(const double* __restrict__ a, int64_t m, int64_t n, int64_t lda,
                    double* __restrict__ partial) {
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        const double* row = a + i * lda;
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
            const double v = row[j];
            acc += v * v;
        }
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Contiguous vector (CSR values): workgroup g owns elements [g*chunk, (g+1)*chunk).
__global__ void __launch_bounds__(kRedThreads)
sumsq_vec_partial(const double* __restrict__ x, int64_t len, int64_t chunk,
                  double* __restrict__ partial) {
    __shared__ double sh[kRedThreads / 64];
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < len ? lo + chunk : len;
    double acc = 0.0;
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
        const double v = x[j];
        acc += v * v;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// out[j] = sum_{g < groups} partial[g * stride + j]; one wave per output: lane l sums
// groups l, l + 64, ... in order, then the 64 lane sums are combined by a fixed xor
// tree.  Used for the final stage of every reduction of per-workgroup partials.
__global__ void __launch_bounds__(256)
sum_partials_kernel(const double* __restrict__ partial, int64_t groups, int64_t stride,
                    int64_t count, double* __restrict__ out) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= count) return;
    double t = 0.0;
    for (int64_t g = lane; g < groups; g += 64) t += partial[g * stride + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0) out[j] = t;
}

// Single workgroup sum of `count` partials (pairwise over threads, fixed order).
__global__ void __launch_bounds__(kRedThreads)
sum_vector_kernel(const double* __restrict__ partial, int64_t count, double* __restrict__ out) {
    __shared__ double sh[kRedThreads / 64];
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < count; j += blockDim.x) acc += partial[j];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = t;
}

// result in out[0]; scratch needs kRedBlocks doubles
hipError_t launch_sumsq_dense(const double* a, int64_t m, int64_t n, int64_t lda,
                              double* scratch, double* out, hipStream_t s) {
    const int64_t g = m < kRedBlocks ? m : kRedBlocks;
    hipLaunchKernelGGL(sumsq_dense_partial, dim3(static_cast<unsigned>(g)), dim3(kRedThreads), 0,
                       s, a, m, n, lda, scratch);
    hipLaunchKernelGGL(sum_vector_kernel, dim3(1), dim3(kRedThreads), 0, s, scratch, g, out);
    return hipGetLastError();
}

hipError_t launch_sumsq_vec(const double* x, int64_t len, double* scratch, double* out,
                            hipStream_t s) {
    if (len <= 0) return launch_fill(out, 1, 0.0, s);
    const int64_t chunk = cdiv(len, kRedBlocks) < 1024 ? 1024 : cdiv(len, kRedBlocks);
    const int64_t g = cdiv(len, chunk);
    hipLaunchKernelGGL(sumsq_vec_partial, dim3(static_cast<unsigned>(g)), dim3(kRedThreads), 0, s,
                       x, len, chunk, scratch);
    hipLaunchKernelGGL(sum_vector_kernel, dim3(1), dim3(kRedThreads), 0, s, scratch, g, out);
    return hipGetLastError();
}

int64_t sumsq_partials() { return kRedBlocks; }

hipError_t launch_sum_vector(const double* partial, int64_t count, double* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_vector_kernel, dim3(1), dim3(kRedThreads), 0, s, partial, count, out);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partial, int64_t groups, int64_t stride,
                               int64_t count, double* out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(static_cast<unsigned>(cdiv(count, 4))),
                       dim3(256), 0, s, partial, groups, stride, count, out);
    return hipGetLastError();
}

}  // namespace qb
