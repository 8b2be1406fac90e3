// Small dense kernels of the block loop:
//  * Cholesky of a b x b Gram matrix X^T X = R^T R with the inverse of R (CholeskyQR:
//    Q = X R^{-1}), reporting breakdown so the host can switch to Householder;
//  * the Householder thin QR of an m x b panel with diag(R) >= 0 (the fallback, and
//    the definition of qr used by the paper's steps 12-13);
//  * R_i = R~_i R_i (Algorithm 4 step 14);
//  * B_i = R_i^{-T} S by forward substitution (step 15, the "\" of Section 4.1), fused
//    with the row sums of squares ||B_i(j,:)||^2 of the error indicator (step 17 and
//    the row-by-row variant 7a-8e of Section 3.1);
//  * gathering the per-block values the host needs for the stopping test.
#include "kernels.h"

namespace qb {

constexpr int kCholThreads = 256;
constexpr int kMaxB = 128;   // largest block size b the library accepts

// Gram (b x b, row-major, only the upper triangle is read) -> R upper (row-major, zero
// below the diagonal) and Rinv = R^{-1}.  flag[0] is set to 1 if some pivot is not
// above tau * max_i Gram(i,i) (the panel is then too ill-conditioned for CholeskyQR).
__global__ void __launch_bounds__(kCholThreads)
chol_upper_inv_kernel(const double* __restrict__ gram, int b, double tau, double* __restrict__ R,
                      double* __restrict__ Rinv, int* __restrict__ flag) {
    __shared__ double M[kMaxB * (kMaxB + 1)];   // b x (b + 1), b <= kMaxB
    __shared__ double dmax;
    __shared__ int bad;
    const int ld = b + 1;
    const int tid = threadIdx.x;
    for (int e = tid; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        M[i * ld + j] = j >= i ? gram[i * b + j] : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double d = 0.0;
        for (int j = 0; j < b; ++j) d = fmax(d, M[j * ld + j]);
        dmax = d;
        bad = 0;
    }
    __syncthreads();
    for (int j = 0; j < b; ++j) {
        const double piv = M[j * ld + j];
        if (!(piv > tau * dmax)) {   // also catches NaN
            if (tid == 0) bad = 1;
            break;
        }
        const double r = sqrt(piv);
        __syncthreads();
        for (int c = j + 1 + tid; c < b; c += blockDim.x) M[j * ld + c] /= r;
        if (tid == 0) M[j * ld + j] = r;
        __syncthreads();
        // trailing update of the upper triangle: M(a, c) -= R(j, a) R(j, c), j < a <= c
        const int t = b - j - 1;
        for (int e = tid; e < t * t; e += blockDim.x) {
            const int a = j + 1 + e / t, c = j + 1 + e % t;
            if (c >= a) M[a * ld + c] -= M[j * ld + a] * M[j * ld + c];
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) flag[0] = 1;
        return;
    }
    for (int e = tid; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        R[e] = j >= i ? M[i * ld + j] : 0.0;
    }
    // R^{-1}: column c by back substitution, one thread per column
    for (int c = tid; c < b; c += blockDim.x) {
        for (int i = b - 1; i > c; --i) Rinv[i * b + c] = 0.0;
        for (int i = c; i >= 0; --i) {
            double t = i == c ? 1.0 : 0.0;
            for (int p = i + 1; p <= c; ++p) t -= M[i * ld + p] * Rinv[p * b + c];
            Rinv[i * b + c] = t / M[i * ld + i];
        }
    }
}

// Rout = Ra * Rb for upper-triangular b x b row-major matrices (Rout may not alias).
__global__ void __launch_bounds__(256)
upper_mul_kernel(const double* __restrict__ Ra, const double* __restrict__ Rb, int b,
                 double* __restrict__ Rout) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= b * b) return;
    const int i = e / b, j = e % b;
    double t = 0.0;
    for (int p = i; p <= j; ++p) t += Ra[i * b + p] * Rb[p * b + j];
    Rout[e] = j >= i ? t : 0.0;
}

// Householder thin QR of the m x b column-major panel X (leading dimension ldx), one
// workgroup.  X is overwritten by the Householder vectors; Qout (column-major, ldq)
// receives the explicit Q, R (b x b row-major) the triangular factor, both sign-fixed
// so that diag(R) >= 0.  tau needs b doubles of scratch.
constexpr int kHhThreads = 1024;

QB_DEV double hh_block_sum(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) t += sh[w];
    return t;
}

__global__ void __launch_bounds__(kHhThreads)
householder_panel_kernel(double* __restrict__ X, int64_t m, int b, int64_t ldx,
                         double* __restrict__ Qout, int64_t ldq, double* __restrict__ R,
                         double* __restrict__ tau) {
    __shared__ double sh[kHhThreads / 64];
    const int tid = threadIdx.x;
    for (int e = tid; e < b * b; e += blockDim.x) R[e] = 0.0;
    for (int j = 0; j < b; ++j) {
        double* x = X + static_cast<int64_t>(j) * ldx;
        double part = 0.0;
        for (int64_t i = j + 1 + tid; i < m; i += blockDim.x) part += x[i] * x[i];
        const double sig = hh_block_sum(part, sh);      // ||x(j+1:m)||^2
        const double alpha = x[j];
        double beta, t;
        if (sig == 0.0) {
            beta = alpha;
            t = 0.0;
        } else {
            const double nrm = sqrt(alpha * alpha + sig);
            beta = alpha >= 0.0 ? -nrm : nrm;
            t = (beta - alpha) / beta;
            const double scale = 1.0 / (alpha - beta);
            for (int64_t i = j + 1 + tid; i < m; i += blockDim.x) x[i] *= scale;
        }
        __syncthreads();
        if (tid == 0) {
            tau[j] = t;
            R[j * b + j] = beta;
            x[j] = 1.0;
        }
        __syncthreads();
        // apply H_j = I - t v v^T to the trailing columns
        for (int c = j + 1; c < b; ++c) {
            double* y = X + static_cast<int64_t>(c) * ldx;
            double p = 0.0;
            for (int64_t i = j + tid; i < m; i += blockDim.x) p += x[i] * y[i];
            const double w = hh_block_sum(p, sh) * t;
            for (int64_t i = j + tid; i < m; i += blockDim.x) y[i] -= w * x[i];
            __syncthreads();
            if (tid == 0) R[j * b + c] = y[j];
        }
        __syncthreads();
    }
    // explicit Q = H_0 ... H_{b-1} [I; 0] by backward accumulation
    for (int c = 0; c < b; ++c) {
        double* q = Qout + static_cast<int64_t>(c) * ldq;
        for (int64_t i = tid; i < m; i += blockDim.x) q[i] = i == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = b - 1; j >= 0; --j) {
        const double* x = X + static_cast<int64_t>(j) * ldx;
        const double t = tau[j];
        for (int c = j; c < b; ++c) {
            double* q = Qout + static_cast<int64_t>(c) * ldq;
            double p = 0.0;
            for (int64_t i = j + tid; i < m; i += blockDim.x) p += x[i] * q[i];
            const double w = hh_block_sum(p, sh) * t;
            for (int64_t i = j + tid; i < m; i += blockDim.x) q[i] -= w * x[i];
            __syncthreads();
        }
    }
    // sign fix: diag(R) >= 0
    for (int j = 0; j < b; ++j) {
        if (R[j * b + j] < 0.0) {
            __syncthreads();
            for (int c = j + tid; c < b; c += blockDim.x) R[j * b + c] = -R[j * b + c];
            double* q = Qout + static_cast<int64_t>(j) * ldq;
            for (int64_t i = tid; i < m; i += blockDim.x) q[i] = -q[i];
            __syncthreads();
        }
    }
}

// Forward substitution R^T X = S for b x n S (row-major, lds) with upper-triangular R
// (b x b row-major); X is written to out (row j at out + j*ldo), and the sum over this
// workgroup's columns of X(j, c)^2 to rowsq_part[blockIdx.x * b + j].  One wave per
// workgroup, one column per lane; the lane's solution vector lives in LDS.
constexpr int kTrsmThreads = 64;

__global__ void __launch_bounds__(kTrsmThreads)
trsm_rowsq_kernel(const double* __restrict__ S, int64_t lds, const double* __restrict__ R,
                  int b, int64_t n, double* __restrict__ out, int64_t ldo,
                  double* __restrict__ rowsq_part) {
    __shared__ double xs[kMaxB * kTrsmThreads];   // b x 64
    const int lane = threadIdx.x;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kTrsmThreads + lane;
    const bool live = c < n;
    for (int j = 0; j < b; ++j) {
        double t = live ? S[j * lds + c] : 0.0;
        for (int p = 0; p < j; ++p) t -= R[p * b + j] * xs[p * kTrsmThreads + lane];
        const double x = live ? t / R[j * b + j] : 0.0;
        xs[j * kTrsmThreads + lane] = x;
        if (live) out[j * ldo + c] = x;
        double q = x * x;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
        if (lane == 0) rowsq_part[static_cast<int64_t>(blockIdx.x) * b + j] = q;
    }
}

// info[0:b] = rowsq, info[b:2b] = diag(R), info[2b:3b] = guard column sums of squares
__global__ void gather_block_info(const double* __restrict__ rowsq, const double* __restrict__ R,
                                  const double* __restrict__ gcol, int b,
                                  double* __restrict__ info) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= b) return;
    info[j] = rowsq[j];
    info[b + j] = R[j * b + j];
    info[2 * b + j] = gcol[j];
}

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double v) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void fill_int_kernel(int* __restrict__ p, int n, int v) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

// ------------------------------------------------------------------------------ host

hipError_t launch_chol_inv(const double* gram, int b, double tau, double* R, double* Rinv,
                           int* flag, hipStream_t s) {
    hipLaunchKernelGGL(chol_upper_inv_kernel, dim3(1), dim3(kCholThreads), 0, s, gram, b, tau, R,
                       Rinv, flag);
    return hipGetLastError();
}

hipError_t launch_upper_mul(const double* Ra, const double* Rb, int b, double* Rout,
                            hipStream_t s) {
    hipLaunchKernelGGL(upper_mul_kernel, dim3(static_cast<unsigned>(cdiv(b * b, 256))), dim3(256),
                       0, s, Ra, Rb, b, Rout);
    return hipGetLastError();
}

hipError_t launch_householder(double* X, int64_t m, int b, int64_t ldx, double* Q, int64_t ldq,
                              double* R, double* tau, hipStream_t s) {
    hipLaunchKernelGGL(householder_panel_kernel, dim3(1), dim3(kHhThreads), 0, s, X, m, b, ldx, Q,
                       ldq, R, tau);
    return hipGetLastError();
}

int64_t trsm_groups(int64_t n) { return cdiv(n, kTrsmThreads); }

hipError_t launch_trsm_rowsq(const double* S, int64_t lds, const double* R, int b, int64_t n,
                             double* out, int64_t ldo, double* rowsq_part, hipStream_t s) {
    hipLaunchKernelGGL(trsm_rowsq_kernel, dim3(static_cast<unsigned>(trsm_groups(n))),
                       dim3(kTrsmThreads), 0, s, S, lds, R, b, n, out, ldo, rowsq_part);
    return hipGetLastError();
}

hipError_t launch_gather_info(const double* rowsq, const double* R, const double* gcol, int b,
                              double* info, hipStream_t s) {
    hipLaunchKernelGGL(gather_block_info, dim3(static_cast<unsigned>(cdiv(b, 256))), dim3(256), 0,
                       s, rowsq, R, gcol, b, info);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(static_cast<unsigned>(cdiv(n, 256))), dim3(256), 0, s, p,
                       n, v);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3(static_cast<unsigned>(cdiv(n, 256))), dim3(256), 0, s,
                       p, n, v);
    return hipGetLastError();
}

}  // namespace qb
