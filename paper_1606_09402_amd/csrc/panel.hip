// Small dense kernels of the block loop:
//  * Cholesky of a b x b Gram matrix X^T X = R^T R with the inverse of R (CholeskyQR:
//    Q = X R^{-1}), reporting breakdown so the host can switch to Householder;
//  * the Householder thin QR of an m x b panel with diag(R) >= 0 (the fallback, and
//    the definition of qr used by the paper's steps 12-13);
//  * R_i = R~_i R_i (Algorithm 4 step 14);
//  * R_i^{-1}, from which the GEMM B_i^T = S^T R_i^{-1} solves R_i^T B_i = S (step 15,
//    the "\" of Section 4.1);
//  * gathering the per-block values the host needs for the stopping test.
#include "kernels.h"

namespace qb {

// Register layout for the b x b kernels (b <= BMAX): thread t owns column c = t mod BMAX
// and rows a = t div BMAX + G q, q < Q, of the working matrix (G = 256 / BMAX row groups).
// One step of a right-looking elimination publishes the pivot row in LDS (double
// buffered, so one barrier per step) and every thread updates its own rows in registers.
template <int BMAX>
struct RegLayout {
    static constexpr int NT = 256, G = NT / BMAX, Q = BMAX / G;
};

// One elimination step per row j = g0 + G Q0 of the right-looking Cholesky, for the
// row slot Q0 (a template parameter, so v[Q0] is a compile-time register); recurses to
// the next slot.  Returns false on a pivot at or below floor_piv.
template <int BMAX, int Q0>
QB_DEV bool chol_slots(double (&v)[RegLayout<BMAX>::Q], double (*row)[BMAX], double* Rs, int b,
                       double floor_piv, int& step) {
    using L = RegLayout<BMAX>;
    if constexpr (Q0 >= L::Q) {
        return true;
    } else {
        constexpr int ld = BMAX + 1;
        const int tid = threadIdx.x, c = tid % BMAX, g = tid / BMAX;
        for (int g0 = 0; g0 < L::G; ++g0) {
            const int j = g0 + L::G * Q0;
            if (j >= b) return true;                  // uniform
            const int buf = step & 1;
            ++step;
            if (g == g0) row[buf][c] = v[Q0];         // publish row j
            __syncthreads();
            const double piv = row[buf][j];
            if (!(piv > floor_piv)) return false;     // uniform (NaN included)
            const double rjj = sqrt(piv);
            const double ir = 1.0 / rjj;
            const double rc = row[buf][c] * ir;       // R(j, c) for c >= j
            if (g == 0) Rs[j * ld + c] = (c >= j && c < b) ? (c == j ? rjj : rc) : 0.0;
            // rows a = g + G q with q < Q0 lie above j and are final
#pragma unroll
            for (int q = Q0; q < L::Q; ++q) {
                const int a = g + L::G * q;
                const double upd = v[q] - (row[buf][a] * ir) * rc;
                v[q] = (a > j && c >= a) ? upd : v[q];
            }
        }
        return chol_slots<BMAX, Q0 + 1>(v, row, Rs, b, floor_piv, step);
    }
}

// Back substitution R X = I for the rows of slot Q0 (descending), then the lower slots:
// row i of X is T(i, :) / R(i, i), then rows a < i lose R(a, i) X(i, :).
template <int BMAX, int Q0>
QB_DEV void inv_slots(double (&v)[RegLayout<BMAX>::Q], double (*row)[BMAX], const double* Rs,
                      int b, double* __restrict__ Rinv, int& step) {
    using L = RegLayout<BMAX>;
    if constexpr (Q0 >= 0) {
        constexpr int ld = BMAX + 1;
        const int tid = threadIdx.x, c = tid % BMAX, g = tid / BMAX;
        for (int g0 = L::G - 1; g0 >= 0; --g0) {
            const int i = g0 + L::G * Q0;
            if (i >= b) continue;                     // uniform
            const int buf = step & 1;
            ++step;
            if (g == g0) row[buf][c] = v[Q0] / Rs[i * ld + i];
            __syncthreads();
            const double xc = row[buf][c];
            if (g == 0 && c < b) Rinv[i * b + c] = c >= i ? xc : 0.0;
            // rows a = g + G q with q > Q0 lie below i and are final
#pragma unroll
            for (int q = 0; q <= Q0; ++q) {
                const int a = g + L::G * q;
                const double upd = v[q] - Rs[a * ld + i] * xc;
                v[q] = a < i ? upd : v[q];
            }
        }
        inv_slots<BMAX, Q0 - 1>(v, row, Rs, b, Rinv, step);
    }
}

// Inverse of the upper-triangular factor held in Rs (pitch BMAX + 1); v[] is the
// thread's register slice of the working matrix T (initialised to I).
template <int BMAX>
QB_DEV void tri_inverse_rows(const double* Rs, int b, double (&v)[RegLayout<BMAX>::Q],
                             double (*row)[BMAX], double* __restrict__ Rinv) {
    using L = RegLayout<BMAX>;
    const int tid = threadIdx.x, c = tid % BMAX, g = tid / BMAX;
#pragma unroll
    for (int q = 0; q < L::Q; ++q) v[q] = (g + L::G * q) == c ? 1.0 : 0.0;
    int step = 0;
    inv_slots<BMAX, L::Q - 1>(v, row, Rs, b, Rinv, step);
}

// Gram (b x b, row-major, only the upper triangle is read) -> R upper (row-major, zero
// below the diagonal) with Gram = R^T R, and Rinv = R^{-1}.  flag[0] is set to 1 if some
// pivot is not above tau * max_i Gram(i,i) (the panel is then too ill-conditioned for
// CholeskyQR).
template <int BMAX>
__global__ void __launch_bounds__(256)
chol_upper_inv_kernel(const double* __restrict__ gram, int b, double tau, double* __restrict__ R,
                      double* __restrict__ Rinv, int* __restrict__ flag) {
    using L = RegLayout<BMAX>;
    constexpr int ld = BMAX + 1;
    __shared__ double Rs[BMAX * ld];
    __shared__ double row[2][BMAX];
    __shared__ double wmax[L::NT / 64];
    const int tid = threadIdx.x, c = tid % BMAX, g = tid / BMAX;
    double v[L::Q];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int a = g + L::G * q;
        v[q] = (a < b && c < b && a <= c) ? gram[a * b + c] : 0.0;
    }
    double d = tid < b ? gram[tid * b + tid] : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off, 64));
    if ((tid & 63) == 0) wmax[tid >> 6] = d;
    __syncthreads();
    double dmax = 0.0;
#pragma unroll
    for (int w = 0; w < L::NT / 64; ++w) dmax = fmax(dmax, wmax[w]);
    int step = 0;
    if (!chol_slots<BMAX, 0>(v, row, Rs, b, tau * dmax, step)) {
        if (tid == 0) flag[0] = 1;
        return;
    }
    __syncthreads();
    for (int e = tid; e < b * b; e += L::NT) {
        const int i = e / b, jj = e - i * b;
        R[e] = jj >= i ? Rs[i * ld + jj] : 0.0;
    }
    tri_inverse_rows<BMAX>(Rs, b, v, row, Rinv);
}

// Rinv = R^{-1} for an upper-triangular b x b row-major R.
template <int BMAX>
__global__ void __launch_bounds__(256)
tri_inv_kernel(const double* __restrict__ R, int b, double* __restrict__ Rinv) {
    using L = RegLayout<BMAX>;
    constexpr int ld = BMAX + 1;
    __shared__ double Rs[BMAX * ld];
    __shared__ double row[2][BMAX];
    for (int e = threadIdx.x; e < b * b; e += L::NT) {
        const int i = e / b, jj = e - i * b;
        Rs[i * ld + jj] = jj >= i ? R[e] : 0.0;
    }
    __syncthreads();
    double v[L::Q];
    tri_inverse_rows<BMAX>(Rs, b, v, row, Rinv);
}

// Out1 = A1 B1 and Out2 = A2 B2 for upper-triangular b x b row-major matrices (used for
// R_i = R~_i R_i and R_i^{-1} = R_i^{-1} R~_i^{-1}); outputs may not alias inputs.
__global__ void __launch_bounds__(256)
upper_mul2_kernel(const double* __restrict__ A1, const double* __restrict__ B1,
                  const double* __restrict__ A2, const double* __restrict__ B2, int b,
                  double* __restrict__ Out1, double* __restrict__ Out2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * b * b) return;
    const int which = e >= b * b;
    const int f = e - which * b * b;
    const double* A = which ? A2 : A1;
    const double* B = which ? B2 : B1;
    const int i = f / b, j = f - i * b;
    double t = 0.0;
    for (int p = i; p <= j; ++p) t += A[i * b + p] * B[p * b + j];
    (which ? Out2 : Out1)[f] = j >= i ? t : 0.0;
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
    if (b <= 32)
        hipLaunchKernelGGL(chol_upper_inv_kernel<32>, dim3(1), dim3(256), 0, s, gram, b, tau, R, Rinv, flag);
    else if (b <= 64)
        hipLaunchKernelGGL(chol_upper_inv_kernel<64>, dim3(1), dim3(256), 0, s, gram, b, tau, R, Rinv, flag);
    else
        hipLaunchKernelGGL(chol_upper_inv_kernel<128>, dim3(1), dim3(256), 0, s, gram, b, tau, R, Rinv, flag);
    return hipGetLastError();
}

hipError_t launch_tri_inv(const double* R, int b, double* Rinv, hipStream_t s) {
    if (b <= 32)
        hipLaunchKernelGGL(tri_inv_kernel<32>, dim3(1), dim3(256), 0, s, R, b, Rinv);
    else if (b <= 64)
        hipLaunchKernelGGL(tri_inv_kernel<64>, dim3(1), dim3(256), 0, s, R, b, Rinv);
    else
        hipLaunchKernelGGL(tri_inv_kernel<128>, dim3(1), dim3(256), 0, s, R, b, Rinv);
    return hipGetLastError();
}

hipError_t launch_upper_mul2(const double* A1, const double* B1, const double* A2, const double* B2,
                             int b, double* Out1, double* Out2, hipStream_t s) {
    hipLaunchKernelGGL(upper_mul2_kernel, dim3(static_cast<unsigned>(cdiv(2 * b * b, 256))),
                       dim3(256), 0, s, A1, B1, A2, B2, b, Out1, Out2);
    return hipGetLastError();
}

hipError_t launch_householder(double* X, int64_t m, int b, int64_t ldx, double* Q, int64_t ldq,
                              double* R, double* tau, hipStream_t s) {
    hipLaunchKernelGGL(householder_panel_kernel, dim3(1), dim3(kHhThreads), 0, s, X, m, b, ldx, Q,
                       ldq, R, tau);
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
