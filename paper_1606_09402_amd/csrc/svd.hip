// Kernels of the approximate SVD from a QB factorisation (eq. (3)): B = U~ diag(s) V~^T
// by a thin QR of B^T (B^T = P T, done by the block orthonormalisation of the library) and
// a one-sided Jacobi SVD of the k x k factor X = T^T.  One-sided Jacobi (Hestenes) rotates
// pairs of columns of X until all are mutually orthogonal: the column norms are then the
// singular values, the normalised columns the left singular vectors, and the accumulated
// rotations W the right singular vectors of X.  Rounds follow the circle ordering, so the
// k/2 pairs of a round are disjoint and run as one launch, a workgroup per pair.  Every
// sum is taken in a fixed order (bit-reproducible results).
#include "kernels.h"

namespace qb {

constexpr int kSvdThreads = 256;
constexpr int kRegK = 8;   // columns of up to kRegK * 256 rows are held in registers

// Fixed-order sum over the workgroup of three values at once.
QB_DEV void block_sum3(double& a, double& b, double& c, double (*sh)[kSvdThreads / 64]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
        c += __shfl_down(c, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
#pragma unroll
    for (int i = 0; i < kSvdThreads / 64; ++i) {
        a += sh[0][i];
        b += sh[1][i];
        c += sh[2][i];
    }
    __syncthreads();
}

// Players of round r of the circle ordering for np (even) players: player 0 stays, the
// others rotate; pair p of the round.
QB_DEV void circle_pair(int np, int r, int p, int& a, int& b) {
    const int m = np - 1;
    a = p == 0 ? 0 : 1 + (r + p - 1) % m;
    b = 1 + (r + m - 1 - p) % m;
}

// One round: workgroup p rotates its pair of columns of X (and of W) when their cosine
// exceeds tol; flag is set to 1 if any pair rotated.
__global__ void __launch_bounds__(kSvdThreads)
jacobi_round_kernel(double* __restrict__ X, double* __restrict__ W, int k, int64_t ld, int np,
                    int round, double tol, int* __restrict__ flag) {
    __shared__ double sh[3][kSvdThreads / 64];
    int a, b;
    circle_pair(np, round, static_cast<int>(blockIdx.x), a, b);
    if (a >= k || b >= k) return;   // the dummy player of an odd k (uniform per workgroup)
    if (a > b) {
        const int t = a;
        a = b;
        b = t;
    }
    double* xa = X + static_cast<int64_t>(a) * ld;
    double* xb = X + static_cast<int64_t>(b) * ld;
    double* wa = W + static_cast<int64_t>(a) * ld;
    double* wb = W + static_cast<int64_t>(b) * ld;
    if (k <= kRegK * kSvdThreads) {
        // the pair's columns of X and W are read once, into registers, before the decision,
        // so that the rotation needs no second trip to memory
        double u[kRegK], v[kRegK], p[kRegK], q[kRegK];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int e = 0; e < kRegK; ++e) {
            const int i = threadIdx.x + e * kSvdThreads;
            const bool in = i < k;
            u[e] = in ? xa[i] : 0.0;
            v[e] = in ? xb[i] : 0.0;
            p[e] = in ? wa[i] : 0.0;
            q[e] = in ? wb[i] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < kRegK; ++e) {
            al += u[e] * u[e];
            be += v[e] * v[e];
            ga += u[e] * v[e];
        }
        block_sum3(al, be, ga, sh);
        if (!(ga != 0.0) || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) return;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
#pragma unroll
        for (int e = 0; e < kRegK; ++e) {
            const int i = threadIdx.x + e * kSvdThreads;
            if (i < k) {
                xa[i] = c * u[e] - s * v[e];
                xb[i] = s * u[e] + c * v[e];
                wa[i] = c * p[e] - s * q[e];
                wb[i] = s * p[e] + c * q[e];
            }
        }
        if (threadIdx.x == 0) flag[0] = 1;
        return;
    }
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int i = threadIdx.x; i < k; i += kSvdThreads) {
        const double u = xa[i], v = xb[i];
        al += u * u;
        be += v * v;
        ga += u * v;
    }
    block_sum3(al, be, ga, sh);
    if (!(ga != 0.0) || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) return;
    const double zeta = (be - al) / (2.0 * ga);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double s = c * t;
    for (int i = threadIdx.x; i < k; i += kSvdThreads) {
        const double u = xa[i], v = xb[i];
        xa[i] = c * u - s * v;
        xb[i] = s * u + c * v;
        const double p = wa[i], q = wb[i];
        wa[i] = c * p - s * q;
        wb[i] = s * p + c * q;
    }
    if (threadIdx.x == 0) flag[0] = 1;
}

// sig[j] = ||X(:, j)||_2 (workgroup per column).
__global__ void __launch_bounds__(kSvdThreads)
column_norm_kernel(const double* __restrict__ X, int k, int64_t ld, double* __restrict__ sig) {
    __shared__ double sh[3][kSvdThreads / 64];
    const double* x = X + static_cast<int64_t>(blockIdx.x) * ld;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < k; i += kSvdThreads) a += x[i] * x[i];
    block_sum3(a, b, c, sh);
    if (threadIdx.x == 0) sig[blockIdx.x] = sqrt(a);
}

// pos[j] = place of column j in descending order of sig (equal values keep index order).
__global__ void svd_order_kernel(const double* __restrict__ sig, int k, int* __restrict__ pos) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    const double v = sig[j];
    int p = 0;
    for (int i = 0; i < k; ++i) {
        const double u = sig[i];
        p += (u > v || (u == v && i < j)) ? 1 : 0;
    }
    pos[j] = p;
}

// Sorted outputs: s[pos[j]] = sig[j], Ut(:, pos[j]) = X(:, j) / sig[j] (zero for a zero
// column), Ws(:, pos[j]) = W(:, j).  Grid: (column blocks of 256 rows, k columns).
__global__ void svd_gather_kernel(const double* __restrict__ X, const double* __restrict__ W, int k,
                                  int64_t ld, const double* __restrict__ sig,
                                  const int* __restrict__ pos, double* __restrict__ s_out,
                                  double* __restrict__ Ut, double* __restrict__ Ws) {
    const int j = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = pos[j];
    const double v = sig[j];
    if (i == 0) s_out[p] = v;
    if (i >= k) return;
    const double inv = v > 0.0 ? 1.0 / v : 0.0;
    Ut[static_cast<int64_t>(p) * ld + i] = X[static_cast<int64_t>(j) * ld + i] * inv;
    Ws[static_cast<int64_t>(p) * ld + i] = W[static_cast<int64_t>(j) * ld + i];
}

// Sign rule: make the entry of largest magnitude of V(:, j) positive (smallest row among
// equal magnitudes), flipping V(:, j) and Ut(:, j) together.  Workgroup per column.
__global__ void __launch_bounds__(kSvdThreads)
sign_rule_kernel(double* __restrict__ V, int64_t n, int64_t ldv, double* __restrict__ Ut,
                 int k, int64_t ldu) {
    __shared__ double sv[kSvdThreads];
    __shared__ int64_t si[kSvdThreads];
    double* v = V + static_cast<int64_t>(blockIdx.x) * ldv;
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t i = threadIdx.x; i < n; i += kSvdThreads) {
        const double a = fabs(v[i]);
        if (a > best) {
            best = a;
            bi = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kSvdThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const double o = sv[threadIdx.x + off];
            const int64_t oi = si[threadIdx.x + off];
            if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (!(v[si[0]] < 0.0)) return;   // uniform: every thread reads the same entry
    for (int64_t i = threadIdx.x; i < n; i += kSvdThreads) v[i] = -v[i];
    double* u = Ut + static_cast<int64_t>(blockIdx.x) * ldu;
    for (int i = threadIdx.x; i < k; i += kSvdThreads) u[i] = -u[i];
}

// W = I (k x k, column-major, ld).
__global__ void identity_kernel(double* __restrict__ W, int k, int64_t ld) {
    const int j = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) W[static_cast<int64_t>(j) * ld + i] = i == j ? 1.0 : 0.0;
}

int jacobi_players(int k) { return k + (k & 1); }

hipError_t launch_jacobi_round(double* X, double* W, int k, int64_t ld, int round, double tol,
                               int* flag, hipStream_t s) {
    const int np = jacobi_players(k);
    hipLaunchKernelGGL(jacobi_round_kernel, dim3(static_cast<unsigned>(np / 2)), dim3(kSvdThreads), 0,
                       s, X, W, k, ld, np, round, tol, flag);
    return hipGetLastError();
}

hipError_t launch_svd_finish(const double* X, const double* W, int k, int64_t ld, double* sig,
                             int* pos, double* s_out, double* Ut, double* Ws, hipStream_t s) {
    hipLaunchKernelGGL(column_norm_kernel, dim3(static_cast<unsigned>(k)), dim3(kSvdThreads), 0, s, X,
                       k, ld, sig);
    hipLaunchKernelGGL(svd_order_kernel, dim3(static_cast<unsigned>(cdiv(k, 256))), dim3(256), 0, s,
                       sig, k, pos);
    hipLaunchKernelGGL(svd_gather_kernel, dim3(static_cast<unsigned>(cdiv(k, 256)), static_cast<unsigned>(k)),
                       dim3(256), 0, s, X, W, k, ld, sig, pos, s_out, Ut, Ws);
    return hipGetLastError();
}

hipError_t launch_sign_rule(double* V, int64_t n, int64_t ldv, double* Ut, int k, int64_t ldu,
                            hipStream_t s) {
    hipLaunchKernelGGL(sign_rule_kernel, dim3(static_cast<unsigned>(k)), dim3(kSvdThreads), 0, s, V, n,
                       ldv, Ut, k, ldu);
    return hipGetLastError();
}

hipError_t launch_identity(double* W, int k, int64_t ld, hipStream_t s) {
    hipLaunchKernelGGL(identity_kernel, dim3(static_cast<unsigned>(cdiv(k, 256)), static_cast<unsigned>(k)),
                       dim3(256), 0, s, W, k, ld);
    return hipGetLastError();
}

}  // namespace qb
