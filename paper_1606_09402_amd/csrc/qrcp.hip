// Kernels of trQRCP, the truncated randomized QR with column pivoting that the Frobenius
// indicator drives as it drives randQB (Remark 3.2).  The l x n sketch S = Omega^T A is
// stored transposed (St, n x l row-major: column j of S is row j of St, l contiguous
// values), so that one wave owns one sketch column.  Each pivot step is two launches: one
// workgroup picks the active column of largest remaining norm and forms its Householder
// reflector, then one wave per active column applies the reflector and recomputes the
// column's remaining norm exactly (no downdating).  Every sum has a fixed order, so the
// pivots are reproducible.
#include "kernels.h"

namespace qb {

constexpr int kPickThreads = 1024;   // also the largest sketch height l

// Butterfly sum over the wave; every lane ends with the same total (each level adds a
// pair of equal partial sums in either order, and IEEE addition is commutative).
QB_DEV double wave_allsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// norm2[j] = sum over the l rows of St(j, :)^2 for active columns; -1 marks the others.
__global__ void qrcp_norms_kernel(const double* __restrict__ St, int64_t n, int l,
                                  const int* __restrict__ active, double* __restrict__ norm2) {
    const int64_t j = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (j >= n) return;   // uniform per wave
    if (!active[j]) {
        if (lane == 0) norm2[j] = -1.0;
        return;
    }
    const double* x = St + j * l;
    double s = 0.0;
    for (int r = lane; r < l; r += 64) s += x[r] * x[r];
    s = wave_allsum(s);
    if (lane == 0) norm2[j] = s;
}

// Step t of the sketch's pivoted QR.  Pivot: the active column of largest norm2 (smallest
// index among equal values).  Its reflector of rows t..l-1 in LAPACK's convention
// (v(t) = 1, beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta, tau = 0 when rows
// t+1.. are zero) goes to hh (v in hh[0..l), tau in hh[l]); the pivot column becomes
// (rows < t unchanged, beta, zeros), a column of the sketch's triangular factor.  The pivot
// is recorded in piv[t], deactivated, and ||A(:, p)||^2 copied to g2[t].  With no active
// column left (the caller never asks for more pivots than there are columns) it records -1
// and an identity reflector.
__global__ void __launch_bounds__(kPickThreads)
qrcp_pick_kernel(double* __restrict__ St, int64_t n, int l, int t, double* __restrict__ norm2,
                 int* __restrict__ active, int* __restrict__ piv, const double* __restrict__ colA,
                 double* __restrict__ g2, double* __restrict__ hh) {
    __shared__ double sv[kPickThreads];
    __shared__ int64_t si[kPickThreads];
    __shared__ double red[kPickThreads / 64];
    __shared__ double s_alpha;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double best = -1.0;   // inactive entries hold -1 and never win
    int64_t bi = -1;
    for (int64_t j = tid; j < n; j += kPickThreads) {
        const double v = norm2[j];
        if (v > best) {   // increasing j: the first of equal values stays
            best = v;
            bi = j;
        }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int off = kPickThreads / 2; off > 0; off >>= 1) {
        if (tid < off) {
            const double o = sv[tid + off];
            const int64_t oi = si[tid + off];
            if (o > sv[tid] || (o == sv[tid] && oi >= 0 && (si[tid] < 0 || oi < si[tid]))) {
                sv[tid] = o;
                si[tid] = oi;
            }
        }
        __syncthreads();
    }
    const int64_t p = si[0];
    if (p < 0) {
        if (tid < l) hh[tid] = 0.0;
        if (tid == 0) {
            hh[l] = 0.0;
            piv[t] = -1;
            g2[t] = 0.0;
        }
        return;
    }
    double* x = St + p * l;
    const double xv = tid < l ? x[tid] : 0.0;
    double part = (tid > t && tid < l) ? xv * xv : 0.0;
    part = wave_allsum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    double sigma = 0.0;
#pragma unroll
    for (int w = 0; w < kPickThreads / 64; ++w) sigma += red[w];
    if (tid == t) s_alpha = xv;
    __syncthreads();
    const double a = s_alpha;
    double tau = 0.0, beta = a, scale = 0.0;
    if (sigma != 0.0) {
        const double nrm = sqrt(a * a + sigma);
        beta = a >= 0.0 ? -nrm : nrm;
        tau = (beta - a) / beta;
        scale = 1.0 / (a - beta);
    }
    if (tid < l) {
        hh[tid] = tid < t ? 0.0 : (tid == t ? 1.0 : xv * scale);
        x[tid] = tid < t ? xv : (tid == t ? beta : 0.0);
    }
    if (tid == 0) {
        hh[l] = tau;
        piv[t] = static_cast<int>(p);
        active[p] = 0;
        norm2[p] = -1.0;
        g2[t] = colA[p];
    }
}

// Applies the reflector of step t to rows t..l-1 of every active column (one wave each) and
// sets norm2 to the column's sum of squares over rows t+1..l-1.
__global__ void qrcp_apply_kernel(double* __restrict__ St, int64_t n, int l, int t,
                                  const double* __restrict__ hh, const int* __restrict__ active,
                                  double* __restrict__ norm2) {
    const int64_t j = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (j >= n || !active[j]) return;   // uniform per wave
    double* x = St + j * l;
    const double tau = hh[l];
    double d = 0.0;
    for (int r = t + lane; r < l; r += 64) d += hh[r] * x[r];
    d = wave_allsum(d);
    const double f = tau * d;
    double s = 0.0;
    for (int r = t + lane; r < l; r += 64) {
        const double y = x[r] - f * hh[r];
        x[r] = y;
        if (r > t) s += y * y;
    }
    s = wave_allsum(s);
    if (lane == 0) norm2[j] = s;
}

// Rs(i, c) = St(piv[c], i) for i <= c, 0 below (bw x bw row-major): the sketch's triangular
// factor R~_11 in pivot order.  Grid: (column blocks, bw rows).
__global__ void qrcp_rs_kernel(const double* __restrict__ St, int l, const int* __restrict__ piv,
                               int bw, double* __restrict__ Rs) {
    const int i = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bw) return;
    const int pc = piv[c];
    Rs[i * bw + c] = (i <= c && pc >= 0) ? St[static_cast<int64_t>(pc) * l + i] : 0.0;
}

// Y(i, c) = X(i, piv[c]) for the row-major rows x * matrix X (ld ldx), into the row-major
// rows x bw matrix Y (ld ldy); a missing pivot (-1) gives a zero column.
__global__ void gather_cols_kernel(const double* __restrict__ X, int64_t ldx, int64_t rows,
                                   const int* __restrict__ piv, int bw, double* __restrict__ Y,
                                   int64_t ldy) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= rows * bw) return;
    const int64_t i = e / bw;
    const int c = static_cast<int>(e - i * bw);
    const int pc = piv[c];
    Y[i * ldy + c] = pc >= 0 ? X[i * ldx + pc] : 0.0;
}

int qrcp_max_rows() { return kPickThreads; }

hipError_t launch_qrcp_norms(const double* St, int64_t n, int l, const int* active, double* norm2,
                             hipStream_t s) {
    hipLaunchKernelGGL(qrcp_norms_kernel, dim3(static_cast<unsigned>(cdiv(n, 4))), dim3(256), 0, s, St,
                       n, l, active, norm2);
    return hipGetLastError();
}

hipError_t launch_qrcp_step(double* St, int64_t n, int l, int t, double* norm2, int* active, int* piv,
                            const double* colA, double* g2, double* hh, hipStream_t s) {
    if (l > kPickThreads || t < 0 || t >= l) return hipErrorInvalidValue;
    hipLaunchKernelGGL(qrcp_pick_kernel, dim3(1), dim3(kPickThreads), 0, s, St, n, l, t, norm2, active,
                       piv, colA, g2, hh);
    hipLaunchKernelGGL(qrcp_apply_kernel, dim3(static_cast<unsigned>(cdiv(n, 4))), dim3(256), 0, s, St, n,
                       l, t, hh, active, norm2);
    return hipGetLastError();
}

hipError_t launch_qrcp_rs(const double* St, int l, const int* piv, int bw, double* Rs, hipStream_t s) {
    hipLaunchKernelGGL(qrcp_rs_kernel, dim3(static_cast<unsigned>(cdiv(bw, 128)), static_cast<unsigned>(bw)),
                       dim3(128), 0, s, St, l, piv, bw, Rs);
    return hipGetLastError();
}

hipError_t launch_gather_cols(const double* X, int64_t ldx, int64_t rows, const int* piv, int bw,
                              double* Y, int64_t ldy, hipStream_t s) {
    if (rows <= 0 || bw <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_cols_kernel, dim3(static_cast<unsigned>(cdiv(rows * bw, 256))), dim3(256), 0,
                       s, X, ldx, rows, piv, bw, Y, ldy);
    return hipGetLastError();
}

}  // namespace qb
