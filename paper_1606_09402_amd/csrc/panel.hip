// Small dense kernels of the block loop:
//  * Cholesky of a b x b Gram matrix X^T X = R^T R with the inverse of R (CholeskyQR:
//    Q = X R^{-1}), reporting breakdown so the host can switch to Householder;
//  * the Householder thin QR of an m x b panel with diag(R) >= 0 (the fallback, and
//    the definition of qr used by the paper's two qr calls per block);
//  * R_i = R~_i R_i (Algorithm 4);
//  * R_i^{-1}, from which the GEMM B_i^T = S^T R_i^{-1} solves R_i^T B_i = S (eq. (23),
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

// ----------------------------------------------------------------------- blocked Cholesky

constexpr int kCb = 16;   // diagonal block of the blocked Cholesky

QB_DEV double readlane_d(double x, int lane) {
    const long long bits = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(bits), lane);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), lane);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Gram (b x b, row-major, only the upper triangle is read) -> R upper (row-major, zero below
// the diagonal) with Gram = R^T R, and Rinv = R^{-1}; flag[0] = 1 if some pivot is not above
// tau * max_i Gram(i, i).  One workgroup of 256 threads.  The matrix, padded with the
// identity to bp = 16 ceil(b / 16) rows, lives in LDS: R fills the upper triangle, R^{-1}'s
// strictly upper part is kept transposed in the strictly lower triangle and 1 / R(i, i) in
// rd[].  For each 16-row block p: one wave factors the diagonal block in registers (lane c
// holds column c; the pivot row reaches the other lanes by readlane), every thread solves
// one column of the block row to its right against R_pp^T, and the trailing matrix is
// updated; three barriers per block.  The inverse follows by blocks: the diagonal blocks'
// inverses T_pp (a wave each, by back substitution in registers), then the off-diagonal
// blocks by block distance d: X_pq = -T_pp sum_{r = p+1..q} R_pr X_rq, two barriers per d.
template <int BMAX>
__global__ void __launch_bounds__(256)
chol_blocked_kernel(const double* __restrict__ gram, int b, double tau, double* __restrict__ R,
                    double* __restrict__ Rinv, int* __restrict__ flag) {
    constexpr int ld = BMAX + 1;
    constexpr int NBMAX = BMAX / kCb;
    constexpr int CH = 16;   // elements per thread in flight when moving the matrix
    __shared__ double S[BMAX * ld];
    __shared__ double U[(NBMAX > 1 ? NBMAX - 1 : 1) * kCb * kCb];
    __shared__ double rd[BMAX];
    __shared__ double wmax[4];
    __shared__ int bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (b + kCb - 1) / kCb, bp = nblk * kCb;
    // load: all of a thread's global reads of a round are issued before its LDS writes; the
    // largest diagonal entry comes from the same reads
    double d = 0.0;
    for (int e0 = 0; e0 < bp * bp; e0 += 256 * CH) {
        double v[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + tid + 256 * u;
            const int i = e / bp, c = e - i * bp;
            v[u] = (e < bp * bp && i < b && c < b && c >= i) ? gram[i * b + c] : (i == c ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + tid + 256 * u;
            const int i = e / bp, c = e - i * bp;
            if (e < bp * bp && c >= i) S[i * ld + c] = v[u];
            if (e < bp * bp && c == i && i < b) d = fmax(d, v[u]);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off, 64));
    if (lane == 0) wmax[wave] = d;
    if (tid == 0) bad = 0;
    __syncthreads();
    const double floor_piv = tau * fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));

    for (int p = 0; p < nblk; ++p) {
        const int p0 = p * kCb;
        // diagonal block: right-looking elimination in wave 0's registers
        if (wave == 0) {
            const int c = lane < kCb ? lane : kCb - 1;
            double v[kCb];
#pragma unroll
            for (int i = 0; i < kCb; ++i) v[i] = i <= c ? S[(p0 + i) * ld + p0 + c] : 0.0;
            bool broke = false;
#pragma unroll
            for (int j = 0; j < kCb; ++j) {
                const double piv = readlane_d(v[j], j);
                if (p0 + j < b && !(piv > floor_piv)) broke = true;
                double rjj, ir;
                sqrt_and_rsqrt(piv, rjj, ir);
                const double rj = v[j] * ir;             // R(p0 + j, p0 + c) for c > j
                v[j] = c == j ? rjj : rj;
                if (lane == j) rd[p0 + j] = ir;
#pragma unroll
                for (int a = j + 1; a < kCb; ++a) v[a] -= readlane_d(rj, a) * rj;
            }
            if (lane < kCb) {
#pragma unroll
                for (int i = 0; i < kCb; ++i)
                    if (i <= lane) S[(p0 + i) * ld + p0 + lane] = v[i];
            }
            if (broke && lane == 0) bad = 1;
        }
        __syncthreads();
        if (bad) {   // uniform
            if (tid == 0) flag[0] = 1;
            return;
        }
        const int t = bp - p0 - kCb;   // trailing size
        if (t == 0) break;
        // block row to the right: R_pp^T X = S(p0:p0+16, c), one column per thread
        if (tid < t) {
            const int c = p0 + kCb + tid;
            double x[kCb];
#pragma unroll
            for (int i = 0; i < kCb; ++i) x[i] = S[(p0 + i) * ld + c];
#pragma unroll
            for (int i = 0; i < kCb; ++i) {
                x[i] *= rd[p0 + i];
#pragma unroll
                for (int k = i + 1; k < kCb; ++k) x[k] -= S[(p0 + i) * ld + p0 + k] * x[i];
            }
#pragma unroll
            for (int i = 0; i < kCb; ++i) S[(p0 + i) * ld + c] = x[i];
        }
        __syncthreads();
        // trailing update of the upper triangle, S(a, c) -= sum_i R(p0+i, a) R(p0+i, c),
        // over its t (t + 1) / 2 elements (row a of the triangle starts at a t - a (a - 1) / 2)
        const int tri = t * (t + 1) / 2;
        for (int e = tid; e < tri; e += 256) {
            int a = static_cast<int>((2.0f * t + 1.0f - sqrtf((2.0f * t + 1.0f) * (2.0f * t + 1.0f) - 8.0f * e)) * 0.5f);
            if (a < 0) a = 0;
            if (a > t - 1) a = t - 1;
            while (a > 0 && a * t - a * (a - 1) / 2 > e) --a;
            while (a < t - 1 && (a + 1) * t - (a + 1) * a / 2 <= e) ++a;
            const int cc = a + (e - (a * t - a * (a - 1) / 2));
            const int ga = p0 + kCb + a, gc = p0 + kCb + cc;
            double acc0 = S[ga * ld + gc], acc1 = 0.0;
#pragma unroll
            for (int i = 0; i < kCb; i += 2) {
                acc0 -= S[(p0 + i) * ld + ga] * S[(p0 + i) * ld + gc];
                acc1 -= S[(p0 + i + 1) * ld + ga] * S[(p0 + i + 1) * ld + gc];
            }
            S[ga * ld + gc] = acc0 + acc1;
        }
        __syncthreads();
    }

    // inverse, diagonal blocks: T_pp = R_pp^{-1} by back substitution, a column per lane
    for (int p = wave; p < nblk; p += 4) {
        const int p0 = p * kCb;
        const int c = lane < kCb ? lane : kCb - 1;
        double r[kCb];
#pragma unroll
        for (int k = 0; k < kCb; ++k) r[k] = k == c ? 1.0 : 0.0;
#pragma unroll
        for (int i = kCb - 1; i >= 0; --i) {
            const double xi = r[i] * rd[p0 + i];
            r[i] = xi;
#pragma unroll
            for (int k = 0; k < i; ++k) r[k] -= S[(p0 + k) * ld + p0 + i] * xi;
        }
        if (lane < kCb) {
#pragma unroll
            for (int i = 0; i < kCb; ++i)
                if (i < lane) S[(p0 + lane) * ld + p0 + i] = r[i];   // T(p0+i, p0+c), i < c
        }
    }
    __syncthreads();
    // off-diagonal blocks by distance: X(i, c) with i < c is stored at S[c][i]
    for (int dd = 1; dd < nblk; ++dd) {
        const int npair = nblk - dd;
        for (int e = tid; e < npair * kCb * kCb; e += 256) {
            const int p = e / (kCb * kCb), k = (e / kCb) % kCb, c = e % kCb;
            const int p0 = p * kCb, q0 = (p + dd) * kCb;
            const double* Rrow = S + (p0 + k) * ld;     // R(p0 + k, :)
            const double* Xcol = S + (q0 + c) * ld;     // X(:, q0 + c), stored transposed
            double acc0 = 0.0, acc1 = 0.0;
            for (int r0 = p0 + kCb; r0 < q0; r0 += kCb) {
#pragma unroll
                for (int kk = 0; kk < kCb; kk += 2) {
                    acc0 += Rrow[r0 + kk] * Xcol[r0 + kk];
                    acc1 += Rrow[r0 + kk + 1] * Xcol[r0 + kk + 1];
                }
            }
            // r = q: X_qq = T_qq (upper; its diagonal is in rd, the rest stored transposed)
#pragma unroll
            for (int kk = 0; kk < kCb; kk += 2) {
                const double t0 = kk < c ? Xcol[q0 + kk] : (kk == c ? rd[q0 + c] : 0.0);
                const double t1 = kk + 1 < c ? Xcol[q0 + kk + 1] : (kk + 1 == c ? rd[q0 + c] : 0.0);
                acc0 += Rrow[q0 + kk] * t0;
                acc1 += Rrow[q0 + kk + 1] * t1;
            }
            U[e] = acc0 + acc1;
        }
        __syncthreads();
        for (int e = tid; e < npair * kCb * kCb; e += 256) {
            const int p = e / (kCb * kCb), i = (e / kCb) % kCb, c = e % kCb;
            const int p0 = p * kCb, q0 = (p + dd) * kCb;
            const double* Up = U + p * kCb * kCb;
            double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
            for (int k = 0; k < kCb; k += 2) {
                // T_pp(i, k): rd on the diagonal, stored transposed above it, zero below
                const double t0 = k > i ? S[(p0 + k) * ld + p0 + i] : (k == i ? rd[p0 + i] : 0.0);
                const double t1 = k + 1 > i ? S[(p0 + k + 1) * ld + p0 + i] : (k + 1 == i ? rd[p0 + i] : 0.0);
                acc0 += t0 * Up[k * kCb + c];
                acc1 += t1 * Up[(k + 1) * kCb + c];
            }
            S[(q0 + c) * ld + p0 + i] = -(acc0 + acc1);
        }
        __syncthreads();
    }
    // store: a thread's LDS reads of a round are issued before its global writes
    for (int e0 = 0; e0 < b * b; e0 += 256 * CH) {
        double rv[CH], iv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + tid + 256 * u;
            const int i = e / b, c = e - i * b;
            const bool in = e < b * b;
            rv[u] = in && c >= i ? S[i * ld + c] : 0.0;
            iv[u] = in && c > i ? S[c * ld + i] : (in && c == i ? rd[i] : 0.0);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int e = e0 + tid + 256 * u;
            if (e < b * b) {
                R[e] = rv[u];
                Rinv[e] = iv[u];
            }
        }
    }
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
// Workgroup (z, y) forms rows [16 y, 16 y + 16) of product z: the rows of B it needs
// (from 16 y on) and its 16 rows of A are first moved to LDS, all loads in flight at once.
constexpr int kMulRows = 16;
template <int BMAX>
__global__ void __launch_bounds__(256)
upper_mul2_kernel(const double* __restrict__ A1, const double* __restrict__ B1,
                  const double* __restrict__ A2, const double* __restrict__ B2, int b,
                  double* __restrict__ Out1, double* __restrict__ Out2) {
    constexpr int ld = BMAX + 1;
    __shared__ double Bs[BMAX * ld];
    __shared__ double As[kMulRows * ld];
    const int which = blockIdx.x;
    const double* A = which ? A2 : A1;
    const double* B = which ? B2 : B1;
    double* Out = which ? Out2 : Out1;
    const int i0 = blockIdx.y * kMulRows;
    const int rows = b - i0;                       // rows i0 .. b-1 of B
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < rows * b; e0 += 256 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + tid + 256 * u;
            v[u] = e < rows * b ? B[static_cast<int64_t>(i0) * b + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + tid + 256 * u;
            if (e < rows * b) Bs[(e / b) * ld + e % b] = v[u];
        }
    }
    const int arows = rows < kMulRows ? rows : kMulRows;
    for (int e = tid; e < arows * b; e += 256) As[(e / b) * ld + e % b] = A[static_cast<int64_t>(i0) * b + e];
    __syncthreads();
    for (int e = tid; e < arows * b; e += 256) {
        const int r = e / b, j = e % b, i = i0 + r;
        double t0 = 0.0, t1 = 0.0;
        int p = i;
        for (; p + 1 <= j; p += 2) {
            t0 += As[r * ld + p] * Bs[(p - i0) * ld + j];
            t1 += As[r * ld + p + 1] * Bs[(p + 1 - i0) * ld + j];
        }
        if (p <= j) t0 += As[r * ld + p] * Bs[(p - i0) * ld + j];
        Out[static_cast<int64_t>(i) * b + j] = j >= i ? t0 + t1 : 0.0;
    }
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

// info[0:b] = rowsq, info[b:2b] = diag(R), info[2b:3b] = guard column sums of squares,
// info[3b] = the CholeskyQR breakdown flag (as a double), so one copy carries them all
__global__ void gather_block_info(const double* __restrict__ rowsq, const double* __restrict__ R,
                                  const double* __restrict__ gcol, int b, const int* __restrict__ flag,
                                  double* __restrict__ info) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) info[3 * b] = static_cast<double>(flag[0]);
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

// ------------------------------------------------------------------ device stopping scan

__global__ void scan_init_kernel(const double* __restrict__ normA2, ScanState* __restrict__ st) {
    if (threadIdx.x != 0) return;
    ScanState z{};
    z.E = normA2[0];
    *st = z;
}

__global__ void scan_resume_kernel(ScanState* __restrict__ st, int* __restrict__ flags) {
    if (threadIdx.x < 8) flags[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        st->halt = 0;
        st->skip = 0;
    }
}

// The row-by-row stopping rule of Section 3.1 (or the whole-block test of Algorithms 1, 2
// and 4) on the device, the same arithmetic in the same order as the host rule it replaces.  One wave:
// lane j loads row j's (and row j + 64's) values and evaluates its guard; lane 0 then runs
// the sequential decrements with the values taken from the other lanes' registers.
__global__ void __launch_bounds__(64)
scan_block_kernel(const double* __restrict__ rowsq, const double* __restrict__ Ri,
                  const double* __restrict__ g2, int bw, double eps2, int row_by_row,
                  double exh_rel, const int* __restrict__ flags, ScanState* __restrict__ st,
                  int64_t* __restrict__ khist, double* __restrict__ ehist, int64_t k_expect) {
    const int lane = threadIdx.x;
    const bool live = !(st->stop || st->halt || st->k != k_expect);
    if (!live) return;   // uniform
    if (flags[0] != 0) {
        if (lane == 0) {
            st->halt = 1;
            st->skip = 1;
        }
        return;
    }
    double r0 = 0.0, r1 = 0.0;
    bool ok0 = true, ok1 = true;
    if (lane < bw) {
        r0 = rowsq[lane];
        ok0 = Ri[lane * bw + lane] > exh_rel * sqrt(g2[lane]);
    }
    if (lane + 64 < bw) {
        r1 = rowsq[lane + 64];
        ok1 = Ri[(lane + 64) * bw + lane + 64] > exh_rel * sqrt(g2[lane + 64]);
    }
    // first row whose guard fails (bw if none)
    const unsigned long long bad0 = __ballot(lane < bw && !ok0), bad1 = __ballot(lane + 64 < bw && !ok1);
    const int first_bad = bad0 ? __ffsll(static_cast<long long>(bad0)) - 1
                               : (bad1 ? 64 + __ffsll(static_cast<long long>(bad1)) - 1 : bw);
    double Et = st->E;
    int keep = first_bad, stop = first_bad < bw ? 1 : 0, exh = stop;
    for (int j = 0; j < 128; ++j) {
        if (j >= first_bad) break;   // uniform
        const double r = readlane_d(j < 64 ? r0 : r1, j & 63);
        Et -= r;
        if (row_by_row && Et < eps2) {
            keep = j + 1;
            stop = 1;
            exh = 0;
            break;
        }
    }
    if (!row_by_row && !stop && Et < eps2) stop = 1;
    if (lane == 0) {
        st->E = Et;
        st->k += keep;
        st->stop = stop;
        st->skip = stop;
        st->exhausted |= exh;
        khist[st->blocks] = st->k;
        ehist[st->blocks] = Et;
        st->rk[st->blocks & 7] = st->k;
        st->re[st->blocks & 7] = Et;
        st->blocks += 1;
    }
}

// ------------------------------------------------------------------------------ host

hipError_t launch_chol_inv(const double* gram, int b, double tau, double* R, double* Rinv,
                           int* flag, hipStream_t s) {
    if (b <= 32)
        hipLaunchKernelGGL(chol_blocked_kernel<32>, dim3(1), dim3(256), 0, s, gram, b, tau, R, Rinv, flag);
    else if (b <= 64)
        hipLaunchKernelGGL(chol_blocked_kernel<64>, dim3(1), dim3(256), 0, s, gram, b, tau, R, Rinv, flag);
    else
        hipLaunchKernelGGL(chol_blocked_kernel<128>, dim3(1), dim3(256), 0, s, gram, b, tau, R, Rinv, flag);
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
    const dim3 grid(2, static_cast<unsigned>(cdiv(b, kMulRows)));
    if (b <= 64)
        hipLaunchKernelGGL(upper_mul2_kernel<64>, grid, dim3(256), 0, s, A1, B1, A2, B2, b, Out1, Out2);
    else
        hipLaunchKernelGGL(upper_mul2_kernel<128>, grid, dim3(256), 0, s, A1, B1, A2, B2, b, Out1, Out2);
    return hipGetLastError();
}

hipError_t launch_householder(double* X, int64_t m, int b, int64_t ldx, double* Q, int64_t ldq,
                              double* R, double* tau, hipStream_t s) {
    hipLaunchKernelGGL(householder_panel_kernel, dim3(1), dim3(kHhThreads), 0, s, X, m, b, ldx, Q,
                       ldq, R, tau);
    return hipGetLastError();
}

hipError_t launch_gather_info(const double* rowsq, const double* R, const double* gcol, int b,
                              const int* flag, double* info, hipStream_t s) {
    hipLaunchKernelGGL(gather_block_info, dim3(static_cast<unsigned>(cdiv(b, 256))), dim3(256), 0,
                       s, rowsq, R, gcol, b, flag, info);
    return hipGetLastError();
}

hipError_t launch_scan_init(const double* normA2, ScanState* st, hipStream_t s) {
    hipLaunchKernelGGL(scan_init_kernel, dim3(1), dim3(64), 0, s, normA2, st);
    return hipGetLastError();
}

hipError_t launch_scan_resume(ScanState* st, int* flags, hipStream_t s) {
    hipLaunchKernelGGL(scan_resume_kernel, dim3(1), dim3(64), 0, s, st, flags);
    return hipGetLastError();
}

hipError_t launch_scan_block(const double* rowsq, const double* Ri, const double* g2, int bw, double eps2,
                             int row_by_row, double exh_rel, const int* flags, ScanState* st,
                             int64_t* khist, double* ehist, int64_t k_expect, hipStream_t s) {
    hipLaunchKernelGGL(scan_block_kernel, dim3(1), dim3(64), 0, s, rowsq, Ri, g2, bw, eps2, row_by_row, exh_rel,
                       flags, st, khist, ehist, k_expect);
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
