// Kernels of trQRCP, the truncated randomized QR with column pivoting that the Frobenius
// indicator drives as it drives randQB (Remark 3.2).  The l x n sketch S = Omega^T A is
// stored transposed (St, n x l row-major: column j of S is row j of St, l contiguous
// values).  A pivot step picks the active column of largest remaining norm, forms its
// Householder reflector, applies it to every other active column and recomputes each
// column's remaining norm exactly (no downdating).  A step is one launch (qrcp_step_kernel):
// every workgroup finds the pivot itself from the per-workgroup best columns the previous
// step left, forms the reflector from the pivot column and updates its own 16 columns, 16
// lanes to a column.  Every sum has a fixed order, so the pivots are reproducible.
#include "kernels.h"

namespace qb {

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

// Pivot step t for sketches of up to kStepRows rows.  Workgroup g owns columns
// [kStepCols g, kStepCols (g + 1)); cv_in / ci_in hold each workgroup's best active column
// (largest norm2, smallest index among equal values; -1 / -1 for none) before the step, and
// cv_out / ci_out receive them after it.  Every workgroup reduces the candidates to the
// pivot p (the column a scan of all norms in index order picks), forms its reflector of rows
// t..l-1 in LAPACK's convention (v(t) = 1, beta = -sign(alpha) ||x||, tau = (beta - alpha) /
// beta, tau = 0 when rows t+1.. are zero; the sum of squares over the four waves in wave
// order), applies it to its active columns other than p and recomputes their norms.  The pivot column itself is
// read by every workgroup and written by none: its diagonal entry beta goes to betas[t] (the
// entries below it are zeros of the triangular factor, never read), and its owner only
// deactivates it.  piv[t], g2[t] = ||A(:, p)||^2 and betas[t] are written by workgroup 0; with
// no active column left (the caller never asks for more pivots than there are columns) piv[t]
// is -1 and nothing changes.
constexpr int kStepThreads = 256;
constexpr int kStepRows = 256;
constexpr int kStepCols = 16;   // columns per workgroup, 16 lanes per column (32 and 64
                                // columns per workgroup, in two and four passes, took 37.1
                                // and 41.0 ms a trQRCP call against 36.2 ms)

QB_DEV bool qrcp_better(double v, int i, double bv, int bi) {
    return v > bv || (v == bv && i >= 0 && (bi < 0 || i < bi));
}

__global__ void __launch_bounds__(kStepThreads)
qrcp_step_kernel(double* __restrict__ St, int64_t n, int l, int t, double* __restrict__ norm2,
                 int* __restrict__ active, int* __restrict__ piv, const double* __restrict__ colA,
                 double* __restrict__ g2, double* __restrict__ betas, int ncand,
                 const double* __restrict__ cv_in, const int* __restrict__ ci_in,
                 double* __restrict__ cv_out, int* __restrict__ ci_out) {
    __shared__ double wv[kStepThreads / 64], red[kStepThreads / 64];
    __shared__ int wi[kStepThreads / 64];
    __shared__ double vsh[kStepRows];
    __shared__ double cval[kStepCols];
    __shared__ int cidx[kStepCols];
    __shared__ double s_alpha;
    const int tid = static_cast<int>(threadIdx.x), lane = tid & 63, wave = tid >> 6;
    // the workgroup's columns (16 lanes each, lane r mod 16 holding rows r, r + 16, ...) are
    // read first: they do not depend on the pivot
    constexpr int kPasses = kStepCols / (kStepThreads / 16);
    constexpr int kU = kStepRows / 16;
    const int grp = tid >> 4, gl = tid & 15;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kStepCols;
    double xr[kPasses][kU];
    bool act[kPasses];
#pragma unroll
    for (int pass = 0; pass < kPasses; ++pass) {
        const int64_t j = c0 + pass * (kStepThreads / 16) + grp;
        act[pass] = j < n && active[j] != 0;
        const double* y = St + j * l;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int r = gl + 16 * u;
            xr[pass][u] = (act[pass] && r >= t && r < l) ? y[r] : 0.0;
        }
    }
    // the pivot: best of the candidates (a total order, so every lane ends with the same one)
    double best = -1.0;
    int bi = -1;
    for (int g = tid; g < ncand; g += kStepThreads) {
        const double v = cv_in[g];
        const int i = ci_in[g];
        if (qrcp_better(v, i, best, bi)) {
            best = v;
            bi = i;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double v = __shfl_xor(best, off, 64);
        const int i = __shfl_xor(bi, off, 64);
        if (qrcp_better(v, i, best, bi)) {
            best = v;
            bi = i;
        }
    }
    if (lane == 0) {
        wv[wave] = best;
        wi[wave] = bi;
    }
    __syncthreads();
    best = wv[0];
    bi = wi[0];
#pragma unroll
    for (int w = 1; w < kStepThreads / 64; ++w)
        if (qrcp_better(wv[w], wi[w], best, bi)) {
            best = wv[w];
            bi = wi[w];
        }
    const int p = bi;
    if (p < 0) {   // no active column left: nothing to apply, no candidates
        if (blockIdx.x == 0 && tid == 0) {
            piv[t] = -1;
            g2[t] = 0.0;
            betas[t] = 0.0;
        }
        if (tid == 0) {
            cv_out[blockIdx.x] = -1.0;
            ci_out[blockIdx.x] = -1;
        }
        return;
    }
    // the reflector of rows t..l-1 of column p
    const double* x = St + static_cast<int64_t>(p) * l;
    const double xv = tid < l ? x[tid] : 0.0;
    double part = (tid > t && tid < l) ? xv * xv : 0.0;
    part = wave_allsum(part);
    if (lane == 0) red[wave] = part;
    if (tid == t) s_alpha = xv;
    __syncthreads();
    double sigma = 0.0;
#pragma unroll
    for (int w = 0; w < kStepThreads / 64; ++w) sigma += red[w];
    const double a = s_alpha;
    double tau = 0.0, beta = a, scale = 0.0;
    if (sigma != 0.0) {
        const double nrm = sqrt(a * a + sigma);
        beta = a >= 0.0 ? -nrm : nrm;
        tau = (beta - a) / beta;
        scale = 1.0 / (a - beta);
    }
    if (tid < l) vsh[tid] = tid < t ? 0.0 : (tid == t ? 1.0 : xv * scale);
    if (blockIdx.x == 0 && tid == 0) {
        piv[t] = p;
        g2[t] = colA[p];
        betas[t] = beta;
    }
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < kPasses; ++pass) {
        const int slot = pass * (kStepThreads / 16) + grp;
        const int64_t j = c0 + slot;
        double nv = -1.0;
        const bool live = act[pass] && j != p;   // uniform over the 16 lanes
        if (live) {
            double* y = St + j * l;
            double d = 0.0;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int r = gl + 16 * u;
                if (r >= t && r < l) d += vsh[r] * xr[pass][u];
            }
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) d += __shfl_xor(d, off, 16);
            const double f = tau * d;
            double sq = 0.0;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int r = gl + 16 * u;
                if (r >= t && r < l) {
                    const double v = xr[pass][u] - f * vsh[r];
                    y[r] = v;
                    if (r > t) sq += v * v;
                }
            }
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 16);
            nv = sq;
            if (gl == 0) norm2[j] = sq;
        } else if (j == p && gl == 0) {
            active[p] = 0;
            norm2[p] = -1.0;
        }
        if (gl == 0) {
            cval[slot] = live ? nv : -1.0;
            cidx[slot] = live ? static_cast<int>(j) : -1;
        }
    }
    __syncthreads();
    if (tid == 0) {   // columns in increasing order: the first of equal values stays
        double cb = -1.0;
        int ci = -1;
        for (int q = 0; q < kStepCols; ++q)
            if (cval[q] > cb) {
                cb = cval[q];
                ci = cidx[q];
            }
        cv_out[blockIdx.x] = cb;
        ci_out[blockIdx.x] = ci;
    }
}

// The per-workgroup best columns of norm2 in qrcp_step_kernel's column split (the state
// before the first step of a block).  A thread per workgroup slot.
__global__ void qrcp_cand_kernel(const double* __restrict__ norm2, int64_t n, int ncand,
                                 double* __restrict__ cv, int* __restrict__ ci) {
    const int g = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= ncand) return;
    double cb = -1.0;
    int bi = -1;
    for (int q = 0; q < kStepCols; ++q) {
        const int64_t j = static_cast<int64_t>(g) * kStepCols + q;
        if (j >= n) break;
        const double v = norm2[j];   // -1 for inactive columns
        if (v > cb) {
            cb = v;
            bi = static_cast<int>(j);
        }
    }
    cv[g] = cb;
    ci[g] = bi;
}

// Rs(i, c) = St(piv[c], i) for i < c, betas[c] for i = c, 0 below (bw x bw row-major): the
// sketch's triangular factor R~_11 in pivot order.  Grid: (column blocks, bw rows).
__global__ void qrcp_rs_kernel(const double* __restrict__ St, int l, const int* __restrict__ piv,
                               const double* __restrict__ betas, int bw, double* __restrict__ Rs) {
    const int i = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bw) return;
    const int pc = piv[c];
    double v = 0.0;
    if (pc >= 0) v = i < c ? St[static_cast<int64_t>(pc) * l + i] : (i == c ? betas[c] : 0.0);
    Rs[i * bw + c] = v;
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

int qrcp_max_rows() { return kStepRows; }
int64_t qrcp_cand_slots(int64_t n) { return cdiv(n, kStepCols); }

hipError_t launch_qrcp_cands(const double* norm2, int64_t n, double* cv, int* ci, hipStream_t s) {
    const int ncand = static_cast<int>(qrcp_cand_slots(n));
    hipLaunchKernelGGL(qrcp_cand_kernel, dim3(static_cast<unsigned>(cdiv(ncand, 256))), dim3(256), 0, s, norm2,
                       n, ncand, cv, ci);
    return hipGetLastError();
}

hipError_t launch_qrcp_norms(const double* St, int64_t n, int l, const int* active, double* norm2,
                             hipStream_t s) {
    hipLaunchKernelGGL(qrcp_norms_kernel, dim3(static_cast<unsigned>(cdiv(n, 4))), dim3(256), 0, s, St,
                       n, l, active, norm2);
    return hipGetLastError();
}

hipError_t launch_qrcp_step(double* St, int64_t n, int l, int t, double* norm2, int* active, int* piv,
                            const double* colA, double* g2, double* betas, double* cv, int* ci, hipStream_t s) {
    if (l > kStepRows || t < 0 || t >= l) return hipErrorInvalidValue;
    const int64_t ncand = qrcp_cand_slots(n);
    const int in = t & 1, out = in ^ 1;
    hipLaunchKernelGGL(qrcp_step_kernel, dim3(static_cast<unsigned>(ncand)), dim3(kStepThreads), 0, s, St, n, l, t,
                       norm2, active, piv, colA, g2, betas, static_cast<int>(ncand), cv + in * ncand, ci + in * ncand,
                       cv + out * ncand, ci + out * ncand);
    return hipGetLastError();
}

hipError_t launch_qrcp_rs(const double* St, int l, const int* piv, const double* betas, int bw, double* Rs,
                          hipStream_t s) {
    hipLaunchKernelGGL(qrcp_rs_kernel, dim3(static_cast<unsigned>(cdiv(bw, 128)), static_cast<unsigned>(bw)),
                       dim3(128), 0, s, St, l, piv, betas, bw, Rs);
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
