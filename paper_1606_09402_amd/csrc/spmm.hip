// Sparse products for CSR input (Section 5.1 stores sparse A in CSR):
//   G = A X        one wavefront per segment of at most kSeg nonzeros of a row; the
//                  lanes span the dense columns so every gathered row of X is read with
//                  coalesced 64-lane loads.  Rows longer than kSeg (the hub columns of a
//                  power-law matrix, as rows of A^T) are split over several wavefronts
//                  whose partial rows are summed in segment order by a second kernel, so
//                  the work is balanced and the result bits are reproducible;
//   H = A^T G      the same on CSR(A^T), built once by a stable sort of the nonzeros by
//                  column (rows stay ascending inside each column).
// The segment plan of a CSR matrix (segments per row, their prefix sums, the row of
// each segment) is built on the device once per call.  No floating-point atomics.
#include <hipcub/hipcub.hpp>

#include "kernels.h"

namespace qb {

constexpr int kSpmmThreads = 256;          // 4 rows per workgroup
constexpr int kSpmmCols = 64 * 4;          // dense columns per wave pass (4 per lane)

// G(i, c0 + t) = sum_e val[e] X(colind[e], c0 + t) for the columns of this pass.
__global__ void __launch_bounds__(kSpmmThreads)
spmm_csr_rowwave_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                        const double* __restrict__ val, int64_t m, const double* __restrict__ X,
                        int64_t ldx, double* __restrict__ G, int64_t ldg, int64_t w) {
    const int lane = threadIdx.x & 63;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * (kSpmmThreads / 64) + (threadIdx.x >> 6);
    if (row >= m) return;
    const int64_t c0 = static_cast<int64_t>(blockIdx.y) * kSpmmCols;
    const int64_t e0 = rowptr[row], e1 = rowptr[row + 1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    bool ok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) ok[t] = c0 + lane + 64 * t < w;
    for (int64_t e = e0; e < e1; ++e) {
        const double v = val[e];
        const double* xr = X + static_cast<int64_t>(colind[e]) * ldx + c0 + lane;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (ok[t]) acc[t] += v * xr[64 * t];
    }
    double* gr = G + row * ldg + c0 + lane;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (ok[t]) gr[64 * t] = acc[t];
}

constexpr int64_t kSeg = 512;   // nonzeros per segment

// Segments of row i: 1 if it has at most kSeg nonzeros, else ceil(len / kSeg); entry
// `rows` of both counts is 0 so that the exclusive scans end with the totals.
__global__ void plan_count_kernel(const int64_t* __restrict__ rowptr, int64_t rows,
                                  int64_t* __restrict__ cnt_s, int64_t* __restrict__ cnt_m) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i > rows) return;
    if (i == rows) {
        cnt_s[i] = 0;
        cnt_m[i] = 0;
        return;
    }
    const int64_t len = rowptr[i + 1] - rowptr[i];
    const int64_t ns = len > kSeg ? (len + kSeg - 1) / kSeg : 1;
    cnt_s[i] = ns;
    cnt_m[i] = ns > 1 ? ns : 0;
}

__global__ void plan_fill_kernel(const int64_t* __restrict__ seg_off, int64_t rows,
                                 int32_t* __restrict__ seg_row) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    for (int64_t q = seg_off[i]; q < seg_off[i + 1]; ++q) seg_row[q] = static_cast<int32_t>(i);
}

// Wavefront per segment: its nonzeros times the rows of X for the 256 columns of this
// pass (4 per lane); a row with one segment is written to G, the segments of a longer row
// to P.  Used for short rows, where the index loads of a segment dominate and wide passes
// amortise them.
__global__ void __launch_bounds__(kSpmmThreads)
spmm_seg_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                const double* __restrict__ val, int64_t rows, const int64_t* __restrict__ seg_off,
                const int64_t* __restrict__ mseg_off, const int32_t* __restrict__ seg_row,
                const double* __restrict__ X, int64_t ldx, double* __restrict__ G, int64_t ldg,
                double* __restrict__ P, int64_t w) {
    const int lane = threadIdx.x & 63;
    const int64_t sg = static_cast<int64_t>(blockIdx.x) * (kSpmmThreads / 64) + (threadIdx.x >> 6);
    if (sg >= seg_off[rows]) return;
    const int64_t row = seg_row[sg];
    const int64_t q = sg - seg_off[row], ns = seg_off[row + 1] - seg_off[row];
    const int64_t c0 = static_cast<int64_t>(blockIdx.y) * kSpmmCols;
    const int64_t e0 = rowptr[row] + q * kSeg;
    const int64_t e1 = e0 + kSeg < rowptr[row + 1] ? e0 + kSeg : rowptr[row + 1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    bool ok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) ok[t] = c0 + lane + 64 * t < w;
    for (int64_t e = e0; e < e1; ++e) {
        const double v = val[e];
        const double* xr = X + static_cast<int64_t>(colind[e]) * ldx + c0 + lane;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (ok[t]) acc[t] += v * xr[64 * t];
    }
    double* out = ns == 1 ? G + row * ldg + c0 + lane : P + (mseg_off[row] + q) * w + c0 + lane;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (ok[t]) out[64 * t] = acc[t];
}

// Wavefront per segment, over one slab of kSlab = 32 dense columns: the two half-waves take
// alternate nonzeros of the segment (lane l: column c0 + l mod 32 of nonzeros e0 + l / 32,
// + 2, ...), each keeping kUnroll gathers of X rows in flight, and are added at the end.  A
// slab of X (32 columns of every row) is at most 128 MB for the matrices of this library's
// sparse workload, so the slab in use stays resident in the last-level cache while its
// segments are processed (all segments of a slab are dispatched before the next slab's); the
// CSR arrays are re-read once per slab.  A row with one segment is written to G, the
// segments of a longer row to P.
constexpr int kSlab = 32;
constexpr int kUnroll = 4;
constexpr int64_t kLongRow = 16;
__global__ void __launch_bounds__(kSpmmThreads)
spmm_seg32_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                  const double* __restrict__ val, int64_t rows, const int64_t* __restrict__ seg_off,
                  const int64_t* __restrict__ mseg_off, const int32_t* __restrict__ seg_row,
                  const double* __restrict__ X, int64_t ldx, double* __restrict__ G, int64_t ldg,
                  double* __restrict__ P, int64_t w) {
    const int lane = threadIdx.x & 63, half = lane >> 5;
    // the segment index is the same for the whole wave
    const int64_t sg = static_cast<int64_t>(blockIdx.x) * (kSpmmThreads / 64) +
                       __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (sg >= seg_off[rows]) return;
    const int64_t row = seg_row[sg];
    const int64_t q = sg - seg_off[row], ns = seg_off[row + 1] - seg_off[row];
    const int64_t c = static_cast<int64_t>(blockIdx.y) * kSlab + (lane & 31);
    const bool ok = c < w;
    const int64_t cc = ok ? c : w - 1;   // columns past w re-read the last one (never stored)
    const int64_t e0 = rowptr[row] + q * kSeg;
    const int64_t e1 = e0 + kSeg < rowptr[row + 1] ? e0 + kSeg : rowptr[row + 1];
    const double* xc = X + cc;
    double acc = 0.0;
    int64_t e = e0 + half;
    for (; e + 2 * (kUnroll - 1) < e1; e += 2 * kUnroll) {
        double v[kUnroll], x[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            v[u] = val[e + 2 * u];
            x[u] = xc[static_cast<int64_t>(colind[e + 2 * u]) * ldx];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += v[u] * x[u];
    }
    for (; e < e1; e += 2) acc += val[e] * xc[static_cast<int64_t>(colind[e]) * ldx];
    // even-indexed nonzeros (lanes 0..31) plus odd-indexed ones (lanes 32..63)
    const double other = __shfl_down(acc, 32, 64);
    if (half != 0 || !ok) return;
    acc += other;
    if (ns == 1) G[row * ldg + c] = acc;
    else P[(mseg_off[row] + q) * w + c] = acc;
}

// Rows with several segments: G row = sum of the segment partials in segment order.
__global__ void __launch_bounds__(kSpmmThreads)
spmm_seg_reduce_kernel(int64_t rows, const int64_t* __restrict__ seg_off,
                       const int64_t* __restrict__ mseg_off, const double* __restrict__ P,
                       double* __restrict__ G, int64_t ldg, int64_t w) {
    const int lane = threadIdx.x & 63;
    const int64_t row = static_cast<int64_t>(blockIdx.x) * (kSpmmThreads / 64) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const int64_t ns = seg_off[row + 1] - seg_off[row];
    if (ns <= 1) return;
    const int64_t c0 = static_cast<int64_t>(blockIdx.y) * kSpmmCols;
    const double* p = P + mseg_off[row] * w + c0 + lane;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (c0 + lane + 64 * t >= w) continue;
        double acc = 0.0;
        for (int64_t q = 0; q < ns; ++q) acc += p[q * w + 64 * t];
        G[row * ldg + c0 + lane + 64 * t] = acc;
    }
}

// Column sums of squares of a row-major rows x w matrix: workgroup g sums rows
// g, g + G, ... for 256 columns; partial[g * w + j].
__global__ void __launch_bounds__(256)
colsq_rowmajor_kernel(const double* __restrict__ Y, int64_t rows, int64_t w, int64_t ld,
                      double* __restrict__ partial) {
    const int64_t j = static_cast<int64_t>(blockIdx.y) * 256 + threadIdx.x;
    if (j >= w) return;
    double t = 0.0;
    for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
        const double v = Y[i * ld + j];
        t += v * v;
    }
    partial[static_cast<int64_t>(blockIdx.x) * w + j] = t;
}

// rowidx[e] = row of nonzero e
__global__ void csr_rowidx_kernel(const int64_t* __restrict__ rowptr, int64_t m,
                                  int32_t* __restrict__ rowidx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) rowidx[e] = static_cast<int32_t>(i);
}

__global__ void iota_kernel(int32_t* __restrict__ p, int64_t n) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < n) p[e] = static_cast<int32_t>(e);
}

// gather the transposed entries and locate column starts by binary search in the
// sorted keys (no atomics)
__global__ void csc_finish_kernel(const int32_t* __restrict__ keys_sorted,
                                  const int32_t* __restrict__ perm, const int32_t* __restrict__ rowidx,
                                  const double* __restrict__ val, int64_t nnz, int64_t n,
                                  int64_t* __restrict__ colptr, int32_t* __restrict__ t_col,
                                  double* __restrict__ t_val) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < nnz) {
        const int32_t src = perm[e];
        t_col[e] = rowidx[src];
        t_val[e] = val[src];
    }
    if (e <= n) {
        int64_t lo = 0, hi = nnz;   // first position with key >= e
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys_sorted[mid] < e) lo = mid + 1; else hi = mid;
        }
        colptr[e] = lo;
    }
}

// ------------------------------------------------------------------------------ host

hipError_t launch_spmm_csr(const int64_t* rowptr, const int32_t* colind, const double* val,
                           int64_t m, const double* X, int64_t ldx, double* G, int64_t ldg,
                           int64_t w, hipStream_t s) {
    if (m <= 0 || w <= 0) return hipSuccess;
    dim3 grid(static_cast<unsigned>(cdiv(m, kSpmmThreads / 64)),
              static_cast<unsigned>(cdiv(w, kSpmmCols)));
    hipLaunchKernelGGL(spmm_csr_rowwave_kernel, grid, dim3(kSpmmThreads), 0, s, rowptr, colind, val,
                       m, X, ldx, G, ldg, w);
    return hipGetLastError();
}

static size_t align256_(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

static size_t scan_bytes(int64_t items) {
    size_t tb = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, tb, static_cast<const int64_t*>(nullptr),
                                     static_cast<int64_t*>(nullptr), static_cast<int>(items));
    return tb + 256;
}

// Segment plan in ws: counts (2 x rows+1), offsets (2 x rows+1), seg_row (rows + nnz/kSeg
// + 1), scan scratch, and P for the partial rows: at most 2 nnz / kSeg segments belong to
// rows with more than one segment, each a row of wmax doubles.
size_t spmm_plan_bytes(int64_t rows, int64_t nnz, int64_t wmax) {
    size_t b = 0;
    b += 2 * align256_(sizeof(int64_t) * (rows + 1));
    b += 2 * align256_(sizeof(int64_t) * (rows + 1));
    b += align256_(sizeof(int32_t) * (rows + nnz / kSeg + 1));
    b += align256_(scan_bytes(rows + 1));
    b += align256_(sizeof(double) * (2 * cdiv(nnz, kSeg) + 1) * wmax);
    return b;
}

hipError_t spmm_plan_build(const int64_t* rowptr, int64_t rows, int64_t nnz, int64_t wmax, char* ws,
                           hipStream_t s, SpmmPlan* plan) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = ws + off;
        off += align256_(bytes);
        return p;
    };
    int64_t* cnt_s = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (rows + 1)));
    int64_t* cnt_m = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (rows + 1)));
    plan->rows = rows;
    plan->nnz = nnz;
    plan->smax = rows + nnz / kSeg + 1;
    plan->seg_off = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (rows + 1)));
    plan->mseg_off = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (rows + 1)));
    plan->seg_row = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * plan->smax));
    const size_t sb = scan_bytes(rows + 1);
    char* tmp = take(sb);
    plan->P = reinterpret_cast<double*>(take(sizeof(double) * (2 * cdiv(nnz, kSeg) + 1) * wmax));
    plan->wmax = wmax;
    const unsigned g = static_cast<unsigned>(cdiv(rows + 1, 256));
    hipLaunchKernelGGL(plan_count_kernel, dim3(g), dim3(256), 0, s, rowptr, rows, cnt_s, cnt_m);
    size_t tb = sb;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt_s, plan->seg_off, static_cast<int>(rows + 1), s);
    if (e != hipSuccess) return e;
    tb = sb;
    e = hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt_m, plan->mseg_off, static_cast<int>(rows + 1), s);
    if (e != hipSuccess) return e;
    if (rows > 0)
        hipLaunchKernelGGL(plan_fill_kernel, dim3(static_cast<unsigned>(cdiv(rows, 256))), dim3(256), 0, s,
                           plan->seg_off, rows, plan->seg_row);
    return hipGetLastError();
}

hipError_t launch_spmm_plan(const SpmmPlan& plan, const int64_t* rowptr, const int32_t* colind,
                            const double* val, const double* X, int64_t ldx, double* G, int64_t ldg,
                            int64_t w, hipStream_t s) {
    if (plan.rows <= 0 || w <= 0) return hipSuccess;
    if (w > plan.wmax) return hipErrorInvalidValue;
    if (plan.nnz >= kLongRow * plan.rows) {
        dim3 grid(static_cast<unsigned>(cdiv(plan.smax, kSpmmThreads / 64)), static_cast<unsigned>(cdiv(w, kSlab)));
        hipLaunchKernelGGL(spmm_seg32_kernel, grid, dim3(kSpmmThreads), 0, s, rowptr, colind, val, plan.rows,
                           plan.seg_off, plan.mseg_off, plan.seg_row, X, ldx, G, ldg, plan.P, w);
    } else {
        dim3 grid(static_cast<unsigned>(cdiv(plan.smax, kSpmmThreads / 64)),
                  static_cast<unsigned>(cdiv(w, kSpmmCols)));
        hipLaunchKernelGGL(spmm_seg_kernel, grid, dim3(kSpmmThreads), 0, s, rowptr, colind, val, plan.rows,
                           plan.seg_off, plan.mseg_off, plan.seg_row, X, ldx, G, ldg, plan.P, w);
    }
    dim3 rgrid(static_cast<unsigned>(cdiv(plan.rows, kSpmmThreads / 64)), static_cast<unsigned>(cdiv(w, kSpmmCols)));
    hipLaunchKernelGGL(spmm_seg_reduce_kernel, rgrid, dim3(kSpmmThreads), 0, s, plan.rows, plan.seg_off,
                       plan.mseg_off, plan.P, G, ldg, w);
    return hipGetLastError();
}

int64_t colsq_groups(int64_t rows) { return rows < 512 ? (rows > 0 ? rows : 1) : 512; }

hipError_t launch_colsq_rowmajor(const double* Y, int64_t rows, int64_t w, int64_t ld,
                                 double* partial, hipStream_t s) {
    if (w <= 0) return hipSuccess;
    dim3 grid(static_cast<unsigned>(colsq_groups(rows)), static_cast<unsigned>(cdiv(w, 256)));
    hipLaunchKernelGGL(colsq_rowmajor_kernel, grid, dim3(256), 0, s, Y, rows, w, ld, partial);
    return hipGetLastError();
}


static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

CscLayout csc_layout(int64_t m, int64_t n, int64_t nnz) {
    (void)m;
    CscLayout L{};
    size_t temp_bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, static_cast<const int32_t*>(nullptr),
                                       static_cast<int32_t*>(nullptr),
                                       static_cast<const int32_t*>(nullptr),
                                       static_cast<int32_t*>(nullptr), static_cast<int>(nnz));
    size_t off = 0;
    L.colptr = off; off = align256(off + sizeof(int64_t) * (n + 1));
    L.t_col = off; off = align256(off + sizeof(int32_t) * nnz);
    L.t_val = off; off = align256(off + sizeof(double) * nnz);
    L.keys_in = off; off = align256(off + sizeof(int32_t) * nnz);
    L.keys_out = off; off = align256(off + sizeof(int32_t) * nnz);
    L.perm_in = off; off = align256(off + sizeof(int32_t) * nnz);
    L.perm_out = off; off = align256(off + sizeof(int32_t) * nnz);
    L.rowidx = off; off = align256(off + sizeof(int32_t) * nnz);
    L.temp = off; off = align256(off + temp_bytes + 256);
    L.temp_bytes = temp_bytes + 256;
    L.total = off;
    return L;
}

// Build CSR(A^T) (= CSC of A) inside ws.  Column count of A^T rows = n.
hipError_t build_csc(const int64_t* rowptr, const int32_t* colind, const double* val, int64_t m,
                     int64_t n, int64_t nnz, char* ws, hipStream_t s) {
    const CscLayout L = csc_layout(m, n, nnz);
    int64_t* colptr = reinterpret_cast<int64_t*>(ws + L.colptr);
    int32_t* t_col = reinterpret_cast<int32_t*>(ws + L.t_col);
    double* t_val = reinterpret_cast<double*>(ws + L.t_val);
    int32_t* keys_in = reinterpret_cast<int32_t*>(ws + L.keys_in);
    int32_t* keys_out = reinterpret_cast<int32_t*>(ws + L.keys_out);
    int32_t* perm_in = reinterpret_cast<int32_t*>(ws + L.perm_in);
    int32_t* perm_out = reinterpret_cast<int32_t*>(ws + L.perm_out);
    int32_t* rowidx = reinterpret_cast<int32_t*>(ws + L.rowidx);
    hipError_t e;
    if (nnz > 0) {
        hipLaunchKernelGGL(csr_rowidx_kernel, dim3(static_cast<unsigned>(cdiv(m, 256))), dim3(256), 0,
                           s, rowptr, m, rowidx);
        hipLaunchKernelGGL(iota_kernel, dim3(static_cast<unsigned>(cdiv(nnz, 256))), dim3(256), 0, s,
                           perm_in, nnz);
        e = hipMemcpyAsync(keys_in, colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        size_t tb = L.temp_bytes;
        e = hipcub::DeviceRadixSort::SortPairs(ws + L.temp, tb, keys_in, keys_out, perm_in, perm_out,
                                               static_cast<int>(nnz), 0, 32, s);
        if (e != hipSuccess) return e;
    }
    const int64_t cnt = (nnz > n + 1 ? nnz : n + 1);
    hipLaunchKernelGGL(csc_finish_kernel, dim3(static_cast<unsigned>(cdiv(cnt, 256))), dim3(256), 0,
                       s, keys_out, perm_out, rowidx, val, nnz, n, colptr, t_col, t_val);
    return hipGetLastError();
}

void csc_views(int64_t m, int64_t n, int64_t nnz, char* ws, const int64_t** colptr,
               const int32_t** t_col, const double** t_val) {
    const CscLayout L = csc_layout(m, n, nnz);
    *colptr = reinterpret_cast<const int64_t*>(ws + L.colptr);
    *t_col = reinterpret_cast<const int32_t*>(ws + L.t_col);
    *t_val = reinterpret_cast<const double*>(ws + L.t_val);
}

}  // namespace qb
