// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64) for every product of the
// QB method: the sketch sweep G = A Omega, H = A^T G (Algorithm 4), EI's
// A Omega_i and A^T Q_i (Algorithm 2), and the tall-skinny block products
// B Omega_i, G_i - Q W, Q^T Q_i, Y^T Q, H_i^T - D B of Algorithm 4's block loop (eq. (23)).
//
//   out(i, j) = alpha * sum_k Aop(i, k) Bop(k, j) + beta * C0(i, j)
//
// Aop(i, k) = A[i*sai + k*sak] with either sak == 1 (layout 0, k contiguous: row-major
// A in A Omega) or sai == 1 (layout 1, i contiguous: A^T of a row-major A, or a
// column-major Q).  Bop(k, j) = B[k*sbk + j*sbj] with sbj == 1 (layout 0) or sbk == 1
// (layout 1).  Tiles are staged through LDS in the operand's own global orientation
// (no transposing stores) with pitches chosen so that the MFMA operand reads of a
// 32-lane pass hit 64 distinct banks.  A reduction over a long K can be split across
// workgroups (split-K); partial tiles are then summed in a fixed order by a second
// kernel, so results are bit-reproducible.  Optionally the epilogue emits per-row-tile
// column sums of squares of the output (used for ||B_i(j,:)||^2 and ||A Omega(:,j)||^2).
#include <cmath>

#include "kernels.h"

namespace qb {

struct GemmArgs {
    int64_t M, N, K;
    const double* A;
    int64_t lda;           // stride of the non-contiguous operand index
    const double* B;
    int64_t ldb;
    double alpha, beta;
    const double* C0;      // read when beta != 0
    int64_t c0_si, c0_sj;
    double* C;             // final output (nsplit == 1)
    int64_t c_si, c_sj;
    double* P;             // split-K partials, nsplit x M x N row-major (nsplit > 1)
    int64_t kchunk;        // K range per split (multiple of BK)
    double* colsq;         // [tiles_m][N] partial column sums of squares, or nullptr
    int tiles_m, tiles_n;
    int vec_a, vec_b;      // 16-byte aligned rows: double2 loads allowed
    const int* gate;       // if set and nonzero when the kernel starts, it does nothing
};

// Output element (row, col) inside a 16x16 f64 MFMA accumulator for lane l, slot r:
// slot r of lane l holds row 4 r + l / 16, column l mod 16 (measured on gfx950; the
// A operand is A(l mod 16, l / 16) and the B operand B(l / 16, l mod 16)).
QB_DEV int acc_row(int lane, int r) { return (r << 2) + (lane >> 4); }
QB_DEV int acc_col(int lane) { return lane & 15; }


// Staging of one operand tile of OUTER x INNER elements whose INNER index is contiguous
// in global memory (row stride ld).  Thread t owns the element pair at inner offset
// 2 (t mod INNER/2) of rows t div (INNER/2) + p RPP, p < PASSES.
template <int OUTER, int INNER, int NT>
struct Stage {
    static constexpr int TPR = INNER / 2;          // threads per row
    static constexpr int RPP = NT / TPR;           // rows per pass
    static constexpr int PASSES = OUTER / RPP;
    static_assert(NT % TPR == 0 && OUTER % RPP == 0, "staging shape");
    double2 r[PASSES];

    // Whole tile in bounds, 16-byte aligned rows: one double2 load per pass.
    QB_DEV void load_vec(const double* __restrict__ g, int64_t ld, int64_t o0, int64_t i0) {
        const int tid = threadIdx.x;
        const int ro = tid / TPR, ri = 2 * (tid % TPR);
        const double* p0 = g + (o0 + ro) * ld + i0 + ri;
#pragma unroll
        for (int p = 0; p < PASSES; ++p)
            r[p] = *reinterpret_cast<const double2*>(p0 + static_cast<int64_t>(p) * RPP * ld);
    }
    // Rows [o0, o0 + OUTER) limited by olim, inner [i0, i0 + INNER) limited by ilim;
    // out-of-range elements read as zero.
    QB_DEV void load_checked(const double* __restrict__ g, int64_t ld, int64_t o0, int64_t i0,
                             int64_t olim, int64_t ilim) {
        const int tid = threadIdx.x;
        const int ro = tid / TPR, ri = 2 * (tid % TPR);
        const double* p0 = g + (o0 + ro) * ld + i0 + ri;
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const int64_t o = o0 + ro + p * RPP;
            const int64_t i = i0 + ri;
            const double* q = p0 + static_cast<int64_t>(p) * RPP * ld;
            const bool ok = o < olim;
            r[p].x = ok && i < ilim ? q[0] : 0.0;
            r[p].y = ok && i + 1 < ilim ? q[1] : 0.0;
        }
    }
    template <int PITCH>
    QB_DEV void store(double* __restrict__ s) const {
        const int tid = threadIdx.x;
        const int ro = tid / TPR, ri = 2 * (tid % TPR);
#pragma unroll
        for (int p = 0; p < PASSES; ++p)
            *reinterpret_cast<double2*>(s + (ro + p * RPP) * PITCH + ri) = r[p];
    }
};

template <int BM, int BN, int BK, int WM, int WN, int AL, int BL>
struct GemmCfg {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int FM = TM / 16, FN = TN / 16;
    // layout 0 tiles are [BM][BK] (k contiguous), layout 1 tiles are [BK][BM]; the
    // pitches make a 32-lane pass of MFMA operand reads hit 64 distinct banks
    static constexpr int A_PITCH = AL == 0 ? BK + 2 : ((BM + 31) / 32) * 32 + 16;
    static constexpr int A_ROWS = AL == 0 ? BM : BK;
    static constexpr int A_INNER = AL == 0 ? BK : BM;
    static constexpr int B_PITCH = BL == 0 ? ((BN + 31) / 32) * 32 + 16 : BK + 2;
    static constexpr int B_ROWS = BL == 0 ? BK : BN;
    static constexpr int B_INNER = BL == 0 ? BN : BK;
    static_assert(TM % 16 == 0 && TN % 16 == 0 && (BK == 16 || BK == 32), "bad tile");
};

template <int BM, int BN, int BK, int WM, int WN, int AL, int BL, int OCC, int STAGES>
__global__ void __launch_bounds__(64 * WM * WN, OCC) gemm_f64_kernel(const GemmArgs g) {
    using C = GemmCfg<BM, BN, BK, WM, WN, AL, BL>;
    static_assert(STAGES == 1 || STAGES == 2, "one or two LDS stages");
    if (g.gate != nullptr && *g.gate != 0) return;
    constexpr int A_STAGE = C::A_ROWS * C::A_PITCH, B_STAGE = C::B_ROWS * C::B_PITCH;
    __shared__ __align__(16) double As[STAGES * A_STAGE];
    __shared__ __align__(16) double Bs[STAGES * B_STAGE];
    __shared__ double red[WM][BN];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int li = lane & 15, lk = lane >> 4;

    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int tile_m, tile_n;
    group_tiles(logical, g.tiles_m, g.tiles_n, tile_m, tile_n);
    const int64_t m0 = static_cast<int64_t>(tile_m) * BM;
    const int64_t n0 = static_cast<int64_t>(tile_n) * BN;
    const int64_t kb = static_cast<int64_t>(blockIdx.y) * g.kchunk;
    const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;

    v4d acc[C::FM][C::FN];
#pragma unroll
    for (int a = 0; a < C::FM; ++a)
#pragma unroll
        for (int b = 0; b < C::FN; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

    Stage<C::A_ROWS, C::A_INNER, C::NT> sa;
    Stage<C::B_ROWS, C::B_INNER, C::NT> sb;
    auto load_fast = [&](int64_t k0) {
        if (AL == 0) sa.load_vec(g.A, g.lda, m0, k0); else sa.load_vec(g.A, g.lda, k0, m0);
        if (BL == 0) sb.load_vec(g.B, g.ldb, k0, n0); else sb.load_vec(g.B, g.ldb, n0, k0);
    };
    auto load_checked = [&](int64_t k0) {
        if (AL == 0) sa.load_checked(g.A, g.lda, m0, k0, g.M, ke);
        else         sa.load_checked(g.A, g.lda, k0, m0, ke, g.M);
        if (BL == 0) sb.load_checked(g.B, g.ldb, k0, n0, ke, g.N);
        else         sb.load_checked(g.B, g.ldb, n0, k0, g.N, ke);
    };
    // tiles fully inside M x N with aligned rows stream their full K tiles through the
    // branch-free vector path; everything else (edge tiles, the K tail) is checked
    const bool fast = g.vec_a && g.vec_b && m0 + BM <= g.M && n0 + BN <= g.N;
    const int64_t kfull = fast ? kb + ((ke - kb) / BK) * BK : kb;   // end of the fast tiles

    const int wm0 = wm * C::TM, wn0 = wn * C::TN;
    // MFMA operands of k-step kk from one LDS stage
    auto read_ops = [&](const double* as, const double* bs, int kk, double (&a)[C::FM],
                        double (&b)[C::FN]) {
#pragma unroll
        for (int fm = 0; fm < C::FM; ++fm) {
            const int i = wm0 + fm * 16 + li;
            a[fm] = AL == 0 ? as[i * C::A_PITCH + kk + lk] : as[(kk + lk) * C::A_PITCH + i];
        }
#pragma unroll
        for (int fn = 0; fn < C::FN; ++fn) {
            const int j = wn0 + fn * 16 + li;
            b[fn] = BL == 0 ? bs[(kk + lk) * C::B_PITCH + j] : bs[j * C::B_PITCH + kk + lk];
        }
    };
    // BK/4 k-steps on one stage; the operands of step kk + 4 are read while the MFMAs
    // of step kk run
    auto compute = [&](const double* as, const double* bs) {
        double a0[C::FM], b0[C::FN], a1[C::FM], b1[C::FN];
        read_ops(as, bs, 0, a0, b0);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 8) {
            read_ops(as, bs, kk + 4, a1, b1);
#pragma unroll
            for (int fm = 0; fm < C::FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < C::FN; ++fn)
                    acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[fm], b0[fn], acc[fm][fn], 0, 0, 0);
            if (kk + 8 < BK) read_ops(as, bs, kk + 8, a0, b0);
#pragma unroll
            for (int fm = 0; fm < C::FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < C::FN; ++fn)
                    acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[fm], b1[fn], acc[fm][fn], 0, 0, 0);
        }
    };

    if (STAGES == 1) {
        for (int64_t k0 = kb; k0 < kfull; k0 += BK) {
            load_fast(k0);
            __syncthreads();
            sa.template store<C::A_PITCH>(As);
            sb.template store<C::B_PITCH>(Bs);
            __syncthreads();
            compute(As, Bs);
        }
        for (int64_t k0 = kfull; k0 < ke; k0 += BK) {
            load_checked(k0);
            __syncthreads();
            sa.template store<C::A_PITCH>(As);
            sb.template store<C::B_PITCH>(Bs);
            __syncthreads();
            compute(As, Bs);
        }
    } else {
        // two-stage ring over the fast tiles: tile t is read from stage t & 1 while tile
        // t + 1 is written to the other stage; one barrier per tile
        int st = 0;
        if (kb < kfull) {
            load_fast(kb);
            sa.template store<C::A_PITCH>(As);
            sb.template store<C::B_PITCH>(Bs);
            __syncthreads();
            int64_t k0 = kb;
            for (; k0 + BK < kfull; k0 += BK) {
                load_fast(k0 + BK);
                compute(As + st * A_STAGE, Bs + st * B_STAGE);
                sa.template store<C::A_PITCH>(As + (st ^ 1) * A_STAGE);
                sb.template store<C::B_PITCH>(Bs + (st ^ 1) * B_STAGE);
                __syncthreads();
                st ^= 1;
            }
            compute(As + st * A_STAGE, Bs + st * B_STAGE);
            st ^= 1;
        }
        for (int64_t k0 = kfull; k0 < ke; k0 += BK) {
            load_checked(k0);
            __syncthreads();
            sa.template store<C::A_PITCH>(As + st * A_STAGE);
            sb.template store<C::B_PITCH>(Bs + st * B_STAGE);
            __syncthreads();
            compute(As + st * A_STAGE, Bs + st * B_STAGE);
        }
    }

    // ---------------------------------------------------------------- epilogue
    if (gridDim.y > 1) {
        double* P = g.P + static_cast<int64_t>(blockIdx.y) * g.M * g.N;
#pragma unroll
        for (int fm = 0; fm < C::FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < C::FN; ++fn)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = m0 + wm0 + fm * 16 + acc_row(lane, r);
                    const int64_t j = n0 + wn0 + fn * 16 + acc_col(lane);
                    if (i < g.M && j < g.N) P[i * g.N + j] = acc[fm][fn][r];
                }
        return;
    }
    double csq[C::FN];
#pragma unroll
    for (int fn = 0; fn < C::FN; ++fn) csq[fn] = 0.0;
#pragma unroll
    for (int fm = 0; fm < C::FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < C::FN; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = m0 + wm0 + fm * 16 + acc_row(lane, r);
                const int64_t j = n0 + wn0 + fn * 16 + acc_col(lane);
                if (i < g.M && j < g.N) {
                    double v = g.alpha * acc[fm][fn][r];
                    if (g.beta != 0.0) v += g.beta * g.C0[i * g.c0_si + j * g.c0_sj];
                    g.C[i * g.c_si + j * g.c_sj] = v;
                    csq[fn] += v * v;
                }
            }
    if (g.colsq != nullptr) {
        // lanes l, l^16, l^32, l^48 share a column; then combine the WM waves in order
#pragma unroll
        for (int fn = 0; fn < C::FN; ++fn) {
            double v = csq[fn];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lk == 0) red[wm][wn0 + fn * 16 + li] = v;
        }
        __syncthreads();
        for (int j = tid; j < BN; j += C::NT) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < WM; ++w) t += red[w][j];
            if (n0 + j < g.N) g.colsq[static_cast<int64_t>(tile_m) * g.N + n0 + j] = t;
        }
    }
}

// Fixed-order sum of split-K partials for small outputs with many splits: 8 threads per
// element (thread r sums splits r, r + 8, ... in order), the 8 sums then added in the order
// r = 0..7 through LDS.  A wave reads 32 consecutive elements of two partials.
constexpr int kRedLanes = 8;
__global__ void __launch_bounds__(256)
splitk_reduce_wide_kernel(const double* __restrict__ P, int nsplit, int64_t M, int64_t N,
                          double alpha, double beta, const double* C0, int64_t c0_si,
                          int64_t c0_sj, double* C, int64_t c_si, int64_t c_sj) {
    constexpr int EPB = 256 / kRedLanes;   // elements per block
    __shared__ double part[kRedLanes][EPB];
    const int el = threadIdx.x % EPB, r = threadIdx.x / EPB;
    const int64_t mn = M * N;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * EPB + el;
    double t0 = 0.0, t1 = 0.0;
    if (e < mn) {
        int s = r;
        for (; s + kRedLanes < nsplit; s += 2 * kRedLanes) {
            t0 += P[s * mn + e];
            t1 += P[(s + kRedLanes) * mn + e];
        }
        if (s < nsplit) t0 += P[s * mn + e];
    }
    part[r][el] = t0 + t1;
    __syncthreads();
    if (r != 0 || e >= mn) return;
    double t = part[0][el];
#pragma unroll
    for (int q = 1; q < kRedLanes; ++q) t += part[q][el];
    const int64_t i = e / N, j = e % N;
    double v = alpha * t;
    if (beta != 0.0) v += beta * C0[i * c0_si + j * c0_sj];
    C[i * c_si + j * c_sj] = v;
}

// Fixed-order sum of split-K partials with the alpha / beta epilogue.
__global__ void __launch_bounds__(256)
splitk_reduce_kernel(const double* __restrict__ P, int nsplit, int64_t M, int64_t N,
                     double alpha, double beta, const double* C0, int64_t c0_si, int64_t c0_sj,
                     double* C, int64_t c_si, int64_t c_sj) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= M * N) return;
    // four interleaved partial sums keep four loads in flight; combined in fixed order
    const int64_t mn = M * N;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
    int s = 0;
    for (; s + 4 <= nsplit; s += 4) {
        t0 += P[(s + 0) * mn + e];
        t1 += P[(s + 1) * mn + e];
        t2 += P[(s + 2) * mn + e];
        t3 += P[(s + 3) * mn + e];
    }
    for (; s < nsplit; ++s) t0 += P[s * mn + e];
    const double t = (t0 + t1) + (t2 + t3);
    const int64_t i = e / N, j = e % N;
    double v = alpha * t;
    if (beta != 0.0) v += beta * C0[i * c0_si + j * c0_sj];
    C[i * c_si + j * c_sj] = v;
}

// Column sums of squares of a strided M x N output after a split-K reduction: partial
// g covers rows [g R, (g + 1) R).  Row-major outputs (sj == 1) put threads on columns;
// column-major outputs (si == 1) give each column a wave whose lanes stride the rows.
__global__ void __launch_bounds__(256)
colsq_strided_kernel(const double* __restrict__ C, int64_t M, int64_t N, int64_t si, int64_t sj,
                     int64_t rows_per_group, double* __restrict__ partial) {
    const int64_t g = blockIdx.x;
    const int64_t r0 = g * rows_per_group;
    const int64_t r1 = r0 + rows_per_group < M ? r0 + rows_per_group : M;
    if (sj == 1) {
        const int64_t j = static_cast<int64_t>(blockIdx.y) * 256 + threadIdx.x;
        if (j >= N) return;
        double t = 0.0;
        for (int64_t i = r0; i < r1; ++i) {
            const double v = C[i * si + j];
            t += v * v;
        }
        partial[g * N + j] = t;
    } else {
        const int64_t j = static_cast<int64_t>(blockIdx.y) * 4 + (threadIdx.x >> 6);
        const int lane = threadIdx.x & 63;
        if (j >= N) return;
        double t = 0.0;
        for (int64_t i = r0 + lane; i < r1; i += 64) {
            const double v = C[i + j * sj];
            t += v * v;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane == 0) partial[g * N + j] = t;
    }
}

// Epilogue-only "GEMM" for K == 0: out = beta * C0 (alpha * empty sum = 0).
__global__ void __launch_bounds__(256)
scale_copy_kernel(int64_t M, int64_t N, double beta, const double* C0, int64_t c0_si,
                  int64_t c0_sj, double* C, int64_t c_si, int64_t c_sj) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= M * N) return;
    const int64_t i = e / N, j = e % N;
    C[i * c_si + j * c_sj] = beta != 0.0 ? beta * C0[i * c0_si + j * c0_sj] : 0.0;
}

// ------------------------------------------------------------------------------ host

hipError_t launch_splitk_reduce(const GemmDesc& d, int nsplit, hipStream_t s) {
    const int64_t tot = d.M * d.N;
    if (nsplit >= 2 * kRedLanes && tot <= (int64_t(1) << 18)) {
        // few outputs, long reduction: spread each element over kRedLanes threads
        hipLaunchKernelGGL(splitk_reduce_wide_kernel, dim3(static_cast<unsigned>(cdiv(tot, 256 / kRedLanes))),
                           dim3(256), 0, s, d.ws, nsplit, d.M, d.N, d.alpha, d.beta, d.C0.p, d.C0.si,
                           d.C0.sj, d.C.p, d.C.si, d.C.sj);
    } else {
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(static_cast<unsigned>(cdiv(tot, 256))), dim3(256), 0,
                           s, d.ws, nsplit, d.M, d.N, d.alpha, d.beta, d.C0.p, d.C0.si, d.C0.sj, d.C.p,
                           d.C.si, d.C.sj);
    }
    return hipGetLastError();
}


template <int BM, int BN, int BK, int WM, int WN, int AL, int BL, int OCC, int STAGES>
static hipError_t run_cfg(const GemmDesc& d, hipStream_t s) {
    GemmArgs g{};
    g.M = d.M; g.N = d.N; g.K = d.K;
    g.A = d.A.p; g.lda = AL == 0 ? d.A.si : d.A.sj;
    g.B = d.B.p; g.ldb = BL == 0 ? d.B.si : d.B.sj;
    g.alpha = d.alpha; g.beta = d.beta;
    g.C0 = d.C0.p; g.c0_si = d.C0.si; g.c0_sj = d.C0.sj;
    g.C = d.C.p; g.c_si = d.C.si; g.c_sj = d.C.sj;
    g.vec_a = (reinterpret_cast<uintptr_t>(g.A) % 16 == 0) && (g.lda % 2 == 0);
    g.vec_b = (reinterpret_cast<uintptr_t>(g.B) % 16 == 0) && (g.ldb % 2 == 0);
    g.tiles_m = static_cast<int>(cdiv(d.M, BM));
    g.tiles_n = static_cast<int>(cdiv(d.N, BN));
    const int64_t tiles = static_cast<int64_t>(g.tiles_m) * g.tiles_n;
    int nsplit = 1;
    const int64_t ktiles = cdiv(d.K, BK);
    if (d.ws != nullptr && tiles < 512) {
        // few output tiles: spread the reduction over about 2048 workgroups (8 per compute
        // unit: the long reductions of the block loop stream Q from HBM and need the
        // occupancy to hide its latency)
        int64_t want = cdiv(2048, tiles);
        if (want > 128) want = 128;
        if (want > ktiles / 4) want = ktiles / 4;
        if (d.max_split > 0 && want > d.max_split) want = d.max_split;
        while (want > 1 && want * d.M * d.N > d.ws_elems) --want;
        if (want > 1) nsplit = static_cast<int>(want);
    } else if (d.ws != nullptr && BK == 16) {
        // the two-per-CU sketch tile: split K in 2, 4 or 6 until there are at least 2400
        // workgroups (measured on the 20000 x 15000 sketch products: G and H of 512 and
        // 1024 columns ran fastest with 4-6 splits; odd counts were slower)
        for (int ns = 2; ns <= 6; ns += 2) {
            if (tiles * (nsplit > 1 ? nsplit : 1) >= 2400) break;
            if (ktiles < 16 * ns || ns * d.M * d.N > d.ws_elems) break;
            nsplit = ns;
        }
    } else if (d.ws != nullptr) {
        // pick 1..4 K splits to shrink the idle tail of the last round of workgroups
        // (the split partials cost one extra pass over M x N); the resident workgroups
        // per CU follow from the LDS footprint
        using Cf = GemmCfg<BM, BN, BK, WM, WN, AL, BL>;
        constexpr int64_t lds = 8 * (STAGES * (Cf::A_ROWS * Cf::A_PITCH + Cf::B_ROWS * Cf::B_PITCH) +
                                     WM * BN);
        constexpr int64_t per_cu = (160 * 1024) / lds < 1 ? 1 : (160 * 1024) / lds;
        const int64_t slots = 256 * per_cu;
        double best = 0.0;
        for (int ns = 1; ns <= 4; ++ns) {
            if (ns > 1 && (ktiles < 16 * ns || ns * d.M * d.N > d.ws_elems)) break;
            const double work = static_cast<double>(tiles * ns) / slots;
            const double eff = work / std::ceil(work) * (1.0 - 0.02 * (ns - 1));
            if (eff > best + 1e-9) { best = eff; nsplit = ns; }
        }
    }
    g.kchunk = cdiv(cdiv(d.K, BK), nsplit) * BK;
    nsplit = static_cast<int>(cdiv(d.K, g.kchunk));
    if (nsplit < 1) nsplit = 1;
    g.P = d.ws;
    g.gate = d.gate;
    g.colsq = nsplit == 1 ? d.colsq : nullptr;   // fused only without a split
    if (d.colsq_groups) *d.colsq_groups = g.tiles_m;
    dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(nsplit));
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, WM, WN, AL, BL, OCC, STAGES>), grid, dim3(64 * WM * WN), 0,
                       s, g);
    if (nsplit > 1) {
        const hipError_t e = launch_splitk_reduce(d, nsplit, s);
        if (e != hipSuccess) return e;
        if (d.colsq != nullptr) {
            // at most tiles_m groups of rows, so the caller's [tiles_m][N] buffer fits
            const int64_t groups = g.tiles_m < 256 ? g.tiles_m : 256;
            const int64_t rpg = cdiv(d.M, groups);
            const int64_t ng = cdiv(d.M, rpg);
            dim3 cg(static_cast<unsigned>(ng),
                    static_cast<unsigned>(d.C.sj == 1 ? cdiv(d.N, 256) : cdiv(d.N, 4)));
            hipLaunchKernelGGL(colsq_strided_kernel, cg, dim3(256), 0, s, d.C.p, d.M, d.N, d.C.si,
                               d.C.sj, rpg, d.colsq);
            if (d.colsq_groups) *d.colsq_groups = static_cast<int>(ng);
        }
    }
    return hipGetLastError();
}

// Tile configuration for an M x N x K product: 0 tall-skinny (m x b panels) with at least
// 512 row tiles of 128 or a long reduction, 1 small output with a long reduction (split K)
// -- also the panels with fewer row tiles and a short reduction (the block loop's
// G_J - Q W and Q_i - Q Z), which run faster in 64-row tiles (measured: 20000 x 64 x 896
// in 77 us against 111 us, while 15000 x 64 x 20000 is slower) -- and 2 the sketch sweep.
static int shape_class(int64_t M, int64_t N, int64_t K) {
    if (N <= 64 && (M >= 512 * 128 || (M >= 4096 && K >= 4096))) return 0;
    if (N <= 64 || M <= 2048) return 1;
    return 2;
}

int64_t gemm_f64_colsq_groups(int64_t M, int64_t N) {
    return cdiv(M, N <= 64 || M <= 2048 ? 64 : 128);   // the most any K gives
}

// Class 0 (tall outputs of at most 64 columns) with a long reduction, e.g. the n x 64
// B_i = (A^T Q_i)^T of randQB_EI and trQRCP, takes the 16-deep two-stage ring, two workgroups
// per CU: 54.9 against 49.6 TFLOP/s on the 15000 x 64 x 20000 products with the 32-deep
// single-stage tile.  With a short one (the sparse workload's Q_i = Y R^-1 and
// B_i^T = S^T R_i^-1, 500000 x 50 x 50) the 32-deep tile measured no slower (902-944 against
// 961 us in traced runs).
// Class 1 (the block loop's k x 64 split-K products) measured the same either way and keeps
// its tile.
template <int AL, int BL>
static hipError_t dispatch_shape(const GemmDesc& d, hipStream_t s) {
    switch (shape_class(d.M, d.N, d.K)) {
        case 0:
            return d.K >= 4096 ? run_cfg<128, 64, 16, 4, 1, AL, BL, 2, 2>(d, s)
                               : run_cfg<128, 64, 32, 4, 1, AL, BL, 2, 1>(d, s);
        case 1: return run_cfg<64, 64, 32, 2, 2, AL, BL, 2, 1>(d, s);
        default: return run_cfg<128, 128, 16, 4, 2, AL, BL, 2, 2>(d, s);
    }
}

hipError_t gemm_f64(const GemmDesc& d, hipStream_t s) {
    if (d.M <= 0 || d.N <= 0) {
        if (d.colsq_groups) *d.colsq_groups = 0;
        return hipSuccess;
    }
    if (d.K <= 0) {
        if (d.colsq != nullptr) return hipErrorInvalidValue;
        const int64_t tot = d.M * d.N;
        hipLaunchKernelGGL(scale_copy_kernel, dim3(static_cast<unsigned>(cdiv(tot, 256))), dim3(256),
                           0, s, d.M, d.N, d.beta, d.C0.p, d.C0.si, d.C0.sj, d.C.p, d.C.si, d.C.sj);
        return hipGetLastError();
    }
    // narrow products (the block loop's m x b and n x b panels) on the register-fed kernels of
    // tsgemm.hip where they were measured faster: the panel form (column-major A) for
    // reductions of 132 .. 16384, and the reduction form (k-contiguous A, column-major B) for
    // reductions of 100000 and more.  Shorter reductions and wider outputs stay on the
    // LDS-tiled kernel below.
    if (d.colsq == nullptr && d.N <= 64 && d.K > 128) {
        // (the panel form splits only the rows: under 8192 of them a long reduction runs on
        // too few workgroups: 315 us at up to 1216 x 64 x 15000, where the split-K kernel
        // below takes a tenth of that)
        if (d.A.si == 1 && d.K <= 32768 && (d.M >= 8192 || d.K <= 4096) && ts_panel_dma_fits(d))
            return ts_panel_dma(d, 2, 4, 4, 1, s, 1);
        // k-contiguous A with a long reduction: k-contiguous B (Q^T Y, Q^T Q_i, Y^T Y), or a
        // row-major B under at least 4096 output rows (A Omega_i of randQB_EI: 703 against
        // 887 us at 20000 x 64 x 15000; W = B Omega_J of the sparse workload: 3.53 against
        // 4.03 ms at 7000 x 50 x 200000; at 1152 rows the tiled kernel was as fast)
        const bool red_b = d.B.si == 1 ? d.K >= 100000 : d.B.sj == 1 && d.M >= 4096 && d.K >= 8192;
        if (d.A.sj == 1 && red_b && ts_red_fits(d)) {
            // about 1024 workgroups (one per CU resident at a time), within the split buffer
            const int64_t tiles = cdiv(d.M, 64);
            int64_t ns = cdiv(1024, tiles);
            if (ns > 256) ns = 256;
            while (ns > 1 && (d.ws == nullptr || ns * d.M * d.N > d.ws_elems)) --ns;
            return ts_red(d, 4, 4, static_cast<int>(ns), s);
        }
    }
    const int al = d.A.sj == 1 ? 0 : 1;
    const int bl = d.B.sj == 1 ? 0 : 1;
    if ((al == 1 && d.A.si != 1) || (bl == 1 && d.B.si != 1)) return hipErrorInvalidValue;
    if (al == 0 && bl == 0) return dispatch_shape<0, 0>(d, s);
    if (al == 0 && bl == 1) return dispatch_shape<0, 1>(d, s);
    if (al == 1 && bl == 0) return dispatch_shape<1, 0>(d, s);
    return dispatch_shape<1, 1>(d, s);
}

}  // namespace qb
