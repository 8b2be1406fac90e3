// Precision form of the sketch sweep: A stored in BF16, G = A_q Omega_q and
// H = A_q^T G_q on BF16 matrix cores with FP32 accumulation, everything the block loop
// sees in FP64.  Theorem 1 applies to A_q exactly (||A_q||^2 is summed in FP64 from the
// stored values), and eq. (23) needs only H = A_q^T G for the same G the block loop uses,
// so G_q (the BF16 rounding of the FP32 product) is both the H operand and, dequantised,
// the G of the block loop; Omega_q likewise.
//
//   * f64 -> bf16 round-to-nearest-even from the binary64 bits (no double rounding);
//   * quantise + transpose Omega (n x w FP64) into Omega_q^T (w x n BF16) and the
//     dequantised Omega_q in place;
//   * ||A_q||^2 in FP64 from 16-byte loads of the stored values;
//   * the BF16 GEMM C(i, j) = sum_k A(i, k) B(j, k) on v_mfma_f32_32x32x16_bf16.  B is N x K
//     with K contiguous; A is either M x K with K contiguous (G = A_q Omega_q) or stored
//     as K rows of M contiguous elements (H = A_q^T G_q reads A_q in place: the tile is
//     transposed on its way into LDS, so A_q is never copied).  Two epilogues: G (FP64
//     dequantised BF16 rounding + the transposed BF16 copy + column sums of squares) and
//     H (FP64).
#include "kernels.h"

namespace qb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------ rounding

// binary64 -> bfloat16 bits, round to nearest, ties to even (finite inputs)
QB_DEV uint16_t f64_to_bf16_rne(double x) {
    const uint64_t u = static_cast<uint64_t>(__double_as_longlong(x));
    const uint16_t sign = static_cast<uint16_t>((u >> 48) & 0x8000u);
    const int e64 = static_cast<int>((u >> 52) & 0x7FF);
    const uint64_t mant = u & 0x000FFFFFFFFFFFFFull;
    if (e64 == 0x7FF) return static_cast<uint16_t>(sign | 0x7F80u | (mant ? 0x40u : 0u));
    if (e64 == 0 && mant == 0) return sign;
    int e = e64 - 1023 + 127;   // bf16 biased exponent of a normal result
    // significand with the implicit bit: 53 bits
    uint64_t sig = (e64 == 0 ? mant : (mant | (1ull << 52)));
    int shift = 45;                       // keep 8 significant bits (1 + 7)
    if (e <= 0) {                         // bf16 subnormal: fewer bits survive
        shift += 1 - e;
        e = 0;
    }
    uint64_t q, rem, half;
    if (shift >= 64) {
        q = 0; rem = sig; half = ~0ull;   // below half of the smallest subnormal
    } else {
        q = sig >> shift;
        rem = sig & ((1ull << shift) - 1);
        half = 1ull << (shift - 1);
    }
    if (rem > half || (rem == half && (q & 1))) ++q;
    // q holds 1.mmmmmmm (normal) or 0.mmmmmmm (subnormal); carry may bump the exponent
    uint32_t bits;
    if (e == 0) {
        bits = static_cast<uint32_t>(q);  // q == 0x80 means the smallest normal
    } else {
        if (q >= 0x100) { q >>= 1; ++e; }
        if (e >= 0xFF) return static_cast<uint16_t>(sign | 0x7F80u);
        bits = (static_cast<uint32_t>(e) << 7) | static_cast<uint32_t>(q & 0x7F);
    }
    return static_cast<uint16_t>(sign | bits);
}

QB_DEV double bf16_to_f64(uint16_t h) {
    return static_cast<double>(__uint_as_float(static_cast<uint32_t>(h) << 16));
}

// binary32 -> bfloat16 bits, round to nearest, ties to even (finite inputs)
QB_DEV uint16_t f32_to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ------------------------------------------------------------------ small kernels

// Omega (n x w FP64, row-major, ld w) -> Omega_q^T (w x n BF16, ld ldt) and Omega
// replaced by its dequantised BF16 rounding.  64 x 64 tiles through LDS.
__global__ void __launch_bounds__(256)
quant_transpose_omega_kernel(double* __restrict__ om, int64_t n, int64_t w,
                             uint16_t* __restrict__ omT, int64_t ldt) {
    __shared__ uint16_t tile[64][66];
    const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 64, c0 = static_cast<int64_t>(blockIdx.x) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = r0 + r, j = c0 + tx;
        uint16_t h = 0;
        if (i < n && j < w) {
            h = f64_to_bf16_rne(om[i * w + j]);
            om[i * w + j] = bf16_to_f64(h);
        }
        tile[r][tx] = h;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t j = c0 + r, i = r0 + tx;
        if (j < w && i < n) omT[j * ldt + i] = tile[tx][r];
    }
}

// Partial sums of squares (FP64) of the BF16 values of an m x n matrix: the squares of
// BF16 values are exact in FP64.  Workgroup g owns rows g, g + G, ...; 16-byte loads when
// every row starts 16-byte aligned.
__global__ void __launch_bounds__(256)
sumsq_bf16_partial(const uint16_t* __restrict__ a, int64_t m, int64_t n, int64_t lda, int vec,
                   double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc = 0.0;
    const int64_t nv = vec ? n / 8 : 0;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        const uint16_t* row = a + i * lda;
        for (int64_t c = threadIdx.x; c < nv; c += blockDim.x) {
            const uint4 q = *reinterpret_cast<const uint4*>(row + 8 * c);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double lo = static_cast<double>(__uint_as_float(w[e] << 16));
                const double hi = static_cast<double>(__uint_as_float(w[e] & 0xFFFF0000u));
                acc += lo * lo;
                acc += hi * hi;
            }
        }
        for (int64_t j = 8 * nv + threadIdx.x; j < n; j += blockDim.x) {
            const double v = bf16_to_f64(row[j]);
            acc += v * v;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// ------------------------------------------------------------------ BF16 GEMM

struct Bf16GemmArgs {
    int64_t M, N, K;
    const uint16_t* A;   // a_km == 0: M x K, element (i, k) at A[i * lda + k]
                         // a_km == 1: element (i, k) at A[k * lda + i]
    int64_t lda;
    const uint16_t* B;   // N x K, element (j, k) at B[j * ldb + k]
    int64_t ldb;
    double* out;         // M x N FP64, row stride ldo
    int64_t ldo;
    uint16_t* outT;      // G epilogue: N x M BF16 copy, row stride ldt
    int64_t ldt;
    double* colsq;       // G epilogue: [tiles_m][N] column sums of squares
    int tiles_m, tiles_n;
    int vec;             // 16-byte aligned operands with row strides divisible by 8
};

// Slot r of lane l of a 32x32 f32 accumulator holds row 8 (r / 4) + 4 (l / 32) + r mod 4,
// column l mod 32 (measured on gfx950).  Operand lane l supplies row (or column) l mod 32
// and 8 consecutive k starting at 8 (l / 32) of the 16-wide k step.
QB_DEV int acc32_row(int lane, int r) { return ((r >> 2) << 3) + ((lane >> 5) << 2) + (r & 3); }

// LDS tiles hold rows of BK elements (K contiguous) with a pitch of BK + 8; the 16-byte
// chunk c of row r sits at chunk position c ^ ((r / 16) mod (BK / 8)).  The operand reads
// (32 rows, one chunk) and the transposed 8-byte stores of the K-major A path (8 rows a
// thread, 32 row octets a wave) then spread over all banks.
template <int BK>
QB_DEV int lds_off(int row, int chunk) {
    constexpr int PITCH = BK + 8, CPR = BK / 8;
    return row * PITCH + 8 * (chunk ^ ((row >> 4) & (CPR - 1)));
}

QB_DEV uint32_t pack_lo(uint32_t a, uint32_t b) { return (a & 0xFFFFu) | (b << 16); }
QB_DEV uint32_t pack_hi(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xFFFF0000u); }

template <int BM, int BN, int BK, int WM, int WN, int EPI, bool AKM>
__global__ void __launch_bounds__(64 * WM * WN, (64 * WM * WN >= 512 ? 1 : 2))
gemm_bf16_kernel(const Bf16GemmArgs g) {
    constexpr int NT = 64 * WM * WN;
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
    constexpr int PITCH = BK + 8;
    constexpr int CPR = BK / 8;                         // 16-byte chunks per tile row
    constexpr int PA = BM * CPR / NT, PB = BN * CPR / NT;
    static_assert(BM * CPR % NT == 0 && BN * CPR % NT == 0 && BK % 16 == 0, "tile shape");
    static_assert(!AKM || ((BM / 8) * (BK / 4) == NT && PA == 4), "K-major A: one k-quad x m-octet per thread");
    __shared__ __align__(16) uint16_t As[2][BM * PITCH];
    __shared__ __align__(16) uint16_t Bs[2][BN * PITCH];
    __shared__ double red[WM][BN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    const int tile_m = logical / g.tiles_n, tile_n = logical % g.tiles_n;
    const int64_t m0 = static_cast<int64_t>(tile_m) * BM, n0 = static_cast<int64_t>(tile_n) * BN;
    const bool fast = g.vec && m0 + BM <= g.M && n0 + BN <= g.N;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f32x16{};

    // K-major A: thread owns rows k0 + 4 kq .. + 3 and columns m0 + 8 mo .. + 7
    const int mo = tid % (BM / 8), kq = tid / (BM / 8);
    uint4 ra[PA], rb[PB];
    auto gather8 = [](const uint16_t* p, int64_t lim) {   // 8 elements, the first lim valid
        uint16_t t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = e < lim ? p[e] : 0;
        return uint4{t[0] | (uint32_t(t[1]) << 16), t[2] | (uint32_t(t[3]) << 16),
                     t[4] | (uint32_t(t[5]) << 16), t[6] | (uint32_t(t[7]) << 16)};
    };
    auto load = [&](int64_t k0) {
        const bool kin = k0 + BK <= g.K;
        if constexpr (AKM) {
#pragma unroll
            for (int q = 0; q < PA; ++q) {
                const int64_t gk = k0 + 4 * kq + q, gi = m0 + 8 * mo;
                if (fast && kin) {
                    ra[q] = *reinterpret_cast<const uint4*>(g.A + gk * g.lda + gi);
                } else {
                    const int64_t lim = gk < g.K ? g.M - gi : 0;
                    ra[q] = gather8(g.A + (gk < g.K ? gk : 0) * g.lda + gi, lim);
                }
            }
        } else {
#pragma unroll
            for (int p = 0; p < PA; ++p) {
                const int c = tid + p * NT, row = c / CPR, col = (c % CPR) * 8;
                const int64_t gi = m0 + row, gk = k0 + col;
                if (fast && kin)
                    ra[p] = *reinterpret_cast<const uint4*>(g.A + gi * g.lda + gk);
                else
                    ra[p] = gather8(g.A + (gi < g.M ? gi : 0) * g.lda + gk, gi < g.M ? g.K - gk : 0);
            }
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int c = tid + p * NT, row = c / CPR, col = (c % CPR) * 8;
            const int64_t gj = n0 + row, gk = k0 + col;
            if (fast && kin)
                rb[p] = *reinterpret_cast<const uint4*>(g.B + gj * g.ldb + gk);
            else
                rb[p] = gather8(g.B + (gj < g.N ? gj : 0) * g.ldb + gk, gj < g.N ? g.K - gk : 0);
        }
    };
    auto store = [&](int st) {
        if constexpr (AKM) {
            // transpose the 4 x 8 block: row 8 mo + e of the tile gets k 4 kq .. 4 kq + 3
            const uint32_t w0[4] = {ra[0].x, ra[0].y, ra[0].z, ra[0].w};
            const uint32_t w1[4] = {ra[1].x, ra[1].y, ra[1].z, ra[1].w};
            const uint32_t w2[4] = {ra[2].x, ra[2].y, ra[2].z, ra[2].w};
            const uint32_t w3[4] = {ra[3].x, ra[3].y, ra[3].z, ra[3].w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int r_even = 8 * mo + 2 * h;
                const uint2 ev{pack_lo(w0[h], w1[h]), pack_lo(w2[h], w3[h])};
                const uint2 od{pack_hi(w0[h], w1[h]), pack_hi(w2[h], w3[h])};
                *reinterpret_cast<uint2*>(&As[st][lds_off<BK>(r_even, kq >> 1) + 4 * (kq & 1)]) = ev;
                *reinterpret_cast<uint2*>(&As[st][lds_off<BK>(r_even + 1, kq >> 1) + 4 * (kq & 1)]) = od;
            }
        } else {
#pragma unroll
            for (int p = 0; p < PA; ++p) {
                const int c = tid + p * NT, row = c / CPR, ch = c % CPR;
                *reinterpret_cast<uint4*>(&As[st][lds_off<BK>(row, ch)]) = ra[p];
            }
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int c = tid + p * NT, row = c / CPR, ch = c % CPR;
            *reinterpret_cast<uint4*>(&Bs[st][lds_off<BK>(row, ch)]) = rb[p];
        }
    };
    const int wm0 = wm * TM, wn0 = wn * TN;
    const int lr = lane & 31, lch = lane >> 5;
    auto compute = [&](int st) {
#pragma unroll
        for (int kk = 0; kk < BK / 8; kk += 2) {
            bf16x8 a[FM], b[FN];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
                a[fm] = *reinterpret_cast<const bf16x8*>(&As[st][lds_off<BK>(wm0 + fm * 32 + lr, kk + lch)]);
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
                b[fn] = *reinterpret_cast<const bf16x8*>(&Bs[st][lds_off<BK>(wn0 + fn * 32 + lr, kk + lch)]);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn)
                    acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[fm], b[fn], acc[fm][fn], 0, 0, 0);
        }
    };

    if (g.K > 0) {
        load(0);
        store(0);
        __syncthreads();
        int st = 0;
        for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
            const bool more = k0 + BK < g.K;
            if (more) load(k0 + BK);
            compute(st);
            if (more) store(st ^ 1);
            __syncthreads();
            st ^= 1;
        }
    }

    // epilogue
    double csq[FN];
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) csq[fn] = 0.0;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t i = m0 + wm0 + fm * 32 + acc32_row(lane, r);
                const int64_t j = n0 + wn0 + fn * 32 + (lane & 31);
                if (i < g.M && j < g.N) {
                    if (EPI == 0) {
                        g.out[i * g.ldo + j] = static_cast<double>(acc[fm][fn][r]);
                    } else {
                        const uint16_t h = f32_to_bf16_rne(acc[fm][fn][r]);
                        const double v = bf16_to_f64(h);
                        g.out[i * g.ldo + j] = v;
                        g.outT[j * g.ldt + i] = h;
                        csq[fn] += v * v;
                    }
                }
            }
    if (EPI == 1 && g.colsq != nullptr) {
        // lanes l and l ^ 32 share a column; then the WM waves in order
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
            double v = csq[fn];
            v += __shfl_xor(v, 32, 64);
            if (lane < 32) red[wm][wn0 + fn * 32 + lane] = v;
        }
        __syncthreads();
        for (int j = tid; j < BN; j += NT) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < WM; ++w) t += red[w][j];
            if (n0 + j < g.N) g.colsq[static_cast<int64_t>(tile_m) * g.N + n0 + j] = t;
        }
    }
}

// ------------------------------------------------------------------ host

hipError_t launch_quant_transpose_omega(double* om, int64_t n, int64_t w, uint16_t* omT,
                                        int64_t ldt, hipStream_t s) {
    if (n <= 0 || w <= 0) return hipSuccess;
    dim3 grid(static_cast<unsigned>(cdiv(w, 64)), static_cast<unsigned>(cdiv(n, 64)));
    hipLaunchKernelGGL(quant_transpose_omega_kernel, grid, dim3(256), 0, s, om, n, w, omT, ldt);
    return hipGetLastError();
}

hipError_t launch_sumsq_bf16(const uint16_t* a, int64_t m, int64_t n, int64_t lda,
                             double* scratch, double* out, hipStream_t s) {
    const int64_t g = m < 1024 ? m : 1024;
    const int vec = (reinterpret_cast<uintptr_t>(a) % 16 == 0) && (lda % 8 == 0);
    hipLaunchKernelGGL(sumsq_bf16_partial, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, a, m,
                       n, lda, vec, scratch);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_vector(scratch, g, out, s);
}

namespace {

// Tile 256 x 256 (8 waves of 128 x 64) when the problem has at least one such tile per
// compute unit, else 128 x 128 (4 waves of 64 x 64).
constexpr int kBigTile = 256, kSmallTile = 128;

bool use_big(int64_t M, int64_t N) { return cdiv(M, kBigTile) * cdiv(N, kBigTile) >= 256; }

}  // namespace

int64_t bf16_gemm_row_groups(int64_t M, int64_t N) {
    return cdiv(M, use_big(M, N) ? kBigTile : kSmallTile);
}

hipError_t gemm_bf16(int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t lda, bool a_km,
                     const uint16_t* B, int64_t ldb, double* out, int64_t ldo, uint16_t* outT,
                     int64_t ldt, double* colsq, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    // the two products of the sketch: G (K-contiguous A, G epilogue) and H (K-major A,
    // FP64 epilogue)
    if (a_km == (outT != nullptr)) return hipErrorInvalidValue;
    Bf16GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb;
    g.out = out; g.ldo = ldo; g.outT = outT; g.ldt = ldt; g.colsq = colsq;
    g.vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (reinterpret_cast<uintptr_t>(B) % 16 == 0) &&
            (lda % 8 == 0) && (ldb % 8 == 0);
    const bool big = use_big(M, N);
    const int t = big ? kBigTile : kSmallTile;
    g.tiles_m = static_cast<int>(cdiv(M, t));
    g.tiles_n = static_cast<int>(cdiv(N, t));
    dim3 grid(static_cast<unsigned>(static_cast<int64_t>(g.tiles_m) * g.tiles_n));
    if (big) {
        if (a_km)
            hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 64, 2, 4, 0, true>), grid, dim3(512), 0, s, g);
        else
            hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 64, 2, 4, 1, false>), grid, dim3(512), 0, s, g);
    } else {
        if (a_km)
            hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 64, 2, 2, 0, true>), grid, dim3(256), 0, s, g);
        else
            hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 64, 2, 2, 1, false>), grid, dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

}  // namespace qb
