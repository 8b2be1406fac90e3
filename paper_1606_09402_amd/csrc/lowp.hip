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
#include <type_traits>

#include "kernels.h"

namespace qb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// Power-of-two scale of Omega before its e4m3 rounding in the e4m3 form: the generator's
// Gaussians stay below 9 in magnitude, so 2^5 Omega is inside the format's range (448).
constexpr double kOmegaE4m3Scale = 32.0;

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

// OCP e4m3fn byte -> bfloat16 bits (exact: 3 significand bits, exponents 2^-9 .. 2^8).
// Normal bytes keep their significand and rebias the exponent (bias 7 -> 127); the
// subnormals m 2^-9 (m = 1..7) are renormalised.  The NaN byte does not occur in data.
QB_DEV uint32_t e4m3_to_bf16(uint32_t v) {
    const uint32_t s = (v & 0x80u) << 8;
    const uint32_t mag = v & 0x7Fu, m = v & 7u;
    const uint32_t normal = (mag << 4) + 0x3C00u;   // (e + 120) << 7 | m << 4
    // m 2^-9: the binary32 value m with its exponent lowered by 9, truncated to 16 bits
    const uint32_t sub = (__float_as_uint(static_cast<float>(m)) - (9u << 23)) >> 16;
    return s | (mag >= 8u ? normal : (m != 0u ? sub : 0u));
}

// 8 e4m3 bytes -> 8 bfloat16 values (same order).  v_cvt_pk_f32_fp8 widens two OCP e4m3
// bytes of a word exactly to binary32 (gfx950 converts the OCP format); an e4m3 value has
// 3 significand bits, so its bfloat16 is the high half of that binary32, and one v_perm_b32
// packs two high halves.  Two conversions and one permute per 4 values.
QB_DEV uint32_t pack_hi16(float lo, float hi) {
    return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
}

QB_DEV uint4 e4m3x8_to_bf16x8(uint2 q) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 a = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(q.x), false);
    const f32x2 b = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(q.x), true);
    const f32x2 c = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(q.y), false);
    const f32x2 d = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(q.y), true);
    return uint4{pack_hi16(a[0], a[1]), pack_hi16(b[0], b[1]), pack_hi16(c[0], c[1]), pack_hi16(d[0], d[1])};
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

// binary64 -> OCP e4m3fn byte, round to nearest, ties to even (finite inputs): 4 significant
// bits for normal results (exponents 2^-6 .. 2^8), multiples of 2^-9 below 2^-6; a result
// beyond 448 has no representation and gives the NaN byte.
QB_DEV uint8_t f64_to_e4m3_rne(double x) {
    const uint64_t u = static_cast<uint64_t>(__double_as_longlong(x));
    const uint32_t sign = static_cast<uint32_t>((u >> 56) & 0x80u);
    const int e64 = static_cast<int>((u >> 52) & 0x7FF);
    const uint64_t mant = u & 0x000FFFFFFFFFFFFFull;
    if (e64 == 0x7FF) return static_cast<uint8_t>(sign | 0x7Fu);
    if (e64 == 0 && mant == 0) return static_cast<uint8_t>(sign);
    int e = e64 - 1023 + 7;                    // e4m3 biased exponent of a normal result
    const uint64_t sig = e64 == 0 ? mant : (mant | (1ull << 52));
    int shift = 49;                            // keep 4 significant bits (1 + 3)
    if (e <= 0) {                              // subnormal result
        shift += 1 - e;
        e = 0;
    }
    uint64_t q = 0;
    if (shift < 64) {
        q = sig >> shift;
        const uint64_t rem = sig & ((1ull << shift) - 1), half = 1ull << (shift - 1);
        if (rem > half || (rem == half && (q & 1))) ++q;
    }
    uint32_t bits;
    if (e == 0) {
        bits = static_cast<uint32_t>(q);       // q == 8 is the smallest normal, 0x08
    } else {
        if (q >= 16) { q >>= 1; ++e; }
        if (e > 15 || (e == 15 && (q & 7) == 7)) return static_cast<uint8_t>(sign | 0x7Fu);
        bits = (static_cast<uint32_t>(e) << 3) | static_cast<uint32_t>(q & 7);
    }
    return static_cast<uint8_t>(sign | bits);
}

// Value of an e4m3fn byte (not NaN) as binary64.
QB_DEV double e4m3_to_f64(uint8_t v) {
    const int e = (v >> 3) & 15, m = v & 7;
    const double mag = e == 0 ? ldexp(static_cast<double>(m), -9) : ldexp(static_cast<double>(8 + m), e - 10);
    return (v & 0x80) ? -mag : mag;
}

// The e4m3 form's Omega: Omega (n x w FP64) -> the bytes e4m3(2^5 Omega) transposed (w x n,
// ld ldt8), the same values / 2^5 in bfloat16 transposed (w x n, ld ldt: exact, e4m3 values
// are bfloat16 values), and Omega replaced by the dequantised e4m3(2^5 Omega) / 2^5.
__global__ void __launch_bounds__(256)
quant_transpose_omega_e4m3_kernel(double* __restrict__ om, int64_t n, int64_t w,
                                  uint16_t* __restrict__ omT, int64_t ldt, uint8_t* __restrict__ omT8,
                                  int64_t ldt8) {
    __shared__ uint8_t tile[64][68];
    const int64_t r0 = static_cast<int64_t>(blockIdx.y) * 64, c0 = static_cast<int64_t>(blockIdx.x) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = r0 + r, j = c0 + tx;
        uint8_t q = 0;
        if (i < n && j < w) {
            q = f64_to_e4m3_rne(om[i * w + j] * kOmegaE4m3Scale);
            om[i * w + j] = e4m3_to_f64(q) / kOmegaE4m3Scale;
        }
        tile[r][tx] = q;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t j = c0 + r, i = r0 + tx;
        if (j < w && i < n) {
            const uint8_t q = tile[tx][r];
            omT8[j * ldt8 + i] = q;
            omT[j * ldt + i] = f64_to_bf16_rne(e4m3_to_f64(q) / kOmegaE4m3Scale);
        }
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

// Partial sums of squares (FP64) of an e4m3 matrix with power-of-two row scales:
// (2^e_i v)^2 is exact in FP64.  8-byte loads when every row starts 8-byte aligned.
__global__ void __launch_bounds__(256)
sumsq_fp8_partial(const uint8_t* __restrict__ a, int64_t m, int64_t n, int64_t lda, int vec,
                  const int32_t* __restrict__ row_exp, double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc = 0.0;
    const int64_t nv = vec ? n / 8 : 0;
    for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
        const uint8_t* row = a + i * lda;
        double r = 0.0;
        for (int64_t c = threadIdx.x; c < nv; c += blockDim.x) {
            const uint4 h = e4m3x8_to_bf16x8(*reinterpret_cast<const uint2*>(row + 8 * c));
            const uint32_t w[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double lo = static_cast<double>(__uint_as_float(w[e] << 16));
                const double hi = static_cast<double>(__uint_as_float(w[e] & 0xFFFF0000u));
                r += lo * lo;
                r += hi * hi;
            }
        }
        for (int64_t j = 8 * nv + threadIdx.x; j < n; j += blockDim.x) {
            const double v = static_cast<double>(__uint_as_float(e4m3_to_bf16(row[j]) << 16));
            r += v * v;
        }
        acc += ldexp(r, 2 * row_exp[i]);
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
                         // (bytes of e4m3 values when the kernel reads an FP8 A)
    int64_t lda;
    const uint16_t* B;   // N x K, element (j, k) at B[j * ldb + k]
    int64_t ldb;
    double* out;         // M x N FP64, row stride ldo
    int64_t ldo;
    uint16_t* outT;      // G epilogue: N x M BF16 copy, row stride ldt
    int64_t ldt;
    double* colsq;       // G epilogue: [tiles_m][N] column sums of squares
    const int32_t* row_exp;  // G epilogue of an FP8 A: output row i scaled by 2^row_exp[i]
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

template <int BM, int BN, int BK, int WM, int WN, int EPI, bool AKM, bool AF8>
__global__ void __launch_bounds__(64 * WM * WN, (64 * WM * WN >= 512 ? 1 : 2))
gemm_bf16_kernel(const Bf16GemmArgs g) {
    constexpr int NT = 64 * WM * WN;
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
    constexpr int PITCH = BK + 8;
    constexpr int CPR = BK / 8;                         // 16-byte chunks per tile row
    constexpr int PA = BM * CPR / NT, PB = BN * CPR / NT;
    static_assert(BM * CPR % NT == 0 && BN * CPR % NT == 0 && BK % 16 == 0, "tile shape");
    // K-major A: the BM/8 x BK/4 blocks of 4 (k) x 8 (m) elements are dealt out to the
    // threads, PA/4 blocks each
    static_assert(!AKM || ((BM / 8) * (BK / 4) % NT == 0 && PA == 4 * ((BM / 8) * (BK / 4) / NT)),
                  "K-major A: whole 4 x 8 blocks per thread");
    __shared__ __align__(16) uint16_t As[2][BM * PITCH];
    __shared__ __align__(16) uint16_t Bs[2][BN * PITCH];
    __shared__ double red[WM][BN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int tile_m, tile_n;
    group_tiles(logical, g.tiles_m, g.tiles_n, tile_m, tile_n);
    const int64_t m0 = static_cast<int64_t>(tile_m) * BM, n0 = static_cast<int64_t>(tile_n) * BN;
    const bool fast = g.vec && m0 + BM <= g.M && n0 + BN <= g.N;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f32x16{};

    // K-major A: block u of this thread covers rows k0 + 4 kq(u) .. + 3 and columns
    // m0 + 8 mo(u) .. + 7
    auto blk_mo = [&](int u) { return (tid + u * NT) % (BM / 8); };
    auto blk_kq = [&](int u) { return (tid + u * NT) / (BM / 8); };
    // staging registers: 8 elements per entry (bfloat16, or e4m3 bytes widened at the store)
    using RawA = typename std::conditional<AF8, uint2, uint4>::type;
    RawA ra[PA];
    uint4 rb[PB];
    auto gather8 = [](const uint16_t* p, int64_t lim) {   // 8 elements, the first lim valid
        uint16_t t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = e < lim ? p[e] : 0;
        return uint4{t[0] | (uint32_t(t[1]) << 16), t[2] | (uint32_t(t[3]) << 16),
                     t[4] | (uint32_t(t[5]) << 16), t[6] | (uint32_t(t[7]) << 16)};
    };
    const uint8_t* A8 = reinterpret_cast<const uint8_t*>(g.A);
    auto gather8_f8 = [](const uint8_t* p, int64_t lim) {   // 8 e4m3 bytes, the first lim valid
        uint32_t t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = e < lim ? p[e] : 0u;
        return uint2{t[0] | (t[1] << 8) | (t[2] << 16) | (t[3] << 24),
                     t[4] | (t[5] << 8) | (t[6] << 16) | (t[7] << 24)};
    };
    // 8 consecutive elements of A starting at element offset off (first lim valid)
    auto loadA8 = [&](int64_t off, bool full, int64_t lim) -> RawA {
        if constexpr (AF8) {
            return full ? *reinterpret_cast<const uint2*>(A8 + off) : gather8_f8(A8 + off, lim);
        } else {
            return full ? *reinterpret_cast<const uint4*>(g.A + off) : gather8(g.A + off, lim);
        }
    };
    auto widen = [](const RawA& r) -> uint4 {
        if constexpr (AF8) return e4m3x8_to_bf16x8(r);
        else return r;
    };
    auto load = [&](int64_t k0) {
        const bool kin = k0 + BK <= g.K;
        if constexpr (AKM) {
#pragma unroll
            for (int q = 0; q < PA; ++q) {
                const int64_t gk = k0 + 4 * blk_kq(q / 4) + q % 4, gi = m0 + 8 * blk_mo(q / 4);
                const bool full = fast && kin;
                const int64_t lim = gk < g.K ? g.M - gi : 0;
                ra[q] = loadA8((full || gk < g.K ? gk : 0) * g.lda + gi, full, lim);
            }
        } else {
#pragma unroll
            for (int p = 0; p < PA; ++p) {
                const int c = tid + p * NT, row = c / CPR, col = (c % CPR) * 8;
                const int64_t gi = m0 + row, gk = k0 + col;
                const bool full = fast && kin;
                ra[p] = loadA8((full || gi < g.M ? gi : 0) * g.lda + gk, full, gi < g.M ? g.K - gk : 0);
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
            // transpose each 4 x 8 block: row 8 mo + e of the tile gets k 4 kq .. 4 kq + 3
#pragma unroll
            for (int u = 0; u < PA / 4; ++u) {
                const int mo = blk_mo(u), kq = blk_kq(u);
                const uint4 c0 = widen(ra[4 * u]), c1 = widen(ra[4 * u + 1]), c2 = widen(ra[4 * u + 2]),
                            c3 = widen(ra[4 * u + 3]);
                const uint32_t w0[4] = {c0.x, c0.y, c0.z, c0.w};
                const uint32_t w1[4] = {c1.x, c1.y, c1.z, c1.w};
                const uint32_t w2[4] = {c2.x, c2.y, c2.z, c2.w};
                const uint32_t w3[4] = {c3.x, c3.y, c3.z, c3.w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int r_even = 8 * mo + 2 * h;
                    const uint2 ev{pack_lo(w0[h], w1[h]), pack_lo(w2[h], w3[h])};
                    const uint2 od{pack_hi(w0[h], w1[h]), pack_hi(w2[h], w3[h])};
                    *reinterpret_cast<uint2*>(&As[st][lds_off<BK>(r_even, kq >> 1) + 4 * (kq & 1)]) = ev;
                    *reinterpret_cast<uint2*>(&As[st][lds_off<BK>(r_even + 1, kq >> 1) + 4 * (kq & 1)]) = od;
                }
            }
        } else {
#pragma unroll
            for (int p = 0; p < PA; ++p) {
                const int c = tid + p * NT, row = c / CPR, ch = c % CPR;
                *reinterpret_cast<uint4*>(&As[st][lds_off<BK>(row, ch)]) = widen(ra[p]);
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
                    } else if (AF8) {
                        // G_q = bf16(2^e_i (A8 Omega_q)(i, j)); the H operand carries the row
                        // scale once more, 2^e_i G_q, so that A8^T (that) = A_q^T G_q
                        const int e = g.row_exp[i];
                        const uint16_t h = f32_to_bf16_rne(ldexpf(acc[fm][fn][r], e));
                        const double v = bf16_to_f64(h);
                        g.out[i * g.ldo + j] = v;
                        g.outT[j * g.ldt + i] =
                            static_cast<uint16_t>(__float_as_uint(ldexpf(__uint_as_float(uint32_t(h) << 16), e)) >> 16);
                        csq[fn] += v * v;
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

// ------------------------------------------------------------------ BF16 GEMM, LDS DMA

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(1))) void* global_ptr_t;

// LDS layout of a tile filled by DMA: rows of BK bfloat16 (BK / 8 chunks of 16 bytes, no
// padding); chunk c of row r sits at slot (BK / 8) r + (c ^ swz(r)), with the XOR chosen so
// that the 16 rows of a 16-lane operand read cover all 16 bank groups of a 256-byte bank
// row: swz(r) = (r / 2) mod 8 for 8 chunks per row, (r / 4) mod 4 for 4.
template <int BK>
QB_DEV int dma_slot(int r, int c) {
    constexpr int CPR = BK / 8;
    return CPR * r + (c ^ (CPR == 8 ? ((r >> 1) & 7) : ((r >> 2) & 3)));
}

// s_waitcnt immediate that waits until at most n vector-memory operations of this wave
// are outstanding (export and LDS counters left at their maxima).
QB_DEV constexpr int vmcnt_imm(int n) { return (n & 0xF) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// Same product as gemm_bf16_kernel for K-contiguous A and B (16-byte aligned rows, K a
// multiple of BK), with the K tiles moved global -> LDS by global_load_lds_dwordx4 through
// a ring of STAGES tiles: tile t + STAGES - 1 is requested while tile t is multiplied, so a
// tile has STAGES - 1 tiles of MFMA time to arrive.  A wave's DMA instruction fills 64
// consecutive slots (lane l -> slot s0 + l), each lane fetching the chunk that the swizzle
// puts there; there are no staging registers and no LDS store instructions.  The operands
// of k-step s + 1 are read while the MFMAs of step s run.  Rows beyond M (columns beyond
// N) re-read the last valid row; their results are never stored.
//
// AT: A is read in place from an M-contiguous array (element (i, k) at A[k * lda + i], the
// H = A_q^T G_q product): its tile is moved by DMA as BK rows of BM elements (the chunk c
// of row k at slot (BM / 8) k + (c ^ 4 (k mod 4)), so that the 8 rows x 4 chunks of one
// transposed read hit every 16-byte bank group twice), and the operand of a k-step is read
// with two ds_read_b64_tr_b16: in each 16-lane group, lane j addresses row k0 + j / 4,
// elements i0 + 4 (j mod 4) .. + 3, and lane i then holds A(i0 + i, k0 .. k0 + 3) (measured
// on gfx950).
//
// A8 (with AT): A holds e4m3 bytes.  Its tile rows are BM bytes (16 chunks of 16 elements,
// chunk c of row k at slot c ^ 2 (k mod 8)), and the operand of a k-step is one
// ds_read_b64_tr_b8: in each 16-lane group lane j addresses row k0 + j / 2, elements
// i0 + 8 (j mod 2) .. + 7, and lane i then holds A(i0 + i, k0 .. k0 + 7) as 8 bytes
// (measured on gfx950), widened exactly to bfloat16 in registers.  The e4m3 row scales are
// already in the other operand (2^e_k G_q).
//
// A8 without AT (G = A_q Omega_q for e4m3 A): a tile row (i) is BK bytes, BK / 16 chunks of
// 16 elements, chunk c of row r at slot c ^ ((r >> 3) & 1); the operand of k-step s of a
// fragment is the 8 bytes at chunk s, half (lane / 32), read with one ds_read_b64 and widened
// in registers.  The epilogue applies the row scales: G_q = bf16(2^e_i (A8 Omega_q)), and the
// H operand 2^e_i G_q.
template <int BM, int BN, int BK, int STAGES, int WM, int WN, int EPI, bool AT = false, bool A8 = false>
__global__ void __launch_bounds__(64 * WM * WN, 1) gemm_bf16_dma_kernel(const Bf16GemmArgs g) {
    static_assert(!A8 || AT || BK == 32, "e4m3 A in the G form: 32-deep tiles (two chunks per row)");
    constexpr int NT = 64 * WM * WN, NW = NT / 64, CPR = BK / 8;
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
    constexpr int A_SLOTS = A8 ? BK * BM / 16 : BM * CPR, B_SLOTS = BN * CPR;
    constexpr int A_INSTR = A_SLOTS / 64 / NW, B_INSTR = B_SLOTS / 64 / NW;
    constexpr int PER_TILE = A_INSTR + B_INSTR;           // DMA instructions per wave per tile
    constexpr int KSTEPS = BK / 16;
    static_assert(A_SLOTS % (64 * NW) == 0 && B_SLOTS % (64 * NW) == 0, "whole DMA instructions per wave");
    constexpr int CP8 = BM / 16;   // A8: 16-byte chunks per row (k) of the A tile
    static_assert((CPR == 8 || CPR == 4) && KSTEPS % 2 == 0, "tile depth 32 or 64");
    __shared__ __align__(16) uint16_t As[STAGES][BM * BK];
    __shared__ __align__(16) uint16_t Bs[STAGES][BN * BK];
    __shared__ double red[WM][BN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int tile_m, tile_n;
    group_tiles(logical, g.tiles_m, g.tiles_n, tile_m, tile_n);
    const int64_t m0 = static_cast<int64_t>(tile_m) * BM, n0 = static_cast<int64_t>(tile_n) * BN;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f32x16{};

    auto slot_rc = [](int sl, int& r, int& c) {
        r = sl / CPR;
        c = (sl % CPR) ^ (CPR == 8 ? ((r >> 1) & 7) : ((r >> 2) & 3));
    };
    constexpr int CPA = BM / 8;   // AT: 16-byte chunks per row (k) of the A tile
    static_assert(!AT || (CPA % 16 == 0 && (BK * CPA) % (64 * NW) == 0), "AT tile shape");
    // One DMA instruction: 16 bytes per lane from src into LDS at lds_base + 16 lane.  It is
    // written as inline assembly so that the compiler does not count it among the memory
    // operations that LDS reads must wait for (it would wait for every tile in flight);
    // this kernel waits for its DMAs itself (s_waitcnt vmcnt before each barrier).  The
    // instruction has no register results.  M0 holds the LDS base; no compiler-generated
    // code of this kernel reads M0 (checked in its gfx950 assembly), so clobbering it here
    // is safe.
    auto dma16 = [](const uint16_t* src, const uint16_t* lds_dst) {
        const uint32_t base = __builtin_amdgcn_readfirstlane(
            static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_ptr_t)lds_dst)));
        asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off"
                     :
                     : "v"(src), "s"(base)
                     : "memory", "m0");
    };
    auto issue = [&](int st, int64_t k0) {
#pragma unroll
        for (int j = 0; j < A_INSTR; ++j) {
            const int s0 = (wave * A_INSTR + j) * 64;
            if constexpr (A8 && !AT) {
                const int sl = s0 + lane, r = sl / (BK / 16), c = (sl % (BK / 16)) ^ ((r >> 3) & 1);
                const int64_t gi = m0 + r < g.M ? m0 + r : g.M - 1;
                const uint8_t* a8 = reinterpret_cast<const uint8_t*>(g.A);
                dma16(reinterpret_cast<const uint16_t*>(a8 + gi * g.lda + k0 + 16 * c), &As[st][s0 * 8]);
            } else if constexpr (A8) {
                const int sl = s0 + lane, kr = sl / CP8, c = (sl % CP8) ^ (2 * (kr & 7));
                const int64_t ci = m0 + 16 * c < g.M - 16 ? m0 + 16 * c : g.M - 16;
                const uint8_t* a8 = reinterpret_cast<const uint8_t*>(g.A);
                dma16(reinterpret_cast<const uint16_t*>(a8 + (k0 + kr) * g.lda + ci), &As[st][s0 * 8]);
            } else if constexpr (AT) {
                const int sl = s0 + lane, kr = sl / CPA, c = (sl % CPA) ^ (4 * (kr & 3));
                const int64_t ci = m0 + 8 * c < g.M - 8 ? m0 + 8 * c : g.M - 8;
                dma16(g.A + (k0 + kr) * g.lda + ci, &As[st][s0 * 8]);
            } else {
                int r, c;
                slot_rc(s0 + lane, r, c);
                const int64_t gi = m0 + r < g.M ? m0 + r : g.M - 1;
                dma16(g.A + gi * g.lda + k0 + 8 * c, &As[st][s0 * 8]);
            }
        }
#pragma unroll
        for (int j = 0; j < B_INSTR; ++j) {
            const int s0 = (wave * B_INSTR + j) * 64;
            int r, c;
            slot_rc(s0 + lane, r, c);
            const int64_t gj = n0 + r < g.N ? n0 + r : g.N - 1;
            dma16(g.B + gj * g.ldb + k0 + 8 * c, &Bs[st][s0 * 8]);
        }
    };
    const int wm0 = wm * TM, wn0 = wn * TN;
    const int lr = lane & 31, lch = lane >> 5;
    // A8 keeps a k-step's A operand as its 8 raw bytes until the MFMAs that use it: the
    // widening then waits for the LDS read only there, after the previous step's MFMAs
    using AOp = std::conditional_t<A8, uint2, bf16x8>;
    auto read_ops = [&](int st, int ks, AOp (&a)[FM], bf16x8 (&b)[FN]) {
        if constexpr (A8 && !AT) {
            const uint8_t* tile = reinterpret_cast<const uint8_t*>(&As[st][0]);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int r = wm0 + fm * 32 + lr;
                a[fm] = *reinterpret_cast<const uint2*>(tile + r * BK + ((ks ^ ((r >> 3) & 1)) << 4) + 8 * lch);
            }
        } else if constexpr (A8) {
            const int grp = lane >> 4, j = lane & 15;
            const int kk = 16 * ks + 8 * (grp >> 1) + (j >> 1);
            const uint8_t* tile = reinterpret_cast<const uint8_t*>(&As[st][0]);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int ii = wm0 + fm * 32 + 16 * (grp & 1) + 8 * (j & 1);
                const int off = kk * BM + (((ii >> 4) ^ (2 * (kk & 7))) << 4) + (ii & 15);
                typedef int i32x2 __attribute__((ext_vector_type(2)));
                typedef __attribute__((address_space(3))) i32x2* lds_i32x2;
                const i32x2 v = __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_i32x2)(lds_ptr_t)(tile + off));
                a[fm] = make_uint2(static_cast<uint32_t>(v[0]), static_cast<uint32_t>(v[1]));
            }
        } else if constexpr (AT) {
            const int grp = lane >> 4, j = lane & 15;
            const int kk = 16 * ks + 8 * (grp >> 1) + (j >> 2);
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int ii = wm0 + fm * 32 + 16 * (grp & 1) + 4 * (j & 3);
                const int e0 = kk * BM + (((ii >> 3) ^ (4 * (kk & 3))) << 3) + (ii & 7);
                const int e1 = e0 + 4 * BM;   // rows kk + 4: same swizzle
                typedef short s16x4 __attribute__((ext_vector_type(4)));
                typedef __attribute__((address_space(3))) s16x4* lds_s16x4;
                const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4)(lds_ptr_t)&As[st][e0]);
                const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4)(lds_ptr_t)&As[st][e1]);
                typedef short s16x8 __attribute__((ext_vector_type(8)));
                const s16x8 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                a[fm] = __builtin_bit_cast(bf16x8, v);
            }
        } else {
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
                a[fm] = *reinterpret_cast<const bf16x8*>(&As[st][dma_slot<BK>(wm0 + fm * 32 + lr, 2 * ks + lch) * 8]);
        }
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
            b[fn] = *reinterpret_cast<const bf16x8*>(&Bs[st][dma_slot<BK>(wn0 + fn * 32 + lr, 2 * ks + lch) * 8]);
    };
    auto mfmas = [&](const AOp (&a)[FM], const bf16x8 (&b)[FN]) {
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) {
            bf16x8 av;
            if constexpr (A8) av = __builtin_bit_cast(bf16x8, e4m3x8_to_bf16x8(a[fm]));
            else av = a[fm];
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
                acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b[fn], acc[fm][fn], 0, 0, 0);
        }
    };
    // the k-steps of one tile, two operand sets in flight (scheduling barriers keep the
    // compiler from sinking the reads back to their use)
    auto compute = [&](int st) {
        AOp a0[FM], a1[FM];
        bf16x8 b0[FN], b1[FN];
        read_ops(st, 0, a0, b0);
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ks += 2) {
            read_ops(st, ks + 1, a1, b1);
            __builtin_amdgcn_sched_barrier(0);
            mfmas(a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            if (ks + 2 < KSTEPS) read_ops(st, ks + 2, a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            mfmas(a1, b1);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    const int64_t T = g.K / BK;   // K tiles
    if (T > 0) {
#pragma unroll
        for (int p = 0; p < STAGES - 1; ++p)
            if (p < T) issue(p, static_cast<int64_t>(p) * BK);
        for (int64_t t = 0; t < T; ++t) {
            // this wave's DMAs for tile t have landed once at most the later tiles' remain
            const int64_t later = T - 1 - t < STAGES - 2 ? T - 1 - t : STAGES - 2;
            if (later >= STAGES - 2) __builtin_amdgcn_s_waitcnt(vmcnt_imm((STAGES - 2) * PER_TILE));
            else if (later == 1) __builtin_amdgcn_s_waitcnt(vmcnt_imm(PER_TILE));
            else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            // every wave's part of tile t is in LDS and tile t - 1 is consumed.  A bare
            // s_barrier: the fence of __syncthreads() would also wait for the later tiles'
            // DMAs; the empty asm statements keep the compiler from moving LDS accesses
            // across it.
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (t + STAGES - 1 < T) issue(static_cast<int>((t + STAGES - 1) % STAGES), (t + STAGES - 1) * BK);
            compute(static_cast<int>(t % STAGES));
        }
        __syncthreads();
    }

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
                    } else if constexpr (A8) {
                        // G_q = bf16(2^e_i (A8 Omega_q)(i, j)); the H operand is 2^e_i G_q
                        const int e = g.row_exp[i];
                        const uint16_t h = f32_to_bf16_rne(ldexpf(acc[fm][fn][r], e));
                        const double v = bf16_to_f64(h);
                        g.out[i * g.ldo + j] = v;
                        g.outT[j * g.ldt + i] =
                            static_cast<uint16_t>(__float_as_uint(ldexpf(__uint_as_float(uint32_t(h) << 16), e)) >> 16);
                        csq[fn] += v * v;
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

// ------------------------------------------------------------------ FP8 G product, LDS DMA

// The G product of the e4m3 form on 8-bit matrix cores: out(i, j) = 2^(e_i - 5) sum_k
// A8(i, k) W8(j, k), A8 the e4m3 bytes of A (M x K, K contiguous, row exponents e_i) and W8
// the bytes e4m3(2^5 Omega)^T (N x K, K contiguous), on v_mfma_f32_32x32x64_f8f6f4 with both
// operands e4m3 and binary32 accumulation (a product of two e4m3 values is exact in
// binary32).  Tiles of BM x BN x 64 bytes move global -> LDS by DMA through a ring of STAGES
// tiles as in gemm_bf16_dma_kernel; a 64-byte tile row has that kernel's chunk layout for
// 32-deep bfloat16 rows (chunk c of row r at slot 4 r + (c ^ ((r >> 2) & 3))).  A lane's
// operand of the tile's k-step is 32 bytes of its row, chunks 2 (lane / 32) and
// 2 (lane / 32) + 1: the instruction pairs equal register bytes of the A and B operands with
// the same k, so one k order shared by both operands gives the sum over the tile's 64 k
// (checked on gfx950 against a host product of one instruction).  Epilogue as the bfloat16
// kernels' e4m3 G epilogue: G_q = bf16(2^(e_i - 5) sums), the H operand 2^e_i G_q in bfloat16,
// and the column sums of squares of G_q.  K must be a multiple of 64; rows beyond M (N)
// re-read the last valid row and are never stored.
template <int BM, int BN, int STAGES, int WM, int WN>
__global__ void __launch_bounds__(64 * WM * WN, 1) gemm_f8_dma_kernel(const Bf16GemmArgs g) {
    constexpr int NT = 64 * WM * WN, NW = NT / 64, BK = 64, CPR = 4;
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
    constexpr int A_INSTR = BM * CPR / 64 / NW, B_INSTR = BN * CPR / 64 / NW;
    constexpr int PER_TILE = A_INSTR + B_INSTR;           // DMA instructions per wave per tile
    static_assert((BM * CPR) % (64 * NW) == 0 && (BN * CPR) % (64 * NW) == 0, "whole DMA instructions per wave");
    __shared__ __align__(16) uint8_t As[STAGES][BM * BK];
    __shared__ __align__(16) uint8_t Bs[STAGES][BN * BK];
    __shared__ double red[WM][BN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    int tile_m, tile_n;
    group_tiles(logical, g.tiles_m, g.tiles_n, tile_m, tile_n);
    const int64_t m0 = static_cast<int64_t>(tile_m) * BM, n0 = static_cast<int64_t>(tile_n) * BN;
    const uint8_t* A8 = reinterpret_cast<const uint8_t*>(g.A);
    const uint8_t* W8 = reinterpret_cast<const uint8_t*>(g.B);

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = f32x16{};

    auto slot_of = [](int r, int c) { return CPR * r + (c ^ ((r >> 2) & 3)); };
    // one DMA instruction, as in gemm_bf16_dma_kernel (no register results; the kernel waits
    // for its DMAs itself before each barrier)
    auto dma16 = [](const uint8_t* src, const uint8_t* lds_dst) {
        const uint32_t base = __builtin_amdgcn_readfirstlane(
            static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_ptr_t)lds_dst)));
        asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off"
                     :
                     : "v"(src), "s"(base)
                     : "memory", "m0");
    };
    auto issue = [&](int st, int64_t k0) {
#pragma unroll
        for (int j = 0; j < A_INSTR; ++j) {
            const int s0 = (wave * A_INSTR + j) * 64;
            const int sl = s0 + lane, r = sl / CPR, c = (sl % CPR) ^ ((r >> 2) & 3);
            const int64_t gi = m0 + r < g.M ? m0 + r : g.M - 1;
            dma16(A8 + gi * g.lda + k0 + 16 * c, &As[st][s0 * 16]);
        }
#pragma unroll
        for (int j = 0; j < B_INSTR; ++j) {
            const int s0 = (wave * B_INSTR + j) * 64;
            const int sl = s0 + lane, r = sl / CPR, c = (sl % CPR) ^ ((r >> 2) & 3);
            const int64_t gj = n0 + r < g.N ? n0 + r : g.N - 1;
            dma16(W8 + gj * g.ldb + k0 + 16 * c, &Bs[st][s0 * 16]);
        }
    };
    const int wm0 = wm * TM, wn0 = wn * TN;
    const int lr = lane & 31, lch = lane >> 5;
    auto operand = [&](const uint8_t* tile, int r) {
        const uint4 lo = *reinterpret_cast<const uint4*>(tile + 16 * slot_of(r, 2 * lch));
        const uint4 hi = *reinterpret_cast<const uint4*>(tile + 16 * slot_of(r, 2 * lch + 1));
        return i32x8{static_cast<int>(lo.x), static_cast<int>(lo.y), static_cast<int>(lo.z), static_cast<int>(lo.w),
                     static_cast<int>(hi.x), static_cast<int>(hi.y), static_cast<int>(hi.z), static_cast<int>(hi.w)};
    };
    auto compute = [&](int st) {
        i32x8 a[FM], b[FN];
#pragma unroll
        for (int fm = 0; fm < FM; ++fm) a[fm] = operand(&As[st][0], wm0 + fm * 32 + lr);
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) b[fn] = operand(&Bs[st][0], wn0 + fn * 32 + lr);
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
                acc[fm][fn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[fm], b[fn], acc[fm][fn], 0, 0, 0, 0,
                                                                              0, 0);
    };

    const int64_t T = g.K / BK;   // K tiles
    if (T > 0) {
#pragma unroll
        for (int p = 0; p < STAGES - 1; ++p)
            if (p < T) issue(p, static_cast<int64_t>(p) * BK);
        for (int64_t t = 0; t < T; ++t) {
            const int64_t later = T - 1 - t < STAGES - 2 ? T - 1 - t : STAGES - 2;
            if (later >= STAGES - 2) __builtin_amdgcn_s_waitcnt(vmcnt_imm((STAGES - 2) * PER_TILE));
            else if (later == 1) __builtin_amdgcn_s_waitcnt(vmcnt_imm(PER_TILE));
            else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (t + STAGES - 1 < T) issue(static_cast<int>((t + STAGES - 1) % STAGES), (t + STAGES - 1) * BK);
            compute(static_cast<int>(t % STAGES));
        }
        __syncthreads();
    }

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
                    const int e = g.row_exp[i];
                    const uint16_t h = f32_to_bf16_rne(ldexpf(acc[fm][fn][r], e - 5));
                    const double v = bf16_to_f64(h);
                    g.out[i * g.ldo + j] = v;
                    g.outT[j * g.ldt + i] =
                        static_cast<uint16_t>(__float_as_uint(ldexpf(__uint_as_float(uint32_t(h) << 16), e)) >> 16);
                    csq[fn] += v * v;
                }
            }
    if (g.colsq != nullptr) {
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

hipError_t launch_quant_transpose_omega_e4m3(double* om, int64_t n, int64_t w, uint16_t* omT, int64_t ldt,
                                             uint8_t* omT8, int64_t ldt8, hipStream_t s) {
    if (n <= 0 || w <= 0) return hipSuccess;
    dim3 grid(static_cast<unsigned>(cdiv(w, 64)), static_cast<unsigned>(cdiv(n, 64)));
    hipLaunchKernelGGL(quant_transpose_omega_e4m3_kernel, grid, dim3(256), 0, s, om, n, w, omT, ldt, omT8, ldt8);
    return hipGetLastError();
}

bool gemm_f8_fits(int64_t K, const void* A, int64_t lda, const void* W, int64_t ldw) {
    return K % 64 == 0 && lda % 16 == 0 && ldw % 16 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
           reinterpret_cast<uintptr_t>(W) % 16 == 0;
}

hipError_t gemm_f8(int64_t M, int64_t N, int64_t K, const uint8_t* A, int64_t lda, const int32_t* row_exp,
                   const uint8_t* W, int64_t ldw, double* out, int64_t ldo, uint16_t* outT, int64_t ldt,
                   double* colsq, int64_t* groups, hipStream_t s) {
    *groups = 0;
    if (M <= 0 || N <= 0) return hipSuccess;
    if (!gemm_f8_fits(K, A, lda, W, ldw) || row_exp == nullptr || outT == nullptr) return hipErrorInvalidValue;
    Bf16GemmArgs g{};
    g.M = M; g.N = N; g.K = K;
    g.A = reinterpret_cast<const uint16_t*>(A); g.lda = lda;
    g.B = reinterpret_cast<const uint16_t*>(W); g.ldb = ldw;
    g.out = out; g.ldo = ldo; g.outT = outT; g.ldt = ldt; g.colsq = colsq; g.row_exp = row_exp;
    constexpr int kTile = 256;
    g.tiles_m = static_cast<int>(cdiv(M, kTile));
    g.tiles_n = static_cast<int>(cdiv(N, kTile));
    *groups = g.tiles_m;
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(g.tiles_m) * g.tiles_n));
    hipLaunchKernelGGL((gemm_f8_dma_kernel<256, 256, 4, 4, 2>), grid, dim3(512), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_sumsq_fp8(const uint8_t* a, const int32_t* row_exp, int64_t m, int64_t n,
                            int64_t lda, double* scratch, double* out, hipStream_t s) {
    const int64_t g = m < sumsq_partials() ? m : sumsq_partials();
    const int vec = (reinterpret_cast<uintptr_t>(a) % 8 == 0) && (lda % 8 == 0);
    hipLaunchKernelGGL(sumsq_fp8_partial, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, a, m, n, lda, vec,
                       row_exp, scratch);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_vector(scratch, g, out, s);
}

hipError_t launch_sumsq_bf16(const uint16_t* a, int64_t m, int64_t n, int64_t lda,
                             double* scratch, double* out, hipStream_t s) {
    const int64_t g = m < sumsq_partials() ? m : sumsq_partials();
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

hipError_t gemm_bf16(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, bool a_km,
                     bool a_fp8, const int32_t* row_exp, const uint16_t* B, int64_t ldb, double* out,
                     int64_t ldo, uint16_t* outT, int64_t ldt, double* colsq, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    // the two products of the sketch: G (K-contiguous A, G epilogue) and H (K-major A,
    // FP64 epilogue)
    if (a_km == (outT != nullptr)) return hipErrorInvalidValue;
    if (a_fp8 && !a_km && row_exp == nullptr) return hipErrorInvalidValue;
    Bf16GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.A = static_cast<const uint16_t*>(A); g.lda = lda; g.B = B; g.ldb = ldb;
    g.out = out; g.ldo = ldo; g.outT = outT; g.ldt = ldt; g.colsq = colsq; g.row_exp = row_exp;
    // 8-element chunks: 16 bytes of bfloat16 or 8 bytes of e4m3
    const uintptr_t a_align = a_fp8 ? 8 : 16;
    g.vec = (reinterpret_cast<uintptr_t>(A) % a_align == 0) && (reinterpret_cast<uintptr_t>(B) % 16 == 0) &&
            (lda % 8 == 0) && (ldb % 8 == 0);
    const bool big = use_big(M, N);
    const int t = big ? kBigTile : kSmallTile;
    g.tiles_m = static_cast<int>(cdiv(M, t));
    g.tiles_n = static_cast<int>(cdiv(N, t));
    dim3 grid(static_cast<unsigned>(static_cast<int64_t>(g.tiles_m) * g.tiles_n));
    if (big && !a_km && !a_fp8 && g.vec && K % 32 == 0) {
        // K-contiguous bfloat16 operands with 16-byte aligned rows, whole K tiles: LDS DMA
        hipLaunchKernelGGL((gemm_bf16_dma_kernel<256, 256, 32, 4, 2, 4, 1>), grid, dim3(512), 0, s, g);
    } else if (big && !a_km && a_fp8 && g.vec && K % 32 == 0 && lda % 16 == 0 &&
               reinterpret_cast<uintptr_t>(A) % 16 == 0) {
        // G: e4m3 A rows moved by DMA as bytes, widened in registers, row scales in the epilogue
        hipLaunchKernelGGL((gemm_bf16_dma_kernel<256, 256, 32, 4, 2, 4, 1, false, true>), grid, dim3(512), 0, s, g);
    } else if (big && a_km && !a_fp8 && g.vec && K % 32 == 0 && M % 8 == 0) {
        // H: bfloat16 A read in place (M-contiguous) through transposed LDS reads
        hipLaunchKernelGGL((gemm_bf16_dma_kernel<256, 256, 32, 4, 2, 4, 0, true>), grid, dim3(512), 0, s, g);
    } else if (big && a_km && a_fp8 && g.vec && K % 32 == 0 && M % 16 == 0 && lda % 16 == 0 &&
               reinterpret_cast<uintptr_t>(A) % 16 == 0) {
        // H: e4m3 A read in place through transposed byte reads, widened in registers
        hipLaunchKernelGGL((gemm_bf16_dma_kernel<256, 256, 32, 4, 2, 4, 0, true, true>), grid, dim3(512), 0, s, g);
    } else if (big) {
        if (a_km && a_fp8)
            hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 64, 2, 4, 0, true, true>), grid, dim3(512), 0, s, g);
        else if (a_km)
            hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 64, 2, 4, 0, true, false>), grid, dim3(512), 0, s, g);
        else if (a_fp8)
            hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 64, 2, 4, 1, false, true>), grid, dim3(512), 0, s, g);
        else
            hipLaunchKernelGGL((gemm_bf16_kernel<256, 256, 64, 2, 4, 1, false, false>), grid, dim3(512), 0, s, g);
    } else {
        if (a_km && a_fp8)
            hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 64, 2, 2, 0, true, true>), grid, dim3(256), 0, s, g);
        else if (a_km)
            hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 64, 2, 2, 0, true, false>), grid, dim3(256), 0, s, g);
        else if (a_fp8)
            hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 64, 2, 2, 1, false, true>), grid, dim3(256), 0, s, g);
        else
            hipLaunchKernelGGL((gemm_bf16_kernel<128, 128, 64, 2, 2, 1, false, false>), grid, dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

}  // namespace qb
