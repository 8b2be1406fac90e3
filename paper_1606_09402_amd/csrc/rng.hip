// Bit-specified Gaussian test matrix Omega (randn of Algorithms 2 and 4).
//
// Philox4x32-10 (Salmon et al., SC'11) on counter (row, pair, stream, batch) and key
// (seed lo, seed hi), two 52-bit uniforms per call, Box-Muller (1958).  ln, sqrt,
// sin, cos are evaluated from their series / Newton definitions with IEEE binary64
// +, -, *, / only and contraction disabled, so every conforming implementation of
// the same operation sequence produces identical bits.
#pragma clang fp contract(off)

#include "kernels.h"

namespace qb {
namespace {

constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;

// ln 2, sqrt(1/2), pi/2 rounded to nearest binary64
constexpr double kLn2 = 0x1.62e42fefa39efp-1;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
constexpr double kHalfPi = 0x1.921fb54442d18p+0;

QB_DEV void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                     uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        const uint32_t hi0 = __umulhi(kMul0, c0), lo0 = kMul0 * c0;
        const uint32_t hi1 = __umulhi(kMul1, c2), lo1 = kMul1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// 52 random bits -> (0, 1), never 0 or 1
QB_DEV double unit_open(uint32_t hi, uint32_t lo) {
    const uint64_t x = ((static_cast<uint64_t>(hi) << 32) | lo) >> 12;
    return (static_cast<double>(x) + 0.5) * 0x1p-52;
}

// ln x for normal 0 < x < 1: x = m 2^e, m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s), s = (m - 1)/(m + 1), series through s^23 / 23.
QB_DEV double ln_series(double x) {
    const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(x));
    int64_t e = static_cast<int64_t>((bits >> 52) & 0x7FF) - 1022;
    double m = __longlong_as_double(
        static_cast<long long>((bits & 0x000FFFFFFFFFFFFFull) | (1022ull << 52)));
    if (m < kSqrtHalf) {
        m = m + m;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    p = p * z + 1.0;
    const double lnm = (s + s) * p;
    return static_cast<double>(e) * kLn2 + lnm;
}

// sqrt y for normal y > 0: halve the biased exponent for a first guess, then six
// Newton (Heron) steps.
QB_DEV double sqrt_newton(double y) {
    const uint64_t yb = static_cast<uint64_t>(__double_as_longlong(y));
    double g = __longlong_as_double(static_cast<long long>((yb >> 1) + 0x1FF8000000000000ull));
#pragma unroll
    for (int i = 0; i < 6; ++i) g = 0.5 * (g + y / g);
    return g;
}

// sin(2 pi u), cos(2 pi u) for 0 < u < 1.
QB_DEV void sincos_turn(double u, double& sn, double& cs) {
    const double v = u * 4.0;
    const int q = static_cast<int>(v);
    const double f = v - static_cast<double>(q);
    const bool fold = f > 0.5;
    const double g = fold ? 1.0 - f : f;
    const double x = g * kHalfPi;
    const double z = x * x;
    // Taylor coefficients (-1)^k / (2k+1)! and (-1)^k / (2k)!, k = 8 .. 1
    double ps = 1.0 / 355687428096000.0;
    ps = ps * z + -1.0 / 1307674368000.0;
    ps = ps * z + 1.0 / 6227020800.0;
    ps = ps * z + -1.0 / 39916800.0;
    ps = ps * z + 1.0 / 362880.0;
    ps = ps * z + -1.0 / 5040.0;
    ps = ps * z + 1.0 / 120.0;
    ps = ps * z + -1.0 / 6.0;
    const double sx = x + x * (z * ps);
    double pc = 1.0 / 20922789888000.0;
    pc = pc * z + -1.0 / 87178291200.0;
    pc = pc * z + 1.0 / 479001600.0;
    pc = pc * z + -1.0 / 3628800.0;
    pc = pc * z + 1.0 / 40320.0;
    pc = pc * z + -1.0 / 720.0;
    pc = pc * z + 1.0 / 24.0;
    pc = pc * z + -1.0 / 2.0;
    const double cx = 1.0 + z * pc;
    const double sf = fold ? cx : sx;
    const double cf = fold ? sx : cx;
    switch (q) {
        case 0: sn = sf; cs = cf; break;
        case 1: sn = cf; cs = -sf; break;
        case 2: sn = -sf; cs = -cf; break;
        default: sn = -cf; cs = sf; break;
    }
}

}  // namespace

QB_DEV void gauss_pair(uint64_t seed, uint32_t stream_id, uint32_t batch, uint32_t row,
                       uint32_t pair, double& z0, double& z1) {
    uint32_t c0 = row, c1 = pair, c2 = stream_id, c3 = batch;
    philox10(c0, c1, c2, c3, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const double u1 = unit_open(c0, c1);
    const double u2 = unit_open(c2, c3);
    const double r = sqrt_newton(-2.0 * ln_series(u1));
    double sn, cs;
    sincos_turn(u2, sn, cs);
    z0 = r * cs;
    z1 = r * sn;
}

// One thread per (row, Box-Muller pair); grid.y strides over rows.
__global__ void __launch_bounds__(256)
gauss_fill_kernel(uint64_t seed, uint32_t stream_id, uint32_t batch, int64_t row0, int64_t col0,
                  int64_t rows, int64_t cols, double* __restrict__ out, int64_t ld) {
    const int64_t p_lo = col0 >> 1;
    const int64_t npairs = ((col0 + cols + 1) >> 1) - p_lo;
    const int64_t pp = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (pp >= npairs) return;
    const int64_t pair = p_lo + pp;
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        double z0, z1;
        gauss_pair(seed, stream_id, batch, static_cast<uint32_t>(row0 + r),
                   static_cast<uint32_t>(pair), z0, z1);
        const int64_t c_even = 2 * pair - col0;  // local column of z0
        double* o = out + r * ld;
        if (c_even >= 0 && c_even < cols) o[c_even] = z0;
        if (c_even + 1 >= 0 && c_even + 1 < cols) o[c_even + 1] = z1;
    }
}

hipError_t launch_gauss_fill(uint64_t seed, uint32_t stream_id, uint32_t batch, int64_t row0,
                             int64_t col0, int64_t rows, int64_t cols, double* out, int64_t ld,
                             hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int64_t npairs = ((col0 + cols + 1) >> 1) - (col0 >> 1);
    dim3 grid(static_cast<unsigned>(cdiv(npairs, 256)),
              static_cast<unsigned>(rows < 65535 ? rows : 65535));
    hipLaunchKernelGGL(gauss_fill_kernel, grid, dim3(256), 0, s, seed, stream_id, batch, row0,
                       col0, rows, cols, out, ld);
    return hipGetLastError();
}

}  // namespace qb
