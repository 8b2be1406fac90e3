// Differentiation form: fixed-rank randQB_FP on a batch of matrices and the adjoint of
// A -> (Q, B) for a fixed Omega.
//
// Forward, per matrix (Algorithm 3 with the re-orthogonalisation of Algorithm 4, i.e.
// Algorithm 4 with P = 0 and no stopping; rank k = t b): G = A Omega, H = A^T G once, then
// per block J
//   W = B Omega_J, Y = G_J - Q W, [Q_i, R] = qr(Y), [Q_i, R~] = qr(Q_i - Q (Q^T Q_i)),
//   R_i = R~ R, B_i = R_i^{-T} (H_J^T - (Y^T Q) B - W^T B)     (eq. (23)).
// In exact arithmetic this is Q = qf(A Omega) (diag(R) > 0) and B = Q^T A, so the map has
// one derivative whatever the blocking.
//
// Backward, given dL/dQ and dL/dB (Qb, Bb):
//   A-bar  = Q Bb + Y-bar Omega^T                      (B = Q^T A, Y = A Omega)
//   Qt     = Qb + A Bb^T                               (total adjoint of Q)
//   Y-bar  = (Qt + Q copyltu(M)) R^{-T},  M = -Qt^T Q  (thin-QR adjoint with R-bar = 0,
//            copyltu(M) = the symmetric matrix built from the lower triangle of M)
// where R = Q^T G is recomputed from G = A Omega (G is not kept from the forward).
//
// Every product runs on one batched MFMA GEMM templated on the element type (binary32
// for speed, binary64 for checking the adjoint to round-off); the b x b Cholesky factors
// and the k x k triangular inverse are one workgroup per matrix.
#include <type_traits>

#include "kernels.h"

namespace qb {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ MFMA traits

template <typename T>
struct Mfma;

// v_mfma_f32_16x16x4f32: operand lane l holds A(l mod 16, l / 16) and B(l / 16, l mod 16);
// accumulator slot r of lane l holds row 4 (l / 16) + r, column l mod 16 (measured).
template <>
struct Mfma<float> {
    using acc_t = f32x4;
    static QB_DEV acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static QB_DEV int row(int lane, int r) { return ((lane >> 4) << 2) + r; }
};

// v_mfma_f64_16x16x4f64: same operands; slot r of lane l holds row 4 r + l / 16 (measured).
template <>
struct Mfma<double> {
    using acc_t = v4d;
    static QB_DEV acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static QB_DEV int row(int lane, int r) { return (r << 2) + (lane >> 4); }
};

// ------------------------------------------------------------------ batched GEMM

// C[z](i, j) = alpha sum_k A[z](i, k) B[z](k, j) + beta C0[z](i, j), z < batch, with
// every operand a strided view: X[z](i, j) = X[z * sz + i * si + j * sj].
template <typename T>
struct BGemm {
    int64_t M, N, K;
    const T* A; int64_t a_si, a_sk, a_sz;
    const T* B; int64_t b_sk, b_sj, b_sz;
    T alpha, beta;
    const T* C0; int64_t c0_si, c0_sj, c0_sz;
    T* C; int64_t c_si, c_sj, c_sz;
    int tiles_n;
    int64_t kchunk;   // K range of one split (blockIdx.y); several splits write partials to P
    T* P;             // [split][batch][M][N] partial sums (gridDim.y > 1)
    // a second reduction segment (bgemm2_kernel only): k in [K1, K) reads A2(i, k - K1) and
    // B2(k - K1, j), so C = alpha [A A2] [B; B2] + beta C0 in one pass over C
    int64_t K1;
    const T* A2; int64_t a2_si, a2_sk, a2_sz;
    const T* B2; int64_t b2_sk, b2_sj, b2_sz;
};

template <typename T, int BM, int BN, int BK>
__global__ void __launch_bounds__(256) bgemm_kernel(const BGemm<T> g) {
    constexpr int NT = 256, WM = 2, WN = 2;
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 16, FN = TN / 16;
    constexpr int PA = BM + 16, PB = BN + 16;   // a 4 x 16 operand read hits distinct banks
    constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
    static_assert(BM * BK % NT == 0 && BN * BK % NT == 0 && BK % 4 == 0, "tile shape");
    __shared__ T As[BK * PA];
    __shared__ T Bs[BK * PB];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t z = blockIdx.z;
    const int tile_m = blockIdx.x / g.tiles_n, tile_n = blockIdx.x % g.tiles_n;
    const int64_t m0 = static_cast<int64_t>(tile_m) * BM, n0 = static_cast<int64_t>(tile_n) * BN;
    const T* A = g.A + z * g.a_sz;
    const T* B = g.B + z * g.b_sz;
    // the contiguous index of each operand runs fastest over the threads
    const bool a_kfast = g.a_sk == 1, b_jfast = g.b_sj == 1;

    using Acc = typename Mfma<T>::acc_t;
    Acc acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = Acc{};

    const int wm0 = wm * TM, wn0 = wn * TN;
    const int64_t kb = static_cast<int64_t>(blockIdx.y) * g.kchunk;
    const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
    for (int64_t k0 = kb; k0 < ke; k0 += BK) {
        T ra[LA], rb[LB];
#pragma unroll
        for (int p = 0; p < LA; ++p) {
            const int e = tid + p * NT;
            const int kk = a_kfast ? e % BK : e / BM, ii = a_kfast ? e / BK : e % BM;
            const int64_t i = m0 + ii, k = k0 + kk;
            ra[p] = (i < g.M && k < ke) ? A[i * g.a_si + k * g.a_sk] : T(0);
        }
#pragma unroll
        for (int p = 0; p < LB; ++p) {
            const int e = tid + p * NT;
            const int kk = b_jfast ? e / BN : e % BK, jj = b_jfast ? e % BN : e / BK;
            const int64_t j = n0 + jj, k = k0 + kk;
            rb[p] = (j < g.N && k < ke) ? B[k * g.b_sk + j * g.b_sj] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < LA; ++p) {
            const int e = tid + p * NT;
            const int kk = a_kfast ? e % BK : e / BM, ii = a_kfast ? e / BK : e % BM;
            As[kk * PA + ii] = ra[p];
        }
#pragma unroll
        for (int p = 0; p < LB; ++p) {
            const int e = tid + p * NT;
            const int kk = b_jfast ? e / BN : e % BK, jj = b_jfast ? e % BN : e / BK;
            Bs[kk * PB + jj] = rb[p];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T a[FM], b[FN];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) a[fm] = As[(kk + lk) * PA + wm0 + fm * 16 + li];
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) b[fn] = Bs[(kk + lk) * PB + wn0 + fn * 16 + li];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = Mfma<T>::op(a[fm], b[fn], acc[fm][fn]);
        }
    }

    if (gridDim.y > 1) {   // split K: raw partial sums, combined by bgemm_splitk_reduce
        T* P = g.P + (static_cast<int64_t>(blockIdx.y) * gridDim.z + z) * g.M * g.N;
#pragma unroll
        for (int fm = 0; fm < FM; ++fm)
#pragma unroll
            for (int fn = 0; fn < FN; ++fn)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = m0 + wm0 + fm * 16 + Mfma<T>::row(lane, r);
                    const int64_t j = n0 + wn0 + fn * 16 + li;
                    if (i < g.M && j < g.N) P[i * g.N + j] = acc[fm][fn][r];
                }
        return;
    }
    const T* C0 = g.C0 + z * g.c0_sz;
    T* C = g.C + z * g.c_sz;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = m0 + wm0 + fm * 16 + Mfma<T>::row(lane, r);
                const int64_t j = n0 + wn0 + fn * 16 + li;
                if (i < g.M && j < g.N) {
                    T v = g.alpha * acc[fm][fn][r];
                    if (g.beta != T(0)) v += g.beta * C0[i * g.c0_si + j * g.c0_sj];
                    C[i * g.c_si + j * g.c_sj] = v;
                }
            }
}

// The same product for large tiles: BM x BN per workgroup of WM x WN waves, BK-deep K tiles
// moved global -> registers -> LDS through two LDS stages (tile t + 1 is loaded while tile
// t is multiplied; one barrier per tile), with 16-byte loads along the contiguous index of
// each operand when the host found it aligned (vec), scalar checked loads otherwise and in
// edge tiles.  Each operand keeps its global orientation in LDS: an operand contiguous in k
// (AKF / BKF) as rows of BK + 4 elements, one contiguous in i (j) as BK rows of BM + 16 (BN +
// 16) elements; both pitches make the 16 x 4 operand reads of an MFMA and the 16-byte
// stores free of bank conflicts.
template <typename T, int BM, int BN, int BK, int WM, int WN, bool AKF, bool BKF>
__global__ void __launch_bounds__(64 * WM * WN) bgemm2_kernel(const BGemm<T> g, int vec_a, int vec_b) {
    constexpr int NT = 64 * WM * WN, TM = BM / WM, TN = BN / WN, FM = TM / 16, FN = TN / 16;
    constexpr int VE = 16 / sizeof(T);                       // elements per 16-byte load
    constexpr int PK = BK + 16 / sizeof(T) * (sizeof(T) == 4 ? 1 : 1);   // k-contiguous row pitch
    constexpr int PA = BM + 64 / sizeof(T), PB = BN + 64 / sizeof(T);    // i / j-contiguous pitches
    constexpr int A_SZ = AKF ? BM * PK : BK * PA, B_SZ = BKF ? BN * PK : BK * PB;
    constexpr int LA = BM * BK / NT, LB = BN * BK / NT;      // elements per thread per tile
    static_assert(LA % VE == 0 && LB % VE == 0 && BK % 4 == 0 && BK % VE == 0, "tile shape");
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    __shared__ __align__(16) T As[2][A_SZ];
    __shared__ __align__(16) T Bs[2][B_SZ];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t z = blockIdx.z;
    const int tile_m = blockIdx.x / g.tiles_n, tile_n = blockIdx.x % g.tiles_n;
    const int64_t m0 = static_cast<int64_t>(tile_m) * BM, n0 = static_cast<int64_t>(tile_n) * BN;
    const T* A1 = g.A + z * g.a_sz;
    const T* B1 = g.B + z * g.b_sz;
    const T* A2 = g.A2 != nullptr ? g.A2 + z * g.a2_sz : nullptr;
    const T* B2 = g.B2 != nullptr ? g.B2 + z * g.b2_sz : nullptr;
    const bool full = m0 + BM <= g.M && n0 + BN <= g.N;
    const bool va = vec_a && full, vb = vec_b && full;

    // element e (a multiple of VE) of the thread's share: (kk, ii) of A, (kk, jj) of B, the VE
    // elements e .. e + VE - 1 running along the operand's contiguous index
    auto a_of = [](int e, int& kk, int& ii) {
        if (AKF) { kk = e % BK; ii = e / BK; } else { kk = e / BM; ii = e % BM; }
    };
    auto b_of = [](int e, int& kk, int& jj) {
        if (BKF) { kk = e % BK; jj = e / BK; } else { kk = e / BN; jj = e % BN; }
    };
    T ra[LA], rb[LB];
    auto load = [&](int64_t kg0, int64_t ke) {
        const bool kin = kg0 + BK <= ke;
        // the segment of this K tile (a tile never straddles K1: K1 and the split chunks are
        // multiples of BK when there are two segments)
        const bool seg2 = kg0 >= g.K1;
        const T* A = seg2 ? A2 : A1;
        const T* B = seg2 ? B2 : B1;
        const int64_t a_si = seg2 ? g.a2_si : g.a_si, a_sk = seg2 ? g.a2_sk : g.a_sk;
        const int64_t b_sk = seg2 ? g.b2_sk : g.b_sk, b_sj = seg2 ? g.b2_sj : g.b_sj;
        const int64_t k0 = seg2 ? kg0 - g.K1 : kg0;
        const int64_t kend = seg2 ? ke - g.K1 : (ke < g.K1 ? ke : g.K1);
#pragma unroll
        for (int p = 0; p < LA / VE; ++p) {
            int kk, ii;
            a_of((tid + p * NT) * VE, kk, ii);
            if (va && kin) {
                const V x = *reinterpret_cast<const V*>(A + (m0 + ii) * a_si + (k0 + kk) * a_sk);
                const T* xs = reinterpret_cast<const T*>(&x);
#pragma unroll
                for (int q = 0; q < VE; ++q) ra[p * VE + q] = xs[q];
            } else {
#pragma unroll
                for (int q = 0; q < VE; ++q) {
                    const int64_t i = m0 + ii + (AKF ? 0 : q), k = k0 + kk + (AKF ? q : 0);
                    ra[p * VE + q] = (i < g.M && k < kend) ? A[i * a_si + k * a_sk] : T(0);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < LB / VE; ++p) {
            int kk, jj;
            b_of((tid + p * NT) * VE, kk, jj);
            if (vb && kin) {
                const V x = *reinterpret_cast<const V*>(B + (k0 + kk) * b_sk + (n0 + jj) * b_sj);
                const T* xs = reinterpret_cast<const T*>(&x);
#pragma unroll
                for (int q = 0; q < VE; ++q) rb[p * VE + q] = xs[q];
            } else {
#pragma unroll
                for (int q = 0; q < VE; ++q) {
                    const int64_t j = n0 + jj + (BKF ? 0 : q), k = k0 + kk + (BKF ? q : 0);
                    rb[p * VE + q] = (j < g.N && k < kend) ? B[k * b_sk + j * b_sj] : T(0);
                }
            }
        }
    };
    auto store = [&](int st) {
#pragma unroll
        for (int p = 0; p < LA / VE; ++p) {
            int kk, ii;
            a_of((tid + p * NT) * VE, kk, ii);
            T* d = &As[st][AKF ? ii * PK + kk : kk * PA + ii];
            *reinterpret_cast<V*>(d) = *reinterpret_cast<const V*>(&ra[p * VE]);
        }
#pragma unroll
        for (int p = 0; p < LB / VE; ++p) {
            int kk, jj;
            b_of((tid + p * NT) * VE, kk, jj);
            T* d = &Bs[st][BKF ? jj * PK + kk : kk * PB + jj];
            *reinterpret_cast<V*>(d) = *reinterpret_cast<const V*>(&rb[p * VE]);
        }
    };

    using Acc = typename Mfma<T>::acc_t;
    Acc acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = Acc{};
    const int wm0 = wm * TM, wn0 = wn * TN;
    auto compute = [&](int st) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T a[FM], b[FN];
#pragma unroll
            for (int fm = 0; fm < FM; ++fm) {
                const int i = wm0 + fm * 16 + li;
                a[fm] = AKF ? As[st][i * PK + kk + lk] : As[st][(kk + lk) * PA + i];
            }
#pragma unroll
            for (int fn = 0; fn < FN; ++fn) {
                const int j = wn0 + fn * 16 + li;
                b[fn] = BKF ? Bs[st][j * PK + kk + lk] : Bs[st][(kk + lk) * PB + j];
            }
#pragma unroll
            for (int fm = 0; fm < FM; ++fm)
#pragma unroll
                for (int fn = 0; fn < FN; ++fn) acc[fm][fn] = Mfma<T>::op(a[fm], b[fn], acc[fm][fn]);
        }
    };

    const int64_t kb = static_cast<int64_t>(blockIdx.y) * g.kchunk;
    const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
    int st = 0;
    if (kb < ke) {
        load(kb, ke);
        store(0);
        __syncthreads();
        for (int64_t k0 = kb; k0 < ke; k0 += BK) {
            const bool more = k0 + BK < ke;
            if (more) load(k0 + BK, ke);
            compute(st);
            if (more) store(st ^ 1);
            __syncthreads();
            st ^= 1;
        }
    }

    T* out;
    int64_t osi, osj;
    const bool split = gridDim.y > 1;
    if (split) {
        out = g.P + (static_cast<int64_t>(blockIdx.y) * gridDim.z + z) * g.M * g.N;
        osi = g.N;
        osj = 1;
    } else {
        out = g.C + z * g.c_sz;
        osi = g.c_si;
        osj = g.c_sj;
    }
    const T* C0 = g.C0 + z * g.c0_sz;
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = m0 + wm0 + fm * 16 + Mfma<T>::row(lane, r);
                const int64_t j = n0 + wn0 + fn * 16 + li;
                if (i < g.M && j < g.N) {
                    if (split) {
                        out[i * osi + j] = acc[fm][fn][r];
                    } else {
                        T v = g.alpha * acc[fm][fn][r];
                        if (g.beta != T(0)) v += g.beta * C0[i * g.c0_si + j * g.c0_sj];
                        out[i * osi + j * osj] = v;
                    }
                }
            }
}

// Fixed-order sum of the K splits with the alpha / beta epilogue.
template <typename T>
__global__ void __launch_bounds__(256)
bgemm_splitk_reduce(const T* __restrict__ P, int nsplit, int64_t batch, int64_t M, int64_t N, T alpha,
                    T beta, const T* C0, int64_t c0_si, int64_t c0_sj, int64_t c0_sz, T* C, int64_t c_si,
                    int64_t c_sj, int64_t c_sz) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t per = M * N;
    if (e >= batch * per) return;
    T t = T(0);
    for (int q = 0; q < nsplit; ++q) t += P[static_cast<int64_t>(q) * batch * per + e];
    const int64_t z = e / per, w = e % per, i = w / N, j = w % N;
    T v = alpha * t;
    if (beta != T(0)) v += beta * C0[z * c0_sz + i * c0_si + j * c0_sj];
    C[z * c_sz + i * c_si + j * c_sj] = v;
}

// Scratch for split-K partial sums.
template <typename T>
struct SplitWs {
    T* p;
    int64_t elems;
};

// A strided batch view.
template <typename T>
struct BV {
    const T* p;
    int64_t si, sj, sz;
};
template <typename T>
struct BMV {
    T* p;
    int64_t si, sj, sz;
};

template <typename T>
hipError_t bgemm(int64_t batch, int64_t M, int64_t N, int64_t K, BV<T> a, BV<T> b, T alpha, T beta,
                 BV<T> c0, BMV<T> c, hipStream_t s, SplitWs<T> sw) {
    if (batch <= 0 || M <= 0 || N <= 0) return hipSuccess;
    BGemm<T> g{};
    g.M = M; g.N = N; g.K = K;
    g.A = a.p; g.a_si = a.si; g.a_sk = a.sj; g.a_sz = a.sz;
    g.B = b.p; g.b_sk = b.si; g.b_sj = b.sj; g.b_sz = b.sz;
    g.alpha = alpha; g.beta = beta;
    g.C0 = c0.p; g.c0_si = c0.si; g.c0_sj = c0.sj; g.c0_sz = c0.sz;
    g.C = c.p; g.c_si = c.si; g.c_sj = c.sj; g.c_sz = c.sz;
    g.K1 = K;   // one reduction segment
    if (batch > 65535) return hipErrorInvalidValue;
    // 128 x 128 tiles (two LDS stages) for outputs of at least 128 x 128 with a reduction
    // of at least 128; else 64 x 64 tiles, 128 x 64 for tall outputs with few tiles per matrix
    const bool big = M >= 128 && N >= 128 && K >= 128;
    const bool tall = !big && M >= 1024 && N <= 64;
    g.tiles_n = static_cast<int>(cdiv(N, big ? 128 : 64));
    const int64_t tiles = cdiv(M, big || tall ? 128 : 64) * g.tiles_n;
    // few workgroups and a long reduction (Gram matrices, Q^T X): split K over about 2048
    // workgroups in chunks of at least 128
    int64_t nsplit = 1;
    if (sw.p != nullptr && tiles * batch < 1024 && K >= 256) {
        nsplit = cdiv(2048, tiles * batch);
        if (nsplit > K / 128) nsplit = K / 128;
        while (nsplit > 1 && nsplit * batch * M * N > sw.elems) --nsplit;
    }
    g.kchunk = cdiv(cdiv(K, 16), nsplit) * 16;
    nsplit = K > 0 ? cdiv(K, g.kchunk) : 1;
    if (nsplit < 1) nsplit = 1;
    g.P = sw.p;
    dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(nsplit), static_cast<unsigned>(batch));
    if (big) {
        // 16-byte loads when the operand's contiguous index is aligned in every matrix
        constexpr int64_t VE = 16 / sizeof(T);
        auto aligned = [&](const T* p, int64_t s1, int64_t s2, int64_t sz) {
            return reinterpret_cast<uintptr_t>(p) % 16 == 0 && s1 % VE == 0 && s2 % VE == 0 && sz % VE == 0;
        };
        const bool akf = g.a_sk == 1, bkf = g.b_sk == 1 && g.b_sj != 1;
        const int va = akf ? aligned(g.A, g.a_si, 0, g.a_sz) : g.a_si == 1 && aligned(g.A, g.a_sk, 0, g.a_sz);
        const int vb = bkf ? aligned(g.B, g.b_sj, 0, g.b_sz) : g.b_sj == 1 && aligned(g.B, g.b_sk, 0, g.b_sz);
        if (akf && bkf) hipLaunchKernelGGL((bgemm2_kernel<T, 128, 128, 32, 4, 2, true, true>), grid, dim3(512), 0, s, g, va, vb);
        else if (akf) hipLaunchKernelGGL((bgemm2_kernel<T, 128, 128, 32, 4, 2, true, false>), grid, dim3(512), 0, s, g, va, vb);
        else if (bkf) hipLaunchKernelGGL((bgemm2_kernel<T, 128, 128, 32, 4, 2, false, true>), grid, dim3(512), 0, s, g, va, vb);
        else hipLaunchKernelGGL((bgemm2_kernel<T, 128, 128, 32, 4, 2, false, false>), grid, dim3(512), 0, s, g, va, vb);
    } else if (tall) {
        hipLaunchKernelGGL((bgemm_kernel<T, 128, 64, 16>), grid, dim3(256), 0, s, g);
    } else {
        hipLaunchKernelGGL((bgemm_kernel<T, 64, 64, 16>), grid, dim3(256), 0, s, g);
    }
    if (nsplit > 1) {
        const int64_t tot = batch * M * N;
        hipLaunchKernelGGL((bgemm_splitk_reduce<T>), dim3(static_cast<unsigned>(cdiv(tot, 256))), dim3(256), 0, s,
                           sw.p, static_cast<int>(nsplit), batch, M, N, alpha, beta, c0.p, c0.si, c0.sj, c0.sz,
                           c.p, c.si, c.sj, c.sz);
    }
    return hipGetLastError();
}

// C = alpha [A1 A2] [B1; B2] + beta C0 over the reductions K1 then K2 (each a multiple of
// 32), on the 128 x 128 two-stage kernel without K splits, so C is written once.  Both A
// segments must share their layout (k-contiguous or not), both B segments likewise;
// hipErrorNotSupported when the shape or the layouts do not fit.
template <typename T>
hipError_t bgemm_2seg(int64_t batch, int64_t M, int64_t N, int64_t K1, BV<T> a1, BV<T> b1, int64_t K2,
                      BV<T> a2, BV<T> b2, T alpha, T beta, BV<T> c0, BMV<T> c, hipStream_t s) {
    if (batch <= 0 || batch > 65535 || M < 128 || N < 128 || K1 <= 0 || K2 <= 0 || K1 % 32 != 0 ||
        K2 % 32 != 0)
        return hipErrorNotSupported;
    const bool akf = a1.sj == 1, bkf = b1.si == 1 && b1.sj != 1;
    if ((a2.sj == 1) != akf || (b2.si == 1 && b2.sj != 1) != bkf) return hipErrorNotSupported;
    BGemm<T> g{};
    g.M = M; g.N = N; g.K = K1 + K2; g.K1 = K1;
    g.A = a1.p; g.a_si = a1.si; g.a_sk = a1.sj; g.a_sz = a1.sz;
    g.B = b1.p; g.b_sk = b1.si; g.b_sj = b1.sj; g.b_sz = b1.sz;
    g.A2 = a2.p; g.a2_si = a2.si; g.a2_sk = a2.sj; g.a2_sz = a2.sz;
    g.B2 = b2.p; g.b2_sk = b2.si; g.b2_sj = b2.sj; g.b2_sz = b2.sz;
    g.alpha = alpha; g.beta = beta;
    g.C0 = c0.p; g.c0_si = c0.si; g.c0_sj = c0.sj; g.c0_sz = c0.sz;
    g.C = c.p; g.c_si = c.si; g.c_sj = c.sj; g.c_sz = c.sz;
    g.tiles_n = static_cast<int>(cdiv(N, 128));
    g.kchunk = g.K;
    g.P = nullptr;
    constexpr int64_t VE = 16 / sizeof(T);
    auto aligned = [&](const T* p, int64_t s1, int64_t sz) {
        return reinterpret_cast<uintptr_t>(p) % 16 == 0 && s1 % VE == 0 && sz % VE == 0;
    };
    // 16-byte loads only when every matrix of both segments allows them
    const int va = akf ? aligned(a1.p, a1.si, a1.sz) && aligned(a2.p, a2.si, a2.sz)
                       : a1.si == 1 && a2.si == 1 && aligned(a1.p, a1.sj, a1.sz) && aligned(a2.p, a2.sj, a2.sz);
    const int vb = bkf ? aligned(b1.p, b1.sj, b1.sz) && aligned(b2.p, b2.sj, b2.sz)
                       : b1.sj == 1 && b2.sj == 1 && aligned(b1.p, b1.si, b1.sz) && aligned(b2.p, b2.si, b2.sz);
    const dim3 grid(static_cast<unsigned>(cdiv(M, 128) * g.tiles_n), 1u, static_cast<unsigned>(batch));
    if (akf && bkf) hipLaunchKernelGGL((bgemm2_kernel<T, 128, 128, 32, 4, 2, true, true>), grid, dim3(512), 0, s, g, va, vb);
    else if (akf) hipLaunchKernelGGL((bgemm2_kernel<T, 128, 128, 32, 4, 2, true, false>), grid, dim3(512), 0, s, g, va, vb);
    else if (bkf) hipLaunchKernelGGL((bgemm2_kernel<T, 128, 128, 32, 4, 2, false, true>), grid, dim3(512), 0, s, g, va, vb);
    else hipLaunchKernelGGL((bgemm2_kernel<T, 128, 128, 32, 4, 2, false, false>), grid, dim3(512), 0, s, g, va, vb);
    return hipGetLastError();
}

// ------------------------------------------------------------------ small factorisations

// Cholesky of each b x b Gram matrix (row-major, batch stride b*b): Gram = R^T R with R
// upper triangular, and R^{-1} by back substitution.  A pivot <= tau * max diag(Gram)
// (or not finite) sets *flag.  One workgroup per matrix, b <= 64.
template <typename T>
__global__ void __launch_bounds__(256)
chol_inv_batched_kernel(const T* __restrict__ gram, int b, T tau, T* __restrict__ R,
                        T* __restrict__ Rinv, int* __restrict__ flag) {
    __shared__ T S[64 * 65];
    __shared__ T V[64 * 65];   // R^{-1}
    __shared__ T piv;
    const int64_t z = blockIdx.x;
    const T* Gz = gram + z * b * b;
    T* Rz = R + z * b * b;
    T* Iz = Rinv + z * b * b;
    const int tid = threadIdx.x;
    for (int e = tid; e < b * b; e += blockDim.x) S[(e / b) * 65 + e % b] = Gz[e];
    __syncthreads();
    T dmax = T(0);
    for (int j = 0; j < b; ++j) dmax = S[j * 65 + j] > dmax ? S[j * 65 + j] : dmax;
    for (int j = 0; j < b; ++j) {
        if (tid == 0) {
            const T d = S[j * 65 + j];
            if (!(d > tau * dmax)) *flag = 1;
            piv = d > T(0) ? sqrt(d) : T(1);
        }
        __syncthreads();
        const T p = piv;
        // row j of R: R(j, c) = S(j, c) / p for c >= j (upper part of S holds the update)
        for (int c = j + tid; c < b; c += blockDim.x) S[j * 65 + c] = c == j ? p : S[j * 65 + c] / p;
        __syncthreads();
        // trailing update S(r, c) -= R(j, r) R(j, c) for j < r <= c
        const int rem = b - j - 1;
        for (int e = tid; e < rem * rem; e += blockDim.x) {
            const int r = j + 1 + e / rem, c = j + 1 + e % rem;
            if (c >= r) S[r * 65 + c] -= S[j * 65 + r] * S[j * 65 + c];
        }
        __syncthreads();
    }
    for (int e = tid; e < b * b; e += blockDim.x) {
        const int r = e / b, c = e % b;
        Rz[e] = c >= r ? S[r * 65 + c] : T(0);
    }
    // R^{-1}: thread c solves R x = e_c from the bottom row up (column c of R^{-1}), in LDS
    __syncthreads();
    if (tid < b) {
        const int c = tid;
        for (int r = b - 1; r >= 0; --r) {
            T v = r == c ? T(1) : T(0);
            for (int t = r + 1; t <= c; ++t) v -= S[r * 65 + t] * V[t * 65 + c];
            V[r * 65 + c] = r <= c ? v / S[r * 65 + r] : T(0);
        }
    }
    __syncthreads();
    for (int e = tid; e < b * b; e += blockDim.x) Iz[e] = V[(e / b) * 65 + e % b];
}

// Inverse of the upper triangle of each k x k matrix (row-major, row stride ld, batch
// stride sz) into Rinv (k x k row-major, batch stride k*k).  One workgroup per matrix,
// k <= 256; thread c computes column c by back substitution reading R from global memory.
template <typename T>
__global__ void __launch_bounds__(256)
tri_inv_batched_kernel(const T* __restrict__ R, int k, int64_t ld, int64_t sz, T* __restrict__ Rinv) {
    const int64_t z = blockIdx.x;
    const T* Rz = R + z * sz;
    T* Iz = Rinv + z * static_cast<int64_t>(k) * k;
    const int c = threadIdx.x;
    if (c >= k) return;
    for (int r = k - 1; r >= 0; --r) {
        T v = r == c ? T(1) : T(0);
        if (r <= c) {
            for (int t = r + 1; t <= c; ++t) v -= Rz[r * ld + t] * Iz[static_cast<int64_t>(t) * k + c];
            v /= Rz[r * ld + r];
        } else {
            v = T(0);
        }
        Iz[static_cast<int64_t>(r) * k + c] = v;
    }
}

// The same inverse with R and R^{-1} in LDS (k <= KMAX): R's entries are read by all threads
// at once, each thread's column of R^{-1} stays in LDS.
template <typename T, int KMAX>
__global__ void __launch_bounds__(256)
tri_inv_lds_kernel(const T* __restrict__ R, int k, int64_t ld, int64_t sz, T* __restrict__ Rinv) {
    __shared__ T S[KMAX * (KMAX + 1)];
    __shared__ T V[KMAX * (KMAX + 1)];
    constexpr int P = KMAX + 1;
    const int64_t z = blockIdx.x;
    const T* Rz = R + z * sz;
    T* Iz = Rinv + z * static_cast<int64_t>(k) * k;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int r = e / k, c = e % k;
        S[r * P + c] = c >= r ? Rz[r * ld + c] : T(0);
    }
    __syncthreads();
    const int c = threadIdx.x;
    if (c < k) {
        for (int r = k - 1; r >= 0; --r) {
            // four interleaved partial sums (fixed order) keep the LDS loads in flight
            T v0 = T(0), v1 = T(0), v2 = T(0), v3 = T(0);
            int t = r + 1;
            for (; t + 3 <= c; t += 4) {
                v0 += S[r * P + t] * V[t * P + c];
                v1 += S[r * P + t + 1] * V[(t + 1) * P + c];
                v2 += S[r * P + t + 2] * V[(t + 2) * P + c];
                v3 += S[r * P + t + 3] * V[(t + 3) * P + c];
            }
            for (; t <= c; ++t) v0 += S[r * P + t] * V[t * P + c];
            const T v = (r == c ? T(1) : T(0)) - ((v0 + v1) + (v2 + v3));
            V[r * P + c] = r <= c ? v / S[r * P + r] : T(0);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) Iz[e] = V[(e / k) * P + e % k];
}

// C = copyltu(M): C(r, c) = M(max(r, c), min(r, c)) for each k x k matrix (batch stride k*k).
template <typename T>
__global__ void __launch_bounds__(256)
copyltu_batched_kernel(const T* __restrict__ M, int k, int64_t total, T* __restrict__ C) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t kk = static_cast<int64_t>(k) * k;
    const int64_t z = e / kk, w = e % kk;
    const int r = static_cast<int>(w / k), c = static_cast<int>(w % k);
    const int hi = r > c ? r : c, lo = r > c ? c : r;
    C[e] = M[z * kk + static_cast<int64_t>(hi) * k + lo];
}

__global__ void __launch_bounds__(256)
f64_to_f32_kernel(const double* __restrict__ x, int64_t len, float* __restrict__ y) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < len) y[e] = static_cast<float>(x[e]);
}

// ------------------------------------------------------------------ host

namespace {

constexpr int kMaxDiffB = 64;
constexpr int kMaxDiffK = 256;

struct DiffLayout {
    size_t om64, om, g, h, y, x, w, z, d, s, gram, r1, r1i, rt, rti, ri, rii, flag,
        r, rinv, qt, mm, cs, yb, omt, split, total;
    int64_t split_elems;
};

// split-K partials: the k x k products of the backward (8 splits) and the k x b ones of
// the forward (16 splits) fit
int64_t split_elems(int64_t batch, int64_t k, int64_t b) {
    int64_t e = 8 * batch * k * k;
    if (e < 16 * batch * k * b) e = 16 * batch * k * b;
    return e < (int64_t(1) << 22) ? (int64_t(1) << 22) : e;
}

size_t al256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

template <typename T>
DiffLayout diff_layout(int64_t batch, int64_t m, int64_t n, int64_t k, int64_t b) {
    DiffLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = al256(off + bytes);
        return o;
    };
    const size_t E = sizeof(T);
    L.om64 = take(sizeof(T) == sizeof(float) ? sizeof(double) * n * k : 0);
    L.om = take(E * n * k);
    L.g = take(E * batch * m * k);
    L.h = take(E * batch * n * k);
    L.y = take(E * batch * m * b);
    L.x = take(E * batch * m * b);
    L.w = take(E * batch * k * b);
    L.z = take(E * batch * k * b);
    L.d = take(E * batch * k * b);
    L.s = take(E * batch * n * b);
    L.gram = take(E * batch * b * b);
    L.r1 = take(E * batch * b * b);
    L.r1i = take(E * batch * b * b);
    L.rt = take(E * batch * b * b);
    L.rti = take(E * batch * b * b);
    L.ri = take(E * batch * b * b);
    L.rii = take(E * batch * b * b);
    L.flag = take(sizeof(int) * 4);
    // backward: R = Q^T G and its inverse, Qt, M, copyltu(M), Y-bar
    L.r = take(E * batch * k * k);
    L.rinv = take(E * batch * k * k);
    L.qt = take(E * batch * m * k);
    L.mm = take(E * batch * k * k);
    L.cs = take(E * batch * k * k);
    L.yb = take(E * batch * m * k);
    L.omt = take(E * k * n);   // Omega^T, rows of n (the backward's last product)
    L.split_elems = split_elems(batch, k, b);
    L.split = take(E * L.split_elems);
    L.total = off + 256;
    return L;
}

size_t diff_bytes(const qb_batch* A, int64_t k, int32_t b) {
    if (A->dtype == QB_F32) return diff_layout<float>(A->batch, A->m, A->n, k, b).total;
    return diff_layout<double>(A->batch, A->m, A->n, k, b).total;
}

int check_batch(const qb_batch* A, int64_t k, int32_t b) {
    if (A == nullptr || A->a == nullptr || A->batch < 1 || A->batch > 65535 || A->m < 1 || A->n < 1 ||
        A->lda < A->n || A->stride_a < 0)
        return QB_ERR_ARG;
    if (A->batch > 1 && A->stride_a < A->m * A->lda) return QB_ERR_ARG;
    if (A->dtype != QB_F32 && A->dtype != QB_F64) return QB_ERR_UNSUPPORTED;
    if (b < 1 || b > kMaxDiffB || k < 1 || k > kMaxDiffK || k % b != 0) return QB_ERR_ARG;
    if (k > A->m || k > A->n) return QB_ERR_ARG;
    return QB_OK;
}

#define QB_DHIP(expr)                                 \
    do {                                              \
        const hipError_t qb_e_ = (expr);              \
        if (qb_e_ != hipSuccess) return QB_ERR_HIP;   \
    } while (0)

// Omega (n x k, row-major) in the element type, from the bit-specified generator
// (binary32: each binary64 value rounded to nearest).
template <typename T>
int make_omega(uint64_t seed, int64_t n, int64_t k, char* ws, const DiffLayout& L, hipStream_t s) {
    if constexpr (sizeof(T) == sizeof(float)) {
        double* om64 = reinterpret_cast<double*>(ws + L.om64);
        QB_DHIP(launch_gauss_fill(seed, 0, 0, 0, 0, n, k, om64, k, s));
        const int64_t len = n * k;
        hipLaunchKernelGGL(f64_to_f32_kernel, dim3(static_cast<unsigned>(cdiv(len, 256))), dim3(256), 0,
                           s, om64, len, reinterpret_cast<float*>(ws + L.om));
        QB_DHIP(hipGetLastError());
    } else {
        QB_DHIP(launch_gauss_fill(seed, 0, 0, 0, 0, n, k, reinterpret_cast<double*>(ws + L.om), k, s));
    }
    return QB_OK;
}

template <typename T>
int cholqr_b(int64_t batch, int64_t m, int b, const T* X, int64_t xsz, T* Qout, int64_t q_si,
             int64_t q_sz, T* gram, T* R, T* Rinv, int* flag, hipStream_t s, SplitWs<T> SW) {
    // Gram = X^T X (X: m x b row-major per matrix)
    QB_DHIP(bgemm<T>(batch, b, b, m, BV<T>{X, 1, b, xsz}, BV<T>{X, b, 1, xsz}, T(1), T(0),
                     BV<T>{nullptr, 0, 0, 0}, BMV<T>{gram, b, 1, static_cast<int64_t>(b) * b}, s, SW));
    const T tau = sizeof(T) == sizeof(float) ? T(1e-6) : T(1e-12);
    hipLaunchKernelGGL((chol_inv_batched_kernel<T>), dim3(static_cast<unsigned>(batch)), dim3(256), 0, s,
                       gram, b, tau, R, Rinv, flag);
    QB_DHIP(hipGetLastError());
    // Q = X R^{-1}
    QB_DHIP(bgemm<T>(batch, m, b, b, BV<T>{X, b, 1, xsz}, BV<T>{Rinv, b, 1, static_cast<int64_t>(b) * b},
                     T(1), T(0), BV<T>{nullptr, 0, 0, 0}, BMV<T>{Qout, q_si, 1, q_sz}, s, SW));
    return QB_OK;
}

template <typename T>
int fixed_fwd(const qb_batch* Ab, int64_t k, int b, uint64_t seed, T* Q, int64_t ldq, int64_t sq, T* B,
              int64_t ldb, int64_t sb, char* ws, const DiffLayout& L, hipStream_t s, int* host_flag,
              int32_t* dev_flag) {
    const int64_t bt = Ab->batch, m = Ab->m, n = Ab->n;
    const T* A = static_cast<const T*>(Ab->a);
    const int64_t lda = Ab->lda, sa = Ab->stride_a;
    auto P = [&](size_t off) { return reinterpret_cast<T*>(ws + off); };
    T *Om = P(L.om), *G = P(L.g), *H = P(L.h), *Y = P(L.y), *X = P(L.x), *W = P(L.w), *Z = P(L.z),
      *D = P(L.d), *S = P(L.s), *gram = P(L.gram), *R1 = P(L.r1), *R1i = P(L.r1i), *Rt = P(L.rt),
      *Rti = P(L.rti), *Ri = P(L.ri), *Rii = P(L.rii);
    int* flag = reinterpret_cast<int*>(ws + L.flag);
    const BV<T> none{nullptr, 0, 0, 0};
    const SplitWs<T> SW{P(L.split), L.split_elems};
    const int64_t bb = static_cast<int64_t>(b) * b;
    QB_DHIP(launch_fill_int(flag, 1, 0, s));
    if (int e = make_omega<T>(seed, n, k, ws, L, s)) return e;
    // G = A Omega (m x k), H = A^T G (n x k), row-major per matrix
    QB_DHIP(bgemm<T>(bt, m, k, n, BV<T>{A, lda, 1, sa}, BV<T>{Om, k, 1, 0}, T(1), T(0), none,
                     BMV<T>{G, k, 1, m * k}, s, SW));
    QB_DHIP(bgemm<T>(bt, n, k, m, BV<T>{A, 1, lda, sa}, BV<T>{G, k, 1, m * k}, T(1), T(0), none,
                     BMV<T>{H, k, 1, n * k}, s, SW));
    for (int64_t j0 = 0; j0 < k; j0 += b) {
        const int64_t ki = j0;   // columns of Q / rows of B so far
        // W = B(0:ki, :) Omega_J  (ki x b)
        QB_DHIP(bgemm<T>(bt, ki, b, n, BV<T>{B, ldb, 1, sb}, BV<T>{Om + j0, k, 1, 0}, T(1), T(0), none,
                         BMV<T>{W, b, 1, k * b}, s, SW));
        // Y = G_J - Q(:, 0:ki) W  (m x b row-major)
        QB_DHIP(bgemm<T>(bt, m, b, ki, BV<T>{Q, ldq, 1, sq}, BV<T>{W, b, 1, k * b}, T(-1), T(1),
                         BV<T>{G + j0, k, 1, m * k}, BMV<T>{Y, b, 1, m * b}, s, SW));
        // first qr: X = Y R1^{-1}
        if (int e = cholqr_b<T>(bt, m, b, Y, m * b, X, b, m * b, gram, R1, R1i, flag, s, SW)) return e;
        // re-orthogonalisation: Z = Q^T X, X2 = X - Q Z -> written into the Q panel
        QB_DHIP(bgemm<T>(bt, ki, b, m, BV<T>{Q, 1, ldq, sq}, BV<T>{X, b, 1, m * b}, T(1), T(0), none,
                         BMV<T>{Z, b, 1, k * b}, s, SW));
        QB_DHIP(bgemm<T>(bt, m, b, ki, BV<T>{Q, ldq, 1, sq}, BV<T>{Z, b, 1, k * b}, T(-1), T(1),
                         BV<T>{X, b, 1, m * b}, BMV<T>{X, b, 1, m * b}, s, SW));
        if (int e = cholqr_b<T>(bt, m, b, X, m * b, Q + j0, ldq, sq, gram, Rt, Rti, flag, s, SW)) return e;
        // R_i = R~ R1 and R_i^{-1} = R1^{-1} R~^{-1}
        QB_DHIP(bgemm<T>(bt, b, b, b, BV<T>{Rt, b, 1, bb}, BV<T>{R1, b, 1, bb}, T(1), T(0), none,
                         BMV<T>{Ri, b, 1, bb}, s, SW));
        QB_DHIP(bgemm<T>(bt, b, b, b, BV<T>{R1i, b, 1, bb}, BV<T>{Rti, b, 1, bb}, T(1), T(0), none,
                         BMV<T>{Rii, b, 1, bb}, s, SW));
        // D = Q(:, 0:ki)^T Y + W  (ki x b)
        QB_DHIP(bgemm<T>(bt, ki, b, m, BV<T>{Q, 1, ldq, sq}, BV<T>{Y, b, 1, m * b}, T(1), T(1),
                         BV<T>{W, b, 1, k * b}, BMV<T>{D, b, 1, k * b}, s, SW));
        // S^T = H_J - B(0:ki, :)^T D  (n x b row-major)
        QB_DHIP(bgemm<T>(bt, n, b, ki, BV<T>{B, 1, ldb, sb}, BV<T>{D, b, 1, k * b}, T(-1), T(1),
                         BV<T>{H + j0, k, 1, n * k}, BMV<T>{S, b, 1, n * b}, s, SW));
        // B_i^T = S^T R_i^{-1}, written transposed into rows j0.. of B
        QB_DHIP(bgemm<T>(bt, n, b, b, BV<T>{S, b, 1, n * b}, BV<T>{Rii, b, 1, bb}, T(1), T(0), none,
                         BMV<T>{B + j0 * ldb, 1, ldb, sb}, s, SW));
    }
    if (dev_flag != nullptr) {   // stream-ordered report, no host wait
        QB_DHIP(hipMemcpyAsync(dev_flag, flag, sizeof(int), hipMemcpyDeviceToDevice, s));
        return QB_OK;
    }
    QB_DHIP(hipMemcpyAsync(host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    QB_DHIP(hipStreamSynchronize(s));
    return QB_OK;
}

template <typename T>
int fixed_bwd(const qb_batch* Ab, int64_t k, uint64_t seed, const T* Q, int64_t ldq, int64_t sq,
              const T* dQ, int64_t lddq, int64_t sdq, const T* dB, int64_t lddb, int64_t sdb, T* dA,
              int64_t ldda, int64_t sda, char* ws, const DiffLayout& L, hipStream_t s) {
    const int64_t bt = Ab->batch, m = Ab->m, n = Ab->n;
    const T* A = static_cast<const T*>(Ab->a);
    const int64_t lda = Ab->lda, sa = Ab->stride_a;
    auto P = [&](size_t off) { return reinterpret_cast<T*>(ws + off); };
    T *Om = P(L.om), *G = P(L.g), *R = P(L.r), *Rinv = P(L.rinv), *Qt = P(L.qt), *Mm = P(L.mm),
      *Cs = P(L.cs), *Yb = P(L.yb);
    const BV<T> none{nullptr, 0, 0, 0};
    const SplitWs<T> SW{P(L.split), L.split_elems};
    const int64_t kk = k * k;
    if (int e = make_omega<T>(seed, n, k, ws, L, s)) return e;
    // recompute G = A Omega and R = Q^T G (upper triangular up to round-off)
    QB_DHIP(bgemm<T>(bt, m, k, n, BV<T>{A, lda, 1, sa}, BV<T>{Om, k, 1, 0}, T(1), T(0), none,
                     BMV<T>{G, k, 1, m * k}, s, SW));
    QB_DHIP(bgemm<T>(bt, k, k, m, BV<T>{Q, 1, ldq, sq}, BV<T>{G, k, 1, m * k}, T(1), T(0), none,
                     BMV<T>{R, k, 1, kk}, s, SW));
    // R^{-1} in LDS when it fits (binary32 k <= 128, binary64 k <= 64), else from global
    constexpr int kLds = sizeof(T) == sizeof(float) ? 128 : 64;
    if (k <= kLds)
        hipLaunchKernelGGL((tri_inv_lds_kernel<T, kLds>), dim3(static_cast<unsigned>(bt)), dim3(256), 0, s, R,
                           static_cast<int>(k), k, kk, Rinv);
    else
        hipLaunchKernelGGL((tri_inv_batched_kernel<T>), dim3(static_cast<unsigned>(bt)), dim3(256), 0, s, R,
                           static_cast<int>(k), k, kk, Rinv);
    QB_DHIP(hipGetLastError());
    // Qt = dQ + A dB^T  (m x k)
    const bool has_dq = dQ != nullptr, has_db = dB != nullptr;
    if (has_db) {
        QB_DHIP(bgemm<T>(bt, m, k, n, BV<T>{A, lda, 1, sa}, BV<T>{dB, 1, lddb, sdb}, T(1),
                         has_dq ? T(1) : T(0), has_dq ? BV<T>{dQ, lddq, 1, sdq} : none,
                         BMV<T>{Qt, k, 1, m * k}, s, SW));
    } else if (has_dq) {
        QB_DHIP(bgemm<T>(bt, m, k, 0, none, none, T(0), T(1), BV<T>{dQ, lddq, 1, sdq},
                         BMV<T>{Qt, k, 1, m * k}, s, SW));
    } else {
        QB_DHIP(bgemm<T>(bt, m, k, 0, none, none, T(0), T(0), none, BMV<T>{Qt, k, 1, m * k}, s, SW));
    }
    // M = -Qt^T Q (k x k), Cs = copyltu(M)
    QB_DHIP(bgemm<T>(bt, k, k, m, BV<T>{Qt, 1, k, m * k}, BV<T>{Q, ldq, 1, sq}, T(-1), T(0), none,
                     BMV<T>{Mm, k, 1, kk}, s, SW));
    const int64_t tot = bt * kk;
    hipLaunchKernelGGL((copyltu_batched_kernel<T>), dim3(static_cast<unsigned>(cdiv(tot, 256))), dim3(256), 0,
                       s, Mm, static_cast<int>(k), tot, Cs);
    QB_DHIP(hipGetLastError());
    // Qt <- Qt + Q Cs ; Y-bar = Qt R^{-T}
    QB_DHIP(bgemm<T>(bt, m, k, k, BV<T>{Q, ldq, 1, sq}, BV<T>{Cs, k, 1, kk}, T(1), T(1),
                     BV<T>{Qt, k, 1, m * k}, BMV<T>{Qt, k, 1, m * k}, s, SW));
    QB_DHIP(bgemm<T>(bt, m, k, k, BV<T>{Qt, k, 1, m * k}, BV<T>{Rinv, 1, k, kk}, T(1), T(0), none,
                     BMV<T>{Yb, k, 1, m * k}, s, SW));
    // dA = Q dB + Y-bar Omega^T.  Omega^T is copied with rows of n (0.5 MB at n = 1024, k = 128)
    // so that both products read their right operand the same way; then, when the shape
    // allows, one pass [Q Y-bar] [dB; Omega^T] writes dA once instead of writing it and
    // reading it back for the second product.
    T* OmT = P(L.omt);
    QB_DHIP(bgemm<T>(1, k, n, 0, none, none, T(0), T(1), BV<T>{Om, 1, k, 0}, BMV<T>{OmT, n, 1, 0}, s, SW));
    if (has_db) {
        const hipError_t e = bgemm_2seg<T>(bt, m, n, k, BV<T>{Q, ldq, 1, sq}, BV<T>{dB, lddb, 1, sdb}, k,
                                           BV<T>{Yb, k, 1, m * k}, BV<T>{OmT, n, 1, 0}, T(1), T(0), none,
                                           BMV<T>{dA, ldda, 1, sda}, s);
        if (e == hipSuccess) return QB_OK;
        if (e != hipErrorNotSupported) return QB_ERR_HIP;
        QB_DHIP(bgemm<T>(bt, m, n, k, BV<T>{Q, ldq, 1, sq}, BV<T>{dB, lddb, 1, sdb}, T(1), T(0), none,
                         BMV<T>{dA, ldda, 1, sda}, s, SW));
    }
    QB_DHIP(bgemm<T>(bt, m, n, k, BV<T>{Yb, k, 1, m * k}, BV<T>{OmT, n, 1, 0}, T(1),
                     has_db ? T(1) : T(0), has_db ? BV<T>{dA, ldda, 1, sda} : none,
                     BMV<T>{dA, ldda, 1, sda}, s, SW));
    return QB_OK;
}

}  // namespace
}  // namespace qb

using namespace qb;

extern "C" {

size_t qb_fixed_rank_workspace_bytes(const qb_batch* A, int64_t k, int32_t b) {
    if (check_batch(A, k, b) != QB_OK) return 0;
    return diff_bytes(A, k, b);
}

int qb_fixed_rank_fwd(const qb_batch* A, int64_t k, int32_t b, uint64_t seed, void* Q, int64_t ldq,
                      int64_t stride_q, void* B, int64_t ldb, int64_t stride_b, void* ws,
                      size_t ws_bytes, int32_t* breakdown, hipStream_t stream) {
    if (int st = check_batch(A, k, b)) return st;
    if (Q == nullptr || B == nullptr || ws == nullptr || ldq < k || ldb < A->n) return QB_ERR_ARG;
    if (A->batch > 1 && (stride_q < A->m * ldq || stride_b < k * ldb)) return QB_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return QB_ERR_ARG;
    if (ws_bytes < diff_bytes(A, k, b)) return QB_ERR_WORKSPACE;
    char* w = static_cast<char*>(ws);
    int flag = 0;
    int st;
    if (A->dtype == QB_F32) {
        const DiffLayout L = diff_layout<float>(A->batch, A->m, A->n, k, b);
        st = fixed_fwd<float>(A, k, b, seed, static_cast<float*>(Q), ldq, stride_q, static_cast<float*>(B),
                              ldb, stride_b, w, L, stream, &flag, breakdown);
    } else {
        const DiffLayout L = diff_layout<double>(A->batch, A->m, A->n, k, b);
        st = fixed_fwd<double>(A, k, b, seed, static_cast<double*>(Q), ldq, stride_q,
                               static_cast<double*>(B), ldb, stride_b, w, L, stream, &flag, breakdown);
    }
    if (st != QB_OK) return st;
    return flag ? QB_NOT_CONVERGED : QB_OK;
}

int qb_fixed_rank_bwd(const qb_batch* A, int64_t k, int32_t b, uint64_t seed, const void* Q,
                      int64_t ldq, int64_t stride_q, const void* dQ, int64_t lddq, int64_t stride_dq,
                      const void* dB, int64_t lddb, int64_t stride_db, void* dA, int64_t ldda,
                      int64_t stride_da, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (int st = check_batch(A, k, b)) return st;
    if (Q == nullptr || dA == nullptr || ws == nullptr || ldq < k || ldda < A->n) return QB_ERR_ARG;
    if (dQ != nullptr && lddq < k) return QB_ERR_ARG;
    if (dB != nullptr && lddb < A->n) return QB_ERR_ARG;
    if (A->batch > 1 && (stride_q < A->m * ldq || stride_da < A->m * ldda ||
                         (dQ != nullptr && stride_dq < A->m * lddq) ||
                         (dB != nullptr && stride_db < k * lddb)))
        return QB_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return QB_ERR_ARG;
    if (ws_bytes < diff_bytes(A, k, b)) return QB_ERR_WORKSPACE;
    char* w = static_cast<char*>(ws);
    if (A->dtype == QB_F32) {
        const DiffLayout L = diff_layout<float>(A->batch, A->m, A->n, k, b);
        return fixed_bwd<float>(A, k, seed, static_cast<const float*>(Q), ldq, stride_q,
                                static_cast<const float*>(dQ), lddq, stride_dq,
                                static_cast<const float*>(dB), lddb, stride_db, static_cast<float*>(dA),
                                ldda, stride_da, w, L, stream);
    }
    const DiffLayout L = diff_layout<double>(A->batch, A->m, A->n, k, b);
    return fixed_bwd<double>(A, k, seed, static_cast<const double*>(Q), ldq, stride_q,
                             static_cast<const double*>(dQ), lddq, stride_dq,
                             static_cast<const double*>(dB), lddb, stride_db, static_cast<double*>(dA),
                             ldda, stride_da, w, L, stream);
}

}  // extern "C"
