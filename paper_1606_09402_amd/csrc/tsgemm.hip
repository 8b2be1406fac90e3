// Narrow FP64 products of the block loop (at most 64 output columns) on CDNA4 matrix cores,
// with the MFMA operands loaded from global memory straight into registers: no LDS staging
// and no barrier in the main loop, so every wave streams its operand independently and keeps
// several k-steps of loads in flight.  These products (the block loop of Algorithm 4 and
// eq. (23): B Omega_J, G_J - Q W, the Gram matrices of CholeskyQR, Q^T Q_i, Q_i - Q Z,
// Q^T Y, H_J - B^T D) each read an m x k or k x n panel once and sit at the ridge of the FP64 roofline (2 b flops per 8 bytes
// of the panel), so the panel has to stream at the rate the matrix cores consume it.
//
// v_mfma_f64_16x16x4f64 takes A(i, k) from lane 16 k + i and B(k, j) from lane 16 k + j, and
// leaves C(4 r + l / 16, l mod 16) in slot r of lane l.  Which reduction index a lane supplies,
// and which output row an MFMA row stands for, are free as long as both operands agree; the
// kernels use that freedom to give each lane 16- or 32-byte contiguous loads:
//
//  * panel form, A column-major (rows contiguous): lane (i, k) loads FM consecutive rows
//    r0 + FM i + e (e < FM) of column k; MFMA e then computes output rows r0 + FM v + e.
//  * reduction form, A(i, k) with k contiguous (A^T of a column-major panel, or a row-major
//    panel) and a long reduction: lane (i, q) loads reduction indices base + 4 q + s (s < 4)
//    of row i, and k-step s of the group uses reduction index base + 4 q + s in both operands.
//
// Reductions split over the waves of a workgroup are combined through LDS in wave order, and
// splits over workgroups through a partial buffer summed in split order by the split-K kernels
// of gemm.hip, so results do not depend on timing.
#include <cstdlib>

#include "kernels.h"

namespace qb {

struct TsArgs {
    int64_t M, N, K;
    const double* A;
    int64_t lda;          // stride of A's non-contiguous index
    const double* B;
    int64_t bsk, bsj;     // B(k, j) = B[k * bsk + j * bsj]
    double alpha, beta;
    const double* C0;
    int64_t c0_si, c0_sj;
    double* C;
    int64_t c_si, c_sj;
    double* P;            // split partials [nsplit][M][N] (gridDim split > 1)
    int64_t kchunk;       // reduction range of one split
    int tiles;            // output row tiles
    int nsplit;
    int nt_a;             // stream A with non-temporal loads
    const int* gate;
};

QB_DEV v4d ts_mfma(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Loads at a wave-uniform base plus a 32-bit per-lane byte offset, as buffer loads: the base
// sits in a scalar resource rebuilt per step, the lane offsets stay fixed in the loop, and no
// 64-bit address is formed per load (the data format word is the one of the gfx9 family).
typedef unsigned int ts_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int ts_u32x2 __attribute__((ext_vector_type(2)));
QB_DEV __amdgpu_buffer_rsrc_t ts_rsrc(const double* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0, 0x7FFFFFFF, 0x00020000);
}
QB_DEV double2 ts_ld2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
QB_DEV double ts_ld1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Sum the accumulators of the WAVES waves of a workgroup into wave 0 in wave order.
template <int NACC, int WAVES>
QB_DEV void ts_wave_reduce(double* red, double (&acc)[NACC], int wave, int lane) {
    if (WAVES == 1) return;
    if (wave > 0) {
#pragma unroll
        for (int x = 0; x < NACC; ++x) red[((wave - 1) * NACC + x) * 64 + lane] = acc[x];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int w = 1; w < WAVES; ++w)
#pragma unroll
            for (int x = 0; x < NACC; ++x) acc[x] += red[((w - 1) * NACC + x) * 64 + lane];
    }
}

// Epilogue of one output element: final value or a split partial.
QB_DEV void ts_store(const TsArgs& g, int split, int64_t i, int64_t j, double v) {
    if (g.nsplit > 1) {
        g.P[(static_cast<int64_t>(split) * g.M + i) * g.N + j] = v;
        return;
    }
    double o = g.alpha * v;
    if (g.beta != 0.0) o += g.beta * g.C0[i * g.c0_si + j * g.c0_sj];
    g.C[i * g.c_si + j * g.c_sj] = o;
}

// ------------------------------------------------------------------ panel form
//
// C(M x N) = alpha A B + beta C0, A column-major (A(i, k) = A[i + k lda]), N <= 64.  A workgroup
// owns 16 FM output rows and the reduction range of its split; its WK waves take contiguous
// thirds/quarters of that range in k-steps of 4 columns.  Each lane keeps D k-steps of loads in
// flight (register ring).  EDGE: the row tile crosses M (clamped scalar loads).
template <int FM, int WK, int D, bool EDGE>
QB_DEV void ts_panel_body(const TsArgs& g, int64_t r0, int64_t kw, int64_t nst, int64_t ke,
                          double (&accf)[FM * 16]) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int64_t il = r0 + FM * li;
    // steps [0, nfull) have all four columns inside the reduction range; a last step that
    // crosses ke is done apart with masked loads
    const int64_t nfull = nst > 0 && kw + 4 * nst > ke ? nst - 1 : nst;
    double a[D][FM], b[D][4];
    constexpr int kPanelLoads = (EDGE || FM == 1 ? FM : FM / 2) + 4;   // vector loads per step
    // per-lane byte offsets from the step's column base A(r0, kcol) and row base B(kcol, 0)
    uint32_t aoff[FM], boff[4];
#pragma unroll
    for (int e = 0; e < FM; ++e) {
        const int64_t i = il + e < g.M ? il + e : g.M - 1;
        aoff[e] = static_cast<uint32_t>((lk * g.lda + (i - r0)) * 8);
    }
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
        const int64_t j = 16 * fn + li < g.N ? 16 * fn + li : g.N - 1;
        boff[fn] = static_cast<uint32_t>((lk * g.bsk + j * g.bsj) * 8);
    }
    // loads of the step whose four columns start at kcol (wave-uniform; kcol + 3 < K)
    auto load_col = [&](double (&av)[FM], double (&bv)[4], int64_t kcol) {
        const __amdgpu_buffer_rsrc_t ra = ts_rsrc(g.A + kcol * g.lda + r0);
        const __amdgpu_buffer_rsrc_t rb = ts_rsrc(g.B + kcol * g.bsk);
        if constexpr (!EDGE && FM == 4) {
            const double2 x0 = ts_ld2(ra, aoff[0]);
            const double2 x1 = ts_ld2(ra, aoff[0] + 16);
            av[0] = x0.x; av[1] = x0.y; av[2] = x1.x; av[3] = x1.y;
        } else if constexpr (!EDGE && FM == 2) {
            const double2 x0 = ts_ld2(ra, aoff[0]);
            av[0] = x0.x; av[1] = x0.y;
        } else {
#pragma unroll
            for (int e = 0; e < FM; ++e) av[e] = ts_ld1(ra, aoff[e]);
        }
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) bv[fn] = ts_ld1(rb, boff[fn]);
    };
    v4d acc[FM][4];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) acc[f][fn] = v4d{0.0, 0.0, 0.0, 0.0};
    auto step = [&](const double (&av)[FM], const double (&bv)[4]) {
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int f = 0; f < FM; ++f) acc[f][fn] = ts_mfma(av[f], bv[fn], acc[f][fn]);
    };
    if (nfull > 0) {
        // prefetch of steps beyond nfull re-reads the last full step (never used)
        auto col = [&](int64_t t) { return kw + 4 * (t < nfull ? t : nfull - 1); };
        // prologue: the first D steps.  The loaded values pass through a select before they
        // enter the loop-carried registers: with bare loads on both edges the compiler would
        // merge them with the loop's loads and issue them at the point of use, undoing the
        // prefetch; and with no load pending at loop entry, the waits inside the loop count
        // only the loop's own loads.  The select waits for the prologue loads once.
#pragma unroll
        for (int s = 0; s < D; ++s) {
            load_col(a[s], b[s], col(s));
            const bool v = s < nfull;
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) b[s][fn] = v ? b[s][fn] : 0.0;
#pragma unroll
            for (int e = 0; e < FM; ++e) a[s][e] = v ? a[s][e] : 0.0;
        }
        int64_t t = 0;
        for (; t + D <= nfull; t += D) {
#pragma unroll
            for (int s = 0; s < D; ++s) {
                step(a[s], b[s]);
                load_col(a[s], b[s], col(t + s + D));
                // keep the issue order MFMAs-then-loads per step, so the loads of step t + s + D
                // leave D - 1 steps of loads in flight behind them
                __builtin_amdgcn_sched_group_barrier(0x008, 4 * FM, 0);
                __builtin_amdgcn_sched_group_barrier(0x020, kPanelLoads, 0);
            }
        }
        const int64_t rem = nfull - t;   // steps t .. nfull - 1 sit in slots 0 .. rem - 1
#pragma unroll
        for (int s = 0; s < D - 1; ++s)
            if (s < rem) step(a[s], b[s]);
    }
    if (nfull < nst) {   // the step that crosses ke: columns at or beyond ke contribute zero
        const int64_t k0 = kw + 4 * nfull, k = k0 + lk;
        const bool v = k < ke;
        const int64_t kc = v ? k : ke - 1;
        double av[FM], bv[4];
#pragma unroll
        for (int e = 0; e < FM; ++e) {
            const int64_t i = il + e < g.M ? il + e : g.M - 1;
            av[e] = g.A[kc * g.lda + i];
        }
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) {
            const int64_t j = 16 * fn + li < g.N ? 16 * fn + li : g.N - 1;
            bv[fn] = v ? g.B[kc * g.bsk + j * g.bsj] : 0.0;
        }
        step(av, bv);
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) accf[(f * 4 + fn) * 4 + r] = acc[f][fn][r];
}

template <int FM, int WK, int D>
__global__ void __launch_bounds__(64 * WK) ts_panel_kernel(const TsArgs g) {
    if (g.gate != nullptr && *g.gate != 0) return;
    constexpr int NACC = FM * 16;
    __shared__ double red[(WK > 1 ? WK - 1 : 1) * NACC * 64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int li = lane & 15, lk = lane >> 4;
    const int tile = blockIdx.x % g.tiles, split = blockIdx.x / g.tiles;
    const int64_t r0 = static_cast<int64_t>(tile) * 16 * FM;
    const int64_t kb = static_cast<int64_t>(split) * g.kchunk;
    const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
    const int64_t steps = (ke - kb + 3) / 4;
    const int64_t t0 = steps * wave / WK, t1 = steps * (wave + 1) / WK;
    double acc[NACC];
    if (r0 + 16 * FM <= g.M)
        ts_panel_body<FM, WK, D, false>(g, r0, kb + 4 * t0, t1 - t0, ke, acc);
    else
        ts_panel_body<FM, WK, D, true>(g, r0, kb + 4 * t0, t1 - t0, ke, acc);
    ts_wave_reduce<NACC, WK>(red, acc, wave, lane);
    if (wave != 0) return;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = r0 + FM * ((r << 2) + lk) + f;
                const int64_t j = 16 * fn + li;
                if (i < g.M && j < g.N) ts_store(g, split, i, j, acc[(f * 4 + fn) * 4 + r]);
            }
}

// Panel form with the operands moved global -> LDS by the wave's own DMA instructions
// (global_load_lds_dwordx4) through a ring of D steps: step t + D - 1 is requested while step
// t is multiplied, and a wave waits only for its own DMAs, so no barrier is needed in the loop.
// No register holds data in flight, which leaves room for several waves per SIMD.  Full row
// tiles only (rows r0 .. r0 + 16 FM - 1 < M), FM 2 or 4, B row-major (bsj == 1) with N >= 2,
// A and B 16-byte aligned with even leading dimensions.
//
// Stage layout (bytes): A at 0 -- DMA h (h < FM / 2) fills 1 KB, lane l fetching rows
// FM (l mod 16) + 2 h, + 1 of column l / 16, which is exactly the MFMA operand pair of lane l;
// B at 512 FM -- DMA q (q < 2) fills rows 2 q, 2 q + 1 of the step's 4 x 64 row-major tile,
// lane l fetching the column pair 2 (l mod 32) of row 2 q + l / 32 (pairs past N re-read the
// last pair; those columns are never stored).
typedef __attribute__((address_space(3))) void* ts_lds_ptr;
QB_DEV constexpr int ts_vmcnt(int n) { return (n & 0xF) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

template <int FM>
struct PanelDma {
    static constexpr int A_BYTES = 512 * FM, STAGE = A_BYTES + 2048, ND = FM / 2 + 2;
};

// One DMA: 16 bytes per lane from base + off (off in bytes) into LDS at lds + 16 lane.  Inline
// assembly, so that the compiler does not make later LDS reads wait for it (the loop waits
// for its own DMAs); it has no register results.  M0 carries the LDS address; the kernels
// that use it have no compiler-generated M0 reads (checked in their gfx950 assembly).
QB_DEV void ts_dma16(const double* base, uint32_t off, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1" : : "v"(off), "s"(base), "s"(lds)
                 : "memory", "m0");
}
// The same for data read once (the streamed panel): non-temporal, so that it does not push the
// small, re-read operand out of L2.
QB_DEV void ts_dma16_nt(const double* base, uint32_t off, uint32_t lds) {
    asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1 nt" : : "v"(off), "s"(base), "s"(lds)
                 : "memory", "m0");
}

// VC: N = 16 FNM + 2 with the last two columns on the vector ALU -- lane l accumulates
// C(r0 + l mod 32, 16 FNM + l / 32) from the A and B tiles already in LDS -- instead of a
// fourth MFMA column block that would be seven-eighths padding (FM == 2; accf[FM * 16]).
template <int FM, int D, int FNM, bool VC>
QB_DEV void ts_panel_dma_body(const TsArgs& g, int64_t r0, int64_t kw, int64_t nst, int64_t ke,
                              uint32_t ring, const char* ring_ptr, double (&accf)[FM * 16 + 1]) {
    using L = PanelDma<FM>;
    static_assert(FM == 2 || FM == 4, "DMA panel tiles");
    static_assert(!VC || (FM == 2 && FNM < 4), "vector-ALU columns need 32-row tiles");
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int vr = lane & 31, vc = 16 * FNM + (lane >> 5);   // this lane's vector-ALU output
    double accv = 0.0;
    const int64_t nfull = nst > 0 && kw + 4 * nst > ke ? nst - 1 : nst;
    // per-lane DMA source offsets (bytes) from A(r0, kcol) and B(kcol, 0)
    uint32_t aoff[FM / 2], boff[2];
#pragma unroll
    for (int h = 0; h < FM / 2; ++h) aoff[h] = static_cast<uint32_t>((lk * g.lda + FM * li + 2 * h) * 8);
    {
        const int64_t pair = 2 * (lane & 31) < g.N - 2 ? 2 * (lane & 31) : g.N - 2;
#pragma unroll
        for (int q = 0; q < 2; ++q) boff[q] = static_cast<uint32_t>(((2 * q + (lane >> 5)) * g.bsk + pair) * 8);
    }
    auto issue = [&](int64_t t) {
        const uint32_t sb = ring + static_cast<uint32_t>(t % D) * L::STAGE;
        const int64_t kcol = kw + 4 * t;
        const double* ab = g.A + kcol * g.lda + r0;
        const double* bb = g.B + kcol * g.bsk;
#pragma unroll
        for (int h = 0; h < FM / 2; ++h) {
            if (g.nt_a) ts_dma16_nt(ab, aoff[h], sb + 1024 * h);
            else ts_dma16(ab, aoff[h], sb + 1024 * h);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) ts_dma16(bb, boff[q], sb + L::A_BYTES + 1024 * q);
    };
    v4d acc[FM][4];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) acc[f][fn] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < D - 1; ++p)
        if (p < nfull) issue(p);
    for (int64_t t = 0; t < nfull; ++t) {
        // this wave's DMAs of step t have landed once at most those of the later steps remain
        const int64_t later = nfull - 1 - t;
        if (later >= D - 2) __builtin_amdgcn_s_waitcnt(ts_vmcnt((D - 2) * L::ND));
        else if (D > 3 && later == 2) __builtin_amdgcn_s_waitcnt(ts_vmcnt(2 * L::ND));
        else if (later == 1) __builtin_amdgcn_s_waitcnt(ts_vmcnt(L::ND));
        else __builtin_amdgcn_s_waitcnt(ts_vmcnt(0));
        asm volatile("" ::: "memory");
        const char* st = ring_ptr + (t % D) * L::STAGE;
        double av[FM], bv[4];
#pragma unroll
        for (int h = 0; h < FM / 2; ++h) {
            const double2 x = *reinterpret_cast<const double2*>(st + 1024 * h + 16 * lane);
            av[2 * h] = x.x;
            av[2 * h + 1] = x.y;
        }
#pragma unroll
        for (int fn = 0; fn < FNM; ++fn)
            bv[fn] = *reinterpret_cast<const double*>(st + L::A_BYTES + 8 * (lk * 64 + 16 * fn + li));
#pragma unroll
        for (int fn = 0; fn < FNM; ++fn)
#pragma unroll
            for (int f = 0; f < FM; ++f) acc[f][fn] = ts_mfma(av[f], bv[fn], acc[f][fn]);
        if constexpr (VC) {
            // A(vr, k) sits at byte 256 k + 8 vr of the 32-row stage, B(k, vc) at row k of B's
            double xa[4], xb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                xa[k] = *reinterpret_cast<const double*>(st + 256 * k + 8 * vr);
                xb[k] = *reinterpret_cast<const double*>(st + L::A_BYTES + 8 * (k * 64 + vc));
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) accv = fma(xa[k], xb[k], accv);
        }
        asm volatile("" ::: "memory");
        // the slot of step t - 1 is free: its operands were consumed by the MFMAs above's
        // predecessors (their LDS reads completed before those MFMAs issued)
        if (t + D - 1 < nfull) issue(t + D - 1);
    }
    if (nfull < nst) {   // the step that crosses ke: register loads, columns >= ke masked
        const int64_t k = kw + 4 * nfull + lk;
        const bool v = k < ke;
        const int64_t kc = v ? k : ke - 1;
        const int64_t il = r0 + FM * li;
        double av[FM], bv[4];
#pragma unroll
        for (int e = 0; e < FM; ++e) av[e] = g.A[kc * g.lda + il + e];
#pragma unroll
        for (int fn = 0; fn < FNM; ++fn) {
            const int64_t j = 16 * fn + li < g.N ? 16 * fn + li : g.N - 1;
            bv[fn] = v ? g.B[kc * g.bsk + j] : 0.0;
        }
#pragma unroll
        for (int fn = 0; fn < FNM; ++fn)
#pragma unroll
            for (int f = 0; f < FM; ++f) acc[f][fn] = ts_mfma(av[f], bv[fn], acc[f][fn]);
        if constexpr (VC) {
            const int64_t k0 = kw + 4 * nfull;
            for (int k = 0; k < 4; ++k)
                if (k0 + k < ke) accv = fma(g.A[(k0 + k) * g.lda + r0 + vr], g.B[(k0 + k) * g.bsk + vc], accv);
        }
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) accf[(f * 4 + fn) * 4 + r] = acc[f][fn][r];
    accf[FM * 16] = accv;
}

template <int FM, int WK, int D, int FNM, bool VC>
__global__ void __launch_bounds__(64 * WK) ts_panel_dma_kernel(const TsArgs g) {
    if (g.gate != nullptr && *g.gate != 0) return;
    constexpr int NACC = FM * 16 + 1;
    constexpr int RING = WK * D * PanelDma<FM>::STAGE;
    constexpr int RED = (WK > 1 ? WK - 1 : 0) * NACC * 64 * 8;
    __shared__ __align__(16) char lds[RING > RED ? RING : RED];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int li = lane & 15, lk = lane >> 4;
    const int tile = blockIdx.x % g.tiles, split = blockIdx.x / g.tiles;
    const int64_t r0 = static_cast<int64_t>(tile) * 16 * FM;
    const int64_t kb = static_cast<int64_t>(split) * g.kchunk;
    const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
    const int64_t steps = (ke - kb + 3) / 4;
    const int64_t t0 = steps * wave / WK, t1 = steps * (wave + 1) / WK;
    double acc[NACC];
    const char* ring_ptr = lds + wave * D * PanelDma<FM>::STAGE;
    const uint32_t ring = __builtin_amdgcn_readfirstlane(
        static_cast<uint32_t>(reinterpret_cast<uintptr_t>((ts_lds_ptr)ring_ptr)));
    const bool full = r0 + 16 * FM <= g.M;
    if (full) {
        ts_panel_dma_body<FM, D, FNM, VC>(g, r0, kb + 4 * t0, t1 - t0, ke, ring, ring_ptr, acc);
    } else {   // the one edge tile: every column on MFMA
        double a16[FM * 16];
        ts_panel_body<FM, WK, 2, true>(g, r0, kb + 4 * t0, t1 - t0, ke, a16);
#pragma unroll
        for (int x = 0; x < FM * 16; ++x) acc[x] = a16[x];
        acc[FM * 16] = 0.0;
    }
    if (WK > 1) __syncthreads();   // every wave is done with its ring before it is reused
    ts_wave_reduce<NACC, WK>(reinterpret_cast<double*>(lds), acc, wave, lane);
    if (wave != 0) return;
    const int64_t jmfma = VC && full ? 16 * FNM : g.N;   // columns written from the MFMA tiles
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = r0 + FM * ((r << 2) + lk) + f;
                const int64_t j = 16 * fn + li;
                if (i < g.M && j < jmfma) ts_store(g, split, i, j, acc[(f * 4 + fn) * 4 + r]);
            }
    if (VC && full) ts_store(g, split, r0 + (lane & 31), 16 * FNM + (lane >> 5), acc[FM * 16]);
}

// ------------------------------------------------------------------ reduction form
//
// C(M x N) = alpha A B + beta C0 with A(i, k) = A[i lda + k] and a long reduction; B(k, j) is
// contiguous in k (BK1: B[k + j bsj]) or in j (B[k bsk + j]).  A workgroup owns 16 FM output
// rows; its reduction range (one split) is cut into groups of 16 indices shared out to its WV
// waves in contiguous runs.  Each lane loads, per group, 4 consecutive reduction indices of its
// FM rows of A and of its 4 columns of B; D groups are kept in flight.
// VC: N = 16 FNM + 2 with the last two columns on the vector ALU: lane (i, q) multiplies its
// rows' A values by the B values of those two columns, which lanes (0, q) and (1, q) already
// hold in their fourth column block (exchanged by a lane permute), and the four partial sums
// of a row are added across q at the end (accf[FM * 16 + 2 f + c]).
template <int FM, int D, bool BK1, int FNM, bool VC>
QB_DEV void ts_red_body(const TsArgs& g, int64_t i0, int64_t kw, int64_t ngr, int64_t ke,
                        double (&accf)[FM * 16 + (VC ? 2 * FM : 0)]) {
    const int lane = threadIdx.x & 63, li = lane & 15, lq = lane >> 4;
    // groups [0, nfull) lie inside the reduction range; a last group that crosses ke is done
    // apart with masked loads
    const int64_t nfull = ngr > 0 && kw + 16 * ngr > ke ? ngr - 1 : ngr;
    double a[D][FM][4], b[D][4][4];
    constexpr int kRedLoads = 2 * FM + (BK1 ? 8 : 16);   // vector loads per group
    int64_t arow[FM], bcol[4];   // element offsets of this lane's rows of A / columns of B
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        const int64_t i = i0 + 16 * f + li;
        arow[f] = (i < g.M ? i : g.M - 1) * g.lda;
    }
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
        const int64_t j = 16 * fn + li;
        bcol[fn] = (j < g.N ? j : g.N - 1) * g.bsj;
    }
    // per-lane byte offsets from the group's bases A(i0, kg) and B(kg, 0) (kg wave-uniform)
    uint32_t aoff[FM], boff[4];
#pragma unroll
    for (int f = 0; f < FM; ++f) aoff[f] = static_cast<uint32_t>((arow[f] - i0 * g.lda + 4 * lq) * 8);
#pragma unroll
    for (int fn = 0; fn < 4; ++fn)
        boff[fn] = static_cast<uint32_t>((BK1 ? bcol[fn] + 4 * lq : 4 * lq * g.bsk + bcol[fn]) * 8);
    const uint32_t bstep = static_cast<uint32_t>(g.bsk * 8);
    // this lane's four reduction indices kg + 4 lq .. + 3 of a full group
    auto load_full = [&](double (&av)[FM][4], double (&bv)[4][4], int64_t kg) {
        const __amdgpu_buffer_rsrc_t ra = ts_rsrc(g.A + i0 * g.lda + kg);
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            const double2 x0 = ts_ld2(ra, aoff[f]);
            const double2 x1 = ts_ld2(ra, aoff[f] + 16);
            av[f][0] = x0.x; av[f][1] = x0.y; av[f][2] = x1.x; av[f][3] = x1.y;
        }
        if constexpr (BK1) {
            const __amdgpu_buffer_rsrc_t rb = ts_rsrc(g.B + kg);
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) {
                const double2 y0 = ts_ld2(rb, boff[fn]);
                const double2 y1 = ts_ld2(rb, boff[fn] + 16);
                bv[fn][0] = y0.x; bv[fn][1] = y0.y; bv[fn][2] = y1.x; bv[fn][3] = y1.y;
            }
        } else {
            const __amdgpu_buffer_rsrc_t rb = ts_rsrc(g.B + kg * g.bsk);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int fn = 0; fn < 4; ++fn) bv[fn][s] = ts_ld1(rb, boff[fn] + s * bstep);
        }
    };
    v4d acc[FM][4];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) acc[f][fn] = v4d{0.0, 0.0, 0.0, 0.0};
    double pv[FM][2];
#pragma unroll
    for (int f = 0; f < FM; ++f) pv[f][0] = pv[f][1] = 0.0;
    auto group = [&](const double (&av)[FM][4], const double (&bv)[4][4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int fn = 0; fn < FNM; ++fn)
#pragma unroll
                for (int f = 0; f < FM; ++f) acc[f][fn] = ts_mfma(av[f][s], bv[fn][s], acc[f][fn]);
        if constexpr (VC) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double x0 = __shfl(bv[FNM][s], (lane & 48) | 0, 64);
                const double x1 = __shfl(bv[FNM][s], (lane & 48) | 1, 64);
#pragma unroll
                for (int f = 0; f < FM; ++f) {
                    pv[f][0] = fma(av[f][s], x0, pv[f][0]);
                    pv[f][1] = fma(av[f][s], x1, pv[f][1]);
                }
            }
        }
    };
    if (nfull > 0) {
        auto k0 = [&](int64_t u) { return kw + 16 * (u < nfull ? u : nfull - 1); };
        // prologue (see ts_panel_body: a select, not a bare load, enters the loop registers)
#pragma unroll
        for (int s = 0; s < D; ++s) {
            load_full(a[s], b[s], k0(s));
            const bool v = s < nfull;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int fn = 0; fn < 4; ++fn) b[s][fn][q] = v ? b[s][fn][q] : 0.0;
#pragma unroll
                for (int f = 0; f < FM; ++f) a[s][f][q] = v ? a[s][f][q] : 0.0;
            }
        }
        int64_t u = 0;
        for (; u + D <= nfull; u += D) {
#pragma unroll
            for (int s = 0; s < D; ++s) {
                group(a[s], b[s]);
                load_full(a[s], b[s], k0(u + s + D));
                __builtin_amdgcn_sched_group_barrier(0x008, 16 * FM, 0);
                __builtin_amdgcn_sched_group_barrier(0x020, kRedLoads, 0);
            }
        }
        const int64_t rem = nfull - u;
#pragma unroll
        for (int s = 0; s < D - 1; ++s)
            if (s < rem) group(a[s], b[s]);
    }
    if (nfull < ngr) {   // the group that crosses ke: clamped scalar loads, indices >= ke masked
        const int64_t kq = kw + 16 * nfull + 4 * lq;
        double av[FM][4], bv[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool v = kq + s < ke;
            const int64_t k = v ? kq + s : ke - 1;
#pragma unroll
            for (int f = 0; f < FM; ++f) av[f][s] = g.A[arow[f] + k];
#pragma unroll
            for (int fn = 0; fn < 4; ++fn) {
                const double x = BK1 ? g.B[bcol[fn] + k] : g.B[k * g.bsk + bcol[fn]];
                bv[fn][s] = v ? x : 0.0;
            }
        }
        group(av, bv);
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) accf[(f * 4 + fn) * 4 + r] = acc[f][fn][r];
    if constexpr (VC) {
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double v = pv[f][c];
                v += __shfl_xor(v, 16, 64);
                v += __shfl_xor(v, 32, 64);
                accf[FM * 16 + 2 * f + c] = v;
            }
    }
}

template <int FM, int WV, int D, bool BK1, int FNM, bool VC>
__global__ void __launch_bounds__(64 * WV) ts_red_kernel(const TsArgs g) {
    if (g.gate != nullptr && *g.gate != 0) return;
    constexpr int NACC = FM * 16 + (VC ? 2 * FM : 0);
    __shared__ double red[(WV > 1 ? WV - 1 : 1) * NACC * 64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int li = lane & 15, lq = lane >> 4;
    // consecutive logical workgroups (the row tiles of one split, which read the same rows of
    // B) share an XCD and its L2
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = logical % g.tiles, split = logical / g.tiles;
    const int64_t i0 = static_cast<int64_t>(tile) * 16 * FM;
    const int64_t kb = static_cast<int64_t>(split) * g.kchunk;
    const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
    const int64_t groups = (ke - kb + 15) / 16;
    const int64_t u0 = groups * wave / WV, u1 = groups * (wave + 1) / WV;
    double acc[NACC];
    ts_red_body<FM, D, BK1, FNM, VC>(g, i0, kb + 16 * u0, u1 - u0, ke, acc);
    ts_wave_reduce<NACC, WV>(red, acc, wave, lane);
    if (wave != 0) return;
    const int64_t jmfma = VC ? 16 * FNM : g.N;   // columns written from the MFMA tiles
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + 16 * f + (r << 2) + lq;
                const int64_t j = 16 * fn + li;
                if (i < g.M && j < jmfma) ts_store(g, split, i, j, acc[(f * 4 + fn) * 4 + r]);
            }
    if constexpr (VC) {
        if (lq == 0) {
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int64_t i = i0 + 16 * f + li, j = 16 * FNM + c;
                    if (i < g.M && j < g.N) ts_store(g, split, i, j, acc[FM * 16 + 2 * f + c]);
                }
        }
    }
}

// ------------------------------------------------------------------ host

static TsArgs ts_args(const GemmDesc& d) {
    TsArgs g{};
    g.M = d.M; g.N = d.N; g.K = d.K;
    g.alpha = d.alpha; g.beta = d.beta;
    g.C0 = d.C0.p; g.c0_si = d.C0.si; g.c0_sj = d.C0.sj;
    g.C = d.C.p; g.c_si = d.C.si; g.c_sj = d.C.sj;
    g.P = d.ws;
    g.gate = d.gate;
    return g;
}

static bool aligned16(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

template <int FM, int WK, int D>
static hipError_t launch_panel(TsArgs g, int nsplit, hipStream_t s) {
    g.tiles = static_cast<int>(cdiv(g.M, 16 * FM));
    g.kchunk = cdiv(cdiv(g.K, nsplit), 4) * 4;
    g.nsplit = static_cast<int>(cdiv(g.K, g.kchunk));
    hipLaunchKernelGGL((ts_panel_kernel<FM, WK, D>), dim3(static_cast<unsigned>(g.tiles * g.nsplit)),
                       dim3(64 * WK), 0, s, g);
    return hipGetLastError();
}

template <int FM, int WK, int D>
static hipError_t launch_panel_dma(TsArgs g, int nsplit, hipStream_t s) {
    g.tiles = static_cast<int>(cdiv(g.M, 16 * FM));
    g.kchunk = cdiv(cdiv(g.K, nsplit), 4) * 4;
    g.nsplit = static_cast<int>(cdiv(g.K, g.kchunk));
    const dim3 grid(static_cast<unsigned>(g.tiles * g.nsplit));
    if constexpr (FM == 2) {
        if (g.N == 50) {   // 48 columns on MFMA, two on the vector ALU
            hipLaunchKernelGGL((ts_panel_dma_kernel<FM, WK, D, 3, true>), grid, dim3(64 * WK), 0, s, g);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((ts_panel_dma_kernel<FM, WK, D, 4, false>), grid, dim3(64 * WK), 0, s, g);
    return hipGetLastError();
}

template <int FM, int WV, int D, bool BK1>
static hipError_t launch_red(TsArgs g, int nsplit, hipStream_t s) {
    g.tiles = static_cast<int>(cdiv(g.M, 16 * FM));
    g.kchunk = cdiv(cdiv(g.K, nsplit), 16) * 16;
    g.nsplit = static_cast<int>(cdiv(g.K, g.kchunk));
    const dim3 grid(static_cast<unsigned>(g.tiles * g.nsplit));
    if constexpr (FM == 4) {
        if (g.N == 50) {   // 48 columns on MFMA, two on the vector ALU
            hipLaunchKernelGGL((ts_red_kernel<FM, WV, D, BK1, 3, true>), grid, dim3(64 * WV), 0, s, g);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((ts_red_kernel<FM, WV, D, BK1, 4, false>), grid, dim3(64 * WV), 0, s, g);
    return hipGetLastError();
}

// Sum the split partials in split order into C (alpha, beta epilogue).
static hipError_t ts_finish(const GemmDesc& d, int nsplit, hipStream_t s) {
    if (nsplit <= 1) return hipSuccess;
    return launch_splitk_reduce(d, nsplit, s);
}

// The per-lane load offsets are 32-bit byte counts: they span at most 4 columns of the panel
// form's A and B, and 64 rows of the reduction form's A and columns of its B.
static bool offsets_fit(int64_t span_elems) { return span_elems >= 0 && span_elems * 8 + 64 < (int64_t(1) << 31); }

bool ts_panel_fits(const GemmDesc& d) {
    if (!(d.N >= 1 && d.N <= 64 && d.A.si == 1 && d.colsq == nullptr && d.M >= 1 && d.K >= 1)) return false;
    return offsets_fit(4 * d.A.sj + 64) && offsets_fit(4 * std::abs(d.B.si) + 64 * std::abs(d.B.sj));
}

bool ts_red_fits(const GemmDesc& d) {
    if (!(d.N >= 1 && d.N <= 64 && d.A.sj == 1 && d.colsq == nullptr && d.M >= 1 && d.K >= 1)) return false;
    if (!aligned16(d.A.p) || d.A.si % 2 != 0 || !offsets_fit(64 * d.A.si + 16)) return false;
    if (d.B.si == 1) return aligned16(d.B.p) && d.B.sj % 2 == 0 && offsets_fit(64 * d.B.sj + 16);
    return d.B.sj == 1 && offsets_fit(16 * d.B.si + 64);
}

hipError_t ts_panel(const GemmDesc& d, int fm, int wk, int nsplit, hipStream_t s) {
    if (!ts_panel_fits(d)) return hipErrorNotSupported;
    if (nsplit > 1 && (d.ws == nullptr || nsplit * d.M * d.N > d.ws_elems)) return hipErrorInvalidValue;
    TsArgs g = ts_args(d);
    g.A = d.A.p; g.lda = d.A.sj;
    g.B = d.B.p; g.bsk = d.B.si; g.bsj = d.B.sj;
    const bool vec = aligned16(d.A.p) && d.A.sj % 2 == 0;
    if (fm > 1 && !vec) fm = 1;
    hipError_t e;
    if (fm == 4 && wk == 4) e = launch_panel<4, 4, 4>(g, nsplit, s);
    else if (fm == 4 && wk == 2) e = launch_panel<4, 2, 4>(g, nsplit, s);
    else if (fm == 4 && wk == 1) e = launch_panel<4, 1, 4>(g, nsplit, s);
    else if (fm == 2 && wk == 4) e = launch_panel<2, 4, 6>(g, nsplit, s);
    else if (fm == 2 && wk == 2) e = launch_panel<2, 2, 6>(g, nsplit, s);
    else if (fm == 2 && wk == 1) e = launch_panel<2, 1, 6>(g, nsplit, s);
    else if (fm == 1 && wk == 4) e = launch_panel<1, 4, 8>(g, nsplit, s);
    else if (fm == 1 && wk == 2) e = launch_panel<1, 2, 8>(g, nsplit, s);
    else e = launch_panel<1, 1, 8>(g, nsplit, s);
    if (e != hipSuccess) return e;
    return ts_finish(d, static_cast<int>(cdiv(d.K, cdiv(cdiv(d.K, nsplit), 4) * 4)), s);
}

bool ts_panel_dma_fits(const GemmDesc& d) {
    return ts_panel_fits(d) && d.N >= 2 && d.B.sj == 1 && aligned16(d.A.p) && d.A.sj % 2 == 0 &&
           aligned16(d.B.p) && d.B.si % 2 == 0 && d.B.si >= 0;
}

hipError_t ts_panel_dma(const GemmDesc& d, int fm, int wk, int depth, int nsplit, hipStream_t s, int nt) {
    if (!ts_panel_dma_fits(d)) return hipErrorNotSupported;
    if (nsplit > 1 && (d.ws == nullptr || nsplit * d.M * d.N > d.ws_elems)) return hipErrorInvalidValue;
    TsArgs g = ts_args(d);
    g.nt_a = nt;
    g.A = d.A.p; g.lda = d.A.sj;
    g.B = d.B.p; g.bsk = d.B.si; g.bsj = 1;
    hipError_t e;
    if (fm == 4 && wk == 1 && depth == 4) e = launch_panel_dma<4, 1, 4>(g, nsplit, s);
    else if (fm == 4 && wk == 1 && depth == 6) e = launch_panel_dma<4, 1, 6>(g, nsplit, s);
    else if (fm == 4 && wk == 1 && depth == 8) e = launch_panel_dma<4, 1, 8>(g, nsplit, s);
    else if (fm == 4 && wk == 2 && depth == 4) e = launch_panel_dma<4, 2, 4>(g, nsplit, s);
    else if (fm == 4 && wk == 4 && depth == 4) e = launch_panel_dma<4, 4, 4>(g, nsplit, s);
    else if (fm == 2 && wk == 1 && depth == 4) e = launch_panel_dma<2, 1, 4>(g, nsplit, s);
    else if (fm == 2 && wk == 1 && depth == 8) e = launch_panel_dma<2, 1, 8>(g, nsplit, s);
    else if (fm == 2 && wk == 2 && depth == 4) e = launch_panel_dma<2, 2, 4>(g, nsplit, s);
    else if (fm == 2 && wk == 4 && depth == 4) e = launch_panel_dma<2, 4, 4>(g, nsplit, s);
    else return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    return ts_finish(d, static_cast<int>(cdiv(d.K, cdiv(cdiv(d.K, nsplit), 4) * 4)), s);
}

hipError_t ts_red(const GemmDesc& d, int fm, int wv, int nsplit, hipStream_t s) {
    if (!ts_red_fits(d)) return hipErrorNotSupported;
    if (nsplit > 1 && (d.ws == nullptr || nsplit * d.M * d.N > d.ws_elems)) return hipErrorInvalidValue;
    TsArgs g = ts_args(d);
    g.A = d.A.p; g.lda = d.A.si;
    g.B = d.B.p; g.bsk = d.B.si; g.bsj = d.B.sj;
    const bool bk1 = d.B.si == 1;
    hipError_t e;
    if (bk1) {
        if (fm == 4 && wv == 4) e = launch_red<4, 4, 2, true>(g, nsplit, s);
        else if (fm == 4 && wv == 2) e = launch_red<4, 2, 2, true>(g, nsplit, s);
        else if (fm == 2 && wv == 4) e = launch_red<2, 4, 3, true>(g, nsplit, s);
        else e = launch_red<1, 4, 4, true>(g, nsplit, s);
    } else {
        if (fm == 4 && wv == 4) e = launch_red<4, 4, 2, false>(g, nsplit, s);
        else if (fm == 4 && wv == 2) e = launch_red<4, 2, 2, false>(g, nsplit, s);
        else if (fm == 2 && wv == 4) e = launch_red<2, 4, 3, false>(g, nsplit, s);
        else e = launch_red<1, 4, 4, false>(g, nsplit, s);
    }
    if (e != hipSuccess) return e;
    return ts_finish(d, static_cast<int>(cdiv(d.K, cdiv(cdiv(d.K, nsplit), 16) * 16)), s);
}

}  // namespace qb
