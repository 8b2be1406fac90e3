// Kernels of the approximate SVD from a QB factorisation (eq. (3)): B = U~ diag(s) V~^T
// by a thin QR of B^T (B^T = P T, done by the block orthonormalisation of the library) and
// a one-sided Jacobi SVD of the k x k factor X = T^T.  One-sided Jacobi (Hestenes) rotates
// pairs of columns of X until all are mutually orthogonal: the column norms are then the
// singular values, the normalised columns the left singular vectors, and the accumulated
// rotations W the right singular vectors of X.  The method works on blocks of columns
// (below): a round of the circle ordering over the blocks is three launches, whatever the
// block width, instead of one launch per round over single columns.  Every sum is taken in
// a fixed order (bit-reproducible results).
#include "kernels.h"

namespace qb {

constexpr int kSvdThreads = 256;

// Fixed-order sum over the workgroup of three values at once.
QB_DEV void block_sum3(double& a, double& b, double& c, double (*sh)[kSvdThreads / 64]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
        c += __shfl_down(c, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][w] = a;
        sh[1][w] = b;
        sh[2][w] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
#pragma unroll
    for (int i = 0; i < kSvdThreads / 64; ++i) {
        a += sh[0][i];
        b += sh[1][i];
        c += sh[2][i];
    }
    __syncthreads();
}

// Players of round r of the circle ordering for np (even) players: player 0 stays, the
// others rotate; pair p of the round.
QB_DEV void circle_pair(int np, int r, int p, int& a, int& b) {
    const int m = np - 1;
    a = p == 0 ? 0 : 1 + (r + p - 1) % m;
    b = 1 + (r + m - 1 - p) % m;
}

// Block form.  The columns of X are cut into blocks of kJb (the last one ragged; an odd
// count gets an empty dummy block), and the circle ordering runs over the blocks: a round
// pairs them into disjoint pairs of 2 kJb columns.  For each pair the round forms the Gram
// matrix of its columns (pair_gram_kernel, split over the rows, partial sums added in split
// order, on the matrix cores), finds the rotations that diagonalise it by cyclic two-sided
// Jacobi (pair_eig_kernel, pair_eig_cross_kernel: the rotation of columns p, q is the one
// the column pair itself would get, read off the Gram entries), and applies their product
// V to the pair's columns of X and of W (pair_apply_kernel, on the matrix cores).  The Gram
// matrix is formed afresh from X in every round, so its rounding does not accumulate; the
// pair test of the next sweep measures the cosine of each column pair from fresh dot
// products, as the scalar method does.
constexpr int kJb = 32;            // columns per block
constexpr int kJp = 2 * kJb;       // columns per pair of blocks
constexpr int kApplyTiles = 2;     // 16-row tiles per wave in the apply kernel
constexpr int kJrows = 16 * kApplyTiles * 4;   // rows per apply workgroup (four waves)
constexpr int kGramH = 2;          // 16-row steps per wave in the Gram kernel
constexpr int kGramRows = 16 * kGramH * 4;   // rows per Gram workgroup (four waves)

// The pair of blocks that workgroup p of a round works on: round r >= 0 of the circle
// ordering over np players, or, for round -1 (the within-block step of a sweep), the
// neighbours 2 p and 2 p + 1.
QB_DEV void round_pair(int np, int round, int p, int& a, int& b) {
    if (round < 0) {
        a = 2 * p;
        b = 2 * p + 1;
        return;
    }
    circle_pair(np, round, p, a, b);
}

// Column of X that slot j (0 .. kJp-1) of the pair of blocks (a, b) holds, or -1.
QB_DEV int pair_col(int a, int b, int nb, int j, int k) {
    const int blk = j < kJb ? a : b;
    if (blk >= nb) return -1;
    const int c = blk * kJb + (j & (kJb - 1));
    return c < k ? c : -1;
}

// v_mfma_f64_16x16x4f64 takes A(i, r) from lane 16 r + i and B(r, j) from lane 16 r + j, and
// leaves C(4 q + l / 16, l mod 16) in slot q of lane l.
using svd_v4d = double __attribute__((ext_vector_type(4)));
QB_DEV svd_v4d svd_mfma(double a, double b, svd_v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Partial Gram matrix of rows [R y, R (y + 1)), R = kGramRows, of the pair's columns on the
// matrix cores: wave w takes 16 kGramH of the rows (16 of them, 64 rows a workgroup, was
// slower: 11.0 against 9.7 us a launch at k = 1250), lane (r, i) = (l / 16, l mod 16) supplying row
// 16 h + 4 t + r at reduction step (h, t) of slot 16 g + i (a column of the same rows for
// both operands, so C = sum over the rows of x_p x_q).  Only the 10 tiles of 16 x 16 on and
// above the diagonal are formed; the waves' sums are added in wave order through LDS, and
// each entry on or above the diagonal is written to both of its places (the result is
// exactly symmetric).  part[(pair * nsplit + y) * kJp^2 + i * kJp + j].
__global__ void __launch_bounds__(kSvdThreads)
pair_gram_kernel(const double* __restrict__ X, int k, int64_t ld, int nb, int np, int round,
                 int nsplit, double* __restrict__ part) {
    constexpr int kTiles = 10;
    __shared__ svd_v4d red[kSvdThreads / 64 - 1][kTiles][64];
    int a, b;
    round_pair(np, round, static_cast<int>(blockIdx.x), a, b);
    const int lane = static_cast<int>(threadIdx.x) & 63, w = static_cast<int>(threadIdx.x) >> 6;
    const int rr = lane >> 4, ii = lane & 15;
    static_assert(kGramRows == 16 * kGramH * (kSvdThreads / 64), "16 kGramH rows per wave");
    const int r0 = (static_cast<int>(blockIdx.y) * (kSvdThreads / 64) + w) * 16 * kGramH;
    double v[4][kGramH][4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int c = pair_col(a, b, nb, 16 * g + ii, k);
#pragma unroll
        for (int h = 0; h < kGramH; ++h)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = r0 + 16 * h + 4 * t + rr;
                v[g][h][t] = (c >= 0 && row < k) ? X[static_cast<int64_t>(c) * ld + row] : 0.0;
            }
    }
    svd_v4d acc[kTiles];
#pragma unroll
    for (int T = 0; T < kTiles; ++T) acc[T] = svd_v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < kGramH; ++h)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int T = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = m; n < 4; ++n, ++T) acc[T] = svd_mfma(v[m][h][t], v[n][h][t], acc[T]);
        }
    if (w > 0) {
#pragma unroll
        for (int T = 0; T < kTiles; ++T) red[w - 1][T][lane] = acc[T];
    }
    __syncthreads();
    if (w != 0) return;
    double* out = part + (static_cast<int64_t>(blockIdx.x) * nsplit + blockIdx.y) * (kJp * kJp);
    int T = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = m; n < 4; ++n, ++T) {
            svd_v4d sum = acc[T];
#pragma unroll
            for (int u = 0; u < kSvdThreads / 64 - 1; ++u) sum += red[u][T][lane];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * m + 4 * q + rr, j = 16 * n + ii;
                if (m == n && i > j) continue;
                out[i * kJp + j] = sum[q];
                out[j * kJp + i] = sum[q];
            }
        }
}

// G[pair] = sum of the pair's partial Gram matrices in split order; a thread per entry, its
// loads issued eight splits at a time.  Grid: (pairs, kJp^2 / 256).
__global__ void __launch_bounds__(kSvdThreads)
pair_reduce_kernel(const double* __restrict__ part, int nsplit, double* __restrict__ G) {
    const int e = static_cast<int>(blockIdx.y) * kSvdThreads + static_cast<int>(threadIdx.x);
    const double* src = part + static_cast<int64_t>(blockIdx.x) * nsplit * (kJp * kJp) + e;
    double acc = 0.0;
    for (int y0 = 0; y0 < nsplit; y0 += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            v[q] = y0 + q < nsplit ? src[static_cast<int64_t>(y0 + q) * (kJp * kJp)] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (y0 + q < nsplit) acc += v[q];
    }
    G[static_cast<int64_t>(blockIdx.x) * (kJp * kJp) + e] = acc;
}

// The rotation of columns p, q from their Gram entries al = g_pp, be = g_qq, ga = g_pq:
// returns false (c = 1, s = t = 0) when |g_pq| <= tol_r sqrt(g_pp g_qq), and sets big when
// |g_pq| > tol_c sqrt(g_pp g_qq).  t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// zeta = (g_qq - g_pp) / (2 g_pq), is evaluated as sign(d) 2 g_pq / (|d| + sqrt(d^2 + 4 g_pq^2)),
// d = g_qq - g_pp.  The angle needs no last-bit accuracy (it only sets how far the pair
// turns; one Newton step on each hardware estimate gives about 46 bits), c^2 + s^2 = 1 does:
// c comes from a fully refined 1 / sqrt.
QB_DEV bool pair_rotation(double al, double be, double ga, double tol_r, double tol_c, double& c,
                          double& s, double& t, bool& big) {
    const double g2 = ga * ga, ab = al * be;
    c = 1.0;
    s = 0.0;
    t = 0.0;
    big = false;
    if (!(ga != 0.0 && g2 > tol_r * tol_r * ab)) return false;
    const double d = be - al, g2x = 2.0 * ga;
    const double hx = fma(d, d, g2x * g2x);
    const double y = __builtin_amdgcn_rsq(hx);
    double h = hx * y;                                  // sqrt(hx), ~23 bits
    h = fma(fma(-h, h, hx), 0.5 * y, h);                // one Newton step
    const double den = fabs(d) + h;
    double ri = __builtin_amdgcn_rcp(den);
    ri = fma(ri, fma(-den, ri, 1.0), ri);               // one Newton step
    t = g2x * ri;
    if (d < 0.0) t = -t;
    double unused;
    sqrt_and_rsqrt(fma(t, t, 1.0), unused, c);
    s = c * t;
    big = g2 > tol_c * tol_c * ab;
    return true;
}

// One workgroup per pair of blocks: G = the pair's Gram matrix, then up to `inner` sweeps
// of cyclic two-sided Jacobi on G (circle ordering over the kJp columns, kJp - 1 rounds of
// kJp / 2 disjoint pairs), accumulating V = product of the rotations.  This is the
// within-block step of a sweep (neighbouring blocks 2p, 2p + 1); the circle rounds over the
// blocks that follow turn only the column pairs across their two blocks
// (pair_eig_cross_kernel), so every column pair turns at least once per sweep.
// Columns p, q rotate when |g_pq| > tol_r sqrt(g_pp g_qq), with the angle of one-sided
// Jacobi: zeta = (g_qq - g_pp) / (2 g_pq), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1 / sqrt(1 + t^2), s = c t, x_p <- c x_p - s x_q, x_q <- s x_p + c x_q; on G that is
// G <- J^T G J, with g_pp - t g_pq, g_qq + t g_pq and a zero g_pq set directly.  skip[pair] is
// 1 when nothing rotated (the apply kernel then leaves the pair), and flag is set when some
// |g_pq| exceeded tol_c sqrt(g_pp g_qq) (the sweep is not the last).
__global__ void __launch_bounds__(kSvdThreads)
pair_eig_kernel(const double* __restrict__ gram, int inner, double tol_r, double tol_c,
                double* __restrict__ Vout, int* __restrict__ skip, int* __restrict__ flag) {
    __shared__ double G[kJp][kJp + 1];
    __shared__ double V[kJp][kJp + 1];
    __shared__ double rc[kJp / 2], rs[kJp / 2], rt[kJp / 2];
    __shared__ int rp[kJp / 2], rq[kJp / 2];
    __shared__ int rot, big;
    const int tid = static_cast<int>(threadIdx.x);
    const double* src = gram + static_cast<int64_t>(blockIdx.x) * (kJp * kJp);
    double gv[kJp * kJp / kSvdThreads];
#pragma unroll
    for (int q = 0; q < kJp * kJp / kSvdThreads; ++q) gv[q] = src[tid + q * kSvdThreads];
#pragma unroll
    for (int q = 0; q < kJp * kJp / kSvdThreads; ++q) {
        const int e = tid + q * kSvdThreads;
        G[e / kJp][e % kJp] = gv[q];
        V[e / kJp][e % kJp] = (e / kJp == e % kJp) ? 1.0 : 0.0;
    }
    __syncthreads();
    // the upper-triangle 2 x 2 blocks (P, Q), P <= Q, this thread owns in every round
    constexpr int kH = kJp / 2;
    constexpr int kUp = kH * (kH + 1) / 2;
    constexpr int kPer = (kUp + kSvdThreads - 1) / kSvdThreads;
    int P[kPer], Q[kPer];
    bool own[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int e = tid + i * kSvdThreads;
        own[i] = e < kUp;
        int pr = 0, rem = own[i] ? e : 0;
        while (rem >= kH - pr) {
            rem -= kH - pr;
            ++pr;
        }
        P[i] = pr;
        Q[i] = pr + rem;
    }
    if (tid == 0) big = 0;
    bool any = false;
    // a pair whose Gram matrix is already diagonal to tol_r rotates nothing in a sweep:
    // leave it at once (every thread tests its own 16 entries)
    bool open = false;
#pragma unroll
    for (int q = 0; q < kJp * kJp / kSvdThreads; ++q) {
        const int e = tid + q * kSvdThreads;
        const int i = e / kJp, j = e % kJp;
        const double gij = gv[q];
        open = open || (i != j && gij != 0.0 && gij * gij > tol_r * tol_r * G[i][i] * G[j][j]);
    }
    if (!__syncthreads_or(open)) {
        if (tid == 0) skip[blockIdx.x] = 1;
        return;
    }
    for (int sw = 0; sw < inner; ++sw) {
        if (tid == 0) rot = 0;
        __syncthreads();
        for (int r = 0; r < kJp - 1; ++r) {
            if (tid < kJp / 2) {
                int pp, qq;
                circle_pair(kJp, r, tid, pp, qq);
                if (pp > qq) {
                    const int t = pp;
                    pp = qq;
                    qq = t;
                }
                double c, s, t;
                bool bg;
                if (pair_rotation(G[pp][pp], G[qq][qq], G[pp][qq], tol_r, tol_c, c, s, t, bg)) {
                    rot = 1;
                    if (bg) big = 1;
                }
                rc[tid] = c;
                rt[tid] = t;
                rs[tid] = s;
                rp[tid] = pp;
                rq[tid] = qq;
            }
            __syncthreads();
            // G <- J^T G J by 2 x 2 blocks (rows of pair P, columns of pair Q) with P <= Q
            // (528 of them, about two per thread, one owner each); only the upper triangle
            // of G is kept up to date, every entry is read and written at (min, max).  All
            // reads come first.
            {
                double c1[kPer], s1[kPer], c2[kPer], s2[kPer], g[kPer][4];
                int p1[kPer], q1[kPer], p2[kPer], q2[kPer];
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    c1[i] = rc[P[i]];
                    s1[i] = rs[P[i]];
                    p1[i] = rp[P[i]];
                    q1[i] = rq[P[i]];
                    c2[i] = rc[Q[i]];
                    s2[i] = rs[Q[i]];
                    p2[i] = rp[Q[i]];
                    q2[i] = rq[Q[i]];
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    g[i][0] = G[min(p1[i], p2[i])][max(p1[i], p2[i])];
                    g[i][1] = G[min(p1[i], q2[i])][max(p1[i], q2[i])];
                    g[i][2] = G[min(q1[i], p2[i])][max(q1[i], p2[i])];
                    g[i][3] = G[min(q1[i], q2[i])][max(q1[i], q2[i])];
                }
#pragma unroll
                for (int i = 0; i < kPer; ++i) {
                    if (!own[i]) continue;
                    if (s1[i] == 0.0 && s2[i] == 0.0) continue;
                    if (P[i] == Q[i]) {   // diagonal block: the rotation's closed form
                        const double t = rt[P[i]];
                        G[p1[i]][p1[i]] = g[i][0] - t * g[i][1];
                        G[q1[i]][q1[i]] = g[i][3] + t * g[i][1];
                        G[p1[i]][q1[i]] = 0.0;
                        continue;
                    }
                    const double h11 = c1[i] * g[i][0] - s1[i] * g[i][2];
                    const double h12 = c1[i] * g[i][1] - s1[i] * g[i][3];
                    const double h21 = s1[i] * g[i][0] + c1[i] * g[i][2];
                    const double h22 = s1[i] * g[i][1] + c1[i] * g[i][3];
                    const double n11 = c2[i] * h11 - s2[i] * h12, n12 = s2[i] * h11 + c2[i] * h12;
                    const double n21 = c2[i] * h21 - s2[i] * h22, n22 = s2[i] * h21 + c2[i] * h22;
                    G[min(p1[i], p2[i])][max(p1[i], p2[i])] = n11;
                    G[min(p1[i], q2[i])][max(p1[i], q2[i])] = n12;
                    G[min(q1[i], p2[i])][max(q1[i], p2[i])] = n21;
                    G[min(q1[i], q2[i])][max(q1[i], q2[i])] = n22;
                }
            }
            // V <- V J: thread t applies rotation t mod 32 to rows t / 32 + 8 j
            {
                const int Pv = tid & (kH - 1), i0 = tid / kH;
                const double c = rc[Pv], s = rs[Pv];
                if (s != 0.0) {
                    const int pp = rp[Pv], qq = rq[Pv];
                    double vp[8], vq[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        vp[j] = V[i0 + 8 * j][pp];
                        vq[j] = V[i0 + 8 * j][qq];
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        V[i0 + 8 * j][pp] = c * vp[j] - s * vq[j];
                        V[i0 + 8 * j][qq] = s * vp[j] + c * vq[j];
                    }
                }
            }
            __syncthreads();
        }
        const bool rotated = rot != 0;   // uniform: read after the round's barrier
        __syncthreads();
        if (!rotated) break;
        any = true;
    }
    if (tid == 0) {
        skip[blockIdx.x] = any ? 0 : 1;
        if (big) flag[0] = 1;
    }
    if (!any) return;
    double* v = Vout + static_cast<int64_t>(blockIdx.x) * (kJp * kJp);
    for (int e = tid; e < kJp * kJp; e += kSvdThreads) v[e] = V[e / kJp][e % kJp];
}

// The cross sweep of pair_eig_kernel (column i of block a against column i + r mod kJb of
// block b in round r) with G and V held in registers.  Slot i of block b holds column
// i + r mod kJb of b in round r, so the round's pairs are (i, i) and G splits into 2 x 2
// blocks M_ij = [[A_ij, C_ij], [C_ji, D_ij]] (A = G_aa, C = G_ab, D = G_bb in slot order)
// that each take J_i^T M_ij J_j with no data from other blocks.  Thread (i, h) -- lane
// i = t mod 32 of half-wave h = t / 32 -- keeps the blocks of columns j = h + 8 q, q < 4, and
// rows h + 8 u, u < 8, of V's columns (a_i, b_i); it computes the rotation of pair i and
// takes those of pairs j from lane j.  Between rounds the slots of b move down by one:
// C and D pass through LDS (ping-pong buffers, one barrier per round; C_ji is re-read from
// the copy of C_ij its owner wrote, so the two copies of an entry never drift apart), V's
// b columns and the diagonal of D through lane shuffles.  After kJb rounds the slots are
// back in column order.  Same tests, skip flag and flag as pair_eig_kernel.
__global__ void __launch_bounds__(kSvdThreads)
pair_eig_cross_kernel(const double* __restrict__ gram, int inner, double tol_r, double tol_c,
                      double* __restrict__ Vout, int* __restrict__ skip, int* __restrict__ flag) {
    static_assert(kJb == 32 && kSvdThreads == 256, "thread (lane, half-wave) layout");
    constexpr int kQ = 4, kU = 8;
    __shared__ double Cs[2][kJb][kJb + 1], Ds[2][kJb][kJb + 1];
    __shared__ int rot, big;
    const int tid = static_cast<int>(threadIdx.x);
    const int i = tid & (kJb - 1), h = tid >> 5;
    const double* g = gram + static_cast<int64_t>(blockIdx.x) * (kJp * kJp);
    double A[kQ], C1[kQ], C2[kQ], D[kQ], Djj[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int j = h + 8 * q;
        A[q] = g[i * kJp + j];
        C1[q] = g[i * kJp + kJb + j];
        C2[q] = g[j * kJp + kJb + i];
        D[q] = g[(kJb + i) * kJp + kJb + j];
        Djj[q] = g[(kJb + j) * (kJp + 1)];
    }
    double aii = g[i * (kJp + 1)], cii = g[i * kJp + kJb + i], dii = g[(kJb + i) * (kJp + 1)];
    if (tid == 0) {
        rot = 0;
        big = 0;
    }
    // a pair whose cross entries already pass the test rotates nothing: leave at once
    bool open = false;
#pragma unroll
    for (int q = 0; q < kQ; ++q)
        open = open || (C1[q] != 0.0 && C1[q] * C1[q] > tol_r * tol_r * aii * Djj[q]);
    if (!__syncthreads_or(open)) {
        if (tid == 0) skip[blockIdx.x] = 1;
        return;
    }
    double va[kU], vb[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int l = h + 8 * u;
        va[u] = l == i ? 1.0 : 0.0;
        vb[u] = l == kJb + i ? 1.0 : 0.0;
    }
    bool any = false;
    for (int sw = 0; sw < inner; ++sw) {
        for (int r = 0; r < kJb; ++r) {
            const int buf = r & 1;
            double ci, si, ti;
            bool bg;
            if (pair_rotation(aii, dii, cii, tol_r, tol_c, ci, si, ti, bg) && h == 0) {
                rot = 1;
                if (bg) big = 1;
            }
            double cj[kQ], sj[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                cj[q] = __shfl(ci, h + 8 * q, kJb);
                sj[q] = __shfl(si, h + 8 * q, kJb);
            }
            // V first (it needs only this lane's rotation, so it covers the shuffles' latency),
            // then b's slots of V move down by one.  No branches: c = 1, s = 0 leave every
            // value exactly as it was.
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const double x = va[u], y = vb[u];
                va[u] = ci * x - si * y;
                vb[u] = si * x + ci * y;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) vb[u] = __shfl(vb[u], (i + 1) & (kJb - 1), kJb);
            // pair i's diagonal entries after its rotation (closed form); every thread of lane
            // i holds them, and the owner of the diagonal block takes the same values
            const bool turned = si != 0.0;
            const double aii2 = turned ? aii - ti * cii : aii;
            const double dii2 = turned ? dii + ti * cii : dii;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                // H = M J_j, then J_i^T H; the diagonal block of a turned pair takes the
                // closed form (its cross entry becomes an exact zero)
                const double h00 = cj[q] * A[q] - sj[q] * C1[q], h01 = sj[q] * A[q] + cj[q] * C1[q];
                const double h10 = cj[q] * C2[q] - sj[q] * D[q], h11 = sj[q] * C2[q] + cj[q] * D[q];
                const bool dg = h + 8 * q == i;
                const double a2 = dg ? aii2 : ci * h00 - si * h10;
                const double d2 = dg ? dii2 : si * h01 + ci * h11;
                C1[q] = dg && turned ? 0.0 : ci * h01 - si * h11;
                A[q] = a2;
                D[q] = d2;
            }
            // publish C and D; the next round's slots move down by one.  A stays, the diagonal
            // of D moves across lanes, the rest through LDS after the barrier.
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int j = h + 8 * q;
                Cs[buf][i][j] = C1[q];
                Ds[buf][i][j] = D[q];
            }
            const int i1 = (i + 1) & (kJb - 1);
            aii = aii2;
            dii = __shfl(dii2, i1, kJb);
            __syncthreads();
            cii = Cs[buf][i][i1];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int j = h + 8 * q, j1 = (j + 1) & (kJb - 1);
                C1[q] = Cs[buf][i][j1];
                C2[q] = Cs[buf][j][i1];
                D[q] = Ds[buf][i1][j1];
            }
        }
        __syncthreads();
        const bool rotated = rot != 0;   // uniform: read after the sweep's last barrier
        __syncthreads();
        if (!rotated) break;
        any = true;
        if (tid == 0) rot = 0;   // rot is written by wave 0 only (h == 0), in program order after this
    }
    if (tid == 0) {
        skip[blockIdx.x] = any ? 0 : 1;
        if (big) flag[0] = 1;
    }
    if (!any) return;
    double* v = Vout + static_cast<int64_t>(blockIdx.x) * (kJp * kJp);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int l = h + 8 * u;
        v[l * kJp + i] = va[u];
        v[l * kJp + kJb + i] = vb[u];
    }
}

// [X_a X_b] <- [X_a X_b] V on rows [kJrows y, kJrows (y + 1)) (grid z = 0), and the same on
// W (z = 1), on the matrix cores as (X V)^T = V^T X^T: wave w takes kApplyTiles tiles of 16
// rows, lane (r, i) supplying row i of a tile's slot 4 s + r at reduction step s, and V^T
// from LDS (one read serves the wave's tiles).  A wave reads all
// of its rows before it writes them, and no other wave touches them, so the update is in
// place; lane l writes rows of one column, 16 lanes to a column.
__global__ void __launch_bounds__(kSvdThreads)
pair_apply_kernel(double* __restrict__ X, double* __restrict__ W, int k, int64_t ld, int nb, int np,
                  int round, const double* __restrict__ Vp, const int* __restrict__ skip) {
    if (skip[blockIdx.x] != 0) return;   // uniform per workgroup
    static_assert(kJrows == 16 * kApplyTiles * (kSvdThreads / 64), "kApplyTiles 16-row tiles per wave");
    __shared__ double vs[kJp * kJp];
    double* M = blockIdx.z == 0 ? X : W;
    int a, b;
    round_pair(np, round, static_cast<int>(blockIdx.x), a, b);
    const double* v = Vp + static_cast<int64_t>(blockIdx.x) * (kJp * kJp);
    {
        double t[kJp * kJp / kSvdThreads];
#pragma unroll
        for (int q = 0; q < kJp * kJp / kSvdThreads; ++q) t[q] = v[threadIdx.x + q * kSvdThreads];
#pragma unroll
        for (int q = 0; q < kJp * kJp / kSvdThreads; ++q) vs[threadIdx.x + q * kSvdThreads] = t[q];
    }
    const int lane = static_cast<int>(threadIdx.x) & 63, w = static_cast<int>(threadIdx.x) >> 6;
    const int rr = lane >> 4, ii = lane & 15;
    const int row0 = static_cast<int>(blockIdx.y) * kJrows + 16 * kApplyTiles * w + ii;
    double x[kApplyTiles][kJp / 4];
#pragma unroll
    for (int st = 0; st < kJp / 4; ++st) {
        const int c = pair_col(a, b, nb, 4 * st + rr, k);
#pragma unroll
        for (int h = 0; h < kApplyTiles; ++h) {
            const int row = row0 + 16 * h;
            x[h][st] = (c >= 0 && row < k) ? M[static_cast<int64_t>(c) * ld + row] : 0.0;
        }
    }
    __syncthreads();
    svd_v4d acc[kApplyTiles][4];
#pragma unroll
    for (int h = 0; h < kApplyTiles; ++h)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[h][m] = svd_v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < kJp / 4; ++st)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const double vt = vs[(4 * st + rr) * kJp + 16 * m + ii];
#pragma unroll
            for (int h = 0; h < kApplyTiles; ++h) acc[h][m] = svd_mfma(vt, x[h][st], acc[h][m]);
        }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = pair_col(a, b, nb, 16 * m + 4 * q + rr, k);
            if (c < 0) continue;
#pragma unroll
            for (int h = 0; h < kApplyTiles; ++h) {
                const int row = row0 + 16 * h;
                if (row < k) M[static_cast<int64_t>(c) * ld + row] = acc[h][m][q];
            }
        }
}

// sig[j] = ||X(:, j)||_2 (workgroup per column).
__global__ void __launch_bounds__(kSvdThreads)
column_norm_kernel(const double* __restrict__ X, int k, int64_t ld, double* __restrict__ sig) {
    __shared__ double sh[3][kSvdThreads / 64];
    const double* x = X + static_cast<int64_t>(blockIdx.x) * ld;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < k; i += kSvdThreads) a += x[i] * x[i];
    block_sum3(a, b, c, sh);
    if (threadIdx.x == 0) sig[blockIdx.x] = sqrt(a);
}

// pos[j] = place of column j in descending order of sig (equal values keep index order).
// sig is read through LDS, 256 values at a time (every value is compared by every thread).
// Launch: 256 threads per workgroup.
__global__ void __launch_bounds__(256)
svd_order_kernel(const double* __restrict__ sig, int k, int* __restrict__ pos) {
    __shared__ double sh[256];
    const int t = static_cast<int>(threadIdx.x);
    const int j = static_cast<int>(blockIdx.x) * 256 + t;
    const double v = j < k ? sig[j] : 0.0;
    int p = 0;
    for (int i0 = 0; i0 < k; i0 += 256) {
        __syncthreads();
        if (i0 + t < k) sh[t] = sig[i0 + t];
        __syncthreads();
        const int n = k - i0 < 256 ? k - i0 : 256;
        for (int q = 0; q < n; ++q) {
            const double u = sh[q];
            p += (u > v || (u == v && i0 + q < j)) ? 1 : 0;
        }
    }
    if (j < k) pos[j] = p;
}

// Sorted outputs: s[pos[j]] = sig[j], Ut(:, pos[j]) = X(:, j) / sig[j] (zero for a zero
// column), Ws(:, pos[j]) = W(:, j).  Grid: (column blocks of 256 rows, k columns).
__global__ void svd_gather_kernel(const double* __restrict__ X, const double* __restrict__ W, int k,
                                  int64_t ld, const double* __restrict__ sig,
                                  const int* __restrict__ pos, double* __restrict__ s_out,
                                  double* __restrict__ Ut, double* __restrict__ Ws) {
    const int j = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = pos[j];
    const double v = sig[j];
    if (i == 0) s_out[p] = v;
    if (i >= k) return;
    const double inv = v > 0.0 ? 1.0 / v : 0.0;
    Ut[static_cast<int64_t>(p) * ld + i] = X[static_cast<int64_t>(j) * ld + i] * inv;
    Ws[static_cast<int64_t>(p) * ld + i] = W[static_cast<int64_t>(j) * ld + i];
}

// Sign rule: make the entry of largest magnitude of V(:, j) positive (smallest row among
// equal magnitudes), flipping V(:, j) and Ut(:, j) together.  Workgroup per column.
__global__ void __launch_bounds__(kSvdThreads)
sign_rule_kernel(double* __restrict__ V, int64_t n, int64_t ldv, double* __restrict__ Ut,
                 int k, int64_t ldu) {
    __shared__ double sv[kSvdThreads];
    __shared__ int64_t si[kSvdThreads];
    double* v = V + static_cast<int64_t>(blockIdx.x) * ldv;
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t i = threadIdx.x; i < n; i += kSvdThreads) {
        const double a = fabs(v[i]);
        if (a > best) {
            best = a;
            bi = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kSvdThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const double o = sv[threadIdx.x + off];
            const int64_t oi = si[threadIdx.x + off];
            if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (!(v[si[0]] < 0.0)) return;   // uniform: every thread reads the same entry
    for (int64_t i = threadIdx.x; i < n; i += kSvdThreads) v[i] = -v[i];
    double* u = Ut + static_cast<int64_t>(blockIdx.x) * ldu;
    for (int i = threadIdx.x; i < k; i += kSvdThreads) u[i] = -u[i];
}

// W = I (k x k, column-major, ld).
__global__ void identity_kernel(double* __restrict__ W, int k, int64_t ld) {
    const int j = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) W[static_cast<int64_t>(j) * ld + i] = i == j ? 1.0 : 0.0;
}

int jacobi_blocks(int k) { return (k + kJb - 1) / kJb; }
int jacobi_rounds(int k) {
    const int nb = jacobi_blocks(k);
    return nb + (nb & 1) - 1;
}
size_t jacobi_part_elems(int k) {
    const int nb = jacobi_blocks(k);
    const int64_t pairs = (nb + (nb & 1)) / 2;
    return static_cast<size_t>(pairs * (cdiv(k, kGramRows) + 1) * kJp * kJp);   // partials, sums
}
size_t jacobi_rot_elems(int k) {
    const int nb = jacobi_blocks(k);
    return static_cast<size_t>((nb + (nb & 1)) / 2) * kJp * kJp;
}

hipError_t launch_jacobi_block_round(double* X, double* W, int k, int64_t ld, int round, double tol_r,
                                     double tol_c, int inner, double* part, double* V, int* skip,
                                     int* flag, hipStream_t s) {
    const int nb = jacobi_blocks(k);
    const int np = nb + (nb & 1);
    const unsigned pairs = static_cast<unsigned>(np / 2);
    const int nsplit = static_cast<int>(cdiv(k, kGramRows));
    hipLaunchKernelGGL(pair_gram_kernel, dim3(pairs, static_cast<unsigned>(nsplit)), dim3(kSvdThreads), 0, s,
                       X, k, ld, nb, np, round, nsplit, part);
    double* gram = part + static_cast<int64_t>(pairs) * nsplit * (kJp * kJp);
    hipLaunchKernelGGL(pair_reduce_kernel, dim3(pairs, (kJp * kJp) / kSvdThreads), dim3(kSvdThreads), 0, s,
                       part, nsplit, gram);
    if (round >= 0)
        hipLaunchKernelGGL(pair_eig_cross_kernel, dim3(pairs), dim3(kSvdThreads), 0, s, gram, inner, tol_r, tol_c,
                           V, skip, flag);
    else
        hipLaunchKernelGGL(pair_eig_kernel, dim3(pairs), dim3(kSvdThreads), 0, s, gram, inner, tol_r, tol_c, V,
                           skip, flag);
    hipLaunchKernelGGL(pair_apply_kernel, dim3(pairs, static_cast<unsigned>(cdiv(k, kJrows)), 2), dim3(kSvdThreads),
                       0, s, X, W, k, ld, nb, np, round, V, skip);
    return hipGetLastError();
}

hipError_t launch_svd_finish(const double* X, const double* W, int k, int64_t ld, double* sig,
                             int* pos, double* s_out, double* Ut, double* Ws, hipStream_t s) {
    hipLaunchKernelGGL(column_norm_kernel, dim3(static_cast<unsigned>(k)), dim3(kSvdThreads), 0, s, X,
                       k, ld, sig);
    hipLaunchKernelGGL(svd_order_kernel, dim3(static_cast<unsigned>(cdiv(k, 256))), dim3(256), 0, s,
                       sig, k, pos);
    hipLaunchKernelGGL(svd_gather_kernel, dim3(static_cast<unsigned>(cdiv(k, 256)), static_cast<unsigned>(k)),
                       dim3(256), 0, s, X, W, k, ld, sig, pos, s_out, Ut, Ws);
    return hipGetLastError();
}

hipError_t launch_sign_rule(double* V, int64_t n, int64_t ldv, double* Ut, int k, int64_t ldu,
                            hipStream_t s) {
    hipLaunchKernelGGL(sign_rule_kernel, dim3(static_cast<unsigned>(k)), dim3(kSvdThreads), 0, s, V, n,
                       ldv, Ut, k, ldu);
    return hipGetLastError();
}

hipError_t launch_identity(double* W, int k, int64_t ld, hipStream_t s) {
    hipLaunchKernelGGL(identity_kernel, dim3(static_cast<unsigned>(cdiv(k, 256)), static_cast<unsigned>(k)),
                       dim3(256), 0, s, W, k, ld);
    return hipGetLastError();
}

}  // namespace qb
