/*
 * qb.h -- C ABI of the MI355X (gfx950) fixed-precision randomized QB library.
 *
 * The library computes A ~ Q B with Q (m x k) orthonormal and B = Q^T A, choosing the
 * rank k adaptively so that ||A - QB||_F < tol ||A||_F, following Yu, Gu, Li,
 * "Efficient randomized algorithms for the fixed-precision low-rank matrix
 * approximation" (arXiv 1606.09402):
 *   - randQB_FP: Algorithm 4 (Algorithm 3 plus the re-orthogonalised blocks,
 *     eq. (23)); one sweep G = A Omega, H = A^T G per chunk of Omega columns, then a
 *     block loop that touches only G, H, Omega, Q, B.  With power parameter P > 0
 *     (binary64 A only) each chunk first runs P rounds G = orth(A Omega),
 *     Omega = orth(A^T G) (the power scheme), on the residual A - QB after the first chunk.
 *   - randQB_EI: Algorithm 2, two passes over A per block.
 *   - both stop with the Frobenius error indicator of Theorem 1 / Algorithm 1,
 *     decremented row by row (Section 3.1) unless row_by_row == 0.
 *   - A may be dense (binary64, or bfloat16 / e4m3 for randQB_FP's precision form), CSR,
 *     or COO (turned into CSR on the device); a batched fixed-rank form with its adjoint
 *     serves differentiation; qb_svd_from_qb turns a QB factorisation into an approximate
 *     truncated SVD (eq. (3)).
 *
 * Conventions shared by every entry point
 *   - All matrix pointers are DEVICE pointers owned by the caller.  The library never
 *     allocates or frees device memory: scratch memory comes from the caller's workspace
 *     (qb_fp_dense_noalloc: from a static array of the library).  Host-side read-backs go
 *     to pageable memory of the calling thread.  A host thread's first call on a device
 *     creates that thread's side stream and timing events for the device; later calls
 *     reuse them (they live until the process ends).
 *   - All device work is ordered after earlier work on the caller's stream, and the call's
 *     results are complete on that stream when it returns (parts may run on private
 *     streams of default priority, joined to the caller's stream by events); calls that
 *     return a rank synchronise that stream before returning.  For randQB_FP and randQB_EI
 *     the stopping rule runs on the device; the host reads its state back once per run of
 *     up to 4 blocks (randQB_FP) or once per block (randQB_EI), so blocks past the stop may
 *     have been enqueued: their products are skipped on the device, and what they leave
 *     lies outside [0, rank).
 *   - Dense A is row-major: A(i, j) at a[i * lda + j], lda >= n.
 *   - Q is column-major m x l_max: Q(i, j) at Q[j * ldq + i], ldq >= m.
 *   - B is row-major l_max x n: B(i, j) at B[i * ldb + j], ldb >= n.
 *     On return columns [0, rank) of Q and rows [0, rank) of B are valid; the rest
 *     of the l_max capacity may hold scratch values.
 *   - Omega is the bit-specified Gaussian matrix described at qb_gaussian_fill.
 *   - No C++ exception crosses this interface; every function returns a qb_status.
 */
#ifndef QB_H
#define QB_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QB_API __attribute__((visibility("default")))

typedef enum {
    QB_OK = 0,               /* converged: E < (tol ||A||_F)^2                                   */
    QB_NOT_CONVERGED = 1,    /* warning: l_max reached, or the numerical rank of A was exhausted
                                (info.exhausted = 1) with E >= eps^2; outputs valid for [0,rank) */
    QB_WARN_TOL_FLOOR = 2,   /* warning: tol below the Theorem 3 floor sqrt(4u/0.01) = 2.1e-7 for
                                binary64; E may be inaccurate.  The call still runs.            */
    QB_ERR_ARG = -1,         /* invalid argument (sizes, strides, NULL pointers, b, l_tilde ...) */
    QB_ERR_NONFINITE = -2,   /* ||A||_F^2 is NaN or Inf                                          */
    QB_ERR_WORKSPACE = -3,   /* workspace smaller than qb_workspace_bytes() reports              */
    QB_ERR_HIP = -4,         /* a HIP runtime call failed                                        */
    QB_ERR_UNSUPPORTED = -5  /* e.g. power > 0 with randQB_EI or a low-precision A, or an
                                element type this entry point lacks                           */
} qb_status;

typedef enum { QB_ALGO_FP = 0, QB_ALGO_EI = 1 } qb_algo;

/* Element type of a dense A.
 *   QB_F64  binary64.
 *   QB_BF16 bfloat16 storage (the precision form of randQB_FP): the matrix factorised
 *           is the stored A_q.  ||A_q||^2 is summed in binary64 from the stored values
 *           (their squares are exact), so Theorem 1 holds for A_q.  The two sketch
 *           products run on bfloat16 matrix cores with binary32 accumulation:
 *             Omega_q = bf16(Omega)       (round to nearest even from binary64),
 *             G_q     = bf16(A_q Omega_q) (binary32 accumulation, then rounded),
 *             H       = A_q^T G_q         (binary32 accumulation, kept in binary64);
 *           the block loop (W, Y_i, both QRs, eq. (23), the indicator) runs in binary64
 *           on Omega_q, G_q and H, i.e. on exactly the operands of the two products,
 *           so B_i = Q_i^T A_q up to the accumulation error of H.  Only randQB_FP
 *           accepts it (randQB_EI forms B_i = Q_i^T A directly and would need Q_i in
 *           bfloat16: QB_ERR_UNSUPPORTED).
 *   QB_FP8E4M3 8-bit storage (OCP e4m3fn: 4 exponent bits, bias 7, 3 stored significand
 *           bits, finite values up to 448) with a power-of-two scale per row:
 *           A_q(i, j) = 2^row_exp[i] * e4m3(a[i * lda + j]).  Every such value is a
 *           bfloat16 value, and the precision form above applies to A_q with an 8-bit
 *           Omega for the G product:
 *             Omega_q = e4m3(2^5 Omega) / 2^5   (round to nearest even; 2^5 |Omega| < 448),
 *             G_q     = bf16(A_q Omega_q)       (8-bit matrix cores, e4m3 x e4m3, binary32
 *                                               accumulation -- each product is exact --
 *                                               when n is a multiple of 64 and the rows of
 *                                               A start 16-byte aligned, else the same
 *                                               values on bfloat16 matrix cores),
 *             H       = A_q^T G_q               (bfloat16 matrix cores, A_q widened on load);
 *           the row scales enter the G epilogue (and the H operand) as exact power-of-two
 *           multiplications, and ||A_q||^2 is summed in binary64 from the scaled stored
 *           values.
 *   QB_F32  binary32 (the differentiation form's batches, qb_batch). */
typedef enum { QB_F64 = 0, QB_BF16 = 1, QB_F32 = 2, QB_FP8E4M3 = 3 } qb_dtype;

/* Dense row-major matrix of element type dtype (a qb_dtype). */
typedef struct {
    int64_t m, n;       /* rows, columns (m, n >= 1)                         */
    int64_t lda;        /* row stride in elements, lda >= n                  */
    int32_t dtype;      /* qb_dtype                                          */
    int32_t reserved;
    const void* a;      /* device pointer to A(0,0)                          */
    const int32_t* row_exp; /* QB_FP8E4M3: device, m per-row exponents in
                               [-100, 100]; ignored for other types           */
} qb_dense;

/* Compressed sparse row matrix (Section 5.1 stores sparse A in CSR).  Column indices
 * must lie in [0, n); duplicates are summed as in the usual CSR semantics. */
typedef struct {
    int64_t m, n, nnz;
    const int64_t* rowptr;  /* device, m + 1 entries, rowptr[0] = 0, rowptr[m] = nnz */
    const int32_t* colind;  /* device, nnz entries                                    */
    const double* val;      /* device, nnz entries                                    */
} qb_csr;

/* Sparse A as coordinate triplets (the COO format that Remark 3.2's experiments also use):
 * entries in any order; entries with the same (row, col) are summed, in their input order. */
typedef struct {
    int64_t m, n, nnz;      /* nnz < 2^31                                                      */
    const int32_t* row;     /* device, nnz entries, 0 <= row < m                              */
    const int32_t* col;     /* device, nnz entries, 0 <= col < n                              */
    const double* val;      /* device, nnz entries                                            */
} qb_coo;

typedef struct {
    double tol_rel;      /* stop when E < (tol_rel ||A||_F)^2 (strict), 0 <= tol_rel       */
    int32_t b;           /* block size, 1 <= b <= 128.  The b x b Cholesky
                            factors and triangular inverses of every block are formed in one
                            workgroup's registers and LDS, which bounds b; Section 5 uses
                            b = 10 to 50.                                                   */
    int32_t power;       /* power-scheme parameter P of Algorithm 4, 0 <= P <= 16.
                            P > 0 is accepted by randQB_FP on binary64 A (dense or CSR) and
                            returns QB_ERR_UNSUPPORTED elsewhere.  Each chunk's Gaussian
                            Omega is replaced by the result of P rounds
                            G = orth((A - QB) Omega), Omega = orth((A - QB)^T G) (Q, B the
                            factors so far; A itself in the first chunk), orth being the Q
                            factor of a thin QR with positive diag(R); a chunk then costs
                            2 P + 2 passes over A.                                          */
    int64_t l_max;       /* capacity of Q / B, 1 <= l_max <= min(m, n)                       */
    int64_t l_tilde;     /* randQB_FP chunk width: a multiple of b, or 0 for min(50 b, l_max)
                            (Section 5.4).  A chunk that runs out is followed by the next
                            l_tilde columns of Omega and a fresh G, H sweep.  -1 selects an
                            adaptive schedule: 8 b columns first, then each new chunk is
                            sized from the decay of E over the second half of the previous
                            one (1.1 x the columns a geometric extrapolation needs to reach
                            eps^2, plus b, rounded up to a multiple of b, within
                            [b, 4 x previous]), never wider than min(50 b, l_max).           */
    uint64_t seed;       /* Philox key of Omega                                              */
    int32_t row_by_row;  /* 1: Section 3.1 row by row (rank any integer); 0: whole-block stop */
    int32_t reserved;
} qb_params;

typedef struct {
    int64_t rank;        /* number of valid columns of Q / rows of B                        */
    double E;            /* final indicator ||A||^2 - ||B||^2 (may be negative, Section 3.3)  */
    double normA2;       /* ||A||_F^2                                                        */
    int32_t status;      /* same as the return value                                         */
    int32_t passes;      /* passes over A (FP: 2 P + 2 per chunk; EI: 2 per block)           */
    int32_t blocks;      /* blocks processed                                                 */
    int32_t chunks;      /* Omega chunks drawn (FP)                                          */
    int32_t exhausted;   /* 1 if R_i(j,j) <= 2^-40 ||A Omega(:,j)||_2 ended the run            */
    int32_t fallbacks;   /* blocks (or power-scheme panels) redone by the Householder fallback */
    double ms[8];        /* device time per phase (ms): 0 ||A||^2, 1 Omega, 2 G = A Omega,
                            3 H = A^T G (EI: 2 = the A Omega_i GEMMs, 3 = the A^T Q_i GEMMs),
                            4 block loop without 2-3, 5 whole call, 6 power-scheme rounds
                            (their products with A and orthonormalisations), 7 COO to CSR
                            conversion (qb_*_coo only; not part of 5)                       */
    double gemm_flops[2];/* algorithmic flops of the timed G and H GEMMs (2 m n l each)      */
} qb_info;

/* Bytes of workspace qb_{fp,ei}_{dense,csr} need for this problem (algo = qb_algo,
 * sparse = 0/1, nnz ignored for dense) with binary64 A.  Returns 0 for invalid
 * arguments. */
QB_API size_t qb_workspace_bytes(int algo, int sparse, int64_t m, int64_t n, int64_t nnz,
                          const qb_params* p);

/* Bytes of workspace qb_fp_dense / qb_ei_dense need for dense A of any dtype (the
 * bfloat16 form adds bfloat16 copies of Omega_q and G_q).
 * A->a is not read.  Returns 0 for invalid arguments or an unsupported combination. */
QB_API size_t qb_dense_workspace_bytes(int algo, const qb_dense* A, const qb_params* p);

/* randQB_FP (Algorithm 4) on dense row-major A of dtype QB_F64, QB_BF16 or QB_FP8E4M3
 * (A->row_exp then gives the per-row power-of-two scales).  p->power > 0 (the power scheme
 * of Algorithm 4) is accepted for QB_F64 only.  ws must hold at least
 * qb_dense_workspace_bytes(QB_ALGO_FP, A, p) bytes of device memory (256-byte aligned).  For
 * the low-precision element types the relative tolerance is taken against ||A_q||_F. */
QB_API int qb_fp_dense(const qb_dense* A, const qb_params* p, double* Q, int64_t ldq, double* B,
                int64_t ldb, void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info);

/* Size of the device scratch array that qb_fp_dense_noalloc works in. */
#define QB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* qb_fp_dense for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same arguments without the
 * workspace.  The call allocates nothing: its workspace is a static device array of
 * QB_NOALLOC_SCRATCH_BYTES bytes inside the library (each device the library runs on holds
 * one until the process ends); it creates no stream or event (everything runs on the
 * caller's stream, and info->ms stays zero), and reads the per-block decision data back into
 * pageable memory of the calling thread.  The first call on a device looks up that
 * device's array address once.  Every call on a device shares that device's array, so
 * calls that overlap on one device (several host threads or streams) race and must be
 * serialised by the caller.  The layout is qb_fp_dense's with the split-K partials cut to
 * what the array leaves, so the products may take fewer K splits: the results agree with
 * qb_fp_dense's to rounding.  Returns QB_ERR_WORKSPACE, before any device work, when the
 * problem's Omega / G / H chunks and block buffers do not fit in the array (for example,
 * binary64 A with m, n about 1000 and a 50 b chunk fits; 4096 x 4096 with b = 64 does not);
 * otherwise as qb_fp_dense. */
QB_API int qb_fp_dense_noalloc(const qb_dense* A, const qb_params* p, double* Q, int64_t ldq,
                               double* B, int64_t ldb, hipStream_t stream, qb_info* info);

/* randQB_EI (Algorithm 2) on dense row-major binary64 A; EI's Omega_i is column block
 * i of the same Omega as randQB_FP uses. */
QB_API int qb_ei_dense(const qb_dense* A, const qb_params* p, double* Q, int64_t ldq, double* B,
                int64_t ldb, void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info);

/* randQB_FP on CSR A: G = A Omega by a row-parallel SpMM, H = A^T G by the same SpMM
 * on CSR(A^T), which the call builds once in the workspace. */
QB_API int qb_fp_csr(const qb_csr* A, const qb_params* p, double* Q, int64_t ldq, double* B,
              int64_t ldb, void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info);

/* randQB_EI on CSR A. */
QB_API int qb_ei_csr(const qb_csr* A, const qb_params* p, double* Q, int64_t ldq, double* B,
              int64_t ldb, void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info);

/* randQB_FP / randQB_EI on COO input: the triplets are first turned into CSR inside the
 * workspace (a stable sort by (row, col), duplicates summed in input order, a fixed-order
 * sum), then the CSR path runs.  Workspace: qb_coo_workspace_bytes.  An index outside the
 * matrix returns QB_ERR_ARG.  info->ms[7] receives the device time of the conversion. */
QB_API size_t qb_coo_workspace_bytes(int algo, const qb_coo* A, const qb_params* p);
QB_API int qb_fp_coo(const qb_coo* A, const qb_params* p, double* Q, int64_t ldq, double* B,
              int64_t ldb, void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info);
QB_API int qb_ei_coo(const qb_coo* A, const qb_params* p, double* Q, int64_t ldq, double* B,
              int64_t ldb, void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info);

/* The conversion alone: CSR arrays of A (rowptr m + 1 entries, colind and val at least
 * A->nnz entries; device memory of the caller) and the CSR entry count in *nnz_out (host).
 * Workspace: qb_coo_to_csr_bytes.  Synchronises the stream.  QB_ERR_ARG on an index outside
 * the matrix. */
QB_API size_t qb_coo_to_csr_bytes(const qb_coo* A);
QB_API int qb_coo_to_csr(const qb_coo* A, int64_t* rowptr, int32_t* colind, double* val,
                         int64_t* nnz_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* trQRCP driven by the indicator (Remark 3.2): the truncated randomized QR with column
 * pivoting of Duersch and Gu, stopped by the same indicator E = ||A||^2 - ||B||^2 and
 * row-by-row rule (Section 3.1) as randQB, on dense row-major binary64 A.  The column
 * permutation does not change the Frobenius norms of B or of its rows, so Theorem 1 holds.
 *   Sketch: S = Omega^T A once, Omega the m x l Gaussian matrix of qb_gaussian_fill with
 *   stream 1 (batch 0, rows 0..m-1, columns 0..l-1), l = b + oversample.
 *   Block (bw = min(b, l_max - k) columns): bw steps of Householder QR with column pivoting
 *   on the sketch pick the pivots J (the remaining sketch column of largest norm, the
 *   smallest index among equal norms); then, as a block of Algorithm 2 with A(:, J) in place
 *   of A Omega_i: Q_i = orth(A(:, J) - Q B(:, J)), re-orthogonalised, B_i = Q_i^T A; the
 *   indicator is decremented row by row with the exhaustion guard against ||A(:, J_j)||; the
 *   sketch follows the residual by the sample update S <- S - S(:, J) R_i^{-1} B_i (no
 *   second pass for it).  passes = 1 + blocks.
 *   Q    out, m x rank, column-major (ldq >= m), orthonormal columns.
 *   B    out, rank x n row-major (ldb >= n) in the ORIGINAL column order, i.e. B = R P^T:
 *        B(:, piv) is upper triangular up to rounding, and A ~ Q B as for randQB.
 *   piv  out, device, at least l_max int32: the pivot columns in pivot order (0..rank-1).
 *   p->power must be 0 (else QB_ERR_UNSUPPORTED); p->l_tilde is ignored; A must be QB_F64
 *   (else QB_ERR_UNSUPPORTED); 0 <= oversample <= 128 (else QB_ERR_ARG).  Workspace:
 *   qb_trqrcp_workspace_bytes (256-byte aligned; 0 for invalid arguments).  Synchronises the
 *   stream once per block.  Returns as qb_fp_dense. */
QB_API size_t qb_trqrcp_workspace_bytes(int64_t m, int64_t n, const qb_params* p, int32_t oversample);
QB_API int qb_trqrcp_dense(const qb_dense* A, const qb_params* p, int32_t oversample, double* Q,
                           int64_t ldq, double* B, int64_t ldb, int32_t* piv, void* ws,
                           size_t ws_bytes, hipStream_t stream, qb_info* info);

/* Omega(row0 + r, col0 + c) for r < rows, c < cols into out[r * ld + c] (row-major,
 * ld >= cols).  The paper only asks for a standard Gaussian matrix (randn in
 * Algorithms 2 and 4); this library pins the draw so that runs are reproducible:
 *   entry (i, 2p + q), q in {0, 1}: Philox4x32-10 with counter (i, p, stream, batch) and
 *   key (seed mod 2^32, seed div 2^32) gives words w0..w3;
 *   u1 = (((w0 << 32 | w1) >> 12) + 1/2) 2^-52, u2 likewise from (w2, w3);
 *   r = sqrt(-2 ln u1); q = 0 -> r cos(2 pi u2), q = 1 -> r sin(2 pi u2);
 *   ln, sqrt, sin, cos evaluated with IEEE binary64 +,-,*,/ only in a fixed order
 *   (atanh series for ln, six Newton steps for sqrt, degree-17/16 Taylor polynomials
 *   on [0, pi/4] with quadrant folding for sin / cos).
 * Enqueued on stream; does not synchronise. */
QB_API int qb_gaussian_fill(uint64_t seed, uint32_t stream_id, uint32_t batch, int64_t row0,
                     int64_t col0, int64_t rows, int64_t cols, double* out, int64_t ld,
                     hipStream_t stream);

/* ||A||_F^2 (Theorem 1 / Algorithm 1) of dense row-major A (QB_F64 or
 * QB_BF16), as a deterministic FP64 tree sum of squares; *out_host receives the value.
 * ws needs qb_sumsq_workspace_bytes() bytes.  Synchronises the stream. */
QB_API size_t qb_sumsq_workspace_bytes(void);
QB_API int qb_sumsq_dense(const qb_dense* A, double* out_host, void* ws, hipStream_t stream);

/* One sketch sweep of randQB_FP (Algorithm 4 with P = 0: Omega, G and H):
 * Omega(:, col0:col0+l) drawn as in qb_gaussian_fill (stream 0, batch 0) into om
 * (n x l, row-major, ld l), G = A Omega into g (m x l row-major, ld l), H = A^T G into
 * h (n x l row-major, ld l).  Enqueued on stream; does not synchronise. */
QB_API int qb_sketch_dense(const qb_dense* A, uint64_t seed, int64_t col0, int64_t l, double* om,
                    double* g, double* h, hipStream_t stream);

/* Single-pass form of the same sweep (Remark 4.2) for binary64 A: A is streamed in panels
 * of panel_rows rows (0: panels of at most 96 MiB of A, a multiple of 128 rows); each panel
 * A_p gives G_p = A_p Omega, and A_p^T G_p is added to H right after, while A_p may still be
 * in the last-level cache.  A leaves HBM once per panel only if the panel and the operands
 * the two products stream beside it fit in that cache together, roughly
 * 8 (panel_rows (n + l) + 2 n l) bytes within 256 MiB; for wider l the n x l operands
 * Omega and H evict the panel and A is read about twice, as by qb_sketch_dense (measured
 * at 20000 x 15000, l = 1024: about three times the algorithmic bytes, and slower than the
 * two-pass sweep).  om, g, h as in qb_sketch_dense; H is summed over the panels in row
 * order (a fixed order, so the result is reproducible; it equals qb_sketch_dense's H up to
 * rounding).  ws (caller-owned device memory, qb_sketch_onepass_bytes bytes; 0 for invalid
 * arguments) holds the split-K partials of the panel products.  Enqueued on stream; does
 * not synchronise. */
QB_API size_t qb_sketch_onepass_bytes(const qb_dense* A, int64_t l, int64_t panel_rows);
QB_API int qb_sketch_onepass(const qb_dense* A, uint64_t seed, int64_t col0, int64_t l,
                             int64_t panel_rows, double* om, double* g, double* h, void* ws,
                             size_t ws_bytes, hipStream_t stream);

/* The same sweep for bfloat16 or row-scaled e4m3 A (dtype QB_BF16 or QB_FP8E4M3),
 * exactly as qb_fp_dense runs it:
 * om receives the dequantised Omega_q (n x l, ld l), g the dequantised G_q (m x l,
 * ld l) and h = A_q^T G_q (n x l, ld l), all binary64.  ws (256-byte aligned) needs
 * qb_sketch_lowp_bytes(A, l) bytes.  Enqueued on stream; does not synchronise. */
QB_API size_t qb_sketch_lowp_bytes(const qb_dense* A, int64_t l);
QB_API int qb_sketch_lowp(const qb_dense* A, uint64_t seed, int64_t col0, int64_t l, double* om,
                          double* g, double* h, void* ws, size_t ws_bytes, hipStream_t stream);

/* Same sweep for CSR A; csc_ws must hold qb_csr_transpose_bytes(A) bytes and is
 * filled with CSR(A^T) on the first call (set *csc_ready = 0 before it). */
QB_API size_t qb_csr_transpose_bytes(const qb_csr* A);
QB_API int qb_sketch_csr(const qb_csr* A, uint64_t seed, int64_t col0, int64_t l, double* om,
                  double* g, double* h, void* csc_ws, int* csc_ready, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Differentiation form: fixed-rank randQB_FP on a batch of matrices and its adjoint.
 *
 * For each matrix A (m x n) of the batch and the fixed Gaussian Omega (n x k, drawn as in
 * qb_gaussian_fill with stream 0, batch 0, columns 0..k-1, rounded to the element type),
 * the forward runs randQB_FP without stopping for t = k / b blocks (Algorithm 3 with the
 * re-orthogonalised blocks and eq. (23); G = A Omega and H = A^T G once).  In exact
 * arithmetic the result is Q = qf(A Omega) with diag(R) > 0 and B = Q^T A, a
 * differentiable function of A; the backward computes dL/dA from dL/dQ and dL/dB by the
 * adjoints of B = Q^T A, of the thin QR (R-bar = 0) and of the triangular solve with R,
 * recomputing G = A Omega and R = Q^T G instead of keeping them from the forward.
 * The element type is QB_F32 (binary32 MFMA throughout) or QB_F64.
 * ------------------------------------------------------------------------------------ */

/* A batch of row-major matrices: matrix z, element (i, j) at a[z * stride_a + i * lda + j]. */
typedef struct {
    int64_t batch;      /* 1 .. 65535                                        */
    int64_t m, n;       /* rows, columns                                     */
    int64_t lda;        /* row stride, lda >= n                              */
    int64_t stride_a;   /* batch stride, >= m * lda when batch > 1           */
    int32_t dtype;      /* QB_F32 or QB_F64                                  */
    int32_t reserved;
    const void* a;      /* device pointer                                    */
} qb_batch;

/* Workspace bytes of qb_fixed_rank_fwd / _bwd (the same buffer serves both): k a
 * multiple of b, 1 <= b <= 64, k <= 256, k <= min(m, n).  0 for invalid arguments. */
QB_API size_t qb_fixed_rank_workspace_bytes(const qb_batch* A, int64_t k, int32_t b);

/* Forward.  Q: per matrix m x k row-major (row stride ldq >= k, batch stride stride_q);
 * B: per matrix k x n row-major (ldb >= n, stride_b).  A CholeskyQR pivot below 1e-6
 * (binary32) or 1e-12 (binary64) of the largest Gram diagonal in some block means that
 * A Omega is numerically rank deficient at rank k and Q, B are unreliable; it is reported
 * through breakdown:
 *   breakdown  device int32, or NULL.  Non-NULL: the call is only enqueued (no host wait) and
 *              *breakdown is set, in stream order, to 1 after such a pivot and 0 otherwise.
 *              NULL: the call synchronises the stream and returns QB_NOT_CONVERGED (a
 *              warning) after such a pivot. */
QB_API int qb_fixed_rank_fwd(const qb_batch* A, int64_t k, int32_t b, uint64_t seed, void* Q,
                             int64_t ldq, int64_t stride_q, void* B, int64_t ldb, int64_t stride_b,
                             void* ws, size_t ws_bytes, int32_t* breakdown, hipStream_t stream);

/* Backward: dA = dL/dA (per matrix m x n row-major, ldda >= n) from the forward's Q and
 * the adjoints dQ (m x k, may be NULL for zero) and dB (k x n, may be NULL).  dA is
 * overwritten.  Enqueued on stream; does not synchronise. */
QB_API int qb_fixed_rank_bwd(const qb_batch* A, int64_t k, int32_t b, uint64_t seed, const void* Q,
                             int64_t ldq, int64_t stride_q, const void* dQ, int64_t lddq,
                             int64_t stride_dq, const void* dB, int64_t lddb, int64_t stride_db,
                             void* dA, int64_t ldda, int64_t stride_da, void* ws, size_t ws_bytes,
                             hipStream_t stream);

/* Approximate truncated SVD from a QB factorisation (eq. (3) of the paper): the SVD of the
 * small factor, B = U~ diag(s) V~^T, turns A ~ QB into A ~ (Q U~) diag(s) V~^T; the leading
 * j columns of U = Q U~ and V = V~ with the leading j values of s approximate the rank-j SVD
 * of A.  B^T is first reduced by a thin QR, B^T = P T (the block orthonormalisation of the
 * power scheme in 64-column blocks: CholeskyQR twice, Householder on breakdown), then the
 * k x k factor T^T is diagonalised by block one-sided Jacobi (blocks of 32 columns; a sweep
 * turns every column pair of neighbouring blocks, then runs the circle ordering over the
 * blocks, turning the column pairs across each pair of blocks; each pair of blocks is
 * rotated by the product of one cyclic Jacobi sweep over its Gram matrix; a column pair is
 * rotated while its cosine exceeds 16 sqrt(k) 2^-53), and V = P W.
 *   Q  m x k, column-major (ldq >= m), orthonormal columns (as qb_fp_* return it)
 *   B  k x n, row-major (ldb >= n)
 *   U  out, m x k column-major (ldu >= m); s out, k values in descending order;
 *   V  out, n x k column-major (ldv >= n).  Sign rule: the entry of largest magnitude of each
 *      column of V is positive (the smallest row index among equal magnitudes); the column
 *      of U flips with it.  A zero singular value leaves its column of U zero.
 *   1 <= k <= min(m, n).  All pointers are device pointers; the workspace (256-byte
 *   aligned, qb_svd_workspace_bytes) holds every temporary.  The call synchronises the
 *   stream (one flag per Jacobi sweep).  *sweeps (may be NULL) receives the sweeps over all
 *   pairs of blocks taken.  Returns QB_OK, QB_NOT_CONVERGED if 40 sweeps did not converge (outputs still
 *   written), QB_ERR_ARG, QB_ERR_WORKSPACE or QB_ERR_HIP. */
QB_API size_t qb_svd_workspace_bytes(int64_t m, int64_t n, int64_t k);
QB_API int qb_svd_from_qb(int64_t m, int64_t n, int64_t k, const double* Q, int64_t ldq,
                          const double* B, int64_t ldb, double* U, int64_t ldu, double* s, double* V,
                          int64_t ldv, void* ws, size_t ws_bytes, hipStream_t stream,
                          int32_t* sweeps);

/* Host-only self-check of the workspace layouts (no device work, no allocation): QB_OK if
 * every region of the workspace that qb_{fp,ei}_{dense,csr} (oversample = 0, element type
 * dtype) or qb_trqrcp_dense (oversample > 0: algo QB_ALGO_EI, sparse 0, QB_F64) would carve
 * for this problem holds what the kernels writing it produce, QB_ERR_WORKSPACE if one is
 * short, QB_ERR_ARG for invalid arguments. */
QB_API int qb_layout_check(int algo, int sparse, int dtype, int64_t m, int64_t n, int64_t nnz,
                           const qb_params* p, int32_t oversample);

/* Human-readable name of a qb_status value (static storage). */
QB_API const char* qb_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* QB_H */
