// Launchers of the library's HIP kernels (host-callable, all enqueue on a stream).
#pragma once

#include "common.h"

namespace qb {

// rng.hip -- bit-specified Gaussian Omega
hipError_t launch_gauss_fill(uint64_t seed, uint32_t stream_id, uint32_t batch, int64_t row0,
                             int64_t col0, int64_t rows, int64_t cols, double* out, int64_t ld,
                             hipStream_t s);

// reduce.hip -- deterministic sums
hipError_t launch_sumsq_dense(const double* a, int64_t m, int64_t n, int64_t lda, double* scratch,
                              double* out, hipStream_t s);
hipError_t launch_sumsq_vec(const double* x, int64_t len, double* scratch, double* out,
                            hipStream_t s);
hipError_t launch_sum_partials(const double* partial, int64_t groups, int64_t stride, int64_t count,
                               double* out, hipStream_t s);
hipError_t launch_sum_vector(const double* partial, int64_t count, double* out, hipStream_t s);
// Partial sums the ||A||^2 launchers write into their scratch (dense, bfloat16, e4m3, vector).
int64_t sumsq_partials();

// gemm.hip -- FP64 MFMA GEMM.  out(i,j) = alpha sum_k Aop(i,k) Bop(k,j) + beta C0(i,j)
struct GemmDesc {
    int64_t M, N, K;
    View A, B;           // Aop(i,k) = A.p[i*A.si + k*A.sj];  Bop(k,j) = B.p[k*B.si + j*B.sj]
    double alpha, beta;
    View C0;
    MutView C;
    double* colsq;       // optional [groups][N] partial column sums of squares of the output,
                         // groups <= ceil(M / 64); fused into the epilogue without split-K
    int* colsq_groups;   // receives the number of partial groups when colsq is set
    double* ws;          // split-K scratch (nullptr: no split)
    int64_t ws_elems;
    int max_split;       // 0 = automatic
    const int* gate;     // device flag: the product is skipped if it is nonzero at launch time
};
hipError_t gemm_f64(const GemmDesc& d, hipStream_t s);
// Fixed-order sum of nsplit partials d.ws[split][M][N] into d.C with the alpha / beta epilogue.
hipError_t launch_splitk_reduce(const GemmDesc& d, int nsplit, hipStream_t s);

// tsgemm.hip -- narrow products (N <= 64) with MFMA operands loaded from global memory.
// Panel form: A column-major (d.A.si == 1); reduction form: A with k contiguous (d.A.sj == 1)
// and B contiguous in k or j.  fm: 16-row blocks per output tile; waves: workgroup waves
// sharing the reduction; nsplit: reduction splits over workgroups (partials in d.ws).
// hipErrorNotSupported when the operands do not fit the form.
bool ts_panel_fits(const GemmDesc& d);
bool ts_red_fits(const GemmDesc& d);
hipError_t ts_panel(const GemmDesc& d, int fm, int waves, int nsplit, hipStream_t s);
hipError_t ts_red(const GemmDesc& d, int fm, int waves, int nsplit, hipStream_t s);
// Panel form through per-wave LDS DMA rings of `depth` steps (full row tiles; B row-major).
bool ts_panel_dma_fits(const GemmDesc& d);
hipError_t ts_panel_dma(const GemmDesc& d, int fm, int waves, int depth, int nsplit, hipStream_t s, int nt = 0);

// Largest number of row groups of the column sums of squares gemm_f64 writes for an M x N
// output (colsq): one per output tile row (the tile height depends on K as well).
int64_t gemm_f64_colsq_groups(int64_t M, int64_t N);

// lowp.hip -- the low-precision (bfloat16 / e4m3-stored) form of the sketch sweep
hipError_t launch_quant_transpose_omega(double* om, int64_t n, int64_t w, uint16_t* omT,
                                        int64_t ldt, hipStream_t s);
// The e4m3 form's Omega: omT8 (w x n bytes, ld ldt8) = e4m3(2^5 Omega)^T, omT (w x n bfloat16,
// ld ldt) the same values / 2^5, om replaced by those values (binary64).
hipError_t launch_quant_transpose_omega_e4m3(double* om, int64_t n, int64_t w, uint16_t* omT, int64_t ldt,
                                             uint8_t* omT8, int64_t ldt8, hipStream_t s);
// G = A_q Omega_q of the e4m3 form on 8-bit matrix cores (A: e4m3 bytes M x K with row
// exponents, W: e4m3(2^5 Omega)^T, N x K bytes): the G epilogue of gemm_bf16.  gemm_f8_fits
// tells whether the shape and alignment suit it (K a multiple of 64, 16-byte rows); *groups
// receives the row groups written to colsq.
bool gemm_f8_fits(int64_t K, const void* A, int64_t lda, const void* W, int64_t ldw);
hipError_t gemm_f8(int64_t M, int64_t N, int64_t K, const uint8_t* A, int64_t lda, const int32_t* row_exp,
                   const uint8_t* W, int64_t ldw, double* out, int64_t ldo, uint16_t* outT, int64_t ldt,
                   double* colsq, int64_t* groups, hipStream_t s);
hipError_t launch_sumsq_bf16(const uint16_t* a, int64_t m, int64_t n, int64_t lda,
                             double* scratch, double* out, hipStream_t s);
hipError_t launch_sumsq_fp8(const uint8_t* a, const int32_t* row_exp, int64_t m, int64_t n,
                            int64_t lda, double* scratch, double* out, hipStream_t s);
// out(i, j) = sum_k A(i, k) B(j, k) on bfloat16 matrix cores with binary32 accumulation.
// B is N x K bfloat16 with K contiguous (row stride ldb).  A is bfloat16, or e4m3 bytes
// (a_fp8) widened to bfloat16 on load.  a_km == false: A is M x K with K contiguous (row
// stride lda), and outT must be set (the G epilogue): out = bf16(sums) as binary64 (for
// an e4m3 A: bf16(2^row_exp[i] sums)), outT (N x M, ld ldt) the same bfloat16 values (for
// an e4m3 A: times 2^row_exp[i] once more), colsq (if set) [bf16_gemm_row_groups(M, N)][N]
// partial column sums of squares of out.  a_km == true: A(i, k) = A[k * lda + i] and
// outT must be nullptr: out = the binary32 sums as binary64.
int64_t bf16_gemm_row_groups(int64_t M, int64_t N);
hipError_t gemm_bf16(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, bool a_km,
                     bool a_fp8, const int32_t* row_exp, const uint16_t* B, int64_t ldb, double* out,
                     int64_t ldo, uint16_t* outT, int64_t ldt, double* colsq, hipStream_t s);

// panel.hip -- small dense kernels of the block loop
hipError_t launch_chol_inv(const double* gram, int b, double tau, double* R, double* Rinv,
                           int* flag, hipStream_t s);
hipError_t launch_tri_inv(const double* R, int b, double* Rinv, hipStream_t s);
hipError_t launch_upper_mul2(const double* A1, const double* B1, const double* A2, const double* B2,
                             int b, double* Out1, double* Out2, hipStream_t s);
hipError_t launch_householder(double* X, int64_t m, int b, int64_t ldx, double* Q, int64_t ldq,
                              double* R, double* tau, hipStream_t s);
hipError_t launch_gather_info(const double* rowsq, const double* R, const double* gcol, int b,
                              const int* flag, double* info, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);

// The stopping state of a randQB call, kept on the device so that blocks can be enqueued
// ahead of the host's decision (the indicator of Theorem 1 decremented row by row, Section
// 3.1, with the exhaustion guard).  skip = stop || halt gates the block products.
struct ScanState {
    double E;            // running indicator ||A||^2 - ||B||^2
    int64_t k;           // rows accepted so far (the rank)
    int stop;            // E fell below eps^2, or the guard fired
    int exhausted;       // the guard fired
    int halt;            // a CholeskyQR breakdown in the block that would start at row k
    int skip;            // stop || halt
    int blocks;          // blocks scanned
    int pad;
    int64_t rk[8];       // k and E after block i at [i mod 8] (the host reads the last few
    double re[8];        // with the state itself, in one copy)
};
// st = {E = *normA2, k = 0, rest 0}
hipError_t launch_scan_init(const double* normA2, ScanState* st, hipStream_t s);
// halt = skip = 0 and flags[0:8] = 0 (before a block is redone)
hipError_t launch_scan_resume(ScanState* st, int* flags, hipStream_t s);
// One block: if st is not stopped or halted and st->k == k_expect, a breakdown flag sets
// halt; otherwise rows j = 0..bw-1 are taken while R_i(j,j) > exh_rel sqrt(g2[j]), each
// lowering E by rowsq[j], stopping at the first E < eps2 (row_by_row) or after the block
// (whole-block rule).  Records (k, E) after the block in khist / ehist[blocks].
hipError_t launch_scan_block(const double* rowsq, const double* Ri, const double* g2, int bw, double eps2,
                             int row_by_row, double exh_rel, const int* flags, ScanState* st,
                             int64_t* khist, double* ehist, int64_t k_expect, hipStream_t s);
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t s);

// spmm.hip -- CSR products and the CSR(A^T) build
hipError_t launch_spmm_csr(const int64_t* rowptr, const int32_t* colind, const double* val,
                           int64_t m, const double* X, int64_t ldx, double* G, int64_t ldg,
                           int64_t w, hipStream_t s);
// Load-balanced CSR product through a segment plan (rows split into segments of at most
// 512 nonzeros, long rows reduced in segment order); built once per matrix per call.
struct SpmmPlan {
    int64_t rows, smax, wmax;
    int64_t nnz;
    int64_t* seg_off;    // rows + 1: exclusive prefix of segments per row (last = total)
    int64_t* mseg_off;   // rows + 1: exclusive prefix of the segments of multi-segment rows
    int32_t* seg_row;    // smax: row of each segment
    double* P;           // partial rows of multi-segment rows, wmax columns each
};
size_t spmm_plan_bytes(int64_t rows, int64_t nnz, int64_t wmax);
hipError_t spmm_plan_build(const int64_t* rowptr, int64_t rows, int64_t nnz, int64_t wmax, char* ws,
                           hipStream_t s, SpmmPlan* plan);
hipError_t launch_spmm_plan(const SpmmPlan& plan, const int64_t* rowptr, const int32_t* colind,
                            const double* val, const double* X, int64_t ldx, double* G, int64_t ldg,
                            int64_t w, hipStream_t s);
int64_t colsq_groups(int64_t rows);
hipError_t launch_colsq_rowmajor(const double* Y, int64_t rows, int64_t w, int64_t ld,
                                 double* partial, hipStream_t s);
struct CscLayout {
    size_t colptr, t_col, t_val, keys_in, keys_out, perm_in, perm_out, rowidx, temp, temp_bytes,
        total;
};
CscLayout csc_layout(int64_t m, int64_t n, int64_t nnz);
hipError_t build_csc(const int64_t* rowptr, const int32_t* colind, const double* val, int64_t m,
                     int64_t n, int64_t nnz, char* ws, hipStream_t s);
void csc_views(int64_t m, int64_t n, int64_t nnz, char* ws, const int64_t** colptr,
               const int32_t** t_col, const double** t_val);

// coo.hip -- COO (any order, duplicates summed) to CSR on the device
size_t coo_bytes(int64_t m, int64_t n, int64_t nnz);
hipError_t coo_to_csr(const int32_t* row, const int32_t* col, const double* val, int64_t m, int64_t n,
                      int64_t nnz, char* ws, int64_t* rowptr, int32_t* colind, double* out_val,
                      hipStream_t s);
void coo_counts(int64_t m, int64_t n, int64_t nnz, char* ws, const int64_t** nruns, const int** bad);

// qrcp.hip -- trQRCP: pivoted QR of the transposed sketch (n x l), gathers of pivot columns
int qrcp_max_rows();
hipError_t launch_qrcp_norms(const double* St, int64_t n, int l, const int* active, double* norm2,
                             hipStream_t s);
// One pivot step, one launch (l <= qrcp_max_rows()).  betas[t] receives the pivot's diagonal
// entry of the sketch's triangular factor; cv / ci hold 2 x qrcp_cand_slots(n) per-workgroup
// best columns (alternating between steps; launch_qrcp_cands fills them before a block's
// first step, after the norms).
hipError_t launch_qrcp_step(double* St, int64_t n, int l, int t, double* norm2, int* active, int* piv,
                            const double* colA, double* g2, double* betas, double* cv, int* ci, hipStream_t s);
int64_t qrcp_cand_slots(int64_t n);
hipError_t launch_qrcp_cands(const double* norm2, int64_t n, double* cv, int* ci, hipStream_t s);
hipError_t launch_qrcp_rs(const double* St, int l, const int* piv, const double* betas, int bw, double* Rs,
                          hipStream_t s);
hipError_t launch_gather_cols(const double* X, int64_t ldx, int64_t rows, const int* piv, int bw,
                              double* Y, int64_t ldy, hipStream_t s);

// svd.hip -- block one-sided Jacobi SVD of a k x k factor (circle ordering over blocks of
// 32 columns) and its outputs.  Round -1 of a sweep turns every column pair of neighbouring
// blocks 2p, 2p+1; rounds 0 .. jacobi_rounds(k)-1 turn the pairs across two blocks.
int jacobi_rounds(int k);
size_t jacobi_part_elems(int k);
size_t jacobi_rot_elems(int k);
hipError_t launch_jacobi_block_round(double* X, double* W, int k, int64_t ld, int round, double tol_r,
                                     double tol_c, int inner, double* part, double* V, int* skip,
                                     int* flag, hipStream_t s);
hipError_t launch_svd_finish(const double* X, const double* W, int k, int64_t ld, double* sig,
                             int* pos, double* s_out, double* Ut, double* Ws, hipStream_t s);
hipError_t launch_sign_rule(double* V, int64_t n, int64_t ldv, double* Ut, int k, int64_t ldu,
                            hipStream_t s);
hipError_t launch_identity(double* W, int k, int64_t ld, hipStream_t s);

}  // namespace qb
