// Host orchestration and C ABI of the QB library.
//
// randQB_FP (Algorithm 4 with P = 0: the re-orthogonalised blocks and eq. (23)) and randQB_EI
// (Algorithm 2), both with the row-by-row error indicator of Section 3.1.  Every
// arithmetic step runs in the HIP kernels of this library; the host only carves the
// caller's workspace, enqueues kernels on the caller's stream, and after each block
// copies b row norms (plus diag(R_i) and ||A Omega_i(:,j)||^2 for the exhaustion guard)
// to decide the rank.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "kernels.h"

namespace qb {

namespace {

constexpr int kMaxB = 128;
constexpr double kExhaustRel = 0x1p-40;     // R_i(j,j) <= 2^-40 ||A Omega(:,j)|| ends the run
constexpr double kCholTau = 1e-12;          // CholeskyQR pivot floor relative to max diag
constexpr double kUnitRoundoff = 0x1p-53;
constexpr int64_t kGramSplitElems = 1 << 22;
constexpr int kMaxPower = 16;               // largest power-scheme parameter P accepted
constexpr int kPowerBlock = 128;            // column block of the power-scheme orth()
constexpr int kLookahead = 4;               // blocks enqueued ahead of the stopping decision
static_assert(kLookahead <= 8, "the scan state keeps the (k, E) of its last 8 blocks");
constexpr int kMaxOversample = 128;         // trQRCP sketch rows beyond b
constexpr uint32_t kSketchStream = 1;       // generator stream of trQRCP's sketch (randQB: 0)

#define QB_HIP(expr)                                  \
    do {                                              \
        const hipError_t qb_e_ = (expr);              \
        if (qb_e_ != hipSuccess) return QB_ERR_HIP;   \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// --------------------------------------------------------------------------- workspace

struct Layout {
    size_t red, scal, om, g, h, gpart, gnorm2, y, x2, s, w, z, d, gram, r1, r1i, rt, rti, ri, rii, tau,
        rowsq_part, rowsq, info, flags, split, csc, plan_a, plan_t, omt, gqt, total;
    size_t split2;          // split-K partials of the products issued on the side stream
    size_t scan, khist, ehist;   // device stopping state and the (k, E) after each block
    size_t ynext, w2;            // randQB_FP look-ahead: the next block's partial Y, second W buffer
    bool ahead;                  // look-ahead regions present
    int64_t nhist;
    // trQRCP: sketch St (n x l), its Gaussian (m x l), ||A(:, j)||^2 and its partials, the
    // remaining sketch norms, active flags, block pivots, their ||A(:, p)||^2, R~_11 and
    // R~_11 R_i^{-1}
    size_t sk, skom, cola, colpart, qn, act, bpiv, g2p, rs, mm;
    size_t qcv, qci, beta;   // per-workgroup best columns of the one-launch pivot steps, diag(R~)
    int64_t lt, split_elems, split2_elems, gpart_groups;
    int64_t ldm16, ldn16;   // row strides (elements) of the bfloat16 copies: m, n rounded to 8
    size_t omt8;            // e4m3 form: e4m3(2^5 Omega)^T bytes (l~ x ldn8)
    int64_t ldn8;           // its row stride: n rounded to 16
};

// Largest chunk of Omega columns: l_tilde, or the paper's min(50 b, l_max) for 0 and for
// the adaptive schedule (-1).
int64_t chunk_width(const qb_params* p) {
    int64_t lt = p->l_tilde <= 0 ? 50 * static_cast<int64_t>(p->b) : p->l_tilde;
    return lt < p->l_max ? lt : p->l_max;
}

int64_t round_up(int64_t x, int64_t b) { return ((x + b - 1) / b) * b; }

// Width of the next chunk of Omega columns starting at column k.  Fixed schedules use the
// full width.  The adaptive schedule starts with 8 b columns; after a chunk of w_prev
// columns whose last span columns took the indicator from e_prev to e_now (span covers the
// chunk's second half: from the end of block floor(nb / 2) of its nb blocks), it assumes
// that per-column geometric decay and asks for 1.1 x the columns that would reach eps^2
// plus one block, rounded up to a multiple of b and kept within [b, 4 w_prev] (never above
// the fixed width).
int64_t next_chunk(const qb_params* p, int64_t cap, int64_t k, int64_t w_prev, int64_t span,
                   double e_prev, double e_now, double eps2) {
    const int64_t b = p->b;
    const int64_t left = p->l_max - k;
    int64_t w;
    if (p->l_tilde != -1) {
        w = cap;
    } else if (w_prev == 0) {
        w = 8 * b;
    } else if (span > 0 && e_now > 0.0 && e_prev > e_now && eps2 > 0.0 && eps2 < e_now) {
        const double rate = log(e_now / e_prev) / static_cast<double>(span);      // < 0
        const double need = log(eps2 / e_now) / rate;                               // > 0
        const double want = 1.1 * need + static_cast<double>(b);
        const double hi = 4.0 * static_cast<double>(w_prev);
        w = want >= hi ? 4 * w_prev : round_up(static_cast<int64_t>(ceil(want)), b);
        if (w < b) w = b;
    } else {
        w = 2 * w_prev;
    }
    if (w > cap) w = cap;
    return w < left ? w : left;
}

// split_cap >= 0 selects the allocation-free sizing: no partials for a side stream, and at most
// split_cap elements of split-K partials (the products then take fewer K splits).
Layout make_layout(int algo, int sparse, int dtype, int64_t m, int64_t n, int64_t nnz,
                   const qb_params* p, int64_t ell = 0, int64_t split_cap = -1) {
    Layout L{};
    const bool lowp = dtype == QB_BF16 || dtype == QB_FP8E4M3;
    const int64_t b = p->b;
    const int64_t lmax = p->l_max;
    const int64_t lt = algo == QB_ALGO_FP ? chunk_width(p) : b;   // EI: one block at a time
    L.lt = lt;
    // split-K partials: small Gram / projection products and tall-skinny (m or n) x b
    // products with a few K splits
    L.split_elems = 512 * b * (b > 64 ? b : 64) + 65536;
    if (L.split_elems < kGramSplitElems) L.split_elems = kGramSplitElems;
    if (L.split_elems < 8 * (m > n ? m : n) * b) L.split_elems = 8 * (m > n ? m : n) * b;
    // A^T Q_i (n x b, K = m): room for the split that gives the 128-row tall-skinny tiles
    // about 2048 workgroups, 2048 * 128 * b partials whatever n is
    if (L.split_elems < int64_t(2048) * 128 * b) L.split_elems = int64_t(2048) * 128 * b;
    // randQB_FP overlaps D = Q^T Y + W and S = H_J - B^T D with the panel QR on a second
    // stream: those products get their own partials buffer
    L.split2_elems = algo == QB_ALGO_FP ? L.split_elems : 0;
    // dense randQB_FP: room for two K splits of the widest sketch GEMM (G, m x l~)
    if (algo == QB_ALGO_FP && !sparse && !lowp && L.split_elems < 2 * (m > n ? m : n) * lt)
        L.split_elems = 2 * (m > n ? m : n) * lt;
    if (split_cap >= 0) {
        if (L.split_elems > split_cap) L.split_elems = split_cap;
        L.split2_elems = 0;
    }
    // row-tile partials of the G column norms: dense GEMM tiles are >= 64 rows
    L.gpart_groups = sparse ? colsq_groups(m) : std::max<int64_t>(cdiv(m, 64), colsq_groups(m));
    // per-block row sums of squares of B_i: partials from a GEMM epilogue over n rows
    // (tiles of >= 64 rows) or from the column reduction (CSR EI)
    int64_t nb_part = cdiv(n, 64);
    if (colsq_groups(n) > nb_part) nb_part = colsq_groups(n);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.red = take(sizeof(double) * 1024);
    L.scal = take(sizeof(double) * 8);
    L.om = take(sizeof(double) * n * lt);
    L.g = take(sizeof(double) * m * lt);
    L.h = algo == QB_ALGO_FP ? take(sizeof(double) * n * lt) : take(0);
    L.gpart = take(sizeof(double) * L.gpart_groups * lt);
    L.gnorm2 = take(sizeof(double) * lt);
    // panels of b columns of m rows; the power scheme's orth() also takes n-row panels
    // (Omega = orth(A^T G)) in blocks of kPowerBlock columns
    const bool pw = p->power > 0;
    const int64_t prow = pw && n > m ? n : m;
    const int64_t pb = pw && b < kPowerBlock ? kPowerBlock : b;   // widest panel block
    L.y = take(sizeof(double) * prow * pb);
    L.x2 = take(sizeof(double) * prow * pb);
    L.s = take(sizeof(double) * b * n);
    L.w = take(sizeof(double) * lmax * b);
    L.z = take(sizeof(double) * lmax * pb);
    L.d = take(sizeof(double) * lmax * b);
    L.gram = take(sizeof(double) * pb * pb);
    L.r1 = take(sizeof(double) * pb * pb);
    L.r1i = take(sizeof(double) * pb * pb);
    L.rt = take(sizeof(double) * pb * pb);
    L.rti = take(sizeof(double) * pb * pb);
    L.ri = take(sizeof(double) * b * b);
    L.rii = take(sizeof(double) * b * b);
    L.tau = take(sizeof(double) * pb);
    L.rowsq_part = take(sizeof(double) * nb_part * b);
    L.rowsq = take(sizeof(double) * b);
    L.info = take(sizeof(double) * (3 * b + 1));
    L.flags = take(sizeof(int) * 8);
    // blocks of a call: at most one per b rows plus one short block per chunk
    L.nhist = 2 * cdiv(lmax, b) + 8;
    L.scan = take(sizeof(ScanState));
    L.khist = take(sizeof(int64_t) * L.nhist);
    L.ehist = take(sizeof(double) * L.nhist);
    L.split = take(sizeof(double) * L.split_elems);
    L.split2 = take(sizeof(double) * L.split2_elems);
    // randQB_FP look-ahead (only with a side stream, so not in the allocation-free sizing):
    // the next block's G_J' - Q W' over the columns of Q known before this block ends, and a
    // second W buffer for that block's W'
    L.ahead = algo == QB_ALGO_FP && split_cap < 0;
    L.ynext = take(L.ahead ? sizeof(double) * m * b : 0);
    L.w2 = take(L.ahead ? sizeof(double) * lmax * b : 0);
    L.csc = sparse ? take(csc_layout(m, n, nnz).total) : take(0);
    // segment plans of CSR(A) and CSR(A^T) for the balanced SpMM (widest product: l~ or b)
    L.plan_a = sparse ? take(spmm_plan_bytes(m, nnz, lt)) : take(0);
    L.plan_t = sparse ? take(spmm_plan_bytes(n, nnz, lt)) : take(0);
    // bfloat16 form: Omega_q^T (l~ x n) and G_q^T (l~ x m), rows padded to multiples of 8
    // elements so that every row starts 16-byte aligned
    L.ldm16 = round_up(m, 8);
    L.ldn16 = round_up(n, 8);
    L.omt = lowp ? take(sizeof(uint16_t) * lt * L.ldn16) : take(0);
    L.gqt = lowp ? take(sizeof(uint16_t) * lt * L.ldm16) : take(0);
    L.ldn8 = round_up(n, 16);
    L.omt8 = dtype == QB_FP8E4M3 ? take(lt * L.ldn8) : take(0);
    if (ell > 0) {
        L.sk = take(sizeof(double) * n * ell);
        L.skom = take(sizeof(double) * m * ell);
        L.cola = take(sizeof(double) * n);
        L.colpart = take(sizeof(double) * colsq_groups(m) * n);
        L.qn = take(sizeof(double) * n);
        L.act = take(sizeof(int) * n);
        L.bpiv = take(sizeof(int) * b);
        L.g2p = take(sizeof(double) * b);
        L.rs = take(sizeof(double) * b * b);
        L.mm = take(sizeof(double) * b * b);
        L.qcv = take(sizeof(double) * 2 * qrcp_cand_slots(n));
        L.qci = take(sizeof(int) * 2 * qrcp_cand_slots(n));
        L.beta = take(sizeof(double) * b);
    }
    L.total = off + 256;
    return L;
}

// --------------------------------------------------------------------------- operator

// The matrix A as seen by the algorithm: products with A and A^T, and ||A||^2.
struct Op {
    int64_t m, n;
    bool sparse;
    int dtype;
    const double* a;
    const uint16_t* aq;   // bfloat16 A (dtype QB_BF16)
    const uint8_t* a8;    // e4m3 A (dtype QB_FP8E4M3) and its row exponents
    const int32_t* row_exp;
    int64_t lda;
    const int64_t* rowptr;
    const int32_t* colind;
    const double* val;
    int64_t nnz;
    const int64_t* t_ptr;
    const int32_t* t_col;
    const double* t_val;
    SpmmPlan plan_a, plan_t;   // segment plans of CSR(A) and CSR(A^T)
};

// Streams and events that a host thread keeps per device across calls: the side stream of
// the randQB_FP block loop with its two ordering events, and a pool of timing events.  They
// are created on the thread's first call on that device and kept until the process ends,
// so a call creates no stream or event once the pool has grown to the call's phase count.
struct DevRes {
    hipStream_t side = nullptr;
    hipEvent_t ev_y = nullptr, ev_s = nullptr, ev_pre = nullptr;
    std::vector<hipEvent_t> pool;
};

constexpr int kMaxDevices = 64;

DevRes* dev_res() {
    thread_local DevRes* res[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    if (res[dev] == nullptr) {
        DevRes* r = new DevRes();
        // non-blocking, so that only the explicit events order it against the caller's
        // stream (which may be the legacy default stream); default priority.  If it cannot
        // be made, the products run on the caller's stream.
        if (hipStreamCreateWithFlags(&r->side, hipStreamNonBlocking) != hipSuccess) r->side = nullptr;
        if (r->side != nullptr && (hipEventCreateWithFlags(&r->ev_y, hipEventDisableTiming) != hipSuccess ||
                                   hipEventCreateWithFlags(&r->ev_s, hipEventDisableTiming) != hipSuccess ||
                                   hipEventCreateWithFlags(&r->ev_pre, hipEventDisableTiming) != hipSuccess)) {
            if (r->ev_y) (void)hipEventDestroy(r->ev_y);
            if (r->ev_s) (void)hipEventDestroy(r->ev_s);
            (void)hipStreamDestroy(r->side);
            r->side = nullptr;
            r->ev_y = r->ev_s = r->ev_pre = nullptr;
        }
        (void)hipGetLastError();
        res[dev] = r;
    }
    return res[dev];
}

// Phase timer: events recorded on the caller's stream at phase boundaries, taken from the
// thread's pool (pool == nullptr: timing off, every mark is a no-op).
struct Timer {
    hipStream_t s;
    std::vector<hipEvent_t>* pool;
    size_t used = 0;
    std::vector<int> phase;
    bool ok = true;
    Timer(hipStream_t st, std::vector<hipEvent_t>* p) : s(st), pool(p) {}
    void mark(int ph) {   // start of phase ph (-1 = end of the previous phase)
        if (pool == nullptr) return;
        if (used == pool->size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { ok = false; return; }
            pool->push_back(e);
        }
        if (hipEventRecord((*pool)[used], s) != hipSuccess) ok = false;
        phase.push_back(ph);
        ++used;
    }
    // accumulate the time between consecutive marks into the phase of the earlier mark
    void collect(double* ms) {
        if (pool == nullptr) return;
        for (size_t i = 0; i + 1 < used; ++i) {
            float t = 0.f;
            if (phase[i] >= 0 && hipEventElapsedTime(&t, (*pool)[i], (*pool)[i + 1]) == hipSuccess)
                ms[phase[i]] += t;
        }
        if (used >= 2) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, (*pool)[0], (*pool)[used - 1]) == hipSuccess) ms[5] = t;
        }
    }
};

struct Ctx {
    Op A;
    const qb_params* p;
    double* Q;
    int64_t ldq;
    double* B;
    int64_t ldb;
    char* ws;
    Layout L;
    hipStream_t s;
    qb_info* info;
    Timer* tm;
    double* host_info;   // 3 b doubles + flags
    hipStream_t side = nullptr;   // randQB_FP: stream of the D, S products (or none)
    hipEvent_t ev_y = nullptr, ev_s = nullptr;
    const int* gate = nullptr;    // device flag that skips the block products (stopped call)
    hipEvent_t ev_pre = nullptr;  // randQB_FP look-ahead done on the side stream
    template <class T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

GemmDesc gdesc(int64_t M, int64_t N, int64_t K, View a, View b, double alpha, double beta, View c0,
               MutView c, const Ctx& x) {
    GemmDesc d{};
    d.M = M; d.N = N; d.K = K; d.A = a; d.B = b; d.alpha = alpha; d.beta = beta; d.C0 = c0; d.C = c;
    d.colsq = nullptr; d.colsq_groups = nullptr;
    d.ws = x.at<double>(x.L.split); d.ws_elems = x.L.split_elems; d.max_split = 0;
    d.gate = x.gate;
    return d;
}

// G(:, 0:w) = A X (X: n x w row-major, ld ldx); also the column sums of squares of G
// into gnorm2[0:w].  ldg is G's row stride.
int apply_A(const Ctx& x, const double* X, int64_t ldx, double* G, int64_t ldg, int64_t w,
            double* gnorm2) {
    const Op& A = x.A;
    double* gpart = x.at<double>(x.L.gpart);
    int groups = 0;
    if (!A.sparse) {
        GemmDesc d = gdesc(A.m, w, A.n, View{A.a, A.lda, 1}, View{X, ldx, 1}, 1.0, 0.0,
                           View{nullptr, 0, 0}, MutView{G, ldg, 1}, x);
        if (w <= 64 && A.m >= 4096) {
            // a block of randQB_EI: the product on the narrow reduction-form kernel, the
            // column norms in a pass of their own over the m x w result
            QB_HIP(gemm_f64(d, x.s));
            QB_HIP(launch_colsq_rowmajor(G, A.m, w, ldg, gpart, x.s));
            groups = static_cast<int>(colsq_groups(A.m));
        } else {
            d.colsq = gpart;
            d.colsq_groups = &groups;
            QB_HIP(gemm_f64(d, x.s));
        }
    } else {
        QB_HIP(launch_spmm_plan(A.plan_a, A.rowptr, A.colind, A.val, X, ldx, G, ldg, w, x.s));
        QB_HIP(launch_colsq_rowmajor(G, A.m, w, ldg, gpart, x.s));
        groups = static_cast<int>(colsq_groups(A.m));
    }
    QB_HIP(launch_sum_partials(gpart, groups, w, w, gnorm2, x.s));
    return QB_OK;
}

// H(:, 0:w) = A^T G (G: m x w row-major, ld ldg) into H (n x w row-major, ld ldh).
int apply_At(const Ctx& x, const double* G, int64_t ldg, double* H, int64_t ldh, int64_t w) {
    const Op& A = x.A;
    if (!A.sparse) {
        GemmDesc d = gdesc(A.n, w, A.m, View{A.a, 1, A.lda}, View{G, ldg, 1}, 1.0, 0.0,
                           View{nullptr, 0, 0}, MutView{H, ldh, 1}, x);
        QB_HIP(gemm_f64(d, x.s));
    } else {
        QB_HIP(launch_spmm_plan(A.plan_t, A.t_ptr, A.t_col, A.t_val, G, ldg, H, ldh, w, x.s));
    }
    return QB_OK;
}

// The low-precision sketch of a chunk: Omega (n x w, ld w, binary64 on entry) is replaced
// by its rounding Omega_q -- bfloat16, or for e4m3-stored A the e4m3 rounding of 2^5 Omega
// divided by 2^5 -- (and copied transposed in bfloat16, and in e4m3 bytes), G = bf16(A_q
// Omega_q) with its column sums of squares (on 8-bit matrix cores for e4m3 A when the shape
// allows, else on bfloat16 ones: the products are exact either way), H = A_q^T G_q reading
// A_q in place (bfloat16, or e4m3 with power-of-two row scales).
int sketch_bf16(const Ctx& x, double* Om, double* G, double* H, int64_t w, double* gnorm2,
                bool time_phases) {
    const Op& A = x.A;
    uint16_t* omt = x.at<uint16_t>(x.L.omt);
    uint16_t* gqt = x.at<uint16_t>(x.L.gqt);
    double* gpart = x.at<double>(x.L.gpart);
    const bool f8 = A.dtype == QB_FP8E4M3;
    uint8_t* omt8 = f8 ? x.at<uint8_t>(x.L.omt8) : nullptr;
    if (f8)
        QB_HIP(launch_quant_transpose_omega_e4m3(Om, A.n, w, omt, x.L.ldn16, omt8, x.L.ldn8, x.s));
    else
        QB_HIP(launch_quant_transpose_omega(Om, A.n, w, omt, x.L.ldn16, x.s));
    if (time_phases) x.tm->mark(2);
    const void* a = f8 ? static_cast<const void*>(A.a8) : static_cast<const void*>(A.aq);
    int64_t groups = bf16_gemm_row_groups(A.m, w);
    if (f8 && gemm_f8_fits(A.n, A.a8, A.lda, omt8, x.L.ldn8)) {
        QB_HIP(gemm_f8(A.m, w, A.n, A.a8, A.lda, A.row_exp, omt8, x.L.ldn8, G, w, gqt, x.L.ldm16, gpart, &groups,
                       x.s));
    } else {
        QB_HIP(gemm_bf16(A.m, w, A.n, a, A.lda, false, f8, A.row_exp, omt, x.L.ldn16, G, w, gqt, x.L.ldm16,
                         gpart, x.s));
    }
    QB_HIP(launch_sum_partials(gpart, groups, w, w, gnorm2, x.s));
    if (time_phases) x.tm->mark(3);
    QB_HIP(gemm_bf16(A.n, w, A.m, a, A.lda, true, f8, nullptr, gqt, x.L.ldm16, H, w, nullptr, 0, nullptr,
                     x.s));
    return QB_OK;
}

// CholeskyQR of the m x bw column-major panel X (ld m) into Qout (column-major, ld ldq):
// gram = X^T X, R, R^{-1}, Qout = X R^{-1}.  A breakdown sets flags[0].
// General form: X is any rows x bw view, Qout any rows x bw destination (not aliasing X).
int cholqr_v(const Ctx& x, int64_t rows, View X, int bw, MutView Qout, double* R, double* Rinv) {
    double* gram = x.at<double>(x.L.gram);
    GemmDesc d = gdesc(bw, bw, rows, View{X.p, X.sj, X.si}, X, 1.0, 0.0, View{nullptr, 0, 0},
                       MutView{gram, bw, 1}, x);
    QB_HIP(gemm_f64(d, x.s));
    QB_HIP(launch_chol_inv(gram, bw, kCholTau, R, Rinv, x.at<int>(x.L.flags), x.s));
    GemmDesc q = gdesc(rows, bw, bw, X, View{Rinv, bw, 1}, 1.0, 0.0, View{nullptr, 0, 0}, Qout, x);
    QB_HIP(gemm_f64(q, x.s));
    return QB_OK;
}

int cholqr(const Ctx& x, const double* X, int bw, double* Qout, int64_t ldq, double* R,
           double* Rinv) {
    const int64_t m = x.A.m;
    return cholqr_v(x, m, View{X, 1, m}, bw, MutView{Qout, 1, ldq}, R, Rinv);
}

// A block of Algorithm 4 up to R_i (as Algorithm 2's block QR): given G_J (m x bw, row-major,
// ld ldgj) and Omega_J (n x bw, row-major, ld ldoj; nullptr when the caller has put W in
// the w buffer already, as trQRCP does with W = B(:, J)), form W = B Omega_J,
// Y = G_J - Q W (kept in the y buffer), Q_i = qr(Y), Q_i = qr(Q_i - Q (Q^T Q_i)) and
// R_i = R~ R.  use_hh selects Householder instead of CholeskyQR for both qr calls.
int fp_block_ds(const Ctx& x, int64_t k, int bw, const double* HJ, int64_t ldhj, const double* W);

// Look-ahead of the randQB_FP block loop.  Block i + 1 (columns J' of the chunk) needs
// W' = B Omega_J' and Y' = G_J' - Q W' over all k + bw rows of B and columns of Q, but the
// first k of them are known when block i starts.  So beside block i's QR, the side stream
// forms W'(0:k, :) = B(0:k, :) Omega_J' (into the W buffer block i does not use) and
// Yp = G_J' - Q(:, 0:k) W'(0:k, :) (into the ynext buffer); block i + 1 then only adds
// W'(k:k+bw, :) = B_i Omega_J' and Y' = Yp - Q_i W'(k:k+bw, :).  The sums regroup the
// same products (Y' to rounding).  Not across a chunk end (the next chunk's sketch
// replaces G and Omega), not after a block redone by Householder QR.
struct Lookahead {
    int cur = 0;            // W buffer of the current block: 0 the w region, 1 the w2 region
    int64_t k = -1;         // start of the block the precomputed parts belong to (-1: none)
    int64_t kp = 0;         // rows of W' (columns of Q) they cover
    int bw = 0;             // that block's width
    bool pending = false;   // enqueued on the side stream, ev_pre recorded after it
    int64_t k_end = 0;      // end of the current chunk
};

int orth_block(const Ctx& x, int64_t k, int bw, const double* GJ, int64_t ldgj, const double* OmJ,
               int64_t ldoj, bool use_hh, const double* HJ, int64_t ldhj, Lookahead* la = nullptr) {
    const int64_t m = x.A.m, n = x.A.n;
    double* Y = x.at<double>(x.L.y);
    double* X2 = x.at<double>(x.L.x2);
    double* W = x.at<double>(la != nullptr && la->cur == 1 ? x.L.w2 : x.L.w);
    double* Z = x.at<double>(x.L.z);
    double* Qi = x.Q + k * x.ldq;
    double* R1 = x.at<double>(x.L.r1);
    double* R1i = x.at<double>(x.L.r1i);
    double* Rt = x.at<double>(x.L.rt);
    double* Rti = x.at<double>(x.L.rti);
    double* tau = x.at<double>(x.L.tau);
    if (la != nullptr && la->pending) {   // the side stream's look-ahead writes W and ynext
        QB_HIP(hipStreamWaitEvent(x.s, x.ev_pre, 0));
        la->pending = false;
    }
    const bool use_ahead = la != nullptr && la->k == k && la->bw == bw && !use_hh && OmJ != nullptr;
    if (la != nullptr) la->k = -1;
    if (use_ahead) {
        const int64_t kp = la->kp;
        // W(kp:k, :) = B(kp:k, :) Omega_J
        GemmDesc d = gdesc(k - kp, bw, n, View{x.B + kp * x.ldb, x.ldb, 1}, View{OmJ, ldoj, 1}, 1.0, 0.0,
                           View{nullptr, 0, 0}, MutView{W + kp * bw, bw, 1}, x);
        QB_HIP(gemm_f64(d, x.s));
        // Y = Yp - Q(:, kp:k) W(kp:k, :)
        GemmDesc e = gdesc(m, bw, k - kp, View{x.Q + kp * x.ldq, 1, x.ldq}, View{W + kp * bw, bw, 1}, -1.0,
                           1.0, View{x.at<double>(x.L.ynext), 1, m}, MutView{Y, 1, m}, x);
        QB_HIP(gemm_f64(e, x.s));
    } else {
        // W = B(0:k, :) Omega_J   (k x bw, row-major ld bw)
        if (k > 0 && OmJ != nullptr) {
            GemmDesc d = gdesc(k, bw, n, View{x.B, x.ldb, 1}, View{OmJ, ldoj, 1}, 1.0, 0.0,
                               View{nullptr, 0, 0}, MutView{W, bw, 1}, x);
            QB_HIP(gemm_f64(d, x.s));
        }
        // Y = G_J - Q W   (m x bw, column-major ld m)
        GemmDesc d = gdesc(m, bw, k, View{x.Q, 1, x.ldq}, View{W, bw, 1}, -1.0, 1.0,
                           View{GJ, ldgj, 1}, MutView{Y, 1, m}, x);
        QB_HIP(gemm_f64(d, x.s));
    }
    // randQB_FP: the parts of eq. (23) that need only Y and W, beside the QR below
    if (HJ != nullptr) {
        if (int st = fp_block_ds(x, k, bw, HJ, ldhj, W)) return st;
        // then the look-ahead of the next block of the chunk on the same side stream
        const int64_t k2 = k + bw;
        if (la != nullptr && x.side != nullptr && x.L.ahead && k > 0 && k2 < la->k_end) {
            const int bw2 = static_cast<int>(x.p->b < la->k_end - k2 ? x.p->b : la->k_end - k2);
            const int nc = la->cur ^ 1;
            double* W2 = x.at<double>(nc == 1 ? x.L.w2 : x.L.w);
            GemmDesc d = gdesc(k, bw2, n, View{x.B, x.ldb, 1}, View{OmJ + bw, ldoj, 1}, 1.0, 0.0,
                               View{nullptr, 0, 0}, MutView{W2, bw2, 1}, x);
            d.ws = x.at<double>(x.L.split2);
            d.ws_elems = x.L.split2_elems;
            QB_HIP(gemm_f64(d, x.side));
            GemmDesc e = gdesc(m, bw2, k, View{x.Q, 1, x.ldq}, View{W2, bw2, 1}, -1.0, 1.0,
                               View{GJ + bw, ldgj, 1}, MutView{x.at<double>(x.L.ynext), 1, m}, x);
            e.ws = x.at<double>(x.L.split2);
            e.ws_elems = x.L.split2_elems;
            QB_HIP(gemm_f64(e, x.side));
            QB_HIP(hipEventRecord(x.ev_pre, x.side));
            la->pending = true;
            la->k = k2;
            la->kp = k;
            la->bw = bw2;
            la->cur = nc;
        }
    }
    // first qr
    if (!use_hh) {
        if (int st = cholqr(x, Y, bw, Qi, x.ldq, R1, R1i)) return st;
    } else {
        QB_HIP(hipMemcpyAsync(X2, Y, sizeof(double) * m * bw, hipMemcpyDeviceToDevice, x.s));
        QB_HIP(launch_householder(X2, m, bw, m, Qi, x.ldq, R1, tau, x.s));
    }
    // re-orthogonalisation: X2 = Q_i - Q (Q^T Q_i)
    if (k > 0) {
        GemmDesc d = gdesc(k, bw, m, View{x.Q, x.ldq, 1}, View{Qi, 1, x.ldq}, 1.0, 0.0,
                           View{nullptr, 0, 0}, MutView{Z, bw, 1}, x);
        QB_HIP(gemm_f64(d, x.s));
    }
    {
        GemmDesc d = gdesc(m, bw, k, View{x.Q, 1, x.ldq}, View{Z, bw, 1}, -1.0, 1.0,
                           View{Qi, 1, x.ldq}, MutView{X2, 1, m}, x);
        QB_HIP(gemm_f64(d, x.s));
    }
    if (!use_hh) {
        if (int st = cholqr(x, X2, bw, Qi, x.ldq, Rt, Rti)) return st;
    } else {
        QB_HIP(launch_householder(X2, m, bw, m, Qi, x.ldq, Rt, tau, x.s));
        QB_HIP(launch_tri_inv(R1, bw, R1i, x.s));
        QB_HIP(launch_tri_inv(Rt, bw, Rti, x.s));
    }
    // R_i = R~ R (Algorithm 4) and its inverse R^{-1} R~^{-1}
    QB_HIP(launch_upper_mul2(Rt, R1, R1i, Rti, bw, x.at<double>(x.L.ri), x.at<double>(x.L.rii), x.s));
    return QB_OK;
}

// Algorithm 4's B_i by eq. (23):
//   B_i = R_i^{-T} (H_J^T - (Y^T Q) B - W^T B) = R_i^{-T} (H_J^T - D^T B),  D = Q^T Y + W.
// fp_block_ds forms D and S = H_J^T - D^T B; they need only Y and W, so when the context has
// a side stream they run there, beside the panel QR of Y on the main stream (the two touch
// disjoint buffers: Q(:, 0:k), Y, W, B and H are only read, D and S only written, and the
// side products have their own split-K partials).
int fp_block_ds(const Ctx& x, int64_t k, int bw, const double* HJ, int64_t ldhj, const double* W) {
    const int64_t m = x.A.m, n = x.A.n;
    double* Y = x.at<double>(x.L.y);
    double* D = x.at<double>(x.L.d);
    double* S = x.at<double>(x.L.s);
    hipStream_t st = x.s;
    if (x.side != nullptr) {
        QB_HIP(hipEventRecord(x.ev_y, x.s));
        QB_HIP(hipStreamWaitEvent(x.side, x.ev_y, 0));
        st = x.side;
    }
    auto side_ws = [&](GemmDesc& d) {
        if (x.side != nullptr) {
            d.ws = x.at<double>(x.L.split2);
            d.ws_elems = x.L.split2_elems;
        }
    };
    if (k > 0) {   // D (k x bw) = Q^T Y + W
        GemmDesc d = gdesc(k, bw, m, View{x.Q, x.ldq, 1}, View{Y, 1, m}, 1.0, 1.0, View{W, bw, 1},
                           MutView{D, bw, 1}, x);
        side_ws(d);
        QB_HIP(gemm_f64(d, st));
    }
    {   // S^T (n x bw) = H_J - B^T D, stored as S (bw x n row-major)
        GemmDesc d = gdesc(n, bw, k, View{x.B, 1, x.ldb}, View{D, bw, 1}, -1.0, 1.0,
                           View{HJ, ldhj, 1}, MutView{S, 1, n}, x);
        side_ws(d);
        QB_HIP(gemm_f64(d, st));
    }
    if (x.side != nullptr) QB_HIP(hipEventRecord(x.ev_s, x.side));
    return QB_OK;
}

// B_i^T = S^T R_i^{-1} (the triangular solve R_i^T B_i = S), written to rows k..k+bw of B
// with the row sums of squares ||B_i(j,:)||^2 into the rowsq buffer.
int fp_block_b(const Ctx& x, int64_t k, int bw) {
    const int64_t n = x.A.n;
    double* S = x.at<double>(x.L.s);
    if (x.side != nullptr) QB_HIP(hipStreamWaitEvent(x.s, x.ev_s, 0));
    double* part = x.at<double>(x.L.rowsq_part);
    int groups = 0;
    GemmDesc d = gdesc(n, bw, bw, View{S, 1, n}, View{x.at<double>(x.L.rii), bw, 1}, 1.0, 0.0,
                       View{nullptr, 0, 0}, MutView{x.B + k * x.ldb, 1, x.ldb}, x);
    d.colsq = part;
    d.colsq_groups = &groups;
    QB_HIP(gemm_f64(d, x.s));
    QB_HIP(launch_sum_partials(part, groups, bw, bw, x.at<double>(x.L.rowsq), x.s));
    return QB_OK;
}

// Algorithm 2's B_i = Q_i^T A, computed as (A^T Q_i)^T into rows k..k+bw of B,
// with the row sums of squares into the rowsq buffer.
int ei_block_b(const Ctx& x, int64_t k, int bw) {
    const Op& A = x.A;
    double* Qi = x.Q + k * x.ldq;
    double* rowsq = x.at<double>(x.L.rowsq);
    double* part = x.at<double>(x.L.rowsq_part);
    if (!A.sparse) {
        int groups = 0;
        GemmDesc d = gdesc(A.n, bw, A.m, View{A.a, 1, A.lda}, View{Qi, 1, x.ldq}, 1.0, 0.0,
                           View{nullptr, 0, 0}, MutView{x.B + k * x.ldb, 1, x.ldb}, x);
        d.colsq = part;
        d.colsq_groups = &groups;
        QB_HIP(gemm_f64(d, x.s));
        QB_HIP(launch_sum_partials(part, groups, bw, bw, rowsq, x.s));
    } else {
        // H-style product into the S buffer (n x bw row-major), then transpose-copy via GEMM
        double* S = x.at<double>(x.L.s);
        // Q_i is column-major; make a row-major copy in X2 (m x bw) for the row-wave SpMM
        double* X2 = x.at<double>(x.L.x2);
        GemmDesc c = gdesc(A.m, bw, 0, View{nullptr, 0, 0}, View{nullptr, 0, 0}, 0.0, 1.0,
                           View{Qi, 1, x.ldq}, MutView{X2, bw, 1}, x);
        QB_HIP(gemm_f64(c, x.s));
        QB_HIP(launch_spmm_plan(A.plan_t, A.t_ptr, A.t_col, A.t_val, X2, bw, S, bw, bw, x.s));
        GemmDesc t = gdesc(A.n, bw, 0, View{nullptr, 0, 0}, View{nullptr, 0, 0}, 0.0, 1.0,
                           View{S, bw, 1}, MutView{x.B + k * x.ldb, 1, x.ldb}, x);
        QB_HIP(gemm_f64(t, x.s));
        QB_HIP(launch_colsq_rowmajor(S, A.n, bw, bw, part, x.s));
        QB_HIP(launch_sum_partials(part, colsq_groups(A.n), bw, bw, rowsq, x.s));
    }
    return QB_OK;
}

// dst = src - V (V^T src) for a rows x bw panel src and a rows x kb basis V (views of V and
// of V^T given); dst may be src itself (the update is elementwise).
int project_out(const Ctx& x, int64_t rows, int bw, View src, MutView dst, View V, View Vt,
                int64_t kb) {
    if (kb == 0) {
        if (dst.p != src.p) {
            GemmDesc c = gdesc(rows, bw, 0, View{nullptr, 0, 0}, View{nullptr, 0, 0}, 0.0, 1.0, src,
                               dst, x);
            QB_HIP(gemm_f64(c, x.s));
        }
        return QB_OK;
    }
    double* Z = x.at<double>(x.L.z);
    GemmDesc d = gdesc(kb, bw, rows, Vt, src, 1.0, 0.0, View{nullptr, 0, 0}, MutView{Z, bw, 1}, x);
    QB_HIP(gemm_f64(d, x.s));
    GemmDesc u = gdesc(rows, bw, kb, V, View{Z, bw, 1}, -1.0, 1.0, src, dst, x);
    QB_HIP(gemm_f64(u, x.s));
    return QB_OK;
}

// orth() of Algorithm 4's power scheme on the rows x w row-major panel X (ld ldx), in place:
// block Gram-Schmidt over b-column blocks (b <= kPowerBlock, the widest the CholeskyQR
// kernel takes; the callers pick b by orth_block_cols: on panels of up to 65536 rows the
// shorter Cholesky chain of 64-column blocks outweighs their narrower products, the
// 128-column one-workgroup Cholesky taking about 190 us against 55 us), each projected twice
// against Q(:, 0:kq)
// and the blocks already done, and orthonormalised after each projection by CholeskyQR
// (or, with use_hh, by Householder QR).  Block j of the result depends only on blocks
// 0..j of X and has diag(R) > 0, as the Q factor of a Householder QR of [Q, X] would.
// A CholeskyQR breakdown sets the flag; the caller then redoes the panel with use_hh.
int orth_panel(const Ctx& x, double* X, int64_t rows, int64_t w, int64_t ldx, int64_t kq,
               bool use_hh, int b = kPowerBlock) {
    double* Y = x.at<double>(x.L.y);     // rows x kPowerBlock, column-major
    double* X2 = x.at<double>(x.L.x2);   // rows x kPowerBlock, column-major
    double* tau = x.at<double>(x.L.tau);
    const View Qv{x.Q, 1, x.ldq}, Qt{x.Q, x.ldq, 1};
    const View Pv{X, ldx, 1}, Pt{X, 1, ldx};   // the finished blocks of X
    for (int64_t j0 = 0; j0 < w; j0 += b) {
        const int bw = static_cast<int>(b < w - j0 ? b : w - j0);
        const View Xj{X + j0, ldx, 1};
        const MutView Xjm{X + j0, ldx, 1};
        const View Yv{Y, 1, rows};
        const MutView Ym{Y, 1, rows};
        const View X2v{X2, 1, rows};
        const MutView X2m{X2, 1, rows};
        // first projection, in place, then qr into Y
        if (int e = project_out(x, rows, bw, Xj, Xjm, Qv, Qt, kq)) return e;
        if (int e = project_out(x, rows, bw, Xj, Xjm, Pv, Pt, j0)) return e;
        if (!use_hh) {
            if (int e = cholqr_v(x, rows, Xj, bw, Ym, x.at<double>(x.L.r1), x.at<double>(x.L.r1i)))
                return e;
        } else {
            if (int e = project_out(x, rows, bw, Xj, X2m, Pv, Pt, 0)) return e;   // copy
            QB_HIP(launch_householder(X2, rows, bw, rows, Y, rows, x.at<double>(x.L.r1), tau, x.s));
        }
        // re-orthogonalisation: X2 = Y - Q (Q^T Y) - P (P^T .), then qr into block j of X
        if (int e = project_out(x, rows, bw, Yv, X2m, Qv, Qt, kq)) return e;
        if (int e = project_out(x, rows, bw, X2v, X2m, Pv, Pt, j0)) return e;
        if (!use_hh) {
            if (int e = cholqr_v(x, rows, X2v, bw, Xjm, x.at<double>(x.L.rt), x.at<double>(x.L.rti)))
                return e;
        } else {
            QB_HIP(launch_householder(X2, rows, bw, rows, Y, rows, x.at<double>(x.L.rt), tau, x.s));
            if (int e = project_out(x, rows, bw, Yv, Xjm, Pv, Pt, 0)) return e;   // copy
        }
    }
    return QB_OK;
}

// Block width of orth_panel for panels of `rows` rows: 64 up to 65536 rows (the shorter
// Cholesky chain wins: the P = 1 call on 20000 x 15000 took 72.6 against 75.2 ms), 128
// above (the wider projections win: the P = 1 call on the 500000 x 200000 CSR matrix took
// 4.92 s with 64 against 4.55 s with 128).
int orth_block_cols(int64_t rows) { return rows <= 65536 ? 64 : kPowerBlock; }

// Whether some CholeskyQR since the last reset broke down (waits for the stream).
int read_flag(const Ctx& x, bool* broken) {
    int* hflag = reinterpret_cast<int*>(x.host_info + 3 * kMaxB);
    QB_HIP(hipMemcpyAsync(hflag, x.at<int>(x.L.flags), sizeof(int), hipMemcpyDeviceToHost, x.s));
    QB_HIP(hipStreamSynchronize(x.s));
    *broken = *hflag != 0;
    return QB_OK;
}

// The power scheme of Algorithm 4 for one chunk of w columns: P rounds of
// G = orth(A Omega) and Omega = orth(A^T G).  After the first chunk (k > 0) the rounds act
// on the residual A - Q B: G is also made orthogonal to Q(:, 0:k), and then
// (A - QB)^T G = A^T G because B = Q^T A.  Omega and H are swapped in every round (the
// new Omega is formed in the H buffer); on return Omega points at the final iterate.
int power_rounds(const Ctx& x, int64_t k, int64_t w, double*& Om, double*& H, double* G,
                 double* gnorm2) {
    const int64_t m = x.A.m, n = x.A.n;
    for (int r = 0; r < x.p->power; ++r) {
        for (int side = 0; side < 2; ++side) {
            for (int attempt = 0; attempt < 2; ++attempt) {
                const bool use_hh = attempt == 1;
                if (use_hh) {
                    QB_HIP(launch_fill_int(x.at<int>(x.L.flags), 8, 0, x.s));
                    x.info->fallbacks += 1;
                }
                if (side == 0) {   // G = orth((I - Q Q^T) A Omega)
                    if (int e = apply_A(x, Om, w, G, w, w, gnorm2)) return e;
                    if (int e = orth_panel(x, G, m, w, w, k, use_hh, orth_block_cols(m))) return e;
                } else {           // Omega = orth(A^T G)
                    if (int e = apply_At(x, G, w, H, w, w)) return e;
                    if (int e = orth_panel(x, H, n, w, w, 0, use_hh, orth_block_cols(n))) return e;
                }
                bool broken = false;
                if (int e = read_flag(x, &broken)) return e;
                if (!broken) break;
            }
        }
        double* t = Om;
        Om = H;
        H = t;
    }
    return QB_OK;
}

// Copy the per-block decision data to the host and wait.  Returns QB_OK or QB_ERR_HIP;
// *breakdown tells whether CholeskyQR failed in this block.
int fetch_block(const Ctx& x, int bw, const double* gnorm2_j, bool* breakdown) {
    double* info = x.at<double>(x.L.info);
    QB_HIP(launch_gather_info(x.at<double>(x.L.rowsq), x.at<double>(x.L.ri), gnorm2_j, bw,
                              x.at<int>(x.L.flags), info, x.s));
    QB_HIP(hipMemcpyAsync(x.host_info, info, sizeof(double) * (3 * bw + 1), hipMemcpyDeviceToHost, x.s));
    QB_HIP(hipStreamSynchronize(x.s));
    *breakdown = x.host_info[3 * bw] != 0.0;
    return QB_OK;
}

// The row-by-row stopping rule of Section 3.1 (or Algorithm 1's whole-block test) with the
// exhaustion guard.
void scan_rows(const double* hinfo, int bw, bool row_by_row, double eps2, double* E, int* keep,
               bool* stop, bool* exhausted) {
    const double* rowsq = hinfo;
    const double* rdiag = hinfo + bw;
    const double* g2 = hinfo + 2 * bw;
    *stop = false;
    *exhausted = false;
    *keep = bw;
    double Et = *E;
    for (int j = 0; j < bw; ++j) {
        if (!(rdiag[j] > kExhaustRel * sqrt(g2[j]))) {
            *keep = j;
            *stop = true;
            *exhausted = true;
            *E = Et;
            return;
        }
        Et -= rowsq[j];
        if (row_by_row && Et < eps2) {
            *keep = j + 1;
            *stop = true;
            *E = Et;
            return;
        }
    }
    *E = Et;
    if (!row_by_row && Et < eps2) *stop = true;
}

int check_params(const qb_params* p, int64_t m, int64_t n) {
    if (p == nullptr) return QB_ERR_ARG;
    if (p->power < 0 || p->power > kMaxPower) return QB_ERR_ARG;
    if (!(p->tol_rel >= 0.0) || !isfinite(p->tol_rel)) return QB_ERR_ARG;
    if (p->b < 1 || p->b > kMaxB) return QB_ERR_ARG;
    const int64_t mn = m < n ? m : n;
    if (p->l_max < 1 || p->l_max > mn) return QB_ERR_ARG;
    if (p->l_tilde < -1) return QB_ERR_ARG;
    if (p->l_tilde > 0 && p->l_tilde % p->b != 0 && p->l_tilde < p->l_max) return QB_ERR_ARG;
    if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31)) return QB_ERR_ARG;
    return QB_OK;
}

// Host buffer of the per-block read-back (pageable memory of the calling thread's stack):
// 3 b doubles of decision data and a flag word.
constexpr int kHostWords = 3 * kMaxB + 64;

// The common driver of the four entry points.  With Lfix set the call runs in the
// allocation-free mode: the workspace layout is the given one (ws_bytes is not checked
// against make_layout), and the call uses no side stream and no timing events.
int run(int algo, Op& A, const qb_params* p, double* Q, int64_t ldq, double* B, int64_t ldb,
        void* ws, size_t ws_bytes, hipStream_t s, qb_info* info, const Layout* Lfix = nullptr) {
    qb_info local{};
    qb_info* inf = info ? info : &local;
    memset(inf, 0, sizeof(*inf));
    int st = check_params(p, A.m, A.n);
    if (st != QB_OK) return inf->status = st;
    if (A.dtype != QB_F64 && (algo != QB_ALGO_FP || A.sparse)) return inf->status = QB_ERR_UNSUPPORTED;
    // the power scheme is Algorithm 4's (randQB_FP), on binary64 A
    if (p->power > 0 && (algo != QB_ALGO_FP || A.dtype != QB_F64))
        return inf->status = QB_ERR_UNSUPPORTED;
    if (Q == nullptr || B == nullptr || ws == nullptr || ldq < A.m || ldb < A.n)
        return inf->status = QB_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return inf->status = QB_ERR_ARG;
    const Layout L = Lfix != nullptr ? *Lfix : make_layout(algo, A.sparse, A.dtype, A.m, A.n, A.nnz, p);
    if (ws_bytes < L.total) return inf->status = QB_ERR_WORKSPACE;
    double host[kHostWords];
    DevRes* res = Lfix != nullptr ? nullptr : dev_res();
    Timer tm(s, res != nullptr ? &res->pool : nullptr);
    const bool side_ok = algo == QB_ALGO_FP && res != nullptr && res->side != nullptr && L.split2_elems > 0;
    const int64_t m = A.m, n = A.n, b = p->b, lmax = p->l_max;
    char* wsb = static_cast<char*>(ws);
    double* scal = reinterpret_cast<double*>(wsb + L.scal);
    double* red = reinterpret_cast<double*>(wsb + L.red);

    // ||A||_F^2 (Algorithm 4).  Dense binary64 randQB_FP without the power scheme sums
    // it on the side stream, beside the first chunk's Omega and G = A Omega on this stream
    // (the chunk's width does not depend on it), and reads it back from the side stream once
    // G is enqueued.
    tm.mark(0);
    const bool early_g = side_ok && algo == QB_ALGO_FP && !A.sparse && A.dtype == QB_F64 && p->power == 0;
    int64_t w_early = 0;
    if (early_g) {
        QB_HIP(hipEventRecord(res->ev_pre, s));
        QB_HIP(hipStreamWaitEvent(res->side, res->ev_pre, 0));
        QB_HIP(launch_sumsq_dense(A.a, m, n, A.lda, red, scal, res->side));
        w_early = next_chunk(p, L.lt, 0, 0, 0, 0.0, 0.0, 0.0);
    } else if (A.dtype == QB_BF16) {
        QB_HIP(launch_sumsq_bf16(A.aq, m, n, A.lda, red, scal, s));
    } else if (A.dtype == QB_FP8E4M3) {
        QB_HIP(launch_sumsq_fp8(A.a8, A.row_exp, m, n, A.lda, red, scal, s));
    } else if (!A.sparse) {
        QB_HIP(launch_sumsq_dense(A.a, m, n, A.lda, red, scal, s));
    } else {
        QB_HIP(launch_sumsq_vec(A.val, A.nnz, red, scal, s));
        // CSR(A^T) for the A^T products, built once; its views must be in A before the
        // context below takes its copy of the operator
        QB_HIP(build_csc(A.rowptr, A.colind, A.val, m, n, A.nnz, wsb + L.csc, s));
        csc_views(m, n, A.nnz, wsb + L.csc, &A.t_ptr, &A.t_col, &A.t_val);
        QB_HIP(spmm_plan_build(A.rowptr, m, A.nnz, L.lt, wsb + L.plan_a, s, &A.plan_a));
        QB_HIP(spmm_plan_build(A.t_ptr, n, A.nnz, L.lt, wsb + L.plan_t, s, &A.plan_t));
    }
    ScanState* scan = reinterpret_cast<ScanState*>(wsb + L.scan);
    const Ctx x{A, p, Q, ldq, B, ldb, wsb, L, s, inf, &tm, host, side_ok ? res->side : nullptr,
                side_ok ? res->ev_y : nullptr, side_ok ? res->ev_s : nullptr, &scan->skip,
                side_ok ? res->ev_pre : nullptr};
    if (early_g) {
        // the first chunk's Omega and G (ungated: the stopping state is not set up yet)
        Ctx xg = x;
        xg.gate = nullptr;
        tm.mark(1);
        QB_HIP(launch_gauss_fill(p->seed, 0, 0, 0, 0, n, w_early, x.at<double>(L.om), w_early, s));
        tm.mark(2);
        if (int e = apply_A(xg, x.at<double>(L.om), w_early, x.at<double>(L.g), w_early, w_early,
                            x.at<double>(L.gnorm2)))
            return inf->status = e;
        // the read-back to pageable memory holds the host until the sum is done; G is queued
        QB_HIP(hipMemcpyAsync(host, scal, sizeof(double), hipMemcpyDeviceToHost, res->side));
        QB_HIP(hipStreamSynchronize(res->side));
        // later work on this stream (the scan state set-up reads the sum) follows the sum
        QB_HIP(hipEventRecord(res->ev_pre, res->side));
        QB_HIP(hipStreamWaitEvent(s, res->ev_pre, 0));
    } else {
        QB_HIP(hipMemcpyAsync(host, scal, sizeof(double), hipMemcpyDeviceToHost, s));
        QB_HIP(hipStreamSynchronize(s));
    }
    const double normA2 = host[0];
    inf->normA2 = normA2;
    if (!isfinite(normA2)) {
        tm.mark(-1);
        if (early_g) QB_HIP(hipStreamSynchronize(s));
        return inf->status = QB_ERR_NONFINITE;
    }
    const double eps2 = p->tol_rel * p->tol_rel * normA2;
    const double floor_tol = sqrt(4.0 * kUnitRoundoff / 0.01);   // Theorem 3, delta = 1%
    const int status_tol = p->tol_rel < floor_tol ? QB_WARN_TOL_FLOOR : QB_OK;
    double E = normA2;
    int64_t k = 0;
    bool exhausted = false;
    int scanned = 0;
    if (!(normA2 == 0.0 || E < eps2)) {
        QB_HIP(launch_fill_int(x.at<int>(L.flags), 8, 0, s));
        QB_HIP(launch_scan_init(scal, scan, s));
        int64_t* khist = x.at<int64_t>(L.khist);
        double* ehist = x.at<double>(L.ehist);
        int64_t chunk_lo = 0, chunk_hi = 0;
        int64_t k_half = 0;       // block end where the current chunk's second half starts
        double e_half = E;        // the indicator there
        double* Om = x.at<double>(L.om);
        double* G = x.at<double>(L.g);
        double* H = x.at<double>(L.h);
        double* gnorm2 = x.at<double>(L.gnorm2);
        bool stop = false;
        bool redo_hh = false;     // the block at row k broke down in CholeskyQR: redo it by Householder
        Lookahead la;             // randQB_FP: the next block's W and Y parts formed beside this block
        double dec = 0.0;         // the indicator's drop per block over the last run of blocks
        double ratio = 0.0;       // and its ratio per block (geometric mean)
        while (k < lmax && !stop) {
            if (algo == QB_ALGO_FP && k == chunk_hi) {
                // draw the next chunk of Omega; G = A Omega, H = A^T G
                const int64_t w = next_chunk(p, L.lt, k, chunk_hi - chunk_lo, chunk_hi - k_half, e_half, E,
                                             eps2);
                chunk_lo = k;
                chunk_hi = k + w;
                la.k_end = chunk_hi;
                la.k = -1;
                k_half = chunk_lo + b * (cdiv(w, b) / 2);
                e_half = E;
                const bool g_done = early_g && chunk_lo == 0 && w == w_early;   // Omega, G enqueued
                tm.mark(g_done ? 3 : 1);
                if (!g_done) QB_HIP(launch_gauss_fill(p->seed, 0, 0, 0, chunk_lo, n, w, Om, w, s));
                if (p->power > 0) {
                    tm.mark(6);
                    if (int e = power_rounds(x, k, w, Om, H, G, gnorm2)) return inf->status = e;
                    inf->passes += 2 * p->power;
                }
                if (A.dtype == QB_BF16 || A.dtype == QB_FP8E4M3) {
                    if (int e = sketch_bf16(x, Om, G, H, w, gnorm2, true)) return inf->status = e;
                } else {
                    if (!g_done) {
                        tm.mark(2);
                        if (int e = apply_A(x, Om, w, G, w, w, gnorm2)) return inf->status = e;
                        tm.mark(3);
                    }
                    if (int e = apply_At(x, G, w, H, w, w)) return inf->status = e;
                }
                tm.mark(4);
                inf->passes += 2;
                inf->chunks += 1;
                inf->gemm_flops[0] += 2.0 * m * n * w;
                inf->gemm_flops[1] += 2.0 * m * n * w;
            }
            // Blocks are enqueued ahead of the stopping decision, which the device takes
            // (scan_block) and the host reads back once per run of blocks.  A run never
            // crosses a chunk end, and holds (at most kLookahead) as many blocks as the last
            // run's indicator says are still needed: block t of the run is needed unless the
            // indicator is below eps^2 after t blocks, predicted both with the last run's
            // drop per block (linear decay) and with its ratio per block (geometric decay,
            // the rule for a geometrically decaying spectrum, where the linear prediction
            // would allow one block per run), the larger of the two.  Few blocks run past
            // the stop; their products are skipped by the gate.
            // randQB_EI runs one block at a time: a block redone after a CholeskyQR breakdown
            // reuses its A Omega_i, which the next block's product would overwrite.
            const int64_t k_end = algo == QB_ALGO_FP ? chunk_hi : lmax;
            int nrun = 1;
            if (algo == QB_ALGO_FP && !redo_hh && dec > 0.0) {
                double t = floor((E - eps2) / dec) + 1.0;
                if (ratio > 0.0 && ratio < 1.0 && E > eps2) {
                    const double tg = floor(log(E / eps2) / log(1.0 / ratio)) + 1.0;
                    if (tg > t) t = tg;
                }
                nrun = t >= kLookahead ? kLookahead : (t >= 1.0 ? static_cast<int>(t) : 1);
            }
            int64_t ks = k;
            for (int t = 0; t < nrun && ks < k_end; ++t) {
                const int64_t bw = b < k_end - ks ? b : k_end - ks;
                const int bwi = static_cast<int>(bw);
                const double *GJ, *OmJ, *HJ = nullptr, *g2J;
                int64_t ldj;
                if (algo == QB_ALGO_FP) {
                    ldj = chunk_hi - chunk_lo;
                    const int64_t J0 = ks - chunk_lo;
                    GJ = G + J0;
                    OmJ = Om + J0;
                    HJ = H + J0;
                    g2J = gnorm2 + J0;
                } else {
                    ldj = bw;
                    if (!(t == 0 && redo_hh)) {   // a redone block keeps its A Omega_i
                        tm.mark(1);
                        QB_HIP(launch_gauss_fill(p->seed, 0, 0, 0, ks, n, bw, Om, bw, s));
                        tm.mark(2);
                        if (int e = apply_A(x, Om, bw, G, bw, bw, gnorm2)) return inf->status = e;
                        tm.mark(4);
                    }
                    GJ = G;
                    OmJ = Om;
                    g2J = gnorm2;
                }
                const bool use_hh = t == 0 && redo_hh;
                if (use_hh) QB_HIP(launch_scan_resume(scan, x.at<int>(L.flags), s));
                if (int e = orth_block(x, ks, bwi, GJ, ldj, OmJ, ldj, use_hh, algo == QB_ALGO_FP ? HJ : nullptr, ldj,
                                       algo == QB_ALGO_FP ? &la : nullptr))
                    return inf->status = e;
                if (algo == QB_ALGO_FP) {
                    if (int e = fp_block_b(x, ks, bwi)) return inf->status = e;
                } else {
                    tm.mark(3);
                    if (int e = ei_block_b(x, ks, bwi)) return inf->status = e;
                    tm.mark(4);
                }
                QB_HIP(launch_scan_block(x.at<double>(L.rowsq), x.at<double>(L.ri), g2J, bwi, eps2,
                                         p->row_by_row != 0, kExhaustRel, x.at<int>(L.flags), scan, khist, ehist,
                                         ks, s));
                ks += bw;
            }
            ScanState hs;
            QB_HIP(hipMemcpyAsync(&hs, scan, sizeof(ScanState), hipMemcpyDeviceToHost, s));
            QB_HIP(hipStreamSynchronize(s));
            if (hs.blocks > scanned) {
                // indicator drop per block over the blocks of this run
                const int first = scanned;
                dec = (E - hs.E) / static_cast<double>(hs.blocks - first);
                ratio = E > 0.0 && hs.E > 0.0 ? pow(hs.E / E, 1.0 / static_cast<double>(hs.blocks - first)) : 0.0;
                if (algo == QB_ALGO_FP && k < k_half && hs.k >= k_half) {
                    // the indicator at the end of the block that ends at k_half (a run holds
                    // at most kLookahead blocks, so the state's ring of 8 still has them)
                    for (int i = first; i < hs.blocks; ++i)
                        if (hs.rk[i & 7] == k_half) e_half = hs.re[i & 7];
                }
                scanned = hs.blocks;
            }
            k = hs.k;
            E = hs.E;
            stop = hs.stop != 0;
            exhausted = hs.exhausted != 0;
            redo_hh = hs.halt != 0;
            if (redo_hh) inf->fallbacks += 1;
        }
        // a look-ahead for a block that did not run still uses the workspace: join it
        if (la.pending) QB_HIP(hipStreamWaitEvent(s, x.ev_pre, 0));
        inf->blocks = scanned;
        if (algo == QB_ALGO_EI) {
            inf->passes = 2 * scanned;
            inf->gemm_flops[0] = inf->gemm_flops[1] = 0.0;
            for (int i = 0; i < scanned; ++i) {
                const double bwd = static_cast<double>(b < lmax - static_cast<int64_t>(i) * b ? b : lmax - i * b);
                inf->gemm_flops[0] += 2.0 * m * n * bwd;
                inf->gemm_flops[1] += 2.0 * m * n * bwd;
            }
        }
    }
    tm.mark(-1);
    QB_HIP(hipStreamSynchronize(s));
    tm.collect(inf->ms);
    inf->rank = k;
    inf->E = E;
    inf->exhausted = exhausted ? 1 : 0;
    if (normA2 == 0.0 || E < eps2)
        st = status_tol;
    else
        st = QB_NOT_CONVERGED;
    return inf->status = st;
}

Op dense_op(const qb_dense* A) {
    Op o{};
    o.m = A->m; o.n = A->n; o.sparse = false; o.dtype = A->dtype;
    if (A->dtype == QB_BF16) {
        o.aq = static_cast<const uint16_t*>(A->a);
    } else if (A->dtype == QB_FP8E4M3) {
        o.a8 = static_cast<const uint8_t*>(A->a);
        o.row_exp = A->row_exp;
    } else {
        o.a = static_cast<const double*>(A->a);
    }
    o.lda = A->lda;
    return o;
}

Op csr_op(const qb_csr* A) {
    Op o{};
    o.m = A->m; o.n = A->n; o.sparse = true; o.dtype = QB_F64;
    o.rowptr = A->rowptr; o.colind = A->colind; o.val = A->val; o.nnz = A->nnz;
    return o;
}

int check_dense(const qb_dense* A) {
    if (A == nullptr || A->a == nullptr || A->m < 1 || A->n < 1 || A->lda < A->n) return QB_ERR_ARG;
    if (A->dtype != QB_F64 && A->dtype != QB_BF16 && A->dtype != QB_FP8E4M3) return QB_ERR_UNSUPPORTED;
    if (A->dtype == QB_FP8E4M3 && A->row_exp == nullptr) return QB_ERR_ARG;
    return QB_OK;
}

int check_csr(const qb_csr* A) {
    if (A == nullptr || A->m < 1 || A->n < 1 || A->nnz < 0 || A->rowptr == nullptr) return QB_ERR_ARG;
    if (A->nnz > 0 && (A->colind == nullptr || A->val == nullptr)) return QB_ERR_ARG;
    if (A->nnz >= (int64_t(1) << 31)) return QB_ERR_ARG;
    return QB_OK;
}

// trQRCP driven by the indicator (Remark 3.2) on dense binary64 A.  The sketch
// S = Omega^T A (Omega: m x l, generator stream 1) is taken once and kept transposed.  Per
// block: bw pivot steps of Householder QR with column pivoting on the sketch choose the
// columns J; the block is then factored as a block of Algorithm 2 with A(:, J) in place of
// A Omega_i (W = B(:, J), Y = A(:, J) - Q W, the two QRs, B_i = Q_i^T A), the indicator is
// decremented row by row, and the sketch follows the residual by the sample update
// S <- S - S(:, J) R_i^{-1} B_i.  In the sketch's rotated basis (after the pivot steps its
// pivot columns hold R~_11 over zeros) that update changes only the first bw rows, by
// R~_11 R_i^{-1} B_i; the pivot columns are inactive from then on.
int qrcp_run(const qb_dense* Ad, const qb_params* p, int oversample, double* Q, int64_t ldq,
             double* B, int64_t ldb, int32_t* piv, void* ws, size_t ws_bytes, hipStream_t s,
             qb_info* info) {
    qb_info local{};
    qb_info* inf = info ? info : &local;
    memset(inf, 0, sizeof(*inf));
    if (int st = check_dense(Ad)) return inf->status = st;
    Op A = dense_op(Ad);
    int st = check_params(p, A.m, A.n);
    if (st != QB_OK) return inf->status = st;
    if (A.dtype != QB_F64 || p->power != 0) return inf->status = QB_ERR_UNSUPPORTED;
    if (oversample < 0 || oversample > kMaxOversample) return inf->status = QB_ERR_ARG;
    if (Q == nullptr || B == nullptr || piv == nullptr || ws == nullptr || ldq < A.m || ldb < A.n)
        return inf->status = QB_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return inf->status = QB_ERR_ARG;
    const int64_t m = A.m, n = A.n, b = p->b, lmax = p->l_max;
    const int ell = p->b + oversample;
    if (ell > qrcp_max_rows()) return inf->status = QB_ERR_ARG;
    const Layout L = make_layout(QB_ALGO_EI, 0, QB_F64, m, n, 0, p, ell);
    if (ws_bytes < L.total) return inf->status = QB_ERR_WORKSPACE;
    double host[kHostWords];
    DevRes* res = dev_res();
    Timer tm(s, res != nullptr ? &res->pool : nullptr);
    char* wsb = static_cast<char*>(ws);
    const Ctx x{A, p, Q, ldq, B, ldb, wsb, L, s, inf, &tm, host};
    double* scal = x.at<double>(L.scal);
    tm.mark(0);
    QB_HIP(launch_sumsq_dense(A.a, m, n, A.lda, x.at<double>(L.red), scal, s));
    QB_HIP(hipMemcpyAsync(host, scal, sizeof(double), hipMemcpyDeviceToHost, s));
    QB_HIP(hipStreamSynchronize(s));
    const double normA2 = host[0];
    inf->normA2 = normA2;
    if (!isfinite(normA2)) {
        tm.mark(-1);
        return inf->status = QB_ERR_NONFINITE;
    }
    const double eps2 = p->tol_rel * p->tol_rel * normA2;
    const double floor_tol = sqrt(4.0 * kUnitRoundoff / 0.01);
    const int status_tol = p->tol_rel < floor_tol ? QB_WARN_TOL_FLOOR : QB_OK;
    double E = normA2;
    int64_t k = 0;
    bool exhausted = false;
    if (!(normA2 == 0.0 || E < eps2)) {
        double* St = x.at<double>(L.sk);
        double* colA = x.at<double>(L.cola);
        double* qn = x.at<double>(L.qn);
        int* act = x.at<int>(L.act);
        int* bpiv = x.at<int>(L.bpiv);
        double* g2p = x.at<double>(L.g2p);
        double* Rs = x.at<double>(L.rs);
        double* M = x.at<double>(L.mm);
        double* Y = x.at<double>(L.g);
        double* Wb = x.at<double>(L.w);
        double* qcv = x.at<double>(L.qcv);
        int* qci = x.at<int>(L.qci);
        double* betas = x.at<double>(L.beta);
        QB_HIP(launch_fill_int(x.at<int>(L.flags), 8, 0, s));
        // ||A(:, j)||^2, the reference of the exhaustion guard
        QB_HIP(launch_colsq_rowmajor(A.a, m, n, A.lda, x.at<double>(L.colpart), s));
        QB_HIP(launch_sum_partials(x.at<double>(L.colpart), colsq_groups(m), n, n, colA, s));
        tm.mark(1);
        QB_HIP(launch_gauss_fill(p->seed, kSketchStream, 0, 0, 0, m, ell, x.at<double>(L.skom), ell, s));
        tm.mark(2);
        if (int e = apply_At(x, x.at<double>(L.skom), ell, St, ell, ell)) return inf->status = e;
        inf->passes += 1;
        inf->gemm_flops[0] += 2.0 * m * n * ell;
        tm.mark(4);
        QB_HIP(launch_fill_int(act, static_cast<int>(n), 1, s));
        QB_HIP(launch_qrcp_norms(St, n, ell, act, qn, s));
        QB_HIP(launch_qrcp_cands(qn, n, qcv, qci, s));
        bool stop = false;
        while (k < lmax && !stop) {
            const int bwi = static_cast<int>(b < lmax - k ? b : lmax - k);
            for (int t = 0; t < bwi; ++t)
                QB_HIP(launch_qrcp_step(St, n, ell, t, qn, act, bpiv, colA, g2p, betas, qcv, qci, s));
            QB_HIP(launch_gather_cols(A.a, A.lda, m, bpiv, bwi, Y, bwi, s));
            if (k > 0) QB_HIP(launch_gather_cols(B, ldb, k, bpiv, bwi, Wb, bwi, s));
            bool breakdown = false;
            for (int attempt = 0; attempt < 2; ++attempt) {
                const bool use_hh = attempt == 1;
                if (use_hh) {
                    QB_HIP(launch_fill_int(x.at<int>(L.flags), 8, 0, s));
                    inf->fallbacks += 1;
                }
                if (int e = orth_block(x, k, bwi, Y, bwi, nullptr, bwi, use_hh, nullptr, 0))
                    return inf->status = e;
                tm.mark(3);
                if (int e = ei_block_b(x, k, bwi)) return inf->status = e;
                tm.mark(4);
                if (int e = fetch_block(x, bwi, g2p, &breakdown)) return inf->status = e;
                if (!breakdown) break;
            }
            QB_HIP(hipMemcpyAsync(piv + k, bpiv, sizeof(int) * bwi, hipMemcpyDeviceToDevice, s));
            inf->blocks += 1;
            inf->passes += 1;
            inf->gemm_flops[1] += 2.0 * m * n * bwi;
            int keep = 0;
            bool exh = false;
            const int64_t k0 = k;
            scan_rows(host, bwi, p->row_by_row != 0, eps2, &E, &keep, &stop, &exh);
            k += keep;
            if (exh) exhausted = true;
            if (!stop && k < lmax) {
                // sample update in the rotated basis: St(:, 0:bw) -= B_i^T (R~_11 R_i^{-1})^T
                QB_HIP(launch_qrcp_rs(St, ell, bpiv, betas, bwi, Rs, s));
                GemmDesc d = gdesc(bwi, bwi, bwi, View{Rs, bwi, 1}, View{x.at<double>(L.rii), bwi, 1}, 1.0,
                                   0.0, View{nullptr, 0, 0}, MutView{M, bwi, 1}, x);
                QB_HIP(gemm_f64(d, s));
                GemmDesc u = gdesc(n, bwi, bwi, View{B + k0 * ldb, 1, ldb}, View{M, 1, bwi}, -1.0, 1.0,
                                   View{St, ell, 1}, MutView{St, ell, 1}, x);
                QB_HIP(gemm_f64(u, s));
                QB_HIP(launch_qrcp_norms(St, n, ell, act, qn, s));
                QB_HIP(launch_qrcp_cands(qn, n, qcv, qci, s));
            }
        }
    }
    tm.mark(-1);
    QB_HIP(hipStreamSynchronize(s));
    tm.collect(inf->ms);
    inf->rank = k;
    inf->E = E;
    inf->exhausted = exhausted ? 1 : 0;
    if (normA2 == 0.0 || E < eps2)
        st = status_tol;
    else
        st = QB_NOT_CONVERGED;
    return inf->status = st;
}

// Workspace of the SVD from QB: P (n x k, the orthonormalised B^T), T / X (k x k), the
// rotations W, the sorted Ut and Ws (k x k each), the values and their order, the block
// Jacobi's partial Gram matrices, pair rotations and skip flags, and the buffers of
// orth_panel (128-column panels of n rows, k x 128 projections, 128 x 128 factors, split-K
// partials).
Layout svd_layout(int64_t m, int64_t n, int64_t k) {
    Layout L{};
    const int64_t pb = kPowerBlock;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.split_elems = 4 * (n > k ? n : k) * pb;
    if (L.split_elems < kGramSplitElems) L.split_elems = kGramSplitElems;
    L.om = take(sizeof(double) * n * k);   // P
    L.g = take(sizeof(double) * k * k);    // T, read as X = T^T (column-major)
    L.h = take(sizeof(double) * k * k);    // W
    L.s = take(sizeof(double) * k * k);    // Ut
    L.d = take(sizeof(double) * k * k);    // Ws
    L.gnorm2 = take(sizeof(double) * k);   // column norms
    L.info = take(sizeof(int) * k);        // order
    L.w = take(sizeof(double) * jacobi_part_elems(static_cast<int>(k)));   // pair Gram partials
    L.ri = take(sizeof(double) * jacobi_rot_elems(static_cast<int>(k)));   // pair rotations
    L.rowsq = take(sizeof(int) * (jacobi_rot_elems(static_cast<int>(k)) + 1));   // skip flags
    L.y = take(sizeof(double) * n * pb);
    L.x2 = take(sizeof(double) * n * pb);
    L.z = take(sizeof(double) * k * pb);
    L.gram = take(sizeof(double) * pb * pb);
    L.r1 = take(sizeof(double) * pb * pb);
    L.r1i = take(sizeof(double) * pb * pb);
    L.rt = take(sizeof(double) * pb * pb);
    L.rti = take(sizeof(double) * pb * pb);
    L.tau = take(sizeof(double) * pb);
    L.flags = take(sizeof(int) * 8);
    L.split = take(sizeof(double) * L.split_elems);
    L.total = off + 256;
    (void)m;
    return L;
}

constexpr int kMaxSweeps = 40;
constexpr int kJacobiInner = 1;   // two-sided Jacobi sweeps on each pair's Gram matrix per round

int svd_from_qb(int64_t m, int64_t n, int64_t k, const double* Q, int64_t ldq, const double* B,
                int64_t ldb, double* U, int64_t ldu, double* sv, double* V, int64_t ldv, void* ws,
                size_t ws_bytes, hipStream_t s, int32_t* sweeps_out) {
    if (sweeps_out) *sweeps_out = 0;
    if (k < 1 || m < 1 || n < 1 || k > m || k > n || k >= (int64_t(1) << 31)) return QB_ERR_ARG;
    if (Q == nullptr || B == nullptr || U == nullptr || sv == nullptr || V == nullptr || ws == nullptr)
        return QB_ERR_ARG;
    if (ldq < m || ldb < n || ldu < m || ldv < n) return QB_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return QB_ERR_ARG;
    const Layout L = svd_layout(m, n, k);
    if (ws_bytes < L.total) return QB_ERR_WORKSPACE;
    double host[kHostWords];
    char* wsb = static_cast<char*>(ws);
    Op none{};
    Ctx x{none, nullptr, nullptr, 0, nullptr, 0, wsb, L, s, nullptr, nullptr, host};
    double* P = x.at<double>(L.om);
    double* T = x.at<double>(L.g);
    double* W = x.at<double>(L.h);
    double* Ut = x.at<double>(L.s);
    double* Ws = x.at<double>(L.d);
    double* sig = x.at<double>(L.gnorm2);
    int* pos = x.at<int>(L.info);
    int* flags = x.at<int>(L.flags);
    const int ki = static_cast<int>(k);
    // B^T = P T: P = orth(B^T) (n x k, row-major), T = P^T B^T
    for (int attempt = 0; attempt < 2; ++attempt) {
        QB_HIP(launch_fill_int(flags, 8, 0, s));
        GemmDesc c = gdesc(n, k, 0, View{nullptr, 0, 0}, View{nullptr, 0, 0}, 0.0, 1.0,
                           View{B, 1, ldb}, MutView{P, k, 1}, x);
        QB_HIP(gemm_f64(c, s));
        if (int e = orth_panel(x, P, n, k, k, 0, attempt == 1, orth_block_cols(n))) return e;
        bool broken = false;
        if (int e = read_flag(x, &broken)) return e;
        if (!broken) break;
    }
    {
        GemmDesc d = gdesc(k, k, n, View{P, 1, k}, View{B, 1, ldb}, 1.0, 0.0, View{nullptr, 0, 0},
                           MutView{T, k, 1}, x);
        QB_HIP(gemm_f64(d, s));
    }
    // block one-sided Jacobi on X = T^T (column-major: the same storage as row-major T).
    // Pairs rotate at cosines above tol = 16 sqrt(k) u, and the sweeps end after one in
    // which none did.  (The usual one-sided threshold is sqrt(k) u; a block rotation
    // applied as one product of 2 kJb columns leaves cosines of a few u sqrt(2 kJb) of its
    // own, so the threshold sits above that floor.)
    QB_HIP(launch_identity(W, ki, k, s));
    const double tol_r = 16.0 * sqrt(static_cast<double>(k)) * kUnitRoundoff;
    const double tol_c = tol_r;
    const int rounds = jacobi_rounds(ki);
    double* jpart = x.at<double>(L.w);
    double* jrot = x.at<double>(L.ri);
    int* jskip = x.at<int>(L.rowsq);
    int st = QB_NOT_CONVERGED;
    int sweeps = 0;
    int* hflag = reinterpret_cast<int*>(host + 3 * kMaxB);
    while (sweeps < kMaxSweeps) {
        QB_HIP(launch_fill_int(flags + 1, 1, 0, s));
        for (int r = -1; r < rounds; ++r)   // the within-block step, then the circle rounds
            QB_HIP(launch_jacobi_block_round(T, W, ki, k, r, tol_r, tol_c, kJacobiInner, jpart, jrot, jskip,
                                             flags + 1, s));
        ++sweeps;
        QB_HIP(hipMemcpyAsync(hflag, flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
        QB_HIP(hipStreamSynchronize(s));
        if (*hflag == 0) {
            st = QB_OK;
            break;
        }
    }
    if (sweeps_out) *sweeps_out = sweeps;
    // values, order, normalised left vectors and rotations in descending order
    QB_HIP(launch_svd_finish(T, W, ki, k, sig, pos, sv, Ut, Ws, s));
    // V = P Ws (n x k, column-major), the sign rule on V and Ut, then U = Q Ut
    {
        GemmDesc d = gdesc(n, k, k, View{P, k, 1}, View{Ws, 1, k}, 1.0, 0.0, View{nullptr, 0, 0},
                           MutView{V, 1, ldv}, x);
        QB_HIP(gemm_f64(d, s));
    }
    QB_HIP(launch_sign_rule(V, n, ldv, Ut, ki, k, s));
    {
        GemmDesc d = gdesc(m, k, k, View{Q, 1, ldq}, View{Ut, 1, k}, 1.0, 0.0, View{nullptr, 0, 0},
                           MutView{U, 1, ldu}, x);
        QB_HIP(gemm_f64(d, s));
    }
    QB_HIP(hipStreamSynchronize(s));
    return st;
}

// COO input: the CSR arrays and the conversion's scratch come first in the workspace, then
// the CSR path's own workspace (sized for nnz, an upper bound of the CSR entry count).
struct CooSplit {
    size_t conv, rowptr, colind, val, run, total;
};

CooSplit coo_split(int algo, const qb_coo* A, const qb_params* p) {
    CooSplit c{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    c.conv = take(coo_bytes(A->m, A->n, A->nnz));
    c.rowptr = take(sizeof(int64_t) * (A->m + 1));
    c.colind = take(sizeof(int32_t) * (A->nnz > 0 ? A->nnz : 1));
    c.val = take(sizeof(double) * (A->nnz > 0 ? A->nnz : 1));
    c.run = off;
    c.total = p != nullptr ? off + make_layout(algo, 1, QB_F64, A->m, A->n, A->nnz, p).total : off;
    return c;
}

int check_coo(const qb_coo* A) {
    if (A == nullptr || A->m < 1 || A->n < 1 || A->nnz < 0) return QB_ERR_ARG;
    if (A->nnz >= (int64_t(1) << 31) || A->m >= (int64_t(1) << 31) || A->n >= (int64_t(1) << 31))
        return QB_ERR_ARG;
    if (A->nnz > 0 && (A->row == nullptr || A->col == nullptr || A->val == nullptr)) return QB_ERR_ARG;
    return QB_OK;
}

// Convert into ws (layout c) and return the CSR entry count on the host; the stream is
// synchronised.  ms (may be null) receives the device time of the conversion.
int coo_convert(const qb_coo* A, const CooSplit& c, char* ws, hipStream_t s, int64_t* nnz_out,
                double* ms) {
    double host[2];
    DevRes* res = ms != nullptr ? dev_res() : nullptr;
    Timer tm(s, res != nullptr ? &res->pool : nullptr);
    tm.mark(0);
    QB_HIP(coo_to_csr(A->row, A->col, A->val, A->m, A->n, A->nnz, ws + c.conv,
                      reinterpret_cast<int64_t*>(ws + c.rowptr), reinterpret_cast<int32_t*>(ws + c.colind),
                      reinterpret_cast<double*>(ws + c.val), s));
    tm.mark(-1);
    const int64_t* nruns;
    const int* bad;
    coo_counts(A->m, A->n, A->nnz, ws + c.conv, &nruns, &bad);
    QB_HIP(hipMemcpyAsync(host, nruns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QB_HIP(hipMemcpyAsync(host + 1, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    QB_HIP(hipStreamSynchronize(s));
    int64_t cnt;
    memcpy(&cnt, host, sizeof(cnt));
    int flag;
    memcpy(&flag, host + 1, sizeof(flag));
    if (ms != nullptr) {
        double t[8] = {};
        tm.collect(t);
        *ms = t[0];
    }
    if (flag != 0) return QB_ERR_ARG;
    *nnz_out = cnt;
    return QB_OK;
}

int coo_run(int algo, const qb_coo* A, const qb_params* p, double* Q, int64_t ldq, double* B,
            int64_t ldb, void* ws, size_t ws_bytes, hipStream_t s, qb_info* info) {
    qb_info local{};
    qb_info* inf = info ? info : &local;
    memset(inf, 0, sizeof(*inf));
    int st = check_coo(A);
    if (st == QB_OK) st = check_params(p, A->m, A->n);
    if (st != QB_OK) return inf->status = st;
    if (Q == nullptr || B == nullptr || ws == nullptr || ldq < A->m || ldb < A->n)
        return inf->status = QB_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return inf->status = QB_ERR_ARG;
    const CooSplit c = coo_split(algo, A, p);
    if (ws_bytes < c.total) return inf->status = QB_ERR_WORKSPACE;
    char* wsb = static_cast<char*>(ws);
    int64_t nnz = 0;
    double conv_ms = 0.0;
    if (int e = coo_convert(A, c, wsb, s, &nnz, &conv_ms)) return inf->status = e;
    qb_csr csr{A->m, A->n, nnz, reinterpret_cast<const int64_t*>(wsb + c.rowptr),
               reinterpret_cast<const int32_t*>(wsb + c.colind), reinterpret_cast<const double*>(wsb + c.val)};
    Op o = csr_op(&csr);
    const int r = run(algo, o, p, Q, ldq, B, ldb, wsb + c.run, ws_bytes - c.run, s, inf);
    inf->ms[7] = conv_ms;
    return r;
}

// ------------------------------------------------------------------ layout check

// Whether every region of the workspace layout holds what its producers write (the extent of
// a region runs to the next region's offset).  The producers' sizes come from the same
// functions their launchers use.
int layout_check(int algo, int sparse, int dtype, int64_t m, int64_t n, int64_t nnz, const qb_params* p,
                 int ell) {
    const Layout L = make_layout(algo, sparse, dtype, m, n, nnz, p, ell);
    std::vector<size_t> offs = {L.red, L.scal, L.om, L.g, L.h, L.gpart, L.gnorm2, L.y, L.x2, L.s, L.w,
                                L.z, L.d, L.gram, L.r1, L.r1i, L.rt, L.rti, L.ri, L.rii, L.tau,
                                L.rowsq_part, L.rowsq, L.info, L.flags, L.scan, L.khist, L.ehist,
                                L.split, L.split2, L.ynext, L.w2, L.csc,
                                L.plan_a, L.plan_t, L.omt, L.gqt, L.omt8, L.total};
    if (ell > 0) offs.insert(offs.end(), {L.sk, L.skom, L.cola, L.colpart, L.qn, L.act, L.bpiv,
                                          L.g2p, L.rs, L.mm, L.qcv, L.qci, L.beta});
    auto extent = [&](size_t off) {
        size_t next = L.total;
        for (size_t o : offs)
            if (o > off && o < next) next = o;
        return next - off;
    };
    bool ok = true;
    auto need = [&](size_t off, double bytes) {
        if ((off & 255) != 0 || static_cast<double>(extent(off)) < bytes) ok = false;
    };
    const bool lowp = dtype == QB_BF16 || dtype == QB_FP8E4M3;
    const int64_t b = p->b, lt = L.lt, lmax = p->l_max;
    const bool pw = p->power > 0;
    const int64_t prow = pw && n > m ? n : m, pb = pw && b < kPowerBlock ? kPowerBlock : b;
    const int64_t D = sizeof(double);
    need(L.red, D * sumsq_partials());
    need(L.scal, D);
    need(L.om, D * n * lt);
    need(L.g, D * m * (ell > 0 ? b : lt));
    if (algo == QB_ALGO_FP) need(L.h, D * n * lt);
    // column sums of squares of G (every chunk width w <= lt; EI: w = b)
    for (int64_t w = 1; w <= lt; ++w) {
        const int64_t groups = sparse ? colsq_groups(m) : lowp ? bf16_gemm_row_groups(m, w)
                                                               : std::max(gemm_f64_colsq_groups(m, w),
                                                                          w <= 64 ? colsq_groups(m) : 0);
        need(L.gpart, D * groups * w);
    }
    need(L.gnorm2, D * lt);
    need(L.y, D * prow * pb);
    need(L.x2, D * prow * pb);
    need(L.s, D * b * n);
    need(L.w, D * lmax * b);
    need(L.z, D * lmax * pb);
    need(L.d, D * lmax * b);
    for (size_t o : {L.gram, L.r1, L.r1i, L.rt, L.rti}) need(o, D * pb * pb);
    need(L.ri, D * b * b);
    need(L.rii, D * b * b);
    need(L.tau, D * pb);
    // row sums of squares of B_i: the B_i product (n x bw, K = bw for randQB_FP, K = m for
    // randQB_EI) or, for CSR randQB_EI, the column reduction of A^T Q_i
    for (int64_t bw = 1; bw <= b; ++bw) {
        const int64_t groups = sparse && algo == QB_ALGO_EI ? colsq_groups(n) : gemm_f64_colsq_groups(n, bw);
        need(L.rowsq_part, D * groups * bw);
    }
    need(L.rowsq, D * b);
    need(L.info, D * (3 * b + 1));
    need(L.flags, sizeof(int) * 8);
    need(L.scan, sizeof(ScanState));
    // scanned blocks: every block but the last keeps at least one row; randQB_FP chunks are
    // multiples of b except the last, so at most cdiv(l_max, b) + chunks blocks, chunks
    // being at most cdiv(l_max, b)
    need(L.khist, 8.0 * (2 * cdiv(lmax, b) + 1));
    need(L.ehist, D * (2 * cdiv(lmax, b) + 1));
    if (L.ahead) {
        need(L.ynext, D * m * b);
        need(L.w2, D * lmax * b);
    }
    if (sparse) {
        need(L.csc, static_cast<double>(csc_layout(m, n, nnz).total));
        need(L.plan_a, static_cast<double>(spmm_plan_bytes(m, nnz, lt)));
        need(L.plan_t, static_cast<double>(spmm_plan_bytes(n, nnz, lt)));
    }
    if (lowp) {
        need(L.omt, 2.0 * lt * L.ldn16);
        need(L.gqt, 2.0 * lt * L.ldm16);
    }
    if (dtype == QB_FP8E4M3) need(L.omt8, 1.0 * lt * L.ldn8);
    if (ell > 0) {
        need(L.sk, D * n * ell);
        need(L.skom, D * m * ell);
        need(L.cola, D * n);
        need(L.colpart, D * colsq_groups(m) * n);
        need(L.qn, D * n);
        need(L.act, sizeof(int) * n);
        need(L.bpiv, sizeof(int) * b);
        need(L.g2p, D * b);
        need(L.rs, D * b * b);
        need(L.mm, D * b * b);
        // the pivot steps' per-workgroup best columns (two step parities) and diag(R~_11)
        need(L.qcv, D * 2 * qrcp_cand_slots(n));
        need(L.qci, sizeof(int) * 2.0 * qrcp_cand_slots(n));
        need(L.beta, D * b);
    }
    return ok ? QB_OK : QB_ERR_WORKSPACE;
}

// ------------------------------------------------------------------ allocation-free entry

// Scratch memory of qb_fp_dense_noalloc: a device array in the library's code object (each
// device the library runs on holds its own copy until the process ends).  In host code the
// name stands for a host-side shadow, never a device address: the device address is looked
// up per device with hipGetSymbolAddress and only that pointer is handed to kernels.
static __device__ __align__(256) char scratch[QB_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// The current device's address of the scratch array, looked up on the first call on that
// device (with it current) and kept.
int scratch_ptr(void** out) {
    int dev = 0;
    QB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return QB_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[dev] == nullptr) {
        void* ptr = nullptr;
        QB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (ptr == nullptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0) return QB_ERR_HIP;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return QB_OK;
}

// Layout of the allocation-free mode inside the scratch array: make_layout's regions with the
// split-K partials cut to the room the other regions leave.  false if they do not fit.
bool noalloc_layout(const Op& A, const qb_params* p, Layout* L) {
    const Layout base = make_layout(QB_ALGO_FP, 0, A.dtype, A.m, A.n, 0, p, 0, 0);
    if (base.total > QB_NOALLOC_SCRATCH_BYTES) return false;
    const int64_t room = static_cast<int64_t>(QB_NOALLOC_SCRATCH_BYTES - base.total) / 8 - 64;
    if (room < 0) return false;
    *L = make_layout(QB_ALGO_FP, 0, A.dtype, A.m, A.n, 0, p, 0, room);
    return L->total <= QB_NOALLOC_SCRATCH_BYTES;
}

}  // namespace
}  // namespace qb

using namespace qb;

extern "C" {

size_t qb_workspace_bytes(int algo, int sparse, int64_t m, int64_t n, int64_t nnz,
                          const qb_params* p) {
    if ((algo != QB_ALGO_FP && algo != QB_ALGO_EI) || m < 1 || n < 1) return 0;
    if (check_params(p, m, n) != QB_OK) return 0;
    return make_layout(algo, sparse != 0, QB_F64, m, n, nnz, p).total;
}

size_t qb_dense_workspace_bytes(int algo, const qb_dense* A, const qb_params* p) {
    if ((algo != QB_ALGO_FP && algo != QB_ALGO_EI) || A == nullptr || A->m < 1 || A->n < 1) return 0;
    const bool lowp = A->dtype == QB_BF16 || A->dtype == QB_FP8E4M3;
    if (A->dtype != QB_F64 && !(lowp && algo == QB_ALGO_FP)) return 0;
    if (check_params(p, A->m, A->n) != QB_OK) return 0;
    return make_layout(algo, 0, A->dtype, A->m, A->n, 0, p).total;
}

int qb_fp_dense(const qb_dense* A, const qb_params* p, double* Q, int64_t ldq, double* B,
                int64_t ldb, void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info) {
    if (int st = check_dense(A)) {
        if (info) info->status = st;
        return st;
    }
    Op o = dense_op(A);
    return run(QB_ALGO_FP, o, p, Q, ldq, B, ldb, ws, ws_bytes, stream, info);
}

int qb_layout_check(int algo, int sparse, int dtype, int64_t m, int64_t n, int64_t nnz,
                    const qb_params* p, int32_t oversample) {
    if ((algo != QB_ALGO_FP && algo != QB_ALGO_EI) || m < 1 || n < 1 || nnz < 0) return QB_ERR_ARG;
    if (check_params(p, m, n) != QB_OK || oversample < 0 || oversample > kMaxOversample) return QB_ERR_ARG;
    const int ell = oversample > 0 ? p->b + oversample : 0;
    return layout_check(algo, sparse != 0, dtype, m, n, nnz, p, ell);
}

int qb_fp_dense_noalloc(const qb_dense* A, const qb_params* p, double* Q, int64_t ldq, double* B,
                        int64_t ldb, hipStream_t stream, qb_info* info) {
    int st = check_dense(A);
    if (st == QB_OK && p == nullptr) st = QB_ERR_ARG;
    if (st == QB_OK) st = check_params(p, A->m, A->n);
    Op o{};
    Layout L{};
    if (st == QB_OK) {
        o = dense_op(A);
        if (!noalloc_layout(o, p, &L)) st = QB_ERR_WORKSPACE;
    }
    void* ws = nullptr;
    if (st == QB_OK) st = scratch_ptr(&ws);
    if (st != QB_OK) {
        if (info) {
            memset(info, 0, sizeof(*info));
            info->status = st;
        }
        return st;
    }
    return run(QB_ALGO_FP, o, p, Q, ldq, B, ldb, ws, QB_NOALLOC_SCRATCH_BYTES, stream, info, &L);
}

int qb_ei_dense(const qb_dense* A, const qb_params* p, double* Q, int64_t ldq, double* B,
                int64_t ldb, void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info) {
    if (int st = check_dense(A)) {
        if (info) info->status = st;
        return st;
    }
    Op o = dense_op(A);
    return run(QB_ALGO_EI, o, p, Q, ldq, B, ldb, ws, ws_bytes, stream, info);
}

size_t qb_trqrcp_workspace_bytes(int64_t m, int64_t n, const qb_params* p, int32_t oversample) {
    if (m < 1 || n < 1 || check_params(p, m, n) != QB_OK) return 0;
    if (oversample < 0 || oversample > kMaxOversample || p->b + oversample > qrcp_max_rows()) return 0;
    return make_layout(QB_ALGO_EI, 0, QB_F64, m, n, 0, p, p->b + oversample).total;
}

int qb_trqrcp_dense(const qb_dense* A, const qb_params* p, int32_t oversample, double* Q, int64_t ldq,
                    double* B, int64_t ldb, int32_t* piv, void* ws, size_t ws_bytes, hipStream_t stream,
                    qb_info* info) {
    return qrcp_run(A, p, oversample, Q, ldq, B, ldb, piv, ws, ws_bytes, stream, info);
}

int qb_fp_csr(const qb_csr* A, const qb_params* p, double* Q, int64_t ldq, double* B, int64_t ldb,
              void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info) {
    if (int st = check_csr(A)) {
        if (info) info->status = st;
        return st;
    }
    Op o = csr_op(A);
    return run(QB_ALGO_FP, o, p, Q, ldq, B, ldb, ws, ws_bytes, stream, info);
}

int qb_ei_csr(const qb_csr* A, const qb_params* p, double* Q, int64_t ldq, double* B, int64_t ldb,
              void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info) {
    if (int st = check_csr(A)) {
        if (info) info->status = st;
        return st;
    }
    Op o = csr_op(A);
    return run(QB_ALGO_EI, o, p, Q, ldq, B, ldb, ws, ws_bytes, stream, info);
}

int qb_gaussian_fill(uint64_t seed, uint32_t stream_id, uint32_t batch, int64_t row0, int64_t col0,
                     int64_t rows, int64_t cols, double* out, int64_t ld, hipStream_t stream) {
    if (rows < 0 || cols < 0 || row0 < 0 || col0 < 0 || (rows > 0 && cols > 0 && out == nullptr) ||
        ld < cols || row0 + rows > (int64_t(1) << 32) || col0 + cols > (int64_t(1) << 33))
        return QB_ERR_ARG;
    return launch_gauss_fill(seed, stream_id, batch, row0, col0, rows, cols, out, ld, stream) ==
                   hipSuccess
               ? QB_OK
               : QB_ERR_HIP;
}

size_t qb_sumsq_workspace_bytes(void) { return sizeof(double) * 1040; }

int qb_sumsq_dense(const qb_dense* A, double* out_host, void* ws, hipStream_t stream) {
    if (int st = check_dense(A)) return st;
    if (out_host == nullptr || ws == nullptr) return QB_ERR_ARG;
    double* part = static_cast<double*>(ws);
    double* res = part + 1024;
    if (A->dtype == QB_BF16)
        QB_HIP(launch_sumsq_bf16(static_cast<const uint16_t*>(A->a), A->m, A->n, A->lda, part, res,
                                 stream));
    else if (A->dtype == QB_FP8E4M3)
        QB_HIP(launch_sumsq_fp8(static_cast<const uint8_t*>(A->a), A->row_exp, A->m, A->n, A->lda, part,
                                res, stream));
    else
        QB_HIP(launch_sumsq_dense(static_cast<const double*>(A->a), A->m, A->n, A->lda, part, res,
                                  stream));
    QB_HIP(hipMemcpyAsync(out_host, res, sizeof(double), hipMemcpyDeviceToHost, stream));
    QB_HIP(hipStreamSynchronize(stream));
    return QB_OK;
}

int qb_sketch_dense(const qb_dense* A, uint64_t seed, int64_t col0, int64_t l, double* om, double* g,
                    double* h, hipStream_t stream) {
    if (int st = check_dense(A)) return st;
    if (A->dtype != QB_F64) return QB_ERR_UNSUPPORTED;
    if (l < 1 || col0 < 0 || om == nullptr || g == nullptr || h == nullptr) return QB_ERR_ARG;
    const int64_t m = A->m, n = A->n;
    QB_HIP(launch_gauss_fill(seed, 0, 0, 0, col0, n, l, om, l, stream));
    GemmDesc d{};
    d.M = m; d.N = l; d.K = n;
    d.A = View{static_cast<const double*>(A->a), A->lda, 1};
    d.B = View{om, l, 1};
    d.alpha = 1.0; d.beta = 0.0;
    d.C = MutView{g, l, 1};
    QB_HIP(gemm_f64(d, stream));
    GemmDesc e{};
    e.M = n; e.N = l; e.K = m;
    e.A = View{static_cast<const double*>(A->a), 1, A->lda};
    e.B = View{g, l, 1};
    e.alpha = 1.0; e.beta = 0.0;
    e.C = MutView{h, l, 1};
    QB_HIP(gemm_f64(e, stream));
    return QB_OK;
}

// Single-pass form of the sketch sweep (Remark 4.2): A is streamed in panels of panel_rows
// rows; panel p gives G_p = A_p Omega, and A_p^T G_p is added to H right after, while A_p
// may still be in the last-level cache (it stays there only if the panel and the n x l
// operands fit in it together).  The H sum runs over the panels in order (fixed order).  The G_p
// products are short (panel_rows x l outputs), so they split K over the workspace.
static int64_t onepass_rows(const qb_dense* A, int64_t panel_rows) {
    if (panel_rows > 0) return panel_rows < A->m ? panel_rows : A->m;
    // default: panels of at most 96 MiB of A, a multiple of 128 rows
    int64_t r = (int64_t(96) << 20) / (8 * (A->lda > 0 ? A->lda : 1));
    r = (r / 128) * 128;
    if (r < 128) r = 128;
    return r < A->m ? r : A->m;
}

static int64_t onepass_ws_elems(int64_t rows, int64_t l) { return 32 * rows * l + 65536; }

size_t qb_sketch_onepass_bytes(const qb_dense* A, int64_t l, int64_t panel_rows) {
    if (check_dense(A) != QB_OK || A->dtype != QB_F64 || l < 1 || panel_rows < 0) return 0;
    return sizeof(double) * onepass_ws_elems(onepass_rows(A, panel_rows), l);
}

int qb_sketch_onepass(const qb_dense* A, uint64_t seed, int64_t col0, int64_t l, int64_t panel_rows,
                      double* om, double* g, double* h, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (int st = check_dense(A)) return st;
    if (A->dtype != QB_F64) return QB_ERR_UNSUPPORTED;
    if (l < 1 || col0 < 0 || panel_rows < 0 || om == nullptr || g == nullptr || h == nullptr ||
        ws == nullptr)
        return QB_ERR_ARG;
    const int64_t m = A->m, n = A->n, pr = onepass_rows(A, panel_rows);
    const int64_t ws_elems = onepass_ws_elems(pr, l);
    if (ws_bytes < sizeof(double) * static_cast<size_t>(ws_elems)) return QB_ERR_WORKSPACE;
    const double* a = static_cast<const double*>(A->a);
    QB_HIP(launch_gauss_fill(seed, 0, 0, 0, col0, n, l, om, l, stream));
    for (int64_t p0 = 0; p0 < m; p0 += pr) {
        const int64_t rows = pr < m - p0 ? pr : m - p0;
        GemmDesc d{};   // G_p = A_p Omega
        d.M = rows; d.N = l; d.K = n;
        d.A = View{a + p0 * A->lda, A->lda, 1};
        d.B = View{om, l, 1};
        d.alpha = 1.0; d.beta = 0.0;
        d.C = MutView{g + p0 * l, l, 1};
        d.ws = static_cast<double*>(ws); d.ws_elems = ws_elems;
        QB_HIP(gemm_f64(d, stream));
        GemmDesc e{};   // H (+)= A_p^T G_p
        e.M = n; e.N = l; e.K = rows;
        e.A = View{a + p0 * A->lda, 1, A->lda};
        e.B = View{g + p0 * l, l, 1};
        e.alpha = 1.0; e.beta = p0 == 0 ? 0.0 : 1.0;
        e.C0 = View{h, l, 1};
        e.C = MutView{h, l, 1};
        QB_HIP(gemm_f64(e, stream));
    }
    return QB_OK;
}

// Workspace of qb_sketch_lowp: the randQB_FP layout with one chunk of l columns (the
// sketch buffers it uses are Omega_q^T, G_q^T, A_q^T and the column-norm partials).
static bool sketch_lowp_layout(const qb_dense* A, int64_t l, Layout* L) {
    if (check_dense(A) != QB_OK || (A->dtype != QB_BF16 && A->dtype != QB_FP8E4M3) || l < 1) return false;
    qb_params p{};
    p.tol_rel = 0.0; p.b = 1; p.l_max = l; p.l_tilde = l;
    *L = make_layout(QB_ALGO_FP, 0, A->dtype, A->m, A->n, 0, &p);
    return true;
}

size_t qb_sketch_lowp_bytes(const qb_dense* A, int64_t l) {
    Layout L{};
    return sketch_lowp_layout(A, l, &L) ? L.total : 0;
}

int qb_sketch_lowp(const qb_dense* A, uint64_t seed, int64_t col0, int64_t l, double* om, double* g,
                   double* h, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (int st = check_dense(A)) return st;
    if (A->dtype != QB_BF16 && A->dtype != QB_FP8E4M3) return QB_ERR_UNSUPPORTED;
    if (l < 1 || col0 < 0 || om == nullptr || g == nullptr || h == nullptr || ws == nullptr)
        return QB_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return QB_ERR_ARG;
    Layout L{};
    if (!sketch_lowp_layout(A, l, &L)) return QB_ERR_ARG;
    if (ws_bytes < L.total) return QB_ERR_WORKSPACE;
    char* wsb = static_cast<char*>(ws);
    Op o = dense_op(A);
    Timer tm(stream, nullptr);
    const Ctx x{o, nullptr, nullptr, 0, nullptr, 0, wsb, L, stream, nullptr, &tm, nullptr};
    QB_HIP(launch_gauss_fill(seed, 0, 0, 0, col0, o.n, l, om, l, stream));
    return sketch_bf16(x, om, g, h, l, x.at<double>(L.gnorm2), false);
}

size_t qb_csr_transpose_bytes(const qb_csr* A) {
    if (check_csr(A) != QB_OK) return 0;
    return csc_layout(A->m, A->n, A->nnz).total;
}

int qb_sketch_csr(const qb_csr* A, uint64_t seed, int64_t col0, int64_t l, double* om, double* g,
                  double* h, void* csc_ws, int* csc_ready, hipStream_t stream) {
    if (int st = check_csr(A)) return st;
    if (l < 1 || col0 < 0 || om == nullptr || g == nullptr || h == nullptr || csc_ws == nullptr ||
        csc_ready == nullptr)
        return QB_ERR_ARG;
    char* ws = static_cast<char*>(csc_ws);
    if (!*csc_ready) {
        QB_HIP(build_csc(A->rowptr, A->colind, A->val, A->m, A->n, A->nnz, ws, stream));
        *csc_ready = 1;
    }
    const int64_t* tp;
    const int32_t* tc;
    const double* tv;
    csc_views(A->m, A->n, A->nnz, ws, &tp, &tc, &tv);
    QB_HIP(launch_gauss_fill(seed, 0, 0, 0, col0, A->n, l, om, l, stream));
    QB_HIP(launch_spmm_csr(A->rowptr, A->colind, A->val, A->m, om, l, g, l, l, stream));
    QB_HIP(launch_spmm_csr(tp, tc, tv, A->n, g, l, h, l, l, stream));
    return QB_OK;
}

size_t qb_coo_workspace_bytes(int algo, const qb_coo* A, const qb_params* p) {
    if ((algo != QB_ALGO_FP && algo != QB_ALGO_EI) || check_coo(A) != QB_OK) return 0;
    if (check_params(p, A->m, A->n) != QB_OK) return 0;
    return coo_split(algo, A, p).total;
}

int qb_fp_coo(const qb_coo* A, const qb_params* p, double* Q, int64_t ldq, double* B, int64_t ldb,
              void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info) {
    return coo_run(QB_ALGO_FP, A, p, Q, ldq, B, ldb, ws, ws_bytes, stream, info);
}

int qb_ei_coo(const qb_coo* A, const qb_params* p, double* Q, int64_t ldq, double* B, int64_t ldb,
              void* ws, size_t ws_bytes, hipStream_t stream, qb_info* info) {
    return coo_run(QB_ALGO_EI, A, p, Q, ldq, B, ldb, ws, ws_bytes, stream, info);
}

size_t qb_coo_to_csr_bytes(const qb_coo* A) {
    if (check_coo(A) != QB_OK) return 0;
    return coo_bytes(A->m, A->n, A->nnz);
}

int qb_coo_to_csr(const qb_coo* A, int64_t* rowptr, int32_t* colind, double* val, int64_t* nnz_out,
                  void* ws, size_t ws_bytes, hipStream_t stream) {
    if (int st = check_coo(A)) return st;
    if (rowptr == nullptr || (A->nnz > 0 && (colind == nullptr || val == nullptr)) || nnz_out == nullptr ||
        ws == nullptr)
        return QB_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return QB_ERR_ARG;
    if (ws_bytes < coo_bytes(A->m, A->n, A->nnz)) return QB_ERR_WORKSPACE;
    double host[2];
    char* wsb = static_cast<char*>(ws);
    QB_HIP(coo_to_csr(A->row, A->col, A->val, A->m, A->n, A->nnz, wsb, rowptr, colind, val, stream));
    const int64_t* nruns;
    const int* bad;
    coo_counts(A->m, A->n, A->nnz, wsb, &nruns, &bad);
    QB_HIP(hipMemcpyAsync(host, nruns, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    QB_HIP(hipMemcpyAsync(host + 1, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
    QB_HIP(hipStreamSynchronize(stream));
    int flag;
    memcpy(&flag, host + 1, sizeof(flag));
    if (flag != 0) return QB_ERR_ARG;
    memcpy(nnz_out, host, sizeof(int64_t));
    return QB_OK;
}

size_t qb_svd_workspace_bytes(int64_t m, int64_t n, int64_t k) {
    if (k < 1 || m < 1 || n < 1 || k > m || k > n) return 0;
    return svd_layout(m, n, k).total;
}

int qb_svd_from_qb(int64_t m, int64_t n, int64_t k, const double* Q, int64_t ldq, const double* B,
                   int64_t ldb, double* U, int64_t ldu, double* s, double* V, int64_t ldv, void* ws,
                   size_t ws_bytes, hipStream_t stream, int32_t* sweeps) {
    return svd_from_qb(m, n, k, Q, ldq, B, ldb, U, ldu, s, V, ldv, ws, ws_bytes, stream, sweeps);
}

const char* qb_status_string(int status) {
    switch (status) {
        case QB_OK: return "QB_OK";
        case QB_NOT_CONVERGED: return "QB_NOT_CONVERGED";
        case QB_WARN_TOL_FLOOR: return "QB_WARN_TOL_FLOOR";
        case QB_ERR_ARG: return "QB_ERR_ARG";
        case QB_ERR_NONFINITE: return "QB_ERR_NONFINITE";
        case QB_ERR_WORKSPACE: return "QB_ERR_WORKSPACE";
        case QB_ERR_HIP: return "QB_ERR_HIP";
        case QB_ERR_UNSUPPORTED: return "QB_ERR_UNSUPPORTED";
        default: return "QB_UNKNOWN_STATUS";
    }
}

}  // extern "C"
