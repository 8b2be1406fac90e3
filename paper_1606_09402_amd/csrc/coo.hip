// COO input: entries (row, col, val) in any order, duplicates summed, turned into CSR on the
// device.  The entries are sorted by the key row * n + col with a stable radix sort (so equal
// keys keep their input order), the first entry of each run of equal keys is marked, an
// exclusive scan of the marks gives each run its place, one thread per run adds the run's
// values in sorted order (a fixed order: the result is reproducible), and the row starts are
// found by binary search in the sorted unique keys.
#include <hipcub/hipcub.hpp>

#include "kernels.h"

namespace qb {

// keys[e] = row * n + col; bad[0] = 1 if an index lies outside the matrix.
__global__ void coo_keys_kernel(const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                                int64_t nnz, int64_t m, int64_t n, uint64_t* __restrict__ keys,
                                int32_t* __restrict__ perm, int* __restrict__ bad) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int64_t r = row[e], c = col[e];
    const bool ok = r >= 0 && r < m && c >= 0 && c < n;
    if (!ok) bad[0] = 1;
    keys[e] = ok ? static_cast<uint64_t>(r * n + c) : 0;
    perm[e] = static_cast<int32_t>(e);
}

// head[e] = 1 where a run of equal sorted keys starts.
__global__ void coo_heads_kernel(const uint64_t* __restrict__ keys, int64_t nnz, int32_t* __restrict__ head) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    head[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1 : 0;
}

// Run starts and unique keys at their places; the run count.
__global__ void coo_runs_kernel(const uint64_t* __restrict__ keys, const int32_t* __restrict__ head,
                                const int32_t* __restrict__ place, int64_t nnz,
                                int64_t* __restrict__ start, uint64_t* __restrict__ ukeys,
                                int64_t* __restrict__ nruns) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    if (head[e]) {
        start[place[e]] = e;
        ukeys[place[e]] = keys[e];
    }
    if (e == nnz - 1) nruns[0] = static_cast<int64_t>(place[e]) + head[e];
}

// CSR arrays: run u's values summed in sorted order, its column, and the row starts.
__global__ void coo_finish_kernel(const int64_t* __restrict__ start, const uint64_t* __restrict__ ukeys,
                                  const int32_t* __restrict__ perm, const double* __restrict__ val,
                                  const int64_t* __restrict__ nruns_p, int64_t nnz, int64_t m,
                                  int64_t n, int64_t* __restrict__ rowptr, int32_t* __restrict__ colind,
                                  double* __restrict__ out_val) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nruns = nruns_p[0];
    if (t < nruns) {
        const int64_t e1 = t + 1 < nruns ? start[t + 1] : nnz;
        double acc = 0.0;
        for (int64_t e = start[t]; e < e1; ++e) acc += val[perm[e]];
        out_val[t] = acc;
        colind[t] = static_cast<int32_t>(ukeys[t] % n);
    }
    if (t <= m) {   // first run whose row is >= t
        const uint64_t key = static_cast<uint64_t>(t * n);
        int64_t lo = 0, hi = nruns;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ukeys[mid] < key) lo = mid + 1; else hi = mid;
        }
        rowptr[t] = lo;
    }
}

struct CooLayout {
    size_t keys_in, keys_out, perm_in, perm_out, head, place, start, ukeys, nruns, bad, temp,
        temp_bytes, total;
};

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

static int key_bits(int64_t m, int64_t n) {
    const uint64_t top = static_cast<uint64_t>(m) * static_cast<uint64_t>(n);
    int bits = 1;
    while (bits < 64 && (uint64_t(1) << bits) < top) ++bits;
    return bits;
}

CooLayout coo_layout(int64_t m, int64_t n, int64_t nnz) {
    CooLayout L{};
    const int cnt = static_cast<int>(nnz > 0 ? nnz : 1);
    size_t sort_bytes = 0, scan_bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, static_cast<const uint64_t*>(nullptr),
                                       static_cast<uint64_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                                       static_cast<int32_t*>(nullptr), cnt, 0, key_bits(m, n));
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, static_cast<const int32_t*>(nullptr),
                                     static_cast<int32_t*>(nullptr), cnt);
    const size_t tb = (sort_bytes > scan_bytes ? sort_bytes : scan_bytes) + 256;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.keys_in = take(sizeof(uint64_t) * cnt);
    L.keys_out = take(sizeof(uint64_t) * cnt);
    L.perm_in = take(sizeof(int32_t) * cnt);
    L.perm_out = take(sizeof(int32_t) * cnt);
    L.head = take(sizeof(int32_t) * cnt);
    L.place = take(sizeof(int32_t) * cnt);
    L.start = take(sizeof(int64_t) * cnt);
    L.ukeys = take(sizeof(uint64_t) * cnt);
    L.nruns = take(sizeof(int64_t));
    L.bad = take(sizeof(int));
    L.temp = take(tb);
    L.temp_bytes = tb;
    L.total = off;
    return L;
}

size_t coo_bytes(int64_t m, int64_t n, int64_t nnz) { return coo_layout(m, n, nnz).total; }

// The run count (the CSR nnz) and the bad-index flag that coo_to_csr leaves in ws.
void coo_counts(int64_t m, int64_t n, int64_t nnz, char* ws, const int64_t** nruns, const int** bad) {
    const CooLayout L = coo_layout(m, n, nnz);
    *nruns = reinterpret_cast<const int64_t*>(ws + L.nruns);
    *bad = reinterpret_cast<const int*>(ws + L.bad);
}

hipError_t coo_to_csr(const int32_t* row, const int32_t* col, const double* val, int64_t m, int64_t n,
                      int64_t nnz, char* ws, int64_t* rowptr, int32_t* colind, double* out_val,
                      hipStream_t s) {
    const CooLayout L = coo_layout(m, n, nnz);
    uint64_t* keys_in = reinterpret_cast<uint64_t*>(ws + L.keys_in);
    uint64_t* keys_out = reinterpret_cast<uint64_t*>(ws + L.keys_out);
    int32_t* perm_in = reinterpret_cast<int32_t*>(ws + L.perm_in);
    int32_t* perm_out = reinterpret_cast<int32_t*>(ws + L.perm_out);
    int32_t* head = reinterpret_cast<int32_t*>(ws + L.head);
    int32_t* place = reinterpret_cast<int32_t*>(ws + L.place);
    int64_t* start = reinterpret_cast<int64_t*>(ws + L.start);
    uint64_t* ukeys = reinterpret_cast<uint64_t*>(ws + L.ukeys);
    int64_t* nruns = reinterpret_cast<int64_t*>(ws + L.nruns);
    int* bad = reinterpret_cast<int*>(ws + L.bad);
    hipError_t e = launch_fill_int(bad, 1, 0, s);
    if (e != hipSuccess) return e;
    if (nnz == 0) {
        e = launch_fill_int(reinterpret_cast<int*>(nruns), 2, 0, s);
        if (e != hipSuccess) return e;
    } else {
        const unsigned g = static_cast<unsigned>(cdiv(nnz, 256));
        hipLaunchKernelGGL(coo_keys_kernel, dim3(g), dim3(256), 0, s, row, col, nnz, m, n, keys_in, perm_in,
                           bad);
        size_t tb = L.temp_bytes;
        e = hipcub::DeviceRadixSort::SortPairs(ws + L.temp, tb, keys_in, keys_out, perm_in, perm_out,
                                               static_cast<int>(nnz), 0, key_bits(m, n), s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(coo_heads_kernel, dim3(g), dim3(256), 0, s, keys_out, nnz, head);
        tb = L.temp_bytes;
        e = hipcub::DeviceScan::ExclusiveSum(ws + L.temp, tb, head, place, static_cast<int>(nnz), s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(coo_runs_kernel, dim3(g), dim3(256), 0, s, keys_out, head, place, nnz, start,
                           ukeys, nruns);
    }
    const int64_t cnt = (nnz > m + 1 ? nnz : m + 1);
    hipLaunchKernelGGL(coo_finish_kernel, dim3(static_cast<unsigned>(cdiv(cnt, 256))), dim3(256), 0, s, start,
                       ukeys, perm_out, val, nruns, nnz, m, n, rowptr, colind, out_val);
    return hipGetLastError();
}

}  // namespace qb
