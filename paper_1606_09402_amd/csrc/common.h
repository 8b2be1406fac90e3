// Shared definitions for the QB library's HIP sources (device and host).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qb.h"

#define QB_DEV __device__ __forceinline__

typedef double v4d __attribute__((ext_vector_type(4)));

namespace qb {

// Rounded-up integer division for sizes.
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Generic strided view of a matrix operand: element (i, j) at p[i * si + j * sj].
struct View {
    const double* p;
    int64_t si, sj;
};
struct MutView {
    double* p;
    int64_t si, sj;
};

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range
// of logical tiles so that tiles sharing an operand row-slab share one L2.
QB_DEV int xcd_remap(int wg, int nwg) {
    const int xcd = wg & 7, local = wg >> 3;
    const int per = nwg >> 3, rem = nwg & 7;
    return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Logical tile t -> (tile_m, tile_n).  Narrow outputs (at most 16 column tiles) go row by
// row, so the few tiles of a row slab sit next to each other and share the A slab in L2.
// Wide outputs go column by column inside groups of 8 row tiles, so that the workgroups
// resident on one XCD at a time cover a compact block and re-read fewer operand slabs
// (measured with FETCH_SIZE: 1.8x fewer L2 misses at 25 column tiles, more at 4 or 10).
QB_DEV void group_tiles(int t, int tiles_m, int tiles_n, int& tile_m, int& tile_n) {
    if (tiles_n <= 16) {
        tile_m = t / tiles_n;
        tile_n = t % tiles_n;
        return;
    }
    constexpr int GM = 8;
    const int per_group = GM * tiles_n;
    const int grp = t / per_group, r = t % per_group;
    const int m0 = grp * GM;
    const int rows = tiles_m - m0 < GM ? tiles_m - m0 : GM;
    tile_m = m0 + r % rows;
    tile_n = r / rows;
}

}  // namespace qb
