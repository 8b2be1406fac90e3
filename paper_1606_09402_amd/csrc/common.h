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

// sqrt(x) and 1 / sqrt(x) for a positive normal x: the hardware reciprocal square root
// (about 23 correct bits) refined by two coupled Newton steps of Goldschmidt's iteration,
// g -> sqrt(x) and h -> 1 / (2 sqrt(x)), each step doubling the correct bits.  One short
// dependent chain gives both values (no separate division for 1 / R(j, j)).
QB_DEV void sqrt_and_rsqrt(double x, double& g, double& ir) {
    const double y = __builtin_amdgcn_rsq(x);
    g = x * y;
    double h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    ir = 2.0 * h;
}

// 1 / x for a normal x: the hardware reciprocal refined by two Newton steps (each step
// doubles the correct bits).
QB_DEV double rcp_refined(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

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
