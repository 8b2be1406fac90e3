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

}  // namespace qb
