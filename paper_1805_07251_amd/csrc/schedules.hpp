// The tile schedules of the plain sweep: tile shape, non-temporal stores and
// minimum waves per SIMD of each k_sweep instantiation the autotuner can pick.
#pragma once

#include "internal.hpp"

namespace vdwlb {

// Tile schedules of the sweep (TX x TY sites per workgroup, non-temporal
// stores, minimum waves per SIMD, rows of sites per thread); the autotuner
// picks one per plan.
#define VDWLB_SCHEDULES(X)        \
    X(0, 64, 4, true, 0, 1)       \
    X(1, 64, 8, true, 0, 1)       \
    X(2, 32, 8, true, 0, 1)       \
    X(3, 64, 16, true, 0, 1)      \
    X(4, 128, 4, true, 0, 1)      \
    X(5, 32, 16, true, 0, 1)      \
    X(6, 32, 32, true, 0, 1)      \
    X(7, 128, 8, true, 0, 1)      \
    X(8, 64, 8, false, 0, 1)      \
    X(9, 32, 16, false, 0, 1)     \
    X(10, 64, 16, false, 0, 1)    \
    X(11, 16, 16, true, 0, 1)     \
    X(12, 64, 8, true, 8, 1)      \
    X(13, 64, 16, true, 8, 1)     \
    X(14, 64, 16, true, 0, 2)     \
    X(15, 64, 32, true, 0, 4)     \
    X(16, 32, 32, true, 0, 2)     \
    X(17, 128, 16, true, 0, 4)    \
    X(18, 64, 16, true, 6, 2)     \
    X(19, 32, 32, true, 6, 2)

#define VDWLB_SCHED_ENTRY(i, tx, ty, nt, occ, ry) {tx, ty, nt, occ, ry},
constexpr Schedule SCHEDULES[] = {VDWLB_SCHEDULES(VDWLB_SCHED_ENTRY)};
#undef VDWLB_SCHED_ENTRY
constexpr int N_SCHEDULES = sizeof(SCHEDULES) / sizeof(SCHEDULES[0]);

}  // namespace vdwlb
