// The tile schedules of the plain sweep: tile shape, non-temporal stores and
// minimum waves per SIMD of each k_sweep instantiation the autotuner can pick.
#pragma once

#include "internal.hpp"

namespace vdwlb {

// Tile schedules of the sweep (TX x TY sites per workgroup, non-temporal
// stores, minimum waves per SIMD); the autotuner picks one per plan.
#define VDWLB_SCHEDULES(X)     \
    X(0, 64, 4, true, 0)       \
    X(1, 64, 8, true, 0)       \
    X(2, 32, 8, true, 0)       \
    X(3, 64, 16, true, 0)      \
    X(4, 128, 4, true, 0)      \
    X(5, 32, 16, true, 0)      \
    X(6, 32, 32, true, 0)      \
    X(7, 128, 8, true, 0)      \
    X(8, 64, 8, false, 0)      \
    X(9, 32, 16, false, 0)     \
    X(10, 64, 16, false, 0)    \
    X(11, 16, 16, true, 0)     \
    X(12, 64, 8, true, 8)      \
    X(13, 64, 16, true, 8)

#define VDWLB_SCHED_ENTRY(i, tx, ty, nt, occ) {tx, ty, nt, occ},
constexpr Schedule SCHEDULES[] = {VDWLB_SCHEDULES(VDWLB_SCHED_ENTRY)};
#undef VDWLB_SCHED_ENTRY
constexpr int N_SCHEDULES = sizeof(SCHEDULES) / sizeof(SCHEDULES[0]);

}  // namespace vdwlb
