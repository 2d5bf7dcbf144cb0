// Host-side internals shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/vdwlb.h"

// Captured part of an adjoint segment (the forward recompute or the reverse
// sweep), bound to its step count, buffers and schedule.
struct AdjointGraph {
    hipGraphExec_t exec = nullptr;
    int kind = 0;  // 0: recompute, 1: reverse sweep
    int nsteps = 0, sched = -1, map_mode = -1;
    bool fused = true;
    const void *fbar = nullptr, *ws = nullptr, *pbar = nullptr;
};

struct vdwlb_plan {
    int dim = 2, nx = 0, ny = 0, C = 0, dtype = 0, force = 0;
    double kT = 0, tau = 1, gamma = 1;
    std::vector<double> a, b, kappa, lam;  // row-major C x C (b: C)
    int64_t plane = 0;
    int device = 0;
    int* d_flag = nullptr;  // sticky unphysical-state flag (device)
    int sched = 0;          // tile schedule index
    int map_mode = 0;       // workgroup -> tile order: 0 row-major ranges, 1 vertical XCD bands
    // captured step sequence, bound to one (fA, fB) pair and schedule
    hipGraphExec_t graph = nullptr;
    const void* gA = nullptr;
    const void* gB = nullptr;
    hipStream_t capture_stream = nullptr;
    bool adj_graphs = false;        // replay adjoint recompute / reverse parts from captured graphs
    std::vector<AdjointGraph> adj;  // captured recompute / reverse graphs of up to two workspaces
};

namespace vdwlb {

// Steps per graph replay = 2 * GRAPH_PAIRS (an even count, so every replay
// returns the newest state to the first buffer).
constexpr int GRAPH_PAIRS = 16;

struct Schedule {
    int tx, ty;
    bool nt;
    int occ;
    int ry;  // rows of sites per thread
};

int schedule_count();
Schedule schedule_at(int k);
// Public schedule numbering (D2Q9): tile schedules in row-major XCD order,
// then the same in vertical-band order; D1Q3 plans have their own short list.
int public_schedule_count(const vdwlb_plan& p);

// Alignment the kernels need for a population buffer: the C components of a
// site are one vector access when C is 2 or 4.
inline size_t state_alignment(int C, int dtype) {
    const size_t e = dtype == VDWLB_F64 ? 8 : 4;
    return (C == 2 || C == 4) ? C * e : e;
}
inline bool state_aligned(const vdwlb_plan& p, const void* f) {
    return reinterpret_cast<uintptr_t>(f) % state_alignment(p.C, p.dtype) == 0;
}
bool apply_public_schedule(vdwlb_plan& p, int k);
int default_schedule(const vdwlb_plan& p);
bool graphs_enabled();
void release_adjoint_graph(vdwlb_plan& p);

// mom: null, or [C][N] densities then [C][2][N] momenta of the pulled state
// (D2Q9 plans only).
hipError_t launch_sweep(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom = nullptr);
hipError_t launch_init(const vdwlb_plan& p, void* f, const void* rho, const void* mom, hipStream_t s);
hipError_t launch_moments(const vdwlb_plan& p, const void* f, void* rho, void* mom, void* mu, void* pr,
                          hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t nbytes, hipStream_t s);

int32_t ensure_graph(vdwlb_plan& p, const void* fA, const void* fB);
void release_graph(vdwlb_plan& p);

bool maxwell_coexistence(double a, double b, double kT, double* rho_gas, double* rho_liquid);

int32_t validate_desc(const vdwlb_desc* d);
vdwlb_plan plan_from_desc(const vdwlb_desc& d);
int32_t set_device_error(hipError_t e, const char* where);

}  // namespace vdwlb
