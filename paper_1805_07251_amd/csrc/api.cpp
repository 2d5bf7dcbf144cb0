// C-ABI of the vdwlb library: plans, validation, kernel dispatch, hipGraph
// replay of long step sequences, the schedule autotuner and the sticky
// device error flag.  Declarations and the contract are in include/vdwlb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/vdwlb.h"
#include "internal.hpp"

using namespace vdwlb;

namespace {

thread_local char g_last_error[256] = "";

vdwlb_status dev_fail(hipError_t e, const char* where) {
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s", where, hipGetErrorString(e));
    return VDWLB_E_DEVICE;
}

#define HIP_TRY(expr)                                            \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return dev_fail(e_, #expr);        \
    } while (0)

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace

namespace vdwlb {

int32_t set_device_error(hipError_t e, const char* where) { return dev_fail(e, where); }

// Sites per velocity plane of a plain plan's state: nx ny rounded up to 64,
// and for D2Q9, when that leaves the byte stride between planes a multiple
// of PLANE_ALIAS, about PLANE_PAD_BYTES more (whole multiples of 64 sites).
// A D2Q9 sweep streams nine planes in and nine out at the same site offsets;
// with a stride of a large power of two all eighteen streams meet the memory
// interleave at the same phase.  Measured on 2048^2 with 2 components:
// FP64 212 -> 208.6-210 us per step, FP32 121.5 -> 113-115 us; 1024^2 with
// 4 components in FP32 61.5 -> 58.5 us.  The D1Q3 line (three planes each
// way) gains nothing and keeps the plain stride.
constexpr int64_t PLANE_ALIAS = 8192, PLANE_PAD_BYTES = 5120;
int64_t plan_plane(int64_t n, int C, int dtype, int dim) {
    const int64_t site = (int64_t)C * (dtype == VDWLB_F64 ? 8 : 4);
    int64_t plane = (n + 63) / 64 * 64;
    if (dim == 2 && plane * site % PLANE_ALIAS == 0) plane += (PLANE_PAD_BYTES / site + 63) / 64 * 64;
    return plane;
}

// Every rule of vdwlb_desc, checked on host data only.
int32_t validate_desc(const vdwlb_desc* d) {
    if (!d) return VDWLB_E_INVALID_ARG;
    const int C = d->ncomp;
    if (d->nx < 1 || d->ny < 1 || C < 1) return VDWLB_E_INVALID_ARG;
    if ((int64_t)d->nx * d->ny > (int64_t)1 << 28) return VDWLB_E_INVALID_ARG;
    if (d->dim != 1 && d->dim != 2) return VDWLB_E_INVALID_ARG;
    if (d->dtype != VDWLB_F64 && d->dtype != VDWLB_F32) return VDWLB_E_INVALID_ARG;
    if (C <= VDWLB_MAX_COMPONENTS) {  // kernels address a plane with 32-bit byte offsets
        const int64_t plane = plan_plane((int64_t)d->nx * d->ny, C, d->dtype, d->dim);
        if (plane * C * (d->dtype == VDWLB_F64 ? 8 : 4) > (int64_t)0xffffffff) return VDWLB_E_INVALID_ARG;
    }
    if (d->force != VDWLB_FORCE_LOG && d->force != VDWLB_FORCE_NID) return VDWLB_E_INVALID_ARG;
    if (!(d->tau > 0.5) || !is_finite(d->tau)) return VDWLB_E_INVALID_ARG;
    if (!(d->kT > 0) || !is_finite(d->kT) || !is_finite(d->gamma_mu)) return VDWLB_E_INVALID_ARG;
    if (!d->a || !d->b || !d->kappa) return VDWLB_E_INVALID_ARG;
    for (int c = 0; c < C; ++c) {
        if (!(d->b[c] > 0) || !is_finite(d->b[c])) return VDWLB_E_INVALID_ARG;
        for (int e = 0; e < C; ++e) {
            const int64_t ce = (int64_t)c * C + e, ec = (int64_t)e * C + c;
            const double a = d->a[ce], k = d->kappa[ce];
            if (!is_finite(a) || !is_finite(k)) return VDWLB_E_INVALID_ARG;
            if (a != d->a[ec] || k != d->kappa[ec]) return VDWLB_E_INVALID_ARG;
            if (d->lambda) {
                const double l = d->lambda[ce];
                if (c != e && (!is_finite(l) || l < 0 || l != d->lambda[ec])) return VDWLB_E_INVALID_ARG;
            }
        }
    }
    if (d->dim == 1 && d->ny != 1) return VDWLB_E_INVALID_ARG;  // D1Q3 lattices are nx x 1
    if (C > VDWLB_MAX_COMPONENTS) return VDWLB_E_UNSUPPORTED;
    return VDWLB_OK;
}

// Host part of a plan (no device resources) from a validated description.
vdwlb_plan plan_from_desc(const vdwlb_desc& d) {
    vdwlb_plan p;
    const int C = d.ncomp;
    p.dim = d.dim;
    p.nx = d.nx;
    p.ny = d.ny;
    p.C = C;
    p.dtype = d.dtype;
    p.force = d.force;
    p.kT = d.kT;
    p.tau = d.tau;
    p.gamma = d.gamma_mu;
    p.a.assign(d.a, d.a + C * C);
    p.b.assign(d.b, d.b + C);
    p.kappa.assign(d.kappa, d.kappa + C * C);
    p.lam.assign(C * C, 1.0);
    if (d.lambda)
        for (int i = 0; i < C * C; ++i) p.lam[i] = d.lambda[i];
    for (int c = 0; c < C; ++c) p.lam[c * C + c] = 0.0;
    const int64_t n = (int64_t)d.nx * d.ny;
    p.plane = (n + 63) / 64 * 64;
    p.sched = default_schedule(p);
    return p;
}

}  // namespace vdwlb

extern "C" {

int32_t vdwlb_abi_version(void) { return VDWLB_ABI_VERSION; }

const char* vdwlb_strerror(vdwlb_status s) {
    switch (s) {
        case VDWLB_OK: return "ok";
        case VDWLB_E_INVALID_ARG: return "invalid argument";
        case VDWLB_E_UNSUPPORTED: return "unsupported configuration";
        case VDWLB_E_DEVICE: return "HIP device error";
        case VDWLB_E_UNPHYSICAL: return "unphysical state (rho <= 0, eta >= 1 or non-finite value)";
        case VDWLB_E_CAPACITY: return "request exceeds the fixed capacity of the no-allocation scratch";
        default: return "unknown status";
    }
}

const char* vdwlb_last_device_error(void) { return g_last_error; }

vdwlb_status vdwlb_plan_create(const vdwlb_desc* d, vdwlb_plan** out) {
    if (!out) return VDWLB_E_INVALID_ARG;
    *out = nullptr;
    const vdwlb_status st = validate_desc(d);
    if (st != VDWLB_OK) return st;
    vdwlb_plan* p = new (std::nothrow) vdwlb_plan(plan_from_desc(*d));
    if (!p) return VDWLB_E_DEVICE;
    p->plane = plan_plane((int64_t)d->nx * d->ny, p->C, p->dtype, p->dim);
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc(&p->d_flag, 256);
    if (e == hipSuccess) e = hipMemset(p->d_flag, 0, 256);
    if (e != hipSuccess) {
        if (p->d_flag) (void)hipFree(p->d_flag);
        delete p;
        return dev_fail(e, "plan device buffers");
    }
    *out = p;
    return VDWLB_OK;
}

vdwlb_status vdwlb_plan_destroy(vdwlb_plan* p) {
    if (!p) return VDWLB_OK;
    release_graph(*p);
    release_adjoint_graph(*p);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->d_flag) (void)hipFree(p->d_flag);
    delete p;
    return VDWLB_OK;
}

int64_t vdwlb_plane_elems(const vdwlb_plan* p) { return p ? p->plane : 0; }

size_t vdwlb_state_bytes(const vdwlb_plan* p) {
    if (!p) return 0;
    return (size_t)(p->dim == 1 ? 3 : 9) * p->C * (size_t)p->plane * (p->dtype == VDWLB_F64 ? 8 : 4);
}

vdwlb_status vdwlb_init(vdwlb_plan* p, void* f, const void* rho, const void* mom, void* stream) {
    if (!p || !f || !rho || !state_aligned(*p, f)) return VDWLB_E_INVALID_ARG;
    hipError_t e = launch_init(*p, f, rho, mom, (hipStream_t)stream);
    return e == hipSuccess ? VDWLB_OK : dev_fail(e, "init kernel");
}

vdwlb_status vdwlb_step(vdwlb_plan* p, void* fA, void* fB, int64_t n, void* stream, int32_t* out_which) {
    if (!p || !fA || !fB || fA == fB || n < 0) return VDWLB_E_INVALID_ARG;
    if (!state_aligned(*p, fA) || !state_aligned(*p, fB)) return VDWLB_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int64_t done = 0;
    const int64_t per_graph = 2 * (int64_t)GRAPH_PAIRS;
    if (n >= per_graph && graphs_enabled()) {
        vdwlb_status st = ensure_graph(*p, fA, fB);
        if (st != VDWLB_OK) return st;
        const int64_t reps = n / per_graph;
        for (int64_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(p->graph, s));
        done = reps * per_graph;
    }
    for (int64_t t = done; t < n; ++t) {
        const bool even = (t & 1) == 0;
        hipError_t e = launch_sweep(*p, even ? fA : fB, even ? fB : fA, s);
        if (e != hipSuccess) return dev_fail(e, "sweep kernel");
    }
    if (out_which) *out_which = (int32_t)(n & 1);
    return VDWLB_OK;
}

vdwlb_status vdwlb_sync_status(vdwlb_plan* p, void* stream) {
    if (!p) return VDWLB_E_INVALID_ARG;
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int h = 0;
    HIP_TRY(hipMemcpy(&h, p->d_flag, sizeof h, hipMemcpyDeviceToHost));
    if (h) {
        HIP_TRY(hipMemset(p->d_flag, 0, sizeof h));
        return VDWLB_E_UNPHYSICAL;
    }
    return VDWLB_OK;
}

vdwlb_status vdwlb_moments(vdwlb_plan* p, const void* f, void* rho, void* mom, void* mu, void* pr, void* stream) {
    if (!p || !f || !rho || !state_aligned(*p, f)) return VDWLB_E_INVALID_ARG;
    hipError_t e = launch_moments(*p, f, rho, mom, mu, pr, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(e, "moments kernels");
    return vdwlb_sync_status(p, stream);
}

int32_t vdwlb_schedule_count(const vdwlb_plan* p) { return p ? public_schedule_count(*p) : 0; }

vdwlb_status vdwlb_set_schedule(vdwlb_plan* p, int32_t k) {
    if (!p) return VDWLB_E_INVALID_ARG;
    const int old_s = p->sched, old_m = p->map_mode;
    if (!apply_public_schedule(*p, k)) return VDWLB_E_INVALID_ARG;
    if (old_s != p->sched || old_m != p->map_mode) release_graph(*p);
    return VDWLB_OK;
}

vdwlb_status vdwlb_autotune(vdwlb_plan* p, const void* fA, void* fB, void* stream, int32_t* chosen) {
    if (!p || !fA || !fB || fA == fB) return VDWLB_E_INVALID_ARG;
    if (!state_aligned(*p, fA) || !state_aligned(*p, fB)) return VDWLB_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    // The timing sweeps run on whatever fA holds and may raise the error flag;
    // the flag is restored afterwards so that it still describes the caller's
    // own steps.
    int keep_flag = 0;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(&keep_flag, p->d_flag, sizeof keep_flag, hipMemcpyDeviceToHost));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int64_t sites = (int64_t)p->nx * p->ny;
    const int reps = sites >= (1 << 20) ? 10 : 50;
    const int keep_s = p->sched, keep_m = p->map_mode;
    // Runs alternate between two state buffers, so the timed launches do too:
    // between fB (first a copy of fA) and a temporary buffer.  Reading one
    // input again and again would time lattices of up to half the 256 MB
    // MALL from the cache, not at the rate of a run.  Without the temporary
    // buffer (allocation failed) every launch reads fA.
    const size_t bytes = vdwlb_state_bytes(p);
    void* tmp = nullptr;
    if (hipMalloc(&tmp, bytes) != hipSuccess) {
        tmp = nullptr;
        (void)hipGetLastError();
    }
    int parity = 0;
    auto launch = [&]() -> hipError_t {
        if (!tmp) return launch_sweep(*p, fA, fB, s);
        const bool odd = (parity++ & 1) != 0;
        return odd ? launch_sweep(*p, tmp, fB, s) : launch_sweep(*p, fB, tmp, s);
    };
    hipError_t e = tmp ? hipMemcpyAsync(fB, fA, bytes, hipMemcpyDeviceToDevice, s) : hipSuccess;
    // average launch time of public schedule k over n launches (after 3 warm-up launches)
    auto time_k = [&](int k, int n, float& ms) -> hipError_t {
        apply_public_schedule(*p, k);
        hipError_t e = hipSuccess;
        for (int w = 0; w < 3 && e == hipSuccess; ++w) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < n && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)n;
        return e;
    };
    // first pass over every schedule, then the four fastest again, twice
    // each in alternation, with four times the launches (single short timings
    // of schedules within a few per cent of each other are noise)
    std::vector<std::pair<float, int>> t;
    for (int k = 0; k < public_schedule_count(*p) && e == hipSuccess; ++k) {
        float ms = 0;
        e = time_k(k, reps, ms);
        t.push_back({ms, k});
    }
    std::sort(t.begin(), t.end());
    const int top = (int)std::min<size_t>(4, t.size());
    std::vector<float> acc(top, 0.0f);
    for (int round = 0; round < 2 && e == hipSuccess; ++round)
        for (int j = 0; j < top && e == hipSuccess; ++j) {
            float ms = 0;
            e = time_k(t[j].second, 4 * reps, ms);
            acc[j] += ms;
        }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(p->d_flag, &keep_flag, sizeof keep_flag, hipMemcpyHostToDevice);
    if (tmp) {
        if (e != hipSuccess) (void)hipStreamSynchronize(s);
        (void)hipFree(tmp);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release_graph(*p);
    p->sched = keep_s;
    p->map_mode = keep_m;
    if (e != hipSuccess) return dev_fail(e, "autotune");
    int best_k = -1;
    float best = 0;
    for (int j = 0; j < top; ++j)
        if (best_k < 0 || acc[j] < best) {
            best = acc[j];
            best_k = t[j].second;
        }
    if (best_k >= 0) apply_public_schedule(*p, best_k);
    if (chosen) *chosen = best_k;
    return VDWLB_OK;
}

vdwlb_status vdwlb_maxwell(double a, double b, double kT, double* rho_gas, double* rho_liquid) {
    if (!rho_gas || !rho_liquid) return VDWLB_E_INVALID_ARG;
    if (!(a > 0) || !(b > 0) || !(kT > 0)) return VDWLB_E_INVALID_ARG;
    return maxwell_coexistence(a, b, kT, rho_gas, rho_liquid) ? VDWLB_OK : VDWLB_E_INVALID_ARG;
}

vdwlb_status vdwlb_copy(void* dst, const void* src, size_t nbytes, void* stream) {
    if (!dst || !src || nbytes % 16 != 0) return VDWLB_E_INVALID_ARG;
    hipError_t e = launch_copy(dst, src, nbytes, (hipStream_t)stream);
    return e == hipSuccess ? VDWLB_OK : dev_fail(e, "copy kernel");
}

}  // extern "C"
