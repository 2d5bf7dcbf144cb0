// Runtime pieces of the library: schedule table, dispatch by precision and
// component count, init / moments / copy launches, hipGraph capture of step
// sequences, and the host-side Maxwell construction helper.
#include <cmath>
#include <cstdlib>

#include "../../include/vdwlb.h"
#include "launch.hpp"

namespace vdwlb {

int schedule_count() { return N_SCHEDULES; }
Schedule schedule_at(int k) { return SCHEDULES[k]; }

int public_schedule_count(const vdwlb_plan& p) { return p.dim == 1 ? N_SCHEDULES1 : 2 * N_SCHEDULES; }

bool apply_public_schedule(vdwlb_plan& p, int k) {
    if (k < 0 || k >= public_schedule_count(p)) return false;
    if (p.dim == 1) {
        p.sched = k;
        p.map_mode = 0;
        return true;
    }
    p.sched = k % N_SCHEDULES;
    p.map_mode = k / N_SCHEDULES;
    return true;
}

int default_schedule(const vdwlb_plan& p) {
    return p.dim == 1 ? 0 : 1;  // 256 sites / 64 x 8 tiles, non-temporal stores
}

bool graphs_enabled() {
    const char* v = std::getenv("VDWLB_NO_GRAPH");
    return !(v && v[0] == '1');
}

hipError_t launch_sweep(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom) {
    return p.dtype == VDWLB_F64 ? launch_sweep_f64(p, fin, fout, s, mom) : launch_sweep_f32(p, fin, fout, s, mom);
}

namespace {

template <typename T, int C>
hipError_t init_c(const vdwlb_plan& p, void* f, const void* rho, const void* mom, hipStream_t s) {
    if (p.dim == 1) {
        const Geometry1 g1 = make_geometry1(p, 256);
        hipLaunchKernelGGL((k_init1<T, C>), dim3((p.nx + 255) / 256), dim3(256), 0, s, (T*)f, (const T*)rho,
                           (const T*)mom, g1);
        return hipGetLastError();
    }
    const Geometry g = make_geometry(p, 64, 1);
    const int n = p.nx * p.ny;
    hipLaunchKernelGGL((k_init<T, C>), dim3((n + 255) / 256), dim3(256), 0, s, (T*)f, (const T*)rho,
                       (const T*)mom, g);
    return hipGetLastError();
}

template <typename T, int C>
hipError_t moments_c(const vdwlb_plan& p, const void* f, void* rho, void* mom, void* mu, void* pr, hipStream_t s) {
    if (p.dim == 1) {
        const Geometry1 g1 = make_geometry1(p, 256);
        const unsigned nb = (unsigned)((p.nx + 255) / 256);
        hipLaunchKernelGGL((k_moments1<T, C>), dim3(nb), dim3(256), 0, s, (const T*)f, (T*)rho, (T*)mom, g1);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || (!mu && !pr)) return e;
        hipLaunchKernelGGL((k_mu_p1<T, C>), dim3(nb), dim3(256), 0, s, (const T*)rho, (T*)mu, (T*)pr, g1,
                           make_coeffs<C, T>(p), p.d_flag);
        return hipGetLastError();
    }
    const Geometry g = make_geometry(p, 64, 1);
    const int n = p.nx * p.ny;
    hipLaunchKernelGGL((k_moments<T, C>), dim3((n + 255) / 256), dim3(256), 0, s, (const T*)f, (T*)rho, (T*)mom,
                       g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || (!mu && !pr)) return e;
    hipLaunchKernelGGL((k_mu_p<T, C>), dim3((n + 255) / 256), dim3(256), 0, s, (const T*)rho, (T*)mu, (T*)pr, g,
                       make_coeffs<C, T>(p), p.d_flag);
    return hipGetLastError();
}

template <typename T>
hipError_t init_t(const vdwlb_plan& p, void* f, const void* rho, const void* mom, hipStream_t s) {
    switch (p.C) {
        case 1: return init_c<T, 1>(p, f, rho, mom, s);
        case 2: return init_c<T, 2>(p, f, rho, mom, s);
        case 3: return init_c<T, 3>(p, f, rho, mom, s);
        case 4: return init_c<T, 4>(p, f, rho, mom, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t moments_t(const vdwlb_plan& p, const void* f, void* rho, void* mom, void* mu, void* pr, hipStream_t s) {
    switch (p.C) {
        case 1: return moments_c<T, 1>(p, f, rho, mom, mu, pr, s);
        case 2: return moments_c<T, 2>(p, f, rho, mom, mu, pr, s);
        case 3: return moments_c<T, 3>(p, f, rho, mom, mu, pr, s);
        case 4: return moments_c<T, 4>(p, f, rho, mom, mu, pr, s);
        default: return hipErrorInvalidValue;
    }
}

// Streaming copy: one 16-byte vector per thread with non-temporal loads and
// stores (the fastest plain copy form measured on the target).
__global__ void __launch_bounds__(256) k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 v;
    v.x = __builtin_nontemporal_load(&src[i].x);
    v.y = __builtin_nontemporal_load(&src[i].y);
    v.z = __builtin_nontemporal_load(&src[i].z);
    v.w = __builtin_nontemporal_load(&src[i].w);
    __builtin_nontemporal_store(v.x, &dst[i].x);
    __builtin_nontemporal_store(v.y, &dst[i].y);
    __builtin_nontemporal_store(v.z, &dst[i].z);
    __builtin_nontemporal_store(v.w, &dst[i].w);
}

}  // namespace

hipError_t launch_init(const vdwlb_plan& p, void* f, const void* rho, const void* mom, hipStream_t s) {
    return p.dtype == VDWLB_F64 ? init_t<double>(p, f, rho, mom, s) : init_t<float>(p, f, rho, mom, s);
}

hipError_t launch_moments(const vdwlb_plan& p, const void* f, void* rho, void* mom, void* mu, void* pr,
                          hipStream_t s) {
    return p.dtype == VDWLB_F64 ? moments_t<double>(p, f, rho, mom, mu, pr, s)
                                : moments_t<float>(p, f, rho, mom, mu, pr, s);
}

hipError_t launch_copy(void* dst, const void* src, size_t nbytes, hipStream_t s) {
    const size_t n = nbytes / 16;
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n);
    return hipGetLastError();
}

void release_graph(vdwlb_plan& p) {
    if (p.graph) (void)hipGraphExecDestroy(p.graph);
    p.graph = nullptr;
    p.gA = p.gB = nullptr;
}

// Capture 2 * GRAPH_PAIRS steps fA -> fB -> fA ... on a private stream (the
// caller's stream may be the null stream, which cannot be captured); the
// graph is then launched on the caller's stream.
int32_t ensure_graph(vdwlb_plan& p, const void* fA, const void* fB) {
    if (p.graph && p.gA == fA && p.gB == fB) return VDWLB_OK;
    release_graph(p);
    hipError_t e = hipSuccess;
    if (!p.capture_stream) e = hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return VDWLB_E_DEVICE;
    e = hipStreamBeginCapture(p.capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return VDWLB_E_DEVICE;
    hipError_t le = hipSuccess;
    for (int t = 0; t < 2 * GRAPH_PAIRS && le == hipSuccess; ++t) {
        const bool even = (t & 1) == 0;
        le = launch_sweep(p, even ? fA : fB, const_cast<void*>(even ? fB : fA), p.capture_stream);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p.capture_stream, &g);
    if (le != hipSuccess || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return VDWLB_E_DEVICE;
    }
    e = hipGraphInstantiate(&p.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        p.graph = nullptr;
        return VDWLB_E_DEVICE;
    }
    p.gA = fA;
    p.gB = fB;
    return VDWLB_OK;
}

// Liquid-gas coexistence of one van der Waals component: equal chemical
// potential and equal pressure (Sec. II) solved by Newton in (rho_g, rho_l),
// started on the outer branches of the isotherm at the mean of the two
// spinodal pressures.
bool maxwell_coexistence(double a, double b, double kT, double* rg_out, double* rl_out) {
    const double kTc = 8.0 * a / (27.0 * b), rc = 1.0 / (3.0 * b);
    if (!(kT < kTc)) return false;
    auto mu = [&](double r) { return kT * (std::log(r / (1 - b * r)) + b * r / (1 - b * r)) - 2 * a * r; };
    auto dmu = [&](double r) { return kT / (r * (1 - b * r) * (1 - b * r)) - 2 * a; };
    auto pr = [&](double r) { return r * kT / (1 - b * r) - a * r * r; };
    auto dpr = [&](double r) { return kT / ((1 - b * r) * (1 - b * r)) - 2 * a * r; };
    auto root = [](auto fn, double lo, double hi) {
        const bool slo = fn(lo) > 0;
        for (int i = 0; i < 200; ++i) {
            const double m = 0.5 * (lo + hi);
            if ((fn(m) > 0) == slo) lo = m;
            else hi = m;
        }
        return 0.5 * (lo + hi);
    };
    const double s_lo = root(dpr, 1e-12, rc), s_hi = root(dpr, rc, (1 - 1e-12) / b);
    const double pstar = 0.5 * (std::fmax(pr(s_hi), 0.0) + pr(s_lo));
    double rg = root([&](double r) { return pr(r) - pstar; }, 1e-300, s_lo);
    double rl = root([&](double r) { return pr(r) - pstar; }, s_hi, (1 - 1e-15) / b);
    for (int it = 0; it < 100; ++it) {
        const double f1 = mu(rg) - mu(rl), f2 = pr(rg) - pr(rl);
        const double j11 = dmu(rg), j12 = -dmu(rl), j21 = dpr(rg), j22 = -dpr(rl);
        const double det = j11 * j22 - j12 * j21;
        const double dg = (f1 * j22 - f2 * j12) / det, dl = (j11 * f2 - j21 * f1) / det;
        double lam = 1.0;
        while (!(rg - lam * dg > 0 && (rl - lam * dl) * b < 1 && rl - lam * dl > rg - lam * dg) && lam > 1e-12)
            lam *= 0.5;
        rg -= lam * dg;
        rl -= lam * dl;
        if (std::fabs(lam * dg) < 1e-16 * rg && std::fabs(lam * dl) < 1e-16 * rl) break;
    }
    *rg_out = rg;
    *rl_out = rl;
    return std::isfinite(rg) && std::isfinite(rl) && rg > 0 && rl > rg;
}

}  // namespace vdwlb
