// Host-side launch helpers shared by the per-precision dispatch units.
#pragma once

#include <type_traits>

#include "internal.hpp"
#include "schedules.hpp"
#include "sweep.hpp"
#include "sweep1.hpp"

namespace vdwlb {

inline Geometry make_geometry(const vdwlb_plan& p, int tx, int ty) {
    Geometry g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.plane = p.plane;
    g.tiles_x = (p.nx + tx - 1) / tx;
    // single-step wrapping needs every index to overshoot an extent by less
    // than the extent itself: tile overhang plus a radius-3 reach
    g.wrap_general = (p.nx < tx + 8 || p.ny < ty + 8) ? 1 : 0;
    g.band_w = (p.map_mode == 1 && g.tiles_x % 8 == 0) ? g.tiles_x / 8 : 0;
    return g;
}

// Kernel coefficients in the kernel's own precision R (each value computed in
// double and rounded once); the symmetric matrices keep one triangle.
template <int C, typename R = double>
Coeffs<C, R> make_coeffs(const vdwlb_plan& p) {
    using K = Coeffs<C, R>;
    K k;
    k.kT = R(p.kT);
    k.omega = R(1.0 / p.tau);
    k.cG = R((p.tau - 0.25) / p.tau);
    k.cL = R(1.0 / (12.0 * p.tau));
    k.gamma = R(p.gamma);
    k.lamt[0] = R(0);
    for (int c = 0; c < C; ++c) {
        k.b[c] = R(p.b[c]);
        for (int d = c; d < C; ++d) {
            k.a2t[K::tri(c, d)] = R(2.0 * p.a[c * C + d]);
            k.kapt[K::tri(c, d)] = R(p.kappa[c * C + d]);
            if (d > c) k.lamt[K::off(c, d)] = R(p.lam[c * C + d]);
        }
    }
    k.fk = R(C >= 2 ? 1.0 / (1.0 + 0.5 * p.lam[1]) : 0.0);
    k.force = p.force;
    return k;
}

template <typename T, int C, int TX, int TY, bool NTS, int OCC, bool TAU1, bool MOM, int RY>
void launch_tile(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom, const Geometry& g,
                 const Coeffs<C, T>& k, int tiles) {
    if constexpr (RY == 1)
        hipLaunchKernelGGL((k_sweep<T, C, TX, TY, NTS, OCC, TAU1, MOM>), dim3(tiles), dim3(TX * TY), 0, s,
                           (const T*)fin, (T*)fout, g, k, p.d_flag, (T*)mom);
    else
        hipLaunchKernelGGL((k_sweep_rows<T, C, TX, TY, NTS, OCC, TAU1, MOM, RY>), dim3(tiles), dim3(TX * TY / RY), 0,
                           s, (const T*)fin, (T*)fout, g, k, p.d_flag, (T*)mom);
}

template <typename T, int C, int TX, int TY, bool NTS, int OCC, int RY>
hipError_t run_sweep(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom) {
    const Geometry g = make_geometry(p, TX, TY);
    const Coeffs<C, T> k = make_coeffs<C, T>(p);
    const int tiles = g.tiles_x * ((p.ny + TY - 1) / TY);
    if (mom) {  // the adjoint's recompute: FP64; C > 2 goes through run_sweep_mom_fixed
        if constexpr (std::is_same<T, double>::value && C <= 2) {
            if (p.tau == 1.0)
                launch_tile<T, C, TX, TY, NTS, OCC, true, true, RY>(p, fin, fout, s, mom, g, k, tiles);
            else
                launch_tile<T, C, TX, TY, NTS, OCC, false, true, RY>(p, fin, fout, s, mom, g, k, tiles);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (p.tau == 1.0)
        launch_tile<T, C, TX, TY, NTS, OCC, true, false, RY>(p, fin, fout, s, nullptr, g, k, tiles);
    else
        launch_tile<T, C, TX, TY, NTS, OCC, false, false, RY>(p, fin, fout, s, nullptr, g, k, tiles);
    return hipGetLastError();
}

template <typename T, int C>
hipError_t run_sweep_sched(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom) {
    switch (p.sched) {
#define VDWLB_SCHED_CASE(i, tx, ty, nt, occ, ry) \
    case i: return run_sweep<T, C, tx, ty, nt, occ, ry>(p, fin, fout, s, mom);
        VDWLB_SCHEDULES(VDWLB_SCHED_CASE)
#undef VDWLB_SCHED_CASE
        default: return hipErrorInvalidValue;
    }
}

inline Geometry1 make_geometry1(const vdwlb_plan& p, int tx) {
    Geometry1 g;
    g.nx = p.nx;
    g.plane = p.plane;
    g.wrap_general = p.nx < tx + 8 ? 1 : 0;
    return g;
}

template <typename T, int C, int TX, bool NTS>
hipError_t run_sweep1(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s) {
    const Geometry1 g = make_geometry1(p, TX);
    const Coeffs<C, T> k = make_coeffs<C, T>(p);
    const int tiles = (p.nx + TX - 1) / TX;
    if (p.tau == 1.0)
        hipLaunchKernelGGL((k_sweep1<T, C, TX, NTS, true>), dim3(tiles), dim3(TX), 0, s, (const T*)fin, (T*)fout, g,
                           k, p.d_flag);
    else
        hipLaunchKernelGGL((k_sweep1<T, C, TX, NTS, false>), dim3(tiles), dim3(TX), 0, s, (const T*)fin, (T*)fout, g,
                           k, p.d_flag);
    return hipGetLastError();
}

// The sweep that also writes the moments, for C > 2: one tile shape (every
// schedule gives the same states bit for bit, so the adjoint's recompute
// need not follow the plan's).
template <typename T, int C>
hipError_t run_sweep_mom_fixed(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom) {
    if constexpr (std::is_same<T, double>::value) {
        constexpr int TX = 32, TY = 8;
        const Geometry g = make_geometry(p, TX, TY);
        const Coeffs<C, T> k = make_coeffs<C, T>(p);
        const int tiles = g.tiles_x * ((p.ny + TY - 1) / TY);
        if (p.tau == 1.0)
            launch_tile<T, C, TX, TY, true, 0, true, true, 1>(p, fin, fout, s, mom, g, k, tiles);
        else
            launch_tile<T, C, TX, TY, true, 0, false, true, 1>(p, fin, fout, s, mom, g, k, tiles);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <typename T, int C>
hipError_t run_any(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom) {
    if (p.dim == 1) {
        if (mom) return hipErrorInvalidValue;  // the moments output is a D2Q9 feature
        switch (p.sched) {
#define VDWLB_SCHED1_CASE(i, tx, nt) \
    case i: return run_sweep1<T, C, tx, nt>(p, fin, fout, s);
            VDWLB_SCHEDULES1(VDWLB_SCHED1_CASE)
#undef VDWLB_SCHED1_CASE
            default: return hipErrorInvalidValue;
        }
    }
    if (mom && C > 2) return run_sweep_mom_fixed<T, C>(p, fin, fout, s, mom);
    return run_sweep_sched<T, C>(p, fin, fout, s, mom);
}

template <typename T>
hipError_t run_sweep_typed(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom) {
    switch (p.C) {
        case 1: return run_any<T, 1>(p, fin, fout, s, mom);
        case 2: return run_any<T, 2>(p, fin, fout, s, mom);
        case 3: return run_any<T, 3>(p, fin, fout, s, mom);
        case 4: return run_any<T, 4>(p, fin, fout, s, mom);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_f64(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom);
hipError_t launch_sweep_f32(const vdwlb_plan& p, const void* fin, void* fout, hipStream_t s, void* mom);

}  // namespace vdwlb
