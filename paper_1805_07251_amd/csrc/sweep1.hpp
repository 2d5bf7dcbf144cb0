// D1Q3 form of the sweep: the paper's own one-dimensional scheme (Sec. V).
//
// Velocities v_0 = 0, v_1 = +1, v_2 = -1 with weights 2/3, 1/6, 1/6 (the
// lattice temperature theta = 1/3).  One step at site x:
//   pull      p_0 = f_0(x), p_1 = f_1(x - 1), p_2 = f_2(x + 1);
//   moments   rho^c = p_0 + p_1 + p_2, j^c = p_1 - p_2;
//   potential mu^c of Eq. discreteChemicalPotential with the D1Q3
//             interaction function psi(0) = kappa - a, psi(+-1) = -kappa/2,
//             i.e. -2 a rho - kappa Lap(rho) with Lap g = g(x+1) + g(x-1) - 2 g(x);
//   force     G0 = -rho grad phi (+ theta grad rho for the log form), the
//             central difference grad g = (g(x+1) - g(x-1))/2;
//   friction  the implicit form of Eq. forceFriction (x component only);
//   collision the explicit D1Q3 update of Sec. V: feq of Eq. feq and
//             F_0 = -S, F_+- = (S +- G)/2 with
//             S = 2 G u + [(tau - 1/4) G^2/rho + Lap(rho)/12]/tau.
// State layout as in 2-D with three planes: f_i^c(x) at (i plane + x) C + c.
#pragma once

#include "sweep.hpp"

namespace vdwlb {

constexpr int Q1 = 3;

struct Geometry1 {
    int nx;
    int wrap_general;  // lattice shorter than a tile plus the stencil reach
    int64_t plane;
};

template <typename T, int C>
__device__ __forceinline__ void pull1(const T* __restrict__ f, int64_t plane, int x, int xm, int xp, T (&p)[C][Q1]) {
    T v[C];
    load_site<T, C>(plane_base<T, C>(f, 0, plane), x, v);
#pragma unroll
    for (int c = 0; c < C; ++c) p[c][0] = v[c];
    load_site<T, C>(plane_base<T, C>(f, 1, plane), xm, v);
#pragma unroll
    for (int c = 0; c < C; ++c) p[c][1] = v[c];
    load_site<T, C>(plane_base<T, C>(f, 2, plane), xp, v);
#pragma unroll
    for (int c = 0; c < C; ++c) p[c][2] = v[c];
}

template <typename T>
__device__ __forceinline__ T density1(const T (&p)[Q1]) {
    return (p[0] + p[1]) + p[2];
}

// 3-point Laplacian and central difference (the isotropic D1Q3 stencils
// 6 sum_i w_i (g(x+v_i) - g(x)) and 3 sum_i w_i v_i g(x+v_i)).
template <typename T>
__device__ __forceinline__ T lap3(T gm, T g0, T gp) {
    return (gp + gm) - T(2) * g0;
}
template <typename T>
__device__ __forceinline__ T grad3(T gm, T gp) {
    return (gp - gm) * T(0.5);
}

// Collision of one component at one site (in place on p).  Opposite
// velocities share the even part of feq and F; the rest population comes
// last, from the mass balance f'_0 = rho - f'_+ - f'_- (as in the D2Q9
// collision: its direct form would drop u^2 terms below the rounding step
// with a fixed sign).
template <typename T, bool TAU1>
__device__ __forceinline__ void collide1(T (&p)[Q1], T rho, T ri, T jx, T gx, T lap, T omega, T cG, T cL) {
    const T ux = jx * ri;
    const T S = T(2) * gx * ux + cG * gx * gx * ri + cL * lap;
    const T base = T(1) - T(1.5) * ux * ux;
    const T r1 = T(1.0 / 6.0) * rho;
    const T ev = r1 * (base + T(4.5) * ux * ux), od = T(3) * r1 * ux;
    const T fe = T(0.5) * S, fo = T(0.5) * gx;
    auto out = [&](int i, T feq, T force) {
        if constexpr (TAU1) p[i] = feq + force;
        else p[i] = p[i] + omega * (feq - p[i]) + force;
    };
    out(1, ev + od, fe + fo);
    out(2, ev - od, fe - fo);
    p[0] = rho - (p[1] + p[2]);
}

// Friction, collision and store of one site (x components only: in 1-D the
// momenta and forces have no y part).
template <typename T, int C, bool NTSTORE, bool TAU1, typename R>
__device__ __forceinline__ void collide_store1(T (&p)[C][Q1], const T (&rho)[C], T (&jx)[C], T (&gx)[C],
                                               const T (&lap)[C], const Coeffs<C, R>& k, T* __restrict__ fout,
                                               int64_t plane, int x) {
    T ri[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ri[c] = recip(rho[c]);
    if constexpr (C > 1) {
        T W[C][C];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int d = 0; d < C; ++d) W[c][d] = T(0);
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int d = c + 1; d < C; ++d) W[c][d] = W[d][c] = T(k.lam(c, d)) * recip(ri[c] + ri[d]);
        friction<T, C>(rho, ri, jx, gx, W, T(k.fk));
    }
#pragma unroll
    for (int c = 0; c < C; ++c) collide1<T, TAU1>(p[c], rho[c], ri[c], jx[c], gx[c], lap[c], T(k.omega), T(k.cG), T(k.cL));
#pragma unroll
    for (int i = 0; i < Q1; ++i) {
        T v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = p[c][i];
        store_site<T, C, NTSTORE>(plane_base<T, C>(fout, i, plane), x, v);
    }
}

// The D1Q3 sweep: one workgroup per TX consecutive sites, one thread per
// site.  Phase 1 pulls the site's populations and the densities of a
// radius-2 ring (two sites on each side) into LDS, phase 2 evaluates phi on
// the tile plus one site on each side, phase 3 takes the stencils from LDS,
// applies friction and collision and stores.
template <typename T, int C, int TX, bool NTSTORE, bool TAU1>
__global__ void __launch_bounds__(TX) k_sweep1(const T* __restrict__ fin, T* __restrict__ fout, Geometry1 g,
                                                Coeffs<C, T> k, int* __restrict__ flag) {
    constexpr int EX = TX + 4, MX = TX + 2;
    __shared__ T s_rho[C][EX];
    __shared__ T s_phi[C][MX];
    const int x0 = blockIdx.x * TX, lx = threadIdx.x, x = x0 + lx;
    const int xs = wrapc(x, g.nx, g.wrap_general);

    T p[C][Q1];
    pull1<T, C>(fin, g.plane, xs, wrapc(xs - 1, g.nx, g.wrap_general), wrapc(xs + 1, g.nx, g.wrap_general), p);
    T rho[C], jx[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rho[c] = density1<T>(p[c]);
        jx[c] = p[c][1] - p[c][2];
        if constexpr (TAU1) pin(jx[c]);
        s_rho[c][lx + 2] = rho[c];
    }
    if (lx < 4) {  // ring sites x0 - 2, x0 - 1, x0 + TX, x0 + TX + 1
        const int ex = lx < 2 ? lx : TX + lx;
        const int xr = wrapc(x0 - 2 + ex, g.nx, g.wrap_general);
        T q[C][Q1];
        pull1<T, C>(fin, g.plane, xr, wrapc(xr - 1, g.nx, g.wrap_general), wrapc(xr + 1, g.nx, g.wrap_general), q);
#pragma unroll
        for (int c = 0; c < C; ++c) s_rho[c][ex] = density1<T>(q[c]);
    }
    __syncthreads();

    bool bad = false;
    for (int m = lx; m < MX; m += TX) {
        T r[C], l[C], ph[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            r[c] = s_rho[c][m + 1];
            l[c] = lap3<T>(s_rho[c][m], r[c], s_rho[c][m + 2]);
        }
        bad |= !potential<T, C>(r, l, k, ph);
#pragma unroll
        for (int c = 0; c < C; ++c) s_phi[c][m] = ph[c];
    }
    if (bad) raise_flag(flag);
    __syncthreads();

    if (x >= g.nx) return;
    T gx[C], lap[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const T rm = s_rho[c][lx + 1], r0 = s_rho[c][lx + 2], rp = s_rho[c][lx + 3];
        lap[c] = lap3<T>(rm, r0, rp);
        gx[c] = -rho[c] * grad3<T>(s_phi[c][lx], s_phi[c][lx + 2]);
        if (k.force == 0) gx[c] += T(THETA) * grad3<T>(rm, rp);
    }
    collide_store1<T, C, NTSTORE, TAU1>(p, rho, jx, gx, lap, k, fout, g.plane, x);
}

// f_i^c = f^0_i(rho^c, u^c) (Eq. feq, D1Q3 weights); mom holds [C][2][nx]
// (the y components are ignored).
template <typename T, int C>
__global__ void k_init1(T* __restrict__ f, const T* __restrict__ rho, const T* __restrict__ mom, Geometry1 g) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    T p[C][Q1];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const T r = rho[(int64_t)c * g.nx + x];
        const T jx = mom ? mom[(int64_t)(2 * c) * g.nx + x] : T(0);
#pragma unroll
        for (int i = 0; i < Q1; ++i) p[c][i] = T(0);
        // collide with omega = 1 and no force from p = 0 gives exactly f^0
        collide1<T, false>(p[c], r, T(1) / r, jx, T(0), T(0), T(1), T(0), T(0));
    }
#pragma unroll
    for (int i = 0; i < Q1; ++i) {
        T v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) v[c] = p[c][i];
        store_site<T, C, false>(plane_base<T, C>(f, i, g.plane), x, v);
    }
}

// rho^c and rho^c u^c (x; the y component is written as 0) of the streamed
// populations.
template <typename T, int C>
__global__ void k_moments1(const T* __restrict__ f, T* __restrict__ rho, T* __restrict__ mom, Geometry1 g) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    T p[C][Q1];
    pull1<T, C>(f, g.plane, x, wrapc(x - 1, g.nx, 1), wrapc(x + 1, g.nx, 1), p);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rho[(int64_t)c * g.nx + x] = density1<T>(p[c]);
        if (mom) {
            mom[(int64_t)(2 * c) * g.nx + x] = p[c][1] - p[c][2];
            mom[(int64_t)(2 * c + 1) * g.nx + x] = T(0);
        }
    }
}

// mu^c (Eq. discreteChemicalPotential without the constant kT) and the bulk
// pressure of Sec. II from a 1-D density field.
template <typename T, int C>
__global__ void k_mu_p1(const T* __restrict__ rho, T* __restrict__ mu, T* __restrict__ pr, Geometry1 g, Coeffs<C, T> k,
                        int* __restrict__ flag) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const int xm = wrapc(x - 1, g.nx, 1), xp = wrapc(x + 1, g.nx, 1);
    T r[C], l[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const T* R = rho + (int64_t)c * g.nx;
        r[c] = R[x];
        l[c] = lap3<T>(R[xm], r[c], R[xp]);
    }
    Coeffs<C, T> kk = k;
    kk.gamma = 1.0;
    kk.force = 0;
    T m[C];
    if (!potential<T, C>(r, l, kk, m)) raise_flag(flag);
    if (mu)
#pragma unroll
        for (int c = 0; c < C; ++c) mu[(int64_t)c * g.nx + x] = m[c];
    if (pr) {
        T eta = T(0), tot = T(0), att = T(0);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            eta += T(k.b[c]) * r[c];
            tot += r[c];
#pragma unroll
            for (int d = 0; d < C; ++d) att += T(0.5) * T(k.a2(c, d)) * r[c] * r[d];
        }
        pr[x] = tot * T(k.kT) / (T(1) - eta) - att;
    }
}

// Tile schedules of the D1Q3 sweep (TX sites per workgroup, non-temporal
// stores).
#define VDWLB_SCHEDULES1(X) \
    X(0, 256, true)         \
    X(1, 512, true)         \
    X(2, 1024, true)        \
    X(3, 256, false)
constexpr int N_SCHEDULES1 = 4;

}  // namespace vdwlb
