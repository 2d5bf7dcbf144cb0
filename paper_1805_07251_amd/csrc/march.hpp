// The march form of the sweep: every wavefront owns a strip of 60 columns
// (its 64 lanes cover the strip plus two halo columns on each side) and
// walks a chunk of rows, one row per iteration, with no workgroup barriers:
//   front row y + 2 dir: pull the populations, density into an LDS ring of
//                        five rows;
//   row y + dir:         potential from the density rows y .. y + 2 dir into
//                        an LDS ring of three rows;
//   row y:               gradients and Laplacian from the rings, friction,
//                        collision, store.
// Consecutive chunks march in opposite directions, so two chunks that share a
// boundary read its halo rows at about the same time (both at their start or
// both at their end) and the re-reads hit L2.  The per-site arithmetic is
// that of the tile kernel (same functions and stencil expressions), so the
// results are bit-identical to every other schedule.
#pragma once

#include "sweep.hpp"

namespace vdwlb {

struct MarchGeometry {
    int n_strips;  // strips of 60 columns
    int n_chunks;  // chunks of h rows
    int h;         // rows per chunk
};

constexpr int MARCH_W = 60;  // output columns per wavefront
constexpr int MARCH_RL = 66; // LDS row length: 64 lanes plus one pad element on each side

// Stencils on three LDS rows given by pointers (y-1, y, y+1); expressions are
// identical to lap9s / grad9s.
template <typename T>
__device__ __forceinline__ T lap9r(const T* dn, const T* r0, const T* up, int e) {
    const T axis = (r0[e + 1] + r0[e - 1]) + (up[e] + dn[e]);
    const T diag = (up[e + 1] + up[e - 1]) + (dn[e - 1] + dn[e + 1]);
    return (T(4) * axis + diag - T(20) * r0[e]) * T(1.0 / 6.0);
}

template <typename T>
__device__ __forceinline__ void grad9r(const T* dn, const T* r0, const T* up, int e, T& gx, T& gy) {
    const T ne = up[e + 1], nw = up[e - 1], sw = dn[e - 1], se = dn[e + 1];
    gx = (T(4) * (r0[e + 1] - r0[e - 1]) + ((ne - nw) + (se - sw))) * T(1.0 / 12.0);
    gy = (T(4) * (up[e] - dn[e]) + ((ne + nw) - (sw + se))) * T(1.0 / 12.0);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int slot5(int y) { return ((y % 5) + 5) % 5; }
__device__ __forceinline__ int slot3(int y) { return ((y % 3) + 3) % 3; }

// KEEP: hold the pulled populations of the two rows between front and
// collision in registers (three sets); otherwise pull them again for the
// collision (the second read hits L2).
template <typename T, int C, int NW, bool KEEP, bool TAU1>
__global__ void __launch_bounds__(64 * NW) k_march(const T* __restrict__ fin, T* __restrict__ fout, Geometry g,
                                                    MarchGeometry mg, Coeffs<C> k, int* __restrict__ flag) {
    constexpr int RL = MARCH_RL;
    // per wave: density ring 5 rows x C, potential ring 3 rows x C
    __shared__ T s_mem[NW][(5 + 3) * C * RL];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T* ring_rho = s_mem[wave];
    T* ring_phi = s_mem[wave] + 5 * C * RL;

    // XCD-aware: contiguous ranges of workgroups per XCD, chunk rows outer
    const int nwg = gridDim.x, b = blockIdx.x;
    const int xcd = b & 7, kk = b >> 3;
    const int q = nwg >> 3, rr = nwg & 7;
    const int wg = xcd * q + (xcd < rr ? xcd : rr) + kk;
    const int item = wg * NW + wave;
    if (item >= mg.n_strips * mg.n_chunks) return;
    const int cy = item / mg.n_strips, sx = item - cy * mg.n_strips;
    const int x0 = sx * MARCH_W;
    const int ya = cy * mg.h;
    const int yb = min(ya + mg.h, g.ny);
    const int dir = (cy & 1) ? -1 : 1;
    const int r0 = dir > 0 ? ya : yb - 1;
    const int nrows = yb - ya;
    const int xl = wrapc(x0 - 2 + lane, g.nx, g.wrap_general);
    const int e = lane + 1;  // column of this lane in an LDS row
    const bool outl = lane >= 2 && lane < 62 && x0 - 2 + lane < g.nx;

    T P0[C][Q], P1[C][Q];  // pulled populations of rows r and r + dir (KEEP)
    bool bad = false;

    auto rho_row = [&](int y, T (&P)[C][Q]) {
        int o[Q];
        pull_offsets(g, xl, wrapc(y, g.ny, g.wrap_general), o);
        pull<T, C>(fin, g, o, P);
        T* R = ring_rho + slot5(y) * C * RL;
#pragma unroll
        for (int c = 0; c < C; ++c) R[c * RL + e] = density<T>(P[c]);
    };
    // Lanes 0 and 63 read the pad elements of the rows: their potentials
    // are never used, and they are left out of the error flag.
    auto phi_row = [&](int y) {
        const T* D = ring_rho + slot5(y - 1) * C * RL;
        const T* M = ring_rho + slot5(y) * C * RL;
        const T* U = ring_rho + slot5(y + 1) * C * RL;
        T r[C], l[C], ph[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            r[c] = M[c * RL + e];
            l[c] = lap9r<T>(D + c * RL, M + c * RL, U + c * RL, e);
        }
        const bool ok = potential<T, C>(r, l, k, ph);
        if (lane >= 1 && lane < 63) bad |= !ok;
        T* Pp = ring_phi + slot3(y) * C * RL;
#pragma unroll
        for (int c = 0; c < C; ++c) Pp[c * RL + e] = ph[c];
    };

    // prologue: densities of rows r0 - 2 dir .. r0 + dir, potentials of r0 - dir, r0
    {
        T Pt[C][Q];
        rho_row(r0 - 2 * dir, Pt);
        rho_row(r0 - dir, Pt);
    }
    rho_row(r0, P0);
    rho_row(r0 + dir, P1);
    wave_sync();
    phi_row(r0 - dir);
    phi_row(r0);

    for (int i = 0; i < nrows; ++i) {
        const int y = r0 + i * dir;
        T P2[C][Q];
        wave_sync();  // the previous row's LDS reads precede this row's writes
        rho_row(y + 2 * dir, P2);
        wave_sync();
        phi_row(y + dir);
        wave_sync();
        // collision of row y
        T p[C][Q];
        if constexpr (KEEP) {
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int qq = 0; qq < Q; ++qq) p[c][qq] = P0[c][qq];
        } else {
            int o[Q];
            pull_offsets(g, xl, wrapc(y, g.ny, g.wrap_general), o);
            pull<T, C>(fin, g, o, p);
        }
        T rho[C], jx[C], jy[C], gx[C], gy[C], lap[C];
        const int yw = wrapc(y, g.ny, g.wrap_general);
        const T* RD = ring_rho + slot5(y - 1) * C * RL;
        const T* RM = ring_rho + slot5(y) * C * RL;
        const T* RU = ring_rho + slot5(y + 1) * C * RL;
        const T* PD = ring_phi + slot3(y - 1) * C * RL;
        const T* PM = ring_phi + slot3(y) * C * RL;
        const T* PU = ring_phi + slot3(y + 1) * C * RL;
        const int ee = e;  // lanes 0, 1, 62, 63 compute unused values
#pragma unroll
        for (int c = 0; c < C; ++c) {
            rho[c] = density<T>(p[c]);
            momentum<T>(p[c], jx[c], jy[c]);
            T px, py, rx, ry;
            grad9r<T>(PD + c * RL, PM + c * RL, PU + c * RL, ee, px, py);
            grad9r<T>(RD + c * RL, RM + c * RL, RU + c * RL, ee, rx, ry);
            lap[c] = lap9r<T>(RD + c * RL, RM + c * RL, RU + c * RL, ee);
            gx[c] = -rho[c] * px;
            gy[c] = -rho[c] * py;
            if (k.force == 0) {
                gx[c] += T(THETA) * rx;
                gy[c] += T(THETA) * ry;
            }
        }
        if (outl)
            collide_store<T, C, true, TAU1>(p, rho, jx, jy, gx, gy, lap, k, fout, g.plane,
                                            yw * g.nx + (x0 - 2 + lane));
        if constexpr (KEEP) {
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int qq = 0; qq < Q; ++qq) {
                    P0[c][qq] = P1[c][qq];
                    P1[c][qq] = P2[c][qq];
                }
        }
    }
    if (bad) atomicOr(flag, 1);
}

}  // namespace vdwlb
