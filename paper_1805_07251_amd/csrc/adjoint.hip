// Hand-written adjoint (reverse mode) of one sweep step, FP64, C = 1 or 2,
// and the segment driver that recomputes the forward pass from a checkpoint.
//
// Forward step at site x (see the plain sweep): pulled populations p, moments
// rho^c, j^c; L^c = Lap(rho^c); mu^c(rho, L) (Eq. discreteChemicalPotential);
// phi^c = gamma mu^c (log) or gamma mu^c - theta ln rho^c (nid); mean-field
// force G0^c = -rho^c grad phi^c [+ theta grad rho^c for log]; implicit
// friction G = G0 + Gf (Eq. forceFriction); collision
// f'_i = (1 - omega) p_i + omega feq_i(rho, j) + F_i(rho, j, G, L).
//
// Given the cotangent fb' of the new state, the adjoint runs three gathers:
//  A (tile, LDS): recompute phi and G at the site from the stored moments;
//     back-propagate through collision and friction: local density and
//     momentum cotangents, the force cotangent G0b and the Laplacian
//     cotangent of the correction term.
//  B: phib = div(rho G0b) (transpose of the gradient stencil applied to
//     Av = rho G0b, formed where it is read), with log forcing also
//     div(G0b) (for theta grad rho), mub = gamma phib, density cotangent
//     through d mu / d rho, total Laplacian cotangent, and the parameter
//     cotangents (kT, a, b, kappa), summed per tile into a running partial.
//
// The segment's reverse sweep runs A for its last step and then one fused
// kernel per earlier step (k_adj_bca: B and C of step t + 1, A of step t);
// kernels A, B and C separately give the same values bit for bit.
//  C: rhob = local + B part + Lap(Lb) (the Laplacian is self-adjoint); the
//     pulled-population cotangent pb_i = (1 - omega) fb'_i + rhob + jb.v_i
//     is un-streamed: fb_i(x - v_i) = pb_i(x).
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "../../include/vdwlb.h"
#include "launch.hpp"

// Workspace of vdwlb_adjoint_segment_noalloc: a fixed array in this code
// object's static device storage, one copy per device, held until the process
// ends.  In host code its name stands for a host-side shadow, not a device
// address: host code takes the device address of each device's copy from
// hipGetSymbolAddress (scratch_address below) and passes only that to kernels
// and copies.
static __device__ __align__(256) unsigned char scratch[VDWLB_ADJOINT_SCRATCH_BYTES];

namespace vdwlb {
namespace adj {

constexpr int TX = 32, TY = 8;  // tile of the reverse-sweep kernels (A, B, fused)
constexpr int BLK = 256;        // workgroup of the per-site kernels (C, moments adjoint, reduction)
constexpr int NTF = 2 * TX * TY;  // workgroup of the fused kernel: two threads per tile site
static_assert(TX * TY == BLK, "a tile is one workgroup of BLK threads");

// number of parameters in the cotangent vector:
// kT, a^{cd} (c <= d), b^c, kappa^{cd} (c <= d)
__host__ __device__ constexpr int n_params(int C) { return 1 + C * (C + 1) / 2 + C + C * (C + 1) / 2; }
__host__ __device__ constexpr int pair_index(int C, int c, int d) {
    // index of (min(c,d), max(c,d)) in the row-major upper triangle
    return (c <= d) ? c * C - c * (c - 1) / 2 + (d - c) : d * C - d * (d - 1) / 2 + (c - d);
}

// Per-step fields of the reverse sweep.  g0b, lb, rhob_loc and jb exist
// twice, by step parity: the fused kernel of step t reads step t + 1's values
// around its tile while it writes step t's.  Kernel B needs the vectors
// av = rho G0b and (log forcing) bv = G0b around each site; only G0b is kept,
// and av is formed where it is read, as the same single product.
struct Fields {
    const double* rho;  // [C][N] moments of the forward step
    const double* mom;  // [C][2][N]
    double* rhob_loc;   // [C][N]
    double* jb;         // [C][2][N]
    double* g0b;        // [C][2][N] cotangent of the mean-field force G0
    double* lb;         // [C][N] Laplacian cotangent from the collision
    double* rhob_b;     // [C][N]
    double* lb_tot;     // [C][N]
};

// Periodic wrap of an index v that lies within a few sites of [0, n): by one
// compare and select, or by a remainder when the geometry is flagged general
// (extents too small for every index of a tile and its rings to lie within
// one period of [0, n)).
__device__ __forceinline__ int wrapg(int v, int n, int general) {
    if (general) {
        const int r = v % n;
        return r < 0 ? r + n : r;
    }
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Discrete divergence with the gradient stencil: sum_i 3 w_i v_i . V(x + v_i)
// (the transpose of the gradient up to a sign), on global fields.
__device__ __forceinline__ double div9(const double* vx, const double* vy, const Geometry& g, int x, int y) {
    const int xm = wrapg(x - 1, g.nx, g.wrap_general), xp = wrapg(x + 1, g.nx, g.wrap_general), ym = wrapg(y - 1, g.ny, g.wrap_general), yp = wrapg(y + 1, g.ny, g.wrap_general);
    const int r0 = y * g.nx, rm = ym * g.nx, rp = yp * g.nx;
    const double ax = 4.0 * (vx[r0 + xp] - vx[r0 + xm]) + ((vx[rp + xp] - vx[rp + xm]) + (vx[rm + xp] - vx[rm + xm]));
    const double ay = 4.0 * (vy[rp + x] - vy[rm + x]) + ((vy[rp + xp] + vy[rp + xm]) - (vy[rm + xm] + vy[rm + xp]));
    return (ax + ay) * (1.0 / 12.0);
}

// The divergence of av = r V on global fields, each product formed on its
// own (as where av is staged) and combined as in div9.
__device__ __forceinline__ double div9r(const double* r, const double* vx, const double* vy, const Geometry& g, int x,
                                        int y) {
    const int xm = wrapg(x - 1, g.nx, g.wrap_general), xp = wrapg(x + 1, g.nx, g.wrap_general), ym = wrapg(y - 1, g.ny, g.wrap_general), yp = wrapg(y + 1, g.ny, g.wrap_general);
    const int r0 = y * g.nx, rm = ym * g.nx, rp = yp * g.nx;
    auto px = [&](int i) { const double p = r[i] * vx[i]; return p; };
    auto py = [&](int i) { const double p = r[i] * vy[i]; return p; };
    const double a0p = px(r0 + xp), a0m = px(r0 + xm), app = px(rp + xp), apm = px(rp + xm), amp = px(rm + xp),
                 amm = px(rm + xm);
    const double bp0 = py(rp + x), bm0 = py(rm + x), bpp = py(rp + xp), bpm = py(rp + xm), bmm = py(rm + xm),
                 bmp = py(rm + xp);
    const double ax = 4.0 * (a0p - a0m) + ((app - apm) + (amp - amm));
    const double ay = 4.0 * (bp0 - bm0) + ((bpp + bpm) - (bmm + bmp));
    return (ax + ay) * (1.0 / 12.0);
}

// The same divergence on LDS arrays with row stride S (identical arithmetic).
template <int S>
__device__ __forceinline__ double div9s(const double* vx, const double* vy, int ex, int ey) {
    const double* a = vx + ey * S + ex;
    const double* b = vy + ey * S + ex;
    const double ax = 4.0 * (a[1] - a[-1]) + ((a[S + 1] - a[S - 1]) + (a[-S + 1] - a[-S - 1]));
    const double ay = 4.0 * (b[S] - b[-S]) + ((b[S + 1] + b[S - 1]) - (b[-S - 1] + b[-S + 1]));
    return (ax + ay) * (1.0 / 12.0);
}

// Isotropic Laplacian on a global field (the arithmetic of lap9s).
__device__ __forceinline__ double lapg(const double* a, const Geometry& g, int x, int y) {
    const int xm = wrapg(x - 1, g.nx, g.wrap_general), xp = wrapg(x + 1, g.nx, g.wrap_general), ym = wrapg(y - 1, g.ny, g.wrap_general), yp = wrapg(y + 1, g.ny, g.wrap_general);
    const int r0 = y * g.nx, rm = ym * g.nx, rp = yp * g.nx;
    const double axis = (a[r0 + xp] + a[r0 + xm]) + (a[rp + x] + a[rm + x]);
    const double diag = (a[rp + xp] + a[rp + xm]) + (a[rm + xm] + a[rm + xp]);
    return (4.0 * axis + diag - 20.0 * a[r0 + x]) * (1.0 / 6.0);
}

// Small dense LU factorisation in place (no pivoting; the friction matrix is
// symmetric positive definite): the unit lower factor's multipliers below the
// diagonal, the upper factor on and above it.
template <int C>
__device__ __forceinline__ void lu_factor(double (&A)[C][C]) {
#pragma unroll
    for (int p = 0; p < C; ++p) {
        const double ip = 1.0 / A[p][p];
#pragma unroll
        for (int q = p + 1; q < C; ++q) {
            const double f = A[q][p] * ip;
            A[q][p] = f;
#pragma unroll
            for (int m = p + 1; m < C; ++m) A[q][m] -= f * A[p][m];
        }
    }
}

// Solves A x = b in place with the factors of lu_factor.
template <int C>
__device__ __forceinline__ void lu_solve(const double (&LU)[C][C], double (&x)[C]) {
#pragma unroll
    for (int q = 1; q < C; ++q)
#pragma unroll
        for (int p = 0; p < q; ++p) x[q] -= LU[q][p] * x[p];
#pragma unroll
    for (int p = C - 1; p >= 0; --p) {
#pragma unroll
        for (int m = p + 1; m < C; ++m) x[p] -= LU[p][m] * x[m];
        x[p] /= LU[p][p];
    }
}

// (L u)^c = sum_d W^{cd} (u^c - u^d), the graph Laplacian of the friction weights.
template <int C>
__device__ __forceinline__ double graph_laplacian(const double (&W)[C][C], const double (&u)[C], int c) {
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < C; ++d)
        if (d != c) acc += W[c][d] * (u[c] - u[d]);
    return acc;
}

// Local part of the adjoint at one site (collision, friction, force):
// given the incoming cotangent fin of the site's new populations, its forward
// moments (rho, j), the potential gradient (dpx, dpy) and the density gradient
// (rx, ry), the local density and momentum cotangents rb, jb, the vectors
// av = rho G0b, bv = G0b (log forcing; 0 for nid) and the Laplacian cotangent
// lb of the correction term.
template <int C>
__device__ __forceinline__ void adjoint_local(const double (&fin)[C][Q], const double (&rho)[C], const double (&jx)[C],
                                              const double (&jy)[C], const double (&dpx)[C], const double (&dpy)[C],
                                              const double (&rx)[C], const double (&ry)[C], const Coeffs<C>& k,
                                              double (&rb)[C], double (&jbx)[C], double (&jby)[C], double (&gbx_out)[C],
                                              double (&gby_out)[C], double (&lb)[C]) {
    const double omega = k.omega, cG = k.cG, cL = k.cL;
    double g0x[C], g0y[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        g0x[c] = -rho[c] * dpx[c];
        g0y[c] = -rho[c] * dpy[c];
        if (k.force == 0) {
            g0x[c] += THETA * rx[c];
            g0y[c] += THETA * ry[c];
        }
    }
    // forward friction (C = 2 closed form)
    double gx[C], gy[C];
    double m = 0, K = 0, d0x = 0, d0y = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        gx[c] = g0x[c];
        gy[c] = g0y[c];
    }
    double ir[C];
#pragma unroll
    for (int c = 0; c < C; ++c) ir[c] = recip(rho[c]);
    if constexpr (C == 2) {
        m = rho[0] * rho[1] * recip(rho[0] + rho[1]);
        K = k.lam(0, 1) * k.fk;  // lambda / (1 + lambda/2)
        d0x = (jx[1] + 0.5 * g0x[1]) * ir[1] - (jx[0] + 0.5 * g0x[0]) * ir[0];
        d0y = (jy[1] + 0.5 * g0y[1]) * ir[1] - (jy[0] + 0.5 * g0y[0]) * ir[0];
        gx[0] += K * m * d0x;
        gx[1] -= K * m * d0x;
        gy[0] += K * m * d0y;
        gy[1] -= K * m * d0y;
    }
    // C > 2 (Eq. forceFriction): weights W^{cd} = lambda rho^c rho^d / (rho^c + rho^d),
    // graph Laplacian (L u)^c = sum_d W^{cd} (u^c - u^d), A = diag(rho) + L / 2,
    // uh = A^-1 (j + G0 / 2) per axis, G = G0 - L uh.  A is factorised once
    // (LU, no pivoting: it is symmetric positive definite) for both axes and
    // for the transposed solve of the adjoint below.
    double Wf[C][C] = {}, LU[C][C] = {}, uhx[C] = {}, uhy[C] = {};
    if constexpr (C > 2) {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int d = c + 1; d < C; ++d) Wf[c][d] = Wf[d][c] = k.lam(c, d) * rho[c] * rho[d] * recip(rho[c] + rho[d]);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            double diag = rho[c];
#pragma unroll
            for (int d = 0; d < C; ++d)
                if (d != c) {
                    diag += 0.5 * Wf[c][d];
                    LU[c][d] = -0.5 * Wf[c][d];
                }
            LU[c][c] = diag;
        }
        lu_factor<C>(LU);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            uhx[c] = jx[c] + 0.5 * g0x[c];
            uhy[c] = jy[c] + 0.5 * g0y[c];
        }
        lu_solve<C>(LU, uhx);
        lu_solve<C>(LU, uhy);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            gx[c] = g0x[c] - graph_laplacian<C>(Wf, uhx, c);
            gy[c] = g0y[c] - graph_laplacian<C>(Wf, uhy, c);
        }
    }

    // collision adjoint: h = omega [rho M0 + 3 j.M + Q(j)/rho] + 3 G.M
    //                        + [2 G.B.j + cG Q(G)]/rho + cL L tr B
    double gbx[C], gby[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double M0 = 0, Mx = 0, My = 0, Mxx = 0, Myy = 0, Mxy = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double w = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
            const double fb = w * fin[c][i];
            const double vx = VX[i], vy = VY[i];
            M0 += fb;
            Mx += fb * vx;
            My += fb * vy;
            Mxx += fb * vx * vx;
            Myy += fb * vy * vy;
            Mxy += fb * vx * vy;
        }
        const double Bxx = 4.5 * Mxx - 1.5 * M0, Byy = 4.5 * Myy - 1.5 * M0, Bxy = 4.5 * Mxy;
        const double ri = ir[c];
        const double Jx = jx[c], Jy = jy[c], Gx = gx[c], Gy = gy[c];
        const double Qj = Bxx * Jx * Jx + Byy * Jy * Jy + 2.0 * Bxy * Jx * Jy;
        const double QG = Bxx * Gx * Gx + Byy * Gy * Gy + 2.0 * Bxy * Gx * Gy;
        const double BJx = Bxx * Jx + Bxy * Jy, BJy = Bxy * Jx + Byy * Jy;
        const double BGx = Bxx * Gx + Bxy * Gy, BGy = Bxy * Gx + Byy * Gy;
        const double GBJ = Gx * BJx + Gy * BJy;
        rb[c] = omega * (M0 - Qj * ri * ri) - (2.0 * GBJ + cG * QG) * ri * ri;
        jbx[c] = omega * (3.0 * Mx + 2.0 * BJx * ri) + 2.0 * BGx * ri;
        jby[c] = omega * (3.0 * My + 2.0 * BJy * ri) + 2.0 * BGy * ri;
        gbx[c] = 3.0 * Mx + 2.0 * (BJx + cG * BGx) * ri;
        gby[c] = 3.0 * My + 2.0 * (BJy + cG * BGy) * ri;
        lb[c] = cL * (Bxx + Byy);
    }
    // friction adjoint: G = G0 + (+-) K m d0
    double g0bx[C], g0by[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        g0bx[c] = gbx[c];
        g0by[c] = gby[c];
    }
    if constexpr (C == 2) {
        const double gfbx = gbx[0] - gbx[1], gfby = gby[0] - gby[1];
        const double mb = K * (gfbx * d0x + gfby * d0y);
        const double dbx = K * m * gfbx, dby = K * m * gfby;
        const double is = recip(rho[0] + rho[1]), is2 = is * is;
        rb[0] += mb * rho[1] * rho[1] * is2;
        rb[1] += mb * rho[0] * rho[0] * is2;
        // d0 = (j1 + G0_1/2)/rho1 - (j0 + G0_0/2)/rho0, per axis
        const double i0 = ir[0], i1 = ir[1];
        jbx[1] += dbx * i1;
        jbx[0] -= dbx * i0;
        jby[1] += dby * i1;
        jby[0] -= dby * i0;
        g0bx[1] += 0.5 * dbx * i1;
        g0bx[0] -= 0.5 * dbx * i0;
        g0by[1] += 0.5 * dby * i1;
        g0by[0] -= 0.5 * dby * i0;
        rb[1] -= (dbx * (jx[1] + 0.5 * g0x[1]) + dby * (jy[1] + 0.5 * g0y[1])) * i1 * i1;
        rb[0] += (dbx * (jx[0] + 0.5 * g0x[0]) + dby * (jy[0] + 0.5 * g0y[0])) * i0 * i0;
    }
    if constexpr (C > 2) {
        // G = G0 - L uh, uh = A^-1 r, r = j + G0/2, per axis with the cotangent
        // Gb of G: ub = -L Gb, rb = A^-1 ub (A symmetric), jb += rb,
        // G0b = Gb + rb/2; matrix cotangents Ab = -rb uh^T, Lb = -Gb uh^T
        // (both axes), then A = diag(rho) + L/2 and L(W), W(rho).
        double rbx[C], rby[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            rbx[c] = -graph_laplacian<C>(Wf, gbx, c);
            rby[c] = -graph_laplacian<C>(Wf, gby, c);
        }
        lu_solve<C>(LU, rbx);
        lu_solve<C>(LU, rby);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            jbx[c] += rbx[c];
            jby[c] += rby[c];
            g0bx[c] += 0.5 * rbx[c];
            g0by[c] += 0.5 * rby[c];
            // Ab_cc = -(rb_c uh_c) over both axes, into rho^c through diag(rho)
            rb[c] -= rbx[c] * uhx[c] + rby[c] * uhy[c];
        }
        // Lb_ab = -Gb_a uh_b - (rb_a uh_b) / 2; W^{cd} enters L_cc, L_dd with +1
        // and L_cd, L_dc with -1
        auto Lb = [&](int a, int b) {
            return -(gbx[a] * uhx[b] + gby[a] * uhy[b]) - 0.5 * (rbx[a] * uhx[b] + rby[a] * uhy[b]);
        };
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int d = c + 1; d < C; ++d) {
                const double wb = (Lb(c, c) + Lb(d, d)) - (Lb(c, d) + Lb(d, c));
                const double s2 = recip(rho[c] + rho[d]);
                const double lw = k.lam(c, d) * wb * s2 * s2;
                rb[c] += lw * rho[d] * rho[d];
                rb[d] += lw * rho[c] * rho[c];
            }
    }
    // force adjoint, local part: G0 = -rho grad phi (+ theta grad rho)
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rb[c] -= g0bx[c] * dpx[c] + g0by[c] * dpy[c];
        gbx_out[c] = g0bx[c];
        gby_out[c] = g0by[c];
    }
}

// Potential part of the adjoint at one site: given rho, its Laplacian L,
// phib = div(av), dbv = div(bv) (log forcing) and the local Laplacian
// cotangent lb, the density cotangent rhob_b and the total Laplacian
// cotangent lb_tot; with ACC, adds the site's parameter cotangents to acc.
template <int C, bool ACC>
__device__ __forceinline__ void adjoint_potential(const double (&rho)[C], const double (&L)[C], const double (&phib)[C],
                                                  const double (&dbv)[C], const double (&lb)[C], const Coeffs<C>& k,
                                                  double (&rhob_b)[C], double (&lb_tot)[C], double* acc) {
    double mub[C], rb[C];
    double eta = 0, tot = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        eta += k.b[c] * rho[c];
        tot += rho[c];
    }
    const double fv = 1.0 - eta, iv = recip(fv);
    double ir[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        ir[c] = recip(rho[c]);
        mub[c] = k.gamma * phib[c];
        rb[c] = 0.0;
        if (k.force == 0)
            rb[c] -= THETA * dbv[c];
        else
            rb[c] -= THETA * phib[c] * ir[c];
    }
    // d mu^c / d rho^d = kT [delta/rho^c + (b^c + b^d)/(1-eta) + b^c b^d tot/(1-eta)^2] - 2 a^{cd}
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int d = 0; d < C; ++d) {
            double J = k.kT * ((k.b[c] + k.b[d]) * iv + k.b[c] * k.b[d] * tot * iv * iv) - k.a2(c, d);
            if (c == d) J += k.kT * ir[c];
            rb[d] += mub[c] * J;
        }
#pragma unroll
    for (int d = 0; d < C; ++d) {
        double lt = lb[d];
#pragma unroll
        for (int c = 0; c < C; ++c) lt -= mub[c] * k.kap(c, d);
        lb_tot[d] = lt;
        rhob_b[d] = rb[d];
    }
    if constexpr (ACC) {
        // parameter cotangents of mu^c = kT [ln(rho^c/(1-eta)) + b^c tot/(1-eta)]
        //                                 - sum_d (2 a^{cd} rho^d + kappa^{cd} L^d)
        const int oa = 1, ob = 1 + C * (C + 1) / 2, ok = ob + C;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            acc[0] += mub[c] * (dlog(rho[c] * iv) + k.b[c] * tot * iv);
#pragma unroll
            for (int d = 0; d < C; ++d) {
                acc[oa + pair_index(C, c, d)] -= 2.0 * mub[c] * rho[d];
                acc[ok + pair_index(C, c, d)] -= mub[c] * L[d];
            }
#pragma unroll
            for (int e = 0; e < C; ++e) {
                double db = rho[e] * iv + k.b[c] * tot * rho[e] * iv * iv;
                if (e == c) db += tot * iv;
                acc[ob + e] += mub[c] * k.kT * db;
            }
        }
    }
}

// Tree reduction of the per-thread parameter cotangents of a workgroup (NT
// threads, fixed order: at each level h = NT/2, ..., 1 thread t < h adds
// thread t + h's value) into the tile's running partial vector out: with
// accumulate, out + sum, else the sum alone (the segment's first reversed
// step).  The levels that cross wavefronts go through LDS; the last six run
// within wavefront 0 by shuffles, with the same pairs in the same order.
// Every thread must call it.
template <int NP, int NT>
__device__ __forceinline__ void reduce_partial(double (&s_red)[NP][NT], const double (&acc)[NP],
                                               double* __restrict__ out, int accumulate) {
    static_assert(NT % 64 == 0 && NT >= 64, "whole wavefronts");
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NP; ++q) s_red[q][t] = acc[q];
    __syncthreads();
    for (int h = NT / 2; h >= 64; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int q = 0; q < NP; ++q) s_red[q][t] += s_red[q][t + h];
        __syncthreads();
    }
    if (t < 64) {
        double v[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) v[q] = s_red[q][t];
#pragma unroll
        for (int h = 32; h > 0; h >>= 1)
#pragma unroll
            for (int q = 0; q < NP; ++q) v[q] += __shfl_down(v[q], h, 64);
        if (t == 0)
#pragma unroll
            for (int q = 0; q < NP; ++q) out[q] = accumulate ? out[q] + v[q] : v[q];
    }
}

// The same reduction of NT values per entry (already in s_red) by one
// wavefront, lane l = threadIdx.x - first: the LDS levels h = NT/2, ..., 64
// of reduce_partial leave at position l the sum of s_red[.][l + 64 j] over j
// combined in the same pairs, which a lane forms directly from the 64-strided
// values; the shuffle levels follow unchanged.  Needs no barrier, so one
// otherwise idle wavefront can reduce while the others go on.  prev: the
// running partial read earlier (used with accumulate, as in reduce_partial).
template <int NP, int NT>
__device__ __forceinline__ void reduce_partial_wave(const double (&s_red)[NP][NT], int first, const double (&prev)[NP],
                                                    double* __restrict__ out, int accumulate) {
    static_assert(NT % 64 == 0 && NT >= 64, "whole wavefronts");
    constexpr int J = NT / 64;
    const int l = (int)threadIdx.x - first;
    double v[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        double x[J];
#pragma unroll
        for (int j = 0; j < J; ++j) x[j] = s_red[q][l + 64 * j];
#pragma unroll
        for (int h = J / 2; h >= 1; h >>= 1)
#pragma unroll
            for (int j = 0; j < h; ++j) x[j] += x[j + h];
        v[q] = x[0];
    }
#pragma unroll
    for (int h = 32; h > 0; h >>= 1)
#pragma unroll
        for (int q = 0; q < NP; ++q) v[q] += __shfl_down(v[q], h, 64);
    if (l == 0)
#pragma unroll
        for (int q = 0; q < NP; ++q) out[q] = accumulate ? prev[q] + v[q] : v[q];
}

// Tile origin of workgroup b.  Workgroup b runs on XCD b mod 8; when the tile
// count divides by 8 each XCD gets a contiguous range of row-major tiles, so
// the rings a tile reads were written by the same XCD (its L2) except at the
// range's first and last tile rows.  Every launch maps b to the same tile, so a
// tile's running parameter partial stays with its workgroup index.
__device__ __forceinline__ void tile_origin(const Geometry& g, int& x0, int& y0) {
    const int tiles_x = (g.nx + TX - 1) / TX;
    const int n = gridDim.x, b = blockIdx.x;
    const int t = (n % 8 == 0) ? (b & 7) * (n >> 3) + (b >> 3) : b;
    x0 = (t % tiles_x) * TX;
    y0 = (t / tiles_x) * TY;
}

// Writes the local adjoint of one site into the step's fields.
template <int C>
__device__ __forceinline__ void store_local(const Fields& F, int64_t N, int s, const double (&rb)[C],
                                            const double (&jbx)[C], const double (&jby)[C], const double (&gbx)[C],
                                            const double (&gby)[C], const double (&lb)[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
        F.rhob_loc[c * N + s] = rb[c];
        F.jb[(2 * c) * N + s] = jbx[c];
        F.jb[(2 * c + 1) * N + s] = jby[c];
        F.g0b[(2 * c) * N + s] = gbx[c];
        F.g0b[(2 * c + 1) * N + s] = gby[c];
        F.lb[c * N + s] = lb[c];
    }
}

// Stages step t's densities on the tile plus a radius-2 ring (s_rho, row
// stride TX + 4).
template <int C>
__device__ __forceinline__ void stage_rho(const Fields& F, const Geometry& g, int x0, int y0,
                                          double (&s_rho)[C][(TX + 4) * (TY + 4)]) {
    constexpr int EX = TX + 4, EY = TY + 4, NT = TX * TY;
    const int64_t N = (int64_t)g.nx * g.ny;
    for (int e = threadIdx.x; e < EX * EY; e += NT) {
        const int ey = e / EX, ex = e - ey * EX;
        const int s = wrapg(y0 - 2 + ey, g.ny, g.wrap_general) * g.nx + wrapg(x0 - 2 + ex, g.nx, g.wrap_general);
#pragma unroll
        for (int c = 0; c < C; ++c) s_rho[c][e] = F.rho[c * N + s];
    }
}

// The potential phi on the tile plus a radius-1 ring (s_phi, row stride
// TX + 2) from the staged densities.
template <int C>
__device__ __forceinline__ void eval_potential(const Coeffs<C>& k, const double (&s_rho)[C][(TX + 4) * (TY + 4)],
                                               double (&s_phi)[C][(TX + 2) * (TY + 2)]) {
    constexpr int EX = TX + 4, MX = TX + 2, MY = TY + 2, NT = TX * TY;
    for (int m = threadIdx.x; m < MX * MY; m += NT) {
        const int my = m / MX, mx = m - my * MX;
        double r[C], l[C], ph[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            r[c] = s_rho[c][(my + 1) * EX + mx + 1];
            l[c] = lap9s<double, EX>(s_rho[c], mx + 1, my + 1);
        }
        potential<double, C>(r, l, k, ph);
#pragma unroll
        for (int c = 0; c < C; ++c) s_phi[c][m] = ph[c];
    }
}

// Forward moments of site s.
template <int C>
__device__ __forceinline__ void load_moments(const Fields& F, int64_t N, int s, double (&rho)[C], double (&jx)[C],
                                             double (&jy)[C]) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
        rho[c] = F.rho[c * N + s];
        jx[c] = F.mom[(2 * c) * N + s];
        jy[c] = F.mom[(2 * c + 1) * N + s];
    }
}

// Potential and density gradients at interior site (lx, ly) of the tile.
template <int C>
__device__ __forceinline__ void local_stencils(int lx, int ly, const double (&s_rho)[C][(TX + 4) * (TY + 4)],
                                               const double (&s_phi)[C][(TX + 2) * (TY + 2)], double (&dpx)[C],
                                               double (&dpy)[C], double (&rx)[C], double (&ry)[C]) {
    constexpr int EX = TX + 4, MX = TX + 2;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        grad9s<double, MX>(s_phi[c], lx + 1, ly + 1, dpx[c], dpy[c]);
        grad9s<double, EX>(s_rho[c], lx + 2, ly + 2, rx[c], ry[c]);
    }
}

// Kernel A: collision, friction and force adjoint at each site of a tile,
// from the cotangent fbn of the step's new state at the same site.
template <int C>
__global__ void __launch_bounds__(TX* TY) k_adj_a(const double* __restrict__ fbn, Geometry g, Coeffs<C> k,
                                                  Fields F) {
    __shared__ double s_rho[C][(TX + 4) * (TY + 4)];
    __shared__ double s_phi[C][(TX + 2) * (TY + 2)];
    const int64_t N = (int64_t)g.nx * g.ny;
    int x0, y0;
    tile_origin(g, x0, y0);
    stage_rho<C>(F, g, x0, y0, s_rho);
    __syncthreads();
    eval_potential<C>(k, s_rho, s_phi);
    __syncthreads();
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= g.nx || y >= g.ny) return;
    const int s = y * g.nx + x;
    double fin[C][Q];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int i = 0; i < Q; ++i) fin[c][i] = fbn[((int64_t)i * g.plane + s) * C + c];
    double rho[C], jx[C], jy[C], dpx[C], dpy[C], rx[C], ry[C];
    load_moments<C>(F, N, s, rho, jx, jy);
    local_stencils<C>(lx, ly, s_rho, s_phi, dpx, dpy, rx, ry);
    double rb[C], jbx[C], jby[C], gbx[C], gby[C], lb[C];
    adjoint_local<C>(fin, rho, jx, jy, dpx, dpy, rx, ry, k, rb, jbx, jby, gbx, gby, lb);
    store_local<C>(F, N, s, rb, jbx, jby, gbx, gby, lb);
}

// Kernel B: potential adjoint and parameter cotangents of each site of a tile
// (one partial vector per tile, reduced in a fixed order).
template <int C>
__global__ void __launch_bounds__(TX* TY) k_adj_b(Geometry g, Coeffs<C> k, Fields F, double* __restrict__ partial,
                                                  int accumulate) {
    constexpr int NP = n_params(C), NT = TX * TY;
    __shared__ double s_red[NP][NT];
    const int64_t N = (int64_t)g.nx * g.ny;
    int x0, y0;
    tile_origin(g, x0, y0);
    const int x = x0 + (int)threadIdx.x % TX, y = y0 + (int)threadIdx.x / TX;
    double acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[q] = 0.0;
    if (x < g.nx && y < g.ny) {
        const int s = y * g.nx + x;
        double rho[C], L[C], phib[C], dbv[C], lb[C], rbb[C], lbt[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            rho[c] = F.rho[c * N + s];
            L[c] = lapg(F.rho + c * N, g, x, y);
            phib[c] = div9r(F.rho + c * N, F.g0b + (2 * c) * N, F.g0b + (2 * c + 1) * N, g, x, y);
            dbv[c] = k.force == 0 ? div9(F.g0b + (2 * c) * N, F.g0b + (2 * c + 1) * N, g, x, y) : 0.0;
            lb[c] = F.lb[c * N + s];
        }
        adjoint_potential<C, true>(rho, L, phib, dbv, lb, k, rbb, lbt, acc);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            F.lb_tot[c * N + s] = lbt[c];
            F.rhob_b[c * N + s] = rbb[c];
        }
    }
    reduce_partial<NP, NT>(s_red, acc, partial + (int64_t)blockIdx.x * NP, accumulate);
}

// The fused kernel of one reversed step: B and C of step t + 1 and (with
// DO_A) A of step t, on one tile.  Kernel B's outputs are needed by C on the
// tile plus a radius-1 ring (the gather of the un-stream) and, through the
// Laplacian of lb_tot, on a radius-2 ring: B is evaluated there from step
// t + 1's fields staged in LDS on a radius-3 ring (its stencils reach one
// further); ring sites are evaluated by several workgroups with the same
// arithmetic, and only a tile's own sites add to its parameter partial, in
// kernel B's order.  Then C's gather at each site gives the cotangent of
// step t's new state (written to fbo) and, with DO_A, A of step t runs on it
// at once.  Results equal the sequence A, B, C bit for bit.
//
// Two threads per tile site (NTF = 2 TX TY, two wavefronts per SIMD): thread
// t < TX TY owns tile site t (B there, the gather and A), thread TX TY + r
// owns radius-2 ring site r (B there); A's potential on the tile plus a
// radius-1 ring is spread over the threads from the top down, so that no
// thread evaluates more than two sites between the barriers.
template <int C, bool DO_A>
__global__ void __launch_bounds__(NTF) k_adj_bca(const double* __restrict__ fbn, double* __restrict__ fbo,
                                                 Geometry g, Coeffs<C> k, Fields Fn, Fields F,
                                                 double* __restrict__ partial, int accumulate) {
    constexpr int NT = TX * TY, NP = n_params(C);
    constexpr int X3 = TX + 6, Y3 = TY + 6, X2 = TX + 4, Y2 = TY + 4, X1 = TX + 2, Y1 = TY + 2;
    constexpr int RING2 = X2 * Y2 - TX * TY;
    static_assert(RING2 <= NTF - NT, "one radius-2 ring site per thread of the upper half");
    static_assert(X1 * Y1 <= NTF, "one potential site per thread");
    __shared__ double s_av[2 * C][X3 * Y3];  // rho G0b of step t + 1, formed when staged
    __shared__ double s_bv[2 * C][X3 * Y3];  // G0b of step t + 1 (log forcing; 0 for nid)
    __shared__ double s_rn[C][X3 * Y3];      // densities of step t + 1
    __shared__ double s_rbb[C][X2 * Y2];
    __shared__ double s_lbt[C][X2 * Y2];
    __shared__ double s_rb[C][X1 * Y1];
    __shared__ double s_jx[C][X1 * Y1];
    __shared__ double s_jy[C][X1 * Y1];
    __shared__ double s_red[NP][NT];
    __shared__ double s_rho[DO_A ? C : 1][(TX + 4) * (TY + 4)];
    __shared__ double s_phi[DO_A ? C : 1][(TX + 2) * (TY + 2)];
    const int64_t N = (int64_t)g.nx * g.ny;
    int x0, y0;
    tile_origin(g, x0, y0);
    const int t = threadIdx.x;
    const bool own = t < NT;
    const int lx = t % TX, ly = (t % NT) / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool inside = own && x < g.nx && y < g.ny;
    const int xw = wrapg(x, g.nx, g.wrap_general), yw = wrapg(y, g.ny, g.wrap_general);
    const int s = yw * g.nx + xw;  // this thread's tile site (wrapped when outside the lattice)
    // the site of the radius-2 grid this thread evaluates B at
    int bx = lx + 2, by = ly + 2;
    const bool has_b = own || t - NT < RING2;
    if (!own && has_b) ring_coords<TX, TY>(t - NT, bx, by);
    const int b_s = wrapg(y0 - 2 + by, g.ny, g.wrap_general) * g.nx + wrapg(x0 - 2 + bx, g.nx, g.wrap_general);

    // Every global read first, into registers, so that their latencies
    // overlap: step t + 1's fields around the tile, step t's densities around
    // it, the Laplacian cotangent of the site this thread evaluates B at, the
    // cotangents the gather takes from the neighbours and step t's moments at
    // the own site; then the LDS stores.
    constexpr int N3 = (X3 * Y3 + NTF - 1) / NTF, N1 = (X1 * Y1 + NTF - 1) / NTF;
    constexpr int N2 = (X2 * Y2 + NTF - 1) / NTF;
    double v3[N3][3 * C], v1[N1][3 * C], v2[N2][C];
#pragma unroll
    for (int it = 0; it < N3; ++it) {
        const int e = t + it * NTF;
        if (e < X3 * Y3) {
            const int ey = e / X3, ex = e - ey * X3;
            const int q = wrapg(y0 - 3 + ey, g.ny, g.wrap_general) * g.nx + wrapg(x0 - 3 + ex, g.nx, g.wrap_general);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                v3[it][c] = Fn.rho[c * N + q];
                v3[it][C + 2 * c] = Fn.g0b[(2 * c) * N + q];
                v3[it][C + 2 * c + 1] = Fn.g0b[(2 * c + 1) * N + q];
            }
        }
    }
#pragma unroll
    for (int it = 0; it < N1; ++it) {
        const int m = t + it * NTF;
        if (m < X1 * Y1) {
            const int my = m / X1, mx = m - my * X1;
            const int q = wrapg(y0 - 1 + my, g.ny, g.wrap_general) * g.nx + wrapg(x0 - 1 + mx, g.nx, g.wrap_general);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                v1[it][c] = Fn.rhob_loc[c * N + q];
                v1[it][C + 2 * c] = Fn.jb[(2 * c) * N + q];
                v1[it][C + 2 * c + 1] = Fn.jb[(2 * c + 1) * N + q];
            }
        }
    }
    if constexpr (DO_A) {
#pragma unroll
        for (int it = 0; it < N2; ++it) {
            const int e = t + it * NTF;
            if (e < X2 * Y2) {
                const int ey = e / X2, ex = e - ey * X2;
                const int q =
                    wrapg(y0 - 2 + ey, g.ny, g.wrap_general) * g.nx + wrapg(x0 - 2 + ex, g.nx, g.wrap_general);
#pragma unroll
                for (int c = 0; c < C; ++c) v2[it][c] = F.rho[c * N + q];
            }
        }
    }
    double lb_b[C], fb_nb[C][Q], rho[C], jx[C], jy[C], prev[NP];
    // the tile's running partial, for the wavefront that adds to it
#pragma unroll
    for (int q = 0; q < NP; ++q) prev[q] = accumulate && t >= NTF - 64 ? partial[(int64_t)blockIdx.x * NP + q] : 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) lb_b[c] = has_b ? Fn.lb[c * N + b_s] : 0.0;
    if (inside) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int src = wrapg(y + VY[i], g.ny, g.wrap_general) * g.nx + wrapg(x + VX[i], g.nx, g.wrap_general);
            double v[C];
            load_site<double, C>(fbn + (int64_t)i * g.plane * C, src, v);
#pragma unroll
            for (int c = 0; c < C; ++c) fb_nb[c][i] = v[c];
        }
        if constexpr (DO_A) load_moments<C>(F, N, s, rho, jx, jy);
    }
#pragma unroll
    for (int it = 0; it < N3; ++it) {
        const int e = t + it * NTF;
        if (e < X3 * Y3)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double ax = v3[it][c] * v3[it][C + 2 * c];
                const double ay = v3[it][c] * v3[it][C + 2 * c + 1];
                s_rn[c][e] = v3[it][c];
                s_av[2 * c][e] = ax;
                s_av[2 * c + 1][e] = ay;
                s_bv[2 * c][e] = k.force == 0 ? v3[it][C + 2 * c] : 0.0;
                s_bv[2 * c + 1][e] = k.force == 0 ? v3[it][C + 2 * c + 1] : 0.0;
            }
    }
#pragma unroll
    for (int it = 0; it < N1; ++it) {
        const int m = t + it * NTF;
        if (m < X1 * Y1)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                s_rb[c][m] = v1[it][c];
                s_jx[c][m] = v1[it][C + 2 * c];
                s_jy[c][m] = v1[it][C + 2 * c + 1];
            }
    }
    if constexpr (DO_A) {
#pragma unroll
        for (int it = 0; it < N2; ++it) {
            const int e = t + it * NTF;
            if (e < X2 * Y2)
#pragma unroll
                for (int c = 0; c < C; ++c) s_rho[c][e] = v2[it][c];
        }
    }
    __syncthreads();

    // A's potential of step t (site NTF - 1 - t of the radius-1 grid), and B
    // of step t + 1 at this thread's site of the radius-2 grid (with the
    // parameter partial when it is an own site in the lattice)
    if constexpr (DO_A) {
        constexpr int EX = TX + 4, MX = TX + 2;
        const int m = NTF - 1 - t;
        if (m < X1 * Y1) {
            const int my = m / MX, mx = m - my * MX;
            double r[C], l[C], ph[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                r[c] = s_rho[c][(my + 1) * EX + mx + 1];
                l[c] = lap9s<double, EX>(s_rho[c], mx + 1, my + 1);
            }
            potential<double, C>(r, l, k, ph);
#pragma unroll
            for (int c = 0; c < C; ++c) s_phi[c][m] = ph[c];
        }
    }
    double acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[q] = 0.0;
    if (has_b) {
        const int e3 = (by + 1) * X3 + bx + 1, e2 = by * X2 + bx;
        double rn[C], L[C], phib[C], dbv[C], rbb[C], lbt[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            rn[c] = s_rn[c][e3];
            L[c] = lap9s<double, X3>(s_rn[c], bx + 1, by + 1);
            phib[c] = div9s<X3>(s_av[2 * c], s_av[2 * c + 1], bx + 1, by + 1);
            dbv[c] = k.force == 0 ? div9s<X3>(s_bv[2 * c], s_bv[2 * c + 1], bx + 1, by + 1) : 0.0;
        }
        if (inside)
            adjoint_potential<C, true>(rn, L, phib, dbv, lb_b, k, rbb, lbt, acc);
        else
            adjoint_potential<C, false>(rn, L, phib, dbv, lb_b, k, rbb, lbt, nullptr);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            s_rbb[c][e2] = rbb[c];
            s_lbt[c][e2] = lbt[c];
        }
    }
    if (own)
#pragma unroll
        for (int q = 0; q < NP; ++q) s_red[q][t] = acc[q];
    __syncthreads();
    // C of step t + 1: total density cotangent on the tile and a radius-1 ring
    if (t < X1 * Y1) {
        const int my = t / X1, mx = t - my * X1;
        const int e2 = (my + 1) * X2 + mx + 1;
#pragma unroll
        for (int c = 0; c < C; ++c)
            s_rb[c][t] = (s_rb[c][t] + s_rbb[c][e2]) + lap9s<double, X2>(s_lbt[c], mx + 1, my + 1);
    }
    __syncthreads();
    // the tile's parameter partial, by the last wavefront (idle from here on)
    static_assert(X1 * Y1 <= NTF - 64 && RING2 <= NTF - 64 - NT, "the last wavefront has no site of its own");
    if (t >= NTF - 64) {
        reduce_partial_wave<NP, NT>(s_red, NTF - 64, prev, partial + (int64_t)blockIdx.x * NP, accumulate);
        return;
    }
    if (!inside) return;
    const double omega = k.omega;
    // the un-streamed cotangent at this site: step t's incoming cotangent
    double fin[C][Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int q = (ly + 1 + VY[i]) * X1 + (lx + 1 + VX[i]);
        double v[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            v[c] = (1.0 - omega) * fb_nb[c][i] + s_rb[c][q] + s_jx[c][q] * VX[i] + s_jy[c][q] * VY[i];
            fin[c][i] = v[c];
        }
        store_site<double, C, false>(fbo + (int64_t)i * g.plane * C, s, v);
    }
    if constexpr (DO_A) {
        double dpx[C], dpy[C], rx[C], ry[C];
        local_stencils<C>(lx, ly, s_rho, s_phi, dpx, dpy, rx, ry);
        double rb[C], jbx[C], jby[C], gbx[C], gby[C], lb[C];
        adjoint_local<C>(fin, rho, jx, jy, dpx, dpy, rx, ry, k, rb, jbx, jby, gbx, gby, lb);
        store_local<C>(F, N, s, rb, jbx, jby, gbx, gby, lb);
    }
}

// Fixed-order reduction of the tiles' running partials of a whole segment
// (n vectors of np entries) into pbar (+=): workgroup q sums entry q.
__global__ void __launch_bounds__(BLK) k_adj_reduce(const double* __restrict__ partial, int n, int np,
                                                     double* __restrict__ pbar) {
    __shared__ double s[BLK];
    const int q = blockIdx.x;
    // each thread sums entries b = threadIdx.x + j BLK in increasing j; the
    // loads of a chunk are issued together (terms past n add an exact 0)
    constexpr int CH = 16;
    double a = 0.0;
    for (int b0 = threadIdx.x; b0 < n; b0 += CH * BLK) {
        double v[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int b = b0 + j * BLK;
            v[j] = b < n ? partial[(int64_t)b * np + q] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) a += v[j];
    }
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = BLK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) pbar[q] += s[0];
}

// Kernel C: total density cotangent and the un-streamed population cotangent.
template <int C>
__global__ void __launch_bounds__(BLK) k_adj_c(const double* __restrict__ fbn, double* __restrict__ fbo, Geometry g,
                                                double omega, Fields F) {
    const int N = g.nx * g.ny;
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
    const int y = s / g.nx, x = s - y * g.nx;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double rb = F.rhob_loc[(int64_t)c * N + s] + F.rhob_b[(int64_t)c * N + s] +
                          lapg(F.lb_tot + (int64_t)c * N, g, x, y);
        const double jbx = F.jb[(int64_t)(2 * c) * N + s], jby = F.jb[(int64_t)(2 * c + 1) * N + s];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double pb = (1.0 - omega) * fbn[((int64_t)i * g.plane + s) * C + c] + rb + jbx * VX[i] +
                              jby * VY[i];
            const int t = wrapg(y - VY[i], g.ny, g.wrap_general) * g.nx + wrapg(x - VX[i], g.nx, g.wrap_general);
            fbo[((int64_t)i * g.plane + t) * C + c] = pb;
        }
    }
}

// Cotangent of a state from the cotangent of its densities and momenta (the
// transpose of the moments read-out): fb_i(x - v_i) = rhob(x) + jb(x).v_i.
template <int C>
__global__ void __launch_bounds__(BLK) k_moments_adj(const double* __restrict__ rhob, const double* __restrict__ momb,
                                                      double* __restrict__ fb, Geometry g) {
    const int N = g.nx * g.ny;
    const int s = blockIdx.x * BLK + threadIdx.x;
    if (s >= N) return;
    const int y = s / g.nx, x = s - y * g.nx;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double rb = rhob ? rhob[(int64_t)c * N + s] : 0.0;
        const double jbx = momb ? momb[(int64_t)(2 * c) * N + s] : 0.0;
        const double jby = momb ? momb[(int64_t)(2 * c + 1) * N + s] : 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int t = wrapg(y - VY[i], g.ny, g.wrap_general) * g.nx + wrapg(x - VX[i], g.nx, g.wrap_general);
            fb[((int64_t)i * g.plane + t) * C + c] = rb + jbx * VX[i] + jby * VY[i];
        }
    }
}

}  // namespace adj
}  // namespace vdwlb

using namespace vdwlb;

void vdwlb::release_adjoint_graph(vdwlb_plan& p) {
    for (AdjointGraph& G : p.adj)
        if (G.exec) (void)hipGraphExecDestroy(G.exec);
    p.adj.clear();
}

namespace {

// Geometry of the reverse kernels: their indices reach 3 sites beyond a tile,
// so the cheap periodic wrap needs extents larger than a tile by that much.
Geometry adjoint_geometry(const vdwlb_plan& p) {
    Geometry g = make_geometry(p, adj::TX, adj::TY);
    g.wrap_general = (p.nx < adj::TX + 8 || p.ny < adj::TY + 8) ? 1 : 0;
    return g;
}

struct Layout {
    int64_t N, plane, state;  // elements
    int64_t f0, f1, fb, moms, fields, partial, total;
    int tiles, np;
};

Layout layout(const vdwlb_plan& p, int nsteps) {
    Layout L;
    L.N = (int64_t)p.nx * p.ny;
    L.plane = p.plane;
    L.state = (int64_t)Q * p.C * p.plane;
    L.np = adj::n_params(p.C);
    L.tiles = ((p.nx + adj::TX - 1) / adj::TX) * ((p.ny + adj::TY - 1) / adj::TY);
    int64_t o = 0;
    L.f0 = o;
    o += L.state;
    L.f1 = o;
    o += L.state;
    L.fb = o;
    o += L.state;
    L.moms = o;
    o += (int64_t)nsteps * 3 * p.C * L.N;
    L.fields = o;
    o += 14 * (int64_t)p.C * L.N;
    L.partial = o;  // one running partial vector per tile
    o += (int64_t)L.tiles * L.np;
    L.total = o;
    return L;
}

// Fields of step t: the moments of its forward recompute, and the adjoint
// fields, those read around a tile by the next kernel (rhob_loc, jb, g0b,
// lb) by step parity.
adj::Fields fields_at(const vdwlb_plan& p, const Layout& L, double* ws, int t) {
    adj::Fields F;
    const int64_t CN = (int64_t)p.C * L.N;
    const double* mom0 = ws + L.moms + (int64_t)t * 3 * CN;
    F.rho = mom0;
    F.mom = mom0 + CN;
    double* f = ws + L.fields + ((t & 1) ? 6 * CN : 0);  // per parity: rhob_loc C, jb 2C, g0b 2C, lb C
    F.rhob_loc = f;
    F.jb = f + CN;
    F.g0b = f + 3 * CN;
    F.lb = f + 5 * CN;
    F.rhob_b = ws + L.fields + 12 * CN;
    F.lb_tot = ws + L.fields + 13 * CN;
    return F;
}

template <int C>
struct StepKernels {
    const vdwlb_plan& p;
    const Layout& L;
    double* ws;
    hipStream_t s;
    Geometry g;
    Coeffs<C> k;
    StepKernels(const vdwlb_plan& p_, const Layout& L_, double* ws_, hipStream_t s_)
        : p(p_), L(L_), ws(ws_), s(s_), g(adjoint_geometry(p_)), k(make_coeffs<C>(p_)) {}
    double* partial() const { return ws + L.partial; }
    void a(int t, const double* fbn) {
        hipLaunchKernelGGL((adj::k_adj_a<C>), dim3(L.tiles), dim3(adj::TX * adj::TY), 0, s, fbn, g, k,
                           fields_at(p, L, ws, t));
    }
    // accumulate: the tiles' running partials already hold a later step's
    void b(int t, int accumulate) {
        hipLaunchKernelGGL((adj::k_adj_b<C>), dim3(L.tiles), dim3(adj::TX * adj::TY), 0, s, g, k,
                           fields_at(p, L, ws, t), partial(), accumulate);
    }
    void c(int t, const double* fbn, double* fbo) {
        const int nb = (int)((L.N + adj::BLK - 1) / adj::BLK);
        hipLaunchKernelGGL((adj::k_adj_c<C>), dim3(nb), dim3(adj::BLK), 0, s, fbn, fbo, g, k.omega,
                           fields_at(p, L, ws, t));
    }
    // B and C of step t + 1 fused with A of step t
    void bca(int t, const double* fbn, double* fbo, int accumulate) {
        hipLaunchKernelGGL((adj::k_adj_bca<C, true>), dim3(L.tiles), dim3(adj::NTF), 0, s, fbn, fbo, g, k,
                           fields_at(p, L, ws, t + 1), fields_at(p, L, ws, t), partial(), accumulate);
    }
    // B and C of step 0
    void bc(const double* fbn, double* fbo, int accumulate) {
        const adj::Fields F0 = fields_at(p, L, ws, 0);
        hipLaunchKernelGGL((adj::k_adj_bca<C, false>), dim3(L.tiles), dim3(adj::NTF), 0, s, fbn, fbo, g, k,
                           F0, F0, partial(), accumulate);
    }
};

bool adjoint_fused() {
    const char* v = std::getenv("VDWLB_ADJ_UNFUSED");
    return !(v && v[0] == '1');
}

// The reverse sweep of a segment from fbar_io; the result ends in bufs[n & 1].
// Unfused: per step A, B, C.  Fused: A of the last step, then one kernel per
// earlier step (B and C of the step after it with its own A), and B and C of
// the first step.  Both compute the same values bit for bit.
template <int C>
hipError_t reverse_steps(const vdwlb_plan& p, const Layout& L, double* ws, int nsteps, double* const (&bufs)[2],
                         hipStream_t s, bool fused) {
    StepKernels<C> K(p, L, ws, s);
    if (C > 2 || !fused) {  // the fused kernel's LDS holds C <= 2
        for (int t = nsteps - 1, k = 0; t >= 0; --t, ++k) {
            K.a(t, bufs[k & 1]);
            K.b(t, t < nsteps - 1);
            K.c(t, bufs[k & 1], bufs[(k + 1) & 1]);
        }
        return hipGetLastError();
    }
    if constexpr (C <= 2) {
        K.a(nsteps - 1, bufs[0]);
        // the running partials start with the last step's (each kernel adds step t + 1's)
        for (int t = nsteps - 2, k = 1; t >= 0; --t, ++k) K.bca(t, bufs[(k - 1) & 1], bufs[k & 1], t < nsteps - 2);
        K.bc(bufs[(nsteps - 1) & 1], bufs[nsteps & 1], nsteps > 1);
    }
    return hipGetLastError();
}

// Forward recompute of a segment from the checkpoint already in the
// workspace, keeping each step's moments.
hipError_t enqueue_recompute(const vdwlb_plan& p, const Layout& L, double* ws, int nsteps, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int t = 0; t < nsteps && e == hipSuccess; ++t) {
        double* cur = ws + ((t & 1) ? L.f1 : L.f0);
        double* nxt = ws + ((t & 1) ? L.f0 : L.f1);
        double* m = ws + L.moms + (int64_t)t * 3 * p.C * L.N;
        e = launch_sweep(p, cur, nxt, s, m);  // the sweep also writes this step's moments
    }
    return e;
}

// The reverse sweep of a recomputed segment from fbar_io and the segment's
// parameter cotangents; the result ends in fbar_io.
hipError_t enqueue_reverse(const vdwlb_plan& p, const Layout& L, double* ws, int nsteps, double* fbar_io,
                           double* pbar, hipStream_t s, bool fused) {
    double* const bufs[2] = {fbar_io, ws + L.fb};
    hipError_t e = p.C == 1   ? reverse_steps<1>(p, L, ws, nsteps, bufs, s, fused)
                   : p.C == 2 ? reverse_steps<2>(p, L, ws, nsteps, bufs, s, fused)
                   : p.C == 3 ? reverse_steps<3>(p, L, ws, nsteps, bufs, s, fused)
                              : reverse_steps<4>(p, L, ws, nsteps, bufs, s, fused);
    if (e == hipSuccess) {  // the parameter cotangents of the whole segment, in a fixed order
        hipLaunchKernelGGL(adj::k_adj_reduce, dim3(L.np), dim3(adj::BLK), 0, s, (const double*)(ws + L.partial),
                           L.tiles, L.np, pbar);
        e = hipGetLastError();
    }
    if (e == hipSuccess && (nsteps & 1))
        e = hipMemcpyAsync(fbar_io, ws + L.fb, (size_t)L.state * sizeof(double), hipMemcpyDeviceToDevice, s);
    return e;
}

// Launches the kernels of one part eagerly on stream s, or, when the plan asks
// for graph replay, replays the captured graph of `key` (capturing it on
// first use).  Holds at most six graphs per plan: the recompute and reverse
// graphs of two workspaces for the full segment length and for a shorter
// last segment.
template <typename Enqueue>
vdwlb_status run_part(vdwlb_plan& p, const AdjointGraph& key, hipStream_t s, Enqueue enqueue, const char* what) {
    if (!p.adj_graphs || !graphs_enabled()) {
        const hipError_t e = enqueue(s);
        return e == hipSuccess ? VDWLB_OK : set_device_error(e, what);
    }
    AdjointGraph* G = nullptr;
    for (AdjointGraph& c : p.adj)
        if (c.exec && c.kind == key.kind && c.nsteps == key.nsteps && c.ws == key.ws && c.fbar == key.fbar &&
            c.pbar == key.pbar && c.sched == key.sched && c.map_mode == key.map_mode && c.fused == key.fused)
            G = &c;
    hipError_t e = hipSuccess;
    if (!G) {
        if (!p.capture_stream) e = hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(p.capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return set_device_error(e, what);
        const hipError_t le = enqueue(p.capture_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(p.capture_stream, &g);
        if (le != hipSuccess || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return set_device_error(le != hipSuccess ? le : e, what);
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return set_device_error(e, what);
        if (p.adj.size() >= 6) {  // drop the oldest, once no launch of it can still be running
            e = hipDeviceSynchronize();
            if (e != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return set_device_error(e, what);
            }
            (void)hipGraphExecDestroy(p.adj.front().exec);
            p.adj.erase(p.adj.begin());
        }
        p.adj.push_back(key);
        G = &p.adj.back();
        G->exec = exec;
    }
    e = hipGraphLaunch(G->exec, s);
    return e == hipSuccess ? VDWLB_OK : set_device_error(e, what);
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (the caller's current device is restored).
hipError_t scratch_address(int device, void** out) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void* ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch));
        if (cur >= 0 && cur != device) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

vdwlb_status check_adjoint(const vdwlb_plan* p, int32_t nsteps, const void* workspace) {
    if (!p || !workspace || nsteps < 1) return VDWLB_E_INVALID_ARG;
    if (!state_aligned(*p, workspace)) return VDWLB_E_INVALID_ARG;
    if (p->dtype != VDWLB_F64 || p->C > 4 || p->dim != 2) return VDWLB_E_UNSUPPORTED;
    const Layout L = layout(*p, nsteps);
    if ((int64_t)nsteps * L.tiles > 0x7fffffff) return VDWLB_E_INVALID_ARG;  // partial-sum count of the segment
    return VDWLB_OK;
}

}  // namespace

extern "C" {

int32_t vdwlb_adjoint_param_count(const vdwlb_plan* p) { return p ? adj::n_params(p->C) : 0; }

size_t vdwlb_adjoint_workspace_bytes(const vdwlb_plan* p, int32_t nsteps) {
    if (!p || nsteps < 1) return 0;
    return (size_t)layout(*p, nsteps).total * sizeof(double);
}

vdwlb_status vdwlb_moments_adjoint(vdwlb_plan* p, const void* rho_bar, const void* mom_bar, void* fbar,
                                   void* stream) {
    if (!p || !fbar || (!rho_bar && !mom_bar) || !state_aligned(*p, fbar)) return VDWLB_E_INVALID_ARG;
    if (p->dtype != VDWLB_F64 || p->C > 4 || p->dim != 2) return VDWLB_E_UNSUPPORTED;
    const Geometry g = adjoint_geometry(*p);
    const int nb = (int)(((int64_t)p->nx * p->ny + adj::BLK - 1) / adj::BLK);
    hipError_t e = hipMemsetAsync(fbar, 0, vdwlb_state_bytes(p), (hipStream_t)stream);
    if (e != hipSuccess) return set_device_error(e, "moments adjoint");
    const double* rb = (const double*)rho_bar;
    const double* mb = (const double*)mom_bar;
    hipStream_t s = (hipStream_t)stream;
    if (p->C == 1)
        hipLaunchKernelGGL((adj::k_moments_adj<1>), dim3(nb), dim3(adj::BLK), 0, s, rb, mb, (double*)fbar, g);
    else if (p->C == 2)
        hipLaunchKernelGGL((adj::k_moments_adj<2>), dim3(nb), dim3(adj::BLK), 0, s, rb, mb, (double*)fbar, g);
    else if (p->C == 3)
        hipLaunchKernelGGL((adj::k_moments_adj<3>), dim3(nb), dim3(adj::BLK), 0, s, rb, mb, (double*)fbar, g);
    else
        hipLaunchKernelGGL((adj::k_moments_adj<4>), dim3(nb), dim3(adj::BLK), 0, s, rb, mb, (double*)fbar, g);
    e = hipGetLastError();
    return e == hipSuccess ? VDWLB_OK : set_device_error(e, "moments adjoint");
}

vdwlb_status vdwlb_adjoint_recompute(vdwlb_plan* p, const void* f_ckpt, int32_t nsteps, void* workspace,
                                     void* stream) {
    vdwlb_status st = check_adjoint(p, nsteps, workspace);
    if (st != VDWLB_OK) return st;
    if (!f_ckpt || !state_aligned(*p, f_ckpt)) return VDWLB_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const Layout L = layout(*p, nsteps);
    double* ws = (double*)workspace;
    // the checkpoint goes into the workspace eagerly, so a captured recompute
    // does not depend on where the caller keeps its checkpoints
    const hipError_t e =
        hipMemcpyAsync(ws + L.f0, f_ckpt, (size_t)L.state * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return set_device_error(e, "adjoint checkpoint copy");
    AdjointGraph key;
    key.kind = 0;
    key.nsteps = nsteps;
    key.ws = workspace;
    key.sched = p->sched;
    key.map_mode = p->map_mode;
    return run_part(
        *p, key, s, [&](hipStream_t cs) { return enqueue_recompute(*p, L, ws, nsteps, cs); }, "adjoint recompute");
}

vdwlb_status vdwlb_adjoint_forward(vdwlb_plan* p, const void* f_in, int32_t nsteps, void* f_out, void* workspace,
                                   void* stream) {
    vdwlb_status st = check_adjoint(p, nsteps, workspace);
    if (st != VDWLB_OK) return st;
    if (!f_in || !f_out || !state_aligned(*p, f_in) || !state_aligned(*p, f_out)) return VDWLB_E_INVALID_ARG;
    st = vdwlb_adjoint_recompute(p, f_in, nsteps, workspace, stream);
    if (st != VDWLB_OK) return st;
    // the recompute leaves step nsteps's state in the first buffer after an
    // even number of steps, in the second after an odd number
    const Layout L = layout(*p, nsteps);
    const double* last = (const double*)workspace + ((nsteps & 1) ? L.f1 : L.f0);
    const hipError_t e =
        hipMemcpyAsync(f_out, last, (size_t)L.state * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? VDWLB_OK : set_device_error(e, "adjoint forward state copy");
}

vdwlb_status vdwlb_adjoint_reverse(vdwlb_plan* p, int32_t nsteps, void* fbar_io, void* workspace,
                                   double* pbar_accum, void* stream) {
    vdwlb_status st = check_adjoint(p, nsteps, workspace);
    if (st != VDWLB_OK) return st;
    if (!fbar_io || !pbar_accum || !state_aligned(*p, fbar_io)) return VDWLB_E_INVALID_ARG;
    const Layout L = layout(*p, nsteps);
    double* ws = (double*)workspace;
    AdjointGraph key;
    key.kind = 1;
    key.nsteps = nsteps;
    key.ws = workspace;
    key.fbar = fbar_io;
    key.pbar = pbar_accum;
    key.fused = adjoint_fused();
    return run_part(
        *p, key, (hipStream_t)stream,
        [&](hipStream_t cs) {
            return enqueue_reverse(*p, L, ws, nsteps, (double*)fbar_io, pbar_accum, cs, key.fused);
        },
        "adjoint reverse");
}

vdwlb_status vdwlb_set_adjoint_graphs(vdwlb_plan* p, int32_t enable) {
    if (!p || (enable != 0 && enable != 1)) return VDWLB_E_INVALID_ARG;
    p->adj_graphs = enable == 1;
    return VDWLB_OK;
}

vdwlb_status vdwlb_adjoint_segment(vdwlb_plan* p, const void* f_ckpt, int32_t nsteps, void* fbar_io, void* workspace,
                                   double* pbar_accum, void* stream) {
    vdwlb_status st = check_adjoint(p, nsteps, workspace);
    if (st != VDWLB_OK) return st;
    if (!f_ckpt || !fbar_io || !pbar_accum || !state_aligned(*p, f_ckpt) || !state_aligned(*p, fbar_io))
        return VDWLB_E_INVALID_ARG;
    st = vdwlb_adjoint_recompute(p, f_ckpt, nsteps, workspace, stream);
    if (st != VDWLB_OK) return st;
    return vdwlb_adjoint_reverse(p, nsteps, fbar_io, workspace, pbar_accum, stream);
}

vdwlb_status vdwlb_adjoint_segment_noalloc(vdwlb_plan* p, const void* f_ckpt, int32_t nsteps, void* fbar_io,
                                           double* pbar_accum, void* stream) {
    if (!p || nsteps < 1) return VDWLB_E_INVALID_ARG;
    if (p->dtype != VDWLB_F64 || p->C > 4 || p->dim != 2) return VDWLB_E_UNSUPPORTED;
    if (!f_ckpt || !fbar_io || !pbar_accum || !state_aligned(*p, f_ckpt) || !state_aligned(*p, fbar_io))
        return VDWLB_E_INVALID_ARG;
    if (vdwlb_adjoint_workspace_bytes(p, nsteps) > VDWLB_ADJOINT_SCRATCH_BYTES) return VDWLB_E_CAPACITY;
    void* ws = nullptr;
    hipError_t e = scratch_address(p->device, &ws);
    if (e != hipSuccess) return set_device_error(e, "adjoint scratch address");
    const vdwlb_status st = check_adjoint(p, nsteps, ws);
    if (st != VDWLB_OK) return st;
    // the kernel sequence of vdwlb_adjoint_recompute and vdwlb_adjoint_reverse,
    // launched one by one instead of replayed from a graph
    const Layout L = layout(*p, nsteps);
    hipStream_t s = (hipStream_t)stream;
    double* w = (double*)ws;
    e = hipMemcpyAsync(w + L.f0, f_ckpt, (size_t)L.state * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = enqueue_recompute(*p, L, w, nsteps, s);
    if (e == hipSuccess) e = enqueue_reverse(*p, L, w, nsteps, (double*)fbar_io, pbar_accum, s, adjoint_fused());
    return e == hipSuccess ? VDWLB_OK : set_device_error(e, "adjoint segment (no allocation)");
}

}  // extern "C"
